// Surface term of Eq. (2): one work-item per face.
//
// For a face with left element L and right element R (layout ids), unit
// normal n (L -> R), measure |f| and the reciprocal square roots of the two
// Jacobian determinants, the work-item
//   1. evaluates both traces at the face quadrature points,
//        u_X(q) = (1/sqrt(det J_X)) sum_j trace[code_X][q][j] c_X[m][j],
//      the right trace being the mirror state on a wall;
//   2. evaluates the Rusanov flux F*_q along n at every point;
//   3. projects:  delta_X[m][j] = |f| / sqrt(det J_X) sum_q proj[code_X][q][j] F*_q[m]
//      and applies rhs[L] -= delta_L, rhs[R] += delta_R.
// MODE selects how step 3 reaches memory:
//   kColored  plain read-modify-write; the caller launches one color at a
//             time (Algorithm 1), so no two work-items of a launch touch the
//             same element;
//   kAtomic   hardware floating-point atomic adds, all faces in one launch;
//   kGather   writes -delta_L / +delta_R to buffer slots 2k / 2k+1 of face
//             position k; a second kernel sums each element's slots.
// The basis tables of all face codes are staged once per work-group in LDS.
#pragma once

#include <hip/hip_runtime.h>

#include "euler_dev.hpp"
#include "team.hpp"
#include "volume_team.hpp"

namespace dgc_dev {

enum { kColored = 0, kAtomic = 1, kGather = 2, kCombine = 3, kVolume = 4, kFlux = 5 };

// Compact buffered variant (kFlux): the face pass stores, per face k, the
// record  |f| F*_q[m]  (q < Q, m < M, point-major) followed by one slot that
// carries the two table codes (left | right << 8) as raw bits; a second pass
// lets every element project the records of its faces.
template <int DIM, int Q>
constexpr int compact_stride() { return Q * (DIM + 2) + 1; }
__device__ __forceinline__ double pack_codes(double, int c) { return __hiloint2double(0, c); }
__device__ __forceinline__ float pack_codes(float, int c) { return __int_as_float(c); }
__device__ __forceinline__ int unpack_codes(double v) { return __double2loint(v); }
__device__ __forceinline__ int unpack_codes(float v) { return __float_as_int(v); }

// First color of a stage with the volume term fused in: on a conforming
// mesh every element has exactly one face of every color, so the first
// color's face lanes, which read the element records for the traces anyway,
// also evaluate the volume term of both elements (Eq. (2), first term) and
// write rhs = volume - delta_L (+ delta_R) without reading rhs.  The tables
// are the volume tables of the element type (vb[q][j], vd[d][q][j]).
struct VolArgs {
    const double *elem_geo;
    const double *vb, *vd;
};

// Last color of a colored pass with the SSP-RK3 stage combination fused in:
// on a conforming mesh every element has exactly one face of every color, so
// when its last-color face is done its right-hand side is complete and the
// face's lanes write out = a x + b (y + dt r) instead of r (y = the stage
// input the traces were read from, x = the stage-0 state, or y itself when
// x is null).  f64 only.  x is read up front with the right-hand side: out
// may be x itself (the last stage), so reads of x interleaved with the stores
// would be serialised.
struct CombineArgs {
    const double *x;
    double *out;
    double a, b, dt;
};

__device__ __forceinline__ void combine_store(const CombineArgs &cmb, size_t idx, double x, double y, double r) {
    cmb.out[idx] = cmb.a * x + cmb.b * (y + cmb.dt * r);
}
template <class T>
__device__ __forceinline__ void combine_store(const CombineArgs &, size_t, T, T, T) {}

template <class T>
__device__ __forceinline__ void atomic_add(T *addr, T v) {
    unsafeAtomicAdd(addr, v);
}

// Work-groups of a launch are dealt round-robin to the 8 XCDs (each with its
// own L2).  With remap set, XCD x processes one contiguous range of logical
// work-groups instead of every eighth one; the map is a bijection of
// [0, gridDim.x).
__device__ __forceinline__ unsigned logical_block(int remap) {
    const unsigned b = blockIdx.x;
    if (!remap) return b;
    const unsigned nb = gridDim.x, x = b % 8u, q = nb / 8u, r = nb % 8u;
    return x * q + (x < r ? x : r) + b / 8u;
}

template <int DIM, int NP, int Q, int MODE, class T>
__global__ __launch_bounds__(256) void surface_kernel(
    int64_t f_begin, int64_t f_end, int64_t n_face, int64_t n_elem,
    const int32_t *__restrict__ face_lr, const uint8_t *__restrict__ face_code,
    const double *__restrict__ face_geo, const double *__restrict__ tab_trace,
    const double *__restrict__ tab_proj, int n_codes,
    const T *__restrict__ U, T *__restrict__ rhs, T *__restrict__ buf, int remap) {
    constexpr int M = DIM + 2;
    constexpr int REC = M * NP;
    extern __shared__ unsigned char smem_raw[];
    T *s_tr = reinterpret_cast<T *>(smem_raw);
    T *s_pr = s_tr + n_codes * Q * NP;
    const int ntab = n_codes * Q * NP;
    for (int i = threadIdx.x; i < ntab; i += blockDim.x) {
        s_tr[i] = T(tab_trace[i]);
        s_pr[i] = T(tab_proj[i]);
    }
    __syncthreads();

    const int64_t k = f_begin + (int64_t)logical_block(remap) * blockDim.x + threadIdx.x;
    if (k >= f_end) return;

    const int32_t L = face_lr[k];
    const int32_t R = face_lr[n_face + k];
    const int cL = face_code[k];
    const int cR = face_code[n_face + k];
    // a malformed face (ids or codes out of range) is skipped, never dereferenced
    if (L < 0 || L >= n_elem || R >= n_elem || cL >= n_codes || cR >= n_codes) return;
    T n[DIM];
#pragma unroll
    for (int d = 0; d < DIM; ++d) n[d] = T(face_geo[d * n_face + k]);
    const double len = face_geo[DIM * n_face + k];
    const double isL = face_geo[(DIM + 1) * n_face + k];
    const double isR = face_geo[(DIM + 2) * n_face + k];

    // traces at the face points
    T qL[Q][M], qR[Q][M];
    {
        const T *uL = U + (size_t)L * REC;
        const T *tl = s_tr + cL * Q * NP;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            T c[NP];
#pragma unroll
            for (int j = 0; j < NP; ++j) c[j] = uL[m * NP + j];
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                T a = 0;
#pragma unroll
                for (int j = 0; j < NP; ++j) a += tl[q * NP + j] * c[j];
                qL[q][m] = a * T(isL);
            }
        }
    }
    if (R >= 0) {
        const T *uR = U + (size_t)R * REC;
        const T *tr = s_tr + cR * Q * NP;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            T c[NP];
#pragma unroll
            for (int j = 0; j < NP; ++j) c[j] = uR[m * NP + j];
#pragma unroll
            for (int q = 0; q < Q; ++q) {
                T a = 0;
#pragma unroll
                for (int j = 0; j < NP; ++j) a += tr[q * NP + j] * c[j];
                qR[q][m] = a * T(isR);
            }
        }
    } else {
#pragma unroll
        for (int q = 0; q < Q; ++q) wall_ghost<DIM, T>(qL[q], n, qR[q]);
    }

    // numerical flux at every point
    T Fs[Q][M];
#pragma unroll
    for (int q = 0; q < Q; ++q) rusanov<DIM, T>(qL[q], qR[q], n, Fs[q]);

    // projection and accumulation, left side
    {
        const T sL = T(len * isL);
        const T *pl = s_pr + cL * Q * NP;
        T *dst = MODE == kGather ? buf + (size_t)(2 * k) * REC : rhs + (size_t)L * REC;
#pragma unroll
        for (int m = 0; m < M; ++m) {
#pragma unroll
            for (int j = 0; j < NP; ++j) {
                T a = 0;
#pragma unroll
                for (int q = 0; q < Q; ++q) a += pl[q * NP + j] * Fs[q][m];
                a *= sL;
                if (MODE == kColored) dst[m * NP + j] -= a;
                else if (MODE == kAtomic) atomic_add<T>(dst + m * NP + j, -a);
                else dst[m * NP + j] = -a;
            }
        }
    }
    if (R >= 0) {
        const T sR = T(len * isR);
        const T *pr = s_pr + cR * Q * NP;
        T *dst = MODE == kGather ? buf + (size_t)(2 * k + 1) * REC : rhs + (size_t)R * REC;
#pragma unroll
        for (int m = 0; m < M; ++m) {
#pragma unroll
            for (int j = 0; j < NP; ++j) {
                T a = 0;
#pragma unroll
                for (int q = 0; q < Q; ++q) a += pr[q * NP + j] * Fs[q][m];
                a *= sR;
                if (MODE == kColored) dst[m * NP + j] += a;
                else if (MODE == kAtomic) atomic_add<T>(dst + m * NP + j, a);
                else dst[m * NP + j] = a;
            }
        }
    }
}

// Callback a face routine runs after it has issued every memory read of its
// face and before it uses the LDS tables: the kernels stage their tables
// there (and meet at the work-group barrier), so that the table reads, the
// face's header reads and its record reads are in flight together instead of
// one after the other.  Every thread of the work-group must reach it.
struct NoMid {
    __device__ __forceinline__ void operator()() const {}
};

// Team form of the face work: TEAM lanes per face (4 for M = 4, 8 for
// M = 5); lane r < M owns conserved variable r.  Each lane reads and
// updates the NP modes of its variable, so one load instruction of a team
// touches one contiguous stretch of the element record instead of one
// record per lane.  The traces of all variables are exchanged inside the
// team; every lane evaluates component r of the flux of the full state
// (rusanov_component: the shared wave speeds and pressures, no selection
// among the components) and projects it.  Same formulas and accumulation
// modes as surface_kernel.  A thread whose face is not `active` (beyond the
// launch's range) or is malformed (ids or codes out of range) reads nothing,
// takes part in `mid` and returns.
template <int DIM, int NP, int Q, int MODE, class T, bool PREFETCH, int QV = 1, class Mid = NoMid>
__device__ __forceinline__ void team_face(
    int64_t k, int r, int64_t n_face, int64_t n_elem,
    const int32_t *__restrict__ face_lr, const uint8_t *__restrict__ face_code,
    const double *__restrict__ face_geo, const T *__restrict__ s_tr, const T *__restrict__ s_pr, int n_codes,
    const T *__restrict__ U, T *__restrict__ rhs, T *__restrict__ buf, const CombineArgs &cmb = CombineArgs{},
    const VolArgs &va = VolArgs{}, bool active = true, const Mid &mid = Mid{}) {
    constexpr int M = DIM + 2;
    constexpr int REC = M * NP;
    constexpr int TEAM = M <= 4 ? 4 : 8;
    constexpr bool RMW = MODE == kColored || MODE == kCombine;
    int32_t L = -1, R = -1;
    int cL = 0, cR = 0;
    T n[DIM];
    double len = 0, isL = 0, isR = 0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) n[d] = 0;
    if (active) {
        L = face_lr[k];
        R = face_lr[n_face + k];
        cL = face_code[k];
        cR = face_code[n_face + k];
#pragma unroll
        for (int d = 0; d < DIM; ++d) n[d] = T(face_geo[d * n_face + k]);
        len = face_geo[DIM * n_face + k];
        isL = face_geo[(DIM + 1) * n_face + k];
        isR = face_geo[(DIM + 2) * n_face + k];
    }
    const bool ok = active && L >= 0 && L < n_elem && R < n_elem && cL < n_codes && cR < n_codes;
    const bool own = r < M;
    const bool rd = ok && own;

    // the right-hand-side reads of a colored update are issued up front with
    // the DOF reads (PREFETCH); the right side's at N_p = 9 in f64 once the
    // traces are formed (LATE_R), when the modes of both sides are dead: the
    // kernel then fits three waves per SIMD instead of two
    constexpr bool LATE_R = PREFETCH && MODE == kColored && sizeof(T) == 8 && NP == 9;
    T pre_L[NP], pre_R[NP];
    if (PREFETCH && RMW && rd) {
        const T *a = rhs + (size_t)L * REC + r * NP;
#pragma unroll
        for (int j = 0; j < NP; ++j) pre_L[j] = a[j];
        if (!LATE_R && R >= 0) {
            const T *b = rhs + (size_t)R * REC + r * NP;
#pragma unroll
            for (int j = 0; j < NP; ++j) pre_R[j] = b[j];
        }
    }
    // the stage-0 state of a fused combination (kCombine with x set)
    T xL[NP], xR[NP];
    if (MODE == kCombine && cmb.x && rd) {
        const double *a = cmb.x + (size_t)L * REC + r * NP;
#pragma unroll
        for (int j = 0; j < NP; ++j) xL[j] = T(a[j]);
        if (R >= 0) {
            const double *b = cmb.x + (size_t)R * REC + r * NP;
#pragma unroll
            for (int j = 0; j < NP; ++j) xR[j] = T(b[j]);
        }
    }
    // my variable's modes on both sides (zero on lanes that own none)
    T cL_[NP], cR_[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) cL_[j] = cR_[j] = T(0);
    if (rd) {
        const T *uL = U + (size_t)L * REC + r * NP;
#pragma unroll
        for (int j = 0; j < NP; ++j) cL_[j] = uL[j];
        if (R >= 0) {
            const T *uR = U + (size_t)R * REC + r * NP;
#pragma unroll
            for (int j = 0; j < NP; ++j) cR_[j] = uR[j];
        }
    }
    // the geometry of both elements for the fused volume term (kVolume)
    T JiL[DIM * DIM], JiR[DIM * DIM];
    double sqL = 1, sqR = 1;
    if constexpr (MODE == kVolume) {
        if (ok) {
            load_elem_geo<DIM, T>(L, n_elem, va.elem_geo, JiL, sqL);
            if (R >= 0) load_elem_geo<DIM, T>(R, n_elem, va.elem_geo, JiR, sqR);
        }
    }
    mid();
    if (!ok) return;

    // the volume term of both elements, my variable (kVolume; the face
    // record's 1/sqrt(det J) is the division's correctly rounded result)
    T vL[NP], vR[NP];
    if constexpr (MODE == kVolume) {
        constexpr int UNR = fused_volume_unroll(NP);
        volume_team_core_geo<DIM, NP, QV, T, double, UNR>(r, JiL, sqL, isL, va.vb, va.vd, cL_, vL);
        if (R >= 0) volume_team_core_geo<DIM, NP, QV, T, double, UNR>(r, JiR, sqR, isR, va.vb, va.vd, cR_, vR);
    }
    // my variable's traces on both sides
    T tL[Q], tR[Q];
    {
        const T *tl = s_tr + cL * Q * NP;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            T a = 0;
#pragma unroll
            for (int j = 0; j < NP; ++j) a += tl[q * NP + j] * cL_[j];
            tL[q] = a * T(isL);
        }
    }
    if (R >= 0) {
        const T *tr = s_tr + cR * Q * NP;
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            T a = 0;
#pragma unroll
            for (int j = 0; j < NP; ++j) a += tr[q * NP + j] * cR_[j];
            tR[q] = a * T(isR);
        }
    }

    if (LATE_R && rd && R >= 0) {
        const T *b = rhs + (size_t)R * REC + r * NP;
#pragma unroll
        for (int j = 0; j < NP; ++j) pre_R[j] = b[j];
    }

    // full states at every point, my component of their flux
    T n_r = 0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) n_r = r == 1 + d ? n[d] : n_r;
    const T sel_e = r == M - 1 ? T(1) : T(0);
    T Fm[Q];
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        T uLq[M], uRq[M];
#pragma unroll
        for (int m = 0; m < M; ++m) uLq[m] = team_bcast<TEAM>(tL[q], m);
        T ownR;
        if (R >= 0) {
#pragma unroll
            for (int m = 0; m < M; ++m) uRq[m] = team_bcast<TEAM>(tR[q], m);
            ownR = tR[q];
        } else {
            wall_ghost<DIM, T>(uLq, n, uRq);
            ownR = uRq[0];
#pragma unroll
            for (int m = 1; m < M; ++m) ownR = r == m ? uRq[m] : ownR;
        }
        Fm[q] = rusanov_component<DIM, T>(uLq, uRq, n, tL[q], ownR, n_r, sel_e);
    }
    if (!own) return;
    if constexpr (MODE == kFlux) {
        T *rec = buf + (size_t)k * compact_stride<DIM, Q>();
#pragma unroll
        for (int q = 0; q < Q; ++q) rec[q * M + r] = Fm[q] * T(len);
        if (r == 0) rec[Q * M] = pack_codes(T(0), cL | (R >= 0 ? cR : 0xFF) << 8);
        return;
    }

    {
        const T sL = T(len * isL);
        const T *pl = s_pr + cL * Q * NP;
        T *dst = (MODE == kGather ? buf + (size_t)(2 * k) * REC : rhs + (size_t)L * REC) + r * NP;
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            T a = 0;
#pragma unroll
            for (int q = 0; q < Q; ++q) a += pl[q * NP + j] * Fm[q];
            a *= sL;
            if (MODE == kColored) dst[j] = (PREFETCH ? pre_L[j] : dst[j]) - a;
            else if (MODE == kVolume) dst[j] = vL[j] - a;
            else if (MODE == kCombine)
                combine_store(cmb, (size_t)L * REC + r * NP + j, cmb.x ? xL[j] : cL_[j], cL_[j],
                              (PREFETCH ? pre_L[j] : dst[j]) - a);
            else if (MODE == kAtomic) atomic_add<T>(dst + j, -a);
            else dst[j] = -a;
        }
    }
    if (R >= 0) {
        const T sR = T(len * isR);
        const T *pr = s_pr + cR * Q * NP;
        T *dst = (MODE == kGather ? buf + (size_t)(2 * k + 1) * REC : rhs + (size_t)R * REC) + r * NP;
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            T a = 0;
#pragma unroll
            for (int q = 0; q < Q; ++q) a += pr[q * NP + j] * Fm[q];
            a *= sR;
            if (MODE == kColored) dst[j] = (PREFETCH ? pre_R[j] : dst[j]) + a;
            else if (MODE == kVolume) dst[j] = vR[j] + a;
            else if (MODE == kCombine)
                combine_store(cmb, (size_t)R * REC + r * NP + j, cmb.x ? xR[j] : cR_[j], cR_[j],
                              (PREFETCH ? pre_R[j] : dst[j]) + a);
            else if (MODE == kAtomic) atomic_add<T>(dst + j, a);
            else dst[j] = a;
        }
    }
}

// Mode-team form of the face work for N_p = 4 (tetrahedra, p = 1): a team
// of 4 lanes per face, lane j owns mode j of every conserved variable.  Each
// lane forms its mode's share of all traces, the shares are summed across
// the quad with DPP, lane j evaluates the flux of the full state at point j
// (Q <= 4; a fourth lane repeats the last point), the quad broadcasts the
// fluxes and lane j projects onto mode j.  Loads and stores of one record are
// 4 consecutive values per instruction (the variable-per-lane team would
// need 8 lanes for M = 5).
template <int DIM, int NP, int Q, int MODE, class T, bool PREFETCH, int QV = 1, class Mid = NoMid>
__device__ __forceinline__ void mode_team_face(
    int64_t k, int j, int64_t n_face, int64_t n_elem,
    const int32_t *__restrict__ face_lr, const uint8_t *__restrict__ face_code,
    const double *__restrict__ face_geo, const T *__restrict__ s_tr, const T *__restrict__ s_pr, int n_codes,
    const T *__restrict__ U, T *__restrict__ rhs, T *__restrict__ buf, const CombineArgs &cmb = CombineArgs{},
    const T *__restrict__ s_vb = nullptr, const T *__restrict__ s_vd = nullptr, const double *elem_geo = nullptr,
    bool active = true, const Mid &mid = Mid{}) {
    static_assert(NP == 4, "mode teams need exactly four modes");
    constexpr int M = DIM + 2;
    constexpr int REC = M * NP;
    constexpr bool RMW = MODE == kColored || MODE == kCombine;
    int32_t L = -1, R = -1;
    int cL = 0, cR = 0;
    T n[DIM];
    double len = 0, isL = 0, isR = 0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) n[d] = 0;
    if (active) {
        L = face_lr[k];
        R = face_lr[n_face + k];
        cL = face_code[k];
        cR = face_code[n_face + k];
#pragma unroll
        for (int d = 0; d < DIM; ++d) n[d] = T(face_geo[d * n_face + k]);
        len = face_geo[DIM * n_face + k];
        isL = face_geo[(DIM + 1) * n_face + k];
        isR = face_geo[(DIM + 2) * n_face + k];
    }
    const bool ok = active && L >= 0 && L < n_elem && R < n_elem && cL < n_codes && cR < n_codes;

    T pre_L[M], pre_R[M];
    if (PREFETCH && RMW && ok) {
#pragma unroll
        for (int m = 0; m < M; ++m) pre_L[m] = rhs[(size_t)L * REC + m * NP + j];
        if (R >= 0) {
#pragma unroll
            for (int m = 0; m < M; ++m) pre_R[m] = rhs[(size_t)R * REC + m * NP + j];
        }
    }
    // the stage-0 state of a fused combination (kCombine with x set)
    T xL[M], xR[M];
    if (MODE == kCombine && cmb.x && ok) {
#pragma unroll
        for (int m = 0; m < M; ++m) xL[m] = T(cmb.x[(size_t)L * REC + m * NP + j]);
        if (R >= 0) {
#pragma unroll
            for (int m = 0; m < M; ++m) xR[m] = T(cmb.x[(size_t)R * REC + m * NP + j]);
        }
    }
    // my mode of every variable on both sides
    T cL_[M], cR_[M];
#pragma unroll
    for (int m = 0; m < M; ++m) cL_[m] = cR_[m] = T(0);
    if (ok) {
#pragma unroll
        for (int m = 0; m < M; ++m) cL_[m] = U[(size_t)L * REC + m * NP + j];
        if (R >= 0) {
#pragma unroll
            for (int m = 0; m < M; ++m) cR_[m] = U[(size_t)R * REC + m * NP + j];
        }
    }
    // the geometry of both elements for the fused volume term (kVolume)
    T JiL[DIM * DIM], JiR[DIM * DIM];
    double sqL = 1, sqR = 1;
    if constexpr (MODE == kVolume) {
        if (ok) {
            load_elem_geo<DIM, T>(L, n_elem, elem_geo, JiL, sqL);
            if (R >= 0) load_elem_geo<DIM, T>(R, n_elem, elem_geo, JiR, sqR);
        }
    }
    mid();
    if (!ok) return;

    // the volume term of both elements, my mode (kVolume; tables in LDS)
    T vL[M], vR[M];
    if constexpr (MODE == kVolume) {
        volume_mode_team_core_geo<DIM, NP, QV, T, T>(j, JiL, sqL, isL, s_vb, s_vd, cL_, vL);
        if (R >= 0) volume_mode_team_core_geo<DIM, NP, QV, T, T>(j, JiR, sqR, isR, s_vb, s_vd, cR_, vR);
    }
    // the traces at every point are sums over the quad of each lane's mode
    // share; lane j keeps those of point min(j, Q - 1) and evaluates the flux
    // there only, and the quad exchanges the fluxes for the projection
    static_assert(Q <= 4, "one quadrature point per lane of the quad");
    const int qo = j < Q ? j : Q - 1;
    T uL[M], uR[M];
#pragma unroll
    for (int m = 0; m < M; ++m) uL[m] = uR[m] = T(0);
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        const T t = s_tr[(cL * Q + q) * NP + j];
#pragma unroll
        for (int m = 0; m < M; ++m) {
            const T v = quad_sum(t * cL_[m]) * T(isL);
            uL[m] = q == qo ? v : uL[m];
        }
    }
    if (R >= 0) {
#pragma unroll
        for (int q = 0; q < Q; ++q) {
            const T t = s_tr[(cR * Q + q) * NP + j];
#pragma unroll
            for (int m = 0; m < M; ++m) {
                const T v = quad_sum(t * cR_[m]) * T(isR);
                uR[m] = q == qo ? v : uR[m];
            }
        }
    } else {
        wall_ghost<DIM, T>(uL, n, uR);
    }
    T Fo[M];
    rusanov<DIM, T>(uL, uR, n, Fo);
    T F[Q][M];
#pragma unroll
    for (int q = 0; q < Q; ++q)
#pragma unroll
        for (int m = 0; m < M; ++m) F[q][m] = team_bcast<4>(Fo[m], q);
    {
        const T sL = T(len * isL);
        T *dst = MODE == kGather ? buf + (size_t)(2 * k) * REC : rhs + (size_t)L * REC;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            T a = 0;
#pragma unroll
            for (int q = 0; q < Q; ++q) a += s_pr[(cL * Q + q) * NP + j] * F[q][m];
            a *= sL;
            if (MODE == kColored) dst[m * NP + j] = (PREFETCH ? pre_L[m] : dst[m * NP + j]) - a;
            else if (MODE == kVolume) dst[m * NP + j] = vL[m] - a;
            else if (MODE == kCombine)
                combine_store(cmb, (size_t)L * REC + m * NP + j, cmb.x ? xL[m] : cL_[m], cL_[m],
                              (PREFETCH ? pre_L[m] : dst[m * NP + j]) - a);
            else if (MODE == kAtomic) atomic_add<T>(dst + m * NP + j, -a);
            else dst[m * NP + j] = -a;
        }
    }
    if (R >= 0) {
        const T sR = T(len * isR);
        T *dst = MODE == kGather ? buf + (size_t)(2 * k + 1) * REC : rhs + (size_t)R * REC;
#pragma unroll
        for (int m = 0; m < M; ++m) {
            T a = 0;
#pragma unroll
            for (int q = 0; q < Q; ++q) a += s_pr[(cR * Q + q) * NP + j] * F[q][m];
            a *= sR;
            if (MODE == kColored) dst[m * NP + j] = (PREFETCH ? pre_R[m] : dst[m * NP + j]) + a;
            else if (MODE == kVolume) dst[m * NP + j] = vR[m] + a;
            else if (MODE == kCombine)
                combine_store(cmb, (size_t)R * REC + m * NP + j, cmb.x ? xR[m] : cR_[m], cR_[m],
                              (PREFETCH ? pre_R[m] : dst[m * NP + j]) + a);
            else if (MODE == kAtomic) atomic_add<T>(dst + m * NP + j, a);
            else dst[m * NP + j] = a;
        }
    }
}

// Occupancy asked of the f32 fused first-color kernels for 2D triangles at
// p = 2 (N_p = 6): six waves per SIMD fit their registers without spills
// (the compiler's own choice leaves them at five); 1 (no request) otherwise.
template <class T>
constexpr int f32_min_waves(int dim, int np) {
    return (sizeof(T) == 4 && dim == 2 && np == 6) ? 6 : 1;
}

// Basis tables of every face code, copied once per work-group into LDS.
template <class T>
__device__ __forceinline__ void stage_tables(T *s_tr, T *s_pr, const double *__restrict__ tab_trace,
                                             const double *__restrict__ tab_proj, int ntab) {
    for (int i = threadIdx.x; i < ntab; i += blockDim.x) {
        s_tr[i] = T(tab_trace[i]);
        s_pr[i] = T(tab_proj[i]);
    }
    __syncthreads();
}

// The same staging in two halves, for kernels that issue their face reads
// in between: issue() reads this thread's share of the tables into
// registers when both tables fit in KT values per thread of a work-group of
// `block` threads (larger tables are copied to LDS right there, before the
// face reads: a copy loop behind the face reads would wait for them once per
// trip); store() writes the registers to LDS and meets the work-group
// barrier.  Issuing the table reads first keeps them ahead of the face
// reads, so the wait for the tables does not wait for the records too.
// s_pr must follow s_tr directly in LDS.
template <class T, int KT = 4>
struct TableStage {
    double v[KT];
    int ntab, block;
    bool fits;

    __device__ __forceinline__ void issue(T *s_tr, const double *__restrict__ tab_trace,
                                          const double *__restrict__ tab_proj, int ntab_, int block_) {
        ntab = ntab_;
        block = block_;
        fits = 2 * ntab <= KT * block;
        if (fits) {
#pragma unroll
            for (int i = 0; i < KT; ++i) {
                const int idx = (int)threadIdx.x + i * block;
                if (idx < 2 * ntab) v[i] = idx < ntab ? tab_trace[idx] : tab_proj[idx - ntab];
            }
        } else {
            for (int i = threadIdx.x; i < ntab; i += block) {
                s_tr[i] = T(tab_trace[i]);
                s_tr[ntab + i] = T(tab_proj[i]);
            }
        }
    }
    __device__ __forceinline__ void store(T *s_tr) const {
        if (fits) {
#pragma unroll
            for (int i = 0; i < KT; ++i) {
                const int idx = (int)threadIdx.x + i * block;
                if (idx < 2 * ntab) s_tr[idx] = T(v[i]);
            }
        }
        __syncthreads();
    }
};

template <int DIM, int NP, int Q, int MODE, class T, bool PREFETCH>
__global__ __launch_bounds__(256) void surface_team_kernel(
    int64_t f_begin, int64_t f_end, int64_t n_face, int64_t n_elem,
    const int32_t *__restrict__ face_lr, const uint8_t *__restrict__ face_code,
    const double *__restrict__ face_geo, const double *__restrict__ tab_trace,
    const double *__restrict__ tab_proj, int n_codes,
    const T *__restrict__ U, T *__restrict__ rhs, T *__restrict__ buf, int remap, int block) {
    constexpr int TEAM = DIM + 2 <= 4 ? 4 : 8;
    extern __shared__ unsigned char smem_raw[];
    T *s_tr = reinterpret_cast<T *>(smem_raw);
    T *s_pr = s_tr + n_codes * Q * NP;
    TableStage<T> tabs;
    tabs.issue(s_tr, tab_trace, tab_proj, n_codes * Q * NP, block);
    const int r = threadIdx.x % TEAM;
    const int64_t k = f_begin + ((int64_t)logical_block(remap) * block + threadIdx.x) / TEAM;
    team_face<DIM, NP, Q, MODE, T, PREFETCH>(k, r, n_face, n_elem, face_lr, face_code, face_geo, s_tr, s_pr, n_codes,
                                             U, rhs, buf, CombineArgs{}, VolArgs{}, k < f_end,
                                             [&] { tabs.store(s_tr); });
}

template <int DIM, int NP, int Q, int MODE, class T>
__global__ __launch_bounds__(256) void surface_mode_team_kernel(
    int64_t f_begin, int64_t f_end, int64_t n_face, int64_t n_elem,
    const int32_t *__restrict__ face_lr, const uint8_t *__restrict__ face_code,
    const double *__restrict__ face_geo, const double *__restrict__ tab_trace,
    const double *__restrict__ tab_proj, int n_codes,
    const T *__restrict__ U, T *__restrict__ rhs, T *__restrict__ buf, int remap, int block) {
    extern __shared__ unsigned char smem_raw[];
    T *s_tr = reinterpret_cast<T *>(smem_raw);
    T *s_pr = s_tr + n_codes * Q * NP;
    TableStage<T> tabs;
    tabs.issue(s_tr, tab_trace, tab_proj, n_codes * Q * NP, block);
    const int64_t k = f_begin + ((int64_t)logical_block(remap) * block + threadIdx.x) / 4;
    mode_team_face<DIM, NP, Q, MODE, T, true>(k, threadIdx.x % 4, n_face, n_elem, face_lr, face_code, face_geo,
                                              s_tr, s_pr, n_codes, U, rhs, buf, CombineArgs{}, nullptr, nullptr,
                                              nullptr, k < f_end, [&] { tabs.store(s_tr); });
}

// Last color of an SSP-RK3 stage with the stage combination fused in (see
// CombineArgs): the team form, or the mode team for tetrahedra at p = 1.
template <int DIM, int NP, int Q, bool MT>
__global__ __launch_bounds__(256) void surface_combine_kernel(
    int64_t f_begin, int64_t f_end, int64_t n_face, int64_t n_elem,
    const int32_t *__restrict__ face_lr, const uint8_t *__restrict__ face_code,
    const double *__restrict__ face_geo, const double *__restrict__ tab_trace,
    const double *__restrict__ tab_proj, int n_codes,
    const double *__restrict__ U, double *__restrict__ rhs, CombineArgs cmb, int block) {
    constexpr int TEAM = MT ? 4 : (DIM + 2 <= 4 ? 4 : 8);
    extern __shared__ unsigned char smem_raw[];
    double *s_tr = reinterpret_cast<double *>(smem_raw);
    double *s_pr = s_tr + n_codes * Q * NP;
    const int64_t k = f_begin + ((int64_t)blockIdx.x * block + threadIdx.x) / TEAM;
    if constexpr (NP >= 15) {
        // at p >= 4 the stage-0 state, the right-hand side and the records of
        // both sides held across the barrier would spill: stage the tables
        // first, then read the face
        stage_tables<double>(s_tr, s_pr, tab_trace, tab_proj, n_codes * Q * NP);
        team_face<DIM, NP, Q, kCombine, double, true>(k, threadIdx.x % TEAM, n_face, n_elem, face_lr, face_code,
                                                       face_geo, s_tr, s_pr, n_codes, U, rhs, nullptr, cmb,
                                                       VolArgs{}, k < f_end);
        return;
    }
    TableStage<double> tabs;
    tabs.issue(s_tr, tab_trace, tab_proj, n_codes * Q * NP, block);
    auto mid = [&] { tabs.store(s_tr); };
    if constexpr (MT)
        mode_team_face<DIM, NP, Q, kCombine, double, true>(k, threadIdx.x % 4, n_face, n_elem, face_lr, face_code,
                                                            face_geo, s_tr, s_pr, n_codes, U, rhs, nullptr, cmb,
                                                            nullptr, nullptr, nullptr, k < f_end, mid);
    else
        team_face<DIM, NP, Q, kCombine, double, true>(k, threadIdx.x % TEAM, n_face, n_elem, face_lr, face_code,
                                                       face_geo, s_tr, s_pr, n_codes, U, rhs, nullptr, cmb,
                                                       VolArgs{}, k < f_end, mid);
}

// First color of a stage with the volume term fused in (see VolArgs): the
// team form, or the mode team for tetrahedra at p = 1 (volume tables staged
// in LDS after the face tables).
template <int DIM, int NP, int Q, int QV, bool MT, class T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(f32_min_waves<T>(DIM, NP), 8)))
void surface_volume_kernel(
    int64_t f_begin, int64_t f_end, int64_t n_face, int64_t n_elem,
    const int32_t *__restrict__ face_lr, const uint8_t *__restrict__ face_code,
    const double *__restrict__ face_geo, const double *__restrict__ tab_trace,
    const double *__restrict__ tab_proj, int n_codes,
    const T *__restrict__ U, T *__restrict__ rhs, VolArgs va, int remap, int block) {
    constexpr int TEAM = MT ? 4 : (DIM + 2 <= 4 ? 4 : 8);
    extern __shared__ unsigned char smem_raw[];
    T *s_tr = reinterpret_cast<T *>(smem_raw);
    T *s_pr = s_tr + n_codes * Q * NP;
    TableStage<T> tabs;
    tabs.issue(s_tr, tab_trace, tab_proj, n_codes * Q * NP, block);
    const int64_t k = f_begin + ((int64_t)logical_block(remap) * block + threadIdx.x) / TEAM;
    if constexpr (MT) {
        T *s_vb = s_pr + n_codes * Q * NP;
        T *s_vd = s_vb + QV * NP;
        mode_team_face<DIM, NP, Q, kVolume, T, false, QV>(
            k, threadIdx.x % 4, n_face, n_elem, face_lr, face_code, face_geo, s_tr, s_pr, n_codes, U, rhs, nullptr,
            CombineArgs{}, s_vb, s_vd, va.elem_geo, k < f_end, [&] {
                for (int i = threadIdx.x; i < QV * NP; i += block) s_vb[i] = T(va.vb[i]);
                for (int i = threadIdx.x; i < DIM * QV * NP; i += block) s_vd[i] = T(va.vd[i]);
                tabs.store(s_tr);  // its barrier covers the volume tables too
            });
    } else {
        team_face<DIM, NP, Q, kVolume, T, false, QV>(k, threadIdx.x % TEAM, n_face, n_elem, face_lr, face_code,
                                                     face_geo, s_tr, s_pr, n_codes, U, rhs, nullptr, CombineArgs{},
                                                     va, k < f_end, [&] { tabs.store(s_tr); });
    }
}

// Second pass of the compact buffered variant: element k (a team of lanes,
// lane r < M owning variable r) visits its faces through elem_slots
// (2 * face + side), reads the face's record (|f| F*_q of its variable and
// the side's table code) and adds  -/+ (1/sqrt(det J_k)) sum_q proj[code][q][j] |f| F*_q
// (minus on the left side, plus on the right) to its right-hand side, which
// it reads and writes once.  The projection tables are staged in LDS.
template <int DIM, int NP, int Q, class T>
__global__ __launch_bounds__(256) void compact_gather_kernel(
    int64_t n_elem, int64_t n_face, int max_slots, const int32_t *__restrict__ elem_slots,
    const double *__restrict__ elem_geo, const double *__restrict__ tab_proj, int n_codes,
    const T *__restrict__ flux, T *__restrict__ rhs) {
    constexpr int M = DIM + 2;
    constexpr int REC = M * NP;
    constexpr int TEAM = M <= 4 ? 4 : 8;
    constexpr int RS = compact_stride<DIM, Q>();
    extern __shared__ unsigned char smem_raw[];
    T *s_pr = reinterpret_cast<T *>(smem_raw);
    for (int i = threadIdx.x; i < n_codes * Q * NP; i += blockDim.x) s_pr[i] = T(tab_proj[i]);
    __syncthreads();
    const int r = threadIdx.x % TEAM;
    const int64_t k = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / TEAM;
    if (k >= n_elem || r >= M) return;
    const T isq = T(1.0 / elem_geo[(size_t)DIM * DIM * n_elem + k]);
    T *dst = rhs + (size_t)k * REC + r * NP;
    T acc[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) acc[j] = dst[j];
    for (int s = 0; s < max_slots; ++s) {
        const int32_t slot = elem_slots[(int64_t)s * n_elem + k];
        if (slot < 0 || slot >= 2 * n_face) continue;
        const int64_t f = slot >> 1;
        const int side = slot & 1;
        const T *rec = flux + (size_t)f * RS;
        T F[Q];
#pragma unroll
        for (int q = 0; q < Q; ++q) F[q] = rec[q * M + r];
        const int code = (unpack_codes(rec[Q * M]) >> (8 * side)) & 0xFF;
        if (code >= n_codes) continue;
        const T *pr = s_pr + code * Q * NP;
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            T a = 0;
#pragma unroll
            for (int q = 0; q < Q; ++q) a += pr[q * NP + j] * F[q];
            a *= isq;
            acc[j] = side ? acc[j] + a : acc[j] - a;
        }
    }
#pragma unroll
    for (int j = 0; j < NP; ++j) dst[j] = acc[j];
}

// One SSP-RK3 stage of the compact buffered variant in one element pass
// (f64, 2D): element k's volume term (the team form, lane = variable), its
// face records projected as in compact_gather_kernel, and the stage
// combination out = a x + b (y + dt rhs) with y = U (x is not read when the
// combination has none); the right-hand side is never stored.  Whole teams
// share k, so the team exchanges of the volume term see every lane.
template <int DIM, int NP, int Q, int QV, int MS>
__global__ __launch_bounds__(256) void compact_stage_kernel(
    int64_t n_elem, int64_t n_face, const int32_t *__restrict__ elem_slots,
    const double *__restrict__ elem_geo, const double *__restrict__ tab_proj, int n_codes,
    const double *__restrict__ vb, const double *__restrict__ vd, const double *__restrict__ flux,
    const double *__restrict__ U, CombineArgs cmb) {
    constexpr int M = DIM + 2;
    constexpr int REC = M * NP;
    constexpr int TEAM = volume_team_size<DIM>();
    static_assert(TEAM >= M, "a team holds every variable");
    constexpr int RS = compact_stride<DIM, Q>();
    extern __shared__ unsigned char smem_raw[];
    double *s_pr = reinterpret_cast<double *>(smem_raw);
    for (int i = threadIdx.x; i < n_codes * Q * NP; i += blockDim.x) s_pr[i] = tab_proj[i];
    __syncthreads();
    const int r = threadIdx.x % TEAM;
    const int64_t k = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / TEAM;
    if (k >= n_elem) return;
    const bool own = r < M;
    // every read is issued before the volume term: the element's record and
    // geometry, its face slots, then (once the slots are in) its faces'
    // records, and the stage-0 state of the combination
    double c[NP];
    const double *u = U + (size_t)k * REC + r * NP;
#pragma unroll
    for (int j = 0; j < NP; ++j) c[j] = own ? u[j] : 0.0;
    double Ji[DIM * DIM];
    double sq;
    load_elem_geo<DIM, double>(k, n_elem, elem_geo, Ji, sq);
    int32_t slot[MS];
#pragma unroll
    for (int s = 0; s < MS; ++s) slot[s] = elem_slots[(int64_t)s * n_elem + k];
    double F[MS][Q];
    int code[MS];
#pragma unroll
    for (int s = 0; s < MS; ++s) {
        const bool ok = own && slot[s] >= 0 && slot[s] < 2 * n_face;
        const double *rec = flux + (size_t)(ok ? slot[s] >> 1 : 0) * RS;
#pragma unroll
        for (int q = 0; q < Q; ++q) F[s][q] = ok ? rec[q * M + r] : 0.0;
        code[s] = ok ? (unpack_codes(rec[Q * M]) >> (8 * (slot[s] & 1))) & 0xFF : 0xFF;
    }
    const size_t base = (size_t)k * REC + r * NP;
    double xs[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) xs[j] = (own && cmb.x) ? cmb.x[base + j] : c[j];
    const double isq = 1.0 / sq;
    double acc[NP];
    volume_team_core_geo<DIM, NP, QV, double>(r, Ji, sq, isq, vb, vd, c, acc);
    if (!own) return;
#pragma unroll
    for (int s = 0; s < MS; ++s) {
        if (code[s] >= n_codes) continue;
        const int side = slot[s] & 1;
        const double *pr = s_pr + code[s] * Q * NP;
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            double a = 0;
#pragma unroll
            for (int q = 0; q < Q; ++q) a += pr[q * NP + j] * F[s][q];
            a *= isq;
            acc[j] = side ? acc[j] + a : acc[j] - a;
        }
    }
#pragma unroll
    for (int j = 0; j < NP; ++j) combine_store(cmb, base + j, xs[j], c[j], acc[j]);
}

// Second pass of the buffered variant: rhs[k] += sum of element k's slots.
template <int DIM, int NP, class T>
__global__ __launch_bounds__(256) void gather_kernel(int64_t n_elem, int max_slots, int64_t n_slots_total,
                                                     const int32_t *__restrict__ elem_slots,
                                                     const T *__restrict__ buf, T *__restrict__ rhs) {
    constexpr int REC = (DIM + 2) * NP;
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_elem) return;
    T acc[REC];
    T *dst = rhs + (size_t)k * REC;
#pragma unroll
    for (int i = 0; i < REC; ++i) acc[i] = dst[i];
    for (int s = 0; s < max_slots; ++s) {
        const int32_t slot = elem_slots[(int64_t)s * n_elem + k];
        if (slot < 0 || slot >= n_slots_total) continue;
        const T *src = buf + (size_t)slot * REC;
#pragma unroll
        for (int i = 0; i < REC; ++i) acc[i] += src[i];
    }
#pragma unroll
    for (int i = 0; i < REC; ++i) dst[i] = acc[i];
}

}  // namespace dgc_dev
