// Streaming team form of the face work for large N_p x Q (tetrahedra at
// p = 2, triangles at p >= 4, parallelograms at p = 3): the same team of
// lanes per face as team_face (lane r < M owns conserved variable r), but
// the quadrature points are visited one at a time in a rolled loop: the
// lane forms its variable's trace at point q on both sides, the team
// exchanges them, every lane evaluates its own component of the flux of the
// full state and adds its projection onto all N_p modes of both sides.  Only one
// point's traces and flux are live, so the kernel keeps its registers at
// large N_p x Q, where team_face holds every point's values at once.  The
// sums run in the same order as in team_face (traces over the modes, each
// mode's projection over the points in order).
#pragma once

#include <hip/hip_runtime.h>

#include "euler_dev.hpp"
#include "surface.hpp"
#include "team.hpp"

namespace dgc_dev {

template <int DIM, int NP, int Q, int MODE, class T, class Mid = NoMid>
__device__ __forceinline__ void team_face_stream(int64_t k, int r, int64_t n_face, int64_t n_elem,
                                                 const int32_t *__restrict__ face_lr,
                                                 const uint8_t *__restrict__ face_code,
                                                 const double *__restrict__ face_geo, const T *__restrict__ s_tr,
                                                 const T *__restrict__ s_pr, int n_codes, const T *__restrict__ U,
                                                 T *__restrict__ rhs, T *__restrict__ buf, bool active = true,
                                                 const Mid &mid = Mid{}) {
    static_assert(MODE == kColored || MODE == kAtomic || MODE == kGather, "plain face modes only");
    constexpr int M = DIM + 2;
    constexpr int REC = M * NP;
    constexpr int TEAM = M <= 4 ? 4 : 8;
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

    T cL_[NP], cR_[NP], aL[NP], aR[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) cL_[j] = cR_[j] = T(0);
    if (ok && own) {
        const T *u = U + (size_t)L * REC + r * NP;
#pragma unroll
        for (int j = 0; j < NP; ++j) cL_[j] = u[j];
        if (R >= 0) {
            const T *v = U + (size_t)R * REC + r * NP;
#pragma unroll
            for (int j = 0; j < NP; ++j) cR_[j] = v[j];
        }
    }
    mid();
    if (!ok) return;
#pragma unroll
    for (int j = 0; j < NP; ++j) aL[j] = aR[j] = 0;
    const T *tl = s_tr + cL * Q * NP;
    const T *tr = s_tr + cR * Q * NP;
    const T *pl = s_pr + cL * Q * NP;
    const T *pr = s_pr + cR * Q * NP;
    T n_r = 0;
#pragma unroll
    for (int d = 0; d < DIM; ++d) n_r = r == 1 + d ? n[d] : n_r;
    const T sel_e = r == M - 1 ? T(1) : T(0);
#pragma unroll 1
    for (int q = 0; q < Q; ++q) {
        T uLq[M], uRq[M];
        T t = 0;
#pragma unroll
        for (int j = 0; j < NP; ++j) t += tl[q * NP + j] * cL_[j];
        t *= T(isL);
#pragma unroll
        for (int m = 0; m < M; ++m) uLq[m] = team_bcast<TEAM>(t, m);
        T ownR;
        if (R >= 0) {
            T s = 0;
#pragma unroll
            for (int j = 0; j < NP; ++j) s += tr[q * NP + j] * cR_[j];
            s *= T(isR);
#pragma unroll
            for (int m = 0; m < M; ++m) uRq[m] = team_bcast<TEAM>(s, m);
            ownR = s;
        } else {
            wall_ghost<DIM, T>(uLq, n, uRq);
            ownR = uRq[0];
#pragma unroll
            for (int m = 1; m < M; ++m) ownR = r == m ? uRq[m] : ownR;
        }
        const T f = rusanov_component<DIM, T>(uLq, uRq, n, t, ownR, n_r, sel_e);
#pragma unroll
        for (int j = 0; j < NP; ++j) aL[j] += pl[q * NP + j] * f;
        if (R >= 0) {
#pragma unroll
            for (int j = 0; j < NP; ++j) aR[j] += pr[q * NP + j] * f;
        }
    }
    if (!own) return;
    {
        const T sL = T(len * isL);
        T *dst = (MODE == kGather ? buf + (size_t)(2 * k) * REC : rhs + (size_t)L * REC) + r * NP;
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            const T a = aL[j] * sL;
            if (MODE == kColored) dst[j] = dst[j] - a;
            else if (MODE == kAtomic) atomic_add<T>(dst + j, -a);
            else dst[j] = -a;
        }
    }
    if (R >= 0) {
        const T sR = T(len * isR);
        T *dst = (MODE == kGather ? buf + (size_t)(2 * k + 1) * REC : rhs + (size_t)R * REC) + r * NP;
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            const T a = aR[j] * sR;
            if (MODE == kColored) dst[j] = dst[j] + a;
            else if (MODE == kAtomic) atomic_add<T>(dst + j, a);
            else dst[j] = a;
        }
    }
}

template <int DIM, int NP, int Q, int MODE, class T>
__global__ __launch_bounds__(256) void surface_stream_kernel(
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
    const int64_t k = f_begin + ((int64_t)logical_block(remap) * block + threadIdx.x) / TEAM;
    team_face_stream<DIM, NP, Q, MODE, T>(k, threadIdx.x % TEAM, n_face, n_elem, face_lr, face_code, face_geo, s_tr,
                                          s_pr, n_codes, U, rhs, buf, k < f_end,
                                          [&] { tabs.store(s_tr); });
}

}  // namespace dgc_dev
