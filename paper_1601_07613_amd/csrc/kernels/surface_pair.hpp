// Pair team of the face work for tetrahedra at p = 1 (N_p = 4, M = 5): four
// lanes per face; lane l owns modes 2h, 2h+1 (h = l & 1) of the variables
// g, g + 2, g + 4 (g = l >> 1; the last only for g = 0).  In the
// element-major record U[k][m][j] those two modes are one aligned 16-byte
// pair, so a record is read and written in three 16-byte instructions of a
// quad instead of the mode team's five 8-byte ones.  A trace value is the
// sum of the two half sums of the lanes (g, 0) and (g, 1) (one DPP exchange),
// and the quads' two lane pairs swap their variables (a second exchange);
// every lane evaluates the flux of the full state at each point and projects
// its variables onto its two modes.
#pragma once

#include <hip/hip_runtime.h>

#include "euler_dev.hpp"
#include "surface.hpp"
#include "team.hpp"

namespace dgc_dev {

template <class T>
struct Pair;
template <>
struct Pair<double> {
    using type = double2;
};
template <>
struct Pair<float> {
    using type = float2;
};

template <int MODE, class T, bool PREFETCH, class Mid = NoMid>
__device__ __forceinline__ void pair_team_face(int64_t k, int l, int64_t n_face, int64_t n_elem,
                                               const int32_t *__restrict__ face_lr,
                                               const uint8_t *__restrict__ face_code,
                                               const double *__restrict__ face_geo, const T *__restrict__ s_tr,
                                               const T *__restrict__ s_pr, int n_codes, const T *__restrict__ U,
                                               T *__restrict__ rhs, T *__restrict__ buf,
                                               const CombineArgs &cmb = CombineArgs{}, bool active = true,
                                               const Mid &mid = Mid{}) {
    constexpr int DIM = 3, NP = 4, Q = 3, M = 5, REC = M * NP;
    static_assert(MODE == kColored || MODE == kAtomic || MODE == kGather || MODE == kCombine,
                  "pair teams evaluate the surface term only");
    constexpr bool RMW = MODE == kColored || MODE == kCombine;
    using P = typename Pair<T>::type;
    const int h = l & 1, g = l >> 1;
    const int nv = g ? 2 : 3;  // variables owned: g, g + 2 (, g + 4)
    int32_t L = -1, R = -1;
    int cL = 0, cR = 0;
    T n[DIM] = {0, 0, 0};
    double len = 0, isL = 0, isR = 0;
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
    // pair p of a record: variable g + 2i, modes 2h, 2h + 1 (pair index 2 (g + 2i) + h)
    P cl[3], cr[3], prl[3], prr[3], xl[3], xr[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) cl[i] = cr[i] = P{T(0), T(0)};
    if (ok) {
        const P *uL = reinterpret_cast<const P *>(U + (size_t)L * REC);
        const P *uR = reinterpret_cast<const P *>(U + (size_t)R * REC);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            if (i < nv) {
                const int p = 2 * (g + 2 * i) + h;
                if (PREFETCH && RMW) prl[i] = reinterpret_cast<const P *>(rhs + (size_t)L * REC)[p];
                if constexpr (MODE == kCombine) {
                    if (cmb.x) {
                        const double *x = cmb.x + (size_t)L * REC + 2 * p;
                        xl[i] = P{T(x[0]), T(x[1])};
                    }
                }
                cl[i] = uL[p];
                if (R >= 0) {
                    if (PREFETCH && RMW) prr[i] = reinterpret_cast<const P *>(rhs + (size_t)R * REC)[p];
                    if constexpr (MODE == kCombine) {
                        if (cmb.x) {
                            const double *x = cmb.x + (size_t)R * REC + 2 * p;
                            xr[i] = P{T(x[0]), T(x[1])};
                        }
                    }
                    cr[i] = uR[p];
                }
            }
        }
    }
    mid();
    if (!ok) return;

    T aL[3][2], aR[3][2];
#pragma unroll
    for (int i = 0; i < 3; ++i) aL[i][0] = aL[i][1] = aR[i][0] = aR[i][1] = T(0);
    const bool hi = g != 0;
#pragma unroll
    for (int q = 0; q < Q; ++q) {
        T uLq[M], uRq[M];
        {
            const T t0 = s_tr[(cL * Q + q) * NP + 2 * h], t1 = s_tr[(cL * Q + q) * NP + 2 * h + 1];
            T v[3], w[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const T s = t0 * cl[i].x + t1 * cl[i].y;
                v[i] = s + quad_xor1(s);
                w[i] = quad_xor2(v[i]);
            }
            uLq[0] = (hi ? w[0] : v[0]) * T(isL);
            uLq[1] = (hi ? v[0] : w[0]) * T(isL);
            uLq[2] = (hi ? w[1] : v[1]) * T(isL);
            uLq[3] = (hi ? v[1] : w[1]) * T(isL);
            uLq[4] = (hi ? w[2] : v[2]) * T(isL);
        }
        if (R >= 0) {
            const T t0 = s_tr[(cR * Q + q) * NP + 2 * h], t1 = s_tr[(cR * Q + q) * NP + 2 * h + 1];
            T v[3], w[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                const T s = t0 * cr[i].x + t1 * cr[i].y;
                v[i] = s + quad_xor1(s);
                w[i] = quad_xor2(v[i]);
            }
            uRq[0] = (hi ? w[0] : v[0]) * T(isR);
            uRq[1] = (hi ? v[0] : w[0]) * T(isR);
            uRq[2] = (hi ? w[1] : v[1]) * T(isR);
            uRq[3] = (hi ? v[1] : w[1]) * T(isR);
            uRq[4] = (hi ? w[2] : v[2]) * T(isR);
        } else {
            wall_ghost<DIM, T>(uLq, n, uRq);
        }
        T F[M];
        rusanov<DIM, T>(uLq, uRq, n, F);
        const T Fi[3] = {hi ? F[1] : F[0], hi ? F[3] : F[2], F[4]};
        const T p0 = s_pr[(cL * Q + q) * NP + 2 * h], p1 = s_pr[(cL * Q + q) * NP + 2 * h + 1];
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            aL[i][0] += p0 * Fi[i];
            aL[i][1] += p1 * Fi[i];
        }
        if (R >= 0) {
            const T r0 = s_pr[(cR * Q + q) * NP + 2 * h], r1 = s_pr[(cR * Q + q) * NP + 2 * h + 1];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                aR[i][0] += r0 * Fi[i];
                aR[i][1] += r1 * Fi[i];
            }
        }
    }
    const T sL = T(len * isL), sR = T(len * isR);
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        if (i >= nv) continue;
        const int p = 2 * (g + 2 * i) + h;
        const T a0 = aL[i][0] * sL, a1 = aL[i][1] * sL;
        if (MODE == kColored) {
            P *dst = reinterpret_cast<P *>(rhs + (size_t)L * REC) + p;
            const P old = PREFETCH ? prl[i] : *dst;
            *dst = P{old.x - a0, old.y - a1};
        } else if (MODE == kCombine) {
            const P old = PREFETCH ? prl[i] : reinterpret_cast<const P *>(rhs + (size_t)L * REC)[p];
            const size_t idx = (size_t)L * REC + 2 * p;
            combine_store(cmb, idx, cmb.x ? xl[i].x : cl[i].x, cl[i].x, old.x - a0);
            combine_store(cmb, idx + 1, cmb.x ? xl[i].y : cl[i].y, cl[i].y, old.y - a1);
        } else if (MODE == kAtomic) {
            T *dst = rhs + (size_t)L * REC + 2 * p;
            atomic_add<T>(dst, -a0);
            atomic_add<T>(dst + 1, -a1);
        } else {
            reinterpret_cast<P *>(buf + (size_t)(2 * k) * REC)[p] = P{-a0, -a1};
        }
        if (R >= 0) {
            const T b0 = aR[i][0] * sR, b1 = aR[i][1] * sR;
            if (MODE == kColored) {
                P *dst = reinterpret_cast<P *>(rhs + (size_t)R * REC) + p;
                const P old = PREFETCH ? prr[i] : *dst;
                *dst = P{old.x + b0, old.y + b1};
            } else if (MODE == kCombine) {
                const P old = PREFETCH ? prr[i] : reinterpret_cast<const P *>(rhs + (size_t)R * REC)[p];
                const size_t idx = (size_t)R * REC + 2 * p;
                combine_store(cmb, idx, cmb.x ? xr[i].x : cr[i].x, cr[i].x, old.x + b0);
                combine_store(cmb, idx + 1, cmb.x ? xr[i].y : cr[i].y, cr[i].y, old.y + b1);
            } else if (MODE == kAtomic) {
                T *dst = rhs + (size_t)R * REC + 2 * p;
                atomic_add<T>(dst, b0);
                atomic_add<T>(dst + 1, b1);
            } else {
                reinterpret_cast<P *>(buf + (size_t)(2 * k + 1) * REC)[p] = P{b0, b1};
            }
        }
    }
}

template <int MODE, class T>
__global__ __launch_bounds__(256) void surface_pair_team_kernel(
    int64_t f_begin, int64_t f_end, int64_t n_face, int64_t n_elem,
    const int32_t *__restrict__ face_lr, const uint8_t *__restrict__ face_code,
    const double *__restrict__ face_geo, const double *__restrict__ tab_trace,
    const double *__restrict__ tab_proj, int n_codes,
    const T *__restrict__ U, T *__restrict__ rhs, T *__restrict__ buf, int remap, int block) {
    extern __shared__ unsigned char smem_raw[];
    T *s_tr = reinterpret_cast<T *>(smem_raw);
    T *s_pr = s_tr + n_codes * 3 * 4;
    TableStage<T> tabs;
    tabs.issue(s_tr, tab_trace, tab_proj, n_codes * 3 * 4, block);
    const int64_t k = f_begin + ((int64_t)logical_block(remap) * block + threadIdx.x) / 4;
    pair_team_face<MODE, T, true>(k, threadIdx.x % 4, n_face, n_elem, face_lr, face_code, face_geo, s_tr, s_pr,
                                  n_codes, U, rhs, buf, CombineArgs{}, k < f_end,
                                  [&] { tabs.store(s_tr); });
}

}  // namespace dgc_dev
