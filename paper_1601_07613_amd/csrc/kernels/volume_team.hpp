// Volume term of Eq. (2), team form: TEAM lanes per element (4 for M = 4,
// 8 for M = 5), lane r < M owning conserved variable r.
//
// Lane r reads the N_p modes of its variable (the team reads the element
// record as one contiguous stretch), forms its variable's value at every
// volume point, and the team exchanges the values (DPP quad broadcasts, or
// ds_bpermute for 8-lane teams) so that every lane holds the full state.
// Every lane evaluates the flux of the full state and keeps its own
// component; the contravariant flux and the projection onto the modes are
// then lane-local, and lane r writes its variable's N_p modes of the result.
// Same arithmetic as volume_elem, in the same order.
#pragma once

#include <hip/hip_runtime.h>

#include "euler_dev.hpp"
#include "surface.hpp"

namespace dgc_dev {

template <int DIM>
constexpr int volume_team_size() {
    return DIM + 2 <= 4 ? 4 : 8;
}

// Lanes per element of the batched volume term: the team form where it is
// the faster vector form, one work-item per element where that is faster
// (tetrahedra; 2D with 9, 10 or 15 modes: quadrilaterals at p = 2, triangles
// at p = 3, 4; measured on 1M-element meshes).  Host and device share this rule.
__host__ __device__ constexpr int batch_volume_lanes(int dim, int np) {
    return (dim == 3 || np == 9 || np == 10 || np == 15) ? 1 : 4;
}

// element k, lane r of its team (all lanes of the team must call); the
// tables may live in global memory (f64) or in LDS
template <int DIM, int NP, int QV, class T, class TAB = double>
__device__ __forceinline__ void volume_team_elem(int64_t k, int r, int64_t n_elem,
                                                 const double *__restrict__ elem_geo, const TAB *__restrict__ vb,
                                                 const TAB *__restrict__ vd, const T *__restrict__ U,
                                                 T *__restrict__ rhs) {
    constexpr int M = DIM + 2;
    constexpr int REC = M * NP;
    constexpr int TEAM = volume_team_size<DIM>();
    const bool own = r < M;
    T Ji[DIM * DIM];
#pragma unroll
    for (int a = 0; a < DIM * DIM; ++a) Ji[a] = T(elem_geo[a * n_elem + k]);
    const double sq = elem_geo[DIM * DIM * n_elem + k];
    const T isq = T(1.0 / sq);
    T c[NP];
    const T *u = U + (size_t)k * REC + r * NP;
#pragma unroll
    for (int j = 0; j < NP; ++j) c[j] = own ? u[j] : T(0);
    T acc[NP];
#pragma unroll
    for (int j = 0; j < NP; ++j) acc[j] = 0;
#pragma unroll
    for (int q = 0; q < QV; ++q) {
        T t = 0;
#pragma unroll
        for (int j = 0; j < NP; ++j) t += T(vb[q * NP + j]) * c[j];
        T uq[M];
#pragma unroll
        for (int m = 0; m < M; ++m) uq[m] = team_bcast<TEAM>(t * isq, m);
        T Fx[M * DIM];
        phys_flux<DIM, T>(uq, Fx);
        T Fm[DIM];
#pragma unroll
        for (int e = 0; e < DIM; ++e) {
            T f = Fx[e];
#pragma unroll
            for (int m = 1; m < M; ++m) f = r == m ? Fx[m * DIM + e] : f;
            Fm[e] = f;
        }
        T G[DIM];
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            T g = 0;
#pragma unroll
            for (int e = 0; e < DIM; ++e) g += Ji[d * DIM + e] * Fm[e];
            G[d] = g;
        }
#pragma unroll
        for (int j = 0; j < NP; ++j) {
            T a = 0;
#pragma unroll
            for (int d = 0; d < DIM; ++d) a += T(vd[(d * QV + q) * NP + j]) * G[d];
            acc[j] += a;
        }
    }
    if (!own) return;
    T *o = rhs + (size_t)k * REC + r * NP;
#pragma unroll
    for (int j = 0; j < NP; ++j) o[j] = acc[j] * T(sq);
}

template <int DIM, int NP, int QV, class T>
__global__ __launch_bounds__(256) void volume_team_kernel(int64_t n_elem, const double *__restrict__ elem_geo,
                                                          const double *__restrict__ vb,
                                                          const double *__restrict__ vd,
                                                          const T *__restrict__ U, T *__restrict__ rhs) {
    constexpr int TEAM = volume_team_size<DIM>();
    const int64_t k = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / TEAM;
    if (k >= n_elem) return;  // whole teams leave together
    volume_team_elem<DIM, NP, QV, T>(k, threadIdx.x % TEAM, n_elem, elem_geo, vb, vd, U, rhs);
}

// Mixed triangle / quadrilateral meshes (2D, N_p = (p+1)^2 slots per
// element): both kinds' volume tables are staged in LDS and each team picks
// its element's block; a triangle's tables are zero beyond its own modes.
template <int NP, int QV, class T>
__global__ __launch_bounds__(256) void volume_team_mixed_kernel(int64_t n_elem, const int8_t *__restrict__ elem_kind,
                                                                const double *__restrict__ elem_geo,
                                                                const double *__restrict__ vb2,
                                                                const double *__restrict__ vd2,
                                                                const T *__restrict__ U, T *__restrict__ rhs) {
    constexpr int TEAM = volume_team_size<2>();
    __shared__ T s_vb[2 * QV * NP];          // [kind][q][j]
    __shared__ T s_vd[2 * 2 * QV * NP];      // [kind][d][q][j]
    for (int i = threadIdx.x; i < 2 * QV * NP; i += blockDim.x) s_vb[i] = T(vb2[i]);
    for (int i = threadIdx.x; i < 4 * QV * NP; i += blockDim.x) s_vd[i] = T(vd2[i]);
    __syncthreads();
    const int64_t k = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / TEAM;
    if (k >= n_elem) return;  // whole teams leave together
    const int kind = elem_kind[k] ? 1 : 0;
    volume_team_elem<2, NP, QV, T, T>(k, threadIdx.x % TEAM, n_elem, elem_geo, s_vb + kind * QV * NP,
                                      s_vd + kind * 2 * QV * NP, U, rhs);
}

}  // namespace dgc_dev
