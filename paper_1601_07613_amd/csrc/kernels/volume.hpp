// Volume term of Eq. (2), one work-item per element:
//   u(x_q)    = (1/sqrt(det J)) sum_j vb[q][j] c[m][j]
//   G_d       = sum_e (J^-1)_{de} F_e(u(x_q))          (contravariant flux)
//   rhs[m][j] = sqrt(det J) sum_q sum_d vd[d][q][j] G_d[m]   (vd carries w_q)
// The tables are read with wave-uniform addresses (scalar loads), the
// element record is read once and the result written once, so the kernel
// moves 2 records + (dim^2 + 1) geometry values per element.
// Also: the SSP-RK3 stage combination out = a x + b (y + dt r).
#pragma once

#include <hip/hip_runtime.h>

#include "euler_dev.hpp"

namespace dgc_dev {

// Unroll of the point loop of the one-work-item form: full for small
// records, rolled from 9 modes on, where a fully unrolled loop runs out of
// registers (measured on 1M-element meshes).
__host__ __device__ constexpr int valu_volume_unroll(int np, int qv) { return np >= 9 ? 1 : qv; }

template <int DIM, int NP, int QV, class T, int UNR = valu_volume_unroll(NP, QV)>
__device__ __forceinline__ void volume_elem(int64_t k, int64_t n_elem, const double *__restrict__ elem_geo,
                                            const double *__restrict__ vb, const double *__restrict__ vd,
                                            const T *__restrict__ U, T *__restrict__ rhs) {
    constexpr int M = DIM + 2;
    constexpr int REC = M * NP;
    T Ji[DIM * DIM];
#pragma unroll
    for (int a = 0; a < DIM * DIM; ++a) Ji[a] = T(elem_geo[a * n_elem + k]);
    const double sq = elem_geo[DIM * DIM * n_elem + k];
    const T isq = T(1.0 / sq);
    T c[REC];
    const T *u = U + (size_t)k * REC;
#pragma unroll
    for (int i = 0; i < REC; ++i) c[i] = u[i];
    T acc[REC];
#pragma unroll
    for (int i = 0; i < REC; ++i) acc[i] = 0;
#pragma unroll UNR
    for (int q = 0; q < QV; ++q) {
        T uq[M];
#pragma unroll
        for (int m = 0; m < M; ++m) {
            T a = 0;
#pragma unroll
            for (int j = 0; j < NP; ++j) a += T(vb[q * NP + j]) * c[m * NP + j];
            uq[m] = a * isq;
        }
        T Fx[M * DIM];
        phys_flux<DIM, T>(uq, Fx);
#pragma unroll
        for (int m = 0; m < M; ++m) {
            T G[DIM];
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
                T g = 0;
#pragma unroll
                for (int e = 0; e < DIM; ++e) g += Ji[d * DIM + e] * Fx[m * DIM + e];
                G[d] = g;
            }
#pragma unroll
            for (int j = 0; j < NP; ++j) {
                T a = 0;
#pragma unroll
                for (int d = 0; d < DIM; ++d) a += T(vd[(d * QV + q) * NP + j]) * G[d];
                acc[m * NP + j] += a;
            }
        }
    }
    T *r = rhs + (size_t)k * REC;
#pragma unroll
    for (int i = 0; i < REC; ++i) r[i] = acc[i] * T(sq);
}

template <int DIM, int NP, int QV, class T>
__global__ __launch_bounds__(256) void volume_kernel(int64_t n_elem, const double *__restrict__ elem_geo,
                                                     const double *__restrict__ vb, const double *__restrict__ vd,
                                                     const T *__restrict__ U, T *__restrict__ rhs) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n_elem) return;
    volume_elem<DIM, NP, QV, T>(k, n_elem, elem_geo, vb, vd, U, rhs);
}

// out = a * x + b * (y + dt * r), f64 accumulation of the stage state
__global__ __launch_bounds__(256) void rk_combine_kernel(int64_t n, double a, double b, double dt,
                                                         const double *__restrict__ x, const double *__restrict__ y,
                                                         const double *__restrict__ r, double *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    out[i] = a * x[i] + b * (y[i] + dt * r[i]);
}

// f32 rhs variant: the stage right-hand side is f32, the stage states f64;
// also refreshes the f32 shadow of the new stage state.
__global__ __launch_bounds__(256) void rk_combine_f32_kernel(int64_t n, double a, double b, double dt,
                                                             const double *__restrict__ x,
                                                             const double *__restrict__ y,
                                                             const float *__restrict__ r, double *__restrict__ out,
                                                             float *__restrict__ shadow) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double v = a * x[i] + b * (y[i] + dt * (double)r[i]);
    out[i] = v;
    if (shadow) shadow[i] = (float)v;
}

__global__ __launch_bounds__(256) void to_f32_kernel(int64_t n, const double *__restrict__ x, float *__restrict__ y) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    y[i] = (float)x[i];
}

}  // namespace dgc_dev
