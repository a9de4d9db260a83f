// Volume term of Eq. (2) for triangles (M = 4) with the two basis
// contractions on the matrix cores.
//
// Per element the term is two small dense products around a pointwise flux:
//   trace       u[m][q]   = (1/sqrt(det J)) sum_j c[m][j] vb[q][j]
//   flux        G[m][q,d] = sum_e (J^-1)_{de} F_e(u[.][q])
//   projection  r[m][j]   = sqrt(det J) sum_(q,d) G[m][q,d] vd[d][q][j]
// Four elements share one v_mfma_f64_16x16x4f64 chain (D[16x16] += A[16x4]
// B[4x16]): the 16 rows are (element, variable) pairs, row i = 4 m + e for
// variable m of the group's element e, so the basis tables are the B
// operands, loaded once per work-item, and the element records the A
// operands.  Operand layouts of this instruction (checked on the device):
// A[i][k] sits in lane i + 16k, B[k][j] in lane j + 16k, and D[i][j] in
// lane j + 16(i%4), register i/4.  After the trace product, lane l therefore
// holds the whole state (all four variables) of element l/16 at point
// q = l%16, so the flux needs no exchange between lanes; the fluxes go
// through LDS to the A layout of the projection.  K of the products is N_p
// and 2 N_qv, padded with zeros to multiples of 4; points q >= N_qv
// contribute zero rows.
#pragma once

#include <hip/hip_runtime.h>

#include "euler_dev.hpp"

namespace dgc_dev {

typedef double mfma_d4 __attribute__((ext_vector_type(4)));

template <int NP, int QV>
__global__ __launch_bounds__(256) void volume_mfma_kernel(int64_t n_elem, const double *__restrict__ elem_geo,
                                                          const double *__restrict__ vb,
                                                          const double *__restrict__ vd,
                                                          const double *__restrict__ U, double *__restrict__ rhs) {
    constexpr int M = 4;
    constexpr int REC = M * NP;
    constexpr int KS1 = (NP + 3) / 4;        // k-steps of the trace product
    constexpr int KS2 = (2 * QV + 3) / 4;    // k-steps of the projection
    constexpr int K2 = 4 * KS2;
    static_assert(NP <= 16 && QV <= 16, "one 16-wide tile per product");
    __shared__ double sG[4][16][K2];         // per wave: row 4 m + e, column (q, d)

    const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
    const int col = lane % 16, kq = lane / 16;

    // B operands: trace table B1[j][q] = vb[q][j], projection table B2[(q,d)][j] = vd[d][q][j]
    double b1[KS1], b2[KS2];
#pragma unroll
    for (int s = 0; s < KS1; ++s) {
        const int j = kq + 4 * s;
        b1[s] = (col < QV && j < NP) ? vb[col * NP + j] : 0.0;
    }
#pragma unroll
    for (int s = 0; s < KS2; ++s) {
        const int k = kq + 4 * s, q = k / 2, d = k % 2;
        b2[s] = (k < 2 * QV && col < NP) ? vd[(d * QV + q) * NP + col] : 0.0;
    }

    // 16 elements per work-group and iteration (4 per wave); the loop count
    // is uniform over the work-group, so the barriers below are reached by all
    const int64_t n_groups = (n_elem + 15) / 16;
    for (int64_t g = blockIdx.x; g < n_groups; g += gridDim.x) {
        const int64_t e0 = g * 16 + w * 4;

        // trace product: A[i][k] = c[e0 + i%4][i/4][k]
        mfma_d4 acc = {0.0, 0.0, 0.0, 0.0};
        {
            const int64_t ea = e0 + col % 4;
            const int m = col / 4;
#pragma unroll
            for (int s = 0; s < KS1; ++s) {
                const int j = kq + 4 * s;
                const double a = (ea < n_elem && j < NP) ? U[(size_t)ea * REC + m * NP + j] : 0.0;
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b1[s], acc, 0, 0, 0);
            }
        }

        // flux of element e0 + kq at point col
        const int64_t e = e0 + kq;
        double G[M][2];
#pragma unroll
        for (int m = 0; m < M; ++m) G[m][0] = G[m][1] = 0.0;
        double sq = 0.0;
        if (e < n_elem) sq = elem_geo[4 * n_elem + e];
        if (e < n_elem && col < QV) {
            double Ji[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) Ji[a] = elem_geo[a * n_elem + e];
            const double isq = 1.0 / sq;
            double u[M], Fx[M * 2];
#pragma unroll
            for (int m = 0; m < M; ++m) u[m] = acc[m] * isq;
            phys_flux<2, double>(u, Fx);
#pragma unroll
            for (int m = 0; m < M; ++m)
#pragma unroll
                for (int d = 0; d < 2; ++d) G[m][d] = Ji[d * 2 + 0] * Fx[m * 2 + 0] + Ji[d * 2 + 1] * Fx[m * 2 + 1];
        }
        if (2 * col < K2) {
#pragma unroll
            for (int m = 0; m < M; ++m)
#pragma unroll
                for (int d = 0; d < 2; ++d)
                    if (2 * col + d < K2) sG[w][m * 4 + kq][2 * col + d] = G[m][d];
        }
        __syncthreads();

        // projection: A[i][k] = G[element e0 + i%4, variable i/4][k]
        mfma_d4 acc2 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int s = 0; s < KS2; ++s)
            acc2 = __builtin_amdgcn_mfma_f64_16x16x4f64(sG[w][col][kq + 4 * s], b2[s], acc2, 0, 0, 0);
        __syncthreads();  // sG is rewritten by the next iteration

        // lane holds r[m][j] of element e0 + kq for m = 0..3, j = col
        if (e < n_elem && col < NP) {
            double *r = rhs + (size_t)e * REC + col;
#pragma unroll
            for (int m = 0; m < M; ++m) r[m * NP] = acc2[m] * sq;
        }
    }
}

}  // namespace dgc_dev
