// Device helpers of the layout and of the refinement map.
//
// permute_records: gather / scatter of element records between the caller's
// element order and the layout order of Section 5 (one work-item per 4-byte
// word of a record).
// child_colors: the closed-form coloring of a 4-way split (Section 3.2):
// the first / second child of a parent edge of color c get c / (c + 3) mod 6
// and each interior edge the color of the parallel parent edge; one
// work-item per split element.
// adapt_transfer: the solution on a refined / coarsened mesh by L2
// projection (copy for an unchanged leaf, P_k c for child k, sum_k P_k^T c_k
// for a merged parent); one work-item per (new element, variable).
#pragma once

#include <hip/hip_runtime.h>

namespace dgc_dev {

__global__ __launch_bounds__(256) void permute_records_kernel(const uint32_t *__restrict__ src,
                                                              uint32_t *__restrict__ dst,
                                                              const int32_t *__restrict__ perm, int64_t n_rec,
                                                              int64_t words, int to_layout) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n_rec * words) return;
    const int64_t i = t / words, w = t % words;
    const int64_t j = perm[i];
    if (j < 0 || j >= n_rec) return;
    if (to_layout)
        dst[j * words + w] = src[i * words + w];
    else
        dst[i * words + w] = src[j * words + w];
}

__global__ __launch_bounds__(256) void child_colors_kernel(const int8_t *__restrict__ parent, int64_t n,
                                                           int8_t *__restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    for (int k = 0; k < 3; ++k) {
        const int c = parent[3 * i + k];
        out[9 * i + 2 * k] = (int8_t)c;
        out[9 * i + 2 * k + 1] = (int8_t)((c + 3) % 6);
        out[9 * i + 6 + k] = (int8_t)c;
    }
}

template <int NP>
__global__ __launch_bounds__(256) void adapt_transfer_kernel(int64_t n_new, int n_var, int64_t n_old,
                                                             const int8_t *__restrict__ kind,
                                                             const int32_t *__restrict__ src,
                                                             const double *__restrict__ P,
                                                             const double *__restrict__ Uold,
                                                             double *__restrict__ Unew) {
    __shared__ double sP[4 * NP * NP];
    for (int t = threadIdx.x; t < 4 * NP * NP; t += blockDim.x) sP[t] = P[t];
    __syncthreads();
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n_new * n_var) return;
    const int64_t i = g / n_var;
    const int m = (int)(g % n_var);
    const int kd = kind[i];
    // source record of variable m, or null when the id is out of range
    auto rec = [&](int a) -> const double * {
        const int32_t s = src[a * n_new + i];
        return (s >= 0 && s < n_old) ? Uold + ((int64_t)s * n_var + m) * NP : nullptr;
    };
    double out[NP];
    bool ok = true;
    if (kd == 0) {
        const double *u = rec(0);
        ok = u != nullptr;
        for (int j = 0; j < NP; ++j) out[j] = ok ? u[j] : 0.0;
    } else if (kd >= 1 && kd <= 4) {
        const double *u = rec(0);
        ok = u != nullptr;
        const double *Pk = sP + (kd - 1) * NP * NP;
        for (int j = 0; j < NP; ++j) {
            double a = 0.0;
            if (ok)
                for (int l = 0; l < NP; ++l) a += Pk[j * NP + l] * u[l];
            out[j] = a;
        }
    } else if (kd == 5) {
        for (int l = 0; l < NP; ++l) out[l] = 0.0;
        for (int k = 0; k < 4 && ok; ++k) {
            const double *u = rec(k);
            ok = u != nullptr;
            if (!ok) break;
            const double *Pk = sP + k * NP * NP;
            for (int j = 0; j < NP; ++j) {
                const double uj = u[j];
                for (int l = 0; l < NP; ++l) out[l] += Pk[j * NP + l] * uj;
            }
        }
    } else {
        ok = false;
    }
    double *o = Unew + (i * n_var + m) * NP;
    for (int j = 0; j < NP; ++j) o[j] = ok ? out[j] : __builtin_nan("");
}

}  // namespace dgc_dev
