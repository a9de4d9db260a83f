// Device helpers of the layout and of the refinement map.
//
// permute_records: gather / scatter of element records between the caller's
// element order and the layout order of Section 5 (one work-item per 4-byte
// word of a record).
// child_colors: the closed-form coloring of a 4-way split (Section 3.2):
// the first / second child of a parent edge of color c get c / (c + 3) mod 6
// and each interior edge the color of the parallel parent edge; one
// work-item per split element.
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

}  // namespace dgc_dev
