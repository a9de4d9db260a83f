// Batched launches: many meshes of one element type and order per launch.
//
// Every work-group reads its mesh from the descriptor's block map (one
// uniform load), then does exactly the per-face / per-element / per-DOF work
// of the single-mesh kernels on that mesh's arrays.  Meshes are disjoint, so
// one launch per color stays race-free (Algorithm 1 applied to the union of
// the meshes), and a mesh's results do not depend on the other members of
// the batch.
#pragma once

#include <hip/hip_runtime.h>

#include "../batch_desc.hpp"
#include "surface.hpp"
#include "volume.hpp"
#include "volume_team.hpp"

namespace dgc_dev {

using dgc_batch::Entry;
using dgc_batch::Header;

__device__ __forceinline__ const Header *bh(const char *desc) { return reinterpret_cast<const Header *>(desc); }

__device__ __forceinline__ const Entry *bentry(const char *desc, int32_t m) {
    return reinterpret_cast<const Entry *>(desc + bh(desc)->off_entries) + m;
}

// Pointers read from the descriptor are generic pointers to the compiler.
// They all point to device global memory; casting them through the global
// address space lets it emit global (not flat) loads and stores, whose
// completion counter does not hold back LDS and scalar loads.
// (Through an integer: a direct cast pair is folded away before the
// address-space inference runs.)
template <class T>
__device__ __forceinline__ T *gptr(T *p) {
    return (T *)((__attribute__((address_space(1))) T *)(uintptr_t)p);
}

// the device arrays of one member, as global pointers
struct Member {
    const int32_t *face_lr;
    const uint8_t *face_code;
    const double *face_geo, *elem_geo;
    double *U;
    dgc_batch::RkWs w;
};

__device__ __forceinline__ Member member(const Entry *e, bool f32) {
    return Member{gptr(e->face_lr), gptr(e->face_code), gptr(e->face_geo), gptr(e->elem_geo), gptr(e->U),
                  dgc_batch::rk_ws(gptr(e->ws), (size_t)e->n_dof, f32)};
}

// stage input of the face and volume work: the state (stage 0), U1, U2; the
// f32 form always reads the f32 shadow of the current stage state
template <class T>
__device__ __forceinline__ const T *stage_input(const Member &mb, int stage);
template <>
__device__ __forceinline__ const double *stage_input<double>(const Member &mb, int stage) {
    return stage == 0 ? mb.U : (stage == 1 ? mb.w.U1 : mb.w.U2);
}
template <>
__device__ __forceinline__ const float *stage_input<float>(const Member &mb, int) {
    return mb.w.shadow;
}

// lanes per face: the mode team (lane = mode) for tetrahedra at p = 1, as the
// single-mesh default; otherwise the variable team
template <int DIM, int NP>
constexpr int batch_team() {
    return (DIM == 3 && NP == 4) ? 4 : (DIM + 2 <= 4 ? 4 : 8);
}

// One color of every mesh.  MODE kColored accumulates into the stage
// right-hand side; kVolume (first color) also evaluates the volume term and
// writes the right-hand side; kCombine (last color, f64) writes the stage
// combination instead of the right-hand side.  The fused modes need every
// member to have exactly one face of each color.
template <int DIM, int NP, int Q, int QV, int MODE, class T>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(MODE == kVolume ? f32_min_waves<T>(DIM, NP) : 1, 8)))
void batch_surface_kernel(const char *__restrict__ desc, int color, int stage) {
    constexpr int TEAM = batch_team<DIM, NP>();
    constexpr bool kMT = DIM == 3 && NP == 4;
    const Header *h = bh(desc);
    extern __shared__ unsigned char smem_raw[];
    T *s_tr = reinterpret_cast<T *>(smem_raw);
    T *s_pr = s_tr + h->n_codes * Q * NP;
    T *s_vb = s_pr + h->n_codes * Q * NP;  // mode team with the volume term: its tables follow
    T *s_vd = s_vb + QV * NP;
    const double *tables = gptr(h->tables);
    if constexpr (kMT && MODE == kVolume) {
        for (int i = threadIdx.x; i < QV * NP; i += blockDim.x) s_vb[i] = T(tables[h->off_vb + i]);
        for (int i = threadIdx.x; i < DIM * QV * NP; i += blockDim.x) s_vd[i] = T(tables[h->off_vd + i]);
    }
    stage_tables<T>(s_tr, s_pr, tables + h->off_trace, tables + h->off_proj, h->n_codes * Q * NP);
    const int32_t m = reinterpret_cast<const int32_t *>(desc + h->off_map_face[color])[blockIdx.x];
    const Entry *e = bentry(desc, m);
    const int64_t local = (int64_t)blockIdx.x - e->blk_face[color];
    const int64_t k = e->color_off[color] + (local * blockDim.x + threadIdx.x) / TEAM;
    if (k >= e->color_off[color + 1]) return;
    const Member mb = member(e, sizeof(T) == 4);
    const T *in = stage_input<T>(mb, stage);
    T *rhs = static_cast<T *>(mb.w.rhs);
    static_assert(MODE != kCombine || sizeof(T) == 8, "the fused stage combination is f64 only");
    CombineArgs cmb{};
    if constexpr (MODE == kCombine) {
        cmb.x = stage == 0 ? nullptr : mb.U;
        cmb.out = stage == 0 ? mb.w.U1 : (stage == 1 ? mb.w.U2 : mb.U);
        cmb.a = stage == 0 ? 0.0 : (stage == 1 ? 0.75 : 1.0 / 3.0);
        cmb.b = stage == 0 ? 1.0 : (stage == 1 ? 0.25 : 2.0 / 3.0);
        cmb.dt = e->dt;
    }
    if constexpr (kMT)
        mode_team_face<DIM, NP, Q, MODE, T, MODE != kVolume, QV>(k, threadIdx.x % TEAM, e->n_face, e->n_elem,
                                                                 mb.face_lr, mb.face_code, mb.face_geo, s_tr, s_pr,
                                                                 h->n_codes, in, rhs, nullptr, cmb, s_vb, s_vd,
                                                                 mb.elem_geo);
    else
        team_face<DIM, NP, Q, MODE, T, MODE != kVolume, QV>(
            k, threadIdx.x % TEAM, e->n_face, e->n_elem, mb.face_lr, mb.face_code, mb.face_geo, s_tr, s_pr,
            h->n_codes, in, rhs, nullptr, cmb, VolArgs{mb.elem_geo, tables + h->off_vb, tables + h->off_vd});
}

template <int DIM, int NP, int QV, class T>
__global__ __launch_bounds__(256) void batch_volume_kernel(const char *__restrict__ desc, int stage) {
    const Header *h = bh(desc);
    const int32_t m = reinterpret_cast<const int32_t *>(desc + h->off_map_elem)[blockIdx.x];
    const Entry *e = bentry(desc, m);
    // a team of lanes per element or one work-item per element (batch_volume_lanes)
    constexpr int LANES = batch_volume_lanes(DIM, NP, sizeof(T) == 4);
    const int64_t k = (((int64_t)blockIdx.x - e->blk_elem) * blockDim.x + threadIdx.x) / LANES;
    if (k >= e->n_elem) return;  // whole teams leave together
    const Member mb = member(e, sizeof(T) == 4);
    const double *tables = gptr(h->tables);
    if constexpr (LANES == 1)
        volume_elem<DIM, NP, QV, T>(k, e->n_elem, mb.elem_geo, tables + h->off_vb, tables + h->off_vd,
                                    stage_input<T>(mb, stage), static_cast<T *>(mb.w.rhs));
    else
        volume_team_elem<DIM, NP, QV, T>(k, threadIdx.x % LANES, e->n_elem, mb.elem_geo, tables + h->off_vb,
                                         tables + h->off_vd, stage_input<T>(mb, stage), static_cast<T *>(mb.w.rhs));
}

// SSP-RK3 stage combination of every mesh, out = a x + b (y + dt r) with the
// mesh's own dt; the f32 form also refreshes the f32 shadow (stages 0, 1).
template <class T>
__global__ __launch_bounds__(256) void batch_combine_kernel(const char *__restrict__ desc, int stage) {
    const Header *h = bh(desc);
    const int32_t m = reinterpret_cast<const int32_t *>(desc + h->off_map_dof)[blockIdx.x];
    const Entry *e = bentry(desc, m);
    const int64_t i = ((int64_t)blockIdx.x - e->blk_dof) * blockDim.x + threadIdx.x;
    if (i >= e->n_dof) return;
    const Member mb = member(e, sizeof(T) == 4);
    const double a = stage == 0 ? 0.0 : (stage == 1 ? 0.75 : 1.0 / 3.0);
    const double b = stage == 0 ? 1.0 : (stage == 1 ? 0.25 : 2.0 / 3.0);
    const double *y = stage == 0 ? mb.U : (stage == 1 ? mb.w.U1 : mb.w.U2);
    double *out = stage == 0 ? mb.w.U1 : (stage == 1 ? mb.w.U2 : mb.U);
    const double v = a * mb.U[i] + b * (y[i] + e->dt * (double)static_cast<const T *>(mb.w.rhs)[i]);
    out[i] = v;
    if (sizeof(T) == 4 && stage < 2) mb.w.shadow[i] = (float)v;
}

__global__ __launch_bounds__(256) void batch_to_f32_kernel(const char *__restrict__ desc) {
    const Header *h = bh(desc);
    const int32_t m = reinterpret_cast<const int32_t *>(desc + h->off_map_dof)[blockIdx.x];
    const Entry *e = bentry(desc, m);
    const int64_t i = ((int64_t)blockIdx.x - e->blk_dof) * blockDim.x + threadIdx.x;
    if (i >= e->n_dof) return;
    const Member mb = member(e, true);
    mb.w.shadow[i] = (float)mb.U[i];
}

}  // namespace dgc_dev
