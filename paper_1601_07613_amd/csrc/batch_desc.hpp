// Layout of a batch descriptor and of the per-mesh SSP-RK3 workspace, shared
// by the host code that writes them and the kernels that read them.
//
// A batch descriptor is one contiguous byte blob (the caller copies it to the
// device):  Header | Entry[n_mesh] | block maps.  A block map lists, for each
// work-group of a batched launch, the mesh it works on; every mesh's
// work-groups are contiguous and start at that mesh's blk_* offset.
#pragma once

#include <stddef.h>
#include <stdint.h>

namespace dgc_batch {

constexpr uint32_t kMagic = 0x44474342u;  // "DGCB"
constexpr int kMaxColors = 8;
constexpr int64_t kHeaderBytes = 512;

struct Entry {
    const int32_t *face_lr;
    const uint8_t *face_code;
    const double *face_geo;
    const double *elem_geo;
    double *U;   // f64 state
    char *ws;    // SSP-RK3 workspace of this mesh (rk_ws layout)
    double dt;
    int64_t n_face, n_elem, n_dof;
    int64_t color_off[kMaxColors + 1];
    int32_t blk_face[kMaxColors];  // first work-group of this mesh in the launch of each color
    int32_t blk_elem, blk_dof;     // first work-group in element-wise / DOF-wise launches
};

struct Header {
    uint32_t magic;
    int32_t n_mesh, n_colors, elem_type, p, n_p, n_var, n_qf, n_qv, n_codes, precision, block, faces_per_block;
    // every member has exactly one face of each color: the RK step may fuse
    // the stage combination into the last color's launch and (fuse_volume)
    // the volume term into the first color's
    int32_t fuse_combine, fuse_volume;
    int32_t nblk_face[kMaxColors];
    int32_t nblk_elem, nblk_dof;
    const double *tables;
    int64_t off_trace, off_proj, off_vb, off_vd;  // into tables, in doubles
    int64_t off_entries;
    int64_t off_map_face[kMaxColors];
    int64_t off_map_elem, off_map_dof;
    int64_t total_bytes;
};

static_assert(sizeof(Header) <= kHeaderBytes, "batch header too large");

// SSP-RK3 workspace of n DOF values: stage states U1, U2 (f64), the stage
// right-hand side (f64 or f32), and for the f32 form an f32 shadow of the
// stage state; sub-buffers start at 256-byte boundaries.
struct RkWs {
    double *U1, *U2;
    void *rhs;
    float *shadow;
    size_t bytes;  // total
};

#if defined(__HIPCC__)
#define DGC_HD __host__ __device__
#else
#define DGC_HD
#endif

DGC_HD inline size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

// byte offsets of U1, U2, rhs, shadow and the total size
DGC_HD inline void rk_ws_offsets(size_t n, int f32, size_t off[4], size_t *total) {
    off[0] = 0;
    off[1] = round256(n * 8);
    off[2] = off[1] + round256(n * 8);
    off[3] = off[2] + round256(n * (f32 ? 4 : 8));
    *total = off[3] + (f32 ? round256(n * 4) : 0);
}

DGC_HD inline RkWs rk_ws(char *base, size_t n, int f32) {
    size_t off[4], total;
    rk_ws_offsets(n, f32, off, &total);
    RkWs w;
    w.U1 = reinterpret_cast<double *>(base + off[0]);
    w.U2 = reinterpret_cast<double *>(base + off[1]);
    w.rhs = base + off[2];
    w.shadow = f32 ? reinterpret_cast<float *>(base + off[3]) : nullptr;
    w.bytes = total;
    return w;
}

}  // namespace dgc_batch
