// Device entry points of the C ABI: argument checks, template dispatch on
// (element type, order, precision) and launches on the caller's stream.
#include <hip/hip_runtime.h>

#include <string>
#include <type_traits>

#include <cmath>
#include <cstring>
#include <mutex>

#include "../batch_desc.hpp"
#include "../host/internal.hpp"
#include "batch.hpp"
#include "layout_dev.hpp"
#include "surface.hpp"
#include "surface_pair.hpp"
#include "surface_stream.hpp"
#include "volume.hpp"
#include "volume_mfma.hpp"
#include "volume_team.hpp"
#include "rk_block.hpp"

using dgc::fail;

namespace {

constexpr int kBlock = 256;

// DGC_FORM_DEFAULT: the face-kernel form measured fastest for each element
// type, order, precision and size (colored pass): the right-hand-side
// prefetch pays only where the launches are large and the records small
// (f64 triangles at p = 1, at p = 2 from 1M faces on; f32 triangles at
// p = 3, 4; parallelograms at p = 2); the streaming team where N_p x Q is
// large (tetrahedra at p = 2, f64 triangles from p = 3 on, f32 triangles at
// p = 5, f64 parallelograms at p = 3: 9-35 % faster than the other forms);
// otherwise the team without prefetch.  Tetrahedra at p = 1: the mode team.
int default_surface_form(int elem_type, int p, bool f32, int64_t n_face) {
    if (elem_type == DGC_TET) {
        if (p == 1) return DGC_FORM_MODE_TEAM;
        if (p == 2) return DGC_FORM_TEAM_STREAM;
        return DGC_FORM_TEAM_PREFETCH;
    }
    if (elem_type == DGC_QUAD || elem_type == DGC_MIXED) {
        if (p == 3) return f32 ? DGC_FORM_TEAM : DGC_FORM_TEAM_STREAM;
        return p == 1 ? DGC_FORM_TEAM : DGC_FORM_TEAM_PREFETCH;
    }
    if (f32) return p >= 5 ? DGC_FORM_TEAM_STREAM : (p >= 3 ? DGC_FORM_TEAM_PREFETCH : DGC_FORM_TEAM);
    if (p <= 1) return DGC_FORM_TEAM_PREFETCH;
    if (p == 2) return n_face >= 1000000 ? DGC_FORM_TEAM_PREFETCH : DGC_FORM_TEAM;
    return DGC_FORM_TEAM_STREAM;
}

int resolved_surface_form(const dgc_dmesh *dm, bool f32) {
    return dm->surf_form == DGC_FORM_DEFAULT ? default_surface_form(dm->elem_type, dm->p, f32, dm->n_face)
                                             : dm->surf_form;
}

// DGC_VOL_DEFAULT: the volume form measured fastest for each element type,
// order and precision (~1M elements; mixed meshes always use their own team
// kernel): in f64 the team (one work-item per element for triangles at
// p = 3), in f32 one work-item per element (the team for quadrilaterals at
// p <= 2), and one work-item per element for tetrahedra, where the 8-lane
// team (5 variables) is 2-9x slower.  The matrix-core form is slower at
// every order measured (its 16 x 16 x 4 tiles are mostly padding).
int default_volume_form(int elem_type, int p, bool f32) {
    if (elem_type == DGC_TET) return DGC_VOL_VALU;
    if (f32) return (elem_type == DGC_QUAD && p <= 2) ? DGC_VOL_TEAM : DGC_VOL_VALU;
    return (elem_type == DGC_TRI && p == 3) ? DGC_VOL_VALU : DGC_VOL_TEAM;
}

// DGC_RK_DEFAULT fuses the volume term into the first color's face kernel
// where the face team carries it without slowing the step down (measured on
// ~1M-element meshes; tetrahedra at p = 1 in f64 only, the f32 form gains
// nothing there; parallelograms at p = 3 in f32 only)
bool default_fuse_volume(int elem_type, int p, bool f32) {
    if (elem_type == DGC_TET) return p == 1 && !f32;
    if (elem_type == DGC_QUAD) return p <= 2 || f32;  // f64 p = 3: the streaming colors win
    return elem_type == DGC_TRI && p <= 3;
}

inline unsigned grid_for(int64_t n, int block = kBlock) { return (unsigned)((n + block - 1) / block); }

dgc_status hip_check(const char *what) {
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(DGC_E_HIP, std::string(what) + ": " + hipGetErrorString(e));
    return DGC_OK;
}

// Validate the device view against the tables the library would build.
dgc_status check_dm(const dgc_dmesh *dm, dgc_table_info *ti) {
    if (!dm) return fail(DGC_E_ARG, "null dgc_dmesh");
    dgc_status s = dgc::build_tables(dm->elem_type, dm->p, ti, nullptr);
    if (s != DGC_OK) return s;
    if (dm->n_p != ti->n_p || dm->n_qf != ti->n_qf || dm->n_qv != ti->n_qv || dm->n_codes != ti->n_codes ||
        dm->n_orient != ti->n_orient || dm->n_var != ti->dim + 2)
        return fail(DGC_E_ARG, "dgc_dmesh sizes do not match the tables of (elem_type, p)");
    if (dm->n_elem <= 0 || dm->n_face <= 0 || dm->n_elem > ((int64_t)1 << 31) - 1 ||
        dm->n_face > ((int64_t)1 << 31) - 1)
        return fail(DGC_E_ARG, "dgc_dmesh: bad element / face count");
    if (!dm->face_lr || !dm->face_code || !dm->face_geo || !dm->elem_geo || !dm->tables)
        return fail(DGC_E_ARG, "dgc_dmesh: null device array");
    if (dm->surf_form < DGC_FORM_DEFAULT || dm->surf_form > DGC_FORM_PAIR_TEAM)
        return fail(DGC_E_ARG, "dgc_dmesh: unknown surf_form");
    if (dm->elem_type == DGC_MIXED && !dm->elem_kind)
        return fail(DGC_E_ARG, "dgc_dmesh: a mixed mesh needs elem_kind");
    if (dm->vol_form < DGC_VOL_DEFAULT || dm->vol_form > DGC_VOL_TEAM)
        return fail(DGC_E_ARG, "dgc_dmesh: unknown vol_form");
    if (dm->block_size != 0 && dm->block_size != 64 && dm->block_size != 128 && dm->block_size != 256)
        return fail(DGC_E_ARG, "dgc_dmesh: block_size must be 0, 64, 128 or 256");
    return DGC_OK;
}

dgc_status check_colors(const dgc_dmesh *dm) {
    if (dm->n_colors <= 0 || dm->n_colors > DGC_MAX_COLORS) return fail(DGC_E_NOT_COLORED, "dgc_dmesh has no colors");
    if (dm->color_off[0] != 0 || dm->color_off[dm->n_colors] != dm->n_face)
        return fail(DGC_E_ARG, "dgc_dmesh: color offsets do not cover the faces");
    for (int c = 0; c < dm->n_colors; ++c)
        if (dm->color_off[c + 1] < dm->color_off[c]) return fail(DGC_E_ARG, "dgc_dmesh: decreasing color offsets");
    return DGC_OK;
}

template <int DIM, int NP, int Q, int QV, class T>
struct Impl {
    static constexpr int REC = (DIM + 2) * NP;
    static constexpr int kDim = DIM, kNp = NP, kQ = Q, kQv = QV;
    using Real = T;

    static dgc_status volume(const dgc_dmesh *dm, const dgc_table_info &ti, const T *U, T *rhs, hipStream_t st) {
        if constexpr (DIM == 2) {
            if (dm->elem_type == DGC_MIXED) {
                // per-element kind: the team form with both kinds' tables in LDS
                hipLaunchKernelGGL((dgc_dev::volume_team_mixed_kernel<NP, QV, T>),
                                   dim3(grid_for(dm->n_elem * dgc_dev::volume_team_size<2>())), dim3(kBlock), 0, st,
                                   dm->n_elem, dm->elem_kind, dm->elem_geo, dm->tables + ti.off_vb,
                                   dm->tables + ti.off_vd, U, rhs);
                return hip_check("volume kernel launch");
            }
        }
        const int vf = dm->vol_form == DGC_VOL_DEFAULT ? default_volume_form(dm->elem_type, dm->p, sizeof(T) == 4)
                                                       : dm->vol_form;
        if constexpr (DIM == 2 && std::is_same_v<T, double> && NP <= 16 && QV <= 16) {
            if (vf == DGC_VOL_MFMA) {
                const int64_t groups = (dm->n_elem + 15) / 16;
                const unsigned grid = (unsigned)(groups < 4096 ? groups : 4096);
                hipLaunchKernelGGL((dgc_dev::volume_mfma_kernel<NP, QV>), dim3(grid), dim3(256), 0, st, dm->n_elem,
                                   dm->elem_geo, dm->tables + ti.off_vb, dm->tables + ti.off_vd, U, rhs);
                return hip_check("volume kernel launch");
            }
        }
        if (vf == DGC_VOL_TEAM) {
            constexpr int TEAM = DIM + 2 <= 4 ? 4 : 8;
            hipLaunchKernelGGL((dgc_dev::volume_team_kernel<DIM, NP, QV, T>), dim3(grid_for(dm->n_elem * TEAM)),
                               dim3(kBlock), 0, st, dm->n_elem, dm->elem_geo, dm->tables + ti.off_vb,
                               dm->tables + ti.off_vd, U, rhs);
            return hip_check("volume kernel launch");
        }
        hipLaunchKernelGGL((dgc_dev::volume_kernel<DIM, NP, QV, T>), dim3(grid_for(dm->n_elem)), dim3(kBlock), 0, st,
                           dm->n_elem, dm->elem_geo, dm->tables + ti.off_vb, dm->tables + ti.off_vd, U, rhs);
        return hip_check("volume kernel launch");
    }

    template <int MODE>
    static dgc_status faces(const dgc_dmesh *dm, const dgc_table_info &ti, int64_t f0, int64_t f1, const T *U, T *rhs,
                            T *buf, hipStream_t st) {
        if (f1 <= f0) return DGC_OK;
        const size_t lds = 2 * (size_t)ti.n_codes * Q * NP * sizeof(T);
        const int block = dm->block_size ? dm->block_size : kBlock;
        const int form = resolved_surface_form(dm, sizeof(T) == 4);
        if constexpr (NP == 4 && DIM == 3) {
            // tetrahedra at p = 1: the mode team (4 lanes, lane = mode)
            if (form == DGC_FORM_MODE_TEAM) {
                hipLaunchKernelGGL((dgc_dev::surface_mode_team_kernel<DIM, NP, Q, MODE, T>),
                                   dim3(grid_for((f1 - f0) * 4, block)), dim3(block), lds, st, f0, f1, dm->n_face,
                                   dm->n_elem, dm->face_lr, dm->face_code, dm->face_geo, dm->tables + ti.off_trace,
                                   dm->tables + ti.off_proj, ti.n_codes, U, rhs, buf, dm->xcd_remap, block);
                return hip_check("surface kernel launch");
            }
        }
        if constexpr (NP == 4 && DIM == 3 && Q == 3) {
            // tetrahedra at p = 1: the pair team (4 lanes, 16-byte record pieces)
            if (form == DGC_FORM_PAIR_TEAM) {
                hipLaunchKernelGGL((dgc_dev::surface_pair_team_kernel<MODE, T>),
                                   dim3(grid_for((f1 - f0) * 4, block)), dim3(block), lds, st, f0, f1, dm->n_face,
                                   dm->n_elem, dm->face_lr, dm->face_code, dm->face_geo, dm->tables + ti.off_trace,
                                   dm->tables + ti.off_proj, ti.n_codes, U, rhs, buf, dm->xcd_remap, block);
                return hip_check("surface kernel launch");
            }
        }
        if (form == DGC_FORM_MODE_TEAM || form == DGC_FORM_PAIR_TEAM)
            return fail(DGC_E_UNSUPPORTED, "mode and pair teams need N_p = 4 in 3D");
        if (form == DGC_FORM_TEAM_STREAM) {
            constexpr int TEAM = DIM + 2 <= 4 ? 4 : 8;
            hipLaunchKernelGGL((dgc_dev::surface_stream_kernel<DIM, NP, Q, MODE, T>),
                               dim3(grid_for((f1 - f0) * TEAM, block)), dim3(block), lds, st, f0, f1, dm->n_face,
                               dm->n_elem, dm->face_lr, dm->face_code, dm->face_geo, dm->tables + ti.off_trace,
                               dm->tables + ti.off_proj, ti.n_codes, U, rhs, buf, dm->xcd_remap, block);
            return hip_check("surface kernel launch");
        }
        if (form == DGC_FORM_THREAD) {
            hipLaunchKernelGGL((dgc_dev::surface_kernel<DIM, NP, Q, MODE, T>), dim3(grid_for(f1 - f0, block)),
                               dim3(block), lds, st, f0, f1, dm->n_face, dm->n_elem, dm->face_lr, dm->face_code,
                               dm->face_geo, dm->tables + ti.off_trace, dm->tables + ti.off_proj, ti.n_codes, U, rhs,
                               buf, dm->xcd_remap);
        } else {
            constexpr int TEAM = DIM + 2 <= 4 ? 4 : 8;
            if (form == DGC_FORM_TEAM_PREFETCH)
                hipLaunchKernelGGL((dgc_dev::surface_team_kernel<DIM, NP, Q, MODE, T, true>),
                                   dim3(grid_for((f1 - f0) * TEAM, block)), dim3(block), lds, st, f0, f1, dm->n_face,
                                   dm->n_elem, dm->face_lr, dm->face_code, dm->face_geo, dm->tables + ti.off_trace,
                                   dm->tables + ti.off_proj, ti.n_codes, U, rhs, buf, dm->xcd_remap, block);
            else
                hipLaunchKernelGGL((dgc_dev::surface_team_kernel<DIM, NP, Q, MODE, T, false>),
                                   dim3(grid_for((f1 - f0) * TEAM, block)), dim3(block), lds, st, f0, f1, dm->n_face,
                                   dm->n_elem, dm->face_lr, dm->face_code, dm->face_geo, dm->tables + ti.off_trace,
                                   dm->tables + ti.off_proj, ti.n_codes, U, rhs, buf, dm->xcd_remap, block);
        }
        return hip_check("surface kernel launch");
    }

    // the whole SSP-RK3 step in one work-group (f64, colored)
    static dgc_status rk_block(const dgc_dmesh *dm, const dgc_table_info &ti, double *U, double *U1, double *U2,
                               double *rhs, double dt, hipStream_t st) {
        dgc_status s = check_colors(dm);
        if (s != DGC_OK) return s;
        dgc_dev::BlockRkArgs a{};
        for (int c = 0; c <= dm->n_colors; ++c) a.color_off[c] = dm->color_off[c];
        a.n_colors = dm->n_colors;
        a.dt = dt;
        const size_t lds = 2 * (size_t)ti.n_codes * Q * NP * sizeof(double);
        hipLaunchKernelGGL((dgc_dev::rk_step_block_kernel<DIM, NP, Q, QV>), dim3(1), dim3(512), lds, st, dm->n_face,
                           dm->n_elem, dm->face_lr, dm->face_code, dm->face_geo, dm->elem_geo,
                           dm->tables + ti.off_trace, dm->tables + ti.off_proj, ti.n_codes, dm->tables + ti.off_vb,
                           dm->tables + ti.off_vd, U, U1, U2, rhs, a);
        return hip_check("single-work-group RK step launch");
    }

    // first color of a stage with the volume term fused in: rhs = volume +
    // first-color surface term, for every element (see DGC_RK_FUSED_VOLUME)
    static dgc_status faces_volume(const dgc_dmesh *dm, const dgc_table_info &ti, int64_t f0, int64_t f1, const T *U,
                                   T *rhs, hipStream_t st) {
        const int block = dm->block_size ? dm->block_size : kBlock;
        const int form = resolved_surface_form(dm, sizeof(T) == 4);
        const dgc_dev::VolArgs va{dm->elem_geo, dm->tables + ti.off_vb, dm->tables + ti.off_vd};
        const size_t lds = 2 * (size_t)ti.n_codes * Q * NP * sizeof(T);
        if constexpr (NP == 4 && DIM == 3) {
            if (form == DGC_FORM_MODE_TEAM) {
                const size_t lds_v = lds + (size_t)(1 + DIM) * QV * NP * sizeof(T);
                hipLaunchKernelGGL((dgc_dev::surface_volume_kernel<DIM, NP, Q, QV, true, T>),
                                   dim3(grid_for((f1 - f0) * 4, block)), dim3(block), lds_v, st, f0, f1, dm->n_face,
                                   dm->n_elem, dm->face_lr, dm->face_code, dm->face_geo, dm->tables + ti.off_trace,
                                   dm->tables + ti.off_proj, ti.n_codes, U, rhs, va, dm->xcd_remap, block);
                return hip_check("fused volume and surface kernel launch");
            }
        }
        if (form != DGC_FORM_TEAM && form != DGC_FORM_TEAM_PREFETCH && form != DGC_FORM_TEAM_STREAM)
            return fail(DGC_E_UNSUPPORTED, "the fused volume term needs a team face form");
        constexpr int TEAM = DIM + 2 <= 4 ? 4 : 8;
        hipLaunchKernelGGL((dgc_dev::surface_volume_kernel<DIM, NP, Q, QV, false, T>),
                           dim3(grid_for((f1 - f0) * TEAM, block)), dim3(block), lds, st, f0, f1, dm->n_face,
                           dm->n_elem, dm->face_lr, dm->face_code, dm->face_geo, dm->tables + ti.off_trace,
                           dm->tables + ti.off_proj, ti.n_codes, U, rhs, va, dm->xcd_remap, block);
        return hip_check("fused volume and surface kernel launch");
    }

    // colors [c0, c1) of a colored pass
    static dgc_status colors(const dgc_dmesh *dm, const dgc_table_info &ti, int c0, int c1, const T *U, T *rhs,
                             hipStream_t st) {
        dgc_status s = DGC_OK;
        for (int c = c0; c < c1 && s == DGC_OK; ++c)
            s = faces<dgc_dev::kColored>(dm, ti, dm->color_off[c], dm->color_off[c + 1], U, rhs, nullptr, st);
        return s;
    }

    // colored pass (from first_color on) whose last color writes the stage
    // combination (f64); *fused is false (and nothing is launched) when the
    // last color is empty
    static dgc_status surface_fused(const dgc_dmesh *dm, const dgc_table_info &ti, const T *U, T *rhs,
                                    const dgc_dev::CombineArgs &cmb, int first_color, bool *fused, hipStream_t st) {
        *fused = false;
        if constexpr (!std::is_same_v<T, double>) {
            return fail(DGC_E_ARG, "fused stage combination is f64 only");
        } else {
            dgc_status s = check_colors(dm);
            if (s != DGC_OK) return s;
            const int nc = dm->n_colors;
            const int64_t f0 = dm->color_off[nc - 1], f1 = dm->color_off[nc];
            if (f1 <= f0 || first_color > nc - 1) return DGC_OK;
            if ((s = colors(dm, ti, first_color, nc - 1, U, rhs, st)) != DGC_OK) return s;
            const size_t lds = 2 * (size_t)ti.n_codes * Q * NP * sizeof(double);
            const int block = dm->block_size ? dm->block_size : kBlock;
            constexpr bool kMT = DIM == 3 && NP == 4;
            if (kMT && resolved_surface_form(dm, false) == DGC_FORM_MODE_TEAM) {
                hipLaunchKernelGGL((dgc_dev::surface_combine_kernel<DIM, NP, Q, kMT>),
                                   dim3(grid_for((f1 - f0) * 4, block)), dim3(block), lds, st, f0, f1, dm->n_face,
                                   dm->n_elem, dm->face_lr, dm->face_code, dm->face_geo, dm->tables + ti.off_trace,
                                   dm->tables + ti.off_proj, ti.n_codes, U, rhs, cmb, block);
            } else {
                constexpr int TEAM = DIM + 2 <= 4 ? 4 : 8;
                hipLaunchKernelGGL((dgc_dev::surface_combine_kernel<DIM, NP, Q, false>),
                                   dim3(grid_for((f1 - f0) * TEAM, block)), dim3(block), lds, st, f0, f1, dm->n_face,
                                   dm->n_elem, dm->face_lr, dm->face_code, dm->face_geo, dm->tables + ti.off_trace,
                                   dm->tables + ti.off_proj, ti.n_codes, U, rhs, cmb, block);
            }
            *fused = true;
            return hip_check("fused surface kernel launch");
        }
    }

    static dgc_status surface(const dgc_dmesh *dm, const dgc_table_info &ti, const T *U, T *rhs, int variant, void *ws,
                              size_t ws_bytes, hipStream_t st) {
        dgc_status s = DGC_OK;
        switch (variant) {
            case DGC_SURF_COLORED:
                if ((s = check_colors(dm)) != DGC_OK) return s;
                for (int c = 0; c < dm->n_colors && s == DGC_OK; ++c)
                    s = faces<dgc_dev::kColored>(dm, ti, dm->color_off[c], dm->color_off[c + 1], U, rhs, nullptr, st);
                return s;
            case DGC_SURF_ATOMIC:
                return faces<dgc_dev::kAtomic>(dm, ti, 0, dm->n_face, U, rhs, nullptr, st);
            case DGC_SURF_GATHER: {
                const size_t need = 2 * (size_t)dm->n_face * REC * sizeof(T);
                if (!ws || ws_bytes < need) return fail(DGC_E_WORKSPACE, "GATHER needs a workspace of " + std::to_string(need) + " bytes");
                if (!dm->elem_slots || dm->max_slots <= 0) return fail(DGC_E_ARG, "GATHER needs elem_slots");
                T *buf = static_cast<T *>(ws);
                if ((s = faces<dgc_dev::kGather>(dm, ti, 0, dm->n_face, U, rhs, buf, st)) != DGC_OK) return s;
                hipLaunchKernelGGL((dgc_dev::gather_kernel<DIM, NP, T>), dim3(grid_for(dm->n_elem)), dim3(kBlock), 0, st,
                                   dm->n_elem, dm->max_slots, 2 * dm->n_face, dm->elem_slots, buf, rhs);
                return hip_check("gather kernel launch");
            }
            case DGC_SURF_COMPACT: {
                const size_t need = (size_t)dm->n_face * dgc_dev::compact_stride<DIM, Q>() * sizeof(T);
                if (!ws || ws_bytes < need)
                    return fail(DGC_E_WORKSPACE, "COMPACT needs a workspace of " + std::to_string(need) + " bytes");
                if (!dm->elem_slots || dm->max_slots <= 0) return fail(DGC_E_ARG, "COMPACT needs elem_slots");
                T *buf = static_cast<T *>(ws);
                constexpr int TEAM = DIM + 2 <= 4 ? 4 : 8;
                const size_t lds = 2 * (size_t)ti.n_codes * Q * NP * sizeof(T);
                hipLaunchKernelGGL((dgc_dev::surface_team_kernel<DIM, NP, Q, dgc_dev::kFlux, T, false>),
                                   dim3(grid_for(dm->n_face * TEAM)), dim3(kBlock), lds, st, (int64_t)0, dm->n_face,
                                   dm->n_face, dm->n_elem, dm->face_lr, dm->face_code, dm->face_geo,
                                   dm->tables + ti.off_trace, dm->tables + ti.off_proj, ti.n_codes, U, rhs, buf, 0,
                                   kBlock);
                if ((s = hip_check("compact face pass launch")) != DGC_OK) return s;
                hipLaunchKernelGGL((dgc_dev::compact_gather_kernel<DIM, NP, Q, T>), dim3(grid_for(dm->n_elem * TEAM)),
                                   dim3(kBlock), lds / 2, st, dm->n_elem, dm->n_face, dm->max_slots, dm->elem_slots,
                                   dm->elem_geo, dm->tables + ti.off_proj, ti.n_codes, buf, rhs);
                return hip_check("compact gather launch");
            }
            default: return fail(DGC_E_ARG, "unknown surface variant");
        }
    }

    // One SSP-RK3 stage of the compact variant (f64, triangles and
    // parallelograms): the face pass writes every face's record, then one
    // element pass adds the volume term and the records and writes the
    // stage combination.
    static dgc_status compact_stage(const dgc_dmesh *dm, const dgc_table_info &ti, const double *U, void *ws,
                                    size_t ws_bytes, const dgc_dev::CombineArgs &cmb, hipStream_t st) {
        if constexpr (DIM == 2 && std::is_same<T, double>::value) {
            const size_t need = (size_t)dm->n_face * dgc_dev::compact_stride<DIM, Q>() * sizeof(double);
            if (!ws || ws_bytes < need)
                return fail(DGC_E_WORKSPACE, "COMPACT needs a workspace of " + std::to_string(need) + " bytes");
            if (!dm->elem_slots || dm->max_slots <= 0) return fail(DGC_E_ARG, "COMPACT needs elem_slots");
            double *buf = static_cast<double *>(ws);
            constexpr int TEAM = 4;
            const size_t lds = 2 * (size_t)ti.n_codes * Q * NP * sizeof(double);
            hipLaunchKernelGGL((dgc_dev::surface_team_kernel<DIM, NP, Q, dgc_dev::kFlux, double, false>),
                               dim3(grid_for(dm->n_face * TEAM)), dim3(kBlock), lds, st, (int64_t)0, dm->n_face,
                               dm->n_face, dm->n_elem, dm->face_lr, dm->face_code, dm->face_geo,
                               dm->tables + ti.off_trace, dm->tables + ti.off_proj, ti.n_codes, U,
                               static_cast<double *>(nullptr), buf, 0, kBlock);
            dgc_status s = hip_check("compact face pass launch");
            if (s != DGC_OK) return s;
            // every element has as many face slots as faces (conforming
            // triangles and parallelograms)
            const int faces = dm->elem_type == DGC_TRI ? 3 : 4;
            if (dm->max_slots != faces)
                return fail(DGC_E_UNSUPPORTED, "the compact stage kernel needs one slot per face");
            if (faces == 3)
                hipLaunchKernelGGL((dgc_dev::compact_stage_kernel<DIM, NP, Q, QV, 3>),
                                   dim3(grid_for(dm->n_elem * TEAM)), dim3(kBlock), lds / 2, st, dm->n_elem,
                                   dm->n_face, dm->elem_slots, dm->elem_geo, dm->tables + ti.off_proj, ti.n_codes,
                                   dm->tables + ti.off_vb, dm->tables + ti.off_vd, buf, U, cmb);
            else
                hipLaunchKernelGGL((dgc_dev::compact_stage_kernel<DIM, NP, Q, QV, 4>),
                                   dim3(grid_for(dm->n_elem * TEAM)), dim3(kBlock), lds / 2, st, dm->n_elem,
                                   dm->n_face, dm->elem_slots, dm->elem_geo, dm->tables + ti.off_proj, ti.n_codes,
                                   dm->tables + ti.off_vb, dm->tables + ti.off_vd, buf, U, cmb);
            return hip_check("compact stage launch");
        } else {
            return fail(DGC_E_UNSUPPORTED, "the compact stage kernel is built for f64 triangles and parallelograms");
        }
    }
};

template <class T, class F>
dgc_status dispatch(const dgc_dmesh *dm, int elem_type, int p, F &&f) {
    if (dm) {
        elem_type = dm->elem_type;
        p = dm->p;
    }
    if (elem_type == DGC_TRI) {
        switch (p) {
            case 0: return f(Impl<2, 1, 1, 1, T>{});
            case 1: return f(Impl<2, 3, 2, 4, T>{});
            case 2: return f(Impl<2, 6, 3, 9, T>{});
            case 3: return f(Impl<2, 10, 4, 16, T>{});
            case 4: return f(Impl<2, 15, 5, 25, T>{});
            case 5: return f(Impl<2, 21, 6, 36, T>{});
            default: break;
        }
    } else if (elem_type == DGC_QUAD) {
        switch (p) {
            case 0: return f(Impl<2, 1, 1, 1, T>{});
            case 1: return f(Impl<2, 4, 2, 4, T>{});
            case 2: return f(Impl<2, 9, 3, 9, T>{});
            case 3: return f(Impl<2, 16, 4, 16, T>{});
            default: break;
        }
    } else if (elem_type == DGC_MIXED) {
        // (p+1)^2 slots per element, the quadrilateral's count
        switch (p) {
            case 0: return f(Impl<2, 1, 1, 1, T>{});
            case 1: return f(Impl<2, 4, 2, 4, T>{});
            case 2: return f(Impl<2, 9, 3, 9, T>{});
            case 3: return f(Impl<2, 16, 4, 16, T>{});
            default: break;
        }
    } else if (elem_type == DGC_TET) {
        switch (p) {
            case 0: return f(Impl<3, 1, 3, 1, T>{});
            case 1: return f(Impl<3, 4, 3, 8, T>{});
            case 2: return f(Impl<3, 10, 9, 27, T>{});
            default: break;
        }
    }
    return fail(DGC_E_UNSUPPORTED, "no kernel built for this element type and order");
}

size_t rec_bytes(const dgc_dmesh *dm, size_t elt) { return (size_t)dm->n_var * dm->n_p * elt; }

}  // namespace

extern "C" {

dgc_status dgc_volume_rhs(const dgc_dmesh *dm, const void *U, void *rhs, int32_t precision, void *stream) {
    dgc_table_info ti;
    dgc_status s = check_dm(dm, &ti);
    if (s != DGC_OK) return s;
    if (!U || !rhs) return fail(DGC_E_ARG, "dgc_volume_rhs: null U or rhs");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (precision == DGC_F64)
        return dispatch<double>(dm, 0, 0, [&](auto impl) {
            return decltype(impl)::volume(dm, ti, static_cast<const double *>(U), static_cast<double *>(rhs), st);
        });
    if (precision == DGC_F32)
        return dispatch<float>(dm, 0, 0, [&](auto impl) {
            return decltype(impl)::volume(dm, ti, static_cast<const float *>(U), static_cast<float *>(rhs), st);
        });
    return fail(DGC_E_ARG, "unknown precision");
}

dgc_status dgc_surface_rhs(const dgc_dmesh *dm, const void *U, void *rhs, int32_t variant, int32_t precision, void *ws,
                           size_t ws_bytes, void *stream) {
    dgc_table_info ti;
    dgc_status s = check_dm(dm, &ti);
    if (s != DGC_OK) return s;
    if (!U || !rhs) return fail(DGC_E_ARG, "dgc_surface_rhs: null U or rhs");
    hipStream_t st = static_cast<hipStream_t>(stream);
    if (precision == DGC_F64)
        return dispatch<double>(dm, 0, 0, [&](auto impl) {
            return decltype(impl)::surface(dm, ti, static_cast<const double *>(U), static_cast<double *>(rhs), variant,
                                           ws, ws_bytes, st);
        });
    if (precision == DGC_F32)
        return dispatch<float>(dm, 0, 0, [&](auto impl) {
            return decltype(impl)::surface(dm, ti, static_cast<const float *>(U), static_cast<float *>(rhs), variant, ws,
                                           ws_bytes, st);
        });
    return fail(DGC_E_ARG, "unknown precision");
}

dgc_status dgc_workspace_bytes(const dgc_dmesh *dm, int32_t what, int32_t variant, int32_t precision, size_t *bytes) {
    dgc_table_info ti;
    dgc_status s = check_dm(dm, &ti);
    if (s != DGC_OK) return s;
    if (!bytes) return fail(DGC_E_ARG, "null bytes");
    if (precision != DGC_F64 && precision != DGC_F32) return fail(DGC_E_ARG, "unknown precision");
    if (variant < DGC_SURF_COLORED || variant > DGC_SURF_COMPACT) return fail(DGC_E_ARG, "unknown variant");
    const size_t elt = precision == DGC_F64 ? 8 : 4;
    const size_t rec = rec_bytes(dm, elt);
    const size_t surf = variant == DGC_SURF_GATHER    ? 2 * (size_t)dm->n_face * rec
                        : variant == DGC_SURF_COMPACT ? (size_t)dm->n_face * (dm->n_qf * dm->n_var + 1) * elt
                                                      : 0;
    if (what == DGC_WS_SURFACE) {
        *bytes = surf;
        return DGC_OK;
    }
    if (what == DGC_WS_RK_STEP) {
        const size_t n = (size_t)dm->n_elem * dm->n_var * dm->n_p;
        size_t off[4], total;
        dgc_batch::rk_ws_offsets(n, precision == DGC_F32, off, &total);  // U1, U2, rhs, f32 shadow
        *bytes = total + surf;
        return DGC_OK;
    }
    return fail(DGC_E_ARG, "unknown workspace kind");
}

dgc_status dgc_rk_step(const dgc_dmesh *dm, double *U, double dt, int32_t variant, int32_t precision, void *ws,
                       size_t ws_bytes, void *stream) {
    dgc_table_info ti;
    dgc_status s = check_dm(dm, &ti);
    if (s != DGC_OK) return s;
    if (!U) return fail(DGC_E_ARG, "dgc_rk_step: null U");
    size_t need = 0;
    if ((s = dgc_workspace_bytes(dm, DGC_WS_RK_STEP, variant, precision, &need)) != DGC_OK) return s;
    if (!ws || ws_bytes < need) return fail(DGC_E_WORKSPACE, "dgc_rk_step needs a workspace of " + std::to_string(need) + " bytes");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const size_t n = (size_t)dm->n_elem * dm->n_var * dm->n_p;
    char *w = static_cast<char *>(ws);
    const dgc_batch::RkWs lay = dgc_batch::rk_ws(w, n, precision == DGC_F32);
    double *U1 = lay.U1;
    double *U2 = lay.U2;
    void *rhs = lay.rhs;
    float *shadow = lay.shadow;
    void *sws = w + lay.bytes;
    size_t sws_bytes = ws_bytes - lay.bytes;

    const double a[3] = {0.0, 0.75, 1.0 / 3.0};
    const double b[3] = {1.0, 0.25, 2.0 / 3.0};
    const double *x_in[3] = {U, U, U};
    const double *stage_in[3] = {U, U1, U2};
    double *stage_out[3] = {U1, U2, U};
    if (shadow) {
        hipLaunchKernelGGL(dgc_dev::to_f32_kernel, dim3(grid_for((int64_t)n)), dim3(kBlock), 0, st, (int64_t)n, U, shadow);
        if ((s = hip_check("f32 shadow launch")) != DGC_OK) return s;
    }
    if (dm->rk_form < DGC_RK_DEFAULT || dm->rk_form > DGC_RK_FUSED_VOLUME)
        return fail(DGC_E_ARG, "dgc_dmesh: unknown rk_form");
    // a small mesh: the whole step in one work-group (see DGC_RK_BLOCK)
    const bool block_ok = !shadow && variant == DGC_SURF_COLORED && dm->elem_type != DGC_MIXED;
    if (dm->rk_form == DGC_RK_BLOCK && !block_ok)
        return fail(DGC_E_UNSUPPORTED, "DGC_RK_BLOCK needs f64, the colored variant and one element type");
    if (block_ok && dm->rk_form == DGC_RK_BLOCK) {
        return dispatch<double>(dm, 0, 0, [&](auto impl) {
            return decltype(impl)::rk_block(dm, ti, U, U1, U2, static_cast<double *>(rhs), dt, st);
        });
    }
    // the compact variant (f64, conforming triangle and parallelogram
    // meshes): a face pass and one element pass per stage, the element pass
    // also evaluating the volume term and writing the stage combination
    if (variant == DGC_SURF_COMPACT && !shadow && dm->rk_form != DGC_RK_SEPARATE &&
        (dm->elem_type == DGC_TRI || dm->elem_type == DGC_QUAD) &&
        dm->max_slots == (dm->elem_type == DGC_TRI ? 3 : 4)) {
        for (int stg = 0; stg < 3; ++stg) {
            const dgc_dev::CombineArgs cmb{stg == 0 ? nullptr : U, stage_out[stg], a[stg], b[stg], dt};
            s = dispatch<double>(dm, 0, 0, [&](auto impl) {
                return decltype(impl)::compact_stage(dm, ti, stage_in[stg], sws, sws_bytes, cmb, st);
            });
            if (s != DGC_OK) return s;
        }
        return DGC_OK;
    }
    // the stage combination rides on the last color's face kernel, and the
    // volume term on the first color's, when every element has exactly one
    // face of each color (see DGC_RK_FUSED and DGC_RK_FUSED_VOLUME)
    if (variant == DGC_SURF_COLORED && (s = check_colors(dm)) != DGC_OK) return s;
    const int faces_per_elem = dm->elem_type == DGC_TRI ? 3 : 4;
    const int sform = resolved_surface_form(dm, shadow != nullptr);
    const bool one_face_per_color = variant == DGC_SURF_COLORED && dm->elem_type != DGC_MIXED &&
                                    dm->n_colors == faces_per_elem && dm->max_slots == faces_per_elem &&
                                    sform != DGC_FORM_THREAD && dm->color_off[1] > dm->color_off[0];
    // (the f32 form keeps its combination kernel: measured faster than a fused
    // one, whose extra f64 reads cost the face kernel registers)
    // (not for tetrahedra from p = 2 on: the combining team kernel runs out of
    // registers there and the separate combination is faster)
    const bool fuse = !shadow && one_face_per_color && dm->rk_form != DGC_RK_SEPARATE &&
                      !(dm->elem_type == DGC_TET && dm->p >= 2 && dm->rk_form == DGC_RK_DEFAULT);
    const bool vol_team_face = sform == DGC_FORM_TEAM || sform == DGC_FORM_TEAM_PREFETCH ||
                               sform == DGC_FORM_TEAM_STREAM ||
                               (sform == DGC_FORM_MODE_TEAM && dm->elem_type == DGC_TET && dm->p == 1);
    const bool fuse_vol = one_face_per_color && vol_team_face &&
                          (dm->rk_form == DGC_RK_FUSED_VOLUME ||
                           (dm->rk_form == DGC_RK_DEFAULT && dm->vol_form == DGC_VOL_DEFAULT &&
                            default_fuse_volume(dm->elem_type, dm->p, shadow != nullptr)));
    const int first = fuse_vol ? 1 : 0;
    for (int stg = 0; stg < 3; ++stg) {
        const void *Uin = shadow ? static_cast<const void *>(shadow) : static_cast<const void *>(stage_in[stg]);
        if (fuse_vol) {
            const int64_t f0 = dm->color_off[0], f1 = dm->color_off[1];
            if (shadow)
                s = dispatch<float>(dm, 0, 0, [&](auto impl) {
                    return decltype(impl)::faces_volume(dm, ti, f0, f1, shadow, static_cast<float *>(rhs), st);
                });
            else
                s = dispatch<double>(dm, 0, 0, [&](auto impl) {
                    return decltype(impl)::faces_volume(dm, ti, f0, f1, stage_in[stg], static_cast<double *>(rhs),
                                                        st);
                });
        } else {
            s = dgc_volume_rhs(dm, Uin, rhs, precision, stream);
        }
        if (s != DGC_OK) return s;
        if (fuse) {
            const dgc_dev::CombineArgs cmb{stg == 0 ? nullptr : U, stage_out[stg], a[stg], b[stg], dt};
            bool fused = false;
            s = dispatch<double>(dm, 0, 0, [&](auto impl) {
                return decltype(impl)::surface_fused(dm, ti, stage_in[stg], static_cast<double *>(rhs), cmb, first,
                                                     &fused, st);
            });
            if (s != DGC_OK) return s;
            if (fused) continue;
        }
        if (first == 0) {
            s = dgc_surface_rhs(dm, Uin, rhs, variant, precision, sws, sws_bytes, stream);
        } else if (shadow) {
            s = dispatch<float>(dm, 0, 0, [&](auto impl) {
                return decltype(impl)::colors(dm, ti, first, dm->n_colors, shadow, static_cast<float *>(rhs), st);
            });
        } else {
            s = dispatch<double>(dm, 0, 0, [&](auto impl) {
                return decltype(impl)::colors(dm, ti, first, dm->n_colors, stage_in[stg], static_cast<double *>(rhs),
                                              st);
            });
        }
        if (s != DGC_OK) return s;
        if (shadow) {
            hipLaunchKernelGGL(dgc_dev::rk_combine_f32_kernel, dim3(grid_for((int64_t)n)), dim3(kBlock), 0, st,
                               (int64_t)n, a[stg], b[stg], dt, x_in[stg], stage_in[stg], static_cast<const float *>(rhs),
                               stage_out[stg], stg < 2 ? shadow : nullptr);
        } else {
            hipLaunchKernelGGL(dgc_dev::rk_combine_kernel, dim3(grid_for((int64_t)n)), dim3(kBlock), 0, st, (int64_t)n,
                               a[stg], b[stg], dt, x_in[stg], stage_in[stg], static_cast<const double *>(rhs),
                               stage_out[stg]);
        }
        if ((s = hip_check("rk combine launch")) != DGC_OK) return s;
    }
    return DGC_OK;
}

// SSP-RK3 step without a caller workspace: the stage states and right-hand
// side live in `scratch`, a device array of fixed size that every GPU holds
// once (at its own address) until the process ends.  Host code never passes
// the array's name to a kernel or a copy: it stands for a host-side shadow
// there.  The device address is looked up once per device, with that device
// current, and kept.
static __device__ __align__(256) unsigned char scratch[DGC_NOALLOC_MAX_BYTES];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};

dgc_status scratch_address(void **out) {
    int dev = -1;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(DGC_E_HIP, std::string("hipGetDevice: ") + hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(DGC_E_HIP, "device ordinal out of range: " + std::to_string(dev));
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(DGC_E_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return DGC_OK;
}

}  // namespace

dgc_status dgc_rk_step_noalloc(const dgc_dmesh *dm, double *U, double dt, int32_t variant, int32_t precision,
                               void *stream) {
    dgc_table_info ti;
    dgc_status s = check_dm(dm, &ti);
    if (s != DGC_OK) return s;
    if (!U) return fail(DGC_E_ARG, "dgc_rk_step_noalloc: null U");
    size_t need = 0;
    if ((s = dgc_workspace_bytes(dm, DGC_WS_RK_STEP, variant, precision, &need)) != DGC_OK) return s;
    if (need > (size_t)DGC_NOALLOC_MAX_BYTES)
        return fail(DGC_E_WORKSPACE, "dgc_rk_step_noalloc: this mesh needs " + std::to_string(need) +
                                         " bytes of stage storage, more than the " +
                                         std::to_string((size_t)DGC_NOALLOC_MAX_BYTES) +
                                         " the library holds; call dgc_rk_step with a workspace");
    void *ws = nullptr;
    if ((s = scratch_address(&ws)) != DGC_OK) return s;
    return dgc_rk_step(dm, U, dt, variant, precision, ws, (size_t)DGC_NOALLOC_MAX_BYTES, stream);
}

}  // extern "C"

// ------------------------------------------------------------------------
// Batched forms
// ------------------------------------------------------------------------

namespace {

template <class F>
dgc_status dispatch_type(int elem_type, int p, int precision, F &&f) {
    if (precision == DGC_F64) return dispatch<double>(nullptr, elem_type, p, f);
    return dispatch<float>(nullptr, elem_type, p, f);
}

dgc_status read_header(const void *host_desc, dgc_batch::Header *h) {
    if (!host_desc) return fail(DGC_E_ARG, "null batch descriptor");
    std::memcpy(h, host_desc, sizeof(*h));
    if (h->magic != dgc_batch::kMagic || h->n_mesh <= 0) return fail(DGC_E_ARG, "not a batch descriptor");
    return DGC_OK;
}

template <int DIM, int NP, int Q, int QV, class T>
struct BatchImpl {
    // color c of every mesh in face-kernel mode MODE
    template <int MODE>
    static dgc_status color(const dgc_batch::Header &h, const char *dev, int stage, int c, hipStream_t st) {
        if (h.nblk_face[c] == 0) return DGC_OK;
        size_t lds = 2 * (size_t)h.n_codes * Q * NP * sizeof(T);
        // the mode team's fused volume term stages the volume tables too
        if (MODE == dgc_dev::kVolume && DIM == 3 && NP == 4) lds += (size_t)(1 + DIM) * QV * NP * sizeof(T);
        hipLaunchKernelGGL((dgc_dev::batch_surface_kernel<DIM, NP, Q, QV, MODE, T>), dim3(h.nblk_face[c]),
                           dim3(h.block), lds, st, dev, c, stage);
        return hip_check("batched surface launch");
    }
    static dgc_status surface(const dgc_batch::Header &h, const char *dev, int stage, hipStream_t st) {
        for (int c = 0; c < h.n_colors; ++c)
            if (dgc_status s = color<dgc_dev::kColored>(h, dev, stage, c, st); s != DGC_OK) return s;
        return DGC_OK;
    }
    // the volume and face work of one SSP-RK3 stage, with the volume term in
    // the first color's launch and (f64) the combination in the last color's
    // as the header allows
    static dgc_status stage_fused(const dgc_batch::Header &h, const char *dev, int stage, hipStream_t st) {
        const int nc = h.n_colors;
        dgc_status s = h.fuse_volume ? color<dgc_dev::kVolume>(h, dev, stage, 0, st) : volume(h, dev, stage, st);
        if (s != DGC_OK) return s;
        for (int c = h.fuse_volume ? 1 : 0; c < nc - 1; ++c)
            if ((s = color<dgc_dev::kColored>(h, dev, stage, c, st)) != DGC_OK) return s;
        if constexpr (std::is_same_v<T, double>)
            if (h.fuse_combine) return color<dgc_dev::kCombine>(h, dev, stage, nc - 1, st);
        return color<dgc_dev::kColored>(h, dev, stage, nc - 1, st);
    }
    static dgc_status volume(const dgc_batch::Header &h, const char *dev, int stage, hipStream_t st) {
        hipLaunchKernelGGL((dgc_dev::batch_volume_kernel<DIM, NP, QV, T>), dim3(h.nblk_elem), dim3(kBlock), 0, st, dev,
                           stage);
        return hip_check("batched volume launch");
    }
};

}  // namespace

extern "C" {

dgc_status dgc_permute_records(const void *src, void *dst, const int32_t *perm, int64_t n_rec, int64_t rec_bytes,
                               int32_t to_layout, void *stream) {
    if (!src || !dst || !perm || n_rec < 0 || rec_bytes <= 0 || rec_bytes % 4 != 0 || src == dst)
        return fail(DGC_E_ARG, "dgc_permute_records: bad argument");
    if (n_rec == 0) return DGC_OK;
    const int64_t words = rec_bytes / 4;
    hipLaunchKernelGGL(dgc_dev::permute_records_kernel, dim3(grid_for(n_rec * words)), dim3(kBlock), 0,
                       static_cast<hipStream_t>(stream), static_cast<const uint32_t *>(src), static_cast<uint32_t *>(dst),
                       perm, n_rec, words, to_layout ? 1 : 0);
    return hip_check("permute kernel launch");
}

dgc_status dgc_child_colors(const int8_t *parent_colors, int64_t n, int8_t *child_colors, void *stream) {
    if (!parent_colors || !child_colors || n < 0) return fail(DGC_E_ARG, "dgc_child_colors: bad argument");
    if (n == 0) return DGC_OK;
    hipLaunchKernelGGL(dgc_dev::child_colors_kernel, dim3(grid_for(n)), dim3(kBlock), 0,
                       static_cast<hipStream_t>(stream), parent_colors, n, child_colors);
    return hip_check("child color kernel launch");
}

dgc_status dgc_adapt_transfer(const dgc_dmesh *dm, const double *U_old, int64_t n_old, double *U_new,
                              const int8_t *kind, const int32_t *src, void *stream) {
    dgc_table_info ti;
    dgc_status s = check_dm(dm, &ti);
    if (s != DGC_OK) return s;
    if (dm->elem_type != DGC_TRI) return fail(DGC_E_UNSUPPORTED, "dgc_adapt_transfer: triangles only");
    if (!U_old || !U_new || !kind || !src || n_old <= 0 || n_old > ((int64_t)1 << 31) - 1)
        return fail(DGC_E_ARG, "dgc_adapt_transfer: bad argument");
    if (U_old == U_new) return fail(DGC_E_ARG, "dgc_adapt_transfer: U_old and U_new must be distinct");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const double *P = dm->tables + ti.off_prolong;
    const int64_t n = dm->n_elem * dm->n_var;
    auto go = [&](auto np_tag) {
        constexpr int NP = decltype(np_tag)::value;
        hipLaunchKernelGGL((dgc_dev::adapt_transfer_kernel<NP>), dim3(grid_for(n)), dim3(kBlock), 0, st, dm->n_elem,
                           dm->n_var, n_old, kind, src, P, U_old, U_new);
        return hip_check("adapt transfer kernel launch");
    };
    switch (dm->p) {
        case 0: return go(std::integral_constant<int, 1>{});
        case 1: return go(std::integral_constant<int, 3>{});
        case 2: return go(std::integral_constant<int, 6>{});
        case 3: return go(std::integral_constant<int, 10>{});
        case 4: return go(std::integral_constant<int, 15>{});
        case 5: return go(std::integral_constant<int, 21>{});
        default: return fail(DGC_E_UNSUPPORTED, "dgc_adapt_transfer: no kernel for this order");
    }
}

dgc_status dgc_rk_workspace_layout(int64_t n, int32_t precision, size_t off[4], size_t *total) {
    if (n < 0 || !off || !total || (precision != DGC_F64 && precision != DGC_F32))
        return fail(DGC_E_ARG, "dgc_rk_workspace_layout: bad argument");
    dgc_batch::rk_ws_offsets((size_t)n, precision == DGC_F32, off, total);
    if (precision != DGC_F32) off[3] = 0;
    return DGC_OK;
}

dgc_status dgc_batch_describe(int32_t n_mesh, const dgc_dmesh *meshes, double *const *U, void *const *ws,
                              const double *dt, int32_t precision, void *host_desc, size_t bytes, size_t *needed) {
    if (n_mesh <= 0 || !meshes || !U || !ws || !dt) return fail(DGC_E_ARG, "dgc_batch_describe: bad argument");
    if (precision != DGC_F64 && precision != DGC_F32) return fail(DGC_E_ARG, "dgc_batch_describe: unknown precision");
    dgc_table_info ti{};
    for (int32_t i = 0; i < n_mesh; ++i) {
        dgc_table_info t;
        if (dgc_status s = check_dm(&meshes[i], &t); s != DGC_OK) return s;
        if (dgc_status s = check_colors(&meshes[i]); s != DGC_OK) return s;
        if (i == 0) ti = t;
        if (meshes[i].elem_type == DGC_MIXED)
            return fail(DGC_E_UNSUPPORTED, "dgc_batch_describe: mixed meshes are not batched");
        if (meshes[i].elem_type != meshes[0].elem_type || meshes[i].p != meshes[0].p)
            return fail(DGC_E_ARG, "dgc_batch_describe: meshes of one batch share element type and order");
        if (!U[i] || !ws[i]) return fail(DGC_E_ARG, "dgc_batch_describe: null state or workspace");
        if (!std::isfinite(dt[i])) return fail(DGC_E_ARG, "dgc_batch_describe: non-finite dt");
    }
    // lanes per face of batch_surface_kernel (batch_team<DIM, NP>)
    const int team = (ti.dim == 3 && ti.n_p == 4) ? 4 : (ti.dim + 2 <= 4 ? 4 : 8);
    const int fpb = kBlock / team;
    // lanes per element of batch_volume_kernel
    const int vteam = dgc_dev::batch_volume_lanes(ti.dim, ti.n_p, precision == DGC_F32);
    int nc = 0;
    for (int32_t i = 0; i < n_mesh; ++i) nc = meshes[i].n_colors > nc ? meshes[i].n_colors : nc;
    // work-group counts
    std::vector<int64_t> nb_face(nc, 0);
    int64_t nb_elem = 0, nb_dof = 0;
    for (int32_t i = 0; i < n_mesh; ++i) {
        const dgc_dmesh &d = meshes[i];
        for (int c = 0; c < nc; ++c) {
            const int64_t nf = c < d.n_colors ? d.color_off[c + 1] - d.color_off[c] : 0;
            nb_face[c] += (nf + fpb - 1) / fpb;
        }
        nb_elem += (d.n_elem * vteam + kBlock - 1) / kBlock;
        nb_dof += (d.n_elem * d.n_var * d.n_p + kBlock - 1) / kBlock;
    }
    for (int c = 0; c < nc; ++c)
        if (nb_face[c] > INT32_MAX) return fail(DGC_E_ARG, "dgc_batch_describe: batch too large");
    if (nb_elem > INT32_MAX || nb_dof > INT32_MAX) return fail(DGC_E_ARG, "dgc_batch_describe: batch too large");
    dgc_batch::Header h{};
    h.magic = dgc_batch::kMagic;
    h.n_mesh = n_mesh;
    h.n_colors = nc;
    h.elem_type = meshes[0].elem_type;
    h.p = meshes[0].p;
    h.n_p = ti.n_p;
    h.n_var = ti.dim + 2;
    h.n_qf = ti.n_qf;
    h.n_qv = ti.n_qv;
    h.n_codes = ti.n_codes;
    h.precision = precision;
    h.block = kBlock;
    h.faces_per_block = fpb;
    {
        // fused stage kernels need exactly one face of each color per element
        const int fpe = h.elem_type == DGC_TRI ? 3 : 4;
        bool one = true;
        for (int32_t i = 0; i < n_mesh; ++i) {
            const dgc_dmesh &d = meshes[i];
            one = one && d.n_colors == fpe && d.max_slots == fpe && d.color_off[1] > d.color_off[0] &&
                  d.color_off[fpe] > d.color_off[fpe - 1];
        }
        h.fuse_combine = one && precision == DGC_F64 ? 1 : 0;
        h.fuse_volume = one && default_fuse_volume(h.elem_type, h.p, precision == DGC_F32) ? 1 : 0;
    }
    h.tables = meshes[0].tables;
    h.off_trace = ti.off_trace;
    h.off_proj = ti.off_proj;
    h.off_vb = ti.off_vb;
    h.off_vd = ti.off_vd;
    int64_t off = dgc_batch::kHeaderBytes;
    h.off_entries = off;
    off += (int64_t)sizeof(dgc_batch::Entry) * n_mesh;
    for (int c = 0; c < nc; ++c) {
        h.off_map_face[c] = off;
        h.nblk_face[c] = (int32_t)nb_face[c];
        off += 4 * nb_face[c];
    }
    h.off_map_elem = off;
    h.nblk_elem = (int32_t)nb_elem;
    off += 4 * nb_elem;
    h.off_map_dof = off;
    h.nblk_dof = (int32_t)nb_dof;
    off += 4 * nb_dof;
    h.total_bytes = off;
    if (needed) *needed = (size_t)off;
    if (!host_desc) return DGC_OK;
    if (bytes < (size_t)off) return fail(DGC_E_ARG, "dgc_batch_describe: destination too small");
    char *out = static_cast<char *>(host_desc);
    std::memset(out, 0, (size_t)off);
    std::memcpy(out, &h, sizeof(h));
    dgc_batch::Entry *ent = reinterpret_cast<dgc_batch::Entry *>(out + h.off_entries);
    std::vector<int64_t> cur(nc, 0);
    int64_t ce = 0, cd = 0;
    for (int32_t i = 0; i < n_mesh; ++i) {
        const dgc_dmesh &d = meshes[i];
        dgc_batch::Entry &e = ent[i];
        e.face_lr = d.face_lr;
        e.face_code = d.face_code;
        e.face_geo = d.face_geo;
        e.elem_geo = d.elem_geo;
        e.U = U[i];
        e.ws = static_cast<char *>(ws[i]);
        e.dt = dt[i];
        e.n_face = d.n_face;
        e.n_elem = d.n_elem;
        e.n_dof = d.n_elem * d.n_var * d.n_p;
        for (int c = 0; c <= nc; ++c) e.color_off[c] = c <= d.n_colors ? d.color_off[c] : d.n_face;
        for (int c = 0; c < nc; ++c) {
            const int64_t nf = e.color_off[c + 1] - e.color_off[c];
            const int64_t nb = (nf + fpb - 1) / fpb;
            e.blk_face[c] = (int32_t)cur[c];
            int32_t *map = reinterpret_cast<int32_t *>(out + h.off_map_face[c]);
            for (int64_t b = 0; b < nb; ++b) map[cur[c] + b] = i;
            cur[c] += nb;
        }
        const int64_t ne = (d.n_elem * vteam + kBlock - 1) / kBlock, nd = (e.n_dof + kBlock - 1) / kBlock;
        e.blk_elem = (int32_t)ce;
        e.blk_dof = (int32_t)cd;
        int32_t *me = reinterpret_cast<int32_t *>(out + h.off_map_elem);
        int32_t *md = reinterpret_cast<int32_t *>(out + h.off_map_dof);
        for (int64_t b = 0; b < ne; ++b) me[ce + b] = i;
        for (int64_t b = 0; b < nd; ++b) md[cd + b] = i;
        ce += ne;
        cd += nd;
    }
    return DGC_OK;
}

dgc_status dgc_surface_rhs_batched(const void *host_desc, const void *dev_desc, int32_t stage, void *stream) {
    dgc_batch::Header h;
    if (dgc_status s = read_header(host_desc, &h); s != DGC_OK) return s;
    if (!dev_desc || stage < 0 || stage > 2) return fail(DGC_E_ARG, "dgc_surface_rhs_batched: bad argument");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const char *dev = static_cast<const char *>(dev_desc);
    return dispatch_type(h.elem_type, h.p, h.precision, [&](auto impl) {
        using I = decltype(impl);
        return BatchImpl<I::kDim, I::kNp, I::kQ, I::kQv, typename I::Real>::surface(h, dev, stage, st);
    });
}

dgc_status dgc_volume_rhs_batched(const void *host_desc, const void *dev_desc, int32_t stage, void *stream) {
    dgc_batch::Header h;
    if (dgc_status s = read_header(host_desc, &h); s != DGC_OK) return s;
    if (!dev_desc || stage < 0 || stage > 2) return fail(DGC_E_ARG, "dgc_volume_rhs_batched: bad argument");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const char *dev = static_cast<const char *>(dev_desc);
    return dispatch_type(h.elem_type, h.p, h.precision, [&](auto impl) {
        using I = decltype(impl);
        return BatchImpl<I::kDim, I::kNp, I::kQ, I::kQv, typename I::Real>::volume(h, dev, stage, st);
    });
}

dgc_status dgc_rk_step_batched(const void *host_desc, const void *dev_desc, void *stream) {
    dgc_batch::Header h;
    if (dgc_status s = read_header(host_desc, &h); s != DGC_OK) return s;
    if (!dev_desc) return fail(DGC_E_ARG, "dgc_rk_step_batched: null device descriptor");
    hipStream_t st = static_cast<hipStream_t>(stream);
    const char *dev = static_cast<const char *>(dev_desc);
    const bool f32 = h.precision == DGC_F32;
    if (f32) {
        hipLaunchKernelGGL(dgc_dev::batch_to_f32_kernel, dim3(h.nblk_dof), dim3(kBlock), 0, st, dev);
        if (dgc_status s = hip_check("batched f32 shadow launch"); s != DGC_OK) return s;
    }
    for (int stage = 0; stage < 3; ++stage) {
        if (h.fuse_combine || h.fuse_volume) {
            dgc_status s = dispatch_type(h.elem_type, h.p, h.precision, [&](auto impl) {
                using I = decltype(impl);
                return BatchImpl<I::kDim, I::kNp, I::kQ, I::kQv, typename I::Real>::stage_fused(h, dev, stage, st);
            });
            if (s != DGC_OK) return s;
            if (h.fuse_combine) continue;
        } else {
            if (dgc_status s = dgc_volume_rhs_batched(host_desc, dev_desc, stage, stream); s != DGC_OK) return s;
            if (dgc_status s = dgc_surface_rhs_batched(host_desc, dev_desc, stage, stream); s != DGC_OK) return s;
        }
        if (f32)
            hipLaunchKernelGGL(dgc_dev::batch_combine_kernel<float>, dim3(h.nblk_dof), dim3(kBlock), 0, st, dev, stage);
        else
            hipLaunchKernelGGL(dgc_dev::batch_combine_kernel<double>, dim3(h.nblk_dof), dim3(kBlock), 0, st, dev, stage);
        if (dgc_status s = hip_check("batched combine launch"); s != DGC_OK) return s;
    }
    return DGC_OK;
}

}  // extern "C"
