// Device entry points of the C ABI: argument checks, template dispatch on
// (element type, order, precision) and launches on the caller's stream.
#include <hip/hip_runtime.h>

#include <string>

#include "../host/internal.hpp"
#include "surface.hpp"
#include "volume.hpp"

using dgc::fail;

namespace {

constexpr int kBlock = 256;

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
    if (dm->surf_form < DGC_FORM_DEFAULT || dm->surf_form > DGC_FORM_TEAM_PREFETCH)
        return fail(DGC_E_ARG, "dgc_dmesh: unknown surf_form");
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

    static dgc_status volume(const dgc_dmesh *dm, const dgc_table_info &ti, const T *U, T *rhs, hipStream_t st) {
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
        if (dm->surf_form == DGC_FORM_THREAD) {
            hipLaunchKernelGGL((dgc_dev::surface_kernel<DIM, NP, Q, MODE, T>), dim3(grid_for(f1 - f0, block)),
                               dim3(block), lds, st, f0, f1, dm->n_face, dm->n_elem, dm->face_lr, dm->face_code,
                               dm->face_geo, dm->tables + ti.off_trace, dm->tables + ti.off_proj, ti.n_codes, U, rhs,
                               buf, dm->xcd_remap);
        } else {
            constexpr int TEAM = DIM + 2 <= 4 ? 4 : 8;
            if (dm->surf_form == DGC_FORM_TEAM_PREFETCH || dm->surf_form == DGC_FORM_DEFAULT)
                hipLaunchKernelGGL((dgc_dev::surface_team_kernel<DIM, NP, Q, MODE, T, true>),
                                   dim3(grid_for((f1 - f0) * TEAM, block)), dim3(block), lds, st, f0, f1, dm->n_face,
                                   dm->n_elem, dm->face_lr, dm->face_code, dm->face_geo, dm->tables + ti.off_trace,
                                   dm->tables + ti.off_proj, ti.n_codes, U, rhs, buf, dm->xcd_remap);
            else
                hipLaunchKernelGGL((dgc_dev::surface_team_kernel<DIM, NP, Q, MODE, T, false>),
                                   dim3(grid_for((f1 - f0) * TEAM, block)), dim3(block), lds, st, f0, f1, dm->n_face,
                                   dm->n_elem, dm->face_lr, dm->face_code, dm->face_geo, dm->tables + ti.off_trace,
                                   dm->tables + ti.off_proj, ti.n_codes, U, rhs, buf, dm->xcd_remap);
        }
        return hip_check("surface kernel launch");
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
            default: return fail(DGC_E_ARG, "unknown surface variant");
        }
    }
};

template <class T, class F>
dgc_status dispatch(const dgc_dmesh *dm, F &&f) {
    if (dm->elem_type == DGC_TRI) {
        switch (dm->p) {
            case 0: return f(Impl<2, 1, 1, 1, T>{});
            case 1: return f(Impl<2, 3, 2, 4, T>{});
            case 2: return f(Impl<2, 6, 3, 9, T>{});
            case 3: return f(Impl<2, 10, 4, 16, T>{});
            default: break;
        }
    } else if (dm->elem_type == DGC_TET) {
        switch (dm->p) {
            case 0: return f(Impl<3, 1, 3, 1, T>{});
            case 1: return f(Impl<3, 4, 3, 8, T>{});
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
        return dispatch<double>(dm, [&](auto impl) {
            return decltype(impl)::volume(dm, ti, static_cast<const double *>(U), static_cast<double *>(rhs), st);
        });
    if (precision == DGC_F32)
        return dispatch<float>(dm, [&](auto impl) {
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
        return dispatch<double>(dm, [&](auto impl) {
            return decltype(impl)::surface(dm, ti, static_cast<const double *>(U), static_cast<double *>(rhs), variant,
                                           ws, ws_bytes, st);
        });
    if (precision == DGC_F32)
        return dispatch<float>(dm, [&](auto impl) {
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
    if (variant < DGC_SURF_COLORED || variant > DGC_SURF_GATHER) return fail(DGC_E_ARG, "unknown variant");
    const size_t elt = precision == DGC_F64 ? 8 : 4;
    const size_t rec = rec_bytes(dm, elt);
    const size_t surf = variant == DGC_SURF_GATHER ? 2 * (size_t)dm->n_face * rec : 0;
    if (what == DGC_WS_SURFACE) {
        *bytes = surf;
        return DGC_OK;
    }
    if (what == DGC_WS_RK_STEP) {
        const size_t n = (size_t)dm->n_elem * dm->n_var * dm->n_p;
        size_t b = 2 * n * 8 + n * elt;  // U1, U2 (f64) + rhs
        if (precision == DGC_F32) b += n * 4;  // f32 shadow of the stage state
        b = (b + 255) & ~(size_t)255;
        *bytes = b + surf;
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
    double *U1 = reinterpret_cast<double *>(w);
    double *U2 = U1 + n;
    const size_t elt = precision == DGC_F64 ? 8 : 4;
    void *rhs = U2 + n;
    float *shadow = precision == DGC_F32 ? reinterpret_cast<float *>(static_cast<char *>(rhs) + n * elt) : nullptr;
    size_t base = 2 * n * 8 + n * elt + (shadow ? n * 4 : 0);
    base = (base + 255) & ~(size_t)255;
    void *sws = w + base;
    size_t sws_bytes = ws_bytes - base;

    const double a[3] = {0.0, 0.75, 1.0 / 3.0};
    const double b[3] = {1.0, 0.25, 2.0 / 3.0};
    const double *x_in[3] = {U, U, U};
    const double *stage_in[3] = {U, U1, U2};
    double *stage_out[3] = {U1, U2, U};
    if (shadow) {
        hipLaunchKernelGGL(dgc_dev::to_f32_kernel, dim3(grid_for((int64_t)n)), dim3(kBlock), 0, st, (int64_t)n, U, shadow);
        if ((s = hip_check("f32 shadow launch")) != DGC_OK) return s;
    }
    for (int stg = 0; stg < 3; ++stg) {
        const void *Uin = shadow ? static_cast<const void *>(shadow) : static_cast<const void *>(stage_in[stg]);
        if ((s = dgc_volume_rhs(dm, Uin, rhs, precision, stream)) != DGC_OK) return s;
        if ((s = dgc_surface_rhs(dm, Uin, rhs, variant, precision, sws, sws_bytes, stream)) != DGC_OK) return s;
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

}  // extern "C"
