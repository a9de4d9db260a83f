// Host entry points of the C ABI: mesh construction, coloring, layout,
// export of host and device-ready arrays, tables, error reporting.
#include <chrono>
#include <cmath>
#include <cstring>
#include <new>

#include "internal.hpp"

namespace dgc {

namespace {
thread_local std::string g_err;
}

void set_error(const std::string &msg) { g_err = msg; }

dgc_status fail(dgc_status code, const std::string &msg) {
    g_err = msg;
    return code;
}

}  // namespace dgc

using dgc::fail;

extern "C" {

const char *dgc_last_error(void) { return dgc::g_err.c_str(); }

const char *dgc_version(void) { return "dgc 0.1 (gfx950)"; }

dgc_status dgc_mesh_build(int32_t elem_type, int64_t n_elem, const int32_t *elem_vert, const double *elem_xyz,
                          dgc_mesh **out) {
    if (!out || !elem_vert || !elem_xyz || n_elem <= 0) return fail(DGC_E_ARG, "dgc_mesh_build: bad argument");
    if (elem_type != DGC_TRI && elem_type != DGC_QUAD && elem_type != DGC_TET && elem_type != DGC_MIXED)
        return fail(DGC_E_ARG, "dgc_mesh_build: unknown element type");
    if (n_elem > (int64_t)1 << 30) return fail(DGC_E_ARG, "dgc_mesh_build: too many elements");
    *out = nullptr;
    try {
        dgc_mesh *h = new dgc_mesh();
        dgc::Mesh &m = h->m;
        m.elem_type = elem_type;
        m.dim = elem_type == DGC_TET ? 3 : 2;
        m.nv = elem_type == DGC_TRI ? 3 : 4;
        m.F = m.nv;
        m.n_orient = m.dim == 2 ? 4 : 6;
        m.K = n_elem;
        m.elem_vert.assign(elem_vert, elem_vert + n_elem * m.nv);
        m.elem_xyz.assign(elem_xyz, elem_xyz + n_elem * m.nv * m.dim);
        m.elem_level.assign(n_elem, 0);
        m.n_vert = 0;
        if (elem_type == DGC_MIXED) {
            // the fourth vertex id -1 marks a triangle
            m.elem_kind.resize(n_elem);
            for (int64_t i = 0; i < n_elem; ++i) m.elem_kind[i] = m.elem_vert[i * 4 + 3] >= 0 ? 1 : 0;
        }
        for (int64_t i = 0; i < n_elem * m.nv; ++i) {
            if (elem_type == DGC_MIXED && i % 4 == 3 && m.elem_kind[i / 4] == 0) continue;
            if (m.elem_vert[i] < 0) {
                delete h;
                return fail(DGC_E_ARG, "dgc_mesh_build: negative vertex id");
            }
            if (m.elem_vert[i] + 1 > m.n_vert) m.n_vert = m.elem_vert[i] + 1;
        }
        dgc_status s = dgc::build_faces(m);
        if (s != DGC_OK) {
            delete h;
            return s;
        }
        *out = h;
        return DGC_OK;
    } catch (const std::bad_alloc &) {
        return fail(DGC_E_ALLOC, "dgc_mesh_build: out of host memory");
    }
}

void dgc_mesh_free(dgc_mesh *m) { delete m; }

dgc_status dgc_color_edges(dgc_mesh *h, uint64_t seed, int64_t max_swaps, uint32_t flags, dgc_color_stats *stats) {
    if (!h) return fail(DGC_E_ARG, "dgc_color_edges: null mesh");
    dgc::Mesh &m = h->m;
    if (m.has_tree()) return fail(DGC_E_UNSUPPORTED, "refined meshes are colored by dgc_mesh_refine");
    uint32_t alg = flags & 0x0Fu, lay = flags & 0xFF0u;
    if (lay == 0) lay = DGC_LAYOUT_PAPER;
    if (alg == 0) alg = DGC_COLOR_PAPER;
    if ((alg != DGC_COLOR_PAPER && alg != DGC_COLOR_GREEDY_STD) ||
        (lay != DGC_LAYOUT_PAPER && lay != DGC_LAYOUT_RENUMBER && lay != DGC_LAYOUT_NONE &&
         lay != DGC_LAYOUT_PAPER_SFC && lay != DGC_LAYOUT_PAIRED))
        return fail(DGC_E_ARG, "dgc_color_edges: bad flags");
    try {
        dgc_color_stats st{};
        auto t0 = std::chrono::steady_clock::now();
        std::vector<int8_t> saved = m.color;
        int saved_n = m.n_colors;
        dgc_status s = alg == DGC_COLOR_PAPER ? dgc::color_paper(m, seed, max_swaps, &st) : dgc::color_greedy_std(m, &st);
        auto t1 = std::chrono::steady_clock::now();
        if (s != DGC_OK) {
            m.color = saved;
            m.n_colors = saved_n;
            if (stats) *stats = st;
            return s;
        }
        std::string why;
        if (!dgc::coloring_valid(m, m.color, &why)) return fail(DGC_E_COLORING_INVALID, "internal: " + why);
        s = dgc::make_layout(m, lay);
        auto t2 = std::chrono::steady_clock::now();
        st.color_ms = std::chrono::duration<double, std::milli>(t1 - t0).count();
        st.layout_ms = std::chrono::duration<double, std::milli>(t2 - t1).count();
        if (stats) *stats = st;
        return s;
    } catch (const std::bad_alloc &) {
        return fail(DGC_E_ALLOC, "dgc_color_edges: out of host memory");
    }
}

dgc_status dgc_set_colors(dgc_mesh *h, const int8_t *colors, uint32_t layout_flags) {
    if (!h || !colors) return fail(DGC_E_ARG, "dgc_set_colors: null argument");
    dgc::Mesh &m = h->m;
    uint32_t lay = layout_flags & 0xFF0u;
    if (lay == 0) lay = DGC_LAYOUT_PAPER;
    if (lay != DGC_LAYOUT_PAPER && lay != DGC_LAYOUT_RENUMBER && lay != DGC_LAYOUT_NONE &&
        lay != DGC_LAYOUT_PAPER_SFC && lay != DGC_LAYOUT_PAIRED)
        return fail(DGC_E_ARG, "dgc_set_colors: bad layout flag");
    std::vector<int8_t> c(colors, colors + m.E);
    std::string why;
    if (!dgc::coloring_valid(m, c, &why)) return fail(DGC_E_COLORING_INVALID, "dgc_set_colors: " + why);
    int nc = 0;
    for (int8_t x : c) nc = x + 1 > nc ? x + 1 : nc;
    m.color.swap(c);
    m.n_colors = nc;
    return dgc::make_layout(m, lay);
}

dgc_status dgc_mesh_info(const dgc_mesh *h, dgc_mesh_info_t *info) {
    if (!h || !info) return fail(DGC_E_ARG, "dgc_mesh_info: null argument");
    const dgc::Mesh &m = h->m;
    dgc_mesh_info_t r{};
    r.elem_type = m.elem_type;
    r.dim = m.dim;
    r.n_vert_per_elem = m.nv;
    r.n_face_per_elem = m.F;
    r.max_slots = m.max_slots;
    r.n_colors = m.laid_out ? m.n_colors : 0;
    r.n_elem = m.K;
    r.n_face = m.E;
    r.n_boundary = m.n_boundary;
    if (m.laid_out)
        for (int c = 0; c <= m.n_colors; ++c) r.color_off[c] = m.color_off[c];
    r.n_orient = m.n_orient;
    r.max_level = m.max_level;
    *info = r;
    return DGC_OK;
}

}  // extern "C"

namespace {

template <class T>
dgc_status copy_out(const std::vector<T> &v, void *dst, size_t bytes, size_t *needed) {
    size_t nb = v.size() * sizeof(T);
    if (needed) *needed = nb;
    if (!dst) return DGC_OK;
    if (bytes < nb) return fail(DGC_E_ARG, "dgc_mesh_export: destination too small");
    if (nb) std::memcpy(dst, v.data(), nb);
    return DGC_OK;
}

}  // namespace

extern "C" {

dgc_status dgc_mesh_export(const dgc_mesh *h, int32_t which, void *dst, size_t bytes, size_t *needed) {
    if (!h) return fail(DGC_E_ARG, "dgc_mesh_export: null mesh");
    const dgc::Mesh &m = h->m;
    const int64_t E = m.E, K = m.K;
    const int dim = m.dim;
    const bool layout_arr = which >= 10 && which < 30;
    if (layout_arr && !m.laid_out) return fail(DGC_E_NOT_COLORED, "dgc_mesh_export: mesh is not colored");
    try {
        switch (which) {
            case DGC_ARR_FACE_ELEM: {
                std::vector<int32_t> v(2 * E);
                for (int64_t f = 0; f < E; ++f) { v[2 * f] = m.face_L[f]; v[2 * f + 1] = m.face_R[f]; }
                return copy_out(v, dst, bytes, needed);
            }
            case DGC_ARR_FACE_LOCAL: {
                std::vector<int8_t> v(2 * E);
                for (int64_t f = 0; f < E; ++f) { v[2 * f] = m.face_fL[f]; v[2 * f + 1] = m.face_fR[f]; }
                return copy_out(v, dst, bytes, needed);
            }
            case DGC_ARR_COLOR: return copy_out(m.color, dst, bytes, needed);
            case DGC_ARR_FACE_NORMAL: return copy_out(m.normal, dst, bytes, needed);
            case DGC_ARR_FACE_MEASURE: return copy_out(m.measure, dst, bytes, needed);
            case DGC_ARR_ELEM_DETJ: return copy_out(m.detJ, dst, bytes, needed);
            case DGC_ARR_ELEM_FACE: return copy_out(m.elem_face, dst, bytes, needed);
            case DGC_ARR_ELEM_NEW: return copy_out(m.elem_new, dst, bytes, needed);
            case DGC_ARR_FACE_ORDER: return copy_out(m.face_order, dst, bytes, needed);
            case DGC_ARR_COLOR_OFF: return copy_out(m.color_off, dst, bytes, needed);
            case DGC_ARR_ELEM_LEVEL: return copy_out(m.elem_level, dst, bytes, needed);
            case DGC_ARR_ELEM_XYZ: return copy_out(m.elem_xyz, dst, bytes, needed);
            case DGC_ARR_ELEM_VERT: return copy_out(m.elem_vert, dst, bytes, needed);
            case DGC_ARR_DEV_ELEM_KIND: {
                if (m.elem_type != DGC_MIXED) return fail(DGC_E_ARG, "dgc_mesh_export: not a mixed mesh");
                std::vector<int8_t> v(K);
                for (int64_t i = 0; i < K; ++i) v[m.elem_new[i]] = m.elem_kind[i];
                return copy_out(v, dst, bytes, needed);
            }
            case DGC_ARR_ADAPT_KIND:
            case DGC_ARR_ADAPT_SRC:
            case DGC_ARR_DEV_ADAPT_KIND:
            case DGC_ARR_DEV_ADAPT_SRC: {
                if (m.adapt_kind.size() != (size_t)K)
                    return fail(DGC_E_ARG, "dgc_mesh_export: mesh was not made by dgc_mesh_refine / dgc_mesh_coarsen");
                if (which == DGC_ARR_ADAPT_KIND) return copy_out(m.adapt_kind, dst, bytes, needed);
                if (which == DGC_ARR_ADAPT_SRC) return copy_out(m.adapt_src, dst, bytes, needed);
                if (which == DGC_ARR_DEV_ADAPT_KIND) {
                    std::vector<int8_t> v(K);
                    for (int64_t i = 0; i < K; ++i) v[m.elem_new[i]] = m.adapt_kind[i];
                    return copy_out(v, dst, bytes, needed);
                }
                std::vector<int32_t> v(4 * K, -1);
                for (int64_t i = 0; i < K; ++i)
                    for (int a = 0; a < 4; ++a) {
                        const int32_t s = m.adapt_src[i * 4 + a];
                        v[a * K + m.elem_new[i]] = s >= 0 ? m.prev_elem_new[s] : -1;
                    }
                return copy_out(v, dst, bytes, needed);
            }
            case DGC_ARR_DEV_FACE_LR: {
                std::vector<int32_t> v(2 * E);
                for (int64_t k = 0; k < E; ++k) {
                    int32_t f = m.face_order[k];
                    v[k] = m.elem_new[m.face_L[f]];
                    v[E + k] = m.face_R[f] >= 0 ? m.elem_new[m.face_R[f]] : -1;
                }
                return copy_out(v, dst, bytes, needed);
            }
            case DGC_ARR_DEV_FACE_CODE: {
                std::vector<uint8_t> v(2 * E);
                for (int64_t k = 0; k < E; ++k) {
                    int32_t f = m.face_order[k];
                    // mixed meshes: the quadrilateral's codes follow the triangle's 3 faces
                    const int offL = m.elem_type == DGC_MIXED && m.elem_kind[m.face_L[f]] ? 3 * m.n_orient : 0;
                    v[k] = (uint8_t)(offL + m.face_fL[f] * m.n_orient + m.face_oL[f]);
                    if (m.face_R[f] >= 0) {
                        const int offR = m.elem_type == DGC_MIXED && m.elem_kind[m.face_R[f]] ? 3 * m.n_orient : 0;
                        v[E + k] = (uint8_t)(offR + m.face_fR[f] * m.n_orient + m.face_oR[f]);
                    } else {
                        v[E + k] = 0;
                    }
                }
                return copy_out(v, dst, bytes, needed);
            }
            case DGC_ARR_DEV_FACE_GEO: {
                std::vector<double> v((dim + 3) * E);
                for (int64_t k = 0; k < E; ++k) {
                    int32_t f = m.face_order[k];
                    for (int d = 0; d < dim; ++d) v[d * E + k] = m.normal[f * dim + d];
                    v[dim * E + k] = m.measure[f];
                    v[(dim + 1) * E + k] = 1.0 / std::sqrt(m.detJ[m.face_L[f]]);
                    v[(dim + 2) * E + k] = m.face_R[f] >= 0 ? 1.0 / std::sqrt(m.detJ[m.face_R[f]]) : 0.0;
                }
                return copy_out(v, dst, bytes, needed);
            }
            case DGC_ARR_DEV_ELEM_GEO: {
                const int G = dim * dim + 1;
                std::vector<double> v(G * K);
                for (int64_t i = 0; i < K; ++i) {
                    int64_t k = m.elem_new[i];
                    for (int a = 0; a < dim * dim; ++a) v[a * K + k] = m.Jinv[i * dim * dim + a];
                    v[dim * dim * K + k] = std::sqrt(m.detJ[i]);
                }
                return copy_out(v, dst, bytes, needed);
            }
            case DGC_ARR_DEV_ELEM_SLOTS: {
                const int S = m.max_slots;
                std::vector<int32_t> v((size_t)S * K, -1);
                std::vector<int32_t> pos(E);
                for (int64_t k = 0; k < E; ++k) pos[m.face_order[k]] = (int32_t)k;
                std::vector<int> fill(K, 0);
                for (int64_t k = 0; k < E; ++k) {
                    int32_t f = m.face_order[k];
                    int32_t l = m.elem_new[m.face_L[f]];
                    v[(size_t)fill[l]++ * K + l] = (int32_t)(2 * k);
                    if (m.face_R[f] >= 0) {
                        int32_t r = m.elem_new[m.face_R[f]];
                        v[(size_t)fill[r]++ * K + r] = (int32_t)(2 * k + 1);
                    }
                }
                return copy_out(v, dst, bytes, needed);
            }
            default: return fail(DGC_E_ARG, "dgc_mesh_export: unknown array " + std::to_string(which));
        }
    } catch (const std::bad_alloc &) {
        return fail(DGC_E_ALLOC, "dgc_mesh_export: out of host memory");
    }
}

dgc_status dgc_tables(int32_t elem_type, int32_t p, dgc_table_info *info, double *dst, size_t bytes, size_t *needed) {
    dgc_table_info ti{};
    dgc_status s = dgc::build_tables(elem_type, p, &ti, nullptr);
    if (s != DGC_OK) return s;
    if (info) *info = ti;
    size_t nb = (size_t)ti.total * sizeof(double);
    if (needed) *needed = nb;
    if (!dst) return DGC_OK;
    if (bytes < nb) return fail(DGC_E_ARG, "dgc_tables: destination too small");
    std::vector<double> v;
    s = dgc::build_tables(elem_type, p, &ti, &v);
    if (s != DGC_OK) return s;
    std::memcpy(dst, v.data(), nb);
    return DGC_OK;
}

}  // extern "C"
