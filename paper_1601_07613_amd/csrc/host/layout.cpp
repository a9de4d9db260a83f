// Color-driven element renumbering and face reordering (Section 5).
//
// 1. faces are grouped by color, original order inside a color;
// 2. the k-th face of the first color gets left element k and right element
//    N_1 + k (Table 5b); interior faces of that color come first so that the
//    numbering stays dense, boundary faces after them;
// 3. faces of later colors are sorted by ascending new left element
//    (Table 6b), without exchanging left and right.
// On meshes where an element can miss a color (refined meshes), colors are
// processed in order and each one first numbers its still-unnumbered left
// elements, then its still-unnumbered right elements, before its sort.
//
// DGC_LAYOUT_PAPER_SFC (an extension, not in the paper): before step 2 the
// faces of the first color are put in Morton (Z-curve) order of their
// midpoints, interior faces still first.  Neighbouring pairs of the first
// color then get neighbouring ids, so the right elements met by the later
// colors lie close in memory to their left elements.
//
// DGC_LAYOUT_PAIRED (an extension, not in the paper): the first color's
// interior faces in Morton order as above, taken in blocks of kPairBlock;
// block b of n faces numbers its left elements 2 kPairBlock b + i and its
// right elements 2 kPairBlock b + n + i (i < n), so a wave of face teams
// still reads one contiguous run of left records and one of right records,
// while the two elements of a face get ids at most 2 kPairBlock apart; its
// boundary faces' left elements follow; later colors as in
// DGC_LAYOUT_PAPER.  Spatial neighbours then get close ids on both sides of
// every color, and the scattered right-element records of the later colors
// share their cache lines with records read at about the same time.
#include <algorithm>
#include <cmath>

#include "internal.hpp"

namespace dgc {

namespace {

// first-color faces per block of the DGC_LAYOUT_PAIRED numbering: the faces
// of one wave of four-lane face teams
constexpr int kPairBlock = 16;

// Morton code of each listed face's midpoint (taken from its left element's
// coordinates), quantised on the bounding box of those midpoints.
std::vector<uint64_t> morton_codes(const Mesh &m, const std::vector<int32_t> &faces) {
    const int dim = m.dim, nfv = dim;
    const int bits = dim == 2 ? 31 : 21;
    const double scale = std::ldexp(1.0, bits);
    std::vector<double> mid(faces.size() * dim);
    double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
    for (size_t i = 0; i < faces.size(); ++i) {
        const int32_t f = faces[i];
        const double *x = &m.elem_xyz[(int64_t)m.face_L[f] * m.nv * dim];
        for (int d = 0; d < dim; ++d) {
            double s = 0.0;
            for (int a = 0; a < nfv; ++a) s += x[face_vertex(m, m.face_L[f], m.face_fL[f], a) * dim + d];
            const double v = s / nfv;
            mid[i * dim + d] = v;
            if (i == 0 || v < lo[d]) lo[d] = v;
            if (i == 0 || v > hi[d]) hi[d] = v;
        }
    }
    std::vector<uint64_t> code(faces.size(), 0);
    for (size_t i = 0; i < faces.size(); ++i) {
        uint64_t c = 0;
        for (int d = 0; d < dim; ++d) {
            const double ext = hi[d] > lo[d] ? hi[d] - lo[d] : 1.0;
            const double t = (mid[i * dim + d] - lo[d]) / ext * scale;
            uint64_t q = t >= scale ? (uint64_t)scale - 1 : (t > 0 ? (uint64_t)t : 0);
            for (int b = 0; b < bits; ++b) c |= ((q >> b) & 1ull) << (b * dim + d);
        }
        code[i] = c;
    }
    return code;
}

void sort_by_morton(const Mesh &m, std::vector<int32_t> &faces) {
    std::vector<uint64_t> code = morton_codes(m, faces);
    std::vector<size_t> idx(faces.size());
    for (size_t i = 0; i < idx.size(); ++i) idx[i] = i;
    std::sort(idx.begin(), idx.end(), [&](size_t a, size_t b) {
        if (code[a] != code[b]) return code[a] < code[b];
        return faces[a] < faces[b];
    });
    std::vector<int32_t> out(faces.size());
    for (size_t i = 0; i < idx.size(); ++i) out[i] = faces[idx[i]];
    faces.swap(out);
}

}  // namespace

dgc_status make_layout(Mesh &m, uint32_t flag) {
    const int nc = m.n_colors;
    if (nc <= 0) return fail(DGC_E_NOT_COLORED, "mesh is not colored");
    const bool renumber = flag != DGC_LAYOUT_NONE;
    const bool reorder = flag == DGC_LAYOUT_PAPER || flag == DGC_LAYOUT_PAPER_SFC || flag == DGC_LAYOUT_PAIRED;
    const bool morton = flag == DGC_LAYOUT_PAPER_SFC || flag == DGC_LAYOUT_PAIRED;

    std::vector<std::vector<int32_t>> groups(nc);
    for (int64_t f = 0; f < m.E; ++f) groups[m.color[f]].push_back((int32_t)f);
    if (renumber) {
        std::vector<int32_t> &g0 = groups[0];
        if (morton) {
            std::vector<int32_t> in, bd;
            for (int32_t f : g0) (m.face_R[f] >= 0 ? in : bd).push_back(f);
            sort_by_morton(m, in);
            sort_by_morton(m, bd);
            g0 = in;
            g0.insert(g0.end(), bd.begin(), bd.end());
        } else {
            std::stable_partition(g0.begin(), g0.end(), [&](int32_t f) { return m.face_R[f] >= 0; });
        }
    }

    m.elem_new.assign(m.K, -1);
    if (!renumber) {
        for (int64_t i = 0; i < m.K; ++i) m.elem_new[i] = (int32_t)i;
    } else {
        int32_t next = 0;
        for (int c = 0; c < nc; ++c) {
            if (c == 0 && flag == DGC_LAYOUT_PAIRED) {
                // no element is numbered yet, and the faces of one color
                // share no element; interior faces come first in groups[0]
                const std::vector<int32_t> &g = groups[0];
                size_t n_in = 0;
                while (n_in < g.size() && m.face_R[g[n_in]] >= 0) ++n_in;
                for (size_t b0 = 0; b0 < n_in; b0 += kPairBlock) {
                    const size_t n = std::min(n_in - b0, (size_t)kPairBlock);
                    for (size_t i = 0; i < n; ++i) m.elem_new[m.face_L[g[b0 + i]]] = next + (int32_t)i;
                    for (size_t i = 0; i < n; ++i) m.elem_new[m.face_R[g[b0 + i]]] = next + (int32_t)(n + i);
                    next += (int32_t)(2 * n);
                }
                for (size_t i = n_in; i < g.size(); ++i) m.elem_new[m.face_L[g[i]]] = next++;
                continue;
            }
            for (int32_t f : groups[c]) {
                int32_t e = m.face_L[f];
                if (m.elem_new[e] < 0) m.elem_new[e] = next++;
            }
            for (int32_t f : groups[c]) {
                int32_t e = m.face_R[f];
                if (e >= 0 && m.elem_new[e] < 0) m.elem_new[e] = next++;
            }
        }
        if (next != m.K) return fail(DGC_E_MESH, "an element has no face");
    }

    m.face_order.clear();
    m.face_order.reserve(m.E);
    m.color_off.assign(nc + 1, 0);
    for (int c = 0; c < nc; ++c) {
        std::vector<int32_t> &g = groups[c];
        if (reorder && c > 0) {
            std::sort(g.begin(), g.end(),
                      [&](int32_t a, int32_t b) { return m.elem_new[m.face_L[a]] < m.elem_new[m.face_L[b]]; });
        }
        m.face_order.insert(m.face_order.end(), g.begin(), g.end());
        m.color_off[c + 1] = (int64_t)m.face_order.size();
    }
    m.laid_out = true;
    return DGC_OK;
}

}  // namespace dgc
