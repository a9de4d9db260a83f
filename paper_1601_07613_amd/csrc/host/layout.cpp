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
#include <algorithm>

#include "internal.hpp"

namespace dgc {

dgc_status make_layout(Mesh &m, uint32_t flag) {
    const int nc = m.n_colors;
    if (nc <= 0) return fail(DGC_E_NOT_COLORED, "mesh is not colored");
    const bool renumber = flag != DGC_LAYOUT_NONE;
    const bool reorder = flag == DGC_LAYOUT_PAPER;

    std::vector<std::vector<int32_t>> groups(nc);
    for (int64_t f = 0; f < m.E; ++f) groups[m.color[f]].push_back((int32_t)f);
    if (renumber) {
        std::vector<int32_t> &g0 = groups[0];
        std::stable_partition(g0.begin(), g0.end(), [&](int32_t f) { return m.face_R[f] >= 0; });
    }

    m.elem_new.assign(m.K, -1);
    if (!renumber) {
        for (int64_t i = 0; i < m.K; ++i) m.elem_new[i] = (int32_t)i;
    } else {
        int32_t next = 0;
        for (int c = 0; c < nc; ++c) {
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
