// Nonconforming refinement of triangle meshes and the six-color map of
// Section 3.2.
//
// A flagged leaf is split into four by its edge midpoints: corner children
// (v0,m01,m20), (m01,v1,m12), (m20,m12,v2) and the center child
// (m12,m20,m01), whose local edge k is parallel to parent edge k.  Coarser
// edge-neighbours of a split leaf are split first (2:1 closure), so a leaf
// edge faces either one leaf of the same level, one coarser leaf (a hanging
// half edge) or two finer leaves.  Edges form a tree: an edge of color c
// splits into a first child (the half at the edge's recorded start vertex)
// of color c and a second child of color (c + 3) mod 6; an interior edge
// takes the color of the parent edge it is parallel to.  The recorded
// orientation makes both sides of an edge agree on which half is "first":
// base edges are oriented counter-clockwise for their left element, children
// inherit it, interior edges are oriented counter-clockwise for the center
// child.
//
// Faces of the refined mesh are the unsplit edges referenced by a leaf; they
// are numbered by first visit scanning leaves and local edges (a split local
// edge visits its two halves).  The coarse side of a hanging face is its
// right element (orientation code 2 / 3: first / second half of its edge,
// traversed in reverse); otherwise the first visitor is the left element.
#include <deque>

#include "internal.hpp"

namespace dgc {

namespace {

using Node = Mesh::EdgeNode;

// Edge tree of a colored conforming triangle mesh: node f = face f.
void base_tree(const Mesh &b, std::vector<Node> &nodes, std::vector<int32_t> &leaf_edge) {
    nodes.resize(b.E);
    for (int64_t f = 0; f < b.E; ++f) {
        const int32_t L = b.face_L[f];
        const int k = b.face_fL[f];
        nodes[f] = {b.elem_vert[(int64_t)L * 3 + k], b.elem_vert[(int64_t)L * 3 + (k + 1) % 3], b.color[f], -1, -1, -1,
                    -1};
    }
    leaf_edge.resize(b.K * 3);
    for (int64_t i = 0; i < b.K; ++i)
        for (int k = 0; k < 3; ++k) leaf_edge[i * 3 + k] = b.elem_face[i * b.max_slots + k];
}

int32_t half_of(const std::vector<Node> &nodes, int32_t e, int32_t a, int32_t b) {
    for (int32_t ch : {nodes[e].child0, nodes[e].child1}) {
        const Node &n = nodes[ch];
        if ((n.start == a && n.end == b) || (n.start == b && n.end == a)) return ch;
    }
    return -1;
}

}  // namespace

}  // namespace dgc

using dgc::fail;

extern "C" dgc_status dgc_mesh_refine(const dgc_mesh *parent, const uint8_t *flags, dgc_mesh **out,
                                      int64_t *n_closure) {
    using Node = dgc::Mesh::EdgeNode;
    if (out) *out = nullptr;
    if (!parent || !flags || !out) return fail(DGC_E_ARG, "dgc_mesh_refine: null argument");
    const dgc::Mesh &P = parent->m;
    if (P.elem_type != DGC_TRI) return fail(DGC_E_UNSUPPORTED, "dgc_mesh_refine: triangles only");
    if (!P.laid_out || P.n_colors <= 0) return fail(DGC_E_NOT_COLORED, "dgc_mesh_refine: parent is not colored");
    if (P.max_level == 0 && P.n_colors > 3)
        return fail(DGC_E_ARG, "dgc_mesh_refine: the conforming base needs a 3-coloring");
    try {
        std::vector<Node> nodes;
        std::vector<int32_t> pedge;
        int64_t n_vert = P.n_vert;
        if (P.max_level == 0) {
            dgc::base_tree(P, nodes, pedge);
        } else {
            nodes = P.nodes;
            pedge = P.leaf_edge;
        }
        const int64_t K0 = P.K;

        // leaves referencing each node (at most two)
        std::vector<int32_t> refA(nodes.size(), -1), refB(nodes.size(), -1);
        for (int64_t i = 0; i < K0; ++i)
            for (int k = 0; k < 3; ++k) {
                int32_t e = pedge[i * 3 + k];
                (refA[e] < 0 ? refA[e] : refB[e]) = (int32_t)i;
            }

        // 2:1 closure
        std::vector<uint8_t> split(K0, 0);
        std::deque<int64_t> work;
        int64_t n_flag = 0;
        for (int64_t i = 0; i < K0; ++i)
            if (flags[i]) {
                split[i] = 1;
                work.push_back(i);
                ++n_flag;
            }
        while (!work.empty()) {
            int64_t i = work.front();
            work.pop_front();
            for (int k = 0; k < 3; ++k) {
                const Node &n = nodes[pedge[i * 3 + k]];
                if (n.child0 >= 0 || n.parent < 0) continue;
                for (int32_t j : {refA[n.parent], refB[n.parent]}) {
                    if (j >= 0 && P.elem_level[j] < P.elem_level[i] && !split[j]) {
                        split[j] = 1;
                        work.push_back(j);
                    }
                }
            }
        }
        int64_t n_split = 0;
        for (int64_t i = 0; i < K0; ++i) n_split += split[i];
        if (n_closure) *n_closure = n_split - n_flag;

        // split the edges of split leaves: new vertex ids in order of need
        for (int64_t i = 0; i < K0; ++i) {
            if (!split[i]) continue;
            for (int k = 0; k < 3; ++k) {
                const int32_t e = pedge[i * 3 + k];
                if (nodes[e].child0 >= 0) continue;
                const int32_t mid = (int32_t)n_vert++;
                const Node n = nodes[e];
                const int32_t c0 = (int32_t)nodes.size();
                nodes.push_back({n.start, mid, n.color, -1, -1, e, -1});
                nodes.push_back({mid, n.end, (n.color + 3) % 6, -1, -1, e, -1});
                nodes[e].child0 = c0;
                nodes[e].child1 = c0 + 1;
                nodes[e].mid = mid;
            }
        }

        // new leaf list: children replace their parent
        dgc_mesh *h = new dgc_mesh();
        dgc::Mesh &m = h->m;
        m.elem_type = DGC_TRI;
        m.dim = 2;
        m.nv = 3;
        m.F = 3;
        m.n_orient = 4;
        const int64_t K = K0 + 3 * n_split;
        m.K = K;
        m.elem_vert.reserve(K * 3);
        m.elem_xyz.reserve(K * 6);
        m.elem_level.reserve(K);
        m.leaf_edge.reserve(K * 3);
        auto add_leaf = [&](int32_t a, int32_t b, int32_t c, const double *xa, const double *xb, const double *xc,
                            int lvl, int32_t e0, int32_t e1, int32_t e2) {
            m.elem_vert.insert(m.elem_vert.end(), {a, b, c});
            m.elem_xyz.insert(m.elem_xyz.end(), {xa[0], xa[1], xb[0], xb[1], xc[0], xc[1]});
            m.elem_level.push_back((int8_t)lvl);
            m.leaf_edge.insert(m.leaf_edge.end(), {e0, e1, e2});
        };
        for (int64_t i = 0; i < K0; ++i) {
            const int32_t *v = &P.elem_vert[i * 3];
            const double *x = &P.elem_xyz[i * 6];
            const int lvl = P.elem_level[i];
            const int32_t E0 = pedge[i * 3], E1 = pedge[i * 3 + 1], E2 = pedge[i * 3 + 2];
            if (!split[i]) {
                add_leaf(v[0], v[1], v[2], x, x + 2, x + 4, lvl, E0, E1, E2);
                continue;
            }
            const int32_t m01 = nodes[E0].mid, m12 = nodes[E1].mid, m20 = nodes[E2].mid;
            const double x01[2] = {0.5 * (x[0] + x[2]), 0.5 * (x[1] + x[3])};
            const double x12[2] = {0.5 * (x[2] + x[4]), 0.5 * (x[3] + x[5])};
            const double x20[2] = {0.5 * (x[4] + x[0]), 0.5 * (x[5] + x[1])};
            const int32_t I0 = (int32_t)nodes.size();
            nodes.push_back({m12, m20, nodes[E0].color, -1, -1, -1, -1});
            nodes.push_back({m20, m01, nodes[E1].color, -1, -1, -1, -1});
            nodes.push_back({m01, m12, nodes[E2].color, -1, -1, -1, -1});
            const int32_t I1 = I0 + 1, I2 = I0 + 2;
            add_leaf(v[0], m01, m20, x, x01, x20, lvl + 1, dgc::half_of(nodes, E0, v[0], m01), I1,
                     dgc::half_of(nodes, E2, m20, v[0]));
            add_leaf(m01, v[1], m12, x01, x + 2, x12, lvl + 1, dgc::half_of(nodes, E0, m01, v[1]),
                     dgc::half_of(nodes, E1, v[1], m12), I2);
            add_leaf(m20, m12, v[2], x20, x12, x + 4, lvl + 1, I0, dgc::half_of(nodes, E1, m12, v[2]),
                     dgc::half_of(nodes, E2, v[2], m20));
            add_leaf(m12, m20, m01, x12, x20, x01, lvl + 1, I0, I1, I2);
        }
        for (int32_t e : m.leaf_edge)
            if (e < 0) {
                delete h;
                return fail(DGC_E_MESH, "dgc_mesh_refine: internal edge-tree inconsistency");
            }
        m.nodes.swap(nodes);
        m.n_vert = n_vert;
        int maxl = 0;
        for (int8_t l : m.elem_level) maxl = l > maxl ? l : maxl;
        m.max_level = maxl;

        // faces: unsplit nodes referenced by leaves, in order of first visit
        std::vector<int32_t> face_of(m.nodes.size(), -1);
        struct FaceAcc { int32_t node; int32_t fine[2][2]; int nfine; int32_t coarse[3]; };
        std::vector<FaceAcc> acc;
        std::vector<std::vector<int32_t>> slots(K);
        auto visit = [&](int32_t node) {
            if (face_of[node] < 0) {
                face_of[node] = (int32_t)acc.size();
                acc.push_back({node, {{-1, -1}, {-1, -1}}, 0, {-1, -1, -1}});
            }
            return face_of[node];
        };
        for (int64_t i = 0; i < K; ++i) {
            for (int k = 0; k < 3; ++k) {
                const int32_t e = m.leaf_edge[i * 3 + k];
                const Node &n = m.nodes[e];
                if (n.child0 < 0) {
                    const int32_t f = visit(e);
                    FaceAcc &a = acc[f];
                    if (a.nfine >= 2) {
                        delete h;
                        return fail(DGC_E_MESH, "dgc_mesh_refine: an edge has more than two leaves");
                    }
                    a.fine[a.nfine][0] = (int32_t)i;
                    a.fine[a.nfine][1] = k;
                    ++a.nfine;
                    slots[i].push_back(f);
                } else {
                    const int32_t w0 = m.elem_vert[i * 3 + k];
                    for (int32_t ch : {n.child0, n.child1}) {
                        if (m.nodes[ch].child0 >= 0) {
                            delete h;
                            return fail(DGC_E_MESH, "dgc_mesh_refine: neighbours differ by more than one level");
                        }
                        const int32_t f = visit(ch);
                        const bool first = m.nodes[ch].start == w0 || m.nodes[ch].end == w0;
                        acc[f].coarse[0] = (int32_t)i;
                        acc[f].coarse[1] = k;
                        acc[f].coarse[2] = first ? 2 : 3;
                        slots[i].push_back(f);
                    }
                }
            }
        }
        const int64_t E = (int64_t)acc.size();
        m.E = E;
        m.face_L.resize(E); m.face_R.resize(E);
        m.face_fL.resize(E); m.face_fR.resize(E);
        m.face_oL.assign(E, 0); m.face_oR.assign(E, 0);
        m.color.resize(E);
        m.edge_start.resize(E);
        m.n_boundary = 0;
        for (int64_t f = 0; f < E; ++f) {
            const FaceAcc &a = acc[f];
            m.color[f] = (int8_t)m.nodes[a.node].color;
            m.edge_start[f] = m.nodes[a.node].start;
            m.face_L[f] = a.fine[0][0];
            m.face_fL[f] = (int8_t)a.fine[0][1];
            if (a.coarse[0] >= 0) {
                m.face_R[f] = a.coarse[0];
                m.face_fR[f] = (int8_t)a.coarse[1];
                m.face_oR[f] = (uint8_t)a.coarse[2];
            } else if (a.nfine == 2) {
                m.face_R[f] = a.fine[1][0];
                m.face_fR[f] = (int8_t)a.fine[1][1];
                m.face_oR[f] = 1;
            } else {
                m.face_R[f] = -1;
                m.face_fR[f] = -1;
                ++m.n_boundary;
            }
            if (m.face_L[f] < 0) {
                delete h;
                return fail(DGC_E_MESH, "dgc_mesh_refine: hanging face without a fine side");
            }
        }
        int ms = 0;
        for (const auto &s : slots) ms = (int)s.size() > ms ? (int)s.size() : ms;
        m.max_slots = ms;
        m.elem_face.assign(K * ms, -1);
        for (int64_t i = 0; i < K; ++i)
            for (size_t a = 0; a < slots[i].size(); ++a) m.elem_face[i * ms + a] = slots[i][a];

        dgc_status s = dgc::elem_geometry(m);
        if (s == DGC_OK) s = dgc::face_geometry(m);
        if (s != DGC_OK) {
            delete h;
            return s;
        }
        int nc = 0;
        for (int8_t c : m.color) nc = c + 1 > nc ? c + 1 : nc;
        m.n_colors = nc;
        std::string why;
        if (!dgc::coloring_valid(m, m.color, &why)) {
            delete h;
            return fail(DGC_E_COLORING_INVALID, "dgc_mesh_refine: " + why);
        }
        s = dgc::make_layout(m, DGC_LAYOUT_PAPER);
        if (s != DGC_OK) {
            delete h;
            return s;
        }
        *out = h;
        return DGC_OK;
    } catch (const std::bad_alloc &) {
        return fail(DGC_E_ALLOC, "dgc_mesh_refine: out of host memory");
    }
}
