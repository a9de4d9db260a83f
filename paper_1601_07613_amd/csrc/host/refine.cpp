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
//
// Coarsening is the inverse split: four leaves that are the children 0..3 of
// one element, all flagged and none with a split edge (which would leave a
// neighbour two levels finer), merge back into that element, which takes the
// place of its first child.  Its edges are the parent edges, which kept
// their colors, so the parent coloring comes back unchanged; a parent edge
// whose halves no leaf references any more is unsplit.  Every leaf records
// where it came from (same leaf, child k of a leaf, parent of four leaves)
// so that the solution can be moved to the new mesh.
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

// Faces, geometry, colors and layout of a leaf set.  m holds the leaves
// (elem_vert, elem_xyz, elem_level, leaf_edge) and the edge tree; faces are
// the unsplit nodes referenced by leaves, in order of first visit.
dgc_status finish_leaves(Mesh &m, const char *who) {
    const int64_t K = m.K;
    for (int32_t e : m.leaf_edge)
        if (e < 0) return fail(DGC_E_MESH, std::string(who) + ": internal edge-tree inconsistency");
    int maxl = 0;
    for (int8_t l : m.elem_level) maxl = l > maxl ? l : maxl;
    m.max_level = maxl;

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
                if (a.nfine >= 2) return fail(DGC_E_MESH, std::string(who) + ": an edge has more than two leaves");
                a.fine[a.nfine][0] = (int32_t)i;
                a.fine[a.nfine][1] = k;
                ++a.nfine;
                slots[i].push_back(f);
            } else {
                const int32_t w0 = m.elem_vert[i * 3 + k];
                for (int32_t ch : {n.child0, n.child1}) {
                    if (m.nodes[ch].child0 >= 0)
                        return fail(DGC_E_MESH, std::string(who) + ": neighbours differ by more than one level");
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
        if (m.face_L[f] < 0) return fail(DGC_E_MESH, std::string(who) + ": hanging face without a fine side");
    }
    int ms = 0;
    for (const auto &sl : slots) ms = (int)sl.size() > ms ? (int)sl.size() : ms;
    m.max_slots = ms;
    m.elem_face.assign(K * ms, -1);
    for (int64_t i = 0; i < K; ++i)
        for (size_t a = 0; a < slots[i].size(); ++a) m.elem_face[i * ms + a] = slots[i][a];

    dgc_status st = elem_geometry(m);
    if (st == DGC_OK) st = face_geometry(m);
    if (st != DGC_OK) return st;
    int nc = 0;
    for (int8_t c : m.color) nc = c + 1 > nc ? c + 1 : nc;
    m.n_colors = nc;
    std::string why;
    if (!coloring_valid(m, m.color, &why)) return fail(DGC_E_COLORING_INVALID, std::string(who) + ": " + why);
    return make_layout(m, DGC_LAYOUT_PAPER);
}

// The tree of P, or a fresh one (one node per face, base leaves) for a
// conforming mesh.
void start_tree(const Mesh &P, std::vector<Node> &nodes, std::vector<int32_t> &pedge, std::vector<int32_t> &pfam,
                std::vector<int8_t> &pchild, std::vector<Mesh::Family> &fams) {
    if (P.has_tree()) {
        nodes = P.nodes;
        pedge = P.leaf_edge;
        pfam = P.leaf_family;
        pchild = P.leaf_child;
        fams = P.families;
    } else {
        base_tree(P, nodes, pedge);
        pfam.assign(P.K, -1);
        pchild.assign(P.K, -1);
        fams.clear();
    }
}

dgc_mesh *new_tri_mesh(int64_t K) {
    dgc_mesh *h = new dgc_mesh();
    Mesh &m = h->m;
    m.elem_type = DGC_TRI;
    m.dim = 2;
    m.nv = 3;
    m.F = 3;
    m.n_orient = 4;
    m.K = K;
    m.elem_vert.reserve(K * 3);
    m.elem_xyz.reserve(K * 6);
    m.elem_level.reserve(K);
    m.leaf_edge.reserve(K * 3);
    m.leaf_family.reserve(K);
    m.leaf_child.reserve(K);
    m.adapt_kind.reserve(K);
    m.adapt_src.reserve(K * 4);
    return h;
}

void add_leaf(Mesh &m, const int32_t v[3], const double *x0, const double *x1, const double *x2, int lvl,
              int32_t e0, int32_t e1, int32_t e2, int32_t fam, int child, int kind, const int32_t src[4]) {
    m.elem_vert.insert(m.elem_vert.end(), {v[0], v[1], v[2]});
    m.elem_xyz.insert(m.elem_xyz.end(), {x0[0], x0[1], x1[0], x1[1], x2[0], x2[1]});
    m.elem_level.push_back((int8_t)lvl);
    m.leaf_edge.insert(m.leaf_edge.end(), {e0, e1, e2});
    m.leaf_family.push_back(fam);
    m.leaf_child.push_back((int8_t)child);
    m.adapt_kind.push_back((int8_t)kind);
    m.adapt_src.insert(m.adapt_src.end(), {src[0], src[1], src[2], src[3]});
}

dgc_status check_parent(const dgc_mesh *parent, const void *flags, dgc_mesh **out, const char *who) {
    if (out) *out = nullptr;
    if (!parent || !flags || !out) return fail(DGC_E_ARG, std::string(who) + ": null argument");
    const Mesh &P = parent->m;
    if (P.elem_type != DGC_TRI) return fail(DGC_E_UNSUPPORTED, std::string(who) + ": triangles only");
    if (!P.laid_out || P.n_colors <= 0) return fail(DGC_E_NOT_COLORED, std::string(who) + ": mesh is not colored");
    if (!P.has_tree() && P.n_colors > 3)
        return fail(DGC_E_ARG, std::string(who) + ": the conforming base needs a 3-coloring");
    return DGC_OK;
}

}  // namespace

}  // namespace dgc

using dgc::fail;

extern "C" dgc_status dgc_mesh_refine(const dgc_mesh *parent, const uint8_t *flags, dgc_mesh **out,
                                      int64_t *n_closure) {
    using Node = dgc::Mesh::EdgeNode;
    if (dgc_status s = dgc::check_parent(parent, flags, out, "dgc_mesh_refine"); s != DGC_OK) return s;
    const dgc::Mesh &P = parent->m;
    dgc_mesh *h = nullptr;
    try {
        std::vector<Node> nodes;
        std::vector<int32_t> pedge, pfam;
        std::vector<int8_t> pchild;
        std::vector<dgc::Mesh::Family> fams;
        dgc::start_tree(P, nodes, pedge, pfam, pchild, fams);
        int64_t n_vert = P.n_vert;
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
        h = dgc::new_tri_mesh(K0 + 3 * n_split);
        dgc::Mesh &m = h->m;
        for (int64_t i = 0; i < K0; ++i) {
            const int32_t *v = &P.elem_vert[i * 3];
            const double *x = &P.elem_xyz[i * 6];
            const int lvl = P.elem_level[i];
            const int32_t E0 = pedge[i * 3], E1 = pedge[i * 3 + 1], E2 = pedge[i * 3 + 2];
            const int32_t src[4] = {(int32_t)i, -1, -1, -1};
            if (!split[i]) {
                dgc::add_leaf(m, v, x, x + 2, x + 4, lvl, E0, E1, E2, pfam[i], pchild[i], 0, src);
                continue;
            }
            const int32_t fam = (int32_t)fams.size();
            dgc::Mesh::Family F{};
            for (int a = 0; a < 3; ++a) F.verts[a] = v[a];
            for (int a = 0; a < 6; ++a) F.xyz[a] = x[a];
            F.edges[0] = E0; F.edges[1] = E1; F.edges[2] = E2;
            F.parent = pfam[i];
            F.child = pchild[i];
            F.level = (int8_t)lvl;
            fams.push_back(F);
            const int32_t m01 = nodes[E0].mid, m12 = nodes[E1].mid, m20 = nodes[E2].mid;
            const double x01[2] = {0.5 * (x[0] + x[2]), 0.5 * (x[1] + x[3])};
            const double x12[2] = {0.5 * (x[2] + x[4]), 0.5 * (x[3] + x[5])};
            const double x20[2] = {0.5 * (x[4] + x[0]), 0.5 * (x[5] + x[1])};
            const int32_t I0 = (int32_t)nodes.size();
            nodes.push_back({m12, m20, nodes[E0].color, -1, -1, -1, -1});
            nodes.push_back({m20, m01, nodes[E1].color, -1, -1, -1, -1});
            nodes.push_back({m01, m12, nodes[E2].color, -1, -1, -1, -1});
            const int32_t I1 = I0 + 1, I2 = I0 + 2;
            const int32_t c0[3] = {v[0], m01, m20}, c1[3] = {m01, v[1], m12}, c2[3] = {m20, m12, v[2]},
                          c3[3] = {m12, m20, m01};
            dgc::add_leaf(m, c0, x, x01, x20, lvl + 1, dgc::half_of(nodes, E0, v[0], m01), I1,
                          dgc::half_of(nodes, E2, m20, v[0]), fam, 0, 1, src);
            dgc::add_leaf(m, c1, x01, x + 2, x12, lvl + 1, dgc::half_of(nodes, E0, m01, v[1]),
                          dgc::half_of(nodes, E1, v[1], m12), I2, fam, 1, 2, src);
            dgc::add_leaf(m, c2, x20, x12, x + 4, lvl + 1, I0, dgc::half_of(nodes, E1, m12, v[2]),
                          dgc::half_of(nodes, E2, v[2], m20), fam, 2, 3, src);
            dgc::add_leaf(m, c3, x12, x20, x01, lvl + 1, I0, I1, I2, fam, 3, 4, src);
        }
        m.nodes.swap(nodes);
        m.families.swap(fams);
        m.n_vert = n_vert;
        m.prev_elem_new = P.elem_new;
        if (dgc_status s = dgc::finish_leaves(m, "dgc_mesh_refine"); s != DGC_OK) {
            delete h;
            return s;
        }
        *out = h;
        return DGC_OK;
    } catch (const std::bad_alloc &) {
        delete h;
        return fail(DGC_E_ALLOC, "dgc_mesh_refine: out of host memory");
    }
}

extern "C" dgc_status dgc_mesh_coarsen(const dgc_mesh *fine, const uint8_t *flags, dgc_mesh **out,
                                       int64_t *n_merged) {
    if (dgc_status s = dgc::check_parent(fine, flags, out, "dgc_mesh_coarsen"); s != DGC_OK) return s;
    const dgc::Mesh &P = fine->m;
    dgc_mesh *h = nullptr;
    try {
        std::vector<dgc::Mesh::EdgeNode> nodes;
        std::vector<int32_t> pedge, pfam;
        std::vector<int8_t> pchild;
        std::vector<dgc::Mesh::Family> fams;
        dgc::start_tree(P, nodes, pedge, pfam, pchild, fams);
        const int64_t K0 = P.K;

        // families to merge: four consecutive leaves that are children 0..3 of
        // one family, all flagged, none with a split edge
        std::vector<int64_t> merge_at;
        for (int64_t i = 0; i < K0;) {
            const int32_t f = pfam[i];
            bool ok = f >= 0 && pchild[i] == 0 && i + 3 < K0;
            for (int k = 0; ok && k < 4; ++k) {
                ok = pfam[i + k] == f && pchild[i + k] == k && flags[i + k];
                for (int e = 0; ok && e < 3; ++e) ok = nodes[pedge[(i + k) * 3 + e]].child0 < 0;
            }
            if (ok) {
                merge_at.push_back(i);
                i += 4;
            } else {
                ++i;
            }
        }
        if (n_merged) *n_merged = (int64_t)merge_at.size();

        h = dgc::new_tri_mesh(K0 - 3 * (int64_t)merge_at.size());
        dgc::Mesh &m = h->m;
        size_t next = 0;
        for (int64_t i = 0; i < K0;) {
            if (next < merge_at.size() && merge_at[next] == i) {
                const dgc::Mesh::Family &F = fams[pfam[i]];
                const int32_t src[4] = {(int32_t)i, (int32_t)i + 1, (int32_t)i + 2, (int32_t)i + 3};
                dgc::add_leaf(m, F.verts, F.xyz, F.xyz + 2, F.xyz + 4, F.level, F.edges[0], F.edges[1], F.edges[2],
                              F.parent, F.child, 5, src);
                ++next;
                i += 4;
                continue;
            }
            const int32_t src[4] = {(int32_t)i, -1, -1, -1};
            dgc::add_leaf(m, &P.elem_vert[i * 3], &P.elem_xyz[i * 6], &P.elem_xyz[i * 6 + 2], &P.elem_xyz[i * 6 + 4],
                          P.elem_level[i], pedge[i * 3], pedge[i * 3 + 1], pedge[i * 3 + 2], pfam[i], pchild[i], 0,
                          src);
            ++i;
        }
        // a merged parent's edge whose halves no leaf references is unsplit
        std::vector<uint8_t> used(nodes.size(), 0);
        for (int32_t e : m.leaf_edge) used[e] = 1;
        for (int64_t i : merge_at)
            for (int e = 0; e < 3; ++e) {
                dgc::Mesh::EdgeNode &n = nodes[fams[pfam[i]].edges[e]];
                if (n.child0 >= 0 && !used[n.child0] && !used[n.child1]) {
                    n.child0 = n.child1 = -1;
                    n.mid = -1;
                }
            }
        m.nodes.swap(nodes);
        m.families.swap(fams);
        m.n_vert = P.n_vert;
        m.prev_elem_new = P.elem_new;
        if (dgc_status s = dgc::finish_leaves(m, "dgc_mesh_coarsen"); s != DGC_OK) {
            delete h;
            return s;
        }
        *out = h;
        return DGC_OK;
    } catch (const std::bad_alloc &) {
        delete h;
        return fail(DGC_E_ALLOC, "dgc_mesh_coarsen: out of host memory");
    }
}
