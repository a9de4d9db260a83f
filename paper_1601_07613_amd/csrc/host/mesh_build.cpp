// Face table and geometry of a conforming mesh of triangles, parallelograms
// (affine quadrilaterals) or tetrahedra.
//
// The paper keeps the connectivity face-wise: each face points to its left
// and right element (Section 5, Table 5a).  Faces are matched here by
// ordering (sorted vertex-id key, visit index) records, which reproduces the
// "first visit creates the face" numbering without a hash table: the visit
// index elem * F + local is unique and increasing in scan order.  The records
// are bucketed by their smallest vertex id with a stable counting sort (a
// bucket holds the few faces around one vertex) and each bucket is sorted by
// the rest of the key; the faces are then numbered by walking the visit
// indices in order.
#include <algorithm>
#include <array>
#include <cmath>
#include <numeric>

#include "internal.hpp"

namespace dgc {

namespace {

// local vertex lists of the faces of the reference element
const int kTriFace[3][2] = {{0, 1}, {1, 2}, {2, 0}};
const int kQuadFace[4][2] = {{0, 1}, {1, 2}, {2, 3}, {3, 0}};
const int kTetFace[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};

struct FaceRec {
    std::array<int32_t, 3> key;  // sorted vertex ids (unused slots = -1)
    int64_t visit;               // elem * F + local face
};

// lexicographic index of a permutation of {0,1,2}
int perm3_index(int p0, int p1, int p2) { return p0 * 2 + (p1 > p2 ? 1 : 0); }

}  // namespace

bool elem_is_quad(const Mesh &m, int64_t elem) {
    return m.elem_type == DGC_QUAD || (m.elem_type == DGC_MIXED && m.elem_kind[elem] == 1);
}

int elem_n_faces(const Mesh &m, int64_t elem) { return m.dim == 3 || elem_is_quad(m, elem) ? 4 : 3; }

int face_vertex(const Mesh &m, int64_t elem, int local_face, int k) {
    if (m.dim == 3) return kTetFace[local_face][k];
    return elem_is_quad(m, elem) ? kQuadFace[local_face][k] : kTriFace[local_face][k];
}

dgc_status elem_geometry(Mesh &m) {
    const int nv = m.nv, dim = m.dim;
    const int64_t K = m.K;
    // element Jacobians
    m.detJ.assign(K, 0.0);
    m.Jinv.assign(K * dim * dim, 0.0);
    for (int64_t i = 0; i < K; ++i) {
        const double *x = &m.elem_xyz[i * nv * dim];
        if (dim == 2) {
            // columns: vertex 1 - vertex 0 and (triangle) vertex 2 - vertex 0 or
            // (quadrilateral) vertex 3 - vertex 0
            const bool quad = elem_is_quad(m, i);
            const int v2 = quad ? 3 : 2;
            double a = x[2] - x[0], b = x[2 * v2] - x[0];      // J[0][0], J[0][1]
            double c = x[3] - x[1], d = x[2 * v2 + 1] - x[1];  // J[1][0], J[1][1]
            if (quad) {
                // an affine image of the unit square: x2 = x1 + x3 - x0
                const double gx = x[4] - x[2] - x[6] + x[0], gy = x[5] - x[3] - x[7] + x[1];
                const double size = std::max(std::max(std::fabs(a), std::fabs(b)), std::max(std::fabs(c), std::fabs(d)));
                if (std::fabs(gx) > 1e-12 * size || std::fabs(gy) > 1e-12 * size)
                    return fail(DGC_E_MESH, "quadrilateral " + std::to_string(i) + " is not a parallelogram");
            }
            double det = a * d - b * c;
            if (!(det > 0.0)) return fail(DGC_E_MESH, "element " + std::to_string(i) + " has non-positive area");
            m.detJ[i] = det;
            double *Ji = &m.Jinv[i * 4];
            Ji[0] = d / det;  Ji[1] = -b / det;
            Ji[2] = -c / det; Ji[3] = a / det;
        } else {
            double J[3][3];
            for (int e = 0; e < 3; ++e)
                for (int d = 0; d < 3; ++d) J[e][d] = x[(d + 1) * 3 + e] - x[e];
            double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
            double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
            double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
            double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
            if (!(det > 0.0)) return fail(DGC_E_MESH, "element " + std::to_string(i) + " has non-positive volume");
            m.detJ[i] = det;
            double *Ji = &m.Jinv[i * 9];
            // inverse = adjugate / det; Jinv[d][e]
            Ji[0] = c00 / det;
            Ji[1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
            Ji[2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
            Ji[3] = c01 / det;
            Ji[4] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
            Ji[5] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
            Ji[6] = c02 / det;
            Ji[7] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
            Ji[8] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
        }
    }

    return DGC_OK;
}

dgc_status face_geometry(Mesh &m) {
    const int nv = m.nv, dim = m.dim;
    const int64_t E = m.E;
    // face geometry from the left element's own coordinates
    m.normal.assign(E * dim, 0.0);
    m.measure.assign(E, 0.0);
    for (int64_t f = 0; f < E; ++f) {
        const int64_t L = m.face_L[f];
        const int fL = m.face_fL[f];
        const double *x = &m.elem_xyz[L * nv * dim];
        if (dim == 2) {
            const double *a = x + 2 * face_vertex(m, L, fL, 0);
            const double *b = x + 2 * face_vertex(m, L, fL, 1);
            double tx = b[0] - a[0], ty = b[1] - a[1];
            double len = std::hypot(tx, ty);
            m.measure[f] = len;
            m.normal[2 * f] = ty / len;
            m.normal[2 * f + 1] = -tx / len;
        } else {
            const double *p0 = x + 3 * kTetFace[fL][0];
            const double *p1 = x + 3 * kTetFace[fL][1];
            const double *p2 = x + 3 * kTetFace[fL][2];
            double u[3] = {p1[0] - p0[0], p1[1] - p0[1], p1[2] - p0[2]};
            double v[3] = {p2[0] - p0[0], p2[1] - p0[1], p2[2] - p0[2]};
            double c[3] = {u[1] * v[2] - u[2] * v[1], u[2] * v[0] - u[0] * v[2], u[0] * v[1] - u[1] * v[0]};
            double ar = std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
            double cen[3] = {0, 0, 0};
            for (int a = 0; a < 4; ++a)
                for (int e = 0; e < 3; ++e) cen[e] += 0.25 * x[3 * a + e];
            double s = (p0[0] - cen[0]) * c[0] + (p0[1] - cen[1]) * c[1] + (p0[2] - cen[2]) * c[2];
            double sg = s < 0 ? -1.0 : 1.0;
            for (int e = 0; e < 3; ++e) m.normal[3 * f + e] = sg * c[e] / ar;
            m.measure[f] = 0.5 * ar;
        }
    }
    return DGC_OK;
}

dgc_status build_faces(Mesh &m) {
    const int nv = m.nv, F = m.F, dim = m.dim, nfv = dim;
    const int64_t K = m.K;

    if (dgc_status g = elem_geometry(m); g != DGC_OK) return g;

    // face matching (an element of a mixed mesh has 3 or 4 faces)
    std::vector<FaceRec> raw;
    raw.reserve(K * F);
    int32_t n_vert = 0;
    for (int64_t i = 0; i < K; ++i) {
        const int Fi = elem_n_faces(m, i);
        for (int k = 0; k < Fi; ++k) {
            FaceRec r;
            r.key = {-1, -1, -1};
            for (int a = 0; a < nfv; ++a) r.key[a] = m.elem_vert[i * nv + face_vertex(m, i, k, a)];
            std::sort(r.key.begin(), r.key.begin() + nfv);
            if (r.key[0] < 0) return fail(DGC_E_MESH, "negative vertex id");
            n_vert = std::max(n_vert, r.key[nfv - 1] + 1);
            r.visit = i * F + k;
            raw.push_back(r);
        }
    }
    // stable counting sort by the smallest vertex id
    std::vector<int64_t> bstart((size_t)n_vert + 1, 0);
    for (const FaceRec &r : raw) ++bstart[(size_t)r.key[0] + 1];
    for (int32_t v = 0; v < n_vert; ++v) bstart[v + 1] += bstart[v];
    std::vector<FaceRec> rec(raw.size());
    {
        std::vector<int64_t> pos(bstart.begin(), bstart.end() - 1);
        for (const FaceRec &r : raw) rec[pos[r.key[0]]++] = r;
    }
    raw.clear();
    raw.shrink_to_fit();
    const auto less = [](const FaceRec &a, const FaceRec &b) {
        if (a.key != b.key) return a.key < b.key;
        return a.visit < b.visit;
    };
    for (int32_t v = 0; v < n_vert; ++v) {
        FaceRec *b = rec.data() + bstart[v], *e = rec.data() + bstart[v + 1];
        if (e - b <= 32) {
            for (FaceRec *x = b + 1; x < e; ++x) {  // insertion sort of a small bucket
                const FaceRec t = *x;
                FaceRec *y = x;
                for (; y > b && less(t, y[-1]); --y) *y = y[-1];
                *y = t;
            }
        } else {
            std::sort(b, e, less);
        }
    }
    // one group per face; walking the first visits in increasing order numbers
    // the faces as the element scan first meets them
    struct Group { int64_t first, second; };
    std::vector<int64_t> partner((size_t)K * F, -2);  // -2: not a first visit
    int64_t n_groups = 0;
    for (size_t s = 0; s < rec.size();) {
        size_t e = s + 1;
        while (e < rec.size() && rec[e].key == rec[s].key) ++e;
        if (e - s > 2) return fail(DGC_E_MESH, "a face is shared by more than two elements");
        partner[rec[s].visit] = e - s == 2 ? rec[s + 1].visit : -1;
        ++n_groups;
        s = e;
    }
    rec.clear();
    rec.shrink_to_fit();
    std::vector<Group> groups;
    groups.reserve(n_groups);
    for (int64_t t = 0; t < K * F; ++t)
        if (partner[t] != -2) groups.push_back({t, partner[t]});

    const int64_t E = (int64_t)groups.size();
    m.E = E;
    m.face_L.resize(E); m.face_R.resize(E);
    m.face_fL.resize(E); m.face_fR.resize(E);
    m.face_oL.assign(E, 0); m.face_oR.assign(E, 0);
    m.max_slots = F;
    m.elem_face.assign(K * F, -1);
    m.n_boundary = 0;
    for (int64_t f = 0; f < E; ++f) {
        const Group &g = groups[f];
        int32_t L = (int32_t)(g.first / F), fL = (int32_t)(g.first % F);
        m.face_L[f] = L; m.face_fL[f] = (int8_t)fL;
        m.elem_face[(int64_t)L * F + fL] = (int32_t)f;
        if (g.second < 0) {
            m.face_R[f] = -1; m.face_fR[f] = -1;
            ++m.n_boundary;
            continue;
        }
        int32_t R = (int32_t)(g.second / F), fR = (int32_t)(g.second % F);
        m.face_R[f] = R; m.face_fR[f] = (int8_t)fR;
        m.elem_face[(int64_t)R * F + fR] = (int32_t)f;
        // how the right element sees the left element's point order
        int32_t vl[3], vr[3];
        for (int a = 0; a < nfv; ++a) {
            vl[a] = m.elem_vert[(int64_t)L * nv + face_vertex(m, L, fL, a)];
            vr[a] = m.elem_vert[(int64_t)R * nv + face_vertex(m, R, fR, a)];
        }
        if (dim == 2) {
            if (!(vl[0] == vr[1] && vl[1] == vr[0]))
                return fail(DGC_E_MESH, "inconsistently oriented neighbours at face " + std::to_string(f));
            m.face_oR[f] = 1;  // reversed
        } else {
            int pi[3];
            for (int q = 0; q < 3; ++q) {
                pi[q] = -1;
                for (int a = 0; a < 3; ++a)
                    if (vr[a] == vl[q]) pi[q] = a;
                if (pi[q] < 0) return fail(DGC_E_MESH, "face vertex mismatch");
            }
            m.face_oR[f] = (uint8_t)perm3_index(pi[0], pi[1], pi[2]);
        }
    }

    if (dgc_status g = face_geometry(m); g != DGC_OK) return g;
    m.edge_start.assign(E, -1);
    if (dim == 2)
        for (int64_t f = 0; f < E; ++f)
            m.edge_start[f] = m.elem_vert[(int64_t)m.face_L[f] * nv + face_vertex(m, m.face_L[f], m.face_fL[f], 0)];
    m.n_colors = 0;
    m.color.assign(E, -1);
    m.laid_out = false;
    return DGC_OK;
}

}  // namespace dgc
