// Host-side internals of libdgc: the mesh object and error plumbing.
#pragma once

#include <cstdint>
#include <string>
#include <vector>

#include "../../../include/dgc.h"

namespace dgc {

// Thread-local error message returned by dgc_last_error().
void set_error(const std::string &msg);
dgc_status fail(dgc_status code, const std::string &msg);

struct Mesh {
    int32_t elem_type = DGC_TRI;
    int dim = 2, nv = 3, F = 3;   // F: conforming faces per element
    int max_slots = 3;            // faces incl. hanging sub-faces per element
    int n_orient = 4;             // orientation codes per local face
    int64_t K = 0, E = 0, n_boundary = 0;

    std::vector<int32_t> elem_vert;  // [K][nv] (mixed meshes: -1 as the fourth vertex of a triangle)
    std::vector<int8_t> elem_kind;   // mixed meshes: [K] 0 triangle, 1 quadrilateral (else empty)
    std::vector<double> elem_xyz;    // [K][nv][dim]
    std::vector<int8_t> elem_level;  // [K] refinement level

    // face table, original ids
    std::vector<int32_t> face_L, face_R;      // R = -1: wall
    std::vector<int8_t> face_fL, face_fR;     // local face index
    std::vector<uint8_t> face_oR;             // orientation code of the right side
    std::vector<uint8_t> face_oL;             // orientation code of the left side (0 unless refined)
    std::vector<int32_t> elem_face;           // [K][max_slots], -1 padded

    // geometry
    std::vector<double> normal;   // [E][dim], left -> right
    std::vector<double> measure;  // [E]
    std::vector<double> detJ;     // [K]
    std::vector<double> Jinv;     // [K][dim][dim], Jinv[d][e] = d xi_d / d x_e

    // coloring / layout
    int n_colors = 0;
    std::vector<int8_t> color;        // [E], original ids
    std::vector<int32_t> elem_new;    // [K]
    std::vector<int32_t> face_order;  // [E]
    std::vector<int64_t> color_off;   // [n_colors + 1]
    bool laid_out = false;

    // refinement: recorded orientation of every edge (start vertex id) used
    // by the child-color map; -1 when not recorded
    std::vector<int32_t> edge_start;  // [E]
    int max_level = 0;

    // edge tree of a refined triangle mesh (empty for a conforming base)
    struct EdgeNode {
        int32_t start, end, color, child0, child1, parent, mid;
    };
    std::vector<EdgeNode> nodes;
    std::vector<int32_t> leaf_edge;   // [K][3] node of each local edge
    int64_t n_vert = 0;               // vertex ids in use
    bool has_tree() const { return !nodes.empty(); }

    // leaf tree: the element each leaf was split from (its "family"), kept so
    // that four siblings can merge back into it
    struct Family {
        int32_t verts[3];
        double xyz[6];
        int32_t edges[3];
        int32_t parent;  // family of the split element itself (-1: a base element)
        int8_t child;    // the split element's index in that family
        int8_t level;
    };
    std::vector<Family> families;
    std::vector<int32_t> leaf_family;  // [K], -1 for base elements
    std::vector<int8_t> leaf_child;    // [K] 0..3 (corner at v0, v1, v2, center)

    // provenance with respect to the mesh this one was adapted from
    std::vector<int8_t> adapt_kind;     // [K] 0 same leaf, 1 + k child k, 5 parent of four
    std::vector<int32_t> adapt_src;     // [K][4] original ids in the previous mesh, -1 padded
    std::vector<int32_t> prev_elem_new; // layout ids of the previous mesh
};

// mesh_build.cpp
dgc_status build_faces(Mesh &m);        // face table + geometry from elem_vert / elem_xyz
dgc_status elem_geometry(Mesh &m);      // detJ, J^-1 of every element
dgc_status face_geometry(Mesh &m);      // normal (from the left element) and measure of every face
int face_vertex(const Mesh &m, int64_t elem, int local_face, int k);  // local vertex of a face
bool elem_is_quad(const Mesh &m, int64_t elem);
int elem_n_faces(const Mesh &m, int64_t elem);
// coloring.cpp
dgc_status color_paper(Mesh &m, uint64_t seed, int64_t max_swaps, dgc_color_stats *st);
dgc_status color_greedy_std(Mesh &m, dgc_color_stats *st);
bool coloring_valid(const Mesh &m, const std::vector<int8_t> &color, std::string *why);
// layout.cpp
dgc_status make_layout(Mesh &m, uint32_t layout_flag);
// tables.cpp
dgc_status build_tables(int32_t elem_type, int p, dgc_table_info *info, std::vector<double> *out);

}  // namespace dgc

struct dgc_mesh {
    dgc::Mesh m;
};
