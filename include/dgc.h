/*
 * dgc.h -- C ABI of libdgc: race-free DG surface integrals on edge-colored
 * unstructured meshes, for AMD Instinct MI355X (gfx950).
 *
 * Method: A. Giuliani and L. Krivodonova, "Edge coloring in unstructured CFD
 * codes" (arXiv:1601.07613).  The surface term of the DG scheme (Eq. 2) is
 * evaluated one face per work item; two faces that share an element would
 * race on that element's right-hand side (Section 1, Figure 1).  The faces
 * are therefore colored so that no element has two faces of one color
 * (Sections 2-3) and processed one color at a time with a barrier between
 * colors (Algorithm 1).  The coloring also drives an element renumbering and
 * face reordering that make the memory accesses of the face kernel
 * contiguous (Section 5, Tables 5-6).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Every function returns a dgc_status: 0 (DGC_OK) on success, a negative
 *   code on failure.  dgc_last_error() then returns a thread-local message.
 *   Nothing is thrown across the ABI and no entry point writes outside the
 *   buffers and sizes it is given.
 * - Host objects (dgc_mesh) are owned by the library: create them with
 *   dgc_mesh_build / dgc_mesh_refine, release them with dgc_mesh_free.
 * - Device buffers are owned by the caller (raw device pointers, e.g. from a
 *   framework's caching allocator).  Device entry points only enqueue work on
 *   the given stream (a hipStream_t passed as void*, NULL = the null stream)
 *   and return; asynchronous faults surface at the caller's synchronisation.
 *   The library allocates no device memory; its only device state is the
 *   fixed stage storage of dgc_rk_step_noalloc (DGC_NOALLOC_MAX_BYTES per
 *   GPU, reserved when the library's code is loaded onto that GPU).
 * - Colors are 0-based (the paper's color c is color c-1 here).
 * - Element ids in device arrays are *layout* ids (after the renumbering of
 *   Section 5); DOF and right-hand-side arrays are indexed by layout ids.
 * - DOF / RHS layout on the device: element-major records,
 *   U[k][m][j] = U[(k * M + m) * N_p + j] for layout element k, conserved
 *   variable m (rho, rho u, rho v[, rho w], E) and mode j.  The coefficient
 *   multiplies v_kj = phi_j / sqrt(det J_k), phi_j the orthonormal Dubiner
 *   function on the unit reference element (mode order: total degree
 *   ascending, then the second collapsed index ascending).
 */
#ifndef DGC_H
#define DGC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    DGC_OK = 0,
    DGC_E_ARG = -1,              /* bad argument: null pointer, size, enum, buffer too small */
    DGC_E_MESH = -2,             /* non-positive element measure, face shared by >2 elements */
    DGC_E_NOT_COLORED = -3,      /* operation needs a colored and laid-out mesh */
    DGC_E_COLOR_CAP = -4,        /* coloring move cap reached; mesh left uncolored */
    DGC_E_COLORING_INVALID = -5, /* a supplied coloring has an element with two faces of one color */
    DGC_E_UNSUPPORTED = -6,      /* element type / order / variant / precision not built */
    DGC_E_WORKSPACE = -7,        /* workspace missing or smaller than dgc_workspace_bytes */
    DGC_E_HIP = -8,              /* a HIP runtime call failed (message names it) */
    DGC_E_ALLOC = -9             /* host allocation failed */
} dgc_status;

enum { DGC_TRI = 0, DGC_QUAD = 1, DGC_TET = 2, DGC_MIXED = 3 };

/* dgc_color_edges flags: one coloring algorithm | one layout */
#define DGC_COLOR_PAPER      0x01u /* modified greedy + conflict resolution (Section 3.1) */
#define DGC_COLOR_GREEDY_STD 0x02u /* standard greedy, first free color (Section 1) */
#define DGC_LAYOUT_PAPER     0x10u /* renumber elements + reorder faces (Section 5) */
#define DGC_LAYOUT_RENUMBER  0x20u /* renumber elements only (Table 5) */
#define DGC_LAYOUT_NONE      0x40u /* faces grouped by color, elements unchanged */
#define DGC_LAYOUT_PAPER_SFC 0x80u /* DGC_LAYOUT_PAPER with the first color's faces taken in
                                      Morton order of their midpoints (an extension) */
#define DGC_LAYOUT_PAIRED   0x100u /* as DGC_LAYOUT_PAPER_SFC, but the first color's interior
                                      faces are numbered in blocks of 16: block b of n faces gets
                                      left elements 32b + i and right elements 32b + n + i
                                      (an extension; boundary faces' left elements follow) */

#define DGC_MAX_COLORS 8

typedef struct dgc_mesh dgc_mesh;

typedef struct {
    int64_t conflicts_after_greedy; /* faces left uncolored by the modified greedy stage */
    int64_t swaps;                  /* conflict moves that keep the conflict count */
    int64_t loop_breaks;            /* loop escapes that add one conflict */
    int64_t deferrals;              /* conflicts re-queued (no same-colored pair to break) */
    int32_t n_colors;
    int32_t pad_;
    int64_t count[DGC_MAX_COLORS];  /* faces per color */
    double color_ms;                /* host wall time of the coloring */
    double layout_ms;               /* host wall time of renumbering + reordering */
} dgc_color_stats;

typedef struct {
    int32_t elem_type;       /* DGC_TRI or DGC_TET */
    int32_t dim;             /* 2 or 3 */
    int32_t n_vert_per_elem; /* 3 or 4 */
    int32_t n_face_per_elem; /* conforming faces per element: 3 or 4 */
    int32_t max_slots;       /* max faces (incl. hanging sub-faces) of one element */
    int32_t n_colors;        /* 0 until colored */
    int64_t n_elem;
    int64_t n_face;
    int64_t n_boundary;
    int64_t color_off[DGC_MAX_COLORS + 1]; /* layout positions: color c = [off[c], off[c+1]) */
    int32_t n_orient;        /* orientation codes per local face (table index = f*n_orient+o) */
    int32_t max_level;       /* refinement level reached (0 = conforming base) */
} dgc_mesh_info_t;

/* Build the face table and geometry of a conforming mesh (face-wise
 * connectivity, Section 5 and Table 5a; left/right elements,
 * Section 3).
 *   elem_type  DGC_TRI (3 vertices, counter-clockwise, 2D), DGC_QUAD (4
 *              vertices, counter-clockwise, a parallelogram: the affine image
 *              of the unit square), DGC_MIXED (triangles and parallelograms
 *              in one 2D mesh, the hybrid meshes of Table 2: 4 vertex slots
 *              per element, -1 as the fourth vertex id of a triangle) or
 *              DGC_TET (4 vertices, positive volume, 3D).
 *   elem_vert  host int32 [n_elem][nv]: vertex ids; periodic images of a
 *              vertex share one id.
 *   elem_xyz   host f64 [n_elem][nv][dim]: each element's own (unwrapped)
 *              vertex coordinates; geometry of a face is taken from its
 *              left element.
 * Faces are numbered by first visit scanning elements 0..K-1 and local faces
 * 0..F-1 (triangle edge k joins local vertices k, k+1 mod 3, quadrilateral
 * edge k local vertices k, k+1 mod 4; tetrahedron face k is opposite vertex
 * k); the first visitor is the left element, the second the right one, a
 * face with one visitor is a reflective wall.  Errors: DGC_E_MESH also for a
 * quadrilateral that is not a parallelogram.
 * Errors: DGC_E_ARG, DGC_E_MESH (non-positive measure, face with >2 elements),
 * DGC_E_ALLOC.  On success *out owns a new mesh. */
dgc_status dgc_mesh_build(int32_t elem_type, int64_t n_elem, const int32_t *elem_vert,
                          const double *elem_xyz, dgc_mesh **out);

/* Color the faces (Section 3.1) and lay the mesh out (Section 5).
 * DGC_COLOR_PAPER uses as many colors as an element has faces at most: 3 for
 * triangles, 4 for quadrilaterals, mixed meshes and tetrahedra: a
 * modified greedy pass with random non-conflicting colors (SplitMix64 seeded
 * with `seed`), then conflict resolution by count-preserving swaps, loop
 * breaks that uncolor a same-colored pair, and deferral of a conflict whose
 * elements hold no such pair.  Moves are capped by max_swaps (<0: 1000 x
 * n_face); reaching the cap returns DGC_E_COLOR_CAP and leaves the mesh
 * uncolored (a caller may retry with another seed).
 * DGC_COLOR_GREEDY_STD gives each face, in id order, the smallest color
 * free on both elements (at most 5 colors for triangles, 7 for tetrahedra).
 * Layout: the first color's k-th face (interior faces first) gets left
 * element k and right element N_1 + k; the faces of later colors are sorted
 * by ascending left element (Tables 5 and 6).  stats may be NULL.
 * Errors: DGC_E_ARG, DGC_E_COLOR_CAP, DGC_E_UNSUPPORTED (refined meshes are
 * colored by dgc_mesh_refine). */
dgc_status dgc_color_edges(dgc_mesh *m, uint64_t seed, int64_t max_swaps, uint32_t flags,
                           dgc_color_stats *stats);

/* Install a caller-supplied coloring (host int8 [n_face], original face ids)
 * and lay the mesh out with the given DGC_LAYOUT_* flag.  The coloring is
 * checked exactly: an uncolored face, a color >= DGC_MAX_COLORS or an
 * element with two faces of one color returns DGC_E_COLORING_INVALID and
 * leaves the mesh unchanged. */
dgc_status dgc_set_colors(dgc_mesh *m, const int8_t *colors, uint32_t layout_flags);

/* Split the flagged leaf triangles of a colored mesh into four (midpoint
 * split, Section 3.2), first splitting coarser neighbours so that adjacent
 * leaves differ by at most one level, and color the new mesh by the
 * closed-form map of Section 3.2: child edges of a parent edge of color c
 * take c and (c + 3) mod 6 (the first child is the one at the parent edge's
 * recorded start vertex); interior edges take the color of the parallel
 * parent edge.  A hanging edge is split into its two sub-edges; the fine
 * element is the left element and the coarse one the right element.
 *   flags     host uint8 [n_elem of parent]: nonzero = refine this leaf.
 *   n_closure out (may be NULL): leaves split only to restore the 2:1 balance.
 * The result is colored (up to 6 colors) and laid out (DGC_LAYOUT_PAPER).
 * Errors: DGC_E_ARG, DGC_E_NOT_COLORED, DGC_E_UNSUPPORTED (tetrahedra). */
dgc_status dgc_mesh_refine(const dgc_mesh *parent, const uint8_t *flags, dgc_mesh **out,
                           int64_t *n_closure);

/* Undo 4-way splits (the coarsening of Section 3.2).  Four leaves merge
 * back into the element they were split from when they are its children
 * 0..3, all four are flagged and none of their edges is split (so no
 * neighbour ends up two levels finer); the merged element takes the place
 * of its first child.  Its edges are the parent edges, whose colors were
 * kept, so coarsening restores the parent coloring without any search; a
 * parent edge whose halves no leaf references any more is unsplit.
 *   fine      a colored mesh (a conforming base has nothing to merge and
 *             comes back with the same leaves, renumbered as a refined mesh
 *             would be).
 *   flags     host uint8 [n_elem]: nonzero = this leaf may merge.
 *   n_merged  out (may be NULL): number of merged families.
 * The result is colored and laid out (DGC_LAYOUT_PAPER); the origin of every
 * leaf is exported as DGC_ARR_ADAPT_* / DGC_ARR_DEV_ADAPT_*, as after
 * dgc_mesh_refine.  Errors: DGC_E_ARG, DGC_E_NOT_COLORED, DGC_E_UNSUPPORTED
 * (tetrahedra). */
dgc_status dgc_mesh_coarsen(const dgc_mesh *fine, const uint8_t *flags, dgc_mesh **out, int64_t *n_merged);

dgc_status dgc_mesh_info(const dgc_mesh *m, dgc_mesh_info_t *info);

/* Arrays that dgc_mesh_export can copy out (host memory, caller-owned). */
enum {
    /* original face ids */
    DGC_ARR_FACE_ELEM = 1,   /* int32 [E][2]: left, right original element (-1 = wall) */
    DGC_ARR_FACE_LOCAL = 2,  /* int8  [E][2]: local face index in left / right element */
    DGC_ARR_COLOR = 3,       /* int8  [E]: color of each face (-1 if uncolored) */
    DGC_ARR_FACE_NORMAL = 4, /* f64   [E][dim]: unit normal, left -> right */
    DGC_ARR_FACE_MEASURE = 5,/* f64   [E]: length / area */
    DGC_ARR_ELEM_DETJ = 6,   /* f64   [K]: det of the reference-to-physical Jacobian */
    DGC_ARR_ELEM_FACE = 7,   /* int32 [K][max_slots]: face ids of each element, -1 padded */
    /* layout */
    DGC_ARR_ELEM_NEW = 10,   /* int32 [K]: layout id of original element i */
    DGC_ARR_FACE_ORDER = 11, /* int32 [E]: original face id at layout position k */
    DGC_ARR_COLOR_OFF = 12,  /* int64 [n_colors + 1] */
    /* device-ready arrays, layout order, structure-of-arrays */
    DGC_ARR_DEV_FACE_LR = 20,   /* int32 [2][E]: layout ids of left / right element (-1 = wall) */
    DGC_ARR_DEV_FACE_CODE = 21, /* uint8 [2][E]: table code of the left / right side */
    DGC_ARR_DEV_FACE_GEO = 22,  /* f64 [dim+3][E]: n_0..n_{dim-1}, |f|, 1/sqrt(detJ_L), 1/sqrt(detJ_R) (0 at walls) */
    DGC_ARR_DEV_ELEM_GEO = 23,  /* f64 [dim*dim+1][K]: (J^-1)_{de} row-major, then sqrt(det J) */
    DGC_ARR_DEV_ELEM_SLOTS = 24,/* int32 [max_slots][K]: 2*face+side of each element's faces, -1 padded */
    DGC_ARR_DEV_ADAPT_KIND = 25,/* int8 [K] (layout order): origin of each leaf, as DGC_ARR_ADAPT_KIND */
    DGC_ARR_DEV_ADAPT_SRC = 26, /* int32 [4][K] (layout order): its source leaves as layout ids of the
                                   previous mesh, -1 padded */
    DGC_ARR_DEV_ELEM_KIND = 27, /* int8 [K] (layout order), mixed meshes: 0 triangle, 1 quadrilateral */
    /* refinement bookkeeping */
    DGC_ARR_ELEM_LEVEL = 30,    /* int8 [K]: refinement level of each leaf (original ids) */
    DGC_ARR_ELEM_XYZ = 31,      /* f64 [K][nv][dim]: element vertex coordinates (original ids) */
    DGC_ARR_ELEM_VERT = 32,     /* int32 [K][nv]: element vertex ids (original ids) */
    /* meshes made by dgc_mesh_refine / dgc_mesh_coarsen: where each leaf came from */
    DGC_ARR_ADAPT_KIND = 33,    /* int8 [K]: 0 the same leaf, 1 + k child k of a leaf (k = 0..2 corner
                                   children at v0, v1, v2, k = 3 the center child), 5 the parent of
                                   four leaves (children 0..3) */
    DGC_ARR_ADAPT_SRC = 34      /* int32 [K][4]: those leaves (original ids of the previous mesh),
                                   -1 padded */
};

/* Copy array `which` into dst (bytes available).  *needed (if not NULL)
 * receives the size in bytes; call with dst = NULL to query it.
 * Errors: DGC_E_ARG (unknown array, dst too small), DGC_E_NOT_COLORED (a
 * layout array of an uncolored mesh). */
dgc_status dgc_mesh_export(const dgc_mesh *m, int32_t which, void *dst, size_t bytes, size_t *needed);

void dgc_mesh_free(dgc_mesh *m);
const char *dgc_last_error(void);

/* Basis and quadrature tables for an element type and order (Eq. 2 with an
 * orthonormal basis; the quadrature is not given by the paper: Gauss-Legendre
 * with p+1 points on edges, the symmetric 3-point rule on tetrahedron faces
 * up to p = 1 and the collapsed Gauss-Jacobi triangle rule with (p+1)^2
 * points from p = 2, collapsed Gauss-Jacobi rules with p+1 points per
 * direction in the volume; tensor Gauss-Legendre on quadrilaterals).
 * Orders: triangles p <= 5, quadrilaterals and mixed meshes p <= 3,
 * tetrahedra p <= 2;
 * DGC_E_UNSUPPORTED beyond.  Layout of the f64 array (offsets in doubles,
 * from info):
 *   trace [n_codes][n_qf][n_p]  phi_j at face point q seen through code c
 *   proj  [n_codes][n_qf][n_p]  w_q * trace (face weights sum to 1)
 *   vb    [n_qv][n_p]           phi_j at volume point q
 *   vd    [dim][n_qv][n_p]      w_q * d phi_j / d xi_d at volume point q
 *   prolong [4][n_p][n_p]       triangles only (empty for tetrahedra): L2
 *                               projection of a parent's modes onto child k
 *                               (corner children at v0, v1, v2, then the
 *                               center child; Section 3.2 split), see
 *                               dgc_adapt_transfer
 * Mixed meshes (DGC_MIXED): n_p = (p+1)^2 slots for every element (a
 * triangle uses its first (p+1)(p+2)/2, its tables are zero beyond them);
 * codes 0..11 are the triangle's, 12..27 the quadrilateral's (12 + f *
 * n_orient + o); vb and vd hold the triangle block, then the quadrilateral
 * block ([2][n_qv][n_p], [2][dim][n_qv][n_p]).
 * Code c = f * n_orient + o addresses local face f seen with orientation o:
 * o = 0 the face's own point order, 2D: 1 reversed, 2 / 3 reversed points on
 * the first / second half of the edge (hanging edge seen from the coarse
 * side); 3D: the o-th permutation pi (lexicographic) of the face's three
 * vertices, vertex u of the left element's face order being vertex pi[u] of
 * this side's face; face point q is placed by its barycentric weights in the
 * left element's order, so both sides evaluate the same physical point. */
typedef struct {
    int32_t elem_type, p, dim, n_p, n_qf, n_qv, n_codes, n_orient;
    int64_t off_trace, off_proj, off_vb, off_vd, off_prolong, total; /* in doubles */
} dgc_table_info;

dgc_status dgc_tables(int32_t elem_type, int32_t p, dgc_table_info *info, double *dst, size_t bytes,
                      size_t *needed);

/* ---------------------------------------------------------------------- */
/* Device entry points                                                     */
/* ---------------------------------------------------------------------- */

enum { DGC_SURF_COLORED = 0, DGC_SURF_ATOMIC = 1, DGC_SURF_GATHER = 2, DGC_SURF_COMPACT = 3 };
enum { DGC_F64 = 0, DGC_F32 = 1 };

/* Device view of one laid-out mesh at one order.  Every pointer is a device
 * pointer to the matching DGC_ARR_DEV_* / dgc_tables array, copied to the
 * device by the caller; color_off is a host copy. */
typedef struct {
    int32_t elem_type, p, n_p, n_var, n_qf, n_qv, n_codes, n_orient;
    int32_t n_colors, max_slots;
    int64_t n_elem, n_face;
    int64_t color_off[DGC_MAX_COLORS + 1];
    const int32_t *face_lr;    /* [2][n_face] */
    const uint8_t *face_code;  /* [2][n_face] */
    const double *face_geo;    /* [dim+3][n_face] */
    const double *elem_geo;    /* [dim*dim+1][n_elem] */
    const int32_t *elem_slots; /* [max_slots][n_elem] (GATHER only; may be NULL otherwise) */
    const double *tables;      /* dgc_tables layout for (elem_type, p) */
    /* launch tuning (0 = library default); any valid choice gives the same
     * result up to the rounding of the accumulation order */
    int32_t surf_form;         /* DGC_FORM_* */
    int32_t block_size;        /* work-items per work-group of the face kernels: 64, 128 or 256 */
    int32_t xcd_remap;         /* 1: work-groups are dealt round-robin to the 8 XCDs, so give
                                  each XCD one contiguous range of faces (shared L2 lines) */
    int32_t vol_form;          /* DGC_VOL_* */
    int32_t rk_form;           /* DGC_RK_* */
    int32_t pad_;
    const int8_t *elem_kind;   /* [n_elem] DGC_ARR_DEV_ELEM_KIND (mixed meshes; NULL otherwise) */
} dgc_dmesh;

/* dgc_rk_step forms: DGC_RK_FUSED fuses each stage's combination into the
 * face kernel of the last color when that is exact (f64, colored variant, a
 * conforming mesh colored with as many colors as an element has faces, so
 * every element has exactly one face of the last color, and a team face
 * form; the f32 form keeps its combination kernel, measured faster than a
 * fused one), else runs it as its own kernel; DGC_RK_SEPARATE always runs the
 * combination as its own kernel; DGC_RK_BLOCK runs the whole step in one
 * work-group of 512 work-items, with barriers between the volume term, the
 * colors and the combinations (f64, colored variant, one element type; an
 * alternative for small meshes, where launches dominate: measured slower
 * than DGC_RK_FUSED even at 512 elements, one CU being too little).
 * DGC_RK_FUSED_VOLUME also moves each stage's volume term into the face
 * kernel of the first color under the same conditions (every element has
 * exactly one face of the first color; f64 and the f32 form; the element
 * records read for the traces feed the volume term too, and the first color
 * writes rhs without reading it): one launch and three record passes fewer
 * per stage; the volume term is then computed by the face team (lane =
 * variable, or lane = mode for tetrahedra at p = 1) whatever vol_form says.
 * Where its conditions fail it falls back to DGC_RK_FUSED.
 * DGC_RK_DEFAULT is DGC_RK_FUSED_VOLUME for triangles at p <= 3, for
 * quadrilaterals (f32 only at p = 3) and for f64 tetrahedra at p = 1 when
 * vol_form is DGC_VOL_DEFAULT (measured 2-18 % faster per step on ~1M
 * elements), and
 * DGC_RK_FUSED otherwise (triangles at p = 4, 5: the face kernel's
 * registers run out; f32 tetrahedra: no gain, the face team evaluates the
 * flux of the volume term on each of its four lanes), except for
 * tetrahedra at p = 2, where the combination stays a kernel of its own (the
 * combining team kernel runs out of registers). */
enum { DGC_RK_DEFAULT = 0, DGC_RK_SEPARATE = 1, DGC_RK_FUSED = 2, DGC_RK_BLOCK = 3, DGC_RK_FUSED_VOLUME = 4 };

/* Volume-kernel forms: DGC_VOL_VALU evaluates each element in one work-item
 * with vector FMAs; DGC_VOL_TEAM gives each element a team of lanes (one
 * per conserved variable, the element record read as one contiguous
 * stretch) that exchange the point values; DGC_VOL_MFMA (2D, f64, at most 16
 * modes and 16 points: triangles p <= 3, quadrilaterals p <= 3; other cases
 * fall back to DGC_VOL_VALU) runs the two basis contractions of four
 * elements at a time on the matrix cores (v_mfma_f64_16x16x4f64) and the
 * flux between them on the vector units.  DGC_VOL_DEFAULT picks the form
 * measured fastest for the element type, order and precision: in f64 the
 * team form (one work-item per element for triangles at p = 3), in f32 one
 * work-item per element (the team form for quadrilaterals at p <= 2), one
 * work-item per element for tetrahedra; mixed meshes always use their own
 * team kernel.  The matrix-core form is an explicit choice only: slower
 * than the vector forms at every order measured. */
enum { DGC_VOL_DEFAULT = 0, DGC_VOL_VALU = 1, DGC_VOL_MFMA = 2, DGC_VOL_TEAM = 3 };

/* Face-kernel forms: DGC_FORM_TEAM gives each face a team of lanes (one lane
 * per conserved variable) so that loads of one element record are
 * contiguous across lanes; DGC_FORM_TEAM_PREFETCH is the same with the
 * right-hand-side reads of the colored update issued before the flux
 * evaluation; DGC_FORM_THREAD gives each face one work-item;
 * DGC_FORM_MODE_TEAM (tetrahedra, p = 1) gives each face 4 lanes, one per
 * mode, and sums the traces across them; DGC_FORM_TEAM_STREAM is the team
 * visiting the quadrature points one at a time (trace, flux and projection
 * per point), for large N_p x Q where the team runs out of registers (the
 * plain colored, atomic and gather passes; the fused RK stages keep the
 * team); DGC_FORM_PAIR_TEAM (tetrahedra, p = 1) gives each face 4 lanes that
 * own two adjacent modes of two or three variables, so that records move in
 * 16-byte pieces (the plain passes and the fused combination).
 * DGC_FORM_DEFAULT picks the form measured fastest for the element
 * type, order, precision and size: the team with prefetch for f64
 * triangles at p = 1 and at p = 2 from 1M faces on, for f32 triangles at
 * p = 3, 4 and for parallelograms (and mixed meshes) at p = 0, 2; the
 * streaming team for tetrahedra at p = 2, f64 triangles at p >= 3, f32
 * triangles at p = 5 and f64 parallelograms at p = 3; the mode team for
 * tetrahedra at p = 1; the team without prefetch otherwise. */
enum { DGC_FORM_DEFAULT = 0, DGC_FORM_TEAM = 1, DGC_FORM_THREAD = 2, DGC_FORM_TEAM_PREFETCH = 3,
       DGC_FORM_MODE_TEAM = 4, DGC_FORM_TEAM_STREAM = 5, DGC_FORM_PAIR_TEAM = 6 };

/* Volume term of Eq. (2): rhs = int F(U) . grad v (overwrites rhs).
 * U, rhs: device [n_elem][n_var][n_p] (f64, or f32 for DGC_F32). */
dgc_status dgc_volume_rhs(const dgc_dmesh *dm, const void *U, void *rhs, int32_t precision, void *stream);

/* Surface term of Eq. (2), accumulated: rhs -= sum_faces int v F* . n.
 * DGC_SURF_COLORED: one launch per color, the launches ordered on `stream`
 *   (the "synchronize threads" of Algorithm 1); each face updates its left
 *   and right element with plain read-modify-write, race-free because no
 *   element has two faces of one color.  Needs no workspace.
 * DGC_SURF_ATOMIC: one launch over all faces, atomic adds (Section 1).
 * DGC_SURF_GATHER: the buffered alternative of Section 1: face j writes its
 *   left / right contributions to slots 2j, 2j+1 of a workspace of
 *   2 * n_face * n_var * n_p values (the memory of Table 4), then a second
 *   kernel adds each element's slots to rhs.
 * DGC_SURF_COMPACT: the buffer alternative of Section 1 with one record per
 *   face instead of two element-sized slots: the face pass writes
 *   |f| F*_q[m] at the Q face points (n_qf * n_var values) and the two
 *   table codes, a workspace of n_face * (n_qf * n_var + 1) values; a second
 *   kernel lets each element project the records of its faces (minus on its
 *   left faces, plus on its right faces) and update its rhs once.
 * Errors: DGC_E_ARG, DGC_E_NOT_COLORED (COLORED without colors),
 * DGC_E_WORKSPACE, DGC_E_UNSUPPORTED, DGC_E_HIP (launch failure). */
dgc_status dgc_surface_rhs(const dgc_dmesh *dm, const void *U, void *rhs, int32_t variant,
                           int32_t precision, void *ws, size_t ws_bytes, void *stream);

/* One SSP-RK3 step (Shu-Osher form) of U (device f64, updated in place):
 * three stages of volume term + surface term (`variant`) + combination,
 * launched as dm->rk_form says (the volume term and the combination may
 * ride on the first and last color's face kernels, see DGC_RK_*).  With
 * DGC_SURF_COMPACT in f64 on conforming triangle and parallelogram meshes
 * (any rk_form but DGC_RK_SEPARATE) a stage is two launches: the face pass, then one element
 * pass that evaluates the volume term (the team form, whatever vol_form
 * says), adds the face records and writes the stage combination.
 * DGC_F32 evaluates both terms on an f32 shadow of the stage state and
 * accumulates the stages in f64.  ws holds the stage states and the RHS
 * (DGC_WS_RK_STEP bytes, dgc_rk_workspace_layout).  Errors: DGC_E_ARG,
 * DGC_E_NOT_COLORED, DGC_E_WORKSPACE, DGC_E_UNSUPPORTED, DGC_E_HIP. */
dgc_status dgc_rk_step(const dgc_dmesh *dm, double *U, double dt, int32_t variant, int32_t precision,
                       void *ws, size_t ws_bytes, void *stream);

/* dgc_rk_step for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid allocation):
 * the same step, same kernels and same results as dgc_rk_step, with the
 * stage states and right-hand side held in a device array of
 * DGC_NOALLOC_MAX_BYTES bytes that the library keeps on every GPU it runs on
 * until the process ends.  The array of the current device is used; `stream`
 * must belong to that device.  Nothing in it needs to start at zero (every
 * part is written before it is read).  Every call on one GPU shares that
 * GPU's array, so calls that overlap on one GPU (two streams, two host
 * threads) race: order them on one stream.  Allocates nothing, host or
 * device.  Errors: as dgc_rk_step, and DGC_E_WORKSPACE when the step needs
 * more than DGC_NOALLOC_MAX_BYTES (dgc_workspace_bytes, DGC_WS_RK_STEP: at
 * p = 2 about 116k triangles in f64); DGC_E_HIP when the array's device
 * address cannot be found. */
#define DGC_NOALLOC_MAX_BYTES (64u << 20)
dgc_status dgc_rk_step_noalloc(const dgc_dmesh *dm, double *U, double dt, int32_t variant, int32_t precision,
                               void *stream);

enum { DGC_WS_SURFACE = 0, DGC_WS_RK_STEP = 1 };

/* Workspace size in bytes for dgc_surface_rhs (what = DGC_WS_SURFACE) or
 * dgc_rk_step (DGC_WS_RK_STEP) with the given variant and precision. */
dgc_status dgc_workspace_bytes(const dgc_dmesh *dm, int32_t what, int32_t variant, int32_t precision,
                               size_t *bytes);

/* Move element records between the caller's element order and the layout
 * order (Section 5) on the device.  src, dst: device [n_rec][rec_bytes]
 * (distinct buffers); perm: device int32 [n_rec], perm[i] = layout id of
 * element i (the DGC_ARR_ELEM_NEW array).  to_layout != 0: dst[perm[i]] =
 * src[i]; otherwise dst[i] = src[perm[i]].  rec_bytes must be a multiple of
 * 4.  Errors: DGC_E_ARG, DGC_E_HIP. */
dgc_status dgc_permute_records(const void *src, void *dst, const int32_t *perm, int64_t n_rec, int64_t rec_bytes,
                               int32_t to_layout, void *stream);

/* The closed-form child coloring of a 4-way split (Section 3.2), computed in
 * parallel on the device.  parent_colors: device int8 [n][3], the colors
 * (0..5) of the three edges of each split element; child_colors: device int8
 * [n][9]: for parent edge k, the colors of its first and second child
 * (entries 2k, 2k+1: c and (c + 3) mod 6; "first" is the half at the edge's
 * recorded start vertex), then the colors of the interior edges parallel to
 * parent edges 0, 1, 2 (entries 6..8).  dgc_mesh_refine applies the same map
 * on the host.  Errors: DGC_E_ARG, DGC_E_HIP. */
dgc_status dgc_child_colors(const int8_t *parent_colors, int64_t n, int8_t *child_colors, void *stream);

/* Move a solution onto a mesh made by dgc_mesh_refine / dgc_mesh_coarsen
 * (refinement under a running solution, Section 3.2), on the device.  Every
 * new leaf gets the L2 projection of the previous solution: an unchanged leaf
 * copies its modes, child k of a split leaf gets P_k c (P_k from the tables'
 * prolong block), a merged parent gets sum_k P_k^T c_k over its four
 * children (exact inverse of the split: sum_k P_k^T P_k = I).
 *   dm      device view of the NEW mesh (triangles, p <= 5).
 *   U_old   device f64 [n_old][n_var][n_p] in the previous mesh's layout order.
 *   U_new   device f64 [dm->n_elem][n_var][n_p] in the new layout order;
 *           must not alias U_old.
 *   kind    device int8 [n_elem]  (DGC_ARR_DEV_ADAPT_KIND of the new mesh)
 *   src     device int32 [4][n_elem] (DGC_ARR_DEV_ADAPT_SRC of the new mesh)
 * A record whose source id falls outside [0, n_old) or whose kind is unknown
 * is filled with NaN.  Errors: DGC_E_ARG, DGC_E_UNSUPPORTED (tetrahedra),
 * DGC_E_HIP. */
dgc_status dgc_adapt_transfer(const dgc_dmesh *dm, const double *U_old, int64_t n_old, double *U_new,
                              const int8_t *kind, const int32_t *src, void *stream);

/* Layout of the dgc_rk_step workspace for n = n_elem * n_var * n_p values:
 * byte offsets of the stage states U1, U2 (f64), the stage right-hand side
 * (f64, or f32 for DGC_F32) and, for DGC_F32, the f32 shadow of the stage
 * state (off[3] is 0 otherwise); each part starts on a 256-byte boundary.
 * *total is the size of that part of the workspace (a GATHER buffer follows
 * it).  Lets a caller read the stage right-hand side, e.g. after a batched
 * volume + surface evaluation. */
dgc_status dgc_rk_workspace_layout(int64_t n, int32_t precision, size_t off[4], size_t *total);

/* ---------------------------------------------------------------------- */
/* Batched forms: many meshes of one element type and order per launch      */
/* ---------------------------------------------------------------------- */

/* Describe a batch of n_mesh meshes (same element type and order, each
 * colored) so that one launch per color covers all of them: meshes are
 * disjoint, so the union of their color-c faces is race-free (Algorithm 1).
 * Writes a descriptor (header, one entry per mesh with its device pointers,
 * and per-launch work-group -> mesh maps) into host_desc; the caller copies
 * the same bytes to device memory and passes both copies to the batched
 * calls.  U[i] is mesh i's f64 state, ws[i] its dgc_rk_step workspace
 * (DGC_WS_RK_STEP bytes for `precision`), dt[i] its time step.  Call with
 * host_desc = NULL to get the size.  The descriptor stays valid while the
 * pointed-to buffers live; rebuild it when the batch membership or a dt
 * changes.  Errors: DGC_E_ARG, DGC_E_NOT_COLORED, DGC_E_UNSUPPORTED. */
dgc_status dgc_batch_describe(int32_t n_mesh, const dgc_dmesh *meshes, double *const *U, void *const *ws,
                              const double *dt, int32_t precision, void *host_desc, size_t bytes, size_t *needed);

/* Surface / volume term of every mesh of the batch for SSP-RK3 stage `stage`
 * (0: input U, 1: U1, 2: U2; the f32 form reads the f32 shadow), accumulated
 * into / written to each mesh's stage right-hand side in its workspace. */
dgc_status dgc_surface_rhs_batched(const void *host_desc, const void *dev_desc, int32_t stage, void *stream);
dgc_status dgc_volume_rhs_batched(const void *host_desc, const void *dev_desc, int32_t stage, void *stream);

/* One SSP-RK3 step of every mesh of the batch with its own dt: a fixed
 * sequence of launches (plus one for the f32 shadow), independent of the
 * number of meshes, so it can be captured once in a graph and replayed.
 * When every member has exactly one face of each color (conforming meshes
 * colored with as many colors as an element has faces), each stage is one
 * launch per color, the first also evaluating the volume term where the
 * single-mesh DGC_RK_DEFAULT step does (triangles p <= 3, quadrilaterals,
 * f64 tetrahedra at p = 1) and, in f64, the last writing the stage
 * combination; otherwise 3 x (volume + one launch per color + combine). */
dgc_status dgc_rk_step_batched(const void *host_desc, const void *dev_desc, void *stream);

/* Library build identification (static string). */
const char *dgc_version(void);

#ifdef __cplusplus
}
#endif

#endif /* DGC_H */
