/*
 * fe.h -- C ABI of libfe: finite element numerical integration for
 * first-order approximations on AMD Instinct MI355X (gfx950).
 *
 * What the library computes (K. Banas, F. Kruzel, J. Bielanski,
 * arXiv:1504.01023): for every element e of a batch of elements of one type,
 * the element stiffness matrix A^e (here K) and load vector b^e (here F) of
 * the weak form of Sec. 2.1 (eq. "weak_form"), i.e. eqs. "sm_local" and
 * "lv_local" of Sec. 2.2 with all coefficient terms c^{i;j}, c^{i;0},
 * c^{0;i}, c^{0;0}, d^i, d^0, evaluated by the change of variables to the
 * reference element (eq. "change_of_variables") and the quadrature sum of
 * eq. "quadrature" (Sec. 2.3). Boundary terms are not computed (the paper
 * neglects them, Sec. 2.1). The inputs mirror the procedure's input list of
 * Sec. 2.3: element type, quadrature points and weights, per-element geometry
 * degrees of freedom (vertex coordinates) and problem-dependent coefficient
 * values; the outputs are stored in device memory for later solution steps
 * (Sec. 3.1).
 *
 * Elements: affine 4-node tetrahedra and 6-node linear prisms. Problems:
 * scalar convection-diffusion-reaction, 3-component isotropic linear
 * elasticity, and the general 3-component convection-diffusion-reaction
 * problem in which every coefficient is a matrix over the components (the
 * vector problems of Sec. 2.1 and Sec. 3.3).
 *
 * Conventions (readings where the paper is silent):
 *  - Reference tetrahedron (0,0,0),(1,0,0),(0,1,0),(0,0,1), shape functions
 *    1-xi-eta-zeta, xi, eta, zeta. Reference prism: unit right triangle in
 *    (xi, eta) times zeta in [-1, 1]; nodes 0-2 at zeta = -1 in triangle
 *    order, node v+3 above node v.
 *  - Coefficient index 0 is the function value, 1..3 the x, y, z
 *    derivatives (Algorithm 1). The first index of c^{a;b} pairs with the
 *    test function (row of K), the second with the trial function (column).
 *  - det J is used signed: inverted elements are integrated as written.
 *  - Vector problems number unknowns node-major: row 3*r + alpha.
 *
 * Memory layout (structure of arrays, element index fastest, so that one
 * wavefront reads and writes whole cache lines; Sec. 4.2 discusses coalesced
 * access):
 *  coords  [(v*3 + d) * ld_in + e]            FP64 always
 *  coeffs  per element: [j * ld_in + e]
 *          per point:   [(j * n_q + q) * ld_in + e]
 *          where j runs over the set bits of coef_mask in increasing slot
 *          order ("compact" layout); FP64 for FE_FP64, FP32 for FE_FP32_BULK.
 *  out_K   [k * ld_out + e], k = packed or full entry index (below)
 *  out_F   [i * ld_out + e]
 * Full K: k = row * N + col. Packed (symmetric problems only): the upper
 * triangle row by row, k = row * N - row * (row - 1) / 2 + (col - row) for
 * col >= row. N = number of shape functions times components.
 *
 * Coefficient slots. Scalar problems (20 slots): slot 4*a + b holds c^{a;b}
 * (a, b in 0..3), slot 16 + a holds d^a. Elasticity (5 slots): E, nu, f_x,
 * f_y, f_z, with Lame parameters lambda = E nu / ((1+nu)(1-2nu)),
 * mu = E / (2 (1+nu)) and the body force as d^0 per component. A slot whose
 * bit is set in coef_mask is read from `coeffs`; every other slot takes the
 * value problem->uniform[slot] (zero for absent terms). With
 * FE_COEF_UNIFORM no slot is read from memory.
 * General 3-component problem (FE_VECTOR_CDR, 156 slots): c^{a;b}_{alpha
 * beta} (alpha: component of the test function, beta: of the trial function)
 * is slot (4a+b)*9 + 3 alpha + beta, d^a_alpha is slot 144 + 3a + alpha.
 * coef_mask has one bit per block: bit 4a+b stands for the nine slots of
 * c^{a;b}, bit 16+a for the three of d^a; the compact array holds the slots
 * of the present blocks in slot order, and absent blocks are zero
 * (problem->uniform is not used). Coefficients per element or per point;
 * K is full.
 *
 * Ownership and streams: every device pointer is owned by the caller and must
 * stay valid until the work enqueued on `stream` has completed. Quadrature
 * rules are host memory read during the call only. Calls enqueue work on
 * `stream` and return without synchronising; device faults surface at the
 * caller's next synchronisation. The library never allocates device memory
 * in fe_integrate / fe_integrate_ex.
 *
 * Errors: every entry point returns FE_OK or a status code; on error nothing
 * has been enqueued and the outputs are untouched. fe_last_error() returns a
 * thread-local description of the last failure of the calling thread.
 * Thread safety: all entry points are reentrant.
 */
#ifndef FE_H
#define FE_H

#include <stdint.h>

#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define FE_API __attribute__((visibility("default")))

typedef enum fe_status {
    FE_OK = 0,
    FE_ERR_INVALID_ARG = 1,   /* null pointer with n_elem > 0, negative size,
                                 bad enum, ld < n_elem, bad rule weights */
    FE_ERR_UNSUPPORTED = 2,   /* n_q outside the supported range, misaligned
                                 pointer, combination not built */
    FE_ERR_NOT_SYMMETRIC = 3, /* packed K requested for a non-symmetric problem */
    FE_ERR_HIP = 4,           /* HIP runtime error; see fe_last_error() */
    FE_ERR_CAPACITY = 5       /* batch, server or table capacity exceeded */
} fe_status;

typedef enum fe_elem_type { FE_TET4 = 0, FE_PRISM6 = 1 } fe_elem_type;
typedef enum fe_problem_kind {
    FE_SCALAR_CDR = 0,
    FE_ELASTICITY = 1,
    FE_VECTOR_CDR = 2  /* general 3-component convection-diffusion-reaction */
} fe_problem_kind;

/* FE_FP32_BULK: coordinates stay FP64 and the Jacobian terms (J, det J, its
 * inverse), the global derivatives and vol are computed in FP64, then rounded
 * to FP32; coefficients, accumulation and outputs are FP32. */
typedef enum fe_precision { FE_FP64 = 0, FE_FP32_BULK = 1 } fe_precision;

/* Coefficients constant over the whole element (Sec. 3.3) or given at each
 * quadrature point (the paper's "Poisson" right-hand side, Sec. 4.1). */
/* FE_COEF_FUNCTION (scalar problems): the slots in coef_mask are computed at
 * every point from the parameters of a coefficient function (the "problem
 * dependent parameters used for computing coefficients" of Sec. 2.3):
 * `coeffs` points to FE_COEF_FN_PARAMS FP64 values in device memory, shared
 * by all elements; slot k's value at the physical point x is
 *   p[6k] + p[6k+1] sin(2 pi (p[6k+2] x + p[6k+3] y + p[6k+4] z) + p[6k+5]),
 * and if p[121] != 0 the diffusion block is then replaced by
 * A A^T + p[120] I, A being the computed block (a symmetric positive definite
 * field for p[120] > 0). Evaluated in FP64 in both tiers. */
#define FE_COEF_FN_PARAMS 122
typedef enum fe_coef_mode {
    FE_COEF_UNIFORM = 0,
    FE_COEF_PER_ELEMENT = 1,
    FE_COEF_PER_QP = 2,
    FE_COEF_FUNCTION = 3
} fe_coef_mode;

typedef enum fe_k_format { FE_K_FULL = 0, FE_K_SYM_PACKED = 1 } fe_k_format;

typedef struct fe_problem {
    int32_t kind;        /* fe_problem_kind */
    int32_t precision;   /* fe_precision */
    int32_t coef_mode;   /* fe_coef_mode */
    uint32_t coef_mask;  /* slots read from `coeffs` (ignored for UNIFORM) */
    int32_t k_format;    /* fe_k_format */
    int32_t reserved;    /* must be 0 */
    double uniform[20];  /* values of the slots not read from memory */
} fe_problem;

/* A quadrature rule on the reference element: n_q points xi[q*3 + k] and
 * weights w[q] (Sec. 2.3). Host memory. 1 <= n_q <= FE_MAX_QP. */
#define FE_MAX_QP 8

/* Node blocks of fe_csr_blocks / fe_assemble_csr_blocks: at most this many
 * nodes, elements at them and vertices of those elements per block (the
 * elements and vertices of a block are staged in one workgroup's LDS). */
#define FE_CSR_BLOCK_NODES 256
#define FE_CSR_BLOCK_ELEMS 2432
#define FE_CSR_BLOCK_VERTS 768
typedef struct fe_quad_rule {
    int32_t n_q;
    const double *xi;
    const double *w;
} fe_quad_rule;

/* Launch variant (the tuning parameters of Sec. 4.3: where reference data
 * lives, plus GPU launch shape). Zero fields mean "library default". */
typedef struct fe_variant {
    int32_t wg_size;           /* 64, 128 or 256 threads */
    int32_t elems_per_thread;  /* 1, 2 or 4 contiguous elements (tetrahedra) */
    int32_t ref_in_lds;        /* 1: stage reference tables in LDS; 2: read
                                  them as wave-uniform kernel arguments */
    int32_t nontemporal;       /* 1: streaming (non-temporal) loads and stores;
                                  2: off; 3: streaming stores only */
    int32_t blocks;            /* grid size; 0 = one element group per thread */
    int32_t row_split;         /* passes over the points with the rows of K split
                                  between them (prism elasticity): 1, 2 or 3 */
    int32_t loop_order;        /* order of the point and shape-function loops
                                  (Sec. 3.3, Algorithms 2, 4, 6) for prism
                                  scalar kernels: 1 QSS, 2 SQS, 3 SSQ */
    int32_t lanes;             /* lanes per element (prism scalar QSS): 1, 2, 3
                                  or 6; the element's points are split between
                                  its lanes, each forms the Jacobian terms of its
                                  own points, and the partial K and F are summed
                                  across the lanes (0 = 1) */
} fe_variant;

/* ---------------------------------------------------------------------
 * Integration (Sec. 2.3, Algorithm 1; the element loop parallelised one
 * element per GPU thread as in Sec. 3.2).
 * ------------------------------------------------------------------- */

/* Integrate n_elem elements with leading dimension n_elem for inputs and
 * outputs. (Writes reach HBM fastest when every output row starts on a
 * cache line: fe_integrate_ex with ld_out a multiple of 64 elements and
 * 256-byte aligned outputs.) coeffs may be NULL when no slot is read from memory.
 * n_elem == 0 returns FE_OK without enqueuing anything. */
FE_API int fe_integrate(const fe_problem *problem, fe_elem_type elem_type, int64_t n_elem,
                        const double *coords, const void *coeffs, const fe_quad_rule *quad_rule,
                        void *out_K, void *out_F, hipStream_t stream);

/* As fe_integrate with explicit leading dimensions (ld_in for coords and
 * coeffs, ld_out for out_K and out_F; both >= n_elem), which lets a caller
 * integrate a slice of a larger batch in place, and an optional forced
 * launch variant (NULL = the tuned or default variant). */
FE_API int fe_integrate_ex(const fe_problem *problem, fe_elem_type elem_type, int64_t n_elem,
                           const double *coords, const void *coeffs, int64_t ld_in,
                           const fe_quad_rule *quad_rule, void *out_K, void *out_F, int64_t ld_out,
                           const fe_variant *variant, hipStream_t stream);

/* Indexed geometry: the geometry degrees of freedom of Sec. 2.3 given as a
 * global node array nodes[3 * id + d] (FP64, n_nodes nodes) and int32
 * connectivity conn[v * ld_conn + e] (local vertex v of element e), instead
 * of coordinates duplicated per element. Coefficients (leading dimension
 * ld_in; pass n_elem when none are read) and outputs are laid out as for
 * fe_integrate_ex. Node ids outside [0, n_nodes) are clamped to the range
 * (those elements' results are then meaningless, but nothing faults). */
FE_API int fe_integrate_indexed(const fe_problem *problem, fe_elem_type elem_type,
                                int64_t n_elem, const double *nodes, int64_t n_nodes,
                                const int32_t *conn, int64_t ld_conn, const void *coeffs,
                                int64_t ld_in, const fe_quad_rule *quad_rule, void *out_K,
                                void *out_F, int64_t ld_out, const fe_variant *variant,
                                hipStream_t stream);

/* Natural (element-contiguous) order, the organisation of the element data
 * that Sec. 4.2 discusses (Fig. 1): every element's values are contiguous,
 * element after element:
 *   coords  [e * 3 NV + 3 v + d]              FP64
 *   coeffs  [e * C + j] per element, [e * C + j * n_q + q] per point
 *           (C = fe_coeff_entries; the compact slots of coef_mask)
 *   out_K   [e * fe_k_entries + k],  out_F [e * fe_f_entries + i]
 * The same per-element code as fe_integrate runs on these records (bitwise
 * identical results) in one of two forms: scalar problems with fewer than 16
 * coefficient rows per element copy a tile of 64 elements' inputs to LDS
 * with coalesced loads (one wavefront per workgroup) and write the tile's
 * outputs back as contiguous blocks; the others (16 or more coefficient
 * rows, elasticity, 3-component problems) let each lane read and write its
 * element's records in place. Every problem class is built. Enqueued on
 * `stream`; no allocation. Pointers aligned to their element size. */
FE_API int fe_integrate_natural(const fe_problem *problem, fe_elem_type elem_type, int64_t n_elem,
                                const double *coords, const void *coeffs,
                                const fe_quad_rule *quad_rule, void *out_K, void *out_F,
                                hipStream_t stream);

/* Matrix-free application of the assembled operator, with the element
 * matrices computed in registers and never stored (Sec. 3.1 leaves open
 * whether element matrices are stored at all; Sec. 3.2 assembles the element
 * contributions at their nodes, by colouring for parallel updates):
 *   y[i] += sum over elements e and local nodes r with conn[r][e] = node(i)
 *           of (K^e x^e)_r,      x^e = x at the element's nodes,
 *   b[i] += the same sum of F^e_r            (when b is not NULL).
 * Inputs as for fe_integrate_indexed (nodes, conn, coeffs with leading
 * dimension ld_in, rule). x, y, b: device arrays of n_nodes * n_comp values
 * in the precision of the tier (FP64, or FP32 for FE_FP32_BULK), node-major
 * (index node * n_comp + component, n_comp = 1 scalar, 3 elasticity); x is
 * read, y and b are accumulated into (zero them first). K^e and F^e are those
 * of fe_integrate (same arithmetic, one element per lane), so K^e x^e differs
 * from a product with stored matrices only by the order of the final sums.
 * Colouring: color_ptr (host, n_colors + 1 offsets from 0 to n_elem) splits
 * the elements into colours whose elements share no node (fe_color_elements
 * computes one; the caller orders conn and coeffs accordingly). Each colour
 * is one launch with plain read-add-write updates: the result is
 * deterministic. n_colors = 0: one launch with hardware atomic adds, in
 * whatever order the elements run (the last bits may vary between runs).
 * Built for every problem class; coefficient modes a class lacks return
 * FE_ERR_UNSUPPORTED. Node ids outside [0, n_nodes)
 * are clamped. Enqueued on `stream`; no allocation. */
FE_API int fe_apply_indexed(const fe_problem *problem, fe_elem_type elem_type, int64_t n_elem,
                            const double *nodes, int64_t n_nodes, const int32_t *conn,
                            int64_t ld_conn, const void *coeffs, int64_t ld_in,
                            const fe_quad_rule *quad_rule, const void *x, void *y, void *b,
                            const int64_t *color_ptr, int32_t n_colors, hipStream_t stream);

/* Greedy colouring on the host: elements of one colour share no node. conn
 * is host memory, conn[v * ld_conn + e] (int32). Writes perm[n_elem] (the
 * original element ids, colour by colour, increasing within a colour) and
 * color_ptr[0 .. n_colors] (offsets into perm); color_ptr must hold
 * max_colors + 1 values. Returns the number of colours, or minus a status
 * (FE_ERR_CAPACITY when more than max_colors are needed, FE_ERR_INVALID_ARG
 * for bad arguments or node ids outside [0, n_nodes)). */
FE_API int fe_color_elements(fe_elem_type elem_type, int64_t n_elem, const int32_t *conn,
                             int64_t ld_conn, int64_t n_nodes, int32_t *perm, int64_t *color_ptr,
                             int32_t max_colors);

/* Sparsity pattern of the assembled matrix (Sec. 3.2: the global matrix is
 * the sum of the element matrices at their nodes), built on the host. conn
 * is host memory as for fe_color_elements. Row R = n_comp * node +
 * component (n_comp 1 or 3); a node's rows hold every component of every
 * node that shares an element with it (itself included), columns
 * ascending, and the rows of one node's components have the same columns.
 * Writes row_ptr[0 .. n_nodes * n_comp] (host) and, when col_idx is not
 * NULL, col_idx[0 .. nnz) (host, int32). Returns nnz, or minus a status:
 * FE_ERR_CAPACITY when col_idx is given and nnz > max_nnz,
 * FE_ERR_INVALID_ARG for bad arguments or node ids outside [0, n_nodes).
 * Call once with col_idx = NULL to learn nnz. */
FE_API int64_t fe_csr_pattern(fe_elem_type elem_type, int64_t n_elem, const int32_t *conn,
                              int64_t ld_conn, int64_t n_nodes, int32_t n_comp, int64_t *row_ptr,
                              int32_t *col_idx, int64_t max_nnz);

/* Assembly of the global matrix and load vector into CSR storage, with the
 * element matrices computed in registers and never stored (Sec. 3.1, 3.2):
 *   values[p] += K^e_rs for every element e and local dofs r, s whose
 *                global row and column meet at entry p,
 *   b[i]      += F^e_r at the element's dofs          (when b is not NULL).
 * Inputs as for fe_apply_indexed. row_ptr (n_nodes * n_comp + 1 values,
 * int64), col_idx (nnz, int32), values (nnz) and b (n_nodes * n_comp): device
 * memory; row_ptr and col_idx as fe_csr_pattern writes them (a pattern with
 * fewer entries drops the missing couplings; reads and writes stay inside
 * [0, nnz)). values and b are in the precision of the tier and are
 * accumulated into (zero them first). A packed symmetric K is added to both
 * triangles. Colouring as for fe_apply_indexed: per colour, plain
 * read-add-write (deterministic); n_colors = 0, hardware atomic adds. An
 * element that repeats a node id is degenerate (det J = 0, non-finite K) and
 * its entries are unspecified; nothing outside values and b is written. Built
 * for the problems fe_apply_indexed supports; others return
 * FE_ERR_UNSUPPORTED. Enqueued on `stream`; no allocation. */
FE_API int fe_assemble_csr(const fe_problem *problem, fe_elem_type elem_type, int64_t n_elem,
                           const double *nodes, int64_t n_nodes, const int32_t *conn,
                           int64_t ld_conn, const void *coeffs, int64_t ld_in,
                           const fe_quad_rule *quad_rule, const int64_t *row_ptr,
                           const int32_t *col_idx, int64_t nnz, void *values, void *b,
                           const int64_t *color_ptr, int32_t n_colors, hipStream_t stream);

/* Elements at each node, built on the host for fe_assemble_csr_rows. conn
 * is host memory as for fe_color_elements. Writes inc_ptr[0 .. n_nodes]
 * (host) and, when inc is not NULL, inc[0 .. n_elem * n_vert) (host): the
 * elements at node i are inc[inc_ptr[i] .. inc_ptr[i + 1]), in increasing
 * element order, each coded element * n_vert + local vertex (n_elem *
 * n_vert must fit in int32). Returns n_elem * n_vert, or minus
 * FE_ERR_INVALID_ARG for bad arguments or node ids outside [0, n_nodes). */
FE_API int64_t fe_node_incidence(fe_elem_type elem_type, int64_t n_elem, const int32_t *conn,
                                 int64_t ld_conn, int64_t n_nodes, int64_t *inc_ptr, int32_t *inc);

/* Node blocks for fe_assemble_csr_blocks, built on the host (Sec. 3.2
 * assembles at the nodes; here consecutive nodes share one workgroup, which
 * reads the elements at them once). Tetrahedra, scalar patterns. conn is
 * host memory as for fe_color_elements; inc_ptr and inc (host) as
 * fe_node_incidence writes them; row_ptr and col_idx (host) as
 * fe_csr_pattern writes them with n_comp = 1. Consecutive nodes form a
 * block while the block's nodes (at most FE_CSR_BLOCK_NODES), the elements
 * at them (at most FE_CSR_BLOCK_ELEMS) and those elements' vertices (at most
 * FE_CSR_BLOCK_VERTS) fit; a node order with neighbours close together (a
 * space-filling curve) keeps the blocks full. Writes sizes[0] = n_blocks,
 * sizes[1] = element slots, sizes[2] = vertex slots (host, 3 values); when
 * blk is not NULL also (host):
 *   blk[3 b + 0, 1, 2]  first node, first element slot, first vertex slot of
 *                       block b, for b = 0 .. n_blocks (the last triple
 *                       holds n_nodes and the two totals);
 *   elems[slot]         the global element id of an element slot (a block's
 *                       elements in the order they first appear along its
 *                       nodes' incidence lists);
 *   verts[slot]         the global node id of a vertex slot (ascending
 *                       within a block);
 *   lconn[slot * 4 + v] the block-local index of vertex v of the element in
 *                       that slot;
 *   linc[k]             inc[k] recoded for the node i whose list holds it:
 *                       bits 0-13 block-local element slot * 4 + local vertex,
 *                       bits 14-19, 20-25, 26-31 the positions in row i
 *                       (offsets from row_ptr[i]) of the element's other
 *                       three vertices in increasing local order, 62 where
 *                       the pattern has no such entry, 63 past offset 61
 *                       (n_elem * 4 values).
 * Returns n_blocks, or minus a status: FE_ERR_CAPACITY when one node's
 * elements or their vertices alone exceed a block, FE_ERR_UNSUPPORTED for
 * prisms, FE_ERR_INVALID_ARG for bad arguments. Call once with blk = NULL to
 * learn the sizes. */
FE_API int64_t fe_csr_blocks(fe_elem_type elem_type, int64_t n_elem, const int32_t *conn,
                             int64_t ld_conn, int64_t n_nodes, const int64_t *inc_ptr,
                             const int32_t *inc, const int64_t *row_ptr, const int32_t *col_idx,
                             int64_t *sizes, int64_t *blk, int32_t *elems, int32_t *verts,
                             uint16_t *lconn, uint32_t *linc);

/* The assembly of fe_assemble_csr_rows over node blocks: one workgroup per
 * block (fe_csr_blocks; device copies of blk, elems, verts, lconn, linc and
 * of inc_ptr) first reads the block's vertices (coordinates from nodes) and
 * elements into LDS, once; then each lane adds one node's row, walking the
 * node's incidence list in the same order against LDS, computing each
 * element as fe_assemble_csr_rows does and adding its values at the
 * positions linc carries (the row's first entries accumulate in LDS): the
 * values and b equal that entry point's bit for bit. row_ptr and col_idx
 * must be the pattern the blocks were built from. Other arguments as for
 * fe_assemble_csr_rows (no conn: the blocks carry the connectivity). Scalar
 * problems on tetrahedra; others return FE_ERR_UNSUPPORTED. Enqueued on
 * `stream`; no allocation. */
FE_API int fe_assemble_csr_blocks(const fe_problem *problem, fe_elem_type elem_type,
                                  int64_t n_elem, const double *nodes, int64_t n_nodes,
                                  const void *coeffs, int64_t ld_in,
                                  const fe_quad_rule *quad_rule, const int64_t *row_ptr,
                                  const int32_t *col_idx, int64_t nnz, void *values, void *b,
                                  const int64_t *inc_ptr, int64_t n_blocks, const int64_t *blk,
                                  const int32_t *elems, const int32_t *verts,
                                  const uint16_t *lconn, const uint32_t *linc,
                                  hipStream_t stream);

/* The same assembly as fe_assemble_csr by row ownership: one lane per node
 * adds the node's rows, walking the elements at the node (inc_ptr, inc:
 * device copies of what fe_node_incidence writes) and computing each
 * element's K and F once per vertex (Sec. 3.2 assembles at the nodes; here
 * the node, not the element, is the unit of parallel work). No colours and
 * no atomic operations: each row is written by one lane, in the order of
 * inc, so the result is deterministic. Other arguments as for
 * fe_assemble_csr. Enqueued on `stream`; no allocation. */
FE_API int fe_assemble_csr_rows(const fe_problem *problem, fe_elem_type elem_type, int64_t n_elem,
                                const double *nodes, int64_t n_nodes, const int32_t *conn,
                                int64_t ld_conn, const void *coeffs, int64_t ld_in,
                                const fe_quad_rule *quad_rule, const int64_t *row_ptr,
                                const int32_t *col_idx, int64_t nnz, void *values, void *b,
                                const int64_t *inc_ptr, const int32_t *inc, hipStream_t stream);

/* Assembly of stored element matrices into CSR storage (Sec. 3.2: the
 * global matrix is the sum of the element contributions at their nodes), the
 * step after an integration entry point has stored K and F (device, the
 * problem's precision and k_format): elem_major = 0, rows as fe_integrate
 * writes them, K [k * ld + e] and F [i * ld + e]; elem_major = 1,
 * element-contiguous as fe_integrate_natural writes them, K [e * nk + k] and
 * F [e * nf + i] (ld ignored; the faster input here: a lane reads an
 * element's entries from one or two cache lines). conn [v * ld_conn + e]
 * (device, int32), row_ptr, col_idx,
 * values and b as for fe_assemble_csr, inc_ptr and inc as for
 * fe_assemble_csr_rows. One lane per node adds the node's rows from the
 * stored matrices of the elements at the node (no colours, no atomic
 * operations, nothing recomputed): with the same incidence lists the values
 * equal those of fe_assemble_csr_rows bit for bit. F may be NULL when b is
 * NULL. Enqueued on `stream`; no allocation. */
FE_API int fe_assemble_csr_stored(const fe_problem *problem, fe_elem_type elem_type, int64_t n_elem,
                                  const int32_t *conn, int64_t ld_conn, int64_t n_nodes,
                                  const void *K, const void *F, int64_t ld, int32_t elem_major,
                                  const int64_t *row_ptr,
                                  const int32_t *col_idx, int64_t nnz, void *values, void *b,
                                  const int64_t *inc_ptr, const int32_t *inc, hipStream_t stream);

/* Diagnostic for the signed-determinant convention (det J is used as it
 * is; inverted elements are integrated as written): adds to *count (device
 * int64, zero it first) the number of elements whose det J is not positive
 * at some point of the rule (at the one constant value for tetrahedra).
 * Coordinates as for fe_integrate_ex. Enqueued on `stream`. */
FE_API int fe_count_inverted(fe_elem_type elem_type, int64_t n_elem, const double *coords,
                             int64_t ld_in, const fe_quad_rule *quad_rule, int64_t *count,
                             hipStream_t stream);

/* ---------------------------------------------------------------------
 * Sizes and accounting (Sec. 4.1, table "memory_requirements"; Sec. 4.4,
 * table "accesses_and_operations"). Each returns -1 on invalid input.
 * ------------------------------------------------------------------- */

/* Rows of out_K per element (N*N full, N(N+1)/2 packed). */
FE_API int64_t fe_k_entries(const fe_problem *problem, fe_elem_type elem_type);
/* Rows of out_F per element (N). */
FE_API int64_t fe_f_entries(const fe_problem *problem, fe_elem_type elem_type);
/* Rows of coeffs for this problem and rule size (popcount(mask) per element,
 * times n_q for per-point data; 0 for uniform; FE_COEF_FN_PARAMS values in
 * total, not per element, for the function mode; for FE_VECTOR_CDR nine rows
 * per c block and three per d block in the mask). */
FE_API int64_t fe_coeff_entries(const fe_problem *problem, fe_elem_type elem_type, int n_q);
/* Algorithmic global-memory bytes per element: every input word read once
 * and every output word written once. */
FE_API int64_t fe_bytes_per_element(const fe_problem *problem, fe_elem_type elem_type, int n_q);
/* Storage row of K entry (row, col) in out_K, or -1 when that entry is not
 * stored (lower triangle of a packed K) or out of range. */
FE_API int64_t fe_k_index(const fe_problem *problem, fe_elem_type elem_type, int row, int col);

/* Built-in rules: tetrahedron 1 point (centroid) and 4 points (degree 2),
 * prism 6 points (3-point triangle rule times 2-point Gauss line). Fills *out
 * with pointers to library-owned static arrays. */
FE_API int fe_quad_rule_builtin(fe_elem_type elem_type, int n_q, fe_quad_rule *out);

FE_API const char *fe_status_string(int status);
FE_API const char *fe_last_error(void);

/* The leading dimension to allocate for rows of n_elem elements: n_elem
 * rounded up to a multiple of 256 elements, so that every row of the SoA
 * inputs and outputs starts on a whole cache line (2 KiB of FP64, 1 KiB of
 * FP32) and every wavefront reads and writes whole lines; rows that start
 * mid-line cost the output stores up to a quarter of their rate (measured on
 * MI355X). Any ld >= n_elem is valid. Returns -1 for negative n_elem. */
FE_API int64_t fe_ld_for(int64_t n_elem);

/* Library version as major*10000 + minor*100 + patch. */
FE_API int fe_version(void);

/* ---------------------------------------------------------------------
 * Tuning (parameter-based tuning by exhaustive search over variants,
 * Sec. 4.3).
 * ------------------------------------------------------------------- */

/* Time every valid variant for this problem on the caller's device buffers
 * (layouts as for fe_integrate_ex; the outputs are overwritten with valid
 * results), keep the fastest in the in-process tuning table and return it in
 * *best (and its mean time in ms). Synchronises `stream`. */
FE_API int fe_autotune(const fe_problem *problem, fe_elem_type elem_type, int64_t n_elem,
                       const double *coords, const void *coeffs, int64_t ld_in,
                       const fe_quad_rule *quad_rule, void *out_K, void *out_F, int64_t ld_out,
                       int reps, fe_variant *best, double *best_ms, hipStream_t stream);
/* The variant a call with variant = NULL uses comes from the caller's
 * tuning table (fe_tuning_set, fe_tuning_load, fe_autotune) when it has an
 * entry for the problem shape, else from the built-in table, else the
 * library's base variant. The built-in table is the one measured on MI355X
 * (gfx950) with ROCm 7.x, compiled into the library; it applies when the
 * device the library first plans a launch on is a gfx950 and the HIP runtime
 * has ROCm major version 7 (every variant gives the same results bit for bit;
 * the tables only choose the fastest).
 *
 * fe_tuning_get returns the entry in effect (the caller's, else the
 * built-in one) and FE_ERR_INVALID_ARG when neither exists; fe_tuning_set
 * sets the caller's entry. */
FE_API int fe_tuning_get(const fe_problem *problem, fe_elem_type elem_type, int n_q,
                         fe_variant *out);
FE_API int fe_tuning_set(const fe_problem *problem, fe_elem_type elem_type, int n_q,
                         const fe_variant *v);
/* Persist / restore the caller's tuning table as text (one entry per line;
 * the format of the built-in table). fe_tuning_clear empties the caller's
 * table; the built-in entries stay in effect. */
FE_API int fe_tuning_save(const char *path);
FE_API int fe_tuning_load(const char *path);
FE_API int fe_tuning_clear(void);
/* Whether the built-in table is in effect (1) or not (0, e.g. another GPU
 * architecture or no device); copies the table's architecture name into
 * arch (arch_len bytes, NUL-terminated) and its entry count in effect into
 * *n_entries, either may be NULL. */
FE_API int fe_tuning_builtin(char *arch, int arch_len, int *n_entries);

/* ---------------------------------------------------------------------
 * Persistent batched launches. Elements of the same type, problem and rule
 * form one "kind" (the same-type element sets of Sec. 3.2 that one
 * integration procedure processes in sequence, Algorithm 1). Requests of any
 * size are cut into chunks of chunk_elems elements; fe_batch_launch replays a
 * HIP graph captured at creation (copy of the chunk table to the device, then
 * one persistent kernel per kind whose workgroups walk that kind's chunks),
 * so many uneven requests cost one graph launch. Every element is computed by
 * the same code path as in fe_integrate with the same kernel variant, so the
 * results are bitwise identical to a plain launch of that variant.
 * A fe_batch object is not thread-safe; calls on it must be serialised.
 * ------------------------------------------------------------------- */
#define FE_MAX_BATCH_KINDS 16

typedef struct fe_batch_kind {
    fe_problem problem;   /* coefficient values of uniform slots are fixed per kind */
    int32_t elem_type;    /* fe_elem_type */
    int32_t n_q;          /* rule, host memory, copied at creation */
    const double *xi;
    const double *w;
} fe_batch_kind;

typedef struct fe_batch fe_batch;

/* Create a batcher for n_kinds kinds (1..FE_MAX_BATCH_KINDS) with a table of
 * max_chunks chunks of chunk_elems elements (a multiple of 4) and
 * blocks_per_kind workgroups per persistent kernel (0 = 4096). Allocates the
 * device and pinned host tables and captures the graphs on the current
 * device. Kernel variants come from the tuning table as at creation. */
FE_API int fe_batch_create(const fe_batch_kind *kinds, int n_kinds, int max_chunks,
                           int64_t chunk_elems, int blocks_per_kind, fe_batch **out);
/* Append a request (device pointers, layouts as for fe_integrate_ex) to the
 * pending table. FE_ERR_CAPACITY when its chunks do not fit (launch first);
 * FE_ERR_UNSUPPORTED when a pointer is not aligned to its element size. A
 * request whose leading dimensions or pointers do not suit the kind's
 * elements per lane is processed element by element (same results, bit for
 * bit). Nothing is enqueued until fe_batch_launch. */
FE_API int fe_batch_add(fe_batch *b, int kind, int64_t n_elem, const double *coords,
                        const void *coeffs, int64_t ld_in, void *out_K, void *out_F,
                        int64_t ld_out);
/* Number of pending chunks, or -1 for a NULL batch. */
FE_API int fe_batch_pending(const fe_batch *b);
/* Enqueue the pending chunks on `stream` (one graph launch) and clear the
 * pending table. Blocks only if the table buffer it needs is still in use by
 * the launch before the previous one. */
FE_API int fe_batch_launch(fe_batch *b, hipStream_t stream);
/* Wait for outstanding launches and free everything. */
FE_API int fe_batch_destroy(fe_batch *b);

/* ---------------------------------------------------------------------
 * Batched integration that allocates nothing, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc). One call integrates a list of requests
 * of up to FE_MAX_BATCH_KINDS kinds with the persistent batched kernels of
 * fe_batch_launch, and gives the same results bit for bit as fe_batch_create
 * + fe_batch_add (each request, in order) + fe_batch_launch with the same
 * kinds, chunk_elems and blocks_per_kind.
 *
 * Memory: the chunk table lives in a device array inside the library of
 * 128 + 64 * FE_BATCH_STATIC_MAX_CHUNKS bytes (about 64 KiB), one per device,
 * held until the process ends. The call writes the table there with small
 * table-writing kernels whose arguments carry it, then launches one
 * persistent kernel per kind present, all on `stream`; it calls no
 * allocating routine and never waits. The caller owns every input and output
 * and keeps them valid until the stream work completes; `kinds` (and their
 * rules) and `requests` are host memory read during the call only.
 *
 * Every call on one device shares that device's table and overwrites it:
 * calls on the same stream are ordered, but calls that overlap on one device
 * (from two streams, or from two host threads) race and give wrong results.
 * Serialise them.
 *
 * Errors: FE_ERR_CAPACITY when the requests need more than
 * FE_BATCH_STATIC_MAX_CHUNKS chunks of chunk_elems elements (use larger
 * chunks or split the list); the other codes as for fe_batch_create and
 * fe_batch_add. Every check is made before anything is enqueued, so on error
 * nothing runs and the outputs are untouched.
 * ------------------------------------------------------------------- */
#define FE_BATCH_STATIC_MAX_CHUNKS 1024

typedef struct fe_batch_request {
    int32_t kind;              /* index into `kinds` */
    int32_t reserved;          /* must be 0 */
    int64_t n_elem;
    const double *coords;      /* layouts as for fe_integrate_ex */
    const void *coeffs;
    int64_t ld_in;
    void *out_K;
    void *out_F;
    int64_t ld_out;
} fe_batch_request;

FE_API int fe_batch_integrate_static(const fe_batch_kind *kinds, int n_kinds,
                                     const fe_batch_request *requests, int n_requests,
                                     int64_t chunk_elems, int blocks_per_kind,
                                     hipStream_t stream);

/* ---------------------------------------------------------------------
 * Continuous-batching server. Requests (one mesh of one kind each) are
 * submitted at any time; a scheduler thread admits them in arrival order
 * while a slot is free and their device bytes (inputs + outputs) fit in the
 * HBM budget, copies host inputs to the device on a copy stream, and fuses
 * the ready requests' chunks into persistent batched launches (fe_batch), so
 * work that arrives while other requests run joins the next launch. Outputs
 * stay resident on the device for the consumer (Sec. 3.1: element matrices
 * are kept in memory available to the following solution steps) until
 * fe_server_release. Host inputs must stay valid until the request
 * completes; for asynchronous copies they should be pinned.
 * ------------------------------------------------------------------- */
#define FE_SERVER_GPU 0
#define FE_SERVER_FAKE 1  /* timing model on the host, no device: for tests */

typedef struct fe_server fe_server;

typedef struct fe_server_config {
    const fe_batch_kind *kinds;  /* copied at creation */
    int32_t n_kinds;
    int32_t max_slots;           /* requests admitted and not yet complete */
    int64_t hbm_budget_bytes;    /* device arena for inputs and outputs */
    int32_t max_chunks;          /* chunks per launch (tick) */
    int32_t blocks_per_kind;     /* persistent workgroups per kind (0 = 4096) */
    int64_t chunk_elems;         /* elements per chunk, multiple of 4 */
    int32_t backend;             /* FE_SERVER_GPU or FE_SERVER_FAKE */
    int32_t reserved;
    double fake_ns_per_elem;     /* FAKE: device time per element */
    double fake_h2d_bytes_per_s; /* FAKE: copy rate */
    double fake_tick_overhead_s; /* FAKE: fixed cost per launch */
} fe_server_config;

typedef struct fe_request {
    int32_t kind;
    int32_t inputs_on_device;  /* 0: host inputs, copied to the device by the
                                  server; 1: device inputs used in place */
    int64_t n_elem;
    const double *coords;      /* layouts as for fe_integrate_ex */
    const void *coeffs;
    int64_t ld_in;             /* leading dimension of coords/coeffs, >= n_elem */
    uint64_t tag;              /* caller's value, returned in the completion */
} fe_request;

typedef struct fe_completion {
    uint64_t id;
    uint64_t tag;
    int32_t status;            /* FE_OK, or why the request failed */
    int32_t kind;
    int64_t n_elem;
    void *out_K;               /* device, [k * ld_out + e]; valid until release */
    void *out_F;
    int64_t ld_out;
    double t_submit, t_admit, t_ready, t_done;  /* fe_server_now() clock, s */
} fe_completion;

typedef struct fe_server_stats {
    int64_t submitted, admitted, completed, failed, in_queue, in_flight;
    int64_t bytes_in_use, bytes_peak, elements_done, ticks;
    double p50_s, p99_s, mean_s;                    /* submit -> done */
    double mean_queue_s, mean_h2d_s, mean_device_s; /* breakdown */
} fe_server_stats;

/* Create a server (on the current device for FE_SERVER_GPU: allocates the
 * arena, streams and the batched graphs once). */
FE_API int fe_server_create(const fe_server_config *cfg, fe_server **out);
/* Queue a request; *id receives its identifier. A request larger than the
 * whole budget completes with FE_ERR_CAPACITY without affecting others. */
FE_API int fe_server_submit(fe_server *s, const fe_request *req, uint64_t *id);
/* Move up to max completions to out, waiting up to timeout_s seconds for the
 * first; returns the number moved, or a negative status. */
FE_API int fe_server_poll(fe_server *s, fe_completion *out, int max, double timeout_s);
/* The consumer is done with a completed request's outputs: free its memory.
 * Returns once the scheduler has put the memory back into the budget (the
 * statistics show it); the outputs must not be used after this call. */
FE_API int fe_server_release(fe_server *s, uint64_t id);
FE_API int fe_server_stats_get(fe_server *s, fe_server_stats *out);
FE_API int fe_server_reset_stats(fe_server *s);
/* Stop the scheduler, wait for the device and free everything. */
FE_API int fe_server_destroy(fe_server *s);
/* The server's clock (steady, seconds). */
FE_API double fe_server_now(void);

/* ---------------------------------------------------------------------
 * Measurement helper: copy n_bytes (a multiple of 16) from src to dst with
 * a plain streaming kernel, used to calibrate HBM counters and the achieved
 * copy ceiling beside the integration kernels.
 * ------------------------------------------------------------------- */
FE_API int fe_stream_copy(void *dst, const void *src, int64_t n_bytes, hipStream_t stream);

/* Measurement helper: the bare access pattern of an integration kernel,
 * with its arithmetic removed. For each element e < n, reads rows_in FP64
 * rows in[r * ld + e] and writes rows_out rows out[w * ld + e] of out_bytes
 * (8: FP64, 4: FP32) with the value sum_r in[r][e] + w, one element per
 * lane, streaming loads and stores (device memory, rows of ld >= n
 * elements). Its rate is the memory system's rate for that pattern: the
 * ceiling of an integration kernel that moves the same rows. Returns
 * FE_ERR_INVALID_ARG for bad sizes or misaligned pointers. Enqueued on
 * `stream`. */
FE_API int fe_stream_pattern(const double *in, int32_t rows_in, void *out, int32_t rows_out,
                             int32_t out_bytes, int64_t n, int64_t ld, hipStream_t stream);

#ifdef __cplusplus
}
#endif

#endif /* FE_H */
