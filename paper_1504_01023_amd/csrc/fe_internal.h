// fe_internal.h -- structures shared by the host dispatcher (fe_api.cpp) and
// the kernel translation units. Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <tuple>
#include <utility>

#include "fe.h"

namespace fe {

// Launches the __global__ function k with the given arguments, converted to
// its parameter types, and returns the launch's own status. (The thread's
// last error is not consulted: it may hold a failure of the caller's earlier
// work, which the library neither reports as its own nor clears.)
template <typename... P, typename... A>
inline hipError_t launch_kernel(void (*k)(P...), dim3 grid, dim3 block, size_t lds,
                                hipStream_t stream, A &&...args)
{
    std::tuple<P...> vals(std::forward<A>(args)...);
    void *ptrs[sizeof...(P) > 0 ? sizeof...(P) : 1];
    std::apply([&ptrs](auto &...v) {
        int i = 0;
        ((ptrs[i++] = static_cast<void *>(&v)), ...);
    }, vals);
    return hipLaunchKernel(reinterpret_cast<const void *>(k), grid, block, ptrs, lds, stream);
}

// Workgroups are handed to the chip's 8 XCDs in turn (workgroup b to XCD
// b mod 8), and each XCD has its own L2. The logical workgroup index
// xcd_block(b, G) gives every XCD one contiguous range of the work (nodes,
// or elements in mesh order), so neighbours, which share elements and
// vertex data, are read through the same L2. A bijection of [0, G): XCD x
// takes q + 1 consecutive indices if x < G mod 8, else q (q = G / 8).
__device__ __forceinline__ int64_t xcd_block(int64_t b, int64_t G)
{
    const int64_t x = b % 8, k = b / 8, q = G / 8, r = G % 8;
    return x < r ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

// Term groups of the scalar weak form (Sec. 2.1, eq. "weak_form"); a kernel
// is compiled for a set of groups and the code for absent groups is removed.
enum TermBits : int {
    T_DIFF = 1,   // c^{i;j}, slots 5-7, 9-11, 13-15
    T_CONVA = 2,  // c^{i;0}, slots 4, 8, 12 (derivative of the test function)
    T_CONVB = 4,  // c^{0;j}, slots 1, 2, 3 (derivative of the trial function)
    T_MASS = 8,   // c^{0;0}, slot 0
    T_DGRAD = 16, // d^i, slots 17-19
    T_D0 = 32,    // d^0, slot 16
};
constexpr int TS_POISSON = T_DIFF | T_D0;
constexpr int TS_FULL = 63;
constexpr int TS_ELAST = 64;  // marker for the elasticity kernels

// Where coefficient values come from.
enum ModeKind : int {
    M_UNIFORM = 0,     // kernel arguments only
    M_ELEM = 1,        // per element, every slot of the term set in memory (dense)
    M_QP = 2,          // per point, dense
    M_ELEM_MIXED = 3,  // per element, slot by slot from memory or arguments
    M_QP_MIXED = 4,    // per point, slot by slot
    M_FUNC = 5,        // per point, computed from coefficient-function parameters
};

enum RefKind : int { REF_KARG = 0, REF_LDS = 1 };

constexpr uint32_t slots_of_terms(int terms)
{
    uint32_t m = 0;
    if (terms & T_DIFF) m |= (1u << 5) | (1u << 6) | (1u << 7) | (1u << 9) | (1u << 10) |
                             (1u << 11) | (1u << 13) | (1u << 14) | (1u << 15);
    if (terms & T_CONVA) m |= (1u << 4) | (1u << 8) | (1u << 12);
    if (terms & T_CONVB) m |= (1u << 1) | (1u << 2) | (1u << 3);
    if (terms & T_MASS) m |= 1u;
    if (terms & T_DGRAD) m |= (1u << 17) | (1u << 18) | (1u << 19);
    if (terms & T_D0) m |= (1u << 16);
    if (terms & TS_ELAST) m = 31u;
    return m;
}

// Kernel arguments, passed by value (they live in the kernel-argument
// segment and are read with wave-uniform scalar loads). Reference data are
// evaluated on the host from the caller's rule: shape-function values and
// reference derivatives at every point, weights, and for tetrahedra the
// weighted moments W = sum_q w_q, m_r = sum_q w_q phi_r(xi_q),
// M_rs = sum_q w_q phi_r(xi_q) phi_s(xi_q).
struct KArgs {
    const double *coords;
    const void *coeffs;
    void *out_K;
    void *out_F;
    int64_t n_elem;
    int64_t ld_in;
    int64_t ld_out;
    int32_t n_q;
    int32_t k_packed;
    int32_t col[20];     // compact column of each slot in coeffs, -1 = uniform
    double uniform[20];
    double w[FE_MAX_QP];
    double phi[FE_MAX_QP][6];
    double dphi[FE_MAX_QP][6][3];
    float phi_f[FE_MAX_QP][6];  // the same tables rounded to FP32 (FP32 tier)
    float dphi_f[FE_MAX_QP][6][3];
    double Wsum;
    double m[6];
    double M[6][6];
};
static_assert(sizeof(KArgs) < 4096, "kernel arguments must stay below 4 KiB");

// Identifies one compiled kernel.
struct KernelKey {
    int elem;      // fe_elem_type
    int kind;      // fe_problem_kind
    int prec;      // fe_precision
    int terms;     // term set (scalar) or TS_ELAST
    int mode;      // ModeKind
    int packed;    // 1 = packed K store
    int vec;       // elements per thread
    int nt;        // non-temporal memory operations
    int ref;       // RefKind
    int nq;        // compiled point count, 0 = runtime loop
    int split;     // passes over the points (row split of K), 1, 2 or 3
    int order;     // loop order (1 QSS, 2 SQS, 3 SSQ)
    int lanes;     // lanes per element (1, or 2, 3, 6 for the prism point split)
};

typedef hipError_t (*LaunchFn)(const KArgs &, unsigned grid, unsigned block, hipStream_t);

// Persistent batched launches: a table of chunks (element ranges of many
// requests), grouped by kind; kind k owns chunks [begin[k], end[k]).
constexpr int MAX_BATCH_KINDS = 16;
struct Chunk {
    const double *coords;
    const void *coeffs;
    void *out_K;
    void *out_F;
    int64_t ld_in;
    int64_t ld_out;
    int64_t e0;  // first element of the chunk (offset into the arrays above)
    int64_t n;   // elements in the chunk; negated when the rows or pointers do
                 // not suit the kind's elements per lane (element by element)
};
static_assert(sizeof(Chunk) == 64, "chunk records are one 64-byte line");
struct BatchHeader {
    int32_t begin[MAX_BATCH_KINDS];
    int32_t end[MAX_BATCH_KINDS];
};
typedef hipError_t (*BatchLaunchFn)(const KArgs &, const BatchHeader *, const Chunk *, int kind,
                              unsigned grid, unsigned block, hipStream_t);

// Indexed geometry: coordinates gathered from a node array through
// connectivity instead of being duplicated per element.
struct IdxArgs {
    const double *nodes;   // [3 * id + d]
    const int32_t *conn;   // [v * ld_conn + e]
    int64_t ld_conn;
    uint32_t n_nodes;      // ids are clamped to [0, n_nodes)
};
typedef hipError_t (*IdxLaunchFn)(const KArgs &, const IdxArgs &, unsigned grid, unsigned block,
                            hipStream_t);

// Matrix-free application: nodal vectors in the precision of the tier,
// node-major (node * components + component).
struct ApplyArgs {
    const void *x;  // read
    void *y;        // y += assembled K x
    void *b;        // b += assembled F, or nullptr
    // Assembly into a CSR matrix instead (vals != nullptr; x and y unused):
    // vals[row_ptr[R] .. row_ptr[R + 1]) hold row R's entries, columns
    // col_idx[] ascending, each node's components in consecutive rows with
    // the same columns (the pattern fe_csr_pattern builds).
    const int64_t *row_ptr;
    const int32_t *col_idx;
    int64_t nnz;
    void *vals;
    // Row ownership (inc != nullptr; the launch then runs over nodes): the
    // elements at node i are inc[inc_ptr[i] .. inc_ptr[i + 1]), each coded
    // element * n_vert + local vertex; the node's thread adds its rows.
    const int64_t *inc_ptr;
    const int32_t *inc;
    int64_t n_own;  // nodes in this launch
    // Row ownership over node blocks (blk != nullptr; one workgroup per
    // block, tetrahedra): block b owns nodes [blk[3b], blk[3b + 3]), its
    // element slots are [blk[3b + 1], blk[3b + 4]) and its vertex slots
    // [blk[3b + 2], blk[3b + 5]). blk_elems / blk_verts give a slot's global
    // element / node id, blk_conn[slot * 4 + v] the block-local index of the
    // element's vertex v, and linc[k] (aligned with inc) codes the incidence
    // inc[k] with the row positions of the element's vertices (the code of
    // fe_csr_blocks_kernel).
    const int64_t *blk;
    const int32_t *blk_elems;
    const int32_t *blk_verts;
    const uint16_t *blk_conn;
    const uint32_t *linc;
};
typedef hipError_t (*ApplyLaunchFn)(const KArgs &, const IdxArgs &, const ApplyArgs &, int atomic,
                              unsigned grid, unsigned block, hipStream_t);

// Natural-order (element-contiguous) inputs and outputs: every element's
// coordinates, coefficients, K and F are contiguous, element after element.
struct AosArgs {
    int32_t coef_rows;  // coefficient values per element
    int32_t k_rows;     // K entries per element
    int32_t f_rows;     // F entries per element
    int32_t tsize;      // bytes per coefficient / output value
    // ceil(2^32 / rows): i / rows = umulhi(i, magic) exactly for the tile
    // indices used (i < 2^16, rows < 2^16)
    uint32_t coef_magic, k_magic, f_magic;
    // 1: no LDS tile; each lane runs the per-element code on its element's
    // contiguous records in place (stream pointers at the element, leading
    // dimension 1), grid over elements with 256 lanes per workgroup
    int32_t direct;
};
typedef hipError_t (*AosLaunchFn)(const KArgs &, const AosArgs &, unsigned grid, size_t lds_bytes,
                            hipStream_t);
constexpr int AOS_TILE = 64;  // elements per workgroup tile (one wavefront)

struct KernelEntry {
    KernelKey key;
    LaunchFn launch;
    const void *func;
    BatchLaunchFn batch;  // persistent batched form, or nullptr
    IdxLaunchFn idx;      // indexed-geometry form, or nullptr
    ApplyLaunchFn apply;  // matrix-free form (one element per lane), or nullptr
    AosLaunchFn aos;      // natural-order form (one element per lane), or nullptr
};

// Registration of compiled kernels (each kernel translation unit registers
// its instantiations at load time).
void register_kernel(const KernelEntry &e);
const KernelEntry *find_kernel(const KernelKey &k);
int kernel_count();
const KernelEntry *kernel_at(int i);

}  // namespace fe
