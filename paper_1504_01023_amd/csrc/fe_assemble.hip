// fe_assemble.hip -- assembly of stored element matrices into CSR storage:
// one lane per node adds the node's rows from the K and F of the elements at
// the node (the global matrix as the sum of the element contributions at
// their nodes). The element matrices are those the integration entry points
// store; nothing is recomputed.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>

#include "fe.h"
#include "fe_api_internal.h"

namespace {

using namespace fe;

struct AsmArgs {
    const void *K;  // entry k of element e at [k * ks + e * es]
    const void *F;  // entry i of element e at [i * fs + e * fes]
    int64_t ks, es, fs, fes;
    const int32_t *conn;  // [v * ld_conn + e]
    int64_t ld_conn;
    uint32_t n_nodes;
    int64_t n_elem;
    const int64_t *row_ptr;
    const int32_t *col_idx;
    int64_t nnz;
    void *vals;
    void *b;
    const int64_t *inc_ptr;
    const int32_t *inc;  // element * NV + local vertex
    int64_t n_own;
};

// Storage row of K entry (r, s) of an N x N matrix: row-major, or the packed
// upper triangle r N - r (r - 1) / 2 + s - r (r <= s; the mirror otherwise).
__device__ __forceinline__ int k_row(int N, bool packed, int r, int s)
{
    if (!packed)
        return r * N + s;
    const int lo = r < s ? r : s, hi = r < s ? s : r;
    return lo * N - lo * (lo - 1) / 2 + (hi - lo);
}

template <int NV, int NC, typename T, bool PACKED, bool WITH_B>
__global__ __launch_bounds__(256) void assemble_stored_kernel(AsmArgs g)
{
    constexpr int N = NV * NC;
    constexpr int RC = 32;  // node columns of a row held in registers
    const T *K = static_cast<const T *>(g.K);
    const T *F = static_cast<const T *>(g.F);
    T *vals = static_cast<T *>(g.vals);
    T *b = static_cast<T *>(g.b);
    const int64_t nnz = g.nnz;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < g.n_own; i += stride) {
        // row bounds clamped into [0, nnz]: never a fault
        int64_t r0 = g.row_ptr[NC * i], r1 = g.row_ptr[NC * i + 1];
        r0 = r0 < 0 ? 0 : (r0 > nnz ? nnz : r0);
        r1 = r1 < r0 ? r0 : (r1 > nnz ? nnz : r1);
        const int64_t len = r1 - r0;
        int32_t cols[RC];
#pragma unroll
        for (int k = 0; k < RC; ++k)
            cols[k] = (int64_t)k * NC < len ? g.col_idx[r0 + (int64_t)k * NC] : -1;
        T fb[NC];
#pragma unroll
        for (int al = 0; al < NC; ++al)
            fb[al] = T(0);
        const int64_t k0 = g.inc_ptr[i], k1 = g.inc_ptr[i + 1];
        // software pipeline over the node's elements: the code of element
        // k + 2 and the vertex ids of element k + 1 are loaded while element
        // k is processed; element k's K entries are loaded before its
        // positions in the row are searched
        auto code_at = [&](int64_t k) -> uint32_t { return k < k1 ? (uint32_t)g.inc[k] : 0u; };
        auto ids_of = [&](uint32_t code, uint32_t (&id)[NV]) {
            const int64_t e = code / NV < g.n_elem ? code / NV : 0;
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const uint32_t u = (uint32_t)g.conn[v * g.ld_conn + e];
                id[v] = u < g.n_nodes ? u : g.n_nodes - 1;  // clamped: never a fault
            }
        };
        uint32_t c_cur = code_at(k0), c_next = code_at(k0 + 1);
        uint32_t id_cur[NV];
        ids_of(c_cur, id_cur);
        for (int64_t k = k0; k < k1; ++k) {
            const uint32_t code = c_cur;
            uint32_t id[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v)
                id[v] = id_cur[v];
            const int64_t e = code / NV;
            const int lv = (int)(code % NV);
            const bool valid = e < g.n_elem;
            const int64_t ee = valid ? e : 0;
            T kv[NC][N];
#pragma unroll
            for (int al = 0; al < NC; ++al)
#pragma unroll
                for (int s = 0; s < N; ++s)
                    kv[al][s] = K[(int64_t)k_row(N, PACKED, NC * lv + al, s) * g.ks + ee * g.es];
            const uint32_t c_after = code_at(k + 2);
            if (k + 1 < k1)
                ids_of(c_next, id_cur);
            c_cur = c_next;
            c_next = c_after;
            if (!valid)
                continue;
            int32_t slot[NV];
#pragma unroll
            for (int u = 0; u < NV; ++u)
                slot[u] = -1;
#pragma unroll
            for (int c = 0; c < RC; ++c)
#pragma unroll
                for (int u = 0; u < NV; ++u)
                    if (cols[c] == (int32_t)(NC * id[u]))
                        slot[u] = c * NC;
            for (int64_t j = (int64_t)RC * NC; j < len; j += NC) {
                const int32_t c = g.col_idx[r0 + j];
#pragma unroll
                for (int u = 0; u < NV; ++u)
                    if (c == (int32_t)(NC * id[u]))
                        slot[u] = (int32_t)j;
            }
#pragma unroll
            for (int al = 0; al < NC; ++al) {
                T old[N];
                int64_t p[N];
#pragma unroll
                for (int s = 0; s < N; ++s) {
                    const int o = slot[s / NC];
                    const int64_t q = r0 + (int64_t)al * len + o + s % NC;
                    p[s] = (o >= 0 && q < nnz) ? q : -1;
                    old[s] = p[s] >= 0 ? vals[p[s]] : T(0);
                }
#pragma unroll
                for (int s = 0; s < N; ++s)
                    if (p[s] >= 0)
                        vals[p[s]] = old[s] + kv[al][s];
                if constexpr (WITH_B)
                    fb[al] += F[(int64_t)(NC * lv + al) * g.fs + e * g.fes];
            }
        }
        if constexpr (WITH_B) {
#pragma unroll
            for (int al = 0; al < NC; ++al)
                b[NC * i + al] += fb[al];
        }
    }
}

// Scalar problems (one unknown per node). The first RC entries of the node's
// row stay in registers from the first element at the node to the last,
// starting from their stored values, so the loop over the elements carries
// no load-add-store through memory; the K row and vertex ids of the next
// element load while the current one is added. Every element adds to each
// held entry either its K value or -0 (x + (-0) is x for every x, -0
// included), so each entry receives the same additions in the same order as
// the read-add-write form above and the results are bitwise the same.
// Entries beyond the first RC keep the read-add-write form.
template <int NV, typename T, bool PACKED, bool WITH_B>
__global__ __launch_bounds__(256) void assemble_scalar_kernel(AsmArgs g)
{
    constexpr int RC = 32;
    const T *K = static_cast<const T *>(g.K);
    const T *F = static_cast<const T *>(g.F);
    T *vals = static_cast<T *>(g.vals);
    T *b = static_cast<T *>(g.b);
    const int64_t nnz = g.nnz;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x; i < g.n_own;
         i += stride) {
        // row bounds clamped into [0, nnz]: never a fault
        int64_t r0 = g.row_ptr[i], r1 = g.row_ptr[i + 1];
        r0 = r0 < 0 ? 0 : (r0 > nnz ? nnz : r0);
        r1 = r1 < r0 ? r0 : (r1 > nnz ? nnz : r1);
        const int64_t len = r1 - r0;
        int32_t cols[RC];
        T acc[RC];
#pragma unroll
        for (int c = 0; c < RC; ++c) {
            const bool in = c < len;
            cols[c] = in ? g.col_idx[r0 + c] : -1;
            acc[c] = in ? vals[r0 + c] : T(0);
        }
        T fb = T(0);
        const int64_t k0 = g.inc_ptr[i], k1 = g.inc_ptr[i + 1];
        auto code_at = [&](int64_t k) -> uint32_t { return k < k1 ? (uint32_t)g.inc[k] : 0u; };
        auto load = [&](uint32_t code, uint32_t (&id)[NV], T (&kv)[NV]) {
            const int64_t e = code / NV < g.n_elem ? code / NV : 0;
            const int lv = (int)(code % NV);
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const uint32_t u = (uint32_t)g.conn[v * g.ld_conn + e];
                id[v] = u < g.n_nodes ? u : g.n_nodes - 1;  // clamped: never a fault
            }
#pragma unroll
            for (int s = 0; s < NV; ++s)
                kv[s] = K[(int64_t)k_row(NV, PACKED, lv, s) * g.ks + e * g.es];
        };
        uint32_t c_cur = code_at(k0), c_next = code_at(k0 + 1);
        uint32_t id_cur[NV];
        T kv_cur[NV];
        load(c_cur, id_cur, kv_cur);
        for (int64_t k = k0; k < k1; ++k) {
            const uint32_t code = c_cur;
            uint32_t id[NV];
            T kv[NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                id[v] = id_cur[v];
                kv[v] = kv_cur[v];
            }
            const uint32_t c_after = code_at(k + 2);
            if (k + 1 < k1)
                load(c_next, id_cur, kv_cur);
            c_cur = c_next;
            c_next = c_after;
            const int64_t e = code / NV;
            if (e >= g.n_elem)
                continue;
            // held entries in chunks of 8; a chunk no lane of the wave has
            // entries in (its columns are all -1) is skipped by the whole wave
#pragma unroll
            for (int q = 0; q < RC / 8; ++q) {
                if (q > 0 && !__any(len > 8 * q))
                    break;
#pragma unroll
                for (int c = 8 * q; c < 8 * q + 8; ++c) {
                    T add = T(-0.0);
#pragma unroll
                    for (int u = 0; u < NV; ++u)
                        if (cols[c] == (int32_t)id[u])
                            add = kv[u];
                    acc[c] += add;
                    // keeps each column's compares beside their selects (all
                    // compares hoisted together need more mask registers than
                    // there are)
                    __builtin_amdgcn_sched_barrier(0);
                }
            }
            for (int64_t j = RC; j < len; ++j) {
                const int32_t c = g.col_idx[r0 + j];
#pragma unroll
                for (int u = 0; u < NV; ++u)
                    if (c == (int32_t)id[u])
                        vals[r0 + j] = vals[r0 + j] + kv[u];
            }
            if constexpr (WITH_B)
                fb += F[(int64_t)(code % NV) * g.fs + e * g.fes];
        }
        // written back where a column is held (cols[c] is -1 for c >= len; a
        // negative column matches no node, so its entry is unchanged)
#pragma unroll
        for (int c = 0; c < RC; ++c)
            if (cols[c] >= 0)
                vals[r0 + c] = acc[c];
        if constexpr (WITH_B)
            b[i] += fb;
    }
}

// Scalar problems take the register-row kernel, 3-component ones the
// read-add-write kernel.
template <int NV, int NC, typename T, bool PACKED, bool WITH_B>
hipError_t launch_one(const AsmArgs &g, unsigned grid, hipStream_t stream)
{
    if constexpr (NC == 1)
        return launch_kernel(&assemble_scalar_kernel<NV, T, PACKED, WITH_B>, dim3(grid), dim3(256), 0,
                           stream, g);
    else
        return launch_kernel(&assemble_stored_kernel<NV, NC, T, PACKED, WITH_B>, dim3(grid), dim3(256),
                           0, stream, g);
}

template <int NV, int NC, typename T>
hipError_t launch(const AsmArgs &g, bool packed, unsigned grid, hipStream_t stream)
{
    if (packed && g.b)
        return launch_one<NV, NC, T, true, true>(g, grid, stream);
    else if (packed)
        return launch_one<NV, NC, T, true, false>(g, grid, stream);
    else if (g.b)
        return launch_one<NV, NC, T, false, true>(g, grid, stream);
    else
        return launch_one<NV, NC, T, false, false>(g, grid, stream);
}

bool aligned_to(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

}  // namespace

extern "C" int fe_assemble_csr_stored(const fe_problem *problem, fe_elem_type elem_type,
                                      int64_t n_elem, const int32_t *conn, int64_t ld_conn,
                                      int64_t n_nodes, const void *K, const void *F, int64_t ld,
                                      int32_t elem_major, const int64_t *row_ptr,
                                      const int32_t *col_idx, int64_t nnz,
                                      void *values, void *b, const int64_t *inc_ptr,
                                      const int32_t *inc, hipStream_t stream)
{
    const int64_t nk = fe_k_entries(problem, elem_type);
    if (nk < 0)
        return fail(FE_ERR_INVALID_ARG, "bad problem or element type");
    const int nv = elem_type == FE_TET4 ? 4 : 6;
    if (n_elem < 0 || n_elem > 0x7fffffffLL / nv)
        return fail(FE_ERR_INVALID_ARG, "n_elem out of range (element * vertex codes fit in int32)");
    if (nnz < 0)
        return fail(FE_ERR_INVALID_ARG, "nnz is negative");
    if (n_elem == 0)
        return FE_OK;
    if (!conn || !K || !row_ptr || !col_idx || !values || !inc_ptr || !inc || (b && !F))
        return fail(FE_ERR_INVALID_ARG, "NULL pointer (F is needed when b is given)");
    if (elem_major != 0 && elem_major != 1)
        return fail(FE_ERR_INVALID_ARG, "elem_major must be 0 or 1");
    if (n_nodes < 1 || n_nodes > 0x7fffffffLL || ld_conn < n_elem || (!elem_major && ld < n_elem))
        return fail(FE_ERR_INVALID_ARG, "need 1 .. 2^31-1 nodes and leading dimensions >= n_elem");
    const size_t tsz = problem->precision == FE_FP64 ? 8 : 4;
    if (!aligned_to(K, tsz) || !aligned_to(F, tsz) || !aligned_to(values, tsz) || !aligned_to(b, tsz) ||
        !aligned_to(conn, 4) || !aligned_to(col_idx, 4) || !aligned_to(inc, 4) ||
        !aligned_to(row_ptr, 8) || !aligned_to(inc_ptr, 8))
        return fail(FE_ERR_UNSUPPORTED, "pointers must be aligned to their element size");
    AsmArgs g;
    std::memset(&g, 0, sizeof(g));
    const int64_t nf = fe_f_entries(problem, elem_type);
    g.K = K;
    g.F = F;
    g.ks = elem_major ? 1 : ld;
    g.es = elem_major ? nk : 1;
    g.fs = elem_major ? 1 : ld;
    g.fes = elem_major ? nf : 1;
    g.conn = conn;
    g.ld_conn = ld_conn;
    g.n_nodes = (uint32_t)n_nodes;
    g.n_elem = n_elem;
    g.row_ptr = row_ptr;
    g.col_idx = col_idx;
    g.nnz = nnz;
    g.vals = values;
    g.b = b;
    g.inc_ptr = inc_ptr;
    g.inc = inc;
    g.n_own = n_nodes;
    const bool packed = problem->k_format == FE_K_SYM_PACKED;
    const int nc = problem->kind == FE_SCALAR_CDR ? 1 : 3;
    int64_t grid = (n_nodes + 255) / 256;
    if (grid > 0x7fffffff)
        grid = 0x7fffffff;
    const bool fp64 = problem->precision == FE_FP64;
    hipError_t err;
    if (nv == 4 && nc == 1)
        err = fp64 ? launch<4, 1, double>(g, packed, (unsigned)grid, stream)
                   : launch<4, 1, float>(g, packed, (unsigned)grid, stream);
    else if (nv == 4)
        err = fp64 ? launch<4, 3, double>(g, packed, (unsigned)grid, stream)
                   : launch<4, 3, float>(g, packed, (unsigned)grid, stream);
    else if (nc == 1)
        err = fp64 ? launch<6, 1, double>(g, packed, (unsigned)grid, stream)
                   : launch<6, 1, float>(g, packed, (unsigned)grid, stream);
    else
        err = fp64 ? launch<6, 3, double>(g, packed, (unsigned)grid, stream)
                   : launch<6, 3, float>(g, packed, (unsigned)grid, stream);
    if (err != hipSuccess)
        return fail(FE_ERR_HIP, "kernel launch failed: %s", hipGetErrorString(err));
    return FE_OK;
}
