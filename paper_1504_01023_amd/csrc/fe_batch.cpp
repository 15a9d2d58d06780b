// fe_batch.cpp -- persistent batched launches replayed from captured HIP
// graphs.
//
// Elements of one "kind" (element type, problem, precision, rule; the sets
// of same-type elements of Sec. 3.2 and Algorithm 1's "sequence of elements
// of the same type and order of approximation") from many requests of
// different sizes are cut into fixed-size chunks and processed by one
// persistent launch per kind. The chunk table lives in pinned host memory,
// is copied to the device by the first node of a HIP graph captured once at
// creation, and the graph (copy -> one persistent kernel per kind, the kinds
// on parallel branches) is replayed for every batch, so a batch costs one graph launch whatever the
// number of requests in it. Two tables and two graph instances alternate so
// the host can fill one while the other is in flight.
#include <hip/hip_runtime.h>

#include <cstring>
#include <new>
#include <vector>

#include "fe.h"
#include "fe_api_internal.h"

using namespace fe;

namespace {

constexpr size_t HEADER_BYTES = 128;
static_assert(sizeof(BatchHeader) == HEADER_BYTES, "batch header layout");

struct Kind {
    Plan plan;
    int vec = 1;
    size_t tsize = 8;
};

struct Buffer {
    void *host = nullptr;
    void *dev = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t done = nullptr;
    bool used = false;
};

}  // namespace

namespace fe {

int batch_kind_plan(const fe_batch_kind &bk, int k, int64_t chunk_elems, int blocks_per_kind,
                    Plan &out)
{
    const fe_quad_rule rule{bk.n_q, bk.xi, bk.w};
    // Resolve the kernel for this kind (validation, tuned variant, reference
    // tables) with an empty batch.
    int st = plan(&bk.problem, bk.elem_type, 0, nullptr, nullptr, 0, &rule, nullptr, nullptr, 0,
                  nullptr, out);
    if (st)
        return st;
    if (!out.entry->batch) {
        // The tuned variant has no batched form: keep its workgroup and
        // width with streaming memory operations, else the base variant.
        const fe_variant tuned = out.variant;
        const fe_variant alts[2] = {
            {tuned.wg_size, tuned.elems_per_thread, tuned.ref_in_lds, 1, 0, tuned.row_split, 1},
            {256, 1, 2, 1, 0, 1, 1}};
        for (const fe_variant &v : alts) {
            Plan alt;
            if (plan(&bk.problem, bk.elem_type, 0, nullptr, nullptr, 0, &rule, nullptr, nullptr, 0,
                     &v, alt) == FE_OK && alt.entry->batch) {
                out = alt;
                break;
            }
        }
    }
    if (!out.entry->batch)
        return fail(FE_ERR_UNSUPPORTED, "kind %d has no batched kernel (elem=%d kind=%d mode=%d)",
                    k, out.key.elem, out.key.kind, out.key.mode);
    // 4096 workgroups per kind: most batches take one or two passes of the
    // tile loop (a long grid-stride loop streams more slowly; measured on
    // MI355X: resident served throughput +8% over 1024)
    out.grid = blocks_per_kind > 0 ? (unsigned)blocks_per_kind : 4096u;
    out.args.n_elem = chunk_elems;  // the kernel's tile count per chunk
    return FE_OK;
}

int batch_check_request(const Plan &pl, int kind, int64_t n_elem, const double *coords,
                        const void *coeffs, int64_t ld_in, const void *out_K, const void *out_F,
                        int64_t ld_out, bool *wide)
{
    bool reads_coeffs = false;
    for (int s = 0; s < 20; ++s)
        reads_coeffs = reads_coeffs || pl.args.col[s] >= 0;
    if (!coords || !out_K || !out_F || (reads_coeffs && !coeffs))
        return fail(FE_ERR_INVALID_ARG, "NULL input or output pointer");
    if (ld_in < n_elem || ld_out < n_elem)
        return fail(FE_ERR_INVALID_ARG, "leading dimension smaller than n_elem");
    const size_t tsize = pl.key.prec == FE_FP64 ? 8 : 4;
    const size_t csize = pl.key.mode == M_FUNC ? 8 : tsize;  // function parameters are FP64
    auto al = [](const void *p, size_t a) { return ((uintptr_t)p % a) == 0; };
    if (!al(coords, 8) || !al(out_K, tsize) || !al(out_F, tsize) ||
        (reads_coeffs && !al(coeffs, csize)))
        return fail(FE_ERR_UNSUPPORTED, "kind %d: pointers must be aligned to their element size",
                    kind);
    // V elements per lane read and write V-wide vectors: the rows must start
    // on multiples of V and the pointers on the vector size; other requests
    // are processed element by element
    const int V = pl.key.vec;
    const size_t ca = V > 1 ? 16 : 8, ta = V > 1 ? (tsize * V < 16 ? tsize * V : 16) : tsize;
    *wide = !(ld_in % V || ld_out % V || !al(coords, ca) || !al(out_K, ta) || !al(out_F, ta) ||
              (reads_coeffs && pl.key.mode != M_FUNC && !al(coeffs, ta)));
    return FE_OK;
}

Chunk batch_chunk(int64_t c, int64_t chunk_elems, int64_t n_elem, const double *coords,
                  const void *coeffs, int64_t ld_in, void *out_K, void *out_F, int64_t ld_out,
                  bool wide)
{
    Chunk ch;
    ch.coords = coords;
    ch.coeffs = coeffs;
    ch.out_K = out_K;
    ch.out_F = out_F;
    ch.ld_in = ld_in;
    ch.ld_out = ld_out;
    ch.e0 = c * chunk_elems;
    ch.n = (n_elem - ch.e0) < chunk_elems ? (n_elem - ch.e0) : chunk_elems;
    if (!wide)
        ch.n = -ch.n;
    return ch;
}

}  // namespace fe

struct fe_batch {
    int n_kinds = 0;
    Kind kinds[MAX_BATCH_KINDS];
    int max_chunks = 0;
    int64_t chunk_elems = 0;
    size_t table_bytes = 0;
    std::vector<Chunk> pending[MAX_BATCH_KINDS];
    int pending_total = 0;
    Buffer buf[2];
    int next = 0;
    hipStream_t capture = nullptr;
    hipStream_t branch[MAX_BATCH_KINDS] = {};
    hipEvent_t forked = nullptr, joined[MAX_BATCH_KINDS] = {};
};

static void destroy_batch(fe_batch *b)
{
    if (!b)
        return;
    for (Buffer &B : b->buf) {
        if (B.used && B.done)
            (void)hipEventSynchronize(B.done);
        if (B.exec)
            (void)hipGraphExecDestroy(B.exec);
        if (B.graph)
            (void)hipGraphDestroy(B.graph);
        if (B.done)
            (void)hipEventDestroy(B.done);
        if (B.dev)
            (void)hipFree(B.dev);
        if (B.host)
            (void)hipHostFree(B.host);
    }
    for (int k = 0; k < MAX_BATCH_KINDS; ++k) {
        if (b->branch[k])
            (void)hipStreamDestroy(b->branch[k]);
        if (b->joined[k])
            (void)hipEventDestroy(b->joined[k]);
    }
    if (b->forked)
        (void)hipEventDestroy(b->forked);
    if (b->capture)
        (void)hipStreamDestroy(b->capture);
    delete b;
}

#define HIP_TRY(expr)                                                                        \
    do {                                                                                     \
        hipError_t err_ = (expr);                                                            \
        if (err_ != hipSuccess) {                                                            \
            destroy_batch(b);                                                                \
            return fail(FE_ERR_HIP, "%s failed: %s", #expr, hipGetErrorString(err_));        \
        }                                                                                    \
    } while (0)

extern "C" {

int fe_batch_create(const fe_batch_kind *kinds, int n_kinds, int max_chunks, int64_t chunk_elems,
                    int blocks_per_kind, fe_batch **out)
{
    if (!out)
        return fail(FE_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!kinds || n_kinds < 1 || n_kinds > FE_MAX_BATCH_KINDS)
        return fail(FE_ERR_INVALID_ARG, "need 1..%d kinds", FE_MAX_BATCH_KINDS);
    if (max_chunks < 1 || max_chunks > (1 << 20))
        return fail(FE_ERR_INVALID_ARG, "max_chunks must be in 1..2^20");
    if (chunk_elems < 4 || chunk_elems % 4)
        return fail(FE_ERR_INVALID_ARG, "chunk_elems must be a positive multiple of 4");
    if (blocks_per_kind < 0 || blocks_per_kind > (1 << 20))
        return fail(FE_ERR_INVALID_ARG, "blocks_per_kind out of range");
    fe_batch *b = new (std::nothrow) fe_batch();
    if (!b)
        return fail(FE_ERR_CAPACITY, "out of host memory");
    b->n_kinds = n_kinds;
    b->max_chunks = max_chunks;
    b->chunk_elems = chunk_elems;
    b->table_bytes = HEADER_BYTES + sizeof(Chunk) * (size_t)max_chunks;
    for (int k = 0; k < n_kinds; ++k) {
        Kind &K = b->kinds[k];
        const int st = batch_kind_plan(kinds[k], k, chunk_elems, blocks_per_kind, K.plan);
        if (st) {
            destroy_batch(b);
            return st;
        }
        K.vec = K.plan.key.vec;
        K.tsize = kinds[k].problem.precision == FE_FP64 ? 8 : 4;
    }
    HIP_TRY(hipStreamCreateWithFlags(&b->capture, hipStreamNonBlocking));
    for (int k = 0; k < n_kinds; ++k) {
        HIP_TRY(hipStreamCreateWithFlags(&b->branch[k], hipStreamNonBlocking));
        HIP_TRY(hipEventCreateWithFlags(&b->joined[k], hipEventDisableTiming));
    }
    HIP_TRY(hipEventCreateWithFlags(&b->forked, hipEventDisableTiming));
    for (Buffer &B : b->buf) {
        HIP_TRY(hipHostMalloc(&B.host, b->table_bytes, hipHostMallocDefault));
        std::memset(B.host, 0, b->table_bytes);
        HIP_TRY(hipMalloc(&B.dev, b->table_bytes));
        HIP_TRY(hipEventCreateWithFlags(&B.done, hipEventDisableTiming));
        HIP_TRY(hipStreamBeginCapture(b->capture, hipStreamCaptureModeThreadLocal));
        hipError_t cerr = hipMemcpyAsync(B.dev, B.host, b->table_bytes, hipMemcpyHostToDevice,
                                         b->capture);
        const BatchHeader *hdr = static_cast<const BatchHeader *>(B.dev);
        const Chunk *chunks =
            reinterpret_cast<const Chunk *>(static_cast<const char *>(B.dev) + HEADER_BYTES);
        // One branch per kind after the table copy, so kinds run side by side.
        if (cerr == hipSuccess)
            cerr = hipEventRecord(b->forked, b->capture);
        for (int k = 0; k < n_kinds && cerr == hipSuccess; ++k) {
            const Kind &K = b->kinds[k];
            cerr = hipStreamWaitEvent(b->branch[k], b->forked, 0);
            if (cerr != hipSuccess)
                break;
            cerr = K.plan.entry->batch(K.plan.args, hdr, chunks, k, K.plan.grid, K.plan.block,
                                       b->branch[k]);
            if (cerr == hipSuccess)
                cerr = hipEventRecord(b->joined[k], b->branch[k]);
            if (cerr == hipSuccess)
                cerr = hipStreamWaitEvent(b->capture, b->joined[k], 0);
        }
        hipError_t eerr = hipStreamEndCapture(b->capture, &B.graph);
        if (cerr != hipSuccess || eerr != hipSuccess) {
            destroy_batch(b);
            return fail(FE_ERR_HIP, "graph capture failed: %s",
                        hipGetErrorString(cerr != hipSuccess ? cerr : eerr));
        }
        HIP_TRY(hipGraphInstantiate(&B.exec, B.graph, nullptr, nullptr, 0));
    }
    *out = b;
    return FE_OK;
}

int fe_batch_add(fe_batch *b, int kind, int64_t n_elem, const double *coords, const void *coeffs,
                 int64_t ld_in, void *out_K, void *out_F, int64_t ld_out)
{
    if (!b)
        return fail(FE_ERR_INVALID_ARG, "batch is NULL");
    if (kind < 0 || kind >= b->n_kinds)
        return fail(FE_ERR_INVALID_ARG, "kind %d out of range", kind);
    if (n_elem < 0)
        return fail(FE_ERR_INVALID_ARG, "n_elem is negative");
    if (n_elem == 0)
        return FE_OK;
    bool wide = true;
    const int st = batch_check_request(b->kinds[kind].plan, kind, n_elem, coords, coeffs, ld_in,
                                       out_K, out_F, ld_out, &wide);
    if (st)
        return st;
    const int64_t n_chunks = (n_elem + b->chunk_elems - 1) / b->chunk_elems;
    if (b->pending_total + n_chunks > b->max_chunks)
        return fail(FE_ERR_CAPACITY, "batch table full (%d of %d chunks pending, %lld more)",
                    b->pending_total, b->max_chunks, (long long)n_chunks);
    for (int64_t c = 0; c < n_chunks; ++c)
        b->pending[kind].push_back(batch_chunk(c, b->chunk_elems, n_elem, coords, coeffs, ld_in,
                                               out_K, out_F, ld_out, wide));
    b->pending_total += (int)n_chunks;
    return FE_OK;
}

int fe_batch_pending(const fe_batch *b) { return b ? b->pending_total : -1; }

int fe_batch_launch(fe_batch *b, hipStream_t stream)
{
    if (!b)
        return fail(FE_ERR_INVALID_ARG, "batch is NULL");
    if (b->pending_total == 0)
        return FE_OK;
    Buffer &B = b->buf[b->next];
    if (B.used) {
        const hipError_t err = hipEventSynchronize(B.done);
        if (err != hipSuccess)
            return fail(FE_ERR_HIP, "waiting for the previous batch failed: %s",
                        hipGetErrorString(err));
    }
    BatchHeader hdr;
    std::memset(&hdr, 0, sizeof(hdr));
    Chunk *dst = reinterpret_cast<Chunk *>(static_cast<char *>(B.host) + HEADER_BYTES);
    int pos = 0;
    for (int k = 0; k < b->n_kinds; ++k) {
        hdr.begin[k] = pos;
        for (const Chunk &c : b->pending[k])
            dst[pos++] = c;
        hdr.end[k] = pos;
    }
    std::memcpy(B.host, &hdr, sizeof(hdr));
    hipError_t err = hipGraphLaunch(B.exec, stream);
    if (err == hipSuccess)
        err = hipEventRecord(B.done, stream);
    if (err != hipSuccess)
        return fail(FE_ERR_HIP, "graph launch failed: %s", hipGetErrorString(err));
    B.used = true;
    b->next ^= 1;
    for (int k = 0; k < b->n_kinds; ++k)
        b->pending[k].clear();
    b->pending_total = 0;
    return FE_OK;
}

int fe_batch_destroy(fe_batch *b)
{
    destroy_batch(b);
    return FE_OK;
}

}  // extern "C"
