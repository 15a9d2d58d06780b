// fe_batch_static.hip -- batched integration that allocates nothing.
//
// The persistent batched kernels (the same kernels fe_batch_launch replays)
// read their chunk table from a file-scope device array instead of memory the
// library allocates, for callers that cannot call hipMalloc. The table does
// not pass through host staging memory either: its records travel in the
// kernel arguments of a small table-writing kernel (at most PIECE records per
// launch), which stores them into the array on the caller's stream, so the
// call never waits and the caller's request array may be reused on return.
#include <hip/hip_runtime.h>

#include <mutex>

#include "fe.h"
#include "fe_api_internal.h"

using namespace fe;

namespace {

constexpr size_t HEADER_BYTES = 128;
static_assert(sizeof(BatchHeader) == HEADER_BYTES, "batch header layout");
constexpr size_t SCRATCH_BYTES = HEADER_BYTES + sizeof(Chunk) * FE_BATCH_STATIC_MAX_CHUNKS;

// The chunk table of the last call on this device (header, then records).
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

// Records per table-writing launch: the piece stays near the size of the
// integration kernels' own arguments (about 2.2 KiB).
constexpr int PIECE = 30;
struct TablePiece {
    BatchHeader hdr;      // written by the piece with with_header = 1
    int32_t first;        // table index of rec[0]
    int32_t count;        // records in this piece, 0..PIECE
    int32_t with_header;
    int32_t pad;
    Chunk rec[PIECE];
};
static_assert(sizeof(TablePiece) <= 2304, "table piece must stay a modest kernel argument");

__global__ __launch_bounds__(256) void write_table_kernel(unsigned char *__restrict__ table,
                                                          TablePiece piece)
{
    // 8-byte words: the header's 16, then the records' 8 each
    const int n_hdr = piece.with_header ? (int)(HEADER_BYTES / 8) : 0;
    const int n_rec = piece.count * (int)(sizeof(Chunk) / 8);
    uint64_t *hdr = reinterpret_cast<uint64_t *>(table);
    uint64_t *rec = reinterpret_cast<uint64_t *>(table + HEADER_BYTES) +
                    (size_t)piece.first * (sizeof(Chunk) / 8);
    const uint64_t *src_hdr = reinterpret_cast<const uint64_t *>(&piece.hdr);
    const uint64_t *src_rec = reinterpret_cast<const uint64_t *>(&piece.rec[0]);
    for (int i = threadIdx.x; i < n_hdr; i += blockDim.x)
        hdr[i] = src_hdr[i];
    for (int i = threadIdx.x; i < n_rec; i += blockDim.x)
        rec[i] = src_rec[i];
}

constexpr int MAX_DEVICES = 64;
std::mutex g_mu;
void *g_table[MAX_DEVICES];  // address of `scratch` on each device, once looked up

// The device address of this device's copy of `scratch` (the array's name in
// host code is only a host-side stand-in, never a device address).
int table_on_current_device(void **out)
{
    int dev = -1;
    hipError_t err = hipGetDevice(&dev);
    if (err != hipSuccess)
        return fail(FE_ERR_HIP, "hipGetDevice failed: %s", hipGetErrorString(err));
    if (dev < 0 || dev >= MAX_DEVICES)
        return fail(FE_ERR_UNSUPPORTED, "device %d beyond the %d supported", dev, MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_mu);
    if (!g_table[dev]) {
        void *ptr = nullptr;
        err = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (err != hipSuccess || !ptr)
            return fail(FE_ERR_HIP, "hipGetSymbolAddress(scratch) failed: %s",
                        hipGetErrorString(err));
        g_table[dev] = ptr;
    }
    *out = g_table[dev];
    return FE_OK;
}

int launch_piece(unsigned char *table, const TablePiece &piece, hipStream_t stream)
{
    const hipError_t err =
        launch_kernel(&write_table_kernel, dim3(1), dim3(256), 0, stream, table, piece);
    if (err != hipSuccess)
        return fail(FE_ERR_HIP, "table write launch failed: %s", hipGetErrorString(err));
    return FE_OK;
}

}  // namespace

extern "C" int fe_batch_integrate_static(const fe_batch_kind *kinds, int n_kinds,
                                         const fe_batch_request *requests, int n_requests,
                                         int64_t chunk_elems, int blocks_per_kind,
                                         hipStream_t stream)
{
    if (!kinds || n_kinds < 1 || n_kinds > FE_MAX_BATCH_KINDS)
        return fail(FE_ERR_INVALID_ARG, "need 1..%d kinds", FE_MAX_BATCH_KINDS);
    if (n_requests < 0 || (n_requests > 0 && !requests))
        return fail(FE_ERR_INVALID_ARG, "requests is NULL or n_requests negative");
    if (chunk_elems < 4 || chunk_elems % 4)
        return fail(FE_ERR_INVALID_ARG, "chunk_elems must be a positive multiple of 4");
    if (blocks_per_kind < 0 || blocks_per_kind > (1 << 20))
        return fail(FE_ERR_INVALID_ARG, "blocks_per_kind out of range");

    // Every kind and request is checked, and the table's size known, before
    // anything is enqueued.
    Plan plans[FE_MAX_BATCH_KINDS];
    for (int k = 0; k < n_kinds; ++k) {
        const int st = batch_kind_plan(kinds[k], k, chunk_elems, blocks_per_kind, plans[k]);
        if (st)
            return st;
    }
    int64_t chunks_of_kind[FE_MAX_BATCH_KINDS] = {};
    int64_t total = 0;
    for (int i = 0; i < n_requests; ++i) {
        const fe_batch_request &r = requests[i];
        if (r.kind < 0 || r.kind >= n_kinds)
            return fail(FE_ERR_INVALID_ARG, "request %d: kind %d out of range", i, r.kind);
        if (r.reserved != 0)
            return fail(FE_ERR_INVALID_ARG, "request %d: reserved field must be 0", i);
        if (r.n_elem < 0)
            return fail(FE_ERR_INVALID_ARG, "request %d: n_elem is negative", i);
        if (r.n_elem == 0)
            continue;
        bool wide = true;
        const int st = batch_check_request(plans[r.kind], r.kind, r.n_elem, r.coords, r.coeffs,
                                           r.ld_in, r.out_K, r.out_F, r.ld_out, &wide);
        if (st)
            return st;
        const int64_t n_chunks = (r.n_elem + chunk_elems - 1) / chunk_elems;
        chunks_of_kind[r.kind] += n_chunks;
        total += n_chunks;
        if (total > FE_BATCH_STATIC_MAX_CHUNKS)
            return fail(FE_ERR_CAPACITY, "the requests need more than %d chunks of %lld elements",
                        FE_BATCH_STATIC_MAX_CHUNKS, (long long)chunk_elems);
    }
    if (total == 0)
        return FE_OK;
    void *table = nullptr;
    int st = table_on_current_device(&table);
    if (st)
        return st;
    unsigned char *tab = static_cast<unsigned char *>(table);

    // Kind-major table: kind k owns records [begin[k], end[k]).
    TablePiece piece;
    piece.hdr = BatchHeader{};
    int64_t pos = 0;
    for (int k = 0; k < n_kinds; ++k) {
        piece.hdr.begin[k] = (int32_t)pos;
        pos += chunks_of_kind[k];
        piece.hdr.end[k] = (int32_t)pos;
    }
    piece.with_header = 1;
    piece.first = 0;
    piece.count = 0;
    piece.pad = 0;
    for (int k = 0; k < n_kinds; ++k) {
        for (int i = 0; i < n_requests; ++i) {
            const fe_batch_request &r = requests[i];
            if (r.kind != k || r.n_elem == 0)
                continue;
            bool wide = true;
            (void)batch_check_request(plans[k], k, r.n_elem, r.coords, r.coeffs, r.ld_in, r.out_K,
                                      r.out_F, r.ld_out, &wide);
            const int64_t n_chunks = (r.n_elem + chunk_elems - 1) / chunk_elems;
            for (int64_t c = 0; c < n_chunks; ++c) {
                piece.rec[piece.count++] = batch_chunk(c, chunk_elems, r.n_elem, r.coords,
                                                       r.coeffs, r.ld_in, r.out_K, r.out_F,
                                                       r.ld_out, wide);
                if (piece.count == PIECE) {
                    if ((st = launch_piece(tab, piece, stream)))
                        return st;
                    piece.first += piece.count;
                    piece.count = 0;
                    piece.with_header = 0;
                }
            }
        }
    }
    if (piece.count > 0 || piece.with_header) {
        if ((st = launch_piece(tab, piece, stream)))
            return st;
    }
    const BatchHeader *hdr = reinterpret_cast<const BatchHeader *>(tab);
    const Chunk *chunks = reinterpret_cast<const Chunk *>(tab + HEADER_BYTES);
    for (int k = 0; k < n_kinds; ++k) {
        if (chunks_of_kind[k] == 0)
            continue;
        const Plan &pl = plans[k];
        const hipError_t err = pl.entry->batch(pl.args, hdr, chunks, k, pl.grid, pl.block, stream);
        if (err != hipSuccess)
            return fail(FE_ERR_HIP, "batched kernel launch failed: %s", hipGetErrorString(err));
    }
    return FE_OK;
}
