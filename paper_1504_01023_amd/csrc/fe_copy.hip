// fe_copy.hip -- a plain streaming copy used to calibrate HBM byte counters
// and to measure the achieved copy ceiling next to the integration kernels,
// and the bare access pattern of an integration kernel (its rows read and
// written, no arithmetic) for the memory-side ceiling of that pattern.
#include <hip/hip_runtime.h>

#include "fe.h"
#include "fe_api_internal.h"

namespace {

typedef double d2_t __attribute__((ext_vector_type(2)));

__global__ __launch_bounds__(256) void stream_copy_kernel(d2_t *__restrict__ dst,
                                                          const d2_t *__restrict__ src, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride)
        __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
}

// rows_in FP64 rows read and rows_out rows of TO written per element, one
// element per lane, streaming loads and stores: out[w][e] = sum_r in[r][e] + w.
template <typename TO>
__global__ __launch_bounds__(256) void stream_pattern_kernel(const double *__restrict__ in,
                                                             int rows_in, TO *__restrict__ out,
                                                             int rows_out, int64_t n, int64_t ld)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n)
        return;
    double s = 0.0;
#pragma unroll 8
    for (int r = 0; r < rows_in; ++r)
        s += __builtin_nontemporal_load(in + r * ld + e);
#pragma unroll 8
    for (int w = 0; w < rows_out; ++w)
        __builtin_nontemporal_store((TO)(s + (double)w), out + w * ld + e);
}

}  // namespace

extern "C" int fe_stream_pattern(const double *in, int32_t rows_in, void *out, int32_t rows_out,
                                 int32_t out_bytes, int64_t n, int64_t ld, hipStream_t stream)
{
    if (rows_in < 0 || rows_out < 1 || n < 0 || ld < n || (out_bytes != 8 && out_bytes != 4))
        return fe::fail(FE_ERR_INVALID_ARG, "bad pattern arguments");
    if (n == 0)
        return FE_OK;
    if (!out || (rows_in > 0 && !in) || ((uintptr_t)in % 8) || ((uintptr_t)out % out_bytes))
        return fe::fail(FE_ERR_INVALID_ARG, "pointers must be non-NULL and aligned");
    int64_t grid = (n + 255) / 256;
    if (grid > 0x7fffffff)
        return fe::fail(FE_ERR_INVALID_ARG, "n too large");
    const hipError_t err =
        out_bytes == 8
            ? fe::launch_kernel(&stream_pattern_kernel<double>, dim3((unsigned)grid), dim3(256), 0,
                                stream, in, (int)rows_in, static_cast<double *>(out),
                                (int)rows_out, n, ld)
            : fe::launch_kernel(&stream_pattern_kernel<float>, dim3((unsigned)grid), dim3(256), 0,
                                stream, in, (int)rows_in, static_cast<float *>(out),
                                (int)rows_out, n, ld);
    if (err != hipSuccess)
        return fe::fail(FE_ERR_HIP, "pattern launch failed: %s", hipGetErrorString(err));
    return FE_OK;
}

extern "C" int fe_stream_copy(void *dst, const void *src, int64_t n_bytes, hipStream_t stream)
{
    if (n_bytes < 0 || (n_bytes % 16) != 0)
        return fe::fail(FE_ERR_INVALID_ARG, "n_bytes must be a non-negative multiple of 16");
    if (n_bytes == 0)
        return FE_OK;
    if (!dst || !src || ((uintptr_t)dst % 16) || ((uintptr_t)src % 16))
        return fe::fail(FE_ERR_INVALID_ARG, "pointers must be non-NULL and 16-byte aligned");
    const int64_t n = n_bytes / 16;
    // one 16-byte element per lane over a full grid (measured on MI355X: a
    // grid-stride loop over a capped grid copies 5-15% slower)
    int64_t grid = (n + 255) / 256;
    if (grid > 0x7fffffff)
        grid = 0x7fffffff;
    const hipError_t err =
        fe::launch_kernel(&stream_copy_kernel, dim3((unsigned)grid), dim3(256), 0, stream,
                          static_cast<d2_t *>(dst), static_cast<const d2_t *>(src), n);
    if (err != hipSuccess)
        return fe::fail(FE_ERR_HIP, "copy launch failed: %s", hipGetErrorString(err));
    return FE_OK;
}
