// fe_orient.hip -- diagnostic count of elements with det J <= 0 at some
// point of a rule. Such elements are integrated as written (signed det J);
// this count lets a caller find them.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstring>

#include "fe.h"
#include "fe_api_internal.h"

namespace {

using namespace fe;

// det J at reference point q from the edge vectors E_r = X_r - X_0 (r >= 1),
// J[i][k] = sum_r E_r,i dphi_r/dxi_k, by cofactor expansion along row 0.
template <int NV>
__device__ __forceinline__ double point_det(const double (&E)[NV * 3], const KArgs &a, int q)
{
    double J[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            double s = 0.0;
#pragma unroll
            for (int r = 1; r < NV; ++r)
                s += E[3 * r + i] * a.dphi[q][r][k];
            J[i][k] = s;
        }
    return J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1]) +
           J[0][1] * (J[1][2] * J[2][0] - J[1][0] * J[2][2]) +
           J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
}

template <int NV>
__global__ __launch_bounds__(256) void count_inverted_kernel(KArgs a, unsigned long long *count)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    // the loop bound is uniform over the workgroup, so every lane reaches the ballot
    for (int64_t base = (int64_t)blockIdx.x * blockDim.x; base < a.n_elem; base += stride) {
        const int64_t e = base + threadIdx.x;
        bool inverted = false;
        if (e < a.n_elem) {
            double E[NV * 3];
#pragma unroll
            for (int s = 0; s < NV * 3; ++s)
                E[s] = a.coords[s * a.ld_in + e];
#pragma unroll
            for (int r = NV - 1; r >= 1; --r)
#pragma unroll
                for (int i = 0; i < 3; ++i)
                    E[3 * r + i] -= E[i];
            const int nq = NV == 4 ? 1 : a.n_q;  // affine tetrahedra: det J is constant
            for (int q = 0; q < nq; ++q)
                inverted = inverted || !(point_det<NV>(E, a, q) > 0.0);
        }
        const unsigned long long m = __ballot(inverted);
        if ((threadIdx.x & 63) == 0 && m)
            atomicAdd(count, (unsigned long long)__popcll(m));
    }
}

}  // namespace

extern "C" int fe_count_inverted(fe_elem_type elem_type, int64_t n_elem, const double *coords,
                                 int64_t ld_in, const fe_quad_rule *quad_rule, int64_t *count,
                                 hipStream_t stream)
{
    if (elem_type != FE_TET4 && elem_type != FE_PRISM6)
        return fail(FE_ERR_INVALID_ARG, "bad element type %d", elem_type);
    if (n_elem < 0)
        return fail(FE_ERR_INVALID_ARG, "n_elem is negative");
    if (const int st = check_rule(quad_rule))
        return st;
    if (n_elem == 0)
        return FE_OK;
    if (!coords || !count || ld_in < n_elem)
        return fail(FE_ERR_INVALID_ARG, "NULL pointer or ld_in smaller than n_elem");
    if (((uintptr_t)coords % 8) || ((uintptr_t)count % 8))
        return fail(FE_ERR_UNSUPPORTED, "pointers must be 8-byte aligned");
    KArgs a;
    std::memset(&a, 0, sizeof(a));
    a.coords = coords;
    a.n_elem = n_elem;
    a.ld_in = ld_in;
    fill_reference(elem_type, *quad_rule, a);
    int64_t grid = (n_elem + 255) / 256;
    if (grid > 4096)
        grid = 4096;
    unsigned long long *c = reinterpret_cast<unsigned long long *>(count);
    const hipError_t err =
        elem_type == FE_TET4
            ? launch_kernel(&count_inverted_kernel<4>, dim3((unsigned)grid), dim3(256), 0, stream, a, c)
            : launch_kernel(&count_inverted_kernel<6>, dim3((unsigned)grid), dim3(256), 0, stream, a, c);
    if (err != hipSuccess)
        return fail(FE_ERR_HIP, "kernel launch failed: %s", hipGetErrorString(err));
    return FE_OK;
}
