// fe_device.h -- gfx950 device code for element-by-element numerical
// integration (Sec. 2.3 of arXiv:1504.01023, parallelised one element per
// thread as in Sec. 3.2).
//
// Design (MI355X / CDNA4):
//  * Element streaming over structure-of-arrays data: every input and output
//    array is indexed [row * ld + e], so a wavefront of 64 lanes touches 64
//    consecutive elements of one row = whole 64-byte segments; with
//    VEC = 2 or 4 contiguous elements per lane the loads and stores become
//    16-byte vector accesses (global_load_dwordx4). This is the "coalesced"
//    organisation of Sec. 4.2, with the data permutation moved into the
//    layout instead of an LDS transpose.
//  * Reference data (weights, shape-function values and reference
//    derivatives at the points, tetrahedron moments) are either read as
//    wave-uniform kernel arguments (scalar loads into SGPRs) or staged once
//    per workgroup in LDS (Sec. 4.3 "shared memory usage"; the choice is a
//    tuning parameter).
//  * Jacobian terms (J, det J, adj J / det J) are always FP64, from FP64
//    coordinates. In the FP32 bulk tier the global derivatives and vol are
//    rounded to FP32 after they are formed and everything after that
//    (coefficients, accumulation, outputs) is FP32.
//  * The loop order is QSS (Algorithms 2 and 3): points outermost, then the
//    two shape-function loops, with the derivative-index loops innermost and
//    specialised per problem (Sec. 3.3). For tetrahedra the geometric terms
//    are hoisted out of the point loop (Algorithm 3), and the sums over
//    points of (weight x coefficient x reference shape values) are formed
//    before the contraction with the constant gradients.
#pragma once

#include <hip/hip_runtime.h>

#include <type_traits>

#include "fe_internal.h"

namespace fe {

typedef double d2_t __attribute__((ext_vector_type(2)));
typedef float f2_t __attribute__((ext_vector_type(2)));
typedef float f4_t __attribute__((ext_vector_type(4)));

// ------------------------------------------------------------------ memory
// Cache policy of the streams (NT): 0 default; 1 streaming (non-temporal)
// loads and stores; 2 streaming stores only.
template <int NT, typename T>
__device__ __forceinline__ T ld1(const T *p)
{
    if constexpr (NT == 1)
        return __builtin_nontemporal_load(p);
    else
        return *p;
}

template <int NT, typename T>
__device__ __forceinline__ void st1(T *p, T v)
{
    if constexpr (NT != 0)
        __builtin_nontemporal_store(v, p);
    else
        *p = v;
}

// Load V consecutive values starting at p. Alignment of p to
// min(16, V * sizeof(T)) bytes is guaranteed by the host dispatcher.
template <int V, int NT>
__device__ __forceinline__ void loadv(const double *p, double (&v)[V])
{
    if constexpr (V == 1) {
        v[0] = ld1<NT>(p);
    } else {
#pragma unroll
        for (int i = 0; i < V; i += 2) {
            const d2_t x = ld1<NT>(reinterpret_cast<const d2_t *>(p + i));
            v[i] = x.x;
            v[i + 1] = x.y;
        }
    }
}

template <int V, int NT>
__device__ __forceinline__ void loadv(const float *p, float (&v)[V])
{
    if constexpr (V == 1) {
        v[0] = ld1<NT>(p);
    } else if constexpr (V == 2) {
        const f2_t x = ld1<NT>(reinterpret_cast<const f2_t *>(p));
        v[0] = x.x;
        v[1] = x.y;
    } else {
        const f4_t x = ld1<NT>(reinterpret_cast<const f4_t *>(p));
        v[0] = x.x;
        v[1] = x.y;
        v[2] = x.z;
        v[3] = x.w;
    }
}

typedef int int2_t __attribute__((ext_vector_type(2)));
typedef int int4_t __attribute__((ext_vector_type(4)));

template <int V, int NT>
__device__ __forceinline__ void loadv(const int32_t *p, int32_t (&v)[V])
{
    if constexpr (V == 1) {
        v[0] = ld1<NT>(p);
    } else if constexpr (V == 2) {
        const int2_t x = ld1<NT>(reinterpret_cast<const int2_t *>(p));
        v[0] = x.x;
        v[1] = x.y;
    } else {
        const int4_t x = ld1<NT>(reinterpret_cast<const int4_t *>(p));
        v[0] = x.x;
        v[1] = x.y;
        v[2] = x.z;
        v[3] = x.w;
    }
}

template <int V, int NT>
__device__ __forceinline__ void storev(double *p, const double (&v)[V])
{
    if constexpr (V == 1) {
        st1<NT>(p, v[0]);
    } else {
#pragma unroll
        for (int i = 0; i < V; i += 2) {
            d2_t x;
            x.x = v[i];
            x.y = v[i + 1];
            st1<NT>(reinterpret_cast<d2_t *>(p + i), x);
        }
    }
}

template <int V, int NT>
__device__ __forceinline__ void storev(float *p, const float (&v)[V])
{
    if constexpr (V == 1) {
        st1<NT>(p, v[0]);
    } else if constexpr (V == 2) {
        f2_t x;
        x.x = v[0];
        x.y = v[1];
        st1<NT>(reinterpret_cast<f2_t *>(p), x);
    } else {
        f4_t x;
        x.x = v[0];
        x.y = v[1];
        x.z = v[2];
        x.w = v[3];
        st1<NT>(reinterpret_cast<f4_t *>(p), x);
    }
}

// Where one batch of elements lives: the kernels read coordinates and
// coefficients and write K and F through this view, so a plain launch
// (one batch) and a persistent launch over a table of chunks of many
// requests share the per-element code.
struct Streams {
    const double *coords;
    const void *coeffs;
    void *out_K;
    void *out_F;
    int64_t ld_in;
    int64_t ld_out;

    // Vertex coordinates of V consecutive elements: X[i][3 v + d].
    template <int NV, int V, int NT>
    __device__ __forceinline__ void load_coords(int64_t e0, double (&X)[V][3 * NV]) const
    {
#pragma unroll
        for (int s = 0; s < 3 * NV; ++s) {
            double t[V];
            loadv<V, NT>(coords + s * ld_in + e0, t);
#pragma unroll
            for (int i = 0; i < V; ++i)
                X[i][s] = t[i];
        }
    }
};

// Indexed geometry: vertex coordinates gathered from a global node array
// nodes[3 * id + d] through connectivity conn[v * ld_conn + e] (int32).
// Neighbouring elements share nodes, so after the first touch the gathers
// are served by L2 / MALL and HBM sees each node about once.
struct StreamsIdx : Streams {
    const double *nodes;
    const int32_t *conn;
    int64_t ld_conn;
    uint32_t n_nodes;

    template <int NV, int V, int NT>
    __device__ __forceinline__ void load_coords(int64_t e0, double (&X)[V][3 * NV]) const
    {
        int32_t id[NV][V];
#pragma unroll
        for (int v = 0; v < NV; ++v)
            loadv<V, NT>(conn + v * ld_conn + e0, id[v]);
#pragma unroll
        for (int i = 0; i < V; ++i)
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                // out-of-range ids are clamped: never a fault, whatever the input
                const uint32_t u = (uint32_t)id[v][i];
                const double *p = nodes + 3 * (int64_t)(u < n_nodes ? u : n_nodes - 1);
                X[i][3 * v + 0] = p[0];
                X[i][3 * v + 1] = p[1];
                X[i][3 * v + 2] = p[2];
            }
    }
};

// ------------------------------------------------------------ small helpers
__host__ __device__ constexpr int popc_below(uint32_t m, int k)
{
    int c = 0;
    for (int i = 0; i < k; ++i)
        c += (m >> i) & 1u;
    return c;
}

// Packed upper-triangle index of (r, s), r <= s, in an N x N matrix.
__host__ __device__ constexpr int pidx(int N, int r, int s) { return r * N - r * (r - 1) / 2 + (s - r); }

// Value of coefficient slot k at point q for V consecutive elements.
template <typename T, int MODE, uint32_t DENSE_SLOTS, int V, int NT>
__device__ __forceinline__ void coef(const KArgs &a, const Streams &st, int k, int q,
                                     int64_t e0, T (&out)[V])
{
    if constexpr (MODE == M_UNIFORM) {
        const T u = (T)a.uniform[k];
#pragma unroll
        for (int i = 0; i < V; ++i)
            out[i] = u;
    } else if constexpr (MODE == M_ELEM || MODE == M_QP) {
        const int j = popc_below(DENSE_SLOTS, k);
        const int64_t row = (MODE == M_QP) ? (int64_t)j * a.n_q + q : (int64_t)j;
        loadv<V, NT>(static_cast<const T *>(st.coeffs) + row * st.ld_in + e0, out);
    } else {
        const int j = a.col[k];
        if (j < 0) {
            const T u = (T)a.uniform[k];
#pragma unroll
            for (int i = 0; i < V; ++i)
                out[i] = u;
        } else {
            const int64_t row = (MODE == M_QP_MIXED) ? (int64_t)j * a.n_q + q : (int64_t)j;
            loadv<V, NT>(static_cast<const T *>(st.coeffs) + row * st.ld_in + e0, out);
        }
    }
}

// Addressing of one problem block. ScalarBlock is the scalar problem itself;
// VecBlock is the (alpha = A, beta = B) block of the general 3-component
// problem: its scalar slot k stands for c^{a;b}_{A B} (k = 4a+b) or d^a_A
// (k = 16+a), read from row col[k] + component of the compact array (col[k]
// < 0: the block is absent and zero), and its K entry (r, s) is the entry
// (3r+A, 3s+B) of the full matrix. F belongs to the B = 0 blocks. A and B are
// wave-uniform run-time values, so the nine blocks share one copy of the code.
struct ScalarBlock {
    __device__ __forceinline__ bool with_f() const { return true; }
    template <typename T, int MODE, uint32_t SL, int V, int NT>
    __device__ __forceinline__ void coef(const KArgs &a, const Streams &st, int k, int q,
                                         int64_t e0, T (&out)[V]) const
    {
        fe::coef<T, MODE, SL, V, NT>(a, st, k, q, e0, out);
    }
    __device__ __forceinline__ int k_index(int NS, int packed, int r, int s) const
    {
        return packed ? pidx(NS, r, s) : NS * r + s;
    }
    __device__ __forceinline__ int f_index(int r) const { return r; }
    // Results: K entry (r, s) of an N x N matrix and F entry r, for V elements.
    template <int V, int NT, typename T>
    __device__ __forceinline__ void put_k(const Streams &st, int N, int packed, int r, int s,
                                          int64_t e0, const T (&val)[V]) const
    {
        storev<V, NT>(static_cast<T *>(st.out_K) + k_index(N, packed, r, s) * st.ld_out + e0, val);
    }
    template <int V, int NT, typename T>
    __device__ __forceinline__ void put_f(const Streams &st, int r, int64_t e0, const T (&val)[V]) const
    {
        storev<V, NT>(static_cast<T *>(st.out_F) + f_index(r) * st.ld_out + e0, val);
    }
};

struct VecBlock {
    int A, B;
    __device__ __forceinline__ bool with_f() const { return B == 0; }
    template <typename T, int MODE, uint32_t SL, int V, int NT>
    __device__ __forceinline__ void coef(const KArgs &a, const Streams &st, int k, int q,
                                         int64_t e0, T (&out)[V]) const
    {
        const int j = a.col[k];
        if (j < 0) {
#pragma unroll
            for (int i = 0; i < V; ++i)
                out[i] = T(0);
            return;
        }
        const int64_t row = j + (k < 16 ? 3 * A + B : A);
        const int64_t r = (MODE == M_QP) ? row * a.n_q + q : row;
        loadv<V, NT>(static_cast<const T *>(st.coeffs) + r * st.ld_in + e0, out);
    }
    __device__ __forceinline__ int k_index(int NS, int, int r, int s) const
    {
        return (3 * r + A) * (3 * NS) + 3 * s + B;
    }
    __device__ __forceinline__ int f_index(int r) const { return 3 * r + A; }
    template <int V, int NT, typename T>
    __device__ __forceinline__ void put_k(const Streams &st, int N, int packed, int r, int s,
                                          int64_t e0, const T (&val)[V]) const
    {
        storev<V, NT>(static_cast<T *>(st.out_K) + k_index(N, packed, r, s) * st.ld_out + e0, val);
    }
    template <int V, int NT, typename T>
    __device__ __forceinline__ void put_f(const Streams &st, int r, int64_t e0, const T (&val)[V]) const
    {
        storev<V, NT>(static_cast<T *>(st.out_F) + f_index(r) * st.ld_out + e0, val);
    }
};

// The (A, B) block of a 3-component problem handed to a consumer of whole
// element matrices (matrix-free application, assembly): block entry (r, s)
// is entry (3r + A, 3s + B) of the full 3NS x 3NS matrix, F entry r of a
// B = 0 block is entry 3r + A. Coefficient addressing is VecBlock's.
template <class IN>
struct VecConsumer : VecBlock {
    const IN *in;
    __device__ __forceinline__ bool with_f() const { return B == 0 && in->with_f(); }
    template <int V, int NT, typename U>
    __device__ __forceinline__ void put_k(const Streams &st, int NS, int, int r, int s, int64_t e0,
                                          const U (&val)[V]) const
    {
        in->template put_k<V, NT>(st, 3 * NS, 0, 3 * r + A, 3 * s + B, e0, val);
    }
    template <int V, int NT, typename U>
    __device__ __forceinline__ void put_f(const Streams &st, int r, int64_t e0, const U (&val)[V]) const
    {
        in->template put_f<V, NT>(st, 3 * r + A, e0, val);
    }
};

// Matrix-free consumer of one element's results (one element per lane): K
// is applied to the element's nodal values x as its entries are produced,
// y_r += K_rs x_s (and y_s += K_rs x_r for the mirrored entry of a packed
// symmetric K), and F is added to b when b is requested. The element matrix
// is never stored. x, y, b are the lane's local arrays.
template <typename T, bool WITH_B>
struct ApplyBlock : ScalarBlock {
    const T *x;
    T *y;
    T *b;  // used when WITH_B
    __device__ __forceinline__ bool with_f() const { return WITH_B; }
    template <int V, int NT, typename U>
    __device__ __forceinline__ void put_k(const Streams &, int, int packed, int r, int s, int64_t,
                                          const U (&val)[V]) const
    {
        static_assert(V == 1, "matrix-free application is one element per lane");
        y[r] += val[0] * x[s];
        if (packed && r != s)
            y[s] += val[0] * x[r];
    }
    template <int V, int NT, typename U>
    __device__ __forceinline__ void put_f(const Streams &, int r, int64_t, const U (&val)[V]) const
    {
        b[r] += val[0];
    }
};

// Assembly into a CSR matrix (one element per lane): each entry of K goes to
// the global entry of its (row, column), and to the mirrored entry for a
// packed symmetric K; F goes to b. The element matrix is never stored.
// Element dof r = NC v + alpha sits in global row NC id[v] + alpha; rp[v] is
// where row NC id[v] starts, len[v] its length (the rows of a node's
// components have equal length and the same columns), off[v][u] the
// position of column NC id[u] in it, or -1 when the pattern lacks it (the
// entry is then dropped; nothing is written outside vals).
// DEFER: the entries are collected in the lane's array kv (and fv) and
// added by the kernel afterwards, all loads before all stores (the plain
// read-add-write of a coloured launch; small K only); otherwise each entry
// is added as it is produced.
template <typename T, bool ATOMIC>
__device__ __forceinline__ void add_at(T *p, T v)
{
    if constexpr (ATOMIC)
        unsafeAtomicAdd(p, v);
    else
        *p += v;
}

template <typename T, int NV, int NC, bool ATOMIC, bool WITH_B, bool DEFER>
struct CsrBlock : ScalarBlock {
    static constexpr int N = NV * NC;
    T *vals;
    T *b;   // used when WITH_B
    T *kv;  // DEFER: N x N entries
    T *fv;  // DEFER: N entries
    int64_t nnz;
    uint32_t id[NV];
    int64_t rp[NV];
    int32_t len[NV];
    int32_t off[NV][NV];
    __device__ __forceinline__ bool with_f() const { return WITH_B; }
    // position of entry (r, s) in vals, or -1
    __device__ __forceinline__ int64_t pos(int r, int s) const
    {
        const int vr = r / NC, al = r % NC, vs = s / NC, be = s % NC;
        const int o = off[vr][vs];
        if (o < 0)
            return -1;
        const int64_t p = rp[vr] + (int64_t)al * len[vr] + o + be;
        return p < nnz ? p : -1;
    }
    __device__ __forceinline__ void add(int r, int s, T v) const
    {
        if constexpr (DEFER) {
            kv[r * N + s] = v;
        } else {
            const int64_t p = pos(r, s);
            if (p >= 0)
                add_at<T, ATOMIC>(vals + p, v);
        }
    }
    template <int V, int NT, typename U>
    __device__ __forceinline__ void put_k(const Streams &, int, int packed, int r, int s, int64_t,
                                          const U (&val)[V]) const
    {
        static_assert(V == 1, "assembly is one element per lane");
        add(r, s, val[0]);
        if (packed && r != s)
            add(s, r, val[0]);
    }
    template <int V, int NT, typename U>
    __device__ __forceinline__ void put_f(const Streams &, int r, int64_t, const U (&val)[V]) const
    {
        if constexpr (WITH_B) {
            if constexpr (DEFER)
                fv[r] = val[0];
            else
                add_at<T, ATOMIC>(b + (int64_t)NC * id[r / NC] + r % NC, val[0]);
        }
    }
    // DEFER: add the collected entries, every load issued before any store
    __device__ __forceinline__ void flush() const
    {
        int64_t p[N * N];
        T old[N * N];
#pragma unroll
        for (int r = 0; r < N; ++r)
#pragma unroll
            for (int s = 0; s < N; ++s) {
                p[r * N + s] = pos(r, s);
                old[r * N + s] = p[r * N + s] >= 0 ? vals[p[r * N + s]] : T(0);
            }
        T oldb[N];
        if constexpr (WITH_B) {
#pragma unroll
            for (int r = 0; r < N; ++r)
                oldb[r] = b[(int64_t)NC * id[r / NC] + r % NC];
        }
#pragma unroll
        for (int k = 0; k < N * N; ++k)
            if (p[k] >= 0)
                vals[p[k]] = old[k] + kv[k];
        if constexpr (WITH_B) {
#pragma unroll
            for (int r = 0; r < N; ++r)
                b[(int64_t)NC * id[r / NC] + r % NC] = oldb[r] + fv[r];
        }
    }
};

// Row ownership (one node per lane): of element e's K and F only the rows
// of the owning node's local vertex lv are kept, kr[alpha][s] = K_{NC lv +
// alpha, s} (a packed symmetric K also gives them from the mirrored
// entries) and fr[alpha] = F_{NC lv + alpha}; the kernel adds them to the
// node's rows.
template <typename T, int NV, int NC>
struct RowBlock : ScalarBlock {
    static constexpr int N = NV * NC;
    int lv;
    T *kr;  // NC x N
    T *fr;  // NC
    __device__ __forceinline__ bool with_f() const { return true; }
    template <int V, int NT, typename U>
    __device__ __forceinline__ void put_k(const Streams &, int, int packed, int r, int s, int64_t,
                                          const U (&val)[V]) const
    {
        static_assert(V == 1, "assembly is one element per lane");
        if (r / NC == lv)
            kr[(r % NC) * N + s] = val[0];
        if (packed && r != s && s / NC == lv)
            kr[(s % NC) * N + r] = val[0];
    }
    template <int V, int NT, typename U>
    __device__ __forceinline__ void put_f(const Streams &, int r, int64_t, const U (&val)[V]) const
    {
        if (r / NC == lv)
            fr[r % NC] = val[0];
    }
};

// Coefficient functions: slot k's value at the physical point x is
// alpha_k + beta_k sin(2 pi (omega_k . x) + theta_k), parameters p[6k..6k+5]
// (read with wave-uniform scalar loads); with p[121] != 0 the diffusion block
// becomes A A^T + p[120] I. Evaluated in FP64 with the device sin; only the
// slots of the term set that the mask marks are computed.
template <uint32_t SL, int V>
__device__ __forceinline__ void fn_values(const KArgs &a, const double *p, const double (&x)[V][3],
                                          double (&fv)[20][V])
{
    const double two_pi = 6.283185307179586476925286766559;
#pragma unroll
    for (int k = 0; k < 20; ++k) {
        if (!((SL >> k) & 1u))
            continue;
        if (a.col[k] < 0) {
#pragma unroll
            for (int v = 0; v < V; ++v)
                fv[k][v] = a.uniform[k];
            continue;
        }
        const double al = p[6 * k], be = p[6 * k + 1], wx = p[6 * k + 2], wy = p[6 * k + 3],
                     wz = p[6 * k + 4], th = p[6 * k + 5];
#pragma unroll
        for (int v = 0; v < V; ++v)
            fv[k][v] = al + be * sin(two_pi * (wx * x[v][0] + wy * x[v][1] + wz * x[v][2]) + th);
    }
    if constexpr ((SL >> 5) & 1u) {
        if (p[121] != 0.0) {
#pragma unroll
            for (int v = 0; v < V; ++v) {
                double A[3][3];
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int j = 0; j < 3; ++j)
                        A[i][j] = fv[4 * (i + 1) + 1 + j][v];
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int j = 0; j < 3; ++j) {
                        double c = A[i][0] * A[j][0] + A[i][1] * A[j][1] + A[i][2] * A[j][2];
                        if (i == j)
                            c += p[120];
                        fv[4 * (i + 1) + 1 + j][v] = c;
                    }
            }
        }
    }
}

// Coefficient values at one point for V elements: read from memory or
// uniform (coef), or computed from the coefficient function.
template <typename T, int MODE, uint32_t SL, int V, int NT, class BL = ScalarBlock>
struct PointCoefs {
    double fv[MODE == M_FUNC ? 20 : 1][V];
    BL bl;

    __device__ __forceinline__ explicit PointCoefs(const BL &b = BL()) : bl(b) {}

    // x: physical coordinates of the point for each element (function mode)
    __device__ __forceinline__ void prepare(const KArgs &a, const double (&x)[V][3])
    {
        if constexpr (MODE == M_FUNC)
            fn_values<SL, V>(a, static_cast<const double *>(a.coeffs), x, fv);
    }

    __device__ __forceinline__ void get(const KArgs &a, const Streams &st, int k, int q,
                                        int64_t e0, T (&out)[V]) const
    {
        if constexpr (MODE == M_FUNC) {
#pragma unroll
            for (int v = 0; v < V; ++v)
                out[v] = (T)fv[k][v];
        } else {
            bl.template coef<T, MODE, SL, V, NT>(a, st, k, q, e0, out);
        }
    }
};

// Reference tables: kernel arguments or an LDS copy.
struct RefLds {
    double w[FE_MAX_QP];
    double phi[FE_MAX_QP][6];
    double dphi[FE_MAX_QP][6][3];
};

template <int REF>
struct Ref {
    const KArgs &a;
    const RefLds *s;
    __device__ __forceinline__ double w(int q) const { return REF == REF_LDS ? s->w[q] : a.w[q]; }
    __device__ __forceinline__ double phi(int q, int r) const
    {
        return REF == REF_LDS ? s->phi[q][r] : a.phi[q][r];
    }
    __device__ __forceinline__ double dphi(int q, int r, int k) const
    {
        return REF == REF_LDS ? s->dphi[q][r][k] : a.dphi[q][r][k];
    }
    // The tables in the arithmetic type U: FP32 reads the rounded copies in
    // the kernel arguments; otherwise the FP64 value is converted.
    template <typename U>
    __device__ __forceinline__ U dphi_t(int q, int r, int k) const
    {
        if constexpr (sizeof(U) == 4 && REF == REF_KARG)
            return a.dphi_f[q][r][k];
        return (U)dphi(q, r, k);
    }
    template <typename U>
    __device__ __forceinline__ U phi_t(int q, int r) const
    {
        if constexpr (sizeof(U) == 4 && REF == REF_KARG)
            return a.phi_f[q][r];
        return (U)phi(q, r);
    }
};

// ------------------------------------------------- tetrahedron geometry
// Affine tetrahedron: the columns of J are X1-X0, X2-X0, X3-X0; the rows of
// J^{-1} are the cross products (b x c, c x a, a x b) / det, which are the
// global gradients of shape functions 1..3; gradient 0 is minus their sum.
template <typename T>
__device__ __forceinline__ void tet_geometry(const double (&X)[12], T (&g)[4][3], T &det_t)
{
    double a[3], b[3], c[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        a[d] = X[3 + d] - X[d];
        b[d] = X[6 + d] - X[d];
        c[d] = X[9 + d] - X[d];
    }
    double n[4][3];
    n[1][0] = b[1] * c[2] - b[2] * c[1];
    n[1][1] = b[2] * c[0] - b[0] * c[2];
    n[1][2] = b[0] * c[1] - b[1] * c[0];
    n[2][0] = c[1] * a[2] - c[2] * a[1];
    n[2][1] = c[2] * a[0] - c[0] * a[2];
    n[2][2] = c[0] * a[1] - c[1] * a[0];
    n[3][0] = a[1] * b[2] - a[2] * b[1];
    n[3][1] = a[2] * b[0] - a[0] * b[2];
    n[3][2] = a[0] * b[1] - a[1] * b[0];
    const double det = a[0] * n[1][0] + a[1] * n[1][1] + a[2] * n[1][2];
    const double inv = 1.0 / det;
#pragma unroll
    for (int d = 0; d < 3; ++d) {
        const double g1 = n[1][d] * inv, g2 = n[2][d] * inv, g3 = n[3][d] * inv;
        g[1][d] = (T)g1;
        g[2][d] = (T)g2;
        g[3][d] = (T)g3;
        g[0][d] = (T)(-(g1 + g2 + g3));
    }
    det_t = (T)det;
}

// Vertex coordinates relative to vertex 0 (edge vectors). The reference
// derivatives sum to zero, so J = sum_r (X_r - X_0) dphi_r/dxi exactly, and
// the edge vectors avoid the cancellation of absolute coordinates in the
// thin direction of sliver elements (the FP64 result stays within a few ulp
// of the exact one there).
template <int NS>
__device__ __forceinline__ void to_edge_vectors(double (&X)[NS * 3])
{
#pragma unroll
    for (int r = NS - 1; r >= 1; --r)
#pragma unroll
        for (int i = 0; i < 3; ++i)
            X[3 * r + i] -= X[i];
}

// Reference derivatives of the linear prism that vanish at every point, for
// any rule: d/dxi of shape functions 2 and 5 and d/deta of 1 and 4 (the
// triangle functions eta and xi do not depend on the other coordinate).
// Their terms are left out of the sums below (adding a zero product leaves
// a finite sum unchanged).
__device__ __forceinline__ constexpr bool prism_zero_derivative(int r, int k)
{
    return (k == 0 && (r == 2 || r == 5)) || (k == 1 && (r == 1 || r == 4));
}

// Element given by tables (prism): Jacobian terms at one point from the
// edge vectors E (E_r = X_r - X_0, r >= 1): J[i][k] = sum_r E_r,i dphi_r/dxi_k,
// Ji[k][i] = (J^{-1})_{k i} and det J.
template <int NS, class R>
__device__ __forceinline__ void point_jacobian(const double (&E)[NS * 3], const R &ref, int q,
                                               double (&Ji)[3][3], double &det)
{
    double J[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            double s = 0.0;
#pragma unroll
            for (int r = 1; r < NS; ++r)
                if (!(NS == 6 && prism_zero_derivative(r, k)))
                    s += E[3 * r + i] * ref.dphi(q, r, k);
            J[i][k] = s;
        }
    const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
    const double inv = 1.0 / det;
    Ji[0][0] = c00 * inv;
    Ji[1][0] = c01 * inv;
    Ji[2][0] = c02 * inv;
    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * inv;
    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * inv;
    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * inv;
    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * inv;
    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * inv;
    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * inv;
}

// Global derivatives at one point: g_r = J^{-T} grad_ref phi_r, and
// vol = det J w_q.
template <int NS, typename T, class R>
__device__ __forceinline__ void point_geometry(const double (&E)[NS * 3], const R &ref, int q,
                                               T (&g)[NS][3], T &vol_t)
{
    double Ji[3][3], det;
    point_jacobian<NS>(E, ref, q, Ji, det);
#pragma unroll
    for (int r = 0; r < NS; ++r) {
        const double d0 = ref.dphi(q, r, 0), d1 = ref.dphi(q, r, 1), d2 = ref.dphi(q, r, 2);
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            if (NS == 6 && prism_zero_derivative(r, 0))
                g[r][i] = (T)(d1 * Ji[1][i] + d2 * Ji[2][i]);
            else if (NS == 6 && prism_zero_derivative(r, 1))
                g[r][i] = (T)(d0 * Ji[0][i] + d2 * Ji[2][i]);
            else
                g[r][i] = (T)(d0 * Ji[0][i] + d1 * Ji[1][i] + d2 * Ji[2][i]);
        }
    }
    vol_t = (T)(det * ref.w(q));
}

// Lame parameters from Young's modulus and Poisson's ratio.
template <typename T>
__device__ __forceinline__ void lame(T E, T nu, T &lam, T &mu)
{
    lam = E * nu / ((T(1) + nu) * (T(1) - T(2) * nu));
    mu = E / (T(2) * (T(1) + nu));
}

// ===================================================== tetrahedron, scalar
template <typename T, int TERMS, int MODE, int PACKED, class BL = ScalarBlock>
struct TetScalar {
    static constexpr uint32_t SL = slots_of_terms(TERMS);
    static constexpr bool DIFF = TERMS & T_DIFF, CA = TERMS & T_CONVA, CB = TERMS & T_CONVB,
                          MASS = TERMS & T_MASS, DG = TERMS & T_DGRAD, D0 = TERMS & T_D0;
    static constexpr bool PER_QP = (MODE == M_QP || MODE == M_QP_MIXED || MODE == M_FUNC);
    // coefficients read from memory by element id
    static constexpr bool ELEM_COEFS = MODE != M_UNIFORM && MODE != M_FUNC;

    template <int V, int NT, int REF, class S>
    __device__ __forceinline__ static void run(const KArgs &a, const S &st, const Ref<REF> &ref,
                                               int64_t e0)
    {
        double X[V][12];
        st.template load_coords<4, V, NT>(e0, X);
        if constexpr (!PER_QP)
            run_const<V, NT>(a, st, X, e0);
        else
            run_qp<V, NT, REF>(a, st, ref, X, e0);
    }

    template <int V, int NT, class B2>
    __device__ __forceinline__ static void store_K(const Streams &st, int r, int s, int64_t e0,
                                                   const T (&val)[V], const B2 &bl)
    {
        bl.template put_k<V, NT>(st, 4, PACKED, r, s, e0, val);
    }

    // One element from its vertex coordinates, results to bl (matrix-free).
    template <int NT, int REF, class B2>
    __device__ __forceinline__ static void apply_x(const KArgs &a, const Streams &st, const Ref<REF> &ref,
                                                   const double (&X)[12], int64_t e, const B2 &bl)
    {
        const double (&Xv)[1][12] = reinterpret_cast<const double (&)[1][12]>(X);
        if constexpr (PER_QP)
            run_qp<1, NT, REF>(a, st, ref, Xv, e, bl);
        else
            run_const<1, NT>(a, st, Xv, e, bl);
    }

    // Coefficients constant over the element: with the (constant) gradients
    // g, the weighted moments W, m_r, M_rs of the reference shape functions
    // carry the whole point sum:
    //   K_rs = det [W g_r . C g_s + (c^{.;0} . g_r) m_s + m_r (c^{0;.} . g_s)
    //               + c^{0;0} M_rs],   F_r = det [W d . g_r + d^0 m_r].
    template <int V, int NT, class B2 = BL>
    __device__ __forceinline__ static void run_const(const KArgs &a, const Streams &st,
                                                     const double (&X)[V][12],
                                                     int64_t e0, const B2 &bl = B2())
    {
        T C[3][3][V], ca[3][V], cb[3][V], c00[V], d[3][V], d0[V];
        if constexpr (DIFF) {
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j)
                    bl.template coef<T, MODE, SL, V, NT>(a, st, 4 * (i + 1) + 1 + j, 0, e0, C[i][j]);
        }
        if constexpr (CA) {
#pragma unroll
            for (int i = 0; i < 3; ++i)
                bl.template coef<T, MODE, SL, V, NT>(a, st, 4 * (i + 1), 0, e0, ca[i]);
        }
        if constexpr (CB) {
#pragma unroll
            for (int j = 0; j < 3; ++j)
                bl.template coef<T, MODE, SL, V, NT>(a, st, 1 + j, 0, e0, cb[j]);
        }
        if constexpr (MASS)
            bl.template coef<T, MODE, SL, V, NT>(a, st, 0, 0, e0, c00);
        const bool wf = bl.with_f();
        if constexpr (DG) {
#pragma unroll
            for (int i = 0; i < 3; ++i) {
#pragma unroll
                for (int v = 0; v < V; ++v)
                    d[i][v] = T(0);
                if (wf)
                    bl.template coef<T, MODE, SL, V, NT>(a, st, 17 + i, 0, e0, d[i]);
            }
        }
        if constexpr (D0) {
#pragma unroll
            for (int v = 0; v < V; ++v)
                d0[v] = T(0);
            if (wf)
                bl.template coef<T, MODE, SL, V, NT>(a, st, 16, 0, e0, d0);
        }

        const T W = (T)a.Wsum;
        T Kv[4][4][V], Fv[4][V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            T g[4][3], det;
            tet_geometry<T>(X[v], g, det);
            const T sw = det * W;
            T al[4], be[4];
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                al[r] = T(0);
                be[r] = T(0);
                if constexpr (CA)
                    al[r] = det * (ca[0][v] * g[r][0] + ca[1][v] * g[r][1] + ca[2][v] * g[r][2]);
                if constexpr (CB)
                    be[r] = det * (cb[0][v] * g[r][0] + cb[1][v] * g[r][1] + cb[2][v] * g[r][2]);
            }
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                T t[3] = {T(0), T(0), T(0)};
                if constexpr (DIFF) {
#pragma unroll
                    for (int i = 0; i < 3; ++i)
                        t[i] = sw * (C[i][0][v] * g[s][0] + C[i][1][v] * g[s][1] + C[i][2][v] * g[s][2]);
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if (PACKED && s < r)
                        continue;
                    T x = T(0);
                    if constexpr (DIFF)
                        x = g[r][0] * t[0] + g[r][1] * t[1] + g[r][2] * t[2];
                    if constexpr (CA)
                        x += al[r] * (T)a.m[s];
                    if constexpr (CB)
                        x += (T)a.m[r] * be[s];
                    if constexpr (MASS)
                        x += det * c00[v] * (T)a.M[r][s];
                    // stored below, element by element within the group
                    Kv[r][s][v] = x;
                }
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                T x = T(0);
                if constexpr (DG)
                    x = sw * (d[0][v] * g[r][0] + d[1][v] * g[r][1] + d[2][v] * g[r][2]);
                if constexpr (D0)
                    x += det * d0[v] * (T)a.m[r];
                Fv[r][v] = x;
            }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int s = (PACKED ? r : 0); s < 4; ++s)
                store_K<V, NT>(st, r, s, e0, Kv[r][s], bl);
        if (bl.with_f()) {
#pragma unroll
            for (int r = 0; r < 4; ++r)
                bl.template put_f<V, NT>(st, r, e0, Fv[r]);
        }
    }

    // Coefficients per point (Algorithm 3 with "calculate possibly
    // coefficients" inside the point loop): the point sums of weight x
    // coefficient x reference values are formed first, then contracted with
    // the constant gradients:
    //   Cb = sum_q w C_q, Pb_s = sum_q w phi_s c^{.;0}_q, Qb_r = sum_q w phi_r c^{0;.}_q,
    //   Mb_rs = sum_q w c^{0;0}_q phi_r phi_s, Db = sum_q w d_q, fb_r = sum_q w d^0_q phi_r,
    //   K_rs = det (g_r . Cb g_s + g_r . Pb_s + Qb_r . g_s + Mb_rs), F_r = det (Db . g_r + fb_r).
    template <int V, int NT, int REF, class B2 = BL>
    __device__ __forceinline__ static void run_qp(const KArgs &a, const Streams &st, const Ref<REF> &ref,
                                                  const double (&X)[V][12], int64_t e0,
                                                  const B2 &bl = B2())
    {
        const bool wf = bl.with_f();
        T Cb[V][3][3], Pb[V][4][3], Qb[V][4][3], Mb[V][4][4], Db[V][3], fb[V][4];
#pragma unroll
        for (int v = 0; v < V; ++v) {
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                Db[v][i] = T(0);
#pragma unroll
                for (int j = 0; j < 3; ++j)
                    Cb[v][i][j] = T(0);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                fb[v][r] = T(0);
#pragma unroll
                for (int i = 0; i < 3; ++i)
                    Pb[v][r][i] = Qb[v][r][i] = T(0);
#pragma unroll
                for (int s = 0; s < 4; ++s)
                    Mb[v][r][s] = T(0);
            }
        }
        for (int q = 0; q < a.n_q; ++q) {
            PointCoefs<T, MODE, SL, V, NT, B2> pc(bl);
            if constexpr (MODE == M_FUNC) {
                // physical point x(xi_q) = X_0 + sum_r phi_r(xi_q) (X_r - X_0)
                double x[V][3];
#pragma unroll
                for (int v = 0; v < V; ++v)
#pragma unroll
                    for (int i = 0; i < 3; ++i)
                        x[v][i] = X[v][i] + ref.phi(q, 1) * (X[v][3 + i] - X[v][i]) +
                                  ref.phi(q, 2) * (X[v][6 + i] - X[v][i]) +
                                  ref.phi(q, 3) * (X[v][9 + i] - X[v][i]);
                pc.prepare(a, x);
            }
            const T w = (T)ref.w(q);
            T wp[4];
#pragma unroll
            for (int r = 0; r < 4; ++r)
                wp[r] = w * (T)ref.phi(q, r);
            T c[V];
            if constexpr (DIFF) {
#pragma unroll
                for (int i = 0; i < 3; ++i)
#pragma unroll
                    for (int j = 0; j < 3; ++j) {
                        pc.get(a, st, 4 * (i + 1) + 1 + j, q, e0, c);
#pragma unroll
                        for (int v = 0; v < V; ++v)
                            Cb[v][i][j] += w * c[v];
                    }
            }
            if constexpr (CA) {
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    pc.get(a, st, 4 * (i + 1), q, e0, c);
#pragma unroll
                    for (int v = 0; v < V; ++v)
#pragma unroll
                        for (int s = 0; s < 4; ++s)
                            Pb[v][s][i] += wp[s] * c[v];
                }
            }
            if constexpr (CB) {
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    pc.get(a, st, 1 + j, q, e0, c);
#pragma unroll
                    for (int v = 0; v < V; ++v)
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            Qb[v][r][j] += wp[r] * c[v];
                }
            }
            if constexpr (MASS) {
                pc.get(a, st, 0, q, e0, c);
#pragma unroll
                for (int v = 0; v < V; ++v)
#pragma unroll
                    for (int r = 0; r < 4; ++r)
#pragma unroll
                        for (int s = 0; s < 4; ++s)
                            Mb[v][r][s] += wp[r] * (T)ref.phi(q, s) * c[v];
            }
            if constexpr (DG) {
                if (wf) {
#pragma unroll
                    for (int i = 0; i < 3; ++i) {
                        pc.get(a, st, 17 + i, q, e0, c);
#pragma unroll
                        for (int v = 0; v < V; ++v)
                            Db[v][i] += w * c[v];
                    }
                }
            }
            if constexpr (D0) {
                if (wf) {
                    pc.get(a, st, 16, q, e0, c);
#pragma unroll
                    for (int v = 0; v < V; ++v)
#pragma unroll
                        for (int r = 0; r < 4; ++r)
                            fb[v][r] += wp[r] * c[v];
                }
            }
        }
        T Kv[4][4][V], Fv[4][V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            T g[4][3], det;
            tet_geometry<T>(X[v], g, det);
#pragma unroll
            for (int s = 0; s < 4; ++s) {
                T t[3];
#pragma unroll
                for (int i = 0; i < 3; ++i) {
                    T x = T(0);
                    if constexpr (DIFF)
                        x = Cb[v][i][0] * g[s][0] + Cb[v][i][1] * g[s][1] + Cb[v][i][2] * g[s][2];
                    if constexpr (CA)
                        x += Pb[v][s][i];
                    t[i] = x;
                }
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    if (PACKED && s < r)
                        continue;
                    T x = T(0);
                    if constexpr (DIFF || CA)
                        x = g[r][0] * t[0] + g[r][1] * t[1] + g[r][2] * t[2];
                    if constexpr (CB)
                        x += Qb[v][r][0] * g[s][0] + Qb[v][r][1] * g[s][1] + Qb[v][r][2] * g[s][2];
                    if constexpr (MASS)
                        x += Mb[v][r][s];
                    Kv[r][s][v] = det * x;
                }
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                T x = T(0);
                if constexpr (DG)
                    x = Db[v][0] * g[r][0] + Db[v][1] * g[r][1] + Db[v][2] * g[r][2];
                if constexpr (D0)
                    x += fb[v][r];
                Fv[r][v] = det * x;
            }
        }
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int s = (PACKED ? r : 0); s < 4; ++s)
                store_K<V, NT>(st, r, s, e0, Kv[r][s], bl);
        if (bl.with_f()) {
#pragma unroll
            for (int r = 0; r < 4; ++r)
                bl.template put_f<V, NT>(st, r, e0, Fv[r]);
        }
    }
};

// ============================================ tetrahedron, 3-component CDR
// The general 3-component problem block by block: the (alpha, beta) block of
// K is the scalar form with the coefficients c^{a;b}_{alpha beta}, and F_alpha
// the scalar load with d^a_alpha, so each of the nine blocks runs the scalar
// contraction on the same vertex coordinates (the geometry is recomputed per
// block; it is a few dozen operations against the block's memory traffic).
template <typename T, int MODE>
struct TetVector {
    static constexpr bool PER_QP = (MODE == M_QP);
    // each block's coefficients are read after earlier blocks are stored
    static constexpr bool INTERLEAVED_IO = true;
    typedef TetScalar<T, TS_FULL, MODE, 0, VecBlock> P;

    template <int V, int NT, int REF, class S>
    __device__ __forceinline__ static void run(const KArgs &a, const S &st, const Ref<REF> &ref,
                                               int64_t e0)
    {
        double X[V][12];
        st.template load_coords<4, V, NT>(e0, X);
#pragma unroll 1
        for (int b = 0; b < 9; ++b) {
            const VecBlock bl{b / 3, b % 3};
            if constexpr (PER_QP)
                P::template run_qp<V, NT, REF>(a, st, ref, X, e0, bl);
            else
                P::template run_const<V, NT>(a, st, X, e0, bl);
        }
    }

    // Matrix-free and assembly consumers: the nine blocks handed to bl.
    template <int NT, int REF, class B2>
    __device__ __forceinline__ static void apply_x(const KArgs &a, const Streams &st, const Ref<REF> &ref,
                                                   const double (&X)[12], int64_t e, const B2 &bl)
    {
        const double (&Xv)[1][12] = reinterpret_cast<const double (&)[1][12]>(X);
#pragma unroll 1
        for (int b = 0; b < 9; ++b) {
            VecConsumer<B2> vb;
            vb.A = b / 3;
            vb.B = b % 3;
            vb.in = &bl;
            if constexpr (PER_QP)
                P::template run_qp<1, NT, REF>(a, st, ref, Xv, e, vb);
            else
                P::template run_const<1, NT>(a, st, Xv, e, vb);
        }
    }
};

// ================================================= tetrahedron, elasticity
// K_(r a),(s b) = det [lam_b g_ra g_sb + mu_b g_rb g_sa + mu_b delta_ab g_r . g_s]
// with lam_b = sum_q w_q lambda_q, mu_b likewise (gradients are constant);
// F_(r a) = det sum_q w_q f_a,q phi_r(xi_q).
template <typename T, int MODE, int PACKED, class BL = ScalarBlock>
struct TetElastic {
    static constexpr uint32_t SL = 31u;
    static constexpr bool PER_QP = (MODE == M_QP || MODE == M_QP_MIXED || MODE == M_FUNC);

    template <int V, int NT, int REF, class S>
    __device__ __forceinline__ static void run(const KArgs &a, const S &st, const Ref<REF> &ref,
                                               int64_t e0)
    {
        double X[V][12];
        st.template load_coords<4, V, NT>(e0, X);
        run_x<V, NT, REF>(a, st, ref, X, e0);
    }

    template <int NT, int REF, class B2>
    __device__ __forceinline__ static void apply_x(const KArgs &a, const Streams &st, const Ref<REF> &ref,
                                                   const double (&X)[12], int64_t e, const B2 &bl)
    {
        run_x<1, NT, REF>(a, st, ref, reinterpret_cast<const double (&)[1][12]>(X), e, bl);
    }

    template <int V, int NT, int REF, class B2 = BL>
    __device__ __forceinline__ static void run_x(const KArgs &a, const Streams &st, const Ref<REF> &ref,
                                                 const double (&X)[V][12], int64_t e0,
                                                 const B2 &bl = B2())
    {
        T lb[V], mb[V], fb[V][4][3];
        if constexpr (!PER_QP) {
            T E[V], nu[V], f[3][V];
            coef<T, MODE, SL, V, NT>(a, st, 0, 0, e0, E);
            coef<T, MODE, SL, V, NT>(a, st, 1, 0, e0, nu);
#pragma unroll
            for (int al = 0; al < 3; ++al)
                coef<T, MODE, SL, V, NT>(a, st, 2 + al, 0, e0, f[al]);
            const T W = (T)a.Wsum;
#pragma unroll
            for (int v = 0; v < V; ++v) {
                T lam, mu;
                lame<T>(E[v], nu[v], lam, mu);
                lb[v] = W * lam;
                mb[v] = W * mu;
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int al = 0; al < 3; ++al)
                        fb[v][r][al] = (T)a.m[r] * f[al][v];
            }
        } else {
#pragma unroll
            for (int v = 0; v < V; ++v) {
                lb[v] = mb[v] = T(0);
#pragma unroll
                for (int r = 0; r < 4; ++r)
#pragma unroll
                    for (int al = 0; al < 3; ++al)
                        fb[v][r][al] = T(0);
            }
            for (int q = 0; q < a.n_q; ++q) {
                const T w = (T)ref.w(q);
                T E[V], nu[V], f[3][V];
                coef<T, MODE, SL, V, NT>(a, st, 0, q, e0, E);
                coef<T, MODE, SL, V, NT>(a, st, 1, q, e0, nu);
#pragma unroll
                for (int al = 0; al < 3; ++al)
                    coef<T, MODE, SL, V, NT>(a, st, 2 + al, q, e0, f[al]);
#pragma unroll
                for (int v = 0; v < V; ++v) {
                    T lam, mu;
                    lame<T>(E[v], nu[v], lam, mu);
                    lb[v] += w * lam;
                    mb[v] += w * mu;
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const T wp = w * (T)ref.phi(q, r);
#pragma unroll
                        for (int al = 0; al < 3; ++al)
                            fb[v][r][al] += wp * f[al][v];
                    }
                }
            }
        }
        T g[V][4][3], det[V];
#pragma unroll
        for (int v = 0; v < V; ++v) {
            tet_geometry<T>(X[v], g[v], det[v]);
            lb[v] *= det[v];
            mb[v] *= det[v];
        }
#pragma unroll
        for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int s = (PACKED ? r : 0); s < 4; ++s) {
                T dot[V];
#pragma unroll
                for (int v = 0; v < V; ++v)
                    dot[v] = mb[v] * (g[v][r][0] * g[v][s][0] + g[v][r][1] * g[v][s][1] +
                                      g[v][r][2] * g[v][s][2]);
#pragma unroll
                for (int al = 0; al < 3; ++al)
#pragma unroll
                    for (int be = 0; be < 3; ++be) {
                        const int row = 3 * r + al, col = 3 * s + be;
                        if (PACKED && col < row)
                            continue;
                        T val[V];
#pragma unroll
                        for (int v = 0; v < V; ++v) {
                            T x = lb[v] * g[v][r][al] * g[v][s][be] + mb[v] * g[v][r][be] * g[v][s][al];
                            if (al == be)
                                x += dot[v];
                            val[v] = x;
                        }
                        bl.template put_k<V, NT>(st, 12, PACKED, row, col, e0, val);
                    }
            }
        if (bl.with_f()) {
#pragma unroll
            for (int r = 0; r < 4; ++r)
#pragma unroll
                for (int al = 0; al < 3; ++al) {
                    T val[V];
#pragma unroll
                    for (int v = 0; v < V; ++v)
                        val[v] = det[v] * fb[v][r][al];
                    bl.template put_f<V, NT>(st, 3 * r + al, e0, val);
                }
        }
    }
};

// ========================================================== prism, scalar
// Algorithm 2 (QSS, geometry per point): for every point the Jacobian terms
// and global derivatives are formed, then the S x S update. PACKED: 0 full
// K, 1 packed upper triangle, 2 a symmetric problem asked for full K (the
// upper triangle is accumulated, both halves stored). With
// u_r = vol g_r, p_r = vol phi_r, t_s = C g_s + phi_s c^{.;0} and
// sigma_s = c^{0;.} . g_s + c^{0;0} phi_s:  K_rs += u_r . t_s + p_r sigma_s,
// F_r += u_r . d + p_r d^0.
template <typename T, int TERMS, int MODE, int PACKED, int NQ, class BL = ScalarBlock>
struct PrismScalar {
    static constexpr uint32_t SL = slots_of_terms(TERMS);
    static constexpr bool DIFF = TERMS & T_DIFF, CA = TERMS & T_CONVA, CB = TERMS & T_CONVB,
                          MASS = TERMS & T_MASS, DG = TERMS & T_DGRAD, D0 = TERMS & T_D0;
    static constexpr bool PER_QP = (MODE == M_QP || MODE == M_QP_MIXED || MODE == M_FUNC);
    static constexpr bool NEED_PHI = CA || CB || MASS || D0;
    // Coefficients that are uniform, per element, or per point slot by slot:
    // the contraction runs in reference coordinates (contract_ref); with
    // every slot per point or coefficient functions the per-point form
    // through the global derivatives measured faster.
    static constexpr bool REF_SPACE = MODE != M_QP && MODE != M_FUNC;

    struct Coefs {
        T C[3][3], ca[3], cb[3], c00, d[3], d0;
    };

    // Physical point x(xi_q) = X_0 + sum_r phi_r(xi_q) E_r from the edge
    // vectors E (function mode only).
    template <class R>
    __device__ __forceinline__ static void point_x(const double (&X0)[3], const double (&E)[18],
                                                   const R &ref, int q, double (&x)[1][3])
    {
#pragma unroll
        for (int i = 0; i < 3; ++i) {
            double s = X0[i];
#pragma unroll
            for (int r = 1; r < 6; ++r)
                s += ref.phi(q, r) * E[3 * r + i];
            x[0][i] = s;
        }
    }

    template <int NT, class R, class B2 = BL>
    __device__ __forceinline__ static void load_coefs(const KArgs &a, const Streams &st, const R &ref,
                                                      int q, int64_t e, const double (&X0)[3],
                                                      const double (&E)[18], Coefs &c,
                                                      const B2 &bl = B2())
    {
        PointCoefs<T, MODE, SL, 1, NT, B2> pc(bl);
        if constexpr (MODE == M_FUNC) {
            double x[1][3];
            point_x(X0, E, ref, q, x);
            pc.prepare(a, x);
        }
        T x[1];
        if constexpr (DIFF) {
#pragma unroll
            for (int i = 0; i < 3; ++i)
#pragma unroll
                for (int j = 0; j < 3; ++j) {
                    pc.get(a, st, 4 * (i + 1) + 1 + j, q, e, x);
                    c.C[i][j] = x[0];
                }
        }
        if constexpr (CA) {
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                pc.get(a, st, 4 * (i + 1), q, e, x);
                c.ca[i] = x[0];
            }
        }
        if constexpr (CB) {
#pragma unroll
            for (int j = 0; j < 3; ++j) {
                pc.get(a, st, 1 + j, q, e, x);
                c.cb[j] = x[0];
            }
        }
        if constexpr (MASS) {
            pc.get(a, st, 0, q, e, x);
            c.c00 = x[0];
        }
        const bool wf = bl.with_f();
        if constexpr (DG) {
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                c.d[i] = T(0);
                if (wf) {
                    pc.get(a, st, 17 + i, q, e, x);
                    c.d[i] = x[0];
                }
            }
        }
        if constexpr (D0) {
            c.d0 = T(0);
            if (wf) {
                pc.get(a, st, 16, q, e, x);
                c.d0 = x[0];
            }
        }
    }

    template <int V, int NT, int REF, class S>
    __device__ __forceinline__ static void run(const KArgs &a, const S &st, const Ref<REF> &ref,
                                               int64_t e)
    {
        static_assert(V == 1, "prisms are processed one element per lane");
        double Xg[1][18];
        st.template load_coords<6, 1, NT>(e, Xg);
        double X[18];
#pragma unroll
        for (int s = 0; s < 18; ++s)
            X[s] = Xg[0][s];
        const double X0[3] = {X[0], X[1], X[2]};
        to_edge_vectors<6>(X);
        body<NT>(a, st, ref, e, X0, X);
    }

    template <int NT, int REF, class B2>
    __device__ __forceinline__ static void apply_x(const KArgs &a, const Streams &st, const Ref<REF> &ref,
                                                   const double (&Xa)[18], int64_t e, const B2 &bl)
    {
        double X[18];
#pragma unroll
        for (int s = 0; s < 18; ++s)
            X[s] = Xa[s];
        const double X0[3] = {X[0], X[1], X[2]};
        to_edge_vectors<6>(X);
        body<NT>(a, st, ref, e, X0, X, bl);
    }

    // Point loop and stores for one element, from vertex 0 and the edge
    // vectors X_r - X_0.
    template <int NT, class R, class B2 = BL>
    __device__ __forceinline__ static void body(const KArgs &a, const Streams &st, const R &ref,
                                                int64_t e, const double (&X0)[3], const double (&X)[18],
                                                const B2 &bl = B2())
    {
        constexpr int NK = PACKED ? 21 : 36;
        T K[NK], F[6];
        accumulate<NT>(a, st, ref, e, X0, X, 0, 1, K, F, bl);
#pragma unroll
        for (int r = 0; r < 6; ++r)
#pragma unroll
            for (int s = (PACKED ? r : 0); s < 6; ++s) {
                const T v[1] = {K[PACKED ? pidx(6, r, s) : 6 * r + s]};
                if constexpr (PACKED == 2) {
                    // symmetric problem stored in full: the upper triangle
                    // is accumulated, both halves are stored
                    bl.template put_k<1, NT>(st, 6, 0, r, s, e, v);
                    if (s != r)
                        bl.template put_k<1, NT>(st, 6, 0, s, r, e, v);
                } else {
                    bl.template put_k<1, NT>(st, 6, PACKED, r, s, e, v);
                }
            }
        if (bl.with_f()) {
#pragma unroll
            for (int r = 0; r < 6; ++r) {
                const T v[1] = {F[r]};
                bl.template put_f<1, NT>(st, r, e, v);
            }
        }
    }

    // One point's contribution to K (and to F when wf) from its gradients g,
    // vol and the shape-function values phi. The trial function is the outer
    // loop: its column of the integrand (the coefficients applied to Phi_s),
    // scaled by vol, meets every test function's Phi_r, so only one column is
    // live at a time.
    template <int NK>
    __device__ __forceinline__ static void contract(const Coefs &c, const T (&g)[6][3], T vol,
                                                    const T (&phi)[6], T (&K)[NK], T (&F)[6],
                                                    bool wf)
    {
#pragma unroll
        for (int s = 0; s < 6; ++s) {
            T ts[3];
#pragma unroll
            for (int i = 0; i < 3; ++i) {
                T x = T(0);
                if constexpr (DIFF)
                    x = c.C[i][0] * g[s][0] + c.C[i][1] * g[s][1] + c.C[i][2] * g[s][2];
                if constexpr (CA)
                    x += phi[s] * c.ca[i];
                ts[i] = vol * x;
            }
            T y = T(0);
            if constexpr (CB)
                y = c.cb[0] * g[s][0] + c.cb[1] * g[s][1] + c.cb[2] * g[s][2];
            if constexpr (MASS)
                y += c.c00 * phi[s];
            const T sgs = vol * y;
#pragma unroll
            for (int r = 0; r < (PACKED ? s + 1 : 6); ++r) {
                const int k = PACKED ? pidx(6, r, s) : 6 * r + s;
                T x = K[k];
                if constexpr (DIFF || CA)
                    x += g[r][0] * ts[0] + g[r][1] * ts[1] + g[r][2] * ts[2];
                if constexpr (CB || MASS)
                    x += phi[r] * sgs;
                K[k] = x;
            }
        }
        if (wf) {
#pragma unroll
            for (int r = 0; r < 6; ++r) {
                if constexpr (DG)
                    F[r] += vol * (g[r][0] * c.d[0] + g[r][1] * c.d[1] + g[r][2] * c.d[2]);
                if constexpr (D0)
                    F[r] += (vol * phi[r]) * c.d0;
            }
        }
    }

    // One point's contribution in reference coordinates, in the tier's
    // arithmetic type U (FP32 starts from the FP64 Jacobian terms): with
    // Jv = vol J^{-1}, the global derivatives never appear, since
    //   vol g_r . C g_s = dphi_r . B dphi_s,     B = Jv C J^{-T}
    //   vol (c^{.;0} . g_r) phi_s = (dphi_r . a) phi_s,   a = Jv c^{.;0}
    //   vol phi_r (c^{0;.} . g_s) = phi_r (b . dphi_s),   b = Jv c^{0;.}
    //   vol g_r . d = dphi_r . f,   f = Jv d,
    // so K_rs += dphi_r . (B dphi_s + a phi_s) + phi_r (b . dphi_s + m phi_s)
    // with m = vol c^{0;0}, and F_r += dphi_r . f + phi_r (vol d^0). The
    // reference derivatives are wave-uniform table values, and the ones that
    // vanish for the prism are skipped.
    template <typename U, class R, int NK>
    __device__ __forceinline__ static void contract_ref(const Coefs &c, const R &ref, int q,
                                                        const double (&Jd)[3][3], double vol,
                                                        T (&K)[NK], T (&F)[6], bool wf)
    {
        U Ji[3][3], Jv[3][3];
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int i = 0; i < 3; ++i)
                Ji[k][i] = (U)Jd[k][i];
#pragma unroll
        for (int k = 0; k < 3; ++k)
#pragma unroll
            for (int i = 0; i < 3; ++i)
                Jv[k][i] = (U)vol * Ji[k][i];
        U B[3][3], av[3], bv[3];
        if constexpr (DIFF) {
            U M[3][3];  // Jv C
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int j = 0; j < 3; ++j)
                    M[k][j] = Jv[k][0] * c.C[0][j] + Jv[k][1] * c.C[1][j] + Jv[k][2] * c.C[2][j];
#pragma unroll
            for (int k = 0; k < 3; ++k)
#pragma unroll
                for (int l = 0; l < 3; ++l)
                    B[k][l] = M[k][0] * Ji[l][0] + M[k][1] * Ji[l][1] + M[k][2] * Ji[l][2];
        }
        if constexpr (CA) {
#pragma unroll
            for (int k = 0; k < 3; ++k)
                av[k] = Jv[k][0] * c.ca[0] + Jv[k][1] * c.ca[1] + Jv[k][2] * c.ca[2];
        }
        if constexpr (CB) {
#pragma unroll
            for (int k = 0; k < 3; ++k)
                bv[k] = Jv[k][0] * c.cb[0] + Jv[k][1] * c.cb[1] + Jv[k][2] * c.cb[2];
        }
        const U m = MASS ? (U)vol * c.c00 : U(0);
#pragma unroll
        for (int s = 0; s < 6; ++s) {
            const U ps = NEED_PHI ? ref.template phi_t<U>(q, s) : U(0);
            U u[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                U x = U(0);
                if constexpr (DIFF) {
#pragma unroll
                    for (int l = 0; l < 3; ++l)
                        if (!prism_zero_derivative(s, l))
                            x += B[k][l] * ref.template dphi_t<U>(q, s, l);
                }
                if constexpr (CA)
                    x += av[k] * ps;
                u[k] = x;
            }
            U sg = U(0);
            if constexpr (CB) {
#pragma unroll
                for (int l = 0; l < 3; ++l)
                    if (!prism_zero_derivative(s, l))
                        sg += bv[l] * ref.template dphi_t<U>(q, s, l);
            }
            if constexpr (MASS)
                sg += m * ps;
#pragma unroll
            for (int r = 0; r < (PACKED ? s + 1 : 6); ++r) {
                const int kk = PACKED ? pidx(6, r, s) : 6 * r + s;
                T x = K[kk];
                if constexpr (DIFF || CA) {
#pragma unroll
                    for (int k = 0; k < 3; ++k)
                        if (!prism_zero_derivative(r, k))
                            x += ref.template dphi_t<U>(q, r, k) * u[k];
                }
                if constexpr (CB || MASS)
                    x += ref.template phi_t<U>(q, r) * sg;
                K[kk] = x;
            }
        }
        if (wf) {
            U fv[3] = {U(0), U(0), U(0)};
            if constexpr (DG) {
#pragma unroll
                for (int k = 0; k < 3; ++k)
                    fv[k] = Jv[k][0] * c.d[0] + Jv[k][1] * c.d[1] + Jv[k][2] * c.d[2];
            }
            const U f0 = D0 ? (U)vol * c.d0 : U(0);
#pragma unroll
            for (int r = 0; r < 6; ++r) {
                if constexpr (DG) {
#pragma unroll
                    for (int k = 0; k < 3; ++k)
                        if (!prism_zero_derivative(r, k))
                            F[r] += ref.template dphi_t<U>(q, r, k) * fv[k];
                }
                if constexpr (D0)
                    F[r] += ref.template phi_t<U>(q, r) * f0;
            }
        }
    }

    // The points q0, q0 + qstep, ... of one element, summed into K and F.
    template <int NT, class R, class B2, int NK>
    __device__ __forceinline__ static void accumulate(const KArgs &a, const Streams &st, const R &ref,
                                                      int64_t e, const double (&X0)[3],
                                                      const double (&X)[18], int q0, int qstep,
                                                      T (&K)[NK], T (&F)[6], const B2 &bl)
    {
#pragma unroll
        for (int k = 0; k < NK; ++k)
            K[k] = T(0);
#pragma unroll
        for (int r = 0; r < 6; ++r)
            F[r] = T(0);
        Coefs c;
        if constexpr (!PER_QP)
            load_coefs<NT>(a, st, ref, 0, e, X0, X, c, bl);
        const bool wf = bl.with_f();
        const int nq = NQ > 0 ? NQ : a.n_q;
#pragma unroll(NQ > 0 ? NQ : 1)
        for (int q = q0; q < nq; q += qstep) {
            if constexpr (PER_QP)
                load_coefs<NT>(a, st, ref, q, e, X0, X, c, bl);
            if constexpr (REF_SPACE) {
                double Ji[3][3], det;
                point_jacobian<6>(X, ref, q, Ji, det);
                contract_ref<T>(c, ref, q, Ji, det * ref.w(q), K, F, wf);
                continue;
            }
            T g[6][3], vol;
            point_geometry<6, T>(X, ref, q, g, vol);
            T phi[6];
#pragma unroll
            for (int r = 0; r < 6; ++r)
                phi[r] = NEED_PHI ? (T)ref.phi(q, r) : T(0);
            contract(c, g, vol, phi, K, F, wf);
        }
    }

    // The three blocks (A, 0), (A, 1), (A, 2) of the 3-component problem in
    // one pass over the points: the Jacobian terms are formed once per point
    // for the three, and each block's sums are those of `accumulate` for it.
    template <int NT, class R>
    __device__ __forceinline__ static void accumulate_row3(const KArgs &a, const Streams &st,
                                                           const R &ref, int64_t e,
                                                           const double (&X0)[3],
                                                           const double (&X)[18], int A,
                                                           T (&K)[3][36], T (&F)[6])
    {
#pragma unroll
        for (int b = 0; b < 3; ++b)
#pragma unroll
            for (int k = 0; k < 36; ++k)
                K[b][k] = T(0);
#pragma unroll
        for (int r = 0; r < 6; ++r)
            F[r] = T(0);
        Coefs c[3];
        if constexpr (!PER_QP) {
#pragma unroll
            for (int b = 0; b < 3; ++b)
                load_coefs<NT>(a, st, ref, 0, e, X0, X, c[b], VecBlock{A, b});
        }
        const int nq = NQ > 0 ? NQ : a.n_q;
#pragma unroll(NQ > 0 ? NQ : 1)
        for (int q = 0; q < nq; ++q) {
            if constexpr (PER_QP) {
#pragma unroll
                for (int b = 0; b < 3; ++b)
                    load_coefs<NT>(a, st, ref, q, e, X0, X, c[b], VecBlock{A, b});
            }
            if constexpr (REF_SPACE) {
                // each block's sums are exactly those `accumulate` forms
                double Ji[3][3], det;
                point_jacobian<6>(X, ref, q, Ji, det);
#pragma unroll
                for (int b = 0; b < 3; ++b)
                    contract_ref<T>(c[b], ref, q, Ji, det * ref.w(q), K[b], F, b == 0);
                continue;
            }
            T g[6][3], vol;
            point_geometry<6, T>(X, ref, q, g, vol);
            T phi[6];
#pragma unroll
            for (int r = 0; r < 6; ++r)
                phi[r] = NEED_PHI ? (T)ref.phi(q, r) : T(0);
#pragma unroll
            for (int b = 0; b < 3; ++b)
                contract(c[b], g, vol, phi, K[b], F, b == 0);
        }
    }

    // G lanes per element (the wavefront-level mapping of the point loop):
    // lane j of the element's group forms the Jacobian terms and the K, F
    // contributions of points j, j + G, ...; the partial sums are then added
    // across the group in lane order (shuffles through the cross-lane
    // network), and lane j stores the entries with index = j mod G.
    // `lead` is the group's first lane in the wavefront; `valid` is false for
    // lanes past the end of the batch, which still join the shuffles.
    template <int G, int NT, int REF>
    __device__ __forceinline__ static void run_lanes(const KArgs &a, const Streams &st,
                                                     const Ref<REF> &ref, int64_t e, int j, int lead,
                                                     bool valid)
    {
        double Xg[1][18];
        st.template load_coords<6, 1, NT>(e, Xg);
        double X[18];
#pragma unroll
        for (int s = 0; s < 18; ++s)
            X[s] = Xg[0][s];
        const double X0[3] = {X[0], X[1], X[2]};
        to_edge_vectors<6>(X);
        static_assert(PACKED != 2, "lane-split kernels store packed or full accumulations");
        constexpr int NK = PACKED ? 21 : 36;
        T K[NK], F[6];
        accumulate<NT>(a, st, ref, e, X0, X, j, G, K, F, ScalarBlock());
        T *outK = static_cast<T *>(st.out_K);
        T *outF = static_cast<T *>(st.out_F);
#pragma unroll
        for (int k = 0; k < NK; ++k) {
            T sum = __shfl(K[k], lead);
#pragma unroll
            for (int i = 1; i < G; ++i)
                sum += __shfl(K[k], lead + i);
            if (valid && k % G == j)
                st1<NT>(outK + k * st.ld_out + e, sum);
        }
#pragma unroll
        for (int r = 0; r < 6; ++r) {
            T sum = __shfl(F[r], lead);
#pragma unroll
            for (int i = 1; i < G; ++i)
                sum += __shfl(F[r], lead + i);
            if (valid && r % G == j)
                st1<NT>(outF + r * st.ld_out + e, sum);
        }
    }
};

// ================================================= prism, 3-component CDR
// Block by block as for tetrahedra: the (alpha, beta) block runs the scalar
// point loop with the block's coefficients, so a lane holds one 6x6 block of
// accumulators (FP64) or one row of three blocks (FP32) at a time instead of
// the whole 18x18 matrix; the per-point Jacobian terms are recomputed for
// each pass.
template <typename T, int MODE, int NQ>
struct PrismVector {
    // each block's coefficients are read after earlier blocks are stored
    static constexpr bool INTERLEAVED_IO = true;
    template <int V, int NT, int REF, class S>
    __device__ __forceinline__ static void run(const KArgs &a, const S &st, const Ref<REF> &ref,
                                               int64_t e)
    {
        static_assert(V == 1, "prisms are processed one element per lane");
        double Xg[1][18];
        st.template load_coords<6, 1, NT>(e, Xg);
        double X[18];
#pragma unroll
        for (int s = 0; s < 18; ++s)
            X[s] = Xg[0][s];
        const double X0[3] = {X[0], X[1], X[2]};
        to_edge_vectors<6>(X);
        typedef PrismScalar<T, TS_FULL, MODE, 0, NQ, VecBlock> PS;
        if constexpr (sizeof(T) == 4) {
            // FP32 tier: a row of three blocks per pass over the points, so
            // the FP64 Jacobian terms are formed three times instead of nine
            // (the three blocks' FP32 sums fit the registers)
#pragma unroll 1
            for (int A = 0; A < 3; ++A) {
                T K[3][36], F[6];
                PS::template accumulate_row3<NT>(a, st, ref, e, X0, X, A, K, F);
#pragma unroll
                for (int b = 0; b < 3; ++b) {
                    const VecBlock bl{A, b};
#pragma unroll
                    for (int r = 0; r < 6; ++r)
#pragma unroll
                        for (int s2 = 0; s2 < 6; ++s2) {
                            const T v[1] = {K[b][6 * r + s2]};
                            bl.template put_k<1, NT>(st, 6, 0, r, s2, e, v);
                        }
                }
                const VecBlock b0{A, 0};
#pragma unroll
                for (int r = 0; r < 6; ++r) {
                    const T v[1] = {F[r]};
                    b0.template put_f<1, NT>(st, r, e, v);
                }
            }
        } else {
            // FP64: one block per pass (three blocks' FP64 sums would not
            // fit the registers)
#pragma unroll 1
            for (int b = 0; b < 9; ++b)
                PS::template body<NT>(a, st, ref, e, X0, X, VecBlock{b / 3, b % 3});
        }
    }

    // Matrix-free and assembly consumers: the nine blocks handed to bl.
    template <int NT, int REF, class B2>
    __device__ __forceinline__ static void apply_x(const KArgs &a, const Streams &st, const Ref<REF> &ref,
                                                   const double (&Xa)[18], int64_t e, const B2 &bl)
    {
        double X[18];
#pragma unroll
        for (int s = 0; s < 18; ++s)
            X[s] = Xa[s];
        const double X0[3] = {X[0], X[1], X[2]};
        to_edge_vectors<6>(X);
#pragma unroll 1
        for (int b = 0; b < 9; ++b) {
            VecConsumer<B2> vb;
            vb.A = b / 3;
            vb.B = b % 3;
            vb.in = &bl;
            PrismScalar<T, TS_FULL, MODE, 0, NQ, VecBlock>::template body<NT>(a, st, ref, e, X0, X, vb);
        }
    }
};

// ====================================== prism, scalar, SQS and SSQ orders
// The other loop orders of Sec. 3.3 for geo_generic elements: SQS
// (Algorithm 4) loops over the rows of K outermost and recomputes the
// Jacobian terms at every point for every row; SSQ (Algorithm 6) loops over
// the entries of K outermost and recomputes them for every entry (with only
// the two global derivatives that entry needs). They hold fewer values at a
// time (one row; one entry) at the price of repeated geometry, and exist to
// compare the orders on gfx950 as the paper's experiments compare them on its
// processors; QSS (PrismScalar) remains the production kernel.
enum LoopOrder { ORDER_QSS = 1, ORDER_SQS = 2, ORDER_SSQ = 3 };

// Jacobian terms at one point: (J^{-1})[k][i] and det J, from edge vectors.
template <class R>
__device__ __forceinline__ void point_jinv(const double (&E)[18], const R &ref, int q,
                                           double (&Ji)[3][3], double &det)
{
    double J[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            double s = 0.0;
#pragma unroll
            for (int r = 1; r < 6; ++r)
                s += E[3 * r + i] * ref.dphi(q, r, k);
            J[i][k] = s;
        }
    const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
    const double inv = 1.0 / det;
    Ji[0][0] = c00 * inv;
    Ji[1][0] = c01 * inv;
    Ji[2][0] = c02 * inv;
    Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) * inv;
    Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) * inv;
    Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) * inv;
    Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) * inv;
    Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) * inv;
    Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) * inv;
}

// Global derivatives of shape function r (r may be a runtime index).
template <typename T, class R>
__device__ __forceinline__ void grad_of(const R &ref, int q, int r, const double (&Ji)[3][3],
                                        T (&g)[3])
{
    const double d0 = ref.dphi(q, r, 0), d1 = ref.dphi(q, r, 1), d2 = ref.dphi(q, r, 2);
#pragma unroll
    for (int i = 0; i < 3; ++i)
        g[i] = (T)(d0 * Ji[0][i] + d1 * Ji[1][i] + d2 * Ji[2][i]);
}

template <typename T, int TERMS, int MODE, int PACKED, int ORDER>
struct PrismScalarOrder {
    using Q = PrismScalar<T, TERMS, MODE, PACKED, 0>;
    static constexpr bool DIFF = Q::DIFF, CA = Q::CA, CB = Q::CB, MASS = Q::MASS, DG = Q::DG,
                          D0 = Q::D0, PER_QP = Q::PER_QP;

    // vol [g_r . C g_s + (c^{.;0} . g_r) phi_s + phi_r (c^{0;.} . g_s) + c^{0;0} phi_r phi_s]
    __device__ __forceinline__ static T entry(const typename Q::Coefs &c, const T (&gr)[3],
                                              const T (&gs)[3], T pr, T ps)
    {
        T x = T(0);
        if constexpr (DIFF) {
#pragma unroll
            for (int i = 0; i < 3; ++i)
                x += gr[i] * (c.C[i][0] * gs[0] + c.C[i][1] * gs[1] + c.C[i][2] * gs[2]);
        }
        if constexpr (CA)
            x += (c.ca[0] * gr[0] + c.ca[1] * gr[1] + c.ca[2] * gr[2]) * ps;
        if constexpr (CB)
            x += pr * (c.cb[0] * gs[0] + c.cb[1] * gs[1] + c.cb[2] * gs[2]);
        if constexpr (MASS)
            x += c.c00 * pr * ps;
        return x;
    }

    __device__ __forceinline__ static T load_entry(const typename Q::Coefs &c, const T (&gr)[3],
                                                   T pr)
    {
        T x = T(0);
        if constexpr (DG)
            x = c.d[0] * gr[0] + c.d[1] * gr[1] + c.d[2] * gr[2];
        if constexpr (D0)
            x += c.d0 * pr;
        return x;
    }

    template <int V, int NT, int REF, class S>
    __device__ __forceinline__ static void run(const KArgs &a, const S &st, const Ref<REF> &ref,
                                               int64_t e)
    {
        static_assert(V == 1, "prisms are processed one element per lane");
        double Xg[1][18];
        st.template load_coords<6, 1, NT>(e, Xg);
        double X[18];
#pragma unroll
        for (int s = 0; s < 18; ++s)
            X[s] = Xg[0][s];
        const double X0[3] = {X[0], X[1], X[2]};
        to_edge_vectors<6>(X);
        typename Q::Coefs c;
        if constexpr (!PER_QP)
            Q::template load_coefs<NT>(a, st, ref, 0, e, X0, X, c);
        T *outK = static_cast<T *>(st.out_K);
        T *outF = static_cast<T *>(st.out_F);
        const int nq = a.n_q;
        if constexpr (ORDER == ORDER_SQS) {
#pragma unroll 1
            for (int r = 0; r < 6; ++r) {
                T Kr[6], Fr = T(0);
#pragma unroll
                for (int s = 0; s < 6; ++s)
                    Kr[s] = T(0);
                for (int q = 0; q < nq; ++q) {
                    if constexpr (PER_QP)
                        Q::template load_coefs<NT>(a, st, ref, q, e, X0, X, c);
                    double Ji[3][3], det;
                    point_jinv(X, ref, q, Ji, det);
                    const T vol = (T)(det * ref.w(q));
                    T gr[3];
                    grad_of<T>(ref, q, r, Ji, gr);
                    const T pr = (T)ref.phi(q, r);
#pragma unroll
                    for (int s = 0; s < 6; ++s) {
                        T gs[3];
                        grad_of<T>(ref, q, s, Ji, gs);
                        Kr[s] += vol * entry(c, gr, gs, pr, (T)ref.phi(q, s));
                    }
                    Fr += vol * load_entry(c, gr, pr);
                }
#pragma unroll
                for (int s = 0; s < 6; ++s) {
                    if (PACKED && s < r)
                        continue;
                    const int k = PACKED ? r * 6 - r * (r - 1) / 2 + (s - r) : 6 * r + s;
                    st1<NT>(outK + k * st.ld_out + e, Kr[s]);
                }
                st1<NT>(outF + r * st.ld_out + e, Fr);
            }
        } else {
#pragma unroll 1
            for (int r = 0; r < 6; ++r) {
#pragma unroll 1
                for (int s = PACKED ? r : 0; s < 6; ++s) {
                    T acc = T(0), fr = T(0);
                    for (int q = 0; q < nq; ++q) {
                        if constexpr (PER_QP)
                            Q::template load_coefs<NT>(a, st, ref, q, e, X0, X, c);
                        double Ji[3][3], det;
                        point_jinv(X, ref, q, Ji, det);
                        const T vol = (T)(det * ref.w(q));
                        T gr[3], gs[3];
                        grad_of<T>(ref, q, r, Ji, gr);
                        grad_of<T>(ref, q, s, Ji, gs);
                        const T pr = (T)ref.phi(q, r);
                        acc += vol * entry(c, gr, gs, pr, (T)ref.phi(q, s));
                        if (r == s)
                            fr += vol * load_entry(c, gr, pr);
                    }
                    const int k = PACKED ? r * 6 - r * (r - 1) / 2 + (s - r) : 6 * r + s;
                    st1<NT>(outK + k * st.ld_out + e, acc);
                    if (r == s)
                        st1<NT>(outF + r * st.ld_out + e, fr);
                }
            }
        }
    }
};

// ====================================================== prism, elasticity
// Coefficients constant over the element: H_rs = sum_q vol_q g_r g_s^T
// (r <= s), then K_(r a),(s b) = lam H_rs[a][b] + mu H_rs[b][a]
// + mu delta_ab tr H_rs, and F_(r a) = f_a sum_q vol_q phi_r(xi_q).
// Coefficients per point: the same expression accumulated point by point
// with lambda_q, mu_q (and f_q), directly into the packed K.
//
// SPLIT = 2 or 3 processes the rows of K in passes over the points (shape
// functions {0,1},{2..5} or {0},{1,2},{3..5} as test functions), recomputing
// the Jacobian terms in every pass: the SQS idea of Algorithm 4 used only to
// bound the live FP64 accumulators (93 or 75 instead of 171) so that more
// waves fit on a SIMD.
template <typename T, int MODE, int PACKED, int NQ, int SPLIT = 1>
struct PrismElastic {
    static constexpr uint32_t SL = 31u;
    static constexpr bool PER_QP = (MODE == M_QP || MODE == M_QP_MIXED || MODE == M_FUNC);
    static constexpr int NP = 171;  // packed entries of the 18 x 18 matrix

    template <int V, int NT>
    __device__ __forceinline__ static void store_block(const Streams &st, int64_t e, int k0,
                                                       int k1, const T *Kp)
    {
        T *outK = static_cast<T *>(st.out_K);
        if constexpr (PACKED) {
#pragma unroll
            for (int k = k0; k < k1; ++k)
                st1<NT>(outK + k * st.ld_out + e, Kp[k - k0]);
        } else {
#pragma unroll
            for (int row = 0; row < 18; ++row)
#pragma unroll
                for (int col = row; col < 18; ++col) {
                    const int k = pidx(18, row, col);
                    if (k < k0 || k >= k1)
                        continue;
                    st1<NT>(outK + (18 * row + col) * st.ld_out + e, Kp[k - k0]);
                    if (col != row)
                        st1<NT>(outK + (18 * col + row) * st.ld_out + e, Kp[k - k0]);
                }
        }
    }

    // Shape functions R0..R1-1 as test functions (rows 3*R0 .. 3*R1-1 of K):
    // accumulate H over the points, transform to K, store (B2 = void) or
    // hand the entries and F to the consumer bl.
    template <int R0, int R1, bool WITH_F, int NT, int REF, class B2 = void>
    __device__ __forceinline__ static void const_pass(const KArgs &a, const Streams &st,
                                                      const Ref<REF> &ref, const double (&X)[18],
                                                      int64_t e, T lam, T mu, const T (&f)[3],
                                                      const B2 *bl = nullptr)
    {
        constexpr int K0 = pidx(18, 3 * R0, 3 * R0);
        constexpr int K1 = R1 == 6 ? NP : pidx(18, 3 * R1, 3 * R1);
        T Kp[K1 - K0];
#pragma unroll
        for (int k = 0; k < K1 - K0; ++k)
            Kp[k] = T(0);
        T sphi[6];
#pragma unroll
        for (int r = 0; r < 6; ++r)
            sphi[r] = T(0);
        const int nq = NQ > 0 ? NQ : a.n_q;
#pragma unroll(NQ > 0 ? NQ : 1)
        for (int q = 0; q < nq; ++q) {
            T g[6][3], vol;
            point_geometry<6, T>(X, ref, q, g, vol);
            if constexpr (WITH_F) {
#pragma unroll
                for (int r = 0; r < 6; ++r)
                    sphi[r] += vol * (T)ref.phi(q, r);
            }
#pragma unroll
            for (int r = R0; r < R1; ++r) {
                const T u[3] = {vol * g[r][0], vol * g[r][1], vol * g[r][2]};
#pragma unroll
                for (int s = r; s < 6; ++s)
#pragma unroll
                    for (int al = 0; al < 3; ++al)
#pragma unroll
                        for (int be = (s == r ? al : 0); be < 3; ++be)
                            Kp[pidx(18, 3 * r + al, 3 * s + be) - K0] += u[al] * g[s][be];
            }
        }
        // H -> K block by block, in place
#pragma unroll
        for (int r = R0; r < R1; ++r)
#pragma unroll
            for (int s = r; s < 6; ++s) {
                T H[3][3];
#pragma unroll
                for (int al = 0; al < 3; ++al)
#pragma unroll
                    for (int be = 0; be < 3; ++be) {
                        if (s == r && be < al)
                            H[al][be] = Kp[pidx(18, 3 * r + be, 3 * s + al) - K0];
                        else
                            H[al][be] = Kp[pidx(18, 3 * r + al, 3 * s + be) - K0];
                    }
                const T tr = mu * (H[0][0] + H[1][1] + H[2][2]);
#pragma unroll
                for (int al = 0; al < 3; ++al)
#pragma unroll
                    for (int be = (s == r ? al : 0); be < 3; ++be) {
                        T x = lam * H[al][be] + mu * H[be][al];
                        if (al == be)
                            x += tr;
                        Kp[pidx(18, 3 * r + al, 3 * s + be) - K0] = x;
                    }
            }
        if constexpr (std::is_void<B2>::value) {
            store_block<1, NT>(st, e, K0, K1, Kp);
            if constexpr (WITH_F) {
                T *outF = static_cast<T *>(st.out_F);
#pragma unroll
                for (int r = 0; r < 6; ++r)
#pragma unroll
                    for (int al = 0; al < 3; ++al)
                        st1<NT>(outF + (3 * r + al) * st.ld_out + e, f[al] * sphi[r]);
            }
        } else {
            // packed entries (upper triangle) to the consumer, which adds
            // the mirrored entry itself
#pragma unroll
            for (int r = R0; r < R1; ++r)
#pragma unroll
                for (int s = r; s < 6; ++s)
#pragma unroll
                    for (int al = 0; al < 3; ++al)
#pragma unroll
                        for (int be = (s == r ? al : 0); be < 3; ++be) {
                            const T v[1] = {Kp[pidx(18, 3 * r + al, 3 * s + be) - K0]};
                            bl->template put_k<1, NT>(st, 18, 1, 3 * r + al, 3 * s + be, e, v);
                        }
            if constexpr (WITH_F) {
#pragma unroll
                for (int r = 0; r < 6; ++r)
#pragma unroll
                    for (int al = 0; al < 3; ++al) {
                        const T v[1] = {f[al] * sphi[r]};
                        bl->template put_f<1, NT>(st, 3 * r + al, e, v);
                    }
            }
        }
    }

    // Per-point coefficients, rows 3*R0 .. 3*R1-1 of K (and F when WITH_F)
    // for a consumer: lambda_q, mu_q and f_q at every point.
    template <int R0, int R1, bool WITH_F, int NT, int REF, class B2>
    __device__ __forceinline__ static void qp_pass(const KArgs &a, const Streams &st,
                                                   const Ref<REF> &ref, const double (&X)[18],
                                                   int64_t e, const B2 &bl)
    {
        constexpr int K0 = pidx(18, 3 * R0, 3 * R0);
        constexpr int K1 = R1 == 6 ? NP : pidx(18, 3 * R1, 3 * R1);
        T Kp[K1 - K0], F[18];
#pragma unroll
        for (int k = 0; k < K1 - K0; ++k)
            Kp[k] = T(0);
#pragma unroll
        for (int k = 0; k < 18; ++k)
            F[k] = T(0);
        const int nq = NQ > 0 ? NQ : a.n_q;
#pragma unroll(NQ > 0 ? NQ : 1)
        for (int q = 0; q < nq; ++q) {
            T E[1], nu[1], f[3][1];
            coef<T, MODE, SL, 1, NT>(a, st, 0, q, e, E);
            coef<T, MODE, SL, 1, NT>(a, st, 1, q, e, nu);
            if constexpr (WITH_F) {
#pragma unroll
                for (int al = 0; al < 3; ++al)
                    coef<T, MODE, SL, 1, NT>(a, st, 2 + al, q, e, f[al]);
            }
            T lam, mu;
            lame<T>(E[0], nu[0], lam, mu);
            T g[6][3], vol;
            point_geometry<6, T>(X, ref, q, g, vol);
            const T vl = vol * lam, vm = vol * mu;
            if constexpr (WITH_F) {
#pragma unroll
                for (int r = 0; r < 6; ++r) {
                    const T pq = vol * (T)ref.phi(q, r);
#pragma unroll
                    for (int al = 0; al < 3; ++al)
                        F[3 * r + al] += pq * f[al][0];
                }
            }
#pragma unroll
            for (int r = R0; r < R1; ++r)
#pragma unroll
                for (int s = r; s < 6; ++s) {
                    const T dot = vm * (g[r][0] * g[s][0] + g[r][1] * g[s][1] + g[r][2] * g[s][2]);
#pragma unroll
                    for (int al = 0; al < 3; ++al)
#pragma unroll
                        for (int be = (s == r ? al : 0); be < 3; ++be) {
                            T x = vl * g[r][al] * g[s][be] + vm * g[r][be] * g[s][al];
                            if (al == be)
                                x += dot;
                            Kp[pidx(18, 3 * r + al, 3 * s + be) - K0] += x;
                        }
                }
        }
#pragma unroll
        for (int r = R0; r < R1; ++r)
#pragma unroll
            for (int s = r; s < 6; ++s)
#pragma unroll
                for (int al = 0; al < 3; ++al)
#pragma unroll
                    for (int be = (s == r ? al : 0); be < 3; ++be) {
                        const T v[1] = {Kp[pidx(18, 3 * r + al, 3 * s + be) - K0]};
                        bl.template put_k<1, NT>(st, 18, 1, 3 * r + al, 3 * s + be, e, v);
                    }
        if constexpr (WITH_F) {
#pragma unroll
            for (int k = 0; k < 18; ++k) {
                const T v[1] = {F[k]};
                bl.template put_f<1, NT>(st, k, e, v);
            }
        }
    }

    // Matrix-free and assembly consumers: absolute vertex coordinates in, K
    // and F handed to bl one row block per pass over the points (six passes:
    // at most 51 live accumulators next to the consumer's own arrays).
    template <int NT, int REF, class B2>
    __device__ __forceinline__ static void apply_x(const KArgs &a, const Streams &st, const Ref<REF> &ref,
                                                   const double (&Xa)[18], int64_t e, const B2 &bl)
    {
        double X[18];
#pragma unroll
        for (int s = 0; s < 18; ++s)
            X[s] = Xa[s];
        to_edge_vectors<6>(X);
        if constexpr (PER_QP) {
            qp_pass<0, 1, true, NT, REF, B2>(a, st, ref, X, e, bl);
            qp_pass<1, 2, false, NT, REF, B2>(a, st, ref, X, e, bl);
            qp_pass<2, 3, false, NT, REF, B2>(a, st, ref, X, e, bl);
            qp_pass<3, 4, false, NT, REF, B2>(a, st, ref, X, e, bl);
            qp_pass<4, 5, false, NT, REF, B2>(a, st, ref, X, e, bl);
            qp_pass<5, 6, false, NT, REF, B2>(a, st, ref, X, e, bl);
        } else {
            T E[1], nu[1], fc[3][1];
            coef<T, MODE, SL, 1, NT>(a, st, 0, 0, e, E);
            coef<T, MODE, SL, 1, NT>(a, st, 1, 0, e, nu);
#pragma unroll
            for (int al = 0; al < 3; ++al)
                coef<T, MODE, SL, 1, NT>(a, st, 2 + al, 0, e, fc[al]);
            T lam, mu;
            lame<T>(E[0], nu[0], lam, mu);
            const T fv[3] = {fc[0][0], fc[1][0], fc[2][0]};
            const_pass<0, 1, true, NT, REF, B2>(a, st, ref, X, e, lam, mu, fv, &bl);
            const_pass<1, 2, false, NT, REF, B2>(a, st, ref, X, e, lam, mu, fv, &bl);
            const_pass<2, 3, false, NT, REF, B2>(a, st, ref, X, e, lam, mu, fv, &bl);
            const_pass<3, 4, false, NT, REF, B2>(a, st, ref, X, e, lam, mu, fv, &bl);
            const_pass<4, 5, false, NT, REF, B2>(a, st, ref, X, e, lam, mu, fv, &bl);
            const_pass<5, 6, false, NT, REF, B2>(a, st, ref, X, e, lam, mu, fv, &bl);
        }
    }

    template <int V, int NT, int REF, class S>
    __device__ __forceinline__ static void run(const KArgs &a, const S &st, const Ref<REF> &ref,
                                               int64_t e)
    {
        static_assert(V == 1, "prisms are processed one element per lane");
        double Xg[1][18];
        st.template load_coords<6, 1, NT>(e, Xg);
        double X[18];
#pragma unroll
        for (int s = 0; s < 18; ++s)
            X[s] = Xg[0][s];
        to_edge_vectors<6>(X);
        if constexpr (!PER_QP) {
            T E[1], nu[1], f[3][1];
            coef<T, MODE, SL, 1, NT>(a, st, 0, 0, e, E);
            coef<T, MODE, SL, 1, NT>(a, st, 1, 0, e, nu);
#pragma unroll
            for (int al = 0; al < 3; ++al)
                coef<T, MODE, SL, 1, NT>(a, st, 2 + al, 0, e, f[al]);
            T lam, mu;
            lame<T>(E[0], nu[0], lam, mu);
            const T fv[3] = {f[0][0], f[1][0], f[2][0]};
            if constexpr (SPLIT == 3) {
                const_pass<0, 1, true, NT, REF>(a, st, ref, X, e, lam, mu, fv);
                const_pass<1, 3, false, NT, REF>(a, st, ref, X, e, lam, mu, fv);
                const_pass<3, 6, false, NT, REF>(a, st, ref, X, e, lam, mu, fv);
            } else if constexpr (SPLIT == 2) {
                const_pass<0, 2, true, NT, REF>(a, st, ref, X, e, lam, mu, fv);
                const_pass<2, 6, false, NT, REF>(a, st, ref, X, e, lam, mu, fv);
            } else {
                const_pass<0, 6, true, NT, REF>(a, st, ref, X, e, lam, mu, fv);
            }
            return;
        } else {
            T Kp[NP], F[18];
#pragma unroll
            for (int k = 0; k < NP; ++k)
                Kp[k] = T(0);
#pragma unroll
            for (int k = 0; k < 18; ++k)
                F[k] = T(0);
            const int nq = NQ > 0 ? NQ : a.n_q;
#pragma unroll(NQ > 0 ? NQ : 1)
            for (int q = 0; q < nq; ++q) {
                T E[1], nu[1], f[3][1];
                coef<T, MODE, SL, 1, NT>(a, st, 0, q, e, E);
                coef<T, MODE, SL, 1, NT>(a, st, 1, q, e, nu);
#pragma unroll
                for (int al = 0; al < 3; ++al)
                    coef<T, MODE, SL, 1, NT>(a, st, 2 + al, q, e, f[al]);
                T lam, mu;
                lame<T>(E[0], nu[0], lam, mu);
                T g[6][3], vol;
                point_geometry<6, T>(X, ref, q, g, vol);
                const T vl = vol * lam, vm = vol * mu;
#pragma unroll
                for (int r = 0; r < 6; ++r) {
                    const T p = vol * (T)ref.phi(q, r);
#pragma unroll
                    for (int al = 0; al < 3; ++al)
                        F[3 * r + al] += p * f[al][0];
#pragma unroll
                    for (int s = r; s < 6; ++s) {
                        const T dot = vm * (g[r][0] * g[s][0] + g[r][1] * g[s][1] + g[r][2] * g[s][2]);
#pragma unroll
                        for (int al = 0; al < 3; ++al)
#pragma unroll
                            for (int be = (s == r ? al : 0); be < 3; ++be) {
                                T x = vl * g[r][al] * g[s][be] + vm * g[r][be] * g[s][al];
                                if (al == be)
                                    x += dot;
                                Kp[pidx(18, 3 * r + al, 3 * s + be)] += x;
                            }
                    }
                }
            }
            store_block<1, NT>(st, e, 0, NP, Kp);
            T *outF = static_cast<T *>(st.out_F);
#pragma unroll
            for (int k = 0; k < 18; ++k)
                st1<NT>(outF + k * st.ld_out + e, F[k]);
        }
    }
};

// ================================================================ kernel
// Grid: element groups of V contiguous elements, one group per lane, with a
// grid-stride loop so a launch may use fewer workgroups than groups. The
// last, partial group is processed element by element.
template <class P, int V, int NT, int REF>
__global__ __launch_bounds__(256) void fe_kernel(KArgs a)
{
    __shared__ RefLds lds_ref[1];
    if constexpr (REF == REF_LDS) {
        const int n_w = a.n_q, n_phi = a.n_q * 6, n_dphi = a.n_q * 18;
        for (int i = threadIdx.x; i < n_w; i += blockDim.x)
            lds_ref[0].w[i] = a.w[i];
        for (int i = threadIdx.x; i < n_phi; i += blockDim.x)
            (&lds_ref[0].phi[0][0])[i] = (&a.phi[0][0])[i];
        for (int i = threadIdx.x; i < n_dphi; i += blockDim.x)
            (&lds_ref[0].dphi[0][0][0])[i] = (&a.dphi[0][0][0])[i];
        __syncthreads();
    }
    const Ref<REF> ref{a, &lds_ref[0]};
    const Streams st{a.coords, a.coeffs, a.out_K, a.out_F, a.ld_in, a.ld_out};
    const int64_t n_groups = (a.n_elem + V - 1) / V;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n_groups; g += stride) {
        const int64_t e0 = g * V;
        if (V == 1 || e0 + V <= a.n_elem) {
            P::template run<V, NT, REF>(a, st, ref, e0);
        } else {
            for (int64_t e = e0; e < a.n_elem; ++e)
                P::template run<1, NT, REF>(a, st, ref, e);
        }
    }
}

// Persistent batched form: the blocks of one launch walk the chunks of one
// kind in the device table (chunk c by block c mod gridDim), so requests of
// different sizes share one launch. Chunk starts are multiples of V, so every
// element is processed by the same code path as in a plain launch. A chunk
// whose rows or pointers do not suit V-wide accesses carries a negative
// element count and is processed element by element (the code path of a
// plain launch's last partial group, which rounds identically).
template <class P, int V, int NT, int REF>
__global__ __launch_bounds__(256) void fe_batch_kernel(KArgs a, const BatchHeader *__restrict__ hdr,
                                                       const Chunk *__restrict__ chunks, int kind)
{
    __shared__ RefLds lds_ref[1];
    if constexpr (REF == REF_LDS) {
        const int n_w = a.n_q, n_phi = a.n_q * 6, n_dphi = a.n_q * 18;
        for (int i = threadIdx.x; i < n_w; i += blockDim.x)
            lds_ref[0].w[i] = a.w[i];
        for (int i = threadIdx.x; i < n_phi; i += blockDim.x)
            (&lds_ref[0].phi[0][0])[i] = (&a.phi[0][0])[i];
        for (int i = threadIdx.x; i < n_dphi; i += blockDim.x)
            (&lds_ref[0].dphi[0][0][0])[i] = (&a.dphi[0][0][0])[i];
        __syncthreads();
    }
    const Ref<REF> ref{a, &lds_ref[0]};
    // Work is handed out per tile (one element group per lane) across all
    // chunks of this kind, so a batch of few chunks still fills the grid.
    // a.n_elem holds the batch's chunk size, the element count of every
    // chunk but a request's last.
    const int begin = hdr->begin[kind], end = hdr->end[kind];
    const int64_t tile = (int64_t)blockDim.x * V;
    const int64_t tiles_per_chunk = (a.n_elem + tile - 1) / tile;
    const int64_t n_tiles = (int64_t)(end - begin) * tiles_per_chunk;
    for (int64_t t = blockIdx.x; t < n_tiles; t += gridDim.x) {
        const Chunk ch = chunks[begin + (int)(t / tiles_per_chunk)];
        const bool by_elem = ch.n < 0;
        const int64_t e0 = ch.e0 + (t % tiles_per_chunk) * tile + (int64_t)threadIdx.x * V;
        const int64_t last = ch.e0 + (by_elem ? -ch.n : ch.n);
        if (e0 >= last)
            continue;
        const Streams st{ch.coords, ch.coeffs, ch.out_K, ch.out_F, ch.ld_in, ch.ld_out};
        if (V == 1 || (!by_elem && e0 + V <= last)) {
            P::template run<V, NT, REF>(a, st, ref, e0);
        } else {
            const int64_t stop = e0 + V < last ? e0 + V : last;
            for (int64_t e = e0; e < stop; ++e)
                P::template run<1, NT, REF>(a, st, ref, e);
        }
    }
}

template <class P, int V, int NT, int REF>
hipError_t launch_fe_batch_kernel(const KArgs &a, const BatchHeader *hdr, const Chunk *chunks, int kind,
                            unsigned grid, unsigned block, hipStream_t stream)
{
    return launch_kernel(&fe_batch_kernel<P, V, NT, REF>, dim3(grid), dim3(block), 0, stream, a, hdr,
                       chunks, kind);
}

// Indexed-geometry form of fe_kernel.
template <class P, int V, int NT, int REF>
__global__ __launch_bounds__(256) void fe_kernel_idx(KArgs a, IdxArgs gi)
{
    __shared__ RefLds lds_ref[1];
    if constexpr (REF == REF_LDS) {
        const int n_w = a.n_q, n_phi = a.n_q * 6, n_dphi = a.n_q * 18;
        for (int i = threadIdx.x; i < n_w; i += blockDim.x)
            lds_ref[0].w[i] = a.w[i];
        for (int i = threadIdx.x; i < n_phi; i += blockDim.x)
            (&lds_ref[0].phi[0][0])[i] = (&a.phi[0][0])[i];
        for (int i = threadIdx.x; i < n_dphi; i += blockDim.x)
            (&lds_ref[0].dphi[0][0][0])[i] = (&a.dphi[0][0][0])[i];
        __syncthreads();
    }
    const Ref<REF> ref{a, &lds_ref[0]};
    StreamsIdx st;
    st.coords = nullptr;
    st.coeffs = a.coeffs;
    st.out_K = a.out_K;
    st.out_F = a.out_F;
    st.ld_in = a.ld_in;
    st.ld_out = a.ld_out;
    st.nodes = gi.nodes;
    st.conn = gi.conn;
    st.ld_conn = gi.ld_conn;
    st.n_nodes = gi.n_nodes;
    const int64_t n_groups = (a.n_elem + V - 1) / V;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; g < n_groups; g += stride) {
        const int64_t e0 = g * V;
        if (V == 1 || e0 + V <= a.n_elem) {
            P::template run<V, NT, REF>(a, st, ref, e0);
        } else {
            for (int64_t e = e0; e < a.n_elem; ++e)
                P::template run<1, NT, REF>(a, st, ref, e);
        }
    }
}

// Vertex ids (clamped into the node array: never a fault) and coordinates
// of element e.
template <int NV, int NT>
__device__ __forceinline__ void gather_vertices(const IdxArgs &gi, int64_t e, uint32_t (&id)[NV],
                                                double (&X)[3 * NV])
{
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        const uint32_t u = (uint32_t)ld1<NT>(gi.conn + v * gi.ld_conn + e);
        id[v] = u < gi.n_nodes ? u : gi.n_nodes - 1;
        const double *pn = gi.nodes + 3 * (int64_t)id[v];
        X[3 * v + 0] = pn[0];
        X[3 * v + 1] = pn[1];
        X[3 * v + 2] = pn[2];
    }
}

template <int REF>
__device__ __forceinline__ void stage_reference(const KArgs &a, RefLds &lds)
{
    if constexpr (REF == REF_LDS) {
        const int n_w = a.n_q, n_phi = a.n_q * 6, n_dphi = a.n_q * 18;
        for (int i = threadIdx.x; i < n_w; i += blockDim.x)
            lds.w[i] = a.w[i];
        for (int i = threadIdx.x; i < n_phi; i += blockDim.x)
            (&lds.phi[0][0])[i] = (&a.phi[0][0])[i];
        for (int i = threadIdx.x; i < n_dphi; i += blockDim.x)
            (&lds.dphi[0][0][0])[i] = (&a.dphi[0][0][0])[i];
        __syncthreads();
    }
}

// Matrix-free application of the assembled operator (indexed geometry, one
// element per lane): gather the vertex ids, coordinates and nodal values x,
// compute the element's K (and F) exactly as the storing kernels do but
// consume them in registers (ApplyBlock), then add the element's K x (and F)
// to y (and b) at its nodes. ATOMIC: hardware atomic adds, any element
// order; otherwise plain read-add-write, for launches over one colour of
// elements that share no node.
template <class P, int NV, int NC, typename T, int NT, int REF, bool ATOMIC, bool WITH_B>
__global__ __launch_bounds__(256) void fe_apply_kernel(KArgs a, IdxArgs gi, ApplyArgs ap)
{
    __shared__ RefLds lds_ref[1];
    stage_reference<REF>(a, lds_ref[0]);
    const Ref<REF> ref{a, &lds_ref[0]};
    const Streams st{nullptr, a.coeffs, nullptr, nullptr, a.ld_in, a.ld_out};
    const T *x = static_cast<const T *>(ap.x);
    T *y = static_cast<T *>(ap.y);
    T *b = static_cast<T *>(ap.b);
    constexpr int N = NV * NC;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = xcd_block(blockIdx.x, gridDim.x) * blockDim.x + threadIdx.x; e < a.n_elem;
         e += stride) {
        uint32_t id[NV];
        double X[3 * NV];
        gather_vertices<NV, NT>(gi, e, id, X);
        T xe[N], ye[N], be[N];
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                xe[NC * v + c] = x[(int64_t)NC * id[v] + c];
                ye[NC * v + c] = T(0);
                be[NC * v + c] = T(0);
            }
        ApplyBlock<T, WITH_B> bl;
        bl.x = xe;
        bl.y = ye;
        bl.b = be;
        P::template apply_x<NT, REF>(a, st, ref, X, e, bl);
#pragma unroll
        for (int v = 0; v < NV; ++v)
#pragma unroll
            for (int c = 0; c < NC; ++c) {
                add_at<T, ATOMIC>(y + (int64_t)NC * id[v] + c, ye[NC * v + c]);
                if constexpr (WITH_B)
                    add_at<T, ATOMIC>(b + (int64_t)NC * id[v] + c, be[NC * v + c]);
            }
    }
}

// Assembly into a CSR matrix (indexed geometry, one element per lane):
// gather the element as the matrix-free kernel does, find where its
// couplings sit in the rows of its nodes (one pass over each row's
// columns), then compute K (and F) and add every entry there (CsrBlock).
// ATOMIC as for the matrix-free kernel.
template <class P, int NV, int NC, typename T, int NT, int REF, bool ATOMIC, bool WITH_B>
__global__ __launch_bounds__(256) void fe_csr_kernel(KArgs a, IdxArgs gi, ApplyArgs ap)
{
    __shared__ RefLds lds_ref[1];
    stage_reference<REF>(a, lds_ref[0]);
    const Ref<REF> ref{a, &lds_ref[0]};
    const Streams st{nullptr, a.coeffs, nullptr, nullptr, a.ld_in, a.ld_out};
    const int64_t nnz = ap.nnz;
    constexpr int N = NV * NC;
    constexpr bool DEFER = !ATOMIC && N * N <= 36;
    constexpr int SB = 16;  // columns loaded together in the row scans
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < a.n_elem; e += stride) {
        CsrBlock<T, NV, NC, ATOMIC, WITH_B, DEFER> bl;
        T kv[DEFER ? N * N : 1], fv[DEFER ? N : 1];
#pragma unroll
        for (int k = 0; k < (DEFER ? N * N : 1); ++k)
            kv[k] = T(0);
#pragma unroll
        for (int k = 0; k < (DEFER ? N : 1); ++k)
            fv[k] = T(0);
        bl.vals = static_cast<T *>(ap.vals);
        bl.b = static_cast<T *>(ap.b);
        bl.kv = kv;
        bl.fv = fv;
        bl.nnz = nnz;
        double X[3 * NV];
        gather_vertices<NV, NT>(gi, e, bl.id, X);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            // row bounds clamped into [0, nnz]: never a fault
            const int64_t row = (int64_t)NC * bl.id[v];
            int64_t r0 = ap.row_ptr[row], r1 = ap.row_ptr[row + 1];
            r0 = r0 < 0 ? 0 : (r0 > nnz ? nnz : r0);
            r1 = r1 < r0 ? r0 : (r1 > nnz ? nnz : r1);
            bl.rp[v] = r0;
            bl.len[v] = (int32_t)(r1 - r0);
#pragma unroll
            for (int u = 0; u < NV; ++u)
                bl.off[v][u] = -1;
            for (int64_t j0 = r0; j0 < r1; j0 += SB * NC) {
                int32_t c[SB];
#pragma unroll
                for (int t = 0; t < SB; ++t) {
                    const int64_t j = j0 + (int64_t)t * NC;
                    c[t] = j < r1 ? ap.col_idx[j] : -1;
                }
#pragma unroll
                for (int t = 0; t < SB; ++t)
#pragma unroll
                    for (int u = 0; u < NV; ++u)
                        if (c[t] == (int32_t)(NC * bl.id[u]))
                            bl.off[v][u] = (int32_t)(j0 - r0) + t * NC;
            }
        }
        P::template apply_x<NT, REF>(a, st, ref, X, e, bl);
        if constexpr (DEFER)
            bl.flush();
    }
}

// Assembly into a CSR matrix by row ownership (one node per lane, no
// colours and no atomics): node i's lane loads the node columns of its
// rows (the first RC in registers), then for each element at the node
// gathers it, finds where the element's nodes sit in the row, computes K
// and F keeping only the node's rows (RowBlock) and adds them; every
// element is computed once per vertex. Each row is written by one lane
// only, so the result does not depend on the schedule. For scalar tets
// (REG_ROW) the first RC entries of the row stay in registers from the
// first element to the last, starting from their stored values, and are
// written once: each element adds its K value or -0 to every held entry
// (x + (-0) is x for every x), the same additions in the same order as a
// read-add-write. Entries beyond the first RC, and the rows of prisms
// (whose element arithmetic already fills the registers), are added
// through memory.
template <class P, int NV, int NC, typename T, int NT, int REF, bool WITH_B>
__global__ __launch_bounds__(256) void fe_csr_rows_kernel(KArgs a, IdxArgs gi, ApplyArgs ap)
{
    __shared__ RefLds lds_ref[1];
    stage_reference<REF>(a, lds_ref[0]);
    const Ref<REF> ref{a, &lds_ref[0]};
    const Streams st{nullptr, a.coeffs, nullptr, nullptr, a.ld_in, a.ld_out};
    constexpr int N = NV * NC;
    constexpr int RC = 32;  // node columns of a row held in registers
    constexpr bool REG_ROW = NC == 1 && NV == 4;
    const int64_t nnz = ap.nnz;
    T *vals = static_cast<T *>(ap.vals);
    T *b = static_cast<T *>(ap.b);
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    // scalar tets: workgroup b takes the nodes of logical workgroup
    // xcd_block(b) (one contiguous range of nodes per XCD, see xcd_block)
    const int64_t blk = REG_ROW ? xcd_block(blockIdx.x, gridDim.x) : (int64_t)blockIdx.x;
    for (int64_t i = blk * blockDim.x + threadIdx.x; i < ap.n_own; i += stride) {
        // row bounds clamped into [0, nnz]: never a fault
        int64_t r0 = ap.row_ptr[NC * i], r1 = ap.row_ptr[NC * i + 1];
        r0 = r0 < 0 ? 0 : (r0 > nnz ? nnz : r0);
        r1 = r1 < r0 ? r0 : (r1 > nnz ? nnz : r1);
        const int64_t len = r1 - r0;
        int32_t cols[RC];
        T acc[REG_ROW ? RC : 1];
#pragma unroll
        for (int k = 0; k < RC; ++k)
            cols[k] = (int64_t)k * NC < len ? ap.col_idx[r0 + (int64_t)k * NC] : -1;
        if constexpr (REG_ROW) {
#pragma unroll
            for (int k = 0; k < RC; ++k)
                acc[k] = k < len ? vals[r0 + k] : T(0);
        }
        T fb[NC];
#pragma unroll
        for (int al = 0; al < NC; ++al)
            fb[al] = T(0);
        const int64_t k0 = ap.inc_ptr[i], k1 = ap.inc_ptr[i + 1];
        // software pipeline over the node's elements: the code of element
        // k + 2 and the vertex ids of element k + 1 are loaded while
        // element k is processed
        auto code_at = [&](int64_t k) -> uint32_t {
            return k < k1 ? (uint32_t)ap.inc[k] : 0u;
        };
        auto ids_of = [&](uint32_t code, uint32_t (&id)[NV]) {
            const int64_t e = code / NV < a.n_elem ? code / NV : 0;
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const uint32_t u = (uint32_t)ld1<NT>(gi.conn + v * gi.ld_conn + e);
                id[v] = u < gi.n_nodes ? u : gi.n_nodes - 1;  // clamped: never a fault
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
            const uint32_t c_after = code_at(k + 2);
            if (k + 1 < k1)
                ids_of(c_next, id_cur);
            c_cur = c_next;
            c_next = c_after;
            const int64_t e = code / NV;
            if (e >= a.n_elem)
                continue;
            RowBlock<T, NV, NC> bl;
            bl.lv = (int)(code % NV);
            T kr[NC * N], fr[NC];
#pragma unroll
            for (int j = 0; j < NC * N; ++j)
                kr[j] = T(0);
#pragma unroll
            for (int al = 0; al < NC; ++al)
                fr[al] = T(0);
            bl.kr = kr;
            bl.fr = fr;
            double X[3 * NV];
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const double *pn = gi.nodes + 3 * (int64_t)id[v];
                X[3 * v + 0] = pn[0];
                X[3 * v + 1] = pn[1];
                X[3 * v + 2] = pn[2];
            }
            if constexpr (REG_ROW) {
                P::template apply_x<NT, REF>(a, st, ref, X, e, bl);
                // held entries in chunks of 8; a chunk no lane of the wave
                // has entries in (its columns are all -1) is skipped by the
                // whole wave
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
                                add = kr[u];
                        acc[c] += add;
                        // keeps each column's compares beside their selects
                        __builtin_amdgcn_sched_barrier(0);
                    }
                }
                for (int64_t j = RC; j < len; ++j) {
                    const int32_t c = ap.col_idx[r0 + j];
#pragma unroll
                    for (int u = 0; u < NV; ++u)
                        if (c == (int32_t)id[u])
                            vals[r0 + j] = vals[r0 + j] + kr[u];
                }
            } else {
                // offset of each element node's first column in the row, or -1
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
                    const int32_t c = ap.col_idx[r0 + j];
#pragma unroll
                    for (int u = 0; u < NV; ++u)
                        if (c == (int32_t)(NC * id[u]))
                            slot[u] = (int32_t)j;
                }
                if constexpr (NC == 1) {
                    // the row's current values are loaded before the element
                    // is computed, so the loads overlap the arithmetic
                    int64_t p[N];
                    T old[N];
#pragma unroll
                    for (int s = 0; s < N; ++s) {
                        const int64_t q = r0 + slot[s];
                        p[s] = (slot[s] >= 0 && q < nnz) ? q : -1;
                        old[s] = p[s] >= 0 ? vals[p[s]] : T(0);
                    }
                    P::template apply_x<NT, REF>(a, st, ref, X, e, bl);
#pragma unroll
                    for (int s = 0; s < N; ++s)
                        if (p[s] >= 0)
                            vals[p[s]] = old[s] + kr[s];
                } else {
                    P::template apply_x<NT, REF>(a, st, ref, X, e, bl);
                    // row by row: the row's loads, then its stores
#pragma unroll
                    for (int al = 0; al < NC; ++al) {
                        int64_t p[N];
                        T old[N];
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
                                vals[p[s]] = old[s] + kr[al * N + s];
                    }
                }
            }
#pragma unroll
            for (int al = 0; al < NC; ++al)
                fb[al] += fr[al];
        }
        if constexpr (REG_ROW) {
            // written back where a column is held (cols[c] is -1 for c >=
            // len; a negative column matches no node, so its entry is
            // unchanged)
#pragma unroll
            for (int c = 0; c < RC; ++c)
                if (cols[c] >= 0)
                    vals[r0 + c] = acc[c];
        }
        if constexpr (WITH_B) {
#pragma unroll
            for (int al = 0; al < NC; ++al)
                b[NC * i + al] += fb[al];
        }
    }
}

// Row ownership over node blocks (scalar tetrahedra): one workgroup per
// block of consecutive nodes. The block's elements (block-local vertex
// indices and, where coefficients are read per element, global ids) and
// their vertices' coordinates are read from HBM into LDS once; then each
// lane walks its node's incidence list in the order fe_csr_rows_kernel
// walks it, computes the element's row for the node (RowBlock) and adds its
// four values where the host-built incidence codes place them: the first RL
// entries of the node's row accumulate in LDS (starting from their stored
// values, written back once), entries past them through memory. Every
// entry receives the same additions in the same order as in
// fe_csr_rows_kernel, so the values are the same bit for bit; and no lane
// compares columns, which is most of that kernel's arithmetic.
// Incidence code: bits 0-13 element slot * 4 + local vertex; bits 14-19,
// 20-25, 26-31 the row positions of the element's other three vertices in
// increasing local order (62: no such entry in the pattern; 63: position
// past 61, found by its column).
template <class P, typename T, int NT, int REF, bool WITH_B>
__global__ __launch_bounds__(FE_CSR_BLOCK_NODES) void fe_csr_blocks_kernel(KArgs a, IdxArgs gi,
                                                                          ApplyArgs ap)
{
    constexpr int NV = 4;
    constexpr int BN = FE_CSR_BLOCK_NODES, BV = FE_CSR_BLOCK_VERTS, BE = FE_CSR_BLOCK_ELEMS;
    constexpr int RL = 16;  // row entries per node accumulated in LDS
    constexpr bool EID = P::ELEM_COEFS;
    __shared__ RefLds lds_ref[1];
    __shared__ double lx[BV], ly[BV], lz[BV];
    __shared__ uint16_t lcn[BE * NV];
    __shared__ int32_t lel[EID ? BE : 1];
    __shared__ T lrow[RL * BN];  // entry c of lane t's row at [c * BN + t]
    stage_reference<REF>(a, lds_ref[0]);
    const Ref<REF> ref{a, &lds_ref[0]};
    const Streams st{nullptr, a.coeffs, nullptr, nullptr, a.ld_in, a.ld_out};
    const int64_t nnz = ap.nnz;
    T *vals = static_cast<T *>(ap.vals);
    T *b = static_cast<T *>(ap.b);
    // workgroup b takes block xcd_block(b): one contiguous range of blocks
    // per XCD
    const int64_t *bp = ap.blk + 3 * xcd_block(blockIdx.x, gridDim.x);
    const int64_t n0 = bp[0], n1 = bp[3], es = bp[1], ve = bp[2];
    // counts clamped to the LDS arrays: never a fault
    const int64_t ne = bp[4] - es, nvx = bp[5] - ve;
    const int32_t n_el = (int32_t)(ne < 0 ? 0 : (ne > BE ? BE : ne));
    const int32_t n_ve = (int32_t)(nvx < 0 ? 0 : (nvx > BV ? BV : nvx));
    for (int j = threadIdx.x; j < n_ve; j += blockDim.x) {
        uint32_t g = (uint32_t)ap.blk_verts[ve + j];
        g = g < gi.n_nodes ? g : gi.n_nodes - 1;
        const double *pn = gi.nodes + 3 * (int64_t)g;
        lx[j] = pn[0];
        ly[j] = pn[1];
        lz[j] = pn[2];
    }
    for (int j = threadIdx.x; j < n_el * NV; j += blockDim.x) {
        const uint16_t l = ap.blk_conn[es * NV + j];
        lcn[j] = l < n_ve ? l : 0;
    }
    if constexpr (EID) {
        for (int j = threadIdx.x; j < n_el; j += blockDim.x)
            lel[j] = ap.blk_elems[es + j];
    }
    const int t = threadIdx.x;
    const int64_t i = n0 + t;
    const bool own = t < BN && i >= 0 && i < n1 && i < ap.n_own;
    int64_t r0 = 0, len = 0;
    int pos_self = 62;
    if (own) {
        // row bounds clamped into [0, nnz]: never a fault
        r0 = ap.row_ptr[i];
        int64_t r1 = ap.row_ptr[i + 1];
        r0 = r0 < 0 ? 0 : (r0 > nnz ? nnz : r0);
        r1 = r1 < r0 ? r0 : (r1 > nnz ? nnz : r1);
        len = r1 - r0;
        for (int64_t j = 0; j < len; ++j)
            if (ap.col_idx[r0 + j] == (int32_t)i) {
                pos_self = j < 62 ? (int)j : 63;
                break;
            }
#pragma unroll
        for (int c = 0; c < RL; ++c)
            lrow[c * BN + t] = c < len ? vals[r0 + c] : T(0);
    }
    __syncthreads();
    if (!own)
        return;
    T fb = T(0);
    const int64_t k0 = ap.inc_ptr[i], k1 = ap.inc_ptr[i + 1];
    auto code_at = [&](int64_t k) -> uint32_t { return k < k1 ? ap.linc[k] : 0u; };
    // adds x to the row entry at position p (62: none; 63: found by the
    // column of block vertex l)
    auto add_at = [&](int p, uint32_t l, T x) {
        if (p < RL) {
            lrow[p * BN + t] += x;
        } else if (p < 62) {
            if (p < len)
                vals[r0 + p] = vals[r0 + p] + x;
        } else if (p == 63) {
            const int32_t g = ap.blk_verts[ve + l];
            for (int64_t j = 0; j < len; ++j)
                if (ap.col_idx[r0 + j] == g)
                    vals[r0 + j] = vals[r0 + j] + x;
        }
    };
    uint32_t c_next = code_at(k0);
    for (int64_t k = k0; k < k1; ++k) {
        const uint32_t code = c_next;
        c_next = code_at(k + 1);
        const uint32_t sl = (code & 0x3fffu) / NV;
        if (sl >= (uint32_t)n_el)
            continue;
        int64_t e = 0;
        if constexpr (EID) {
            e = lel[sl];
            if (e < 0 || e >= a.n_elem)
                continue;
        }
        const int lv = (int)(code & 3u);
        uint32_t lid[NV];
        double X[3 * NV];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            lid[v] = lcn[sl * NV + v];
            X[3 * v + 0] = lx[lid[v]];
            X[3 * v + 1] = ly[lid[v]];
            X[3 * v + 2] = lz[lid[v]];
        }
        RowBlock<T, NV, 1> bl;
        bl.lv = lv;
        T kr[NV], fr[1];
#pragma unroll
        for (int j = 0; j < NV; ++j)
            kr[j] = T(0);
        fr[0] = T(0);
        bl.kr = kr;
        bl.fr = fr;
        P::template apply_x<NT, REF>(a, st, ref, X, e, bl);
        // positions of the element's vertices in the row: the node's own
        // for lv, the code's fields for the others in increasing order
        const int f0 = (int)((code >> 14) & 63u), f1 = (int)((code >> 20) & 63u),
                  f2 = (int)((code >> 26) & 63u);
#pragma unroll
        for (int u = 0; u < NV; ++u) {
            const int p = u == lv ? pos_self : (u < lv ? (u == 0 ? f0 : (u == 1 ? f1 : f2))
                                                       : (u == 1 ? f0 : (u == 2 ? f1 : f2)));
            add_at(p, lid[u], kr[u]);
        }
        fb += fr[0];
    }
#pragma unroll
    for (int c = 0; c < RL; ++c)
        if (c < len)
            vals[r0 + c] = lrow[c * BN + t];
    if constexpr (WITH_B)
        b[i] += fb;
}

template <class P, int NV, int NC, typename T, int NT, int REF>
hipError_t launch_fe_apply(const KArgs &a, const IdxArgs &gi, const ApplyArgs &ap, int atomic,
                     unsigned grid, unsigned block, hipStream_t stream)
{
    if (ap.vals && ap.blk) {
        if constexpr (NV == 4 && NC == 1) {
            if (block != FE_CSR_BLOCK_NODES)
                return hipErrorInvalidValue;
            if (ap.b)
                return launch_kernel(&fe_csr_blocks_kernel<P, T, NT, REF, true>, dim3(grid),
                                     dim3(block), 0, stream, a, gi, ap);
            else
                return launch_kernel(&fe_csr_blocks_kernel<P, T, NT, REF, false>, dim3(grid),
                                     dim3(block), 0, stream, a, gi, ap);
        }
        return hipErrorInvalidValue;
    }
    if (ap.vals && ap.inc) {
        if (ap.b)
            return launch_kernel(&fe_csr_rows_kernel<P, NV, NC, T, NT, REF, true>, dim3(grid),
                               dim3(block), 0, stream, a, gi, ap);
        else
            return launch_kernel(&fe_csr_rows_kernel<P, NV, NC, T, NT, REF, false>, dim3(grid),
                               dim3(block), 0, stream, a, gi, ap);
    }
    if (ap.vals) {
        if (atomic && ap.b)
            return launch_kernel(&fe_csr_kernel<P, NV, NC, T, NT, REF, true, true>, dim3(grid),
                               dim3(block), 0, stream, a, gi, ap);
        else if (atomic)
            return launch_kernel(&fe_csr_kernel<P, NV, NC, T, NT, REF, true, false>, dim3(grid),
                               dim3(block), 0, stream, a, gi, ap);
        else if (ap.b)
            return launch_kernel(&fe_csr_kernel<P, NV, NC, T, NT, REF, false, true>, dim3(grid),
                               dim3(block), 0, stream, a, gi, ap);
        else
            return launch_kernel(&fe_csr_kernel<P, NV, NC, T, NT, REF, false, false>, dim3(grid),
                               dim3(block), 0, stream, a, gi, ap);
    }
    if (atomic && ap.b)
        return launch_kernel(&fe_apply_kernel<P, NV, NC, T, NT, REF, true, true>, dim3(grid), dim3(block),
                           0, stream, a, gi, ap);
    else if (atomic)
        return launch_kernel(&fe_apply_kernel<P, NV, NC, T, NT, REF, true, false>, dim3(grid),
                           dim3(block), 0, stream, a, gi, ap);
    else if (ap.b)
        return launch_kernel(&fe_apply_kernel<P, NV, NC, T, NT, REF, false, true>, dim3(grid),
                           dim3(block), 0, stream, a, gi, ap);
    else
        return launch_kernel(&fe_apply_kernel<P, NV, NC, T, NT, REF, false, false>, dim3(grid),
                           dim3(block), 0, stream, a, gi, ap);
}

// G lanes per element: each wavefront takes 64 / G consecutive elements
// (lanes past G * (64 / G) idle); the loop bound is uniform over the
// wavefront, so every lane reaches every cross-lane exchange.
template <class P, int G, int NT, int REF>
__global__ __launch_bounds__(256) void fe_kernel_lanes(KArgs a)
{
    __shared__ RefLds lds_ref[1];
    if constexpr (REF == REF_LDS) {
        const int n_w = a.n_q, n_phi = a.n_q * 6, n_dphi = a.n_q * 18;
        for (int i = threadIdx.x; i < n_w; i += blockDim.x)
            lds_ref[0].w[i] = a.w[i];
        for (int i = threadIdx.x; i < n_phi; i += blockDim.x)
            (&lds_ref[0].phi[0][0])[i] = (&a.phi[0][0])[i];
        for (int i = threadIdx.x; i < n_dphi; i += blockDim.x)
            (&lds_ref[0].dphi[0][0][0])[i] = (&a.dphi[0][0][0])[i];
        __syncthreads();
    }
    const Ref<REF> ref{a, &lds_ref[0]};
    const Streams st{a.coords, a.coeffs, a.out_K, a.out_F, a.ld_in, a.ld_out};
    constexpr int PER_WAVE = 64 / G;
    const int lane = threadIdx.x & 63;
    const int slot = lane / G, j = lane % G;
    const int lead = (slot < PER_WAVE ? slot : PER_WAVE - 1) * G;
    const int64_t waves = (int64_t)gridDim.x * (blockDim.x / 64);
    const int64_t wave = (int64_t)blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
    for (int64_t base = wave * PER_WAVE; base < a.n_elem; base += waves * PER_WAVE) {
        const int64_t e = base + (slot < PER_WAVE ? slot : PER_WAVE - 1);
        const bool valid = slot < PER_WAVE && e < a.n_elem;
        // lanes without an element of their own work on the batch's last
        // element (in bounds) and store nothing
        P::template run_lanes<G, NT, REF>(a, st, ref, valid ? e : a.n_elem - 1,
                                          slot < PER_WAVE ? j : 0, lead, valid);
    }
}

template <class P, int G, int NT, int REF>
hipError_t launch_fe_kernel_lanes(const KArgs &a, unsigned grid, unsigned block, hipStream_t stream)
{
    return launch_kernel(&fe_kernel_lanes<P, G, NT, REF>, dim3(grid), dim3(block), 0, stream, a);
}

// Natural-order inputs and outputs (the element-contiguous organisation
// of Sec. 4.2 and its Fig. 1): a workgroup of one wavefront takes a tile of
// AOS_TILE consecutive elements, copies the tile's contiguous input block to
// LDS with coalesced loads, transposed to rows (row-major by value, element
// fastest), runs the unchanged per-element code on that LDS tile (the
// stream pointers are LDS addresses, the leading dimension AOS_TILE), and
// writes the tile's K and F back as contiguous element-major blocks with
// coalesced stores. LDS tile: inputs [3 NV rows FP64 | coef rows], and the
// outputs [K rows | F rows] over the same bytes: the problem classes read
// every input of an element before they write its first output, and the
// one wavefront executes its instructions in order, so no lane's output
// overwrites an input another lane has still to read (except those marked
// INTERLEAVED_IO below, whose outputs get bytes of their own).
__device__ __forceinline__ uint32_t div_magic(uint32_t i, uint32_t magic) { return __umulhi(i, magic); }

// Problem classes whose block loop reads the next block's coefficients
// after storing earlier blocks (INTERLEAVED_IO) break that order; for them
// the outputs follow the inputs in LDS instead of sharing their bytes.
template <class P, class = void>
struct aos_separate : std::false_type {};
template <class P>
struct aos_separate<P, std::void_t<decltype(P::INTERLEAVED_IO)>>
    : std::integral_constant<bool, P::INTERLEAVED_IO> {};

template <class P, int NV, int NT, int REF>
__global__ __launch_bounds__(64) void fe_kernel_aos(KArgs a, AosArgs ao)
{
    extern __shared__ __align__(16) unsigned char lds_raw[];
    __shared__ RefLds lds_ref[1];
    if constexpr (REF == REF_LDS) {
        const int n_w = a.n_q, n_phi = a.n_q * 6, n_dphi = a.n_q * 18;
        for (int i = threadIdx.x; i < n_w; i += blockDim.x)
            lds_ref[0].w[i] = a.w[i];
        for (int i = threadIdx.x; i < n_phi; i += blockDim.x)
            (&lds_ref[0].phi[0][0])[i] = (&a.phi[0][0])[i];
        for (int i = threadIdx.x; i < n_dphi; i += blockDim.x)
            (&lds_ref[0].dphi[0][0][0])[i] = (&a.dphi[0][0][0])[i];
        __syncthreads();
    }
    const Ref<REF> ref{a, &lds_ref[0]};
    constexpr int NC3 = 3 * NV;
    double *l_x = reinterpret_cast<double *>(lds_raw);
    unsigned char *l_c = lds_raw + sizeof(double) * NC3 * AOS_TILE;
    unsigned char *l_k =
        aos_separate<P>::value ? l_c + (size_t)ao.tsize * ao.coef_rows * AOS_TILE : lds_raw;
    unsigned char *l_f = l_k + (size_t)ao.tsize * ao.k_rows * AOS_TILE;
    const Streams st{l_x, l_c, l_k, l_f, AOS_TILE, AOS_TILE};
    const int lane = threadIdx.x;
    for (int64_t t0 = (int64_t)blockIdx.x * AOS_TILE; t0 < a.n_elem; t0 += (int64_t)gridDim.x * AOS_TILE) {
        const int n = (int)(a.n_elem - t0 < AOS_TILE ? a.n_elem - t0 : AOS_TILE);
        // tile inputs: element-major in memory, row-major in LDS
        const double *gx = a.coords + t0 * NC3;
        for (int i = lane; i < n * NC3; i += AOS_TILE)
            l_x[(i % NC3) * AOS_TILE + i / NC3] = ld1<NT>(gx + i);
        const int cr = ao.coef_rows;
        if (ao.tsize == 8) {
            const double *gc = static_cast<const double *>(a.coeffs) + t0 * cr;
            double *lc = reinterpret_cast<double *>(l_c);
            for (int i = lane; i < n * cr; i += AOS_TILE) {
                const int q = (int)div_magic((uint32_t)i, ao.coef_magic);
                lc[(i - q * cr) * AOS_TILE + q] = ld1<NT>(gc + i);
            }
        } else {
            const float *gc = static_cast<const float *>(a.coeffs) + t0 * cr;
            float *lc = reinterpret_cast<float *>(l_c);
            for (int i = lane; i < n * cr; i += AOS_TILE) {
                const int q = (int)div_magic((uint32_t)i, ao.coef_magic);
                lc[(i - q * cr) * AOS_TILE + q] = ld1<NT>(gc + i);
            }
        }
        __syncthreads();
        if (lane < n)
            P::template run<1, 0, REF>(a, st, ref, (int64_t)lane);
        __syncthreads();
        // tile outputs: row-major in LDS, element-major in memory
        const int kr = ao.k_rows, fr = ao.f_rows;
        if (ao.tsize == 8) {
            double *gk = static_cast<double *>(a.out_K) + t0 * kr;
            double *gf = static_cast<double *>(a.out_F) + t0 * fr;
            const double *lk = reinterpret_cast<const double *>(l_k);
            const double *lf = reinterpret_cast<const double *>(l_f);
            for (int i = lane; i < n * kr; i += AOS_TILE) {
                const int q = (int)div_magic((uint32_t)i, ao.k_magic);
                st1<NT>(gk + i, lk[(i - q * kr) * AOS_TILE + q]);
            }
            for (int i = lane; i < n * fr; i += AOS_TILE) {
                const int q = (int)div_magic((uint32_t)i, ao.f_magic);
                st1<NT>(gf + i, lf[(i - q * fr) * AOS_TILE + q]);
            }
        } else {
            float *gk = static_cast<float *>(a.out_K) + t0 * kr;
            float *gf = static_cast<float *>(a.out_F) + t0 * fr;
            const float *lk = reinterpret_cast<const float *>(l_k);
            const float *lf = reinterpret_cast<const float *>(l_f);
            for (int i = lane; i < n * kr; i += AOS_TILE) {
                const int q = (int)div_magic((uint32_t)i, ao.k_magic);
                st1<NT>(gk + i, lk[(i - q * kr) * AOS_TILE + q]);
            }
            for (int i = lane; i < n * fr; i += AOS_TILE) {
                const int q = (int)div_magic((uint32_t)i, ao.f_magic);
                st1<NT>(gf + i, lf[(i - q * fr) * AOS_TILE + q]);
            }
        }
        __syncthreads();
    }
}

// Natural order without LDS: lane e's streams start at element e's records
// (coordinates, coefficients, K, F) with leading dimension 1, so the
// unchanged per-element code reads and writes them in place. Lanes touch
// addresses one record apart; the lines of a record are reused through the
// caches as the code walks it.
template <class P, int NV, int NT, int REF>
__global__ __launch_bounds__(256) void fe_kernel_aos_direct(KArgs a, AosArgs ao)
{
    __shared__ RefLds lds_ref[1];
    stage_reference<REF>(a, lds_ref[0]);
    const Ref<REF> ref{a, &lds_ref[0]};
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const unsigned char *cb = static_cast<const unsigned char *>(a.coeffs);
    unsigned char *kb = static_cast<unsigned char *>(a.out_K);
    unsigned char *fb = static_cast<unsigned char *>(a.out_F);
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < a.n_elem; e += stride) {
        const Streams st{a.coords + e * 3 * NV,
                         ao.coef_rows ? cb + e * ao.coef_rows * ao.tsize : a.coeffs,
                         kb + e * ao.k_rows * ao.tsize, fb + e * ao.f_rows * ao.tsize, 1, 1};
        P::template run<1, 0, REF>(a, st, ref, (int64_t)0);
    }
}

template <class P, int NV, int NT, int REF>
hipError_t launch_fe_kernel_aos(const KArgs &a, const AosArgs &ao, unsigned grid, size_t lds_bytes,
                          hipStream_t stream)
{
    if (ao.direct)
        return launch_kernel(&fe_kernel_aos_direct<P, NV, NT, REF>, dim3(grid), dim3(256), 0, stream,
                           a, ao);
    else
        return launch_kernel(&fe_kernel_aos<P, NV, NT, REF>, dim3(grid), dim3(AOS_TILE), lds_bytes,
                           stream, a, ao);
}

template <class P, int V, int NT, int REF>
hipError_t launch_fe_kernel_idx(const KArgs &a, const IdxArgs &gi, unsigned grid, unsigned block,
                          hipStream_t stream)
{
    return launch_kernel(&fe_kernel_idx<P, V, NT, REF>, dim3(grid), dim3(block), 0, stream, a, gi);
}

template <class P, int V, int NT, int REF>
hipError_t launch_fe_kernel(const KArgs &a, unsigned grid, unsigned block, hipStream_t stream)
{
    return launch_kernel(&fe_kernel<P, V, NT, REF>, dim3(grid), dim3(block), 0, stream, a);
}

}  // namespace fe
