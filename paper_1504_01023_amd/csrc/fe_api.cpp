// fe_api.cpp -- host side of the libfe C ABI: argument validation, reference
// tables built from the caller's quadrature rule, kernel selection and
// launch. Every per-element step runs in the HIP kernels; the host only
// evaluates the reference element's shape functions at the rule's points
// (an input of the integration procedure, Sec. 2.3) and picks a compiled
// kernel.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "fe.h"
#include "fe_api_internal.h"
#include "fe_internal.h"

namespace fe {

static std::vector<KernelEntry> &registry()
{
    static std::vector<KernelEntry> r;
    return r;
}

void register_kernel(const KernelEntry &e) { registry().push_back(e); }

static bool same_key(const KernelKey &a, const KernelKey &b)
{
    return a.elem == b.elem && a.kind == b.kind && a.prec == b.prec && a.terms == b.terms &&
           a.mode == b.mode && a.packed == b.packed && a.vec == b.vec && a.nt == b.nt &&
           a.ref == b.ref && a.nq == b.nq && a.split == b.split && a.order == b.order &&
           a.lanes == b.lanes;
}

const KernelEntry *find_kernel(const KernelKey &k)
{
    for (const KernelEntry &e : registry())
        if (same_key(e.key, k))
            return &e;
    return nullptr;
}

int kernel_count() { return (int)registry().size(); }
const KernelEntry *kernel_at(int i)
{
    return (i >= 0 && i < kernel_count()) ? &registry()[i] : nullptr;
}

static thread_local std::string g_last_error;

int fail(int status, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return status;
}

// ------------------------------------------------------------ reference data
// The library's own evaluation of the reference shape functions (the same
// reference elements as documented in fe.h).
static void ref_shape(int elem, const double *xi, double *phi, double (*dphi)[3])
{
    if (elem == FE_TET4) {
        phi[0] = 1.0 - xi[0] - xi[1] - xi[2];
        phi[1] = xi[0];
        phi[2] = xi[1];
        phi[3] = xi[2];
        for (int k = 0; k < 3; ++k) {
            dphi[0][k] = -1.0;
            for (int r = 1; r < 4; ++r)
                dphi[r][k] = (r - 1 == k) ? 1.0 : 0.0;
        }
    } else {
        const double t[3] = {1.0 - xi[0] - xi[1], xi[0], xi[1]};
        const double tx[3] = {-1.0, 1.0, 0.0}, ty[3] = {-1.0, 0.0, 1.0};
        const double b = 0.5 * (1.0 - xi[2]), u = 0.5 * (1.0 + xi[2]);
        for (int v = 0; v < 3; ++v) {
            phi[v] = t[v] * b;
            phi[v + 3] = t[v] * u;
            dphi[v][0] = tx[v] * b;
            dphi[v][1] = ty[v] * b;
            dphi[v][2] = -0.5 * t[v];
            dphi[v + 3][0] = tx[v] * u;
            dphi[v + 3][1] = ty[v] * u;
            dphi[v + 3][2] = 0.5 * t[v];
        }
    }
}

void fill_reference(int elem, const fe_quad_rule &rule, KArgs &a)
{
    const int ns = elem == FE_TET4 ? 4 : 6;
    std::memset(a.w, 0, sizeof(a.w));
    std::memset(a.phi, 0, sizeof(a.phi));
    std::memset(a.dphi, 0, sizeof(a.dphi));
    std::memset(a.phi_f, 0, sizeof(a.phi_f));
    std::memset(a.dphi_f, 0, sizeof(a.dphi_f));
    std::memset(a.m, 0, sizeof(a.m));
    std::memset(a.M, 0, sizeof(a.M));
    a.Wsum = 0.0;
    a.n_q = rule.n_q;
    for (int q = 0; q < rule.n_q; ++q) {
        double phi[6], dphi[6][3];
        ref_shape(elem, rule.xi + 3 * q, phi, dphi);
        a.w[q] = rule.w[q];
        a.Wsum += rule.w[q];
        for (int r = 0; r < ns; ++r) {
            a.phi[q][r] = phi[r];
            a.phi_f[q][r] = (float)phi[r];
            for (int k = 0; k < 3; ++k) {
                a.dphi[q][r][k] = dphi[r][k];
                a.dphi_f[q][r][k] = (float)dphi[r][k];
            }
            a.m[r] += rule.w[q] * phi[r];
            for (int s = 0; s < ns; ++s)
                a.M[r][s] += rule.w[q] * phi[r] * phi[s];
        }
    }
}

// ------------------------------------------------------------- validation
static int n_shape(int elem) { return elem == FE_TET4 ? 4 : 6; }
static int n_comp(int kind) { return kind == FE_SCALAR_CDR ? 1 : 3; }
// mask bits: slots (scalar, elasticity) or blocks of slots (3-component CDR)
static int n_slots(int kind) { return kind == FE_ELASTICITY ? 5 : 20; }
// 3-component CDR: coefficient rows of the blocks present in the mask
static int vector_rows(uint32_t mask)
{
    int n = 0;
    for (int k = 0; k < 20; ++k)
        if (mask >> k & 1u)
            n += k < 16 ? 9 : 3;
    return n;
}

static int check_problem(const fe_problem *p, int elem)
{
    if (!p)
        return fail(FE_ERR_INVALID_ARG, "problem is NULL");
    if (elem != FE_TET4 && elem != FE_PRISM6)
        return fail(FE_ERR_INVALID_ARG, "bad element type %d", elem);
    if (p->kind != FE_SCALAR_CDR && p->kind != FE_ELASTICITY && p->kind != FE_VECTOR_CDR)
        return fail(FE_ERR_INVALID_ARG, "bad problem kind %d", p->kind);
    if (p->precision != FE_FP64 && p->precision != FE_FP32_BULK)
        return fail(FE_ERR_INVALID_ARG, "bad precision %d", p->precision);
    if (p->coef_mode < FE_COEF_UNIFORM || p->coef_mode > FE_COEF_FUNCTION)
        return fail(FE_ERR_INVALID_ARG, "bad coefficient mode %d", p->coef_mode);
    if (p->coef_mode == FE_COEF_FUNCTION && p->kind != FE_SCALAR_CDR)
        return fail(FE_ERR_UNSUPPORTED, "coefficient functions are built for scalar problems");
    if (p->k_format != FE_K_FULL && p->k_format != FE_K_SYM_PACKED)
        return fail(FE_ERR_INVALID_ARG, "bad K format %d", p->k_format);
    if (p->reserved != 0)
        return fail(FE_ERR_INVALID_ARG, "reserved field must be 0");
    if (p->kind == FE_VECTOR_CDR) {
        if (p->coef_mode != FE_COEF_PER_ELEMENT && p->coef_mode != FE_COEF_PER_QP)
            return fail(FE_ERR_UNSUPPORTED,
                        "the 3-component problem takes coefficients per element or per point");
        if (p->k_format != FE_K_FULL)
            return fail(FE_ERR_UNSUPPORTED, "the 3-component problem stores K in full");
    }
    if (p->coef_mode != FE_COEF_UNIFORM && (p->coef_mask >> n_slots(p->kind)) != 0)
        return fail(FE_ERR_INVALID_ARG, "coef_mask has bits beyond slot %d", n_slots(p->kind) - 1);
    return FE_OK;
}

static uint32_t effective_mask(const fe_problem *p)
{
    return p->coef_mode == FE_COEF_UNIFORM ? 0u : p->coef_mask;
}

// Term groups a scalar problem needs: any slot read from memory or nonzero.
static int needed_terms(const fe_problem *p)
{
    const uint32_t mask = effective_mask(p);
    int t = 0;
    const int groups[6] = {T_DIFF, T_CONVA, T_CONVB, T_MASS, T_DGRAD, T_D0};
    for (int g : groups) {
        const uint32_t sl = slots_of_terms(g);
        bool need = (mask & sl) != 0;
        for (int k = 0; k < 20; ++k)
            if ((sl >> k & 1u) && p->uniform[k] != 0.0)
                need = true;
        if (need)
            t |= g;
    }
    return t;
}

static int check_symmetry(const fe_problem *p)
{
    if (p->k_format != FE_K_SYM_PACKED || p->kind != FE_SCALAR_CDR)
        return FE_OK;
    const uint32_t mask = effective_mask(p);
    const uint32_t conv = slots_of_terms(T_CONVA) | slots_of_terms(T_CONVB);
    if (mask & conv)
        return fail(FE_ERR_NOT_SYMMETRIC,
                    "packed K requested with convection coefficients read from memory");
    for (int i = 1; i <= 3; ++i) {
        if (p->uniform[4 * i] != p->uniform[i])
            return fail(FE_ERR_NOT_SYMMETRIC, "packed K requested with c^{%d;0} != c^{0;%d}", i, i);
        for (int j = i + 1; j <= 3; ++j)
            if (!(mask >> (4 * i + j) & 1u) && !(mask >> (4 * j + i) & 1u) &&
                p->uniform[4 * i + j] != p->uniform[4 * j + i])
                return fail(FE_ERR_NOT_SYMMETRIC, "packed K requested with non-symmetric c^{i;j}");
    }
    return FE_OK;
}

int check_rule(const fe_quad_rule *r)
{
    if (!r)
        return fail(FE_ERR_INVALID_ARG, "quad_rule is NULL");
    if (r->n_q < 1 || r->n_q > FE_MAX_QP)
        return fail(FE_ERR_UNSUPPORTED, "rule has %d points; 1..%d supported", r->n_q, FE_MAX_QP);
    if (!r->xi || !r->w)
        return fail(FE_ERR_INVALID_ARG, "rule points or weights are NULL");
    for (int q = 0; q < r->n_q; ++q) {
        if (!std::isfinite(r->w[q]))
            return fail(FE_ERR_INVALID_ARG, "rule weight %d is not finite", q);
        for (int k = 0; k < 3; ++k)
            if (!std::isfinite(r->xi[3 * q + k]))
                return fail(FE_ERR_INVALID_ARG, "rule point %d is not finite", q);
    }
    return FE_OK;
}

static bool aligned(const void *p, size_t a) { return ((uintptr_t)p % a) == 0; }

// K is symmetric whatever the per-element data: no convection term, and the
// diffusion tensor uniform and symmetric (the mass term is symmetric).
static bool symmetric_full(const fe_problem *p, int elem)
{
    if (elem != FE_PRISM6 || p->kind != FE_SCALAR_CDR || p->coef_mode == FE_COEF_FUNCTION)
        return false;
    if (needed_terms(p) & (T_CONVA | T_CONVB))
        return false;
    if (effective_mask(p) & slots_of_terms(T_DIFF))
        return false;
    for (int i = 0; i < 3; ++i)
        for (int j = i + 1; j < 3; ++j)
            if (p->uniform[4 * (i + 1) + 1 + j] != p->uniform[4 * (j + 1) + 1 + i])
                return false;
    return true;
}

// ---------------------------------------------------------------- planning
int plan(const fe_problem *problem, int elem, int64_t n_elem, const double *coords,
         const void *coeffs, int64_t ld_in, const fe_quad_rule *rule, void *out_K, void *out_F,
         int64_t ld_out, const fe_variant *variant, Plan &pl, int form, const int32_t *conn,
         int64_t ld_conn)
{
    int st = check_problem(problem, elem);
    if (st)
        return st;
    if (n_elem < 0)
        return fail(FE_ERR_INVALID_ARG, "n_elem is negative");
    if ((st = check_rule(rule)))
        return st;
    if ((st = check_symmetry(problem)))
        return st;
    const uint32_t mask = effective_mask(problem);
    if (form >= 1)
        coords = nullptr;  // indexed geometry: no per-element coordinates
    if (n_elem > 0) {
        // form 0: per-element coordinates; 1: indexed; 2: indexed, matrix-free
        // (no K, F); 3: as 2 over node blocks (block-local connectivity)
        const bool by_conn = form == 1 || form == 2;
        if ((form == 0 && !coords) || (by_conn && !conn) || (form < 2 && (!out_K || !out_F)))
            return fail(FE_ERR_INVALID_ARG, "NULL coordinates, connectivity or output pointer");
        if (by_conn && ld_conn < n_elem)
            return fail(FE_ERR_INVALID_ARG, "connectivity leading dimension smaller than n_elem");
        if (mask && !coeffs)
            return fail(FE_ERR_INVALID_ARG, "coeffs is NULL but coef_mask reads %u slots",
                        (unsigned)__builtin_popcount(mask));
        if (ld_in < n_elem || ld_out < n_elem)
            return fail(FE_ERR_INVALID_ARG, "leading dimension smaller than n_elem");
    }
    const size_t tsz = problem->precision == FE_FP64 ? 8 : 4;
    const bool fn = problem->coef_mode == FE_COEF_FUNCTION;
    const size_t csz = fn ? 8 : tsz;  // function parameters are FP64
    if (!aligned(coords, 8) || !aligned(out_K, tsz) || !aligned(out_F, tsz) ||
        (mask && !aligned(coeffs, csz)) || !aligned(conn, 4))
        return fail(FE_ERR_UNSUPPORTED, "pointers must be aligned to their element size");

    KernelKey k{};
    k.elem = elem;
    k.kind = problem->kind;
    k.prec = problem->precision;
    if (problem->kind == FE_ELASTICITY) {
        k.terms = TS_ELAST;
    } else if (problem->kind == FE_VECTOR_CDR) {
        k.terms = TS_FULL;
    } else {
        const int need = needed_terms(problem);
        k.terms = ((need & ~TS_POISSON) == 0) ? TS_POISSON : TS_FULL;
    }
    const bool per_qp = problem->coef_mode == FE_COEF_PER_QP;
    if (mask == 0)
        k.mode = M_UNIFORM;
    else if (fn)
        k.mode = M_FUNC;
    else if (mask == slots_of_terms(k.terms) || problem->kind == FE_VECTOR_CDR)
        k.mode = per_qp ? M_QP : M_ELEM;  // 3-component blocks are addressed through col[]
    else
        k.mode = per_qp ? M_QP_MIXED : M_ELEM_MIXED;
    k.packed = (problem->k_format == FE_K_SYM_PACKED) ? 1 : 0;
    if (k.packed == 0 && symmetric_full(problem, elem)) {
        // a symmetric prism problem asked for full K: accumulate the upper
        // triangle only, where such kernels are built
        KernelKey s = k;
        s.packed = 2;
        for (int i = 0; i < kernel_count(); ++i) {
            const KernelKey &x = kernel_at(i)->key;
            if (x.elem == s.elem && x.kind == s.kind && x.prec == s.prec && x.terms == s.terms &&
                x.mode == s.mode && x.packed == 2) {
                k.packed = 2;
                break;
            }
        }
    }

    // variant: forced, tuned, or default
    fe_variant v{};
    bool forced = variant != nullptr;
    if (forced) {
        v = *variant;
    } else if (tuning_lookup(k, rule->n_q, v) != FE_OK) {
        v = fe_variant{};
    }
    const int wg = v.wg_size ? v.wg_size : 256;
    if (wg != 64 && wg != 128 && wg != 256)
        return fail(FE_ERR_UNSUPPORTED, "workgroup size %d not supported (64, 128, 256)", wg);
    int vec = v.elems_per_thread ? v.elems_per_thread : (elem == FE_TET4 ? 2 : 1);
    // cache policy: variant 1 (or 0) streaming loads and stores, 2 default,
    // 3 streaming stores only -> kernel NT 1, 0, 2
    const int nt = v.nontemporal == 2 ? 0 : (v.nontemporal == 3 ? 2 : 1);
    const int ref = (v.ref_in_lds == 1) ? REF_LDS : REF_KARG;
    const int split = (v.row_split == 2 || v.row_split == 3) ? v.row_split : 1;
    const int order = (v.loop_order == 2 || v.loop_order == 3) ? v.loop_order : 1;
    const int lanes = (v.lanes == 2 || v.lanes == 3 || v.lanes == 6) ? v.lanes : 1;

    // vector width needs aligned rows
    auto vec_ok = [&](int V) {
        if (V == 1)
            return true;
        if (ld_in % V || ld_out % V)
            return false;
        const size_t ca = std::min<size_t>(16, 8 * V), ta = std::min<size_t>(16, tsz * V);
        const size_t ia = std::min<size_t>(16, 4 * V);
        if ((form == 1 || form == 2) && (ld_conn % V || !aligned(conn, ia)))
            return false;
        return aligned(coords, ca) && aligned(out_K, ta) && aligned(out_F, ta) &&
               (!mask || fn || aligned(coeffs, ta));
    };
    if (!vec_ok(vec)) {
        if (forced && v.elems_per_thread > 1)
            return fail(FE_ERR_UNSUPPORTED, "elements per thread %d needs rows aligned to it", vec);
        vec = 1;
    }
    k.vec = vec;
    k.nt = nt;
    k.ref = ref;
    k.split = split;
    k.order = order;
    k.lanes = lanes;
    k.nq = rule->n_q;
    const KernelKey kv = k;  // the chosen variant, before any fallback
    auto usable = [&](const KernelEntry *x) {
        return x && (form == 0 || (form == 1 && x->idx != nullptr) || (form >= 2 && x->apply != nullptr));
    };
    const int nq_rule = k.nq;
    // the kernel of key k, compiled for the rule's point count or for any
    auto find_nq = [&]() {
        k.nq = nq_rule;
        const KernelEntry *x = find_kernel(k);
        if (!usable(x)) {
            k.nq = 0;
            x = find_kernel(k);
        }
        return x;
    };
    auto to_base = [&]() {
        k.vec = 1;
        k.nt = 1;
        k.ref = REF_KARG;
        k.split = 1;
        k.order = 1;
        k.lanes = 1;
    };
    const KernelEntry *e = find_nq();
    // Fallbacks, keeping the accumulation (packed 2: the upper triangle of a
    // symmetric K, mirrored) as long as some variant has it, so that every
    // form of a problem (stored, indexed, consumers) rounds alike: the
    // always-built base variant of the same accumulation, then the full-K
    // accumulation in the chosen variant, then in the base variant.
    if (!usable(e) && !forced && k.packed == 2) {
        to_base();
        e = find_nq();
    }
    if (!usable(e) && k.packed == 2) {
        k.packed = 0;
        if (!forced) {
            k.vec = kv.vec;
            k.nt = kv.nt;
            k.ref = kv.ref;
            k.split = kv.split;
            k.order = kv.order;
            k.lanes = kv.lanes;
        }
        e = find_nq();
    }
    if (!usable(e) && !forced) {
        to_base();
        e = find_nq();
        if (!usable(e)) {
            k.nq = 0;
            e = find_kernel(k);
        }
    }
    if (!usable(e))
        e = nullptr;
    if (!e)
        return fail(FE_ERR_UNSUPPORTED,
                    "no compiled kernel for elem=%d kind=%d prec=%d terms=%d mode=%d packed=%d "
                    "vec=%d nt=%d ref=%d nq=%d split=%d order=%d lanes=%d",
                    k.elem, k.kind, k.prec, k.terms, k.mode, k.packed, k.vec, k.nt, k.ref, k.nq,
                    k.split, k.order, k.lanes);

    KArgs &a = pl.args;
    std::memset(&a, 0, sizeof(a));
    a.coords = coords;
    a.coeffs = coeffs;
    a.out_K = out_K;
    a.out_F = out_F;
    a.n_elem = n_elem;
    a.ld_in = ld_in;
    a.ld_out = ld_out;
    a.k_packed = k.packed;
    int col = 0;
    for (int s = 0; s < 20; ++s) {
        if (problem->kind == FE_VECTOR_CDR) {
            // first row of block s in the compact array
            a.col[s] = (mask >> s & 1u) ? col : -1;
            col += (mask >> s & 1u) ? (s < 16 ? 9 : 3) : 0;
            a.uniform[s] = 0.0;
        } else {
            a.col[s] = (s < n_slots(problem->kind) && (mask >> s & 1u)) ? col++ : -1;
            a.uniform[s] = problem->uniform[s];
        }
    }
    fill_reference(elem, *rule, a);
    pl.entry = e;
    pl.block = (unsigned)wg;
    // threads: one per group of vec elements, or whole wavefronts of
    // 64 / lanes elements for the lane-split kernels
    const int64_t groups = k.lanes > 1 ? (n_elem + 64 / k.lanes - 1) / (64 / k.lanes) * 64
                                       : (n_elem + k.vec - 1) / k.vec;
    int64_t grid = (groups + wg - 1) / wg;
    if (v.blocks > 0 && v.blocks < grid)
        grid = v.blocks;
    if (grid > 0x7fffffff)
        grid = 0x7fffffff;
    pl.grid = (unsigned)(grid > 0 ? grid : 1);
    pl.key = k;
    pl.variant = fe_variant{wg, k.vec, ref == REF_LDS ? 1 : 2, nt == 0 ? 2 : (nt == 2 ? 3 : 1),
                            v.blocks, k.split, k.order, k.lanes};
    return FE_OK;
}

int launch(const Plan &pl, hipStream_t stream)
{
    if (pl.args.n_elem == 0)
        return FE_OK;
    const hipError_t err = pl.entry->launch(pl.args, pl.grid, pl.block, stream);
    if (err != hipSuccess)
        return fail(FE_ERR_HIP, "kernel launch failed: %s", hipGetErrorString(err));
    return FE_OK;
}

int launch_indexed(const Plan &pl, const IdxArgs &gi, hipStream_t stream)
{
    if (pl.args.n_elem == 0)
        return FE_OK;
    const hipError_t err = pl.entry->idx(pl.args, gi, pl.grid, pl.block, stream);
    if (err != hipSuccess)
        return fail(FE_ERR_HIP, "kernel launch failed: %s", hipGetErrorString(err));
    return FE_OK;
}

}  // namespace fe

using namespace fe;

// ------------------------------------------------------------------ C ABI
extern "C" {

int fe_integrate_ex(const fe_problem *problem, fe_elem_type elem_type, int64_t n_elem,
                    const double *coords, const void *coeffs, int64_t ld_in,
                    const fe_quad_rule *quad_rule, void *out_K, void *out_F, int64_t ld_out,
                    const fe_variant *variant, hipStream_t stream)
{
    Plan pl;
    int st = plan(problem, elem_type, n_elem, coords, coeffs, ld_in, quad_rule, out_K, out_F,
                  ld_out, variant, pl);
    if (st)
        return st;
    return launch(pl, stream);
}

int fe_integrate_indexed(const fe_problem *problem, fe_elem_type elem_type, int64_t n_elem,
                         const double *nodes, int64_t n_nodes, const int32_t *conn,
                         int64_t ld_conn, const void *coeffs, int64_t ld_in,
                         const fe_quad_rule *quad_rule, void *out_K, void *out_F, int64_t ld_out,
                         const fe_variant *variant, hipStream_t stream)
{
    if (n_elem > 0 && (!nodes || n_nodes < 1 || n_nodes > 0x7fffffffLL))
        return fail(FE_ERR_INVALID_ARG, "need a node array with 1 .. 2^31-1 nodes");
    if (nodes && ((uintptr_t)nodes % 8))
        return fail(FE_ERR_UNSUPPORTED, "nodes must be 8-byte aligned");
    Plan pl;
    int st = plan(problem, elem_type, n_elem, nullptr, coeffs, ld_in, quad_rule, out_K, out_F,
                  ld_out, variant, pl, 1, conn, ld_conn);
    if (st)
        return st;
    IdxArgs gi{nodes, conn, ld_conn, (uint32_t)n_nodes};
    return launch_indexed(pl, gi, stream);
}

// The consumers of indexed geometry that never store K: the matrix-free
// application (ap.x, ap.y) and the assembly into a CSR matrix (ap.vals).
// With colours, one launch per colour with plain read-add-write; without,
// one launch with atomic adds.
static int indexed_consumer(const fe_problem *problem, fe_elem_type elem_type, int64_t n_elem,
                            const double *nodes, int64_t n_nodes, const int32_t *conn,
                            int64_t ld_conn, const void *coeffs, int64_t ld_in,
                            const fe_quad_rule *quad_rule, const ApplyArgs &ap, bool csr,
                            const int64_t *color_ptr, int32_t n_colors, hipStream_t stream)
{
    const void *x = ap.x;
    void *y = ap.y, *b = ap.b;
    if (n_elem > 0 && (!nodes || n_nodes < 1 || n_nodes > 0x7fffffffLL))
        return fail(FE_ERR_INVALID_ARG, "need a node array with 1 .. 2^31-1 nodes");
    if (nodes && ((uintptr_t)nodes % 8))
        return fail(FE_ERR_UNSUPPORTED, "nodes must be 8-byte aligned");
    if (n_colors < 0 || (n_colors > 0 && !color_ptr))
        return fail(FE_ERR_INVALID_ARG, "n_colors must be >= 0, with color_ptr for n_colors > 0");
    if (n_colors > 0) {
        if (color_ptr[0] != 0 || color_ptr[n_colors] != n_elem)
            return fail(FE_ERR_INVALID_ARG, "color_ptr must run from 0 to n_elem");
        for (int c = 0; c < n_colors; ++c)
            if (color_ptr[c + 1] < color_ptr[c])
                return fail(FE_ERR_INVALID_ARG, "color_ptr must not decrease");
    }
    // the matrix-free form exists for the base variant: one element per lane
    const fe_variant base{256, 1, 2, 1, 0, 1, 1, 1};
    Plan pl;
    int st = plan(problem, elem_type, n_elem, nullptr, coeffs, ld_in, quad_rule, nullptr, nullptr,
                  n_elem, &base, pl, 2, conn, ld_conn);
    if (st)
        return st;
    if (!pl.entry->apply)
        return fail(FE_ERR_UNSUPPORTED, csr ? "no assembly form for this problem"
                                                : "no matrix-free form for this problem");
    const size_t tsz = problem->precision == FE_FP64 ? 8 : 4;
    if (!aligned(x, tsz) || !aligned(y, tsz) || !aligned(b, tsz) || !aligned(ap.vals, tsz))
        return fail(FE_ERR_UNSUPPORTED, "nodal vectors and values must be aligned to their element size");
    if (n_elem == 0)
        return FE_OK;
    const bool fn = problem->coef_mode == FE_COEF_FUNCTION;
    auto run = [&](int64_t e0, int64_t cnt, int atomic) -> int {
        if (cnt == 0)
            return FE_OK;
        KArgs a = pl.args;
        a.n_elem = cnt;
        if (a.coeffs && !fn)
            a.coeffs = static_cast<const char *>(a.coeffs) + tsz * e0;
        const IdxArgs gi{nodes, conn + e0, ld_conn, (uint32_t)n_nodes};
        int64_t grid = (cnt + pl.block - 1) / pl.block;
        if (grid > 0x7fffffff)
            grid = 0x7fffffff;
        const hipError_t err = pl.entry->apply(a, gi, ap, atomic, (unsigned)grid, pl.block, stream);
        if (err != hipSuccess)
            return fail(FE_ERR_HIP, "kernel launch failed: %s", hipGetErrorString(err));
        return FE_OK;
    };
    if (n_colors == 0)
        return run(0, n_elem, 1);
    for (int c = 0; c < n_colors; ++c)
        if ((st = run(color_ptr[c], color_ptr[c + 1] - color_ptr[c], 0)))
            return st;
    return FE_OK;
}

int fe_apply_indexed(const fe_problem *problem, fe_elem_type elem_type, int64_t n_elem,
                     const double *nodes, int64_t n_nodes, const int32_t *conn, int64_t ld_conn,
                     const void *coeffs, int64_t ld_in, const fe_quad_rule *quad_rule,
                     const void *x, void *y, void *b, const int64_t *color_ptr, int32_t n_colors,
                     hipStream_t stream)
{
    if (n_elem > 0 && (!x || !y))
        return fail(FE_ERR_INVALID_ARG, "x and y must not be NULL");
    ApplyArgs ap{};
    ap.x = x;
    ap.y = y;
    ap.b = b;
    return indexed_consumer(problem, elem_type, n_elem, nodes, n_nodes, conn, ld_conn, coeffs,
                            ld_in, quad_rule, ap, false, color_ptr, n_colors, stream);
}

int fe_assemble_csr(const fe_problem *problem, fe_elem_type elem_type, int64_t n_elem,
                    const double *nodes, int64_t n_nodes, const int32_t *conn, int64_t ld_conn,
                    const void *coeffs, int64_t ld_in, const fe_quad_rule *quad_rule,
                    const int64_t *row_ptr, const int32_t *col_idx, int64_t nnz, void *values,
                    void *b, const int64_t *color_ptr, int32_t n_colors, hipStream_t stream)
{
    if (n_elem > 0 && (!row_ptr || !col_idx || !values))
        return fail(FE_ERR_INVALID_ARG, "row_ptr, col_idx and values must not be NULL");
    if (nnz < 0 || nnz > 0x7fffffffffffLL)
        return fail(FE_ERR_INVALID_ARG, "nnz out of range");
    if (!aligned(row_ptr, 8) || !aligned(col_idx, 4))
        return fail(FE_ERR_UNSUPPORTED, "row_ptr and col_idx must be aligned to their element size");
    ApplyArgs ap{};
    ap.b = b;
    ap.row_ptr = row_ptr;
    ap.col_idx = col_idx;
    ap.nnz = nnz;
    ap.vals = values;  // non-null whenever a kernel is launched: selects the assembly form
    return indexed_consumer(problem, elem_type, n_elem, nodes, n_nodes, conn, ld_conn, coeffs,
                            ld_in, quad_rule, ap, true, color_ptr, n_colors, stream);
}

int fe_assemble_csr_rows(const fe_problem *problem, fe_elem_type elem_type, int64_t n_elem,
                         const double *nodes, int64_t n_nodes, const int32_t *conn,
                         int64_t ld_conn, const void *coeffs, int64_t ld_in,
                         const fe_quad_rule *quad_rule, const int64_t *row_ptr,
                         const int32_t *col_idx, int64_t nnz, void *values, void *b,
                         const int64_t *inc_ptr, const int32_t *inc, hipStream_t stream)
{
    if (n_elem > 0 && (!nodes || n_nodes < 1 || n_nodes > 0x7fffffffLL))
        return fail(FE_ERR_INVALID_ARG, "need a node array with 1 .. 2^31-1 nodes");
    if (n_elem > 0 && (!row_ptr || !col_idx || !values || !inc_ptr || !inc))
        return fail(FE_ERR_INVALID_ARG, "row_ptr, col_idx, values, inc_ptr and inc must not be NULL");
    if (nnz < 0 || nnz > 0x7fffffffffffLL)
        return fail(FE_ERR_INVALID_ARG, "nnz out of range");
    if (elem_type == FE_TET4 || elem_type == FE_PRISM6) {
        if (n_elem > 0x7fffffffLL / n_shape(elem_type))
            return fail(FE_ERR_INVALID_ARG, "element * vertex codes must fit in int32");
    }
    if (!aligned(nodes, 8) || !aligned(row_ptr, 8) || !aligned(col_idx, 4) ||
        !aligned(inc_ptr, 8) || !aligned(inc, 4))
        return fail(FE_ERR_UNSUPPORTED, "pointers must be aligned to their element size");
    // the assembly form exists for the base variant: one element per lane
    const fe_variant base{256, 1, 2, 1, 0, 1, 1, 1};
    Plan pl;
    int st = plan(problem, elem_type, n_elem, nullptr, coeffs, ld_in, quad_rule, nullptr, nullptr,
                  n_elem, &base, pl, 2, conn, ld_conn);
    if (st)
        return st;
    if (!pl.entry->apply)
        return fail(FE_ERR_UNSUPPORTED, "no assembly form for this problem");
    const size_t tsz = problem->precision == FE_FP64 ? 8 : 4;
    if (!aligned(values, tsz) || !aligned(b, tsz))
        return fail(FE_ERR_UNSUPPORTED, "values and b must be aligned to their element size");
    if (n_elem == 0)
        return FE_OK;
    ApplyArgs ap{};
    ap.b = b;
    ap.row_ptr = row_ptr;
    ap.col_idx = col_idx;
    ap.nnz = nnz;
    ap.vals = values;
    ap.inc_ptr = inc_ptr;
    ap.inc = inc;
    ap.n_own = n_nodes;
    const IdxArgs gi{nodes, conn, ld_conn, (uint32_t)n_nodes};
    int64_t grid = (n_nodes + pl.block - 1) / pl.block;
    if (grid > 0x7fffffff)
        grid = 0x7fffffff;
    const hipError_t err = pl.entry->apply(pl.args, gi, ap, 0, (unsigned)grid, pl.block, stream);
    if (err != hipSuccess)
        return fail(FE_ERR_HIP, "kernel launch failed: %s", hipGetErrorString(err));
    return FE_OK;
}

int fe_assemble_csr_blocks(const fe_problem *problem, fe_elem_type elem_type, int64_t n_elem,
                           const double *nodes, int64_t n_nodes, const void *coeffs,
                           int64_t ld_in, const fe_quad_rule *quad_rule, const int64_t *row_ptr,
                           const int32_t *col_idx, int64_t nnz, void *values, void *b,
                           const int64_t *inc_ptr, int64_t n_blocks, const int64_t *blk,
                           const int32_t *elems, const int32_t *verts, const uint16_t *lconn,
                           const uint32_t *linc, hipStream_t stream)
{
    if (elem_type != FE_TET4 || !problem || problem->kind != FE_SCALAR_CDR)
        return fail(FE_ERR_UNSUPPORTED, "node blocks are built for scalar problems on tetrahedra");
    if (n_elem > 0 && (!nodes || n_nodes < 1 || n_nodes > 0x7fffffffLL))
        return fail(FE_ERR_INVALID_ARG, "need a node array with 1 .. 2^31-1 nodes");
    if (n_elem > 0x7fffffffLL / 4)
        return fail(FE_ERR_INVALID_ARG, "element * vertex codes must fit in int32");
    if (n_blocks < 0 || n_blocks > 0x7fffffffLL || (n_elem > 0 && n_blocks < 1))
        return fail(FE_ERR_INVALID_ARG, "n_blocks out of range");
    if (n_elem > 0 && (!row_ptr || !col_idx || !values || !inc_ptr || !blk || !elems || !verts ||
                       !lconn || !linc))
        return fail(FE_ERR_INVALID_ARG,
                    "row_ptr, col_idx, values, inc_ptr and the node block arrays must not be NULL");
    if (nnz < 0 || nnz > 0x7fffffffffffLL)
        return fail(FE_ERR_INVALID_ARG, "nnz out of range");
    if (!aligned(nodes, 8) || !aligned(row_ptr, 8) || !aligned(col_idx, 4) ||
        !aligned(inc_ptr, 8) || !aligned(blk, 8) || !aligned(elems, 4) || !aligned(verts, 4) ||
        !aligned(lconn, 2) || !aligned(linc, 4))
        return fail(FE_ERR_UNSUPPORTED, "pointers must be aligned to their element size");
    const fe_variant base{256, 1, 2, 1, 0, 1, 1, 1};
    Plan pl;
    int st = plan(problem, elem_type, n_elem, nullptr, coeffs, ld_in, quad_rule, nullptr, nullptr,
                  n_elem, &base, pl, 3, nullptr, 0);
    if (st)
        return st;
    if (!pl.entry->apply)
        return fail(FE_ERR_UNSUPPORTED, "no assembly form for this problem");
    const size_t tsz = problem->precision == FE_FP64 ? 8 : 4;
    if (!aligned(values, tsz) || !aligned(b, tsz))
        return fail(FE_ERR_UNSUPPORTED, "values and b must be aligned to their element size");
    if (n_elem == 0)
        return FE_OK;
    ApplyArgs ap{};
    ap.b = b;
    ap.row_ptr = row_ptr;
    ap.col_idx = col_idx;
    ap.nnz = nnz;
    ap.vals = values;
    ap.inc_ptr = inc_ptr;
    ap.n_own = n_nodes;
    ap.blk = blk;
    ap.blk_elems = elems;
    ap.blk_verts = verts;
    ap.blk_conn = lconn;
    ap.linc = linc;
    const IdxArgs gi{nodes, nullptr, 0, (uint32_t)n_nodes};
    const hipError_t err =
        pl.entry->apply(pl.args, gi, ap, 0, (unsigned)n_blocks, FE_CSR_BLOCK_NODES, stream);
    if (err != hipSuccess)
        return fail(FE_ERR_HIP, "kernel launch failed: %s", hipGetErrorString(err));
    return FE_OK;
}

int fe_integrate_natural(const fe_problem *problem, fe_elem_type elem_type, int64_t n_elem,
                         const double *coords, const void *coeffs, const fe_quad_rule *quad_rule,
                         void *out_K, void *out_F, hipStream_t stream)
{
    // the natural-order form exists for the base variant: one element per lane
    const fe_variant base{AOS_TILE, 1, 2, 1, 0, 1, 1, 1};
    Plan pl;
    int st = plan(problem, elem_type, n_elem, coords, coeffs, n_elem, quad_rule, out_K, out_F,
                  n_elem, &base, pl);
    if (st)
        return st;
    if (!pl.entry->aos)
        return fail(FE_ERR_UNSUPPORTED, "no natural-order form for this problem");
    const bool fn = problem->coef_mode == FE_COEF_FUNCTION;
    AosArgs ao{};
    ao.tsize = problem->precision == FE_FP64 ? 8 : 4;
    ao.coef_rows = fn ? 0 : (int32_t)fe_coeff_entries(problem, elem_type, quad_rule->n_q);
    ao.k_rows = (int32_t)fe_k_entries(problem, elem_type);
    ao.f_rows = (int32_t)fe_f_entries(problem, elem_type);
    auto magic = [](int32_t d) -> uint32_t {
        return d > 0 ? (uint32_t)(((uint64_t)1 << 32) / (uint64_t)d + 1) : 0u;
    };
    ao.coef_magic = magic(ao.coef_rows);
    ao.k_magic = magic(ao.k_rows);
    ao.f_magic = magic(ao.f_rows);
    const int nv = elem_type == FE_TET4 ? 4 : 6;
    // the outputs reuse the inputs' LDS (every input of an element is read
    // before its first output is written, and a tile is one wavefront),
    // except for the 3-component problems, whose block loop reads
    // coefficients after storing earlier blocks: their outputs follow the
    // inputs
    const size_t in_b = 8 * 3 * nv + (size_t)ao.tsize * ao.coef_rows;
    const size_t out_b = (size_t)ao.tsize * (ao.k_rows + ao.f_rows);
    const bool separate = problem->kind == FE_VECTOR_CDR;
    const size_t lds = (size_t)AOS_TILE * (separate ? in_b + out_b : (in_b > out_b ? in_b : out_b));
    // the device's LDS per workgroup (160 KiB on gfx950; 64 KiB when it
    // cannot be queried) less the kernel's static reference tables
    size_t lds_max = 64 * 1024;
    int dev = 0, attr = 0;
    const hipError_t pending = hipPeekAtLastError();
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&attr, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess &&
        attr > 0)
        lds_max = (size_t)attr;
    else if (pending == hipSuccess)
        (void)hipGetLastError();  // clear only what the failed query left
    const size_t lds_dyn_max = lds_max > 2048 ? lds_max - 2048 : 0;
    // Two forms (measured on MI355X): the LDS tile suits records with few
    // coefficient rows (uniform data, a per-point right-hand side); records
    // with 16 or more coefficient rows, elasticity and the 3-component
    // problems run faster read and written in place, and tiles of more than
    // 64 KiB (one workgroup, one wavefront per CU) always do
    ao.direct = (problem->kind != FE_SCALAR_CDR || ao.coef_rows >= 16 || lds > 64 * 1024 ||
                 lds > lds_dyn_max)
                    ? 1
                    : 0;
    if (n_elem == 0)
        return FE_OK;
    int64_t grid = ao.direct ? (n_elem + 255) / 256 : (n_elem + AOS_TILE - 1) / AOS_TILE;
    if (grid > 0x7fffffff)
        grid = 0x7fffffff;
    const hipError_t err = pl.entry->aos(pl.args, ao, (unsigned)grid, ao.direct ? 0 : lds, stream);
    if (err != hipSuccess)
        return fail(FE_ERR_HIP, "kernel launch failed: %s", hipGetErrorString(err));
    return FE_OK;
}

int fe_color_elements(fe_elem_type elem_type, int64_t n_elem, const int32_t *conn, int64_t ld_conn,
                      int64_t n_nodes, int32_t *perm, int64_t *color_ptr, int32_t max_colors)
{
    if (elem_type != FE_TET4 && elem_type != FE_PRISM6)
        return -fail(FE_ERR_INVALID_ARG, "bad element type %d", elem_type);
    if (n_elem < 0 || n_elem > 0x7fffffffLL || n_nodes < 1 || n_nodes > 0x7fffffffLL ||
        max_colors < 1 || (n_elem > 0 && (!conn || !perm || ld_conn < n_elem)) || !color_ptr)
        return -fail(FE_ERR_INVALID_ARG, "bad colouring arguments");
    const int nv = n_shape(elem_type);
    const int words = (max_colors + 63) / 64;
    std::vector<uint64_t> used((size_t)n_nodes * words, 0);  // colours taken at each node
    std::vector<int32_t> color((size_t)n_elem);
    int n_colors = 0;
    for (int64_t e = 0; e < n_elem; ++e) {
        int32_t id[6];
        for (int v = 0; v < nv; ++v) {
            id[v] = conn[v * ld_conn + e];
            if (id[v] < 0 || id[v] >= n_nodes)
                return -fail(FE_ERR_INVALID_ARG, "element %lld has node id %d outside [0, %lld)",
                             (long long)e, id[v], (long long)n_nodes);
        }
        int c = -1;
        for (int w = 0; w < words && c < 0; ++w) {
            uint64_t taken = 0;
            for (int v = 0; v < nv; ++v)
                taken |= used[(size_t)id[v] * words + w];
            if (~taken) {
                const int cand = 64 * w + __builtin_ctzll(~taken);
                if (cand < max_colors)
                    c = cand;
            }
        }
        if (c < 0)
            return -fail(FE_ERR_CAPACITY, "more than %d colours needed", max_colors);
        for (int v = 0; v < nv; ++v)
            used[(size_t)id[v] * words + c / 64] |= 1ull << (c % 64);
        color[e] = c;
        n_colors = std::max(n_colors, c + 1);
    }
    // elements colour by colour, in their original order within a colour
    std::vector<int64_t> count((size_t)n_colors + 1, 0);
    for (int64_t e = 0; e < n_elem; ++e)
        ++count[color[e] + 1];
    for (int c = 0; c < n_colors; ++c)
        count[c + 1] += count[c];
    for (int c = 0; c <= n_colors; ++c)
        color_ptr[c] = count[c];
    for (int64_t e = 0; e < n_elem; ++e)
        perm[count[color[e]]++] = (int32_t)e;
    return n_colors;
}

int64_t fe_node_incidence(fe_elem_type elem_type, int64_t n_elem, const int32_t *conn,
                          int64_t ld_conn, int64_t n_nodes, int64_t *inc_ptr, int32_t *inc)
{
    if (elem_type != FE_TET4 && elem_type != FE_PRISM6)
        return -fail(FE_ERR_INVALID_ARG, "bad element type %d", elem_type);
    const int nv = n_shape(elem_type);
    if (n_elem < 0 || n_elem > 0x7fffffffLL / nv || n_nodes < 1 || n_nodes > 0x7fffffffLL ||
        (n_elem > 0 && (!conn || ld_conn < n_elem)) || !inc_ptr)
        return -fail(FE_ERR_INVALID_ARG, "bad incidence arguments");
    for (int64_t i = 0; i <= n_nodes; ++i)
        inc_ptr[i] = 0;
    for (int v = 0; v < nv; ++v)
        for (int64_t e = 0; e < n_elem; ++e) {
            const int32_t id = conn[v * ld_conn + e];
            if (id < 0 || id >= n_nodes)
                return -fail(FE_ERR_INVALID_ARG, "element %lld has node id %d outside [0, %lld)",
                             (long long)e, id, (long long)n_nodes);
            ++inc_ptr[id + 1];
        }
    for (int64_t i = 0; i < n_nodes; ++i)
        inc_ptr[i + 1] += inc_ptr[i];
    if (inc) {
        std::vector<int64_t> fill(inc_ptr, inc_ptr + n_nodes);
        for (int64_t e = 0; e < n_elem; ++e)
            for (int v = 0; v < nv; ++v)
                inc[fill[conn[v * ld_conn + e]]++] = (int32_t)(e * nv + v);
    }
    return inc_ptr[n_nodes];
}

static_assert(FE_CSR_BLOCK_ELEMS * 4 <= 0x4000, "element slot and vertex fit 14 bits of a code");

int64_t fe_csr_blocks(fe_elem_type elem_type, int64_t n_elem, const int32_t *conn, int64_t ld_conn,
                      int64_t n_nodes, const int64_t *inc_ptr, const int32_t *inc,
                      const int64_t *row_ptr, const int32_t *col_idx, int64_t *sizes,
                      int64_t *blk, int32_t *elems, int32_t *verts, uint16_t *lconn,
                      uint32_t *linc)
{
    if (elem_type == FE_PRISM6)
        return -fail(FE_ERR_UNSUPPORTED, "node blocks are built for tetrahedra");
    if (elem_type != FE_TET4)
        return -fail(FE_ERR_INVALID_ARG, "bad element type %d", elem_type);
    const int nv = 4;
    if (n_elem < 0 || n_elem > 0x7fffffffLL / nv || n_nodes < 1 || n_nodes > 0x7fffffffLL ||
        (n_elem > 0 && (!conn || ld_conn < n_elem)) || !inc_ptr || !inc || !row_ptr ||
        !col_idx || !sizes)
        return -fail(FE_ERR_INVALID_ARG, "bad node block arguments");
    for (int64_t i = 0; i < n_nodes; ++i)
        if (row_ptr[i + 1] < row_ptr[i] || row_ptr[i] < 0)
            return -fail(FE_ERR_INVALID_ARG, "row_ptr decreases at row %lld", (long long)i);
    if (inc_ptr[0] != 0 || inc_ptr[n_nodes] != n_elem * nv)
        return -fail(FE_ERR_INVALID_ARG, "inc_ptr does not cover n_elem * n_vert incidences");
    for (int64_t i = 0; i < n_nodes; ++i)
        if (inc_ptr[i + 1] < inc_ptr[i])
            return -fail(FE_ERR_INVALID_ARG, "inc_ptr decreases at node %lld", (long long)i);
    for (int64_t k = 0; k < n_elem * nv; ++k)
        if (inc[k] < 0 || inc[k] >= n_elem * nv)
            return -fail(FE_ERR_INVALID_ARG, "incidence %lld codes no element", (long long)k);
    for (int v = 0; v < nv; ++v)
        for (int64_t e = 0; e < n_elem; ++e)
            if (conn[v * ld_conn + e] < 0 || conn[v * ld_conn + e] >= n_nodes)
                return -fail(FE_ERR_INVALID_ARG, "element %lld has node id %d outside [0, %lld)",
                             (long long)e, conn[v * ld_conn + e], (long long)n_nodes);
    // greedy partition of the node order: a block grows node by node while
    // its nodes, their elements and those elements' vertices fit
    std::vector<int64_t> e_mark((size_t)n_elem, -1), v_mark((size_t)n_nodes, -1);
    std::vector<int64_t> bounds{0};
    int64_t n_in = 0, e_in = 0, v_in = 0, e_tot = 0, v_tot = 0, trial = 0;
    const int64_t block_id_base = n_nodes + 1;  // marks of committed blocks
    int64_t cur = block_id_base;
    auto count_new = [&](int64_t i, int64_t &ne, int64_t &nvx) {
        // elements and vertices node i adds to the current block
        ++trial;
        ne = nvx = 0;
        for (int64_t k = inc_ptr[i]; k < inc_ptr[i + 1]; ++k) {
            const int64_t e = inc[k] / nv;
            if (e_mark[e] == cur || e_mark[e] == -2 - trial)
                continue;
            e_mark[e] = -2 - trial;
            ++ne;
            for (int v = 0; v < nv; ++v) {
                const int32_t g = conn[v * ld_conn + e];
                if (v_mark[g] == cur || v_mark[g] == -2 - trial)
                    continue;
                v_mark[g] = -2 - trial;
                ++nvx;
            }
        }
    };
    auto commit = [&](int64_t i) {
        for (int64_t k = inc_ptr[i]; k < inc_ptr[i + 1]; ++k) {
            const int64_t e = inc[k] / nv;
            e_mark[e] = cur;
            for (int v = 0; v < nv; ++v)
                v_mark[conn[v * ld_conn + e]] = cur;
        }
    };
    for (int64_t i = 0; i < n_nodes; ++i) {
        int64_t ne, nvx;
        count_new(i, ne, nvx);
        if (n_in > 0 && (n_in + 1 > FE_CSR_BLOCK_NODES || e_in + ne > FE_CSR_BLOCK_ELEMS ||
                         v_in + nvx > FE_CSR_BLOCK_VERTS)) {
            bounds.push_back(i);
            e_tot += e_in;
            v_tot += v_in;
            n_in = e_in = v_in = 0;
            ++cur;
            count_new(i, ne, nvx);
        }
        if (ne > FE_CSR_BLOCK_ELEMS || nvx > FE_CSR_BLOCK_VERTS)
            return -fail(FE_ERR_CAPACITY, "node %lld alone has %lld elements and %lld vertices "
                         "(a block holds %d and %d)", (long long)i, (long long)ne, (long long)nvx,
                         FE_CSR_BLOCK_ELEMS, FE_CSR_BLOCK_VERTS);
        commit(i);
        ++n_in;
        e_in += ne;
        v_in += nvx;
    }
    bounds.push_back(n_nodes);
    e_tot += e_in;
    v_tot += v_in;
    const int64_t nb = (int64_t)bounds.size() - 1;
    sizes[0] = nb;
    sizes[1] = e_tot;
    sizes[2] = v_tot;
    if (!blk)
        return nb;
    if (!elems || !verts || !lconn || !linc)
        return -fail(FE_ERR_INVALID_ARG, "NULL node block output");
    // fill: per block, its elements in the order of first appearance along
    // the nodes' incidence lists, its vertices ascending
    std::vector<int32_t> e_loc((size_t)n_elem, -1), v_loc((size_t)n_nodes, -1);
    std::vector<int32_t> el, vl;
    int64_t es = 0, vs = 0;
    for (int64_t bb = 0; bb < nb; ++bb) {
        const int64_t n0 = bounds[bb], n1 = bounds[bb + 1];
        el.clear();
        vl.clear();
        for (int64_t i = n0; i < n1; ++i)
            for (int64_t k = inc_ptr[i]; k < inc_ptr[i + 1]; ++k) {
                const int64_t e = inc[k] / nv;
                if (e_loc[e] >= 0 && e_loc[e] < (int32_t)el.size() && el[e_loc[e]] == e)
                    continue;
                e_loc[e] = (int32_t)el.size();
                el.push_back((int32_t)e);
            }
        for (int32_t e : el)
            for (int v = 0; v < nv; ++v) {
                const int32_t g = conn[v * ld_conn + e];
                if (v_loc[g] == (int32_t)bb)
                    continue;
                v_loc[g] = (int32_t)bb;
                vl.push_back(g);
            }
        std::sort(vl.begin(), vl.end());
        for (size_t j = 0; j < vl.size(); ++j)
            v_loc[vl[j]] = (int32_t)j;
        blk[3 * bb + 0] = n0;
        blk[3 * bb + 1] = es;
        blk[3 * bb + 2] = vs;
        for (size_t j = 0; j < el.size(); ++j) {
            elems[es + j] = el[j];
            for (int v = 0; v < nv; ++v)
                lconn[(es + (int64_t)j) * nv + v] = (uint16_t)v_loc[conn[v * ld_conn + el[j]]];
        }
        for (size_t j = 0; j < vl.size(); ++j)
            verts[vs + j] = vl[j];
        for (int64_t i = n0; i < n1; ++i) {
            const int32_t *cb = col_idx + row_ptr[i], *ce = col_idx + row_ptr[i + 1];
            for (int64_t k = inc_ptr[i]; k < inc_ptr[i + 1]; ++k) {
                const int64_t e = inc[k] / nv;
                const int lv = (int)(inc[k] % nv);
                uint32_t code = (uint32_t)(e_loc[e] * nv + lv);
                int f = 0;
                for (int u = 0; u < nv; ++u) {
                    if (u == lv)
                        continue;
                    // position of vertex u's column in row i (ascending
                    // columns): 62 absent, 63 past offset 61
                    const int32_t g = conn[u * ld_conn + e];
                    const int32_t *at = std::lower_bound(cb, ce, g);
                    const int64_t pos = at - cb;
                    const uint32_t field = (at == ce || *at != g) ? 62u : (pos < 62 ? (uint32_t)pos : 63u);
                    code |= field << (14 + 6 * f);
                    ++f;
                }
                linc[k] = code;
            }
        }
        // vertex marks of the next block must not match this block's
        // local indices: reset the ones used here
        for (int32_t g : vl)
            v_loc[g] = -1;
        es += (int64_t)el.size();
        vs += (int64_t)vl.size();
    }
    blk[3 * nb + 0] = n_nodes;
    blk[3 * nb + 1] = es;
    blk[3 * nb + 2] = vs;
    return nb;
}

int64_t fe_csr_pattern(fe_elem_type elem_type, int64_t n_elem, const int32_t *conn,
                       int64_t ld_conn, int64_t n_nodes, int32_t n_comp, int64_t *row_ptr,
                       int32_t *col_idx, int64_t max_nnz)
{
    if (elem_type != FE_TET4 && elem_type != FE_PRISM6)
        return -fail(FE_ERR_INVALID_ARG, "bad element type %d", elem_type);
    if (n_comp != 1 && n_comp != 3)
        return -fail(FE_ERR_INVALID_ARG, "n_comp must be 1 or 3");
    if (n_elem < 0 || n_elem > 0x7fffffffLL || n_nodes < 1 ||
        n_nodes * n_comp > 0x7fffffffLL || (n_elem > 0 && (!conn || ld_conn < n_elem)) ||
        !row_ptr || max_nnz < 0)
        return -fail(FE_ERR_INVALID_ARG, "bad pattern arguments");
    const int nv = n_shape(elem_type);
    // elements at each node
    std::vector<int64_t> at((size_t)n_nodes + 1, 0);
    for (int v = 0; v < nv; ++v)
        for (int64_t e = 0; e < n_elem; ++e) {
            const int32_t id = conn[v * ld_conn + e];
            if (id < 0 || id >= n_nodes)
                return -fail(FE_ERR_INVALID_ARG, "element %lld has node id %d outside [0, %lld)",
                             (long long)e, id, (long long)n_nodes);
            ++at[(size_t)id + 1];
        }
    for (int64_t i = 0; i < n_nodes; ++i)
        at[i + 1] += at[i];
    std::vector<int32_t> elems((size_t)at[n_nodes]);
    {
        std::vector<int64_t> fill(at.begin(), at.end() - 1);
        for (int64_t e = 0; e < n_elem; ++e)
            for (int v = 0; v < nv; ++v)
                elems[fill[conn[v * ld_conn + e]]++] = (int32_t)e;
    }
    // node neighbours (the node itself included), ascending
    std::vector<int64_t> nb_ptr((size_t)n_nodes + 1, 0);
    std::vector<int32_t> nb;
    std::vector<int32_t> mark((size_t)n_nodes, -1);
    nb.reserve((size_t)at[n_nodes] * 2);
    for (int64_t i = 0; i < n_nodes; ++i) {
        const size_t first = nb.size();
        for (int64_t k = at[i]; k < at[i + 1]; ++k)
            for (int v = 0; v < nv; ++v) {
                const int32_t j = conn[v * ld_conn + elems[k]];
                if (mark[j] != (int32_t)i) {
                    mark[j] = (int32_t)i;
                    nb.push_back(j);
                }
            }
        std::sort(nb.begin() + first, nb.end());
        nb_ptr[i + 1] = (int64_t)nb.size();
    }
    // rows of the components of a node: the same columns, every component of
    // every neighbour
    const int64_t nc = n_comp;
    int64_t nnz = 0;
    row_ptr[0] = 0;
    for (int64_t i = 0; i < n_nodes; ++i) {
        const int64_t len = nc * (nb_ptr[i + 1] - nb_ptr[i]);
        for (int64_t a = 0; a < nc; ++a) {
            nnz += len;
            row_ptr[nc * i + a + 1] = nnz;
        }
    }
    if (!col_idx)
        return nnz;
    if (nnz > max_nnz)
        return -fail(FE_ERR_CAPACITY, "the pattern has %lld entries; col_idx holds %lld",
                     (long long)nnz, (long long)max_nnz);
    for (int64_t i = 0; i < n_nodes; ++i)
        for (int64_t a = 0; a < nc; ++a) {
            int32_t *out = col_idx + row_ptr[nc * i + a];
            for (int64_t k = nb_ptr[i]; k < nb_ptr[i + 1]; ++k)
                for (int64_t b = 0; b < nc; ++b)
                    *out++ = (int32_t)(nc * nb[k] + b);
        }
    return nnz;
}

int fe_integrate(const fe_problem *problem, fe_elem_type elem_type, int64_t n_elem,
                 const double *coords, const void *coeffs, const fe_quad_rule *quad_rule,
                 void *out_K, void *out_F, hipStream_t stream)
{
    return fe_integrate_ex(problem, elem_type, n_elem, coords, coeffs, n_elem, quad_rule, out_K,
                           out_F, n_elem, nullptr, stream);
}

int64_t fe_k_entries(const fe_problem *problem, fe_elem_type elem_type)
{
    if (check_problem(problem, elem_type))
        return -1;
    const int64_t N = n_shape(elem_type) * n_comp(problem->kind);
    return problem->k_format == FE_K_SYM_PACKED ? N * (N + 1) / 2 : N * N;
}

int64_t fe_f_entries(const fe_problem *problem, fe_elem_type elem_type)
{
    if (check_problem(problem, elem_type))
        return -1;
    return n_shape(elem_type) * n_comp(problem->kind);
}

int64_t fe_coeff_entries(const fe_problem *problem, fe_elem_type elem_type, int n_q)
{
    if (check_problem(problem, elem_type) || n_q < 1 || n_q > FE_MAX_QP)
        return -1;
    const int64_t c = problem->kind == FE_VECTOR_CDR ? vector_rows(effective_mask(problem))
                                                     : __builtin_popcount(effective_mask(problem));
    if (problem->coef_mode == FE_COEF_FUNCTION)
        return c ? FE_COEF_FN_PARAMS : 0;
    return problem->coef_mode == FE_COEF_PER_QP ? c * n_q : c;
}

int64_t fe_bytes_per_element(const fe_problem *problem, fe_elem_type elem_type, int n_q)
{
    const int64_t nk = fe_k_entries(problem, elem_type);
    const int64_t nf = fe_f_entries(problem, elem_type);
    const int64_t nc = fe_coeff_entries(problem, elem_type, n_q);
    if (nk < 0 || nf < 0 || nc < 0)
        return -1;
    const int64_t t = problem->precision == FE_FP64 ? 8 : 4;
    // function parameters are read once per launch, not per element
    const int64_t ncpe = problem->coef_mode == FE_COEF_FUNCTION ? 0 : nc;
    return 8 * 3 * n_shape(elem_type) + t * (ncpe + nk + nf);
}

int64_t fe_k_index(const fe_problem *problem, fe_elem_type elem_type, int row, int col)
{
    if (check_problem(problem, elem_type))
        return -1;
    const int N = n_shape(elem_type) * n_comp(problem->kind);
    if (row < 0 || col < 0 || row >= N || col >= N)
        return -1;
    if (problem->k_format == FE_K_SYM_PACKED)
        return col >= row ? (int64_t)row * N - (int64_t)row * (row - 1) / 2 + (col - row) : -1;
    return (int64_t)row * N + col;
}

// Built-in rules, written out here independently of any other component.
static double g_tet1_xi[3], g_tet1_w[1], g_tet4_xi[12], g_tet4_w[4], g_pri6_xi[18], g_pri6_w[6];
static std::once_flag g_rules_once;

static void init_rules()
{
    g_tet1_xi[0] = g_tet1_xi[1] = g_tet1_xi[2] = 0.25;
    g_tet1_w[0] = 1.0 / 6.0;
    const double r5 = std::sqrt(5.0);
    const double hi = (5.0 + 3.0 * r5) / 20.0, lo = (5.0 - r5) / 20.0;
    for (int q = 0; q < 4; ++q) {
        for (int k = 0; k < 3; ++k)
            g_tet4_xi[3 * q + k] = (q == k + 1) ? hi : lo;
        g_tet4_w[q] = 1.0 / 24.0;
    }
    const double tri[3][2] = {{2.0 / 3.0, 1.0 / 6.0}, {1.0 / 6.0, 2.0 / 3.0}, {1.0 / 6.0, 1.0 / 6.0}};
    const double z = 1.0 / std::sqrt(3.0);
    for (int t = 0; t < 3; ++t)
        for (int l = 0; l < 2; ++l) {
            const int q = 2 * t + l;
            g_pri6_xi[3 * q] = tri[t][0];
            g_pri6_xi[3 * q + 1] = tri[t][1];
            g_pri6_xi[3 * q + 2] = l ? z : -z;
            g_pri6_w[q] = 1.0 / 6.0;
        }
}

int fe_quad_rule_builtin(fe_elem_type elem_type, int n_q, fe_quad_rule *out)
{
    if (!out)
        return fail(FE_ERR_INVALID_ARG, "out is NULL");
    std::call_once(g_rules_once, init_rules);
    if (elem_type == FE_TET4 && n_q == 1) {
        *out = fe_quad_rule{1, g_tet1_xi, g_tet1_w};
        return FE_OK;
    }
    if (elem_type == FE_TET4 && n_q == 4) {
        *out = fe_quad_rule{4, g_tet4_xi, g_tet4_w};
        return FE_OK;
    }
    if (elem_type == FE_PRISM6 && n_q == 6) {
        *out = fe_quad_rule{6, g_pri6_xi, g_pri6_w};
        return FE_OK;
    }
    return fail(FE_ERR_UNSUPPORTED, "no built-in rule for element %d with %d points", elem_type, n_q);
}

const char *fe_status_string(int status)
{
    switch (status) {
    case FE_OK: return "ok";
    case FE_ERR_INVALID_ARG: return "invalid argument";
    case FE_ERR_UNSUPPORTED: return "unsupported";
    case FE_ERR_NOT_SYMMETRIC: return "packed K requested for a non-symmetric problem";
    case FE_ERR_HIP: return "HIP runtime error";
    case FE_ERR_CAPACITY: return "capacity exceeded";
    default: return "unknown status";
    }
}

const char *fe_last_error(void) { return g_last_error.c_str(); }

int fe_version(void) { return 1 * 10000 + 1 * 100 + 0; }

int64_t fe_ld_for(int64_t n_elem)
{
    if (n_elem < 0)
        return -1;
    return (n_elem + 255) / 256 * 256;
}

}  // extern "C"
