/*
 * fe_oracle.c -- plain, slow, FP64 CPU oracle for per-element finite element
 * numerical integration with first-order approximations (K. Banas,
 * F. Kruzel, J. Bielanski, arXiv:1504.01023).
 *
 * TEST INFRASTRUCTURE. Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library. It shares no code, header,
 * table or constant with the GPU library: shape functions, quadrature rules
 * and the element loop are written out here independently.
 *
 * What it computes. For every element e, the element stiffness matrix and
 * load vector of eqs. "sm_local" and "lv_local" (Sec. 2.2) as their
 * definition gives them after the change of variables to the reference
 * element (eq. "change_of_variables") and the quadrature rule the caller
 * passes (eq. "quadrature", Sec. 2.3):
 *   K[r][s] = sum_q vol_q sum_{a,b} c^{a;b}(x_q) Phi_r[a](x_q) Phi_s[b](x_q),
 *   F[r]    = sum_q vol_q sum_a d^a(x_q) Phi_r[a](x_q),
 * vol_q = det J(xi_q) w_q, Phi_r = (phi_r, its x, y, z derivatives); for
 * 3-component problems every coefficient also carries the component indices
 * of the test and trial functions. Each term is evaluated as written, point
 * by point; nothing is hoisted, reduced in advance or fused.
 *
 * Readings where the paper is silent (stated again in the design notes):
 *  - first coefficient index pairs with the test function (row r), the second
 *    with the trial function (column s);
 *  - reference tetrahedron (0,0,0),(1,0,0),(0,1,0),(0,0,1) with shape
 *    functions 1-xi-eta-zeta, xi, eta, zeta; reference prism = unit right
 *    triangle x [-1,1], bottom nodes 0-2 at zeta=-1, top node v+3 above v;
 *  - det J is used signed (no absolute value);
 *  - the Jacobian is formed from the edge vectors X_r - X_0 (see
 *    jacobian_terms);
 *  - 3-component problems number unknowns node-major (3 r + alpha); the
 *    isotropic elasticity tensor is C_{i alpha j beta} = lambda d_{i alpha}
 *    d_{j beta} + mu (d_ij d_{alpha beta} + d_{i beta} d_{j alpha}) for the
 *    product w^alpha_{,i} u^beta_{,j}, lambda and mu from E and nu, and the
 *    body force enters as d^0_alpha;
 *  - the general 3-component problem (every c^{a;b} and d^a of the weak form
 *    a 3x3 matrix or 3-vector over the components, Sec. 2.1 and 3.3) keeps the
 *    component of the test function first: c^{a;b}_{alpha beta} multiplies
 *    the alpha component of the test function and the beta component of the
 *    trial function.
 *
 * Input layouts (identical to what the GPU library consumes):
 *  coords[(v*3+d)*ld + e]; coefficient array in "compact" form: only the
 *  slots whose bit is set in `mask`, in increasing slot order j; per element
 *  coeffs[j*ldc + e], per point coeffs[(j*n_q + q)*ldc + e]. Slots whose bit
 *  is clear take the value uniform[slot]. Scalar slots: 4a+b -> c[a][b],
 *  16+a -> d[a]. Elasticity slots: E, nu, f_x, f_y, f_z. In the function
 *  mode `coeffs` holds the 122 parameters of the coefficient function (see
 *  fn_raw) and the slots in `mask` are computed from it at every point.
 *  General 3-component problem: 156 slots, (4a+b)*9 + 3 alpha + beta ->
 *  c^{a;b}_{alpha beta} for the first 144 and 144 + 3a + alpha -> d^a_alpha;
 *  `mask` has one bit per block (bit 4a+b: the nine c^{a;b}_{..}; bit 16+a:
 *  the three d^a_.), a block whose bit is clear is zero, and the compact
 *  array holds the slots of the present blocks in slot order.
 *
 * Output: full matrices, element-major: K[e*N*N + row*N + col], F[e*N + row],
 * N = number of shape functions times components.
 *
 * Compiled with -O2 -fno-fast-math -ffp-contract=off.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_TET4 0
#define OR_PRISM6 1
#define OR_SCALAR 0
#define OR_ELASTICITY 1
#define OR_VECTOR 2
#define OR_MAX_SLOTS 156
#define OR_UNIFORM 0
#define OR_PER_ELEMENT 1
#define OR_PER_QP 2
#define OR_FUNCTION 3
#define OR_FN_PARAMS 122

#define OR_OK 0
#define OR_EINVAL 1
#define OR_ENOMEM 2

/* ------------------------------------------------------------------------
 * Reference elements (reading of Sec. 2.3's "reference element").
 * ---------------------------------------------------------------------- */

/* Affine tetrahedron: values and reference derivatives d/dxi_k. */
static void tet4_shape(const double xi[3], double phi[6], double dphi[6][3])
{
    phi[0] = 1.0 - xi[0] - xi[1] - xi[2];
    phi[1] = xi[0];
    phi[2] = xi[1];
    phi[3] = xi[2];
    for (int k = 0; k < 3; ++k) {
        dphi[0][k] = -1.0;
        dphi[1][k] = (k == 0) ? 1.0 : 0.0;
        dphi[2][k] = (k == 1) ? 1.0 : 0.0;
        dphi[3][k] = (k == 2) ? 1.0 : 0.0;
    }
}

/* Linear prism: triangle functions N = (1-xi-eta, xi, eta) times the linear
 * functions (1-zeta)/2 (bottom, nodes 0-2) and (1+zeta)/2 (top, nodes 3-5). */
static void prism6_shape(const double xi[3], double phi[6], double dphi[6][3])
{
    const double N[3] = {1.0 - xi[0] - xi[1], xi[0], xi[1]};
    const double dNdxi[3] = {-1.0, 1.0, 0.0};
    const double dNdeta[3] = {-1.0, 0.0, 1.0};
    const double lo = 0.5 * (1.0 - xi[2]);
    const double hi = 0.5 * (1.0 + xi[2]);
    for (int i = 0; i < 3; ++i) {
        phi[i] = N[i] * lo;
        phi[i + 3] = N[i] * hi;
        dphi[i][0] = dNdxi[i] * lo;
        dphi[i][1] = dNdeta[i] * lo;
        dphi[i][2] = -0.5 * N[i];
        dphi[i + 3][0] = dNdxi[i] * hi;
        dphi[i + 3][1] = dNdeta[i] * hi;
        dphi[i + 3][2] = 0.5 * N[i];
    }
}

static int n_shape(int elem) { return elem == OR_TET4 ? 4 : 6; }

/* ------------------------------------------------------------------------
 * Quadrature rules (reading of Sec. 2.3's "Gaussian quadratures" and the
 * point counts of Sec. 4.1). Points are given in reference coordinates.
 *  tet, 1 point : centroid, weight 1/6 (degree 1).
 *  tet, 4 points: barycentric permutations of (a,b,b,b), a = (5+3 sqrt5)/20,
 *                 b = (5-sqrt5)/20, weight 1/24 (degree 2); point q has the
 *                 large barycentric weight on vertex q.
 *  prism, 6 pts : triangle points (2/3,1/6), (1/6,2/3), (1/6,1/6), weight 1/6,
 *                 times Gauss-Legendre zeta = -+1/sqrt3 with weight 1; point
 *                 index 2 t + l, l = 0 at zeta = -1/sqrt3.
 * ---------------------------------------------------------------------- */
int oracle_quad_rule(int elem, int n_q, double *xi, double *w)
{
    if (elem == OR_TET4 && n_q == 1) {
        xi[0] = xi[1] = xi[2] = 0.25;
        w[0] = 1.0 / 6.0;
        return OR_OK;
    }
    if (elem == OR_TET4 && n_q == 4) {
        const double s5 = sqrt(5.0);
        const double a = (5.0 + 3.0 * s5) / 20.0;
        const double b = (5.0 - s5) / 20.0;
        for (int q = 0; q < 4; ++q) {
            /* barycentric weights (l0, l1, l2, l3); xi = (l1, l2, l3) */
            for (int k = 0; k < 3; ++k)
                xi[3 * q + k] = (q == k + 1) ? a : b;
            w[q] = 1.0 / 24.0;
        }
        return OR_OK;
    }
    if (elem == OR_PRISM6 && n_q == 6) {
        const double tp[3][2] = {{2.0 / 3.0, 1.0 / 6.0}, {1.0 / 6.0, 2.0 / 3.0}, {1.0 / 6.0, 1.0 / 6.0}};
        const double g = 1.0 / sqrt(3.0);
        for (int t = 0; t < 3; ++t) {
            for (int l = 0; l < 2; ++l) {
                const int q = 2 * t + l;
                xi[3 * q + 0] = tp[t][0];
                xi[3 * q + 1] = tp[t][1];
                xi[3 * q + 2] = (l == 0) ? -g : g;
                w[q] = 1.0 / 6.0;
            }
        }
        return OR_OK;
    }
    return OR_EINVAL;
}

/* Reference shape functions at one point, exported for tests. */
int oracle_shape(int elem, const double *xi, double *phi, double *dphi)
{
    double p[6], d[6][3];
    if (elem == OR_TET4)
        tet4_shape(xi, p, d);
    else if (elem == OR_PRISM6)
        prism6_shape(xi, p, d);
    else
        return OR_EINVAL;
    for (int r = 0; r < n_shape(elem); ++r) {
        phi[r] = p[r];
        for (int k = 0; k < 3; ++k)
            dphi[3 * r + k] = d[r][k];
    }
    return OR_OK;
}

/* ------------------------------------------------------------------------
 * Coefficient functions (the paper's option of computing the coefficients
 * at the integration points from problem-dependent parameters, Sec. 2.3 and
 * Sec. 3.3). Parameters, for slot k: p[6k..6k+5] = alpha, beta, omega_x,
 * omega_y, omega_z, theta; the raw value at point x is
 *   alpha + beta sin(2 pi (omega . x) + theta).
 * If p[121] != 0, the diffusion block is then replaced by A A^T + p[120] I
 * with A[i][j] the raw value of slot 4(i+1)+1+j (symmetric positive
 * definite for p[120] > 0).
 * ---------------------------------------------------------------------- */
static double fn_raw(const double *p, int k, const double x[3])
{
    const double *a = p + 6 * k;
    const double two_pi = 6.283185307179586476925286766559;
    return a[0] + a[1] * sin(two_pi * (a[2] * x[0] + a[3] * x[1] + a[4] * x[2]) + a[5]);
}

static void fn_spd_diffusion(const double *p, double *par)
{
    if (p[121] == 0.0)
        return;
    double A[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            A[i][j] = par[4 * (i + 1) + 1 + j];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double c = 0.0;
            for (int m = 0; m < 3; ++m)
                c += A[i][m] * A[j][m];
            if (i == j)
                c += p[120];
            par[4 * (i + 1) + 1 + j] = c;
        }
}

/* ------------------------------------------------------------------------
 * The element loop.
 * ---------------------------------------------------------------------- */
typedef struct {
    int elem, kind, coef_mode;
    unsigned mask;
    const double *uniform;
    int64_t n_elem;
    const double *coords;
    int64_t ld;
    const double *coeffs;
    int64_t ldc;
    int n_q;
    const double *xi, *w;
    double *K, *F;
    int n_slots;
    int slot_col[OR_MAX_SLOTS]; /* compact column of each slot, -1 = uniform (or 0) */
    const double *fn; /* coefficient-function parameters (OR_FUNCTION) */
} job_t;

/* Jacobian terms at one point: J[i][k] = dx_i/dxi_k. Because the reference
 * derivatives of the shape functions sum to zero, x(xi) = X_0 + sum_r
 * phi_r(xi) (X_r - X_0) and J[i][k] = sum_r (X[r][i] - X[0][i]) dphi_r/dxi_k
 * exactly; forming J from these edge vectors instead of absolute coordinates
 * avoids cancellation on thin elements. det J by cofactor expansion along
 * row 0, inverse = adjugate / det. */
static void jacobian_terms(int ns, const double X[6][3], const double dphi[6][3],
                           double *det_out, double Jinv[3][3])
{
    double J[3][3];
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k) {
            double s = 0.0;
            for (int r = 0; r < ns; ++r)
                s += (X[r][i] - X[0][i]) * dphi[r][k];
            J[i][k] = s;
        }
    const double c00 = J[1][1] * J[2][2] - J[1][2] * J[2][1];
    const double c01 = J[1][2] * J[2][0] - J[1][0] * J[2][2];
    const double c02 = J[1][0] * J[2][1] - J[1][1] * J[2][0];
    const double det = J[0][0] * c00 + J[0][1] * c01 + J[0][2] * c02;
    /* adj[k][i] = cofactor[i][k] */
    double adj[3][3];
    adj[0][0] = c00;
    adj[1][0] = c01;
    adj[2][0] = c02;
    adj[0][1] = J[0][2] * J[2][1] - J[0][1] * J[2][2];
    adj[1][1] = J[0][0] * J[2][2] - J[0][2] * J[2][0];
    adj[2][1] = J[0][1] * J[2][0] - J[0][0] * J[2][1];
    adj[0][2] = J[0][1] * J[1][2] - J[0][2] * J[1][1];
    adj[1][2] = J[0][2] * J[1][0] - J[0][0] * J[1][2];
    adj[2][2] = J[0][0] * J[1][1] - J[0][1] * J[1][0];
    for (int k = 0; k < 3; ++k)
        for (int i = 0; i < 3; ++i)
            Jinv[k][i] = adj[k][i] / det;
    *det_out = det;
}

static double kd(int a, int b) { return a == b ? 1.0 : 0.0; }

/* What the integrands of eqs. "sm_local" and "lv_local" need at one point of
 * the rule, after the change of variables (eq. "change_of_variables"): the
 * factor vol = det J(xi_q) w_q of the quadrature sum (eq. "quadrature", det J
 * signed), the physical point x(xi_q), and for every shape function r the
 * 4-vector Phi_r = (phi_r, d phi_r/dx, d phi_r/dy, d phi_r/dz), the global
 * derivatives being J^{-T} times the reference ones. */
typedef struct {
    double vol;
    double x[3];
    double Phi[6][4];
} point_t;

static void point_values(int elem, const double X[6][3], const double xi[3], double w,
                         point_t *pt)
{
    const int ns = n_shape(elem);
    double ph[6], dph[6][3], Jinv[3][3], det;
    if (elem == OR_TET4)
        tet4_shape(xi, ph, dph);
    else
        prism6_shape(xi, ph, dph);
    jacobian_terms(ns, X, dph, &det, Jinv);
    pt->vol = det * w;
    for (int i = 0; i < 3; ++i) {
        pt->x[i] = 0.0;
        for (int r = 0; r < ns; ++r)
            pt->x[i] += ph[r] * X[r][i];
    }
    for (int r = 0; r < ns; ++r) {
        pt->Phi[r][0] = ph[r];
        for (int i = 0; i < 3; ++i) {
            double g = 0.0;
            for (int k = 0; k < 3; ++k)
                g += dph[r][k] * Jinv[k][i];
            pt->Phi[r][1 + i] = g;
        }
    }
}

/* The coefficients of the weak form (eq. "weak_form") at one point, as
 * c[a][b][alpha][beta] and d[a][alpha] over the derivative indices a, b
 * (0: the function, 1..3: x, y, z) and the components alpha, beta of the
 * test and trial functions. Scalar problems use component 0 only. */
typedef struct {
    double c[4][4][3][3];
    double d[4][3];
} coef_t;

/* Slot values at point q of element e: read from memory (per element or per
 * point), computed from the coefficient function at x, or the uniform
 * values. */
static void slot_values(const job_t *jb, int64_t e, int q, const double x[3], double *par)
{
    for (int k = 0; k < jb->n_slots; ++k) {
        const int j = jb->slot_col[k];
        double v = (jb->kind == OR_VECTOR) ? 0.0 : jb->uniform[k];
        if (j >= 0) {
            if (jb->coef_mode == OR_FUNCTION)
                v = fn_raw(jb->fn, k, x);
            else if (jb->coef_mode == OR_PER_QP)
                v = jb->coeffs[((int64_t)j * jb->n_q + q) * jb->ldc + e];
            else
                v = jb->coeffs[(int64_t)j * jb->ldc + e];
        }
        par[k] = v;
    }
    if (jb->coef_mode == OR_FUNCTION)
        fn_spd_diffusion(jb->fn, par);
}

static void coefficients(const job_t *jb, const double *p, coef_t *cf)
{
    memset(cf, 0, sizeof(*cf));
    if (jb->kind == OR_SCALAR) {
        for (int a = 0; a < 4; ++a) {
            for (int b = 0; b < 4; ++b)
                cf->c[a][b][0][0] = p[4 * a + b];
            cf->d[a][0] = p[16 + a];
        }
    } else if (jb->kind == OR_VECTOR) {
        for (int a = 0; a < 4; ++a)
            for (int b = 0; b < 4; ++b)
                for (int al = 0; al < 3; ++al)
                    for (int be = 0; be < 3; ++be)
                        cf->c[a][b][al][be] = p[(4 * a + b) * 9 + 3 * al + be];
        for (int a = 0; a < 4; ++a)
            for (int al = 0; al < 3; ++al)
                cf->d[a][al] = p[144 + 3 * a + al];
    } else {
        /* isotropic elasticity: only the derivative-derivative terms, the
         * tensor of (i, alpha), (j, beta) with i = a - 1, j = b - 1 */
        const double E = p[0], nu = p[1];
        const double lambda = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu));
        const double mu = E / (2.0 * (1.0 + nu));
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j)
                for (int al = 0; al < 3; ++al)
                    for (int be = 0; be < 3; ++be)
                        cf->c[1 + i][1 + j][al][be] =
                            lambda * kd(i, al) * kd(j, be) +
                            mu * (kd(i, j) * kd(al, be) + kd(i, be) * kd(j, al));
        for (int al = 0; al < 3; ++al)
            cf->d[0][al] = p[2 + al];
    }
}

/* The integrand of eq. "sm_local" for test function (r, alpha) and trial
 * function (s, beta): sum over a, b of c^{a;b}_{alpha beta} Phi_r[a] Phi_s[b]. */
static double stiffness_integrand(const coef_t *cf, const double Phi_r[4], const double Phi_s[4],
                                  int al, int be)
{
    double v = 0.0;
    for (int a = 0; a < 4; ++a)
        for (int b = 0; b < 4; ++b)
            v += cf->c[a][b][al][be] * Phi_r[a] * Phi_s[b];
    return v;
}

/* The integrand of eq. "lv_local" for test function (r, alpha): sum over a of
 * d^a_alpha Phi_r[a]. */
static double load_integrand(const coef_t *cf, const double Phi_r[4], int al)
{
    double v = 0.0;
    for (int a = 0; a < 4; ++a)
        v += cf->d[a][al] * Phi_r[a];
    return v;
}

/* K and F of element e: the quadrature sums over the rule's points of vol
 * times the integrands, for every unknown (r, alpha), number 3 r + alpha
 * (r for scalar problems). */
static void integrate_element(const job_t *jb, int64_t e)
{
    const int ns = n_shape(jb->elem);
    const int nc = (jb->kind == OR_SCALAR) ? 1 : 3;
    const int N = ns * nc;
    double *Ke = jb->K + (size_t)e * N * N;
    double *Fe = jb->F + (size_t)e * N;

    double X[6][3];
    for (int v = 0; v < ns; ++v)
        for (int d = 0; d < 3; ++d)
            X[v][d] = jb->coords[(int64_t)(v * 3 + d) * jb->ld + e];
    for (int i = 0; i < N * N; ++i)
        Ke[i] = 0.0;
    for (int i = 0; i < N; ++i)
        Fe[i] = 0.0;

    for (int q = 0; q < jb->n_q; ++q) {
        point_t pt;
        point_values(jb->elem, X, &jb->xi[3 * q], jb->w[q], &pt);
        double par[OR_MAX_SLOTS];
        slot_values(jb, e, q, pt.x, par);
        coef_t cf;
        coefficients(jb, par, &cf);
        for (int r = 0; r < ns; ++r)
            for (int al = 0; al < nc; ++al) {
                const int row = nc * r + al;
                for (int s = 0; s < ns; ++s)
                    for (int be = 0; be < nc; ++be)
                        Ke[row * N + nc * s + be] +=
                            pt.vol * stiffness_integrand(&cf, pt.Phi[r], pt.Phi[s], al, be);
                Fe[row] += pt.vol * load_integrand(&cf, pt.Phi[r], al);
            }
    }
}

typedef struct {
    const job_t *jb;
    int64_t e0, e1;
    int status;
} range_t;

static void *run_range(void *arg)
{
    range_t *rg = (range_t *)arg;
    for (int64_t e = rg->e0; e < rg->e1; ++e)
        integrate_element(rg->jb, e);
    rg->status = OR_OK;
    return NULL;
}

/* Integrate n_elem elements; see the header comment for layouts. n_threads
 * workers each take one contiguous range of elements. */
int oracle_integrate(int elem, int kind, int coef_mode, unsigned mask, const double *uniform,
                     int64_t n_elem, const double *coords, int64_t ld, const double *coeffs,
                     int64_t ldc, int n_q, const double *xi, const double *w, double *K,
                     double *F, int n_threads)
{
    if ((elem != OR_TET4 && elem != OR_PRISM6) ||
        (kind != OR_SCALAR && kind != OR_ELASTICITY && kind != OR_VECTOR) ||
        coef_mode < OR_UNIFORM || coef_mode > OR_FUNCTION || n_elem < 0 || n_q < 1 || !uniform ||
        !xi || !w)
        return OR_EINVAL;
    if (kind == OR_VECTOR && coef_mode != OR_PER_ELEMENT && coef_mode != OR_PER_QP)
        return OR_EINVAL;
    if (n_elem == 0)
        return OR_OK;
    if (!coords || !K || !F || ld < n_elem)
        return OR_EINVAL;
    job_t jb;
    memset(&jb, 0, sizeof(jb));
    jb.elem = elem;
    jb.kind = kind;
    jb.coef_mode = coef_mode;
    int col = 0;
    if (kind == OR_VECTOR) {
        /* one mask bit per block of slots */
        jb.n_slots = OR_MAX_SLOTS;
        jb.mask = mask & 0xFFFFFu;
        for (int k = 0; k < OR_MAX_SLOTS; ++k) {
            const int block = (k < 144) ? k / 9 : 16 + (k - 144) / 3;
            jb.slot_col[k] = (jb.mask >> block & 1u) ? col++ : -1;
        }
    } else {
        jb.n_slots = (kind == OR_SCALAR) ? 20 : 5;
        jb.mask = (coef_mode == OR_UNIFORM) ? 0u : (mask & ((1u << jb.n_slots) - 1u));
        for (int k = 0; k < jb.n_slots; ++k)
            jb.slot_col[k] = (jb.mask >> k & 1u) ? col++ : -1;
    }
    if (coef_mode == OR_FUNCTION) {
        if (kind != OR_SCALAR || (col > 0 && !coeffs))
            return OR_EINVAL;
        jb.fn = coeffs;
    } else if (col > 0 && (!coeffs || ldc < n_elem)) {
        return OR_EINVAL;
    }
    jb.uniform = uniform;
    jb.n_elem = n_elem;
    jb.coords = coords;
    jb.ld = ld;
    jb.coeffs = coeffs;
    jb.ldc = ldc;
    jb.n_q = n_q;
    jb.xi = xi;
    jb.w = w;
    jb.K = K;
    jb.F = F;

    if (n_threads < 1)
        n_threads = 1;
    if (n_threads > 256)
        n_threads = 256;
    if ((int64_t)n_threads > n_elem)
        n_threads = (int)n_elem;
    range_t rg[256];
    pthread_t th[256];
    for (int t = 0; t < n_threads; ++t) {
        rg[t].jb = &jb;
        rg[t].e0 = n_elem * t / n_threads;
        rg[t].e1 = n_elem * (t + 1) / n_threads;
        rg[t].status = OR_OK;
    }
    if (n_threads == 1) {
        run_range(&rg[0]);
        return rg[0].status;
    }
    int started = 0;
    for (int t = 0; t < n_threads; ++t) {
        if (pthread_create(&th[t], NULL, run_range, &rg[t]) != 0) {
            run_range(&rg[t]);
            th[t] = 0;
        } else {
            ++started;
        }
    }
    int status = OR_OK;
    for (int t = 0; t < n_threads; ++t) {
        if (th[t])
            pthread_join(th[t], NULL);
        if (rg[t].status != OR_OK)
            status = rg[t].status;
    }
    (void)started;
    return status;
}

/* ------------------------------------------------------------------------
 * A second, independent route for isotropic elasticity: K += vol B^T D B in
 * Voigt notation (strain order xx, yy, zz, yz, xz, xy with engineering
 * shears), D from lambda and mu; F_(r,alpha) += vol f_alpha phi_r. Used only
 * to pin the tensor form of the main loop. Same layouts and outputs as
 * oracle_integrate with kind = elasticity.
 * ---------------------------------------------------------------------- */
int oracle_elasticity_voigt(int elem, int coef_mode, unsigned mask, const double *uniform,
                            int64_t n_elem, const double *coords, int64_t ld, const double *coeffs,
                            int64_t ldc, int n_q, const double *xi, const double *w, double *K,
                            double *F)
{
    if ((elem != OR_TET4 && elem != OR_PRISM6) || n_elem < 0 || n_q < 1 || !uniform || !xi || !w)
        return OR_EINVAL;
    const int ns = n_shape(elem);
    const int N = 3 * ns;
    int slot_col[5];
    int col = 0;
    for (int k = 0; k < 5; ++k)
        slot_col[k] = (coef_mode != OR_UNIFORM && (mask >> k & 1u)) ? col++ : -1;
    for (int64_t e = 0; e < n_elem; ++e) {
        double X[6][3];
        for (int v = 0; v < ns; ++v)
            for (int d = 0; d < 3; ++d)
                X[v][d] = coords[(int64_t)(v * 3 + d) * ld + e];
        double *Ke = K + (size_t)e * N * N;
        double *Fe = F + (size_t)e * N;
        memset(Ke, 0, sizeof(double) * N * N);
        memset(Fe, 0, sizeof(double) * N);
        for (int q = 0; q < n_q; ++q) {
            double p[5];
            for (int k = 0; k < 5; ++k) {
                p[k] = uniform[k];
                if (slot_col[k] >= 0)
                    p[k] = (coef_mode == OR_PER_QP)
                               ? coeffs[((int64_t)slot_col[k] * n_q + q) * ldc + e]
                               : coeffs[(int64_t)slot_col[k] * ldc + e];
            }
            const double lambda = p[0] * p[1] / ((1.0 + p[1]) * (1.0 - 2.0 * p[1]));
            const double mu = p[0] / (2.0 * (1.0 + p[1]));
            double D[6][6];
            memset(D, 0, sizeof(D));
            for (int i = 0; i < 3; ++i) {
                for (int j = 0; j < 3; ++j)
                    D[i][j] = lambda;
                D[i][i] = lambda + 2.0 * mu;
                D[3 + i][3 + i] = mu;
            }
            double ph[6], dph[6][3], Jinv[3][3], det;
            if (elem == OR_TET4)
                tet4_shape(&xi[3 * q], ph, dph);
            else
                prism6_shape(&xi[3 * q], ph, dph);
            jacobian_terms(ns, X, dph, &det, Jinv);
            const double vol = det * w[q];
            double B[6][18];
            memset(B, 0, sizeof(B));
            for (int r = 0; r < ns; ++r) {
                double g[3];
                for (int i = 0; i < 3; ++i) {
                    g[i] = 0.0;
                    for (int k = 0; k < 3; ++k)
                        g[i] += dph[r][k] * Jinv[k][i];
                }
                B[0][3 * r + 0] = g[0];
                B[1][3 * r + 1] = g[1];
                B[2][3 * r + 2] = g[2];
                B[3][3 * r + 1] = g[2];
                B[3][3 * r + 2] = g[1];
                B[4][3 * r + 0] = g[2];
                B[4][3 * r + 2] = g[0];
                B[5][3 * r + 0] = g[1];
                B[5][3 * r + 1] = g[0];
            }
            double DB[6][18];
            for (int i = 0; i < 6; ++i)
                for (int c = 0; c < N; ++c) {
                    double s = 0.0;
                    for (int k = 0; k < 6; ++k)
                        s += D[i][k] * B[k][c];
                    DB[i][c] = s;
                }
            for (int a = 0; a < N; ++a)
                for (int c = 0; c < N; ++c) {
                    double s = 0.0;
                    for (int k = 0; k < 6; ++k)
                        s += B[k][a] * DB[k][c];
                    Ke[a * N + c] += vol * s;
                }
            for (int r = 0; r < ns; ++r)
                for (int al = 0; al < 3; ++al)
                    Fe[3 * r + al] += vol * p[2 + al] * ph[r];
        }
    }
    return OR_OK;
}
