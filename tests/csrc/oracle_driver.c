/* Drives every entry point of the oracle over small fixed meshes, in one and
 * in several threads, for the sanitizer builds (address and undefined
 * behaviour; data races). Exit status = number of failures. Test
 * infrastructure only. */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

int oracle_quad_rule(int elem, int n_q, double *xi, double *w);
int oracle_integrate(int elem, int kind, int coef_mode, unsigned mask, const double *uniform,
                     int64_t n_elem, const double *coords, int64_t ld, const double *coeffs,
                     int64_t ldc, int n_q, const double *xi, const double *w, double *K,
                     double *F, int n_threads);
int oracle_elasticity_voigt(int elem, int coef_mode, unsigned mask, const double *uniform,
                            int64_t n_elem, const double *coords, int64_t ld, const double *coeffs,
                            int64_t ldc, int n_q, const double *xi, const double *w, double *K,
                            double *F);

static uint64_t g_state = 88172645463325252ull;
static double rnd(void) /* xorshift64, uniform in [0, 1) */
{
    g_state ^= g_state << 13;
    g_state ^= g_state >> 7;
    g_state ^= g_state << 17;
    return (double)(g_state >> 11) / 9007199254740992.0;
}

int main(void)
{
    enum { NE = 37 };
    static const double tet[4][3] = {{0, 0, 0}, {1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
    static const double pri[6][3] = {{0, 0, -1}, {1, 0, -1}, {0, 1, -1}, {0, 0, 1}, {1, 0, 1}, {0, 1, 1}};
    int failures = 0;
    for (int elem = 0; elem < 2; ++elem) {
        const int nv = elem ? 6 : 4, nq = elem ? 6 : 4;
        double *coords = malloc(sizeof(double) * nv * 3 * NE);
        for (int e = 0; e < NE; ++e)
            for (int v = 0; v < nv; ++v)
                for (int d = 0; d < 3; ++d)
                    coords[(v * 3 + d) * NE + e] = (elem ? pri[v][d] : tet[v][d]) + 0.1 * (rnd() - 0.5);
        double xi[8 * 3], w[8];
        if (oracle_quad_rule(elem, nq, xi, w) != 0)
            ++failures;
        for (int kind = 0; kind < 3; ++kind) {
            const int N = nv * (kind ? 3 : 1);
            for (int mode = 0; mode < 4; ++mode) {
                if (kind == 2 && (mode == 0 || mode == 3))
                    continue;                      /* per element or per point only */
                if (kind == 1 && mode == 3)
                    continue;                      /* coefficient functions: scalar */
                const unsigned mask = kind == 1 ? 31u : 0xFFFFFu;
                int rows = kind == 0 ? 20 : (kind == 1 ? 5 : 156);
                if (mode == 2)
                    rows *= nq;
                const int64_t nc = mode == 3 ? 122 : (int64_t)rows * NE;
                double *coeffs = malloc(sizeof(double) * nc);
                for (int64_t i = 0; i < nc; ++i)
                    coeffs[i] = kind == 1 ? 0.2 + 0.2 * rnd() : rnd() - 0.5;
                if (mode == 3)
                    coeffs[121] = 1.0;
                double uniform[20];
                for (int k = 0; k < 20; ++k)
                    uniform[k] = rnd();
                uniform[1] = 0.3;
                double *K1 = malloc(sizeof(double) * N * N * NE), *F1 = malloc(sizeof(double) * N * NE);
                double *K4 = malloc(sizeof(double) * N * N * NE), *F4 = malloc(sizeof(double) * N * NE);
                const unsigned m = mode == 0 ? 0u : mask;
                int st = oracle_integrate(elem, kind, mode, m, uniform, NE, coords, NE,
                                          mode == 0 ? NULL : coeffs, NE, nq, xi, w, K1, F1, 1);
                st |= oracle_integrate(elem, kind, mode, m, uniform, NE, coords, NE,
                                       mode == 0 ? NULL : coeffs, NE, nq, xi, w, K4, F4, 4);
                if (st) {
                    fprintf(stderr, "elem %d kind %d mode %d: status %d\n", elem, kind, mode, st);
                    ++failures;
                }
                if (memcmp(K1, K4, sizeof(double) * N * N * NE) || memcmp(F1, F4, sizeof(double) * N * NE)) {
                    fprintf(stderr, "elem %d kind %d mode %d: threads change the result\n", elem, kind, mode);
                    ++failures;
                }
                for (int64_t i = 0; i < (int64_t)N * N * NE; ++i)
                    if (!isfinite(K1[i])) {
                        ++failures;
                        break;
                    }
                if (kind == 1 && mode < 3 &&
                    oracle_elasticity_voigt(elem, mode, m, uniform, NE, coords, NE,
                                            mode == 0 ? NULL : coeffs, NE, nq, xi, w, K4, F4))
                    ++failures;
                free(coeffs);
                free(K1);
                free(F1);
                free(K4);
                free(F4);
            }
        }
        free(coords);
    }
    printf("oracle driver: %d failures\n", failures);
    return failures;
}
