/*
 * Driver for the sanitizer test of the CPU oracle (test infrastructure):
 * built together with oracle/bfsft_oracle.c under AddressSanitizer and
 * UndefinedBehaviorSanitizer, it runs the direct sum (eq. (1)) and the
 * butterfly of Section 2.2 on small 2D and 3D problems that reach every code
 * path the tests use (start levels, level dumps, N not a power of two,
 * points on box faces and at x = N, empty and single-point sets), and checks
 * that the butterfly matches the direct sum at the accuracy of its p.  Any
 * memory error or undefined behaviour aborts the run.  Exit status 0: all
 * checks passed.
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

void or_direct(int d, double N, const double *x, const double *k, const double *f, int64_t nk,
               const int64_t *idx, int64_t ns, double *u);
void *or_bf_create(int d, int64_t N, int p, const double *x, int64_t nx, const double *k, int64_t nk);
void or_bf_destroy(void *h);
int or_bf_levels(void *h);
int64_t or_bf_count(void *h, int side, int m);
void or_bf_boxes(void *h, int side, int m, int64_t *coords);
void or_bf_matrix_M(void *h, int64_t iA, int64_t iB, double *out);
void or_bf_matrix_E(void *h, int64_t iA, int64_t ic, double *out);
int or_bf_run(void *h, const double *f_in, double *u_out, int dump_level, double *dump_u, double *dump_f,
              int start);

static uint64_t rng = 88172645463325252ull;
static double uniform(void)
{
    rng ^= rng << 13;
    rng ^= rng >> 7;
    rng ^= rng << 17;
    return (double)(rng >> 11) * (1.0 / 9007199254740992.0);
}

/* points on a circle (2D) or a sphere (3D) of radius r about the centre, scaled by N */
static double *curve(int d, int n, double N, double r)
{
    double *x = malloc(sizeof(double) * (size_t)(n > 0 ? n : 1) * d);
    for (int i = 0; i < n; ++i) {
        const double t = 2.0 * M_PI * (i + 0.5) / n;
        if (d == 2) {
            x[2 * i] = N * (0.5 + r * cos(t));
            x[2 * i + 1] = N * (0.5 + r * sin(t));
        } else {
            const double z = 1.0 - (2.0 * i + 1.0) / n, s = sqrt(1.0 - z * z), ph = i * M_PI * (3.0 - sqrt(5.0));
            x[3 * i] = N * (0.5 + r * s * cos(ph));
            x[3 * i + 1] = N * (0.5 + r * s * sin(ph));
            x[3 * i + 2] = N * (0.5 + r * z);
        }
    }
    return x;
}

static int failures = 0;

/* butterfly at start levels 0 .. smax (with a dump of every level at start
 * 0) against the direct sum: relative l2 within tol */
static void check(const char *name, int d, int64_t N, int p, const double *x, int nx, const double *k, int nk,
                  int smax, double tol)
{
    double *f = malloc(sizeof(double) * 2 * (size_t)(nk > 0 ? nk : 1));
    for (int j = 0; j < 2 * nk; ++j) f[j] = uniform() - 0.5;
    double *ud = calloc(2 * (size_t)(nx > 0 ? nx : 1), sizeof(double));
    double *ub = calloc(2 * (size_t)(nx > 0 ? nx : 1), sizeof(double));
    int64_t *idx = malloc(sizeof(int64_t) * (size_t)(nx > 0 ? nx : 1));
    for (int i = 0; i < nx; ++i) idx[i] = i;
    or_direct(d, (double)N, x, k, f, nk, idx, nx, ud);
    void *h = or_bf_create(d, N, p, x, nx, k, nk);
    if (!h) {
        printf("%s: create failed\n", name);
        ++failures;
        return;
    }
    const int L = or_bf_levels(h);
    for (int m = 0; m <= L; ++m)
        for (int side = 0; side < 2; ++side) {
            const int64_t c = or_bf_count(h, side, m);
            int64_t *co = malloc(sizeof(int64_t) * (size_t)(c > 0 ? c : 1) * d);
            or_bf_boxes(h, side, m, co);
            free(co);
        }
    double M[2 * 16 * 16];
    or_bf_matrix_M(h, 1, 2, M);
    or_bf_matrix_E(h, 1, 3, M);
    for (int s0 = 0; s0 <= smax && s0 <= L; ++s0) {
        for (int lvl = (s0 == 0 ? 0 : -1); lvl <= (s0 == 0 ? L : -1); ++lvl) {
            double *du = NULL, *df = NULL;
            if (lvl >= 0 && nx > 0 && nk > 0) {
                int64_t pd = 1;
                for (int a = 0; a < d; ++a) pd *= p;
                const int64_t n = or_bf_count(h, 0, L - lvl) * or_bf_count(h, 1, lvl) * pd;
                du = malloc(sizeof(double) * 2 * (size_t)(n > 0 ? n : 1));
                df = malloc(sizeof(double) * 2 * (size_t)(n > 0 ? n : 1));
            }
            const int rc = or_bf_run(h, f, ub, du ? lvl : -1, du, df, s0);
            free(du);
            free(df);
            double num = 0, den = 0;
            for (int i = 0; i < 2 * nx; ++i) {
                num += (ub[i] - ud[i]) * (ub[i] - ud[i]);
                den += ud[i] * ud[i];
            }
            const double err = den > 0 ? sqrt(num / den) : sqrt(num);
            if (rc != 0 || !(err <= tol)) {
                printf("%s: start %d dump %d: rc %d err %.3e > %.1e\n", name, s0, lvl, rc, err, tol);
                ++failures;
            }
        }
    }
    or_bf_destroy(h);
    free(f);
    free(ud);
    free(ub);
    free(idx);
}

int main(void)
{
    /* 2D, N a power of two, p = 5 and 9 */
    double *x = curve(2, 160, 64.0, 0.4), *k = curve(2, 130, 64.0, 0.3);
    check("2d N=64 p=5", 2, 64, 5, x, 160, k, 130, 3, 1e-2);
    check("2d N=64 p=9", 2, 64, 9, x, 160, k, 130, 2, 1e-6);
    free(x);
    free(k);
    /* 2D, N not a power of two (leaf width rho < 1), p = 7 */
    x = curve(2, 300, 77.0, 0.45);
    k = curve(2, 250, 77.0, 0.35);
    check("2d N=77 p=7", 2, 77, 7, x, 300, k, 250, 2, 1e-3);
    free(x);
    free(k);
    /* 2D, points on box faces and at x = N */
    double g[2 * 81];
    for (int i = 0; i < 9; ++i)
        for (int j = 0; j < 9; ++j) {
            g[2 * (9 * i + j)] = 4.0 * i;
            g[2 * (9 * i + j) + 1] = 4.0 * j;
        }
    check("2d faces N=32", 2, 32, 6, g, 81, g, 81, 2, 1e-3);
    /* single points, empty sets */
    check("2d one source", 2, 32, 5, g, 81, g + 2 * 40, 1, 1, 1e-2);
    check("2d no sources", 2, 32, 5, g, 81, g, 0, 0, 1e-300);
    check("2d no targets", 2, 32, 5, g, 0, g, 81, 0, 1e-300);
    /* 3D */
    x = curve(3, 200, 8.0, 0.4);
    k = curve(3, 150, 8.0, 0.3);
    check("3d N=8 p=4", 3, 8, 4, x, 200, k, 150, 2, 3e-2);
    free(x);
    free(k);
    x = curve(3, 120, 6.0, 0.4);
    k = curve(3, 100, 6.0, 0.3);
    check("3d N=6 p=5", 3, 6, 5, x, 120, k, 100, 1, 1e-2);
    free(x);
    free(k);
    printf("%s (%d failures)\n", failures ? "FAILED" : "all checks passed", failures);
    return failures ? 1 : 0;
}
