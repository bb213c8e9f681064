/*
 * CPU ORACLE for the butterfly sparse Fourier transform.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, calls or
 * includes this file; only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark load it.  It shares no code, header, table or
 * helper with the GPU path.
 *
 * Paper: L. Ying, "Sparse Fourier Transform via Butterfly Algorithm" (2007).
 *
 * Two parts:
 *   O1  or_direct     - eq. (1) of Section 1 written out: u_i = sum_j
 *                       exp(2 pi i x_i.k_j / N) f_j, in FP64, with the phase
 *                       x_i.k_j / N reduced modulo 1 in double-double.
 *   O2  or_bf_*       - the butterfly algorithm of Section 2.2 (steps 1-4),
 *                       f-form (equivalent charges), in the paper's
 *                       order: check potentials u^{AB} are evaluated from the
 *                       children's charges with E = E1 (x) E2 (Section 2.1,
 *                       eq. E1), then f^{AB} = M^{-1} u^{AB} with
 *                       M = M1 (x) M2 (Section 2.1, eq. M1).  The diagonal
 *                       factors of eqs. (M1) and (E1) are evaluated from exact
 *                       rational phases: with box corners c = i w, every
 *                       phase is an integer multiple of rho/(q 2^k), reduced
 *                       modulo 1 in 128-bit integers before one sin/cos.
 *                       G^{-1} is applied by an LU solve with partial
 *                       pivoting.  The butterfly's arithmetic (phases,
 *                       solves, products, sums) is x87 long double: in the
 *                       f-form the charges inherit the conditioning of G
 *                       (about 3e8 at p = 9, 5e11 at p = 11, 1e13 at p = 12)
 *                       and FP64 loses field accuracy from p = 11 on.
 *
 * Readings where the paper is silent (they are shared with the GPU library by
 * specification, not by code):
 *   - N need not be a power of two: L = ceil(log2 N), leaf width
 *     rho = N / 2^L, so paired boxes satisfy w^A w^B = rho N <= N.
 *   - a point's leaf index along an axis is floor(x * 2^L / N) in IEEE FP64
 *     (the product by 2^L is exact), clamped to [0, 2^L - 1]; the index at
 *     level m is that leaf index shifted right by L - m (half-open boxes).
 *   - p^d tensors are stored row-major [l1][l2][l3] with axis 1 slowest;
 *     (M1 (x) M2) vec(F) = M1 F M2^T (plain transpose).
 *   - the sign of the exponent is + (eq. 1).
 *   - step 4 is read as u_i for x_i in the T_X leaf A (the paper's u_j, x_j
 *     are a typo).
 */
#define _GNU_SOURCE
#include <complex.h>
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef long double complex cplx;   /* butterfly (O2) */
typedef double complex dcplx;       /* direct sum (O1) */
typedef unsigned __int128 u128;

#define OR_PMAX 16

/* ------------------------------------------------------------------------- */
/* exponentials                                                               */
/* ------------------------------------------------------------------------- */

/* exp(2 pi i t) for t given in turns */
static cplx expi_turns(long double t)
{
    t -= nearbyintl(t);
    long double s, c;
    sincosl(2.0L * M_PIl * t, &s, &c);
    return CMPLXL(c, s);
}

/* the same in FP64, for the direct sum */
static dcplx expi_turns_d(double t)
{
    t -= nearbyint(t);
    double s, c;
    sincos(2.0 * M_PI * t, &s, &c);
    return CMPLX(c, s);
}

/* exp(2 pi i a rho / b) with rho = N / 2^L, a >= 0, b >= 1: the numerator
 * a*N is reduced modulo b*2^L in exact integer arithmetic. */
static cplx expi_rational(uint64_t a, uint64_t b, int64_t N, int L)
{
    u128 num = (u128)a * (u128)(uint64_t)N;
    u128 den = (u128)b << L;
    u128 r = num % den;
    return expi_turns((long double)(uint64_t)r / (long double)(uint64_t)den);
}

/* double-double helpers for O1 and for phases of arbitrary coordinates */
typedef struct { double hi, lo; } dd_t;

static inline dd_t two_prod(double a, double b)
{
    double p = a * b;
    return (dd_t){p, fma(a, b, -p)};
}

static inline dd_t two_sum(double a, double b)
{
    double s = a + b;
    double bb = s - a;
    return (dd_t){s, (a - (s - bb)) + (b - bb)};
}

static inline dd_t dd_add(dd_t a, dd_t b)
{
    dd_t s = two_sum(a.hi, b.hi);
    double lo = s.lo + a.lo + b.lo;
    return two_sum(s.hi, lo);
}

static inline dd_t dd_div(dd_t a, double b)
{
    double q1 = a.hi / b;
    dd_t pr = two_prod(q1, b);
    double r = ((a.hi - pr.hi) - pr.lo) + a.lo;
    return two_sum(q1, r / b);
}

/* exp(2 pi i t) for t = hi + lo given in turns */
static cplx expi_dd(dd_t t)
{
    double n = nearbyint(t.hi);
    return expi_turns((long double)(t.hi - n) + (long double)t.lo);
}

static dcplx expi_dd_d(dd_t t)
{
    double n = nearbyint(t.hi);
    return expi_turns_d((t.hi - n) + t.lo);
}

/* ------------------------------------------------------------------------- */
/* O1: direct evaluation of eq. (1)                                           */
/* ------------------------------------------------------------------------- */

/* u[s] = sum_j exp(2 pi i x_{idx[s]} . k_j / N) f_j, s = 0..ns-1.
 * x: [nx][d], k: [nk][d], f: [nk] complex (interleaved re, im), u: [ns]. */
void or_direct(int d, double N, const double *x, const double *k,
               const double *f, int64_t nk, const int64_t *idx, int64_t ns,
               double *u)
{
    const dcplx *fc = (const dcplx *)f;
    dcplx *uc = (dcplx *)u;
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t s = 0; s < ns; ++s) {
        const double *xi = x + idx[s] * d;
        dcplx acc = 0;
        for (int64_t j = 0; j < nk; ++j) {
            const double *kj = k + j * d;
            dd_t t = two_prod(xi[0], kj[0]);
            for (int a = 1; a < d; ++a)
                t = dd_add(t, two_prod(xi[a], kj[a]));
            acc += expi_dd_d(dd_div(t, N)) * fc[j];
        }
        uc[s] = acc;
    }
}

/* ------------------------------------------------------------------------- */
/* O2: trees (step 1)                                                          */
/* ------------------------------------------------------------------------- */

typedef struct {
    int64_t n;           /* non-empty boxes at this level */
    uint64_t *key;       /* sorted lexicographic keys (axis 1 most significant) */
} or_level;

typedef struct {
    int d, p, q, L;
    int64_t N;
    int64_t nx, nk;
    double *x, *k;               /* copies, [n][d] */
    or_level *tx, *tk;           /* [L+1] each */
    int64_t *xperm, *xbeg;       /* targets sorted by leaf; leaf a owns xperm[xbeg[a]..xbeg[a+1]) */
    int64_t *kperm, *kbeg;       /* sources sorted by leaf */
    cplx G[OR_PMAX * OR_PMAX];   /* G_rho, eq. (M1) centre factor */
    cplx H[OR_PMAX * OR_PMAX];   /* H_rho, eq. (E1) centre factor */
    cplx GLU[OR_PMAX * OR_PMAX]; /* LU factors of G with row pivots */
    int piv[OR_PMAX];
} or_plan;

static uint64_t box_key(const int64_t *idx, int d, int m)
{
    uint64_t key = 0;
    for (int a = 0; a < d; ++a)
        key = (key << m) | (uint64_t)idx[a];
    return key;
}

static void key_coords(uint64_t key, int d, int m, int64_t *idx)
{
    uint64_t mask = (m >= 64) ? ~0ull : ((1ull << m) - 1ull);
    for (int a = d - 1; a >= 0; --a) {
        idx[a] = (int64_t)(key & mask);
        key >>= m;
    }
}

static void leaf_index(const double *pt, int d, int64_t N, int L, int64_t *idx)
{
    int64_t nleaf = (int64_t)1 << L;
    for (int a = 0; a < d; ++a) {
        double v = floor(ldexp(pt[a], L) / (double)N);
        int64_t i = (int64_t)v;
        if (v < 0) i = 0;
        if (i > nleaf - 1) i = nleaf - 1;
        idx[a] = i;
    }
}

static int cmp_u64(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x > y) - (x < y);
}

typedef struct { uint64_t key; int64_t id; } key_id;

static int cmp_key_id(const void *a, const void *b)
{
    const key_id *x = a, *y = b;
    if (x->key != y->key) return (x->key > y->key) - (x->key < y->key);
    return (x->id > y->id) - (x->id < y->id);
}

/* Non-empty boxes of every level for one point set, plus the points of each
 * leaf.  Level m holds boxes of width N / 2^m; a box's index at level m is
 * the leaf index shifted right by L - m. */
static void build_tree(const double *pts, int64_t n, int d, int64_t N, int L,
                       or_level *lv, int64_t **perm_out, int64_t **beg_out)
{
    int64_t *leaf = malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1) * d);
    for (int64_t i = 0; i < n; ++i)
        leaf_index(pts + i * d, d, N, L, leaf + i * d);

    uint64_t *tmp = malloc(sizeof(uint64_t) * (size_t)(n > 0 ? n : 1));
    for (int m = 0; m <= L; ++m) {
        for (int64_t i = 0; i < n; ++i) {
            int64_t idx[3];
            for (int a = 0; a < d; ++a) idx[a] = leaf[i * d + a] >> (L - m);
            tmp[i] = box_key(idx, d, m);
        }
        qsort(tmp, (size_t)n, sizeof(uint64_t), cmp_u64);
        int64_t u = 0;
        for (int64_t i = 0; i < n; ++i)
            if (i == 0 || tmp[i] != tmp[i - 1]) tmp[u++] = tmp[i];
        lv[m].n = u;
        lv[m].key = malloc(sizeof(uint64_t) * (size_t)(u > 0 ? u : 1));
        memcpy(lv[m].key, tmp, sizeof(uint64_t) * (size_t)u);
    }

    key_id *ki = malloc(sizeof(key_id) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i) {
        ki[i].key = box_key(leaf + i * d, d, L);
        ki[i].id = i;
    }
    qsort(ki, (size_t)n, sizeof(key_id), cmp_key_id);
    int64_t nl = lv[L].n;
    int64_t *perm = malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
    int64_t *beg = malloc(sizeof(int64_t) * (size_t)(nl + 1));
    int64_t b = 0;
    for (int64_t i = 0; i < n; ++i) {
        perm[i] = ki[i].id;
        if (i == 0 || ki[i].key != ki[i - 1].key) beg[b++] = i;
    }
    beg[nl] = n;
    *perm_out = perm;
    *beg_out = beg;
    free(ki);
    free(tmp);
    free(leaf);
}

/* index of `key` among the sorted keys of a level, or -1 */
static int64_t find_box(const or_level *lv, uint64_t key)
{
    int64_t lo = 0, hi = lv->n - 1;
    while (lo <= hi) {
        int64_t mid = lo + (hi - lo) / 2;
        if (lv->key[mid] == key) return mid;
        if (lv->key[mid] < key) lo = mid + 1; else hi = mid - 1;
    }
    return -1;
}

/* ------------------------------------------------------------------------- */
/* O2: per-axis operators of Section 2.1                                      */
/* ------------------------------------------------------------------------- */

/* Diagonal factors of eq. (M1) for a pair (A, B) with w^A w^B = rho N, box
 * indices iA, iB along one axis:
 *   (M1)_{ll'} = m11_l * G_{ll'} * m12_{l'},
 *   m11_l  = exp(2 pi i (c^A + l w^A/q) c^B / N) = exp(2 pi i (q iA + l) iB rho / q),
 *   m12_l' = exp(2 pi i c^A l' w^B / (q N))      = exp(2 pi i iA l' rho / q),
 *   G_ll'  = exp(2 pi i l l' rho / q^2).                                     */
static void m_diagonals(const or_plan *P, int64_t iA, int64_t iB, cplx *m11, cplx *m12)
{
    for (int l = 0; l < P->p; ++l) {
        m11[l] = expi_rational((uint64_t)(P->q * iA + l) * (uint64_t)iB, (uint64_t)P->q, P->N, P->L);
        m12[l] = expi_rational((uint64_t)iA * (uint64_t)l, (uint64_t)P->q, P->N, P->L);
    }
}

/* Diagonal factors of eq. (E1) for A and a child B_c (index ic) of B, with
 * w^A w^{B_c} = rho N / 2:
 *   (E1)_{ll'} = e11_l * H_{ll'} * e12_{l'},
 *   e11_l  = exp(2 pi i (q iA + l) ic rho / (2q)),
 *   e12_l' = exp(2 pi i iA l' rho / (2q)),
 *   H_ll'  = exp(2 pi i l l' rho / (2 q^2)).                                  */
static void e_diagonals(const or_plan *P, int64_t iA, int64_t ic, cplx *e11, cplx *e12)
{
    for (int l = 0; l < P->p; ++l) {
        e11[l] = expi_rational((uint64_t)(P->q * iA + l) * (uint64_t)ic, (uint64_t)(2 * P->q), P->N, P->L);
        e12[l] = expi_rational((uint64_t)iA * (uint64_t)l, (uint64_t)(2 * P->q), P->N, P->L);
    }
}

/* LU factorisation with partial pivoting of a p x p complex matrix (in place) */
static void lu_factor(cplx *A, int *piv, int p)
{
    for (int c = 0; c < p; ++c) {
        int r = c;
        long double best = cabsl(A[c * p + c]);
        for (int i = c + 1; i < p; ++i)
            if (cabsl(A[i * p + c]) > best) { best = cabsl(A[i * p + c]); r = i; }
        piv[c] = r;
        if (r != c)
            for (int j = 0; j < p; ++j) { cplx t = A[c * p + j]; A[c * p + j] = A[r * p + j]; A[r * p + j] = t; }
        for (int i = c + 1; i < p; ++i) {
            A[i * p + c] /= A[c * p + c];
            for (int j = c + 1; j < p; ++j) A[i * p + j] -= A[i * p + c] * A[c * p + j];
        }
    }
}

/* solve (LU) y = b in place, b of length p with stride s */
static void lu_solve(const cplx *LU, const int *piv, int p, cplx *b, int s)
{
    for (int c = 0; c < p; ++c)
        if (piv[c] != c) { cplx t = b[c * s]; b[c * s] = b[piv[c] * s]; b[piv[c] * s] = t; }
    for (int i = 1; i < p; ++i)
        for (int j = 0; j < i; ++j) b[i * s] -= LU[i * p + j] * b[j * s];
    for (int i = p - 1; i >= 0; --i) {
        for (int j = i + 1; j < p; ++j) b[i * s] -= LU[i * p + j] * b[j * s];
        b[i * s] /= LU[i * p + i];
    }
}

/* ------------------------------------------------------------------------- */
/* p^d tensor helpers: fibres along one axis                                  */
/* ------------------------------------------------------------------------- */

/* stride of axis a in a row-major p^d tensor */
static int axis_stride(int p, int d, int a)
{
    int s = 1;
    for (int b = d - 1; b > a; --b) s *= p;
    return s;
}

/* X <- A applied along axis a:  X[.., l, ..] = sum_l' A[l][l'] X[.., l', ..] */
static void mode_apply(cplx *X, const cplx *A, int p, int d, int a)
{
    int s = axis_stride(p, d, a);
    int P = 1;
    for (int b = 0; b < d; ++b) P *= p;
    cplx fib[OR_PMAX], out[OR_PMAX];
    for (int base = 0; base < P; ++base) {
        if ((base / s) % p != 0) continue;        /* base = start of a fibre */
        for (int l = 0; l < p; ++l) fib[l] = X[base + l * s];
        for (int l = 0; l < p; ++l) {
            cplx acc = 0;
            for (int m = 0; m < p; ++m) acc += A[l * p + m] * fib[m];
            out[l] = acc;
        }
        for (int l = 0; l < p; ++l) X[base + l * s] = out[l];
    }
}

/* X <- G^{-1} applied along axis a (LU solve per fibre) */
static void mode_solve(cplx *X, const or_plan *P, int a)
{
    int p = P->p, d = P->d;
    int s = axis_stride(p, d, a);
    int n = 1;
    for (int b = 0; b < d; ++b) n *= p;
    for (int base = 0; base < n; ++base) {
        if ((base / s) % p != 0) continue;
        lu_solve(P->GLU, P->piv, p, X + base, s);
    }
}

/* X[.., l, ..] *= v[l] along axis a */
static void mode_scale(cplx *X, const cplx *v, int p, int d, int a, int inverse)
{
    int s = axis_stride(p, d, a);
    int n = 1;
    for (int b = 0; b < d; ++b) n *= p;
    for (int i = 0; i < n; ++i) {
        int l = (i / s) % p;
        X[i] = inverse ? X[i] / v[l] : X[i] * v[l];
    }
}

/* f = M(A,B)^{-1} u  with M = (x)_axis diag(m11) G diag(m12)  (eq. M1) */
static void solve_matching(const or_plan *P, const int64_t *iA, const int64_t *iB, cplx *X)
{
    cplx m11[OR_PMAX], m12[OR_PMAX];
    for (int a = 0; a < P->d; ++a) {
        m_diagonals(P, iA[a], iB[a], m11, m12);
        mode_scale(X, m11, P->p, P->d, a, 1);
        mode_solve(X, P, a);
        mode_scale(X, m12, P->p, P->d, a, 1);
    }
}

/* ------------------------------------------------------------------------- */
/* O2: plan                                                                   */
/* ------------------------------------------------------------------------- */

static int ceil_log2(int64_t N)
{
    int L = 0;
    while (((int64_t)1 << L) < N) ++L;
    return L;
}

void *or_bf_create(int d, int64_t N, int p, const double *x, int64_t nx,
                   const double *k, int64_t nk)
{
    if (d < 1 || d > 3 || p < 2 || p > OR_PMAX || N < 2) return NULL;
    or_plan *P = calloc(1, sizeof(or_plan));
    P->d = d; P->p = p; P->q = p - 1; P->N = N; P->L = ceil_log2(N);
    P->nx = nx; P->nk = nk;
    P->x = malloc(sizeof(double) * (size_t)(nx > 0 ? nx : 1) * d);
    P->k = malloc(sizeof(double) * (size_t)(nk > 0 ? nk : 1) * d);
    memcpy(P->x, x, sizeof(double) * (size_t)nx * d);
    memcpy(P->k, k, sizeof(double) * (size_t)nk * d);
    P->tx = calloc((size_t)P->L + 1, sizeof(or_level));
    P->tk = calloc((size_t)P->L + 1, sizeof(or_level));
    build_tree(P->x, nx, d, N, P->L, P->tx, &P->xperm, &P->xbeg);
    build_tree(P->k, nk, d, N, P->L, P->tk, &P->kperm, &P->kbeg);
    int q = P->q;
    for (int l = 0; l < p; ++l)
        for (int m = 0; m < p; ++m) {
            P->G[l * p + m] = expi_rational((uint64_t)(l * m), (uint64_t)(q * q), N, P->L);
            P->H[l * p + m] = expi_rational((uint64_t)(l * m), (uint64_t)(2 * q * q), N, P->L);
        }
    memcpy(P->GLU, P->G, sizeof(P->G));
    lu_factor(P->GLU, P->piv, p);
    return P;
}

void or_bf_destroy(void *h)
{
    or_plan *P = h;
    if (!P) return;
    for (int m = 0; m <= P->L; ++m) { free(P->tx[m].key); free(P->tk[m].key); }
    free(P->tx); free(P->tk);
    free(P->xperm); free(P->xbeg); free(P->kperm); free(P->kbeg);
    free(P->x); free(P->k);
    free(P);
}

int or_bf_levels(void *h) { return ((or_plan *)h)->L; }

/* number of non-empty boxes at level m of T_X (side 0) or T_K (side 1) */
int64_t or_bf_count(void *h, int side, int m)
{
    or_plan *P = h;
    if (m < 0 || m > P->L) return -1;
    return side == 0 ? P->tx[m].n : P->tk[m].n;
}

/* box coordinates of level m, [n][d] */
void or_bf_boxes(void *h, int side, int m, int64_t *coords)
{
    or_plan *P = h;
    or_level *lv = side == 0 ? &P->tx[m] : &P->tk[m];
    for (int64_t i = 0; i < lv->n; ++i) key_coords(lv->key[i], P->d, m, coords + i * P->d);
}

/* per-axis matrices for tests: M(iA, iB) of eq. (M1) at T_K level lvl, and
 * E(iA, ic) of eq. (E1) for a child index ic at T_K level lvl + 1 */
void or_bf_matrix_M(void *h, int64_t iA, int64_t iB, double *out)
{
    or_plan *P = h;
    cplx m11[OR_PMAX], m12[OR_PMAX];
    m_diagonals(P, iA, iB, m11, m12);
    dcplx *o = (dcplx *)out;
    for (int l = 0; l < P->p; ++l)
        for (int m = 0; m < P->p; ++m) o[l * P->p + m] = (dcplx)(m11[l] * P->G[l * P->p + m] * m12[m]);
}

void or_bf_matrix_E(void *h, int64_t iA, int64_t ic, double *out)
{
    or_plan *P = h;
    cplx e11[OR_PMAX], e12[OR_PMAX];
    e_diagonals(P, iA, ic, e11, e12);
    dcplx *o = (dcplx *)out;
    for (int l = 0; l < P->p; ++l)
        for (int m = 0; m < P->p; ++m) o[l * P->p + m] = (dcplx)(e11[l] * P->H[l * P->p + m] * e12[m]);
}

/* ------------------------------------------------------------------------- */
/* O2: steps 2-4                                                               */
/* ------------------------------------------------------------------------- */

/*
 * Runs the butterfly on sources f (complex, original order) and writes u
 * (complex, original target order).  If dump_level is in [0, L], the check
 * potentials u^{AB} and charges f^{AB} of T_K level dump_level are copied to
 * dump_u / dump_f (layout [nA][nB][p^d], boxes in the order of or_bf_boxes;
 * A at T_X level L - dump_level).
 *
 * start = s0 in [0, L] is the number of T_K levels above the leaves at
 * which the sweep begins: the charges of the pairs (A at T_X level s0, B at
 * T_K level L - s0) are matched to potentials summed directly over the
 * sources in B (the plain procedure of Section 2.1), and step 3 continues
 * from there.  s0 = 0 is step 2 of Section 2.2 (B a leaf, A the root).
 * Returns 0, -1 on allocation failure, -3 for a bad start level.
 */
int or_bf_run(void *h, const double *f_in, double *u_out, int dump_level,
              double *dump_u, double *dump_f, int start)
{
    or_plan *P = h;
    const int d = P->d, p = P->p, q = P->q, L = P->L;
    int PD = 1;
    for (int a = 0; a < d; ++a) PD *= p;
    const dcplx *f = (const dcplx *)f_in;
    dcplx *u = (dcplx *)u_out;
    dcplx *du = (dcplx *)dump_u, *df = (dcplx *)dump_f;

    for (int64_t i = 0; i < P->nx; ++i) u[i] = 0;
    if (P->nx == 0 || P->nk == 0) return 0;
    if (start < 0 || start > L) return -3;

    /* step 2 (at level l0 = L - s0): for every B at T_K level l0 and A at
     * T_X level s0, u^{AB}_l = sum_{k_j in B} exp(2 pi i x^A_l . k_j / N) f_j
     * with x^A_l = (i_A + l/q) N / 2^s0 per axis, so the phase of axis a is
     * (q i_A + l) k_a / (q 2^s0) turns; then f^{AB} = M^{-1} u^{AB}. */
    const int s0 = start, l0 = L - start;
    const or_level *XS = &P->tx[s0], *KS = &P->tk[l0];
    int64_t nAs = XS->n, nBs = KS->n;
    cplx *cur = malloc(sizeof(cplx) * (size_t)nAs * nBs * PD);
    /* sources of every box B of T_K level l0 (counting sort by box) */
    int64_t *sbeg = calloc((size_t)nBs + 1, sizeof(int64_t));
    int64_t *sidx = malloc(sizeof(int64_t) * (size_t)P->nk);
    int64_t *sbox = malloc(sizeof(int64_t) * (size_t)P->nk);
    if (!cur || !sbeg || !sidx || !sbox) { free(cur); free(sbeg); free(sidx); free(sbox); return -1; }
    for (int64_t j = 0; j < P->nk; ++j) {
        int64_t idx[3];
        leaf_index(P->k + j * d, d, P->N, L, idx);
        for (int a = 0; a < d; ++a) idx[a] >>= s0;
        sbox[j] = find_box(KS, box_key(idx, d, l0));
        sbeg[sbox[j] + 1]++;
    }
    for (int64_t b = 0; b < nBs; ++b) sbeg[b + 1] += sbeg[b];
    {
        int64_t *fill = malloc(sizeof(int64_t) * (size_t)nBs);
        if (!fill) { free(cur); free(sbeg); free(sidx); free(sbox); return -1; }
        memcpy(fill, sbeg, sizeof(int64_t) * (size_t)nBs);
        for (int64_t j = 0; j < P->nk; ++j) sidx[fill[sbox[j]]++] = j;
        free(fill);
    }
    free(sbox);
    const double qs = (double)((int64_t)q << s0);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t ab = 0; ab < nAs * nBs; ++ab) {
        int64_t a = ab / nBs, b = ab % nBs;
        cplx *X = cur + ab * PD;
        int64_t iA[3], iB[3];
        key_coords(XS->key[a], d, s0, iA);
        key_coords(KS->key[b], d, l0, iB);
        for (int e = 0; e < PD; ++e) X[e] = 0;
        for (int64_t t = sbeg[b]; t < sbeg[b + 1]; ++t) {
            int64_t j = sidx[t];
            const double *kj = P->k + j * d;
            cplx ph[3][OR_PMAX];
            for (int s = 0; s < d; ++s)
                for (int l = 0; l < p; ++l)
                    ph[s][l] = expi_dd(dd_div(two_prod((double)(q * iA[s] + l), kj[s]), qs));
            for (int e = 0; e < PD; ++e) {
                cplx w = f[j];
                int r = e;
                for (int s = d - 1; s >= 0; --s) { w *= ph[s][r % p]; r /= p; }
                X[e] += w;
            }
        }
        if (dump_level == l0 && du)
            for (int e = 0; e < PD; ++e) du[ab * PD + e] = (dcplx)X[e];
        solve_matching(P, iA, iB, X);
        if (dump_level == l0 && df)
            for (int e = 0; e < PD; ++e) df[ab * PD + e] = (dcplx)X[e];
    }
    free(sbeg);
    free(sidx);

    /* step 3: for l = l0-1 .. 0, every B at T_K level l and every A at T_X
     * level L-l:  u^{AB} = sum_c E(A, B_c) f^{A' B_c},  f^{AB} = M^{-1} u^{AB}. */
    for (int lvl = l0 - 1; lvl >= 0; --lvl) {
        const or_level *XA = &P->tx[L - lvl], *XP = &P->tx[L - lvl - 1];
        const or_level *KB = &P->tk[lvl], *KC = &P->tk[lvl + 1];
        int64_t nA = XA->n, nBo = KB->n, nBc = KC->n;
        cplx *nxt = malloc(sizeof(cplx) * (size_t)nA * nBo * PD);
        if (!nxt) { free(cur); return -1; }
        int ok = 1;
#pragma omp parallel for schedule(dynamic, 64)
        for (int64_t ab = 0; ab < nA * nBo; ++ab) {
            int64_t a = ab / nBo, b = ab % nBo;
            int64_t iA[3], iB[3], iAp[3];
            key_coords(XA->key[a], d, L - lvl, iA);
            key_coords(KB->key[b], d, lvl, iB);
            for (int t = 0; t < d; ++t) iAp[t] = iA[t] >> 1;
            int64_t ap = find_box(XP, box_key(iAp, d, L - lvl - 1));
            if (ap < 0) { ok = 0; continue; }
            cplx *U = nxt + ab * PD;
            for (int e = 0; e < PD; ++e) U[e] = 0;
            cplx Y[OR_PMAX * OR_PMAX * OR_PMAX];
            for (int c = 0; c < (1 << d); ++c) {
                int64_t ic[3];
                for (int t = 0; t < d; ++t) ic[t] = 2 * iB[t] + ((c >> (d - 1 - t)) & 1);
                int64_t bc = find_box(KC, box_key(ic, d, lvl + 1));
                if (bc < 0) continue;                    /* empty child */
                memcpy(Y, cur + (ap * nBc + bc) * PD, sizeof(cplx) * PD);
                for (int t = 0; t < d; ++t) {
                    cplx e11[OR_PMAX], e12[OR_PMAX], E[OR_PMAX * OR_PMAX];
                    e_diagonals(P, iA[t], ic[t], e11, e12);
                    for (int l = 0; l < p; ++l)
                        for (int m = 0; m < p; ++m) E[l * p + m] = e11[l] * P->H[l * p + m] * e12[m];
                    mode_apply(Y, E, p, d, t);
                }
                for (int e = 0; e < PD; ++e) U[e] += Y[e];
            }
            if (dump_level == lvl && du)
                for (int e = 0; e < PD; ++e) du[ab * PD + e] = (dcplx)U[e];
            solve_matching(P, iA, iB, U);
            if (dump_level == lvl && df)
                for (int e = 0; e < PD; ++e) df[ab * PD + e] = (dcplx)U[e];
        }
        free(cur);
        cur = nxt;
        if (!ok) { free(cur); return -2; }
    }

    /* step 4: u_i = sum_l exp(2 pi i x_i . k^{B0}_l / N) f^{A B0}_l for x_i in
     * leaf A of T_X; k^{B0}_l = l N / q per axis, so the phase is x_i . l / q. */
    const or_level *XL = &P->tx[L];
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t a = 0; a < XL->n; ++a) {
        const cplx *F = cur + a * PD;
        for (int64_t t = P->xbeg[a]; t < P->xbeg[a + 1]; ++t) {
            int64_t i = P->xperm[t];
            const double *xi = P->x + i * d;
            cplx ph[3][OR_PMAX];
            for (int s = 0; s < d; ++s)
                for (int l = 0; l < p; ++l)
                    ph[s][l] = expi_dd(dd_div(two_prod((double)l, xi[s]), (double)q));
            cplx acc = 0;
            for (int e = 0; e < PD; ++e) {
                cplx w = F[e];
                int r = e;
                for (int s = d - 1; s >= 0; --s) { w *= ph[s][r % p]; r /= p; }
                acc += w;
            }
            u[i] = (dcplx)acc;
        }
    }
    free(cur);
    return 0;
}

void or_set_threads(int n)
{
    if (n > 0) omp_set_num_threads(n);
}

int or_max_threads(void) { return omp_get_max_threads(); }
