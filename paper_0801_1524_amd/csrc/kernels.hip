// Steps 2-4 of Section 2.2 on gfx950: leaf initialisation, the level sweep
// and the evaluation at the leaves of T_X.
//
// State representation.  The paper stores equivalent charges f^{AB}
// (Section 2.1) and recomputes check potentials u^{AB} = M f^{AB} from the
// children at every level.  Here the state of a box pair is its check
// potential itself, with B's corner phase divided out:
//
//     w^{AB}_l = exp(-2 pi i x^A_l . c^B / N) u^{AB}_l ,   l in {0..p-1}^d.
//
// In exact arithmetic this is the same computation (u^{AB} = M f^{AB}, and M
// is invertible), but every operator becomes well conditioned:
//  * the field of (A', B_c) inside A' is a polynomial of degree p-1 (per
//    axis) in Z = exp(2 pi i xi rho / q) that takes the values w^{A'B_c} at
//    the p check nodes Z_k = exp(2 pi i rho k / q^2); evaluating it at the
//    check points of A = child t of A' is Lagrange interpolation, so the
//    translation of eq. (E1) followed by M^{-1} of eq. (M1) is, per axis,
//        U_{s,t}[l][l'] = e^{i pi rho t s} e^{i pi rho l s / q} L_t[l][l'],
//        L_t[l][l'] = ell_{l'}( exp(i pi rho (t q + l) / q^2) ),
//    times the scalar exp(2 pi i rho i_{A'} s) (1 when rho = 1);
//  * the leaf state (step 2) is sum_j exp(2 pi i l . k'_j / q) f_j with the
//    local offset k' = k - rho i_B, so no phase argument exceeds 2 pi d;
//  * evaluation (step 4) is barycentric interpolation of w^{AB_0} at the
//    local offset x' = x - rho i_A.
// No inverse of the Vandermonde matrix G (cond ~ 3e8 at p = 9) is formed.
//
// Rotation.  Nodes and check points lie on the unit circle, where
// ell_k(Y) = exp(i q (arg Y - arg Z_k) / 2) times a real product of sines, so
// L_t = diag(D_t) R_t diag(E) with R_t real, E[k] = exp(-i pi rho k / q) and
// D_t[l] = exp(i pi rho (t q + l) / (2 q)).  Every kernel therefore keeps the
// rotated state w^ = (E x ... x E) w, which is B's check potential with the
// phase of B's centre (not its corner) divided out, up to a factor of A:
// the leaf sums take offsets from the centre, the start-level direct sums
// multiply by E, the translations apply the real R_t with the phases
// G(s, t, l) = E[l] D_t[l] f(s, t, l) on the outputs, and the evaluation
// folds conj(E) into its weights.
//
// The sweep of one level is a streaming pass: for a parent a' of T_X and a
// tile of boxes b of T_K, the children of b are contiguous in the input row
// a' (Morton order), and the outputs are rows a = children of a'.
#include "bfsft_impl.h"
#include "cplx.h"
#include "dispatch.h"

#include <type_traits>

namespace bfsft {

namespace {

// exp(2 pi i num / den) with the numerator reduced exactly (den > 0)
__device__ double2 expi_ratio(int64_t num, int64_t den)
{
    int64_t r = num % den;
    if (r < 0) r += den;
    double s, c;
    sincospi(2.0 * (double)r / (double)den, &s, &c);
    return make_double2(c, s);
}

__device__ double2 dmul(double2 a, double2 b) { return cmul(a, b); }

__device__ double2 ddiv(double2 a, double2 b)
{
    const double den = b.x * b.x + b.y * b.y;
    return make_double2((a.x * b.x + a.y * b.y) / den, (a.y * b.x - a.x * b.y) / den);
}

// exp(2 pi i a) - exp(2 pi i b) = 2 i sin(pi (a - b)) exp(i pi (a + b)), for
// a - b and a + b given in turns: no cancellation between close points
__device__ double2 diff_unit(double amb, double apb)
{
    double s, c;
    sincospi(apb, &s, &c);
    const double sn = 2.0 * sinpi(amb);
    return make_double2(-sn * s, sn * c);
}

// ---------------------------------------------------------------- tables --

// One thread block, FP64.  rho = N / 2^L; all turns are exact rationals
// N n / (2 q^2 2^L) (or N n / (4 q 2^L)) rounded once.
//   L64  Lagrange rows L_t[l][k] = ell_k(exp(i pi rho (t q + l) / q^2)),
//   R64  their real factor: for points on the unit circle
//        ell_k(Y) = exp(i q (arg Y - arg Z_k) / 2) prod_{j != k} sin((arg Y - arg Z_j) / 2)
//                                                       / sin((arg Z_k - arg Z_j) / 2),
//        so R_t[l][k] is the sine product, taken directly,
//   C64  G(0, t, l) = E[l] D_t[l] = exp(i pi rho (t q - l) / (2 q)) and
//        G(1, t, l) = G(0, t, l) exp(i pi rho (t q + l) / q),
//   erot E[k] = exp(-i pi rho k / q).
__global__ void k_tables(int p, int64_t N, int L, double2 *L64, double2 *PH64, double *R64, float *R32,
                         double2 *C64, float2 *C32, double2 *erot, double2 *nodes, double2 *bary,
                         double *node_turns)
{
    const int q = p - 1;
    const double den = ldexp(2.0 * q * q, L);  // 2 q^2 2^L
    __shared__ double2 lam[16];
    const int tid = threadIdx.x;
    if (tid < p) {
        // barycentric weight of node k: 1 / prod_{j != k} (Z_k - Z_j), Z_k at 2k/(2q^2) rho turns
        const int k = tid;
        double2 prod = make_double2(1.0, 0.0);
        for (int j = 0; j < p; ++j) {
            if (j == k) continue;
            const double amb = (double)(N * (int64_t)(2 * (k - j))) / den;
            const double apb = (double)(N * (int64_t)(2 * (k + j))) / den;
            prod = dmul(prod, diff_unit(amb, apb));
        }
        lam[k] = ddiv(make_double2(1.0, 0.0), prod);
        bary[k] = lam[k];
        nodes[k] = expi_ratio(N * (int64_t)(2 * k), (int64_t)(2 * q * q) << L);
        node_turns[k] = (double)(N * (int64_t)k) / ldexp((double)(q * q), L);
        erot[k] = expi_ratio(-N * (int64_t)k, (int64_t)(2 * q) << L);
    }
    __syncthreads();
    if (tid < 2 * p) {
        const int t = tid / p, l = tid % p;
        const int num = t * q + l;  // point exp(i pi rho num / q^2)
        double2 w[16];
        double2 sum = make_double2(0.0, 0.0);
        int exact = -1;
        for (int k = 0; k < p; ++k) {
            if (num == 2 * k) exact = k;
            const double amb = (double)(N * (int64_t)(num - 2 * k)) / den;
            const double apb = (double)(N * (int64_t)(num + 2 * k)) / den;
            w[k] = ddiv(lam[k], diff_unit(amb, apb));
            sum.x += w[k].x;
            sum.y += w[k].y;
        }
        for (int k = 0; k < p; ++k) {
            double2 v;
            double r = 0.0;
            if (exact >= 0) {
                v = make_double2(k == exact ? 1.0 : 0.0, 0.0);
                r = k == exact ? 1.0 : 0.0;
            } else {
                v = ddiv(w[k], sum);
                r = 1.0;
                for (int j = 0; j < p; ++j) {
                    if (j == k) continue;
                    r *= sinpi((double)(N * (int64_t)(num - 2 * j)) / den) /
                         sinpi((double)(N * (int64_t)(2 * k - 2 * j)) / den);
                }
            }
            L64[(t * p + l) * p + k] = v;
            R64[(t * p + l) * p + k] = r;
            R32[(t * p + l) * p + k] = (float)r;
        }
        // phase of the child at offset s = 1: exp(i pi rho (t q + l) / q)
        PH64[t * p + l] = expi_ratio(N * (int64_t)num, (int64_t)(2 * q) << L);
        const double2 g0 = expi_ratio(N * (int64_t)(t * q - l), (int64_t)(4 * q) << L);
        const double2 g1 = expi_ratio(N * (int64_t)(3 * t * q + l), (int64_t)(4 * q) << L);
        C64[t * p + l] = g0;
        C64[(2 + t) * p + l] = g1;
        C32[t * p + l] = make_float2((float)g0.x, (float)g0.y);
        C32[(2 + t) * p + l] = make_float2((float)g1.x, (float)g1.y);
    }
}

__global__ void k_sigma(const uint64_t *__restrict__ keys, int64_t n, int d, int m, int L,
                        int64_t N, double2 *__restrict__ sig)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const uint64_t key = keys[i];
    for (int a = 0; a < d; ++a) {
        int64_t c = 0;
        for (int b = 0; b < m; ++b) c |= (int64_t)((key >> (b * d + a)) & 1ull) << b;
        // exp(2 pi i rho c) with rho c = N c / 2^L
        sig[i * d + a] = expi_ratio(N * c, (int64_t)1 << L);
    }
}

// ------------------------------------------------------------------ leaf --

// Step 2: w^{A0 B}_l = sum_{k_j in B} exp(2 pi i l . k'_j / q) f_j for every
// leaf B of T_K (A0 = root of T_X), stored rotated: E[l_a] = exp(-2 pi i
// l_a (rho / 2) / q) per axis turns the offset k' from B's corner into the
// offset k' - rho / 2 from its centre.  One thread per (leaf, grid point).
template <int D, typename S>
__device__ __forceinline__ void leaf_item(int p, int64_t nleaf, const double2 *__restrict__ f,
                                          const int32_t *__restrict__ perm,
                                          const int32_t *__restrict__ beg,
                                          const double *__restrict__ local, double shift,
                                          typename CV<S>::t *__restrict__ state, int64_t gid)
{
    int PD = p;
    for (int a = 1; a < D; ++a) PD *= p;
    if (gid >= nleaf * PD) return;
    const int64_t b = gid / PD;
    const int e = (int)(gid - b * PD);
    int lidx[3] = {0, 0, 0};
    {
        int r = e;
        for (int a = D - 1; a >= 0; --a) {
            lidx[a] = r % p;
            r /= p;
        }
    }
    const double invq = 1.0 / (double)(p - 1);
    double2 acc = make_double2(0.0, 0.0);
    for (int t = beg[b]; t < beg[b + 1]; ++t) {
        const int j = perm[t];
        double turns = 0.0;
        for (int a = 0; a < D; ++a) turns = fma((double)lidx[a], local[(int64_t)j * D + a] - shift, turns);
        double s, c;
        sincospi(2.0 * turns * invq, &s, &c);
        const double2 fj = f[j];
        acc.x += c * fj.x - s * fj.y;
        acc.y += c * fj.y + s * fj.x;
    }
    typename CV<S>::t o;
    o.x = (S)acc.x;
    o.y = (S)acc.y;
    state[gid] = o;
}

template <int D, typename S>
__global__ __launch_bounds__(256) void k_leaf(int p, int64_t nleaf,
                                             const double2 *__restrict__ f,
                                             const int32_t *__restrict__ perm,
                                             const int32_t *__restrict__ beg,
                                             const double *__restrict__ local, double shift,
                                             typename CV<S>::t *__restrict__ state)
{
    leaf_item<D, S>(p, nleaf, f, perm, beg, local, shift, state, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// ---------------------------------------------------------- start level --
// The sweep may begin s0 levels above the leaves: the twisted check
// potentials of every pair (A at T_X level s0, B at T_K level L - s0) are
// summed directly over the sources in B (the plain procedure of
// Section 2.1):
//     w^{AB}_l = sum_{k_j in B} exp(2 pi i x^A_l . (k_j - c^B) / N) f_j,
//     x^A_l = (i_A + l / q) N / 2^s0 per axis,
// so the phase of axis a is (q i_A + l) (k_j - c^B)_a / (q 2^s0) turns.
// Each offset k_j - c^B = rho m + loc is stored split: m = leaf index mod
// 2^s0 (an integer), loc = offset inside the leaf (exact).

// offsets of the sources, in the trees' sorted order
// and the phase step between grid points of every axis,
// exp(2 pi i (rho m + loc) / (q 2^s0))
template <int D>
__global__ void k_source_offsets(int64_t n, int s0, int q, double rho, const int32_t *__restrict__ perm,
                                 const int32_t *__restrict__ leaf_of, const uint64_t *__restrict__ leaf_keys,
                                 const double *__restrict__ local, int32_t *__restrict__ sm,
                                 double *__restrict__ sloc, double2 *__restrict__ sratio)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= n) return;
    const int j = perm[t];
    const uint64_t key = leaf_keys[leaf_of[j]];
#pragma unroll
    for (int a = 0; a < D; ++a) {
        int m = 0;
        for (int b = 0; b < s0; ++b) m |= (int)((key >> (b * D + a)) & 1) << b;
        sm[t * D + a] = m;
        sloc[t * D + a] = local[(int64_t)j * D + a];
        double sn, cs;
        sincospi(2.0 * (rho * m + local[(int64_t)j * D + a]) / ldexp((double)q, s0), &sn, &cs);
        sratio[t * D + a] = make_double2(cs, sn);
    }
}

// turns of (q i_A + l) (rho m + loc) / (q 2^s0) modulo 1 (up to one extra
// turn): the rho m part is the exact rational X / (q 2^E) with
// X = (q i_A + l) m N and E = s0 + L, reduced in integers as
// X mod q 2^E = ((X >> E) mod q) 2^E + (X mod 2^E)  (X < 2^64 for s0 <= 18,
// q a compile-time constant); the loc part is below two turns, in FP64
template <int Q>
__device__ __forceinline__ double direct_turns(int64_t qil, int m, double loc, int E, double inv_den,
                                               double inv_qs, int64_t N)
{
    const uint64_t X = (uint64_t)(qil * (int64_t)m) * (uint64_t)N;
    const uint64_t r = (((X >> E) % (uint64_t)Q) << E) | (X & ((1ull << E) - 1ull));
    return (double)r * inv_den + (double)qil * loc * inv_qs;
}

__device__ __forceinline__ double2 expi_turns(double t)
{
    double s, c;
    sincospi(2.0 * t, &s, &c);
    return make_double2(c, s);
}

// One thread per (pair, group of G lines).  A line fixes the grid indices
// of the leading d - 1 axes; a group holds G consecutive indices of axis
// d - 2.  Per source the thread takes one phase per leading axis and one
// along the last axis from sincospi, steps along axis d - 2 (G values) and
// along the last axis (p values) by the source's per-axis phase steps, and
// accumulates G x p outputs.
// waves per SIMD the direct sums' registers must allow (their 3p complex
// accumulators and phase chains): three up to p = 8, two above
template <int P> constexpr int direct_waves() { return P <= 8 ? 3 : 2; }

template <int D, int P, int G> constexpr int direct_groups() { return D == 2 ? (P + G - 1) / G : P * ((P + G - 1) / G); }

template <int D, int P, int G, typename S>
__device__ __forceinline__ void direct_item(const DirectDesc &dd, int64_t gid)
{
    constexpr int Q = P - 1;
    constexpr int NG = (P + G - 1) / G;              // groups along axis d - 2
    constexpr int GL = direct_groups<D, P, G>();     // groups per pair
    constexpr int PD = D == 2 ? P * P : P * P * P;
    const int s0 = dd.s0, L = dd.L;
    const int64_t N = dd.N, nB = dd.nB;
    if (gid >= dd.nA * nB * GL) return;
    // B-major: the threads of a wave mostly share the box B, hence the
    // source loop's trip count and the addresses of its loads.  Item
    // indices fit 32 bits (checked at launch).
    const int g32 = (int)gid;
    const int per_b = (int)dd.nA * GL;
    const int b = g32 / per_b;
    const int rem = g32 - b * per_b;
    const int a = rem / GL;
    const int grp = rem - a * GL;
    const int64_t ab = (int64_t)a * nB + b;
    int64_t iA[3] = {0, 0, 0};
    {
        const uint64_t key = dd.xkeys[a];
        for (int ax = 0; ax < D; ++ax)
            for (int bit = 0; bit < s0; ++bit) iA[ax] |= (int64_t)((key >> (bit * D + ax)) & 1) << bit;
    }
    // grid index of axis 0 (3D only) and the first index of the group on axis d - 2
    const int l_outer = D == 3 ? grp / NG : 0;
    const int lg0 = (D == 3 ? grp - l_outer * NG : grp) * G;
    const int E = s0 + L;
    const double inv_den = 1.0 / ldexp((double)Q, E);
    const double inv_qs = 1.0 / ldexp((double)Q, s0);
    const int2 lr = dd.box_leaf[b];
    const int t0 = dd.leaf_beg[lr.x], t1 = dd.leaf_beg[lr.y];
    const int32_t *__restrict__ sm = dd.sm;
    const double *__restrict__ sloc = dd.sloc;
    const double2 *__restrict__ sstep = dd.sstep;
    double2 acc[G][P];
#pragma unroll
    for (int g = 0; g < G; ++g)
#pragma unroll
        for (int l = 0; l < P; ++l) acc[g][l] = make_double2(0.0, 0.0);
    for (int t = t0; t < t1; ++t) {
        double2 w = dd.f[dd.perm[t]];
        if (D == 3)
            w = cmul(w, expi_turns(direct_turns<Q>(Q * iA[0] + l_outer, sm[(int64_t)t * D], sloc[(int64_t)t * D],
                                                   E, inv_den, inv_qs, N)));
        constexpr int AG = D - 2, AL = D - 1;  // the group axis and the last axis
        double2 c[G];
        c[0] = cmul(w, expi_turns(direct_turns<Q>(Q * iA[AG] + lg0, sm[(int64_t)t * D + AG],
                                                  sloc[(int64_t)t * D + AG], E, inv_den, inv_qs, N)));
        const double2 rg = sstep[(int64_t)t * D + AG];
#pragma unroll
        for (int g = 1; g < G; ++g) c[g] = cmul(c[g - 1], rg);
        double2 e = expi_turns(direct_turns<Q>(Q * iA[AL], sm[(int64_t)t * D + AL], sloc[(int64_t)t * D + AL], E,
                                               inv_den, inv_qs, N));
        const double2 rl = sstep[(int64_t)t * D + AL];
#pragma unroll
        for (int l = 0; l < P; ++l) {
#pragma unroll
            for (int g = 0; g < G; ++g) cfma(acc[g][l], c[g], e);
            e = cmul(e, rl);
        }
    }
    // rotated state: times E[l_a] of every axis.  All factors are read
    // before the first store (the table could alias the state for all the
    // compiler knows); the uniform ones through scalar loads.
    typename CV<S>::t *o = (typename CV<S>::t *)dd.state + ab * PD + ((int64_t)l_outer * P + lg0) * P;
    const cptr<double> er = (cptr<double>)(const void *)dd.erot;
    double2 el[P];
#pragma unroll
    for (int l = 0; l < P; ++l) el[l] = ldc<double2>(er, l);
    const double2 eo = D == 3 ? dd.erot[l_outer] : make_double2(1.0, 0.0);
    double2 eg[G];
#pragma unroll
    for (int g = 0; g < G; ++g) eg[g] = cmul(eo, lg0 + g < P ? dd.erot[lg0 + g] : make_double2(1.0, 0.0));
#pragma unroll
    for (int g = 0; g < G; ++g) {
        if (lg0 + g >= P) break;
#pragma unroll
        for (int l = 0; l < P; ++l) {
            const double2 r = cmul(acc[g][l], cmul(eg[g], el[l]));
            typename CV<S>::t v;
            v.x = (S)r.x;
            v.y = (S)r.y;
            o[g * P + l] = v;
        }
    }
}

template <int D, int P, int G, typename S>
__global__ __launch_bounds__(256, (direct_waves<P>())) void k_direct(DirectDesc dd)
{
    direct_item<D, P, G, S>(dd, (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

// index of the descriptor owning flat item `i` (prefix[t] <= i < prefix[t+1])
__device__ __forceinline__ int owner(const int64_t *__restrict__ prefix, int n, int64_t i)
{
    int lo = 0, hi = n - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= i) lo = mid; else hi = mid - 1;
    }
    return lo;
}

template <int D, typename S>
__global__ __launch_bounds__(256) void k_leaf_batched(int p, const LeafDesc *__restrict__ ds,
                                                     const int64_t *__restrict__ prefix, int n,
                                                     int64_t total)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const LeafDesc &d = ds[owner(prefix, n, i)];
    leaf_item<D, S>(p, d.nleaf, (const double2 *)d.f, d.perm, d.beg, d.local, d.shift,
                    (typename CV<S>::t *)d.state, i - d.first);
}

// descriptor i, read through the constant address space (uniform: scalar
// loads), field by field
__device__ __forceinline__ DirectDesc load_direct_desc(const DirectDesc *descs, int i)
{
    using CT = const __attribute__((address_space(4))) DirectDesc;
    CT *p = (CT *)descs + i;
    DirectDesc d;
    d.s0 = p->s0;
    d.L = p->L;
    d.N = p->N;
    d.nA = p->nA;
    d.nB = p->nB;
    d.xkeys = p->xkeys;
    d.box_leaf = p->box_leaf;
    d.steps = nullptr;
    d.wg_first = nullptr;
    d.nwg = d.nwaves = 0;
    d.gam = d.geo = nullptr;
    d.nk = 0;
    d.leaf_beg = p->leaf_beg;
    d.perm = p->perm;
    d.sm = p->sm;
    d.sloc = p->sloc;
    d.sstep = p->sstep;
    d.f = p->f;
    d.erot = p->erot;
    d.state = p->state;
    d.first = p->first;
    return d;
}

// Every transform's items start on a work-group boundary (the prefix is
// padded to 256), so the owner is uniform across a work-group: it is found
// from the work-group's first item and its descriptor held in scalar
// registers.
template <int D, int P, int G, typename S>
__global__ __launch_bounds__(256, (direct_waves<P>())) void k_direct_batched(const DirectDesc *__restrict__ ds,
                                                       const int64_t *__restrict__ prefix, int n,
                                                       int64_t total)
{
    const int64_t i0 = (int64_t)blockIdx.x * blockDim.x;
    const DirectDesc d = load_direct_desc(ds, owner(prefix, n, i0));
    const int64_t i = i0 + threadIdx.x;
    if (i >= total) return;
    direct_item<D, P, G, S>(d, i - d.first);
}

// ----------------------------------------------------------------- final --

// Step 4: u_i = sum_l prod_a ell_{l_a}(exp(2 pi i x'_{i,a} / q)) w^{A B0}_l for
// x_i in leaf A of T_X (barycentric Lagrange interpolation); the state is
// rotated, w = conj(E x ... x E) w^, so each weight takes conj(E[l_a]).

// exp(i pi node_turns[k]) for every node, by recurrence from the first
// (node_turns[k] is k node_turns[1] up to one rounding; the products drift
// by a few ulps at most)
template <int P>
__device__ __forceinline__ void node_phases(const double *__restrict__ node_turns, double2 *nph)
{
    double s, c;
    sincospi(node_turns[1], &s, &c);
    nph[0] = make_double2(1.0, 0.0);
#pragma unroll
    for (int k = 1; k < P; ++k) nph[k] = cmul(nph[k - 1], make_double2(c, s));
}

// The P weights of one axis at xt turns of z = exp(2 pi i x'/q), each times
// conj(E[k]); a point on a node takes that node's E alone.
template <int P>
__device__ __forceinline__ void axis_weights(double xt, const double2 *__restrict__ bary,
                                             const double *__restrict__ node_turns,
                                             const double2 *__restrict__ erot, const double2 *nph, double2 *ell)
{
    double sx, cx;
    sincospi(xt, &sx, &cx);
    int exact = -1;
    double2 sum = make_double2(0.0, 0.0);
#pragma unroll
    for (int k = 0; k < P; ++k) {
        // z - z_k = 2 i sin(pi (xt - t_k)) e with e = exp(i pi (xt + t_k)),
        // |e| = 1, so 1 / (z - z_k) = -i conj(e) / (2 sin(pi (xt - t_k))):
        // the difference of the turns is taken exactly (no cancellation
        // between close points), and one real division per node
        const double amb = xt - node_turns[k];
        if (amb == 0.0) exact = k;  // that node's weight is replaced below
        const double2 e = cmul(make_double2(cx, sx), nph[k]);
        const double h = 0.5 / sinpi(amb);
        const double2 w = cmul(bary[k], make_double2(-e.y * h, -e.x * h));
        ell[k] = w;
        sum.x += w.x;
        sum.y += w.y;
    }
    const double n2 = sum.x * sum.x + sum.y * sum.y;
    const double2 rs = make_double2(sum.x / n2, -sum.y / n2);  // 1 / sum
#pragma unroll
    for (int k = 0; k < P; ++k) {
        const double2 e = make_double2(erot[k].x, -erot[k].y);
        ell[k] = exact >= 0 ? (k == exact ? e : make_double2(0.0, 0.0)) : cmul(cmul(ell[k], rs), e);
    }
}

// rows of the 2D sum taken by the first lane of a pair (k_final2); the
// one-lane form sums the same two halves in the same order, so both give
// the same bits
template <int P> constexpr int final_half() { return (P + 1) / 2; }

template <int D, int P, typename S>
__device__ __forceinline__ void final_item(int64_t nx, const typename CV<S>::t *__restrict__ state,
                                           const int32_t *__restrict__ leaf_of,
                                           const double *__restrict__ local,
                                           const double2 *__restrict__ bary,
                                           const double *__restrict__ node_turns,
                                           const double2 *__restrict__ erot,
                                           double2 *__restrict__ u, int64_t i)
{
    if (i >= nx) return;
    constexpr int q = P - 1;
    double2 nph[P];
    node_phases<P>(node_turns, nph);
    double2 ell[D][P];
#pragma unroll
    for (int a = 0; a < D; ++a) axis_weights<P>(local[i * D + a] / (double)q, bary, node_turns, erot, nph, ell[a]);
    constexpr int PD = (D == 2) ? P * P : P * P * P;
    const typename CV<S>::t *w = state + (int64_t)leaf_of[i] * PD;
    double2 acc = make_double2(0.0, 0.0);
    if (D == 2) {
        constexpr int LH = final_half<P>();
        double2 half[2] = {make_double2(0.0, 0.0), make_double2(0.0, 0.0)};
#pragma unroll
        for (int l = 0; l < P; ++l) {
            double2 r = make_double2(0.0, 0.0);
#pragma unroll
            for (int m = 0; m < P; ++m) cfma(r, ell[1][m], cvt<double2>(w[l * P + m]));
            cfma(half[l >= LH], ell[0][l], r);
        }
        acc = make_double2(half[0].x + half[1].x, half[0].y + half[1].y);
    } else {
#pragma unroll
        for (int l = 0; l < P; ++l) {
            double2 r1 = make_double2(0.0, 0.0);
            for (int m = 0; m < P; ++m) {
                double2 r2 = make_double2(0.0, 0.0);
#pragma unroll
                for (int n = 0; n < P; ++n) cfma(r2, ell[D - 1][n], cvt<double2>(w[(l * P + m) * P + n]));
                cfma(r1, ell[1][m], r2);
            }
            cfma(acc, ell[0][l], r1);
        }
    }
    u[i] = acc;
}

// 2D with two lanes per target: lane a of the pair computes the weights of
// axis a (the pair exchanges them) and half of the rows l of the sum; the
// halves are added as in final_item.
template <int P, typename S>
__global__ __launch_bounds__(256) void k_final2(int64_t nx, const typename CV<S>::t *__restrict__ state,
                                               const int32_t *__restrict__ leaf_of,
                                               const double *__restrict__ local,
                                               const double2 *__restrict__ bary,
                                               const double *__restrict__ node_turns,
                                               const double2 *__restrict__ erot,
                                               double2 *__restrict__ u)
{
    constexpr int q = P - 1, LH = final_half<P>();
    const int64_t g = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i0 = g >> 1;
    const int a = (int)(g & 1);
    // clamped, so that both lanes of every pair run the exchanges below
    const int64_t i = i0 < nx ? i0 : nx - 1;
    double2 nph[P];
    node_phases<P>(node_turns, nph);
    double2 own[P];
    axis_weights<P>(local[i * 2 + a] / (double)q, bary, node_turns, erot, nph, own);
    double2 e0[P], e1[P];
#pragma unroll
    for (int k = 0; k < P; ++k) {
        const double2 o = make_double2(__shfl_xor(own[k].x, 1), __shfl_xor(own[k].y, 1));
        e0[k] = a ? o : own[k];
        e1[k] = a ? own[k] : o;
    }
    const typename CV<S>::t *w = state + (int64_t)leaf_of[i] * (P * P);
    double2 acc = make_double2(0.0, 0.0);
#pragma unroll
    for (int k = 0; k < LH; ++k) {
        const int l = a * LH + k;  // lane 1: rows LH .. P - 1
        if (l < P) {
            double2 r = make_double2(0.0, 0.0);
#pragma unroll
            for (int m = 0; m < P; ++m) cfma(r, e1[m], cvt<double2>(w[l * P + m]));
            const double2 wl = (LH + k < P && a) ? e0[LH + k < P ? LH + k : 0] : e0[k];
            cfma(acc, wl, r);
        }
    }
    const double2 o = make_double2(__shfl_xor(acc.x, 1), __shfl_xor(acc.y, 1));
    if (a == 0 && i0 < nx) u[i0] = make_double2(acc.x + o.x, acc.y + o.y);
}

template <int D, int P, typename S>
__global__ __launch_bounds__(256) void k_final(int64_t nx, const typename CV<S>::t *__restrict__ state,
                                              const int32_t *__restrict__ leaf_of,
                                              const double *__restrict__ local,
                                              const double2 *__restrict__ bary,
                                              const double *__restrict__ node_turns,
                                              const double2 *__restrict__ erot,
                                              double2 *__restrict__ u)
{
    final_item<D, P, S>(nx, state, leaf_of, local, bary, node_turns, erot, u,
                        (int64_t)blockIdx.x * blockDim.x + threadIdx.x);
}

template <int D, int P, typename S>
__global__ __launch_bounds__(256) void k_final_batched(const FinalDesc *__restrict__ ds,
                                                      const int64_t *__restrict__ prefix, int n,
                                                      int64_t total)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const FinalDesc &d = ds[owner(prefix, n, i)];
    final_item<D, P, S>(d.nx, (const typename CV<S>::t *)d.state, d.leaf_of, d.local,
                        (const double2 *)d.bary, d.node_turns, (const double2 *)d.erot, (double2 *)d.u,
                        i - d.first);
}

// ----------------------------------------------------------------- export --

// Parity probe: pot[a][b][l] = exp(2 pi i x^A_l . c^B / N) w^{AB}_l, i.e. the
// paper's check potential u^{AB} at T_K level lvl, from the rotated state
// w^ = E w; the phase is sum_a [rho i_B (q i_A + l_a) / q + rho l_a / (2 q)]
// turns, its numerator over 2 q 2^L reduced exactly.
template <typename S>
__global__ void k_export(int d, int p, const typename CV<S>::t *__restrict__ st,
                         const uint64_t *__restrict__ xkeys, int64_t nA,
                         const uint64_t *__restrict__ kkeys, int64_t nB, int lvl, int L,
                         int64_t N, double2 *__restrict__ pot)
{
    int PD = p;
    for (int a = 1; a < d; ++a) PD *= p;
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (gid >= nA * nB * PD) return;
    const int64_t ab = gid / PD;
    const int e = (int)(gid - ab * PD);
    const int64_t ia = ab / nB, ib = ab - ia * nB;
    const int q = p - 1;
    const uint64_t D = (uint64_t)q << L;
    const uint64_t Nm = (uint64_t)N % D;
    const uint64_t D2 = 2 * D;
    const uint64_t N2 = (uint64_t)N % D2;
    const int mA = L - lvl;
    uint64_t tot = 0;
    int r = e;
    int lix[3];
    for (int a = d - 1; a >= 0; --a) {
        lix[a] = r % p;
        r /= p;
    }
    for (int a = 0; a < d; ++a) {
        uint64_t cA = 0, cB = 0;
        for (int b = 0; b < mA; ++b) cA |= ((xkeys[ia] >> (b * d + a)) & 1ull) << b;
        for (int b = 0; b < lvl; ++b) cB |= ((kkeys[ib] >> (b * d + a)) & 1ull) << b;
        const uint64_t n = (cB * ((uint64_t)q * cA + (uint64_t)lix[a])) % D;
        tot = (tot + (Nm * n) % D) % D;
    }
    uint64_t tot2 = 2 * tot;
    for (int a = 0; a < d; ++a) tot2 = (tot2 + N2 * (uint64_t)lix[a]) % D2;
    double s, c;
    sincospi(2.0 * (double)tot2 / (double)D2, &s, &c);
    const double2 w = cvt<double2>(st[gid]);
    pot[gid] = make_double2(c * w.x - s * w.y, c * w.y + s * w.x);
}

__global__ void k_zero_u64(unsigned long long *p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0ULL;
}

__global__ void k_conj(const double2 *__restrict__ in, double2 *__restrict__ out, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = make_double2(in[i].x, -in[i].y);
}

__global__ void k_zero_c128(double2 *u, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) u[i] = make_double2(0.0, 0.0);
}

// blocks of t threads covering n items; a launch must stay below 2^32
// work-items (a larger one would run only part of its grid)
inline int nblk(int64_t n, int t)
{
    if (n > ((int64_t)1 << 32) - t) throw Error{BFSFT_EINVAL, "a launch would exceed 2^32 work-items"};
    return (int)((n + t - 1) / t);
}

}  // namespace

void build_tables(Tables &tb, int p, int64_t N, int L, Arena &arena, hipStream_t s)
{
    tb.R64 = (double *)arena.alloc(sizeof(double) * 2 * p * p);
    tb.R32 = (float *)arena.alloc(sizeof(float) * 2 * p * p);
    tb.C64 = (double *)arena.alloc(sizeof(double2) * 4 * p);
    tb.C32 = (float *)arena.alloc(sizeof(float2) * 4 * p);
    tb.erot = (double *)arena.alloc(sizeof(double2) * p);
    tb.L64 = (double *)arena.alloc(sizeof(double2) * 2 * p * p);
    tb.PH64 = (double *)arena.alloc(sizeof(double2) * 2 * p);
    tb.nodes = (double *)arena.alloc(sizeof(double2) * p);
    tb.bary = (double *)arena.alloc(sizeof(double2) * p);
    tb.node_turns = (double *)arena.alloc(sizeof(double) * p);
    k_tables<<<1, 64, 0, s>>>(p, N, L, (double2 *)tb.L64, (double2 *)tb.PH64, tb.R64, tb.R32,
                              (double2 *)tb.C64, (float2 *)tb.C32, (double2 *)tb.erot,
                              (double2 *)tb.nodes, (double2 *)tb.bary, tb.node_turns);
    BF_HIP(hipGetLastError());
    if (p >= 5 && p <= 9) {
        tb.mf = (double *)arena.alloc(sizeof(double) * translate_mfma_table_doubles(p));
        build_mfma_tables(tb, p, tb.mf, s);
    }
}

void build_start(StartLevel &st, const Tree &tk, int s0, int d, int q, double rho, Arena &arena, hipStream_t s)
{
    st.s0 = s0;
    if (s0 == 0 || tk.npts == 0) return;
    const int L = tk.L, l0 = L - s0;
    // leaves under every box of T_K level l0, composed from the child ranges
    std::vector<int2> br((size_t)tk.count[l0]);
    for (int64_t b = 0; b < tk.count[l0]; ++b) {
        int32_t lo = (int32_t)b, hi = (int32_t)b + 1;
        for (int m = l0; m < L; ++m) {
            lo = tk.child_beg_host[m][lo];
            hi = tk.child_beg_host[m][hi];
        }
        br[(size_t)b] = make_int2(lo, hi);
    }
    st.box_leaf = (int2 *)arena.alloc(sizeof(int2) * br.size());
    BF_HIP(hipMemcpyAsync(st.box_leaf, br.data(), sizeof(int2) * br.size(), hipMemcpyHostToDevice, s));
    st.sm = (int32_t *)arena.alloc(sizeof(int32_t) * (size_t)tk.npts * d);
    st.sloc = (double *)arena.alloc(sizeof(double) * (size_t)tk.npts * d);
    st.sratio = (double2 *)arena.alloc(sizeof(double2) * (size_t)tk.npts * d);
    if (d == 2)
        k_source_offsets<2><<<nblk(tk.npts, 256), 256, 0, s>>>(tk.npts, s0, q, rho, tk.perm, tk.leaf_of,
                                                               tk.keys[L], tk.local, st.sm, st.sloc, st.sratio);
    else
        k_source_offsets<3><<<nblk(tk.npts, 256), 256, 0, s>>>(tk.npts, s0, q, rho, tk.perm, tk.leaf_of,
                                                               tk.keys[L], tk.local, st.sm, st.sloc, st.sratio);
    BF_HIP(hipGetLastError());
    BF_HIP(hipStreamSynchronize(s));  // br is a host temporary
}

constexpr int kDirectG = 3;  // grid lines per thread of the direct sums

DirectDesc direct_desc(const StartLevel &st, const double *f, const Tree &tx, const Tree &tk, int64_t N,
                       const Tables &tb, void *state)
{
    DirectDesc d;
    d.s0 = st.s0;
    d.L = tk.L;
    d.N = N;
    d.nA = tx.count[st.s0];
    d.nB = tk.count[tk.L - st.s0];
    d.xkeys = tx.keys[st.s0];
    d.box_leaf = st.box_leaf;
    d.steps = st.steps;
    d.wg_first = st.wg_first;
    d.nwg = st.nwg;
    d.nwaves = st.nwaves;
    d.gam = st.gam;
    d.geo = st.geo;
    d.nk = tk.npts;
    d.leaf_beg = tk.leaf_beg;
    d.perm = tk.perm;
    d.sm = st.sm;
    d.sloc = st.sloc;
    d.sstep = st.sratio;
    d.f = (const double2 *)f;
    d.erot = (const double2 *)tb.erot;
    d.state = state;
    d.first = 0;
    return d;
}

int64_t direct_items(int d, int p, const DirectDesc &dd)
{
    const int ng = (p + kDirectG - 1) / kDirectG;
    const int64_t n = dd.nA * dd.nB * (d == 2 ? ng : p * ng);
    if (n >= ((int64_t)1 << 31)) throw Error{BFSFT_EINVAL, "start level: too many direct-sum items"};
    return n;
}

void launch_direct(const Launch &c, const StartLevel &st, const double *f, const Tree &tx, const Tree &tk,
                   int64_t N, void *state)
{
    const DirectDesc dd = direct_desc(st, f, tx, tk, N, *c.tb, state);
    if (st.kind == 1) {
        launch_direct_mfma(c, dd);
        return;
    }
    const int64_t n = direct_items(c.d, c.p, dd);
    if (n == 0) return;
    const bool f32 = c.precision != BFSFT_FP64;
    auto go = [&](auto dim, auto tag) {
        constexpr int D = decltype(dim)::value;
        constexpr int P = decltype(tag)::value;
        if (f32)
            k_direct<D, P, kDirectG, float><<<nblk(n, 256), 256, 0, c.stream>>>(dd);
        else
            k_direct<D, P, kDirectG, double><<<nblk(n, 256), 256, 0, c.stream>>>(dd);
    };
    if (c.d == 2)
        dispatch_p(c.p, [&](auto tag) { go(std::integral_constant<int, 2>{}, tag); });
    else
        dispatch_p3(c.p, [&](auto tag) { go(std::integral_constant<int, 3>{}, tag); });
    BF_HIP(hipGetLastError());
}

void launch_direct_batched(const Launch &c, const DirectDesc *ds, const int64_t *prefix, int n, int64_t total)
{
    if (total == 0) return;
    const bool f32 = c.precision != BFSFT_FP64;
    const int g = nblk(total, 256);
    auto go = [&](auto dim, auto tag) {
        constexpr int D = decltype(dim)::value;
        constexpr int P = decltype(tag)::value;
        if (f32)
            k_direct_batched<D, P, kDirectG, float><<<g, 256, 0, c.stream>>>(ds, prefix, n, total);
        else
            k_direct_batched<D, P, kDirectG, double><<<g, 256, 0, c.stream>>>(ds, prefix, n, total);
    };
    if (c.d == 2)
        dispatch_p(c.p, [&](auto tag) { go(std::integral_constant<int, 2>{}, tag); });
    else
        dispatch_p3(c.p, [&](auto tag) { go(std::integral_constant<int, 3>{}, tag); });
    BF_HIP(hipGetLastError());
}

void launch_leaf(const Launch &c, const double *f, const Tree &tk, double rho, void *state)
{
    const int64_t nl = tk.count[tk.L];
    int PD = c.p;
    for (int a = 1; a < c.d; ++a) PD *= c.p;
    const int64_t n = nl * PD;
    if (n == 0) return;
    const bool f32 = c.precision != BFSFT_FP64;
    const double sh = 0.5 * rho;
    if (c.d == 2) {
        if (f32)
            k_leaf<2, float><<<nblk(n, 256), 256, 0, c.stream>>>(c.p, nl, (const double2 *)f, tk.perm,
                                                               tk.leaf_beg, tk.local, sh, (float2 *)state);
        else
            k_leaf<2, double><<<nblk(n, 256), 256, 0, c.stream>>>(c.p, nl, (const double2 *)f, tk.perm,
                                                                tk.leaf_beg, tk.local, sh, (double2 *)state);
    } else {
        if (f32)
            k_leaf<3, float><<<nblk(n, 256), 256, 0, c.stream>>>(c.p, nl, (const double2 *)f, tk.perm,
                                                               tk.leaf_beg, tk.local, sh, (float2 *)state);
        else
            k_leaf<3, double><<<nblk(n, 256), 256, 0, c.stream>>>(c.p, nl, (const double2 *)f, tk.perm,
                                                                tk.leaf_beg, tk.local, sh, (double2 *)state);
    }
    BF_HIP(hipGetLastError());
}

void launch_final(const Launch &c, const void *state, const Tree &tx, double, int64_t nx, double *u)
{
    if (nx == 0) return;
    const bool f32 = c.precision != BFSFT_FP64;
    dispatch_p(c.p, [&](auto tag) {
        constexpr int P = decltype(tag)::value;
        if (c.d == 2) {  // two lanes per target (k_final2)
            if (f32)
                k_final2<P, float><<<nblk(2 * nx, 256), 256, 0, c.stream>>>(
                    nx, (const float2 *)state, tx.leaf_of, tx.local, (const double2 *)c.tb->bary,
                    c.tb->node_turns, (const double2 *)c.tb->erot, (double2 *)u);
            else
                k_final2<P, double><<<nblk(2 * nx, 256), 256, 0, c.stream>>>(
                    nx, (const double2 *)state, tx.leaf_of, tx.local, (const double2 *)c.tb->bary,
                    c.tb->node_turns, (const double2 *)c.tb->erot, (double2 *)u);
        } else if constexpr (P <= 8) {
            if (f32)
                k_final<3, P, float><<<nblk(nx, 256), 256, 0, c.stream>>>(
                    nx, (const float2 *)state, tx.leaf_of, tx.local, (const double2 *)c.tb->bary,
                    c.tb->node_turns, (const double2 *)c.tb->erot, (double2 *)u);
            else
                k_final<3, P, double><<<nblk(nx, 256), 256, 0, c.stream>>>(
                    nx, (const double2 *)state, tx.leaf_of, tx.local, (const double2 *)c.tb->bary,
                    c.tb->node_turns, (const double2 *)c.tb->erot, (double2 *)u);
        } else {
            throw Error{BFSFT_EINVAL, "p > 8 in 3D"};
        }
    });
    BF_HIP(hipGetLastError());
}

void launch_export(const Launch &c, const void *state, const uint64_t *xkeys, int64_t nA,
                   const uint64_t *kkeys, int64_t nB, int lvl, int L, int64_t N, double *pot)
{
    int PD = c.p;
    for (int a = 1; a < c.d; ++a) PD *= c.p;
    const int64_t n = nA * nB * PD;
    if (n == 0) return;
    if (c.precision == BFSFT_FP64)
        k_export<double><<<nblk(n, 256), 256, 0, c.stream>>>(c.d, c.p, (const double2 *)state, xkeys,
                                                            nA, kkeys, nB, lvl, L, N, (double2 *)pot);
    else
        k_export<float><<<nblk(n, 256), 256, 0, c.stream>>>(c.d, c.p, (const float2 *)state, xkeys,
                                                           nA, kkeys, nB, lvl, L, N, (double2 *)pot);
    BF_HIP(hipGetLastError());
}

void launch_zero_u64(unsigned long long *p, int64_t n, hipStream_t s)
{
    if (n <= 0) return;
    k_zero_u64<<<nblk(n, 256), 256, 0, s>>>(p, n);
    BF_HIP(hipGetLastError());
}

void launch_conj(const double *in, double *out, int64_t n, hipStream_t s)
{
    if (n <= 0) return;
    k_conj<<<nblk(n, 256), 256, 0, s>>>((const double2 *)in, (double2 *)out, n);
    BF_HIP(hipGetLastError());
}

void launch_zero_c128(double *u, int64_t n, hipStream_t s)
{
    if (n == 0) return;
    k_zero_c128<<<nblk(n, 256), 256, 0, s>>>((double2 *)u, n);
    BF_HIP(hipGetLastError());
}

void launch_sigma(const uint64_t *keys, int64_t n, int d, int m, int L, int64_t N, double *sig,
                  hipStream_t s)
{
    if (n == 0) return;
    k_sigma<<<nblk(n, 256), 256, 0, s>>>(keys, n, d, m, L, N, (double2 *)sig);
    BF_HIP(hipGetLastError());
}

void launch_leaf_batched(const Launch &c, const LeafDesc *ds, const int64_t *prefix, int n,
                         int64_t total)
{
    if (total == 0) return;
    const bool f32 = c.precision != BFSFT_FP64;
    const int g = nblk(total, 256);
    if (c.d == 2) {
        if (f32) k_leaf_batched<2, float><<<g, 256, 0, c.stream>>>(c.p, ds, prefix, n, total);
        else k_leaf_batched<2, double><<<g, 256, 0, c.stream>>>(c.p, ds, prefix, n, total);
    } else {
        if (f32) k_leaf_batched<3, float><<<g, 256, 0, c.stream>>>(c.p, ds, prefix, n, total);
        else k_leaf_batched<3, double><<<g, 256, 0, c.stream>>>(c.p, ds, prefix, n, total);
    }
    BF_HIP(hipGetLastError());
}

void launch_final_batched(const Launch &c, const FinalDesc *ds, const int64_t *prefix, int n,
                          int64_t total)
{
    if (total == 0) return;
    const bool f32 = c.precision != BFSFT_FP64;
    const int g = nblk(total, 256);
    dispatch_p(c.p, [&](auto tag) {
        constexpr int P = decltype(tag)::value;
        if (c.d == 2) {
            if (f32) k_final_batched<2, P, float><<<g, 256, 0, c.stream>>>(ds, prefix, n, total);
            else k_final_batched<2, P, double><<<g, 256, 0, c.stream>>>(ds, prefix, n, total);
        } else if constexpr (P <= 8) {
            if (f32) k_final_batched<3, P, float><<<g, 256, 0, c.stream>>>(ds, prefix, n, total);
            else k_final_batched<3, P, double><<<g, 256, 0, c.stream>>>(ds, prefix, n, total);
        } else {
            throw Error{BFSFT_EINVAL, "p > 8 in 3D"};
        }
    });
    BF_HIP(hipGetLastError());
}

}  // namespace bfsft
