// Start-level direct sums on the FP64 matrix cores.
//
// The check potentials of a pair (A at T_X level s0, B at T_K level L - s0)
// at grid point l (Section 2.1, summed directly over the sources in B) have
// the phase (q i_A + l) . delta_j / (q 2^s0) per axis, delta_j = k_j - c^B.
// It splits into a part that depends on A and the source only and a part
// that depends on the source and the grid point only:
//     w^{AB}_l = sum_j Gamma[A][j] T_j[l],
//     Gamma[A][j] = exp(2 pi i sum_a i_{A,a} delta_{j,a} / 2^s0),
//     T_j[l]      = f_j prod_a exp(2 pi i l_a delta_{j,a} / (q 2^s0)).
// For one B this is a complex matrix product (rows: the A boxes, inner
// index: the sources of B, columns: the p^d grid points), computed here as
// four real products on v_mfma_f64_16x16x4f64.  The state rotation E[l_a]
// of every axis is folded into T: E[l] = E[1]^l, so it joins the chains of
// the phase steps.
//
// Gamma is exact to rounding: delta = rho m + loc (m = leaf index mod 2^s0,
// an integer; loc = offset inside the leaf), and the turns i_A rho m / 2^s0
// = (i_A m N mod 2^E) / 2^E with E = s0 + L are reduced in 64-bit integers
// (the product wraps modulo 2^64, a multiple of 2^E); the loc part is below
// one turn per axis.  T takes the phase steps
// beta_a = exp(2 pi i delta_a / (q 2^s0)) of every source and chains their
// powers (at most 2 (p - 1) products per entry).
#include "bfsft_impl.h"
#include "cplx.h"
#include "dispatch.h"

#include <algorithm>
#include <cstdlib>
#include <cstring>

namespace bfsft {

namespace {

typedef double dx4 __attribute__((ext_vector_type(4)));

constexpr int kChunk = 16;  // sources of B per LDS chunk: four K-steps of 4

template <int D, int P> struct DirectShape {
    static constexpr int PD = D == 2 ? P * P : P * P * P;  // grid points (columns)
    // p^d = 16 k + 1 (p = 7, 9 in 2D): the last column is summed by the
    // producers instead of padding a whole 16-column tile for it
    static constexpr int XC = (PD % 16 == 1 && PD > 16) ? 1 : 0;
    static constexpr int NT = XC ? PD / 16 : (PD + 15) / 16;  // 16-column tiles on the matrix cores
    static constexpr int NC = NT * 16;                        // their columns
    static constexpr int NR = PD / P;                         // column rows of P points: leading indices
};

template <int D, int P> constexpr bool mfma_shape_ok() { return DirectShape<D, P>::NT <= 9; }

__device__ __forceinline__ double2 cpow_chain(double2 b, int n)
{
    double2 r = make_double2(1.0, 0.0);
    for (int e = 0; e < n; ++e) r = cmul(r, b);
    return r;
}

// inputs of one source held by a producer lane
template <int D> struct SourceRegs {
    double fx, fy;
    double bx[D], by[D];
    double loc[D];
    int m[D];
};

constexpr int kProducers = 4;  // producer waves per work-group
// consumer waves (16-row tiles) per work-group: two per SIMD where the
// accumulators of a tile fit three waves per SIMD (at most 6 column tiles),
// else one
constexpr int max_consumers(int nt) { return nt <= 6 ? 8 : 4; }

// Persistent work-groups of W consumer waves (W = 1..8: one per 16-row tile
// of a block of A rows; two per SIMD keep the matrix cores busy, one does
// not reach half their rate) and four producer waves.  A step is one chunk of at
// most 16 sources of a box B for one block of 16 W rows; the steps of one
// (block, B) item are consecutive and every work-group walks its own
// contiguous range of steps (built at plan time, balanced, cut at item
// ends).  While the consumers run the products of step s on the matrix
// cores (their instruction stream is LDS reads and MFMAs only), the
// producers build T, Gamma and the descriptor of step s + 1 into the other
// LDS buffer on the VALU of the same SIMDs and issue the loads of the steps
// after it: source inputs one step ahead, the source permutation two,
// descriptors three.  One barrier per step.
//
// Producer lane (source j = tp mod 16, group g = tp / 16 of its 256
// lanes): T rows g and g + 16 (leading grid indices), Gamma rows g + 16 k.
//
// Operands of v_mfma_f64_16x16x4f64: lane i + 16 kq holds A[i][kq] and
// B[kq][i]; register r of the result holds D[4 r + kq][i].  Here A = Gamma
// (row i: A box, kq: source), B = T (kq: source, i: grid point).
template <int D, int P, typename S, bool PRE>
__global__ __launch_bounds__(64 * (max_consumers(DirectShape<D, P>::NT) + kProducers), 1) void k_direct_mfma(DirectDesc dd)
{
    using SH = DirectShape<D, P>;
    constexpr int PD = SH::PD, NT = SH::NT, NC = SH::NC, NR = SH::NR;
    constexpr int MAXC = max_consumers(NT);
    constexpr int XC = SH::XC;
    constexpr int TS = (XC ? PD : NC) + 1, GS = kChunk + 1;  // padded row strides (no bank conflicts)
    __shared__ double2 sT[2][kChunk][TS];
    __shared__ double2 sG[2][16 * MAXC][GS];
    __shared__ int4 s_desc[2];  // descriptor of the step held in each buffer

    const int W = (int)(blockDim.x >> 6) - kProducers;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nB = (int)dd.nB, nA = (int)dd.nA;

    // work-groups numbered so that consecutive ranges (adjacent boxes B,
    // adjacent state segments) run on one XCD: the hardware deals
    // work-groups to the 8 XCDs round-robin (a bijection of [0, nblk))
    const int nblk = gridDim.x, bid = blockIdx.x;
    const int q8 = nblk >> 3, r8 = nblk & 7, x = bid & 7;
    const int lw = x * q8 + min(x, r8) + (bid >> 3);
    const int s_beg = dd.wg_first[lw], s_end = dd.wg_first[lw + 1];
    if (s_beg >= s_end) return;  // the whole work-group

    // step descriptor: x first source, y count | first << 8 | last << 9,
    // z box b, w row block.  Loaded clamped to the range (a uniform load
    // with no branch); `valid` gives count 0 past the range where it is
    // used, long after the load
    auto step = [&](int s) { return dd.steps[min(s, s_end - 1)]; };
    auto valid = [&](int4 q, int s) {
        q.y = s < s_end ? q.y : 0;
        return q;
    };
    auto count = [](const int4 &q) { return q.y & 255; };

    for (int e = threadIdx.x; e < 2 * kChunk * (TS - PD); e += blockDim.x) {
        const int buf = e / (kChunk * (TS - PD)), rem = e - buf * kChunk * (TS - PD);
        const int j = rem / (TS - PD);
        sT[buf][j][PD + rem - j * (TS - PD)] = make_double2(0.0, 0.0);
    }
    __syncthreads();  // padding in place

    if (wave < W) {
        // ------------------------------------------------------ consumer
        const int i = lane & 15, kq = lane >> 4;
        using SV = typename CV<S>::t;
        SV *out = (SV *)dd.state;
        dx4 cre[NT], cim[NT];
#pragma unroll
        for (int nt = 0; nt < NT; ++nt) {
            cre[nt] = dx4{0.0, 0.0, 0.0, 0.0};
            cim[nt] = dx4{0.0, 0.0, 0.0, 0.0};
        }
        double2 xsum = make_double2(0.0, 0.0);  // last column (XC): this lane's sources of row i
        __syncthreads();  // step s_beg built
        for (int s = s_beg; s < s_end; ++s) {
            const int buf = (s - s_beg) & 1;
            const int4 d = s_desc[buf];
            const int row0 = (d.w * W + wave) * 16;
            if (row0 < nA) {
                const int nks = (count(d) + 3) >> 2;
                const double2 *grow = &sG[buf][wave * 16 + i][0];
                // operands of K-step ks into (g, bv); products of one K-step
                // the last grid column (XC) rides along: its T entry with the
                // operands, one complex FMA per K-step on the VALU
                double2 xa = make_double2(0.0, 0.0), xta, xtb;
                auto fetch = [&](int ks, double2 &g, double2 (&bv)[NT], double2 &xt) {
                    const int jr = ks * 4 + kq;
                    g = grow[jr];
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) bv[nt] = sT[buf][jr][nt * 16 + i];
                    if (XC) xt = sT[buf][jr][PD - 1];
                };
                auto products = [&](const double2 &g, const double2 (&bv)[NT], const double2 &xt) {
                    if (XC) cfma(xa, g, xt);
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) {
                        cre[nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(g.x, bv[nt].x, cre[nt], 0, 0, 0);
                        cim[nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(g.x, bv[nt].y, cim[nt], 0, 0, 0);
                    }
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) {
                        cre[nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(-g.y, bv[nt].y, cre[nt], 0, 0, 0);
                        cim[nt] = __builtin_amdgcn_mfma_f64_16x16x4f64(g.y, bv[nt].x, cim[nt], 0, 0, 0);
                    }
                };
                // two operand sets in turn: the reads of K-step ks + 1 are
                // issued before the products of K-step ks
                double2 ga, gb, ba[NT], bb[NT];
                fetch(0, ga, ba, xta);
                if (nks > 1) fetch(1, gb, bb, xtb);
                __builtin_amdgcn_sched_barrier(0);
                products(ga, ba, xta);
                if (nks > 1) {
                    if (nks > 2) fetch(2, ga, ba, xta);
                    __builtin_amdgcn_sched_barrier(0);
                    products(gb, bb, xtb);
                }
                if (nks > 2) {
                    if (nks > 3) fetch(3, gb, bb, xtb);
                    __builtin_amdgcn_sched_barrier(0);
                    products(ga, ba, xta);
                }
                if (nks > 3) products(gb, bb, xtb);
                xsum = cadd(xsum, xa);
                if ((d.y >> 9) & 1) {  // the item's last step: its potentials
                    if (XC) {  // the last column: the four source lanes kq of row i
                        xsum.x += __shfl_xor(xsum.x, 16);
                        xsum.y += __shfl_xor(xsum.y, 16);
                        xsum.x += __shfl_xor(xsum.x, 32);
                        xsum.y += __shfl_xor(xsum.y, 32);
                        const int ar = row0 + i;
                        if (kq == 0 && ar < nA) {
                            SV v;
                            v.x = (S)xsum.x;
                            v.y = (S)xsum.y;
                            out[((int64_t)ar * nB + d.z) * PD + PD - 1] = v;
                        }
                        xsum = make_double2(0.0, 0.0);
                    }
#pragma unroll
                    for (int nt = 0; nt < NT; ++nt) {
                        const int col = nt * 16 + i;
#pragma unroll
                        for (int r = 0; r < 4; ++r) {
                            const int ar = row0 + 4 * r + kq;
                            if (col < PD && ar < nA) {
                                SV v;
                                v.x = (S)cre[nt][r];
                                v.y = (S)cim[nt][r];
                                out[((int64_t)ar * nB + d.z) * PD + col] = v;
                            }
                        }
                        cre[nt] = dx4{0.0, 0.0, 0.0, 0.0};
                        cim[nt] = dx4{0.0, 0.0, 0.0, 0.0};
                    }
                }
            }
            __syncthreads();  // step s + 1 built; buffer buf free
        }
        return;
    }

    // ---------------------------------------------------------- producer
    const int tp = (int)threadIdx.x - 64 * W;  // 0 .. 255
    const int j = tp & 15, grp = tp >> 4;
    constexpr int kRows = MAXC;                 // Gamma rows per lane: grp + 16 k
    // this lane's source of a step: a valid source index whether or not j
    // is below the step's count (no branch around the loads)
    auto lane_src = [&](const int4 &q) { return q.x + min(j, max(count(q) - 1, 0)); };

    if constexpr (PRE) {
        // Gamma and T / f from the plan-time tables: per step, loads, one
        // complex multiply per T entry and stores only
        constexpr int NRL = (NR + 15) / 16;  // T rows of this lane: grp, grp + 16
        struct PreRegs {
            double2 f;
            double2 g[kRows];
            double2 t[NRL][P];
        };
        const int64_t nk = dd.nk;
        auto load_pre = [&](const int4 &q, int pidx, PreRegs &r) {
            const int tt = lane_src(q);
            r.f = dd.f[pidx];
            const int base = q.w * 16 * W;
#pragma unroll
            for (int k = 0; k < kRows; ++k) r.g[k] = dd.gam[(int64_t)min(base + grp + 16 * k, nA - 1) * nk + tt];
#pragma unroll
            for (int rr = 0; rr < NRL; ++rr) {
                const double2 *src = dd.geo + (int64_t)tt * PD + min(grp + 16 * rr, NR - 1) * P;
#pragma unroll
                for (int l = 0; l < P; ++l) r.t[rr][l] = src[l];
            }
        };
        auto build_pre = [&](int buf, const int4 &q, const PreRegs &r) {
            if (tp == 0) s_desc[buf] = q;
            const bool on = j < count(q);
#pragma unroll
            for (int rr = 0; rr < NRL; ++rr) {
                const int row = grp + 16 * rr;
                if (row >= NR) break;
                double2 *dst = &sT[buf][j][row * P];
#pragma unroll
                for (int l = 0; l < P; ++l) dst[l] = on ? cmul(r.f, r.t[rr][l]) : make_double2(0.0, 0.0);
            }
            const int base = q.w * 16 * W;
#pragma unroll
            for (int k = 0; k < kRows; ++k) {
                const int rr = grp + 16 * k;
                if (rr >= 16 * W) break;
                sG[buf][rr][j] = (on && base + rr < nA) ? r.g[k] : make_double2(0.0, 0.0);
            }
        };
        int4 d1 = step(s_beg + 1), d2 = step(s_beg + 2), d3 = step(s_beg + 3);
        PreRegs r;
        {
            const int4 d0 = step(s_beg);
            load_pre(d0, dd.perm[lane_src(d0)], r);
            build_pre(0, d0, r);
        }
        load_pre(d1, dd.perm[lane_src(d1)], r);
        int pn = dd.perm[lane_src(d2)];
        __syncthreads();
        for (int s = s_beg; s < s_end; ++s) {
            const int4 d4 = step(s + 4);
            const int4 q1 = valid(d1, s + 1);
            if (count(q1) > 0) build_pre((s + 1 - s_beg) & 1, q1, r);
            // loads of step s + 2 and the source permutation of step s + 3
            load_pre(d2, pn, r);
            pn = dd.perm[lane_src(d3)];
            d1 = d2;
            d2 = d3;
            d3 = d4;
            __syncthreads();  // step s + 1 built; buffer of step s free
        }
        return;
    }

    const int E = dd.s0 + dd.L;
    const uint64_t mask = (1ull << E) - 1ull;
    const double inv_2E = ldexp(1.0, -E), inv_2s0 = ldexp(1.0, -dd.s0);
    const uint64_t N = (uint64_t)dd.N;
    // the rotation E[l] = E[1]^l joins the phase steps: beta E[1] per axis
    const double2 e1 = dd.erot[1];

    auto load_inputs = [&](int tt, int pidx, SourceRegs<D> &r) {
        const double2 fv = dd.f[pidx];
        r.fx = fv.x;
        r.fy = fv.y;
#pragma unroll
        for (int ax = 0; ax < D; ++ax) {
            const double2 bv = dd.sstep[(int64_t)tt * D + ax];
            r.bx[ax] = bv.x;
            r.by[ax] = bv.y;
            r.loc[ax] = dd.sloc[(int64_t)tt * D + ax];
            r.m[ax] = dd.sm[(int64_t)tt * D + ax];
        }
    };
    // Morton keys of this lane's Gamma rows in row block blk (rows past nA
    // read a valid key that is never used)
    auto row_keys = [&](int blk, uint64_t (&key)[kRows]) {
#pragma unroll
        for (int k = 0; k < kRows; ++k) key[k] = dd.xkeys[min(blk * 16 * W + grp + 16 * k, nA - 1)];
    };
    auto decode = [&](const uint64_t (&key)[kRows], int (&iA)[kRows][D]) {
#pragma unroll
        for (int k = 0; k < kRows; ++k)
#pragma unroll
            for (int ax = 0; ax < D; ++ax) {
                int v = 0;  // below 2^s0 <= 2^18
                for (int bit = 0; bit < dd.s0; ++bit) v |= (int)((key[k] >> (bit * D + ax)) & 1) << bit;
                iA[k][ax] = v;
            }
    };
    // T rows and Gamma entries of one step into buffer buf
    auto build = [&](int buf, const int4 &q, const SourceRegs<D> &r, const int (&iA)[kRows][D]) {
        if (tp == 0) s_desc[buf] = q;
        const bool on = j < count(q);
        const double2 f = make_double2(r.fx, r.fy);
        for (int row = grp; row < NR; row += 16) {
            double2 *dst = &sT[buf][j][row * P];
            if (!on) {
#pragma unroll
                for (int l = 0; l < P; ++l) dst[l] = make_double2(0.0, 0.0);
                continue;
            }
            double2 w = f;
            if (D == 2) {
                w = cmul(w, cpow_chain(cmul(make_double2(r.bx[0], r.by[0]), e1), row));
            } else {
                const int l0 = row / P, l1 = row - l0 * P;
                w = cmul(w, cpow_chain(cmul(make_double2(r.bx[0], r.by[0]), e1), l0));
                w = cmul(w, cpow_chain(cmul(make_double2(r.bx[D == 3 ? 1 : 0], r.by[D == 3 ? 1 : 0]), e1), l1));
            }
            const double2 bl = cmul(make_double2(r.bx[D - 1], r.by[D - 1]), e1);
#pragma unroll
            for (int l = 0; l < P; ++l) {
                dst[l] = w;
                w = cmul(w, bl);
            }
        }
        const int blk = q.w;
#pragma unroll
        for (int k = 0; k < kRows; ++k) {
            const int rr = grp + 16 * k;
            if (rr >= 16 * W) break;
            double2 g = make_double2(0.0, 0.0);
            if (on && blk * 16 * W + rr < nA) {
                double th = 0.0;
#pragma unroll
                for (int ax = 0; ax < D; ++ax) {
                    const uint64_t red = ((uint64_t)iA[k][ax] * (uint64_t)r.m[ax] * N) & mask;
                    th += (double)red * inv_2E + (double)iA[k][ax] * r.loc[ax] * inv_2s0;
                }
                double sn, cs;
                sincospi(2.0 * th, &sn, &cs);
                g = make_double2(cs, sn);
            }
            sG[buf][rr][j] = g;
        }
    };

    // prologue: build step s_beg; inputs of step s_beg + 1, the permutation
    // of step s_beg + 2 and the descriptor of step s_beg + 3 in flight.
    // In the loop, dK is the raw descriptor of step s + K.
    int4 d1 = step(s_beg + 1), d2 = step(s_beg + 2), d3 = step(s_beg + 3);
    int iA[kRows][D];
    uint64_t keys[kRows];
    {
        const int4 d0 = step(s_beg);
        SourceRegs<D> r0;
        const int tt = lane_src(d0);
        load_inputs(tt, dd.perm[tt], r0);
        row_keys(d0.w, keys);
        decode(keys, iA);
        build(0, d0, r0, iA);
    }
    SourceRegs<D> nxt;
    {
        const int tt = lane_src(d1);
        load_inputs(tt, dd.perm[tt], nxt);
    }
    int pn = dd.perm[lane_src(d2)];
    row_keys(d1.w, keys);
    __syncthreads();
    for (int s = s_beg; s < s_end; ++s) {
        const int4 d4 = step(s + 4);  // in flight during the build
        // build step s + 1 (inputs in nxt, row keys in keys) into the other buffer
        const int4 q1 = valid(d1, s + 1);
        if (count(q1) > 0) {
            if ((q1.y >> 8) & 1) decode(keys, iA);
            build((s + 1 - s_beg) & 1, q1, nxt, iA);
        }
        // loads for the steps ahead: inputs and row keys of s + 2,
        // permutation of s + 3 (all unconditional)
        load_inputs(lane_src(d2), pn, nxt);
        row_keys(d2.w, keys);
        pn = dd.perm[lane_src(d3)];
        d1 = d2;
        d2 = d3;
        d3 = d4;
        __syncthreads();  // step s + 1 built; buffer of step s free
    }
}

// Plan-time tables of the matrix-core direct sums (the parts that depend on
// the points only; the same formulas the producers evaluate otherwise).
// Gamma[a][t]: one thread per (A box a, source t in sorted order).
template <int D>
__global__ void k_gamma_table(int64_t nA, int64_t nk, int s0, int L, int64_t Nv, const uint64_t *__restrict__ xkeys,
                              const int32_t *__restrict__ sm, const double *__restrict__ sloc,
                              double2 *__restrict__ gam)
{
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nA * nk) return;
    const int64_t a = e / nk, t = e - a * nk;
    const uint64_t key = xkeys[a];
    const int E = s0 + L;
    const uint64_t mask = (1ull << E) - 1ull, N = (uint64_t)Nv;
    double th = 0.0;
#pragma unroll
    for (int ax = 0; ax < D; ++ax) {
        uint64_t iA = 0;
        for (int bit = 0; bit < s0; ++bit) iA |= ((key >> (bit * D + ax)) & 1ull) << bit;
        const uint64_t red = (iA * (uint64_t)sm[t * D + ax] * N) & mask;
        th += (double)red * ldexp(1.0, -E) + (double)iA * sloc[t * D + ax] * ldexp(1.0, -s0);
    }
    double sn, cs;
    sincospi(2.0 * th, &sn, &cs);
    gam[e] = make_double2(cs, sn);
}

// T_j[l] / f_j = prod_a (beta_a E[1])^{l_a}: one thread per (source t,
// leading grid indices r), p entries along the last axis
template <int D, int P>
__global__ void k_geo_table(int64_t nk, const double2 *__restrict__ sstep, const double2 *__restrict__ erot,
                            double2 *__restrict__ geo)
{
    constexpr int PD = D == 2 ? P * P : P * P * P, NR = PD / P;
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= nk * NR) return;
    const int64_t t = e / NR;
    const int r = (int)(e - t * NR);
    const double2 e1 = erot[1];
    double2 w = make_double2(1.0, 0.0);
    if (D == 2) {
        w = cpow_chain(cmul(sstep[t * D], e1), r);
    } else {
        const int l0 = r / P, l1 = r - l0 * P;
        w = cmul(cpow_chain(cmul(sstep[t * D], e1), l0), cpow_chain(cmul(sstep[t * D + (D == 3 ? 1 : 0)], e1), l1));
    }
    const double2 bl = cmul(sstep[t * D + D - 1], e1);
    double2 *dst = geo + t * PD + (int64_t)r * P;
#pragma unroll
    for (int l = 0; l < P; ++l) {
        dst[l] = w;
        w = cmul(w, bl);
    }
}

}  // namespace

bool direct_mfma_supported(int d, int p)
{
    return (d == 2 && p >= 3 && p <= 12) || (d == 3 && p >= 3 && p <= 5);
}

int direct_kinds(int d, int p)
{
    const bool mfma = direct_mfma_supported(d, p);
    if (const char *e = std::getenv("BFSFT_DIRECT")) {
        if (std::strcmp(e, "valu") == 0) return 1;
        if (std::strcmp(e, "mfma") == 0) return mfma ? 2 : 1;
    }
    return mfma ? 3 : 1;
}

// consumer waves per work-group for nA rows: one 16-row tile each
int direct_mfma_waves(int d, int p, int64_t nA)
{
    const int pd = d == 2 ? p * p : p * p * p;
    const int nt = (pd % 16 == 1 && pd > 16) ? pd / 16 : (pd + 15) / 16;  // as DirectShape::NT
    return (int)std::max<int64_t>(1, std::min<int64_t>(max_consumers(nt), (nA + 15) / 16));
}

template <typename F> void dispatch_direct(int d, int p, bool f32, bool pre, F &&f)
{
    auto go = [&](auto dim, auto tag) {
        constexpr int D = decltype(dim)::value;
        constexpr int Pc = decltype(tag)::value;
        if constexpr (mfma_shape_ok<D, Pc>()) {
            if (f32)
                pre ? f(k_direct_mfma<D, Pc, float, true>) : f(k_direct_mfma<D, Pc, float, false>);
            else
                pre ? f(k_direct_mfma<D, Pc, double, true>) : f(k_direct_mfma<D, Pc, double, false>);
        }
    };
    if (d == 2)
        dispatch_p(p, [&](auto tag) { go(std::integral_constant<int, 2>{}, tag); });
    else
        dispatch_p3(p, [&](auto tag) {
            if constexpr (decltype(tag)::value <= 5) go(std::integral_constant<int, 3>{}, tag);
        });
}

// budget of the plan-time tables (BFSFT_DIRECT_TABLE_MB, default 2048 MB;
// 0 disables them)
int64_t direct_table_budget()
{
    int64_t mb = 2048;
    if (const char *e = std::getenv("BFSFT_DIRECT_TABLE_MB")) {
        char *end = nullptr;
        const long long v = std::strtoll(e, &end, 10);
        if (end != e && v >= 0) mb = v;
    }
    return mb << 20;
}

void build_direct_steps(StartLevel &st, const Tree &tx, const Tree &tk, const Tables &tb, int d, int p,
                        int64_t N, Arena &arena, hipStream_t s)
{
    if (!direct_mfma_supported(d, p)) throw Error{BFSFT_EINVAL, "matrix-core direct sums: unsupported (d, p)"};
    const int s0 = st.s0, L = tk.L, l0 = L - s0;
    const int64_t nA = tx.count[s0], nB = tk.count[l0];
    if (nA >= ((int64_t)1 << 30) || nB >= ((int64_t)1 << 30) || tk.npts >= ((int64_t)1 << 30))
        throw Error{BFSFT_EINVAL, "start level: too many boxes for the matrix-core direct sums"};
    if (s0 + L > 62) throw Error{BFSFT_EINVAL, "start level: phase reduction exceeds 64 bits"};
    // source range of every box B (the leaf ranges composed on the host)
    std::vector<int32_t> leaf_beg((size_t)tk.count[L] + 1);
    std::vector<int2> br((size_t)nB);
    BF_HIP(hipMemcpyAsync(leaf_beg.data(), tk.leaf_beg, sizeof(int32_t) * leaf_beg.size(), hipMemcpyDeviceToHost, s));
    BF_HIP(hipMemcpyAsync(br.data(), st.box_leaf, sizeof(int2) * br.size(), hipMemcpyDeviceToHost, s));
    BF_HIP(hipStreamSynchronize(s));
    const int w = direct_mfma_waves(d, p, nA);
    const int64_t blocks = (nA + 16 * w - 1) / (16 * w);
    std::vector<int4> steps;
    std::vector<int64_t> item_end;  // first step after each item
    for (int64_t blk = 0; blk < blocks; ++blk)
        for (int64_t b = 0; b < nB; ++b) {
            const int t0 = leaf_beg[(size_t)br[(size_t)b].x], t1 = leaf_beg[(size_t)br[(size_t)b].y];
            for (int tc = t0; tc < t1; tc += kChunk) {
                const int nc = std::min(kChunk, t1 - tc);
                const int flags = (tc == t0 ? 1 : 0) | (tc + kChunk >= t1 ? 2 : 0);
                steps.push_back(make_int4(tc, nc | (flags << 8), (int)b, (int)blk));
            }
            item_end.push_back((int64_t)steps.size());
        }
    if (steps.size() >= ((size_t)1 << 31)) throw Error{BFSFT_EINVAL, "start level: too many direct-sum steps"};
    // resident work-groups: the occupancy of the kernel at w waves on every CU
    int dev = 0, ncu = 0, per_cu = 0;
    BF_HIP(hipGetDevice(&dev));
    BF_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    // plan-time tables when they fit the budget and the plan's byte cap
    const int pd = d == 2 ? p * p : p * p * p;
    const int64_t nk = tk.npts;
    const int64_t table_bytes = (nA * nk + nk * pd) * (int64_t)sizeof(double2);
    const bool pre = table_bytes <= direct_table_budget() &&
                     (arena.cap < 0 || arena.bytes + table_bytes + (int64_t)(1 << 20) <= arena.cap);
    if (pre) {
        st.gam = (double2 *)arena.alloc(sizeof(double2) * (size_t)(nA * nk));
        st.geo = (double2 *)arena.alloc(sizeof(double2) * (size_t)(nk * pd));
        const int64_t ng = nA * nk;
        const int64_t nr = nk * (pd / p);
        const unsigned gg = (unsigned)((ng + 255) / 256), gr = (unsigned)((nr + 255) / 256);
        const double2 *erot = (const double2 *)tb.erot;
        if (d == 2)
            k_gamma_table<2><<<gg, 256, 0, s>>>(nA, nk, s0, L, N, tx.keys[s0], st.sm, st.sloc, st.gam);
        else
            k_gamma_table<3><<<gg, 256, 0, s>>>(nA, nk, s0, L, N, tx.keys[s0], st.sm, st.sloc, st.gam);
        auto geo = [&](auto dim, auto tag) {
            constexpr int D = decltype(dim)::value, Pc = decltype(tag)::value;
            k_geo_table<D, Pc><<<gr, 256, 0, s>>>(nk, st.sratio, erot, st.geo);
        };
        if (d == 2)
            dispatch_p(p, [&](auto tag) { geo(std::integral_constant<int, 2>{}, tag); });
        else
            dispatch_p3(p, [&](auto tag) {
                if constexpr (decltype(tag)::value <= 5) geo(std::integral_constant<int, 3>{}, tag);
            });
        BF_HIP(hipGetLastError());
    }
    dispatch_direct(d, p, false, pre, [&](auto kern) {
        BF_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 64 * (w + kProducers), 0));
    });
    const int64_t items = (int64_t)item_end.size();
    const int64_t nwg = std::max<int64_t>(1, std::min<int64_t>(items, (int64_t)std::max(1, ncu) * std::max(1, per_cu)));
    // contiguous ranges of about equal step counts, cut at item ends
    std::vector<int32_t> first((size_t)nwg + 1, 0);
    const double total = (double)steps.size();
    int64_t it = 0;
    for (int64_t g = 1; g < nwg; ++g) {
        const double target = total * (double)g / (double)nwg;
        while (it < items && (double)item_end[(size_t)it] < target) ++it;
        // the item end nearest the target, not before the previous cut
        int64_t cut = it < items ? item_end[(size_t)it] : (int64_t)steps.size();
        if (it > 0 && it < items && target - (double)item_end[(size_t)it - 1] < (double)item_end[(size_t)it] - target)
            cut = item_end[(size_t)it - 1];
        first[(size_t)g] = (int32_t)std::max<int64_t>(first[(size_t)g - 1], cut);
    }
    first[(size_t)nwg] = (int32_t)steps.size();
    st.steps = (int4 *)arena.alloc(sizeof(int4) * std::max<size_t>(1, steps.size()));
    st.wg_first = (int32_t *)arena.alloc(sizeof(int32_t) * first.size());
    BF_HIP(hipMemcpyAsync(st.steps, steps.data(), sizeof(int4) * steps.size(), hipMemcpyHostToDevice, s));
    BF_HIP(hipMemcpyAsync(st.wg_first, first.data(), sizeof(int32_t) * first.size(), hipMemcpyHostToDevice, s));
    BF_HIP(hipStreamSynchronize(s));  // host vectors are temporaries
    st.nwg = (int)nwg;
    st.nwaves = w;
}

void launch_direct_mfma(const Launch &c, const DirectDesc &dd)
{
    if (dd.nA == 0 || dd.nB == 0) return;
    if (!dd.steps || !dd.wg_first || dd.nwg < 1 || dd.nwaves < 1 || dd.nwaves > 8)
        throw Error{BFSFT_EINVAL, "matrix-core direct sums: no step list"};
    dispatch_direct(c.d, c.p, c.precision != BFSFT_FP64, dd.gam != nullptr, [&](auto kern) {
        kern<<<(unsigned)dd.nwg, 64 * (dd.nwaves + kProducers), 0, c.stream>>>(dd);
    });
    BF_HIP(hipGetLastError());
}

}  // namespace bfsft
