// Step 3 of Section 2.2 (the level sweep) on gfx950.
//
// For a box pair (A, B) at T_K level l, A = child t of A' and B with
// children B_s, the state (B's check potential at A's check points, B's
// corner phase divided out; see kernels.hip for the derivation) is, per
// axis, interpolated from the children's states:
//
//   w^{AB}[l] = sum_s f(s, t, l) * (L_t w^{A'B_s})[l],
//   f(0, t, l) = 1,   f(1, t, l) = sigma_{A'} exp(i pi rho (t q + l) / q),
//   L_t[l][l'] = ell_{l'}( exp(i pi rho (t q + l) / q^2) ).
//
// The nodes and the targets of this interpolation lie on the unit circle,
// where the Lagrange basis is a phase times a real product of sines:
// L_t = diag(D_t) R_t diag(E) with R_t real and E[k] = exp(-i pi rho k / q).
// The state is therefore kept rotated, w^ = (E x E) w, and a level is
//
//   w^{AB}[l] = sum_s sigma^s G(s, t, l) (R_t w^{A'B_s})[l],
//   G(0, t, l) = exp(i pi rho (t q - l) / (2 q)),
//   G(1, t, l) = G(0, t, l) exp(i pi rho (t q + l) / q),
//
// so every contraction multiplies complex state by a real operator (two
// FMAs per term instead of four) and the phases are applied once per
// output.  The check point (t + l/q)/2 of A coincides with the node
// (t q + l)/2 / q of A' whenever t q + l is even; those rows of R_t are unit
// vectors, so about half of every 1D interpolation is a copy and only the
// other rows are dot products (4 of 9 at p = 9).  Which rows are copies
// depends only on (p, t), so it is resolved at compile time.
//
// Work decomposition.  A work-group takes R consecutive rows a' of T_X level
// L-l-1 and one tile of boxes b of T_K level l; the children of the tile are
// a contiguous range of every input row (Morton order), and the outputs are
// the rows a = children of each a'.
//   stage 1: one thread per input row (a', j, l): Y = R_t2 along axis 2 for
//            each output position t2 the row a' needs,
//   stage 2: one thread per (t2, a', b, m): sum the children with the same
//            s1, each times its G(s2, t2, m), apply R_t1 along axis 1 for
//            t1 = 0 and 1, combine the two sums with G(s1, t1, .), write.
// The operators of each stage depend only on t, so they are uniform across
// the work-group and read through scalar loads.  The per-item tables come
// from the trees' child-position slot words, one load per box and row.
#include "bfsft_impl.h"
#include "cplx.h"
#include "dispatch.h"
#include "translate2d.h"

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <type_traits>

namespace bfsft {

namespace {

using namespace tr;

// Whether the 3D work-group holds the axis-1 results of both output
// positions t1 at once (one box with all its children, 8 + 4 blocks, fits
// the LDS of a work-group); otherwise one t1 at a time (8 + 2 blocks).
template <int P, typename S> constexpr bool both3d()
{
    return (size_t)12 * P * P * P * sizeof(typename CV<S>::t) <= kLdsMax;
}

// Step 3, 3D (octrees, p^3 grids, axis 0 = l slowest, axis 2 = n fastest).
// Child positions s and output positions t carry the parity of axis a in bit
// a.  Per output position t2 along axis 2:
//   stage 1 (axis 2): rows (j, l, m):  Y1 = R_t2 along n,
//   stage 2 (axis 1): lines (b, e0, l, n): sum the children over bit 2, each
//                     times G(e2, t2, n) (and sigma of axis 2 for e2 = 1),
//                     then Y2[b][t1][e0] = sum over bit 1 of G(e1, t1, .)
//                     R_t1 along m, for both t1 from the same sums,
//   stage 3 (axis 0): lines (b, t1, m, n): out_t = sum over bit 0 of
//                     G(e0, t0, .) R_t0 along l, written to HBM.
// When Y2 has room for one t1 only, stages 2 and 3 run once per t1.
template <int P, bool RHO1, typename S, typename C>
__device__ __forceinline__ void translate3d_item(const TArgs &a, int64_t gid, unsigned char *smem)
{
    using Sv = typename CV<S>::t;
    using Cv = typename CV<C>::t;
    using Yv = typename YT<S, C>::t;
    constexpr int P2 = P * P, P3 = P * P * P;
    __shared__ int s_out[kRowsMax * 8];
    __shared__ int s_bits[kRowsMax];  // bit t: output t; bit 8+t2: some output with t2;
                                      // bit 16 + 2*t2 + t1: some output with (t1, t2)
    __shared__ Cv s_sig[kRowsMax * 3];
    __shared__ __align__(8) signed char s_cj[kInMax * 8];  // read as one 64-bit word per box
    __shared__ Cv s_gc[4 * P];  // G(s, t, l) as [2 s][2 t][P]: stage 2 reads it at the lane's n

    const int64_t g = gid / a.ntile;
    const int tile = (int)(gid - g * a.ntile);
    const int64_t ap0 = g * a.rows;
    const int R = (int)min((int64_t)a.rows, a.nap - ap0);
    const int4 bt = a.tiles[tile];
    const int b0 = bt.x, nb = bt.y - bt.x;
    const int J0 = bt.z;
    const int nin = bt.w - bt.z;
    constexpr bool BOTH = both3d<P, S>();
    constexpr int NT1 = BOTH ? 2 : 1;       // positions t1 per stage-2 pass
    Yv *Y1 = reinterpret_cast<Yv *>(smem);  // [R][nin][P3]
    Yv *Y2 = Y1 + R * nin * P3;             // [R][nb][NT1][2 e0][P3]

    // stage-1 rows (r, j, l, m) of the item, flattened; a thread's rows are
    // v = tid, tid + kTT, ...; loads are unconditional (clamped to the last
    // row), so the compiler does not wait for them where a branch joins
    const int rowlen = nin * P2;
    const int nrows = R * rowlen;
    const float inv_rowlen = 1.0f / (float)rowlen;
    const Sv *in0 = reinterpret_cast<const Sv *>(a.in) + (ap0 * a.in_row + J0) * P3;
    const int64_t in_rs = a.in_row * P3;
    auto load_row3 = [&](int v, Sv *xn) {
        v = min(v, nrows - 1);
        const int r = (int)(((float)v + 0.5f) * inv_rowlen);
        const Sv *src = in0 + r * in_rs + (v - r * rowlen) * P;
#pragma unroll
        for (int m = 0; m < P; ++m) xn[m] = src[m];
    };

    // tables from the child-position slot words: one load per box and row,
    // issued ahead of the first input row, which stays in flight through
    // the table fill and its barrier
    const int tid = threadIdx.x;
    Cv gval = load_gc<P, C>(a);  // first: see pin_after
    const int bl_ = min(tid, nb - 1), r_ = min(tid, R - 1);
    const int kcb = a.k_cb[b0 + bl_];
    const uint64_t kw = a.k_slot[b0 + bl_];
    const int xcb = a.x_cb[ap0 + r_];
    const uint64_t xw = a.x_slot[ap0 + r_];
    __builtin_amdgcn_sched_barrier(0);
    Sv xn[P];
    load_row3(tid, xn);
    pin_after(gval);
    if (tid < 4 * P) s_gc[tid] = gval;
    for (int bl = tid; bl < nb; bl += kTT) {  // nb <= kInMax < kTT: one pass
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            const int o = (int)((kw >> (8 * s)) & 0xffu);
            s_cj[bl * 8 + s] = o == 0xff ? (signed char)-1 : (signed char)(kcb + o - J0);
        }
    }
    if (tid < R) {
        const int r = tid;
        const int64_t ap = ap0 + r;
        int bits = 0;
#pragma unroll
        for (int t = 0; t < 8; ++t) {
            const int o = (int)((xw >> (8 * t)) & 0xffu);
            s_out[r * 8 + t] = o == 0xff ? -1 : xcb + o;
            if (o != 0xff) bits |= (1 << t) | (1 << (8 + (t >> 2))) | (1 << (16 + 2 * (t >> 2) + ((t >> 1) & 1)));
        }
        s_bits[r] = bits;
        Cv one;
        one.x = 1;
        one.y = 0;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) s_sig[r * 3 + ax] = (!RHO1 && a.sig) ? cvt<Cv>(a.sig[ap * 3 + ax]) : one;
    }
    __syncthreads();
    int all = 0;
    for (int r = 0; r < R; ++r) all |= s_bits[r];

    const cptr<C> Rt = (cptr<C>)(a.R);
    const cptr<C> Ct = (cptr<C>)(a.C);
    bool first = true;  // xn holds the thread's first row
    // unrolled: each position t2 gets its own registers for the rows, so no
    // copy (and no wait for a load in flight) joins the two passes
#pragma unroll
    for (int t2 = 0; t2 < 2; ++t2) {
        if (!(all & (1 << (8 + t2)))) continue;  // uniform
        // stage 1: rows of the rows a' that need t2 (with one row per
        // thread, xn still holds it from the first position)
        if (!first && nrows > kTT) load_row3(tid, xn);
        first = false;
        auto row = [&](int v, const Cv *x) {
            const int r = (int)(((float)v + 0.5f) * inv_rowlen);
            const int w = v - r * rowlen;
            if (!((s_bits[r] >> (8 + t2)) & 1)) return;
            Yv *dst = Y1 + r * rowlen * P + w * P;
            if (t2 == 0)
                row_interp<P, 0, C>(Rt, x, dst);
            else
                row_interp<P, 1, C>(Rt, x, dst);
        };
        if (nrows <= kTT) {
            // at most one row per thread (uniform): no next row to load
            if (tid < nrows) {
                Cv x[P];
#pragma unroll
                for (int m = 0; m < P; ++m) x[m] = cvt<Cv>(xn[m]);
                row(tid, x);
            }
        } else {
            for (int v = tid; v < nrows; v += kTT) {
                Cv x[P];
#pragma unroll
                for (int m = 0; m < P; ++m) x[m] = cvt<Cv>(xn[m]);
                load_row3(v + kTT, xn);
                row(v, x);
            }
        }
        __syncthreads();
        for (int pass = 0; pass < 2 / NT1; ++pass) {
            // bit t1 of the positions this pass produces
            const int mask = BOTH ? 3 : 1 << pass;
            if (!((all >> (16 + 2 * t2)) & mask)) continue;  // uniform
            // stage 2: lines along m, for (r, b, e0, l, n)
            const int len2 = nb * 2 * P2;
            const float inv_len2 = 1.0f / (float)len2;
            for (int v = tid; v < R * len2; v += kTT) {
                const int r = (int)(((float)v + 0.5f) * inv_len2);
                const int rn = (s_bits[r] >> (16 + 2 * t2)) & mask;
                if (!rn) continue;
                const int vr = v - r * len2;
                const Yv *Yr = Y1 + r * nin * P3;
                Yv *Y2r = Y2 + r * nb * NT1 * 2 * P3;
                const Cv sg1 = s_sig[r * 3 + 1], sg2 = s_sig[r * 3 + 2];
                const int bl = vr / (2 * P2);
                const int rem = vr - bl * 2 * P2;
                const int e0 = rem / P2;
                const int ln = rem - e0 * P2;
                const int l = ln / P, n = ln - l * P;
                const Cv g0 = s_gc[t2 * P + n];
                Cv g1 = s_gc[(2 + t2) * P + n];
                if (!RHO1) g1 = cmul(g1, sg2);
                Cv z0[P], z1[P];
#pragma unroll
                for (int m = 0; m < P; ++m) z0[m] = z1[m] = czero<Cv>();
                // the box's eight child slots in one read; a child's line is
                // read whole before it is used (one LDS wait per child)
                const uint64_t cw = *reinterpret_cast<const uint64_t *>(s_cj + bl * 8);
#pragma unroll
                for (int e12 = 0; e12 < 4; ++e12) {  // e1 = bit 0 of e12, e2 = bit 1
                    const int c = (int)(signed char)((cw >> (8 * (e0 + 2 * e12))) & 0xffu);
                    if (c < 0) continue;
                    const Cv gw = (e12 & 2) ? g1 : g0;
                    const Yv *yp = Yr + c * P3 + l * P2 + n;
                    Yv y[P];
#pragma unroll
                    for (int m = 0; m < P; ++m) y[m] = yp[m * P];
                    __builtin_amdgcn_sched_barrier(0);
                    if (e12 & 1) {
#pragma unroll
                        for (int m = 0; m < P; ++m) cfma(z1[m], gw, cvt<Cv>(y[m]));
                    } else {
#pragma unroll
                        for (int m = 0; m < P; ++m) cfma(z0[m], gw, cvt<Cv>(y[m]));
                    }
                }
                if (!RHO1) {
#pragma unroll
                    for (int m = 0; m < P; ++m) z1[m] = cmul(z1[m], sg1);
                }
                // Y2r[bl][t1][e0]
                Yv *dst = Y2r + (bl * NT1 * 2 + e0) * P3 + l * P2 + n;
                if (BOTH) {
                    if (rn & 1) line_interp<P, 0, C>(Rt, Ct, z0, z1, dst, P);
                    if (rn & 2) line_interp<P, 1, C>(Rt, Ct, z0, z1, dst + 2 * P3, P);
                } else if (pass == 0) {
                    line_interp<P, 0, C>(Rt, Ct, z0, z1, dst, P);
                } else {
                    line_interp<P, 1, C>(Rt, Ct, z0, z1, dst, P);
                }
            }
            __syncthreads();
            // stage 3: lines along l, for (r, b, t1, m, n); both output positions t0
            const int len3 = nb * NT1 * P2;
            const float inv_len3 = 1.0f / (float)len3;
            for (int v = tid; v < R * len3; v += kTT) {
                const int r = (int)(((float)v + 0.5f) * inv_len3);
                const int bits = s_bits[r];
                const int vr = v - r * len3;
                const int bl = vr / (NT1 * P2);
                const int rem = vr - bl * NT1 * P2;
                const int k = BOTH ? rem / P2 : 0;
                const int mn = rem - k * P2;
                const int t1 = BOTH ? k : pass;
                if (!(bits & (1 << (16 + 2 * t2 + t1)))) continue;
                const Yv *Y2r = Y2 + r * nb * NT1 * 2 * P3;
                const Cv sg0 = s_sig[r * 3 + 0];
                const int ta = 4 * t2 + 2 * t1;
                const int a0 = s_out[r * 8 + ta], a1 = s_out[r * 8 + ta + 1];
                Cv z0[P], z1[P];
                const Yv *y0 = Y2r + ((bl * NT1 + k) * 2 + 0) * P3 + mn;
                const Yv *y1 = y0 + P3;
                // a child slot is present when its byte is >= 0 (sign bit clear)
                const uint64_t cw = *reinterpret_cast<const uint64_t *>(s_cj + bl * 8);
                const bool h1 = (~cw & 0x8000800080008000ull) != 0;  // slots 1, 3, 5, 7
                const bool h0 = (~cw & 0x0080008000800080ull) != 0;  // slots 0, 2, 4, 6
                // both lines read whole first (in the tile's Y2 whatever the
                // flags: one LDS wait), absent halves then taken as zero
                Yv v0[P], v1[P];
#pragma unroll
                for (int l = 0; l < P; ++l) {
                    v0[l] = y0[l * P2];
                    v1[l] = y1[l * P2];
                }
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int l = 0; l < P; ++l) {
                    z0[l] = h0 ? cvt<Cv>(v0[l]) : czero<Cv>();
                    z1[l] = h1 ? cvt<Cv>(v1[l]) : czero<Cv>();
                    if (!RHO1) z1[l] = cmul(z1[l], sg0);
                }
                if (a0 >= 0)
                    line_interp<P, 0, C>(Rt, Ct, z0, z1,
                        reinterpret_cast<Sv *>(a.out) + ((int64_t)a0 * a.out_row + b0 + bl) * P3 + mn, P2);
                if (a1 >= 0)
                    line_interp<P, 1, C>(Rt, Ct, z0, z1,
                        reinterpret_cast<Sv *>(a.out) + ((int64_t)a1 * a.out_row + b0 + bl) * P3 + mn, P2);
            }
            __syncthreads();
        }
    }
}

// One work item per work-group (single transform).

template <int P, bool RHO1, typename S, typename C>
__global__ __launch_bounds__(kTT, (min_waves<2, P>())) void k_translate2d(TArgs a, int64_t item0)
{
    extern __shared__ __align__(16) unsigned char smem[];
    translate2d_item<P, RHO1, S, C>(a, item0 + blockIdx.x, smem);
}

template <int P, bool RHO1, typename S, typename C>
__global__ __launch_bounds__(kTT) void k_translate3d(TArgs a, int64_t item0)
{
    extern __shared__ __align__(16) unsigned char smem[];
    translate3d_item<P, RHO1, S, C>(a, item0 + blockIdx.x, smem);
}

// Persistent batched step: the work items of all transforms still active at
// this sweep step form one index space (prefix[t] = first item of transform
// t).  Work-groups take the next item from a counter that starts at zero
// for every step, so late-starting work-groups cannot leave a tail; a
// work-group finishes when the counter passes the end.
template <int D, int P, typename S, typename C>
__global__ __launch_bounds__(kTT, (min_waves<D, P>())) void k_translate_batched(
    const TArgs *__restrict__ descs,
                                                             const int64_t *__restrict__ prefix,
                                                             int ndesc, int64_t total,
                                                             unsigned long long *__restrict__ next)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int64_t s_item;
    for (;;) {
        if (threadIdx.x == 0) s_item = (int64_t)atomicAdd(next, 1ULL);
        __syncthreads();
        // the item is the same for the whole work-group: keep it (and all
        // that is derived from it) in scalar registers
        const int64_t raw = s_item;
        const int64_t item =
            (int64_t)(((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(raw >> 32)) << 32) |
                      (uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(raw & 0xffffffff)));
        if (item >= total) break;
        int lo = 0, hi = ndesc - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (prefix[mid] <= item) lo = mid; else hi = mid - 1;
        }
        const TArgs a = load_desc(descs, lo);
        if constexpr (D == 2)
            translate2d_item<P, false, S, C>(a, item - prefix[lo], smem);
        else
            translate3d_item<P, false, S, C>(a, item - prefix[lo], smem);
        __syncthreads();  // the LDS and s_item are reused by the next item
    }
}

// The same step with one work-group per work item (the hardware scheduler
// balances the items; no counter).
template <int D, int P, typename S, typename C>
__global__ __launch_bounds__(kTT, (min_waves<D, P>())) void k_translate_batched_flat(const TArgs *__restrict__ descs,
                                                                  const int64_t *__restrict__ prefix,
                                                                  int ndesc, int64_t item0)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int64_t item = item0 + blockIdx.x;
    int lo = 0, hi = ndesc - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= item) lo = mid; else hi = mid - 1;
    }
    const TArgs a = load_desc(descs, lo);
    if constexpr (D == 2)
        translate2d_item<P, false, S, C>(a, item - prefix[lo], smem);
    else
        translate3d_item<P, false, S, C>(a, item - prefix[lo], smem);
}

// BFSFT_LDS_KB if it names a budget the d-dimensional kernels can launch
// (8 KB up to kLdsMax2D in 2D, kLdsMax in 3D), else 32 KB
int lds_budget_default(int d)
{
    const char *s = std::getenv("BFSFT_LDS_KB");
    const int v = s ? std::atoi(s) : 0;
    const int vmax = (int)((d == 2 ? kLdsMax2D : kLdsMax) / 1024);
    return ((v >= 8 && v <= vmax) ? v : 32) * 1024;
}

}  // namespace

int translate_default_lds(int d) { return lds_budget_default(d); }

// Blocks of axis-1 results per box of a 3D tile: both t1 (4) when a box
// with all its children fits that way, else one t1 (2); the kernels take
// the same decision from their template arguments (both3d)
static int y2_blocks(int p, int precision)
{
    const size_t elem = precision == BFSFT_FP64 ? 16 : 8;
    return (size_t)12 * p * p * p * elem <= kLdsMax ? 4 : 2;
}

// LDS blocks (p^d elements of the intermediate type) a work-group may hold
// within `budget` bytes
int translate_cap_blocks(int d, int p, int precision, int budget)
{
    int PD = p;
    for (int a = 1; a < d; ++a) PD *= p;
    const int elem = precision == BFSFT_FP64 ? 16 : 8;
    int cap = budget / (PD * elem);
    const int one_box = d == 2 ? 2 * 4 : 8 + y2_blocks(p, precision);  // a single box with all children
    if (cap < one_box) cap = one_box;
    return cap;
}

// LDS blocks a tile of nb boxes with nin children needs: the VALU kernels
// hold the axis-2 results (2D: both t2) or two stages (3D); the matrix-core
// kernel also stages the input blocks
int translate_tile_cost(int d, int p, int precision, int nin, int nb, int kind)
{
    if (kind == 1) return 3 * nin;
    return d == 2 ? 2 * nin : nin + y2_blocks(p, precision) * nb;
}

bool translate_fits(int d, int p, int precision)
{
    int PD = p;
    for (int a = 1; a < d; ++a) PD *= p;
    const int elem = precision == BFSFT_FP64 ? 16 : 8;
    const int one_box = d == 2 ? 2 * 4 : 8 + y2_blocks(p, precision);
    return (size_t)one_box * PD * elem <= kLdsMax;
}

int translate_rows(int cap, int cost_max, int64_t nap, int kind)
{
    if (kind == 1) cap -= 1;  // the zero block of absent children
    int R = cap / std::max(1, cost_max);
    R = std::max(1, std::min(R, kRowsMax));
    return (int)std::min<int64_t>(R, std::max<int64_t>(1, nap));
}

namespace {

size_t ysize(int precision) { return precision == BFSFT_FP64 ? 16 : 8; }

}  // namespace

size_t translate_lds_bytes(int d, int p, int precision, int rows, int cost_max, int kind)
{
    size_t PD = (size_t)p * p * (d == 3 ? p : 1);
    return ((size_t)rows * cost_max + (kind == 1 ? 1 : 0)) * PD * ysize(precision);
}

int64_t translate_items(const LevelArgs &la)
{
    if (la.nap == 0 || la.ntile == 0) return 0;
    return ((la.nap + la.rows - 1) / la.rows) * (int64_t)la.ntile;
}

size_t translate_desc_size() { return sizeof(TArgs); }

void translate_fill_desc(const Launch &c, const LevelArgs &la, void *dst)
{
    const TArgs a = make_targs(c, la);
    std::memcpy(dst, &a, sizeof(TArgs));
}

void launch_translate(const Launch &c, const LevelArgs &la)
{
    if (la.kind == 1) {
        launch_translate_mfma(c, la);
        return;
    }
    if (la.kind == 2) {
        launch_translate_xdl(c, la);
        return;
    }
    const int64_t grid = translate_items(la);
    if (grid == 0) return;
    const TArgs a = make_targs(c, la);
    const size_t lds = translate_lds_bytes(c.d, c.p, c.precision, la.rows, la.cost_max);
    if (lds > (c.d == 2 ? kLdsMax2D : kLdsMax)) throw Error{BFSFT_EINVAL, "translation tile exceeds LDS"};
    auto body = [&](auto tag, auto *sp, auto *cp, auto d3) {
        constexpr int P = decltype(tag)::value;
        using S = std::remove_pointer_t<decltype(sp)>;
        using C = std::remove_pointer_t<decltype(cp)>;
        // chunks of at most kMaxGroups work-groups (see kMaxGroups)
        const int64_t chunk = max_groups();
        for (int64_t i0 = 0; i0 < grid; i0 += chunk) {
            const unsigned g = (unsigned)std::min<int64_t>(chunk, grid - i0);
            if constexpr (decltype(d3)::value) {
                if (la.sig)
                    k_translate3d<P, false, S, C><<<g, kTT, lds, c.stream>>>(a, i0);
                else
                    k_translate3d<P, true, S, C><<<g, kTT, lds, c.stream>>>(a, i0);
            } else {
                if (la.sig)
                    k_translate2d<P, false, S, C><<<g, kTT, lds, c.stream>>>(a, i0);
                else
                    k_translate2d<P, true, S, C><<<g, kTT, lds, c.stream>>>(a, i0);
            }
        }
    };
    if (c.d == 2)
        dispatch_p(c.p, [&](auto tag) {
            dispatch_prec(c.precision, [&](auto *sp, auto *cp) { body(tag, sp, cp, std::false_type{}); });
        });
    else
        dispatch_p3(c.p, [&](auto tag) {
            dispatch_prec(c.precision, [&](auto *sp, auto *cp) { body(tag, sp, cp, std::true_type{}); });
        });
    BF_HIP(hipGetLastError());
}

void launch_translate_batched(const Launch &c, const void *descs, const int64_t *prefix, int ndesc,
                              int64_t total, size_t lds, int grid, unsigned long long *next)
{
    if (total == 0) return;
    if (split_precision(c.precision)) {  // stage 1 on the matrix cores
        launch_translate_batched_xdl(c, descs, prefix, ndesc, total, lds, grid, next);
        return;
    }
    if (lds > kLdsMax) throw Error{BFSFT_EINVAL, "translation tile exceeds LDS"};
    const unsigned g = (unsigned)std::min<int64_t>(grid, total);
    auto body = [&](auto tag, auto *sp, auto *cp, auto dd) {
        constexpr int P = decltype(tag)::value;
        constexpr int D = decltype(dd)::value;
        using S = std::remove_pointer_t<decltype(sp)>;
        using C = std::remove_pointer_t<decltype(cp)>;
        if (grid <= 0)
            for (int64_t i0 = 0, chunk = max_groups(); i0 < total; i0 += chunk)  // see kMaxGroups
                k_translate_batched_flat<D, P, S, C>
                    <<<(unsigned)std::min<int64_t>(chunk, total - i0), kTT, lds, c.stream>>>(
                        (const TArgs *)descs, prefix, ndesc, i0);
        else
            k_translate_batched<D, P, S, C><<<g, kTT, lds, c.stream>>>((const TArgs *)descs, prefix, ndesc,
                                                                       total, next);
    };
    if (c.d == 2)
        dispatch_p(c.p, [&](auto tag) {
            dispatch_prec(c.precision, [&](auto *sp, auto *cp) {
                body(tag, sp, cp, std::integral_constant<int, 2>{});
            });
        });
    else
        dispatch_p3(c.p, [&](auto tag) {
            dispatch_prec(c.precision, [&](auto *sp, auto *cp) {
                body(tag, sp, cp, std::integral_constant<int, 3>{});
            });
        });
    BF_HIP(hipGetLastError());
}

}  // namespace bfsft
