// The 2D translation of step 3 of Section 2.2 (rotated state, real
// interpolation operators; see translate.hip): its per-item tables, stage 1
// on the VALU, stage 2, and the pieces the 3D kernel shares.  Internal to
// the library; included by the translation sources.
#pragma once

#include "translate_common.h"

namespace bfsft {

namespace {

using namespace tr;

// coefficient G(s, t, l) of the table [2 s][2 t][P]
template <typename Cv, typename C>
__device__ __forceinline__ Cv gcoef(cptr<C> Ct, int s, int t, int l, int P)
{
    return ldc<Cv>(Ct, (2 * s + t) * P + l);
}

// stage 1 for one input row x and one output position T2: the dot rows of
// R_t2 and the copy rows; no phases
template <int P, int T2, typename C, typename Yv>
__device__ __forceinline__ void row_interp(cptr<C> Rt, const typename CV<C>::t *x, Yv *dst)
{
    using Cv = typename CV<C>::t;
    using RW = Rows<P, T2>;
    constexpr int PP = P * P, Q = P - 1;
#pragma unroll
    for (int k = 0; k < RW::ndot; ++k) {
        const int m = RW::first_dot + 2 * k;
        Cv y = czero<Cv>();
#pragma unroll
        for (int mp = 0; mp < P; ++mp) rfma(y, Rt[T2 * PP + m * P + mp], x[mp]);
        st(dst + m, y);
    }
#pragma unroll
    for (int m = 0; m < P; ++m) {
        if (!RW::copy(m)) continue;
        st(dst + m, x[(T2 * Q + m) / 2]);
    }
}

// One output line at position T along the contracted axis, written with
// stride `stride` to a destination of element type Dv (LDS or HBM):
//   o[l] = G(0, T, l) (R_T z0)[l] + G(1, T, l) (R_T z1)[l],
// z1 carrying sigma already.
template <int P, int T, typename C, typename Dv>
__device__ __forceinline__ void line_interp(cptr<C> Rt, cptr<C> Ct, const typename CV<C>::t *z0,
                                            const typename CV<C>::t *z1, Dv *dst, int stride)
{
    using Cv = typename CV<C>::t;
    using RW = Rows<P, T>;
    constexpr int PP = P * P, Q = P - 1;
#pragma unroll
    for (int k = 0; k < RW::ndot; ++k) {
        const int l = RW::first_dot + 2 * k;
        Cv a = czero<Cv>(), b = czero<Cv>();
#pragma unroll
        for (int lp = 0; lp < P; ++lp) {
            const auto r = Rt[T * PP + l * P + lp];
            rfma(a, r, z0[lp]);
            rfma(b, r, z1[lp]);
        }
        Cv o = cmul(gcoef<Cv>(Ct, 0, T, l, P), a);
        cfma(o, gcoef<Cv>(Ct, 1, T, l, P), b);
        st(dst + l * stride, o);
    }
#pragma unroll
    for (int l = 0; l < P; ++l) {
        if (!RW::copy(l)) continue;
        const int n = (T * Q + l) / 2;
        Cv o = cmul(gcoef<Cv>(Ct, 0, T, l, P), z0[n]);
        cfma(o, gcoef<Cv>(Ct, 1, T, l, P), z1[n]);
        st(dst + l * stride, o);
    }
}

// Y element type: the state precision for the FP32-state paths, FP64 otherwise
template <typename S, typename C> struct YT { using t = typename CV<S>::t; };

// Waves per SIMD the register allocation must allow: four (at most 128
// VGPRs) up to p = 9 (five, at 96 VGPRs, spills in stage 2 and is slower);
// the larger grids of p >= 10 need the full register file.
template <int D, int P> constexpr int min_waves() { return (D == 2 && P <= 9) ? 4 : 1; }

// Per-work-group tables of a 2D item (static LDS).
template <typename Cv> struct Tables2D {
    int out[kRowsMax * 4];       // [r][t]: output row a of child t of row a' (or -1)
    int bits[kRowsMax];          // bit t: child t present; bit 4 + t2: a child with that t2
    Cv sig[kRowsMax * 2];        // [r][axis]: exp(2 pi i rho i_{A'}) (1 when rho = 1)
    signed char cj[kInMax * 4];  // [b][s]: local input index of child s of box b (or -1)
    Cv gc[4 * kPMax2];           // G(s, t, l) as the table [2 s][2 t][P]: stage 2 reads it at
                                 // the lane's column, which from LDS costs no memory latency
};

// What a thread loads ahead of an item's tables: the slot words of box
// tid and of row tid (Tree::slots) with their first children.
struct Slots2D {
    int kcb = 0, xcb = 0;
    uint64_t kslot = ~0ull, xslot = ~0ull;
};

// The loads are unconditional (indices clamped into range): a load under a
// branch makes the compiler wait for it where the branch joins.
__device__ __forceinline__ Slots2D load_slots(const TArgs &a, const Item2D &it)
{
    Slots2D h;
    const int tid = threadIdx.x;
    const int bl = min(tid, it.nb - 1), r = min(tid, it.R - 1);
    h.kcb = a.k_cb[it.b0 + bl];
    h.kslot = a.k_slot[it.b0 + bl];
    h.xcb = a.x_cb[it.ap0 + r];
    h.xslot = a.x_slot[it.ap0 + r];
    return h;
}

// The G entry of thread tid (clamped, so the load is unconditional).
template <int P, typename C>
__device__ __forceinline__ typename CV<C>::t load_gc(const TArgs &a)
{
    return ldc<typename CV<C>::t>((cptr<C>)(a.C), min((int)threadIdx.x, 4 * P - 1));
}

// Marks v as used here.  Without it the compiler moves the load of an
// entry that only some threads store into their branch, after the input
// rows' loads; the wait for it there then waits for those rows too (the
// counter of outstanding loads drains in order).  Placed after the rows'
// loads are issued, the wait covers the entry's load alone.
template <typename Cv> __device__ __forceinline__ void pin_after(Cv &v)
{
    asm volatile("" : "+v"(v.x), "+v"(v.y));
}

// Fill the tables from the slot words (ends with a barrier; sets it.all).
template <bool RHO1, typename Cv>
__device__ __forceinline__ void fill_tables(const TArgs &a, Item2D &it, const Slots2D &h, Tables2D<Cv> &tb,
                                            const Cv &gval, int ngc)
{
    const int tid = threadIdx.x;
    if (tid < ngc) tb.gc[tid] = gval;
    if (tid < it.nb) {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int o = (int)((h.kslot >> (8 * s)) & 0xffu);
            tb.cj[tid * 4 + s] = o == 0xff ? (signed char)-1 : (signed char)(h.kcb + o - it.J0);
        }
    }
    if (tid < it.R) {
        int bits = 0;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int o = (int)((h.xslot >> (8 * t)) & 0xffu);
            tb.out[tid * 4 + t] = o == 0xff ? -1 : h.xcb + o;
            if (o != 0xff) bits |= (1 << t) | (1 << (4 + (t >> 1)));
        }
        tb.bits[tid] = bits;
        Cv one;
        one.x = 1;
        one.y = 0;
        const int64_t ap = it.ap0 + tid;
        tb.sig[tid * 2] = (!RHO1 && a.sig) ? cvt<Cv>(a.sig[ap * 2]) : one;
        tb.sig[tid * 2 + 1] = (!RHO1 && a.sig) ? cvt<Cv>(a.sig[ap * 2 + 1]) : one;
    }
    __syncthreads();
    int all = 0;
    for (int r = 0; r < it.R; ++r) all |= tb.bits[r];
    it.all = all;
}

// The stage-1 row v of an item: row a' from a float reciprocal (exact: the
// index is below 2^16, so the error is far below the distance 0.5 / rowlen).
template <int P, typename Sv>
__device__ __forceinline__ const Sv *row_src(const TArgs &a, const Item2D &it, int v)
{
    constexpr int PP = P * P;
    const int rowlen = it.nin * P;
    const int r = (int)(((float)v + 0.5f) * (1.0f / (float)rowlen));
    return reinterpret_cast<const Sv *>(a.in) + ((it.ap0 + r) * a.in_row + it.J0) * PP + (v - r * rowlen) * P;
}

// row v, clamped to the last row (an unconditional load, see load_slots)
template <int P, typename Sv>
__device__ __forceinline__ void load_row(const TArgs &a, const Item2D &it, int v, Sv *xn)
{
    const Sv *src = row_src<P, Sv>(a, it, min(v, it.R * it.nin * P - 1));
#pragma unroll
    for (int m = 0; m < P; ++m) xn[m] = src[m];
}

// Stage 1: every input row once, both output positions t2 it is needed
// for; the rows a' of the work-group are processed side by side.  xn holds
// the thread's first row on entry; each next row is loaded while the
// current one is computed.
template <int P, typename S, typename C>
__device__ __forceinline__ void stage1_2d(const TArgs &a, const Item2D &it, typename CV<S>::t *xn,
                                          typename YT<S, C>::t *Y, const int *s_bits)
{
    using Cv = typename CV<C>::t;
    using Yv = typename YT<S, C>::t;
    constexpr int PP = P * P;
    const cptr<C> Rt = (cptr<C>)(a.R);
    const int rowlen = it.nin * P;
    const int nrows = it.R * rowlen;
    const int ysz = it.R * it.nin * PP;  // one t2 half of Y
    const float inv_rowlen = 1.0f / (float)rowlen;
    auto row = [&](int v, const Cv *x) {
        const int r = (int)(((float)v + 0.5f) * inv_rowlen);
        const int w = v - r * rowlen;
        const int bits = s_bits[r];
        Yv *Yr = Y + r * it.nin * PP + w * P;
        if (bits & (1 << 4)) row_interp<P, 0, C>(Rt, x, Yr);
        if (bits & (1 << 5)) row_interp<P, 1, C>(Rt, x, Yr + ysz);
    };
    if (nrows <= kTT) {
        // at most one row per thread (uniform): no next row to load, so
        // nothing is left in flight for the compiler to wait on before the
        // barrier that follows
        if ((int)threadIdx.x < nrows) {
            Cv x[P];
#pragma unroll
            for (int m = 0; m < P; ++m) x[m] = cvt<Cv>(xn[m]);
            row(threadIdx.x, x);
        }
        return;
    }
    for (int v = threadIdx.x; v < nrows; v += kTT) {
        Cv x[P];
#pragma unroll
        for (int m = 0; m < P; ++m) x[m] = cvt<Cv>(xn[m]);
        load_row<P>(a, it, v + kTT, xn);
        row(v, x);
    }
}

// Stage 2: one work unit per (t2, output column), over the positions t2
// some row needs, each with both output positions t1 and the whole column.
// (Splitting a column's rows over several threads, to keep all waves busy
// when units are few, repeats the children's sums and is slower: idle waves
// cost no issue slots.)
template <int P, bool RHO1, typename S, typename C>
__device__ __forceinline__ void stage2_2d(const TArgs &a, const Item2D &it, const typename YT<S, C>::t *Y,
                                          const Tables2D<typename CV<C>::t> &tb)
{
    using Sv = typename CV<S>::t;
    using Cv = typename CV<C>::t;
    using Yv = typename YT<S, C>::t;
    constexpr int PP = P * P;
    const cptr<C> Rt = (cptr<C>)(a.R);
    const cptr<C> Ct = (cptr<C>)(a.C);
    const int nin = it.nin, b0 = it.b0;
    const int ysz = it.R * nin * PP;
    const int ncol = it.nb * P;
    const float inv_ncol = 1.0f / (float)ncol;
    const int ntot = it.R * ncol;
    const int need = (it.all >> 4) & 3;  // t2 = 0, 1 needed by some row (uniform)
    const int units = ((need & 1) + (need >> 1)) * ntot;
    const int tfirst = (need & 1) ? 0 : 1;
    for (int u = threadIdx.x; u < units; u += kTT) {
        const bool second = u >= ntot;  // only when both positions are needed
        const int t2 = second ? 1 : tfirst;
        const int v = second ? u - ntot : u;
        const int r = (int)(((float)v + 0.5f) * inv_ncol);
        const int col = v - r * ncol;
        const int bits = tb.bits[r];
        if (!(bits & (1 << (4 + t2)))) continue;
        const int bl = col / P, m = col - bl * P;
        const Yv *Yr = Y + t2 * ysz + r * nin * PP;
        const int a0 = tb.out[r * 4 + (t2 << 1)], a1 = tb.out[r * 4 + 1 + (t2 << 1)];
        const int c0 = tb.cj[bl * 4 + 0], c2 = tb.cj[bl * 4 + 2];
        const int c1 = tb.cj[bl * 4 + 1], c3 = tb.cj[bl * 4 + 3];
        // weights of the children at column m: G(s2, t2, m), sigma of
        // axis 2 with s2 = 1, sigma of axis 1 on the s1 = 1 sum
        Cv g0 = tb.gc[t2 * P + m], g1 = tb.gc[(2 + t2) * P + m];
        if (!RHO1) g1 = cmul(g1, tb.sig[r * 2 + 1]);
        Cv h0 = g0, h1 = g1;
        if (!RHO1) {
            const Cv sg = tb.sig[r * 2];
            h0 = cmul(h0, sg);
            h1 = cmul(h1, sg);
        }
        // one branch per child slot, not per element; a child's column is
        // read whole before it is used, so its reads wait on LDS once
        // (interleaved, each read waited for the previous one's use)
        auto column = [&](int c, Yv *v) {
            const Yv *yp = Yr + c * PP + m;
#pragma unroll
            for (int l = 0; l < P; ++l) v[l] = yp[l * P];
            __builtin_amdgcn_sched_barrier(0);
        };
        Cv z0[P], z1[P];
#pragma unroll
        for (int l = 0; l < P; ++l) z0[l] = z1[l] = czero<Cv>();
        if (c0 >= 0) {
            Yv v[P];
            column(c0, v);
#pragma unroll
            for (int l = 0; l < P; ++l) z0[l] = cmul(g0, cvt<Cv>(v[l]));
        }
        if (c2 >= 0) {
            Yv v[P];
            column(c2, v);
#pragma unroll
            for (int l = 0; l < P; ++l) cfma(z0[l], g1, cvt<Cv>(v[l]));
        }
        if (c1 >= 0) {
            Yv v[P];
            column(c1, v);
#pragma unroll
            for (int l = 0; l < P; ++l) z1[l] = cmul(h0, cvt<Cv>(v[l]));
        }
        if (c3 >= 0) {
            Yv v[P];
            column(c3, v);
#pragma unroll
            for (int l = 0; l < P; ++l) cfma(z1[l], h1, cvt<Cv>(v[l]));
        }
        Sv *o0 = reinterpret_cast<Sv *>(a.out) + ((int64_t)a0 * a.out_row + b0 + bl) * PP + m;
        Sv *o1 = reinterpret_cast<Sv *>(a.out) + ((int64_t)a1 * a.out_row + b0 + bl) * PP + m;
        if (a0 >= 0) line_interp<P, 0, C>(Rt, Ct, z0, z1, o0, P);
        if (a1 >= 0) line_interp<P, 1, C>(Rt, Ct, z0, z1, o1, P);
    }
}

// One 2D work item: its tables from the slot words (independent loads),
// the thread's first input row loaded alongside, stage 1, stage 2.
template <int P, bool RHO1, typename S, typename C>
__device__ __forceinline__ void translate2d_item(const TArgs &a, int64_t gid, unsigned char *smem)
{
    using Sv = typename CV<S>::t;
    using Cv = typename CV<C>::t;
    using Yv = typename YT<S, C>::t;
    __shared__ Tables2D<Cv> tb;
    Yv *Y = reinterpret_cast<Yv *>(smem);  // [2 t2][R][nin][P][P]
    Item2D it = item2d(a, gid);
    // the G entry and the slot words first (the tables need them first),
    // then the first input row, which stays in flight through the table
    // fill and its barrier
    Cv gval = load_gc<P, C>(a);
    const Slots2D h = load_slots(a, it);
    __builtin_amdgcn_sched_barrier(0);  // keep these loads ahead of the row's
    Sv xn[P];
    load_row<P>(a, it, threadIdx.x, xn);
    pin_after(gval);
    fill_tables<RHO1>(a, it, h, tb, gval, 4 * P);
    stage1_2d<P, S, C>(a, it, xn, Y, tb.bits);
    __syncthreads();
    stage2_2d<P, RHO1, S, C>(a, it, Y, tb);
}

}  // namespace

}  // namespace bfsft
