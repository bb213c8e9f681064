// Step 3 of Section 2.2 (the level sweep) on gfx950.
//
// For a box pair (A, B) at T_K level l, A = child t of A' and B with
// children B_s, the state (B's check potential at A's check points, B's
// corner phase divided out) is, per axis, interpolated from the children's
// states (see kernels.hip for the derivation):
//
//   w^{AB}[l] = sum_s f(s, t, l) * (L_t w^{A'B_s})[l],
//   f(0, t, l) = 1,   f(1, t, l) = sigma_{A'} exp(i pi rho (t q + l) / q),
//   L_t[l][l'] = ell_{l'}( exp(i pi rho (t q + l) / q^2) ).
//
// The check point (t + l/q)/2 of A coincides with the node (t q + l)/2 / q of
// A' whenever t q + l is even; those rows of L_t are unit vectors, so about
// half of every 1D interpolation is a copy and only the other rows are dot
// products (4 of 9 at p = 9).  Which rows are copies depends only on (p, t),
// so it is resolved at compile time.
//
// Work decomposition.  A work-group takes R consecutive rows a' of T_X level
// L-l-1 and one tile of boxes b of T_K level l; the children of the tile are
// a contiguous range of every input row (Morton order), and the outputs are
// the rows a = children of each a'.  Per output position t2 along axis 2:
//   stage 1: one thread per input row (a', j, l): Y = L_t2 along axis 2,
//   stage 2: one thread per output column (a', b, m): sum the children with
//            the same s1, apply L_t1 along axis 1, write the column.
// The interpolation operator of each stage depends only on t, so it is
// uniform across the work-group and read through scalar loads.
#include "bfsft_impl.h"
#include "cplx.h"
#include "dispatch.h"
#include "translate_common.h"

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <type_traits>

namespace bfsft {

namespace {

using namespace tr;

// phase of a child at offset 1 along an axis, output index l, position t:
// sigma_{A'} * PH_t[l]; sigma = 1 when rho = 1 (RHO1)
template <bool RHO1, typename Cv, typename C>
__device__ __forceinline__ Cv child_phase(cptr<C> PH, int t, int l, int P, const Cv sg)
{
    const Cv ph = ldc<Cv>(PH, t * P + l);
    return RHO1 ? ph : cmul(sg, ph);
}

// stage 1 for one input row x and one output position T2 along axis 2
template <int P, int T2, bool RHO1, typename C, typename Yv>
__device__ __forceinline__ void row_interp(cptr<C> Lt, cptr<C> PH, const typename CV<C>::t *x,
                                           bool s2, const typename CV<C>::t sg, Yv *dst)
{
    using Cv = typename CV<C>::t;
    using RW = Rows<P, T2>;
    constexpr int PP = P * P, Q = P - 1;
#pragma unroll 1
    for (int k = 0; k < RW::ndot; ++k) {
        const int m = RW::first_dot + 2 * k;
        Cv y = czero<Cv>();
#pragma unroll
        for (int mp = 0; mp < P; ++mp) cfma(y, ldc<Cv>(Lt, T2 * PP + m * P + mp), x[mp]);
        if (s2) y = cmul(y, child_phase<RHO1, Cv>(PH, T2, m, P, sg));
        st(dst + m, y);
    }
#pragma unroll
    for (int m = 0; m < P; ++m) {
        if (!RW::copy(m)) continue;
        Cv y = x[(T2 * Q + m) / 2];
        if (s2) y = cmul(y, child_phase<RHO1, Cv>(PH, T2, m, P, sg));
        st(dst + m, y);
    }
}

// Output column of stage 2 (2D) at position T1, restricted to the output
// rows of group g of G (dot rows k = g, g+G, ... and every G-th copy row; g
// is uniform across the wave).  z0 sums the children at s1 = 0, z1 those at
// s1 = 1 with sigma_{A'} of axis 1 already applied, so the s1 = 1 rows use
// the folded table LP = diag(PH_t) L_t and every dot row is one accumulator.
template <int P, int T1, typename S, typename C>
__device__ __forceinline__ void col_interp_g(cptr<C> Lt, cptr<C> LP, cptr<C> PH,
                                             const typename CV<C>::t *z0,
                                             const typename CV<C>::t *z1, bool h1,
                                             typename CV<S>::t *dst, int g, int G)
{
    using Cv = typename CV<C>::t;
    using RW = Rows<P, T1>;
    constexpr int PP = P * P, Q = P - 1;
#pragma unroll 1
    for (int k = g; k < RW::ndot; k += G) {
        const int l = RW::first_dot + 2 * k;
        Cv o = czero<Cv>();
#pragma unroll
        for (int lp = 0; lp < P; ++lp) {
            cfma(o, ldc<Cv>(Lt, T1 * PP + l * P + lp), z0[lp]);
            cfma(o, ldc<Cv>(LP, T1 * PP + l * P + lp), z1[lp]);
        }
        st(dst + l * P, o);
    }
#pragma unroll
    for (int l = 0; l < P; ++l) {
        if (!RW::copy(l)) continue;
        if (RW::copy_index(l) % G != g) continue;
        Cv o = z0[(T1 * Q + l) / 2];
        if (h1) o = cadd(o, cmul(z1[(T1 * Q + l) / 2], ldc<Cv>(PH, T1 * P + l)));
        st(dst + l * P, o);
    }
}

// Y element type: the state precision for the FP32-state paths, FP64 otherwise
#ifdef BFSFT_MIXED_Y64
template <typename S, typename C> struct YT { using t = typename CV<C>::t; };
#else
template <typename S, typename C> struct YT { using t = typename CV<S>::t; };
#endif

// Strided variant of col_interp: the output column has stride `stride`
// elements and goes to a destination of element type Dv (LDS or HBM).
template <int P, int T, bool RHO1, typename C, typename Dv>
__device__ __forceinline__ void col_interp_s(cptr<C> Lt, cptr<C> PH, const typename CV<C>::t *z0,
                                             const typename CV<C>::t *z1, bool h1,
                                             const typename CV<C>::t sg, Dv *dst, int stride)
{
    using Cv = typename CV<C>::t;
    using RW = Rows<P, T>;
    constexpr int PP = P * P, Q = P - 1;
#pragma unroll 1
    for (int k = 0; k < RW::ndot; ++k) {
        const int l = RW::first_dot + 2 * k;
        Cv o0 = czero<Cv>(), o1 = czero<Cv>();
#pragma unroll
        for (int lp = 0; lp < P; ++lp) {
            const Cv lv = ldc<Cv>(Lt, T * PP + l * P + lp);
            cfma(o0, lv, z0[lp]);
            cfma(o1, lv, z1[lp]);
        }
        if (h1) o0 = cadd(o0, cmul(o1, child_phase<RHO1, Cv>(PH, T, l, P, sg)));
        st(dst + l * stride, o0);
    }
#pragma unroll
    for (int l = 0; l < P; ++l) {
        if (!RW::copy(l)) continue;
        Cv o = z0[(T * Q + l) / 2];
        if (h1) o = cadd(o, cmul(z1[(T * Q + l) / 2], child_phase<RHO1, Cv>(PH, T, l, P, sg)));
        st(dst + l * stride, o);
    }
}

// Step 3, 3D (octrees, p^3 grids, axis 0 = l slowest, axis 2 = n fastest).
// Child positions s and output positions t carry the parity of axis a in bit
// a.  Per output position (t2 along axis 2, then t1 along axis 1):
//   stage 1 (axis 2): rows (j, l, m):  Y1 = L_t2 along n, phase of bit 2,
//   stage 2 (axis 1): lines (b, e0, l, n): sum the children over bit 2,
//                     Y2[b][e0] = sum over bit 1 of phase * L_t1 along m,
//   stage 3 (axis 0): lines (b, m, n): out_t = sum over bit 0 of phase *
//                     L_t0 along l, written to HBM.
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
    __shared__ unsigned char s_pos[kInMax];
    __shared__ signed char s_cj[kInMax * 8];

    const int64_t g = gid / a.ntile;
    const int tile = (int)(gid - g * a.ntile);
    const int64_t ap0 = g * a.rows;
    const int R = (int)min((int64_t)a.rows, a.nap - ap0);
    const int2 bt = a.tiles[tile];
    const int b0 = bt.x, nb = bt.y - bt.x;
    const int J0 = a.k_cb[b0];
    const int nin = a.k_cb[bt.y] - J0;
    Yv *Y1 = reinterpret_cast<Yv *>(smem);  // [R][nin][P3]
    Yv *Y2 = Y1 + R * nin * P3;             // [R][nb][2][P3]

    for (int i = threadIdx.x; i < nin; i += kTT) s_pos[i] = (unsigned char)(a.k_keys[J0 + i] & 7);
    for (int bl = threadIdx.x; bl < nb; bl += kTT) {
        signed char cj[8] = {-1, -1, -1, -1, -1, -1, -1, -1};
        for (int j = a.k_cb[b0 + bl]; j < a.k_cb[b0 + bl + 1]; ++j)
            cj[a.k_keys[j] & 7] = (signed char)(j - J0);
#pragma unroll
        for (int s = 0; s < 8; ++s) s_cj[bl * 8 + s] = cj[s];
    }
    if (threadIdx.x < R) {
        const int r = threadIdx.x;
        const int64_t ap = ap0 + r;
        int bits = 0;
        int o[8] = {-1, -1, -1, -1, -1, -1, -1, -1};
        for (int i = a.x_cb[ap]; i < a.x_cb[ap + 1]; ++i) {
            const int t = (int)(a.x_keys[i] & 7);
            o[t] = i;
            bits |= (1 << t) | (1 << (8 + (t >> 2))) | (1 << (16 + 2 * (t >> 2) + ((t >> 1) & 1)));
        }
#pragma unroll
        for (int t = 0; t < 8; ++t) s_out[r * 8 + t] = o[t];
        s_bits[r] = bits;
        Cv one;
        one.x = 1;
        one.y = 0;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) s_sig[r * 3 + ax] = a.sig ? cvt<Cv>(a.sig[ap * 3 + ax]) : one;
    }
    __syncthreads();
    int all = 0;
    for (int r = 0; r < R; ++r) all |= s_bits[r];

    const cptr<C> Lt = (cptr<C>)(a.Lt);
    const cptr<C> PH = (cptr<C>)(a.PH);
    for (int t2 = 0; t2 < 2; ++t2) {
        if (!(all & (1 << (8 + t2)))) continue;
        // stage 1
        for (int r = 0; r < R; ++r) {
            if (!(s_bits[r] & (1 << (8 + t2)))) continue;
            const Sv *in = reinterpret_cast<const Sv *>(a.in) + ((ap0 + r) * a.in_row + J0) * P3;
            Yv *Yr = Y1 + r * nin * P3;
            const Cv sg = s_sig[r * 3 + 2];
            for (int v = threadIdx.x; v < nin * P2; v += kTT) {
                const int j = v / P2;
                const Sv *src = in + v * P;
                Cv x[P];
#pragma unroll
                for (int m = 0; m < P; ++m) x[m] = cvt<Cv>(src[m]);
                const bool e2 = (s_pos[j] >> 2) & 1;
                if (t2 == 0)
                    row_interp<P, 0, RHO1, C>(Lt, PH, x, e2, sg, Yr + v * P);
                else
                    row_interp<P, 1, RHO1, C>(Lt, PH, x, e2, sg, Yr + v * P);
            }
        }
        __syncthreads();
        for (int t1 = 0; t1 < 2; ++t1) {
            if (!(all & (1 << (16 + 2 * t2 + t1)))) continue;
            // stage 2: lines along m, for (b, e0, l, n)
            for (int r = 0; r < R; ++r) {
                if (!(s_bits[r] & (1 << (16 + 2 * t2 + t1)))) continue;
                const Yv *Yr = Y1 + r * nin * P3;
                Yv *Y2r = Y2 + r * nb * 2 * P3;
                const Cv sg = s_sig[r * 3 + 1];
                for (int v = threadIdx.x; v < nb * 2 * P2; v += kTT) {
                    const int bl = v / (2 * P2);
                    const int rem = v - bl * 2 * P2;
                    const int e0 = rem / P2;
                    const int ln = rem - e0 * P2;
                    const int l = ln / P, n = ln - l * P;
                    Cv z0[P], z1[P];
#pragma unroll
                    for (int m = 0; m < P; ++m) z0[m] = z1[m] = czero<Cv>();
                    bool h1 = false;
#pragma unroll
                    for (int e12 = 0; e12 < 4; ++e12) {  // e1 = bit 0 of e12, e2 = bit 1
                        const int c = s_cj[bl * 8 + e0 + 2 * e12];
                        if (c < 0) continue;
                        const Yv *yp = Yr + c * P3 + l * P2 + n;
                        if (e12 & 1) {
                            h1 = true;
#pragma unroll
                            for (int m = 0; m < P; ++m) z1[m] = cadd(z1[m], ld<Cv>(yp + m * P));
                        } else {
#pragma unroll
                            for (int m = 0; m < P; ++m) z0[m] = cadd(z0[m], ld<Cv>(yp + m * P));
                        }
                    }
                    Yv *dst = Y2r + (bl * 2 + e0) * P3 + l * P2 + n;
                    if (t1 == 0)
                        col_interp_s<P, 0, RHO1, C>(Lt, PH, z0, z1, h1, sg, dst, P);
                    else
                        col_interp_s<P, 1, RHO1, C>(Lt, PH, z0, z1, h1, sg, dst, P);
                }
            }
            __syncthreads();
            // stage 3: lines along l, for (b, m, n); both output positions t0
            for (int r = 0; r < R; ++r) {
                const int bits = s_bits[r];
                if (!(bits & (1 << (16 + 2 * t2 + t1)))) continue;
                const Yv *Y2r = Y2 + r * nb * 2 * P3;
                const Cv sg = s_sig[r * 3 + 0];
                const int ta = 4 * t2 + 2 * t1;
                const int a0 = s_out[r * 8 + ta], a1 = s_out[r * 8 + ta + 1];
                for (int v = threadIdx.x; v < nb * P2; v += kTT) {
                    const int bl = v / P2, mn = v - bl * P2;
                    Cv z0[P], z1[P];
                    const Yv *y0 = Y2r + (bl * 2 + 0) * P3 + mn;
                    const Yv *y1 = Y2r + (bl * 2 + 1) * P3 + mn;
                    const bool h1 = (s_cj[bl * 8 + 1] >= 0) | (s_cj[bl * 8 + 3] >= 0) |
                                    (s_cj[bl * 8 + 5] >= 0) | (s_cj[bl * 8 + 7] >= 0);
                    const bool h0 = (s_cj[bl * 8 + 0] >= 0) | (s_cj[bl * 8 + 2] >= 0) |
                                    (s_cj[bl * 8 + 4] >= 0) | (s_cj[bl * 8 + 6] >= 0);
#pragma unroll
                    for (int l = 0; l < P; ++l) {
                        z0[l] = h0 ? ld<Cv>(y0 + l * P2) : czero<Cv>();
                        z1[l] = h1 ? ld<Cv>(y1 + l * P2) : czero<Cv>();
                    }
                    if (a0 >= 0)
                        col_interp_s<P, 0, RHO1, C>(Lt, PH, z0, z1, h1, sg,
                            reinterpret_cast<Sv *>(a.out) + ((int64_t)a0 * a.out_row + b0 + bl) * P3 + mn, P2);
                    if (a1 >= 0)
                        col_interp_s<P, 1, RHO1, C>(Lt, PH, z0, z1, h1, sg,
                            reinterpret_cast<Sv *>(a.out) + ((int64_t)a1 * a.out_row + b0 + bl) * P3 + mn, P2);
                }
            }
            __syncthreads();
        }
    }
}


template <int P, bool RHO1, typename S, typename C>
__device__ __forceinline__ void translate2d_item(const TArgs &a, int64_t gid, unsigned char *smem)
{
    using Sv = typename CV<S>::t;
    using Cv = typename CV<C>::t;
    using Yv = typename YT<S, C>::t;
    constexpr int PP = P * P;
    Yv *Y = reinterpret_cast<Yv *>(smem);  // [2 t2][R][nin][P][P]
    __shared__ int s_out[kRowsMax * 4];
    __shared__ int s_bits[kRowsMax];
    __shared__ Cv s_sig[kRowsMax * 2];
    __shared__ unsigned char s_pos[kInMax];
    __shared__ signed char s_cj[kInMax * 4];  // [b][s]: local child index or -1
    const Item2D it = setup2d<Cv>(a, gid, s_out, s_bits, s_sig, s_pos, s_cj);
    const int64_t ap0 = it.ap0;
    const int R = it.R, b0 = it.b0, nb = it.nb, J0 = it.J0, nin = it.nin, all = it.all;

    const cptr<C> Lt = (cptr<C>)(a.Lt);
    const cptr<C> PH = (cptr<C>)(a.PH);
    const cptr<C> LP = (cptr<C>)(a.LP);
    const int ysz = R * nin * PP;  // one t2 half of Y

    // stage 1: every input row once, both output positions t2 it is needed
    // for; the rows a' of the work-group are processed side by side
    // row a' of a flat index through a float reciprocal (exact: the index
    // is below 2^16, so the error is far below the distance 0.5 / rowlen)
    const int rowlen = nin * P;
    const float inv_rowlen = 1.0f / (float)rowlen;
    for (int v = threadIdx.x; v < R * rowlen; v += kTT) {
        const int r = (int)(((float)v + 0.5f) * inv_rowlen);
        const int w = v - r * rowlen;
        const int j = w / P;
        const int bits = s_bits[r];
        const Sv *src = reinterpret_cast<const Sv *>(a.in) + ((ap0 + r) * a.in_row + J0) * PP + w * P;
        Cv x[P];
#pragma unroll
        for (int m = 0; m < P; ++m) x[m] = cvt<Cv>(src[m]);
        const bool s2 = (s_pos[j] >> 1) & 1;
        const Cv sg = s_sig[r * 2 + 1];
        Yv *Yr = Y + r * nin * PP + w * P;
        if (bits & (1 << 4)) row_interp<P, 0, RHO1, C>(Lt, PH, x, s2, sg, Yr);
        if (bits & (1 << 5)) row_interp<P, 1, RHO1, C>(Lt, PH, x, s2, sg, Yr + ysz);
    }
    __syncthreads();

    // stage 2: every output column once per t2, both output positions t1,
    // all rows side by side.  Narrow work splits the output rows over G
    // wave-aligned groups of threads, so all four waves work.
    const int ncol = nb * P;
    const float inv_ncol = 1.0f / (float)ncol;
    const int ntot = R * ncol;
    const int G = (ntot <= 64 && kWaves >= 4) ? 4 : ((ntot <= 128 && kWaves >= 2) ? 2 : 1);
    const int span = kTT / G;
    const int grp = __builtin_amdgcn_readfirstlane((int)threadIdx.x / span);
    const int lane = (int)threadIdx.x - grp * span;
    for (int t2 = 0; t2 < 2; ++t2) {
        if (!(all & (1 << (4 + t2)))) continue;  // uniform
        for (int v = lane; v < ntot; v += span) {
            const int r = (int)(((float)v + 0.5f) * inv_ncol);
            const int col = v - r * ncol;
            const int bits = s_bits[r];
            if (!(bits & (1 << (4 + t2)))) continue;
            const int bl = col / P, m = col - bl * P;
            const Yv *Yr = Y + t2 * ysz + r * nin * PP;
            const int a0 = s_out[r * 4 + (t2 << 1)], a1 = s_out[r * 4 + 1 + (t2 << 1)];
            const int c0 = s_cj[bl * 4 + 0], c2 = s_cj[bl * 4 + 2];
            const int c1 = s_cj[bl * 4 + 1], c3 = s_cj[bl * 4 + 3];
            // one branch per child slot, not per element
            Cv z0[P], z1[P];
#pragma unroll
            for (int l = 0; l < P; ++l) z0[l] = z1[l] = czero<Cv>();
            if (c0 >= 0) {
                const Yv *yp = Yr + c0 * PP + m;
#pragma unroll
                for (int l = 0; l < P; ++l) z0[l] = ld<Cv>(yp + l * P);
            }
            if (c2 >= 0) {
                const Yv *yp = Yr + c2 * PP + m;
#pragma unroll
                for (int l = 0; l < P; ++l) z0[l] = cadd(z0[l], ld<Cv>(yp + l * P));
            }
            if (c1 >= 0) {
                const Yv *yp = Yr + c1 * PP + m;
#pragma unroll
                for (int l = 0; l < P; ++l) z1[l] = ld<Cv>(yp + l * P);
            }
            if (c3 >= 0) {
                const Yv *yp = Yr + c3 * PP + m;
#pragma unroll
                for (int l = 0; l < P; ++l) z1[l] = cadd(z1[l], ld<Cv>(yp + l * P));
            }
            const bool h1 = (c1 >= 0) | (c3 >= 0);
            if (!RHO1 && h1) {
                const Cv sg = s_sig[r * 2];
#pragma unroll
                for (int l = 0; l < P; ++l) z1[l] = cmul(sg, z1[l]);
            }
            if (a0 >= 0)
                col_interp_g<P, 0, S, C>(Lt, LP, PH, z0, z1, h1,
                    reinterpret_cast<Sv *>(a.out) + ((int64_t)a0 * a.out_row + b0 + bl) * PP + m, grp, G);
            if (a1 >= 0)
                col_interp_g<P, 1, S, C>(Lt, LP, PH, z0, z1, h1,
                    reinterpret_cast<Sv *>(a.out) + ((int64_t)a1 * a.out_row + b0 + bl) * PP + m, grp, G);
        }
    }
}

// One work item per work-group (single transform).
// Waves per SIMD the register allocation must allow: five (at most 96
// VGPRs) up to p = 9; the larger grids of p >= 10 need the full register file.
template <int D, int P> constexpr int min_waves() { return (D == 2 && P <= 9) ? 5 : 1; }

template <int P, bool RHO1, typename S, typename C>
__global__ __launch_bounds__(kTT, (min_waves<2, P>())) void k_translate2d(TArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    translate2d_item<P, RHO1, S, C>(a, blockIdx.x, smem);
}

template <int P, bool RHO1, typename S, typename C>
__global__ __launch_bounds__(kTT) void k_translate3d(TArgs a)
{
    extern __shared__ __align__(16) unsigned char smem[];
    translate3d_item<P, RHO1, S, C>(a, blockIdx.x, smem);
}

// Persistent batched step: the work items of all transforms still active at
// this sweep step form one index space (prefix[t] = first item of transform
// t).  Work-groups take the next item from a counter that starts at zero
// for every step, so late-starting work-groups cannot leave a tail; a
// work-group finishes when the counter passes the end.
template <int D, int P, typename S, typename C>
__global__ __launch_bounds__(kTT, (min_waves<D, P>() > 1 ? 4 : 1)) void k_translate_batched(
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
                                                                  int ndesc)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int64_t item = blockIdx.x;
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

int lds_budget_default()
{
    const char *s = std::getenv("BFSFT_LDS_KB");
    const int v = s ? std::atoi(s) : 0;
    return ((v >= 8 && v <= 64) ? v : 32) * 1024;
}

}  // namespace

int translate_default_lds() { return lds_budget_default(); }

// LDS blocks (p^d elements of the intermediate type) a work-group may hold
// within `budget` bytes
int translate_cap_blocks(int d, int p, int precision, int budget)
{
    int PD = p;
    for (int a = 1; a < d; ++a) PD *= p;
#ifdef BFSFT_MIXED_Y64
    const int elem = precision != BFSFT_FP32 ? 16 : 8;
#else
    const int elem = precision == BFSFT_FP64 ? 16 : 8;
#endif
    int cap = budget / (PD * elem);
    const int one_box = d == 2 ? 2 * 4 : 8 + 2;  // a single box with all children
    if (cap < one_box) cap = one_box;
    return cap;
}

// LDS blocks a tile of nb boxes with nin children needs: the VALU kernels
// hold the axis-2 results (2D: both t2) or two stages (3D); the matrix-core
// kernel also stages the input blocks
int translate_tile_cost(int d, int nin, int nb, int kind)
{
    if (kind == 1) return 3 * nin;
    return d == 2 ? 2 * nin : nin + 2 * nb;
}

bool translate_fits(int d, int p, int precision)
{
    int PD = p;
    for (int a = 1; a < d; ++a) PD *= p;
    const int elem = precision == BFSFT_FP64 ? 16 : 8;
    const int one_box = d == 2 ? 2 * 4 : 8 + 2;
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

#ifdef BFSFT_MIXED_Y64
size_t ysize(int precision) { return precision != BFSFT_FP32 ? 16 : 8; }
#else
size_t ysize(int precision) { return precision == BFSFT_FP64 ? 16 : 8; }
#endif

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
    const int64_t grid = translate_items(la);
    if (grid == 0) return;
    const TArgs a = make_targs(c, la);
    const size_t lds = translate_lds_bytes(c.d, c.p, c.precision, la.rows, la.cost_max);
    if (lds > kLdsMax) throw Error{BFSFT_EINVAL, "translation tile exceeds LDS"};
    auto body = [&](auto tag, auto *sp, auto *cp, auto d3) {
        constexpr int P = decltype(tag)::value;
        using S = std::remove_pointer_t<decltype(sp)>;
        using C = std::remove_pointer_t<decltype(cp)>;
        if constexpr (decltype(d3)::value) {
            if (la.sig)
                k_translate3d<P, false, S, C><<<(unsigned)grid, kTT, lds, c.stream>>>(a);
            else
                k_translate3d<P, true, S, C><<<(unsigned)grid, kTT, lds, c.stream>>>(a);
        } else {
            if (la.sig)
                k_translate2d<P, false, S, C><<<(unsigned)grid, kTT, lds, c.stream>>>(a);
            else
                k_translate2d<P, true, S, C><<<(unsigned)grid, kTT, lds, c.stream>>>(a);
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
    if (lds > kLdsMax) throw Error{BFSFT_EINVAL, "translation tile exceeds LDS"};
    const unsigned g = (unsigned)std::min<int64_t>(grid, total);
    auto body = [&](auto tag, auto *sp, auto *cp, auto dd) {
        constexpr int P = decltype(tag)::value;
        constexpr int D = decltype(dd)::value;
        using S = std::remove_pointer_t<decltype(sp)>;
        using C = std::remove_pointer_t<decltype(cp)>;
        if (grid <= 0)
            k_translate_batched_flat<D, P, S, C><<<(unsigned)total, kTT, lds, c.stream>>>(
                (const TArgs *)descs, prefix, ndesc);
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
