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

#include <algorithm>
#include <cstdlib>
#include <type_traits>

namespace bfsft {

namespace {

constexpr int kTT = 256;       // threads of a translation work-group
constexpr int kRowsMax = 32;   // rows a' per work-group
constexpr int kInMax = 160;    // inputs of a tile

struct TArgs {
    const void *in;
    void *out;
    int64_t in_row, out_row;
    const int32_t *x_cb;
    const uint64_t *x_keys;
    const int32_t *k_cb;
    const uint64_t *k_keys;
    const int2 *tiles;
    int ntile;
    int rows;
    int64_t nap;
    const double2 *sig;
    const void *Lt;  // [2][P][P] complex, compute precision
    const void *PH;  // [2][P] complex, compute precision
};

// Row structure of L_t: row l is the unit vector of node (t q + l) / 2 when
// t q + l is even, a full interpolation row otherwise.
template <int P, int T> struct Rows {
    static constexpr int Q = P - 1;
    static constexpr __host__ __device__ bool copy(int l) { return ((T * Q + l) & 1) == 0; }
    static constexpr int first_dot = (1 + T * Q) & 1;
    static constexpr int ndot = (P - first_dot + 1) / 2;
};

template <int P, int T2, typename S, typename C>
__device__ __forceinline__ void stage1(const TArgs &a, int R, int64_t ap0, int J0, int nin,
                                       const int *s_bits, const typename CV<C>::t *s_sig,
                                       const unsigned char *s_pos, typename CV<C>::t *Y)
{
    using Sv = typename CV<S>::t;
    using Cv = typename CV<C>::t;
    using RW = Rows<P, T2>;
    constexpr int PP = P * P, Q = P - 1;
    const cptr<C> Lt = (cptr<C>)(a.Lt);
    const cptr<C> PH = (cptr<C>)(a.PH);
    const Sv *in = reinterpret_cast<const Sv *>(a.in);
    const int per_row = nin * P;
    for (int v = threadIdx.x; v < R * per_row; v += kTT) {
        const int r = v / per_row;
        const int rem = v - r * per_row;
        const int j = rem / P, l = rem - j * P;
        if (!(s_bits[r] & (1 << (4 + T2)))) continue;
        const Sv *src = in + ((ap0 + r) * a.in_row + J0 + j) * PP + l * P;
        Cv x[P];
#pragma unroll
        for (int m = 0; m < P; ++m) x[m] = cvt<Cv>(src[m]);
        const bool s2 = (s_pos[j] >> 1) & 1;
        const Cv sg = s_sig[r * 2 + 1];
        Cv *dst = Y + (r * nin + j) * PP + l * P;
#pragma unroll 1
        for (int k = 0; k < RW::ndot; ++k) {
            const int m = RW::first_dot + 2 * k;
            Cv y = czero<Cv>();
#pragma unroll
            for (int mp = 0; mp < P; ++mp) cfma(y, ldc<Cv>(Lt, T2 * PP + m * P + mp), x[mp]);
            if (s2) y = cmul(y, cmul(sg, ldc<Cv>(PH, T2 * P + m)));
            dst[m] = y;
        }
#pragma unroll
        for (int m = 0; m < P; ++m) {
            if (!RW::copy(m)) continue;
            Cv y = x[(T2 * Q + m) / 2];
            if (s2) y = cmul(y, cmul(sg, ldc<Cv>(PH, T2 * P + m)));
            dst[m] = y;
        }
    }
}

template <int P, int T1, typename S, typename C>
__device__ __forceinline__ void stage2(const TArgs &a, int R, int t2, int nin, int b0, int nb,
                                       const int *s_out, const typename CV<C>::t *s_sig,
                                       const unsigned char *s_pos, const int *s_cb,
                                       const typename CV<C>::t *Y)
{
    using Sv = typename CV<S>::t;
    using Cv = typename CV<C>::t;
    using RW = Rows<P, T1>;
    constexpr int PP = P * P, Q = P - 1;
    const cptr<C> Lt = (cptr<C>)(a.Lt);
    const cptr<C> PH = (cptr<C>)(a.PH);
    Sv *out = reinterpret_cast<Sv *>(a.out);
    const int t = T1 | (t2 << 1);
    const int per_row = nb * P;
    for (int v = threadIdx.x; v < R * per_row; v += kTT) {
        const int r = v / per_row;
        const int rem = v - r * per_row;
        const int bl = rem / P, m = rem - bl * P;
        const int ao = s_out[r * 4 + t];
        if (ao < 0) continue;
        Cv z0[P], z1[P];
#pragma unroll
        for (int l = 0; l < P; ++l) z0[l] = z1[l] = czero<Cv>();
        bool h1 = false;
        for (int j = s_cb[bl]; j < s_cb[bl + 1]; ++j) {
            const Cv *yp = Y + (r * nin + j) * PP + m;
            if (s_pos[j] & 1) {
                h1 = true;
#pragma unroll
                for (int l = 0; l < P; ++l) z1[l] = cadd(z1[l], yp[l * P]);
            } else {
#pragma unroll
                for (int l = 0; l < P; ++l) z0[l] = cadd(z0[l], yp[l * P]);
            }
        }
        const Cv sg = s_sig[r * 2];
        Sv *dst = out + ((int64_t)ao * a.out_row + b0 + bl) * PP + m;
#pragma unroll 1
        for (int k = 0; k < RW::ndot; ++k) {
            const int l = RW::first_dot + 2 * k;
            Cv o0 = czero<Cv>(), o1 = czero<Cv>();
#pragma unroll
            for (int lp = 0; lp < P; ++lp) {
                const Cv lv = ldc<Cv>(Lt, T1 * PP + l * P + lp);
                cfma(o0, lv, z0[lp]);
                cfma(o1, lv, z1[lp]);
            }
            if (h1) o0 = cadd(o0, cmul(o1, cmul(sg, ldc<Cv>(PH, T1 * P + l))));
            Sv so;
            so.x = (S)o0.x;
            so.y = (S)o0.y;
            dst[l * P] = so;
        }
#pragma unroll
        for (int l = 0; l < P; ++l) {
            if (!RW::copy(l)) continue;
            Cv o = z0[(T1 * Q + l) / 2];
            if (h1) o = cadd(o, cmul(z1[(T1 * Q + l) / 2], cmul(sg, ldc<Cv>(PH, T1 * P + l))));
            Sv so;
            so.x = (S)o.x;
            so.y = (S)o.y;
            dst[l * P] = so;
        }
    }
}

template <int P, typename S, typename C>
__global__ __launch_bounds__(kTT) void k_translate2d(TArgs a)
{
    using Cv = typename CV<C>::t;
    extern __shared__ __align__(16) unsigned char smem[];
    Cv *Y = reinterpret_cast<Cv *>(smem);
    __shared__ int s_out[kRowsMax * 4];
    __shared__ int s_bits[kRowsMax];
    __shared__ Cv s_sig[kRowsMax * 2];
    __shared__ unsigned char s_pos[kInMax];
    __shared__ int s_cb[kInMax + 1];

    const int64_t gid = blockIdx.x;
    const int64_t g = gid / a.ntile;
    const int tile = (int)(gid - g * a.ntile);
    const int64_t ap0 = g * a.rows;
    const int R = (int)min((int64_t)a.rows, a.nap - ap0);
    const int2 bt = a.tiles[tile];
    const int b0 = bt.x, nb = bt.y - bt.x;
    const int J0 = a.k_cb[b0];
    const int nin = a.k_cb[bt.y] - J0;

    for (int i = threadIdx.x; i < nin; i += kTT) s_pos[i] = (unsigned char)(a.k_keys[J0 + i] & 3);
    for (int i = threadIdx.x; i <= nb; i += kTT) s_cb[i] = a.k_cb[b0 + i] - J0;
    if (threadIdx.x < R) {
        const int r = threadIdx.x;
        const int64_t ap = ap0 + r;
        int bits = 0;
        int o[4] = {-1, -1, -1, -1};
        for (int i = a.x_cb[ap]; i < a.x_cb[ap + 1]; ++i) {
            const int t = (int)(a.x_keys[i] & 3);
            o[t] = i;
            bits |= (1 << t) | (1 << (4 + (t >> 1)));
        }
#pragma unroll
        for (int t = 0; t < 4; ++t) s_out[r * 4 + t] = o[t];
        s_bits[r] = bits;
        Cv one;
        one.x = 1;
        one.y = 0;
        s_sig[r * 2] = a.sig ? cvt<Cv>(a.sig[ap * 2]) : one;
        s_sig[r * 2 + 1] = a.sig ? cvt<Cv>(a.sig[ap * 2 + 1]) : one;
    }
    __syncthreads();
    int all = 0;
    for (int r = 0; r < R; ++r) all |= s_bits[r];

    for (int t2 = 0; t2 < 2; ++t2) {
        if (!(all & (1 << (4 + t2)))) continue;
        if (t2 == 0)
            stage1<P, 0, S, C>(a, R, ap0, J0, nin, s_bits, s_sig, s_pos, Y);
        else
            stage1<P, 1, S, C>(a, R, ap0, J0, nin, s_bits, s_sig, s_pos, Y);
        __syncthreads();
        if (all & (1 << (t2 << 1)))
            stage2<P, 0, S, C>(a, R, t2, nin, b0, nb, s_out, s_sig, s_pos, s_cb, Y);
        if (all & (1 << (1 | (t2 << 1))))
            stage2<P, 1, S, C>(a, R, t2, nin, b0, nb, s_out, s_sig, s_pos, s_cb, Y);
        __syncthreads();
    }
}

int lds_budget()
{
    static int kb = [] {
        const char *s = std::getenv("BFSFT_LDS_KB");
        int v = s ? std::atoi(s) : 0;
        return (v >= 8 && v <= 150) ? v : 40;
    }();
    return kb * 1024;
}

}  // namespace

int translate_max_inputs(int d, int p, int precision)
{
    const int csize = precision == BFSFT_FP32 ? 8 : 16;
    int PD = p;
    for (int a = 1; a < d; ++a) PD *= p;
    int m = lds_budget() / (PD * csize);
    if (m > kInMax) m = kInMax;
    if (m < (1 << d)) m = 1 << d;
    return m;
}

int translate_rows(int d, int p, int precision, int nin_max, int64_t nap)
{
    int R = translate_max_inputs(d, p, precision) / std::max(1, nin_max);
    R = std::max(1, std::min(R, kRowsMax));
    return (int)std::min<int64_t>(R, std::max<int64_t>(1, nap));
}

void launch_translate(const Launch &c, const LevelArgs &la)
{
    if (la.nap == 0 || la.ntile == 0) return;
    if (c.d != 2) throw Error{BFSFT_EINVAL, "3D translation not built"};
    TArgs a;
    a.in = la.in;
    a.out = la.out;
    a.in_row = la.in_row;
    a.out_row = la.out_row;
    a.x_cb = la.x_cb;
    a.x_keys = la.x_keys;
    a.k_cb = la.k_cb;
    a.k_keys = la.k_keys;
    a.tiles = la.tiles;
    a.ntile = la.ntile;
    a.nap = la.nap;
    a.rows = translate_rows(c.d, c.p, c.precision, la.nin_max, la.nap);
    a.sig = reinterpret_cast<const double2 *>(la.sig);
    const bool f32 = c.precision == BFSFT_FP32;
    a.Lt = f32 ? (const void *)c.tb->L32 : (const void *)c.tb->L64;
    a.PH = f32 ? (const void *)c.tb->PH32 : (const void *)c.tb->PH64;
    const int64_t groups = (la.nap + a.rows - 1) / a.rows;
    const int64_t grid = groups * la.ntile;
    dispatch_p(c.p, [&](auto tag) {
        constexpr int P = decltype(tag)::value;
        dispatch_prec(c.precision, [&](auto *sp, auto *cp) {
            using S = std::remove_pointer_t<decltype(sp)>;
            using C = std::remove_pointer_t<decltype(cp)>;
            const size_t lds = (size_t)a.rows * la.nin_max * P * P * sizeof(typename CV<C>::t);
            k_translate2d<P, S, C><<<(unsigned)grid, kTT, lds, c.stream>>>(a);
        });
    });
    BF_HIP(hipGetLastError());
}

}  // namespace bfsft
