// Step 3 of Section 2.2 in 2D with the axis-2 interpolation (stage 1) on the
// matrix cores.
//
// Stage 1 applies the real interpolation operator R_t2 to every input line
// (one child block row, p complex values along axis 2) for both output
// positions t2.  As a product it is Y = X R^T with X the lines (real and
// imaginary parts as separate rows) and R^T the p x (dot rows of t2 = 0 and
// 1) operator, at most 16 columns for p <= 12: a 16-line group of a wave is
// one 16x16 result tile per part.  The copy rows of R_t2 are written from
// the loaded elements directly.  Stage 2 (children sums with the phases
// G(s2, t2, m), axis-1 interpolation and the output phases) is the VALU
// stage of the 2D kernel in compute precision C.
//
// Contraction formats of stage 1 (accumulation in FP32 inside the matrix
// core in every format):
//   FP32    v_mfma_f32_16x16x4_f32 on the FP32 state and R rounded to FP32;
//   FP16X2  v_mfma_f32_16x16x16_f16 on two-term splits x = x_hi + x_lo and
//           R = R_hi + R_lo (11 + 11 significant bits), three products
//           x_hi R_hi + x_hi R_lo + x_lo R_hi; every line is scaled by a
//           power of two so that its largest part lies in [2^14, 2^15)
//           (FP16 range), and its results are scaled back exactly;
//   BF16X3  v_mfma_f32_16x16x16_bf16 on exact three-term splits of the FP32
//           values (8 + 8 + 8 significant bits, each piece rounded to nearest
//           even) and of R rounded to FP32, six products x_a R_b with
//           a + b <= 2; BF16 has the FP32 exponent range, so no scaling.
//
// Operand layouts (checked on the GPU with an in-bounds probe): for the
// 16x16x4 f32 product lane i + 16k holds A[i][k] and B[k][i]; for the
// 16x16x16 f16/bf16 products lane i + 16g holds A[i][4g .. 4g+3] and
// B[4g .. 4g+3][i]; the 16x16 result leaves D[4g + r][j] in register r of
// lane j + 16g.
#include "bfsft_impl.h"
#include "cplx.h"
#include "dispatch.h"
#include "translate2d.h"

#include <algorithm>
#include <type_traits>

namespace bfsft {

namespace {

using namespace tr;

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef float f32x2 __attribute__((ext_vector_type(2)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));

constexpr int kF32 = 0, kF16X2 = 1, kBF16X3 = 2;

// Result column j (0..15) of a stage-1 tile: output position t2 and dot row
// m of R_t2 (the dot rows of t2 = 0 first, then those of t2 = 1).
template <int P> struct XCols {
    static constexpr int n0 = Rows<P, 0>::ndot, n1 = Rows<P, 1>::ndot;
    static_assert(n0 + n1 <= 16, "dot rows of both positions must fit one 16-column tile");
    static __device__ __forceinline__ bool valid(int j) { return j < n0 + n1; }
    static __device__ __forceinline__ int t2(int j) { return j < n0 ? 0 : 1; }
    static __device__ __forceinline__ int m(int j)
    {
        return j < n0 ? Rows<P, 0>::first_dot + 2 * j : Rows<P, 1>::first_dot + 2 * (j - n0);
    }
};

// Elements of its line a lane holds: F32, K-step s holds element 4 s + k
// (k = lane / 16); the 16-wide formats hold elements 4 g .. 4 g + 3 (g = lane / 16).
template <int P, int F> struct XLane {
    static constexpr int NE = F == kF32 ? (P + 3) / 4 : 4;
    static __device__ __forceinline__ int elem(int e, int g) { return F == kF32 ? 4 * e + g : 4 * g + e; }
};

// The operator operand of one lane (uniform over the lines): B[k][j] =
// R_t2(j)[m(j)][k], zero outside the dot rows and beyond k = p - 1.
template <int P, int F> struct XOp;

template <int P> struct XOp<P, kF32> {
    float b[XLane<P, kF32>::NE];
};
template <int P> struct XOp<P, kF16X2> {
    f16x4 hi, lo;
};
template <int P> struct XOp<P, kBF16X3> {
    bf16x4 b0, b1, b2;
};

__device__ __forceinline__ short bf16_bits(float x) { return (short)(__float_as_uint(x) >> 16); }

// Two FP32 values rounded to BF16 (to nearest even, one v_cvt_pk_bf16_f32),
// as packed bits and as FP32 values.  Round to nearest keeps the terms a
// split drops unbiased: truncation makes them all of one sign.
__device__ __forceinline__ unsigned bf16_pair(float a, float b, float &ra, float &rb)
{
    const bf16x2v h = __builtin_convertvector(f32x2{a, b}, bf16x2v);
    const unsigned u = __builtin_bit_cast(unsigned, h);
    ra = __uint_as_float(u << 16);
    rb = __uint_as_float(u & 0xffff0000u);
    return u;
}

// Exact three-term splits of two FP32 values into BF16 pieces, packed in
// pairs: x = x0 + x1 + x2 (x - x0 has at most 16 significant bits and
// x - x0 - x1 at most 8, so both differences are exact in FP32).
__device__ __forceinline__ void bf16_split3_pair(float a, float b, unsigned &p0, unsigned &p1, unsigned &p2)
{
    float a0, b0, a1, b1, a2, b2;
    p0 = bf16_pair(a, b, a0, b0);
    const float da = a - a0, db = b - b0;
    p1 = bf16_pair(da, db, a1, b1);
    p2 = bf16_pair(da - a1, db - b1, a2, b2);
}

// Two FP32 values (already scaled into the FP16 range) as FP16 hi + lo
// pieces, each rounded to nearest (v_cvt_pk_f16_f32): x = hi + lo + O(2^-22 x)
__device__ __forceinline__ void f16_split2_pair(float a, float b, unsigned &hi, unsigned &lo)
{
    const f16x2 h = __builtin_convertvector(f32x2{a, b}, f16x2);
    const f32x2 hf = __builtin_convertvector(h, f32x2);
    const f16x2 l = __builtin_convertvector(f32x2{a - hf.x, b - hf.y}, f16x2);
    hi = __builtin_bit_cast(unsigned, h);
    lo = __builtin_bit_cast(unsigned, l);
}

template <int P, int F, typename C>
__device__ __forceinline__ XOp<P, F> make_op(const TArgs &a)
{
    const cptr<C> Rt = (cptr<C>)(a.R);
    constexpr int PP = P * P;
    const int lane = threadIdx.x & 63, j = lane & 15, g = lane >> 4;
    const bool jv = XCols<P>::valid(j);
    const int base = jv ? XCols<P>::t2(j) * PP + XCols<P>::m(j) * P : 0;
    XOp<P, F> o;
#pragma unroll
    for (int e = 0; e < XLane<P, F>::NE; ++e) {
        const int k = XLane<P, F>::elem(e, g);
        const double r = (jv && k < P) ? (double)Rt[base + k] : 0.0;
        if constexpr (F == kF32) {
            o.b[e] = (float)r;
        } else if constexpr (F == kF16X2) {
            const _Float16 h = (_Float16)r;
            o.hi[e] = h;
            o.lo[e] = (_Float16)(r - (double)h);
        } else {
            unsigned p0, p1, p2;
            bf16_split3_pair((float)r, 0.f, p0, p1, p2);
            o.b0[e] = (short)(p0 & 0xffffu);
            o.b1[e] = (short)(p1 & 0xffffu);
            o.b2[e] = (short)(p2 & 0xffffu);
        }
    }
    return o;
}

// The lane's elements of line v (zeros beyond the line)
template <int P, int F>
__device__ __forceinline__ void load_elems(const TArgs &a, const Item2D &it, int v, float2 *x)
{
    const float2 *src = row_src<P, float2>(a, it, v);
    const int g = (threadIdx.x & 63) >> 4;
#pragma unroll
    for (int e = 0; e < XLane<P, F>::NE; ++e) {
        const int n = XLane<P, F>::elem(e, g);
        x[e] = n < P ? src[n] : make_float2(0.f, 0.f);
    }
}

// Y = X R^T for the 16 lines of the group, real and imaginary parts; the
// results of lane j + 16 g are lines 4 g + r, column j.
template <int P, int F>
__device__ __forceinline__ void products(const float2 *x, const XOp<P, F> &op, f32x4 &re, f32x4 &im, float4 &scale_back)
{
    re = f32x4{0.f, 0.f, 0.f, 0.f};
    im = f32x4{0.f, 0.f, 0.f, 0.f};
    scale_back = make_float4(1.f, 1.f, 1.f, 1.f);
    if constexpr (F == kF32) {
#pragma unroll
        for (int e = 0; e < XLane<P, F>::NE; ++e) {
            re = __builtin_amdgcn_mfma_f32_16x16x4f32(x[e].x, op.b[e], re, 0, 0, 0);
            im = __builtin_amdgcn_mfma_f32_16x16x4f32(x[e].y, op.b[e], im, 0, 0, 0);
        }
    } else if constexpr (F == kF16X2) {
        // the line's scale: its largest part, over the four lanes holding it
        float mx = 0.f;
#pragma unroll
        for (int e = 0; e < 4; ++e) mx = fmaxf(mx, fmaxf(fabsf(x[e].x), fabsf(x[e].y)));
        mx = fmaxf(mx, __shfl_xor(mx, 16));
        mx = fmaxf(mx, __shfl_xor(mx, 32));
        const int ex = mx > 0.f ? max(-100, min(100, ilogbf(mx))) : 0;
        const float sc = ldexpf(1.f, 14 - ex), inv = ldexpf(1.f, ex - 14);
        // pieces of elements (0, 1) and (2, 3), real and imaginary parts
        unsigned rh[2], rl[2], ih[2], il[2];
#pragma unroll
        for (int e = 0; e < 2; ++e) {  // scaling by powers of two is exact
            f16_split2_pair(x[2 * e].x * sc, x[2 * e + 1].x * sc, rh[e], rl[e]);
            f16_split2_pair(x[2 * e].y * sc, x[2 * e + 1].y * sc, ih[e], il[e]);
        }
        const f16x4 rhv = __builtin_bit_cast(f16x4, make_uint2(rh[0], rh[1]));
        const f16x4 rlv = __builtin_bit_cast(f16x4, make_uint2(rl[0], rl[1]));
        const f16x4 ihv = __builtin_bit_cast(f16x4, make_uint2(ih[0], ih[1]));
        const f16x4 ilv = __builtin_bit_cast(f16x4, make_uint2(il[0], il[1]));
        re = __builtin_amdgcn_mfma_f32_16x16x16f16(rlv, op.hi, re, 0, 0, 0);
        re = __builtin_amdgcn_mfma_f32_16x16x16f16(rhv, op.lo, re, 0, 0, 0);
        re = __builtin_amdgcn_mfma_f32_16x16x16f16(rhv, op.hi, re, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f32_16x16x16f16(ilv, op.hi, im, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f32_16x16x16f16(ihv, op.lo, im, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f32_16x16x16f16(ihv, op.hi, im, 0, 0, 0);
        // result rows 4 g + r belong to lines 4 g + r, whose scale lane 4 g + r holds
        const int g = (threadIdx.x & 63) >> 4;
        scale_back.x = __shfl(inv, 4 * g + 0);
        scale_back.y = __shfl(inv, 4 * g + 1);
        scale_back.z = __shfl(inv, 4 * g + 2);
        scale_back.w = __shfl(inv, 4 * g + 3);
    } else {
        // pieces of elements (0, 1) and (2, 3), real and imaginary parts
        unsigned q0[2], q1[2], q2[2], j0[2], j1[2], j2[2];
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            bf16_split3_pair(x[2 * e].x, x[2 * e + 1].x, q0[e], q1[e], q2[e]);
            bf16_split3_pair(x[2 * e].y, x[2 * e + 1].y, j0[e], j1[e], j2[e]);
        }
        const bf16x4 r0 = __builtin_bit_cast(bf16x4, make_uint2(q0[0], q0[1]));
        const bf16x4 r1 = __builtin_bit_cast(bf16x4, make_uint2(q1[0], q1[1]));
        const bf16x4 r2 = __builtin_bit_cast(bf16x4, make_uint2(q2[0], q2[1]));
        const bf16x4 i0 = __builtin_bit_cast(bf16x4, make_uint2(j0[0], j0[1]));
        const bf16x4 i1 = __builtin_bit_cast(bf16x4, make_uint2(j1[0], j1[1]));
        const bf16x4 i2 = __builtin_bit_cast(bf16x4, make_uint2(j2[0], j2[1]));
        // x_a R_b with a + b <= 2, smallest terms first
        re = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(r2, op.b0, re, 0, 0, 0);
        re = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(r1, op.b1, re, 0, 0, 0);
        re = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(r0, op.b2, re, 0, 0, 0);
        re = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(r1, op.b0, re, 0, 0, 0);
        re = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(r0, op.b1, re, 0, 0, 0);
        re = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(r0, op.b0, re, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(i2, op.b0, im, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(i1, op.b1, im, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(i0, op.b2, im, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(i1, op.b0, im, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(i0, op.b1, im, 0, 0, 0);
        im = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(i0, op.b0, im, 0, 0, 0);
    }
}

// Groups of 16 lines a wave loads at once in stage 1: a work item's lines
// (about 225 at the tuned tiles of p = 9) usually fit one batch, so stage 1
// waits for memory once, as the VALU kernel's one-line-per-thread pass does.
constexpr int kBatch = 4;

// The lane's elements of the wave's batch of groups starting at line `base`
template <int P, int F>
__device__ __forceinline__ void load_batch(const TArgs &a, const Item2D &it, int base, int nlines,
                                           float2 (&x)[kBatch][XLane<P, F>::NE])
{
    const int i = threadIdx.x & 15;
#pragma unroll
    for (int b = 0; b < kBatch; ++b) load_elems<P, F>(a, it, min(base + 16 * kWaves * b + i, nlines - 1), x[b]);
}

// Stage 1 on the matrix cores: wave w takes the groups of 16 consecutive
// input lines starting at 16 w, 16 (w + kWaves), ... (lines past the end
// are loaded clamped and not stored); every lane of the wave takes part in
// every product.  x holds the lane's elements of the wave's first batch on
// entry.
template <int P, int F>
__device__ __forceinline__ void stage1_xdl(const TArgs &a, const Item2D &it, float2 (&x)[kBatch][XLane<P, F>::NE],
                                           float2 *Y, const XOp<P, F> &op)
{
    constexpr int NE = XLane<P, F>::NE, Q = P - 1;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int i = lane & 15, g = lane >> 4;
    const int rowlen = it.nin * P;
    const int nlines = it.R * rowlen;
    const int ysz = it.R * it.nin * P * P;  // one t2 half of Y
    const bool jv = XCols<P>::valid(i);
    const int jt = XCols<P>::t2(i), jm = XCols<P>::m(i);
    for (int base = 16 * wave; base < nlines; base += 16 * kWaves * kBatch) {  // uniform in the wave
        if (base != 16 * wave) load_batch<P, F>(a, it, base, nlines, x);
#pragma unroll
        for (int b = 0; b < kBatch; ++b) {
            const int g0 = base + 16 * kWaves * b;
            if (g0 >= nlines) break;  // uniform in the wave
            f32x4 re, im;
            float4 sb;
            products<P, F>(x[b], op, re, im, sb);
            // dot rows: lines g0 + 4 g + r, column i.  Both positions t2 are
            // stored whether or not the line's row a' needs them (stage 2
            // reads only the needed ones; Y holds both).
            if (jv) {
                const float s4[4] = {sb.x, sb.y, sb.z, sb.w};
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int w = g0 + 4 * g + r;
                    if (w >= nlines) continue;
                    // only the FP16 format scales its lines
                    Y[jt * ysz + w * P + jm] = F == kF16X2 ? make_float2(re[r] * s4[r], im[r] * s4[r])
                                                           : make_float2(re[r], im[r]);
                }
            }
            // copy rows: the lane's own elements n of line g0 + i go to row 2n
            // (t2 = 0) and 2n - q (t2 = 1)
            const int v = g0 + i;
            if (v < nlines) {
#pragma unroll
                for (int e = 0; e < NE; ++e) {
                    const int n = XLane<P, F>::elem(e, g);
                    if (n >= P) continue;
                    if (2 * n <= Q) Y[v * P + 2 * n] = x[b][e];
                    if (2 * n >= Q) Y[ysz + v * P + 2 * n - Q] = x[b][e];
                }
            }
        }
    }
}

// One 2D work item with stage 1 on the matrix cores (FP32 state, stage 2
// in C).
template <int P, bool RHO1, typename C, int F>
__device__ __forceinline__ void translate2d_xdl_item(const TArgs &a, int64_t gid, unsigned char *smem)
{
    using Cv = typename CV<C>::t;
    __shared__ Tables2D<Cv> tb;
    float2 *Y = reinterpret_cast<float2 *>(smem);  // [2 t2][R][nin][P][P]
    Item2D it = item2d(a, gid);
    Cv gval = load_gc<P, C>(a);  // first: see pin_after
    const Slots2D h = load_slots(a, it);
    __builtin_amdgcn_sched_barrier(0);  // keep these loads ahead of the lines'
    // the wave's first batch of lines, in flight through the table fill
    float2 x[kBatch][XLane<P, F>::NE];
    load_batch<P, F>(a, it, 16 * (int)(threadIdx.x >> 6), it.R * it.nin * P, x);
    pin_after(gval);
    const XOp<P, F> op = make_op<P, F, C>(a);
    fill_tables<RHO1>(a, it, h, tb, gval, 4 * P);
    stage1_xdl<P, F>(a, it, x, Y, op);
    __syncthreads();
    stage2_2d<P, RHO1, float, C>(a, it, Y, tb);
}

template <int P, bool RHO1, typename C, int F>
__global__ __launch_bounds__(kTT, (min_waves<2, P>())) void k_translate2d_xdl(TArgs a, int64_t item0)
{
    extern __shared__ __align__(16) unsigned char smem[];
    translate2d_xdl_item<P, RHO1, C, F>(a, item0 + blockIdx.x, smem);
}

// Batched step forms (see translate.hip): one work-group per item, and
// persistent work-groups taking items from a counter.
template <int P, typename C, int F>
__global__ __launch_bounds__(kTT, (min_waves<2, P>())) void k_translate_batched_xdl_flat(
    const TArgs *__restrict__ descs, const int64_t *__restrict__ prefix, int ndesc, int64_t item0)
{
    extern __shared__ __align__(16) unsigned char smem[];
    const int64_t item = item0 + blockIdx.x;
    int lo = 0, hi = ndesc - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (prefix[mid] <= item) lo = mid; else hi = mid - 1;
    }
    const TArgs a = load_desc(descs, lo);
    translate2d_xdl_item<P, false, C, F>(a, item - prefix[lo], smem);
}

template <int P, typename C, int F>
__global__ __launch_bounds__(kTT, (min_waves<2, P>())) void k_translate_batched_xdl(
    const TArgs *__restrict__ descs, const int64_t *__restrict__ prefix, int ndesc, int64_t total,
    unsigned long long *__restrict__ next)
{
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ int64_t s_item;
    for (;;) {
        if (threadIdx.x == 0) s_item = (int64_t)atomicAdd(next, 1ULL);
        __syncthreads();
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
        translate2d_xdl_item<P, false, C, F>(a, item - prefix[lo], smem);
        __syncthreads();  // the LDS and s_item are reused by the next item
    }
}

// (stage-2 compute scalar, contraction format) of a precision
template <typename Fn> void dispatch_xdl(int precision, Fn &&fn)
{
    switch (precision) {
    case BFSFT_FP32: fn((float *)nullptr, std::integral_constant<int, kF32>{}); break;
    case BFSFT_FP16X2: fn((double *)nullptr, std::integral_constant<int, kF16X2>{}); break;
    case BFSFT_BF16X3: fn((double *)nullptr, std::integral_constant<int, kBF16X3>{}); break;
    default: throw Error{BFSFT_EINVAL, "no matrix-core stage 1 for this precision"};
    }
}

}  // namespace

bool translate_xdl_supported(int d, int p, int precision)
{
    return d == 2 && p >= 3 && p <= 12 &&
           (precision == BFSFT_FP32 || precision == BFSFT_FP16X2 || precision == BFSFT_BF16X3);
}

void launch_translate_xdl(const Launch &c, const LevelArgs &la)
{
    if (!translate_xdl_supported(c.d, c.p, c.precision))
        throw Error{BFSFT_EINVAL, "matrix-core stage 1 not available for this plan"};
    const int64_t grid = translate_items(la);
    if (grid == 0) return;
    const TArgs a = make_targs(c, la);
    const size_t lds = translate_lds_bytes(2, c.p, c.precision, la.rows, la.cost_max, 0);
    if (lds > kLdsMax2D) throw Error{BFSFT_EINVAL, "translation tile exceeds LDS"};
    dispatch_p(c.p, [&](auto tag) {
        constexpr int P = decltype(tag)::value;
        dispatch_xdl(c.precision, [&](auto *cp, auto fmt) {
            using C = std::remove_pointer_t<decltype(cp)>;
            constexpr int F = decltype(fmt)::value;
            const int64_t chunk = max_groups();  // see kMaxGroups
            for (int64_t i0 = 0; i0 < grid; i0 += chunk) {
                const unsigned g = (unsigned)std::min<int64_t>(chunk, grid - i0);
                if (la.sig)
                    k_translate2d_xdl<P, false, C, F><<<g, kTT, lds, c.stream>>>(a, i0);
                else
                    k_translate2d_xdl<P, true, C, F><<<g, kTT, lds, c.stream>>>(a, i0);
            }
        });
    });
    BF_HIP(hipGetLastError());
}

void launch_translate_batched_xdl(const Launch &c, const void *descs, const int64_t *prefix, int ndesc,
                                  int64_t total, size_t lds, int grid, unsigned long long *next)
{
    if (total == 0) return;
    if (c.d != 2 || lds > kLdsMax) throw Error{BFSFT_EINVAL, "matrix-core batched step: 2D only, tile within LDS"};
    const unsigned g = (unsigned)std::min<int64_t>(grid, total);
    dispatch_p(c.p, [&](auto tag) {
        constexpr int P = decltype(tag)::value;
        dispatch_xdl(c.precision, [&](auto *cp, auto fmt) {
            using C = std::remove_pointer_t<decltype(cp)>;
            constexpr int F = decltype(fmt)::value;
            if (grid <= 0)
                for (int64_t i0 = 0, chunk = max_groups(); i0 < total; i0 += chunk)  // see kMaxGroups
                    k_translate_batched_xdl_flat<P, C, F>
                        <<<(unsigned)std::min<int64_t>(chunk, total - i0), kTT, lds, c.stream>>>(
                            (const TArgs *)descs, prefix, ndesc, i0);
            else
                k_translate_batched_xdl<P, C, F><<<g, kTT, lds, c.stream>>>((const TArgs *)descs, prefix, ndesc,
                                                                            total, next);
        });
    });
    BF_HIP(hipGetLastError());
}

}  // namespace bfsft
