// Step 3 of Section 2.2 in 2D on the FP64 matrix cores of gfx950.
//
// The translation of a level is the same as in translate.hip: per axis,
// w^{AB}[l] = sum_s f(s, t, l) (L_t w^{A'B_s})[l], here applied to the
// rotated state w^ = E w, i.e. with the operator E L_t E^{-1} (E = diag of
// exp(-i pi rho k / q)), whose copy rows carry the phase E[l] / E[node].
// Only the dot rows (floor(p/2) per t) are contractions, and those run as
// v_mfma_f64_16x16x4f64 products with the operator as the 16-row A
// operand and 16 state lines as the B operand.  Complex products are
// written in real form: a complex row (w_0 .. w_{p-1}) becomes the 2p reals
// (re w_0, im w_0, ...), and the operator entry W becomes the 2x2 block
// [[re W, -im W], [im W, re W]].
//
//   stage 1 (axis 2): D1[(t2, k, re/im)][line] = sum over the 2p reals of
//       the input line: both output positions t2 and all floor(p/2) dot
//       rows k in one 16-row output tile (p <= 9).  The phase of the
//       child's offsets, f(s2, t2, .) and, when rho != 1, sigma of axis 1,
//       is applied to the result; the copy rows (unit rows of L_t2) are
//       moved by the VALU with the same phases.
//   stage 2 (axis 1): D2[(t1, k, re/im)][column] = sum over the 4p reals
//       (z_0, z_1 at every node, z_s1 = sum of the children with that s1)
//       with the phase of s1 = 1 folded into the operator.  Each lane
//       builds complete z values of the nodes it owns, so the copy rows of
//       stage 2 are formed from its own registers.
//
// The input block of every child is first copied from HBM into LDS with
// coalesced loads.  Absent children read a zero block.  Everything is FP64
// arithmetic; the state and the LDS intermediates are stored in the state
// precision (FP32 for the mixed path).
#include "bfsft_impl.h"
#include "cplx.h"
#include "dispatch.h"
#include "translate_common.h"

#include <type_traits>

namespace bfsft {

namespace {

using namespace tr;

typedef double dx4 __attribute__((ext_vector_type(4)));

// Shape of the per-lane operator tables of order p.
struct MShape {
    int P, Q, ND, NC, KS1, NB, REM;
    int oT1, oT2, oDPH, oNPH, oCF, size;
    __host__ __device__ constexpr explicit MShape(int p)
        : P(p), Q(p - 1), ND(p / 2), NC(p - p / 2), KS1((2 * p + 3) / 4), NB(p / 4), REM(p % 4),
          oT1(0), oT2(((2 * p + 3) / 4) * 64), oDPH(((2 * p + 3) / 4) * 64 + p * 64),
          oNPH(((2 * p + 3) / 4) * 64 + p * 64 + 256), oCF(((2 * p + 3) / 4) * 64 + p * 64 + 256 + 2 * p),
          size(((2 * p + 3) / 4) * 64 + p * 64 + 256 + 6 * p)
    {
    }
};

// output row of dot k of L_t
__host__ __device__ constexpr int dot_row(int P, int t, int k) { return ((1 + t * (P - 1)) & 1) + 2 * k; }

// entry of the real form of a complex operator entry w: output part (0 re,
// 1 im) times input part
__device__ __forceinline__ double realform(int part, int kpart, double2 w)
{
    return part == 0 ? (kpart == 0 ? w.x : -w.y) : (kpart == 0 ? w.y : w.x);
}

// Per-lane tables, one wave.  Operands of v_mfma_f64_16x16x4f64: lane
// i + 16 kq holds A[i][kq] and B[kq][i] of each 16x4 / 4x16 step, and
// register r of the result holds D[4 r + kq][i].  Output row i is ordered
// so that a lane's four result registers are the (re, im) pairs of the
// complex outputs 2 kq and 2 kq + 1:  row i <-> complex output
// 2 (i mod 4) + floor(i / 8), part (floor(i / 4) mod 2).
//   T1[s][lane]:  output row lane % 16 (complex output c = t2 ND + k),
//                 input real 4 s + kq of a line (2p reals, zero beyond),
//   T2[s][lane]:  output o as above with t1, input (node, component) of
//                 step s: steps 4b..4b+3 give components 0..3 (re z0,
//                 im z0, re z1, im z1) of node 4b + kq; the p mod 4 last
//                 steps give component kq of the remaining nodes,
//   DPH[h][lane]: phase PH_t[row] of complex output 2 kq + h of stage 1,
//   NPH[node]:    phase of the copy rows through node (same for t = 0, 1),
//   CF[t][node]:  entry E[l] / E[node] of the copy row l = 2 node - t q.
// Operator entries are those of the rotated state, E[row] L_t[row][k] / E[k].
__global__ void k_mfma_tables(int p, const double2 *__restrict__ L64, const double2 *__restrict__ PH64,
                              const double2 *__restrict__ erot, double *__restrict__ mt)
{
    const MShape m(p);
    auto lrot = [&](int t, int row, int k) {
        const double2 ek = erot[k];
        return cmul(cmul(erot[row], L64[(t * p + row) * p + k]), make_double2(ek.x, -ek.y));
    };
    const int lane = threadIdx.x, i = lane & 15, kq = lane >> 4;
    const int co = 2 * (i & 3) + (i >> 3), part = (i >> 2) & 1;
    const bool orow = co < 2 * m.ND;
    const int t = orow ? co / m.ND : 0, kk = orow ? co % m.ND : 0, row = dot_row(p, t, kk);
    for (int s = 0; s < m.KS1; ++s) {
        const int k = 4 * s + kq;
        double v = 0.0;
        if (orow && k < 2 * p) v = realform(part, k & 1, lrot(t, row, k >> 1));
        mt[m.oT1 + s * 64 + lane] = v;
    }
    for (int s = 0; s < p; ++s) {
        int node, comp;
        if (s < 4 * m.NB) {
            node = 4 * (s >> 2) + kq;
            comp = s & 3;
        } else {
            node = 4 * m.NB + (s - 4 * m.NB);
            comp = kq;
        }
        double v = 0.0;
        if (orow) {
            double2 w = lrot(t, row, node);
            if (comp >= 2) w = cmul(PH64[t * p + row], w);
            v = realform(part, comp & 1, w);
        }
        mt[m.oT2 + s * 64 + lane] = v;
    }
    for (int h = 0; h < 2; ++h) {
        const int c2 = 2 * kq + h;
        double2 ph = make_double2(1.0, 0.0);
        if (c2 < 2 * m.ND) ph = PH64[(c2 / m.ND) * p + dot_row(p, c2 / m.ND, c2 % m.ND)];
        mt[m.oDPH + (2 * h) * 64 + lane] = ph.x;
        mt[m.oDPH + (2 * h + 1) * 64 + lane] = ph.y;
    }
    if (lane < p) {
        const int nd = lane;
        const double2 ph = 2 * nd <= m.Q ? PH64[2 * nd] : PH64[p + 2 * nd - m.Q];
        mt[m.oNPH + 2 * nd] = ph.x;
        mt[m.oNPH + 2 * nd + 1] = ph.y;
    }
    if (lane < 2 * p) {
        const int t = lane / p, nd = lane % p, l = 2 * nd - t * m.Q;
        double2 cf = make_double2(0.0, 0.0);
        if (l >= 0 && l < p) {
            const double2 en = erot[nd];
            cf = cmul(erot[l], make_double2(en.x, -en.y));
        }
        mt[m.oCF + 2 * lane] = cf.x;
        mt[m.oCF + 2 * lane + 1] = cf.y;
    }
}

template <int P, bool RHO1, typename S>
__global__ __launch_bounds__(kTT) void k_translate2d_mfma(TArgs a, const double *__restrict__ mt, int64_t item0)
{
    constexpr MShape M(P);
    constexpr int PP = P * P, Q = P - 1, ND = M.ND, NC = M.NC, KS1 = M.KS1, NB = M.NB, REM = M.REM;
    static_assert(4 * ND <= 16, "stage outputs must fit one 16-row tile");
    using Sv = typename CV<S>::t;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ __align__(16) int s_out[kRowsMax * 4];
    __shared__ int s_bits[kRowsMax];
    __shared__ double2 s_sig[kRowsMax * 2];
    __shared__ unsigned char s_pos[kInMax];
    __shared__ int s_cj4[kInMax];  // [b]: local child index of slots 0..3, one byte each
    __shared__ double2 s_nph[P];
    __shared__ double2 s_cf[2 * P];

    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6, kq = lane >> 4, j16 = lane & 15;
    if (tid < P) s_nph[tid] = make_double2(mt[M.oNPH + 2 * tid], mt[M.oNPH + 2 * tid + 1]);
    if (tid < 2 * P) s_cf[tid] = make_double2(mt[M.oCF + 2 * tid], mt[M.oCF + 2 * tid + 1]);
    const Item2D it = setup2d<double2>(a, item0 + blockIdx.x, s_out, s_bits, s_sig, s_pos,
                                       reinterpret_cast<signed char *>(s_cj4));
    const int R = it.R, nb = it.nb, nin = it.nin;
    const int nblk = R * nin;
    const int ysz = nblk * PP;  // one t2 half of Y
    Sv *X = reinterpret_cast<Sv *>(smem);  // [R][nin][P][P] input blocks
    Sv *Y = X + ysz;                       // [2 t2][R][nin][P][P] after stage 1
    Sv *Zb = Y + 2 * ysz;                  // [P][P] zeros (absent children)

    // zero block; input rows of the work-group (one contiguous segment per
    // row a'), coalesced
    for (int e = tid; e < PP; e += kTT) {
        Sv z;
        z.x = 0;
        z.y = 0;
        Zb[e] = z;
    }
    {
        const int seg = nin * PP;
        const Sv *in = reinterpret_cast<const Sv *>(a.in) + (it.ap0 * a.in_row + it.J0) * PP;
        const int64_t rs = a.in_row * PP;
        for (int r = 0; r < R; ++r) {
            const Sv *src = in + r * rs;
            Sv *dst = X + r * seg;
            for (int e0 = tid; e0 < seg; e0 += 4 * kTT) {
                Sv v[4];
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (e0 + u * kTT < seg) v[u] = src[e0 + u * kTT];
#pragma unroll
                for (int u = 0; u < 4; ++u)
                    if (e0 + u * kTT < seg) dst[e0 + u * kTT] = v[u];
            }
        }
    }
    __syncthreads();

    // row a' of a child block index cc = r nin + j: a float reciprocal is
    // exact here (cc < 2^12, so the error is far below 0.5 / nin)
    const float inv_nin = 1.0f / (float)nin;
    const int nrow = nblk * P;  // input lines (r, j, l1')

    // ---- stage 1 (axis 2): dot rows on the matrix cores, two tiles of 16
    // lines per wave and step; copy rows in the epilogue
    {
        double t1[KS1];
#pragma unroll
        for (int s = 0; s < KS1; ++s) t1[s] = mt[M.oT1 + s * 64 + lane];
        double2 dph[2];
#pragma unroll
        for (int h = 0; h < 2; ++h)
            dph[h] = make_double2(mt[M.oDPH + 2 * h * 64 + lane], mt[M.oDPH + (2 * h + 1) * 64 + lane]);
        const S *xr = reinterpret_cast<const S *>(X);
        // results of line n: the two dot outputs of this lane, then its share
        // (combinations kq, kq + 4, ...) of the 2 NC copy rows
        auto epilogue = [&](int n, const dx4 &acc) {
            const int cc = n / P;
            const int r = (int)(((float)cc + 0.5f) * inv_nin);
            const int pos = s_pos[cc - r * nin];
            const int bits = s_bits[r];
            const bool s1 = pos & 1, s2 = (pos >> 1) & 1;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int co = 2 * kq + h;
                if (co >= 2 * ND) continue;
                double2 y = make_double2(acc[2 * h], acc[2 * h + 1]);
                if (s2) y = cmul(y, RHO1 ? dph[h] : cmul(s_sig[r * 2 + 1], dph[h]));
                if (!RHO1 && s1) y = cmul(y, s_sig[r * 2]);
                const int t2 = co >= ND ? 1 : 0, k = co - t2 * ND;
                st(Y + t2 * ysz + n * P + dot_row(P, t2, k), y);
            }
#pragma unroll
            for (int i = 0; i < (2 * NC + 3) / 4; ++i) {
                const int c = kq + 4 * i;
                if (c >= 2 * NC) continue;
                const int t2 = c >= NC ? 1 : 0, jc = c - t2 * NC;
                if (!((bits >> (4 + t2)) & 1)) continue;
                const int l2 = 2 * jc + (t2 & Q & 1);
                const int node = (t2 * Q + l2) >> 1;
                double2 v = cmul(ld<double2>(X + n * P + node), s_cf[t2 * P + node]);
                if (s2) v = cmul(v, RHO1 ? s_nph[node] : cmul(s_sig[r * 2 + 1], s_nph[node]));
                if (!RHO1 && s1) v = cmul(v, s_sig[r * 2]);
                st(Y + t2 * ysz + n * P + l2, v);
            }
        };
        const int nt = (nrow + 15) >> 4;
        for (int tile = wave; tile < nt; tile += 2 * kWaves) {
            const int n0 = tile * 16 + j16, n1 = n0 + 16 * kWaves;  // tiles `tile`, `tile + kWaves`
            const int c0 = min(n0, nrow - 1), c1 = min(n1, nrow - 1);
            double b0[KS1], b1[KS1];
#pragma unroll
            for (int s = 0; s < KS1; ++s) {
                const int k = 4 * s + kq;
                const bool kin = k < 2 * P;
                const int kc = kin ? k : 0;
                const double x0 = (double)xr[c0 * 2 * P + kc];
                const double x1 = (double)xr[c1 * 2 * P + kc];
                b0[s] = (kin && n0 < nrow) ? x0 : 0.0;
                b1[s] = (kin && n1 < nrow) ? x1 : 0.0;
            }
            dx4 acc0 = {0.0, 0.0, 0.0, 0.0}, acc1 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int s = 0; s < KS1; ++s) {
                acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(t1[s], b0[s], acc0, 0, 0, 0);
                acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(t1[s], b1[s], acc1, 0, 0, 0);
            }
            if (n0 < nrow) epilogue(n0, acc0);
            if (n1 < nrow) epilogue(n1, acc1);
        }
    }
    __syncthreads();

    // ---- stage 2 (axis 1): columns (r, b, l2) of both output positions t1
    {
        double tv[P];
#pragma unroll
        for (int s = 0; s < P; ++s) tv[s] = mt[M.oT2 + s * 64 + lane];
        const int ncol = R * nb * P;
        const int nt = (ncol + 15) >> 4;
        const float inv_nb = 1.0f / (float)nb;
        Sv *out = reinterpret_cast<Sv *>(a.out);
        for (int t2 = 0; t2 < 2; ++t2) {
            if (!((it.all >> (4 + t2)) & 1)) continue;  // uniform
            const Sv *Yt = Y + t2 * ysz;
            for (int tile = wave; tile < nt; tile += kWaves) {
                const int n = tile * 16 + j16;
                int r = 0, bl = 0, l2 = 0;
                bool valid = n < ncol;
                if (valid) {
                    const int bb = n / P;
                    l2 = n - bb * P;
                    r = (int)(((float)bb + 0.5f) * inv_nb);
                    bl = bb - r * nb;
                    valid = (s_bits[r] >> (4 + t2)) & 1;
                }
                if (__ballot(valid) == 0) continue;  // whole tile unused at this t2
                const int cj = valid ? s_cj4[bl] : -1;  // four bytes of -1 when invalid
                const Sv *yb[4];
                const int base = r * nin;
#pragma unroll
                for (int s = 0; s < 4; ++s) {
                    const int c = (int)(signed char)((cj >> (8 * s)) & 0xff);
                    yb[s] = (c >= 0 ? Yt + (base + c) * PP : Zb) + l2;
                }
                double bv[P];
                double2 z0o[NB > 0 ? NB : 1], z1o[NB > 0 ? NB : 1];
#pragma unroll
                for (int bk = 0; bk < NB; ++bk) {
                    const int node = 4 * bk + kq;
                    z0o[bk] = cadd(ld<double2>(yb[0] + node * P), ld<double2>(yb[2] + node * P));
                    z1o[bk] = cadd(ld<double2>(yb[1] + node * P), ld<double2>(yb[3] + node * P));
                    bv[4 * bk + 0] = z0o[bk].x;
                    bv[4 * bk + 1] = z0o[bk].y;
                    bv[4 * bk + 2] = z1o[bk].x;
                    bv[4 * bk + 3] = z1o[bk].y;
                }
                double2 z0r[REM > 0 ? REM : 1], z1r[REM > 0 ? REM : 1];
#pragma unroll
                for (int j = 0; j < REM; ++j) {
                    const int node = 4 * NB + j;
                    z0r[j] = cadd(ld<double2>(yb[0] + node * P), ld<double2>(yb[2] + node * P));
                    z1r[j] = cadd(ld<double2>(yb[1] + node * P), ld<double2>(yb[3] + node * P));
                    const double2 zz = kq < 2 ? z0r[j] : z1r[j];
                    bv[4 * NB + j] = (kq & 1) ? zz.y : zz.x;
                }
                dx4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
                for (int s = 0; s < P; ++s) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(tv[s], bv[s], acc, 0, 0, 0);
                if (!valid) continue;
                const int2 ao = *reinterpret_cast<const int2 *>(s_out + r * 4 + (t2 << 1));
                const int64_t col = (int64_t)(it.b0 + bl) * PP + l2;
                Sv *o0 = ao.x >= 0 ? out + (int64_t)ao.x * a.out_row * PP + col : nullptr;
                Sv *o1 = ao.y >= 0 ? out + (int64_t)ao.y * a.out_row * PP + col : nullptr;
#pragma unroll
                for (int h = 0; h < 2; ++h) {
                    const int co = 2 * kq + h;
                    if (co >= 2 * ND) continue;
                    const int t1 = co >= ND ? 1 : 0, k = co - t1 * ND;
                    Sv *o = t1 ? o1 : o0;
                    if (o) st(o + dot_row(P, t1, k) * P, make_double2(acc[2 * h], acc[2 * h + 1]));
                }
                // copy rows through the nodes this lane owns: row l1 of
                // position t1 with t1 q + l1 = 2 node
                auto copies = [&](int node, double2 z0, double2 z1) {
                    const double2 v = cadd(z0, cmul(s_nph[node], z1));
                    if (o0 && 2 * node <= Q) st(o0 + (2 * node) * P, cmul(v, s_cf[node]));
                    if (o1 && 2 * node >= Q) st(o1 + (2 * node - Q) * P, cmul(v, s_cf[P + node]));
                };
#pragma unroll
                for (int bk = 0; bk < NB; ++bk) copies(4 * bk + kq, z0o[bk], z1o[bk]);
#pragma unroll
                for (int j = 0; j < REM; ++j)
                    if (kq == (j & 3)) copies(4 * NB + j, z0r[j], z1r[j]);
            }
        }
    }
}

template <typename F> void dispatch_p59(int p, F &&f)
{
    switch (p) {
    case 5: f(std::integral_constant<int, 5>{}); break;
    case 6: f(std::integral_constant<int, 6>{}); break;
    case 7: f(std::integral_constant<int, 7>{}); break;
    case 8: f(std::integral_constant<int, 8>{}); break;
    case 9: f(std::integral_constant<int, 9>{}); break;
    default: throw Error{BFSFT_EINVAL, "matrix-core translation needs 5 <= p <= 9"};
    }
}

}  // namespace

bool translate_mfma_supported(int d, int p, int precision)
{
    return d == 2 && p >= 5 && p <= 9 && (precision == BFSFT_FP64 || precision == BFSFT_MIXED);
}

size_t translate_mfma_table_doubles(int p) { return (size_t)MShape(p).size; }

void build_mfma_tables(const Tables &tb, int p, double *dst, hipStream_t s)
{
    k_mfma_tables<<<1, 64, 0, s>>>(p, reinterpret_cast<const double2 *>(tb.L64),
                                   reinterpret_cast<const double2 *>(tb.PH64),
                                   reinterpret_cast<const double2 *>(tb.erot), dst);
    BF_HIP(hipGetLastError());
}

void launch_translate_mfma(const Launch &c, const LevelArgs &la)
{
    if (!translate_mfma_supported(c.d, c.p, c.precision) || !c.tb->mf)
        throw Error{BFSFT_EINVAL, "matrix-core translation not available for this plan"};
    const int64_t grid = translate_items(la);
    if (grid == 0) return;
    const TArgs a = make_targs(c, la);
    const size_t lds = translate_lds_bytes(2, c.p, c.precision, la.rows, la.cost_max, 1);
    if (lds > kLdsMax2D) throw Error{BFSFT_EINVAL, "translation tile exceeds LDS"};
    dispatch_p59(c.p, [&](auto tag) {
        constexpr int P = decltype(tag)::value;
        // chunks of at most kMaxGroups work-groups (see kMaxGroups)
        const int64_t chunk = max_groups();
        for (int64_t i0 = 0; i0 < grid; i0 += chunk) {
            const unsigned g = (unsigned)std::min<int64_t>(chunk, grid - i0);
            if (c.precision == BFSFT_FP64) {
                if (la.sig)
                    k_translate2d_mfma<P, false, double><<<g, kTT, lds, c.stream>>>(a, c.tb->mf, i0);
                else
                    k_translate2d_mfma<P, true, double><<<g, kTT, lds, c.stream>>>(a, c.tb->mf, i0);
            } else {
                if (la.sig)
                    k_translate2d_mfma<P, false, float><<<g, kTT, lds, c.stream>>>(a, c.tb->mf, i0);
                else
                    k_translate2d_mfma<P, true, float><<<g, kTT, lds, c.stream>>>(a, c.tb->mf, i0);
            }
        }
    });
    BF_HIP(hipGetLastError());
}

}  // namespace bfsft
