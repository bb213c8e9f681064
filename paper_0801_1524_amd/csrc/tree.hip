// Step 1 of Section 2.2 on the device: the trees T_X and T_K.
//
// A point's box index along an axis is floor(x * 2^L / N) (clamped to
// [0, 2^L - 1]; the product by 2^L is exact), so boxes are half-open and a
// box at level m is the leaf index shifted right by L - m.  The indices of
// all axes are interleaved into a Morton key (bit b of axis a at key bit
// b*d + a); sorting the keys puts the children of every box next to each
// other, at every level, which is what makes the level sweep a streaming
// pass.  Sorting is an LSD radix sort on 8-bit digits with a stable in-tile
// ranking built from wavefront ballots; unique boxes and parent/child maps
// come from flag + exclusive-scan + compaction passes.
#include "bfsft_impl.h"

#include <algorithm>
#include <cstdlib>

namespace bfsft {

namespace {

constexpr int kThreads = 256;
constexpr int kItems = 8;
constexpr int kTile = kThreads * kItems;

// ------------------------------------------------------------ scan --------

__device__ uint32_t block_scan_exclusive(uint32_t v, uint32_t *total)
{
    __shared__ uint32_t wsum[kThreads / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t x = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        uint32_t y = __shfl_up(x, o);
        if (lane >= o) x += y;
    }
    if (lane == 63) wsum[w] = x;
    __syncthreads();
    uint32_t before = 0, tot = 0;
#pragma unroll
    for (int i = 0; i < kThreads / 64; ++i) {
        if (i < w) before += wsum[i];
        tot += wsum[i];
    }
    __syncthreads();
    *total = tot;
    return before + x - v;
}

__global__ __launch_bounds__(kThreads) void k_scan_tiles(const uint32_t *__restrict__ in,
                                                        uint32_t *__restrict__ out, int n,
                                                        uint32_t *__restrict__ sums)
{
    const int base = blockIdx.x * kTile + threadIdx.x * kItems;
    uint32_t v[kItems];
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
        uint32_t t = (base + i < n) ? in[base + i] : 0u;
        v[i] = s;
        s += t;
    }
    uint32_t tot;
    uint32_t pre = block_scan_exclusive(s, &tot);
#pragma unroll
    for (int i = 0; i < kItems; ++i)
        if (base + i < n) out[base + i] = pre + v[i];
    if (sums && threadIdx.x == 0) sums[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kThreads) void k_scan_add(uint32_t *__restrict__ out, int n,
                                                      const uint32_t *__restrict__ sums)
{
    const uint32_t add = sums[blockIdx.x];
    const int base = blockIdx.x * kTile;
    for (int i = threadIdx.x; i < kTile; i += kThreads)
        if (base + i < n) out[base + i] += add;
}

// ------------------------------------------------------------ keys --------

__device__ uint64_t morton(const int64_t *idx, int d, int L)
{
    uint64_t key = 0;
    for (int b = 0; b < L; ++b)
        for (int a = 0; a < d; ++a)
            key |= (uint64_t)((idx[a] >> b) & 1) << (b * d + a);
    return key;
}

__global__ void k_point_keys(const double *__restrict__ pts, int64_t n, int d, int L, int64_t N,
                             uint64_t *__restrict__ keys, int32_t *__restrict__ vals,
                             double *__restrict__ local)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int64_t nleaf = (int64_t)1 << L;
    int64_t idx[3] = {0, 0, 0};
    for (int a = 0; a < d; ++a) {
        const double x = pts[i * d + a];
        double v = floor(ldexp(x, L) / (double)N);
        int64_t c = (int64_t)v;
        if (v < 0.0) c = 0;
        if (c > nleaf - 1) c = nleaf - 1;
        idx[a] = c;
        // corner of the leaf: rho * c = N c / 2^L, exact; the difference is
        // exact as well (Sterbenz), so the local offset carries no rounding
        local[i * d + a] = x - ldexp((double)N * (double)c, -L);
    }
    keys[i] = morton(idx, d, L);
    vals[i] = (int32_t)i;
}

__global__ void k_validate(const double *__restrict__ pts, int64_t n, double N,
                           int *__restrict__ bad)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double v = pts[i];
    if (!(v >= 0.0 && v <= N)) atomicOr(bad, 1);  // NaN fails both comparisons
}

// ------------------------------------------------------------ sort --------

__global__ __launch_bounds__(kThreads) void k_rs_hist(const uint64_t *__restrict__ keys, int n,
                                                     int shift, uint32_t *__restrict__ hist,
                                                     int ntiles)
{
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    const int base = blockIdx.x * kTile;
    for (int r = 0; r < kItems; ++r) {
        const int i = base + r * kThreads + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[threadIdx.x * ntiles + blockIdx.x] = h[threadIdx.x];
}

// Stable scatter: item r*256 + t of a tile is ranked after every earlier item
// of the tile with the same digit (ballot match within the wavefront, then
// the counts of the earlier wavefronts and rounds).
__global__ __launch_bounds__(kThreads) void k_rs_scatter(const uint64_t *__restrict__ kin,
                                                        const int32_t *__restrict__ vin,
                                                        uint64_t *__restrict__ kout,
                                                        int32_t *__restrict__ vout, int n,
                                                        int shift,
                                                        const uint32_t *__restrict__ offs,
                                                        int ntiles)
{
    __shared__ uint32_t run[256];
    __shared__ uint32_t cnt[kThreads / 64][256];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    run[tid] = offs[tid * ntiles + blockIdx.x];
    const int base = blockIdx.x * kTile;
    const uint64_t below = (1ull << lane) - 1ull;
    for (int r = 0; r < kItems; ++r) {
#pragma unroll
        for (int w = 0; w < kThreads / 64; ++w) cnt[w][tid] = 0;
        __syncthreads();
        const int i = base + r * kThreads + tid;
        const bool act = i < n;
        const uint64_t key = act ? kin[i] : 0ull;
        const int32_t val = act ? vin[i] : 0;
        const uint32_t dig = (uint32_t)((key >> shift) & 255u);
        uint64_t peers = __ballot(act);
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (dig >> b) & 1u;
            const uint64_t m = __ballot(bit);
            peers &= bit ? m : ~m;
        }
        const uint32_t rank = __popcll(peers & below);
        if (act && rank == 0) cnt[wave][dig] = __popcll(peers);
        __syncthreads();
        if (act) {
            uint32_t off = run[dig] + rank;
            for (int w = 0; w < wave; ++w) off += cnt[w][dig];
            kout[off] = key;
            vout[off] = val;
        }
        __syncthreads();
        uint32_t add = 0;
#pragma unroll
        for (int w = 0; w < kThreads / 64; ++w) add += cnt[w][tid];
        run[tid] += add;
        __syncthreads();
    }
}

// ------------------------------------------------------------ unique ------

__global__ void k_flags(const uint64_t *__restrict__ keys, int n, int shift,
                        uint32_t *__restrict__ flags)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    flags[i] = (i == 0 || (keys[i] >> shift) != (keys[i - 1] >> shift)) ? 1u : 0u;
}

__global__ void k_compact(const uint64_t *__restrict__ keys, int n, int shift,
                          const uint32_t *__restrict__ flags, const uint32_t *__restrict__ pos,
                          uint64_t *__restrict__ out_keys, int32_t *__restrict__ out_beg)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (flags[i]) {
        out_keys[pos[i]] = keys[i] >> shift;
        out_beg[pos[i]] = i;
    }
}

__global__ void k_leaf_of(const int32_t *__restrict__ perm, const uint32_t *__restrict__ flags,
                          const uint32_t *__restrict__ pos, int n, int32_t *__restrict__ leaf_of)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    leaf_of[perm[i]] = (int32_t)(pos[i] + flags[i]) - 1;
}

__global__ void k_store_i32(int32_t *p, int32_t v) { *p = v; }

// child-position slots of every box of a level: byte s of slots[b] is the
// offset (from child_beg[b]) of the child at position s, 0xff if absent
__global__ void k_slots(const uint64_t *__restrict__ child_keys, const int32_t *__restrict__ child_beg, int n,
                        int d, uint64_t *__restrict__ slots)
{
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n) return;
    const uint64_t pm = (1ull << d) - 1ull;
    uint64_t w = ~0ull;
    const int j0 = child_beg[b];
    for (int j = j0; j < child_beg[b + 1]; ++j) {
        const int s = (int)(child_keys[j] & pm);
        w &= ~(0xffull << (8 * s));
        w |= (uint64_t)(j - j0) << (8 * s);
    }
    slots[b] = w;
}

// blocks of t threads covering n items; a launch must stay below 2^32
// work-items (a larger one would run only part of its grid)
inline int nblk(int64_t n, int t)
{
    if (n > ((int64_t)1 << 32) - t) throw Error{BFSFT_EINVAL, "a launch would exceed 2^32 work-items"};
    return (int)((n + t - 1) / t);
}

uint32_t read_count(const uint32_t *flags, const uint32_t *pos, int n, hipStream_t s)
{
    if (n == 0) return 0;
    uint32_t a = 0, b = 0;
    BF_HIP(hipMemcpyAsync(&a, flags + n - 1, 4, hipMemcpyDeviceToHost, s));
    BF_HIP(hipMemcpyAsync(&b, pos + n - 1, 4, hipMemcpyDeviceToHost, s));
    BF_HIP(hipStreamSynchronize(s));
    return a + b;
}

}  // namespace

void scan_exclusive_u32(const uint32_t *in, uint32_t *out, int n, hipStream_t s, TempList &tmp)
{
    if (n <= 0) return;
    const int nt = nblk(n, kTile);
    if (nt == 1) {
        k_scan_tiles<<<1, kThreads, 0, s>>>(in, out, n, nullptr);
        BF_HIP(hipGetLastError());
        return;
    }
    uint32_t *sums = (uint32_t *)tmp.alloc(sizeof(uint32_t) * nt);
    uint32_t *sums_scan = (uint32_t *)tmp.alloc(sizeof(uint32_t) * nt);
    k_scan_tiles<<<nt, kThreads, 0, s>>>(in, out, n, sums);
    BF_HIP(hipGetLastError());
    scan_exclusive_u32(sums, sums_scan, nt, s, tmp);
    k_scan_add<<<nt, kThreads, 0, s>>>(out, n, sums_scan);
    BF_HIP(hipGetLastError());
}

int validate_points(const double *pts, int64_t n, int d, int64_t N, Arena &arena, hipStream_t s)
{
    if (n == 0) return 0;
    TempList tmp(arena);
    int *bad = (int *)tmp.alloc(sizeof(int));
    int zero = 0, host = 0;
    BF_HIP(hipMemcpyAsync(bad, &zero, sizeof(int), hipMemcpyHostToDevice, s));
    k_validate<<<nblk(n * d, 256), 256, 0, s>>>(pts, n * d, (double)N, bad);
    BF_HIP(hipGetLastError());
    BF_HIP(hipMemcpyAsync(&host, bad, sizeof(int), hipMemcpyDeviceToHost, s));
    BF_HIP(hipStreamSynchronize(s));
    return host;
}

void build_tree(Tree &t, const double *pts, int64_t n64, int d, int L, int64_t N, Arena &arena,
                hipStream_t s)
{
    t.d = d;
    t.L = L;
    t.npts = n64;
    t.count.assign(L + 1, 0);
    t.keys.assign(L + 1, nullptr);
    t.child_beg.assign(L, nullptr);
    t.slots.assign(L, nullptr);
    t.child_beg_host.assign(L, {});
    if (n64 == 0) return;
    const int n = (int)n64;

    TempList tmp(arena);
    uint64_t *ka = (uint64_t *)tmp.alloc(sizeof(uint64_t) * n);
    uint64_t *kb = (uint64_t *)tmp.alloc(sizeof(uint64_t) * n);
    int32_t *vb = (int32_t *)tmp.alloc(sizeof(int32_t) * n);
    uint32_t *flags = (uint32_t *)tmp.alloc(sizeof(uint32_t) * n);
    uint32_t *pos = (uint32_t *)tmp.alloc(sizeof(uint32_t) * n);
    int32_t *va = (int32_t *)tmp.alloc(sizeof(int32_t) * n);
    t.local = (double *)arena.alloc(sizeof(double) * n * d);
    t.leaf_of = (int32_t *)arena.alloc(sizeof(int32_t) * n);

    k_point_keys<<<nblk(n, 256), 256, 0, s>>>(pts, n, d, L, N, ka, va, t.local);
    BF_HIP(hipGetLastError());

    // LSD radix sort of (key, original index) on the d*L used key bits
    const int ntiles = nblk(n, kTile);
    uint32_t *hist = (uint32_t *)tmp.alloc(sizeof(uint32_t) * 256 * ntiles);
    uint32_t *offs = (uint32_t *)tmp.alloc(sizeof(uint32_t) * 256 * ntiles);
    TempList &scan_tmp = tmp;
    for (int shift = 0; shift < d * L; shift += 8) {
        k_rs_hist<<<ntiles, kThreads, 0, s>>>(ka, n, shift, hist, ntiles);
        BF_HIP(hipGetLastError());
        scan_exclusive_u32(hist, offs, 256 * ntiles, s, scan_tmp);
        k_rs_scatter<<<ntiles, kThreads, 0, s>>>(ka, va, kb, vb, n, shift, offs, ntiles);
        BF_HIP(hipGetLastError());
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    // the sorted permutation must live in the arena
    int32_t *perm = (int32_t *)arena.alloc(sizeof(int32_t) * n);
    BF_HIP(hipMemcpyAsync(perm, va, sizeof(int32_t) * n, hipMemcpyDeviceToDevice, s));
    t.perm = perm;

    // leaves: unique sorted keys, point ranges, leaf of every point
    k_flags<<<nblk(n, 256), 256, 0, s>>>(ka, n, 0, flags);
    BF_HIP(hipGetLastError());
    scan_exclusive_u32(flags, pos, n, s, scan_tmp);
    const int nl = (int)read_count(flags, pos, n, s);
    t.count[L] = nl;
    t.keys[L] = (uint64_t *)arena.alloc(sizeof(uint64_t) * nl);
    t.leaf_beg = (int32_t *)arena.alloc(sizeof(int32_t) * (nl + 1));
    k_compact<<<nblk(n, 256), 256, 0, s>>>(ka, n, 0, flags, pos, t.keys[L], t.leaf_beg);
    k_store_i32<<<1, 1, 0, s>>>(t.leaf_beg + nl, n);
    k_leaf_of<<<nblk(n, 256), 256, 0, s>>>(t.perm, flags, pos, n, t.leaf_of);
    BF_HIP(hipGetLastError());

    // coarser levels: parents are keys >> d of the finer level's boxes
    for (int m = L - 1; m >= 0; --m) {
        const int nc = (int)t.count[m + 1];
        k_flags<<<nblk(nc, 256), 256, 0, s>>>(t.keys[m + 1], nc, d, flags);
        BF_HIP(hipGetLastError());
        scan_exclusive_u32(flags, pos, nc, s, scan_tmp);
        const int np = (int)read_count(flags, pos, nc, s);
        t.count[m] = np;
        t.keys[m] = (uint64_t *)arena.alloc(sizeof(uint64_t) * np);
        t.child_beg[m] = (int32_t *)arena.alloc(sizeof(int32_t) * (np + 1));
        k_compact<<<nblk(nc, 256), 256, 0, s>>>(t.keys[m + 1], nc, d, flags, pos, t.keys[m],
                                               t.child_beg[m]);
        k_store_i32<<<1, 1, 0, s>>>(t.child_beg[m] + np, nc);
        t.slots[m] = (uint64_t *)arena.alloc(sizeof(uint64_t) * np);
        k_slots<<<nblk(np, 256), 256, 0, s>>>(t.keys[m + 1], t.child_beg[m], np, d, t.slots[m]);
        BF_HIP(hipGetLastError());
    }
    for (int m = 0; m < L; ++m) {
        t.child_beg_host[m].resize(t.count[m] + 1);
        BF_HIP(hipMemcpyAsync(t.child_beg_host[m].data(), t.child_beg[m],
                              sizeof(int32_t) * (t.count[m] + 1), hipMemcpyDeviceToHost, s));
    }
    BF_HIP(hipStreamSynchronize(s));
}

}  // namespace bfsft
