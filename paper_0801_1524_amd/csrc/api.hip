// C ABI of bfsft (include/bfsft.h): validation, plan construction and the
// stream-ordered execution of steps 2-4 of Section 2.2 for one transform.
// Batched plans live in batched.hip.
#include "plan.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <fstream>
#include <mutex>
#include <new>
#include <sstream>
#include <string>

namespace bfsft {

// batched.hip
void create_batched(bfsft_plan *B, int count, const bfsft_problem *probs);
void execute_batched(bfsft_plan *B, const double *f, double *u, bool serial);
void release_batched(bfsft_plan *B);
void info_batched(const bfsft_plan *B, bfsft_info *o);

namespace {
thread_local std::string g_last_error;
}

void set_last_error(const std::string &m) { g_last_error = m; }

void *Arena::alloc(size_t n)
{
    if (n == 0) n = 16;
    n = (n + 255) & ~(size_t)255;
    if (cap >= 0 && bytes + (int64_t)n > cap)
        throw Error{BFSFT_ENOMEM, "BFSFT_MAX_DEVICE_BYTES exceeded (" + std::to_string(bytes + n) +
                                      " > " + std::to_string(cap) + ")"};
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, n);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        throw Error{BFSFT_ENOMEM, std::string("hipMalloc(") + std::to_string(n) + "): " + hipGetErrorString(e)};
    }
    ptrs.push_back(p);
    bytes += (int64_t)n;
    return p;
}

void Arena::release()
{
    for (void *p : ptrs) (void)hipFree(p);
    ptrs.clear();
    bytes = 0;
}

void *Arena::alloc_temp(size_t n)
{
    if (n == 0) n = 16;
    n = (n + 255) & ~(size_t)255;
    if (cap >= 0 && bytes + temp_bytes + (int64_t)n > cap)
        throw Error{BFSFT_ENOMEM, "BFSFT_MAX_DEVICE_BYTES exceeded by plan-time temporaries (" +
                                      std::to_string(bytes + temp_bytes + n) + " > " + std::to_string(cap) + ")"};
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, n);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        throw Error{BFSFT_ENOMEM, std::string("hipMalloc(") + std::to_string(n) + "): " + hipGetErrorString(e)};
    }
    temp_bytes += (int64_t)n;
    return p;
}

void Arena::free_temp(void *p, size_t n)
{
    if (n == 0) n = 16;
    n = (n + 255) & ~(size_t)255;
    (void)hipFree(p);
    temp_bytes -= (int64_t)n;
}

void *TempList::alloc(size_t n)
{
    void *q = arena.alloc_temp(n);
    p.emplace_back(q, n);
    return q;
}

TempList::~TempList()
{
    for (auto &e : p) arena.free_temp(e.first, e.second);
}

int ceil_log2(int64_t N)
{
    int L = 0;
    while (((int64_t)1 << L) < N) ++L;
    return L;
}

int64_t env_cap()
{
    const char *s = std::getenv("BFSFT_MAX_DEVICE_BYTES");
    if (!s || !*s) return -1;
    char *end = nullptr;
    long long v = std::strtoll(s, &end, 10);
    return v < 0 ? -1 : (int64_t)v;
}

Launch launch_of(const bfsft_plan *P)
{
    Launch c;
    c.d = P->d;
    c.p = P->p;
    c.precision = P->precision;
    c.tb = &P->tb;
    c.stream = P->stream;
    return c;
}

// Arguments of the translation producing T_K level l (rows a' at T_X level
// L-l-1, outputs at T_X level L-l).
LevelArgs level_args(const bfsft_plan *P, int l, const void *in, void *out)
{
    const int L = P->L;
    LevelArgs a;
    a.in = in;
    a.out = out;
    a.in_row = P->tk.count[l + 1];
    a.out_row = P->tk.count[l];
    a.x_cb = P->tx.child_beg[L - l - 1];
    a.k_cb = P->tk.child_beg[l];
    a.x_slot = P->tx.slots[L - l - 1];
    a.k_slot = P->tk.slots[l];
    a.tiles = P->tiles[l];
    a.ntile = P->ntile[l];
    a.cost_max = P->cost_max[l];
    a.rows = P->rows[l];
    a.kind = P->kind.empty() ? 0 : P->kind[l];
    a.nap = P->tx.count[L - l - 1];
    a.sig = P->sig[L - l - 1];
    return a;
}

namespace {

// Tiles of T_K level l: ranges [b0, b1) whose LDS cost (translate_tile_cost
// of their children count and size) is at most `cap`, with at most 120
// children; a single box always fits, so every tile is non-empty.  A tile
// record is (b0, b1, cb[b0], cb[b1]): the children range comes with it.
std::vector<int4> make_tiles(const std::vector<int32_t> &cb, int d, int p, int precision, int cap, int kind)
{
    std::vector<int4> t;
    const int n = (int)cb.size() - 1;
    if (kind == 1) cap -= 1;  // the zero block of the matrix-core kernel
    int b0 = 0;
    while (b0 < n) {
        int b1 = b0 + 1;
        while (b1 < n && cb[b1 + 1] - cb[b0] <= 120 &&
               translate_tile_cost(d, p, precision, cb[b1 + 1] - cb[b0], b1 + 1 - b0, kind) <= cap)
            ++b1;
        t.push_back(make_int4(b0, b1, cb[b0], cb[b1]));
        b0 = b1;
    }
    return t;
}

template <typename F> int guarded(F &&f)
{
    try {
        f();
        return BFSFT_OK;
    } catch (const Error &e) {
        set_last_error(e.msg);
        return e.status;
    } catch (const std::bad_alloc &) {
        set_last_error("host allocation failed");
        return BFSFT_ENOMEM;
    } catch (...) {
        set_last_error("unexpected exception");
        return BFSFT_EDEVICE;
    }
}

void check_scalars(int d, int64_t N, int p, int precision, int64_t nx, int64_t nk, const void *x,
                   const void *k)
{
    if (d != 2 && d != 3) throw Error{BFSFT_EINVAL, "d must be 2 or 3"};
    if (precision != BFSFT_FP64 && precision != BFSFT_MIXED && precision != BFSFT_FP32 &&
        !split_precision(precision))
        throw Error{BFSFT_EINVAL, "unknown precision"};
    if (split_precision(precision) && d != 2)
        throw Error{BFSFT_EINVAL, "the FP16X2 and BF16X3 contraction formats are 2D only"};
    const int pmax = d == 2 ? 12 : 8;
    if (p < 3 || p > pmax)
        throw Error{BFSFT_EINVAL, "p must be in [3, " + std::to_string(pmax) + "] for d = " + std::to_string(d)};
    const int64_t nmax = d == 2 ? ((int64_t)1 << 24) : ((int64_t)1 << 16);
    if (N < 2 || N > nmax) throw Error{BFSFT_EINVAL, "N out of range"};
    if (nx < 0 || nk < 0) throw Error{BFSFT_EINVAL, "negative point count"};
    if (nx > INT32_MAX / 4 || nk > INT32_MAX / 4) throw Error{BFSFT_EINVAL, "too many points"};
    if ((nx > 0 && !x) || (nk > 0 && !k)) throw Error{BFSFT_EINVAL, "NULL point array"};
    if (!translate_fits(d, p, precision))
        throw Error{BFSFT_EINVAL, "p too large for d = 3 at this precision (LDS)"};
}

void init_plan(bfsft_plan *P, int d, int64_t N, int p, int precision, int64_t nx, int64_t nk,
               hipStream_t stream)
{
    P->d = d;
    P->p = p;
    P->precision = precision;
    P->N = N;
    P->nx = nx;
    P->nk = nk;
    P->L = ceil_log2(N);
    P->rho = std::ldexp((double)N, -P->L);
    P->PD = d == 2 ? p * p : p * p * p;
    P->stream = stream;
    P->state_size = precision == BFSFT_FP64 ? 16 : 8;
    P->arena.cap = env_cap();
}

const char *prec_name(int precision)
{
    switch (precision) {
    case BFSFT_FP64: return "fp64";
    case BFSFT_FP32: return "fp32";
    case BFSFT_FP16X2: return "fp16x2";
    case BFSFT_BF16X3: return "bf16x3";
    default: return "mixed";
    }
}

size_t state_bytes(const bfsft_plan *P)
{
    size_t m = 0;
    for (int l = 0; l <= P->L; ++l)
        m = std::max(m, (size_t)P->tx.count[P->L - l] * (size_t)P->tk.count[l]);
    return m * P->PD * P->state_size;
}

// Time one sweep of a single plan level by level, eagerly: ms[l] is the
// best of `reps` runs (after one warm-up) of the launch producing T_K level l.
std::vector<double> time_levels(bfsft_plan *P, int reps)
{
    const Launch c = launch_of(P);
    const int L = P->L;
    std::vector<hipEvent_t> ev(L + 1);
    for (auto &e : ev) BF_HIP(hipEventCreate(&e));
    std::vector<double> best(L, 1e30);
    for (int r = 0; r < reps + 1; ++r) {
        BF_HIP(hipEventRecord(ev[0], P->stream));
        int cur = 0;
        for (int l = L - 1; l >= 0; --l) {
            launch_translate(c, level_args(P, l, P->buf[cur], P->buf[cur ^ 1]));
            BF_HIP(hipEventRecord(ev[L - l], P->stream));
            cur ^= 1;
        }
        BF_HIP(hipEventSynchronize(ev[L]));
        if (r == 0) continue;
        for (int i = 0; i < L; ++i) {
            float ms = 0.f;
            BF_HIP(hipEventElapsedTime(&ms, ev[i], ev[i + 1]));
            const int l = L - 1 - i;
            best[l] = std::min(best[l], (double)ms);
        }
    }
    for (auto &e : ev) (void)hipEventDestroy(e);
    return best;
}

// Kernels the tuner may use for this plan: bit k allows kind k (0 the VALU
// kernel, 1 the FP64 matrix-core kernel, 2 stage 1 on the matrix cores in
// the precision's contraction format).  The split formats have only kind 2;
// otherwise BFSFT_TRANSLATE=valu, =mfma or =xdl restricts the choice to one
// kind where the plan allows it.  Members of a batched plan use the VALU
// kernel (kind 2 for the split formats).
int kernel_choices(const bfsft_plan *P)
{
    if (split_precision(P->precision)) return 4;
    int m = 1;
    if (!P->valu_only && translate_mfma_supported(P->d, P->p, P->precision)) m |= 2;
    if (!P->valu_only && translate_xdl_supported(P->d, P->p, P->precision)) m |= 4;
    if (const char *s = std::getenv("BFSFT_TRANSLATE")) {
        if (std::strcmp(s, "valu") == 0) m &= 1;
        else if (std::strcmp(s, "mfma") == 0 && (m & 2)) m = 2;
        else if (std::strcmp(s, "xdl") == 0 && (m & 4)) m = 4;
    }
    return m;
}

// the kind of a single choice (untuned plans): the lowest allowed
int first_kind(int choices) { return (choices & 1) ? 0 : (choices & 2) ? 1 : 2; }

// Choose the kernel and the tile LDS budget of every level of a single plan
// by timing the sweep on the plan's own shapes.  Neither changes what is
// computed, only the order of the floating-point operations inside an
// output and the speed.  Cached per (architecture, d, p, precision, L,
// allowed kernels).
void autotune_single(bfsft_plan *P)
{
    const int choices = kernel_choices(P);
    const std::string key = "single5/d" + std::to_string(P->d) + "/p" + std::to_string(P->p) + "/" +
                            prec_name(P->precision) + "/L" + std::to_string(P->L) + "/k" +
                            std::to_string(choices);
    std::vector<int> v;
    if (tune_lookup(key, v) && (int)v.size() == P->L) {
        std::vector<int> b(P->L), k(P->L);
        for (int l = 0; l < P->L; ++l) {
            k[l] = v[l] / 100;
            b[l] = (v[l] % 100) * 1024;
        }
        build_tiles_levels(P, b, k);
        return;
    }
    // clear the state once (a plan-time fill, never captured) so the timed
    // arithmetic runs on finite values
    const size_t bytes = state_bytes(P);
    BF_HIP(hipMemsetAsync(P->buf[0], 0, bytes, P->stream));
    BF_HIP(hipMemsetAsync(P->buf[1], 0, bytes, P->stream));
    // budgets a few KB apart: the threads a tile fills depend on them finely;
    // 2D also tries tiles of two work-groups per CU (kLdsMax2D)
    std::vector<int> cand = {8, 12, 16, 20, 24, 28, 30, 32, 34, 36, 38, 40, 44, 48, 54, 60};
    if (P->d == 2) cand.insert(cand.end(), {66, 72, 76});
    std::vector<double> best(P->L, 1e30);
    std::vector<int> pick(P->L, 32), pk(P->L, first_kind(choices));
    for (int kind = 0; kind < 3; ++kind) {
        if (!(choices & (1 << kind))) continue;
        for (int kb : cand) {
            build_tiles_levels(P, std::vector<int>(P->L, kb * 1024), std::vector<int>(P->L, kind));
            const std::vector<double> ms = time_levels(P, 3);
            for (int l = 0; l < P->L; ++l)
                if (ms[l] < best[l]) {
                    best[l] = ms[l];
                    pick[l] = kb;
                    pk[l] = kind;
                }
        }
    }
    std::vector<int> b(P->L), store(P->L);
    for (int l = 0; l < P->L; ++l) {
        b[l] = pick[l] * 1024;
        store[l] = pk[l] * 100 + pick[l];
    }
    build_tiles_levels(P, b, pk);
    tune_store(key, store);
}

// Steps 2-4 for sources f into u.  The two state buffers are the plan's own
// unless `bufs` names others (each at least state_bytes(P)).
void run(bfsft_plan *P, const double *f, double *u, int probe_level, double *pot, void *const *bufs = nullptr)
{
    void *const B[2] = {bufs ? bufs[0] : P->buf[0], bufs ? bufs[1] : P->buf[1]};
    if (P->nx == 0) return;
    if (P->nk == 0) {
        launch_zero_c128(u, P->nx, P->stream);
        return;
    }
    const Launch c = launch_of(P);
    const int L = P->L;
    hipEvent_t *ev = nullptr;
    if (P->tcount < P->tmax) ev = &P->tev[(size_t)P->tcount++ * (L + 3)];
    const int s0 = P->start.s0, l0 = L - s0;
    if (ev) BF_HIP(hipEventRecord(ev[0], P->stream));
    if (s0 == 0)
        launch_leaf(c, f, P->tk, P->rho, B[0]);
    else
        launch_direct(c, P->start, f, P->tx, P->tk, P->N, B[0]);
    if (ev) BF_HIP(hipEventRecord(ev[1], P->stream));
    if (probe_level == l0)
        launch_export(c, B[0], P->tx.keys[s0], P->tx.count[s0], P->tk.keys[l0], P->tk.count[l0], l0, L,
                      P->N, pot);
    // levels above the start have no translation and record no event (each
    // event between two launches delays the next by a few microseconds);
    // bfsft_timing_end reports zero for them
    int cur = 0;
    for (int l = l0 - 1; l >= 0; --l) {
        launch_translate(c, level_args(P, l, B[cur], B[cur ^ 1]));
        if (ev) BF_HIP(hipEventRecord(ev[2 + (L - 1 - l)], P->stream));
        cur ^= 1;
        if (probe_level == l)
            launch_export(c, B[cur], P->tx.keys[L - l], P->tx.count[L - l], P->tk.keys[l],
                          P->tk.count[l], l, L, P->N, pot);
    }
    launch_final(c, B[cur], P->tx, P->rho, P->nx, u);
    if (ev) BF_HIP(hipEventRecord(ev[L + 2], P->stream));
}

// ------------------------------------------------ no-allocation execute --
// Scratch of bfsft_execute_noalloc: the sweep's two state buffers, in a
// static device array the library holds on every GPU it runs on until the
// process ends.  In host code `scratch` names a host-side stand-in, not the
// device memory: its device address is taken once per device with
// hipGetSymbolAddress (with that device current) and only that address is
// handed to kernels.
constexpr size_t kScratchBytes = (size_t)64 << 20;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch[kMaxDevices] = {};

// device address of `scratch` on the current device
void *scratch_ptr()
{
    int dev = 0;
    BF_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) throw Error{BFSFT_EDEVICE, "device index beyond the scratch table"};
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            throw Error{BFSFT_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e)};
        g_scratch[dev] = ptr;
    }
    return g_scratch[dev];
}

void free_events(bfsft_plan *P)
{
    for (hipEvent_t e : P->tev) (void)hipEventDestroy(e);
    P->tev.clear();
    P->tmax = P->tcount = 0;
}

}  // namespace

// Tiles, rows per work-group and LDS cost of every level for per-level tile
// budgets (bytes).
void build_tiles_levels(bfsft_plan *P, const std::vector<int> &lds_bytes, const std::vector<int> &kinds)
{
    P->lds_level = lds_bytes;
    P->kind = kinds.empty() ? std::vector<int>(P->L, 0) : kinds;
    P->lds = lds_bytes.empty() ? translate_default_lds(P->d) : lds_bytes[0];
    P->tiles.assign(P->L, nullptr);
    P->ntile.assign(P->L, 0);
    P->cost_max.assign(P->L, 0);
    P->rows.assign(P->L, 1);
    if (P->nx == 0 || P->nk == 0) return;
    std::vector<int4> all;
    std::vector<size_t> off(P->L);
    for (int l = 0; l < P->L; ++l) {
        const int cap = translate_cap_blocks(P->d, P->p, P->precision, lds_bytes[l]);
        const std::vector<int32_t> &cb = P->tk.child_beg_host[l];
        const int kind = P->kind[l];
        std::vector<int4> t = make_tiles(cb, P->d, P->p, P->precision, cap, kind);
        off[l] = all.size();
        P->ntile[l] = (int)t.size();
        for (const int4 &b : t)
            P->cost_max[l] =
                std::max(P->cost_max[l], translate_tile_cost(P->d, P->p, P->precision, cb[b.y] - cb[b.x], b.y - b.x, kind));
        P->rows[l] = translate_rows(cap, P->cost_max[l], P->tx.count[P->L - l - 1], kind);
        all.insert(all.end(), t.begin(), t.end());
    }
    int4 *dev = (int4 *)P->arena.alloc(sizeof(int4) * all.size());
    BF_HIP(hipMemcpyAsync(dev, all.data(), sizeof(int4) * all.size(), hipMemcpyHostToDevice, P->stream));
    BF_HIP(hipStreamSynchronize(P->stream));  // `all` is a host temporary
    for (int l = 0; l < P->L; ++l) P->tiles[l] = dev + off[l];
}

void build_tiles(bfsft_plan *P, int lds_bytes)
{
    // untuned: the VALU kernel unless the precision or BFSFT_TRANSLATE asks
    // for another
    const int kind = first_kind(kernel_choices(P));
    build_tiles_levels(P, std::vector<int>(P->L, lds_bytes), std::vector<int>(P->L, kind));
}

// Start level of the sweep (the number of T_K levels above the leaves at
// which potentials are summed directly), chosen from the tree counts alone so
// that it never depends on timing: the s0 that minimises a cost model (ns on
// one MI355X, constants fitted to the kernels' measured times)
//   direct sums at level L - s0:  0.0066 (1 + 0.15 (d - 2)) per pair, source and
//                                 line of p^(d-1),
//   translations below it:        (d = 2: 6.4e-4, d = 3: 1.54e-3) p^(d+1) per pair,
//   leaf initialisation (s0 = 0): 5.7e-3 per source and grid point.
// A start above the leaves is taken only if it saves at least 3 % of the
// modelled time.  BFSFT_START_LEVEL=n forces n (clamped to [0, min(L, kStartMax)]).
// Start level and direct-sum kernel from a cost model of the measured
// kernel times (ns): translations per output pair, VALU direct sums per
// (pair, source, grid line), matrix-core direct sums per padded complex
// multiply-add on the busiest SIMD (about 45 ns per FP64 MFMA with two
// consumer waves per SIMD, a third more with one) plus the producers' work
// per step (which the SIMD does not overlap with the products; far less with
// the plan-time tables of the point-only factors).  The
// matrix-core kernel is taken in 3D and where at least 5 row tiles give two
// consumer waves per SIMD; BFSFT_DIRECT restricts the choice.
StartChoice choose_start(const bfsft_plan *P)
{
    StartChoice c;
    if (P->nx == 0 || P->nk == 0) return c;
    const int L = P->L, d = P->d;
    // a transform of a batched plan: its direct sums run in the batched
    // graph's VALU launch
    const int kinds = P->valu_only ? 1 : direct_kinds(d, P->p);
    int dev = 0, ncu = 0;
    BF_HIP(hipGetDevice(&dev));
    BF_HIP(hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev));
    ncu = std::max(1, ncu);
    const double p = P->p;
    const double lines = d == 2 ? p : p * p;
    auto pairs = [&](int l) { return (double)P->tx.count[L - l] * (double)P->tk.count[l]; };
    const double tr = (d == 2 ? 6.4e-4 : 1.54e-3) * std::pow(p, d + 1);
    const double dr = 0.0066 * (1.0 + 0.15 * (d - 2));
    const int pd = d == 2 ? P->p * P->p : P->p * P->p * P->p;
    const int nt = (pd % 16 == 1 && pd > 16) ? pd / 16 : (pd + 15) / 16;  // the kernel's column tiles
    const int maxc = nt <= 6 ? 8 : 4;
    auto direct_cost = [&](int l0, int s, int kind) {
        const double nk = (double)P->nk, nB = (double)P->tk.count[l0], nA = (double)P->tx.count[s];
        if (kind == 0) return dr * pairs(l0) * (nk / nB) * lines;
        const double tiles = std::ceil(nA / 16.0);
        const double w = std::min<double>(maxc, tiles);
        const double full = std::floor(tiles / w), rem = tiles - full * w;
        const double simd_rows = 16.0 * (full * std::ceil(w / 4.0) + std::ceil(rem / 4.0));
        const double blocks = std::ceil(tiles / w);
        const double load = simd_rows * (nk + 1.5 * nB) * 16.0 * nt;  // complex multiply-adds
        const double steps = blocks * (nk / 16.0 + 0.5 * nB);
        const double t_mfma = 45.0 * (d == 2 && w <= 4 ? 1.33 : 1.0);
        // the producers' work per step: loads and stores with the plan-time
        // tables, the phases and chains without them
        const double table_bytes = (nA * nk + nk * pd) * 16.0;
        const bool tables = table_bytes <= (double)direct_table_budget() &&
                            (P->arena.cap < 0 || (double)P->arena.bytes + table_bytes <= (double)P->arena.cap);
        const double per_step = tables ? 200.0 * w + 300.0 : 450.0 * w + 300.0;
        return t_mfma * load / (256.0 * ncu) + steps / ncu * per_step;
    };
    // the kernel at start level s: in 2D the matrix cores from 5 row tiles
    // on (with fewer, one consumer wave per SIMD, the VALU kernel measures
    // faster); in 3D the cheaper of the two in the model
    auto kind_at = [&](int s) {
        if (!(kinds & 2)) return 0;
        if (!(kinds & 1)) return 1;
        if (d == 2) return P->tx.count[s] > 64 ? 1 : 0;
        return direct_cost(L - s, s, 1) < direct_cost(L - s, s, 0) ? 1 : 0;
    };
    if (const char *e = std::getenv("BFSFT_START_LEVEL")) {
        char *end = nullptr;
        const long v = std::strtol(e, &end, 10);
        if (end != e) {
            c.s0 = (int)std::max(0L, std::min((long)std::min(L, kStartMax), v));
            c.kind = c.s0 > 0 ? kind_at(c.s0) : 0;
            return c;
        }
    }
    std::vector<double> below(L + 1, 0.0);  // below[l0]: translations producing levels < l0
    for (int l = 1; l <= L; ++l) below[l] = below[l - 1] + tr * pairs(l - 1);
    const double leaf_cost = 5.7e-3 * (double)P->nk * std::pow(p, d) + below[L];
    double best_cost = leaf_cost;
    for (int s = 1; s <= std::min(L, kStartMax); ++s) {
        const int l0 = L - s, kind = kind_at(s);
        const double cost = direct_cost(l0, s, kind) + below[l0];
        if (cost < best_cost) {
            best_cost = cost;
            c.s0 = s;
            c.kind = kind;
        }
    }
    // the leaf start of the paper unless the model predicts a clear gain
    // (it is within a few per cent of the measured times)
    if (!(best_cost < 0.97 * leaf_cost)) c = StartChoice{};
    return c;
}

void build_plan(bfsft_plan *P, const double *x, const double *k)
{
    hipStream_t s = P->stream;
    if (validate_points(x, P->nx, P->d, P->N, P->arena, s) || validate_points(k, P->nk, P->d, P->N, P->arena, s))
        throw Error{BFSFT_EDOMAIN, "a coordinate is not finite or lies outside [0, N]"};
    build_tree(P->tx, x, P->nx, P->d, P->L, P->N, P->arena, s);
    build_tree(P->tk, k, P->nk, P->d, P->L, P->N, P->arena, s);
    build_tables(P->tb, P->p, P->N, P->L, P->arena, s);
    P->sig.assign(P->L, nullptr);
    if (P->nx == 0 || P->nk == 0) {
        build_tiles(P, translate_default_lds(P->d));
        BF_HIP(hipStreamSynchronize(s));
        return;
    }
    if (P->rho != 1.0) {
        for (int m = 0; m < P->L; ++m) {
            P->sig[m] = (double *)P->arena.alloc(sizeof(double) * 2 * P->d * P->tx.count[m]);
            launch_sigma(P->tx.keys[m], P->tx.count[m], P->d, m, P->L, P->N, P->sig[m], s);
        }
    }
    const size_t bytes = state_bytes(P);
    P->buf[0] = P->arena.alloc(bytes);
    P->buf[1] = P->arena.alloc(bytes);
    const StartChoice sc = choose_start(P);
    P->start.kind = sc.kind;
    build_start(P->start, P->tk, sc.s0, P->d, P->p - 1, P->rho, P->arena, s);
    if (P->start.kind == 1 && P->start.s0 > 0)
        build_direct_steps(P->start, P->tx, P->tk, P->tb, P->d, P->p, P->N, P->arena, s);
    build_tiles(P, translate_default_lds(P->d));
    BF_HIP(hipStreamSynchronize(s));
}

void release_plan(bfsft_plan *P)
{
    (void)hipStreamSynchronize(P->stream);
    if (P->adj) {
        release_plan(P->adj);  // its trees and tables belong to P
        delete P->adj;
        P->adj = nullptr;
    }
    free_events(P);
    P->arena.release();
}

// The adjoint of a single plan: the same trees with the roles of x and k
// exchanged (T_X of the adjoint is P's T_K and vice versa) and the same
// tables; its own sigma tables, tiles, start level and input staging.  Its
// pairs at level l are P's pairs at level L - l, so its largest level has
// P's size: it shares P's two state buffers (executes on one plan are
// stream-ordered, never concurrent).  Built with the plan, so no execute
// call allocates.
bfsft_plan *make_adjoint(bfsft_plan *P)
{
    bfsft_plan *A = new bfsft_plan();
    try {
        init_plan(A, P->d, P->N, P->p, P->precision, P->nk, P->nx, P->stream);
        A->arena.cap = P->arena.cap < 0 ? -1 : std::max<int64_t>(0, P->arena.cap - P->arena.bytes);
        A->tx = P->tk;
        A->tk = P->tx;
        A->tb = P->tb;
        A->sig.assign(A->L, nullptr);
        A->adj_in = (double *)A->arena.alloc(sizeof(double) * 2 * std::max<int64_t>(1, A->nk));
        if (A->nx > 0 && A->nk > 0) {
            if (A->rho != 1.0)
                for (int m = 0; m < A->L; ++m) {
                    A->sig[m] = (double *)A->arena.alloc(sizeof(double) * 2 * A->d * A->tx.count[m]);
                    launch_sigma(A->tx.keys[m], A->tx.count[m], A->d, m, A->L, A->N, A->sig[m], A->stream);
                }
            if (state_bytes(A) > state_bytes(P)) throw Error{BFSFT_EDEVICE, "adjoint state larger than the plan's"};
            A->buf[0] = P->buf[0];
            A->buf[1] = P->buf[1];
            const StartChoice sc = choose_start(A);
            A->start.kind = sc.kind;
            build_start(A->start, A->tk, sc.s0, A->d, A->p - 1, A->rho, A->arena, A->stream);
            if (A->start.kind == 1 && A->start.s0 > 0)
                build_direct_steps(A->start, A->tx, A->tk, A->tb, A->d, A->p, A->N, A->arena, A->stream);
        }
        build_tiles(A, translate_default_lds(A->d));
        if (A->nx > 0 && A->nk > 0 && autotune_enabled()) autotune_single(A);
        BF_HIP(hipStreamSynchronize(A->stream));
    } catch (...) {
        (void)hipStreamSynchronize(A->stream);
        A->arena.release();
        delete A;
        throw;
    }
    return A;
}

void run_single(bfsft_plan *P, const double *f, double *u) { run(P, f, u, -1, nullptr); }

// ------------------------------------------------------------ tuning cache --

bool autotune_enabled()
{
    const char *s = std::getenv("BFSFT_AUTOTUNE");
    return !(s && s[0] == '0');
}

namespace {
std::string tune_path()
{
    if (const char *s = std::getenv("BFSFT_TUNE_CACHE")) return s;
    if (const char *h = std::getenv("HOME")) return std::string(h) + "/.cache/bfsft_tune.txt";
    return "";
}

std::string arch_tag()
{
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "gpu";
    std::string a = prop.gcnArchName;
    return a.substr(0, a.find(':'));
}
}  // namespace

bool tune_lookup(const std::string &key, std::vector<int> &vals)
{
    const std::string path = tune_path();
    if (path.empty()) return false;
    std::ifstream in(path);
    std::string line;
    const std::string full = arch_tag() + "/" + key;
    bool found = false;
    while (std::getline(in, line)) {  // the last entry for a key wins
        std::istringstream ss(line);
        std::string k;
        ss >> k;
        if (k != full) continue;
        std::vector<int> v;
        int x;
        while (ss >> x) v.push_back(x);
        if (!v.empty()) {
            vals = v;
            found = true;
        }
    }
    return found;
}

void tune_store(const std::string &key, const std::vector<int> &vals)
{
    const std::string path = tune_path();
    if (path.empty()) return;
    std::ofstream out(path, std::ios::app);
    if (!out) return;  // read-only or missing directory: tuning is simply not cached
    out << arch_tag() << "/" << key;
    for (int v : vals) out << " " << v;
    out << "\n";
}

}  // namespace bfsft

using namespace bfsft;

extern "C" {

const char *bfsft_strerror(int status)
{
    switch (status) {
    case BFSFT_OK: return "success";
    case BFSFT_EINVAL: return "invalid argument";
    case BFSFT_EDOMAIN: return "point outside [0, N]^d or not finite";
    case BFSFT_ENOMEM: return "out of device memory";
    case BFSFT_EDEVICE: return "HIP runtime error";
    default: return "unknown status";
    }
}

const char *bfsft_last_error(void) { return g_last_error.c_str(); }

int bfsft_plan_create(bfsft_plan **out, int d, int64_t N, int p, int precision, const double *x,
                      int64_t nx, const double *k, int64_t nk, void *stream)
{
    if (!out) {
        set_last_error("out is NULL");
        return BFSFT_EINVAL;
    }
    *out = nullptr;
    bfsft_plan *P = nullptr;
    int rc = guarded([&] {
        check_scalars(d, N, p, precision, nx, nk, x, k);
        P = new bfsft_plan();
        init_plan(P, d, N, p, precision, nx, nk, (hipStream_t)stream);
        build_plan(P, x, k);
        if (nx > 0 && nk > 0 && autotune_enabled()) autotune_single(P);
        P->adj = make_adjoint(P);
        BF_HIP(hipStreamSynchronize(P->stream));
    });
    if (rc != BFSFT_OK) {
        if (P) {
            release_plan(P);
            delete P;
        }
        return rc;
    }
    *out = P;
    return BFSFT_OK;
}

int bfsft_execute(bfsft_plan *plan, const double *f, double *u)
{
    return guarded([&] {
        if (!plan) throw Error{BFSFT_EINVAL, "plan is NULL"};
        if (plan->batched) throw Error{BFSFT_EINVAL, "batched plan: use bfsft_execute_batched"};
        if ((plan->nk > 0 && !f) || (plan->nx > 0 && !u)) throw Error{BFSFT_EINVAL, "NULL f or u"};
        if (plan->nx > 0 && plan->nk > 0 && (const void *)f == (const void *)u)
            throw Error{BFSFT_EINVAL, "u aliases f"};
        run(plan, f, u, -1, nullptr);
    });
}

int bfsft_execute_noalloc(bfsft_plan *plan, const double *f, double *u)
{
    return guarded([&] {
        if (!plan) throw Error{BFSFT_EINVAL, "plan is NULL"};
        if (plan->batched) throw Error{BFSFT_EINVAL, "batched plan: use bfsft_execute_batched"};
        if ((plan->nk > 0 && !f) || (plan->nx > 0 && !u)) throw Error{BFSFT_EINVAL, "NULL f or u"};
        if (plan->nx > 0 && plan->nk > 0 && (const void *)f == (const void *)u)
            throw Error{BFSFT_EINVAL, "u aliases f"};
        if (plan->nx == 0 || plan->nk == 0) {  // no state: the plain execute allocates nothing either
            run(plan, f, u, -1, nullptr);
            return;
        }
        const size_t one = (state_bytes(plan) + 255) & ~(size_t)255;
        if (2 * one > kScratchBytes)
            throw Error{BFSFT_EINVAL, "the plan's state (2 x " + std::to_string(one) +
                                          " bytes) exceeds the no-allocation scratch (" +
                                          std::to_string(kScratchBytes) + " bytes)"};
        unsigned char *base = static_cast<unsigned char *>(scratch_ptr());
        void *const bufs[2] = {base, base + one};
        run(plan, f, u, -1, nullptr, bufs);
    });
}

int bfsft_execute_adjoint(bfsft_plan *plan, const double *g, double *v)
{
    return guarded([&] {
        if (!plan) throw Error{BFSFT_EINVAL, "plan is NULL"};
        if (plan->batched) throw Error{BFSFT_EINVAL, "batched plans have no adjoint"};
        if ((plan->nx > 0 && !g) || (plan->nk > 0 && !v)) throw Error{BFSFT_EINVAL, "NULL g or v"};
        if (plan->nx > 0 && plan->nk > 0 && (const void *)g == (const void *)v)
            throw Error{BFSFT_EINVAL, "v aliases g"};
        if (plan->nk == 0) return;
        bfsft_plan *A = plan->adj;  // built with the plan
        if (!A) throw Error{BFSFT_EINVAL, "plan has no adjoint"};
        launch_conj(g, A->adj_in, plan->nx, plan->stream);
        run(A, A->adj_in, v, -1, nullptr);
        launch_conj(v, v, plan->nk, plan->stream);
    });
}

int bfsft_execute_probe(bfsft_plan *plan, const double *f, double *u, int level, double *pot)
{
    return guarded([&] {
        if (!plan || plan->batched) throw Error{BFSFT_EINVAL, "plan is NULL or batched"};
        if (level < 0 || level > plan->L - plan->start.s0)
            throw Error{BFSFT_EINVAL, "level out of range (above the start level there are no potentials)"};
        if (!pot || !f || !u) throw Error{BFSFT_EINVAL, "NULL pointer"};
        if (plan->nx == 0 || plan->nk == 0) throw Error{BFSFT_EINVAL, "empty plan has no levels"};
        run(plan, f, u, level, pot);
    });
}

int bfsft_timing_begin(bfsft_plan *P, int max_execs)
{
    return guarded([&] {
        if (!P || P->batched || max_execs < 1) throw Error{BFSFT_EINVAL, "bad timing request"};
        free_events(P);
        P->tev.resize((size_t)max_execs * (P->L + 3));
        for (auto &e : P->tev) BF_HIP(hipEventCreate(&e));
        P->tmax = max_execs;
    });
}

int bfsft_timing_end(bfsft_plan *P, double *out, int n)
{
    return guarded([&] {
        if (!P || P->batched || !out || n < 3 + P->L) throw Error{BFSFT_EINVAL, "bad timing output"};
        const int L = P->L;
        for (int i = 0; i < n; ++i) out[i] = 0.0;
        out[0] = P->tcount;
        // events: 0 start, 1 after the leaf or direct sums, 2 + (L - 1 - l)
        // after translation level l (only l < l0, the translated levels),
        // L + 2 after the final evaluation
        const int l0 = L - P->start.s0;
        for (int r = 0; r < P->tcount; ++r) {
            hipEvent_t *ev = &P->tev[(size_t)r * (L + 3)];
            BF_HIP(hipEventSynchronize(ev[L + 2]));
            float ms = 0.f;
            BF_HIP(hipEventElapsedTime(&ms, ev[0], ev[1]));
            out[1] += ms;
            BF_HIP(hipEventElapsedTime(&ms, l0 > 0 ? ev[L + 1] : ev[1], ev[L + 2]));
            out[2] += ms;
            for (int l = l0 - 1; l >= 0; --l) {
                const hipEvent_t before = l == l0 - 1 ? ev[1] : ev[2 + (L - 1 - (l + 1))];
                BF_HIP(hipEventElapsedTime(&ms, before, ev[2 + (L - 1 - l)]));
                out[3 + l] += ms;
            }
        }
        free_events(P);
    });
}

void bfsft_destroy(bfsft_plan *plan)
{
    if (!plan) return;
    if (plan->batched)
        release_batched(plan);
    else
        release_plan(plan);
    delete plan;
}

int bfsft_plan_info(const bfsft_plan *P, bfsft_info *o)
{
    return guarded([&] {
        if (!P || !o) throw Error{BFSFT_EINVAL, "NULL argument"};
        std::memset(o, 0, sizeof(*o));
        if (P->batched) {
            info_batched(P, o);
            return;
        }
        o->d = P->d;
        o->p = P->p;
        o->precision = P->precision;
        o->levels = P->L;
        o->N = P->N;
        o->nx = P->nx;
        o->nk = P->nk;
        o->rho = P->rho;
        o->transforms = 1;
        o->device_bytes = P->arena.bytes + (P->adj ? P->adj->arena.bytes : 0);
        o->lds_kb = P->lds / 1024;
        o->start_level = P->start.s0;
        o->start_kernel = P->start.s0 > 0 ? P->start.kind : 0;
        o->start_tables = P->start.s0 > 0 && P->start.gam ? 1 : 0;
        for (int l = 0; l < P->L && l < (int)P->kind.size(); ++l) {
            o->level_kernel[l] = P->kind[l];
            o->level_lds_kb[l] = P->lds_level[l] / 1024;
        }
        if (P->nx == 0 || P->nk == 0) return;
        for (int m = 0; m <= P->L; ++m) {
            o->x_boxes[m] = P->tx.count[m];
            o->k_boxes[m] = P->tk.count[m];
        }
        for (int l = 0; l <= P->L; ++l) o->pairs[l] = o->x_boxes[P->L - l] * o->k_boxes[l];
        const double unit = P->d == 2 ? 48.0 * P->p * P->p * P->p : 112.0 * P->p * P->p * P->p * P->p;
        double bytes = 0, flops = 0;
        for (int l = 0; l < P->L - P->start.s0; ++l) {  // the translated levels
            bytes += (double)(o->pairs[l + 1] + o->pairs[l]) * P->PD * (double)P->state_size;
            flops += (double)o->pairs[l] * unit;
        }
        o->sweep_bytes = bytes;
        o->sweep_flops = flops;
    });
}

int bfsft_plan_tables(const bfsft_plan *P, double *R, double *G, double *E)
{
    return guarded([&] {
        if (!P || P->batched || !R || !G || !E) throw Error{BFSFT_EINVAL, "NULL argument or batched plan"};
        const size_t p = (size_t)P->p;
        BF_HIP(hipMemcpyAsync(R, P->tb.R64, sizeof(double) * 2 * p * p, hipMemcpyDeviceToHost, P->stream));
        BF_HIP(hipMemcpyAsync(G, P->tb.C64, sizeof(double) * 2 * 4 * p, hipMemcpyDeviceToHost, P->stream));
        BF_HIP(hipMemcpyAsync(E, P->tb.erot, sizeof(double) * 2 * p, hipMemcpyDeviceToHost, P->stream));
        BF_HIP(hipStreamSynchronize(P->stream));
    });
}

int bfsft_plan_boxes(const bfsft_plan *P, int side, int m, int64_t *coords)
{
    return guarded([&] {
        if (!P || !coords || P->batched) throw Error{BFSFT_EINVAL, "NULL argument or batched plan"};
        if (m < 0 || m > P->L || (side != 0 && side != 1)) throw Error{BFSFT_EINVAL, "bad side or level"};
        const Tree &t = side == 0 ? P->tx : P->tk;
        if (t.npts == 0) return;
        std::vector<uint64_t> keys(t.count[m]);
        BF_HIP(hipMemcpyAsync(keys.data(), t.keys[m], sizeof(uint64_t) * keys.size(),
                              hipMemcpyDeviceToHost, P->stream));
        BF_HIP(hipStreamSynchronize(P->stream));
        for (size_t i = 0; i < keys.size(); ++i)
            for (int a = 0; a < P->d; ++a) {
                int64_t c = 0;
                for (int b = 0; b < m; ++b) c |= (int64_t)((keys[i] >> (b * P->d + a)) & 1ull) << b;
                coords[i * P->d + a] = c;
            }
    });
}

int bfsft_plan_create_batched(bfsft_plan **out, int count, const bfsft_problem *probs, int d, int p,
                              int precision, void *stream)
{
    if (!out) {
        set_last_error("out is NULL");
        return BFSFT_EINVAL;
    }
    *out = nullptr;
    bfsft_plan *B = nullptr;
    int rc = guarded([&] {
        if (count < 1 || !probs) throw Error{BFSFT_EINVAL, "count < 1 or NULL problems"};
        int64_t N0 = 2;
        for (int t = 0; t < count; ++t) {
            check_scalars(d, probs[t].N, p, precision, probs[t].nx, probs[t].nk, probs[t].x, probs[t].k);
            N0 = std::max<int64_t>(N0, probs[t].N);
        }
        B = new bfsft_plan();
        init_plan(B, d, N0, p, precision, 0, 0, (hipStream_t)stream);
        B->batched = true;
        for (int t = 0; t < count; ++t) {
            bfsft_plan *S = new bfsft_plan();
            B->subs.push_back(S);
            init_plan(S, d, probs[t].N, p, precision, probs[t].nx, probs[t].nk, (hipStream_t)stream);
            S->valu_only = true;
            S->arena.cap = -1;  // the cap applies to the batched plan as a whole
            build_plan(S, probs[t].x, probs[t].k);
        }
        create_batched(B, count, probs);
    });
    if (rc != BFSFT_OK) {
        if (B) {
            release_batched(B);
            delete B;
        }
        return rc;
    }
    *out = B;
    return BFSFT_OK;
}

int bfsft_execute_batched(bfsft_plan *B, const double *f, double *u)
{
    return guarded([&] {
        if (!B || !B->batched) throw Error{BFSFT_EINVAL, "not a batched plan"};
        if ((B->nk > 0 && !f) || (B->nx > 0 && !u)) throw Error{BFSFT_EINVAL, "NULL f or u"};
        execute_batched(B, f, u, false);
    });
}

int bfsft_execute_batched_serial(bfsft_plan *B, const double *f, double *u)
{
    return guarded([&] {
        if (!B || !B->batched) throw Error{BFSFT_EINVAL, "not a batched plan"};
        if ((B->nk > 0 && !f) || (B->nx > 0 && !u)) throw Error{BFSFT_EINVAL, "NULL f or u"};
        execute_batched(B, f, u, true);
    });
}

}  // extern "C"
