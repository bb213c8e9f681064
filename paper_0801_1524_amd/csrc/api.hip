// C ABI of bfsft (include/bfsft.h): validation, plan construction and the
// stream-ordered execution of steps 2-4 of Section 2.2.
#include "bfsft_impl.h"

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>

namespace bfsft {

int validate_points(const double *pts, int64_t n, int d, int64_t N, hipStream_t s);

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

}  // namespace bfsft

using namespace bfsft;

struct bfsft_plan {
    int d = 0, p = 0, precision = 0, L = 0;
    int64_t N = 0, nx = 0, nk = 0;
    double rho = 1.0;
    int PD = 0;
    hipStream_t stream = nullptr;
    Arena arena;
    Tree tx, tk;
    Tables tb;
    std::vector<int2 *> tiles;    // per T_K level l = 0..L-1 (output level of the step)
    std::vector<int> ntile;
    std::vector<int> cost_max;    // most LDS blocks a tile of level l needs
    std::vector<double *> sig;    // per T_X level m = 0..L-1 (rows a'), null when rho == 1
    void *buf[2] = {nullptr, nullptr};
    size_t state_size = 16;
    // timing events: per execute, L + 3 of them (see bfsft_timing_begin)
    std::vector<hipEvent_t> tev;
    int tmax = 0, tcount = 0;
};

namespace {

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

// Tiles of T_K level l: ranges [b0, b1) whose LDS cost (translate_tile_cost
// of their children count and size) is at most `cap`; a single box always
// fits, so every tile is non-empty.
std::vector<int2> make_tiles(const std::vector<int32_t> &cb, int d, int cap)
{
    std::vector<int2> t;
    const int n = (int)cb.size() - 1;
    int b0 = 0;
    while (b0 < n) {
        int b1 = b0 + 1;
        while (b1 < n && cb[b1 + 1] - cb[b0] <= 120 &&
               translate_tile_cost(d, cb[b1 + 1] - cb[b0], b1 + 1 - b0) <= cap)
            ++b1;
        t.push_back(make_int2(b0, b1));
        b0 = b1;
    }
    return t;
}

void check_scalars(int d, int64_t N, int p, int precision, int64_t nx, int64_t nk, const void *x,
                   const void *k)
{
    if (d != 2 && d != 3) throw Error{BFSFT_EINVAL, "d must be 2 or 3"};
    if (precision != BFSFT_FP64 && precision != BFSFT_MIXED && precision != BFSFT_FP32)
        throw Error{BFSFT_EINVAL, "unknown precision"};
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

void build_plan(bfsft_plan *P, const double *x, const double *k)
{
    hipStream_t s = P->stream;
    if (validate_points(x, P->nx, P->d, P->N, s) || validate_points(k, P->nk, P->d, P->N, s))
        throw Error{BFSFT_EDOMAIN, "a coordinate is not finite or lies outside [0, N]"};
    build_tree(P->tx, x, P->nx, P->d, P->L, P->N, P->arena, s);
    build_tree(P->tk, k, P->nk, P->d, P->L, P->N, P->arena, s);
    build_tables(P->tb, P->p, P->N, P->L, P->arena, s);
    P->tiles.assign(P->L, nullptr);
    P->ntile.assign(P->L, 0);
    P->cost_max.assign(P->L, 0);
    P->sig.assign(P->L, nullptr);
    if (P->nx == 0 || P->nk == 0) {
        BF_HIP(hipStreamSynchronize(s));
        return;
    }
    const int cap = translate_cap_blocks(P->d, P->p, P->precision);
    size_t maxpairs = 0;
    for (int l = 0; l <= P->L; ++l)
        maxpairs = std::max(maxpairs, (size_t)P->tx.count[P->L - l] * (size_t)P->tk.count[l]);
    for (int l = 0; l < P->L; ++l) {
        const std::vector<int32_t> &cb = P->tk.child_beg_host[l];
        std::vector<int2> t = make_tiles(cb, P->d, cap);
        P->ntile[l] = (int)t.size();
        for (const int2 &b : t)
            P->cost_max[l] = std::max(P->cost_max[l], translate_tile_cost(P->d, cb[b.y] - cb[b.x], b.y - b.x));
        P->tiles[l] = (int2 *)P->arena.alloc(sizeof(int2) * t.size());
        BF_HIP(hipMemcpyAsync(P->tiles[l], t.data(), sizeof(int2) * t.size(), hipMemcpyHostToDevice, s));
        BF_HIP(hipStreamSynchronize(s));  // t is a host temporary
    }
    if (P->rho != 1.0) {
        for (int m = 0; m < P->L; ++m) {
            P->sig[m] = (double *)P->arena.alloc(sizeof(double) * 2 * P->d * P->tx.count[m]);
            launch_sigma(P->tx.keys[m], P->tx.count[m], P->d, m, P->L, P->N, P->sig[m], s);
        }
    }
    const size_t bytes = maxpairs * (size_t)P->PD * P->state_size;
    P->buf[0] = P->arena.alloc(bytes);
    P->buf[1] = P->arena.alloc(bytes);
    BF_HIP(hipStreamSynchronize(s));
}

void run(bfsft_plan *P, const double *f, double *u, int probe_level, double *pot)
{
    if (P->nx == 0) return;
    if (P->nk == 0) {
        launch_zero_c128(u, P->nx, P->stream);
        return;
    }
    const Launch c = launch_of(P);
    const int L = P->L;
    hipEvent_t *ev = nullptr;
    if (P->tcount < P->tmax) ev = &P->tev[(size_t)P->tcount++ * (L + 3)];
    if (ev) BF_HIP(hipEventRecord(ev[0], P->stream));
    launch_leaf(c, f, P->tk, P->rho, P->buf[0]);
    if (ev) BF_HIP(hipEventRecord(ev[1], P->stream));
    if (probe_level == L)
        launch_export(c, P->buf[0], P->tx.keys[0], 1, P->tk.keys[L], P->tk.count[L], L, L, P->N, pot);
    int cur = 0;
    for (int l = L - 1; l >= 0; --l) {
        LevelArgs a;
        a.in = P->buf[cur];
        a.out = P->buf[cur ^ 1];
        a.in_row = P->tk.count[l + 1];
        a.out_row = P->tk.count[l];
        a.x_cb = P->tx.child_beg[L - l - 1];
        a.x_keys = P->tx.keys[L - l];
        a.k_cb = P->tk.child_beg[l];
        a.k_keys = P->tk.keys[l + 1];
        a.tiles = P->tiles[l];
        a.ntile = P->ntile[l];
        a.cost_max = P->cost_max[l];
        a.nap = P->tx.count[L - l - 1];
        a.sig = P->sig[L - l - 1];
        launch_translate(c, a);
        if (ev) BF_HIP(hipEventRecord(ev[2 + (L - 1 - l)], P->stream));
        cur ^= 1;
        if (probe_level == l)
            launch_export(c, P->buf[cur], P->tx.keys[L - l], P->tx.count[L - l], P->tk.keys[l],
                          P->tk.count[l], l, L, P->N, pot);
    }
    launch_final(c, P->buf[cur], P->tx, P->rho, P->nx, u);
    if (ev) BF_HIP(hipEventRecord(ev[L + 2], P->stream));
}

void free_events(bfsft_plan *P)
{
    for (hipEvent_t e : P->tev) (void)hipEventDestroy(e);
    P->tev.clear();
    P->tmax = P->tcount = 0;
}

}  // namespace

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
        P->d = d;
        P->p = p;
        P->precision = precision;
        P->N = N;
        P->nx = nx;
        P->nk = nk;
        P->L = ceil_log2(N);
        P->rho = std::ldexp((double)N, -P->L);
        P->PD = d == 2 ? p * p : p * p * p;
        P->stream = (hipStream_t)stream;
        P->state_size = precision == BFSFT_FP64 ? 16 : 8;
        P->arena.cap = env_cap();
        build_plan(P, x, k);
    });
    if (rc != BFSFT_OK) {
        if (P) {
            (void)hipStreamSynchronize(P->stream);
            P->arena.release();
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
        if ((plan->nk > 0 && !f) || (plan->nx > 0 && !u)) throw Error{BFSFT_EINVAL, "NULL f or u"};
        if (plan->nx > 0 && plan->nk > 0 && (const void *)f == (const void *)u)
            throw Error{BFSFT_EINVAL, "u aliases f"};
        run(plan, f, u, -1, nullptr);
    });
}

int bfsft_execute_probe(bfsft_plan *plan, const double *f, double *u, int level, double *pot)
{
    return guarded([&] {
        if (!plan) throw Error{BFSFT_EINVAL, "plan is NULL"};
        if (level < 0 || level > plan->L) throw Error{BFSFT_EINVAL, "level out of range"};
        if (!pot || !f || !u) throw Error{BFSFT_EINVAL, "NULL pointer"};
        if (plan->nx == 0 || plan->nk == 0) throw Error{BFSFT_EINVAL, "empty plan has no levels"};
        run(plan, f, u, level, pot);
    });
}

int bfsft_timing_begin(bfsft_plan *P, int max_execs)
{
    return guarded([&] {
        if (!P || max_execs < 1) throw Error{BFSFT_EINVAL, "bad timing request"};
        free_events(P);
        P->tev.resize((size_t)max_execs * (P->L + 3));
        for (auto &e : P->tev) BF_HIP(hipEventCreate(&e));
        P->tmax = max_execs;
    });
}

int bfsft_timing_end(bfsft_plan *P, double *out, int n)
{
    return guarded([&] {
        if (!P || !out || n < 3 + P->L) throw Error{BFSFT_EINVAL, "bad timing output"};
        const int L = P->L;
        for (int i = 0; i < n; ++i) out[i] = 0.0;
        out[0] = P->tcount;
        for (int r = 0; r < P->tcount; ++r) {
            hipEvent_t *ev = &P->tev[(size_t)r * (L + 3)];
            BF_HIP(hipEventSynchronize(ev[L + 2]));
            float ms = 0.f;
            BF_HIP(hipEventElapsedTime(&ms, ev[0], ev[1]));
            out[1] += ms;
            BF_HIP(hipEventElapsedTime(&ms, ev[L + 1], ev[L + 2]));
            out[2] += ms;
            for (int i = 0; i < L; ++i) {
                BF_HIP(hipEventElapsedTime(&ms, ev[1 + i], ev[2 + i]));
                out[3 + (L - 1 - i)] += ms;
            }
        }
        free_events(P);
    });
}

void bfsft_destroy(bfsft_plan *plan)
{
    if (!plan) return;
    (void)hipStreamSynchronize(plan->stream);
    free_events(plan);
    plan->arena.release();
    delete plan;
}

int bfsft_plan_info(const bfsft_plan *P, bfsft_info *o)
{
    return guarded([&] {
        if (!P || !o) throw Error{BFSFT_EINVAL, "NULL argument"};
        std::memset(o, 0, sizeof(*o));
        o->d = P->d;
        o->p = P->p;
        o->precision = P->precision;
        o->levels = P->L;
        o->N = P->N;
        o->nx = P->nx;
        o->nk = P->nk;
        o->rho = P->rho;
        o->transforms = 1;
        o->device_bytes = P->arena.bytes;
        if (P->nx == 0 || P->nk == 0) return;
        for (int m = 0; m <= P->L; ++m) {
            o->x_boxes[m] = P->tx.count[m];
            o->k_boxes[m] = P->tk.count[m];
        }
        for (int l = 0; l <= P->L; ++l) o->pairs[l] = o->x_boxes[P->L - l] * o->k_boxes[l];
        const double unit = P->d == 2 ? 48.0 * P->p * P->p * P->p : 112.0 * P->p * P->p * P->p * P->p;
        double bytes = 0, flops = 0;
        for (int l = 0; l < P->L; ++l) {
            bytes += (double)(o->pairs[l + 1] + o->pairs[l]) * P->PD * (double)P->state_size;
            flops += (double)o->pairs[l] * unit;
        }
        o->sweep_bytes = bytes;
        o->sweep_flops = flops;
    });
}

int bfsft_plan_boxes(const bfsft_plan *P, int side, int m, int64_t *coords)
{
    return guarded([&] {
        if (!P || !coords) throw Error{BFSFT_EINVAL, "NULL argument"};
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

int bfsft_plan_create_batched(bfsft_plan **out, int, const bfsft_problem *, int, int, int, void *)
{
    if (out) *out = nullptr;
    set_last_error("batched plans are not available in this build");
    return BFSFT_EINVAL;
}

int bfsft_execute_batched(bfsft_plan *, const double *, double *)
{
    set_last_error("batched plans are not available in this build");
    return BFSFT_EINVAL;
}

int bfsft_execute_batched_serial(bfsft_plan *, const double *, double *)
{
    set_last_error("batched plans are not available in this build");
    return BFSFT_EINVAL;
}

}  // extern "C"
