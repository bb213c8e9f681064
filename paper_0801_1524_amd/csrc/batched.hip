// Batched plans: many independent transforms of the same d, p and precision
// but their own N and points.  All transforms start with their leaves at the
// same time; sweep step s (s = 1 .. max L_t) runs T_K level L_t - s of every
// transform that still has levels, as one persistent launch over the
// concatenated work items; transforms with fewer levels retire early.  Leaf
// initialisation, the steps and the final evaluation are captured once into
// a HIP graph; an execute copies the packed sources into the plan, launches
// the graph and copies the packed outputs out.
#include "plan.h"

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

namespace bfsft {

void run_single(bfsft_plan *P, const double *f, double *u);

namespace {

Launch batch_launch(const bfsft_plan *B, hipStream_t s)
{
    Launch c;
    c.d = B->d;
    c.p = B->p;
    c.precision = B->precision;
    c.tb = nullptr;  // batched kernels read each transform's tables from its descriptor
    c.stream = s;
    return c;
}

bool active(const bfsft_plan *S) { return S->nx > 0 && S->nk > 0; }

template <typename T> T *upload(bfsft_plan *B, const std::vector<T> &v)
{
    T *d = (T *)B->arena.alloc(sizeof(T) * std::max<size_t>(1, v.size()));
    if (!v.empty()) {
        BF_HIP(hipMemcpyAsync(d, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice, B->stream));
        BF_HIP(hipStreamSynchronize(B->stream));  // v is a host temporary
    }
    return d;
}

// Translation descriptors of every sweep step under the sub-plans' current tiles.
void build_steps(bfsft_plan *B)
{
    int Lmax = 0;
    for (bfsft_plan *S : B->subs)
        if (active(S)) Lmax = std::max(Lmax, S->L);
    B->steps.assign(Lmax, {});
    const size_t dsz = translate_desc_size();
    for (int s = 1; s <= Lmax; ++s) {
        bfsft_plan::Step st;
        std::vector<unsigned char> descs;
        std::vector<int64_t> prefix;
        for (bfsft_plan *S : B->subs) {
            // transform S translates at steps start + 1 .. L
            if (!active(S) || S->L < s || s <= S->start.s0) continue;
            const int l = S->L - s;
            const LevelArgs la = level_args(S, l, S->buf[(s - 1) & 1], S->buf[s & 1]);
            const int64_t items = translate_items(la);
            if (items == 0) continue;
            const size_t at = descs.size();
            descs.resize(at + dsz);
            translate_fill_desc(launch_of(S), la, descs.data() + at);
            prefix.push_back(st.total);
            st.total += items;
            st.lds = std::max(st.lds, translate_lds_bytes(S->d, S->p, S->precision, la.rows, la.cost_max));
            ++st.ndesc;
        }
        st.desc = upload(B, descs);
        st.prefix = upload(B, prefix);
        B->steps[s - 1] = st;
    }
}

void build_leaf_final(bfsft_plan *B)
{
    std::vector<LeafDesc> ld;
    std::vector<DirectDesc> dd;
    std::vector<FinalDesc> fd;
    std::vector<int64_t> lp, dp, fp;
    int64_t lt = 0, dt = 0, ft = 0;
    for (size_t t = 0; t < B->subs.size(); ++t) {
        bfsft_plan *S = B->subs[t];
        if (!active(S)) continue;
        if (S->start.s0 > 0) {
            // the state of level L - s0 goes where step s0 + 1 reads it
            DirectDesc a = direct_desc(S->start, B->f_stage + 2 * B->f_off[t], S->tx, S->tk, S->N, S->tb,
                                       S->buf[S->start.s0 & 1]);
            a.first = dt;
            dp.push_back(dt);
            // each transform's items start on a work-group boundary (the
            // batched kernel finds one owner per work-group)
            dt += (direct_items(S->d, S->p, a) + 255) / 256 * 256;
            dd.push_back(a);
        }
        LeafDesc a;
        a.f = B->f_stage + 2 * B->f_off[t];
        a.perm = S->tk.perm;
        a.beg = S->tk.leaf_beg;
        a.local = S->tk.local;
        a.state = S->buf[0];
        a.nleaf = S->tk.count[S->L];
        a.shift = 0.5 * S->rho;
        a.first = lt;
        if (S->start.s0 == 0) {
            lp.push_back(lt);
            lt += a.nleaf * S->PD;
            ld.push_back(a);
        }
        FinalDesc b;
        b.state = S->buf[S->L & 1];
        b.leaf_of = S->tx.leaf_of;
        b.local = S->tx.local;
        b.bary = S->tb.bary;
        b.node_turns = S->tb.node_turns;
        b.erot = S->tb.erot;
        b.u = B->u_stage + 2 * B->u_off[t];
        b.nx = S->nx;
        b.first = ft;
        fp.push_back(ft);
        ft += S->nx;
        fd.push_back(b);
    }
    B->leaf_desc = upload(B, ld);
    B->leaf_prefix = upload(B, lp);
    B->leaf_n = (int)ld.size();
    B->leaf_total = lt;
    B->direct_desc = upload(B, dd);
    B->direct_prefix = upload(B, dp);
    B->direct_n = (int)dd.size();
    B->direct_total = dt;
    B->final_desc = upload(B, fd);
    B->final_prefix = upload(B, fp);
    B->final_n = (int)fd.size();
    B->final_total = ft;
}

void enqueue(bfsft_plan *B, hipStream_t s)
{
    const Launch c = batch_launch(B, s);
    // item counters of all steps start at zero (a kernel, not a memset node)
    launch_zero_u64(B->step_next, (int64_t)B->steps.size(), s);
    launch_leaf_batched(c, B->leaf_desc, B->leaf_prefix, B->leaf_n, B->leaf_total);
    launch_direct_batched(c, B->direct_desc, B->direct_prefix, B->direct_n, B->direct_total);
    for (size_t i = 0; i < B->steps.size(); ++i) {
        const bfsft_plan::Step &st = B->steps[i];
        launch_translate_batched(c, st.desc, st.prefix, st.ndesc, st.total, st.lds, B->grid, B->step_next + i);
    }
    launch_final_batched(c, B->final_desc, B->final_prefix, B->final_n, B->final_total);
}

double time_steps(bfsft_plan *B, int reps)
{
    const Launch c = batch_launch(B, B->stream);
    hipEvent_t e0, e1;
    BF_HIP(hipEventCreate(&e0));
    BF_HIP(hipEventCreate(&e1));
    double best = 1e30;
    for (int r = 0; r < reps + 1; ++r) {
        launch_zero_u64(B->step_next, (int64_t)B->steps.size(), B->stream);
        BF_HIP(hipEventRecord(e0, B->stream));
        for (size_t i = 0; i < B->steps.size(); ++i) {
            const bfsft_plan::Step &st = B->steps[i];
            launch_translate_batched(c, st.desc, st.prefix, st.ndesc, st.total, st.lds, B->grid,
                                     B->step_next + i);
        }
        BF_HIP(hipEventRecord(e1, B->stream));
        BF_HIP(hipEventSynchronize(e1));
        float ms = 0.f;
        BF_HIP(hipEventElapsedTime(&ms, e0, e1));
        if (r > 0) best = std::min(best, (double)ms);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return best;
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

// BFSFT_BATCHED_WG: forced persistent work-groups per CU (0 = one work-group
// per item), or -1 when unset
int batched_wg_env()
{
    const char *e = std::getenv("BFSFT_BATCHED_WG");
    if (!e || !*e) return -1;
    char *end = nullptr;
    const long v = std::strtol(e, &end, 10);
    if (end == e || v < 0 || v > 32) return -1;
    return (int)v;
}

}  // namespace

void create_batched(bfsft_plan *B, int count, const bfsft_problem *probs)
{
    int64_t fo = 0, uo = 0;
    for (int t = 0; t < count; ++t) {
        B->f_off.push_back(fo);
        B->u_off.push_back(uo);
        fo += probs[t].nk;
        uo += probs[t].nx;
    }
    B->nk = fo;
    B->nx = uo;
    B->f_stage = (double *)B->arena.alloc(sizeof(double) * 2 * std::max<int64_t>(1, fo));
    B->u_stage = (double *)B->arena.alloc(sizeof(double) * 2 * std::max<int64_t>(1, uo));
    launch_zero_c128(B->f_stage, fo, B->stream);
    launch_zero_c128(B->u_stage, uo, B->stream);  // transforms without sources keep u = 0
    B->L = 0;
    for (bfsft_plan *S : B->subs) B->L = std::max(B->L, S->L);
    B->step_next = (unsigned long long *)B->arena.alloc(sizeof(unsigned long long) * std::max(1, B->L));

    int dev = 0, ncu = 256;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess)
        ncu = prop.multiProcessorCount;

    const int64_t cap = env_cap();
    int64_t total = 0;
    for (bfsft_plan *S : B->subs) total += S->arena.bytes;
    if (cap >= 0 && total + B->arena.bytes > cap)
        throw Error{BFSFT_ENOMEM, "BFSFT_MAX_DEVICE_BYTES exceeded by the batched plan"};

    // autotuning: tile LDS budget x persistent work-groups per CU, timed on
    // the plan's own steps (results do not depend on either);
    // BFSFT_BATCHED_WG=n forces the launch form (0: one work-group per item,
    // n > 0: n persistent work-groups per CU) and tunes only the budget
    const int forced_wg = batched_wg_env();
    std::vector<int> wg_cand = {0, 4, 5, 8};
    if (forced_wg >= 0) wg_cand = {forced_wg};
    const std::string key = "batched3/d" + std::to_string(B->d) + "/p" + std::to_string(B->p) + "/" +
                            prec_name(B->precision) + "/n" + std::to_string(count) +
                            (forced_wg >= 0 ? "/w" + std::to_string(forced_wg) : std::string());
    std::vector<int> best;
    if (!tune_lookup(key, best) || best.size() != 2) {
        best = {32, forced_wg >= 0 ? forced_wg : 4};
        if (autotune_enabled()) {
            double best_ms = 1e30;
            // one plain execute per transform (zero sources) leaves finite
            // state in every buffer the timed steps read
            for (size_t t = 0; t < B->subs.size(); ++t)
                if (active(B->subs[t]))
                    run_single(B->subs[t], B->f_stage + 2 * B->f_off[t], B->u_stage + 2 * B->u_off[t]);
            for (int kb : {16, 20, 24, 28, 32, 36, 40}) {
                for (bfsft_plan *S : B->subs) build_tiles(S, kb * 1024);
                build_steps(B);
                for (int wg : wg_cand) {  // 0: one work-group per item
                    B->grid = ncu * wg;
                    const double ms = time_steps(B, 2);
                    if (ms < best_ms) {
                        best_ms = ms;
                        best = {kb, wg};
                    }
                }
            }
            // the staging output was used as scratch while timing
            launch_zero_c128(B->u_stage, uo, B->stream);
            tune_store(key, best);
        }
    }
    for (bfsft_plan *S : B->subs) build_tiles(S, best[0] * 1024);
    B->lds = best[0] * 1024;
    B->wg_per_cu = best[1];
    B->grid = ncu * best[1];
    build_steps(B);
    build_leaf_final(B);

    // capture leaf, steps and final into one graph on a private stream
    BF_HIP(hipStreamCreate(&B->cap_stream));
    BF_HIP(hipStreamBeginCapture(B->cap_stream, hipStreamCaptureModeRelaxed));
    try {
        enqueue(B, B->cap_stream);
    } catch (...) {
        hipGraph_t g = nullptr;
        (void)hipStreamEndCapture(B->cap_stream, &g);
        if (g) (void)hipGraphDestroy(g);
        throw;
    }
    BF_HIP(hipStreamEndCapture(B->cap_stream, &B->graph));
    BF_HIP(hipGraphInstantiate(&B->gexec, B->graph, nullptr, nullptr, 0));
    BF_HIP(hipStreamSynchronize(B->stream));
}

void execute_batched(bfsft_plan *B, const double *f, double *u, bool serial)
{
    if (serial) {
        for (size_t t = 0; t < B->subs.size(); ++t) {
            bfsft_plan *S = B->subs[t];
            if (S->nx == 0) continue;
            run_single(S, f + 2 * B->f_off[t], u + 2 * B->u_off[t]);
        }
        return;
    }
    if (B->nk > 0)
        BF_HIP(hipMemcpyAsync(B->f_stage, f, sizeof(double) * 2 * B->nk, hipMemcpyDeviceToDevice, B->stream));
    BF_HIP(hipGraphLaunch(B->gexec, B->stream));
    if (B->nx > 0)
        BF_HIP(hipMemcpyAsync(u, B->u_stage, sizeof(double) * 2 * B->nx, hipMemcpyDeviceToDevice, B->stream));
}

void release_batched(bfsft_plan *B)
{
    (void)hipStreamSynchronize(B->stream);
    if (B->gexec) (void)hipGraphExecDestroy(B->gexec);
    if (B->graph) (void)hipGraphDestroy(B->graph);
    if (B->cap_stream) (void)hipStreamDestroy(B->cap_stream);
    B->gexec = nullptr;
    B->graph = nullptr;
    B->cap_stream = nullptr;
    for (bfsft_plan *S : B->subs) {
        release_plan(S);
        delete S;
    }
    B->subs.clear();
    B->arena.release();
}

void info_batched(const bfsft_plan *B, bfsft_info *o)
{
    o->d = B->d;
    o->p = B->p;
    o->precision = B->precision;
    o->levels = B->L;
    o->N = B->N;
    o->nx = B->nx;
    o->nk = B->nk;
    o->rho = 0.0;
    o->transforms = (int64_t)B->subs.size();
    o->lds_kb = B->lds / 1024;
    o->wg_per_cu = B->wg_per_cu;
    int64_t bytes = B->arena.bytes;
    double sb = 0, sf = 0;
    for (const bfsft_plan *S : B->subs) {
        bytes += S->arena.bytes;
        if (!active(S)) continue;
        bfsft_info si;
        std::memset(&si, 0, sizeof(si));
        const double unit = S->d == 2 ? 48.0 * S->p * S->p * S->p : 112.0 * S->p * S->p * S->p * S->p;
        for (int l = 0; l < S->L; ++l) {
            const double pl = (double)S->tx.count[S->L - l] * S->tk.count[l];
            const double pl1 = (double)S->tx.count[S->L - l - 1] * S->tk.count[l + 1];
            sb += (pl + pl1) * S->PD * (double)S->state_size;
            sf += pl * unit;
            // pairs[s] summed over transforms, by sweep step s = L_t - l
            o->pairs[S->L - l] += (int64_t)pl;
        }
    }
    o->device_bytes = bytes;
    o->sweep_bytes = sb;
    o->sweep_flops = sf;
}

}  // namespace bfsft
