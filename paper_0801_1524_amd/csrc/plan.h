// The plan object behind the opaque bfsft_plan handle (host side).
#pragma once

#include "bfsft_impl.h"

#include <string>
#include <vector>

struct bfsft_plan {
    int d = 0, p = 0, precision = 0, L = 0;
    int64_t N = 0, nx = 0, nk = 0;
    double rho = 1.0;
    int PD = 0;
    hipStream_t stream = nullptr;
    bfsft::Arena arena;

    // ---- one transform
    bfsft::Tree tx, tk;
    bfsft::Tables tb;
    bfsft::StartLevel start;            // the sweep begins at T_K level L - start.s0
    int lds = 0;                        // LDS budget of a translation tile (bytes), most levels
    std::vector<int> lds_level;         // per T_K level l: tile LDS budget (bytes)
    std::vector<int> kind;              // per T_K level l: 0 VALU kernel, 1 matrix-core kernel
    bool valu_only = false;             // member of a batched plan (its kernel is the VALU one)
    bfsft_plan *adj = nullptr;          // adjoint: trees exchanged, built on first use
    double *adj_in = nullptr;           // adjoint plan: conjugated input staging [nk] complex
    std::vector<int4 *> tiles;          // per T_K level l = 0..L-1 (output level of the step)
    std::vector<int> ntile;
    std::vector<int> cost_max;          // most LDS blocks a tile of level l needs
    std::vector<int> rows;              // rows a' per work-group at level l
    std::vector<double *> sig;          // per T_X level m = 0..L-1 (rows a'), null when rho == 1
    void *buf[2] = {nullptr, nullptr};  // ping-pong state of two adjacent levels
    size_t state_size = 16;
    std::vector<hipEvent_t> tev;        // timing events, L + 3 per execute
    int tmax = 0, tcount = 0;

    // ---- batched: independent transforms sharing d, p, precision
    bool batched = false;
    std::vector<bfsft_plan *> subs;
    std::vector<int64_t> f_off, u_off;  // offsets of each transform in the packed arrays
    double *f_stage = nullptr, *u_stage = nullptr;
    struct Step {
        void *desc = nullptr;           // [ndesc] translation descriptors
        int64_t *prefix = nullptr;      // [ndesc] first work item of each
        int ndesc = 0;
        int64_t total = 0;
        size_t lds = 0;
    };
    std::vector<Step> steps;            // sweep step s = 1..Lmax at index s-1
    bfsft::LeafDesc *leaf_desc = nullptr;
    int64_t *leaf_prefix = nullptr;
    int leaf_n = 0;
    int64_t leaf_total = 0;
    bfsft::DirectDesc *direct_desc = nullptr;  // transforms that start above their leaves
    int64_t *direct_prefix = nullptr;
    int direct_n = 0;
    int64_t direct_total = 0;
    bfsft::FinalDesc *final_desc = nullptr;
    int64_t *final_prefix = nullptr;
    int final_n = 0;
    int64_t final_total = 0;
    unsigned long long *step_next = nullptr;  // [steps] item counters of the step launches
    int grid = 0;                       // work-groups of a persistent step launch
    int wg_per_cu = 0;
    hipStream_t cap_stream = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t gexec = nullptr;
};

namespace bfsft {

// shared by the single and batched plan code
Launch launch_of(const bfsft_plan *P);
LevelArgs level_args(const bfsft_plan *P, int l, const void *in, void *out);
void build_tiles(bfsft_plan *P, int lds_bytes);
void build_tiles_levels(bfsft_plan *P, const std::vector<int> &lds_bytes, const std::vector<int> &kinds);
void build_plan(bfsft_plan *P, const double *x, const double *k);
void release_plan(bfsft_plan *P);
int ceil_log2(int64_t N);
int64_t env_cap();
// start level of the sweep and its direct-sum kernel (0 VALU, 1 matrix cores)
struct StartChoice {
    int s0 = 0, kind = 0;
};
StartChoice choose_start(const bfsft_plan *P);

// autotuning cache (text file, one "key value..." line per entry)
bool tune_lookup(const std::string &key, std::vector<int> &vals);
void tune_store(const std::string &key, const std::vector<int> &vals);
bool autotune_enabled();

}  // namespace bfsft
