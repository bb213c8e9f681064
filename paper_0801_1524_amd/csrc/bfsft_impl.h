// Internal declarations of the bfsft library (gfx950).  Not part of the ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <utility>
#include <vector>

#include "bfsft.h"

namespace bfsft {

// ---------------------------------------------------------------- errors --
struct Error {
    int status;
    std::string msg;
};

void set_last_error(const std::string &m);

#define BF_HIP(call)                                                                  \
    do {                                                                              \
        hipError_t e_ = (call);                                                       \
        if (e_ != hipSuccess)                                                         \
            throw ::bfsft::Error{BFSFT_EDEVICE, std::string(#call) + ": " +           \
                                                    hipGetErrorString(e_)};           \
    } while (0)

// ------------------------------------------------------------ allocation --
// Device allocations of a plan are tracked so that BFSFT_MAX_DEVICE_BYTES can
// be enforced before any allocation is made.
struct Arena {
    std::vector<void *> ptrs;
    int64_t bytes = 0;
    int64_t temp_bytes = 0;  // live plan-time temporaries (TempList), also under the cap
    int64_t cap = -1;        // -1: no cap
    void *alloc(size_t n);
    void release();
    // plan-time temporaries: counted against the cap while alive
    void *alloc_temp(size_t n);
    void free_temp(void *p, size_t n);
};

// Temporaries of one plan-time step, freed when the list goes out of scope.
struct TempList {
    Arena &arena;
    std::vector<std::pair<void *, size_t>> p;
    explicit TempList(Arena &a) : arena(a) {}
    TempList(const TempList &) = delete;
    TempList &operator=(const TempList &) = delete;
    void *alloc(size_t n);
    ~TempList();
};

// -------------------------------------------------------------- tree ------
// One quadtree / octree over a point set, built on the device (step 1).
// Level m holds the non-empty boxes of width N / 2^m in Morton order.
struct Tree {
    int d = 0, L = 0;
    int64_t npts = 0;
    std::vector<int64_t> count;        // [L+1] boxes per level
    std::vector<uint64_t *> keys;      // [L+1] device, Morton keys of level m
    std::vector<int32_t *> child_beg;  // [L] device, level m: [count[m]+1] first child in level m+1
    std::vector<uint64_t *> slots;     // [L] device, level m: [count[m]] byte s = child at position s,
                                       //   as an offset from child_beg (0xff: no such child)
    std::vector<std::vector<int32_t>> child_beg_host;  // same, host copies (tiling)
    int32_t *perm = nullptr;           // device [npts]: Morton-sorted position -> original index
    int32_t *leaf_beg = nullptr;       // device [count[L]+1]: sorted points of each leaf
    int32_t *leaf_of = nullptr;        // device [npts]: leaf of each point, original order
    double *local = nullptr;           // device [npts][d]: x - rho*leaf_index, original order
};

void build_tree(Tree &t, const double *pts_dev, int64_t n, int d, int L, int64_t N,
                Arena &arena, hipStream_t s);

// device scan used by the tree build (exclusive, uint32); temporary storage
// from `tmp`
void scan_exclusive_u32(const uint32_t *in, uint32_t *out, int n, hipStream_t s, TempList &tmp);
int validate_points(const double *pts, int64_t n, int d, int64_t N, Arena &arena, hipStream_t s);

// ------------------------------------------------------------- kernels ----
// Operator tables of one leaf width rho (Section 2.1, as interpolation rows).
// The state is kept rotated, w^ = (E x ... x E) w with E[k] = exp(-i pi rho k / q),
// which makes the interpolation operator of every axis real:
//   L_t = diag(D_t) R_t diag(E),  D_t[l] = exp(i pi rho (t q + l) / (2 q)),
// so a level is w^_out[l] = sum_s sigma^s G(s, t, l) (R_t w^_s)[l] per axis.
struct Tables {
    double *R64 = nullptr;   // [2][p][p] real: R_t
    float *R32 = nullptr;
    double *C64 = nullptr;   // [2 s][2 t][p] complex: G(s, t, l)
    float *C32 = nullptr;
    double *erot = nullptr;  // [p] complex: E[k]
    double *L64 = nullptr;   // [2][p][p] complex: Lagrange rows L_t (matrix-core tables)
    double *PH64 = nullptr;  // [2][p] complex: phase of a child at offset s = 1
    double *nodes = nullptr; // [p] complex  Z_k (unused by kernels; kept for probes)
    double *bary = nullptr;  // [p] complex  barycentric weights of the nodes
    double *node_turns = nullptr; // [p] real  rho*k/q^2
    double *mf = nullptr;    // per-lane operator tables of the matrix-core kernel (5 <= p <= 9)
};

void build_tables(Tables &tb, int p, int64_t N, int L, Arena &arena, hipStream_t s);

// per-level arguments of the translation kernels
struct LevelArgs {
    const void *in;          // state of T_K level l+1, rows a' (T_X level L-l-1)
    void *out;               // state of T_K level l,   rows a  (T_X level L-l)
    int64_t in_row;          // boxes per input row  = count_K[l+1]
    int64_t out_row;         // boxes per output row = count_K[l]
    const int32_t *x_cb;     // T_X level L-l-1: children range in level L-l, [nap+1]
    const int32_t *k_cb;     // T_K level l: children range in level l+1
    const uint64_t *x_slot;  // T_X level L-l-1: child-position slots (Tree::slots)
    const uint64_t *k_slot;  // T_K level l: child-position slots
    const int4 *tiles;       // [ntile] (b0, b1, first child, end of children)
    int ntile;
    int cost_max;            // most LDS blocks any tile needs (translate_tile_cost)
    int rows;                // rows a' per work-group
    int kind;                // 0: VALU kernel, 1: FP64 matrix-core kernel (2D), 2: stage 1 on
                             //   the matrix cores in the precision's contraction format (2D)
    int64_t nap;             // rows a'
    const double *sig;       // [nap][d] complex exp(2 pi i rho i_{A'}) or null (rho == 1)
};

struct Launch {
    int d, p, precision;
    const Tables *tb;
    hipStream_t stream;
};

int translate_default_lds(int d);
int translate_cap_blocks(int d, int p, int precision, int budget);
int translate_tile_cost(int d, int p, int precision, int nin, int nb, int kind = 0);
bool translate_fits(int d, int p, int precision);
int translate_rows(int cap, int cost_max, int64_t nap, int kind = 0);
size_t translate_lds_bytes(int d, int p, int precision, int rows, int cost_max, int kind = 0);
int64_t translate_items(const LevelArgs &la);
size_t translate_desc_size();
void translate_fill_desc(const Launch &c, const LevelArgs &la, void *dst);
// `next` is the step's item counter; it must be zero when the launch starts
void launch_translate_batched(const Launch &c, const void *descs, const int64_t *prefix, int ndesc,
                              int64_t total, size_t lds, int grid, unsigned long long *next);

// per-transform descriptors of the batched leaf and final launches; `first`
// is the transform's first flat item
struct LeafDesc {
    const double *f;
    const int32_t *perm;
    const int32_t *beg;
    const double *local;
    void *state;
    int64_t nleaf;
    double shift;  // rho / 2: the leaf phase is taken from B's centre (rotated state)
    int64_t first;
};

struct FinalDesc {
    const void *state;
    const int32_t *leaf_of;
    const double *local;
    const double *bary;
    const double *node_turns;
    const double *erot;
    double *u;
    int64_t nx;
    int64_t first;
};

void launch_leaf_batched(const Launch &c, const LeafDesc *ds, const int64_t *prefix, int n,
                         int64_t total);
void launch_final_batched(const Launch &c, const FinalDesc *ds, const int64_t *prefix, int n,
                          int64_t total);
void launch_translate(const Launch &c, const LevelArgs &a);

// Start of the sweep s0 levels above the leaves (s0 = 0: the leaves).
struct StartLevel {
    int s0 = 0;
    int kind = 0;               // direct-sum kernel: 0 VALU, 1 FP64 matrix cores
    // matrix-core kernel: its steps (one chunk of at most 16 sources of a box
    // B for one block of A rows), in order, and each work-group's range of them
    int4 *steps = nullptr;      // [nsteps] x first source, y count | first << 8 | last << 9,
                                //   z box b, w row block
    int32_t *wg_first = nullptr;// [nwg + 1] first step of every work-group
    int nwg = 0, nwaves = 0;
    // matrix-core kernel, when they fit the table budget: the parts of the
    // direct sums that depend on the points only, computed at plan time
    double2 *gam = nullptr;     // [nA][npts] Gamma[A][j] (sources in sorted order)
    double2 *geo = nullptr;     // [npts][p^d] T_j[l] / f_j
    int2 *box_leaf = nullptr;   // [count_K[L - s0]] leaf range of every box of T_K level L - s0
    int32_t *sm = nullptr;      // [npts][d] leaf index mod 2^s0 of every source (sorted order)
    double *sloc = nullptr;     // [npts][d] offset inside its leaf (sorted order)
    double2 *sratio = nullptr;  // [npts][d] phase step between grid points, per axis
};
// s0 <= 18 keeps the exact phase reduction of the direct sums in 64-bit integers
constexpr int kStartMax = 18;
void build_start(StartLevel &st, const Tree &tk, int s0, int d, int q, double rho, Arena &arena, hipStream_t s);
void launch_direct(const Launch &c, const StartLevel &st, const double *f, const Tree &tx, const Tree &tk,
                   int64_t N, void *state);

// direct-sum kernels: the VALU one takes every (d, p); the matrix-core one
// 2D p <= 12 and 3D p <= 5.  Bit 0: VALU allowed, bit 1: matrix cores;
// BFSFT_DIRECT=valu or =mfma allows one only (mfma falls back to valu where
// unsupported).
bool direct_mfma_supported(int d, int p);
int direct_kinds(int d, int p);
// byte budget of the matrix-core direct sums' plan-time tables
int64_t direct_table_budget();

// one transform of a (batched) direct start-level launch
struct DirectDesc {
    int s0, L;
    int64_t N, nA, nB;          // pairs: T_X boxes of level s0 x T_K boxes of level L - s0
    const uint64_t *xkeys;      // T_X keys of level s0
    const int2 *box_leaf;
    const int4 *steps;          // matrix-core kernel only (single plans)
    const int32_t *wg_first;
    int nwg, nwaves;
    const double2 *gam, *geo;   // matrix-core kernel: plan-time tables, or NULL
    int64_t nk;                 // sources (row length of gam)
    const int32_t *leaf_beg;
    const int32_t *perm;
    const int32_t *sm;
    const double *sloc;
    const double2 *sstep;
    const double2 *f;           // sources, original order
    const double2 *erot;        // [p] E[k] of the state rotation
    void *state;                // output state of level L - s0
    int64_t first;              // first flat item (batched)
};
DirectDesc direct_desc(const StartLevel &st, const double *f, const Tree &tx, const Tree &tk, int64_t N,
                       const Tables &tb, void *state);
int64_t direct_items(int d, int p, const DirectDesc &dd);
void launch_direct_mfma(const Launch &c, const DirectDesc &dd);
// the matrix-core kernel's step list for start level st.s0 (st.kind == 1)
void build_direct_steps(StartLevel &st, const Tree &tx, const Tree &tk, const Tables &tb, int d, int p,
                        int64_t N, Arena &arena, hipStream_t s);
void launch_direct_batched(const Launch &c, const DirectDesc *ds, const int64_t *prefix, int n, int64_t total);

// 2D translation with stage 1 on the matrix cores in the FP32, FP16X2 or
// BF16X3 contraction format (FP32 state); kind 2 of a level
bool translate_xdl_supported(int d, int p, int precision);
void launch_translate_xdl(const Launch &c, const LevelArgs &la);
void launch_translate_batched_xdl(const Launch &c, const void *descs, const int64_t *prefix, int ndesc,
                                  int64_t total, size_t lds, int grid, unsigned long long *next);
// split-precision formats (stage 1 on the matrix cores only)
inline bool split_precision(int precision) { return precision == BFSFT_FP16X2 || precision == BFSFT_BF16X3; }

// matrix-core (MFMA) 2D translation with FP64 arithmetic (mixed and FP64)
bool translate_mfma_supported(int d, int p, int precision);
size_t translate_mfma_table_doubles(int p);
void build_mfma_tables(const Tables &tb, int p, double *dst, hipStream_t s);
void launch_translate_mfma(const Launch &c, const LevelArgs &la);
void launch_leaf(const Launch &c, const double *f, const Tree &tk, double rho, void *state);
void launch_final(const Launch &c, const void *state, const Tree &tx, double rho, int64_t nx,
                  double *u);
void launch_export(const Launch &c, const void *state, const uint64_t *xkeys, int64_t nA,
                   const uint64_t *kkeys, int64_t nB, int lvl, int L, int64_t N, double *pot);
void launch_zero_c128(double *u, int64_t n, hipStream_t s);
void launch_zero_u64(unsigned long long *p, int64_t n, hipStream_t s);
void launch_conj(const double *in, double *out, int64_t n, hipStream_t s);  // out = conj(in), n complex
void launch_sigma(const uint64_t *keys, int64_t n, int d, int m, int L, int64_t N,
                  double *sig, hipStream_t s);

}  // namespace bfsft
