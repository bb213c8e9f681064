// Pieces shared by the two 2D/3D translation kernels of step 3 of
// Section 2.2: the VALU kernels (translate.hip) and the matrix-core kernel
// (translate_mfma.hip).  Internal to the library.
#pragma once

#include "bfsft_impl.h"
#include "cplx.h"

#include <cstdlib>

namespace bfsft {
namespace tr {

#ifndef BFSFT_TT
#define BFSFT_TT 256
#endif
constexpr int kTT = BFSFT_TT;  // threads of a translation work-group
constexpr int kWaves = kTT / 64;
constexpr int kRowsMax = 32;   // rows a' per work-group
constexpr int kInMax = 127;    // inputs of a tile (local child indices fit a signed char)
constexpr int kPMax2 = 12;     // largest 2D grid size p
constexpr size_t kLdsMax = 60 * 1024;  // dynamic LDS of one work-group (static use stays below 4 KB)
// 2D single-transform tiles may be larger: two work-groups of this size and
// their static tables still fit the 160 KB of a CU (for the last levels,
// whose rows hold few boxes, so a tile needs many rows to fill stage 2)
constexpr size_t kLdsMax2D = 76 * 1024;
// Work-groups of one launch: its work-items (work-groups x kTT) must stay
// below 2^32, or the dispatch runs only part of the grid.  Launches of more
// work items are split into chunks of this many, each told its first item.
constexpr int64_t kMaxGroups = (((int64_t)1 << 32) / kTT) - 1;

// chunk size of the translation launches: kMaxGroups, or less when
// BFSFT_MAX_GROUPS asks for it (tests of the chunked launches)
inline int64_t max_groups()
{
    const char *e = std::getenv("BFSFT_MAX_GROUPS");
    const long long v = e ? std::atoll(e) : 0;
    return v >= 1 && v < kMaxGroups ? (int64_t)v : kMaxGroups;
}

struct TArgs {
    const void *in;
    void *out;
    int64_t in_row, out_row;
    const int32_t *x_cb;
    const int32_t *k_cb;
    const uint64_t *x_slot;
    const uint64_t *k_slot;
    const int4 *tiles;
    int ntile;
    int rows;
    int64_t nap;
    const double2 *sig;
    const void *R;   // [2][P][P] real, compute precision: R_t
    const void *C;   // [2 s][2 t][P] complex, compute precision: G(s, t, l)
};

// Descriptor i of a device array, read through the constant address space:
// it is uniform and read-only, so every field becomes a scalar load (the
// fields are copied one by one; the struct holds only pointers and integers)
__device__ __forceinline__ TArgs load_desc(const TArgs *descs, int i)
{
    using CT = const __attribute__((address_space(4))) TArgs;
    CT *d = (CT *)descs + i;
    TArgs a;
    a.in = d->in;
    a.out = d->out;
    a.in_row = d->in_row;
    a.out_row = d->out_row;
    a.x_cb = d->x_cb;
    a.k_cb = d->k_cb;
    a.x_slot = d->x_slot;
    a.k_slot = d->k_slot;
    a.tiles = d->tiles;
    a.ntile = d->ntile;
    a.rows = d->rows;
    a.nap = d->nap;
    a.sig = d->sig;
    a.R = d->R;
    a.C = d->C;
    return a;
}

inline TArgs make_targs(const Launch &c, const LevelArgs &la)
{
    TArgs a;
    a.in = la.in;
    a.out = la.out;
    a.in_row = la.in_row;
    a.out_row = la.out_row;
    a.x_cb = la.x_cb;
    a.k_cb = la.k_cb;
    a.x_slot = la.x_slot;
    a.k_slot = la.k_slot;
    a.tiles = la.tiles;
    a.ntile = la.ntile;
    a.nap = la.nap;
    a.rows = la.rows;
    a.sig = reinterpret_cast<const double2 *>(la.sig);
    const bool f32 = c.precision == BFSFT_FP32;
    a.R = f32 ? (const void *)c.tb->R32 : (const void *)c.tb->R64;
    a.C = f32 ? (const void *)c.tb->C32 : (const void *)c.tb->C64;
    return a;
}

// Row structure of R_t (and L_t): row l is the unit vector of node (t q + l) / 2
// when t q + l is even, a full interpolation row otherwise.
template <int P, int T> struct Rows {
    static constexpr int Q = P - 1;
    static constexpr __host__ __device__ bool copy(int l) { return ((T * Q + l) & 1) == 0; }
    static constexpr int first_dot = (1 + T * Q) & 1;
    static constexpr int ndot = (P - first_dot + 1) / 2;
    // position of copy row l among the copy rows
    static constexpr __host__ __device__ int copy_index(int l)
    {
        int c = 0;
        for (int i = 0; i < l; ++i) c += copy(i) ? 1 : 0;
        return c;
    }
};

// complex value of type Cv from an LDS/state element of another precision
template <typename Cv, typename V> __device__ __forceinline__ Cv ld(const V *p)
{
    return cvt<Cv>(*p);
}

template <typename V, typename Cv> __device__ __forceinline__ void st(V *p, const Cv v)
{
    V o;
    o.x = (decltype(o.x))v.x;
    o.y = (decltype(o.y))v.y;
    *p = o;
}

// Work item of a 2D translation work-group: R rows a' starting at ap0 and
// the boxes [b0, b0 + nb) of T_K level l, whose nin children start at J0.
struct Item2D {
    int64_t ap0;
    int R, b0, nb, J0, nin;
    int all;  // union of the rows' output bits
};

// Uniform description of work item gid (no memory but the tile record).
__device__ __forceinline__ Item2D item2d(const TArgs &a, int64_t gid)
{
    Item2D it;
    const int64_t g = gid / a.ntile;
    const int tile = (int)(gid - g * a.ntile);
    it.ap0 = g * a.rows;
    it.R = (int)min((int64_t)a.rows, a.nap - it.ap0);
    const int4 bt = a.tiles[tile];
    it.b0 = bt.x;
    it.nb = bt.y - bt.x;
    it.J0 = bt.z;
    it.nin = bt.w - bt.z;
    it.all = 0;
    return it;
}

// Per-work-group tables of a 2D item, filled cooperatively (ends with a
// barrier; sets it.all):
//   s_out[r][t]   output row a of child t of row a' (or -1),
//   s_bits[r]     bit t: child t present; bit 4 + t2: a child with that t2,
//   s_sig[r][ax]  exp(2 pi i rho i_{A'}) per axis (1 when rho = 1),
//   s_pos[j]      child position s of input j of the tile,
//   s_cj[b][s]    local input index of child s of box b (or -1).
template <typename Cv>
__device__ __forceinline__ void tables2d(const TArgs &a, Item2D &it, int *s_out, int *s_bits, Cv *s_sig,
                                         unsigned char *s_pos, signed char *s_cj)
{
    // from the child-position slot words: one load per box and per row
    for (int bl = threadIdx.x; bl < it.nb; bl += kTT) {
        const int kcb = a.k_cb[it.b0 + bl];
        const uint64_t w = a.k_slot[it.b0 + bl];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int o = (int)((w >> (8 * s)) & 0xffu);
            s_cj[bl * 4 + s] = o == 0xff ? (signed char)-1 : (signed char)(kcb + o - it.J0);
            if (o != 0xff) s_pos[kcb + o - it.J0] = (unsigned char)s;
        }
    }
    if ((int)threadIdx.x < it.R) {
        const int r = threadIdx.x;
        const int64_t ap = it.ap0 + r;
        const int xcb = a.x_cb[ap];
        const uint64_t w = a.x_slot[ap];
        int bits = 0;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            const int o = (int)((w >> (8 * t)) & 0xffu);
            s_out[r * 4 + t] = o == 0xff ? -1 : xcb + o;
            if (o != 0xff) bits |= (1 << t) | (1 << (4 + (t >> 1)));
        }
        s_bits[r] = bits;
        Cv one;
        one.x = 1;
        one.y = 0;
        s_sig[r * 2] = a.sig ? cvt<Cv>(a.sig[ap * 2]) : one;
        s_sig[r * 2 + 1] = a.sig ? cvt<Cv>(a.sig[ap * 2 + 1]) : one;
    }
    __syncthreads();
    int all = 0;
    for (int r = 0; r < it.R; ++r) all |= s_bits[r];
    it.all = all;
}

template <typename Cv>
__device__ __forceinline__ Item2D setup2d(const TArgs &a, int64_t gid, int *s_out, int *s_bits,
                                          Cv *s_sig, unsigned char *s_pos, signed char *s_cj)
{
    Item2D it = item2d(a, gid);
    tables2d<Cv>(a, it, s_out, s_bits, s_sig, s_pos, s_cj);
    return it;
}

}  // namespace tr

}  // namespace bfsft
