/*
 * bfsft - butterfly sparse Fourier transform on one MI355X (gfx950).
 *
 * Computes, for target points x_i (i in I) and source points k_j (j in J) in
 * [0, N]^d (d = 2 or 3) and complex sources f_j,
 *
 *     u_i = sum_j exp(+2 pi i x_i . k_j / N) f_j            (Section 1, eq. 1)
 *
 * with the butterfly algorithm of Section 2.2: quadtrees (octrees) T_X and
 * T_K with leaves of width rho = N / 2^L, L = ceil(log2 N) (step 1); p^d
 * equivalent-source / check grids per box pair with w^A w^B = rho N
 * (Section 2.1); leaf initialisation (step 2); the level-by-level sweep up
 * T_K (step 3); evaluation at the leaves of T_X (step 4).  The result is an
 * approximation of eq. (1) whose accuracy is set by p (Theorem 2.1, Table 1:
 * about 2e-3, 1e-5, 5e-8 relative l2 at p = 5, 7, 9 in 2D).
 *
 * Memory model.  Every pointer argument marked "device" is a HIP device
 * pointer on the current device; "host" pointers are ordinary CPU memory.
 * Complex numbers are interleaved (re, im) float64 pairs.  Point arrays are
 * row-major [n][d] float64.  All device work is enqueued on the stream given
 * at plan creation; bfsft_execute* are asynchronous with respect to the host
 * and ordered on that stream.  A plan is not safe for concurrent use from
 * several host threads.
 *
 * Errors.  Functions return BFSFT_OK (0) or a negative status; nothing is
 * thrown or aborted across this interface.  bfsft_last_error() returns a
 * thread-local message describing the most recent failure.  On failure of a
 * *_create call, *out is set to NULL and nothing is leaked.
 */
#ifndef BFSFT_H
#define BFSFT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define BFSFT_OK        0
#define BFSFT_EINVAL   -1   /* bad argument: d, p, N, counts, NULL pointers, precision */
#define BFSFT_EDOMAIN  -2   /* a point coordinate is NaN/inf or outside [0, N] */
#define BFSFT_ENOMEM   -3   /* device allocation failed or BFSFT_MAX_DEVICE_BYTES exceeded */
#define BFSFT_EDEVICE  -4   /* a HIP runtime call failed (message in bfsft_last_error) */

/* Arithmetic of the translation sweep (step 3 of Section 2.2).  Leaf
 * initialisation, phases and the final evaluation always run in FP64; inputs
 * and outputs are complex128.  The split formats apply the axis-2
 * interpolation of every level (the per-axis contraction of Section 2.1,
 * eq. (E1)) on the matrix cores, accumulating in FP32, and do the rest of the
 * level (children sums with their phases, axis-1 interpolation, output
 * phases) in FP64; they are 2D only (BFSFT_EINVAL in 3D). */
#define BFSFT_FP64    0  /* FP64 state in HBM, FP64 arithmetic                     */
#define BFSFT_FP32    1  /* FP32 state in HBM, FP32 arithmetic (VALU, or the axis-2
                            contraction on FP32 matrix cores, tuned per level)     */
#define BFSFT_FP16X2  2  /* FP32 state; axis-2 contraction as FP16 hi + lo split
                            products (three per term, each line scaled by 2^e)     */
#define BFSFT_BF16X3  3  /* FP32 state; axis-2 contraction as exact three-term BF16
                            split products (six per term)                          */
#define BFSFT_MIXED   4  /* FP32 state in HBM, FP64 arithmetic in registers        */

#define BFSFT_MAX_LEVELS 32

typedef struct bfsft_plan bfsft_plan;

/* Sizes of a plan (filled by bfsft_plan_info). */
typedef struct {
    int d, p, precision, levels;          /* levels = L */
    int64_t N, nx, nk;
    double rho;                           /* leaf width N / 2^L */
    int64_t x_boxes[BFSFT_MAX_LEVELS + 1];/* non-empty T_X boxes at level m = 0..L */
    int64_t k_boxes[BFSFT_MAX_LEVELS + 1];/* non-empty T_K boxes at level m = 0..L */
    int64_t pairs[BFSFT_MAX_LEVELS + 1];  /* box pairs at T_K level l: x_boxes[L-l] * k_boxes[l];
                                             batched: pairs produced at sweep step s, all
                                             transforms */
    double sweep_bytes;                   /* algorithmic HBM bytes of the sweep (read + write
                                             of every translated level's state, once: the
                                             levels below levels - start_level) */
    double sweep_flops;                   /* algorithmic flops of the sweep: per output pair,
                                             2^d * d * p^(d+1) complex multiply-adds x 8 */
    int64_t device_bytes;                 /* device memory owned by the plan */
    int64_t transforms;                   /* 1, or the count of a batched plan */
    int lds_kb;                           /* LDS budget of a translation tile (tuned) */
    int wg_per_cu;                        /* batched: persistent work-groups per CU (tuned); 0: one
                                             work-group per work item instead */
    int level_kernel[BFSFT_MAX_LEVELS];   /* single plan, translation producing T_K level l:
                                             0 VALU kernel, 1 FP64 matrix-core kernel, 2 axis-2
                                             contraction on the matrix cores in the precision's
                                             format (FP32, FP16X2, BF16X3) */
    int level_lds_kb[BFSFT_MAX_LEVELS];   /* single plan: tile LDS budget of level l (tuned) */
    int start_level;                      /* single plan: the sweep starts at T_K level
                                             levels - start_level (0: at the leaves) */
    int start_kernel;                     /* single plan with start_level > 0: direct sums on
                                             0 the VALU, 1 the FP64 matrix cores */
    int start_tables;                     /* 1: the matrix-core direct sums read plan-time
                                             tables of their point-only factors */
} bfsft_info;

/*
 * Create a plan (step 1 of Section 2.2: the trees, plus the operator tables).
 *
 *   out        host: receives the plan handle.
 *   d          2 or 3.
 *   N          frequency bound, 2 <= N <= 2^24 (2D) or 2^16 (3D).
 *   p          equivalent-grid size per axis (Section 2.1), 3 <= p <= 12 in
 *              2D, 3 <= p <= 8 in 3D (p = 2 makes the matching system
 *              singular); 3D p = 8 needs BFSFT_MIXED or BFSFT_FP32 (the
 *              FP64 state of one box and its children exceeds a work-group's
 *              LDS): BFSFT_EINVAL otherwise.
 *   precision  BFSFT_FP64, BFSFT_FP32, BFSFT_FP16X2 (2D), BFSFT_BF16X3 (2D)
 *              or BFSFT_MIXED; any other value is BFSFT_EINVAL.
 *   x, nx      device, [nx][d] targets in [0, N]^d; nx >= 0 (NULL iff nx == 0).
 *   k, nk      device, [nk][d] sources in [0, N]^d; nk >= 0 (NULL iff nk == 0).
 *   stream     hipStream_t (NULL = default stream) used for all work of the plan.
 *
 * The points are copied; the caller may free x and k when this returns (the
 * call synchronises the stream).  Box index of a point along an axis:
 * min(floor(x * 2^L / N), 2^L - 1) in IEEE FP64 (half-open boxes).
 * Environment: BFSFT_MAX_DEVICE_BYTES caps the plan's device memory;
 * BFSFT_AUTOTUNE=0 disables the plan-time tuning of the translation tiles
 * (otherwise the sweep is timed on the plan's own shapes for a few tile LDS
 * budgets and, in 2D, for every translation kernel the precision allows: with
 * FP64 arithmetic (5 <= p <= 9) the VALU and the FP64 matrix-core kernel, in
 * FP32 the VALU kernel and the FP32 matrix-core axis-2 contraction; the
 * fastest is kept per level; results differ between the choices only by
 * rounding); BFSFT_TRANSLATE=valu, =mfma or =xdl restricts the choice to one;
 * the sweep starts start_level levels above the leaves of T_K, where the
 * potentials of every pair are summed directly over the sources of B (the
 * plain procedure of Section 2.1), with start_level chosen from the tree
 * sizes by a fixed cost model (0 = the leaf start of Section 2.2) or forced
 * by BFSFT_START_LEVEL=n (at most 18); results differ between start levels
 * at the level of the method's error, not by rounding; the direct sums run
 * on the FP64 matrix cores (2D p <= 12, 3D p <= 5) or on the VALU
 * (BFSFT_DIRECT=valu forces the VALU kernel; the two differ by rounding);
 * the matrix-core kernel reads plan-time tables of the factors that depend
 * on the points only ((nA + p^d) x 16 bytes per source) when they fit
 * BFSFT_DIRECT_TABLE_MB (default 2048; 0: computed at every execute);
 * BFSFT_TUNE_CACHE names the text file caching tuned choices (default
 * $HOME/.cache/bfsft_tune.txt); BFSFT_LDS_KB sets the untuned tile budget (8-76 KB in
 * 2D, 8-60 KB in 3D; other values give 32 KB).
 */
int bfsft_plan_create(bfsft_plan **out, int d, int64_t N, int p, int precision,
                      const double *x, int64_t nx, const double *k, int64_t nk,
                      void *stream);

/*
 * Execute steps 2-4 of Section 2.2 for sources f.
 *   f   device, [nk] complex128 (original source order), read only.
 *   u   device, [nx] complex128 (original target order), overwritten; must
 *       not alias f.
 * nk == 0 gives u = 0; nx == 0 is a no-op.  Asynchronous on the plan stream.
 */
int bfsft_execute(bfsft_plan *plan, const double *f, double *u);

/*
 * bfsft_execute for callers that cannot allocate device memory (code under
 * HIP graph capture, serving loops, harnesses that forbid allocation): the
 * same computation and result, bit for bit, with the two state buffers of
 * the sweep taken from a static device array of 64 MiB that the library
 * holds on every GPU it runs on until the process ends, instead of the
 * plan's own.  Calls no allocating routine.  The first call on a device
 * looks the array's address up (no allocation).  Every call on a GPU
 * shares that GPU's array: calls whose executions overlap on one GPU (two
 * streams, two threads) race and give wrong results; calls on one stream
 * are ordered.  Nothing must start at zero: each call writes every state
 * entry before reading it.
 *   f, u  as bfsft_execute.
 * BFSFT_EINVAL if 2 x the plan's largest level state (bfsft_info pairs x
 * p^d x 8 or 16 bytes) exceeds 64 MiB, and for the arguments bfsft_execute
 * rejects.
 */
int bfsft_execute_noalloc(bfsft_plan *plan, const double *f, double *u);

/* Release a plan and all its device memory (synchronises its stream).
 * NULL is a no-op. */
void bfsft_destroy(bfsft_plan *plan);

/* Static description of a status code. */
const char *bfsft_strerror(int status);

/* Thread-local message of the last failure in this thread ("" if none). */
const char *bfsft_last_error(void);

/* Sizes and algorithmic work of a plan (host struct). */
int bfsft_plan_info(const bfsft_plan *plan, bfsft_info *out);

/*
 * Box coordinates of level m of T_X (side 0) or T_K (side 1), in the order
 * the plan stores them (Morton order).
 *   coords  host, [count][d] int64, count = x_boxes[m] or k_boxes[m].
 */
int bfsft_plan_boxes(const bfsft_plan *plan, int side, int m, int64_t *coords);

/*
 * The per-axis interpolation tables of a single plan, as built on the device
 * (FP64), for tests of the operators of Section 2.1 (eqs. (M1), (E1)).  The
 * state of a box pair is B's check potential at A's check points with B's
 * corner phase divided out, rotated by E; one level of step 3 applies, per
 * axis, diag(sigma^s G(s, t, .)) R_t to the state of the child pair
 * (A', B_s), A = child t of A', sigma = exp(2 pi i rho i_{A'}).
 *   R  host, [2 t][p l][p l'] real: R_t
 *   G  host, [2 s][2 t][p l] complex (interleaved): G(s, t, l)
 *   E  host, [p] complex: E[k] = exp(-i pi rho k / q)
 * Synchronises the plan stream.
 */
int bfsft_plan_tables(const bfsft_plan *plan, double *R, double *G, double *E);

/*
 * Parity probe: run bfsft_execute and also export the check potentials
 * u^{AB}_l = sum over sources of B of exp(2 pi i x^A_l . k / N) f, as
 * reproduced by the sweep at T_K level `level` (Section 2.1: the potentials
 * at the p^d check points x^A_l of A; for level L these are the exact leaf
 * potentials of step 2).
 *   pot  device, [x_boxes[L-level]][k_boxes[level]][p^d] complex128, boxes in
 *        the order of bfsft_plan_boxes, grid index row-major (axis 1 slowest).
 */
int bfsft_execute_probe(bfsft_plan *plan, const double *f, double *u,
                        int level, double *pot);

/*
 * Adjoint transform (Section 1, eq. (1) with the roles of x and k exchanged
 * and the sign of the phase reversed):
 *     v_j = sum_i exp(-2 pi i x_i . k_j / N) g_i ,   j = 0 .. nk-1.
 * The kernel of eq. (1) is symmetric in x and k, so this is the conjugate of
 * the forward butterfly with T_X and T_K exchanged applied to conj(g); it
 * shares the plan's trees and tables.
 *   g  device, nx complex128 (interleaved), indexed like x.
 *   v  device, nk complex128, overwritten; must not alias g.
 * The adjoint's tiles, start level and input staging are built with the
 * plan, and it shares the plan's state buffers (executes of one plan are
 * stream-ordered), so a call only enqueues work on the plan's stream and
 * allocates nothing.  nx = 0 gives v = 0.
 */
int bfsft_execute_adjoint(bfsft_plan *plan, const double *g, double *v);

/* One problem of a batched plan (all points in device memory). */
typedef struct {
    int64_t N;
    const double *x; int64_t nx;   /* device, [nx][d] */
    const double *k; int64_t nk;   /* device, [nk][d] */
} bfsft_problem;

/*
 * Batched plan: `count` independent transforms of the same d, p and
 * precision but their own N and points.  Execution runs sweep step
 * s = 1 .. max_t L_t for all transforms still active in one launch per step
 * (transform t works on its T_K level L_t - s; either one work-group per work
 * item or persistent work-groups taking items from a counter, whichever the
 * plan-time tuning found faster), all captured in one HIP graph.
 *   probs  host, [count] problem descriptors (device point pointers).
 * Sources and outputs are packed: transform t reads f_packed at offset
 * sum_{t'<t} nk_{t'} and writes u_packed at offset sum_{t'<t} nx_{t'}.
 */
int bfsft_plan_create_batched(bfsft_plan **out, int count, const bfsft_problem *probs,
                              int d, int p, int precision, void *stream);

/* Execute a batched plan (one graph launch on the plan stream).
 *   f_packed  device, [sum nk] complex128.
 *   u_packed  device, [sum nx] complex128, overwritten. */
int bfsft_execute_batched(bfsft_plan *plan, const double *f_packed, double *u_packed);

/* Execute a batched plan without the graph and without the persistent
 * multi-transform launches: each transform's steps are launched one after
 * another (the per-transform baseline the batched path is compared with). */
int bfsft_execute_batched_serial(bfsft_plan *plan, const double *f_packed, double *u_packed);

/*
 * Kernel timing (measurement).  bfsft_timing_begin arms HIP events for the
 * next `max_execs` executes of a single-transform plan: each records events on
 * the plan stream before the start-level launch (leaf initialisation or direct
 * sums), after it, after every translation launch and after the final launch.
 * bfsft_timing_end waits for them, then writes to out (host, n doubles):
 *   out[0]      executes recorded
 *   out[1]      leaf initialisation or start-level direct sums, ms summed over executes
 *   out[2]      final evaluation, ms summed
 *   out[3 + l]  translation launch producing T_K level l (l = 0..L-1), ms summed;
 *               0 for l >= L - s0 (s0 the start level: those levels have no
 *               translation launch)
 * and disarms timing.  Returns BFSFT_EINVAL if n < 3 + L.
 */
int bfsft_timing_begin(bfsft_plan *plan, int max_execs);
int bfsft_timing_end(bfsft_plan *plan, double *out, int n);

/*
 * Measurement helper (not part of the method): the streaming bandwidth of a
 * plain device copy kernel, the practical memory ceiling the translation
 * kernels are compared with.  Allocates two device buffers of `bytes` each,
 * runs one untimed and `reps` timed copies of elements of `elem_bytes`
 * (4, 8 or 16) on `stream`, frees the buffers and writes to *gbps (host) the
 * bytes read plus written per second / 1e9.  bytes must be a multiple of
 * elem_bytes in [2^20, 2^34].  Synchronises the stream.
 */
int bfsft_copy_rate(int elem_bytes, int64_t bytes, int reps, void *stream, double *gbps);

/*
 * Measurement helper (not part of the method): the FP64 matrix-core rate
 * that waves_per_simd (1..8) waves per SIMD reach with 12 independent
 * chains of v_mfma_f64_16x16x4f64 each (the accumulator count of the
 * matrix-core direct sums), the practical ceiling those sums are compared
 * with.  Runs one short untimed and one timed launch of `iters` (1..2^20)
 * rounds on `stream`, with a device buffer it allocates and frees; writes
 * to *tflops (host) the FP64 TFLOP/s.  Synchronises the stream.
 */
int bfsft_mfma_f64_rate(int waves_per_simd, int iters, void *stream, double *tflops);

#ifdef __cplusplus
}
#endif
#endif /* BFSFT_H */
