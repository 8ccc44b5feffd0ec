/*
 * fcc_dct.h -- C ABI of the MI355X (gfx950) fast FCC cosine transform.
 *
 * The transform (Seifert, Hueper, Uhl, "Fast cosine transform for FCC
 * lattices", Sec. IV-A, Definition 2 and eq. SU4ChebyshevTransformExplicitForm):
 *
 *     X[j] = sum_{k in [0,n)^3} T_k(theta_j) x[k],   theta_j = ((r,s,t) + j) / n,
 *
 * where T_k are the three-variable Chebyshev polynomials of the Weyl group
 * S_4 (Sec. III, Definition 1) and the rows j are the common zeros of the
 * skew ideal (Lemma 2).  The default skew (r,s,t) = (1/8, 0, 3/8) gives the
 * FCC cosine transform DCT_{n x n x n}.  Input x holds the coefficients of the
 * basis b_n = (T_k | k in [0,n)^3) (eq. ZTransformFCC); output X holds the
 * values at the zeros.  Both are flattened lexicographically:
 * (a,b,c) -> (a*n + b)*n + c.  No normalisation is applied; the inverse is the
 * exact matrix inverse (the matrix is not unitary).
 *
 * The fast path is the radix-2x2x2 factorisation of Sec. IV-B (eq.
 * FastAlgorithm), applied level by level:
 *     DCT_n(r,s,t) = P_n (+)_i DCT_{n/2}(((r,s,t)+i)/2) (DCT_2(r,s,t) (x) I) B_n(r,s,t).
 * It needs n = 2^d (Sec. IV-B).
 *
 * Conventions for every call:
 *   - Data pointers are DEVICE pointers (hipMalloc'd memory or torch tensors),
 *     at least 16-byte aligned, owned by the caller.  Calls are out of place:
 *     input and output must not overlap.
 *   - Real arrays hold n^3 elements; complex arrays hold n^3 interleaved
 *     (re, im) pairs.  The element type is set by the plan's precision:
 *       FCC_PREC_FP64                    : double / double2
 *       FCC_PREC_FP32, FCC_PREC_SPLIT_*  : float  / float2
 *   - `hip_stream` is a hipStream_t (NULL = the default stream).  Calls only
 *     enqueue work on it and never synchronise; errors raised by kernels show
 *     up at the caller's next synchronisation.
 *   - Every call returns a status and never throws.  A plan executes on one
 *     stream at a time (it owns scratch buffers).
 *   - Debugging: with the environment variable FCC_POISON_SCRATCH set (and
 *     not "0") when a plan or a batched call allocates scratch, the scratch
 *     starts as all-ones bytes (NaN in FP32 and FP64) instead of unspecified
 *     contents; results are unchanged unless a kernel reads scratch it did
 *     not write.  FCC_FAIL_ALLOC_AT=k makes the k-th device allocation of the
 *     library (counted from when the variable last changed) fail as out of
 *     memory, for testing the error paths: the call returns FCC_ERR_OOM and
 *     frees what it had allocated.
 */
#ifndef FCC_DCT_H
#define FCC_DCT_H

#ifdef __cplusplus
extern "C" {
#endif

typedef struct fcc_plan_s* fcc_plan_t;

typedef enum {
  FCC_OK = 0,
  FCC_ERR_INVALID_ARG = 1,   /* null or misaligned pointer, bad count/direction   */
  FCC_ERR_NOT_POW2 = 2,      /* n is not a power of two in [1, 1024]              */
  FCC_ERR_SINGULAR_SKEW = 3, /* (r,s,t) gives coinciding zeros somewhere in the tree */
  FCC_ERR_OOM = 4,           /* device or host allocation failed                   */
  FCC_ERR_HIP = 5,           /* a HIP runtime call failed                          */
  FCC_ERR_UNSUPPORTED = 6    /* valid request the library does not serve (a size or flag combination) */
} fcc_status;

typedef enum {
  FCC_PREC_FP64 = 0,       /* FP64 data, FP64 stages                                */
  FCC_PREC_FP32 = 1,       /* FP32 data; stage precision chosen by the plan (below) */
  FCC_PREC_SPLIT_BF16 = 2, /* FP32 data; dense base on MFMA, split hi+lo BF16, FP32 acc */
  FCC_PREC_SPLIT_FP16 = 3  /* FP32 data; dense base on MFMA, split hi+lo FP16, FP32 acc */
} fcc_precision;

enum {
  /* Forward input is real (n^3 reals); the inverse then writes the real part. */
  FCC_REAL_INPUT = 1u << 0,
  /* Force FP32 intermediate stages for FCC_PREC_FP32 (fast, but the skew
   * sub-transforms lose accuracy with depth; see the plan's error model).      */
  FCC_STAGES_FP32 = 1u << 1,
  /* Force FP64 intermediate stages for FCC_PREC_FP32.                          */
  FCC_STAGES_FP64 = 1u << 2,
  /* FCC_PREC_FP32 with FP64 stages: run the top level (and the inverse's last
   * level) in FP32 arithmetic with a complex64 intermediate.  Faster top level;
   * round-trip error ~4e-6 instead of ~5e-8 at n = 32..128.                    */
  FCC_LEVEL0_FP32 = 1u << 3,
  /* The transposed transform, the literal reading of the row/column labels
   * after eq. SU4ChebyshevTransformExplicitForm: forward X[k] =
   * sum_j T_k(theta_j) x[j] (input indexed by the zeros, output by the
   * basis), inverse its exact inverse.  Runs the factors of eq. FastAlgorithm
   * transposed, in reverse order (orbit-block launches at every level with
   * node size >= 4, then DCT_2^T per cube).  FP64 or FP32 data, n <= 256;
   * not with FCC_LEVEL0_FP32, FCC_HERMITIAN_PACKED or the split precisions. */
  FCC_TRANSPOSED = 1u << 4,
  /* With FCC_REAL_INPUT: the spectrum of real input in Hermitian-packed form.
   * The zeros pair up as j' = (c - g^T j) mod n with X[j'] = conj X[j] (g in W
   * and c fixed by the skew; the conjugation symmetry of Sec. III); the forward
   * writes one value per pair (the member with the smaller flat index) and
   * the self-paired zeros, in increasing flat index: fcc_dct_packed_size
   * values.  The inverse reads that form.  Skews without such a pairing return
   * FCC_ERR_UNSUPPORTED; fcc_dct_batched does not take these plans. */
  FCC_HERMITIAN_PACKED = 1u << 5,
  /* A variant, not the paper's factorisation: the same transform through the
   * fold+FFT form that follows from the explicit matrix (Sec. IV-A, eq.
   * SU4ChebyshevTransformExplicitForm, with the two sums exchanged):
   * X = N IDFT_3(Fh), Fh[mu] = (1/24) sum_{g kappa = mu mod n} x[kappa]
   * exp(2 pi i (g kappa).rst / n); the inverse takes Fh = DFT_3(X) / N and
   * undoes the fold orbit by orbit (the Gram blocks of the fold).  All
   * arithmetic in the data precision (FCC_PREC_FP32 runs FP32 throughout).
   * Needs 8 rst integral (the default skew is); FP64 or FP32; n <= 512; not
   * with the other flags except FCC_REAL_INPUT. */
  FCC_FOLD_FFT = 1u << 6,
  /* Hybrid depth (Sec. IV-B, the stepwise decomposition with n = 2^Lt M):
   * the forward runs the radix-2 levels down to node size M and then, per
   * node J of level Lt, the dense DCT_M(phi_J), phi_J = ((r,s,t) + J) / 2^Lt,
   * as a twiddled fold onto the M-torus and a DFT_M^3 shared by all nodes
   * (the explicit form of Sec. IV-A at the node's skew), one LDS-resident
   * launch.  M = 2^tail_levels[0] of the schedule (4, 8 or 16, at most
   * n / 2; default min(16, n / 2)).  The inverse is unchanged (the radix-2
   * levels; the fold at a node skew has dense orbit blocks up to 24 x 24).
   * Stage precision as without the flag.  Needs 8 rst integral and
   * 8 <= n <= 1024 (else FCC_ERR_UNSUPPORTED); not with FCC_TRANSPOSED,
   * FCC_FOLD_FFT or the split precisions.  A schedule with tail_levels[0]
   * outside 2..log2(n) - 1 is FCC_ERR_INVALID_ARG. */
  FCC_FOLD_BASE = 1u << 7
};

/* Build a plan for DCT_{n x n x n}(r,s,t) (Definition 2).
 *   plan  : receives the new plan (set to NULL on failure).
 *   n     : size parameter, a power of two in [1, 1024] (fast algorithm, Sec. IV-B).
 *           Levels with node size above 256 run as orbit-block launches
 *           (the per-row gather tables pack node-local coordinates in 8
 *           bits); the default schedule has them at every node size >= 16.
 *   rst   : host pointer to the skew (r,s,t), or NULL for (1/8, 0, 3/8).
 *   prec  : data/compute precision (fcc_precision).  The split-MFMA precisions
 *           apply the dense transform matrix and need n <= 8.
 *   flags : FCC_REAL_INPUT | FCC_STAGES_FP32 | FCC_STAGES_FP64 | FCC_LEVEL0_FP32 |
 *           FCC_TRANSPOSED | FCC_HERMITIAN_PACKED | FCC_FOLD_FFT | FCC_FOLD_BASE.
 * Derives the basis-change patterns on the host (cached per node size),
 * uploads them, generates FP64 tables on the GPU on `hip_stream`, allocates
 * scratch, and synchronises `hip_stream` once before returning.
 * Errors: FCC_ERR_NOT_POW2, FCC_ERR_SINGULAR_SKEW, FCC_ERR_INVALID_ARG,
 * FCC_ERR_UNSUPPORTED (split precisions with n > 8, the flag limits above),
 * FCC_ERR_OOM,
 * FCC_ERR_HIP. */
fcc_status fcc_dct_plan(fcc_plan_t* plan, int n, const double rst[3], fcc_precision prec,
                        unsigned flags, void* hip_stream);

/* X = DCT_n(r,s,t) x  (eq. FastAlgorithm applied recursively, output
 * permutation P_n folded into the addressing).
 *   x : n^3 reals (FCC_REAL_INPUT) or complex; X : n^3 complex. */
fcc_status fcc_dct_forward(fcc_plan_t plan, const void* x, void* X, void* hip_stream);

/* fcc_dct_forward for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same kernels and result bits, but the two scratch buffers come from a
 * static device array of 8 MiB per device instead of the plan's buffers, and
 * the call makes no allocation of any kind.
 *   plan : a plan made on the current device (its set-up looked up the
 *          array's address on that device).
 *   x, X : as for fcc_dct_forward (device pointers, 16-byte aligned, disjoint).
 * Limit: 2 n^3 stage-precision complex values must fit in 8 MiB, i.e.
 * n <= 64 (FP64 or FP32 stages); larger n returns FCC_ERR_UNSUPPORTED.  Dense
 * (split-MFMA) plans keep their per-row scale there too.
 * Every call on one device shares that device's array, which keeps the last
 * call's contents (no call needs it cleared): calls that overlap in time on one
 * device (two streams, two threads) race and give wrong results.
 * Errors: FCC_ERR_INVALID_ARG (null or misaligned pointers, current device is
 * not the plan's), FCC_ERR_UNSUPPORTED (in place, n above the limit),
 * FCC_ERR_HIP (the array's address could not be looked up). */
fcc_status fcc_dct_forward_static(fcc_plan_t plan, const void* x, void* X, void* hip_stream);

/* x = DCT_n(r,s,t)^{-1} X: the factors of eq. FastAlgorithm inverted in reverse
 * order (P_n^T, inverse skew sub-transforms, DCT_2^{-1} (x) I, then the
 * product expansion C_n = B_n^{-1}).
 *   X : n^3 complex; x : n^3 complex, or the real part only (FCC_REAL_INPUT). */
fcc_status fcc_dct_inverse(fcc_plan_t plan, const void* X, void* x, void* hip_stream);

/* Many independent transforms in one call; plans may differ in n.
 *   plans[i], in[i], out[i] for i < count; direction +1 forward (in -> out),
 *   -1 inverse (in -> out), 0 forward then inverse (in -> out, then out -> in,
 *   overwriting in[i] with the round trip).
 * The first call with a given (plans, pointers, direction) records the launch
 * sequence into a HIP graph; later identical calls replay it (at most 4
 * recorded graphs are kept, least recently used freed first; see
 * fcc_dct_batched_release).  Volumes with the same plan configuration form a
 * group and share each level launch, in chunks of up to 2^25 points that
 * reuse one scratch pair; groups run on up to 4 concurrent branches of the
 * graph.  Calls that overlap in time must not pass the same buffers.
 * Errors: FCC_ERR_INVALID_ARG (count < 1, null entries, direction), plus the
 * errors of the single-volume calls. */
fcc_status fcc_dct_batched(const fcc_plan_t* plans, int count, const void* const* in,
                           void* const* out, int direction, void* hip_stream);

/* Number of complex values in the forward output of a plan: n^3, or the
 * packed count with FCC_HERMITIAN_PACKED.  Errors: FCC_ERR_INVALID_ARG. */
fcc_status fcc_dct_packed_size(fcc_plan_t plan, long long* count);

/* Host-only (no device call): the unfold tables of the FCC_FOLD_FFT inverse
 * for size n and skew rst (8 rst integral).  Point k (flat index) has the row
 * K[pid[k]] of 24 complex values, one per element u of W (in the closure order
 * of the generators of eq. GeneratorMatricesS4, identity first), and
 *   x[k] = sum_u K[pid[k]][u] exp(-2 pi i (u k).rst / n) Fh[u k mod n],
 *   Fh = DFT_3(X) / n^3,
 * inverts the transform.  pid: n^3 bytes; K: 256 * 24 * 2 doubles
 * (interleaved complex), caller-owned; *npat receives the number of rows.
 * Errors: FCC_ERR_INVALID_ARG (null pointers, n not a power of two <= 1024),
 * FCC_ERR_UNSUPPORTED (8 rst not integral, more than 256 distinct rows),
 * FCC_ERR_SINGULAR_SKEW (a singular block), FCC_ERR_OOM. */
fcc_status fcc_fold_unfold_tables(int n, const double rst[3], unsigned char* pid, double* K, int* npat);

/* Free every graph (and its scratch) that fcc_dct_batched has recorded.  At
 * most 4 are kept anyway (the least recently used is freed when a new one is
 * recorded); this releases them at once.  Waits for the device first.
 * Errors: FCC_ERR_HIP. */
fcc_status fcc_dct_batched_release(void);

/* Free the plan's device tables, scratch and cached graphs.  NULL is a no-op. */
fcc_status fcc_dct_destroy(fcc_plan_t plan);

/* Static description of a status code. */
const char* fcc_status_string(fcc_status s);

/* ---- schedule tuning ---------------------------------------------------- */

/* How a plan schedules the levels of eq. FastAlgorithm on the GPU.  Tiles,
 * block numbering and node groups change no result bit (every output row is
 * summed in the same order).  A different tail depth, FCC_MAP_SPLIT or
 * FCC_MAP_BALANCE evaluates the same expressions, at the same stage
 * precision, in another kernel or order and may differ in the last bits.  Index [0] is the forward
 * transform, [1] the inverse.
 *   tail_levels[d] : the last 1..4 levels (node sizes <= 2^tail_levels) run
 *                    fused in one launch with the data resident in LDS (the
 *                    last level alone, where B_2 = C_2 = I, is a per-cube
 *                    DCT_2 pass).
 *   tile[d][L][.]  : at levels L = 0, 1 the gather pass of the basis change
 *                    walks the cubes of a node in tiles of 2^t0 x 2^t1 x 2^t2
 *                    cubes (log2 sizes; {0,0,0} = plain lexicographic order).
 *                    Each side is clamped to the node's n / 2^(L+1) cubes.
 *   map[d][L]      : thread map of the gather pass at level L = 0..9.
 *                    FCC_MAP_XCD numbers the blocks so that each XCD takes one
 *                    contiguous range of rows; FCC_MAP_XCD16 gives each XCD
 *                    runs of 16 consecutive blocks instead (it takes precedence over
 *                    FCC_MAP_XCD).  FCC_MAP_F_INNER puts the 8 rows
 *                    of a cube next to each other (otherwise the row's position
 *                    in its cube is the slowest index).  From level 2 on,
 *                    FCC_MAP_NODES8 / FCC_MAP_NODES64 run all rows of an
 *                    aligned group of 8 / 64 consecutive nodes before the next
 *                    group (otherwise all nodes of one row run together); the
 *                    tile and the node-group bits are ignored where they do
 *                    not apply.  Forward levels run the basis change and
 *                    DCT_2 (x) I in one launch, the 8 rows of each cube on 8
 *                    adjacent lanes (FCC_MAP_F_INNER is implied there);
 *                    FCC_MAP_SPLIT runs them as two launches instead (gather,
 *                    then DCT_2 on the cubes).  The inverse always uses two.
 *                    FCC_MAP_BALANCE (two-pass gathers only) sums each long
 *                    row on 2 or 4 adjacent lanes (by the mean row length of
 *                    its position in the cube) and adds the parts; it changes
 *                    the summation order, so results may differ in the last
 *                    bits.  It takes precedence over FCC_MAP_F_INNER.
 *                    FCC_MAP_CLUSTER (gather passes at levels 0 and 1 where
 *                    the node has a multiple of 4 slices of cubes) runs the
 *                    slices in blocks of 4, the 8 f of a block one after the
 *                    other, and orders the slices so that the cubes of one
 *                    block of B_nl (C_nl) run together: a block is an orbit
 *                    of (generically) 24 cubes whose rows read the same
 *                    sources and no others, so with FCC_MAP_XCD or
 *                    FCC_MAP_XCD16 those sources are fetched into one XCD's
 *                    L2 once.  It takes precedence over FCC_MAP_F_INNER and
 *                    FCC_MAP_BALANCE and changes no result bit.
 *                    FCC_MAP_ORBIT (node sizes n / 2^L >= 8) runs the
 *                    level as one launch over the orbits of W on the node's
 *                    cube grid: a block loads the sources of 1 to 64 orbits
 *                    of one kind (fewer the more cubes an orbit has) once,
 *                    forms their rows from the kind's template (the
 *                    basis change is block diagonal over the orbits) and
 *                    applies DCT_2 (x) I (inverse: DCT_2^{-1} (x) I, then C)
 *                    before storing; no per-row table is read.  It takes
 *                    precedence over every other bit of the level.  Plans with
 *                    n > 256 need it on every level with node size >= 32 in
 *                    both directions (the per-row tables pack coordinates in
 *                    8 bits). */
enum {
  FCC_MAP_XCD = 1u << 0,
  FCC_MAP_F_INNER = 1u << 1,
  FCC_MAP_NODES8 = 1u << 2,
  FCC_MAP_NODES64 = 1u << 3,
  FCC_MAP_SPLIT = 1u << 4,
  FCC_MAP_BALANCE = 1u << 5,
  FCC_MAP_XCD16 = 1u << 6,
  FCC_MAP_CLUSTER = 1u << 7,
  FCC_MAP_ORBIT = 1u << 8
};
typedef struct {
  int tail_levels[2];
  int tile[2][2][3];
  unsigned map[2][10];
} fcc_tuning;

/* fcc_dct_plan with an explicit schedule.  tuning == NULL takes the schedule
 * fcc_dct_plan would take (see fcc_dct_autotune).  Errors: those of
 * fcc_dct_plan, and FCC_ERR_INVALID_ARG for tail_levels outside 1..4, a tile
 * size outside 0..9, unknown map bits or both node-group bits. */
fcc_status fcc_dct_plan_tuned(fcc_plan_t* plan, int n, const double rst[3], fcc_precision prec,
                              unsigned flags, const fcc_tuning* tuning, void* hip_stream);

/* The schedule a plan runs with. */
fcc_status fcc_dct_get_tuning(fcc_plan_t plan, fcc_tuning* out);

/* Search the schedule for (n, prec, flags) on the current device: the fused
 * tail depth of each direction first (whole-transform time), then tile shape
 * and thread map of each gather pass one level at a time (time of that
 * launch), each candidate timed `reps` times on synthetic data
 * with HIP events on `hip_stream`.  The winner is written to *best (may be
 * NULL) and remembered for the process: later fcc_dct_plan calls for the same
 * (device, n, prec, flags) use it.  With the environment variable
 * FCC_AUTOTUNE_CACHE naming a file, the winner is also appended to that file
 * (one text line, tagged with the device's architecture), and each process
 * reads the file at its first plan on a device, so searches persist across
 * processes (later lines win; unreadable or malformed lines are skipped).  Without a search, fcc_dct_plan uses
 * built-in defaults.  Allocates and frees its own buffers and synchronises
 * `hip_stream`.  Errors: those of fcc_dct_plan, FCC_ERR_INVALID_ARG for
 * reps < 1. */
fcc_status fcc_dct_autotune(int n, const double rst[3], fcc_precision prec, unsigned flags, int reps,
                            fcc_tuning* best, void* hip_stream);

/* ---- measurement ------------------------------------------------------- */

/* Per-launch timing of one direction of the fast path: enqueues `reps`
 * transforms of `in` into `out` (direction +1 forward, -1 inverse) on
 * `hip_stream`, each kernel launched with its own start and stop event
 * (recorded at the kernel's start and end), waits for them, and writes the
 * average duration in ms of each launch slot to ms[k].
 * Slots in launch order, with Lt = D - tail_levels (at least 0) of the
 * direction: forward = for levels 0..Lt-1 one slot (one-pass level) or two
 * (FCC_MAP_SPLIT: gather pass, DCT_2 pass), then the fused tail (with fused depth 1 after
 * a two-pass level D - 2, n >= 8, that level's DCT_2 pass and the last level are one slot);
 * inverse = the fused tail, then (DCT_2^{-1} pass, C gather
 * pass) for levels Lt-1 down to 0 (with fused depth 1, n >= 8, the last level
 * and the DCT_2^{-1} pass of level D - 2 are one slot, and for n >= 16 that
 * slot also does level D - 2's C gather).  Orbit-block levels are one slot.  n = 1 and the dense precisions have one
 * slot.  *count receives the number of slots; with ms == NULL only *count is
 * set.
 * Errors: FCC_ERR_INVALID_ARG (cap too small, bad pointers or direction),
 * FCC_ERR_HIP. */
fcc_status fcc_dct_time_launches(fcc_plan_t plan, const void* in, void* out, int direction, int reps,
                                 float* ms, int cap, int* count, void* hip_stream);

/* One launch slot of a transform: kernel and level(s), the points it covers,
 * and the algorithmic bytes per point it reads and writes -- each element of
 * the method's own input and output once, in the plan's data precision (real
 * 4 or 8 bytes, complex 8 or 16), whatever the stage precision. */
typedef struct {
  char name[64];
  long long points;
  int in_bytes, out_bytes;
} fcc_launch_info;

/* The launch slots of one transform in `direction` (+1 forward, -1 inverse),
 * in the order fcc_dct_time_launches reports them.  *count receives their
 * number; info (may be NULL) receives up to cap entries.
 * Errors: FCC_ERR_INVALID_ARG (bad plan or direction, cap too small). */
fcc_status fcc_dct_describe_launches(fcc_plan_t plan, int direction, fcc_launch_info* info, int cap, int* count);

/* Per-launch timing of fcc_dct_batched's work: the same groups (volumes with
 * the same plan configuration) and chunks of volumes, enqueued eagerly on
 * `hip_stream` one group after the other, `reps` times, each kernel between
 * its own start and stop events.  ms[k] receives the average duration of slot
 * k and info[k] (may be NULL) its description, named "n<n> x<volumes> <kernel
 * and levels>"; *nslots receives the slot count (with ms == NULL only that is
 * set).  direction as for fcc_dct_batched (0 overwrites in[i] with the round
 * trip).  Allocates and frees its own scratch and waits for `hip_stream`.
 * Errors: those of fcc_dct_batched, FCC_ERR_INVALID_ARG (cap too small, reps < 1). */
fcc_status fcc_dct_batched_time_launches(const fcc_plan_t* plans, int count, const void* const* in,
                                         void* const* out, int direction, int reps, float* ms,
                                         fcc_launch_info* info, int cap, int* nslots, void* hip_stream);

/* FP64 round-trip residual on the GPU: *result = max_k |x_k - y_k| / max_k |x_k|
 * over the plan's n^3 elements, x and y laid out like the forward input
 * (real with FCC_REAL_INPUT, else complex; float or double per precision).
 * Typically y = inverse(forward(x)).  A NaN in x - y counts as an infinite
 * difference, so a round trip that produced NaN never reports a small
 * residual.  Waits for `hip_stream` (the result is a host value).  Errors: FCC_ERR_INVALID_ARG, FCC_ERR_HIP. */
fcc_status fcc_dct_roundtrip_residual(fcc_plan_t plan, const void* x, const void* y, double* result,
                                      void* hip_stream);

/* ---- block-wise coding ------------------------------------------------- */

/* Threshold and quantise FCC spectra for block-wise volumetric coding (the
 * application motivating the transform, Sec. I and Sec. V): for each of
 * `count` complex64 coefficients X[k] (device, interleaved float2),
 *   keep_k = re^2 + im^2 >= threshold^2,
 *   codes[k] = keep_k ? (rint(re / step), rint(im / step)) : (0, 0)  (int16 pairs, saturated),
 *   Xq[k] = step * codes[k]  (the dequantised spectrum, float2),
 * every operation a single FP32 rounding (no fused multiply-add), so the
 * integer decisions are reproducible in any IEEE FP32 arithmetic.  *kept
 * (a device counter, set to zero first) receives the number of kept
 * coefficients.  codes or Xq may be NULL.  Asynchronous on hip_stream.
 * Errors: FCC_ERR_INVALID_ARG (null X or kept, step <= 0, negative or
 * non-finite threshold, misaligned pointers), FCC_ERR_UNSUPPORTED (Xq == X),
 * FCC_ERR_HIP. */
fcc_status fcc_spectrum_quantise(const void* X, long long count, float threshold, float step, void* codes,
                                 void* Xq, unsigned long long* kept, void* hip_stream);

/* ---- introspection (host logic; no GPU needed) ------------------------- */

/* Host view of the basis-change tables for one node size nl = 2m (2 <= nl <= 1024).
 * Gather form, grouped by 2x2x2 cube:
 *   forward (B_nl): row r = cube*8 + d, cube = (a*m+b)*m+c for abc in [0,m)^3,
 *     d = (d0*2+d1)*2+d2 for def in {0,1}^3; the row yields the coordinate of
 *     b~_(def,abc) = T_abc * T_{m*def}, stored at node-local position def + 2*abc.
 *     Entries: source node-local index kappa packed as (kx<<20)|(ky<<10)|kz and a
 *     coefficient-polynomial id.
 *   inverse (C_nl): row r = cube*8 + i, for node-local kappa = i + 2*abc; entries
 *     name the source position def + 2*abc (packed the same way).
 *   Polynomial p has coefficients poly[p*nmono + q] of the monomial
 *     c1^e1 c2^e2 c3^e3 with (e1,e2,e3) = mono[3q..3q+2], c = (sigma,tau,rho)(node).
 *   Blocks of B: cubes whose B rows read a common source are in one block,
 *     and the rows of a block read no source of another block (a generic
 *     block is an orbit of 24 cubes).  Block ids are the smallest cube index
 *     of the block.  C = B^{-1} is block diagonal the other way round: row
 *     kappa of C reads only positions of cubes in block kappa_block[kappa].
 * Pointers stay valid until the process ends.  Returns FCC_ERR_NOT_POW2 for a
 * bad nl, FCC_ERR_OOM if the derivation cannot allocate. */
typedef struct {
  int nl, m, nmono, npoly;
  const int* mono;       /* 3*nmono exponents                      */
  const double* poly;    /* npoly*nmono coefficients               */
  const int* b_rowptr;   /* 8*m^3 + 1                              */
  const unsigned* b_src; /* b_rowptr[8 m^3] packed source indices  */
  const unsigned short* b_pid;
  const int* c_rowptr;   /* 8*m^3 + 1                              */
  const unsigned* c_src;
  const unsigned short* c_pid;
  const int* cube_block;  /* m^3: per cube, the smallest cube of its block of B   */
  const int* kappa_block; /* nl^3: per source kappa, the block that reads it in B */
} fcc_level_tables;

fcc_status fcc_asp_tables(int nl, fcc_level_tables* out);

/* Orbit-block form of the same basis change (node size nl = 2m, 4 <= nl <= 1024).
 * Let W act on the cube grid [0,m)^3 by q -> (g q) mod m.  For each orbit O,
 * the B_nl rows (def, q), q in O, read exactly the sources kappa = q' + m o
 * (q' in O, o in {0,1}^3), and no other rows read them; C_nl = B_nl^{-1} has
 * the same blocks.  Labelled relative to its representative p0 (the orbit's
 * smallest cube index), a block's matrix depends only on the orbit's kind,
 * so a level is described by a few templates and the representatives of
 * each kind:
 *   template t: cube slot j < nc is the cube q_j = (G[w[j]] p0) mod m;
 *     B row j*8 + def gives the coordinate stored at position def + 2 q_j, with
 *       entries (s << 8) | poly reading the source q_{s/8} + m o, o = s % 8
 *       as (o>>2, (o>>1)&1, o&1);
 *     C row s = j'*8 + o gives x at q_{j'} + m o, with entries (j*8 + def) << 8 | poly
 *       reading position def + 2 q_j;
 *   rep[i]: representative p0 packed (x << 20) | (y << 10) | z, Morton order.
 *   poly p: coefficients poly[5p + q] of the monomials 1, c3, c1, c2, c1 c3 of
 *     c = (sigma, tau, rho)(node); ids below nconst are constants.
 *   group: the 24 matrices G[w] of W, row-major 3x3 integers.
 * Templates are read off the derived tables of one small node size and the
 * orbits of nl are classified into them (Sec. IV-B, B_n; see the tests).
 * Pointers stay valid until the process ends.  Errors: FCC_ERR_NOT_POW2 for a
 * bad nl, FCC_ERR_UNSUPPORTED if an orbit matches no template, FCC_ERR_OOM. */
typedef struct {
  int nc;
  const int* w;
  const int* b_rowptr;          /* 8 nc + 1 */
  const unsigned short* b_ent;
  const int* c_rowptr;          /* 8 nc + 1 */
  const unsigned short* c_ent;
  int nrep;
  const unsigned* rep;
} fcc_orbit_template;
typedef struct {
  int nl, m, npoly, nconst, ntempl;
  const double* poly;
  const int* group;
  fcc_orbit_template templ[16];
} fcc_orbit_blocks;

fcc_status fcc_asp_orbit_blocks(int nl, fcc_orbit_blocks* out);

#ifdef __cplusplus
}
#endif
#endif /* FCC_DCT_H */
