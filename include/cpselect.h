/*
 * cpselect.h - exact k-th order statistic selection on one MI355X (gfx950) GPU,
 * by Kelley's cutting-plane minimisation of a convex piecewise-linear objective.
 *
 * Method (Beliakov, "Parallel calculation of the median and order statistics on
 * GPUs with application to robust regression"):
 *   - Section 1: x_(k) is the k-th smallest element of x (1-based k); the median
 *     is x_([(n+1)/2]), the lower median for even n.
 *   - Section 3, Eq. 2: x_(k) minimises f(y) = sum_i max(alpha (x_i - y), beta (y - x_i))
 *     with alpha = k - 1/2 and beta = n - k + 1/2 (this orientation is the one whose
 *     minimiser is the k-th smallest; the printed weights are swapped).  Its Clarke
 *     subdifferential at y is [n (L - k + 1/2), n (L + E - k + 1/2)] with L = #(x<y),
 *     E = #(x=y), so 0 lies in it exactly when L < k <= L + E.
 *   - Section 4, Algorithm 1: Kelley's cutting plane keeps a bracket [y_L, y_R] and
 *     moves to the intersection of the two supporting lines at its ends; step 0 takes
 *     the data extremes, with f and g there from min, max and sum(x) in one reduction.
 *     The hybrid at the end of Section 4 stops the iterations early, copies the
 *     elements inside the open bracket to a smaller array and selects there exactly.
 *
 * Every call is asynchronous on `stream` (a hipStream_t; NULL means the default
 * stream) and returns CPS_OK or a negative synchronous error code.  Results land in
 * caller-owned DEVICE memory; nothing is copied to the host and the library never
 * synchronises the stream.  Input arrays are caller-owned device memory, read only,
 * and must stay valid until the stream reaches the call.  Errors found on the device
 * while running (NaN in the data, a wait that timed out) are reported in the result's
 * `status` field, not as a return code.
 *
 * Data types: CPS_F32 (float) and CPS_F64 (double).  Ordering is IEEE "<": -0.0 and
 * +0.0 are equal, and the selected value is returned with +0.0 for zero.  NaN is not
 * ordered: an input holding NaN yields status CPS_STATUS_NAN.
 */
#ifndef CPSELECT_H
#define CPSELECT_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ codes */

enum cps_dtype { CPS_F32 = 0, CPS_F64 = 1 };

enum cps_error {
  CPS_OK = 0,
  CPS_EINVAL = -1,   /* bad argument: null pointer, n < 1, k outside [1, n], bad dtype or size */
  CPS_ENOMEM = -2,   /* the workspace could not be allocated */
  CPS_EHIP = -3,     /* a HIP runtime call failed (see cps_last_hip_error) */
  CPS_ECAPTURE = -4, /* the call would have to allocate while the stream is being captured */
  CPS_ENODEV = -5,   /* no usable gfx950 device */
  CPS_ESTATE = -6,   /* the handle is in an unusable state */
  CPS_EIO = -7,      /* a network file could not be opened, read or written */
  CPS_EFORMAT = -8,  /* a network file is not a valid file of this network (see cps_model_load) */
  CPS_ESCRATCH = -9  /* select_kth_noalloc: the call needs more than its static scratch array */
};

/* Asynchronous status, written by the device into cps_result.status. */
enum cps_status {
  CPS_STATUS_OK = 0,
  CPS_STATUS_NAN = 1,     /* the array holds NaN; value is NaN, counts are 0 */
  CPS_STATUS_TIMEOUT = 2, /* a device-side wait exceeded the spin limit; result invalid */
  CPS_STATUS_INTERNAL = 3, /* an internal consistency check failed; result invalid */
  CPS_STATUS_BADARG = 4    /* batched calls: this array's pointer, size or rank is invalid */
};

/* ------------------------------------------------------------------ records */

/* Result of one selection (48 bytes, device memory).
 * value_bits: raw bits of the selected element in its own type, zero-extended (f32 in
 *             the low 32 bits); the bit-exact comparison key.
 * value:      the selected element widened to double.
 * less, equal, greater: #(x < value), #(x == value), #(x > value).
 * passes:     full reads of the input array (pass 0 included) the call made.
 * status:     a cps_status value. */
typedef struct cps_result {
  uint64_t value_bits;
  double value;
  int64_t less, equal, greater;
  int32_t passes;
  int32_t status;
} cps_result;

/* Objective and counts at one trial point y (Section 3), 80 bytes, device memory.
 * f = alpha A + beta B; A = sum over x_i > y of (x_i - y); B = sum over x_i < y of (y - x_i);
 * L, E, G = #(x<y), #(x=y), #(x>y); pred = largest x_i < y (-inf if none), succ = smallest
 * x_i > y (+inf if none); gminus = n (L - k + 1/2), gplus = n (L + E - k + 1/2).
 * Comparisons and terms are taken in double precision on the widened element. */
typedef struct cps_eval {
  double f, A, B;
  int64_t L, E, G;
  double pred, succ;
  double gminus, gplus;
} cps_eval;

/* Tuning and test options for select_kth_ex.  Fill with cps_default_options first.
 * maxit:            cutting-plane iterations before the method falls back to bisection of
 *                   the bracket in the ordered bit pattern of T (which bounds the passes).
 * final_threshold:  when the bracket holds at most this many elements, one workgroup
 *                   finishes with an exact radix select (Section 4's final exact step).
 * partition_fraction: once the bracket holds at most this fraction of n, each pass also
 *                   splits the bracket's elements at the trial point into a workspace
 *                   buffer, and later passes read only the side that still holds x_(k)
 *                   (the count-and-compact of Section 4, applied at every later pass).
 *                   0 disables splitting (plain passes over x, then one compaction).
 *                   Default 1.0 (split from the first trial point on).
 * grid_blocks, block_threads: launch shape; 0 picks the tuned default.
 * spin_limit:       bound on device-side waiting loops (iterations); 0 = default.
 * bracket_lo/hi, use_bracket: a caller-supplied starting bracket (tests; the proposal
 *                   path).  Pass 0 counts #(x <= lo) and #(x < hi) and keeps each end only
 *                   where the counts prove it (#(x <= lo) < k, k <= #(x < hi)); the result
 *                   never depends on it.
 * compact_proposal: with a proposed bracket, pass 0 also writes the elements strictly
 *                   inside it to the split workspace (at most half of each wavefront's
 *                   share); when both ends hold and everything fit, later passes read only
 *                   those elements and the input is read once.  1 (default) or 0.
 * hist_bits:        once the bracket's elements are compacted, finish with exact passes
 *                   that count them in 2^hist_bits bins of their ordered bit patterns and
 *                   keep the bin holding the rank (a multi-workgroup radix select on the
 *                   compacted elements; the paper sorts them).  1..12, default 12; 0 keeps
 *                   cutting-plane passes to the end.
 * count_first:      with hist_bits > 0, the evaluation at which the first split from the
 *                   input would happen counts the elements on either side of the trial point
 *                   in those key bins instead of writing them; the bracket narrows to the
 *                   bin holding the rank, and the next pass over the input counts that
 *                   bin's elements and copies them to the workspace (when they are at most a
 *                   quarter of n).  From 256 MiB of input on, the counting evaluation also
 *                   copies the elements of a likely interval (sample quantiles around the
 *                   rank) to the workspace, and when the narrowed bracket lies inside it the
 *                   copy replaces that next pass over x.  1 (default) or 0 (the split writes
 *                   both sides and counts them as it goes).
 * cooperative:      the kernel's workgroups wait for each other between passes, so all of
 *                   them must be resident at once (the grid never exceeds what fits).  0
 *                   (default): an ordinary launch, which on a GPU not running another such
 *                   kernel gives exactly that; a selection started while another one (a
 *                   different handle, another stream) still runs may find some of its
 *                   workgroups unable to start until that one ends, and if both wait on
 *                   each other the waits give up after spin_limit and the call reports
 *                   CPS_STATUS_TIMEOUT.  1: a cooperative launch, for which the runtime
 *                   guarantees residency (about 17 us more per call on this part).
 * transform:        1: the cutting plane minimises the objective of F(x) = log(1 + x - min x),
 *                   the monotone transform of Section 5.3 for data with a few huge values
 *                   (~1e20, where the sums over x lose every smaller term): one evaluation
 *                   at the minimum forms F's objective at both ends, then every trial point is
 *                   Kelley's step on F's scale mapped back by F^-1, and every evaluation sums
 *                   F(x) (formed to float precision: the exact exponent of 1 + x - min x and
 *                   the hardware base-2 logarithm of its mantissa) in double precision;
 *                   counts, comparisons and the result stay on x
 *                   (exact whatever F rounds).  Runs without splits (count_first is then
 *                   forced on when hist_bits > 0, and partition_fraction to 0 when it is 0);
 *                   not with use_bracket or a proposal.  0 (default): the objective of x. */
typedef struct cps_options {
  int32_t maxit;
  int32_t final_threshold;
  double partition_fraction;
  int32_t grid_blocks;
  int32_t block_threads;
  int64_t spin_limit;
  int32_t use_bracket;
  int32_t compact_proposal;
  double bracket_lo, bracket_hi;
  int32_t hist_bits;
  int32_t count_first;
  int32_t transform;
  int32_t cooperative;
} cps_options;

#define CPS_STATS_MAX_PASSES 96

/* Per-call trace written by select_kth_ex when stats_dev is not NULL (device memory).
 * passes:       full reads of the input (pass 0 included).
 * work_passes:  all reduction passes, including those over the split buffers.
 * kelley_steps, bisect_steps: how each trial point was chosen.
 * final_select_size: elements the exact select read.
 * bracket_used: which proposed bracket ends the counts proved and pass 0 adopted (bit 0:
 *               the lower end, bit 1: the upper end).
 * elements_read, elements_written: elements the passes moved (algorithmic traffic).
 * population[i]: elements inside the open bracket after pass i.
 * working[i]:   elements pass i read.
 * t_start, t_arrive[i], t_publish[i]: device wall clock (100 MHz ticks) at the launch, when
 *               the last workgroup finished pass i, and when the state after pass i was
 *               published (the difference is the cutting-plane update and, on the last
 *               pass, the exact select).
 * kind[i]:      what pass i was (enum cps_pass_kind).  The remaining arrays hold what the
 *               pass's own reduction produced, as the cutting-plane update used it:
 *   CPS_PASS_ZERO (Section 4, step 0): trial = minimum, A = sum(x) - n_f min (A at the
 *               minimum), B = n_f max - sum(x) (B at the maximum), L = #min, G = #max,
 *               pred = minimum, succ = maximum (n_f: finite elements, sum over those).
 *   CPS_PASS_EVAL (Section 3, Eq. 2, one cutting-plane evaluation at trial[i]): A, B, L, G
 *               of the whole array (a pass over the bracket's compacted elements adds the
 *               parts outside the bracket), pred / succ: the largest / smallest element of
 *               the pass's working set below / above the trial point (-inf / +inf if none).
 *   CPS_PASS_COUNT (the counting evaluation): L, G of the whole array at trial[i]; A and B
 *               are not formed (0).
 *   the others: only kind and working. */
typedef struct cps_stats {
  int32_t passes;
  int32_t work_passes;
  int32_t kelley_steps;
  int32_t bisect_steps;
  int32_t final_select_size;
  int32_t bracket_used;
  int64_t elements_read;
  int64_t elements_written;
  int64_t population[CPS_STATS_MAX_PASSES];
  int64_t working[CPS_STATS_MAX_PASSES];
  uint64_t t_start;
  uint64_t t_arrive[CPS_STATS_MAX_PASSES];
  uint64_t t_publish[CPS_STATS_MAX_PASSES];
  int32_t kind[CPS_STATS_MAX_PASSES];
  double trial[CPS_STATS_MAX_PASSES];
  double A[CPS_STATS_MAX_PASSES], B[CPS_STATS_MAX_PASSES];
  int64_t L[CPS_STATS_MAX_PASSES], G[CPS_STATS_MAX_PASSES];
  double pred[CPS_STATS_MAX_PASSES], succ[CPS_STATS_MAX_PASSES];
} cps_stats;

/* Pass kinds of cps_stats.kind. */
enum cps_pass_kind {
  CPS_PASS_ZERO = 0,   /* pass 0: extremes, their multiplicities and the sum */
  CPS_PASS_EVAL = 1,   /* fused evaluation of A, B, counts and neighbours at a trial point */
  CPS_PASS_COUNT = 2,  /* counting evaluation: the two sides of a trial point in key bins */
  CPS_PASS_HIST = 3,   /* key-histogram pass of the exact finish */
  CPS_PASS_GATHER = 4, /* gather of the bracket's elements */
  CPS_PASS_FINAL = 5   /* one-workgroup exact select */
};

typedef struct cps_handle cps_handle;

/* ------------------------------------------------------------------ handle */

/* Create a handle bound to HIP device `device` (which must be gfx950).  The handle owns
 * the workspace (grown on demand outside stream capture) and the launch configuration.
 * Returns CPS_ENODEV when the device is missing or not gfx950.
 *
 * Streams: the calls made with one handle share its workspaces (the selection state, its
 * synchronisation counters, split and gather buffers, the batched queue, the proposal's
 * bracket), so the device work of two calls with one handle must not overlap.  Calls on
 * one stream are ordered by the stream; calls on different streams with one handle must
 * be ordered by the caller (events), or use one handle per stream.  The host side of a
 * handle is thread-safe (a mutex), which orders the launches but not their device work. */
int cps_create(int device, cps_handle **out);

/* Destroy a handle.  The caller must have synchronised every stream used with it. */
int cps_destroy(cps_handle *h);

/* Human-readable text for a cps_error or cps_status code (static storage). */
const char *cps_status_string(int code);

/* The last HIP error code seen by the library in this thread (0 if none). */
int cps_last_hip_error(void);

/* Defaults for select_kth_ex. */
void cps_default_options(cps_options *opt);

/* Make sure the workspace can serve a single-array call of n elements of `dtype`, so
 * that a later call made under stream capture does not need to allocate. */
int cps_reserve(cps_handle *h, int64_t n, int dtype);

/* ------------------------------------------------------------------ selection */

/* The k-th smallest element of x[0..n) (1-based k), with its counts.
 * x: device pointer to n elements of `dtype` (any alignment of the element type).
 * out_dev: device pointer to one cps_result.
 * Errors: CPS_EINVAL for a null pointer, n < 1, k outside [1, n] or a bad dtype. */
int select_kth(cps_handle *h, const void *x, int64_t n, int64_t k, int dtype,
               cps_result *out_dev, void *stream);

/* select_kth with options (may be NULL) and an optional device-side trace (may be NULL). */
int select_kth_ex(cps_handle *h, const void *x, int64_t n, int64_t k, int dtype,
                  const cps_options *opt, cps_result *out_dev, cps_stats *stats_dev,
                  void *stream);

/* select_kth for callers that cannot allocate device memory: code under stream capture,
 * serving loops, harnesses that forbid hipMalloc.  The call allocates nothing (no hipMalloc,
 * hipFree or allocating library routine) and takes none of the handle's workspace: its
 * scratch words (the selection state, the grid's synchronisation words, 2 x 4096 histogram
 * counters, the workgroups' partials and a gather buffer of 8192 elements) live in one
 * file-scope device array of 1 MiB per GPU, which that GPU holds until the process ends.
 * cps_create takes the array's device address for its device.
 * The selection is that of select_kth's defaults without the split buffers: pass 0, the
 * counting evaluation at the first trial point, then key-histogram passes over x that count
 * the narrowed bracket without copying it (each keeps one of 4096 bins), the gather of the
 * last few thousand elements and the exact select.  Results (value, counts, status) are
 * identical to select_kth's; it reads x about twice as often on large inputs.
 * The launch is a fill kernel that zeroes the synchronisation words and histogram counters,
 * then the selection kernel: both may be captured in a graph.
 * Every call on one GPU shares that GPU's array, which keeps the last call's contents:
 * calls whose device work overlaps on one GPU (different streams, or different handles of
 * the same device) race and give wrong results; the caller must order them.
 * Arguments, layout and errors as select_kth, and CPS_ESTATE when the handle's device has
 * no scratch address, CPS_ESCRATCH when the launch shape would need more than the array
 * (it does not on any device of up to 1024 resident workgroups). */
int select_kth_noalloc(cps_handle *h, const void *x, int64_t n, int64_t k, int dtype,
                       cps_result *out_dev, void *stream);

/* f, A, B, counts, neighbours and subgradient end points at each of ny points ys_dev
 * (device doubles), for the rank-k objective of x[0..n) (Section 3, Eq. 2): the quantities a
 * cutting-plane pass forms, computed here by a separate two-stage kernel that widens every
 * element to double before comparing and summing (a reference evaluation on the device, not
 * the hot path's own pass: what the selection's passes formed is in cps_stats' per-pass
 * trace).  Uses its own region of the handle's workspace.
 * out_dev: device pointer to ny cps_eval records. */
int cps_objective(cps_handle *h, const void *x, int64_t n, int64_t k, int dtype,
                  const double *ys_dev, int64_t ny, cps_eval *out_dev, void *stream);

/* ------------------------------------------------------------------ batched selection */

/* Tuning of the batched kernel.  Fill with cps_default_batch_options first (1024 threads,
 * split capacity 2^17, final threshold 4096, split fraction 1, 2^12 bins, count first, the
 * sampled bracket, one workgroup per array);
 * 0 fields pick the tuned (or default) value.
 * block_threads:   workgroup size, 256, 512 or 1024 (one workgroup runs one array at a time).
 * blocks_per_cu:   resident workgroups per compute unit.
 * split_capacity:  elements of each of a workgroup's two split buffers; a bracket is split
 *                  (count-and-compact, end of Section 4) once it holds at most this many.
 *                  Unused (no buffers) with count_first and hist_bits > 0, which never split.
 * final_threshold, maxit, partition_fraction, hist_bits: as in cps_options (the histogram
 *                  passes count in the workgroup's LDS).
 * count_first:     as in cps_options, with 2^11 bins per side (the two sides share the
 *                  workgroup's LDS histogram); the bin's elements are then counted by
 *                  histogram passes over the array (no copy) until few are left for the
 *                  gather.  The split capacity does not limit it.  1 (default) or 0.
 * proposal:        1 (default): an array of at least 2^15 elements starts from a sampled
 *                  bracket (not in the paper): S of its elements (S = 4096, or 16384 from
 *                  2^18 elements on; runs of 16 neighbours) counted in 2^12 key bins over
 *                  their range, and the values just outside the bins of sample ranks
 *                  S p -/+ (4 sqrt(S p (1 - p)) + 2), p = (k - 1/2) / n.  Pass 0 counts #(x <= a) and #(x < b), keeps each
 *                  end only where the counts prove it (as cps_options.use_bracket), counts the
 *                  elements strictly inside in key bins and copies every 16-byte vector of x
 *                  that holds one to a buffer; when both ends hold, the bracket narrows to the
 *                  bin of the rank at once and every later pass reads only the copy.  The
 *                  result never depends on it.  Needs hist_bits > 0 (ignored otherwise).
 *                  0: every array from [min, max].
 * blocks_per_array, elements_per_block: with the proposal, an array of n > elements_per_block
 *                  elements is split into min(blocks_per_array, ceil(n / elements_per_block))
 *                  contiguous parts, each taken by its own workgroup for pass 0 (the one pass
 *                  over the whole array); the last part to arrive folds the parts' partials
 *                  (in part order) and finishes the array alone.  Only the 1024 largest arrays
 *                  of a batch of at most 4096 may be split.  blocks_per_array in [1, 16]
 *                  (default 1: one workgroup per array), elements_per_block >= 2^15
 *                  (default 2^18).
 * team_capacity:   elements of the buffer that holds an array's copied vectors (default 2^18:
 *                  enough for arrays of about a million elements); a copy that does not fit
 *                  makes pass 0's counts decide alone and the array continues over its full
 *                  length (exact, slower).  Each workgroup has one such buffer, and each
 *                  split array one more.  The autotuner sizes it from the batch's largest
 *                  array. */
typedef struct cps_batch_options {
  int32_t block_threads;
  int32_t blocks_per_cu;
  int64_t split_capacity;
  int32_t final_threshold;
  int32_t maxit;
  double partition_fraction;
  int32_t hist_bits;
  int32_t count_first;
  int32_t proposal;
  int32_t blocks_per_array;
  int64_t elements_per_block;
  int64_t team_capacity;
} cps_batch_options;

void cps_default_batch_options(cps_batch_options *opt);

/* The k-th smallest element of each of `count` arrays of uneven sizes, in one launch: the
 * method of Sections 3-4 run per array by one workgroup of a persistent grid that takes
 * arrays largest first (the paper motivates batching when many medians are needed,
 * Section 2).  The launch allocates nothing and leaves its queue reset, so it may be
 * captured in a graph and replayed once the workspace is reserved (cps_reserve_batched).
 * ptrs_dev:  device array of `count` device pointers to the arrays (each aligned to its
 *            element type); sizes_dev, ks_dev: device arrays of int64 sizes and 1-based ranks.
 * out_dev:   device array of `count` cps_result.  An invalid array (null pointer, size < 1,
 *            rank outside [1, size]) gets status CPS_STATUS_BADARG; the others are unaffected.
 * Errors: CPS_EINVAL for a null handle or descriptor pointer, count < 1 or a bad dtype. */
int select_kth_batched(cps_handle *h, const void *const *ptrs_dev, const int64_t *sizes_dev,
                       const int64_t *ks_dev, int64_t count, int dtype, cps_result *out_dev,
                       void *stream);

/* select_kth_batched with explicit tuning (NULL: the handle's autotuned choice, else the
 * defaults). */
int select_kth_batched_ex(cps_handle *h, const void *const *ptrs_dev, const int64_t *sizes_dev,
                          const int64_t *ks_dev, int64_t count, int dtype,
                          const cps_batch_options *opt, cps_result *out_dev, void *stream);

/* Allocate the batched workspace for `opt` (NULL: the current choice) ahead of stream capture. */
int cps_reserve_batched(cps_handle *h, int dtype, const cps_batch_options *opt);

/* Autotuner: time each candidate launch shape (256, 512, 1024 threads) with the sampled
 * bracket and one workgroup per array or 4, 8 or 16 per array at 2^16 .. 2^18 elements per
 * workgroup, without it (the counting evaluation from [min, max]), and with splits at split
 * capacities 2^17 and 2^19, on this very batch (the call synchronises `stream`; the
 * candidates with the sampled bracket get a team_capacity of a quarter of the largest
 * array's elements, between the default 2^18 and 2^22); keep the
 * fastest as the handle's choice for `dtype`, and return it in best (may be NULL) with its
 * time in *best_ms (may be NULL).  The results in out_dev are those of the last timed
 * candidate. */
int cps_autotune_batched(cps_handle *h, const void *const *ptrs_dev, const int64_t *sizes_dev,
                         const int64_t *ks_dev, int64_t count, int dtype, cps_result *out_dev,
                         void *stream, cps_batch_options *best, double *best_ms);

/* ------------------------------------------------------------------ least median of squares */

/* For each of m candidate parameter vectors b (rows of betas_dev, m x p, row-major doubles),
 * the lower median (rank floor((n+1)/2)) of the squared residuals
 *     r_i = (y_i - sum_{j=0..p-1} X_ij b_j)^2,   i = 0..n-1,
 * the objective of the least-median-of-squares estimator (Section 6).  The sum runs left to
 * right in j and every product and sum is rounded on its own (no fused multiply-add), so the
 * residuals are bit-identical to that sequence in IEEE double precision; the medians are
 * then exact.  out_dev[c] receives candidate c's median with its counts among the r_i.
 * X_dev: n x p row-major doubles; y_dev: n doubles (device memory, caller-owned).
 * Same as lms_median_sq_residuals_ex with form CPS_LMS_AUTO.
 * Errors: CPS_EINVAL for null pointers, n < 1, p outside [1, 16], m < 1 or m > 1048560. */
int lms_median_sq_residuals(cps_handle *h, const double *X_dev, const double *y_dev,
                            const double *betas_dev, int64_t n, int32_t p, int64_t m,
                            cps_result *out_dev, void *stream);

/* How lms_median_sq_residuals_ex finds the medians (all forms give the same value, counts
 * and status):
 * CPS_LMS_MATERIALISED: every r_i is written to the handle's workspace (m * n doubles) and
 *   the batched kernel selects within each candidate's n squares.
 * CPS_LMS_FILTERED (n from 2^15 to 2^31 - 1): each candidate's sampled bracket (a, b) is
 *   taken from the squares of a fixed sample of rows (as the batched kernel samples an array
 *   of n elements), one kernel forms every r_i and keeps only those in (a, b) (and NaN),
 *   with #(r <= a), and the kept squares are packed and selected at rank k - #(r <= a).  A
 *   candidate whose bracket does not hold the median, or whose kept squares exceed n/8, gets
 *   its whole array written and selected as in the materialised form.  The workspace holds
 *   m * n + m * (n/8) doubles.  `passes` then counts the one pass that forms the residuals
 *   plus the selection's passes over the packed squares.
 * CPS_LMS_AUTO: the filtered form where n allows it, else the materialised one. */
enum cps_lms_form { CPS_LMS_AUTO = 0, CPS_LMS_MATERIALISED = 1, CPS_LMS_FILTERED = 2 };

/* lms_median_sq_residuals with a choice of form (above).  Errors: as
 * lms_median_sq_residuals, and CPS_EINVAL for a form outside cps_lms_form, or
 * CPS_LMS_FILTERED with n outside [2^15, 2^31). */
int lms_median_sq_residuals_ex(cps_handle *h, const double *X_dev, const double *y_dev,
                               const double *betas_dev, int64_t n, int32_t p, int64_t m,
                               int32_t form, cps_result *out_dev, void *stream);

/* The k-th smallest element of each array (as select_kth_batched_ex) and the sum of each
 * array's k smallest elements, ksum_dev[i] = sum_{x < v} x + (k - #(x < v)) v with v = x_(k)
 * (Section 6: the least-trimmed-squares objective is this sum over squared residuals, and
 * the weight rho there is 1 below v, a/b at v with a = k - #(x < v) and b = #(x = v)).
 * Formed in double precision; with the sampled bracket the elements below the bracket's
 * lower end are summed by pass 0 and those inside from its copy (in the copy's order, which
 * varies from run to run, so the last bits may differ between runs), else by one more pass
 * over the array.  ksum_dev: device array of `count` doubles (NaN for an array whose status
 * is not OK).  Other arguments and errors as select_kth_batched_ex. */
int select_kth_batched_ksum(cps_handle *h, const void *const *ptrs_dev, const int64_t *sizes_dev,
                            const int64_t *ks_dev, int64_t count, int dtype,
                            const cps_batch_options *opt, cps_result *out_dev, double *ksum_dev,
                            void *stream);

/* Least trimmed squares (Section 6), 48 bytes, device memory: for one candidate, the sum F of
 * the h smallest squared residuals, their h-th smallest m, below = #(r < m), a = h - below,
 * b = #(r = m), and the selection's status. */
typedef struct cps_trim {
  double F;
  double m;
  int64_t below, a, b;
  int32_t status;
  int32_t pad;
} cps_trim;

/* For each of m candidate parameter vectors (rows of betas_dev, m x p), the least-trimmed-
 * squares objective: the sum of the h smallest of r_i = (y_i - sum_j X_ij b_j)^2, found
 * through the h-th order statistic as Section 6 writes it, F = sum_{r < m} r + a m.  The
 * residuals are formed as in lms_median_sq_residuals (bit-identical), h is 1-based
 * (Section 6 takes h = floor((n+1)/2), the rank of the median; Rousseeuw's h = floor((n+p)/2)
 * works the same).  out_dev receives m cps_trim records.  Errors: as
 * lms_median_sq_residuals, and CPS_EINVAL for h outside [1, n]. */
int lts_trimmed_sq(cps_handle *h, const double *X_dev, const double *y_dev,
                   const double *betas_dev, int64_t n, int32_t p, int64_t m, int64_t hk,
                   cps_trim *out_dev, void *stream);

/* lts_trimmed_sq with a choice of form (cps_lms_form; CPS_LMS_AUTO is lts_trimmed_sq).  In
 * the filtered form the bracket is taken for rank hk, the filter also sums the squares at or
 * below its lower end (per row segment, in row order; the segments' sums added in a fixed
 * order), and one more pass over the packed squares sums those below the selected value, so
 * F is formed in double precision in a fixed order.  Errors: as lts_trimmed_sq, and
 * CPS_EINVAL for a form outside cps_lms_form, or CPS_LMS_FILTERED with n outside
 * [2^15, 2^31). */
int lts_trimmed_sq_ex(cps_handle *h, const double *X_dev, const double *y_dev,
                      const double *betas_dev, int64_t n, int32_t p, int64_t m, int64_t hk,
                      int32_t form, cps_trim *out_dev, void *stream);

/* k nearest neighbours (Section 6, last paragraph), 32 bytes, device memory: for one query,
 * the mean ordinate of its k nearest points, the k-th smallest squared distance dk, the
 * counts #(d < dk) and #(d = dk), and the selection's status. */
typedef struct cps_knn {
  double mean;
  float dk;
  int32_t status;
  int64_t below, equal;
} cps_knn;

/* For each of nq queries (rows of Q_dev, nq x dim floats, row-major), the squared Euclidean
 * distances d_i = sum_j (P_ij - q_j)^2 to the n points (rows of P_dev, n x dim), each
 * difference, square and sum rounded to float in order j = 0..dim-1 (no fused multiply-add);
 * their k-th smallest dk by the batched selection; and the mean ordinate of the k nearest
 * points, (sum_{d < dk} f_i + (a / b) sum_{d = dk} f_i) / k with b = #(d = dk),
 * a = k - #(d < dk) (Section 6's rho as an indicator: exactly k points' worth), summed in
 * double precision in a fixed order.  f_dev: n floats.  In the materialised form the
 * distances are written to the handle's workspace (nq x n floats) for the selection and read
 * back by the reduction.
 * Errors: CPS_EINVAL for null pointers, n < 1, dim outside [1, 16], nq outside [1, 65535],
 * k outside [1, n]. */
int knn_mean(cps_handle *h, const float *P_dev, const float *f_dev, const float *Q_dev, int64_t n,
             int32_t dim, int64_t nq, int64_t k, cps_knn *out_dev, void *stream);

/* knn_mean with a choice of form (cps_lms_form; CPS_LMS_AUTO is knn_mean, which takes the
 * filtered form from n = 2^15 on).  Filtered: each query's sampled bracket (a, b) from the
 * distances of the points the batched kernel would sample, one pass over the points that
 * keeps the distances in (a, b) (and NaN) with their ordinates (at most 8128 per query),
 * counting d <= a and summing its ordinates; d_k by a radix select among the kept ones, the
 * sums below and at d_k in a fixed order.  A query whose bracket misses d_k, or that keeps
 * more, is selected by one workgroup over its distances recomputed.  Same results (the
 * ordinates' sum over d <= a is added over segments in no fixed order, so its last bits may
 * vary).  Errors: as knn_mean, and CPS_EINVAL for a form outside cps_lms_form, or
 * CPS_LMS_FILTERED with n outside [2^15, 2^31). */
int knn_mean_ex(cps_handle *h, const float *P_dev, const float *f_dev, const float *Q_dev,
                int64_t n, int32_t dim, int64_t nq, int64_t k, int32_t form, cps_knn *out_dev,
                void *stream);

/* ------------------------------------------------------------------ learned bracket proposal
 *
 * An extension of the method (not in the paper): a small network reads a sketch of the
 * array and proposes a bracket around x_(k), which the two-point pass 0 checks by counts
 * (see cps_options.use_bracket); a wrong proposal costs nothing in exactness.
 *
 * Features of an array (n elements, rank k): the fixed-stride sample
 * x[i * floor(n / S)], i < S = min(n, 4096); its minimum lo and maximum hi (a zero extreme
 * as +0); its histogram in 64 equal bins over [lo, hi], bin = min(63,
 * floor(64 (v - lo) / (hi - lo))) in double precision (all in bin 0 when hi == lo), as
 * cumulative fractions (feature b: the fraction of the sample in bins 0..b);
 * lo / (1 + |lo|), hi / (1 + |hi|) and k / n.  Each of the 67 features is formed in double
 * precision and rounded once to float.  A sample holding NaN or an infinity gives no
 * proposal.
 *
 * Network: 67 -> 64 (ReLU) -> 64 (ReLU) -> 2 in float, outputs (u, s).  Parameters are one
 * float array of CPS_MLP_PARAMS values: W1 (64 x 67, row-major, row = hidden unit), b1 (64),
 * W2 (64 x 64), b2 (64), W3 (2 x 64), b3 (2).  The histogram position h is where the
 * cumulative features F cross the k/n feature p: (b + (p - F_{b-1}) / (F_b - F_{b-1})) / 64,
 * b the first bin with F_b >= p (F_{-1} = 0), in double precision.  Proposed bracket:
 * y0 -+ w with y0 = lo + (hi - lo)(h + u), w = (hi - lo) exp(clamp(s, -20, 4)), formed in
 * double precision.
 *
 * Training loss of one example with label u* = (x_(k) - lo) / (hi - lo) - h (0 when
 * hi == lo), d = u - u*, omega = exp(clamp(s, -20, 4)):
 *     100 d^2 + max(0, |d| - omega) + 0.02 omega,
 * averaged over the batch.  ReLU'(0) = 0, sign(0) = 0, and the clamp passes gradient only
 * strictly inside (-20, 4). */

#define CPS_MLP_INPUTS 67
#define CPS_MLP_HIDDEN 64
#define CPS_MLP_OUTPUTS 2
#define CPS_MLP_PARAMS 8642

/* Synthetic training and test arrays: `count` float arrays of n elements, array
 * first_id + a at x_dev + a * n, each drawn from a random mixture of 1-4 components
 * (Gaussian, lognormal, uniform), with its rank k in ks_dev[a] (may be NULL).  Array
 * (seed, id) is defined by the Philox4x32-10 counter-based generator (Salmon et al.,
 * SC'11) at counters (i mod 2^32, i div 2^32, id, j), key (seed mod 2^32, seed div 2^32):
 *   parameters from the blocks at counters (0, 0, id, 4..8), twenty words w0..w19:
 *     ncomp = 1 + (w0 >> 30); type_c = (3 w_{1+c}) >> 32 (0 Gaussian, 1 lognormal,
 *     2 uniform); ua = w_{5+c} 2^-32, ub = w_{9+c} 2^-32; weight q_c = 1 + (w_{13+c} >> 8),
 *     cumulative weights (q_0 + .. + q_c) / (q_0 + .. + q_{ncomp-1});
 *     Gaussian mean -100 + 200 ua, sd exp((-2 + 3 ub) ln 10); lognormal log-mean
 *     -2 + 4 ua, log-sd 0.25 + 1.25 ub; uniform on [p1, p1 + p2] with p1 = -100 + 200 ua,
 *     p2 = exp((-2 + 4 ub) ln 10); k = 1 + floor(((w17 << 32) | w18) n / 2^64);
 *   element i from the blocks j = 0..3 at its counter: g = (sum of the twelve words of
 *     blocks 0-2, each as (w >> 8) 2^-24) - 6; block 3's first word r picks the component
 *     (the number of cumulative weights <= r 2^-32 among the first three, capped at
 *     ncomp - 1) and its second word v gives the uniform v 2^-32; the value is p1 + p2 g,
 *     exp(p1 + p2 g) or p1 + p2 v in double precision, rounded to float.
 * exp here is 2^floor(t) times the degree-14 Taylor polynomial of e^(f ln 2) in Horner
 * form, t = z log2(e), f = t - floor(t), with coefficients 1/j! formed by successive
 * division; every step is an integer or a correctly rounded double operation, so any
 * implementation of this definition gives the same bits.
 * Errors: CPS_EINVAL for null x_dev, count < 1, n < 1, or ids beyond 2^32. */
int cps_mixture_generate(cps_handle *h, uint64_t seed, int64_t first_id, int64_t count,
                         int64_t n, float *x_dev, int64_t *ks_dev, void *stream);

/* Features of `count` arrays (descriptors as in select_kth_batched; dtype CPS_F32 or
 * CPS_F64): feat_dev receives count x 67 floats, range_dev count x 2 doubles (lo, hi),
 * valid_dev count int32 (1, or 0 when the sample is not finite or the descriptor is
 * invalid; the features are then zero). */
int cps_features(cps_handle *h, const void *const *ptrs_dev, const int64_t *sizes_dev,
                 const int64_t *ks_dev, int64_t count, int dtype, float *feat_dev,
                 double *range_dev, int32_t *valid_dev, void *stream);

/* Network outputs (u, s) for `count` feature rows: out_dev count x 2 floats. */
int cps_mlp_forward(cps_handle *h, const float *params_dev, const float *feat_dev,
                    int64_t count, float *out_dev, void *stream);

/* Mean training loss (loss_dev: one float, may be NULL) and its gradient (grad_dev:
 * CPS_MLP_PARAMS floats) over `count` examples (feature rows and labels ustar_dev),
 * by back-propagation in float with a fixed summation order (deterministic).  Uses the
 * handle's workspace (about count / 32 x 35 KB). */
int cps_mlp_loss_grad(cps_handle *h, const float *params_dev, const float *feat_dev,
                      const float *ustar_dev, int64_t count, float *grad_dev, float *loss_dev,
                      void *stream);

/* One Adam step (Kingma and Ba, 2015), step = 1, 2, ...: m = b1 m + (1 - b1) g,
 * v = b2 v + (1 - b2) g^2, p -= lr (m / (1 - b1^step)) / (sqrt(v / (1 - b2^step)) + eps). */
int cps_mlp_adam(cps_handle *h, float *params_dev, const float *grad_dev, float *m_dev,
                 float *v_dev, int64_t step, float lr, float beta1, float beta2, float eps,
                 void *stream);

/* Initial parameters: weights uniform in +-sqrt(6 / fan_in) from Philox4x32-10 (key
 * seed, counter (index, 0, 0, 0xC0FFEE), first word's top 24 bits), W3 scaled by 0.01,
 * b1 = b2 = 0 and b3 = (0, ln 0.05): the histogram position with a 5 % half-width. */
int cps_mlp_init(cps_handle *h, uint64_t seed, float *params_dev, void *stream);

/* The proposed bracket for one array: bracket_dev receives three doubles (a, b, use), use
 * = 0 when the sample gives no proposal. */
int cps_learned_bracket(cps_handle *h, const void *x, int64_t n, int64_t k, int dtype,
                        const float *params_dev, double *bracket_dev, void *stream);

/* select_kth with the learned proposal: the bracket kernel, then the selection whose pass 0
 * checks the proposal by counts (and, where it holds, compacts its elements).  Results are
 * identical to select_kth's; only the number of passes changes.  opt may be NULL. */
int select_kth_learned(cps_handle *h, const void *x, int64_t n, int64_t k, int dtype,
                       const float *params_dev, const cps_options *opt, cps_result *out_dev,
                       cps_stats *stats_dev, void *stream);

/* The non-learned baseline of the proposal, for one array: the fixed-stride sample of
 * S = min(n, 4096) elements (element i * floor(n / S)) and the bracket between its order
 * statistics of 0-based ranks floor(c - z sd) - 1 and ceil(c + z sd), c = S k / n,
 * sd = sqrt(S p (1 - p)) + 1 with p = k / n (an end beyond the sample is open: -inf or
 * +inf), selected on the device (one workgroup: key bins, then exact ranks inside the two
 * bins that hold them).  bracket_dev receives three doubles (a, b, use), use = 0 when the
 * sample holds NaN or an infinity.  Errors: CPS_EINVAL for null pointers, n < 1, k outside
 * [1, n], a misaligned x or z < 0. */
int cps_sample_bracket(cps_handle *h, const void *x, int64_t n, int64_t k, int dtype, double z,
                       double *bracket_dev, void *stream);

/* select_kth with that bracket (cps_sample_bracket's kernel, then the selection whose pass 0
 * checks it by counts like any proposal); results are identical to select_kth's.
 * Errors: as select_kth, and CPS_EINVAL for z < 0. */
int select_kth_sampled(cps_handle *h, const void *x, int64_t n, int64_t k, int dtype, double z,
                       const cps_options *opt, cps_result *out_dev, cps_stats *stats_dev,
                       void *stream);

/* Network files.  A trained proposal network is kept in a little-endian binary file of 8-byte
 * header words followed by the parameters:
 *   bytes  0..7    magic "CPSMLP01"
 *   uint32 8       format version (1)
 *   uint32 12..23  inputs, hidden units per layer, outputs (67, 64, 2)
 *   uint32 24      feature specification (1: the features and outputs documented above)
 *   uint32 28      parameter count (CPS_MLP_PARAMS)
 *   uint64 32      FNV-1a 64-bit hash (Fowler, Noll, Vo) of the parameter bytes
 *   float  40..    the CPS_MLP_PARAMS parameters in the layout documented above.
 * cps_model_save copies params_dev (device, CPS_MLP_PARAMS floats) to the host and writes the
 * file (replacing it); cps_model_load checks every header field and the hash, then copies the
 * parameters to params_dev.  Both synchronise the device (hipMemcpy) and need no handle.
 * Errors: CPS_EINVAL for null arguments, CPS_EIO when the file cannot be opened, read or
 * written, CPS_EFORMAT for a wrong magic, version, shape, feature specification, count, hash
 * or length (params_dev is then left unchanged), CPS_EHIP for a failed copy. */
int cps_model_save(const float *params_dev, const char *path);
int cps_model_load(const char *path, float *params_dev);

/* Training driver: draws n_arrays arrays of array_size elements (cps_mixture_generate,
 * seed, ids 0..n_arrays-1), labels them exactly with select_kth_batched, and runs `epochs`
 * passes of Adam over them in minibatches of `batch`; then measures the trained proposal
 * on `holdout` arrays of seed holdout_seed.  init = 1 starts from cps_mlp_init(seed).
 * Synchronises `stream` at the end. */
typedef struct cps_train_options {
  uint64_t seed;
  int64_t n_arrays;
  int64_t array_size;
  int32_t epochs;
  int32_t batch;
  float lr;
  int32_t init;
  int64_t holdout;
  uint64_t holdout_seed;
} cps_train_options;

typedef struct cps_train_report {
  double first_loss;       /* mean loss of the first minibatch */
  double final_loss;       /* mean loss over the last epoch's minibatches */
  double holdout_coverage; /* fraction of holdout arrays whose x_(k) lies strictly inside */
  double holdout_width;    /* mean 2 w / (hi - lo) over the holdout arrays */
  int64_t steps;           /* Adam steps taken */
  int64_t examples;        /* training examples with a valid sample */
} cps_train_report;

int cps_mlp_train(cps_handle *h, const cps_train_options *opt, float *params_dev,
                  cps_train_report *report, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* CPSELECT_H */
