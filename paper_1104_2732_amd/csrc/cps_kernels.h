// Kernel argument blocks and launchers shared by the C ABI and the kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/cpselect.h"
#include "batch_queue.h"
#include "cp_state.h"

namespace cps {

// Launch shape of the single-array kernel (build-time tunables).
#ifndef CPS_SELECT_BLOCK
#define CPS_SELECT_BLOCK 1024
#endif
#ifndef CPS_SELECT_UNROLL
#define CPS_SELECT_UNROLL 4
#endif
#ifndef CPS_SPLIT_UNROLL
#define CPS_SPLIT_UNROLL 2
#endif
constexpr int kWaveSize = 64;
constexpr int kSelectBlock = CPS_SELECT_BLOCK;
#ifndef CPS_SELECT_PREFETCH
#define CPS_SELECT_PREFETCH 1
#endif
// the streaming passes over full tiles issue the next tile's loads before processing the
// current one
constexpr bool kSelectPrefetch = CPS_SELECT_PREFETCH != 0;
constexpr int kSelectUnroll = CPS_SELECT_UNROLL;  // 16-byte loads in flight per thread, plain passes
constexpr int kSplitUnroll = CPS_SPLIT_UNROLL;    // the same for passes that also write
constexpr int kHistMaxBins = 4096;  // bins of a histogram pass (2^hist_bits, hist_bits <= 12)
constexpr int kHistWords = 2 * kHistMaxBins;  // global counters: one set per part of a split
constexpr int kGroup = 16;       // workgroups per first-level arrival counter
constexpr int kMaxGroups = 256;  // so at most 4096 workgroups

// Grid-synchronisation words of the single-array kernel, each on its own 128-byte line.
// Workgroups arrive on grp[bid / kGroup]; the last of each group arrives on `top`; the last
// overall advances the state and bumps `gen`, on which the others wait.  gcur hands out
// write offsets in the gather buffer.  `exits` counts the workgroups that have left the
// launch: the last one clears the arrival counters, which a wait that timed out can leave
// part-way counted, so every launch starts from zeroed counters.  A workgroup whose wait
// timed out sets `tmo`; the last one out then also clears the histogram counters, which a
// pass that was abandoned half-way may have left counted.
struct SyncCtl {
  uint32_t top;
  uint32_t gen;
  uint32_t pad0[30];
  uint64_t gcur;
  uint64_t pad1[15];
  uint32_t exits;
  uint32_t pad2[31];
  uint32_t tmo;
  uint32_t pad3[31];
  uint32_t grp[kMaxGroups][32];
};

template <typename T> struct SelectArgs {
  const T *x;
  int64_t n, k;
  CpState *st;
  SyncCtl *sync;
  double *sd;          // per-workgroup partials, 8 fields x slot_stride
  int64_t *si;         // per-workgroup integer partials, 8 fields x slot_stride
  int64_t slot_stride;
  T *z[2];             // split buffers: one region of seg_R elements per wavefront
  int64_t seg_R;
  T *zf;               // gather buffer, cfg.zcap elements
  cps_result *out;
  cps_stats *stats;    // may be null
  CpConfig cfg;
  int64_t spin_limit;
  const double *bracket;  // device [a, b, use] read by pass 0 in place of cfg's, or null
  int64_t p0_cap;      // elements per wavefront region a bracketed pass 0 may write (0: none)
  uint64_t *ghist;     // kHistWords counters (zero between passes): a histogram pass uses the
                       // first kHistMaxBins, a split pass that counts its parts both halves
  uint64_t *phist;     // kHistMaxBins counters, zeroed by the proposal kernel before this
                       // launch: pass 0 counts a proposal's interior in them (or null)
  T *smp;              // pass 0's sample for the likely interval: the first vector of every
                       // tile of x (smp_n elements), or null
  int64_t smp_n;
};

// ---- batched selection


// Work queue of the batched kernel (each counter on its own 128-byte line).  Both reset
// to zero when the last workgroup leaves, so consecutive launches need no clearing.
struct BatchCtl {
  uint64_t queue;
  uint64_t pad0[15];
  uint64_t exits;
  uint64_t pad1[15];
};

// An array split over several workgroups (a team): each takes a contiguous part of pass 0
// and leaves its partial here; the last to arrive folds them and finishes the array alone.
// Every field is back at zero when that workgroup is done, so records are reused across
// launches without clearing (the records live in a buffer of their own, zeroed once).
constexpr int kTeamMax = 16;        // workgroups per array at most
constexpr int kTeamRecords = 1024;  // arrays that may be split (the largest ones)
struct TeamCtl {
  uint32_t arrive;
  uint32_t overflow;         // some part's interior did not fit the team buffer
  uint32_t pad0[30];
  unsigned long long cursor; // 16-byte vectors written to the team buffer
  uint64_t pad1[15];
  double pd[kTeamMax][3];    // per part: min, max, sum of the elements at or below a
  int64_t pi[kTeamMax][6];   // per part: #min, #max, #(x <= a), #NaN, #(a < x < b), unused
  uint32_t hist[kHistMaxBins];  // the interior's key bins, summed over the parts
};

template <typename T> struct BatchArgs {
  const T *const *ptrs;  // device array of `count` device pointers
  const int64_t *sizes;  // device array
  const int64_t *ks;     // device array (1-based ranks)
  int64_t count;
  cps_result *out;       // device array of `count` results
  BatchCtl *ctl;
  T *zbuf;               // per workgroup: split buffers of `cap` (two, or one when nothing is
                         // ever split) and a gather buffer
  int64_t cap;
  int64_t ws_stride;     // elements of workspace per workgroup
  int64_t gb_off;        // the gather buffer's offset in a workgroup's workspace
  CpConfig cfg;
  int32_t proposal;      // 1: arrays of at least kBatchPropMin elements start from a sampled
                         // bracket checked by pass 0's counts (hist_bits > 0 required)
  int32_t team_max;      // workgroups per array at most (1: one per array)
  int64_t team_chunk;    // elements per workgroup of a split array
  int64_t team_cap;      // elements of each team buffer
  int64_t team_records;  // records (and team buffers): largest-first slots below this may split
  TeamCtl *teams;        // team_records records
  T *tbuf;               // team_records buffers of team_cap elements
  double *ksum;          // per array: the sum of its k smallest elements (or null)
};

template <typename T>
hipError_t launch_batched(const BatchArgs<T> &a, int grid, int block, hipStream_t stream);
template <typename T> int batched_max_blocks_per_cu(int block);

hipError_t launch_lms_residuals(const double *X, const double *y, const double *betas, int64_t n,
                                int32_t p, int64_t m, int64_t rank, double *R, const double **ptrs,
                                int64_t *sizes, int64_t *ks, int cu_count, hipStream_t stream);
// The filtered least-median-of-squares form: the workspace's parts (device memory) and shape.
struct LmsFilterBufs {
  double *R;             // m x n: each candidate's kept squares by segment; the whole array
                         // of a candidate whose bracket missed
  double *C;             // m x cap: each candidate's kept squares, packed
  int64_t cap;
  double *Rs;            // m x S: the squares of the sampled rows (S <= 16384)
  double *ab;            // 2m: the sampled brackets
  uint32_t *cnt;         // 2 x m x nseg: kept and #(r <= a) per candidate and segment
  double *psum;          // m x nseg: the sum of the r <= a per candidate and segment (with
                         // the trimmed sums only)
  int32_t *full;         // m: 1 where the candidate's whole array is formed and selected
  int64_t bx, nseg, seg;  // the fallback kernel's workgroups per candidate group; segments
                          // per candidate and rows per segment of the filter
};
void lms_filter_shape(int64_t n, int64_t m, int32_t p, bool vec, int cu_count, int64_t *bx,
                      int64_t *nseg, int64_t *seg);
int64_t lms_filter_cap(int64_t n);
// Every kernel of the filtered form; the medians land in out (m records).
// ksum (or null): m doubles, each candidate's sum of its `rank` smallest squares.
hipError_t launch_lms_filtered(const double *X, const double *y, const double *betas, int64_t n,
                               int32_t p, int64_t m, int64_t rank, const LmsFilterBufs &w,
                               cps_result *out, double *ksum, hipStream_t stream);
hipError_t launch_lts_finish(const cps_result *sel, const double *ksum, int64_t m, int64_t h,
                             cps_trim *out, hipStream_t stream);

// ---- k nearest neighbours
// The filtered kNN form's workspace (device memory) and shape.
struct KnnFilterBufs {
  float *Ds;           // nq x S: distances of the sampled points (S <= 16384)
  float *ab;           // 2 nq: the sampled brackets
  uint32_t *cnt;       // 2 nq: kept count (cursor), #(d <= a)
  double *fsum;        // nq: the ordinates' sum over d <= a
  float *K;            // nq x kKnnCap x 2: kept distances and ordinates
  int64_t nseg, seg;   // the filter's segments and points per segment
};
// kept distances per query (the filtered form); 8128 keeps the select kernel under half a
// CU's LDS (two workgroups per CU; at 8192 it was 208 bytes over and ran one)
constexpr int64_t kKnnKeptCap = 8128;
void knn_filter_shape(int64_t n, int64_t nq, int cu_count, int64_t *nseg, int64_t *seg);
hipError_t launch_knn_filtered(const float *P, const float *f, const float *Q, int64_t n,
                               int32_t dim, int64_t nq, int64_t k, const KnnFilterBufs &w,
                               cps_knn *out, hipStream_t stream);
hipError_t launch_knn_distances(const float *P, const float *Q, int64_t n, int32_t dim, int64_t nq,
                                int64_t k, float *Dst, const float **ptrs, int64_t *sizes,
                                int64_t *ks, int cu_count, hipStream_t stream);
hipError_t launch_knn_reduce(const float *P, const float *f, const float *Q, const float *Dst,
                             int64_t n, int32_t dim, int64_t nq, int64_t k, const cps_result *sel,
                             double *pd, int64_t *pi, cps_knn *out, hipStream_t stream);

template <typename T>
hipError_t launch_select(const SelectArgs<T> &a, int grid, bool cooperative, hipStream_t stream);
template <typename T> int select_max_blocks_per_cu();
template <typename T>
hipError_t launch_objective(const T *x, int64_t n, int64_t k, const double *ys, int64_t ny,
                            cps_eval *out, double *pd, int64_t *pi, int nb, hipStream_t stream);

// ---- the selection without allocation (select_kth_noalloc)

// Size of the per-device scratch array, and the largest grid it serves: the state, the
// synchronisation words, 2 x 4096 histogram counters, 16 partial words per workgroup and a
// gather buffer of the final threshold (8192 elements): about 300 KiB at 1024 workgroups.
constexpr size_t kNoAllocScratchBytes = (size_t)1 << 20;
constexpr int kNoAllocMaxGrid = 1024;

// Take the scratch array's device address on `device`, which must be current (once per
// device; later calls return at once).
hipError_t noalloc_bind(int device);
// That address, or null when noalloc_bind has not run for the device.
void *noalloc_scratch(int device);
// Zero `bytes` (a multiple of 8) at p with a fill kernel.
hipError_t launch_scratch_clear(void *p, size_t bytes, hipStream_t stream);

// ---- learned bracket proposal

hipError_t launch_mixture_gen(uint64_t seed, int64_t first_id, int64_t count, int64_t n,
                              float *out, int64_t *ks, hipStream_t stream);
template <typename T>
hipError_t launch_features(const T *const *ptrs, const int64_t *sizes, const int64_t *ks,
                           int64_t count, float *feat, double *range, int32_t *valid,
                           hipStream_t stream);
hipError_t launch_mlp_forward(const float *P, const float *feat, int64_t count, float *out,
                              hipStream_t stream);
size_t mlp_grad_workspace(int64_t count);
hipError_t launch_mlp_loss_grad(const float *P, const float *feat, const float *ustar,
                                int64_t count, float *grad, float *loss, float *ws,
                                hipStream_t stream);
hipError_t launch_mlp_adam(float *P, const float *g, float *m, float *v, int64_t step, float lr,
                           float b1, float b2, float eps, hipStream_t stream);
hipError_t launch_mlp_init(uint64_t seed, float *P, hipStream_t stream);
template <typename T>
hipError_t launch_learned_bracket(const T *x, int64_t n, int64_t k, const float *P,
                                  uint64_t *zero_hist, double *bracket, hipStream_t stream);
template <typename T>
hipError_t launch_sample_bracket(const T *x, int64_t n, int64_t k, double z, uint64_t *zero_hist,
                                 double *bracket, hipStream_t stream);
hipError_t launch_batch_descriptors(const float *base, int64_t n, int64_t count, const float **ptrs,
                                    int64_t *sizes, hipStream_t stream);
hipError_t launch_labels(const cps_result *res, const float *feat, const double *range,
                         const int32_t *valid, int64_t count, float *ustar, hipStream_t stream);
hipError_t launch_holdout(const float *out, const float *feat, const double *range,
                          const int32_t *valid, const cps_result *res, int64_t count, double *acc,
                          hipStream_t stream);

}  // namespace cps
