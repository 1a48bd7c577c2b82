// C ABI of the selection library: handles, argument checks, workspace, launches.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <string>
#include <type_traits>
#include <mutex>
#include <vector>

#include "cps_kernels.h"

namespace {

thread_local int g_last_hip = 0;

inline int hip_fail(hipError_t e) {
  g_last_hip = (int)e;
  return CPS_EHIP;
}

inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

}  // namespace

struct cps_handle {
  int device = 0;
  int cu_count = 0;
  int max_blocks_f32 = 0;
  int max_blocks_f64 = 0;
  void *ws = nullptr;   // single-array workspace
  size_t ws_bytes = 0;
  void *bws = nullptr;  // batched workspace (queue counters first)
  size_t bws_bytes = 0;
  cps::TeamCtl *tws = nullptr;  // team records of the batched kernel (zeroed once)
  void *lws = nullptr;  // least-median-of-squares residuals and descriptors
  size_t lws_bytes = 0;
  void *mws = nullptr;  // per-workgroup gradient partials of the proposal network
  size_t mws_bytes = 0;
  void *ows = nullptr;  // partials of the reference objective (cps_objective)
  size_t ows_bytes = 0;
  double *bracket = nullptr;  // the learned proposal handed to the selection (a, b, use)
  uint64_t *phist = nullptr;  // counters of the proposal's interior (same allocation)
  cps_batch_options tuned[2];
  bool has_tuned[2] = {false, false};
  std::mutex mu;
};

namespace {

// Workspace layout of a single-array selection: state, synchronisation words, per-workgroup
// partials, two split buffers (one region of seg_R elements per workgroup each) and the
// gather buffer.
struct SelectLayout {
  size_t st, sync, gh, sd, si, z0, z1, zf, sm, total;
  int64_t slot_stride, seg_R, zcap, smp_n;
};

SelectLayout select_layout(int64_t seg_R, int grid, int64_t zcap, int gmax, size_t esize,
                           int64_t smp_n = 0) {
  SelectLayout L;
  size_t off = 0;
  L.st = off;
  off = align_up(off + sizeof(cps::CpState), 256);
  L.sync = off;
  off = align_up(off + sizeof(cps::SyncCtl), 256);
  L.gh = off;  // histogram counters, inside the cleared first part of fresh memory
  off = align_up(off + cps::kHistWords * sizeof(uint64_t), 256);
  L.slot_stride = gmax;
  L.sd = off;
  off = align_up(off + 8 * (size_t)gmax * sizeof(double), 256);
  L.si = off;
  off = align_up(off + 8 * (size_t)gmax * sizeof(int64_t), 256);
  L.seg_R = seg_R;
  L.z0 = off;
  const size_t zbytes = (size_t)seg_R * grid * (cps::kSelectBlock / cps::kWaveSize) * esize;
  off = align_up(off + zbytes, 256);
  L.z1 = off;
  off = align_up(off + zbytes, 256);
  L.zcap = zcap;
  L.zf = off;
  off = align_up(off + (size_t)zcap * esize, 256);
  L.smp_n = smp_n;
  L.sm = off;
  off = align_up(off + (size_t)smp_n * esize, 256);
  L.total = off;
  return L;
}

// Elements of pass 0's sample for the likely interval: one 16-byte vector per tile of x, when
// the input is large enough for the counting evaluation's copy (0 otherwise).
int64_t spec_sample_elems(int64_t n, size_t esize, int64_t spec_min_n) {
  if (spec_min_n <= 0 || n < spec_min_n) return 0;
  const int64_t vec = 16 / (int64_t)esize;
  const int64_t tile = (int64_t)cps::kSelectBlock * cps::kSelectUnroll;  // vectors per tile
  const int64_t tiles = (n / vec + tile - 1) / tile;
  return (tiles < 1 ? 1 : tiles) * vec;
}

// Grow a workspace buffer to at least `bytes`.  The synchronisation words at the start of
// every layout must be zero on first use, so fresh memory is cleared synchronously.
int ensure_buffer(void *&buf, size_t &have, size_t bytes, hipStream_t stream);

int ensure_workspace(cps_handle *h, size_t bytes, hipStream_t stream) {
  return ensure_buffer(h->ws, h->ws_bytes, bytes, stream);
}

int ensure_buffer(void *&buf, size_t &have, size_t bytes, hipStream_t stream) {
  if (bytes <= have) return CPS_OK;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (stream != nullptr) {
    hipError_t e = hipStreamIsCapturing(stream, &cs);
    if (e != hipSuccess) return hip_fail(e);
    if (cs != hipStreamCaptureStatusNone) return CPS_ECAPTURE;
  }
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e);
  if (buf) {
    (void)hipFree(buf);
    buf = nullptr;
    have = 0;
  }
  size_t want = align_up(bytes + bytes / 8, 1 << 20);
  e = hipMalloc(&buf, want);
  if (e != hipSuccess) {
    g_last_hip = (int)e;
    buf = nullptr;
    return CPS_ENOMEM;
  }
  e = hipMemset(buf, 0, want < (1 << 21) ? want : (1 << 21));
  if (e != hipSuccess) return hip_fail(e);
  have = want;
  return CPS_OK;
}

// The team records of the batched kernel: allocated and zeroed once per handle (every use
// leaves them zero again).
int ensure_team_records(cps_handle *h, hipStream_t stream) {
  if (h->tws) return CPS_OK;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (stream != nullptr) {
    hipError_t e = hipStreamIsCapturing(stream, &cs);
    if (e != hipSuccess) return hip_fail(e);
    if (cs != hipStreamCaptureStatusNone) return CPS_ECAPTURE;
  }
  const size_t bytes = (size_t)cps::kTeamRecords * sizeof(cps::TeamCtl);
  void *p = nullptr;
  hipError_t e = hipMalloc(&p, bytes);
  if (e != hipSuccess) {
    g_last_hip = (int)e;
    return CPS_ENOMEM;
  }
  e = hipMemset(p, 0, bytes);
  if (e == hipSuccess) e = hipDeviceSynchronize();
  if (e != hipSuccess) {
    (void)hipFree(p);
    return hip_fail(e);
  }
  h->tws = (cps::TeamCtl *)p;
  return CPS_OK;
}

inline size_t dtype_size(int dtype) { return dtype == CPS_F32 ? 4 : (dtype == CPS_F64 ? 8 : 0); }

struct Resolved {
  cps::CpConfig cfg;
  int grid;
  int64_t seg_R;
  int64_t spin_limit;
  int compact_proposal;
  bool cooperative;
};

int resolve(cps_handle *h, int64_t n, int dtype, const cps_options *opt, Resolved &r) {
  cps_options o;
  cps_default_options(&o);
  if (opt) o = *opt;
  if (o.maxit < 0 || o.final_threshold < 1 || !(o.partition_fraction >= 0.0) ||
      o.partition_fraction > 1.0 || o.grid_blocks < 0 || o.spin_limit < 0 ||
      o.cooperative < 0 || o.cooperative > 1)
    return CPS_EINVAL;
  r.cooperative = o.cooperative != 0;
  if (o.block_threads != 0 && o.block_threads != cps::kSelectBlock) return CPS_EINVAL;
  if (o.hist_bits < 0 || (1 << o.hist_bits) > cps::kHistMaxBins) return CPS_EINVAL;
  r.cfg = cps::CpConfig{};
  r.cfg.maxit = o.maxit;
  r.cfg.dtype = dtype;
  r.cfg.final_threshold = o.final_threshold;
  r.cfg.final_direct_max = 4 * (int64_t)o.final_threshold;
  r.cfg.theta = o.partition_fraction;
  r.cfg.zcap = o.final_threshold;
  r.cfg.use_bracket = o.use_bracket ? 1 : 0;
  r.cfg.bracket_lo = o.bracket_lo;
  r.cfg.bracket_hi = o.bracket_hi;
  r.cfg.hist_bits = o.hist_bits;
  r.cfg.hist_compact = 1;  // the single-array kernel compacts in its histogram passes
  r.cfg.count_first = o.count_first ? 1 : 0;
  if (o.transform) {
    // the transformed objective runs without splits, and never with a proposed bracket
    if (o.transform != 1 || o.use_bracket) return CPS_EINVAL;
    r.cfg.transform = 1;
    if (o.hist_bits > 0) r.cfg.count_first = 1;
    else r.cfg.theta = 0.0;
  }
  // from 256 MiB of input on (2^26 float or 2^25 double elements), the counting evaluation
  // also copies a likely interval; below, the pass over x that the copy saves costs about
  // what the copy and the interval's sample cost (measured: 2^24 float32 selections 0.169-
  // 0.21 ms with it against 0.156-0.196 without; 2^25 float32 even; 2^26 float32 5 %,
  // 2^25 float64 4 %, 2^26 float64 10 % and 2^28 ones ~20 % faster with it)
  r.cfg.spec_min_n = ((int64_t)1 << 28) / (int64_t)dtype_size(dtype);
  const int per_cu = dtype == CPS_F32 ? h->max_blocks_f32 : h->max_blocks_f64;
  const int gmax = h->cu_count * per_cu;
  if (gmax < 1) return CPS_ENODEV;
  const int64_t tile = (int64_t)cps::kSelectBlock * cps::kSelectUnroll * (16 / dtype_size(dtype));
  int64_t g = o.grid_blocks ? o.grid_blocks : (int64_t)h->cu_count * per_cu;
  const int64_t tiles = (n + tile - 1) / tile;
  if (g > tiles) g = tiles;
  if (g > gmax) g = gmax;
  if (g > (int64_t)cps::kGroup * cps::kMaxGroups) g = (int64_t)cps::kGroup * cps::kMaxGroups;
  if (g < 1) g = 1;
  r.grid = (int)g;
  // Each wavefront's split region holds everything it can read in a pass over the input
  // that writes to it (the first split, with half the unroll, or the histogram pass that
  // compacts a counted bin, with the full unroll): its share of each of its workgroup's
  // steps, plus the unaligned edge elements, rounded to 64 elements.
  int64_t seg = 0;
  if (o.partition_fraction > 0.0) {
    const int64_t vec = 16 / (int64_t)dtype_size(dtype);
    const int64_t nvec = n / vec + 1;
    for (const int64_t su : {(int64_t)cps::kSplitUnroll, (int64_t)cps::kSelectUnroll}) {
      const int64_t step_vecs = (int64_t)cps::kSelectBlock * su;
      const int64_t steps = (nvec + step_vecs - 1) / step_vecs;
      const int64_t steps_per_wg = (steps + g - 1) / g;
      const int64_t need = (steps_per_wg * cps::kWaveSize * su * vec + 8 + 63) / 64 * 64;
      if (need > seg) seg = need;
    }
  }
  r.seg_R = seg;
  r.spin_limit = o.spin_limit ? o.spin_limit : (int64_t)1 << 22;
  r.compact_proposal = o.compact_proposal ? 1 : 0;
  return CPS_OK;
}

// bracket_dev: a device-side proposal (a, b, use) read by pass 0, or null.
template <typename T>
int run_select(cps_handle *h, const T *x, int64_t n, int64_t k, const cps_options *opt,
               cps_result *out, cps_stats *stats, hipStream_t stream,
               const double *bracket_dev = nullptr) {
  Resolved r;
  int rc = resolve(h, n, sizeof(T) == 4 ? CPS_F32 : CPS_F64, opt, r);
  if (rc) return rc;
  const int per_cu = sizeof(T) == 4 ? h->max_blocks_f32 : h->max_blocks_f64;
  const SelectLayout L = select_layout(r.seg_R, r.grid, r.cfg.zcap, h->cu_count * per_cu, sizeof(T),
                                       spec_sample_elems(n, sizeof(T), r.cfg.spec_min_n));
  rc = ensure_workspace(h, L.total, stream);
  if (rc) return rc;
  char *base = (char *)h->ws;
  cps::SelectArgs<T> a;
  a.x = x;
  a.n = n;
  a.k = k;
  a.st = (cps::CpState *)(base + L.st);
  a.sync = (cps::SyncCtl *)(base + L.sync);
  a.sd = (double *)(base + L.sd);
  a.si = (int64_t *)(base + L.si);
  a.slot_stride = L.slot_stride;
  a.z[0] = (T *)(base + L.z0);
  a.z[1] = (T *)(base + L.z1);
  a.seg_R = L.seg_R;
  a.zf = (T *)(base + L.zf);
  a.out = out;
  a.stats = stats;
  a.cfg = r.cfg;
  a.spin_limit = r.spin_limit;
  a.bracket = bracket_dev;
  // the proposal kernel that wrote bracket_dev also cleared the interior's counters
  a.phist = (bracket_dev != nullptr && bracket_dev == h->bracket) ? h->phist : nullptr;
  // a proposed bracket's interior may take up to half of each wavefront's region in pass 0
  // (past about two thirds of the input, the passes over x that compaction would spare
  // cost less than reading the compacted elements again)
  const bool proposal = bracket_dev != nullptr || r.cfg.use_bracket != 0;
  if (proposal && r.cfg.transform) return CPS_EINVAL;
  a.p0_cap = (proposal && r.compact_proposal) ? L.seg_R / 2 : 0;
  a.ghist = (uint64_t *)(base + L.gh);
  a.smp = L.smp_n > 0 ? (T *)(base + L.sm) : nullptr;
  a.smp_n = L.smp_n;
  hipError_t e = cps::launch_select<T>(a, r.grid, r.cooperative, stream);
  if (e != hipSuccess) return hip_fail(e);
  return CPS_OK;
}

int check_common(cps_handle *h, const void *x, int64_t n, int64_t k, int dtype) {
  if (!h || !x || n < 1 || k < 1 || k > n) return CPS_EINVAL;
  const size_t es = dtype_size(dtype);
  if (!es) return CPS_EINVAL;
  if (((uintptr_t)x) % es) return CPS_EINVAL;
  return CPS_OK;
}

// ---- batched selection

struct BatchResolved {
  cps::CpConfig cfg;
  int grid, block;
  int64_t cap, ws_stride, gb_off;
  int32_t proposal, team_max;
  int64_t team_chunk, team_cap, team_records;
  size_t wg_off, bytes;  // per-workgroup buffers at wg_off (after the team buffers)
};

int resolve_batched(cps_handle *h, int dtype, int64_t count, const cps_batch_options *opt,
                    BatchResolved &r) {
  cps_batch_options o;
  cps_default_batch_options(&o);
  const int di = dtype == CPS_F32 ? 0 : 1;
  if (opt) o = *opt;
  else if (h->has_tuned[di]) o = h->tuned[di];
  if (o.block_threads == 0) o.block_threads = 1024;
  if (o.block_threads != 256 && o.block_threads != 512 && o.block_threads != 1024) return CPS_EINVAL;
  if (o.blocks_per_cu < 0 || o.split_capacity < 0 || o.final_threshold < 0 || o.maxit < 0 ||
      !(o.partition_fraction >= 0.0) || o.partition_fraction > 1.0 || o.hist_bits < 0 ||
      (1 << o.hist_bits) > cps::kHistMaxBins || o.proposal < 0 || o.proposal > 1 ||
      o.blocks_per_array < 0 || o.blocks_per_array > cps::kTeamMax || o.elements_per_block < 0 ||
      (o.elements_per_block > 0 && o.elements_per_block < ((int64_t)1 << 15)) ||
      o.team_capacity < 0)
    return CPS_EINVAL;
  const size_t es = dtype_size(dtype);
  const int per_cu = dtype == CPS_F32 ? cps::batched_max_blocks_per_cu<float>(o.block_threads)
                                      : cps::batched_max_blocks_per_cu<double>(o.block_threads);
  if (per_cu < 1) return CPS_ENODEV;
  int bpc = o.blocks_per_cu ? o.blocks_per_cu : per_cu;
  if (bpc > per_cu) bpc = per_cu;
  r.block = o.block_threads;
  r.grid = h->cu_count * bpc;
  const int64_t ft = o.final_threshold ? o.final_threshold : 4096;
  r.proposal = (o.proposal && o.hist_bits > 0) ? 1 : 0;
  r.team_max = r.proposal ? (o.blocks_per_array ? o.blocks_per_array : 1) : 1;
  r.team_chunk = o.elements_per_block ? o.elements_per_block : ((int64_t)1 << 18);
  r.team_cap = ((o.team_capacity ? o.team_capacity : ((int64_t)1 << 18)) + 63) / 64 * 64;
  r.cap = o.split_capacity ? o.split_capacity : ((int64_t)1 << 17);
  // with the counting evaluation (and key bins) nothing is ever split: no split buffers,
  // except one for the sampled bracket's copy of an array taken by one workgroup (the team
  // capacity: the copied vectors are ~23 % of a float array, ~12 % of a double one)
  if (o.count_first && o.hist_bits > 0) r.cap = !r.proposal ? ft : r.team_cap;
  if (r.cap < ft) r.cap = ft;
  r.cap = (r.cap + 63) / 64 * 64;
  // (the counting evaluation never splits: the second split buffer is not needed)
  r.gb_off = ((o.count_first && o.hist_bits > 0) ? 1 : 2) * r.cap;
  r.ws_stride = r.gb_off + (ft + 63) / 64 * 64;
  // team records for the largest-first slots that may be split (sorted batches only)
  r.team_records = 0;
  if (r.team_max > 1 && count <= cps::kBatchSortMax)
    r.team_records = count < cps::kTeamRecords ? count : cps::kTeamRecords;
  r.wg_off = align_up(sizeof(cps::BatchCtl), 256) +
             align_up((size_t)r.team_records * r.team_cap * es, 256);
  r.bytes = r.wg_off + (size_t)r.grid * r.ws_stride * es;
  r.cfg = cps::CpConfig{};
  r.cfg.maxit = o.maxit ? o.maxit : 64;
  r.cfg.dtype = dtype;
  r.cfg.final_threshold = ft;
  r.cfg.final_direct_max = 4 * ft;
  r.cfg.theta = o.partition_fraction;
  r.cfg.zcap = ft;
  r.cfg.split_cap = r.cap;
  r.cfg.hist_bits = o.hist_bits;
  r.cfg.count_first = o.count_first ? 1 : 0;
  return CPS_OK;
}

template <typename T>
int run_batched(cps_handle *h, const void *const *ptrs, const int64_t *sizes, const int64_t *ks,
                int64_t count, const cps_batch_options *opt, cps_result *out, double *ksum,
                hipStream_t stream) {
  BatchResolved r;
  int rc = resolve_batched(h, sizeof(T) == 4 ? CPS_F32 : CPS_F64, count, opt, r);
  if (rc) return rc;
  rc = ensure_buffer(h->bws, h->bws_bytes, r.bytes, stream);
  if (rc) return rc;
  if (r.team_records > 0 && (rc = ensure_team_records(h, stream))) return rc;
  cps::BatchArgs<T> a;
  a.ptrs = (const T *const *)ptrs;
  a.sizes = sizes;
  a.ks = ks;
  a.count = count;
  a.out = out;
  a.ctl = (cps::BatchCtl *)h->bws;
  a.tbuf = (T *)((char *)h->bws + align_up(sizeof(cps::BatchCtl), 256));
  a.zbuf = (T *)((char *)h->bws + r.wg_off);
  a.cap = r.cap;
  a.ws_stride = r.ws_stride;
  a.gb_off = r.gb_off;
  a.cfg = r.cfg;
  a.proposal = r.proposal;
  a.team_max = r.team_max;
  a.team_chunk = r.team_chunk;
  a.team_cap = r.team_cap;
  a.team_records = r.team_records;
  a.teams = h->tws;
  a.ksum = ksum;
  hipError_t e = cps::launch_batched<T>(a, r.grid, r.block, stream);
  if (e != hipSuccess) return hip_fail(e);
  return CPS_OK;
}

int check_batched(cps_handle *h, const void *const *ptrs, const int64_t *sizes, const int64_t *ks,
                  int64_t count, int dtype, cps_result *out) {
  if (!h || !ptrs || !sizes || !ks || !out || count < 1 || !dtype_size(dtype)) return CPS_EINVAL;
  return CPS_OK;
}

}  // namespace

extern "C" {

void cps_default_batch_options(cps_batch_options *opt) {
  if (!opt) return;
  std::memset(opt, 0, sizeof(*opt));
  opt->block_threads = 1024;
  opt->blocks_per_cu = 0;
  opt->split_capacity = (int64_t)1 << 17;
  opt->final_threshold = 4096;
  opt->maxit = 64;
  opt->partition_fraction = 1.0;
  opt->hist_bits = 12;
  opt->count_first = 1;
  opt->proposal = 1;
  opt->blocks_per_array = 1;
  opt->elements_per_block = (int64_t)1 << 18;
  opt->team_capacity = (int64_t)1 << 18;
}

int select_kth_batched_ksum(cps_handle *h, const void *const *ptrs_dev, const int64_t *sizes_dev,
                            const int64_t *ks_dev, int64_t count, int dtype,
                            const cps_batch_options *opt, cps_result *out_dev, double *ksum_dev,
                            void *stream) {
  int rc = check_batched(h, ptrs_dev, sizes_dev, ks_dev, count, dtype, out_dev);
  if (rc) return rc;
  std::lock_guard<std::mutex> lk(h->mu);
  if (dtype == CPS_F32)
    return run_batched<float>(h, ptrs_dev, sizes_dev, ks_dev, count, opt, out_dev, ksum_dev,
                              (hipStream_t)stream);
  return run_batched<double>(h, ptrs_dev, sizes_dev, ks_dev, count, opt, out_dev, ksum_dev,
                             (hipStream_t)stream);
}

int select_kth_batched_ex(cps_handle *h, const void *const *ptrs_dev, const int64_t *sizes_dev,
                          const int64_t *ks_dev, int64_t count, int dtype,
                          const cps_batch_options *opt, cps_result *out_dev, void *stream) {
  return select_kth_batched_ksum(h, ptrs_dev, sizes_dev, ks_dev, count, dtype, opt, out_dev,
                                 nullptr, stream);
}

int select_kth_batched(cps_handle *h, const void *const *ptrs_dev, const int64_t *sizes_dev,
                       const int64_t *ks_dev, int64_t count, int dtype, cps_result *out_dev,
                       void *stream) {
  return select_kth_batched_ex(h, ptrs_dev, sizes_dev, ks_dev, count, dtype, nullptr, out_dev, stream);
}

int cps_reserve_batched(cps_handle *h, int dtype, const cps_batch_options *opt) {
  if (!h || !dtype_size(dtype)) return CPS_EINVAL;
  std::lock_guard<std::mutex> lk(h->mu);
  BatchResolved r;
  // workspace for the largest batch that may split arrays
  int rc = resolve_batched(h, dtype, cps::kBatchSortMax, opt, r);
  if (rc) return rc;
  rc = ensure_buffer(h->bws, h->bws_bytes, r.bytes, nullptr);
  if (rc) return rc;
  return r.team_records > 0 ? ensure_team_records(h, nullptr) : CPS_OK;
}

// The filtered form's workspace and launches (the handle's lock held): R (m x n), C (m x cap),
// sampled squares, brackets, segment counts, flags, and with ksum_out the segments' sums and
// m records and sums of its own (the selections then land there, *sel_out and *ksum_out
// point at them).
static int lms_filtered_run(cps_handle *h, const double *X_dev, const double *y_dev,
                            const double *betas_dev, int64_t n, int32_t p, int64_t m, int64_t rank,
                            cps_result *out_dev, cps_result **sel_out, double **ksum_out,
                            hipStream_t s) {
  const size_t dsz = align_up((size_t)m * 8, 256);
  cps::LmsFilterBufs w;
  const bool vec = (uintptr_t)X_dev % 16 == 0 && (uintptr_t)y_dev % 16 == 0;
  cps::lms_filter_shape(n, m, p, vec, h->cu_count, &w.bx, &w.nseg, &w.seg);
  w.cap = cps::lms_filter_cap(n);
  const bool sums = ksum_out != nullptr;
  const size_t off_c = align_up((size_t)m * (size_t)n * sizeof(double), 256);
  const size_t off_rs = off_c + align_up((size_t)m * (size_t)w.cap * sizeof(double), 256);
  const size_t off_ab = off_rs + align_up((size_t)m * 16384 * sizeof(double), 256);
  const size_t off_cnt = off_ab + 2 * dsz;
  const size_t off_full = off_cnt + align_up((size_t)2 * m * w.nseg * sizeof(uint32_t), 256);
  const size_t off_psum = off_full + dsz;
  const size_t off_sel = off_psum + (sums ? align_up((size_t)m * w.nseg * sizeof(double), 256) : 0);
  const size_t off_ksum = off_sel + (sums ? align_up((size_t)m * sizeof(cps_result), 256) : 0);
  const size_t bytes = off_ksum + (sums ? dsz : 0);
  int rc = ensure_buffer(h->lws, h->lws_bytes, bytes, s);
  if (rc) return rc;
  char *base = (char *)h->lws;
  w.R = (double *)base;
  w.C = (double *)(base + off_c);
  w.Rs = (double *)(base + off_rs);
  w.ab = (double *)(base + off_ab);
  w.cnt = (uint32_t *)(base + off_cnt);
  w.full = (int32_t *)(base + off_full);
  w.psum = sums ? (double *)(base + off_psum) : nullptr;
  cps_result *sel = sums ? (cps_result *)(base + off_sel) : out_dev;
  double *ksum = sums ? (double *)(base + off_ksum) : nullptr;
  if (sel_out) *sel_out = sel;
  if (ksum_out) *ksum_out = ksum;
  hipError_t e = cps::launch_lms_filtered(X_dev, y_dev, betas_dev, n, p, m, rank, w, sel, ksum, s);
  return e == hipSuccess ? CPS_OK : hip_fail(e);
}

static bool lms_can_filter(int64_t n) { return n >= ((int64_t)1 << 15) && n < ((int64_t)1 << 31); }

int lms_median_sq_residuals_ex(cps_handle *h, const double *X_dev, const double *y_dev,
                               const double *betas_dev, int64_t n, int32_t p, int64_t m,
                               int32_t form, cps_result *out_dev, void *stream) {
  if (!h || !X_dev || !y_dev || !betas_dev || !out_dev || n < 1 || p < 1 || p > 16 || m < 1 ||
      m > (int64_t)65535 * 16 || form < CPS_LMS_AUTO || form > CPS_LMS_FILTERED)
    return CPS_EINVAL;
  const bool can_filter = lms_can_filter(n);
  if (form == CPS_LMS_FILTERED && !can_filter) return CPS_EINVAL;
  const bool filtered = form == CPS_LMS_FILTERED || (form == CPS_LMS_AUTO && can_filter);
  hipStream_t s = (hipStream_t)stream;
  const int64_t rank = (n + 1) / 2;
  std::lock_guard<std::mutex> lk(h->mu);
  if (filtered)
    return lms_filtered_run(h, X_dev, y_dev, betas_dev, n, p, m, rank, out_dev, nullptr, nullptr, s);
  const size_t dsz = align_up((size_t)m * 8, 256);
  const size_t off_desc = align_up((size_t)m * (size_t)n * sizeof(double), 256);
  const size_t bytes = off_desc + 3 * dsz;
  int rc = ensure_buffer(h->lws, h->lws_bytes, bytes, s);
  if (rc) return rc;
  char *base = (char *)h->lws;
  hipError_t e = cps::launch_lms_residuals(X_dev, y_dev, betas_dev, n, p, m, rank, (double *)base,
                                           (const double **)(base + off_desc),
                                           (int64_t *)(base + off_desc + dsz),
                                           (int64_t *)(base + off_desc + 2 * dsz), h->cu_count, s);
  if (e != hipSuccess) return hip_fail(e);
  // the batched defaults: one 1024-thread workgroup per candidate at a time, the counting
  // evaluation at the first trial point
  cps_batch_options o;
  cps_default_batch_options(&o);
  return run_batched<double>(h, (const void *const *)(base + off_desc),
                             (const int64_t *)(base + off_desc + dsz),
                             (const int64_t *)(base + off_desc + 2 * dsz), m, &o, out_dev, nullptr,
                             s);
}

int lms_median_sq_residuals(cps_handle *h, const double *X_dev, const double *y_dev,
                            const double *betas_dev, int64_t n, int32_t p, int64_t m,
                            cps_result *out_dev, void *stream) {
  return lms_median_sq_residuals_ex(h, X_dev, y_dev, betas_dev, n, p, m, CPS_LMS_AUTO, out_dev,
                                    stream);
}

int lts_trimmed_sq_ex(cps_handle *h, const double *X_dev, const double *y_dev,
                      const double *betas_dev, int64_t n, int32_t p, int64_t m, int64_t hk,
                      int32_t form, cps_trim *out_dev, void *stream) {
  if (!h || !X_dev || !y_dev || !betas_dev || !out_dev || n < 1 || p < 1 || p > 16 || m < 1 ||
      m > (int64_t)65535 * 16 || hk < 1 || hk > n || form < CPS_LMS_AUTO || form > CPS_LMS_FILTERED)
    return CPS_EINVAL;
  const bool can_filter = lms_can_filter(n);
  if (form == CPS_LMS_FILTERED && !can_filter) return CPS_EINVAL;
  const bool filtered = form == CPS_LMS_FILTERED || (form == CPS_LMS_AUTO && can_filter);
  hipStream_t s = (hipStream_t)stream;
  if (filtered) {
    std::lock_guard<std::mutex> lk(h->mu);
    cps_result *sel = nullptr;
    double *ksum = nullptr;
    int rc = lms_filtered_run(h, X_dev, y_dev, betas_dev, n, p, m, hk, nullptr, &sel, &ksum, s);
    if (rc) return rc;
    hipError_t e = cps::launch_lts_finish(sel, ksum, m, hk, out_dev, s);
    return e == hipSuccess ? CPS_OK : hip_fail(e);
  }
  // residuals, then descriptors, selections, sums and records, in the workspace
  const size_t off_desc = align_up((size_t)m * (size_t)n * sizeof(double), 256);
  const size_t dsz = align_up((size_t)m * 8, 256);
  const size_t off_sel = off_desc + 3 * dsz;
  const size_t off_sum = off_sel + align_up((size_t)m * sizeof(cps_result), 256);
  const size_t bytes = off_sum + dsz;
  char *base;
  {
    std::lock_guard<std::mutex> lk(h->mu);
    int rc = ensure_buffer(h->lws, h->lws_bytes, bytes, s);
    if (rc) return rc;
    base = (char *)h->lws;
    hipError_t e = cps::launch_lms_residuals(X_dev, y_dev, betas_dev, n, p, m, hk, (double *)base,
                                             (const double **)(base + off_desc),
                                             (int64_t *)(base + off_desc + dsz),
                                             (int64_t *)(base + off_desc + 2 * dsz), h->cu_count, s);
    if (e != hipSuccess) return hip_fail(e);
  }
  cps_batch_options o;
  cps_default_batch_options(&o);
  int rc = select_kth_batched_ksum(h, (const void *const *)(base + off_desc),
                                   (const int64_t *)(base + off_desc + dsz),
                                   (const int64_t *)(base + off_desc + 2 * dsz), m, CPS_F64, &o,
                                   (cps_result *)(base + off_sel), (double *)(base + off_sum),
                                   stream);
  if (rc) return rc;
  hipError_t e = cps::launch_lts_finish((const cps_result *)(base + off_sel),
                                        (const double *)(base + off_sum), m, hk, out_dev, s);
  return e == hipSuccess ? CPS_OK : hip_fail(e);
}

int lts_trimmed_sq(cps_handle *h, const double *X_dev, const double *y_dev,
                   const double *betas_dev, int64_t n, int32_t p, int64_t m, int64_t hk,
                   cps_trim *out_dev, void *stream) {
  return lts_trimmed_sq_ex(h, X_dev, y_dev, betas_dev, n, p, m, hk, CPS_LMS_AUTO, out_dev, stream);
}

int knn_mean_ex(cps_handle *h, const float *P_dev, const float *f_dev, const float *Q_dev,
                int64_t n, int32_t dim, int64_t nq, int64_t k, int32_t form, cps_knn *out_dev,
                void *stream) {
  if (!h || !P_dev || !f_dev || !Q_dev || !out_dev || n < 1 || dim < 1 || dim > 16 || nq < 1 ||
      nq > 65535 || k < 1 || k > n || form < CPS_LMS_AUTO || form > CPS_LMS_FILTERED)
    return CPS_EINVAL;
  const bool can_filter = lms_can_filter(n);
  if (form == CPS_LMS_FILTERED && !can_filter) return CPS_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  if (form == CPS_LMS_FILTERED || (form == CPS_LMS_AUTO && can_filter)) {
    // sampled distances, brackets, counters, ordinate sums, kept distances and ordinates
    std::lock_guard<std::mutex> lk(h->mu);
    cps::KnnFilterBufs w;
    cps::knn_filter_shape(n, nq, h->cu_count, &w.nseg, &w.seg);
    const size_t off_ab = align_up((size_t)nq * 16384 * sizeof(float), 256);
    const size_t off_cnt = off_ab + align_up((size_t)nq * 2 * sizeof(float), 256);
    const size_t off_fs = off_cnt + align_up((size_t)nq * 2 * sizeof(uint32_t), 256);
    const size_t off_k = off_fs + align_up((size_t)nq * sizeof(double), 256);
    const size_t bytes = off_k + (size_t)nq * cps::kKnnKeptCap * 2 * sizeof(float);
    int rc = ensure_buffer(h->lws, h->lws_bytes, bytes, s);
    if (rc) return rc;
    char *base = (char *)h->lws;
    w.Ds = (float *)base;
    w.ab = (float *)(base + off_ab);
    w.cnt = (uint32_t *)(base + off_cnt);
    w.fsum = (double *)(base + off_fs);
    w.K = (float *)(base + off_k);
    hipError_t e = cps::launch_knn_filtered(P_dev, f_dev, Q_dev, n, dim, nq, k, w, out_dev, s);
    return e == hipSuccess ? CPS_OK : hip_fail(e);
  }
  const size_t off_desc = align_up((size_t)nq * (size_t)n * sizeof(float), 256);
  const size_t dsz = align_up((size_t)nq * 8, 256);
  const size_t off_sel = off_desc + 3 * dsz;
  const size_t off_pd = off_sel + align_up((size_t)nq * sizeof(cps_result), 256);
  const size_t psz = align_up((size_t)nq * 16 * 8, 256);
  const size_t bytes = off_pd + 2 * psz;
  char *base;
  {
    std::lock_guard<std::mutex> lk(h->mu);
    int rc = ensure_buffer(h->lws, h->lws_bytes, bytes, s);
    if (rc) return rc;
    base = (char *)h->lws;
    hipError_t e = cps::launch_knn_distances(P_dev, Q_dev, n, dim, nq, k, (float *)base,
                                             (const float **)(base + off_desc),
                                             (int64_t *)(base + off_desc + dsz),
                                             (int64_t *)(base + off_desc + 2 * dsz), h->cu_count, s);
    if (e != hipSuccess) return hip_fail(e);
  }
  cps_batch_options o;
  cps_default_batch_options(&o);
  int rc = select_kth_batched_ex(h, (const void *const *)(base + off_desc),
                                 (const int64_t *)(base + off_desc + dsz),
                                 (const int64_t *)(base + off_desc + 2 * dsz), nq, CPS_F32, &o,
                                 (cps_result *)(base + off_sel), stream);
  if (rc) return rc;
  hipError_t e = cps::launch_knn_reduce(P_dev, f_dev, Q_dev, (const float *)base, n, dim, nq, k,
                                        (const cps_result *)(base + off_sel),
                                        (double *)(base + off_pd), (int64_t *)(base + off_pd + psz),
                                        out_dev, s);
  return e == hipSuccess ? CPS_OK : hip_fail(e);
}

int knn_mean(cps_handle *h, const float *P_dev, const float *f_dev, const float *Q_dev, int64_t n,
             int32_t dim, int64_t nq, int64_t k, cps_knn *out_dev, void *stream) {
  return knn_mean_ex(h, P_dev, f_dev, Q_dev, n, dim, nq, k, CPS_LMS_AUTO, out_dev, stream);
}

int cps_autotune_batched(cps_handle *h, const void *const *ptrs_dev, const int64_t *sizes_dev,
                         const int64_t *ks_dev, int64_t count, int dtype, cps_result *out_dev,
                         void *stream, cps_batch_options *best, double *best_ms) {
  int rc = check_batched(h, ptrs_dev, sizes_dev, ks_dev, count, dtype, out_dev);
  if (rc) return rc;
  hipStream_t s = (hipStream_t)stream;
  const int blocks[3] = {256, 512, 1024};
  // candidates per workgroup size: the sampled bracket with one workgroup per array, or
  // 4, 8 or 16 per array at 2^16 .. 2^18 elements per workgroup; the counting evaluation
  // from [min, max]; splits at capacities 2^17 and 2^19
  struct Cand {
    int proposal, bpa;
    int64_t epb;
    int count_first;
    int64_t cap;
  };
  const Cand cands[] = {{1, 1, 0, 1, 0},
                        {1, 4, (int64_t)1 << 18, 1, 0},
                        {1, 8, (int64_t)1 << 17, 1, 0},
                        {1, 16, (int64_t)1 << 16, 1, 0},
                        {1, 16, (int64_t)1 << 18, 1, 0},
                        {0, 1, 0, 1, 0},
                        {0, 1, 0, 0, (int64_t)1 << 17},
                        {0, 1, 0, 0, (int64_t)1 << 19}};
  // A sampled bracket's copy holds the 16-byte vectors of x that hold an interior element
  // (~23 % of a float array of ~10^6 elements, ~12 % of a double one); a copy that does not
  // fit sends the array back over its full length with one workgroup.  The candidates that
  // copy get room for a quarter of the batch's largest array (at least the default 2^18
  // elements, at most 2^22).
  int64_t team_cap = 0;
  {
    std::vector<int64_t> hs((size_t)count);
    if (hipMemcpyAsync(hs.data(), sizes_dev, (size_t)count * sizeof(int64_t),
                       hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
      return CPS_EHIP;
    int64_t mx = 0;
    for (const int64_t v : hs) mx = v > mx ? v : mx;
    const int64_t q = (mx / 4 + 63) / 64 * 64;
    if (q > ((int64_t)1 << 18)) team_cap = q < ((int64_t)1 << 22) ? q : ((int64_t)1 << 22);
  }
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return CPS_EHIP;
  double best_t = 1e300;
  cps_batch_options best_o;
  cps_default_batch_options(&best_o);
  int last_rc = CPS_OK;
  for (int b : blocks) {
    for (const Cand &cd : cands) {
      cps_batch_options o;
      cps_default_batch_options(&o);
      o.block_threads = b;
      o.proposal = cd.proposal;
      o.blocks_per_array = cd.bpa;
      if (cd.epb) o.elements_per_block = cd.epb;
      o.count_first = cd.count_first;
      if (cd.cap) o.split_capacity = cd.cap;
      if (cd.proposal && team_cap) o.team_capacity = team_cap;
      rc = select_kth_batched_ex(h, ptrs_dev, sizes_dev, ks_dev, count, dtype, &o, out_dev, stream);
      if (rc == CPS_ENOMEM) continue;  // this candidate's workspace does not fit
      if (rc) { last_rc = rc; break; }
      (void)hipEventRecord(e0, s);
      for (int rep = 0; rep < 2; ++rep)
        rc = select_kth_batched_ex(h, ptrs_dev, sizes_dev, ks_dev, count, dtype, &o, out_dev, stream);
      (void)hipEventRecord(e1, s);
      if (hipEventSynchronize(e1) != hipSuccess) { last_rc = CPS_EHIP; break; }
      float ms = 0;
      (void)hipEventElapsedTime(&ms, e0, e1);
      if (ms / 2 < best_t) {
        best_t = ms / 2;
        best_o = o;
      }
    }
    if (last_rc) break;
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (last_rc) return last_rc;
  {
    std::lock_guard<std::mutex> lk(h->mu);
    const int di = dtype == CPS_F32 ? 0 : 1;
    h->tuned[di] = best_o;
    h->has_tuned[di] = true;
  }
  if (best) *best = best_o;
  if (best_ms) *best_ms = best_t;
  return CPS_OK;
}


void cps_default_options(cps_options *opt) {
  if (!opt) return;
  std::memset(opt, 0, sizeof(*opt));
  opt->maxit = 64;
  opt->final_threshold = 8192;
  opt->partition_fraction = 1.0;
  opt->grid_blocks = 0;
  opt->block_threads = 0;
  opt->spin_limit = 0;
  opt->use_bracket = 0;
  opt->compact_proposal = 1;
  opt->hist_bits = 12;
  opt->count_first = 1;
}

int cps_last_hip_error(void) { return g_last_hip; }

const char *cps_status_string(int code) {
  switch (code) {
    case CPS_OK: return "ok";
    case CPS_EINVAL: return "invalid argument";
    case CPS_ENOMEM: return "workspace allocation failed";
    case CPS_EHIP: return "HIP runtime error";
    case CPS_ECAPTURE: return "allocation needed during stream capture";
    case CPS_ENODEV: return "no usable gfx950 device";
    case CPS_ESTATE: return "handle in an unusable state";
    case CPS_EIO: return "network file could not be opened, read or written";
    case CPS_EFORMAT: return "not a valid network file";
    case CPS_ESCRATCH: return "the call needs more than the static scratch of select_kth_noalloc";
    default: break;
  }
  return "unknown code";
}

int cps_create(int device, cps_handle **out) {
  if (!out) return CPS_EINVAL;
  *out = nullptr;
  int count = 0;
  hipError_t e = hipGetDeviceCount(&count);
  if (e != hipSuccess || device < 0 || device >= count) {
    g_last_hip = (int)e;
    return CPS_ENODEV;
  }
  hipDeviceProp_t prop;
  e = hipGetDeviceProperties(&prop, device);
  if (e != hipSuccess) return hip_fail(e);
  if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) return CPS_ENODEV;
  int coop = 0;
  (void)hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, device);
  if (!coop) return CPS_ENODEV;
  e = hipSetDevice(device);
  if (e != hipSuccess) return hip_fail(e);
  // the device address of select_kth_noalloc's scratch array on this device (once per device)
  e = cps::noalloc_bind(device);
  if (e != hipSuccess) return hip_fail(e);
  cps_handle *h = new cps_handle();
  h->device = device;
  h->cu_count = prop.multiProcessorCount;
  h->max_blocks_f32 = cps::select_max_blocks_per_cu<float>();
  h->max_blocks_f64 = cps::select_max_blocks_per_cu<double>();
  if (h->max_blocks_f32 < 1 || h->max_blocks_f64 < 1) {
    delete h;
    return CPS_ENODEV;
  }
  e = hipMalloc(&h->bracket, 256 + cps::kHistMaxBins * sizeof(uint64_t));
  if (e != hipSuccess) {
    delete h;
    g_last_hip = (int)e;
    return CPS_ENOMEM;
  }
  h->phist = (uint64_t *)((char *)h->bracket + 256);
  *out = h;
  return CPS_OK;
}

int cps_destroy(cps_handle *h) {
  if (!h) return CPS_EINVAL;
  if (h->ws) (void)hipFree(h->ws);
  if (h->bws) (void)hipFree(h->bws);
  if (h->tws) (void)hipFree(h->tws);
  if (h->lws) (void)hipFree(h->lws);
  if (h->mws) (void)hipFree(h->mws);
  if (h->ows) (void)hipFree(h->ows);
  if (h->bracket) (void)hipFree(h->bracket);
  delete h;
  return CPS_OK;
}

int cps_reserve(cps_handle *h, int64_t n, int dtype) {
  if (!h || n < 1 || !dtype_size(dtype)) return CPS_EINVAL;
  std::lock_guard<std::mutex> lk(h->mu);
  Resolved r;
  int rc = resolve(h, n, dtype, nullptr, r);
  if (rc) return rc;
  const int per_cu = dtype == CPS_F32 ? h->max_blocks_f32 : h->max_blocks_f64;
  const SelectLayout L =
      select_layout(r.seg_R, r.grid, r.cfg.zcap, h->cu_count * per_cu, dtype_size(dtype),
                    spec_sample_elems(n, dtype_size(dtype), r.cfg.spec_min_n));
  return ensure_workspace(h, L.total, nullptr);
}

int select_kth_ex(cps_handle *h, const void *x, int64_t n, int64_t k, int dtype,
                  const cps_options *opt, cps_result *out_dev, cps_stats *stats_dev,
                  void *stream) {
  int rc = check_common(h, x, n, k, dtype);
  if (rc) return rc;
  if (!out_dev) return CPS_EINVAL;
  std::lock_guard<std::mutex> lk(h->mu);
  hipStream_t s = (hipStream_t)stream;
  if (dtype == CPS_F32)
    return run_select<float>(h, (const float *)x, n, k, opt, out_dev, stats_dev, s);
  return run_select<double>(h, (const double *)x, n, k, opt, out_dev, stats_dev, s);
}

int select_kth(cps_handle *h, const void *x, int64_t n, int64_t k, int dtype,
               cps_result *out_dev, void *stream) {
  return select_kth_ex(h, x, n, k, dtype, nullptr, out_dev, nullptr, stream);
}

int select_kth_noalloc(cps_handle *h, const void *x, int64_t n, int64_t k, int dtype,
                       cps_result *out_dev, void *stream) {
  int rc = check_common(h, x, n, k, dtype);
  if (rc) return rc;
  if (!out_dev) return CPS_EINVAL;
  char *base = (char *)cps::noalloc_scratch(h->device);
  if (!base) return CPS_ESTATE;
  std::lock_guard<std::mutex> lk(h->mu);
  hipStream_t s = (hipStream_t)stream;
  Resolved r;
  rc = resolve(h, n, dtype, nullptr, r);
  if (rc) return rc;
  // The defaults without the split buffers: the counting evaluation at the first trial point,
  // then histogram passes over x that count the narrowed bracket without copying it, and the
  // gather of its last few elements.  No likely-interval copy.
  r.cfg.hist_compact = 0;
  r.cfg.spec_min_n = 0;
  r.seg_R = 0;
  if (r.grid > cps::kNoAllocMaxGrid) r.grid = cps::kNoAllocMaxGrid;
  const size_t es = dtype_size(dtype);
  const SelectLayout L = select_layout(0, r.grid, r.cfg.zcap, r.grid, es);
  if (L.total > cps::kNoAllocScratchBytes) return CPS_ESCRATCH;
  // every word the kernel expects zero at launch: the synchronisation words and the
  // histogram counters (the state and the partials are written before they are read)
  hipError_t e = cps::launch_scratch_clear(base + L.sync, L.sd - L.sync, s);
  if (e != hipSuccess) return hip_fail(e);
  auto fill = [&](auto *xt) {
    using T = std::remove_const_t<std::remove_pointer_t<decltype(xt)>>;
    cps::SelectArgs<T> a{};
    a.x = xt;
    a.n = n;
    a.k = k;
    a.st = (cps::CpState *)(base + L.st);
    a.sync = (cps::SyncCtl *)(base + L.sync);
    a.sd = (double *)(base + L.sd);
    a.si = (int64_t *)(base + L.si);
    a.slot_stride = L.slot_stride;
    a.z[0] = a.z[1] = nullptr;
    a.seg_R = 0;
    a.zf = (T *)(base + L.zf);
    a.out = out_dev;
    a.stats = nullptr;
    a.cfg = r.cfg;
    a.spin_limit = r.spin_limit;
    a.bracket = nullptr;
    a.p0_cap = 0;
    a.ghist = (uint64_t *)(base + L.gh);
    a.phist = nullptr;
    a.smp = nullptr;
    a.smp_n = 0;
    return cps::launch_select<T>(a, r.grid, r.cooperative, s);
  };
  e = dtype == CPS_F32 ? fill((const float *)x) : fill((const double *)x);
  return e == hipSuccess ? CPS_OK : hip_fail(e);
}

int cps_objective(cps_handle *h, const void *x, int64_t n, int64_t k, int dtype,
                  const double *ys_dev, int64_t ny, cps_eval *out_dev, void *stream) {
  int rc = check_common(h, x, n, k, dtype);
  if (rc) return rc;
  if (!ys_dev || !out_dev || ny < 0 || ny > 65535) return CPS_EINVAL;
  if (ny == 0) return CPS_OK;
  std::lock_guard<std::mutex> lk(h->mu);
  hipStream_t s = (hipStream_t)stream;
  int64_t nb = (n + 256 * 8 - 1) / (256 * 8);
  if (nb > 4 * (int64_t)h->cu_count) nb = 4 * (int64_t)h->cu_count;
  if (nb < 1) nb = 1;
  const size_t pd_bytes = align_up((size_t)ny * nb * 4 * sizeof(double), 256);
  const size_t pi_bytes = align_up((size_t)ny * nb * 3 * sizeof(int64_t), 256);
  rc = ensure_buffer(h->ows, h->ows_bytes, pd_bytes + pi_bytes, s);
  if (rc) return rc;
  double *pd = (double *)h->ows;
  int64_t *pi = (int64_t *)((char *)h->ows + pd_bytes);
  hipError_t e;
  if (dtype == CPS_F32)
    e = cps::launch_objective<float>((const float *)x, n, k, ys_dev, ny, out_dev, pd, pi, (int)nb, s);
  else
    e = cps::launch_objective<double>((const double *)x, n, k, ys_dev, ny, out_dev, pd, pi, (int)nb, s);
  if (e != hipSuccess) return hip_fail(e);
  return CPS_OK;
}

// ------------------------------------------------------------------ learned proposal

int cps_mixture_generate(cps_handle *h, uint64_t seed, int64_t first_id, int64_t count,
                         int64_t n, float *x_dev, int64_t *ks_dev, void *stream) {
  if (!h || !x_dev || count < 1 || n < 1 || first_id < 0 ||
      first_id + count > ((int64_t)1 << 32))
    return CPS_EINVAL;
  hipError_t e = cps::launch_mixture_gen(seed, first_id, count, n, x_dev, ks_dev,
                                         (hipStream_t)stream);
  return e == hipSuccess ? CPS_OK : hip_fail(e);
}

int cps_features(cps_handle *h, const void *const *ptrs_dev, const int64_t *sizes_dev,
                 const int64_t *ks_dev, int64_t count, int dtype, float *feat_dev,
                 double *range_dev, int32_t *valid_dev, void *stream) {
  if (!h || !ptrs_dev || !sizes_dev || !ks_dev || !feat_dev || !range_dev || !valid_dev ||
      count < 1 || !dtype_size(dtype))
    return CPS_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  if (dtype == CPS_F32)
    e = cps::launch_features<float>((const float *const *)ptrs_dev, sizes_dev, ks_dev, count,
                                    feat_dev, range_dev, valid_dev, s);
  else
    e = cps::launch_features<double>((const double *const *)ptrs_dev, sizes_dev, ks_dev, count,
                                     feat_dev, range_dev, valid_dev, s);
  return e == hipSuccess ? CPS_OK : hip_fail(e);
}

int cps_mlp_forward(cps_handle *h, const float *params_dev, const float *feat_dev, int64_t count,
                    float *out_dev, void *stream) {
  if (!h || !params_dev || !feat_dev || !out_dev || count < 1 || count > ((int64_t)1 << 36))
    return CPS_EINVAL;
  hipError_t e = cps::launch_mlp_forward(params_dev, feat_dev, count, out_dev, (hipStream_t)stream);
  return e == hipSuccess ? CPS_OK : hip_fail(e);
}

int cps_mlp_loss_grad(cps_handle *h, const float *params_dev, const float *feat_dev,
                      const float *ustar_dev, int64_t count, float *grad_dev, float *loss_dev,
                      void *stream) {
  if (!h || !params_dev || !feat_dev || !ustar_dev || !grad_dev || count < 1 ||
      count > ((int64_t)1 << 26))
    return CPS_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  std::lock_guard<std::mutex> lk(h->mu);
  int rc = ensure_buffer(h->mws, h->mws_bytes, cps::mlp_grad_workspace(count), s);
  if (rc) return rc;
  hipError_t e = cps::launch_mlp_loss_grad(params_dev, feat_dev, ustar_dev, count, grad_dev,
                                           loss_dev, (float *)h->mws, s);
  return e == hipSuccess ? CPS_OK : hip_fail(e);
}

int cps_mlp_adam(cps_handle *h, float *params_dev, const float *grad_dev, float *m_dev,
                 float *v_dev, int64_t step, float lr, float beta1, float beta2, float eps,
                 void *stream) {
  if (!h || !params_dev || !grad_dev || !m_dev || !v_dev || step < 1 || !(lr > 0.0f) ||
      !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
    return CPS_EINVAL;
  hipError_t e = cps::launch_mlp_adam(params_dev, grad_dev, m_dev, v_dev, step, lr, beta1, beta2,
                                      eps, (hipStream_t)stream);
  return e == hipSuccess ? CPS_OK : hip_fail(e);
}

int cps_mlp_init(cps_handle *h, uint64_t seed, float *params_dev, void *stream) {
  if (!h || !params_dev) return CPS_EINVAL;
  hipError_t e = cps::launch_mlp_init(seed, params_dev, (hipStream_t)stream);
  return e == hipSuccess ? CPS_OK : hip_fail(e);
}

int cps_learned_bracket(cps_handle *h, const void *x, int64_t n, int64_t k, int dtype,
                        const float *params_dev, double *bracket_dev, void *stream) {
  int rc = check_common(h, x, n, k, dtype);
  if (rc) return rc;
  if (!params_dev || !bracket_dev) return CPS_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  if (dtype == CPS_F32)
    e = cps::launch_learned_bracket<float>((const float *)x, n, k, params_dev, nullptr, bracket_dev, s);
  else
    e = cps::launch_learned_bracket<double>((const double *)x, n, k, params_dev, nullptr, bracket_dev,
                                            s);
  return e == hipSuccess ? CPS_OK : hip_fail(e);
}

int select_kth_learned(cps_handle *h, const void *x, int64_t n, int64_t k, int dtype,
                       const float *params_dev, const cps_options *opt, cps_result *out_dev,
                       cps_stats *stats_dev, void *stream) {
  int rc = check_common(h, x, n, k, dtype);
  if (rc) return rc;
  if (!params_dev || !out_dev) return CPS_EINVAL;
  std::lock_guard<std::mutex> lk(h->mu);
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  if (dtype == CPS_F32)
    e = cps::launch_learned_bracket<float>((const float *)x, n, k, params_dev, h->phist, h->bracket,
                                           s);
  else
    e = cps::launch_learned_bracket<double>((const double *)x, n, k, params_dev, h->phist, h->bracket,
                                            s);
  if (e != hipSuccess) return hip_fail(e);
  if (dtype == CPS_F32)
    return run_select<float>(h, (const float *)x, n, k, opt, out_dev, stats_dev, s, h->bracket);
  return run_select<double>(h, (const double *)x, n, k, opt, out_dev, stats_dev, s, h->bracket);
}

int cps_sample_bracket(cps_handle *h, const void *x, int64_t n, int64_t k, int dtype, double z,
                       double *bracket_dev, void *stream) {
  int rc = check_common(h, x, n, k, dtype);
  if (rc) return rc;
  if (!bracket_dev || !(z >= 0.0) || z > 1e6) return CPS_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  if (dtype == CPS_F32)
    e = cps::launch_sample_bracket<float>((const float *)x, n, k, z, nullptr, bracket_dev, s);
  else
    e = cps::launch_sample_bracket<double>((const double *)x, n, k, z, nullptr, bracket_dev, s);
  return e == hipSuccess ? CPS_OK : hip_fail(e);
}

int select_kth_sampled(cps_handle *h, const void *x, int64_t n, int64_t k, int dtype, double z,
                       const cps_options *opt, cps_result *out_dev, cps_stats *stats_dev,
                       void *stream) {
  int rc = check_common(h, x, n, k, dtype);
  if (rc) return rc;
  if (!out_dev || !(z >= 0.0) || z > 1e6) return CPS_EINVAL;
  std::lock_guard<std::mutex> lk(h->mu);
  hipStream_t s = (hipStream_t)stream;
  hipError_t e;
  if (dtype == CPS_F32)
    e = cps::launch_sample_bracket<float>((const float *)x, n, k, z, h->phist, h->bracket, s);
  else
    e = cps::launch_sample_bracket<double>((const double *)x, n, k, z, h->phist, h->bracket, s);
  if (e != hipSuccess) return hip_fail(e);
  if (dtype == CPS_F32)
    return run_select<float>(h, (const float *)x, n, k, opt, out_dev, stats_dev, s, h->bracket);
  return run_select<double>(h, (const double *)x, n, k, opt, out_dev, stats_dev, s, h->bracket);
}

}  // extern "C"

namespace {

// Device buffers of one training run, freed together.
struct TrainBuffers {
  std::vector<void *> bufs;
  ~TrainBuffers() {
    for (void *p : bufs) (void)hipFree(p);
  }
  template <typename P> int get(P *&p, size_t bytes) {
    void *q = nullptr;
    hipError_t e = hipMalloc(&q, bytes < 256 ? 256 : bytes);
    if (e != hipSuccess) {
      g_last_hip = (int)e;
      return CPS_ENOMEM;
    }
    bufs.push_back(q);
    p = (P *)q;
    return CPS_OK;
  }
};

// Generate arrays [first, first + count) of `seed` in chunks, with features, ranges,
// validity and exact labels; optionally the network outputs and the coverage counters.
int label_arrays(cps_handle *h, uint64_t seed, int64_t count, int64_t n, int64_t chunk,
                 float *xbuf, int64_t *ks, const float **ptrs, int64_t *sizes, cps_result *res,
                 float *feat, double *range, int32_t *valid, float *ustar, const float *params,
                 float *outs, double *acc, hipStream_t s) {
  for (int64_t c0 = 0; c0 < count; c0 += chunk) {
    const int64_t c = count - c0 < chunk ? count - c0 : chunk;
    int rc = cps_mixture_generate(h, seed, c0, c, n, xbuf, ks, s);
    if (rc) return rc;
    hipError_t e = cps::launch_batch_descriptors(xbuf, n, c, ptrs, sizes, s);
    if (e != hipSuccess) return hip_fail(e);
    float *f = feat + (feat && !outs ? c0 * CPS_MLP_INPUTS : 0);
    double *rg = range + (outs ? 0 : 2 * c0);
    int32_t *vd = valid + (outs ? 0 : c0);
    rc = cps_features(h, (const void *const *)ptrs, sizes, ks, c, CPS_F32, f, rg, vd, s);
    if (rc) return rc;
    rc = select_kth_batched_ex(h, (const void *const *)ptrs, sizes, ks, c, CPS_F32, nullptr, res, s);
    if (rc) return rc;
    if (!outs) {
      e = cps::launch_labels(res, f, rg, vd, c, ustar + c0, s);
      if (e != hipSuccess) return hip_fail(e);
    } else {
      rc = cps_mlp_forward(h, params, f, c, outs, s);
      if (rc) return rc;
      e = cps::launch_holdout(outs, f, rg, vd, res, c, acc, s);
      if (e != hipSuccess) return hip_fail(e);
    }
  }
  return CPS_OK;
}

}  // namespace

extern "C" {

int cps_mlp_train(cps_handle *h, const cps_train_options *opt, float *params_dev,
                  cps_train_report *report, void *stream) {
  if (!h || !opt || !params_dev || opt->n_arrays < 1 || opt->array_size < 1 || opt->epochs < 0 ||
      opt->batch < 1 || opt->batch > (1 << 20) || !(opt->lr > 0.0f) || opt->holdout < 0 ||
      opt->n_arrays > ((int64_t)1 << 32) || opt->holdout > ((int64_t)1 << 32))
    return CPS_EINVAL;
  hipStream_t s = (hipStream_t)stream;
  const int64_t N = opt->n_arrays, n = opt->array_size;
  // arrays in flight: up to 4096 per chunk and about 2 GiB of values
  int64_t chunk = (((int64_t)1 << 29) + n - 1) / n;
  if (chunk > 4096) chunk = 4096;
  if (chunk < 1) chunk = 1;
  const int64_t cmax = chunk > opt->holdout ? chunk : opt->holdout;
  TrainBuffers tb;
  float *xbuf, *feat, *ustar, *grad, *m, *v, *losses, *outs, *hfeat;
  int64_t *ks, *sizes;
  const float **ptrs;
  cps_result *res;
  double *range, *hrange, *acc;
  int32_t *valid, *hvalid;
  const int64_t spe = N / opt->batch > 0 ? N / opt->batch : 1;  // steps per epoch
  const int64_t B = N / opt->batch > 0 ? opt->batch : N;
  const int64_t steps = spe * opt->epochs;
  int rc = CPS_OK;
  if ((rc = tb.get(xbuf, (size_t)chunk * n * sizeof(float))) ||
      (rc = tb.get(ks, (size_t)cmax * sizeof(int64_t))) ||
      (rc = tb.get(sizes, (size_t)cmax * sizeof(int64_t))) ||
      (rc = tb.get(ptrs, (size_t)cmax * sizeof(float *))) ||
      (rc = tb.get(res, (size_t)cmax * sizeof(cps_result))) ||
      (rc = tb.get(feat, (size_t)N * CPS_MLP_INPUTS * sizeof(float))) ||
      (rc = tb.get(range, (size_t)N * 2 * sizeof(double))) ||
      (rc = tb.get(valid, (size_t)N * sizeof(int32_t))) ||
      (rc = tb.get(ustar, (size_t)N * sizeof(float))) ||
      (rc = tb.get(grad, CPS_MLP_PARAMS * sizeof(float))) ||
      (rc = tb.get(m, CPS_MLP_PARAMS * sizeof(float))) ||
      (rc = tb.get(v, CPS_MLP_PARAMS * sizeof(float))) ||
      (rc = tb.get(losses, (size_t)(steps > 0 ? steps : 1) * sizeof(float))) ||
      (rc = tb.get(outs, (size_t)chunk * 2 * sizeof(float))) ||
      (rc = tb.get(hfeat, (size_t)chunk * CPS_MLP_INPUTS * sizeof(float))) ||
      (rc = tb.get(hrange, (size_t)chunk * 2 * sizeof(double))) ||
      (rc = tb.get(hvalid, (size_t)chunk * sizeof(int32_t))) ||
      (rc = tb.get(acc, 4 * sizeof(double))))
    return rc;
  hipError_t e;
  if ((e = hipMemsetAsync(m, 0, CPS_MLP_PARAMS * sizeof(float), s)) != hipSuccess ||
      (e = hipMemsetAsync(v, 0, CPS_MLP_PARAMS * sizeof(float), s)) != hipSuccess ||
      (e = hipMemsetAsync(acc, 0, 4 * sizeof(double), s)) != hipSuccess)
    return hip_fail(e);
  if (opt->init && (rc = cps_mlp_init(h, opt->seed, params_dev, s))) return rc;
  // the training set: features and exact labels of every array
  rc = label_arrays(h, opt->seed, N, n, chunk, xbuf, ks, ptrs, sizes, res, feat, range, valid,
                    ustar, params_dev, nullptr, nullptr, s);
  if (rc) return rc;
  // Adam over minibatches of consecutive examples (the arrays are independent draws)
  int64_t step = 0;
  for (int ep = 0; ep < opt->epochs; ++ep) {
    for (int64_t b = 0; b < spe; ++b) {
      const int64_t r0 = b * B;
      rc = cps_mlp_loss_grad(h, params_dev, feat + r0 * CPS_MLP_INPUTS, ustar + r0, B, grad,
                             losses + step, s);
      if (rc) return rc;
      ++step;
      rc = cps_mlp_adam(h, params_dev, grad, m, v, step, opt->lr, 0.9f, 0.999f, 1e-8f, s);
      if (rc) return rc;
    }
  }
  // held-out arrays: coverage and width of the trained proposal
  if (opt->holdout > 0) {
    rc = label_arrays(h, opt->holdout_seed, opt->holdout, n, chunk, xbuf, ks, ptrs, sizes, res,
                      hfeat, hrange, hvalid, nullptr, params_dev, outs, acc, s);
    if (rc) return rc;
  }
  if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e);
  if (report) {
    std::vector<float> hl((size_t)(steps > 0 ? steps : 0));
    double ha[4] = {0, 0, 0, 0};
    if (steps > 0 &&
        (e = hipMemcpy(hl.data(), losses, hl.size() * sizeof(float), hipMemcpyDeviceToHost)) !=
            hipSuccess)
      return hip_fail(e);
    if ((e = hipMemcpy(ha, acc, sizeof(ha), hipMemcpyDeviceToHost)) != hipSuccess)
      return hip_fail(e);
    report->first_loss = steps > 0 ? hl[0] : 0.0;
    double last = 0.0;
    for (int64_t i = steps - spe; i < steps; ++i)
      if (i >= 0) last += hl[(size_t)i];
    report->final_loss = steps > 0 ? last / (double)spe : 0.0;
    report->holdout_coverage = ha[2] > 0 ? ha[0] / ha[2] : 0.0;
    report->holdout_width = ha[2] > 0 ? ha[1] / ha[2] : 0.0;
    report->steps = steps;
    report->examples = N;
  }
  return CPS_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ network files

namespace {

constexpr char kModelMagic[8] = {'C', 'P', 'S', 'M', 'L', 'P', '0', '1'};
constexpr uint32_t kModelVersion = 1;
constexpr uint32_t kFeatureSpec = 1;
constexpr size_t kModelHeader = 40;

// FNV-1a, 64-bit (offset basis and prime as published by Fowler, Noll and Vo).
uint64_t fnv1a64(const unsigned char *p, size_t n) {
  uint64_t h = 14695981039346656037ull;
  for (size_t i = 0; i < n; ++i) {
    h ^= p[i];
    h *= 1099511628211ull;
  }
  return h;
}

void put_u32(unsigned char *p, uint32_t v) {
  for (int i = 0; i < 4; ++i) p[i] = (unsigned char)(v >> (8 * i));
}
void put_u64(unsigned char *p, uint64_t v) {
  for (int i = 0; i < 8; ++i) p[i] = (unsigned char)(v >> (8 * i));
}
uint32_t get_u32(const unsigned char *p) {
  uint32_t v = 0;
  for (int i = 0; i < 4; ++i) v |= (uint32_t)p[i] << (8 * i);
  return v;
}
uint64_t get_u64(const unsigned char *p) {
  uint64_t v = 0;
  for (int i = 0; i < 8; ++i) v |= (uint64_t)p[i] << (8 * i);
  return v;
}

}  // namespace

extern "C" {

int cps_model_save(const float *params_dev, const char *path) {
  if (!params_dev || !path) return CPS_EINVAL;
  std::vector<unsigned char> buf(kModelHeader + CPS_MLP_PARAMS * sizeof(float));
  hipError_t e = hipMemcpy(buf.data() + kModelHeader, params_dev, CPS_MLP_PARAMS * sizeof(float),
                           hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e);
  std::memcpy(buf.data(), kModelMagic, 8);
  put_u32(buf.data() + 8, kModelVersion);
  put_u32(buf.data() + 12, CPS_MLP_INPUTS);
  put_u32(buf.data() + 16, CPS_MLP_HIDDEN);
  put_u32(buf.data() + 20, CPS_MLP_OUTPUTS);
  put_u32(buf.data() + 24, kFeatureSpec);
  put_u32(buf.data() + 28, CPS_MLP_PARAMS);
  put_u64(buf.data() + 32, fnv1a64(buf.data() + kModelHeader, CPS_MLP_PARAMS * sizeof(float)));
  // write a sibling file, then rename it over the target, so a failed write leaves no
  // truncated network behind
  const std::string tmp = std::string(path) + ".tmp";
  FILE *f = std::fopen(tmp.c_str(), "wb");
  if (!f) return CPS_EIO;
  const bool ok = std::fwrite(buf.data(), 1, buf.size(), f) == buf.size();
  const bool closed = std::fclose(f) == 0;
  if (!ok || !closed || std::rename(tmp.c_str(), path) != 0) {
    std::remove(tmp.c_str());
    return CPS_EIO;
  }
  return CPS_OK;
}

int cps_model_load(const char *path, float *params_dev) {
  if (!path || !params_dev) return CPS_EINVAL;
  FILE *f = std::fopen(path, "rb");
  if (!f) return CPS_EIO;
  const size_t want = kModelHeader + CPS_MLP_PARAMS * sizeof(float);
  std::vector<unsigned char> buf(want + 1);
  const size_t got = std::fread(buf.data(), 1, buf.size(), f);
  const bool err = std::ferror(f) != 0;
  std::fclose(f);
  if (err) return CPS_EIO;
  if (got != want) return CPS_EFORMAT;  // truncated, or trailing bytes
  if (std::memcmp(buf.data(), kModelMagic, 8) != 0 || get_u32(buf.data() + 8) != kModelVersion ||
      get_u32(buf.data() + 12) != CPS_MLP_INPUTS || get_u32(buf.data() + 16) != CPS_MLP_HIDDEN ||
      get_u32(buf.data() + 20) != CPS_MLP_OUTPUTS || get_u32(buf.data() + 24) != kFeatureSpec ||
      get_u32(buf.data() + 28) != CPS_MLP_PARAMS ||
      get_u64(buf.data() + 32) != fnv1a64(buf.data() + kModelHeader, CPS_MLP_PARAMS * sizeof(float)))
    return CPS_EFORMAT;
  hipError_t e = hipMemcpy(params_dev, buf.data() + kModelHeader, CPS_MLP_PARAMS * sizeof(float),
                           hipMemcpyHostToDevice);
  return e == hipSuccess ? CPS_OK : hip_fail(e);
}

}  // extern "C"
