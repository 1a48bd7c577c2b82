// C ABI of the selection library: handles, argument checks, workspace, launches.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstring>
#include <mutex>

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
  void *ws = nullptr;
  size_t ws_bytes = 0;
  std::mutex mu;
};

namespace {

// Workspace layout of a single-array selection: state, synchronisation words, per-workgroup
// partials, two split buffers (one region of seg_R elements per workgroup each) and the
// gather buffer.
struct SelectLayout {
  size_t st, sync, sd, si, z0, z1, zf, total;
  int64_t slot_stride, seg_R, zcap;
};

SelectLayout select_layout(int64_t seg_R, int grid, int64_t zcap, int gmax, size_t esize) {
  SelectLayout L;
  size_t off = 0;
  L.st = off;
  off = align_up(off + sizeof(cps::CpState), 256);
  L.sync = off;
  off = align_up(off + sizeof(cps::SyncCtl), 256);
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
  L.total = off;
  return L;
}

// Grow the workspace to at least `bytes`.  The synchronisation words at the start of
// every layout must be zero on first use, so fresh memory is cleared synchronously.
int ensure_workspace(cps_handle *h, size_t bytes, hipStream_t stream) {
  if (bytes <= h->ws_bytes) return CPS_OK;
  hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
  if (stream != nullptr) {
    hipError_t e = hipStreamIsCapturing(stream, &cs);
    if (e != hipSuccess) return hip_fail(e);
    if (cs != hipStreamCaptureStatusNone) return CPS_ECAPTURE;
  }
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e);
  if (h->ws) {
    (void)hipFree(h->ws);
    h->ws = nullptr;
    h->ws_bytes = 0;
  }
  size_t want = align_up(bytes + bytes / 8, 1 << 20);
  e = hipMalloc(&h->ws, want);
  if (e != hipSuccess) {
    g_last_hip = (int)e;
    h->ws = nullptr;
    return CPS_ENOMEM;
  }
  e = hipMemset(h->ws, 0, want < (1 << 21) ? want : (1 << 21));
  if (e != hipSuccess) return hip_fail(e);
  h->ws_bytes = want;
  return CPS_OK;
}

inline size_t dtype_size(int dtype) { return dtype == CPS_F32 ? 4 : (dtype == CPS_F64 ? 8 : 0); }

struct Resolved {
  cps::CpConfig cfg;
  int grid;
  int64_t seg_R;
  int64_t spin_limit;
};

int resolve(cps_handle *h, int64_t n, int dtype, const cps_options *opt, Resolved &r) {
  cps_options o;
  cps_default_options(&o);
  if (opt) o = *opt;
  if (o.maxit < 0 || o.final_threshold < 1 || !(o.partition_fraction >= 0.0) ||
      o.partition_fraction > 1.0 || o.grid_blocks < 0 || o.spin_limit < 0)
    return CPS_EINVAL;
  if (o.block_threads != 0 && o.block_threads != cps::kSelectBlock) return CPS_EINVAL;
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
  const int per_cu = dtype == CPS_F32 ? h->max_blocks_f32 : h->max_blocks_f64;
  const int gmax = h->cu_count * per_cu;
  if (gmax < 1) return CPS_ENODEV;
  const int64_t tile = (int64_t)cps::kSelectBlock * cps::kSelectUnroll * (16 / dtype_size(dtype));
  int64_t g = o.grid_blocks ? o.grid_blocks : (int64_t)h->cu_count * (per_cu < 2 ? per_cu : 2);
  const int64_t tiles = (n + tile - 1) / tile;
  if (g > tiles) g = tiles;
  if (g > gmax) g = gmax;
  if (g > (int64_t)cps::kGroup * cps::kMaxGroups) g = (int64_t)cps::kGroup * cps::kMaxGroups;
  if (g < 1) g = 1;
  r.grid = (int)g;
  // Each wavefront's split region holds everything it can read in the first split (a
  // pass over the input with half the unroll): its share of each of its workgroup's
  // steps, plus the unaligned edge elements, rounded to 64 elements.
  int64_t seg = 0;
  if (o.partition_fraction > 0.0) {
    const int64_t vec = 16 / (int64_t)dtype_size(dtype);
    const int64_t su = cps::kSelectUnroll / 2 > 0 ? cps::kSelectUnroll / 2 : 1;
    const int64_t step_vecs = (int64_t)cps::kSelectBlock * su;
    const int64_t nvec = n / vec + 1;
    const int64_t steps = (nvec + step_vecs - 1) / step_vecs;
    const int64_t steps_per_wg = (steps + g - 1) / g;
    seg = (steps_per_wg * cps::kWaveSize * su * vec + 8 + 63) / 64 * 64;
  }
  r.seg_R = seg;
  r.spin_limit = o.spin_limit ? o.spin_limit : (int64_t)1 << 22;
  return CPS_OK;
}

template <typename T>
int run_select(cps_handle *h, const T *x, int64_t n, int64_t k, const cps_options *opt,
               cps_result *out, cps_stats *stats, hipStream_t stream) {
  Resolved r;
  int rc = resolve(h, n, sizeof(T) == 4 ? CPS_F32 : CPS_F64, opt, r);
  if (rc) return rc;
  const int per_cu = sizeof(T) == 4 ? h->max_blocks_f32 : h->max_blocks_f64;
  const SelectLayout L = select_layout(r.seg_R, r.grid, r.cfg.zcap, h->cu_count * per_cu, sizeof(T));
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
  hipError_t e = cps::launch_select<T>(a, r.grid, stream);
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

}  // namespace

extern "C" {

void cps_default_options(cps_options *opt) {
  if (!opt) return;
  std::memset(opt, 0, sizeof(*opt));
  opt->maxit = 64;
  opt->final_threshold = 8192;
  opt->partition_fraction = 0.5;
  opt->grid_blocks = 0;
  opt->block_threads = 0;
  opt->spin_limit = 0;
  opt->use_bracket = 0;
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
  cps_handle *h = new cps_handle();
  h->device = device;
  h->cu_count = prop.multiProcessorCount;
  h->max_blocks_f32 = cps::select_max_blocks_per_cu<float>();
  h->max_blocks_f64 = cps::select_max_blocks_per_cu<double>();
  if (h->max_blocks_f32 < 1 || h->max_blocks_f64 < 1) {
    delete h;
    return CPS_ENODEV;
  }
  *out = h;
  return CPS_OK;
}

int cps_destroy(cps_handle *h) {
  if (!h) return CPS_EINVAL;
  if (h->ws) (void)hipFree(h->ws);
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
      select_layout(r.seg_R, r.grid, r.cfg.zcap, h->cu_count * per_cu, dtype_size(dtype));
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
  // keep clear of the select layout's state and synchronisation words at the start
  const size_t off = align_up(sizeof(cps::CpState), 256) + align_up(sizeof(cps::SyncCtl), 256);
  rc = ensure_workspace(h, off + pd_bytes + pi_bytes, s);
  if (rc) return rc;
  double *pd = (double *)((char *)h->ws + off);
  int64_t *pi = (int64_t *)((char *)h->ws + off + pd_bytes);
  hipError_t e;
  if (dtype == CPS_F32)
    e = cps::launch_objective<float>((const float *)x, n, k, ys_dev, ny, out_dev, pd, pi, (int)nb, s);
  else
    e = cps::launch_objective<double>((const double *)x, n, k, ys_dev, ny, out_dev, pd, pi, (int)nb, s);
  if (e != hipSuccess) return hip_fail(e);
  return CPS_OK;
}

}  // extern "C"
