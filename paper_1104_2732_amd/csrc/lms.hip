// Least median of squares (Section 6): the lower median of the squared residuals of many
// candidate parameter vectors, via the batched selection.
//
// The residual kernels form r_i = (y_i - sum_j X_ij b_j)^2 for a group of candidates per
// thread row: each X row and y_i are read once per group, the sum runs left to right in
// j with every product and sum rounded on its own (the library is built without fused
// multiply-add).
//
// Two forms.  The materialised form writes every square candidate-major in the workspace,
// one array of n per candidate, and the batched kernel selects rank floor((n+1)/2) of every
// array.  The filtered form never writes the whole arrays: a first kernel takes each
// candidate's sampled bracket (a, b) from the squares of a fixed sample of rows (the rows
// the batched kernel would sample), the filter kernel forms every square once and keeps
// only those in (a, b), with #(r <= a), and a gather kernel packs the kept squares of each
// candidate into one array.  Where #(r <= a) < k <= #(r <= a) + #(a < r < b) the k-th
// smallest of all n squares is the (k - #(r <= a))-th smallest of the kept ones, found by
// the batched kernel; a candidate whose bracket misses (or whose kept squares exceed the
// packed array's room) gets its full array written and selected as in the materialised
// form.  Both give the same value and counts.
#include "cps_device.h"
#include "cps_kernels.h"
#include "cps_sample.h"
#include "cps_wgsel.h"

namespace cps {

#ifndef CPS_LMS_GROUP
#define CPS_LMS_GROUP 64
#endif
constexpr int kLmsGroup = CPS_LMS_GROUP;  // candidates per thread row (X read once per group)
constexpr int kLmsBlock = 256;
#ifndef CPS_LMS_ROWS
#define CPS_LMS_ROWS 2
#endif
constexpr int kLmsRows = CPS_LMS_ROWS;  // rows per thread of the 16-byte residual kernel

// ONLY: write only the candidates whose flag in `only` is set (the filtered form's
// fallback); a workgroup whose candidates have none returns at once.
template <int P, bool ONLY>
__global__ __launch_bounds__(kLmsBlock) void lms_residual_kernel(
    const double *__restrict__ X, const double *__restrict__ y, const double *__restrict__ betas,
    int64_t n, int32_t p, int64_t m, double *__restrict__ R, const int32_t *__restrict__ only) {
  __shared__ double sb[kLmsGroup * 16];
  __shared__ int32_t sf[kLmsGroup];
  const int64_t c0 = (int64_t)blockIdx.y * kLmsGroup;
  const int nc = (int)((m - c0) < kLmsGroup ? (m - c0) : kLmsGroup);
  for (int q = threadIdx.x; q < nc * p; q += kLmsBlock) sb[q] = betas[c0 * p + q];
  if (ONLY && threadIdx.x < nc) sf[threadIdx.x] = only[c0 + threadIdx.x];
  if (ONLY) {
    if (!__syncthreads_or(threadIdx.x < nc && only[c0 + threadIdx.x] != 0)) return;
  } else {
    __syncthreads();
  }
  const CPS_GLOBAL double *Xg = (const CPS_GLOBAL double *)X;
  const CPS_GLOBAL double *yg = (const CPS_GLOBAL double *)y;
  CPS_GLOBAL double *Rg = (CPS_GLOBAL double *)R;
  for (int64_t i = (int64_t)blockIdx.x * kLmsBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kLmsBlock) {
    double row[P > 0 ? P : 16];
    const int pp = P > 0 ? P : p;
#pragma unroll
    for (int j = 0; j < (P > 0 ? P : 16); ++j)
      if (j < pp) row[j] = Xg[i * pp + j];
    const double yi = yg[i];
    for (int c = 0; c < nc; ++c) {
      if (ONLY && sf[c] == 0) continue;
      const double *b = sb + c * pp;
      double s = row[0] * b[0];
#pragma unroll
      for (int j = 1; j < (P > 0 ? P : 16); ++j) {
        if (j < pp) {
          const double prod = row[j] * b[j];
          s = s + prod;
        }
      }
      const double d = yi - s;
      __builtin_nontemporal_store(d * d, &Rg[(c0 + c) * n + i]);  // written once, read later
    }
  }
}

// The same residuals for p = P columns, R consecutive rows per thread: each thread's X rows
// are R*P contiguous doubles (16-byte loads) and each candidate's R residuals one or two
// 16-byte stores, so a wavefront writes R*512 contiguous bytes per candidate.  Needs n to be a
// multiple of R (every candidate's array then starts 16-byte aligned).
template <int P, int R, bool ONLY>
__global__ __launch_bounds__(kLmsBlock) void lms_residual_rows_kernel(
    const double *__restrict__ X, const double *__restrict__ y, const double *__restrict__ betas,
    int64_t n, int64_t m, double *__restrict__ R_out, const int32_t *__restrict__ only) {
  static_assert(R % 2 == 0 && (P * R) % 2 == 0, "16-byte groups");
  __shared__ double sb[kLmsGroup * P];
  __shared__ int32_t sf[kLmsGroup];
  const int64_t c0 = (int64_t)blockIdx.y * kLmsGroup;
  const int nc = (int)((m - c0) < kLmsGroup ? (m - c0) : kLmsGroup);
  for (int q = threadIdx.x; q < nc * P; q += kLmsBlock) sb[q] = betas[c0 * P + q];
  if (ONLY && threadIdx.x < nc) sf[threadIdx.x] = only[c0 + threadIdx.x];
  if (ONLY) {
    if (!__syncthreads_or(threadIdx.x < nc && only[c0 + threadIdx.x] != 0)) return;
  } else {
    __syncthreads();
  }
  using D2 = double __attribute__((ext_vector_type(2)));
  const CPS_GLOBAL D2 *Xg = (const CPS_GLOBAL D2 *)X;
  const CPS_GLOBAL D2 *yg = (const CPS_GLOBAL D2 *)y;
  CPS_GLOBAL double *Rg = (CPS_GLOBAL double *)R_out;
  const int64_t groups = n / R;
  for (int64_t g = (int64_t)blockIdx.x * kLmsBlock + threadIdx.x; g < groups;
       g += (int64_t)gridDim.x * kLmsBlock) {
    const int64_t i0 = g * R;
    double row[R][P];
#pragma unroll
    for (int v = 0; v < R * P / 2; ++v) {
      const D2 w = Xg[i0 * P / 2 + v];
      row[(2 * v) / P][(2 * v) % P] = w.x;
      row[(2 * v + 1) / P][(2 * v + 1) % P] = w.y;
    }
    double yi[R];
#pragma unroll
    for (int v = 0; v < R / 2; ++v) {
      const D2 w = yg[i0 / 2 + v];
      yi[2 * v] = w.x;
      yi[2 * v + 1] = w.y;
    }
    for (int c = 0; c < nc; ++c) {
      if (ONLY && sf[c] == 0) continue;
      const double *b = sb + c * P;
      double r[R];
#pragma unroll
      for (int q = 0; q < R; ++q) {
        double s = row[q][0] * b[0];
#pragma unroll
        for (int j = 1; j < P; ++j) {
          const double prod = row[q][j] * b[j];
          s = s + prod;
        }
        const double d = yi[q] - s;
        r[q] = d * d;
      }
      CPS_GLOBAL D2 *dst = (CPS_GLOBAL D2 *)(Rg + (c0 + c) * n + i0);
#pragma unroll
      for (int v = 0; v < R / 2; ++v) {
        D2 w;
        w.x = r[2 * v];
        w.y = r[2 * v + 1];
        __builtin_nontemporal_store(w, dst + v);  // written once, read later
      }
    }
  }
}

// ------------------------------------------------------------------ the filtered form

// One squared residual, in the order of the materialised kernels (bit-identical to them).
template <int P>
__device__ __forceinline__ double sq_residual(const double *row, double yi, const double *b, int p) {
  const int pp = P > 0 ? P : p;
  double s = row[0] * b[0];
#pragma unroll
  for (int j = 1; j < (P > 0 ? P : 16); ++j) {
    if (j < pp) {
      const double prod = row[j] * b[j];
      s = s + prod;
    }
  }
  const double d = yi - s;
  return d * d;
}

// The squares of the sampled rows (the rows the batched kernel samples in an array of n
// elements: runs of kPropRun neighbours at sample_stride apart), one candidate per lane as in
// the filter, to Rs[c * S + i].
template <int P>
__global__ __launch_bounds__(kLmsBlock) void lms_sample_kernel(
    const double *__restrict__ X, const double *__restrict__ y, const double *__restrict__ betas,
    int64_t n, int32_t p, int64_t m, double *__restrict__ Rs) {
  constexpr int PM = P > 0 ? P : 16;
  const int pp = P > 0 ? P : p;
  const int64_t c = (int64_t)blockIdx.y * kLmsBlock + threadIdx.x;
  const bool live = c < m;
  double b[PM];
#pragma unroll
  for (int j = 0; j < PM; ++j) b[j] = live && j < pp ? betas[c * pp + j] : 0.0;
  const int S = sample_size(n);
  const int64_t stride = sample_stride(n, S);
  CPS_GLOBAL double *dst = (CPS_GLOBAL double *)Rs + (live ? c : 0) * S;
  // each workgroup takes a share of the sample's runs, two rows per step (both rows' scalar
  // loads issued together)
  const int runs = S / kPropRun;
  const int per = (runs + (int)gridDim.x - 1) / (int)gridDim.x;
  const int r0 = (int)blockIdx.x * per, r1 = r0 + per < runs ? r0 + per : runs;
  for (int run = r0; run < r1; ++run) {
    for (int q = 0; q < kPropRun; q += 2) {
      const int64_t i = (int64_t)run * stride + q;
      double x0[PM], x1[PM];
#pragma unroll
      for (int j = 0; j < PM; ++j) {
        x0[j] = j < pp ? X[i * pp + j] : 0.0;
        x1[j] = j < pp ? X[(i + 1) * pp + j] : 0.0;
      }
      const double v0 = sq_residual<P>(x0, y[i], b, pp);
      const double v1 = sq_residual<P>(x1, y[i + 1], b, pp);
      if (live) {
        dst[run * kPropRun + q] = v0;
        dst[run * kPropRun + q + 1] = v1;
      }
    }
  }
}

constexpr int kLmsBracketBlock = 256;
struct LmsBracketShared {
  uint64_t kext[2];
  int32_t flag;
  SampleLds smp;
  uint64_t wsum[kLmsBracketBlock / kWave];
  uint32_t rh[kHistMaxBins];
};

// One workgroup per candidate: the sampled bracket of its squared residuals from the sampled
// squares Rs, to ab[2c], ab[2c+1].  A candidate without one gets (+inf, -inf): the filter
// then keeps nothing of it but NaN, and the gather sends it down the materialised path.
__global__ __launch_bounds__(kLmsBracketBlock) void lms_bracket_kernel(
    const double *__restrict__ Rs, int64_t n, int64_t k, double *__restrict__ ab) {
  __shared__ LmsBracketShared sh;
  const int64_t c = blockIdx.x;
  const int S = sample_size(n);
  const CPS_GLOBAL double *src = (const CPS_GLOBAL double *)Rs + c * S;
  auto sample = [&](int i) -> double { return src[i]; };
  double a, b;
  const bool use = sample_bracket_rule<double, kLmsBracketBlock>(sample, S, n, k, sh, a, b);
  if (threadIdx.x == 0) {
    ab[2 * c] = use ? a : __builtin_inf();
    ab[2 * c + 1] = use ? b : -__builtin_inf();
  }
}

// The filter: kLmsLane candidates per lane (c = blockIdx.y * kLmsCands + u * kLmsBlock +
// thread for u < kLmsLane), every row of segment s = blockIdx.x (rows [s * seg,
// min((s + 1) * seg, n))) in order.  The rows are the same for every lane, so each row of X
// and its y are scalar loads (registers shared by the wavefront, read by the vector
// arithmetic as operands; the workgroup's wavefronts read the same rows), two rows per step,
// and each row serves the lane's kLmsLane candidates.  A square r of candidate c with
// a < r < b (or NaN) is kept: written to c's array of the workspace at the segment's first
// row plus the number kept before it in the segment (so a segment's kept squares stay inside
// the segment's own rows, in row order).  The counts land in cnt[0][c][s] (kept) and
// cnt[1][c][s] (#(r <= a)), nseg = gridDim.x segments per candidate; SUM: the segment's sum of
// the r <= a (in row order) in psum[c][s].
constexpr int kLmsLane = 2;
constexpr int kLmsCands = kLmsBlock * kLmsLane;  // candidates per workgroup
#ifndef CPS_LMS_STAGE
#define CPS_LMS_STAGE 4
#endif
constexpr int kLmsStage = CPS_LMS_STAGE;  // kept squares staged in LDS per candidate
template <int P, bool SUM>
__global__ __launch_bounds__(kLmsBlock) void lms_filter_kernel(
    const double *__restrict__ X, const double *__restrict__ y, const double *__restrict__ betas,
    const double *__restrict__ ab, int64_t n, int32_t p, int64_t m, int64_t seg,
    double *__restrict__ R_out, uint32_t *__restrict__ cnt, double *__restrict__ psum) {
  constexpr int PM = P > 0 ? P : 16;
  constexpr int U = kLmsLane;
  // Each candidate's kept squares gather in LDS and go out kLmsStage at a time, as 16-byte
  // stores of contiguous places (single squares scattered over many candidates' arrays left
  // most of each written line empty).
  __shared__ double stg[kLmsCands][kLmsStage];
  const bool pairs = n % 2 == 0;  // (every segment then starts 16-byte aligned)
  const int pp = P > 0 ? P : p;
  const int tid = threadIdx.x;
  const int64_t sg = blockIdx.x, nseg = gridDim.x;
  const int64_t rb = sg * seg;
  const int64_t re = rb + seg < n ? rb + seg : n;
  int64_t c[U];
  bool live[U];
  double b[U][PM], lo[U], hi[U];
  CPS_GLOBAL double *dst[U];
  CPS_GLOBAL double *put[U];  // the place of the first staged square
  uint32_t below[U];          // #(r <= a)
  double sbelow[U];           // SUM: their sum, in row order
  int staged[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    c[u] = (int64_t)blockIdx.y * kLmsCands + u * kLmsBlock + tid;
    live[u] = c[u] < m;
#pragma unroll
    for (int j = 0; j < PM; ++j) b[u][j] = live[u] && j < pp ? betas[c[u] * pp + j] : 0.0;
    // a lane without a candidate stores nothing
    lo[u] = live[u] ? ab[2 * c[u]] : __builtin_inf();
    hi[u] = live[u] ? ab[2 * c[u] + 1] : -__builtin_inf();
    dst[u] = (CPS_GLOBAL double *)R_out + (live[u] ? c[u] : 0) * n + rb;
    put[u] = dst[u];
    below[u] = 0;
    sbelow[u] = 0.0;
    staged[u] = 0;
  }
  auto flush = [&](int u, int k) {
    const double *st = &stg[u * kLmsBlock + tid][0];
    if (k == kLmsStage && pairs) {
      using D2 = double __attribute__((ext_vector_type(2)));
#pragma unroll
      for (int v = 0; v < kLmsStage / 2; ++v)
        ((CPS_GLOBAL D2 *)put[u])[v] = D2{st[2 * v], st[2 * v + 1]};
    } else {
      for (int v = 0; v < k; ++v) put[u][v] = st[v];
    }
    put[u] += k;
  };
  // the squares of a step first (independent chains of dependent double additions, which
  // the scheduler interleaves), then their tests and stores (a branch each)
  auto keep = [&](int u, double r) {
    const bool le = r <= lo[u];
    if (live[u] && !le && !(r >= hi[u])) {
      stg[u * kLmsBlock + tid][staged[u]] = r;
      if (++staged[u] == kLmsStage) {
        flush(u, kLmsStage);
        staged[u] = 0;
      }
    }
    below[u] += le ? 1u : 0u;
    if (SUM && le) sbelow[u] += r;
  };
  int64_t i = rb;
  for (; i + 1 < re; i += 2) {  // two rows per step: both rows' scalar loads issued together
    double x0[PM], x1[PM];
#pragma unroll
    for (int j = 0; j < PM; ++j) {
      x0[j] = j < pp ? X[i * pp + j] : 0.0;
      x1[j] = j < pp ? X[(i + 1) * pp + j] : 0.0;
    }
    const double y0 = y[i], y1 = y[i + 1];
    // the 2U sums advance together, term by term (each in its own left-to-right order), so
    // that consecutive instructions are independent
    double s0[U], s1[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      s0[u] = x0[0] * b[u][0];
      s1[u] = x1[0] * b[u][0];
    }
#pragma unroll
    for (int j = 1; j < PM; ++j) {
      if (j < pp) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
          const double q0 = x0[j] * b[u][j], q1 = x1[j] * b[u][j];
          s0[u] = s0[u] + q0;
          s1[u] = s1[u] + q1;
        }
      }
    }
    double r0[U], r1[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const double d0 = y0 - s0[u], d1 = y1 - s1[u];
      r0[u] = d0 * d0;
      r1[u] = d1 * d1;
    }
    // (an empty statement that takes every square: the compiler would otherwise move each
    // chain down to its branch, and the chains would run one after another)
#pragma unroll
    for (int u = 0; u < U; ++u) asm volatile("" : "+v"(r0[u]), "+v"(r1[u]));
#pragma unroll
    for (int u = 0; u < U; ++u) keep(u, r0[u]);
#pragma unroll
    for (int u = 0; u < U; ++u) keep(u, r1[u]);
  }
  if (i < re) {
    double x0[PM];
#pragma unroll
    for (int j = 0; j < PM; ++j) x0[j] = j < pp ? X[i * pp + j] : 0.0;
    const double y0 = y[i];
#pragma unroll
    for (int u = 0; u < U; ++u) keep(u, sq_residual<P>(x0, y0, b[u], pp));
  }
#pragma unroll
  for (int u = 0; u < U; ++u) {
    if (live[u]) {
      flush(u, staged[u]);
      cnt[c[u] * nseg + sg] = (uint32_t)(put[u] - dst[u]);
      cnt[(m + c[u]) * nseg + sg] = below[u];
      if (SUM) psum[c[u] * nseg + sg] = sbelow[u];
    }
  }
}

constexpr int kLmsGatherBlock = 256;
constexpr int kLmsMaxSegs = 4096;  // segments per candidate (the gather's scan in LDS)
// Filter workgroups per resident set: one set left some CUs a second, lone workgroup (1.5 ms
// against 1.2 ms with four); more segments cost the gather more
constexpr int kLmsRounds = 2;

// ---- the filtered form's finish: one workgroup's exact select (cps_wgsel.h) over an array

// elements a narrowed key range may hold to finish in LDS (992: the gather kernel then fits
// four workgroups per CU, so 1024 candidates run in one round; 1024 left a second round of
// 256 on a third of the chip)
constexpr int kLmsSelCap = 992;
using WgSelLds = WgSelShared<kLmsGatherBlock>;

// The k-th smallest of W[0, len) (wg_select_pass over the array, eight loads per step).
template <int BLOCK>
__device__ __forceinline__ WgSelOut wg_select(const double *W, int64_t len, int64_t k, uint64_t klo,
                              uint64_t khi, int64_t below0, int64_t inrange0, uint32_t *hist,
                              double *buf, WgSelLds &sh) {
  const CPS_GLOBAL double *Wg = (const CPS_GLOBAL double *)W;
  auto pass = [&](auto f) { for_each8<BLOCK>(Wg, len, f); };
  return wg_select_pass<double, BLOCK>(pass, k, klo, khi, below0, inrange0, hist, buf,
                                       kLmsSelCap, sh);
}

// The record of a selection among all n squares.
__device__ inline void lms_write_result(cps_result *out, uint64_t key, int64_t less,
                                        int64_t equal, int64_t n, int32_t passes) {
  cps_result r;
  const double v = Traits<double>::unkey(key);
  r.value_bits = __builtin_bit_cast(uint64_t, v);
  r.value = v;
  r.less = less;
  r.equal = equal;
  r.greater = n - less - equal;
  r.passes = passes;
  r.status = CPS_STATUS_OK;
  *out = r;
}

__device__ inline void lms_write_nan(cps_result *out, int32_t passes) {
  cps_result r;
  r.value = __builtin_nan("");
  r.value_bits = __builtin_bit_cast(uint64_t, r.value);
  r.less = r.equal = r.greater = 0;
  r.passes = passes;
  r.status = CPS_STATUS_NAN;
  *out = r;
}

// The sum of the k smallest of a candidate's n squares: below (the squares under the
// selection's bracket, if any) plus those of W[0, len) below the selected value v, plus
// (k - #(r < v)) v (Section 6's trimmed sum with the multiplicity of v); one more pass over W.
template <int BLOCK>
__device__ inline double lms_ksum(const CPS_GLOBAL double *W, int64_t len, double v, int64_t k,
                                  int64_t less, double below, double *wred) {
  double part = 0.0;
  for_each8<BLOCK>(W, len, [&](double r) {
    if (r < v) part += r;
  });
  const double s = block_sum_fixed<BLOCK>(part, wred);
  return below + s + (double)(k - less) * v;
}

// One workgroup per candidate: the segments' counts and the bracket's test; where it holds,
// the kept squares packed into C + c * cap in segment order, counted on the way in 2^12 key
// bins over the bracket's open interval (a, b) (NaN noted), and the select of rank
// k - #(r <= a) among them from that histogram on, written as candidate c's result over all
// n squares.  Where it does not hold, full[c] = 1 and the candidate's whole array is formed
// and selected by the two kernels that follow.  passes: the filter, the packing, and the
// select's passes over the packed squares.
__global__ __launch_bounds__(kLmsGatherBlock) void lms_gather_kernel(
    const double *__restrict__ R, const uint32_t *__restrict__ cnt, const double *__restrict__ ab,
    int64_t n, int64_t m, int64_t nseg, int64_t seg, int64_t k, int64_t cap, double *__restrict__ C,
    const double *__restrict__ psum, cps_result *__restrict__ out, double *__restrict__ ksum,
    int32_t *__restrict__ full) {
  __shared__ uint32_t pre[kLmsMaxSegs + 1];
  __shared__ uint32_t hist[kHistMaxBins];
  __shared__ double buf[kLmsSelCap];
  __shared__ WgSelLds sh;
  __shared__ uint64_t tot[2];
  __shared__ double wred[kLmsGatherBlock / kWave];
  constexpr int SPT = kLmsMaxSegs / kLmsGatherBlock;
  const int64_t c = blockIdx.x;
  const int tid = threadIdx.x;
  uint32_t kv[SPT];
  uint64_t kcount = 0, bsum = 0;
#pragma unroll
  for (int j = 0; j < SPT; ++j) {
    const int64_t s = (int64_t)tid * SPT + j;
    kv[j] = s < nseg ? cnt[c * nseg + s] : 0u;
    kcount += kv[j];
    bsum += s < nseg ? cnt[(m + c) * nseg + s] : 0u;
  }
  uint64_t run = block_exclusive_scan<kLmsGatherBlock>(kcount, sh.wsum);
  const uint64_t bpre = block_exclusive_scan<kLmsGatherBlock>(bsum, sh.wsum);
  if (tid == kLmsGatherBlock - 1) {
    tot[0] = run + kcount;
    tot[1] = bpre + bsum;
    pre[kLmsMaxSegs] = (uint32_t)(run + kcount);
  }
  if (tid == 0) sh.flag = 0u;
#pragma unroll
  for (int j = 0; j < SPT; ++j) {
    pre[tid * SPT + j] = (uint32_t)run;
    run += kv[j];
  }
  for (int b = tid; b < kHistMaxBins; b += kLmsGatherBlock) hist[b] = 0u;
  __syncthreads();
  const int64_t inside = (int64_t)tot[0], bel = (int64_t)tot[1];
  const double lo = ab[2 * c], hi = ab[2 * c + 1];
  const bool holds = lo < hi && bel < k && k <= bel + inside && inside <= cap;
  if (tid == 0) full[c] = holds ? 0 : 1;
  if (!holds) return;  // (uniform)
  // the keys of a < r < b
  const uint64_t ka = Traits<double>::key(lo) + 1, kb = Traits<double>::key(hi) - 1;
  int shift = 0;
  while (((kb - ka) >> shift) >= (uint64_t)kHistMaxBins) ++shift;
  // packed place j comes from the segment s with pre[s] <= j < pre[s + 1]; each thread's
  // places rise, so its segment only moves forward (pre[kLmsMaxSegs] = inside ends it); the
  // places of a step are consecutive over the threads, so the stores are (packing by
  // segments per thread, its own places together, took 2.5 times as long); four places per
  // step keep four loads in flight
  const CPS_GLOBAL double *Rc = (const CPS_GLOBAL double *)(R + c * n);
  CPS_GLOBAL double *Cc = (CPS_GLOBAL double *)(C + c * cap);
  constexpr int U = 4;
  int sg = 0;
  bool nan = false;
  for (int64_t j0 = tid; j0 < inside; j0 += U * kLmsGatherBlock) {
    double v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t j = j0 + (int64_t)u * kLmsGatherBlock;
      if (j < inside) {
        while ((int64_t)pre[sg + 1] <= j) ++sg;
        v[u] = Rc[(int64_t)sg * seg + (j - (int64_t)pre[sg])];
      }
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t j = j0 + (int64_t)u * kLmsGatherBlock;
      if (j < inside) {
        Cc[j] = v[u];
        const uint64_t kk = Traits<double>::key(v[u]);
        nan = nan || !(v[u] == v[u]);
        if (kk >= ka && kk <= kb) atomicAdd(&hist[(uint32_t)((kk - ka) >> shift)], 1u);
      }
    }
  }
  if (nan) atomicOr(&sh.flag, 1u);
  __syncthreads();  // (the packed squares, written by this workgroup, are read below)
  if (sh.flag != 0u) {  // (uniform)
    if (tid == 0) {
      lms_write_nan(out + c, 2);
      if (ksum) ksum[c] = __builtin_nan("");
    }
    return;
  }
  // the bin of rank k - #(r <= a) among the packed squares
  const int64_t rr = k - bel;
  constexpr int BPT = kHistMaxBins / kLmsGatherBlock;
  uint64_t hv[BPT];
  uint64_t hs = 0;
#pragma unroll
  for (int j = 0; j < BPT; ++j) {
    hv[j] = hist[tid * BPT + j];
    hs += hv[j];
  }
  uint64_t cum = block_exclusive_scan<kLmsGatherBlock>(hs, sh.wsum);
#pragma unroll
  for (int j = 0; j < BPT; ++j) {
    if (cum < (uint64_t)rr && (uint64_t)rr <= cum + hv[j]) {
      sh.bin = tid * BPT + j;
      sh.cum = (int64_t)cum;
      sh.inb = (int64_t)hv[j];
    }
    cum += hv[j];
  }
  __syncthreads();
  const uint64_t b = (uint64_t)sh.bin;
  const int64_t below0 = sh.cum, in0 = sh.inb;
  __syncthreads();
  const uint64_t nlo = ka + (b << shift);
  uint64_t nhi = nlo + ((1ull << shift) - 1);
  if (nhi > kb || nhi < nlo) nhi = kb;
  const WgSelOut r = wg_select<kLmsGatherBlock>(C + c * cap, inside, rr, nlo, nhi, below0, in0,
                                                hist, buf, sh);
  if (tid == 0) lms_write_result(out + c, r.key, bel + r.less, r.equal, n, 3 + r.passes);
  if (ksum) {  // (uniform)
    // the squares under a: the segments' sums, each thread's run of segments in order
    double sb = 0.0;
#pragma unroll
    for (int j = 0; j < SPT; ++j) {
      const int64_t s2 = (int64_t)tid * SPT + j;
      if (s2 < nseg) sb += psum[c * nseg + s2];
    }
    const double below_sum = block_sum_fixed<kLmsGatherBlock>(sb, wred);
    const double v = Traits<double>::unkey(r.key);
    const double t = lms_ksum<kLmsGatherBlock>(Cc, inside, v, rr, r.less, below_sum, wred);
    if (tid == 0) ksum[c] = t;
  }
}

// After the fallback residual kernel: the candidates whose bracket missed, over their whole
// arrays of n squares (a first pass for the key range and NaN, then wg_select); the others'
// workgroups return at once.
__global__ __launch_bounds__(kLmsGatherBlock) void lms_full_select_kernel(
    const double *__restrict__ R, int64_t n, int64_t k, const int32_t *__restrict__ full,
    cps_result *__restrict__ out, double *__restrict__ ksum) {
  __shared__ uint32_t hist[kHistMaxBins];
  __shared__ double buf[kLmsSelCap];
  __shared__ WgSelLds sh;
  __shared__ double wred[kLmsGatherBlock / kWave];
  const int64_t c = blockIdx.x;
  const int tid = threadIdx.x;
  if (full[c] == 0) return;  // (uniform)
  if (tid == 0) {
    sh.kext[0] = ~0ull;
    sh.kext[1] = 0ull;
    sh.flag = 0u;
  }
  __syncthreads();
  const CPS_GLOBAL double *Rc = (const CPS_GLOBAL double *)(R + c * n);
  uint64_t kmn = ~0ull, kmx = 0ull;
  bool nan = false;
  for_each8<kLmsGatherBlock>(Rc, n, [&](double v) {
    const uint64_t kk = Traits<double>::key(v);
    nan = nan || !(v == v);
    kmn = kk < kmn ? kk : kmn;
    kmx = kk > kmx ? kk : kmx;
  });
  atomicMin(&sh.kext[0], (unsigned long long)kmn);
  atomicMax(&sh.kext[1], (unsigned long long)kmx);
  if (nan) atomicOr(&sh.flag, 1u);
  __syncthreads();
  if (sh.flag != 0u) {  // (uniform)
    if (tid == 0) {
      lms_write_nan(out + c, 3);
      if (ksum) ksum[c] = __builtin_nan("");
    }
    return;
  }
  const WgSelOut r = wg_select<kLmsGatherBlock>(R + c * n, n, k, sh.kext[0], sh.kext[1], 0, n,
                                                hist, buf, sh);
  if (tid == 0) lms_write_result(out + c, r.key, r.less, r.equal, n, 3 + r.passes);
  if (ksum) {  // (uniform)
    const double t = lms_ksum<kLmsGatherBlock>(Rc, n, Traits<double>::unkey(r.key), k, r.less,
                                               0.0, wred);
    if (tid == 0) ksum[c] = t;
  }
}

__global__ void lms_descriptor_kernel(const double *R, int64_t n, int64_t m, int64_t rank,
                                      const double **ptrs, int64_t *sizes, int64_t *ks) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < m;
       c += (int64_t)gridDim.x * blockDim.x) {
    ptrs[c] = R + c * n;
    sizes[c] = n;
    ks[c] = rank;
  }
}

// Least trimmed squares (Section 6): from the selection of rank h among a candidate's squared
// residuals (m = r_(h), #(r < m), #(r = m)) and the sum of its h smallest, the record with
// a = h - #(r < m), the weight of m in Section 6's rho.
__global__ void lts_finish_kernel(const cps_result *__restrict__ sel, const double *__restrict__ ksum,
                                  int64_t m, int64_t h, cps_trim *__restrict__ out) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < m;
       c += (int64_t)gridDim.x * blockDim.x) {
    const cps_result r = sel[c];
    cps_trim t;
    t.F = r.status == 0 ? ksum[c] : __builtin_nan("");
    t.m = r.value;
    t.below = r.less;
    t.a = r.status == 0 ? h - r.less : 0;
    t.b = r.equal;
    t.status = r.status;
    t.pad = 0;
    out[c] = t;
  }
}

hipError_t launch_lts_finish(const cps_result *sel, const double *ksum, int64_t m, int64_t h,
                             cps_trim *out, hipStream_t stream) {
  lts_finish_kernel<<<dim3((unsigned)((m + 255) / 256)), dim3(256), 0, stream>>>(sel, ksum, m, h, out);
  return hipGetLastError();
}

hipError_t launch_lms_residuals(const double *X, const double *y, const double *betas, int64_t n,
                                int32_t p, int64_t m, int64_t rank, double *R, const double **ptrs,
                                int64_t *sizes, int64_t *ks, int cu_count, hipStream_t stream) {
  const int64_t groups = (m + kLmsGroup - 1) / kLmsGroup;
  int64_t bx = (n + kLmsBlock - 1) / kLmsBlock;
  const int64_t want = (int64_t)cu_count * 8 / (groups < 1 ? 1 : groups) + 1;
  if (bx > want) bx = want;
  if (bx < 1) bx = 1;
  const dim3 grid((unsigned)bx, (unsigned)groups);
  const bool aligned = ((uintptr_t)X % 16 == 0) && ((uintptr_t)y % 16 == 0) && ((uintptr_t)R % 16 == 0);
  if (p == 8 && aligned && n % kLmsRows == 0) {
    const int64_t rb = (n / kLmsRows + kLmsBlock - 1) / kLmsBlock;
    const dim3 g2((unsigned)(bx < rb ? bx : rb), (unsigned)groups);
    lms_residual_rows_kernel<8, kLmsRows, false>
        <<<g2, dim3(kLmsBlock), 0, stream>>>(X, y, betas, n, m, R, nullptr);
  } else if (p == 8) {
    lms_residual_kernel<8, false><<<grid, dim3(kLmsBlock), 0, stream>>>(X, y, betas, n, p, m, R, nullptr);
  } else {
    lms_residual_kernel<0, false><<<grid, dim3(kLmsBlock), 0, stream>>>(X, y, betas, n, p, m, R, nullptr);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  lms_descriptor_kernel<<<dim3((unsigned)((m + 255) / 256)), dim3(256), 0, stream>>>(R, n, m, rank,
                                                                                    ptrs, sizes, ks);
  return hipGetLastError();
}

void lms_filter_shape(int64_t n, int64_t m, int32_t p, bool vec, int cu_count, int64_t *bx,
                      int64_t *nseg, int64_t *seg) {
  // the filter: kLmsRounds times as many workgroups as are resident at once over (segments x
  // groups of kLmsCands candidates), a multiple of 16 rows per segment (at least 256), every
  // segment holding rows
  int per_cu = 0;
  (void)vec;
  const hipError_t e =
      p == 8 ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, lms_filter_kernel<8, false>, kLmsBlock, 0)
             : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, lms_filter_kernel<0, false>, kLmsBlock, 0);
  if (e != hipSuccess || per_cu < 1) per_cu = 4;
  const int64_t fgroups = (m + kLmsCands - 1) / kLmsCands;
  int64_t ns = (int64_t)cu_count * per_cu * kLmsRounds / fgroups;
  const int64_t nmax = (n + 255) / 256;
  if (ns > nmax) ns = nmax;
  if (ns > kLmsMaxSegs) ns = kLmsMaxSegs;
  if (ns < 1) ns = 1;
  const int64_t sl = ((n + ns - 1) / ns + 15) / 16 * 16;
  *nseg = (n + sl - 1) / sl;
  *seg = sl;
  // the fallback residual kernel's grid, as the materialised form's
  const int64_t groups = (m + kLmsGroup - 1) / kLmsGroup;
  int64_t b = (n + kLmsBlock - 1) / kLmsBlock;
  const int64_t want = (int64_t)cu_count * 8 / groups + 1;
  if (b > want) b = want;
  *bx = b < 1 ? 1 : b;
}

int64_t lms_filter_cap(int64_t n) { return (n / 8 + 1 + 31) / 32 * 32; }

hipError_t launch_lms_filtered(const double *X, const double *y, const double *betas, int64_t n,
                               int32_t p, int64_t m, int64_t rank, const LmsFilterBufs &w,
                               cps_result *out, double *ksum, hipStream_t stream) {
  const int64_t groups = (m + kLmsGroup - 1) / kLmsGroup;
  const int64_t fgroups = (m + kLmsCands - 1) / kLmsCands;
  const int64_t sgroups = (m + kLmsBlock - 1) / kLmsBlock;
  // one run of the sample per workgroup
  const dim3 sg((unsigned)(sample_runs(n)), (unsigned)sgroups);
  if (p == 8)
    lms_sample_kernel<8><<<sg, dim3(kLmsBlock), 0, stream>>>(X, y, betas, n, p, m, w.Rs);
  else
    lms_sample_kernel<0><<<sg, dim3(kLmsBlock), 0, stream>>>(X, y, betas, n, p, m, w.Rs);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  lms_bracket_kernel<<<dim3((unsigned)m), dim3(kLmsBracketBlock), 0, stream>>>(w.Rs, n, rank, w.ab);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const bool aligned = ((uintptr_t)X % 16 == 0) && ((uintptr_t)y % 16 == 0);
  const dim3 fgrid((unsigned)w.nseg, (unsigned)fgroups);
  if (p == 8 && !ksum)
    lms_filter_kernel<8, false><<<fgrid, dim3(kLmsBlock), 0, stream>>>(
        X, y, betas, w.ab, n, p, m, w.seg, w.R, w.cnt, nullptr);
  else if (p == 8)
    lms_filter_kernel<8, true><<<fgrid, dim3(kLmsBlock), 0, stream>>>(
        X, y, betas, w.ab, n, p, m, w.seg, w.R, w.cnt, w.psum);
  else if (!ksum)
    lms_filter_kernel<0, false><<<fgrid, dim3(kLmsBlock), 0, stream>>>(
        X, y, betas, w.ab, n, p, m, w.seg, w.R, w.cnt, nullptr);
  else
    lms_filter_kernel<0, true><<<fgrid, dim3(kLmsBlock), 0, stream>>>(
        X, y, betas, w.ab, n, p, m, w.seg, w.R, w.cnt, w.psum);
  const dim3 grid((unsigned)w.bx, (unsigned)groups);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  lms_gather_kernel<<<dim3((unsigned)m), dim3(kLmsGatherBlock), 0, stream>>>(
      w.R, w.cnt, w.ab, n, m, w.nseg, w.seg, rank, w.cap, w.C, w.psum, out, ksum, w.full);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  // the candidates whose bracket missed: their whole arrays (workgroups without one return)
  if (p == 8 && aligned && (uintptr_t)w.R % 16 == 0 && n % kLmsRows == 0) {
    int64_t rb = (n / kLmsRows + kLmsBlock - 1) / kLmsBlock;
    if (rb > w.bx) rb = w.bx;
    lms_residual_rows_kernel<8, kLmsRows, true>
        <<<dim3((unsigned)rb, (unsigned)groups), dim3(kLmsBlock), 0, stream>>>(X, y, betas, n, m, w.R,
                                                                           w.full);
  } else {
    lms_residual_kernel<0, true><<<grid, dim3(kLmsBlock), 0, stream>>>(X, y, betas, n, p, m, w.R,
                                                                        w.full);
  }
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  lms_full_select_kernel<<<dim3((unsigned)m), dim3(kLmsGatherBlock), 0, stream>>>(w.R, n, rank,
                                                                                w.full, out, ksum);
  return hipGetLastError();
}

}  // namespace cps
