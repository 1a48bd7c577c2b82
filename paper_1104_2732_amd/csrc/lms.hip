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

// The filter: one candidate per lane (c = blockIdx.y * kLmsBlock + thread), every row of
// segment s = blockIdx.x (rows [s * seg, min((s + 1) * seg, n))) in order.  The rows are the
// same for every lane: the workgroup stages them through LDS in tiles of kLmsTile rows (one
// row per thread, the next tile's loads in flight while the current one is used; one barrier
// per tile), and each lane reads every row of a tile as a broadcast.  A square r of candidate
// c with a < r < b (or NaN) is kept: written to c's array of the workspace at the segment's
// first row plus the number kept before it in the segment (so a segment's kept squares stay
// inside the segment's own rows, in row order).  The counts land in cnt[0][c][s] (kept) and
// cnt[1][c][s] (#(r <= a)), nseg = gridDim.x segments per candidate.  VEC: X and y are
// 16-byte aligned and P = 8 (each staged row is four 16-byte loads).
constexpr int kLmsTile = 128;
template <int P, bool VEC>
__global__ __launch_bounds__(kLmsBlock) void lms_filter_kernel(
    const double *__restrict__ X, const double *__restrict__ y, const double *__restrict__ betas,
    const double *__restrict__ ab, int64_t n, int32_t p, int64_t m, int64_t seg,
    double *__restrict__ R_out, uint32_t *__restrict__ cnt) {
  constexpr int PM = P > 0 ? P : 16;
  static_assert(!VEC || PM % 2 == 0, "16-byte rows");
  // a staged row: its PM values, then y, padded to a 16-byte multiple
  constexpr int RW = (PM + 1 + 1) / 2 * 2;
  __shared__ double sx[2][kLmsTile][RW];
  const int pp = P > 0 ? P : p;
  const int tid = threadIdx.x;
  const int64_t c = (int64_t)blockIdx.y * kLmsBlock + tid;
  const bool live = c < m;
  double b[PM];
#pragma unroll
  for (int j = 0; j < PM; ++j) b[j] = live && j < pp ? betas[c * pp + j] : 0.0;
  // a lane without a candidate stores nothing
  const double lo = live ? ab[2 * c] : __builtin_inf();
  const double hi = live ? ab[2 * c + 1] : -__builtin_inf();
  const int64_t sg = blockIdx.x, nseg = gridDim.x;
  const int64_t rb = sg * seg;
  const int64_t re = rb + seg < n ? rb + seg : n;
  CPS_GLOBAL double *dst = (CPS_GLOBAL double *)R_out + (live ? c : 0) * n + rb;
  const CPS_GLOBAL double *Xg = (const CPS_GLOBAL double *)X;
  const CPS_GLOBAL double *yg = (const CPS_GLOBAL double *)y;
  // one row per thread of the first kLmsTile threads
  double lx[PM], ly = 0.0;
  auto load_row = [&](int64_t t0) {
    const int64_t i = t0 + tid;
    const bool ok = tid < kLmsTile && i < re;
    if (VEC) {
      using D2 = double __attribute__((ext_vector_type(2)));
#pragma unroll
      for (int v = 0; v < PM / 2; ++v) {
        const D2 w = ok ? ((const CPS_GLOBAL D2 *)(Xg + i * PM))[v] : D2{0.0, 0.0};
        lx[2 * v] = w.x;
        lx[2 * v + 1] = w.y;
      }
    } else {
#pragma unroll
      for (int j = 0; j < PM; ++j) lx[j] = ok && j < pp ? Xg[i * pp + j] : 0.0;
    }
    ly = ok ? yg[i] : 0.0;
  };
  auto store_row = [&](int buf) {
    if (tid < kLmsTile) {
#pragma unroll
      for (int j = 0; j < PM; ++j) sx[buf][tid][j] = lx[j];
      sx[buf][tid][PM] = ly;
    }
  };
  // #(r <= a), and the next kept square's place
  uint32_t below = 0;
  CPS_GLOBAL double *put = dst;
  load_row(rb);
  store_row(0);
  __syncthreads();
  int buf = 0;
  for (int64_t t0 = rb; t0 < re; t0 += kLmsTile) {
    const bool more = t0 + kLmsTile < re;
    if (more) load_row(t0 + kLmsTile);
    const int rows = re - t0 < kLmsTile ? (int)(re - t0) : kLmsTile;
    // (the tile's address as a lane value, so that one register holds it through the rows)
    const double *tile = &sx[buf][0][0] + __builtin_amdgcn_mbcnt_lo(0u, 0u);
#pragma unroll 4
    for (int q = 0; q < rows; ++q) {
      double xv[PM];
#pragma unroll
      for (int j = 0; j < PM; ++j) xv[j] = tile[q * RW + j];
      const double r = sq_residual<P>(xv, tile[q * RW + PM], b, pp);
      const bool le = r <= lo;
      if (live && !le && !(r >= hi)) *put++ = r;
      below += le ? 1u : 0u;
    }
    if (more) store_row(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
  const uint32_t kept = (uint32_t)(put - dst);
  if (live) {
    cnt[c * nseg + sg] = kept;
    cnt[(m + c) * nseg + sg] = below;
  }
}

constexpr int kLmsGatherBlock = 256;
constexpr int kLmsMaxSegs = 4096;  // segments per candidate (the gather's scan in LDS)

// One workgroup per candidate: the segments' counts, the bracket's test, and, where it holds,
// the kept squares packed into C + c * cap in segment order; then the batched call's
// descriptors and side[2c], side[2c+1] = #(r <= a), #(r >= b) (-1, -1 and full[c] = 1 where
// the candidate takes the materialised path).
__global__ __launch_bounds__(kLmsGatherBlock) void lms_gather_kernel(
    const double *__restrict__ R, const uint32_t *__restrict__ cnt, const double *__restrict__ ab,
    int64_t n, int64_t m, int64_t nseg, int64_t seg, int64_t k, int64_t cap, double *__restrict__ C,
    const double **ptrs, int64_t *sizes, int64_t *ks, int64_t *side, int32_t *full) {
  __shared__ uint32_t pre[kLmsMaxSegs + 1];
  __shared__ uint64_t wsum[kLmsGatherBlock / kWave];
  __shared__ uint64_t tot[2];
  constexpr int SPT = kLmsMaxSegs / kLmsGatherBlock;
  const int64_t c = blockIdx.x;
  const int tid = threadIdx.x;
  uint32_t kv[SPT];
  uint64_t ksum = 0, bsum = 0;
#pragma unroll
  for (int j = 0; j < SPT; ++j) {
    const int64_t s = (int64_t)tid * SPT + j;
    kv[j] = s < nseg ? cnt[c * nseg + s] : 0u;
    ksum += kv[j];
    bsum += s < nseg ? cnt[(m + c) * nseg + s] : 0u;
  }
  uint64_t run = block_exclusive_scan<kLmsGatherBlock>(ksum, wsum);
  const uint64_t bpre = block_exclusive_scan<kLmsGatherBlock>(bsum, wsum);
  if (tid == kLmsGatherBlock - 1) {
    tot[0] = run + ksum;
    tot[1] = bpre + bsum;
    pre[kLmsMaxSegs] = (uint32_t)(run + ksum);
  }
#pragma unroll
  for (int j = 0; j < SPT; ++j) {
    pre[tid * SPT + j] = (uint32_t)run;
    run += kv[j];
  }
  __syncthreads();
  const int64_t inside = (int64_t)tot[0], bel = (int64_t)tot[1];
  const double lo = ab[2 * c], hi = ab[2 * c + 1];
  const bool holds = lo < hi && bel < k && k <= bel + inside && inside <= cap;
  if (holds) {
    // packed place j comes from the segment s with pre[s] <= j < pre[s + 1]; each thread's
    // places rise, so its segment only moves forward (pre[kLmsMaxSegs] = inside ends it);
    // four places per step keep four loads in flight
    const CPS_GLOBAL double *Rc = (const CPS_GLOBAL double *)(R + c * n);
    CPS_GLOBAL double *Cc = (CPS_GLOBAL double *)(C + c * cap);
    constexpr int U = 4;
    int sg = 0;
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
        if (j < inside) Cc[j] = v[u];
      }
    }
  }
  if (tid == 0) {
    ptrs[c] = holds ? C + c * cap : R + c * n;
    sizes[c] = holds ? inside : n;
    ks[c] = holds ? k - bel : k;
    side[2 * c] = holds ? bel : -1;
    side[2 * c + 1] = holds ? n - bel - inside : -1;
    full[c] = holds ? 0 : 1;
  }
}

// After the batched selection: a packed candidate's counts over all n squares (the
// selection saw only the kept ones), and its one pass over the residuals.
__global__ void lms_fixup_kernel(cps_result *__restrict__ out, const int64_t *__restrict__ side,
                                 int64_t m) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < m;
       c += (int64_t)gridDim.x * blockDim.x) {
    if (side[2 * c] < 0 || out[c].status != CPS_STATUS_OK) continue;
    out[c].less += side[2 * c];
    out[c].greater += side[2 * c + 1];
    out[c].passes += 1;
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
  // the filter: as many workgroups as are resident at once over (segments x groups of
  // kLmsBlock candidates), so that no tail of lone workgroups is left; segments of at least
  // 256 rows, every segment holding rows
  int per_cu = 0;
  const hipError_t e =
      vec && p == 8
          ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, lms_filter_kernel<8, true>, kLmsBlock, 0)
          : hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, lms_filter_kernel<0, false>, kLmsBlock, 0);
  if (e != hipSuccess || per_cu < 1) per_cu = 4;
  const int64_t fgroups = (m + kLmsBlock - 1) / kLmsBlock;
  int64_t ns = (int64_t)cu_count * per_cu / fgroups;
  const int64_t nmax = (n + 255) / 256;
  if (ns > nmax) ns = nmax;
  if (ns > kLmsMaxSegs) ns = kLmsMaxSegs;
  if (ns < 1) ns = 1;
  const int64_t sl = (n + ns - 1) / ns;
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
                               hipStream_t stream) {
  const int64_t groups = (m + kLmsGroup - 1) / kLmsGroup;
  const int64_t fgroups = (m + kLmsBlock - 1) / kLmsBlock;
  // one run of the sample per workgroup
  const dim3 sg((unsigned)(sample_runs(n)), (unsigned)fgroups);
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
  if (p == 8 && aligned)
    lms_filter_kernel<8, true><<<fgrid, dim3(kLmsBlock), 0, stream>>>(X, y, betas, w.ab, n, p, m,
                                                                       w.seg, w.R, w.cnt);
  else
    lms_filter_kernel<0, false><<<fgrid, dim3(kLmsBlock), 0, stream>>>(X, y, betas, w.ab, n, p, m,
                                                                        w.seg, w.R, w.cnt);
  const dim3 grid((unsigned)w.bx, (unsigned)groups);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  lms_gather_kernel<<<dim3((unsigned)m), dim3(kLmsGatherBlock), 0, stream>>>(
      w.R, w.cnt, w.ab, n, m, w.nseg, w.seg, rank, w.cap, w.C, w.ptrs, w.sizes, w.ks, w.side, w.full);
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
  return hipGetLastError();
}

hipError_t launch_lms_fixup(cps_result *out, const int64_t *side, int64_t m, hipStream_t stream) {
  lms_fixup_kernel<<<dim3((unsigned)((m + 255) / 256)), dim3(256), 0, stream>>>(out, side, m);
  return hipGetLastError();
}

}  // namespace cps
