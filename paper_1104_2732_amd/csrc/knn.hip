// k nearest neighbours (Section 6, last paragraph): for each query point, the squared
// Euclidean distances to every data point, their k-th smallest d_k by the batched selection,
// and the mean ordinate of the k nearest points, formed by a reduction with the weight of
// Section 6's rho adapted to an indicator: 1 below d_k, a/b at d_k (b points at d_k, a = k -
// #(d < d_k) of them count), 0 above.
//
// The distance kernel forms d_i = sum_j (P_ij - q_j)^2 for a group of queries per thread row
// (each data point read once per group), left to right in j with every difference, square
// and sum rounded on its own in float (the library is built without fused multiply-add), and
// writes them query-major, one array of n per query.  The reduction reads the distance
// arrays back (one read of 4 bytes per distance; recomputing them from the points instead
// reads the points once per query from the caches and measured 13 % slower in all) and sums
// the ordinates below and at d_k in double precision, per block in a fixed order, then per
// query in block order.
#include "cps_device.h"
#include "cps_kernels.h"
#include "cps_passes.h"
#include "cps_sample.h"
#include "cps_wgsel.h"

namespace cps {

#ifndef CPS_KNN_GROUP
#define CPS_KNN_GROUP 64
#endif
#ifndef CPS_KNN_READ
#define CPS_KNN_READ 1
#endif
constexpr int kKnnGroup = CPS_KNN_GROUP;  // queries per thread row of the distance kernel
// the reduction reads the distance arrays back (1) or recomputes the distances (0)
constexpr bool kKnnRead = CPS_KNN_READ != 0;
constexpr int kKnnBlock = 256;
constexpr int kKnnRedBlocks = 8;  // reduction blocks per query

template <int D>
__device__ inline float knn_dist(const float (&row)[D > 0 ? D : 16], const float *q, int dim) {
  const int dd = D > 0 ? D : dim;
  float s = 0.0f;
#pragma unroll
  for (int j = 0; j < (D > 0 ? D : 16); ++j) {
    if (j < dd) {
      const float e = row[j] - q[j];
      const float sq = e * e;
      s = j == 0 ? sq : s + sq;
    }
  }
  return s;
}

template <int D>
__global__ __launch_bounds__(kKnnBlock) void knn_distance_kernel(
    const float *__restrict__ P, const float *__restrict__ Q, int64_t n, int32_t dim, int64_t nq,
    float *__restrict__ Dst) {
  __shared__ float sq[kKnnGroup * 16];  // (up to 16 coordinates per query)
  const int64_t c0 = (int64_t)blockIdx.y * kKnnGroup;
  const int nc = (int)((nq - c0) < kKnnGroup ? (nq - c0) : kKnnGroup);
  for (int t = threadIdx.x; t < nc * dim; t += kKnnBlock) sq[t] = Q[c0 * dim + t];
  __syncthreads();
  const CPS_GLOBAL float *Pg = (const CPS_GLOBAL float *)P;
  CPS_GLOBAL float *Dg = (CPS_GLOBAL float *)Dst;
  for (int64_t i = (int64_t)blockIdx.x * kKnnBlock + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * kKnnBlock) {
    float row[D > 0 ? D : 16];
    const int dd = D > 0 ? D : dim;
#pragma unroll
    for (int j = 0; j < (D > 0 ? D : 16); ++j)
      if (j < dd) row[j] = Pg[i * dd + j];
    for (int c = 0; c < nc; ++c)
      __builtin_nontemporal_store(knn_dist<D>(row, sq + c * dd, dim), &Dg[(c0 + c) * n + i]);
  }
}

__global__ void knn_descriptor_kernel(const float *Dst, int64_t n, int64_t nq, int64_t k,
                                      const float **ptrs, int64_t *sizes, int64_t *ks) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nq;
       c += (int64_t)gridDim.x * blockDim.x) {
    ptrs[c] = Dst + c * n;
    sizes[c] = n;
    ks[c] = k;
  }
}

// Partial sums of the ordinates below and at d_k over this block's slice of the points.
template <int D>
__global__ __launch_bounds__(kKnnBlock) void knn_partial_kernel(
    const float *__restrict__ P, const float *__restrict__ f, const float *__restrict__ Q,
    int64_t n, int32_t dim, const cps_result *__restrict__ sel, double *__restrict__ pd,
    int64_t *__restrict__ pi) {
  __shared__ double sd[8][kKnnBlock / kWave];
  __shared__ int64_t si[8][kKnnBlock / kWave];
  __shared__ float sq[16];
  const int64_t c = blockIdx.y;
  if (threadIdx.x < dim) sq[threadIdx.x] = Q[c * dim + threadIdx.x];
  __syncthreads();
  const float dk = (float)sel[c].value;
  const int64_t per = (n + gridDim.x - 1) / gridDim.x;
  const int64_t lo = (int64_t)blockIdx.x * per;
  const int64_t hi = lo + per < n ? lo + per : n;
  double sb = 0.0, se = 0.0;
  int64_t nb = 0, ne = 0;
  const int dd = D > 0 ? D : dim;
  for (int64_t i = lo + threadIdx.x; i < hi; i += kKnnBlock) {
    float row[D > 0 ? D : 16];
#pragma unroll
    for (int j = 0; j < (D > 0 ? D : 16); ++j)
      if (j < dd) row[j] = P[i * dd + j];
    const float d = knn_dist<D>(row, sq, dim);
    const double fi = (double)f[i];
    if (d < dk) {
      sb += fi;
      ++nb;
    } else if (d == dk) {
      se += fi;
      ++ne;
    }
  }
  double dv[8] = {sb, se, 0, 0, 0, 0, 0, 0};
  int dop[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int64_t iv[8] = {nb, ne, 0, 0, 0, 0, 0, 0};
  block_reduce<kKnnBlock, 2, 2>(dv, dop, iv, false, sd, si);
  if (threadIdx.x == 0) {
    const int64_t slot = c * gridDim.x + blockIdx.x;
    pd[2 * slot] = dv[0];
    pd[2 * slot + 1] = dv[1];
    pi[2 * slot] = iv[0];
    pi[2 * slot + 1] = iv[1];
  }
}

// The same partial sums from the distance arrays the distance kernel wrote (query c's at
// D + c n): 16-byte loads of distances and ordinates when n is a multiple of 4.
template <bool VEC>
__global__ __launch_bounds__(kKnnBlock) void knn_partial_read_kernel(
    const float *__restrict__ D, const float *__restrict__ f, int64_t n,
    const cps_result *__restrict__ sel, double *__restrict__ pd, int64_t *__restrict__ pi) {
  __shared__ double sd[8][kKnnBlock / kWave];
  __shared__ int64_t si[8][kKnnBlock / kWave];
  const int64_t c = blockIdx.y;
  const float dk = (float)sel[c].value;
  int64_t per = (n + gridDim.x - 1) / gridDim.x;
  per = (per + 3) / 4 * 4;
  const int64_t lo = (int64_t)blockIdx.x * per;
  const int64_t hi = lo + per < n ? lo + per : n;
  const float *Dr = D + c * n;
  double sb = 0.0, se = 0.0;
  int64_t nb = 0, ne = 0;
  auto one = [&](float d, float fi) {
    if (d < dk) {
      sb += (double)fi;
      ++nb;
    } else if (d == dk) {
      se += (double)fi;
      ++ne;
    }
  };
  if (VEC) {
    using F4 = float __attribute__((ext_vector_type(4)));
    for (int64_t i = lo + 4 * (int64_t)threadIdx.x; i < hi; i += 4 * (int64_t)kKnnBlock) {
      const F4 d = __builtin_nontemporal_load((const F4 *)(Dr + i));
      const F4 fv = *(const F4 *)(f + i);
      one(d.x, fv.x);
      one(d.y, fv.y);
      one(d.z, fv.z);
      one(d.w, fv.w);
    }
  } else {
    for (int64_t i = lo + threadIdx.x; i < hi; i += kKnnBlock) one(Dr[i], f[i]);
  }
  double dv[8] = {sb, se, 0, 0, 0, 0, 0, 0};
  int dop[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int64_t iv[8] = {nb, ne, 0, 0, 0, 0, 0, 0};
  block_reduce<kKnnBlock, 2, 2>(dv, dop, iv, false, sd, si);
  if (threadIdx.x == 0) {
    const int64_t slot = c * gridDim.x + blockIdx.x;
    pd[2 * slot] = dv[0];
    pd[2 * slot + 1] = dv[1];
    pi[2 * slot] = iv[0];
    pi[2 * slot + 1] = iv[1];
  }
}

__global__ void knn_final_kernel(int64_t nq, int64_t k, int nb, const cps_result *__restrict__ sel,
                                 const double *__restrict__ pd, const int64_t *__restrict__ pi,
                                 cps_knn *__restrict__ out) {
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nq;
       c += (int64_t)gridDim.x * blockDim.x) {
    double sb = 0.0, se = 0.0;
    int64_t below = 0, eq = 0;
    for (int b = 0; b < nb; ++b) {
      sb += pd[2 * (c * nb + b)];
      se += pd[2 * (c * nb + b) + 1];
      below += pi[2 * (c * nb + b)];
      eq += pi[2 * (c * nb + b) + 1];
    }
    const cps_result r = sel[c];
    cps_knn o;
    o.dk = (float)r.value;
    o.status = r.status;
    o.below = below;
    o.equal = eq;
    // the reduction's counts are the selection's (anything else: the data changed)
    if (r.status == 0 && (below != r.less || eq != r.equal)) o.status = CPS_STATUS_INTERNAL;
    const double a = (double)(k - below);
    o.mean = (o.status == 0 && eq > 0) ? (sb + a * se / (double)eq) / (double)k
                                       : __builtin_nan("");
    out[c] = o;
  }
}

// ------------------------------------------------------------------ the filtered form
//
// For small k the k nearest are a sliver of the n points: a sampled bracket (a, b) of each
// query's distances (the batched kernel's rule over the distances of the sampled points)
// keeps only the distances in (a, b), with their ordinates, and the selection and the
// reductions run over those.  #(d <= a) and the ordinates' sum there come from the same
// pass; a query whose bracket does not hold d_k (or keeps more than kKnnCap) is selected by
// its own workgroup over recomputed distances.  Results equal the materialised form's.

constexpr int kKnnCap = (int)kKnnKeptCap;  // (the select holds them in LDS)

// d = sum_j (P_ij - q_j)^2 for a row and a query both in registers, in the order knn_dist uses
template <int D>
__device__ __forceinline__ float knn_dist_reg(const float (&row)[D > 0 ? D : 16],
                                              const float (&qv)[D > 0 ? D : 16], int dim) {
  const int dd = D > 0 ? D : dim;
  float s = 0.0f;
#pragma unroll
  for (int j = 0; j < (D > 0 ? D : 16); ++j) {
    if (j < dd) {
      const float e = row[j] - qv[j];
      const float sq = e * e;
      s = j == 0 ? sq : s + sq;
    }
  }
  return s;
}

// The distances of the sampled points (runs of kPropRun at sample_stride apart), one query
// per lane, the points as scalar loads; one run per workgroup along x.
template <int D>
__global__ __launch_bounds__(kKnnBlock) void knn_sample_kernel(
    const float *__restrict__ P, const float *__restrict__ Q, int64_t n, int32_t dim, int64_t nq,
    float *__restrict__ Ds) {
  constexpr int DM = D > 0 ? D : 16;
  const int dd = D > 0 ? D : dim;
  const int64_t q = (int64_t)blockIdx.y * kKnnBlock + threadIdx.x;
  const bool live = q < nq;
  float qv[DM];
#pragma unroll
  for (int j = 0; j < DM; ++j) qv[j] = live && j < dd ? Q[q * dd + j] : 0.0f;
  const int S = sample_size(n);
  const int64_t stride = sample_stride(n, S);
  const int run = blockIdx.x;
  for (int r = 0; r < kPropRun; ++r) {
    const int64_t i = (int64_t)run * stride + r;
    float row[DM];
#pragma unroll
    for (int j = 0; j < DM; ++j) row[j] = j < dd ? P[i * dd + j] : 0.0f;
    const float d = knn_dist_reg<D>(row, qv, dim);
    if (live) Ds[q * S + run * kPropRun + r] = d;
  }
}

struct KnnBracketShared {
  uint64_t kext[2];
  int32_t flag;
  SampleLds smp;
  uint64_t wsum[kKnnBlock / kWave];
  uint32_t rh[kHistMaxBins];
};

// One workgroup per query: its sampled bracket to ab[2c], ab[2c+1] ((+inf, -inf) where there
// is none: the filter then keeps nothing but NaN and the select recomputes), and the filter's
// counters of c cleared.
__global__ __launch_bounds__(kKnnBlock) void knn_bracket_kernel(
    const float *__restrict__ Ds, int64_t n, int64_t k, int64_t nq, float *__restrict__ ab,
    uint32_t *__restrict__ cnt, double *__restrict__ fsum) {
  __shared__ KnnBracketShared sh;
  const int64_t c = blockIdx.x;
  if (threadIdx.x < 2) cnt[threadIdx.x * nq + c] = 0u;
  if (threadIdx.x == 2) fsum[c] = 0.0;
  const int S = sample_size(n);
  const CPS_GLOBAL float *src = (const CPS_GLOBAL float *)Ds + c * S;
  auto sample = [&](int i) -> float { return src[i]; };
  float a, b;
  const bool use = sample_bracket_rule<float, kKnnBlock>(sample, S, n, k, sh, a, b);
  if (threadIdx.x == 0) {
    ab[2 * c] = use ? a : __builtin_inff();
    ab[2 * c + 1] = use ? b : -__builtin_inff();
  }
}

// The filter: one query per lane, the points of segment blockIdx.x as scalar loads.  A
// distance with a < d < b (or NaN) is kept with its ordinate at a place reserved on the
// query's cursor (rare for small k), if below kKnnCap; d <= a is counted and its ordinate
// summed (in point order; the segments' sums added atomically).
template <int D>
__global__ __launch_bounds__(kKnnBlock) void knn_filter_kernel(
    const float *__restrict__ P, const float *__restrict__ f, const float *__restrict__ Q,
    const float *__restrict__ ab, int64_t n, int32_t dim, int64_t nq, int64_t seg,
    float *__restrict__ K, uint32_t *__restrict__ cnt, double *__restrict__ fsum) {
  constexpr int DM = D > 0 ? D : 16;
  const int dd = D > 0 ? D : dim;
  const int64_t q = (int64_t)blockIdx.y * kKnnBlock + threadIdx.x;
  const bool live = q < nq;
  float qv[DM];
#pragma unroll
  for (int j = 0; j < DM; ++j) qv[j] = live && j < dd ? Q[q * dd + j] : 0.0f;
  const float lo = live ? ab[2 * q] : __builtin_inff();
  const float hi = live ? ab[2 * q + 1] : -__builtin_inff();
  const int64_t rb = (int64_t)blockIdx.x * seg;
  const int64_t re = rb + seg < n ? rb + seg : n;
  uint32_t below = 0;
  double fb = 0.0;
  for (int64_t i = rb; i < re; ++i) {
    float row[DM];
#pragma unroll
    for (int j = 0; j < DM; ++j) row[j] = j < dd ? P[i * dd + j] : 0.0f;
    const float fi = f[i];
    const float d = knn_dist_reg<D>(row, qv, dim);
    const bool le = d <= lo;
    if (live && !le && !(d >= hi)) {
      const uint32_t at = atomicAdd(&cnt[q], 1u);
      if (at < (uint32_t)kKnnCap) {
        K[2 * (q * kKnnCap + at)] = d;
        K[2 * (q * kKnnCap + at) + 1] = fi;
      }
    }
    if (le) {
      ++below;
      fb += (double)fi;
    }
  }
  if (live && below) {
    atomicAdd(&cnt[nq + q], below);
    atomicAdd(&fsum[q], fb);
  }
}

__device__ inline void knn_write(cps_knn *out, double mean, float dk, int32_t status,
                                 int64_t below, int64_t equal) {
  cps_knn o;
  o.mean = mean;
  o.dk = dk;
  o.status = status;
  o.below = below;
  o.equal = equal;
  *out = o;
}

// One workgroup per query: where the bracket holds d_k (#(d <= a) < k <= #(d <= a) + kept,
// kept <= kKnnCap), the kept distances and ordinates in LDS, d_k by a radix select of rank
// k - #(d <= a) among them, and the sums of the ordinates below and at d_k (fixed order);
// else the same over the query's n distances recomputed (key range, histogram narrowing,
// a last pass for the sums).  The mean as the materialised form's final kernel forms it.
template <int D>
__global__ __launch_bounds__(kKnnBlock) void knn_select_kernel(
    const float *__restrict__ K, const uint32_t *__restrict__ cnt,
    const double *__restrict__ fsum, const float *__restrict__ ab, const float *__restrict__ P,
    const float *__restrict__ f, const float *__restrict__ Q, int64_t n, int32_t dim, int64_t nq,
    int64_t k, cps_knn *__restrict__ out) {
  constexpr int DM = D > 0 ? D : 16;
  __shared__ float kd[kKnnCap];
  __shared__ float kf[kKnnCap];
  __shared__ uint32_t hist[kHistMaxBins];
  __shared__ WgSelShared<kKnnBlock> sh;
  __shared__ double wred[kKnnBlock / kWave];
  __shared__ float sq[16];
  const int64_t c = blockIdx.x;
  const int tid = threadIdx.x;
  const int dd = D > 0 ? D : dim;
  const int64_t len = cnt[c], below = cnt[nq + c];
  const float lo = ab[2 * c], hi = ab[2 * c + 1];
  const bool holds = lo < hi && below < k && k <= below + len && len <= kKnnCap;
  if (tid < dd) sq[tid] = Q[c * dd + tid];
  if (tid == 0) {
    sh.flag = 0u;
    sh.kext[0] = ~0ull;
    sh.kext[1] = 0ull;
  }
  __syncthreads();
  if (holds) {  // (uniform)
    bool nan = false;
    for (int64_t i = tid; i < len; i += kKnnBlock) {
      const float d = K[2 * (c * kKnnCap + i)];
      kd[i] = d;
      kf[i] = K[2 * (c * kKnnCap + i) + 1];
      nan = nan || !(d == d);
    }
    if (nan) atomicOr(&sh.flag, 1u);
    __syncthreads();
    if (sh.flag != 0u) {
      if (tid == 0) knn_write(out + c, __builtin_nan(""), __builtin_nanf(""), CPS_STATUS_NAN, 0, 0);
      return;
    }
    uint32_t key;
    int64_t b_in, eq;
    block_radix_select<float, kKnnBlock>(kd, len, false, 0.0f, 0.0f, k - below, hist, sh.misc,
                                         key, b_in, eq);
    const float dk = Traits<float>::unkey(key);
    double slt = 0.0, seq = 0.0;
    for (int64_t i = tid; i < len; i += kKnnBlock) {
      if (kd[i] < dk) slt += (double)kf[i];
      else if (kd[i] == dk) seq += (double)kf[i];
    }
    slt = block_sum_fixed<kKnnBlock>(slt, wred);
    seq = block_sum_fixed<kKnnBlock>(seq, wred);
    const int64_t less = below + b_in;
    if (tid == 0) {
      const double a = (double)(k - less);
      const double mean = (fsum[c] + slt + a * seq / (double)eq) / (double)k;
      knn_write(out + c, mean, dk, CPS_STATUS_OK, less, eq);
    }
    return;
  }
  // the query's distances, recomputed in point order from its share
  float qv[DM];
#pragma unroll
  for (int j = 0; j < DM; ++j) qv[j] = j < dd ? sq[j] : 0.0f;
  auto pass = [&](auto fn) {
    for (int64_t i = tid; i < n; i += kKnnBlock) {
      float row[DM];
#pragma unroll
      for (int j = 0; j < DM; ++j) row[j] = j < dd ? P[i * dd + j] : 0.0f;
      fn(knn_dist_reg<D>(row, qv, dim));
    }
  };
  uint32_t kmn = ~0u, kmx = 0u;
  bool nan = false;
  pass([&](float d) {
    const uint32_t kk = Traits<float>::key(d);
    nan = nan || !(d == d);
    kmn = kk < kmn ? kk : kmn;
    kmx = kk > kmx ? kk : kmx;
  });
  atomicMin(&sh.kext[0], (unsigned long long)kmn);
  atomicMax(&sh.kext[1], (unsigned long long)kmx);
  if (nan) atomicOr(&sh.flag, 1u);
  __syncthreads();
  if (sh.flag != 0u) {  // (uniform)
    if (tid == 0) knn_write(out + c, __builtin_nan(""), __builtin_nanf(""), CPS_STATUS_NAN, 0, 0);
    return;
  }
  const WgSelOut r = wg_select_pass<float, kKnnBlock>(pass, k, sh.kext[0], sh.kext[1], 0, n, hist,
                                                      kd, kKnnCap, sh);
  const float dk = Traits<float>::unkey((uint32_t)r.key);
  double slt = 0.0, seq = 0.0;
  for (int64_t i = tid; i < n; i += kKnnBlock) {
    float row[DM];
#pragma unroll
    for (int j = 0; j < DM; ++j) row[j] = j < dd ? P[i * dd + j] : 0.0f;
    const float d = knn_dist_reg<D>(row, qv, dim);
    if (d < dk) slt += (double)f[i];
    else if (d == dk) seq += (double)f[i];
  }
  slt = block_sum_fixed<kKnnBlock>(slt, wred);
  seq = block_sum_fixed<kKnnBlock>(seq, wred);
  if (tid == 0) {
    const double a = (double)(k - r.less);
    knn_write(out + c, (slt + a * seq / (double)r.equal) / (double)k, dk, CPS_STATUS_OK, r.less,
              r.equal);
  }
}

void knn_filter_shape(int64_t n, int64_t nq, int cu_count, int64_t *nseg, int64_t *seg) {
  // about 4 x 8 workgroups per CU over (segments x groups of kKnnBlock queries), segments of
  // at least 256 points
  const int64_t groups = (nq + kKnnBlock - 1) / kKnnBlock;
  int64_t ns = (int64_t)cu_count * 32 / groups;
  const int64_t nmax = (n + 255) / 256;
  if (ns > nmax) ns = nmax;
  if (ns > 65535) ns = 65535;
  if (ns < 1) ns = 1;
  const int64_t sl = (n + ns - 1) / ns;
  *nseg = (n + sl - 1) / sl;
  *seg = sl;
}

hipError_t launch_knn_filtered(const float *P, const float *f, const float *Q, int64_t n,
                               int32_t dim, int64_t nq, int64_t k, const KnnFilterBufs &w,
                               cps_knn *out, hipStream_t stream) {
  const int64_t groups = (nq + kKnnBlock - 1) / kKnnBlock;
  const dim3 sg((unsigned)sample_runs(n), (unsigned)groups);
  if (dim == 8)
    knn_sample_kernel<8><<<sg, dim3(kKnnBlock), 0, stream>>>(P, Q, n, dim, nq, w.Ds);
  else
    knn_sample_kernel<0><<<sg, dim3(kKnnBlock), 0, stream>>>(P, Q, n, dim, nq, w.Ds);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  knn_bracket_kernel<<<dim3((unsigned)nq), dim3(kKnnBlock), 0, stream>>>(w.Ds, n, k, nq, w.ab,
                                                                        w.cnt, w.fsum);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const dim3 fg((unsigned)w.nseg, (unsigned)groups);
  if (dim == 8)
    knn_filter_kernel<8><<<fg, dim3(kKnnBlock), 0, stream>>>(P, f, Q, w.ab, n, dim, nq, w.seg, w.K,
                                                              w.cnt, w.fsum);
  else
    knn_filter_kernel<0><<<fg, dim3(kKnnBlock), 0, stream>>>(P, f, Q, w.ab, n, dim, nq, w.seg, w.K,
                                                              w.cnt, w.fsum);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  if (dim == 8)
    knn_select_kernel<8><<<dim3((unsigned)nq), dim3(kKnnBlock), 0, stream>>>(
        w.K, w.cnt, w.fsum, w.ab, P, f, Q, n, dim, nq, k, out);
  else
    knn_select_kernel<0><<<dim3((unsigned)nq), dim3(kKnnBlock), 0, stream>>>(
        w.K, w.cnt, w.fsum, w.ab, P, f, Q, n, dim, nq, k, out);
  return hipGetLastError();
}

hipError_t launch_knn_distances(const float *P, const float *Q, int64_t n, int32_t dim, int64_t nq,
                                int64_t k, float *Dst, const float **ptrs, int64_t *sizes,
                                int64_t *ks, int cu_count, hipStream_t stream) {
  const int64_t groups = (nq + kKnnGroup - 1) / kKnnGroup;
  int64_t bx = (n + kKnnBlock - 1) / kKnnBlock;
  const int64_t want = (int64_t)cu_count * 8 / (groups < 1 ? 1 : groups) + 1;
  if (bx > want) bx = want;
  if (bx < 1) bx = 1;
  const dim3 grid((unsigned)bx, (unsigned)groups);
  if (dim == 8)
    knn_distance_kernel<8><<<grid, dim3(kKnnBlock), 0, stream>>>(P, Q, n, dim, nq, Dst);
  else
    knn_distance_kernel<0><<<grid, dim3(kKnnBlock), 0, stream>>>(P, Q, n, dim, nq, Dst);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  knn_descriptor_kernel<<<dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, stream>>>(
      Dst, n, nq, k, ptrs, sizes, ks);
  return hipGetLastError();
}

hipError_t launch_knn_reduce(const float *P, const float *f, const float *Q, const float *Dst,
                             int64_t n, int32_t dim, int64_t nq, int64_t k, const cps_result *sel,
                             double *pd, int64_t *pi, cps_knn *out, hipStream_t stream) {
  const dim3 grid((unsigned)kKnnRedBlocks, (unsigned)nq);
  const bool vec = n % 4 == 0 && (uintptr_t)f % 16 == 0 && (uintptr_t)Dst % 16 == 0;
  if (kKnnRead && vec)
    knn_partial_read_kernel<true><<<grid, dim3(kKnnBlock), 0, stream>>>(Dst, f, n, sel, pd, pi);
  else if (kKnnRead)
    knn_partial_read_kernel<false><<<grid, dim3(kKnnBlock), 0, stream>>>(Dst, f, n, sel, pd, pi);
  else if (dim == 8)
    knn_partial_kernel<8><<<grid, dim3(kKnnBlock), 0, stream>>>(P, f, Q, n, dim, sel, pd, pi);
  else
    knn_partial_kernel<0><<<grid, dim3(kKnnBlock), 0, stream>>>(P, f, Q, n, dim, sel, pd, pi);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  knn_final_kernel<<<dim3((unsigned)((nq + 255) / 256)), dim3(256), 0, stream>>>(
      nq, k, kKnnRedBlocks, sel, pd, pi, out);
  return hipGetLastError();
}

}  // namespace cps
