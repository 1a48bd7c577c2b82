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
