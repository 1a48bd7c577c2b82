// Least median of squares (Section 6): the lower median of the squared residuals of many
// candidate parameter vectors, via the batched selection.
//
// The residual kernel forms r_i = (y_i - sum_j X_ij b_j)^2 for a group of candidates per
// thread row: each X row and y_i are read once per group, the sum runs left to right in
// j with every product and sum rounded on its own (the library is built without fused
// multiply-add), and the squares land candidate-major in the workspace, one array of n
// per candidate.  A second tiny kernel writes the batched call's descriptors on the device,
// and the batched kernel then selects rank floor((n+1)/2) of every candidate's array.
#include "cps_device.h"
#include "cps_kernels.h"

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

template <int P>
__global__ __launch_bounds__(kLmsBlock) void lms_residual_kernel(
    const double *__restrict__ X, const double *__restrict__ y, const double *__restrict__ betas,
    int64_t n, int32_t p, int64_t m, double *__restrict__ R) {
  __shared__ double sb[kLmsGroup * 16];
  const int64_t c0 = (int64_t)blockIdx.y * kLmsGroup;
  const int nc = (int)((m - c0) < kLmsGroup ? (m - c0) : kLmsGroup);
  for (int q = threadIdx.x; q < nc * p; q += kLmsBlock) sb[q] = betas[c0 * p + q];
  __syncthreads();
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
template <int P, int R>
__global__ __launch_bounds__(kLmsBlock) void lms_residual_rows_kernel(
    const double *__restrict__ X, const double *__restrict__ y, const double *__restrict__ betas,
    int64_t n, int64_t m, double *__restrict__ R_out) {
  static_assert(R % 2 == 0 && (P * R) % 2 == 0, "16-byte groups");
  __shared__ double sb[kLmsGroup * P];
  const int64_t c0 = (int64_t)blockIdx.y * kLmsGroup;
  const int nc = (int)((m - c0) < kLmsGroup ? (m - c0) : kLmsGroup);
  for (int q = threadIdx.x; q < nc * P; q += kLmsBlock) sb[q] = betas[c0 * P + q];
  __syncthreads();
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
    lms_residual_rows_kernel<8, kLmsRows><<<g2, dim3(kLmsBlock), 0, stream>>>(X, y, betas, n, m, R);
  } else if (p == 8) {
    lms_residual_kernel<8><<<grid, dim3(kLmsBlock), 0, stream>>>(X, y, betas, n, p, m, R);
  } else {
    lms_residual_kernel<0><<<grid, dim3(kLmsBlock), 0, stream>>>(X, y, betas, n, p, m, R);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  lms_descriptor_kernel<<<dim3((unsigned)((m + 255) / 256)), dim3(256), 0, stream>>>(R, n, m, rank,
                                                                                    ptrs, sizes, ks);
  return hipGetLastError();
}

}  // namespace cps
