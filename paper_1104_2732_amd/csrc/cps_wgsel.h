// One workgroup's exact select of the k-th smallest among values it can pass over any
// number of times (an array in memory, or values it recomputes), by key histograms.
#pragma once

#include "cps_device.h"
#include "cps_kernels.h"

namespace cps {

template <int BLOCK>
struct WgSelShared {
  unsigned long long kext[2];  // key minimum and maximum
  uint32_t flag;               // NaN seen
  uint32_t cursor;             // LDS copy cursor
  int64_t misc[4];             // block_radix_select's words
  int64_t bin, cum, inb;       // a histogram pass's bin, count below it, its own count
  uint64_t wsum[BLOCK / kWave];
};

struct WgSelOut {
  uint64_t key;  // the selected value's key (zero-extended for float)
  int64_t less, equal;
  int32_t passes;
};

// f(W[i]) for every i < len of this workgroup's share (i = thread + j * BLOCK), eight loads
// issued before the eight calls (a single workgroup's pass is otherwise bound by the latency
// of one load after another).
template <int BLOCK, typename T, typename F>
__device__ __forceinline__ void for_each8(const CPS_GLOBAL T *W, int64_t len, F f) {
  constexpr int U = 8;
  for (int64_t i0 = threadIdx.x; i0 < len; i0 += U * BLOCK) {
    T v[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t i = i0 + (int64_t)u * BLOCK;
      v[u] = i < len ? W[i] : T(0);
    }
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (i0 + (int64_t)u * BLOCK < len) f(v[u]);
  }
}

// The k-th smallest (1-based) of the values pass(f) hands to f (each thread its share; no NaN
// among them), given that below0 of them have keys below klo and inrange0 have keys in
// [klo, khi] (and k lies among those): key histograms of 2^12 bins narrow the key range to the
// bin that holds rank k (counting the values below it), until the range holds one key (every
// value in it equals the result) or at most `cap` values, which are copied to LDS (`buf`)
// and radix-selected there.  `hist` is kHistMaxBins words of LDS.
template <typename T, int BLOCK, typename Pass>
__device__ __forceinline__ WgSelOut wg_select_pass(Pass pass, int64_t k, uint64_t klo,
                                                   uint64_t khi, int64_t below0, int64_t inrange0,
                                                   uint32_t *hist, T *buf, int cap,
                                                   WgSelShared<BLOCK> &sh) {
  using Key = typename Traits<T>::Key;
  const int tid = threadIdx.x;
  int64_t below = below0, rr = k - below0, inrange = inrange0;
  int32_t passes = 0;
  for (;;) {
    if (klo == khi) return {klo, below, inrange, passes};  // (uniform)
    if (inrange <= cap) {
      if (tid == 0) sh.cursor = 0u;
      __syncthreads();
      pass([&](T v) {
        const uint64_t kk = (uint64_t)Traits<T>::key(v);
        if (kk >= klo && kk <= khi) buf[atomicAdd(&sh.cursor, 1u)] = v;
      });
      __syncthreads();
      Key key;
      int64_t b_in, eq;
      block_radix_select<T, BLOCK>(buf, inrange, false, T(0), T(0), rr, hist, sh.misc, key, b_in,
                                   eq);
      return {(uint64_t)key, below + b_in, eq, passes + 1};
    }
    int shift = 0;
    while (((khi - klo) >> shift) >= (uint64_t)kHistMaxBins) ++shift;
    for (int b = tid; b < kHistMaxBins; b += BLOCK) hist[b] = 0u;
    __syncthreads();
    pass([&](T v) {
      const uint64_t kk = (uint64_t)Traits<T>::key(v);
      if (kk >= klo && kk <= khi) atomicAdd(&hist[(uint32_t)((kk - klo) >> shift)], 1u);
    });
    __syncthreads();
    ++passes;
    constexpr int BPT = kHistMaxBins / BLOCK;
    uint64_t hv[BPT];
    uint64_t tot = 0;
#pragma unroll
    for (int j = 0; j < BPT; ++j) {
      hv[j] = hist[tid * BPT + j];
      tot += hv[j];
    }
    uint64_t cum = block_exclusive_scan<BLOCK>(tot, sh.wsum);
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
    below += sh.cum;
    rr -= sh.cum;
    inrange = sh.inb;
    __syncthreads();
    const uint64_t nlo = klo + (b << shift);
    uint64_t nhi = nlo + ((1ull << shift) - 1);
    if (nhi > khi || nhi < nlo) nhi = khi;
    klo = nlo;
    khi = nhi;
  }
}

// Sum over the workgroup in a fixed order (each wavefront's lanes by row moves, then the
// wavefronts in order); `wred` holds one double per wavefront.  Every thread gets the sum.
template <int BLOCK>
__device__ inline double block_sum_fixed(double v, double *wred) {
  const double w = wave_sum(v);
  if (threadIdx.x % kWave == 0) wred[threadIdx.x / kWave] = w;
  __syncthreads();
  double t = 0.0;
#pragma unroll
  for (int i = 0; i < BLOCK / kWave; ++i) t += wred[i];
  __syncthreads();
  return t;
}

}  // namespace cps
