// Device-side building blocks shared by the selection kernels: element traits,
// wave64 reductions, agent-scope synchronisation and the one-workgroup radix select.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "cp_state.h"

namespace cps {

constexpr int kWave = 64;

// Global-memory pointers: loads and stores through them compile to global_* instructions
// (with a scalar base where the compiler can prove it) instead of flat_* ones.
#define CPS_GLOBAL __attribute__((address_space(1)))
#define CPS_LDS __attribute__((address_space(3)))

template <typename T> struct Traits;
template <> struct Traits<float> {
  using Vec = float __attribute__((ext_vector_type(4)));  // 16-byte loads
  using Key = uint32_t;
  static constexpr int kVec = 4;
  static constexpr int kDigits = 4;   // 8-bit radix digits in the key
  __device__ static Key key(float v) { return key32(v); }
  __device__ static float unkey(Key k) { return unkey32(k); }
};
template <> struct Traits<double> {
  using Vec = double __attribute__((ext_vector_type(2)));
  using Key = uint64_t;
  static constexpr int kVec = 2;
  static constexpr int kDigits = 8;
  __device__ static Key key(double v) { return key64(v); }
  __device__ static double unkey(Key k) { return unkey64(k); }
};

template <typename T> __device__ inline void vec_to_arr(const typename Traits<T>::Vec &v, T *e) {
#pragma unroll
  for (int j = 0; j < Traits<T>::kVec; ++j) e[j] = v[j];
}

// ------------------------------------------------------------------ wave helpers

__device__ inline uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }
__device__ inline uint32_t popc(uint64_t m) { return (uint32_t)__popcll(m); }
// A pointer every lane of the wavefront holds, moved to scalar registers.
template <typename P> __device__ inline P *uniform_ptr(P *p) {
  const uint64_t v = (uint64_t)p;
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
  return (P *)(((uint64_t)hi << 32) | lo);
}
// number of set bits of m in lanes below this lane
__device__ inline uint32_t lane_rank(uint64_t m) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Wavefront reductions with DPP row moves (no LDS round trips): four row shifts fold each
// 16-lane row into its lane 15, two row broadcasts fold the rows into lane 63, and lane 63
// is read as a scalar.  The order of the operations is fixed, so the results are
// deterministic; every lane receives the result.
template <int CTRL, int ROWS>
__device__ inline double dpp_move(double v, double fill) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint64_t f = __builtin_bit_cast(uint64_t, fill);
  const int lo = __builtin_amdgcn_update_dpp((int)(uint32_t)f, (int)(uint32_t)b, CTRL, ROWS, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(uint32_t)(f >> 32), (int)(uint32_t)(b >> 32), CTRL,
                                             ROWS, 0xF, false);
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

__device__ inline double lane63(double v) {
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, 63);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), 63);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// OP 0: sum, 1: min, 2: max
template <int OP> __device__ inline double dpp_op(double a, double b) {
  return OP == 0 ? a + b : (OP == 1 ? fmin(a, b) : fmax(a, b));
}

template <int OP> __device__ inline double wave_reduce(double v) {
  const double id = OP == 0 ? 0.0 : (OP == 1 ? __builtin_inf() : -__builtin_inf());
  v = dpp_op<OP>(v, dpp_move<0x111, 0xF>(v, id));  // row_shr:1
  v = dpp_op<OP>(v, dpp_move<0x112, 0xF>(v, id));  // row_shr:2
  v = dpp_op<OP>(v, dpp_move<0x114, 0xF>(v, id));  // row_shr:4
  v = dpp_op<OP>(v, dpp_move<0x118, 0xF>(v, id));  // row_shr:8
  v = dpp_op<OP>(v, dpp_move<0x142, 0xA>(v, id));  // row_bcast:15 into rows 1 and 3
  v = dpp_op<OP>(v, dpp_move<0x143, 0xC>(v, id));  // row_bcast:31 into rows 2 and 3
  return lane63(v);
}

__device__ inline double wave_sum(double v) { return wave_reduce<0>(v); }
__device__ inline double wave_min(double v) { return wave_reduce<1>(v); }
__device__ inline double wave_max(double v) { return wave_reduce<2>(v); }
// integer sums through double: exact while the wavefront's total stays below 2^53
__device__ inline int64_t wave_sum_i64(int64_t v) { return (int64_t)wave_reduce<0>((double)v); }

// Exclusive prefix sum over the workgroup in thread order (wsum: one slot per wavefront).
template <int BLOCK>
__device__ inline uint64_t block_exclusive_scan(uint64_t v, uint64_t *wsum) {
  const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
  uint64_t x = v;
#pragma unroll
  for (int o = 1; o < kWave; o <<= 1) {
    const uint64_t y = __shfl_up(x, o);
    if (lane >= o) x += y;
  }
  if (lane == kWave - 1) wsum[wv] = x;
  __syncthreads();
  uint64_t off = 0;
  for (int w = 0; w < wv; ++w) off += wsum[w];
  __syncthreads();
  return off + x - v;
}

// ------------------------------------------------------------------ agent-scope sync
// The eight XCDs have separate L2 caches; agent-scope release/acquire makes the
// compiler write back / invalidate them around the synchronising operation.

__device__ inline uint32_t atomic_add_acq_rel(uint32_t *p, uint32_t v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline uint32_t atomic_add_release(uint32_t *p, uint32_t v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline uint64_t atomic_add_relaxed(uint64_t *p, uint64_t v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline uint32_t load_acquire(const uint32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline uint32_t load_relaxed(const uint32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline uint64_t load_relaxed(const uint64_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void store_release(uint32_t *p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void store_relaxed(uint32_t *p, uint32_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline void fence_acquire() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }
__device__ inline void fence_release() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }

// ------------------------------------------------------------------ radix select
// Exact select of the element of rank r (1-based) among the elements w of W[0..m)
// with lo_ex < w < hi_ex (when `filter`), by most-significant-digit radix select on
// the ordered keys: one histogram of 256 bins per 8-bit digit, kept in LDS.  Run by
// one whole workgroup of BLOCK threads.  Returns the key of the selected element,
// the number of candidates strictly below it and its multiplicity.
template <typename T, int BLOCK>
__device__ __noinline__ void block_radix_select(const T *__restrict__ W, int64_t m, bool filter, T lo_ex,
                                   T hi_ex, int64_t r, uint32_t *hist /* 256 in LDS */,
                                   int64_t *s_misc /* 4 in LDS */,
                                   typename Traits<T>::Key &key_out, int64_t &below_out,
                                   int64_t &equal_out) {
  using Key = typename Traits<T>::Key;
  const int tid = threadIdx.x;
  Key prefix = 0, mask = 0;
  int64_t below = 0, rr = r, eq = 0;
  for (int d = Traits<T>::kDigits - 1; d >= 0; --d) {
    const int shift = 8 * d;
    for (int b = tid; b < 256; b += BLOCK) hist[b] = 0;
    __syncthreads();
    for (int64_t i = tid; i < m; i += BLOCK) {
      const T v = W[i];
      const bool in = !filter || (v > lo_ex && v < hi_ex);
      const Key kk = Traits<T>::key(v);
      if (in && (kk & mask) == prefix) atomicAdd(&hist[(uint32_t)(kk >> shift) & 255u], 1u);
    }
    __syncthreads();
    if (tid < kWave) {
      // lane l owns bins 4l .. 4l+3
      uint32_t c0 = hist[4 * tid], c1 = hist[4 * tid + 1], c2 = hist[4 * tid + 2],
               c3 = hist[4 * tid + 3];
      int64_t own = (int64_t)c0 + c1 + c2 + c3;
      int64_t incl = own;
#pragma unroll
      for (int o = 1; o < kWave; o <<= 1) {
        int64_t up = __shfl_up(incl, o);
        if (tid >= o) incl += up;
      }
      const int64_t excl = incl - own;
      if (excl < rr && rr <= incl) {
        int64_t acc = excl;
        int bin = 4 * tid;
        uint32_t cs[4] = {c0, c1, c2, c3};
        for (int j = 0; j < 4; ++j) {
          if (rr <= acc + cs[j]) { bin = 4 * tid + j; break; }
          acc += cs[j];
        }
        s_misc[0] = bin;
        s_misc[1] = acc;
        s_misc[2] = hist[bin];
      }
    }
    __syncthreads();
    const int bin = (int)s_misc[0];
    const int64_t acc = s_misc[1];
    eq = s_misc[2];
    below += acc;
    rr -= acc;
    prefix |= (Key)bin << shift;
    mask |= (Key)255 << shift;
    __syncthreads();
  }
  key_out = prefix;
  below_out = below;
  equal_out = eq;
}

}  // namespace cps
