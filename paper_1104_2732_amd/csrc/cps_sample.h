// The sampled bracket: a likely interval for the k-th smallest of n values, from S of them.
//
// Used by the batched kernel (its arrays' pass 0 classifies against it) and by the least-
// median-of-squares filter (which keeps only the residuals inside it).  The counts taken
// over the whole array decide whether the bracket holds, so no result depends on it.
#pragma once

#include "cps_device.h"
#include "cps_kernels.h"
#include "cps_passes.h"

namespace cps {

constexpr int kPropSample = 4096;       // sample elements of arrays below kPropBigN
constexpr int kPropSampleBig = 16384;   // ... and from kPropBigN on (a quarter as wide a bracket)
constexpr int64_t kPropBigN = (int64_t)1 << 18;
constexpr int kPropRun = 16;
constexpr int64_t kBatchPropMin = (int64_t)1 << 15;

template <typename T> __device__ constexpr int32_t c_dtype() { return sizeof(T) == 4 ? 0 : 1; }

// Sample size for n values (n >= kBatchPropMin), and the distance between the starts of
// consecutive runs of kPropRun sampled neighbours: the runs lie inside the n values and do
// not overlap.
__device__ __forceinline__ int sample_size(int64_t n) {
  return n >= kPropBigN ? kPropSampleBig : kPropSample;
}
__device__ __forceinline__ int64_t sample_stride(int64_t n, int S) { return n / (S / kPropRun); }
// (the host's count of the runs)
inline int sample_runs(int64_t n) {
  return (n >= kPropBigN ? kPropSampleBig : kPropSample) / kPropRun;
}

// The rule's own LDS words (set by single threads between barriers).
struct SampleLds {
  int64_t b0, b1;          // the bins (then sub-bins) holding the two sample ranks
  int64_t below0, in0;     // samples below the lower rank's bin, and in it
  int64_t below1, in1;     // the same for the upper rank's bin
};

// The bracket rule over S sampled values, sample(i) for i in [0, S) (each read two or three
// times), with the workgroup's LDS in `sh` (members kext[2], flag, smp, rh[kHistMaxBins] and
// wsum, as the scan needs).  The sample is counted in 2^12 key bins over its own range; the
// bracket runs from just below the bin that holds sample rank floor(q - d) to just above the
// bin that holds rank ceil(q + d), where q = S (k - 1/2) / n is the rank's place among the S
// sampled values and d = 4 sqrt(S p (1 - p)) + 2, p = (k - 1/2) / n (four binomial standard
// deviations).  Where those bins hold more than 1.25 times the sampled values between the
// two ranks (a sample whose key range is wide, as one holding an exact zero among values
// near 1, or whose ranks fall in crowded bins), each end's bin is split again into 2^11
// sub-bins and the bracket runs from the sub-bins that hold the ranks.  An end whose rank falls outside the sample is open (-inf or
// +inf).  False (no bracket) when the sample holds NaN or an infinity, only one value, or
// both ends would be open.  Every workgroup that calls it on the same sample computes the
// same bracket.
template <typename T, int BLOCK, typename Sh, typename F>
__device__ __forceinline__ bool sample_bracket_rule(F sample, int S, int64_t n, int64_t k, Sh &sh,
                                                    T &pa, T &pb) {
  using Key = typename Traits<T>::Key;
  const int tid = threadIdx.x;
  if (tid == 0) {
    sh.kext[0] = ~0ull;
    sh.kext[1] = 0ull;
    sh.flag = 0;
    sh.smp.b0 = sh.smp.b1 = 0;
  }
  __syncthreads();
  Key kmn = (Key)~(Key)0, kmx = 0;
  bool bad = false;
#pragma unroll 8
  for (int i = tid; i < S; i += BLOCK) {  // the sample's key range (the keys are read again below)
    const T v = sample(i);
    bad = bad || !(v == v) || v == t_inf<T>() || v == -t_inf<T>();
    const Key kv = Traits<T>::key(v);
    kmn = kv < kmn ? kv : kmn;
    kmx = kv > kmx ? kv : kmx;
  }
  atomicMin(reinterpret_cast<unsigned long long *>(&sh.kext[0]), (unsigned long long)kmn);
  atomicMax(reinterpret_cast<unsigned long long *>(&sh.kext[1]), (unsigned long long)kmx);
  if (bad) atomicOr(&sh.flag, 1);
  __syncthreads();
  const uint64_t klo = sh.kext[0], khi = sh.kext[1];
  if (sh.flag != 0 || klo >= khi) return false;  // (uniform)
  int shift = 0;
  while (((khi - klo) >> shift) >= (uint64_t)kHistMaxBins) ++shift;
  const int nbins = (int)((khi - klo) >> shift) + 1;
  for (int b = tid; b < nbins; b += BLOCK) sh.rh[b] = 0u;
  __syncthreads();
#pragma unroll 8
  for (int i = tid; i < S; i += BLOCK)
    atomicAdd(&sh.rh[(uint32_t)(((uint64_t)Traits<T>::key(sample(i)) - klo) >> shift)], 1u);
  __syncthreads();
  const double Sd = (double)S;
  const double p = ((double)k - 0.5) / (double)n;
  const double q = Sd * p, d = 4.0 * __builtin_sqrt(Sd * p * (1.0 - p)) + 2.0;
  const double r0 = __builtin_floor(q - d), r1 = __builtin_ceil(q + d);
  const bool open0 = r0 < 1.0, open1 = r1 > Sd;
  if (open0 && open1) return false;
  const uint64_t rank0 = open0 ? 1 : (uint64_t)r0, rank1 = open1 ? (uint64_t)S : (uint64_t)r1;
  // the bins holding the two sample ranks: an exclusive scan of the bins in a fixed order
  constexpr int BPT = kHistMaxBins / BLOCK;
  uint64_t hv[BPT];
  uint64_t tot = 0;
#pragma unroll
  for (int j = 0; j < BPT; ++j) {
    const int b = tid * BPT + j;
    hv[j] = b < nbins ? sh.rh[b] : 0u;
    tot += hv[j];
  }
  uint64_t cum = block_exclusive_scan<BLOCK>(tot, sh.wsum);
#pragma unroll
  for (int j = 0; j < BPT; ++j) {
    if (cum < rank0 && rank0 <= cum + hv[j]) {
      sh.smp.b0 = tid * BPT + j;
      sh.smp.below0 = (int64_t)cum;
      sh.smp.in0 = (int64_t)hv[j];
    }
    if (cum < rank1 && rank1 <= cum + hv[j]) {
      sh.smp.b1 = tid * BPT + j;
      sh.smp.below1 = (int64_t)cum;
      sh.smp.in1 = (int64_t)hv[j];
    }
    cum += hv[j];
  }
  __syncthreads();
  const uint64_t b0 = (uint64_t)sh.smp.b0, b1 = (uint64_t)sh.smp.b1;
  const uint64_t below0 = (uint64_t)sh.smp.below0, in0 = (uint64_t)sh.smp.in0;
  const uint64_t below1 = (uint64_t)sh.smp.below1, in1 = (uint64_t)sh.smp.in1;
  __syncthreads();
  // the first key of the lower end's bin and the last key of the upper end's
  uint64_t first0 = klo + (b0 << shift);
  uint64_t last1 = klo + ((b1 + 1) << shift) - 1;
  const uint64_t want = rank1 - rank0 + 1;
  if (shift > 0 && below1 + in1 - below0 > want + want / 4) {  // (uniform)
    // each end's bin in sub-bins: the lower end's in rh[0, 2048), the upper end's after it
    constexpr int kHalf = kHistMaxBins / 2;
    const int sub = shift > 11 ? shift - 11 : 0;
    for (int b = tid; b < kHistMaxBins; b += BLOCK) sh.rh[b] = 0u;
    __syncthreads();
    for (int i = tid; i < S; i += BLOCK) {
      const uint64_t dk = (uint64_t)Traits<T>::key(sample(i)) - klo;
      const uint64_t bin = dk >> shift;
      if (!open0 && bin == b0) atomicAdd(&sh.rh[(uint32_t)((dk - (b0 << shift)) >> sub)], 1u);
      if (!open1 && bin == b1)
        atomicAdd(&sh.rh[kHalf + (uint32_t)((dk - (b1 << shift)) >> sub)], 1u);
    }
    __syncthreads();
    // the ranks' places in the scan of both halves (the upper half follows the lower bin's
    // count, or nothing when the lower end is open)
    const uint64_t t0 = rank0 - below0;
    const uint64_t t1 = (open0 ? 0 : in0) + (rank1 - below1);
    uint64_t hv2[BPT];
    uint64_t tot2 = 0;
#pragma unroll
    for (int j = 0; j < BPT; ++j) {
      hv2[j] = sh.rh[tid * BPT + j];
      tot2 += hv2[j];
    }
    uint64_t cum2 = block_exclusive_scan<BLOCK>(tot2, sh.wsum);
#pragma unroll
    for (int j = 0; j < BPT; ++j) {
      const int e = tid * BPT + j;
      if (e < kHalf && cum2 < t0 && t0 <= cum2 + hv2[j]) sh.smp.b0 = e;
      if (e >= kHalf && cum2 < t1 && t1 <= cum2 + hv2[j]) sh.smp.b1 = e - kHalf;
      cum2 += hv2[j];
    }
    __syncthreads();
    if (!open0) first0 += (uint64_t)sh.smp.b0 << sub;
    if (!open1) last1 = klo + (b1 << shift) + (((uint64_t)sh.smp.b1 + 1) << sub) - 1;
    __syncthreads();
  }
  if (last1 > khi || last1 < klo) last1 = khi;
  // the largest value below the lower end's (sub-)bin, the smallest above the upper one's
  // (keys of finite values, so both neighbours are keys of values: +-inf at worst)
  pa = open0 ? -t_inf<T>() : Traits<T>::unkey((Key)(first0 - 1));
  pb = open1 ? t_inf<T>() : Traits<T>::unkey((Key)(last1 + 1));
  // the interior (a, b) holds at least one value of T (its key bins are not empty)
  return pa < pb && next_up((double)pa, c_dtype<T>()) <= next_down((double)pb, c_dtype<T>());
}

}  // namespace cps
