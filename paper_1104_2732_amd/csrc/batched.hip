// Batched exact selection: many independent arrays of uneven sizes in one launch.
//
// A persistent grid of workgroups pulls arrays from a device-side queue, largest first
// (every workgroup sorts the sizes in LDS on its own, so no grid-wide wait is needed),
// and runs the whole cutting-plane method of Section 4 on each array by itself: pass 0,
// evaluation passes, splits of the bracket into the workgroup's private buffers once the
// bracket is small, a gather, and the exact radix select.  The state machine is the one
// of the single-array kernel (cp_state.h), kept in LDS; every synchronisation is a
// workgroup barrier, so workgroups never wait on each other and the launch needs no
// co-residency.  The queue and exit counters reset themselves at the end, so the launch
// can be captured in a graph and replayed.
#include "batch_queue.h"
#include "cps_device.h"
#include "cps_kernels.h"
#include "cps_passes.h"
#include "cps_sample.h"

namespace cps {

__device__ __noinline__ void bdev_after_pass0(CpState &s, const Pass0Result &r, const CpConfig &c) {
  cp_after_pass0(s, r, c);
}
__device__ __noinline__ void bdev_after_eval(CpState &s, const EvalResult &r, const CpConfig &c) {
  cp_after_eval(s, r, c);
}
__device__ __noinline__ void bdev_after_gather(CpState &s, int64_t gathered) {
  cp_after_gather(s, gathered);
}
__device__ __noinline__ void bdev_after_final(CpState &s, double v, int64_t below, int64_t eq) {
  cp_after_final(s, v, below, eq);
}
__device__ __noinline__ void bdev_after_hist(CpState &s, int32_t b, int64_t below, int64_t cnt,
                                             const CpConfig &c) {
  cp_after_hist(s, b, below, cnt, c);
}
__device__ __noinline__ void bdev_hist_narrow(CpState &s, const HistGeom<uint64_t> &g, int32_t b,
                                              int64_t below, int64_t cnt, const CpConfig &c) {
  cp_hist_narrow(s, g, b, below, cnt, c);
}

// Key bins per side of a counting evaluation: the two sides share the workgroup's LDS
// histogram, half each.
constexpr int kBatchSideBits = 11;

template <typename T, int BLOCK> struct BShared {
  CpState st;
  double d[8][BLOCK / kWave];
  int64_t i[8][BLOCK / kWave];
  uint32_t hist[256];
  int64_t misc[8];
  int64_t cur[2];
  uint64_t wsum[BLOCK / kWave];  // wavefront totals of a workgroup scan
  int64_t job;
  int64_t items;                  // work items of the launch
  int64_t jslot, jindex;          // the current item's largest-first slot and array index
  int32_t jpart, jparts;          // its part, and the parts of that array
  int32_t flag;                   // workgroup-wide flags (sampled bracket, last arrival)
  uint64_t kext[2];               // sampled keys' minimum and maximum
  SampleLds smp;                  // the sampled bracket's bins
  int64_t kcopy;                  // elements of the sampled bracket's copy (-1: not whole)
  double kpa, kpb;                // the sampled bracket
  double ksuma;                   // sum of the elements at or below the bracket's lower end
  uint64_t order[kBatchSortMax];  // (size << 12 | index) sorted by size, largest first; then
                                  // item_entry(first work item, index) per slot
  uint32_t rh[kHistMaxBins];      // key histogram of a histogram pass
  // The state machine's arguments, built by thread 0 in LDS: as private variables whose
  // address a call takes they would sit in scratch memory, and the compiler may write them
  // there from every lane.
  CpConfig cfg;        // the launch's configuration
  CpConfig cfg_arg;    // a per-call variant of it (the sampled bracket, the sides' bins)
  Pass0Result p0r;
  EvalResult evr;
  HistGeom<uint64_t> hg;
  HistGeom<uint64_t> pg[2];  // the two sides' bins of a counting evaluation
};

// The passes load with the nontemporal hint, as the single-array kernel's (each line is read
// once per pass; the LMS call's 8 GB of residuals went 7.7 -> 7.3 ms).

// Split (or gather) one tile's elements into this workgroup's buffer: the low side grows
// up from out[0], the high side down from out[cap-1].  GATHER: every valid element inside
// (lo_ex, hi_ex) goes low.  Each wavefront reserves its place on either side with one LDS
// atomic on the workgroup's cursors, so no workgroup barrier is needed; the order of the
// elements in the buffer follows the wavefronts' arrival, which nothing downstream depends
// on (the histograms, the gather and the final select are order-free; sums over a part only
// position later trial points).
template <typename T, int BLOCK, int U, bool FILTER, bool GATHER>
__device__ inline void block_split_tile(const T (&e)[U][Traits<T>::kVec], const bool (&valid)[U],
                                        int nslot, T t, T lo_ex, T hi_ex, CPS_GLOBAL T *out,
                                        int64_t cap, BShared<T, BLOCK> &sh) {
  constexpr int V = Traits<T>::kVec;
  const int tid = threadIdx.x, lane = tid % kWave;
  auto low = [&](T v, bool ok) -> bool {
    if (GATHER) return ok && (!FILTER || (v > lo_ex && v < hi_ex));
    return ok && v < t && (!FILTER || v > lo_ex);
  };
  auto high = [&](T v, bool ok) -> bool {
    if (GATHER) return false;
    return ok && v > t && (!FILTER || v < hi_ex);
  };
  uint32_t wl = 0, wr = 0;
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int j = 0; j < V; ++j) {
      if (u * V + j >= nslot) continue;
      wl += popc(ballot(low(e[u][j], valid[u])));
      wr += popc(ballot(high(e[u][j], valid[u])));
    }
  if (wl == 0 && wr == 0) return;  // wave-uniform
  uint64_t ol = 0, orr = 0;
  if (lane == 0) {
    if (wl) ol = atomicAdd(reinterpret_cast<unsigned long long *>(&sh.cur[0]), (unsigned long long)wl);
    if (wr) orr = atomicAdd(reinterpret_cast<unsigned long long *>(&sh.cur[1]), (unsigned long long)wr);
  }
  ol = __shfl(ol, 0);
  orr = __shfl(orr, 0);
#pragma unroll
  for (int u = 0; u < U; ++u)
#pragma unroll
    for (int j = 0; j < V; ++j) {
      if (u * V + j >= nslot) continue;
      const bool l = low(e[u][j], valid[u]);
      const uint64_t ml = ballot(l);
      if (l) out[ol + lane_rank(ml)] = e[u][j];
      ol += popc(ml);
      if (!GATHER) {
        const bool r = high(e[u][j], valid[u]);
        const uint64_t mr = ballot(r);
        if (r) out[cap - 1 - (int64_t)(orr + lane_rank(mr))] = e[u][j];
        orr += popc(mr);
      }
    }
}

// One evaluation pass of this workgroup over span sp, optionally splitting into `out`.
template <typename T, int BLOCK, int U, bool CLAMP, bool SPLIT, bool FILTER, bool GATHER>
__device__ void block_pass(const Span<T> &sp, T t, T yL, T yR, T fmin, T fmax,
                           CPS_GLOBAL T *out, int64_t cap, BShared<T, BLOCK> &sh,
                           EvalAcc<T> &acc) {
  constexpr int V = Traits<T>::kVec;
  using Vec = typename Traits<T>::Vec;
  const int tid = threadIdx.x, lane = tid % kWave;
  for (int64_t base = 0; base < sp.nvec; base += (int64_t)BLOCK * U) {
    Vec raw[U];
    bool valid[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t vi = base + (int64_t)u * BLOCK + tid;
      valid[u] = vi < sp.nvec;
      if (valid[u]) raw[u] = __builtin_nontemporal_load(&sp.V[vi]);
    }
    T e[U][V];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      vec_to_arr<T>(raw[u], e[u]);
      if (!GATHER) {
        T a_part = 0, b_part = 0;
#pragma unroll
        for (int j = 0; j < V; ++j) eval_one<T, CLAMP>(e[u][j], valid[u], t, fmin, fmax, a_part, b_part, acc);
        acc.A += (double)a_part;
        acc.B += (double)b_part;
      }
    }
    if (SPLIT || GATHER)
      block_split_tile<T, BLOCK, U, FILTER, GATHER>(e, valid, U * V, t, yL, yR, out, cap, sh);
  }
  if (sp.nedge > 0) {
    // the unaligned head and tail, one element per lane of the first wavefront
    const bool have = tid < sp.nedge;
    T v = have ? sp.W[edge_index(sp, tid)] : T(0);
    if (!GATHER) {
      T a_part = 0, b_part = 0;
      eval_one<T, CLAMP>(v, have, t, fmin, fmax, a_part, b_part, acc);
      acc.A += (double)a_part;
      acc.B += (double)b_part;
    }
    if (SPLIT || GATHER) {
      T e[U][V];
      bool valid[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        valid[u] = false;
#pragma unroll
        for (int j = 0; j < V; ++j) e[u][j] = v;
      }
      valid[0] = have;
      block_split_tile<T, BLOCK, U, FILTER, GATHER>(e, valid, 1, t, yL, yR, out, cap, sh);
    }
  }
  (void)lane;
}

// Histogram pass of this workgroup over span sp: elements whose ordered key lies in
// [klo, khi] are counted in LDS bin (key - klo) >> shift.
template <typename T, int BLOCK, int U>
__device__ void block_hist(const Span<T> &sp, typename Traits<T>::Key klo,
                           typename Traits<T>::Key khi, int shift, uint32_t *rh) {
  constexpr int V = Traits<T>::kVec;
  using Vec = typename Traits<T>::Vec;
  using Key = typename Traits<T>::Key;
  const int tid = threadIdx.x;
  for (int64_t base = 0; base < sp.nvec; base += (int64_t)BLOCK * U) {
    Vec raw[U];
    bool valid[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t vi = base + (int64_t)u * BLOCK + tid;
      valid[u] = vi < sp.nvec;
      if (valid[u]) raw[u] = __builtin_nontemporal_load(&sp.V[vi]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      T e[V];
      vec_to_arr<T>(raw[u], e);
#pragma unroll
      for (int j = 0; j < V; ++j) {
        const Key K = Traits<T>::key(e[j]);
        const Key d = K - klo;  // in range: klo <= K <= khi
        if (valid[u] & (d <= (Key)(khi - klo))) atomicAdd(&rh[(uint32_t)(d >> shift)], 1u);
      }
    }
  }
  if (sp.nedge > 0 && tid < sp.nedge) {
    const Key K = Traits<T>::key(sp.W[edge_index(sp, tid)]);
    if (K >= klo && K <= khi) atomicAdd(&rh[(uint32_t)((K - klo) >> shift)], 1u);
  }
}

// Counting evaluation of this workgroup over the input: the counts below and above t, and
// the bracket's elements on either side in the key bins of that side (LDS counters
// rh[0..) for the low side, rh[kHistMaxBins / 2..) for the high side).  Nothing is written.
template <typename T> struct SideBins {
  typename Traits<T>::Key klo[2];
  typename Traits<T>::Key span[2];  // khi - klo
  bool has[2];                      // the side's key range is not empty
  int shift[2];
};

// On the element's ordered key alone: the low side's elements are those with keys in
// [key(lo), key(t-)], the high side's those in [key(t+), key(hi)] (the bracket's elements
// below and above t exactly); the counts below and above t follow from the bins' totals.
template <typename T>
__device__ inline void count_side(T v, bool valid, const SideBins<T> &sb, uint32_t *rh) {
  using Key = typename Traits<T>::Key;
  const Key K = Traits<T>::key(v);
  const Key d0 = K - sb.klo[0], d1 = K - sb.klo[1];
  const bool l = valid & sb.has[0] & (d0 <= sb.span[0]);
  const bool h = valid & sb.has[1] & (d1 <= sb.span[1]);
  if (l | h) {
    const uint32_t bin = l ? (uint32_t)(d0 >> sb.shift[0])
                           : (uint32_t)(d1 >> sb.shift[1]) + (uint32_t)(kHistMaxBins / 2);
    atomicAdd(&rh[bin], 1u);
  }
}

template <typename T, int BLOCK, int U>
__device__ void block_count(const Span<T> &sp, const SideBins<T> &sb, uint32_t *rh) {
  constexpr int V = Traits<T>::kVec;
  using Vec = typename Traits<T>::Vec;
  const int tid = threadIdx.x;
  for (int64_t base = 0; base < sp.nvec; base += (int64_t)BLOCK * U) {
    Vec raw[U];
    bool valid[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t vi = base + (int64_t)u * BLOCK + tid;
      valid[u] = vi < sp.nvec;
      if (valid[u]) raw[u] = __builtin_nontemporal_load(&sp.V[vi]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      T e[V];
      vec_to_arr<T>(raw[u], e);
#pragma unroll
      for (int j = 0; j < V; ++j) count_side<T>(e[j], valid[u], sb, rh);
    }
  }
  if (sp.nedge > 0 && tid < sp.nedge) count_side<T>(sp.W[edge_index(sp, tid)], true, sb, rh);
}

// The bin holding rank r of `nbins` LDS counters: an exclusive scan in a fixed order.
// Leaves the bin in misc[0] (-1 when none holds it), the count below it in misc[1] and its
// own count in misc[2]; ends with a workgroup barrier.
template <typename T, int BLOCK>
__device__ void block_pick(const uint32_t *bins, int nbins, uint64_t r, BShared<T, BLOCK> &sh) {
  const int tid = threadIdx.x;
  constexpr int BPT = kHistMaxBins / BLOCK;
  uint64_t hv[BPT];
  uint64_t tot = 0;
#pragma unroll
  for (int j = 0; j < BPT; ++j) {
    const int b = tid * BPT + j;
    hv[j] = b < nbins ? bins[b] : 0u;
    tot += hv[j];
  }
  if (tid == 0) sh.misc[0] = -1;
  uint64_t cum = block_exclusive_scan<BLOCK>(tot, sh.wsum);
#pragma unroll
  for (int j = 0; j < BPT; ++j) {
    if (cum < r && r <= cum + hv[j]) {
      sh.misc[0] = tid * BPT + j;
      sh.misc[1] = (int64_t)cum;
      sh.misc[2] = (int64_t)hv[j];
    }
    cum += hv[j];
  }
  __syncthreads();
}

template <typename T, int BLOCK, int U, bool CLASSIFY>
__device__ void block_pass0(const Span<T> &sp, P0Acc<T> &acc) {
  constexpr int V = Traits<T>::kVec;
  using Vec = typename Traits<T>::Vec;
  const int tid = threadIdx.x;
  const T ba = 0, bb = 0;
  for (int64_t base = 0; base < sp.nvec; base += (int64_t)BLOCK * U) {
    Vec raw[U];
    bool valid[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t vi = base + (int64_t)u * BLOCK + tid;
      valid[u] = vi < sp.nvec;
      if (valid[u]) raw[u] = __builtin_nontemporal_load(&sp.V[vi]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      T e[V];
      vec_to_arr<T>(raw[u], e);
      T aa = 0, bA = 0, ab = 0, bB = 0;
      if (!CLASSIFY) {
        // the running extremes change only where an element reaches the wavefront's (as in
        // the single-array pass 0)
        p0_extremes_wave<T, V>(e, valid[u], acc);
#pragma unroll
        for (int j = 0; j < V; ++j)
          pass0_one<T, false, false, true>(e[j], valid[u], ba, bb, aa, bA, ab, bB, acc);
      } else {
#pragma unroll
        for (int j = 0; j < V; ++j)
          pass0_one<T, true, false>(e[j], valid[u], ba, bb, aa, bA, ab, bB, acc);
      }
    }
  }
  if (sp.nedge > 0) {
    const bool have = tid < sp.nedge;
    const T v = have ? sp.W[edge_index(sp, tid)] : T(0);
    T aa = 0, bA = 0, ab = 0, bB = 0;
    pass0_one<T, CLASSIFY, false>(v, have, ba, bb, aa, bA, ab, bB, acc);
  }
}

// ------------------------------------------------------------------ sampled bracket

// The sampled bracket of one array (used by arrays of at least kBatchPropMin elements):
// sample_size(n) elements in runs of kPropRun neighbours at evenly spaced places (so the
// sample touches few lines); the rule is sample_bracket_rule's.  Pass 0's counts decide
// whether each end holds.  Every workgroup of an array computes the same bracket.
template <typename T, int BLOCK>
__device__ __noinline__ bool sample_bracket(const T *x, int64_t n, int64_t k, BShared<T, BLOCK> &sh, T &pa,
                               T &pb) {
  const int S = sample_size(n);
  const int64_t stride = sample_stride(n, S);
  auto sample = [&](int i) -> T { return x[(int64_t)(i / kPropRun) * stride + i % kPropRun]; };
  return sample_bracket_rule<T, BLOCK>(sample, S, n, k, sh, pa, pb);
}

// Pass 0 of an array with a sampled bracket (a, b), over one part of it: the extremes and
// their multiplicities, #(x <= a) and #(a < x < b) (on the ordered keys, which order the
// values as the compares do), the interior's keys in the bins `ib` (LDS), and every 16-byte
// vector of x that holds an interior element copied whole to `out` (one coalesced store per
// vector slot, at places reserved with one atomic per wavefront and tile on `cursor`: the
// workgroup's LDS cursor, or the team's device cursor when TEAM, counted in vectors), at most
// `cap` elements; `ovf` is set when some did not fit.  The copy is a superset of the
// interior: its other elements lie at or below a or at or above b, outside the bracket that
// pass 0 leaves, and the later passes skip them.  The sum of x is not formed: it only places
// cutting-plane trial points, and a bracket that holds at either end is finished by key
// histograms (one that holds at neither end falls back to trial points inside the bracket,
// bisection at worst, with the same exact result).  NaN is counted; NaN or an infinity (an
// infinite extreme) makes the state machine repeat pass 0 with the classification.
template <typename T> struct PropBins {
  typename Traits<T>::Key ka, kb;   // keys of a and b
  typename Traits<T>::Key klo;      // first key of the interior (a's successor)
  typename Traits<T>::Key span;     // last key - klo
  int shift;
};

// Reserve `tot` vectors on the cursor for the wavefront (lane 0's atomic, broadcast).
template <bool TEAM>
__device__ inline int64_t prop_reserve(uint32_t tot, unsigned long long *cursor) {
  unsigned long long base = 0;
  if (threadIdx.x % kWave == 0) {
    if (TEAM)
      base = __hip_atomic_fetch_add(cursor, (unsigned long long)tot, __ATOMIC_RELAXED,
                                    __HIP_MEMORY_SCOPE_AGENT);
    else
      base = atomicAdd(cursor, (unsigned long long)tot);
  }
  return (int64_t)__shfl(base, 0);
}

template <typename T, int BLOCK, int U, bool TEAM, bool SUMA>
__device__ void block_pass0_prop(const Span<T> &sp, T pa, const PropBins<T> &ib, uint32_t *rh,
                                 P0Acc<T> &acc, CPS_GLOBAL T *out, int64_t cap,
                                 unsigned long long *cursor, uint32_t &ovf) {
  constexpr int V = Traits<T>::kVec;
  using Vec = typename Traits<T>::Vec;
  using Key = typename Traits<T>::Key;
  const int tid = threadIdx.x;
  CPS_GLOBAL Vec *outv = (CPS_GLOBAL Vec *)out;
  const int64_t capv = cap / V;
  auto one = [&](T v, bool valid) -> bool {
    acc.nnan += (valid & (v != v)) ? 1u : 0u;
    const Key K = Traits<T>::key(v);
    const bool le = valid & (K <= ib.ka);
    acc.cle_a += le ? 1u : 0u;
    if (SUMA) acc.Aa += le ? (double)v : 0.0;  // the sum of the elements at or below a
    const Key d = K - ib.klo;
    const bool in = valid & (d <= ib.span);
    acc.clt_b += in ? 1u : 0u;  // (here: the interior's count)
    if (in) atomicAdd(&rh[(uint32_t)(d >> ib.shift)], 1u);
    return in;
  };
  for (int64_t base = 0; base < sp.nvec; base += (int64_t)BLOCK * U) {
    Vec raw[U];
    bool valid[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t vi = base + (int64_t)u * BLOCK + tid;
      valid[u] = vi < sp.nvec;
      if (valid[u]) raw[u] = __builtin_nontemporal_load(&sp.V[vi]);
    }
    bool hit[U];
    uint64_t mv[U];
    uint32_t tot = 0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      T w[V];
      vec_to_arr<T>(raw[u], w);
      p0_extremes_wave<T, V>(w, valid[u], acc);
      hit[u] = false;
#pragma unroll
      for (int j = 0; j < V; ++j) hit[u] |= one(w[j], valid[u]);
      mv[u] = ballot(hit[u]);
      tot += popc(mv[u]);
    }
    if (tot != 0) {  // (wave-uniform)
      int64_t off = prop_reserve<TEAM>(tot, cursor);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int64_t at = off + lane_rank(mv[u]);
        if (hit[u]) {
          if (at < capv) outv[at] = raw[u];
          else ovf = 1u;
        }
        off += popc(mv[u]);
      }
    }
  }
  if (sp.nedge > 0) {
    // the unaligned head and tail, one element per lane of the first wavefront; an interior
    // one is copied as a vector padded with a (which lies outside the bracket)
    const bool have = tid < sp.nedge;
    const T v = have ? sp.W[edge_index(sp, tid)] : T(0);
    p0_extremes<T>(v, have, acc);
    const bool in = one(v, have);
    if (tid < kWave) {
      const uint64_t m = ballot(in);
      if (m != 0) {
        const int64_t off = prop_reserve<TEAM>(popc(m), cursor);
        if (in) {
          T w[V];
          w[0] = v;
#pragma unroll
          for (int j = 1; j < V; ++j) w[j] = pa;
          Vec vv;
#pragma unroll
          for (int j = 0; j < V; ++j) vv[j] = w[j];
          const int64_t at = off + lane_rank(m);
          if (at < capv) outv[at] = vv;
          else ovf = 1u;
        }
      }
    }
  }
}

template <typename T> __device__ inline void write_batch_result(cps_result *out, const CpState &s) {
  cps_result r;
  const T v = (T)s.value + T(0);
  uint64_t bits;
  if (sizeof(T) == 4) bits = (uint64_t)__builtin_bit_cast(uint32_t, (float)v);
  else bits = __builtin_bit_cast(uint64_t, (double)v);
  r.value_bits = bits;
  r.value = (double)v;
  r.less = s.less;
  r.equal = s.equal;
  r.greater = s.n - s.less - s.equal;
  r.passes = s.passes;
  r.status = s.status;
  if (s.status != ST_OK) r.less = r.equal = r.greater = 0;
  *out = r;
}

// Pass 0 of one array (or of its part `part` of `parts`) from the sampled bracket (pa, pb),
// then the state after it.  A split array's parts leave their partials in the team record;
// the last to arrive folds them in part order (deterministic) and returns true, the others
// false (they are done with the array).  With one part the workgroup goes on at once.
template <typename T, int BLOCK, int U>
__device__ __noinline__ bool prop_pass0(const T *x, int64_t n, int64_t k, T pa, T pb, int part, int parts,
                           TeamCtl *tc, CPS_GLOBAL T *ibuf, int64_t icap,
                           bool suma, BShared<T, BLOCK> &sh) {
  using Key = typename Traits<T>::Key;
  const int tid = threadIdx.x;
  const int32_t dt = sh.cfg.dtype;
  const HistGeom<uint64_t> g0 =
      hist_geometry(next_up((double)pa, dt), next_down((double)pb, dt), dt, sh.cfg.hist_bits);
  PropBins<T> ib;
  ib.ka = Traits<T>::key(pa);
  ib.kb = Traits<T>::key(pb);
  ib.klo = (Key)g0.klo;
  ib.span = (Key)(g0.khi - g0.klo);
  ib.shift = g0.shift;
  for (int b = tid; b < g0.nbins; b += BLOCK) sh.rh[b] = 0u;
  if (tid == 0) sh.cur[0] = 0;
  __syncthreads();
  // this part: [lo, lo + len), parts of n / parts elements and the remainder spread first
  const int64_t q = n / parts, rem = n % parts;
  const int64_t lo = q * part + (part < rem ? part : rem);
  const int64_t len = q + (part < rem ? 1 : 0);
  const Span<T> sp = make_span(x + lo, len);
  P0Acc<T> acc;
  acc.sum = 0;
  acc.mn = t_inf<T>();
  acc.mx = -t_inf<T>();
  acc.wmn = t_inf<T>();
  acc.wmx = -t_inf<T>();
  acc.cmn = acc.cmx = 0;
  acc.nnan = acc.nneg = acc.npos = acc.cle_a = acc.clt_b = 0;
  acc.Aa = acc.Ba = acc.Ab = acc.Bb = 0;
  uint32_t ovf = 0;
  unsigned long long *lcur = reinterpret_cast<unsigned long long *>(&sh.cur[0]);
  if (parts > 1) {
    if (suma) block_pass0_prop<T, BLOCK, U, true, true>(sp, pa, ib, sh.rh, acc, ibuf, icap, &tc->cursor, ovf);
    else block_pass0_prop<T, BLOCK, U, true, false>(sp, pa, ib, sh.rh, acc, ibuf, icap, &tc->cursor, ovf);
  } else {
    if (suma) block_pass0_prop<T, BLOCK, U, false, true>(sp, pa, ib, sh.rh, acc, ibuf, icap, lcur, ovf);
    else block_pass0_prop<T, BLOCK, U, false, false>(sp, pa, ib, sh.rh, acc, ibuf, icap, lcur, ovf);
  }
  double mn = (double)acc.mn, mx = (double)acc.mx;
  int64_t cmn = acc.cmn, cmx = acc.cmx;
    double dv[8] = {acc.Aa, 0, 0, 0, 0, 0, 0, 0};
  int64_t iv[8] = {(int64_t)acc.cle_a, (int64_t)acc.nnan, (int64_t)ovf, (int64_t)acc.clt_b, 0, 0,
                   0, 0};
  int dop[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  block_reduce_pair<BLOCK, 1, 4>(dv, dop, iv, mn, cmn, mx, cmx, sh.d, sh.i);
  int64_t written = 0;
  if (parts > 1) {
    // leave the partial, add the bins, arrive; the last part folds
    for (int b = tid; b < g0.nbins; b += BLOCK) {
      const uint32_t c = sh.rh[b];
      if (c) __hip_atomic_fetch_add(&tc->hist[b], c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (tid == 0) {
      tc->pd[part][0] = mn;
      tc->pd[part][1] = mx;
      tc->pd[part][2] = dv[0];
      tc->pi[part][0] = cmn;
      tc->pi[part][1] = cmx;
      tc->pi[part][2] = iv[0];
      tc->pi[part][3] = iv[1];
      tc->pi[part][4] = iv[3];
      if (iv[2]) __hip_atomic_fetch_or(&tc->overflow, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    // the workgroup barrier completes every wavefront's stores to this XCD's L2; thread 0's
    // release then writes them back for the other XCDs, and the last part's acquire makes
    // them visible to its whole workgroup (one L2 write-back and invalidation per part)
    __syncthreads();
    if (tid == 0) sh.flag = atomic_add_acq_rel(&tc->arrive, 1u) == (uint32_t)parts - 1 ? 1 : 0;
    __syncthreads();
    if (!sh.flag) return false;
    // the last part: the bins of every part, then the team record back to zero
    for (int b = tid; b < g0.nbins; b += BLOCK) {
      sh.rh[b] = __hip_atomic_load(&tc->hist[b], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      tc->hist[b] = 0u;
    }
    if (tid == 0) {
      double fmn = __builtin_inf(), fmx = -__builtin_inf(), sa = 0.0;
      int64_t c0 = 0, c1 = 0, le = 0, nan = 0, inner = 0;
      for (int p = 0; p < parts; ++p) {
        sa += tc->pd[p][2];
        const double m0 = tc->pd[p][0], m1 = tc->pd[p][1];
        if (m0 < fmn) { fmn = m0; c0 = tc->pi[p][0]; } else if (m0 == fmn) c0 += tc->pi[p][0];
        if (m1 > fmx) { fmx = m1; c1 = tc->pi[p][1]; } else if (m1 == fmx) c1 += tc->pi[p][1];
        le += tc->pi[p][2];
        nan += tc->pi[p][3];
        inner += tc->pi[p][4];
      }
      mn = fmn; cmn = c0; mx = fmx; cmx = c1;
      dv[0] = sa;
      iv[0] = le;
      iv[1] = nan;
      iv[3] = inner;
      iv[2] = __hip_atomic_load(&tc->overflow, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      written = (int64_t)__hip_atomic_load(&tc->cursor, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) *
                Traits<T>::kVec;
      __hip_atomic_store(&tc->cursor, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&tc->overflow, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&tc->arrive, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  } else if (tid == 0) {
    written = sh.cur[0] * Traits<T>::kVec;
  }
  if (tid == 0) {
    Pass0Result &r = sh.p0r;
    r = Pass0Result{};
    r.classified = 0;
    r.sums = 0;  // only the counts at the ends were formed: an adopted bracket ends by histograms
    r.sum = iv[1] > 0 ? __builtin_nan("") : 0.0;  // (NaN: repeat with the classification)
    r.fmin = mn;
    r.fmax = mx;
    r.cmin = cmn;
    r.cmax = cmx;
    r.c_le_a = iv[0];
    r.c_lt_b = iv[0] + iv[3];  // the interior's keys lie between those of a and b
    r.split_overflow = iv[2] != 0 ? 1 : 0;
    r.split_written = written;  // whole vectors: a superset of the interior
    // for the sum of the k smallest: the copy holds every element of (a, b), and the sum of
    // those at or below a
    sh.kcopy = (iv[2] == 0 && iv[1] == 0) ? written : -1;
    sh.ksuma = dv[0];
    CpState &st = sh.st;
    st = CpState{};
    st.n = n;
    st.k = k;
    st.phase = PH_PASS0;
    CpConfig &c = sh.cfg_arg;
    c = sh.cfg;
    c.use_bracket = 1;
    c.bracket_lo = (double)pa;
    c.bracket_hi = (double)pb;
    c.p0_split = 1;
    bdev_after_pass0(st, r, c);
  }
  __syncthreads();
  // both ends proven and the interior's bins are those of the bracket: narrow at once
  const CpState &s1 = sh.st;
  if (s1.phase == PH_HIST && s1.bracket_used == 3 && s1.wbuf == 0) {
    const HistGeom<uint64_t> g = hist_geometry(s1.lo, s1.hi, dt, sh.cfg.hist_bits);
    if (g.klo == g0.klo && g.khi == g0.khi && g.shift == g0.shift) {
      block_pick<T, BLOCK>(sh.rh, g.nbins, (uint64_t)(s1.k - s1.cL), sh);
      if (tid == 0) {
        const int32_t bsel = (int32_t)sh.misc[0];
        sh.hg = g;
        bdev_hist_narrow(sh.st, sh.hg, bsel, bsel < 0 ? 0 : sh.misc[1],
                         bsel < 0 ? 0 : sh.misc[2], sh.cfg);
      }
      __syncthreads();
    }
  }
  return true;
}

// The sum of the elements w of span sp with lo_ex < w < hi_ex (w < hi_ex alone without LO),
// in double precision (a fixed order for a fixed span); valid in thread 0.
template <typename T, int BLOCK, int U, bool LO>
__device__ double block_sum_range(const Span<T> &sp, T lo_ex, T hi_ex, BShared<T, BLOCK> &sh) {
  constexpr int V = Traits<T>::kVec;
  using Vec = typename Traits<T>::Vec;
  const int tid = threadIdx.x;
  double acc = 0.0;
  for (int64_t base = 0; base < sp.nvec; base += (int64_t)BLOCK * U) {
    Vec raw[U];
    bool valid[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t vi = base + (int64_t)u * BLOCK + tid;
      valid[u] = vi < sp.nvec;
      if (valid[u]) raw[u] = __builtin_nontemporal_load(&sp.V[vi]);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      T w[V];
      vec_to_arr<T>(raw[u], w);
#pragma unroll
      for (int j = 0; j < V; ++j)
        acc += (valid[u] & (!LO | (w[j] > lo_ex)) & (w[j] < hi_ex)) ? (double)w[j] : 0.0;
    }
  }
  if (sp.nedge > 0 && tid < sp.nedge) {
    const T w = sp.W[edge_index(sp, tid)];
    acc += ((!LO || w > lo_ex) && w < hi_ex) ? (double)w : 0.0;
  }
  double dv[8] = {acc, 0, 0, 0, 0, 0, 0, 0};
  int dop[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  int64_t iv[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  block_reduce<BLOCK, 1, 0>(dv, dop, iv, false, sh.d, sh.i);
  return dv[0];
}

// The whole method on one array (part `part` of `parts` of it; slot: its largest-first slot,
// which names its team record), by this workgroup.  With ksum (not null), also the sum of
// the array's k smallest elements.
template <typename T, int BLOCK, int U>
__device__ void select_one(const T *x, int64_t n, int64_t k, cps_result *out, double *ksum,
                           const BatchArgs<T> &a, BShared<T, BLOCK> &sh, int64_t slot, int part,
                           int parts) {
  const int tid = threadIdx.x;
  constexpr int SU = U / 2 > 0 ? U / 2 : 1;
  const int64_t cap = a.cap;
  // the two split buffers, as two scalars: a private array indexed by the state's buffer
  // number would live in scratch memory, written by every lane on every pass
  CPS_GLOBAL T *zb0 = (CPS_GLOBAL T *)(a.zbuf + (int64_t)blockIdx.x * a.ws_stride);
  CPS_GLOBAL T *const zb1 = (CPS_GLOBAL T *)(a.zbuf + (int64_t)blockIdx.x * a.ws_stride + cap);
  CPS_GLOBAL T *gb = (CPS_GLOBAL T *)(a.zbuf + (int64_t)blockIdx.x * a.ws_stride + a.gb_off);
  if (!batch_array_valid((uint64_t)(uintptr_t)x, n, k, (uint32_t)sizeof(T))) {
    if (tid == 0 && part == 0) {
      cps_result r = {};
      r.status = ST_BADARG;
      *out = r;
      if (ksum) *ksum = __builtin_nan("");
    }
    return;
  }
  if (tid == 0) sh.kcopy = -1;
  bool slow = false, p0_done = false;
  if (a.proposal && a.cfg.hist_bits > 0 && n >= kBatchPropMin) {
    T pa, pb;
    const bool prop = sample_bracket<T, BLOCK>(x, n, k, sh, pa, pb);
    if (!prop && part > 0) return;  // no bracket: the first part runs the array alone
    if (prop) {
      TeamCtl *tc = parts > 1 ? a.teams + slot : nullptr;
      CPS_GLOBAL T *ibuf = parts > 1 ? (CPS_GLOBAL T *)(a.tbuf + slot * a.team_cap) : zb0;
      if (!prop_pass0<T, BLOCK, U>(x, n, k, pa, pb, part, parts, tc, ibuf, parts > 1 ? a.team_cap : cap,
                                   a.ksum != nullptr, sh))
        return;
      zb0 = ibuf;  // the interior's elements are the working set from here on
      if (tid == 0) {
        sh.kpa = (double)pa;
        sh.kpb = (double)pb;
      }
      if (sh.st.phase == PH_PASS0 && sh.st.p0_slow) slow = true;  // NaN or an infinity
      else p0_done = true;
      __syncthreads();
      if (slow && tid == 0) sh.kcopy = -1;
    }
  } else if (part > 0) {
    return;  // (parts are formed only for arrays that take the sampled bracket)
  }
  const Span<T> sx = make_span(x, n);
  while (!p0_done) {  // pass 0 (repeated once with infinity classification if needed)
    P0Acc<T> acc;
    acc.sum = 0;
    acc.mn = t_inf<T>();
    acc.mx = -t_inf<T>();
    acc.wmn = t_inf<T>();
    acc.wmx = -t_inf<T>();
    acc.cmn = acc.cmx = 0;
    acc.nnan = acc.nneg = acc.npos = acc.cle_a = acc.clt_b = 0;
    acc.Aa = acc.Ba = acc.Ab = acc.Bb = 0;
    if (slow) block_pass0<T, BLOCK, SU, true>(sx, acc);
    else block_pass0<T, BLOCK, U, false>(sx, acc);
    double mn = (double)acc.mn, mx = (double)acc.mx;
    int64_t cmn = acc.cmn, cmx = acc.cmx;
        double dv[8] = {acc.sum, 0, 0, 0, 0, 0, 0, 0};
    int64_t iv[8] = {(int64_t)acc.nnan, (int64_t)acc.nneg, (int64_t)acc.npos, 0, 0, 0, 0, 0};
    int dop[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    block_reduce_pair<BLOCK, 1, 3>(dv, dop, iv, mn, cmn, mx, cmx, sh.d, sh.i);
    if (tid == 0) {
      Pass0Result &r = sh.p0r;
      r = Pass0Result{};
      r.classified = slow ? 1 : 0;
      r.sums = 1;
      r.sum = dv[0];
      r.nnan = iv[0];
      r.nneg = iv[1];
      r.npos = iv[2];
      r.fmin = mn;
      r.fmax = mx;
      r.cmin = cmn;
      r.cmax = cmx;
      CpState &s = sh.st;
      if (!slow) {
        s = CpState{};
        s.n = n;
        s.k = k;
      }
      s.phase = PH_PASS0;
      bdev_after_pass0(s, r, sh.cfg);
    }
    __syncthreads();
    if (sh.st.phase == PH_PASS0 && sh.st.p0_slow && !slow) {
      slow = true;
      continue;
    }
    break;
  }
  while (sh.st.phase == PH_EVAL || sh.st.phase == PH_GATHER || sh.st.phase == PH_HIST) {
    const CpState &s = sh.st;
    const T t = (T)s.t, yL = (T)s.yL, yR = (T)s.yR, fmn = (T)s.fmin, fmx = (T)s.fmax;
    const T *W;
    if (s.wbuf < 0) W = x;
    else if (s.wbuf == 2) W = (const T *)gb;
    else W = (const T *)(s.wbuf == 0 ? zb0 : zb1) + (s.side == 0 ? 0 : cap - s.wlen);
    const Span<T> sp = make_span(W, s.wbuf < 0 ? n : s.wlen);
    if (s.phase == PH_HIST) {
      // key histogram of the compacted bracket in LDS, then the bin holding rank k - cL
      const HistGeom<uint64_t> g = hist_geometry(s.lo, s.hi, a.cfg.dtype, a.cfg.hist_bits);
      for (int b = tid; b < g.nbins; b += BLOCK) sh.rh[b] = 0u;
      __syncthreads();
      block_hist<T, BLOCK, U>(sp, (typename Traits<T>::Key)g.klo, (typename Traits<T>::Key)g.khi,
                              g.shift, sh.rh);
      __syncthreads();
      block_pick<T, BLOCK>(sh.rh, g.nbins, (uint64_t)(s.k - s.cL), sh);
      if (tid == 0) {
        const int32_t bsel = (int32_t)sh.misc[0];
        bdev_after_hist(sh.st, bsel, bsel < 0 ? 0 : sh.misc[1], bsel < 0 ? 0 : sh.misc[2], sh.cfg);
      }
      __syncthreads();
      continue;
    }
    EvalAcc<T> acc;
    acc.A = acc.B = 0;
    acc.pred = -t_inf<T>();
    acc.succ = t_inf<T>();
    acc.L = acc.G = 0;
    if (s.counted) {
      // count both sides of t in key bins (half of the LDS histogram each), then narrow the
      // bracket to the bin of the rank on the side that holds it
      CpConfig cs = a.cfg;
      cs.hist_bits = a.cfg.hist_bits > kBatchSideBits ? kBatchSideBits : a.cfg.hist_bits;
      const HistGeom<uint64_t> pg0 = split_part_geometry(s, 0, cs);
      const HistGeom<uint64_t> pg1 = split_part_geometry(s, 1, cs);
      SideBins<T> sb;
      sb.klo[0] = (typename Traits<T>::Key)pg0.klo;
      sb.has[0] = pg0.nbins > 0;
      sb.span[0] = pg0.nbins > 0 ? (typename Traits<T>::Key)(pg0.khi - pg0.klo) : 0;
      sb.shift[0] = pg0.shift;
      sb.klo[1] = (typename Traits<T>::Key)pg1.klo;
      sb.has[1] = pg1.nbins > 0;
      sb.span[1] = pg1.nbins > 0 ? (typename Traits<T>::Key)(pg1.khi - pg1.klo) : 0;
      sb.shift[1] = pg1.shift;
      if (tid == 0) {  // for the narrowing after the count (kept in LDS, not in registers)
        sh.pg[0] = pg0;
        sh.pg[1] = pg1;
      }
      for (int b = tid; b < kHistMaxBins; b += BLOCK) sh.rh[b] = 0u;
      __syncthreads();
      block_count<T, BLOCK, U>(sp, sb, sh.rh);
      __syncthreads();
      // each side's total: L = #(x <= yL) + the low side, G = #(x >= yR) + the high side
      double dv[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      int dop[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      int64_t iv[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      for (int b = tid; b < kHistMaxBins / 2; b += BLOCK) {
        iv[0] += sh.rh[b];
        iv[1] += sh.rh[kHistMaxBins / 2 + b];
      }
      block_reduce<BLOCK, 0, 2>(dv, dop, iv, false, sh.d, sh.i);
      if (tid == 0) {
        EvalResult &r = sh.evr;
        r.A = r.B = 0.0;
        r.pred = -__builtin_inf();
        r.succ = __builtin_inf();
        r.L = sh.st.cL + iv[0];
        r.G = (sh.st.n - sh.st.cR) + iv[1];
        r.written = 0;
        bdev_after_eval(sh.st, r, sh.cfg);
      }
      __syncthreads();
      if (sh.st.phase == PH_HIST) {
        const int p = sh.st.side;
        block_pick<T, BLOCK>(sh.rh + p * (kHistMaxBins / 2), sh.pg[p].nbins,
                             (uint64_t)(sh.st.k - sh.st.cL), sh);
        if (tid == 0) {
          const int32_t bsel = (int32_t)sh.misc[0];
          bdev_hist_narrow(sh.st, sh.pg[p], bsel, bsel < 0 ? 0 : sh.misc[1],
                           bsel < 0 ? 0 : sh.misc[2], sh.cfg);
        }
        __syncthreads();
      }
      continue;
    }
    if (tid == 0) sh.cur[0] = sh.cur[1] = 0;
    __syncthreads();
    const bool gather = s.phase == PH_GATHER;
    const bool clamp = s.has_inf && s.wbuf < 0;
    if (gather) {
      if (s.filter) block_pass<T, BLOCK, SU, false, false, true, true>(sp, t, yL, yR, fmn, fmx, gb, cap, sh, acc);
      else block_pass<T, BLOCK, SU, false, false, false, true>(sp, t, yL, yR, fmn, fmx, gb, cap, sh, acc);
    } else if (!s.split) {
      if (clamp) block_pass<T, BLOCK, SU, true, false, false, false>(sp, t, yL, yR, fmn, fmx, nullptr, cap, sh, acc);
      else block_pass<T, BLOCK, U, false, false, false, false>(sp, t, yL, yR, fmn, fmx, nullptr, cap, sh, acc);
    } else if (s.filter) {
      block_pass<T, BLOCK, SU, false, true, true, false>(sp, t, yL, yR, fmn, fmx, s.zout == 0 ? zb0 : zb1, cap, sh, acc);
    } else {
      block_pass<T, BLOCK, SU, false, true, false, false>(sp, t, yL, yR, fmn, fmx, s.zout == 0 ? zb0 : zb1, cap, sh, acc);
    }
    double dv[8] = {acc.A, acc.B, (double)acc.pred, (double)acc.succ, 0, 0, 0, 0};
    int dop[8] = {0, 0, 2, 1, 0, 0, 0, 0};
    int64_t iv[8] = {(int64_t)acc.L, (int64_t)acc.G, 0, 0, 0, 0, 0, 0};
    block_reduce<BLOCK, 4, 2>(dv, dop, iv, false, sh.d, sh.i);
    if (tid == 0) {
      CpState &w = sh.st;
      if (gather) {
        bdev_after_gather(w, sh.cur[0]);
      } else {
        EvalResult &r = sh.evr;
        r.A = dv[0]; r.B = dv[1]; r.pred = dv[2]; r.succ = dv[3];
        r.L = iv[0]; r.G = iv[1];
        r.written = sh.cur[0] + sh.cur[1];
        bdev_after_eval(w, r, sh.cfg);
      }
    }
    __syncthreads();
  }
  if (sh.st.phase == PH_FINAL) {
    const CpState &s = sh.st;
    const T *W = s.wbuf < 0 ? x : (const T *)gb;
    typename Traits<T>::Key key;
    int64_t below, eq;
    block_radix_select<T, BLOCK>(W, s.wlen, !s.on_bracket, (T)s.yL, (T)s.yR, s.k - s.cL,
                                 sh.hist, sh.misc, key, below, eq);
    if (tid == 0) bdev_after_final(sh.st, (double)Traits<T>::unkey(key), below, eq);
    __syncthreads();
  }
  if (ksum) {
    // the sum of the k smallest elements: those below x_(k), plus k - #(x < x_(k)) copies of
    // it; the elements below come from the sampled bracket's copy and pass 0's sum at or
    // below its lower end when x_(k) lies inside the bracket, else from a pass over x
    __syncthreads();
    const CpState &s = sh.st;
    if (s.status == ST_OK) {
      const T v = (T)s.value;
      const T pa = (T)sh.kpa, pb = (T)sh.kpb;
      double below;
      if (sh.kcopy >= 0 && pa < v && v < pb)
        below = sh.ksuma +
                block_sum_range<T, BLOCK, U, true>(make_span((const T *)zb0, sh.kcopy), pa, v, sh);
      else
        below = block_sum_range<T, BLOCK, U, false>(make_span(x, n), v, v, sh);
      if (tid == 0) *ksum = below + (double)(s.k - s.less) * (double)v;
    } else if (tid == 0) {
      *ksum = __builtin_nan("");
    }
  }
  if (tid == 0) write_batch_result<T>(out, sh.st);
  __syncthreads();
}

template <typename T, int BLOCK, int U>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_num_vgpr(128)))
void batched_select_kernel(BatchArgs<T> a) {
  __shared__ BShared<T, BLOCK> sh;
  const int tid = threadIdx.x;
  const int64_t count = a.count;
  if (tid == 0) sh.cfg = a.cfg;  // (read after the barriers below)
  // Largest first: every workgroup sorts (size, index) in LDS by itself.
  const bool sorted = count <= kBatchSortMax;
  if (sorted) {
    int64_t m = 1;
    while (m < count) m <<= 1;
    for (int64_t j = tid; j < m; j += BLOCK) sh.order[j] = j < count ? lpt_key(a.sizes[j], j) : 0;
    __syncthreads();
    // bitonic sort, descending
    for (int64_t kk = 2; kk <= m; kk <<= 1) {
      for (int64_t jj = kk >> 1; jj > 0; jj >>= 1) {
        for (int64_t i = tid; i < m; i += BLOCK) bitonic_exchange(sh.order, i, jj, kk);
        __syncthreads();
      }
    }
  }
  if (sorted) {
    // the work items: each slot's array in team_blocks parts (the largest arrays, in the
    // slots that have a team record), one part otherwise; slot j becomes
    // item_entry(its first item, its array's index)
    constexpr int PER = kBatchSortMax / BLOCK;
    const int64_t j0 = (int64_t)tid * PER;
    int64_t mine = 0;
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int64_t j = j0 + p;
      if (j < count)
        mine += j < a.team_records ? team_blocks((int64_t)(sh.order[j] >> 12), a.team_chunk, a.team_max)
                                   : 1;
    }
    int64_t first = (int64_t)block_exclusive_scan<BLOCK>((uint64_t)mine, sh.wsum);
    if (tid == BLOCK - 1) sh.items = first + mine;
#pragma unroll
    for (int p = 0; p < PER; ++p) {
      const int64_t j = j0 + p;
      if (j < count) {
        const uint64_t key = sh.order[j];
        sh.order[j] = item_entry(first, lpt_index(key));
        first += j < a.team_records ? team_blocks((int64_t)(key >> 12), a.team_chunk, a.team_max) : 1;
      }
    }
    __syncthreads();
  } else if (tid == 0) {
    sh.items = count;
  }
  for (;;) {
    if (tid == 0) {
      const int64_t q = (int64_t)atomic_add_relaxed(&a.ctl->queue, 1ull);
      sh.job = q;
      if (q < sh.items) {
        if (sorted) {
          const int64_t j = item_slot(sh.order, count, q);
          const int64_t f = item_first(sh.order[j]);
          const int64_t nf = j + 1 < count ? item_first(sh.order[j + 1]) : sh.items;
          sh.jslot = j;
          sh.jindex = item_index(sh.order[j]);
          sh.jpart = (int32_t)(q - f);
          sh.jparts = (int32_t)(nf - f);
        } else {
          sh.jslot = q;
          sh.jindex = q;
          sh.jpart = 0;
          sh.jparts = 1;
        }
      }
    }
    __syncthreads();
    const int64_t q = sh.job, items = sh.items;
    const int64_t j = sh.jslot, i = sh.jindex;
    const int part = sh.jpart, parts = sh.jparts;
    __syncthreads();
    if (q >= items) break;
    select_one<T, BLOCK, U>(a.ptrs[i], a.sizes[i], a.ks[i], a.out + i, a.ksum ? a.ksum + i : nullptr,
                            a, sh, j, part, parts);
  }
  // the last workgroup out resets the queue for the next launch (graph replays included)
  if (tid == 0) {
    const uint64_t e = atomic_add_relaxed(&a.ctl->exits, 1ull);
    if (e == (uint64_t)gridDim.x - 1) {
      __hip_atomic_store(&a.ctl->queue, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __hip_atomic_store(&a.ctl->exits, 0ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
  }
}

template <typename T>
hipError_t launch_batched(const BatchArgs<T> &a, int grid, int block, hipStream_t stream) {
  if (block == 256)
    batched_select_kernel<T, 256, kSelectUnroll><<<dim3(grid), dim3(256), 0, stream>>>(a);
  else if (block == 512)
    batched_select_kernel<T, 512, kSelectUnroll><<<dim3(grid), dim3(512), 0, stream>>>(a);
  else
    batched_select_kernel<T, 1024, kSelectUnroll><<<dim3(grid), dim3(1024), 0, stream>>>(a);
  return hipGetLastError();
}

template <typename T> int batched_max_blocks_per_cu(int block) {
  int nb = 0;
  hipError_t e;
  if (block == 256)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batched_select_kernel<T, 256, kSelectUnroll>, 256, 0);
  else if (block == 512)
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batched_select_kernel<T, 512, kSelectUnroll>, 512, 0);
  else
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, batched_select_kernel<T, 1024, kSelectUnroll>, 1024, 0);
  return e == hipSuccess ? nb : 0;
}

template hipError_t launch_batched<float>(const BatchArgs<float> &, int, int, hipStream_t);
template hipError_t launch_batched<double>(const BatchArgs<double> &, int, int, hipStream_t);
template int batched_max_blocks_per_cu<float>(int);
template int batched_max_blocks_per_cu<double>(int);

}  // namespace cps
