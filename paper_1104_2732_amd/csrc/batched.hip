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
  uint64_t order[kBatchSortMax];  // (size << 12 | index), sorted by size, largest first
  uint32_t rh[kHistMaxBins];      // key histogram of a histogram pass
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
        // the running extremes change only where a lane's element reaches them (as in the
        // single-array pass 0: the wavefront tests first, NaN compares false in both)
        bool near = false;
#pragma unroll
        for (int j = 0; j < V; ++j) near |= valid[u] & ((e[j] <= acc.mn) | (e[j] >= acc.mx));
        if (ballot(near) != 0) {
#pragma unroll
          for (int j = 0; j < V; ++j) p0_extremes<T>(e[j], valid[u], acc);
        }
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

// The whole method on one array, by this workgroup.
template <typename T, int BLOCK, int U>
__device__ void select_one(const T *x, int64_t n, int64_t k, cps_result *out,
                           const BatchArgs<T> &a, BShared<T, BLOCK> &sh) {
  const int tid = threadIdx.x;
  constexpr int SU = U / 2 > 0 ? U / 2 : 1;
  const int64_t cap = a.cap;
  CPS_GLOBAL T *zb[2] = {(CPS_GLOBAL T *)(a.zbuf + (int64_t)blockIdx.x * a.ws_stride),
                         (CPS_GLOBAL T *)(a.zbuf + (int64_t)blockIdx.x * a.ws_stride + cap)};
  CPS_GLOBAL T *gb = (CPS_GLOBAL T *)(a.zbuf + (int64_t)blockIdx.x * a.ws_stride + 2 * cap);
  if (!batch_array_valid((uint64_t)(uintptr_t)x, n, k, (uint32_t)sizeof(T))) {
    if (tid == 0) {
      cps_result r = {};
      r.status = ST_BADARG;
      *out = r;
    }
    return;
  }
  const Span<T> sx = make_span(x, n);
  bool slow = false;
  for (;;) {  // pass 0 (repeated once with infinity classification if needed)
    P0Acc<T> acc;
    acc.sum = 0;
    acc.mn = t_inf<T>();
    acc.mx = -t_inf<T>();
    acc.cmn = acc.cmx = 0;
    acc.nnan = acc.nneg = acc.npos = acc.cle_a = acc.clt_b = 0;
    acc.Aa = acc.Ba = acc.Ab = acc.Bb = 0;
    if (slow) block_pass0<T, BLOCK, SU, true>(sx, acc);
    else block_pass0<T, BLOCK, U, false>(sx, acc);
    double mn = (double)acc.mn, mx = (double)acc.mx;
    int64_t cmn = acc.cmn, cmx = acc.cmx;
    block_pair_fold<BLOCK>(mn, cmn, mx, cmx, sh.d, sh.i);
    double dv[8] = {acc.sum, 0, 0, 0, 0, 0, 0, 0};
    int64_t iv[8] = {(int64_t)acc.nnan, (int64_t)acc.nneg, (int64_t)acc.npos, 0, 0, 0, 0, 0};
    int dop[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    block_reduce<BLOCK, 1, 3>(dv, dop, iv, false, sh.d, sh.i);
    if (tid == 0) {
      Pass0Result r = {};
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
      bdev_after_pass0(s, r, a.cfg);
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
    else W = (const T *)zb[s.wbuf] + (s.side == 0 ? 0 : cap - s.wlen);
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
        bdev_after_hist(sh.st, bsel, bsel < 0 ? 0 : sh.misc[1], bsel < 0 ? 0 : sh.misc[2], a.cfg);
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
      HistGeom<uint64_t> pg[2];
      SideBins<T> sb;
      for (int p = 0; p < 2; ++p) {
        pg[p] = split_part_geometry(s, p, cs);
        sb.klo[p] = (typename Traits<T>::Key)pg[p].klo;
        sb.has[p] = pg[p].nbins > 0;
        sb.span[p] = pg[p].nbins > 0 ? (typename Traits<T>::Key)(pg[p].khi - pg[p].klo) : 0;
        sb.shift[p] = pg[p].shift;
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
        EvalResult r;
        r.A = r.B = 0.0;
        r.pred = -__builtin_inf();
        r.succ = __builtin_inf();
        r.L = sh.st.cL + iv[0];
        r.G = (sh.st.n - sh.st.cR) + iv[1];
        r.written = 0;
        bdev_after_eval(sh.st, r, a.cfg);
      }
      __syncthreads();
      if (sh.st.phase == PH_HIST) {
        const int p = sh.st.side;
        block_pick<T, BLOCK>(sh.rh + p * (kHistMaxBins / 2), pg[p].nbins,
                             (uint64_t)(sh.st.k - sh.st.cL), sh);
        if (tid == 0) {
          const int32_t bsel = (int32_t)sh.misc[0];
          bdev_hist_narrow(sh.st, pg[p], bsel, bsel < 0 ? 0 : sh.misc[1],
                           bsel < 0 ? 0 : sh.misc[2], a.cfg);
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
      block_pass<T, BLOCK, SU, false, true, true, false>(sp, t, yL, yR, fmn, fmx, zb[s.zout], cap, sh, acc);
    } else {
      block_pass<T, BLOCK, SU, false, true, false, false>(sp, t, yL, yR, fmn, fmx, zb[s.zout], cap, sh, acc);
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
        EvalResult r;
        r.A = dv[0]; r.B = dv[1]; r.pred = dv[2]; r.succ = dv[3];
        r.L = iv[0]; r.G = iv[1];
        r.written = sh.cur[0] + sh.cur[1];
        bdev_after_eval(w, r, a.cfg);
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
  if (tid == 0) write_batch_result<T>(out, sh.st);
  __syncthreads();
}

template <typename T, int BLOCK, int U>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_num_vgpr(128)))
void batched_select_kernel(BatchArgs<T> a) {
  __shared__ BShared<T, BLOCK> sh;
  const int tid = threadIdx.x;
  const int64_t count = a.count;
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
  for (;;) {
    if (tid == 0) sh.job = (int64_t)atomic_add_relaxed(&a.ctl->queue, 1ull);
    __syncthreads();
    const int64_t j = sh.job;
    __syncthreads();
    if (j >= count) break;
    const int64_t i = sorted ? lpt_index(sh.order[j]) : j;
    select_one<T, BLOCK, U>(a.ptrs[i], a.sizes[i], a.ks[i], a.out + i, a, sh);
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
