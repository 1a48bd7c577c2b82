// Exact k-th element selection by Kelley's cutting plane, single array, one launch.
//
// One persistent kernel runs every pass of the method (Section 4, Algorithm 1 and the
// hybrid that ends it):
//   pass 0      min, max (with multiplicities) and sum of x in one reduction (step 0),
//               with NaN detection; repeated with infinity classification only when
//               an extreme is infinite; optionally with the two-point check of a
//               proposed bracket;
//   eval passes A(t), B(t), #(w<t), #(w>t), largest w<t and smallest w>t over the working
//               set at the trial point t (the objective and subgradient of Section 3 in
//               one fused reduction).  Once the bracket is small enough the exact finish
//               starts: by default the evaluation at that trial point only counts the
//               bracket's elements on either side of t in key bins (and, for large
//               inputs, copies a likely interval of values sampled after pass 0), and the
//               bracket narrows to the bin of the rank; otherwise the pass splits the
//               bracket's elements at t into per-wavefront private regions of a
//               workspace buffer (count-and-compact, with no atomics), and later passes
//               read only the side that holds x_(k);
//   histogram   each pass counts the working set in key bins of the bracket's value range
//               and narrows the bracket to the bin holding the remaining rank (an exact
//               select, in place of the paper's sort of the compacted elements); a pass
//               over x also copies the narrowed bracket's elements when they are few;
//   gather      the bracket's remaining elements are copied into one contiguous buffer;
//   final       one workgroup selects the remaining rank exactly (radix select on the
//               ordered keys).
// Between passes the grid synchronises through two-level arrival counters; the last
// workgroup to arrive reduces the per-workgroup partials in a fixed order and advances
// the cutting-plane state (cp_state.h), so no pass needs the host.  The kernel is
// launched cooperatively, which guarantees that every workgroup is resident.
#include "cps_device.h"
#include "cps_kernels.h"
#include "cps_passes.h"

namespace cps {

// The scalar cutting-plane update runs in one thread per pass, inside the out-of-line
// last_update (so its registers stay out of the streaming loops' budget).  Inlined there,
// its records live in registers: out of line they went through the stack in scratch
// memory, a chain of dependent memory round trips that cost ~10 us per update.
__device__ __attribute__((always_inline)) inline void dev_after_pass0(CpState &s, const Pass0Result &r, const CpConfig &c) {
  cp_after_pass0(s, r, c);
}
__device__ __attribute__((always_inline)) inline void dev_after_eval(CpState &s, const EvalResult &r, const CpConfig &c) {
  cp_after_eval(s, r, c);
}
__device__ __attribute__((always_inline)) inline void dev_after_gather(CpState &s, int64_t gathered) {
  cp_after_gather(s, gathered);
}
__device__ __attribute__((always_inline)) inline void dev_after_final(CpState &s, double v, int64_t below, int64_t eq) {
  cp_after_final(s, v, below, eq);
}
__device__ __attribute__((always_inline)) inline void dev_after_hist(CpState &s, int32_t b, int64_t below, int64_t cnt,
                                            const CpConfig &c) {
  cp_after_hist(s, b, below, cnt, c);
}
__device__ __attribute__((always_inline)) inline void dev_adopt_spec(CpState &s, int64_t written,
                                                                    const CpConfig &c) {
  cp_adopt_spec(s, written, c);
}
__device__ __attribute__((always_inline)) inline void dev_hist_narrow(CpState &s, const HistGeom<uint64_t> &g, int32_t b,
                                             int64_t below, int64_t cnt, const CpConfig &c) {
  cp_hist_narrow(s, g, b, below, cnt, c);
}

// How the threads of a workgroup walk the working set.  BLOCK mode: the whole input,
// tiles of BLOCK*U vectors dealt round-robin to workgroups (vector u*BLOCK + tid of a
// tile belongs to thread tid).  WAVE mode: each wavefront walks its own segment of a
// split buffer, 64*U vectors at a time.  The edge elements of a span go to the first
// lanes of its owner.
template <typename T> struct Walk {
  Span<T> sp;
  bool wave_mode;
  bool edge_owner;
};

// ------------------------------------------------------------------ kernel

// Split staging: each lane keeps the elements it sends to either part of a split in its own
// column of an LDS block (slot-major, so a wavefront's writes fall in distinct banks) and
// moves them to global memory one 16-byte vector at a time, at a place given by a prefix
// count over the wavefront's lanes that hold a full vector.
template <typename T> struct Stage {
  static constexpr uint32_t kV = Traits<T>::kVec;  // elements per 16-byte vector
  static constexpr uint32_t kS = 2 * kV;           // slots per lane and part
  static constexpr uint32_t kSlots = kS * kWave;   // per part and wavefront
};

template <typename T, int BLOCK> struct Shared {
  CpState st;
  double d[8][BLOCK / kWave];
  int64_t i[8][BLOCK / kWave];
  int64_t wseg[2][BLOCK / kWave];  // per wavefront: low / high counts of its last split
  uint64_t gbase[BLOCK / kWave];
  uint32_t hist[256];
  int64_t misc[8];
  int last;
  int timed_out;
  uint32_t lcnt;  // elements a gather pass staged in LDS
  uint32_t rh[kHistWords];  // key histogram of a histogram pass, or of both parts of a split
  T ring[BLOCK / kWave][2][Stage<T>::kSlots];  // split staging, per wavefront and part
  // The launch's arguments for the out-of-line update: a reference to the kernel's own
  // argument would make the compiler copy it to every lane's scratch memory at launch
  // (~280 bytes per lane, ~70 MB for a full grid).
  SelectArgs<T> args;
};

// Which side of the trial point an element goes to in a split: the bracket's elements
// below t to the low part, above t to the high part.  FILTER: the working set is the
// whole input, so the bracket ends are tested too.
template <typename T, bool FILTER>
__device__ inline bool goes_low(T v, bool valid, T t, T lo_ex) {
  return valid && v < t && (!FILTER || v > lo_ex);
}
template <typename T, bool FILTER>
__device__ inline bool goes_high(T v, bool valid, T t, T hi_ex) {
  return valid && v > t && (!FILTER || v < hi_ex);
}

// Per-wavefront split output: the low part grows up from the start of the wavefront's
// region, the high part down from its end.  lo / hi count the elements in the region
// (wave-uniform).  Every writer stages in LDS first (per lane: cl / ch elements staged,
// fl / fh of them moved): splits both parts, the compactions and copies the low part.
template <typename T> struct WaveOut {
  CPS_GLOBAL T *region;  // wave-uniform
  uint32_t top;          // Rw - 1
  uint32_t lo, hi;       // a region holds fewer than 2^32 elements
  uint32_t cl, ch, fl, fh;
  T *ring_lo, *ring_hi;  // Stage<T>::kSlots each
};

// Stage v in this lane's column: it is always written to the next free slot, which is
// kept only when `sel`.
template <typename T>
__device__ inline void stage_one(T v, bool sel, T *ring, uint32_t &c, int lane) {
  ring[(c & (Stage<T>::kS - 1)) * kWave + lane] = v;
  c += sel ? 1u : 0u;
}

// Key bins of the two parts of a split (low part: counters rh[0..), high part: counters
// rh[kHistMaxBins..)), for a split pass that also counts the parts' elements.
template <typename T> struct PartBins {
  typename Traits<T>::Key klo[2];
  typename Traits<T>::Key span[2];  // khi - klo: a part's elements have klo <= key <= klo + span
  bool has[2];                      // the part's key range is not empty
  typename Traits<T>::Key ka, kab;  // a counting evaluation's copy: ka <= key <= ka + kab
  uint32_t last[2];  // nbins - 1
  int shift[2];
  uint32_t *rh;
};

// One element of a counting evaluation (over the input), on its ordered key alone: the low
// side's elements are those with keys in [klo0, khi0] = [key(lo), key(t-)], the high
// side's those in [klo1, khi1] = [key(t+), key(hi)] (the bracket's elements below and above
// t exactly, as lo and hi bound them), so the side and the bin come from one key and two
// unsigned range tests.  SPEC: an element of the copy's interval is staged in the lane's
// LDS column.
template <typename T, bool SPEC>
__device__ inline void count_key(T v, bool valid, const PartBins<T> &pb, WaveOut<T> &o,
                                 int lane) {
  using Key = typename Traits<T>::Key;
  const Key K = Traits<T>::key(v);
  const Key d0 = K - pb.klo[0], d1 = K - pb.klo[1];
  const bool l = valid & pb.has[0] & (d0 <= pb.span[0]);
  const bool h = valid & pb.has[1] & (d1 <= pb.span[1]);
  if (l | h) {
    const uint32_t bin = l ? (uint32_t)(d0 >> pb.shift[0])
                           : (uint32_t)(d1 >> pb.shift[1]) + (uint32_t)kHistMaxBins;
    atomicAdd(&pb.rh[bin], 1u);
  }
  if (SPEC) {
    if (valid & (K - pb.ka <= pb.kab)) {
      o.ring_lo[(o.cl & (Stage<T>::kS - 1)) * kWave + lane] = v;
      o.cl += 1;
    }
  }
}

// Count an element of the low part (l) or the high part (h) in that part's key bins.
template <typename T>
__device__ inline void count_part(T v, bool l, bool h, const PartBins<T> &pb) {
  using Key = typename Traits<T>::Key;
  if (l || h) {
    // An element of a part lies in that part's key range (the ranges come from the bracket's
    // bounds and the neighbours of t in T, and keys are monotone), so its bin is in range;
    // the clamp only keeps the counters safe.
    const int p = l ? 0 : 1;
    const Key K = Traits<T>::key(v);
    uint32_t bin = (uint32_t)((K - pb.klo[p]) >> pb.shift[p]);
    bin = bin < pb.last[p] ? bin : pb.last[p];
    atomicAdd(&pb.rh[p * kHistMaxBins + bin], 1u);
  }
}

template <typename T, bool FILTER, bool HIST>
__device__ inline void split_one(T v, bool valid, T t, T yL, T yR, WaveOut<T> &o, int lane,
                                 const PartBins<T> &pb) {
  const bool l = goes_low<T, FILTER>(v, valid, t, yL);
  const bool h = goes_high<T, FILTER>(v, valid, t, yR);
  stage_one<T>(v, l, o.ring_lo, o.cl, lane);
  stage_one<T>(v, h, o.ring_hi, o.ch, lane);
  if (HIST) count_part<T>(v, l, h, pb);
}


// Move every lane's full vector of either part to the region.  Called after each vector of
// input, so a lane holds fewer than two vectors of a part and moves at most one.
template <typename T, bool HIGH>
__device__ inline void flush_part(WaveOut<T> &o, const T *ring, uint32_t c, uint32_t &f,
                                  int lane) {
  using S = Stage<T>;
  using Vec = typename Traits<T>::Vec;
  const bool full = c - f >= S::kV;
  const uint64_t m = ballot(full);
  if (m == 0) return;
  if (full) {
    // f is a multiple of kV, so the vector's slots do not wrap
    const T *col = ring + (f & (S::kS - 1)) * kWave + lane;
    Vec d;
#pragma unroll
    for (uint32_t j = 0; j < S::kV; ++j) d[j] = col[j * kWave];
    const uint32_t at = S::kV * lane_rank(m);
    const uint32_t pos = HIGH ? o.top + 1 - o.hi - at - S::kV : o.lo + at;
    *reinterpret_cast<CPS_GLOBAL Vec *>(o.region + pos) = d;
    f += S::kV;
  }
  if (HIGH) o.hi += S::kV * popc(m);
  else o.lo += S::kV * popc(m);
}

template <typename T>
__device__ inline void split_flush(WaveOut<T> &o, int lane) {
  __builtin_amdgcn_wave_barrier();
  flush_part<T, false>(o, o.ring_lo, o.cl, o.fl, lane);
  flush_part<T, true>(o, o.ring_hi, o.ch, o.fh, lane);
  __builtin_amdgcn_wave_barrier();
}

// Move what is left (at most one vector per lane and part) at the end of a split pass.
template <typename T>
__device__ inline void split_drain(WaveOut<T> &o, int lane) {
  using S = Stage<T>;
  __builtin_amdgcn_wave_barrier();
  const T *cl = o.ring_lo + (o.fl & (S::kS - 1)) * kWave + lane;  // fl, fh: multiples of kV
  const T *ch = o.ring_hi + (o.fh & (S::kS - 1)) * kWave + lane;
#pragma unroll
  for (uint32_t j = 0; j < S::kV; ++j) {
    const bool sl = o.cl - o.fl > j;
    const uint64_t ml = ballot(sl);
    if (sl) o.region[o.lo + lane_rank(ml)] = cl[j * kWave];
    o.lo += popc(ml);
    const bool sh = o.ch - o.fh > j;
    const uint64_t mh = ballot(sh);
    if (sh) o.region[o.top - (o.hi + lane_rank(mh))] = ch[j * kWave];
    o.hi += popc(mh);
  }
  o.fl = o.cl;
  o.fh = o.ch;
}

// Pass 0 with a proposed bracket (a, b) may also write the elements strictly inside it to
// its wavefront's region, up to `cap` of them (the count goes on past the cap, so an
// overflowing region is seen and its contents are not used).
// Key bins of a proposal's interior, counted by pass 0 (one set of counters in LDS).
template <typename T> struct InteriorBins {
  typename Traits<T>::Key klo;
  typename Traits<T>::Key span;    // khi - klo: the interior's keys are klo .. klo + span
  typename Traits<T>::Key ka, kb;  // keys of the proposed ends
  uint32_t last;  // nbins - 1
  int shift;
  uint32_t *rh;
};

// The device proposal's pass 0 on one element's ordered key (after its extremes and sum):
// #(x <= a) and #(x < b) by key compares, and an interior element (key in [key(a+),
// key(b-)]) staged in the lane's column and counted in its bin.  The keys order the values
// as the compares do (NaN aside: a NaN makes this fast pass 0 repeat with the
// classification, whose counts are taken by value).
template <typename T>
__device__ inline void p0_key(T v, bool valid, const InteriorBins<T> &ib, P0Acc<T> &acc,
                              WaveOut<T> &o, int lane) {
  using Key = typename Traits<T>::Key;
  const Key K = Traits<T>::key(v);
  acc.cle_a += (valid & (K <= ib.ka)) ? 1u : 0u;
  acc.clt_b += (valid & (K < ib.kb)) ? 1u : 0u;
  const Key d = K - ib.klo;
  if (valid & (d <= ib.span)) {
    o.ring_lo[(o.cl & (Stage<T>::kS - 1)) * kWave + lane] = v;
    o.cl += 1;
    atomicAdd(&ib.rh[(uint32_t)(d >> ib.shift)], 1u);
  }
}

// An interior element goes to this lane's staging column (low part) and, with HIST, to its
// key bin.
template <typename T, bool HIST>
__device__ inline void stage_inside(T v, bool valid, T a, T b, WaveOut<T> &o, int lane,
                                    const InteriorBins<T> &ib) {
  const bool in = valid & (v > a) & (v < b);
  if (in) {
    o.ring_lo[(o.cl & (Stage<T>::kS - 1)) * kWave + lane] = v;
    o.cl += 1;
  }
  if (HIST && in) {
    // an interior element's key lies in the interior's range; the clamp keeps LDS safe
    uint32_t bin = (uint32_t)((Traits<T>::key(v) - ib.klo) >> ib.shift);
    atomicAdd(&ib.rh[bin < ib.last ? bin : ib.last], 1u);
  }
}

// Move every lane's full staged vector to the region, at most `cap` elements in all (the
// count goes on past the cap).  After each vector of input a lane holds fewer than two.
template <typename T>
__device__ inline void flush_inside(WaveOut<T> &o, int lane, uint32_t cap) {
  using S = Stage<T>;
  using Vec = typename Traits<T>::Vec;
  __builtin_amdgcn_wave_barrier();
  const bool full = o.cl - o.fl >= S::kV;
  const uint64_t m = ballot(full);
  if (m != 0) {
    if (full) {
      const T *col = o.ring_lo + (o.fl & (S::kS - 1)) * kWave + lane;
      Vec d;
#pragma unroll
      for (uint32_t j = 0; j < S::kV; ++j) d[j] = col[j * kWave];
      const uint32_t pos = o.lo + S::kV * lane_rank(m);  // a multiple of kV: aligned
      if (pos + S::kV <= cap) *reinterpret_cast<CPS_GLOBAL Vec *>(o.region + pos) = d;
      o.fl += S::kV;
    }
    o.lo += S::kV * popc(m);
  }
  __builtin_amdgcn_wave_barrier();
}

// What is left in the columns at the end of the pass, one element per lane at a time.
template <typename T>
__device__ inline void drain_inside(WaveOut<T> &o, int lane, uint32_t cap) {
  using S = Stage<T>;
  __builtin_amdgcn_wave_barrier();
  const T *col = o.ring_lo + (o.fl & (S::kS - 1)) * kWave + lane;
#pragma unroll
  for (uint32_t j = 0; j < S::kV; ++j) {
    const bool sel = o.cl - o.fl > j;
    const uint64_t m = ballot(sel);
    const uint32_t pos = o.lo + lane_rank(m);
    if (sel && pos < cap) o.region[pos] = col[j * kWave];
    o.lo += popc(m);
  }
}

// Streaming passes load with the nontemporal hint: a pass over x reads each line once, and
// keeping those lines out of the caches' way made the passes over a 1 GiB input ~10 %
// faster (pass 0 at 2^28 float32: 230 -> 195 us).

// One tile of an evaluation pass: U vectors per thread.  FULL: every vector of the tile
// lies inside the span (no bounds tests; every tile but a span's last is full).
// SPEC (a counting evaluation only): the elements of the copy's key range (pb.ka, pb.kab)
// also go to the wavefront's region of split buffer 0, staged in its LDS columns.
// The U vectors of a tile that belong to thread `me` (vector base + u*per_u + me), with the
// nontemporal hint; FULL: the whole tile lies inside the span.
template <typename T, int U, bool FULL>
__device__ __attribute__((always_inline)) inline void tile_load(const Span<T> &sp, int64_t base, int per_u, int me,
                                 typename Traits<T>::Vec (&raw)[U], bool (&valid)[U]) {
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int64_t vi = base + (int64_t)u * per_u + me;
    valid[u] = FULL || vi < sp.nvec;
    if (valid[u]) raw[u] = __builtin_nontemporal_load(&sp.V[vi]);
  }
}

// Walk the full tiles of a pass from `base` on (every `stride` vectors) with the next tile's
// loads issued before the current tile is processed, so that each wavefront keeps its loads
// in flight while it computes; returns the base of the first tile that is not full (a last
// partial tile, or the end), which the caller walks without the prefetch.
template <typename T, int U, typename Body>
__device__ __attribute__((always_inline)) inline int64_t walk_full_tiles(const Span<T> &sp, int64_t base, int64_t stride,
                                          int per_u, int me, Body &&body) {
  using Vec = typename Traits<T>::Vec;
  const int64_t last_full = sp.nvec - (int64_t)U * per_u;  // tiles at base <= last_full are full
  if (base > last_full) return base;
  Vec cur[U];
  bool valid[U];
  tile_load<T, U, true>(sp, base, per_u, me, cur, valid);
  for (;;) {
    const int64_t nb = base + stride;
    const bool more = nb <= last_full;  // (uniform over the walk's threads)
    Vec nxt[U];
    if (more) tile_load<T, U, true>(sp, nb, per_u, me, nxt, valid);
    body(cur, base);
    base = nb;
    if (!more) return base;
#pragma unroll
    for (int u = 0; u < U; ++u) cur[u] = nxt[u];
  }
}

template <typename T, int U, bool CLAMP, bool SPLIT, bool FILTER, bool HIST, bool FULL,
          bool SPEC = false>
__device__ __attribute__((always_inline)) inline void eval_tile_data(const typename Traits<T>::Vec (&raw)[U],
                                      const bool (&valid)[U], int me, T t, T yL, T yR, T fmin,
                                      T fmax, WaveOut<T> &o, EvalAcc<T> &acc,
                                      const PartBins<T> &pb) {
  constexpr int V = Traits<T>::kVec;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    T e[V];
    vec_to_arr<T>(raw[u], e);
    if (!SPLIT && HIST) {
      // a counting evaluation: the key bins of either side of t only (the bracket narrows
      // by the bins right after it, so f at t is not needed, and the counts below and above
      // t follow from the bins' totals and the bracket's counts)
#pragma unroll
      for (int j = 0; j < V; ++j) count_key<T, SPEC>(e[j], valid[u], pb, o, me % kWave);
      if (SPEC) flush_inside<T>(o, me % kWave, o.top + 1);
      continue;
    }
    T a_part = 0, b_part = 0;
#pragma unroll
    for (int j = 0; j < V; ++j) eval_one<T, CLAMP>(e[j], valid[u], t, fmin, fmax, a_part, b_part, acc);
    acc.A += (double)a_part;
    acc.B += (double)b_part;
    if (SPLIT) {
#pragma unroll
      for (int j = 0; j < V; ++j)
        split_one<T, FILTER, HIST>(e[j], valid[u], t, yL, yR, o, me % kWave, pb);
      split_flush<T>(o, me % kWave);
    }
  }
}

template <typename T, int U, bool CLAMP, bool SPLIT, bool FILTER, bool HIST, bool FULL,
          bool SPEC = false>
__device__ __attribute__((always_inline)) inline void eval_tile(const Span<T> &sp, int64_t base, int per_u, int me, T t, T yL,
                                 T yR, T fmin, T fmax, WaveOut<T> &o, EvalAcc<T> &acc,
                                 const PartBins<T> &pb) {
  typename Traits<T>::Vec raw[U];
  bool valid[U];
  tile_load<T, U, FULL>(sp, base, per_u, me, raw, valid);
  eval_tile_data<T, U, CLAMP, SPLIT, FILTER, HIST, FULL, SPEC>(raw, valid, me, t, yL, yR, fmin,
                                                               fmax, o, acc, pb);
}

// F(x) = log(1 + d), d = x - min x >= 0, to float precision: the exponent of 1 + d taken
// exactly and the hardware base-2 logarithm of its mantissa (the transformed scale only
// places trial points, so a relative error of ~1e-7 costs nothing in exactness, and the
// library logarithm's registers would spill the streaming loop).
__device__ inline double fast_log1p(double d) {
  int e;
  const double m = frexp(1.0 + d, &e);  // 1 + d = m 2^e, m in [1/2, 1)
  return 0.6931471805599453 * ((double)e + (double)__builtin_amdgcn_logf((float)m));
}

// An evaluation pass on the transformed scale (CpConfig::transform): the counts below and
// above t and t's neighbours on x, the sums A and B on F(x) = log(1 + x - xmin) (fast_log1p,
// summed in double precision; with CLAMP, infinities first clamped to the finite extremes).
// Ft = F(t).
template <typename T, int BLOCK, int U, bool CLAMP>
__device__ inline void eval_pass_log(const Walk<T> &wk, T t, double xmin, double Ft, T fmin,
                                     T fmax, EvalAcc<T> &acc) {
  constexpr int V = Traits<T>::kVec;
  using Vec = typename Traits<T>::Vec;
  const int tid = threadIdx.x, lane = tid % kWave;
  const Span<T> &sp = wk.sp;
  auto one = [&](T v, bool valid) {
    if (CLAMP) v = tmin(tmax(v, fmin), fmax);
    const bool l = valid && (v < t);
    const bool g = valid && (v > t);
    const double F = fast_log1p((double)v - xmin);
    acc.A += g ? F - Ft : 0.0;
    acc.B += l ? Ft - F : 0.0;
    acc.pred = tmax(acc.pred, l ? v : -t_inf<T>());
    acc.succ = tmin(acc.succ, g ? v : t_inf<T>());
    acc.L += l ? 1u : 0u;
    acc.G += g ? 1u : 0u;
  };
  // (the working set is x: the transform runs without splits)
  const int64_t step_vecs = (int64_t)BLOCK * U;
  for (int64_t base = (int64_t)blockIdx.x * step_vecs; base < sp.nvec;
       base += (int64_t)gridDim.x * step_vecs) {
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
      for (int j = 0; j < V; ++j) one(e[j], valid[u]);
    }
  }
  if (sp.nedge > 0 && wk.edge_owner && tid < kWave) {
    const bool have = lane < sp.nedge;
    one(have ? sp.W[edge_index(sp, lane)] : T(0), have);
  }
}

// One evaluation pass (optionally splitting) over this thread's share of the walk.
template <typename T, int BLOCK, int U, bool CLAMP, bool SPLIT, bool FILTER, bool HIST,
          bool SPEC = false>
__device__ inline void eval_pass(const Walk<T> &wk, T t, T yL, T yR, T fmin, T fmax,
                                       WaveOut<T> &o, EvalAcc<T> &acc, const PartBins<T> &pb) {
  const int tid = threadIdx.x, lane = tid % kWave;
  const Span<T> &sp = wk.sp;
  const int64_t step_vecs = wk.wave_mode ? (int64_t)kWave * U : (int64_t)BLOCK * U;
  const int64_t first = wk.wave_mode ? 0 : (int64_t)blockIdx.x * step_vecs;
  const int64_t stride = wk.wave_mode ? step_vecs : (int64_t)gridDim.x * step_vecs;
  const int me = wk.wave_mode ? lane : tid;
  const int per_u = wk.wave_mode ? kWave : BLOCK;
  int64_t base = first;
  if (kSelectPrefetch && !SPLIT) {  // (a split's staging leaves no registers for it)
    bool all_valid[U];
#pragma unroll
    for (int u = 0; u < U; ++u) all_valid[u] = true;
    base = walk_full_tiles<T, U>(sp, base, stride, per_u, me,
                                 [&](const typename Traits<T>::Vec (&raw)[U], int64_t) {
                                   eval_tile_data<T, U, CLAMP, SPLIT, FILTER, HIST, true, SPEC>(
                                       raw, all_valid, me, t, yL, yR, fmin, fmax, o, acc, pb);
                                 });
  }
  for (; base < sp.nvec; base += stride) {
    if (base + (int64_t)U * per_u <= sp.nvec)
      eval_tile<T, U, CLAMP, SPLIT, FILTER, HIST, true, SPEC>(sp, base, per_u, me, t, yL, yR, fmin,
                                                              fmax, o, acc, pb);
    else
      eval_tile<T, U, CLAMP, SPLIT, FILTER, HIST, false, SPEC>(sp, base, per_u, me, t, yL, yR, fmin,
                                                               fmax, o, acc, pb);
  }
  if (sp.nedge > 0 && wk.edge_owner && (wk.wave_mode || tid < kWave)) {
    const bool have = lane < sp.nedge;
    T v = have ? sp.W[edge_index(sp, lane)] : T(0);
    if (!SPLIT && HIST) {
      count_key<T, SPEC>(v, have, pb, o, lane);
      if (SPEC) flush_inside<T>(o, lane, o.top + 1);
    } else {
      T a_part = 0, b_part = 0;
      eval_one<T, CLAMP>(v, have, t, fmin, fmax, a_part, b_part, acc);
      acc.A += (double)a_part;
      acc.B += (double)b_part;
      if (SPLIT) split_one<T, FILTER, HIST>(v, have, t, yL, yR, o, lane, pb);
    }
  }
  if (SPLIT) split_drain<T>(o, lane);
  if (SPEC) drain_inside<T>(o, lane, o.top + 1);
}

template <typename T, int U, bool CLASSIFY, bool BRACKET, bool SPLIT, bool HIST, bool FULL,
          bool SAMPLE = false>
__device__ __attribute__((always_inline)) inline void pass0_tile_data(const typename Traits<T>::Vec (&raw)[U],
                                       const bool (&valid)[U], int me, T ba, T bb, P0Acc<T> &acc,
                                       WaveOut<T> &o, uint32_t cap, const InteriorBins<T> &ib,
                                       CPS_GLOBAL typename Traits<T>::Vec *smp, int64_t tile) {
  constexpr int V = Traits<T>::kVec;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    T e[V];
    vec_to_arr<T>(raw[u], e);
    T aa = 0, bA = 0, ab = 0, bB = 0;
    if (!CLASSIFY) {
      // Past the first tiles an element rarely reaches the wavefront's running extremes:
      // the wavefront tests that first (compares against uniform values) and updates the
      // lanes' extremes and their counts only when some element passes.
      p0_extremes_wave<T, V>(e, valid[u], acc);
      if (BRACKET && SPLIT && HIST) {  // the device proposal that counts its interior
#pragma unroll
        for (int j = 0; j < V; ++j)
          pass0_one<T, false, false, true>(e[j], valid[u], ba, bb, aa, bA, ab, bB, acc);
        const int lane = me % kWave;
#pragma unroll
        for (int j = 0; j < V; ++j) p0_key<T>(e[j], valid[u], ib, acc, o, lane);
        flush_inside<T>(o, lane, cap);
      } else {
#pragma unroll
        for (int j = 0; j < V; ++j)
          pass0_one<T, false, BRACKET, true, !HIST>(e[j], valid[u], ba, bb, aa, bA, ab,
                                                    bB, acc);
      }
    } else {
#pragma unroll
      for (int j = 0; j < V; ++j)
        pass0_one<T, true, BRACKET>(e[j], valid[u], ba, bb, aa, bA, ab, bB, acc);
    }
    if (SPLIT && !(BRACKET && HIST && !CLASSIFY)) {
      // staged in LDS and moved in 16-byte vectors (per-element stores of a small interior
      // cost a store instruction per element position)
      const int lane = me % kWave;
#pragma unroll
      for (int j = 0; j < V; ++j) stage_inside<T, HIST>(e[j], valid[u], ba, bb, o, lane, ib);
      flush_inside<T>(o, lane, cap);
    }
    if (BRACKET) {
      acc.Aa += (double)aa;
      acc.Ba += (double)bA;
      acc.Ab += (double)ab;
      acc.Bb += (double)bB;
    }
  }
  // the sample of the likely interval: every tile's first vector (its first thread's)
  if (SAMPLE && me == 0) smp[tile] = raw[0];
}

template <typename T, int U, bool CLASSIFY, bool BRACKET, bool SPLIT, bool HIST, bool FULL,
          bool SAMPLE = false>
__device__ __attribute__((always_inline)) inline void pass0_tile(const Span<T> &sp, int64_t base, int per_u, int me, T ba, T bb,
                                  P0Acc<T> &acc, WaveOut<T> &o, uint32_t cap,
                                  const InteriorBins<T> &ib,
                                  CPS_GLOBAL typename Traits<T>::Vec *smp, int64_t tile) {
  typename Traits<T>::Vec raw[U];
  bool valid[U];
  tile_load<T, U, FULL>(sp, base, per_u, me, raw, valid);
  pass0_tile_data<T, U, CLASSIFY, BRACKET, SPLIT, HIST, FULL, SAMPLE>(raw, valid, me, ba, bb, acc,
                                                                     o, cap, ib, smp, tile);
}

template <typename T, int BLOCK, int U, bool CLASSIFY, bool BRACKET, bool SPLIT, bool HIST = false>
__device__ inline void pass0(const Walk<T> &wk, T ba, T bb, P0Acc<T> &acc, WaveOut<T> &o,
                             uint32_t cap, const InteriorBins<T> &ib,
                             CPS_GLOBAL typename Traits<T>::Vec *smp = nullptr) {
  const int tid = threadIdx.x, lane = tid % kWave;
  const Span<T> &sp = wk.sp;
  const int64_t step_vecs = (int64_t)BLOCK * U;
  int64_t base = (int64_t)blockIdx.x * step_vecs;
  if (kSelectPrefetch && !CLASSIFY && !BRACKET && !SPLIT) {  // the plain fast pass 0
    bool all_valid[U];
#pragma unroll
    for (int u = 0; u < U; ++u) all_valid[u] = true;
    const int64_t stride = (int64_t)gridDim.x * step_vecs;
    if (smp)
      base = walk_full_tiles<T, U>(sp, base, stride, BLOCK, tid,
                                   [&](const typename Traits<T>::Vec (&raw)[U], int64_t b) {
                                     pass0_tile_data<T, U, false, false, false, HIST, true, true>(
                                         raw, all_valid, tid, ba, bb, acc, o, cap, ib, smp,
                                         b / step_vecs);
                                   });
    else
      base = walk_full_tiles<T, U>(sp, base, stride, BLOCK, tid,
                                   [&](const typename Traits<T>::Vec (&raw)[U], int64_t) {
                                     pass0_tile_data<T, U, false, false, false, HIST, true>(
                                         raw, all_valid, tid, ba, bb, acc, o, cap, ib, smp, 0);
                                   });
  }
  for (int64_t tile = base / step_vecs; base < sp.nvec;
       base += (int64_t)gridDim.x * step_vecs, tile += gridDim.x) {
    if (base + step_vecs > sp.nvec)
      pass0_tile<T, U, CLASSIFY, BRACKET, SPLIT, HIST, false>(sp, base, BLOCK, tid, ba, bb, acc, o,
                                                              cap, ib, smp, tile);
    else if (!CLASSIFY && !BRACKET && smp)
      pass0_tile<T, U, CLASSIFY, BRACKET, SPLIT, HIST, true, true>(sp, base, BLOCK, tid, ba, bb,
                                                                   acc, o, cap, ib, smp, tile);
    else
      pass0_tile<T, U, CLASSIFY, BRACKET, SPLIT, HIST, true>(sp, base, BLOCK, tid, ba, bb, acc, o,
                                                             cap, ib, smp, tile);
  }
  if (sp.nedge > 0 && wk.edge_owner && tid < kWave) {
    const bool have = lane < sp.nedge;
    const T v = have ? sp.W[edge_index(sp, lane)] : T(0);
    T aa = 0, bA = 0, ab = 0, bB = 0;
    pass0_one<T, CLASSIFY, BRACKET, false, !HIST>(v, have, ba, bb, aa, bA, ab, bB, acc);
    if (SPLIT) {
      stage_inside<T, HIST>(v, have, ba, bb, o, lane, ib);
      flush_inside<T>(o, lane, cap);
    }
    if (BRACKET) {
      acc.Aa += (double)aa;
      acc.Ba += (double)bA;
      acc.Ab += (double)ab;
      acc.Bb += (double)bB;
    }
  }
  if (SPLIT) drain_inside<T>(o, lane, cap);
}

// Gather: every element of the walk inside (yL, yR) goes to the gather buffer.  STAGE: the
// elements go to the workgroup's LDS buffer `lbuf` first, at places taken with one LDS atomic
// on `lcnt` per wavefront-step that holds any, and the caller moves them out with one device
// atomic per workgroup (the bracket's population must fit the buffer).  Otherwise the places
// come from one device atomic on `gcur` per such wavefront-step, which all workgroups contend
// for.
template <typename T, int BLOCK, int U, bool STAGE>
__device__ inline void gather_walk(const Walk<T> &wk, T yL, T yR, T *zf, uint64_t *gcur,
                                   CPS_LDS T *lbuf, CPS_LDS uint32_t *lcnt, uint32_t lcap,
                                   int64_t &written) {
  constexpr int V = Traits<T>::kVec;
  using Vec = typename Traits<T>::Vec;
  const int tid = threadIdx.x, lane = tid % kWave;
  const Span<T> &sp = wk.sp;
  const int64_t step_vecs = wk.wave_mode ? (int64_t)kWave * U : (int64_t)BLOCK * U;
  const int64_t first = wk.wave_mode ? 0 : (int64_t)blockIdx.x * step_vecs;
  const int64_t stride = wk.wave_mode ? step_vecs : (int64_t)gridDim.x * step_vecs;
  const int me = wk.wave_mode ? lane : tid;
  const int per_u = wk.wave_mode ? kWave : BLOCK;
  for (int64_t base = first; base < sp.nvec; base += stride) {
    // all of the step's loads first; most steps hold no element of the bracket.  `in`
    // has a bit per element of this lane inside the bracket (bitwise tests: no branches).
    Vec raw[U];
    uint32_t in = 0;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t vi = base + (int64_t)u * per_u + me;
      const bool vld = vi < sp.nvec;
      raw[u] = vld ? __builtin_nontemporal_load(&sp.V[vi]) : Vec{};
      T e[V];
      vec_to_arr<T>(raw[u], e);
#pragma unroll
      for (int j = 0; j < V; ++j)
        in |= (uint32_t)(vld & (e[j] > yL) & (e[j] < yR)) << (u * V + j);
    }
    if (ballot(in != 0) == 0) continue;
#pragma unroll
    for (int u = 0; u < U; ++u) {
      T e[V];
      vec_to_arr<T>(raw[u], e);
      uint32_t cnt = 0;
#pragma unroll
      for (int j = 0; j < V; ++j) cnt += popc(ballot((in >> (u * V + j)) & 1u));
      if (cnt == 0) continue;
      uint64_t off = 0;
      if (lane == 0) off = STAGE ? (uint64_t)atomicAdd((uint32_t *)lcnt, cnt) : atomic_add_relaxed(gcur, cnt);
      off = __shfl(off, 0);
      if (!STAGE) written += cnt;
#pragma unroll
      for (int j = 0; j < V; ++j) {
        const bool sel = (in >> (u * V + j)) & 1u;
        const uint64_t m = ballot(sel);
        if (sel) {
          // (a workgroup never holds more than the bracket's population, which fits; the test
          // only keeps LDS safe should the counts and the data ever disagree)
          if (STAGE) {
            if (off + lane_rank(m) < lcap) lbuf[off + lane_rank(m)] = e[j];
          } else {
            zf[off + lane_rank(m)] = e[j];
          }
        }
        off += popc(m);
      }
    }
  }
  if (sp.nedge > 0 && wk.edge_owner && (wk.wave_mode || tid < kWave)) {
    const bool have = lane < sp.nedge;
    const T v = have ? sp.W[edge_index(sp, lane)] : T(0);
    const bool in = have && v > yL && v < yR;
    const uint64_t m = ballot(in);
    if (m) {
      uint64_t off = 0;
      if (lane == 0)
        off = STAGE ? (uint64_t)atomicAdd((uint32_t *)lcnt, (uint32_t)popc(m))
                    : atomic_add_relaxed(gcur, (uint64_t)popc(m));
      off = __shfl(off, 0);
      if (in) {
        if (STAGE) {
          if (off + lane_rank(m) < lcap) lbuf[off + lane_rank(m)] = v;
        } else {
          zf[off + lane_rank(m)] = v;
        }
      }
      if (!STAGE) written += popc(m);
    }
  }
}

// Histogram pass: every element of the walk whose ordered key lies in [klo, khi] is counted
// in LDS bin (key - klo) >> shift.
template <typename T, int U, bool COMPACT, bool FULL>
__device__ inline void hist_tile(const Span<T> &sp, int64_t base, int per_u, int me,
                                 typename Traits<T>::Key klo, typename Traits<T>::Key khi,
                                 int shift, uint32_t *rh, WaveOut<T> &o) {
  constexpr int V = Traits<T>::kVec;
  using Vec = typename Traits<T>::Vec;
  using Key = typename Traits<T>::Key;
  Vec raw[U];
  bool valid[U];
#pragma unroll
  for (int u = 0; u < U; ++u) {
    const int64_t vi = base + (int64_t)u * per_u + me;
    valid[u] = FULL || vi < sp.nvec;
    raw[u] = Vec{};
    if (valid[u]) raw[u] = __builtin_nontemporal_load(&sp.V[vi]);
  }
  // keys and range tests first: after the first narrowing most elements of a tile lie
  // outside the bracket, and a wavefront with none in range skips the counting
  uint32_t in = 0;  // a bit per element of this lane in range (bitwise tests: no branches)
#pragma unroll
  for (int u = 0; u < U; ++u) {
    T e[V];
    vec_to_arr<T>(raw[u], e);
#pragma unroll
    for (int j = 0; j < V; ++j) {
      const Key K = Traits<T>::key(e[j]);
      in |= (uint32_t)(valid[u] & (K >= klo) & (K <= khi)) << (u * V + j);
    }
  }
  if (ballot(in != 0) == 0) return;
  const int lane = me % kWave;
#pragma unroll
  for (int u = 0; u < U; ++u) {
    T e[V];
    vec_to_arr<T>(raw[u], e);
#pragma unroll
    for (int j = 0; j < V; ++j) {
      const Key K = Traits<T>::key(e[j]);
      if ((in >> (u * V + j)) & 1u) {
        atomicAdd(&rh[(uint32_t)((K - klo) >> shift)], 1u);
        if (COMPACT) {  // into this lane's staging column (low part)
          o.ring_lo[(o.cl & (Stage<T>::kS - 1)) * kWave + lane] = e[j];
          o.cl += 1;
        }
      }
    }
    if (COMPACT) {  // at most kV new elements per lane since the last call
      __builtin_amdgcn_wave_barrier();
      flush_part<T, false>(o, o.ring_lo, o.cl, o.fl, lane);
      __builtin_amdgcn_wave_barrier();
    }
  }
}

template <typename T, int BLOCK, int U, bool COMPACT>
__device__ inline void hist_walk(const Walk<T> &wk, typename Traits<T>::Key klo,
                                 typename Traits<T>::Key khi, int shift, uint32_t *rh,
                                 WaveOut<T> &o) {
  using Key = typename Traits<T>::Key;
  const int tid = threadIdx.x, lane = tid % kWave;
  const Span<T> &sp = wk.sp;
  const int64_t step_vecs = wk.wave_mode ? (int64_t)kWave * U : (int64_t)BLOCK * U;
  const int64_t first = wk.wave_mode ? 0 : (int64_t)blockIdx.x * step_vecs;
  const int64_t stride = wk.wave_mode ? step_vecs : (int64_t)gridDim.x * step_vecs;
  const int me = wk.wave_mode ? lane : tid;
  const int per_u = wk.wave_mode ? kWave : BLOCK;
  for (int64_t base = first; base < sp.nvec; base += stride) {
    if (base + (int64_t)U * per_u <= sp.nvec)
      hist_tile<T, U, COMPACT, true>(sp, base, per_u, me, klo, khi, shift, rh, o);
    else
      hist_tile<T, U, COMPACT, false>(sp, base, per_u, me, klo, khi, shift, rh, o);
  }
  if (sp.nedge > 0 && wk.edge_owner && (wk.wave_mode || tid < kWave)) {
    const bool have = lane < sp.nedge;
    const T v = have ? sp.W[edge_index(sp, lane)] : T(0);
    const Key K = Traits<T>::key(v);
    const bool in = have && K >= klo && K <= khi;
    if (in) atomicAdd(&rh[(uint32_t)((K - klo) >> shift)], 1u);
    if (COMPACT) stage_one<T>(v, in, o.ring_lo, o.cl, lane);
  }
  if (COMPACT) split_drain<T>(o, lane);
}

// The bin holding rank r of a histogram's counts: an exclusive scan of the counts in a fixed
// order.  Leaves the bin in misc[0] (-1 when no bin holds it), the count below it in
// misc[1] and its own count in misc[2]; ends with a workgroup barrier.
// The same on counts the caller has loaded (thread t holds bins t * BPT .. t * BPT + BPT-1).
template <int BLOCK>
__device__ inline void hist_pick_loaded(const uint64_t (&hv)[kHistMaxBins / BLOCK], uint64_t r,
                                        uint64_t *wsum, int64_t *misc) {
  const int tid = threadIdx.x;
  constexpr int BPT = kHistMaxBins / BLOCK;
  uint64_t tot = 0;
#pragma unroll
  for (int j = 0; j < BPT; ++j) tot += hv[j];
  if (tid == 0) misc[0] = -1;
  uint64_t cum = block_exclusive_scan<BLOCK>(tot, wsum);
#pragma unroll
  for (int j = 0; j < BPT; ++j) {
    if (cum < r && r <= cum + hv[j]) {
      misc[0] = tid * BPT + j;
      misc[1] = (int64_t)cum;
      misc[2] = (int64_t)hv[j];
    }
    cum += hv[j];
  }
  __syncthreads();
}

template <int BLOCK>
__device__ inline void hist_pick(const uint64_t *gh, int nbins, uint64_t r, uint64_t *wsum,
                                 int64_t *misc) {
  const int tid = threadIdx.x;
  constexpr int BPT = kHistMaxBins / BLOCK;
  uint64_t hv[BPT];
  uint64_t tot = 0;
#pragma unroll
  for (int j = 0; j < BPT; ++j) {
    const int b = tid * BPT + j;
    hv[j] = b < nbins ? gh[b] : 0;
    tot += hv[j];
  }
  if (tid == 0) misc[0] = -1;
  uint64_t cum = block_exclusive_scan<BLOCK>(tot, wsum);
#pragma unroll
  for (int j = 0; j < BPT; ++j) {
    if (cum < r && r <= cum + hv[j]) {
      misc[0] = tid * BPT + j;
      misc[1] = (int64_t)cum;
      misc[2] = (int64_t)hv[j];
    }
    cum += hv[j];
  }
  __syncthreads();
}

template <typename T>
__device__ inline void write_result(const SelectArgs<T> &a, const CpState &s) {
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
  if (s.status == ST_NAN || s.status == ST_INTERNAL || s.status == ST_TIMEOUT) {
    r.less = r.equal = r.greater = 0;
  }
  *a.out = r;
  if (a.stats) {
    cps_stats *st = a.stats;
    st->passes = s.passes;
    st->work_passes = s.work_passes;
    st->kelley_steps = s.kelley;
    st->bisect_steps = s.bisect;
    st->final_select_size = (int32_t)s.final_size;
    st->bracket_used = s.bracket_used;
    st->elements_read = s.elements_read;
    st->elements_written = s.elements_written;
  }
}

// Arrive at the end of a pass.  Workgroups arrive in groups of kGroup on their own
// counter; the last of a group arrives at the top counter.  Returns true in exactly one
// workgroup (the last to arrive overall), which then sees every partial written before
// the arrivals.  Called by thread 0 only.
__device__ inline bool arrive(SyncCtl *sync, int bid, int G) {
  const int g = bid / kGroup;
  const int ng = (G + kGroup - 1) / kGroup;
  const int gsz = (g + 1) * kGroup <= G ? kGroup : G - g * kGroup;
  const uint32_t p = atomic_add_release(&sync->grp[g][0], 1u);
  if (p != (uint32_t)(gsz - 1)) return false;
  fence_acquire();
  store_relaxed(&sync->grp[g][0], 0u);
  const uint32_t q = atomic_add_release(&sync->top, 1u);
  if (q != (uint32_t)(ng - 1)) return false;
  fence_acquire();
  store_relaxed(&sync->top, 0u);
  return true;
}

// Key bins of the interior (ba, bb) of a device proposal, as the histogram pass after the
// proposal's adoption takes them: [a+, b-], the neighbours of the ends inside in T.  None
// when there are no counters for them.
template <typename T>
__device__ inline HistGeom<uint64_t> interior_geometry(const SelectArgs<T> &a, T ba, T bb) {
  HistGeom<uint64_t> g;
  g.klo = 1;
  g.khi = 0;
  g.shift = 0;
  g.nbins = 0;
  if (!a.phist || a.cfg.hist_bits <= 0 || !(ba < bb)) return g;
  const double lo = next_up((double)ba, a.cfg.dtype), hi = next_down((double)bb, a.cfg.dtype);
  if (!(lo <= hi)) return g;
  return hist_geometry(lo, hi, a.cfg.dtype, a.cfg.hist_bits);
}

// A gather pass that tests the bracket (over the input, or a split buffer that holds elements
// outside a narrowed bracket).  A workgroup holds at most the bracket's population `pop`: when
// that fits the split staging block of LDS (idle in this pass), the elements are staged there
// and reserved with one device atomic per workgroup.  Out of line (inlined into the pass loop,
// its registers pushed the streaming loops into spills), with everything passed by value so
// that nothing the loop reads can alias its stores.  Returns the count to report (thread 0).
template <typename T, int BLOCK, int UNROLL>
__device__ __noinline__ int64_t gather_filtered(Walk<T> wk, T yL, T yR, int64_t pop, T *zf,
                                                uint64_t *gcur, int64_t zcap, T *ring,
                                                uint32_t *lcnt, uint64_t *gbase) {
  constexpr int WPB = BLOCK / kWave;
  constexpr int64_t kCap = (int64_t)WPB * 2 * Stage<T>::kSlots;
  const int tid = threadIdx.x;
  CPS_LDS T *lbuf = (CPS_LDS T *)ring;
  CPS_LDS uint32_t *lc = (CPS_LDS uint32_t *)lcnt;
  int64_t written = 0;
  if (pop <= kCap) {
    if (tid == 0) *lc = 0;
    __syncthreads();
    gather_walk<T, BLOCK, UNROLL, true>(wk, yL, yR, zf, gcur, lbuf, lc, (uint32_t)kCap, written);
    __syncthreads();
    // more than kCap cannot happen while the counts hold; the gathered total then differs
    // from the bracket's population and the state machine reports an internal error
    const uint32_t got = *lc;
    const uint32_t cnt = got < (uint32_t)kCap ? got : (uint32_t)kCap;
    CPS_LDS uint64_t *gb = (CPS_LDS uint64_t *)gbase;
    if (tid == 0) *gb = cnt ? atomic_add_relaxed(gcur, (uint64_t)cnt) : 0;
    __syncthreads();
    const uint64_t base = *gb;
    CPS_GLOBAL T *z = (CPS_GLOBAL T *)zf;
    for (uint32_t i = tid; i < cnt; i += BLOCK)
      if (base + i < (uint64_t)zcap) z[base + i] = lbuf[i];
    written = tid == 0 ? (int64_t)got : 0;  // counted once (lane 0 of wavefront 0)
  } else {
    gather_walk<T, BLOCK, UNROLL, false>(wk, yL, yR, zf, gcur, lbuf, lc, 0u, written);
  }
  return written;
}

// The likely interval of a counting evaluation's copy, by the whole last workgroup after pass
// 0: the sample every workgroup stored during pass 0 (the first 16-byte vector of each tile of
// the input: 4 or 2 neighbours every 16384 or 8192 elements, 64K elements at 2^28) in the key
// bins of the bracket's range, then the bins of
// the sample ranks q -/+ d around the rank's place q = p m among the m sampled elements
// inside the bracket (p = (k - cL - 1/2) / (cR - cL), d = 4 sqrt(m p (1 - p)) + 2, four
// binomial standard deviations).  The interval runs from the first key of the lower bin to
// the last key of the upper one; with too few sampled elements nothing is set.

template <typename T, int BLOCK>
__device__ __noinline__ void spec_interval(const T *smp, int64_t nsmp, const CpConfig &c,
                                           Shared<T, BLOCK> &sh) {
  using Key = typename Traits<T>::Key;
  const int tid = threadIdx.x;
  const CpState &s = sh.st;
  const HistGeom<uint64_t> g = hist_geometry(s.lo, s.hi, c.dtype, c.hist_bits);
  for (int b = tid; b < g.nbins; b += BLOCK) sh.rh[b] = 0u;
  __syncthreads();
  const Key klo = (Key)g.klo, khi = (Key)g.khi;
  // eight 16-byte loads in flight per thread, then their keys into the bins (sixteen would
  // take the whole sample of a 2^28 float input in one round trip, but spill this function's
  // registers)
  using Vec = typename Traits<T>::Vec;
  constexpr int V = Traits<T>::kVec, R = 8;
  const Vec *sv = (const Vec *)smp;
  const int64_t nv = nsmp / V;
  for (int64_t i0 = tid; i0 < nv; i0 += (int64_t)BLOCK * R) {
    Vec w[R];
#pragma unroll
    for (int r = 0; r < R; ++r)
      if (i0 + (int64_t)r * BLOCK < nv) w[r] = sv[i0 + (int64_t)r * BLOCK];
#pragma unroll
    for (int r = 0; r < R; ++r) {
      if (i0 + (int64_t)r * BLOCK >= nv) break;
#pragma unroll
      for (int j = 0; j < V; ++j) {
        const Key K = Traits<T>::key(w[r][j]);
        if (K >= klo && K <= khi) atomicAdd(&sh.rh[(uint32_t)((K - klo) >> g.shift)], 1u);
      }
    }
  }
  __syncthreads();
  constexpr int BPT = kHistMaxBins / BLOCK;
  uint64_t hv[BPT];
  uint64_t tot = 0;
#pragma unroll
  for (int j = 0; j < BPT; ++j) {
    const int b = tid * BPT + j;
    hv[j] = b < g.nbins ? sh.rh[b] : 0u;
    tot += hv[j];
  }
  uint64_t cum = block_exclusive_scan<BLOCK>(tot, sh.gbase);
  if (tid == BLOCK - 1) sh.misc[3] = (int64_t)(cum + tot);
  if (tid == 0) sh.misc[4] = sh.misc[5] = -1;
  __syncthreads();
  const double m = (double)sh.misc[3];
  const double p = ((double)(s.k - s.cL) - 0.5) / (double)(s.cR - s.cL);
  const double q = p * m, d = 4.0 * __builtin_sqrt(m * p * (1.0 - p)) + 2.0;
  double rl = __builtin_floor(q - d), rh = __builtin_ceil(q + d);
  rl = rl < 1.0 ? 1.0 : (rl > m ? m : rl);
  rh = rh < rl ? rl : (rh > m ? m : rh);
  const uint64_t r0 = (uint64_t)rl, r1 = (uint64_t)rh;
#pragma unroll
  for (int j = 0; j < BPT; ++j) {
    if (cum < r0 && r0 <= cum + hv[j]) sh.misc[4] = tid * BPT + j;
    if (cum < r1 && r1 <= cum + hv[j]) sh.misc[5] = tid * BPT + j;
    cum += hv[j];
  }
  __syncthreads();
  if (tid == 0 && m >= 16.0 && sh.misc[4] >= 0 && sh.misc[5] >= 0) {
    CpState &w = sh.st;
    const uint64_t a0 = g.klo + ((uint64_t)sh.misc[4] << g.shift);
    uint64_t b1 = g.klo + (((uint64_t)sh.misc[5] + 1) << g.shift) - 1;
    if (b1 > g.khi || b1 < a0) b1 = g.khi;
    w.spec = 1;
    w.spec_a = unkey_T(a0, c.dtype);
    w.spec_b = unkey_T(b1, c.dtype);
  }
  __syncthreads();
}

// Workgroup partials each lane of the folding wavefront loads at once.
constexpr int kFold = 4;

// One pass by this workgroup; leaves the workgroup's partial in thread 0's dv / iv.
template <typename T, int BLOCK, int UNROLL>
__device__ inline void run_pass(const SelectArgs<T> &a, Shared<T, BLOCK> &sh, int phase,
                                      bool p0_slow, double (&dv)[8], int64_t (&iv)[8]) {
  // passes that also write or check a bracket hold fewer vectors in flight
  constexpr int SU = kSplitUnroll;
  constexpr int WPB = BLOCK / kWave;
  const int tid = threadIdx.x, wv = tid / kWave, lane = tid % kWave;
  const int bid = blockIdx.x;
  int dop[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  Walk<T> wk;
  if (phase == PH_PASS0) {
    bool use_br = a.cfg.use_bracket != 0;
    double bl = a.cfg.bracket_lo, bh = a.cfg.bracket_hi;
    if (a.bracket) {
      use_br = a.bracket[2] != 0.0;
      bl = a.bracket[0];
      bh = a.bracket[1];
    }
    const T ba = (T)bl, bb = (T)bh;
    const bool p0s = use_br && a.p0_cap > 0;
    const uint32_t cap = (uint32_t)a.p0_cap;
    // the fast pass 0 also counts the compacted interior in key bins when the proposal came
    // from the device (its kernel cleared the counters); they serve the first histogram step
    const HistGeom<uint64_t> g0 = interior_geometry(a, ba, bb);
    const bool p0h = p0s && !p0_slow && g0.nbins > 0;
    InteriorBins<T> ib;
    ib.klo = (typename Traits<T>::Key)g0.klo;
    ib.span = g0.nbins > 0 ? (typename Traits<T>::Key)(g0.khi - g0.klo) : 0;
    ib.ka = Traits<T>::key(ba);
    ib.kb = Traits<T>::key(bb);
    ib.last = g0.nbins > 0 ? (uint32_t)(g0.nbins - 1) : 0u;
    ib.shift = g0.shift;
    ib.rh = sh.rh;
    if (p0h) {
      for (int b = tid; b < g0.nbins; b += BLOCK) sh.rh[b] = 0u;
      __syncthreads();
    }
    WaveOut<T> o;
    const int wvu = __builtin_amdgcn_readfirstlane(wv);
    o.region = (CPS_GLOBAL T *)uniform_ptr(a.z[0] + ((int64_t)bid * WPB + wvu) * a.seg_R);
    o.top = (uint32_t)(a.seg_R - 1);
    o.lo = o.hi = o.cl = o.ch = o.fl = o.fh = 0;
    o.ring_lo = sh.ring[wv][0];  // the interior is staged in this wavefront's LDS columns
    o.ring_hi = nullptr;
    wk.sp = make_span(a.x, a.n);
    wk.wave_mode = false;
    wk.edge_owner = bid == 0;
    P0Acc<T> acc;
    acc.sum = 0;
    acc.mn = t_inf<T>();
    acc.mx = -t_inf<T>();
    acc.wmn = t_inf<T>();
    acc.wmx = -t_inf<T>();
    acc.cmn = acc.cmx = 0;
    acc.nnan = acc.nneg = acc.npos = acc.cle_a = acc.clt_b = 0;
    acc.Aa = acc.Ba = acc.Ab = acc.Bb = 0;
    if (!p0_slow) {
      if (p0h) pass0<T, BLOCK, UNROLL, false, true, true, true>(wk, ba, bb, acc, o, cap, ib);
      else if (p0s) pass0<T, BLOCK, SU, false, true, true>(wk, ba, bb, acc, o, cap, ib);
      else if (use_br) pass0<T, BLOCK, SU, false, true, false>(wk, ba, bb, acc, o, cap, ib);
      else pass0<T, BLOCK, UNROLL, false, false, false>(wk, ba, bb, acc, o, cap, ib,
                                                        (CPS_GLOBAL typename Traits<T>::Vec *)a.smp);
    } else {
      if (p0s) pass0<T, BLOCK, SU, true, true, true>(wk, ba, bb, acc, o, cap, ib);
      else if (use_br) pass0<T, BLOCK, SU, true, true, false>(wk, ba, bb, acc, o, cap, ib);
      else pass0<T, BLOCK, SU, true, false, false>(wk, ba, bb, acc, o, cap, ib);
    }
    if (p0h) {
      __syncthreads();
      for (int b = tid; b < g0.nbins; b += BLOCK) {
        const uint32_t c = sh.rh[b];
        if (c) atomic_add_relaxed(&a.phist[b], (uint64_t)c);
      }
    }
    if (p0s && lane == 0) {
      sh.wseg[0][wv] = o.lo;
      sh.wseg[1][wv] = 0;
    }
    // (the histogram counters are zero here: cleared with the workspace's first part when it
    // is allocated, by the last workgroup after every pass that counted into them, and by the
    // last workgroup out after a wait that timed out; clearing them here too held workgroup 0
    // at the next barrier until its 64 KB of stores had completed)
    double mn = (double)acc.mn, mx = (double)acc.mx;
    int64_t cmn = acc.cmn, cmx = acc.cmx;
    if (!use_br && !p0_slow) {
      // the plain fast pass 0 forms only the sum and the extremes' pairs (the classification
      // counts and the proposal's fields are zero): fold those alone
      dv[0] = acc.sum;
      block_reduce_pair<BLOCK, 1, 0>(dv, dop, iv, mn, cmn, mx, cmx, sh.d, sh.i);
      dv[1] = dv[2] = dv[3] = dv[4] = 0.0;
      iv[0] = iv[1] = iv[2] = iv[3] = iv[4] = iv[5] = 0;
      dv[5] = mn; dv[6] = mx; dv[7] = 0.0;
      iv[6] = cmn; iv[7] = cmx;
      return;
    }
    dv[0] = acc.sum; dv[1] = acc.Aa; dv[2] = acc.Ba; dv[3] = acc.Ab; dv[4] = acc.Bb;
    dv[5] = dv[6] = dv[7] = 0;
    iv[0] = (int64_t)acc.nnan; iv[1] = (int64_t)acc.nneg; iv[2] = (int64_t)acc.npos;
    iv[3] = (int64_t)acc.cle_a; iv[4] = (int64_t)acc.clt_b;
    iv[5] = (p0s && lane == 0 && o.lo > cap) ? 1 : 0;  // overflowing wavefronts
    iv[6] = iv[7] = 0;
    block_reduce_pair<BLOCK, 5, 6>(dv, dop, iv, mn, cmn, mx, cmx, sh.d, sh.i);
    if (tid == 0) {
      dv[5] = mn; dv[6] = mx; iv[6] = cmn; iv[7] = cmx;
    }
    return;
  }
  const CpState &s = sh.st;
  const T t = (T)s.t, yL = (T)s.yL, yR = (T)s.yR, fmn = (T)s.fmin, fmx = (T)s.fmax;
  const int64_t Rw = a.seg_R;  // elements per wavefront region of a split buffer
  if (s.wbuf < 0) {
    wk.sp = make_span(a.x, a.n);
    wk.wave_mode = false;
    wk.edge_owner = bid == 0;
  } else {
    // this wavefront's segment of its region in split buffer wbuf
    const T *region = a.z[s.wbuf] + ((int64_t)bid * WPB + wv) * Rw;
    const int64_t len = sh.wseg[s.side][wv];
    wk.sp = make_span(s.side == 0 ? region : region + (Rw - len), len);
    wk.wave_mode = true;
    wk.edge_owner = true;
  }
  EvalAcc<T> acc;
  acc.A = acc.B = 0;
  acc.pred = -t_inf<T>();
  acc.succ = t_inf<T>();
  acc.L = acc.G = 0;
  int64_t written = 0;
  if (s.phase == PH_HIST) {
    const HistGeom<uint64_t> g = hist_geometry(s.lo, s.hi, a.cfg.dtype, a.cfg.hist_bits);
    for (int b = tid; b < g.nbins; b += BLOCK) sh.rh[b] = 0u;
    __syncthreads();
    WaveOut<T> o;
    o.lo = o.hi = o.cl = o.ch = o.fl = o.fh = 0;
    if (s.compact) {  // the bracket's elements also go to this wavefront's region of zout
      const int wvu = __builtin_amdgcn_readfirstlane(wv);
      o.region = (CPS_GLOBAL T *)uniform_ptr(a.z[s.zout] + ((int64_t)bid * WPB + wvu) * Rw);
      o.top = (uint32_t)(Rw - 1);
      o.ring_lo = sh.ring[wv][0];
      o.ring_hi = sh.ring[wv][1];
      hist_walk<T, BLOCK, UNROLL, true>(wk, (typename Traits<T>::Key)g.klo,
                                        (typename Traits<T>::Key)g.khi, g.shift, sh.rh, o);
      if (lane == 0) {
        sh.wseg[0][wv] = o.lo;
        sh.wseg[1][wv] = 0;
        written = o.lo;
      }
    } else {
      o.region = nullptr;
      o.top = 0;
      o.ring_lo = o.ring_hi = nullptr;
      hist_walk<T, BLOCK, UNROLL, false>(wk, (typename Traits<T>::Key)g.klo,
                                         (typename Traits<T>::Key)g.khi, g.shift, sh.rh, o);
    }
    __syncthreads();
    for (int b = tid; b < g.nbins; b += BLOCK) {
      const uint32_t c = sh.rh[b];
      if (c) atomic_add_relaxed(&a.ghist[b], (uint64_t)c);
    }
  } else if (s.phase == PH_GATHER) {
    if (s.wbuf < 0 || s.filter) {
      written = gather_filtered<T, BLOCK, UNROLL>(wk, yL, yR, s.cR - s.cL, a.zf, &a.sync->gcur,
                                                  a.cfg.zcap, &sh.ring[0][0][0], &sh.lcnt,
                                                  &sh.gbase[0]);
    } else {
      // every element of a segment lies inside the bracket: one offset per workgroup
      const int64_t len = wk.sp.m;
      if (lane == 0) sh.gbase[wv] = (uint64_t)len;
      __syncthreads();
      if (tid == 0) {
        uint64_t tot = 0;
        for (int w = 0; w < WPB; ++w) {
          const uint64_t l = sh.gbase[w];
          sh.gbase[w] = tot;
          tot += l;
        }
        const uint64_t base = tot ? atomic_add_relaxed(&a.sync->gcur, tot) : 0;
        for (int w = 0; w < WPB; ++w) sh.gbase[w] += base;
      }
      __syncthreads();
      const uint64_t off = sh.gbase[wv];
      CPS_GLOBAL T *zf = (CPS_GLOBAL T *)a.zf;
      for (int64_t i = lane; i < len; i += kWave) zf[off + i] = wk.sp.W[i];
      if (lane == 0) written = len;
    }
  } else {
    WaveOut<T> o;
    const int wvu = __builtin_amdgcn_readfirstlane(wv);
    // (a counting evaluation's copy of the likely interval goes to split buffer 0)
    const int zo = s.counted ? 0 : s.zout;
    o.region = (CPS_GLOBAL T *)uniform_ptr(a.z[zo] + ((int64_t)bid * WPB + wvu) * Rw);
    o.top = (uint32_t)(Rw - 1);
    o.lo = o.hi = o.cl = o.ch = o.fl = o.fh = 0;
    o.ring_lo = sh.ring[wv][0];
    o.ring_hi = sh.ring[wv][1];
    const bool clamp = s.has_inf && s.wbuf < 0;
    const bool hist = (s.split || s.counted) && a.cfg.hist_bits > 0;
    PartBins<T> pb;
    pb.rh = sh.rh;
    int nb[2] = {0, 0};
    if (hist) {
      using Key = typename Traits<T>::Key;
      for (int p = 0; p < 2; ++p) {
        const HistGeom<uint64_t> g = split_part_geometry(s, p, a.cfg);
        pb.klo[p] = (Key)g.klo;
        pb.has[p] = g.nbins > 0;
        pb.span[p] = g.nbins > 0 ? (Key)(g.khi - g.klo) : (Key)0;
        pb.last[p] = g.nbins > 0 ? (uint32_t)(g.nbins - 1) : 0u;
        pb.shift[p] = g.shift;
        nb[p] = g.nbins;
        for (int b = tid; b < g.nbins; b += BLOCK) sh.rh[p * kHistMaxBins + b] = 0u;
      }
      pb.ka = pb.kab = 0;
      if (s.counted && s.spec) {  // spec_a <= spec_b, both values of T
        pb.ka = Traits<T>::key((T)s.spec_a);
        pb.kab = Traits<T>::key((T)s.spec_b) - pb.ka;
      }
      __syncthreads();
    }
    if (s.counted) {  // (never with infinities: those inputs do not split or count)
      if (s.spec && Rw > 0) {
        eval_pass<T, BLOCK, UNROLL, false, false, true, true, true>(
            wk, t, yL, yR, fmn, fmx, o, acc, pb);
        if (lane == 0) {
          sh.wseg[0][wv] = o.lo;
          sh.wseg[1][wv] = 0;
          written = o.lo;
        }
      } else {
        eval_pass<T, BLOCK, UNROLL, false, false, true, true>(wk, t, yL, yR, fmn, fmx, o, acc, pb);
      }
    } else if (!s.split) {
      if (s.tf) {  // the transformed scale (x is the working set: no splits with the transform)
        const double Ft = fast_log1p(s.t - s.fmin);
        if (clamp) eval_pass_log<T, BLOCK, SU, true>(wk, t, s.fmin, Ft, fmn, fmx, acc);
        else eval_pass_log<T, BLOCK, SU, false>(wk, t, s.fmin, Ft, fmn, fmx, acc);
      } else if (clamp) {
        eval_pass<T, BLOCK, SU, true, false, false, false>(wk, t, yL, yR, fmn, fmx, o, acc, pb);
      } else {
        eval_pass<T, BLOCK, UNROLL, false, false, false, false>(wk, t, yL, yR, fmn, fmx, o, acc, pb);
      }
    } else if (s.filter) {
      if (hist) eval_pass<T, BLOCK, SU, false, true, true, true>(wk, t, yL, yR, fmn, fmx, o, acc, pb);
      else eval_pass<T, BLOCK, SU, false, true, true, false>(wk, t, yL, yR, fmn, fmx, o, acc, pb);
    } else {
      if (hist) eval_pass<T, BLOCK, SU, false, true, false, true>(wk, t, yL, yR, fmn, fmx, o, acc, pb);
      else eval_pass<T, BLOCK, SU, false, true, false, false>(wk, t, yL, yR, fmn, fmx, o, acc, pb);
    }
    if (s.split && lane == 0) {
      sh.wseg[0][wv] = o.lo;
      sh.wseg[1][wv] = o.hi;
      written = (int64_t)o.lo + o.hi;
    }
    if (hist) {
      __syncthreads();
      for (int p = 0; p < 2; ++p)
        for (int b = tid; b < nb[p]; b += BLOCK) {
          const uint32_t c = sh.rh[p * kHistMaxBins + b];
          if (c) atomic_add_relaxed(&a.ghist[p * kHistMaxBins + b], (uint64_t)c);
        }
    }
  }
  if (s.phase == PH_EVAL && !s.counted) {
    dv[0] = acc.A; dv[1] = acc.B; dv[2] = (double)acc.pred; dv[3] = (double)acc.succ;
    dop[2] = 2; dop[3] = 1;
    dv[4] = dv[5] = dv[6] = dv[7] = 0;
    iv[0] = (int64_t)acc.L; iv[1] = (int64_t)acc.G;
    iv[2] = lane == 0 ? written : 0;  // per wavefront, counted once
    iv[3] = iv[4] = iv[5] = iv[6] = iv[7] = 0;
    block_reduce<BLOCK, 4, 3>(dv, dop, iv, false, sh.d, sh.i);
    return;
  }
  // a counting evaluation, a histogram pass or a gather: only the elements written are
  // folded (the counts come from the key bins; A, B and the neighbours are not formed), the
  // other fields take their identities
  iv[0] = lane == 0 ? written : 0;
  block_reduce<BLOCK, 0, 1>(dv, dop, iv, false, sh.d, sh.i);
  iv[2] = iv[0];
  iv[0] = iv[1] = iv[3] = iv[4] = iv[5] = iv[6] = iv[7] = 0;
  dv[0] = dv[1] = 0.0;
  dv[2] = -__builtin_inf();
  dv[3] = __builtin_inf();
  dv[4] = dv[5] = dv[6] = dv[7] = 0.0;
}

// Trace of pass i in the stats record (thread 0 of the last workgroup only).
__device__ inline void trace_pass(cps_stats *st, int i, int32_t kind, double t, double A, double B,
                                  int64_t L, int64_t G, double pred, double succ) {
  if (!st || i >= CPS_STATS_MAX_PASSES) return;
  st->kind[i] = kind;
  st->trial[i] = t;
  st->A[i] = A;
  st->B[i] = B;
  st->L[i] = L;
  st->G[i] = G;
  st->pred[i] = pred;
  st->succ[i] = succ;
}

// Pass 0's reduction as the state machine takes it: f at the extremes from the sum
// (Section 4, step 0), the extremes and their multiplicities.
__device__ inline void trace_pass0(cps_stats *st, int i, int64_t n, const Pass0Result &r) {
  const double nf = (double)(n - r.nneg - r.npos - r.nnan);
  trace_pass(st, i, CPS_PASS_ZERO, r.fmin, r.sum - nf * r.fmin, nf * r.fmax - r.sum, r.cmin,
             r.cmax, r.fmin, r.fmax);
}

// The last workgroup to arrive: reduce every workgroup's partial in a fixed order, advance
// the cutting-plane state, run the exact select when the bracket is small, and write the
// new state to global memory (the caller then releases it).
template <typename T, int BLOCK>
__device__ __noinline__ void last_update(const SelectArgs<T> &a, Shared<T, BLOCK> &sh, int phase,
                                         bool p0_slow) {
  const int tid = threadIdx.x;
  const int G = gridDim.x;
  const int64_t stride = a.slot_stride;
  const uint64_t t_arrive = wall_clock64();
  int pidx = 0;  // index of the pass that just ended
  double rd[8];
  int64_t ri[8];
  if (phase == PH_PASS0) {
    // the first wavefront folds the partials: lane l takes workgroups l, l + 64, ... in
    // order, then the wavefront's fixed tree (deterministic); no workgroup barrier
    double mn = __builtin_inf(), mx = -__builtin_inf();
    int64_t cmn = 0, cmx = 0;
    if (tid < kWave) {
      for (int f = 0; f < 8; ++f) { rd[f] = 0; ri[f] = 0; }
      // the fields every pass 0 produces: kFold workgroups per lane at a time, all of
      // their loads issued before the first is used (one memory round trip per round)
      for (int b0 = tid; b0 < G; b0 += kWave * kFold) {
        double sm[kFold], m2[kFold], x2[kFold];
        int64_t c2[kFold], d2[kFold];
#pragma unroll
        for (int q = 0; q < kFold; ++q) {
          const int b = b0 + q * kWave < G ? b0 + q * kWave : 0;
          sm[q] = a.sd[0 * stride + b];
          m2[q] = a.sd[5 * stride + b];
          x2[q] = a.sd[6 * stride + b];
          c2[q] = a.si[6 * stride + b];
          d2[q] = a.si[7 * stride + b];
        }
#pragma unroll
        for (int q = 0; q < kFold; ++q) {
          if (b0 + q * kWave >= G) break;
          rd[0] += sm[q];
          if (m2[q] < mn) { mn = m2[q]; cmn = c2[q]; } else if (m2[q] == mn) cmn += c2[q];
          if (x2[q] > mx) { mx = x2[q]; cmx = d2[q]; } else if (x2[q] == mx) cmx += d2[q];
        }
      }
      // the classification counts (slow pass 0) and the proposal's fields, when present
      const bool more = p0_slow || a.cfg.use_bracket || (a.bracket && a.bracket[2] != 0.0);
      if (more)
        for (int b = tid; b < G; b += kWave) {
          for (int f = 1; f < 5; ++f) rd[f] += a.sd[f * stride + b];
          for (int f = 0; f < 6; ++f) ri[f] += a.si[f * stride + b];
        }
      for (int f = 0; f < 5; ++f) rd[f] = wave_sum(rd[f]);
      for (int f = 0; f < 6; ++f) ri[f] = wave_sum_i64(ri[f]);
      wave_pair_fold(mn, cmn, mx, cmx);
    }
    if (tid == 0) {
      Pass0Result r;
      r.classified = p0_slow ? 1 : 0;
      r.sum = rd[0]; r.A_a = rd[1]; r.B_a = rd[2]; r.A_b = rd[3]; r.B_b = rd[4];
      r.nnan = ri[0]; r.nneg = ri[1]; r.npos = ri[2]; r.c_le_a = ri[3]; r.c_lt_b = ri[4];
      r.fmin = mn; r.fmax = mx; r.cmin = cmn; r.cmax = cmx;
      r.split_overflow = ri[5];
      r.split_written = 0;  // (exactly the interior)
      // the pass that counted the interior formed only the two counts at the ends
      r.sums = (!p0_slow && a.phist && a.bracket && a.bracket[2] != 0.0 && a.p0_cap > 0 &&
                interior_geometry(a, (T)a.bracket[0], (T)a.bracket[1]).nbins > 0) ? 0 : 1;
      CpConfig c = a.cfg;
      if (a.bracket) {
        c.use_bracket = a.bracket[2] != 0.0 ? 1 : 0;
        c.bracket_lo = a.bracket[0];
        c.bracket_hi = a.bracket[1];
      }
      c.p0_split = (c.use_bracket && a.p0_cap > 0) ? 1 : 0;
      CpState &s = sh.st;
      if (!p0_slow) {
        s = CpState{};
        s.n = a.n;
        s.k = a.k;
      }
      pidx = s.work_passes;
      s.phase = PH_PASS0;
      trace_pass0(a.stats, pidx, a.n, r);
      dev_after_pass0(s, r, c);
      if (a.stats && pidx < CPS_STATS_MAX_PASSES) {
        a.stats->population[pidx] = s.phase == PH_DONE ? 0 : s.cR - s.cL;
        a.stats->working[pidx] = a.n;
      }
    }
    __syncthreads();
    // A proven proposal whose interior pass 0 compacted and counted: the first histogram
    // step needs no pass (the counts are those of the interior, in the bins it would use).
    const CpState &s1 = sh.st;
    if (a.phist && a.bracket && a.bracket[2] != 0.0 && a.p0_cap > 0 && s1.phase == PH_HIST &&
        s1.bracket_used == 3 && s1.on_bracket && s1.wbuf == 0) {
      const HistGeom<uint64_t> g0 = interior_geometry(a, (T)a.bracket[0], (T)a.bracket[1]);
      const HistGeom<uint64_t> g = hist_geometry(s1.lo, s1.hi, a.cfg.dtype, a.cfg.hist_bits);
      if (g0.nbins > 0 && g.klo == g0.klo && g.khi == g0.khi && g.shift == g0.shift) {
        hist_pick<BLOCK>(a.phist, g.nbins, (uint64_t)(s1.k - s1.cL), sh.gbase, sh.misc);
        if (tid == 0) {
          CpState &s = sh.st;
          const int32_t bsel = (int32_t)sh.misc[0];
          dev_hist_narrow(s, g, bsel, bsel < 0 ? 0 : sh.misc[1], bsel < 0 ? 0 : sh.misc[2], a.cfg);
          if (a.stats && pidx < CPS_STATS_MAX_PASSES)
            a.stats->population[pidx] = s.phase == PH_DONE ? 0 : s.cR - s.cL;
        }
      }
    }
    // a large input about to be counted from: the likely interval for the evaluation's copy
    __syncthreads();
    if (a.cfg.spec_min_n > 0 && a.n >= a.cfg.spec_min_n && a.seg_R > 0 && a.smp &&
        sh.st.phase == PH_EVAL && sh.st.counted && sh.st.wbuf < 0)
      spec_interval<T, BLOCK>(a.smp, a.smp_n, a.cfg, sh);
  } else if (phase == PH_HIST) {
    const CpState &s0 = sh.st;
    const HistGeom<uint64_t> g = hist_geometry(s0.lo, s0.hi, a.cfg.dtype, a.cfg.hist_bits);
    hist_pick<BLOCK>(a.ghist, g.nbins, (uint64_t)(s0.k - s0.cL), sh.gbase, sh.misc);
    for (int b = tid; b < g.nbins; b += BLOCK) a.ghist[b] = 0;  // ready for the next pass
    if (tid == 0) {
      CpState &s = sh.st;
      pidx = s.work_passes;
      const int64_t wl = s.wlen;
      const int32_t bsel = (int32_t)sh.misc[0];
      trace_pass(a.stats, pidx, CPS_PASS_HIST, 0, 0, 0, 0, 0, 0, 0);
      dev_after_hist(s, bsel, bsel < 0 ? 0 : sh.misc[1], bsel < 0 ? 0 : sh.misc[2], a.cfg);
      if (a.stats && pidx < CPS_STATS_MAX_PASSES) {
        a.stats->population[pidx] = s.phase == PH_DONE ? 0 : s.cR - s.cL;
        a.stats->working[pidx] = wl;
      }
    }
  } else {
    // a split pass that counted its parts, or an evaluation that only counted them: their
    // key bins, from the state it ran with
    const bool counted =
        sh.st.phase == PH_EVAL && (sh.st.split || sh.st.counted) && a.cfg.hist_bits > 0;
    const bool count_only = counted && !sh.st.split;
    HistGeom<uint64_t> pg[2];
    if (counted) {
      pg[0] = split_part_geometry(sh.st, 0, a.cfg);
      pg[1] = split_part_geometry(sh.st, 1, a.cfg);
    }
    // a counting evaluation: both sides' bins, loaded once (their totals give the counts
    // below and above t; the side that holds x_(k) is then narrowed from the same values)
    constexpr int BPT = kHistMaxBins / BLOCK;
    uint64_t hv0[BPT], hv1[BPT];
    if (count_only) {
      uint64_t t0 = 0, t1 = 0;
#pragma unroll
      for (int j = 0; j < BPT; ++j) {
        const int b = tid * BPT + j;
        hv0[j] = b < pg[0].nbins ? a.ghist[b] : 0;
        hv1[j] = b < pg[1].nbins ? a.ghist[kHistMaxBins + b] : 0;
        t0 += hv0[j];
        t1 += hv1[j];
      }
      t0 = (uint64_t)wave_sum_i64((int64_t)t0);
      t1 = (uint64_t)wave_sum_i64((int64_t)t1);
      if (tid % kWave == 0) {
        sh.i[0][tid / kWave] = (int64_t)t0;
        sh.i[1][tid / kWave] = (int64_t)t1;
      }
    }
    __syncthreads();  // every thread has read the state before thread 0 advances it
    // the first wavefront folds the partials (as after pass 0)
    if (tid < kWave) {
      for (int f = 0; f < 8; ++f) { rd[f] = 0; ri[f] = 0; }
      rd[2] = -__builtin_inf();
      rd[3] = __builtin_inf();
      // kFold workgroups per lane at a time, all of their loads issued first; a counting
      // evaluation has only its counts (A, B, pred and succ are not formed)
      for (int b0 = tid; b0 < G; b0 += kWave * kFold) {
        double A[kFold], B[kFold], pr[kFold], su[kFold];
        int64_t L[kFold], Gt[kFold], W[kFold];
#pragma unroll
        for (int q = 0; q < kFold; ++q) {
          const int b = b0 + q * kWave < G ? b0 + q * kWave : 0;
          L[q] = a.si[0 * stride + b];
          Gt[q] = a.si[1 * stride + b];
          W[q] = a.si[2 * stride + b];
          if (!count_only) {
            A[q] = a.sd[0 * stride + b];
            B[q] = a.sd[1 * stride + b];
            pr[q] = a.sd[2 * stride + b];
            su[q] = a.sd[3 * stride + b];
          }
        }
#pragma unroll
        for (int q = 0; q < kFold; ++q) {
          if (b0 + q * kWave >= G) break;
          ri[0] += L[q];
          ri[1] += Gt[q];
          ri[2] += W[q];
          if (!count_only) {
            rd[0] += A[q];
            rd[1] += B[q];
            rd[2] = fmax(rd[2], pr[q]);
            rd[3] = fmin(rd[3], su[q]);
          }
        }
      }
      rd[0] = wave_sum(rd[0]);
      rd[1] = wave_sum(rd[1]);
      rd[2] = wave_max(rd[2]);
      rd[3] = wave_min(rd[3]);
      for (int f = 0; f < 3; ++f) ri[f] = wave_sum_i64(ri[f]);
    }
    if (tid == 0) {
      CpState &s = sh.st;
      pidx = s.work_passes;
      const int64_t wl = s.wlen;
      if (s.phase == PH_GATHER) {
        trace_pass(a.stats, pidx, CPS_PASS_GATHER, 0, 0, 0, 0, 0, 0, 0);
        dev_after_gather(s, ri[2]);
      } else {
        EvalResult r;
        r.A = rd[0]; r.B = rd[1]; r.pred = rd[2]; r.succ = rd[3];
        r.L = ri[0]; r.G = ri[1]; r.written = ri[2];
        if (count_only) {  // L = #(x <= yL) + the low side, G = #(x >= yR) + the high side
          int64_t t0 = 0, t1 = 0;
          for (int w = 0; w < BLOCK / kWave; ++w) {
            t0 += sh.i[0][w];
            t1 += sh.i[1][w];
          }
          r.L = s.cL + t0;
          r.G = (s.n - s.cR) + t1;
          trace_pass(a.stats, pidx, CPS_PASS_COUNT, s.t, 0, 0, r.L, r.G, r.pred, r.succ);
        } else {
          const FullEval fe = cp_full_eval(s, r);
          trace_pass(a.stats, pidx, CPS_PASS_EVAL, s.t, fe.A, fe.B, fe.L, fe.G, r.pred, r.succ);
        }
        dev_after_eval(s, r, a.cfg);
      }
      if (a.stats && pidx < CPS_STATS_MAX_PASSES) {
        a.stats->population[pidx] = s.phase == PH_DONE ? 0 : s.cR - s.cL;
        a.stats->working[pidx] = wl;
      }
    }
    if (counted) {
      __syncthreads();
      // the state asks for a histogram pass over the part that holds x_(k): its counts are
      // here already, so the bracket narrows now
      if (sh.st.phase == PH_HIST && (sh.st.on_bracket || count_only)) {
        const CpState &s1 = sh.st;
        const int p = s1.side;
        if (count_only) {
          uint64_t hv[BPT];
#pragma unroll
          for (int j = 0; j < BPT; ++j) hv[j] = p ? hv1[j] : hv0[j];  // selects, no indexing
          hist_pick_loaded<BLOCK>(hv, (uint64_t)(s1.k - s1.cL), sh.gbase, sh.misc);
        } else
          hist_pick<BLOCK>(a.ghist + p * kHistMaxBins, pg[p].nbins, (uint64_t)(s1.k - s1.cL),
                           sh.gbase, sh.misc);
        if (tid == 0) {
          CpState &s = sh.st;
          const int32_t bsel = (int32_t)sh.misc[0];
          dev_hist_narrow(s, pg[p], bsel, bsel < 0 ? 0 : sh.misc[1], bsel < 0 ? 0 : sh.misc[2],
                          a.cfg);
          if (a.stats && pidx < CPS_STATS_MAX_PASSES)
            a.stats->population[pidx] = s.phase == PH_DONE ? 0 : s.cR - s.cL;
        }
      }
      // a counting evaluation that also copied the likely interval: adopt the copy when the
      // bracket now lies inside it
      if (count_only && tid == 0) {
        dev_adopt_spec(sh.st, ri[2], a.cfg);
        if (a.stats && pidx < CPS_STATS_MAX_PASSES)
          a.stats->population[pidx] = sh.st.phase == PH_DONE ? 0 : sh.st.cR - sh.st.cL;
      }
      for (int p = 0; p < 2; ++p)  // ready for the next pass
        for (int b = tid; b < pg[p].nbins; b += BLOCK) a.ghist[p * kHistMaxBins + b] = 0;
    }
  }
  __syncthreads();
  if (tid == 0 && a.stats && pidx < CPS_STATS_MAX_PASSES) {
    a.stats->t_arrive[pidx] = t_arrive;
    a.stats->t_publish[pidx] = wall_clock64();
  }
  // ---- exact finish in this workgroup when the bracket is small
  if (sh.st.phase == PH_FINAL) {
    const CpState &s = sh.st;
    const T *W = s.wbuf < 0 ? a.x : a.zf;
    typename Traits<T>::Key key;
    int64_t below, eq;
    block_radix_select<T, BLOCK>(W, s.wlen, !s.on_bracket, (T)s.yL, (T)s.yR, s.k - s.cL,
                                 sh.hist, sh.misc, key, below, eq);
    if (tid == 0) {
      CpState &w = sh.st;
      const int fi = w.work_passes;
      const int64_t wl = w.wlen;
      dev_after_final(w, (double)Traits<T>::unkey(key), below, eq);
      trace_pass(a.stats, fi, CPS_PASS_FINAL, 0, 0, 0, 0, 0, 0, 0);
      if (a.stats && fi < CPS_STATS_MAX_PASSES) {
        a.stats->population[fi] = 0;
        a.stats->working[fi] = wl;
        a.stats->t_arrive[fi] = wall_clock64();
        a.stats->t_publish[fi] = a.stats->t_arrive[fi];
      }
    }
    __syncthreads();
  }
  // write the new state: every thread copies words; the waits before the workgroup
  // barrier that follows make the stores complete, and thread 0's release covers them
  constexpr int NW = sizeof(CpState) / 8;
  for (int w = tid; w < NW; w += BLOCK)
    reinterpret_cast<uint64_t *>(a.st)[w] = reinterpret_cast<const uint64_t *>(&sh.st)[w];
  if (tid == 0) {
    const CpState &s = sh.st;
    if (s.phase == PH_DONE) write_result<T>(a, s);
    if (s.phase == PH_GATHER) a.sync->gcur = 0;
  }
}

template <typename T, int BLOCK, int UNROLL>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_num_vgpr(128))) void cp_select_kernel(SelectArgs<T> a) {
  __shared__ Shared<T, BLOCK> sh;
  const int tid = threadIdx.x, wv = tid / kWave, lane = tid % kWave;
  const int G = gridDim.x, bid = blockIdx.x;
  uint32_t gen = 0;
  if (tid == 0) sh.args = a;  // (read by last_update, after the pass's barriers)
  if (tid == 0) {
    gen = load_relaxed(&a.sync->gen);
    if (bid == 0) {
      // a pending record; overwritten on completion, left in place if a wait times out
      cps_result r = {};
      r.status = ST_TIMEOUT;
      *a.out = r;
      if (a.stats) a.stats->t_start = wall_clock64();
    }
  }
  if (lane == 0) sh.wseg[0][wv] = sh.wseg[1][wv] = 0;
  int phase = PH_PASS0;
  bool p0_slow = false;
  for (;;) {
    double dv[8];
    int64_t iv[8];
    run_pass<T, BLOCK, UNROLL>(a, sh, phase, p0_slow, dv, iv);
    // ---- publish this workgroup's partial and arrive
    if (tid == 0) {
      const int64_t stride = a.slot_stride;
#pragma unroll
      for (int f = 0; f < 8; ++f) {
        a.sd[f * stride + bid] = dv[f];
        a.si[f * stride + bid] = iv[f];
      }
      sh.last = arrive(a.sync, bid, G) ? 1 : 0;  // the last arrival has acquired already
    }
    __syncthreads();
    if (sh.last) {
      last_update<T, BLOCK>(sh.args, sh, phase, p0_slow);
      __syncthreads();
      if (tid == 0) {
        store_release(&a.sync->gen, gen + 1u);
        gen = gen + 1u;
      }
    } else {
      if (tid == 0) {
        // poll with device-scope loads, which are served coherently across the XCDs
        int64_t spins = 0;
        bool timed_out = false;
        while (load_relaxed(&a.sync->gen) == gen) {
          __builtin_amdgcn_s_sleep(2);
          if (++spins > a.spin_limit) { timed_out = true; break; }
        }
        sh.timed_out = timed_out ? 1 : 0;
        if (!timed_out) gen = gen + 1u;
        else store_relaxed(&a.sync->tmo, 1u);
      }
      __syncthreads();
      if (sh.timed_out) {
        if (tid == 0) {
          sh.st.phase = PH_DONE;
          sh.st.status = ST_TIMEOUT;
        }
      } else {
        // Read the state the last workgroup published, with device-scope loads as well:
        // its release wrote the state back before the generation word moved, and these
        // loads are served at the device's coherence point, so no acquire (an invalidation
        // of this XCD's L2, which took up to ~10 us with the XCD's 32 workgroups issuing it
        // together) is needed.  Nothing else another workgroup wrote is read by a waiting
        // workgroup: each reads only its own split regions, the input and, through device
        // atomics, the shared counters; the last workgroup acquires in `arrive`.
        constexpr int NW = sizeof(CpState) / 8;
        for (int w = tid; w < NW; w += BLOCK)
          reinterpret_cast<uint64_t *>(&sh.st)[w] =
              load_relaxed(reinterpret_cast<const uint64_t *>(a.st) + w);
      }
    }
    __syncthreads();
    phase = sh.st.phase;
    p0_slow = sh.st.p0_slow != 0;
    if (phase == PH_DONE) break;
  }
  // Leave the launch.  Normally every arrival counter is back at zero here; after a wait
  // that timed out, a workgroup that went on alone has left its group counter (and maybe
  // the top counter) part-way counted, and an abandoned histogram pass its counters.  Every
  // wait is bounded, so every workgroup gets here, and the last one clears them for the
  // next launch on this workspace.
  if (tid == 0) {
    const uint32_t e = __hip_atomic_fetch_add(&a.sync->exits, 1u, __ATOMIC_ACQ_REL,
                                              __HIP_MEMORY_SCOPE_AGENT);
    sh.last = e == (uint32_t)G - 1u ? 1 : 0;
  }
  __syncthreads();
  if (sh.last) {
    if (load_relaxed(&a.sync->tmo) != 0u)
      for (int b = tid; b < kHistWords; b += BLOCK) a.ghist[b] = 0;
    if (tid == 0) {
      const int ng = (G + kGroup - 1) / kGroup;
      for (int g = 0; g < ng; ++g) store_relaxed(&a.sync->grp[g][0], 0u);
      store_relaxed(&a.sync->top, 0u);
      store_relaxed(&a.sync->tmo, 0u);
      store_release(&a.sync->exits, 0u);
    }
  }
}

// ------------------------------------------------------------------ objective at given y

// Partial sums of the objective pieces at ys[blockIdx.y] over this block's slice of x.
template <typename T, int BLOCK>
__global__ __launch_bounds__(BLOCK) void objective_partial_kernel(const T *__restrict__ x,
                                                                  int64_t n,
                                                                  const double *__restrict__ ys,
                                                                  double *__restrict__ pd,
                                                                  int64_t *__restrict__ pi) {
  __shared__ double sd[8][BLOCK / kWave];
  __shared__ int64_t si[8][BLOCK / kWave];
  const double y = ys[blockIdx.y];
  double A = 0, B = 0, pred = -__builtin_inf(), succ = __builtin_inf();
  int64_t L = 0, E = 0, Gc = 0;
  for (int64_t i = (int64_t)blockIdx.x * BLOCK + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * BLOCK) {
    const double v = (double)x[i];
    const double d = v - y;
    if (v > y) { A += d; Gc++; succ = fmin(succ, v); }
    else if (v < y) { B -= d; L++; pred = fmax(pred, v); }
    else if (v == y) { E++; }
  }
  double dv[8] = {A, B, pred, succ, 0, 0, 0, 0};
  int dop[8] = {0, 0, 2, 1, 0, 0, 0, 0};
  int64_t iv[8] = {L, E, Gc, 0, 0, 0, 0, 0};
  block_reduce<BLOCK, 4, 3>(dv, dop, iv, false, sd, si);
  if (threadIdx.x == 0) {
    const int64_t slot = (int64_t)blockIdx.y * gridDim.x + blockIdx.x;
    for (int f = 0; f < 4; ++f) pd[slot * 4 + f] = dv[f];
    for (int f = 0; f < 3; ++f) pi[slot * 3 + f] = iv[f];
  }
}

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void objective_final_kernel(int64_t n, int64_t k, int nb,
                                                                const double *__restrict__ pd,
                                                                const int64_t *__restrict__ pi,
                                                                cps_eval *__restrict__ out) {
  __shared__ double sd[8][BLOCK / kWave];
  __shared__ int64_t si[8][BLOCK / kWave];
  const int64_t y = blockIdx.x;
  double dv[8] = {0, 0, -__builtin_inf(), __builtin_inf(), 0, 0, 0, 0};
  int dop[8] = {0, 0, 2, 1, 0, 0, 0, 0};
  int64_t iv[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (int b = threadIdx.x; b < nb; b += BLOCK) {
    const int64_t slot = y * nb + b;
    dv[0] += pd[slot * 4 + 0];
    dv[1] += pd[slot * 4 + 1];
    dv[2] = fmax(dv[2], pd[slot * 4 + 2]);
    dv[3] = fmin(dv[3], pd[slot * 4 + 3]);
    iv[0] += pi[slot * 3 + 0];
    iv[1] += pi[slot * 3 + 1];
    iv[2] += pi[slot * 3 + 2];
  }
  block_reduce<BLOCK, 4, 3>(dv, dop, iv, false, sd, si);
  if (threadIdx.x == 0) {
    const double alpha = (double)k - 0.5, beta = (double)n - (double)k + 0.5;
    cps_eval e;
    e.A = dv[0];
    e.B = dv[1];
    e.f = alpha * dv[0] + beta * dv[1];
    e.L = iv[0];
    e.E = iv[1];
    e.G = iv[2];
    e.pred = dv[2];
    e.succ = dv[3];
    e.gminus = (double)n * ((double)iv[0] - (double)k + 0.5);
    e.gplus = (double)n * ((double)(iv[0] + iv[1]) - (double)k + 0.5);
    out[y] = e;
  }
}

// ------------------------------------------------------------------ launchers

template <typename T>
hipError_t launch_select(const SelectArgs<T> &a, int grid, bool cooperative, hipStream_t stream) {
  // The grid never exceeds the workgroups that fit at once (one per CU), so an ordinary launch
  // on a GPU not running another grid-synchronising kernel has them all resident; the
  // cooperative launch guarantees it in every case but costs ~17 us more per call (measured:
  // an empty kernel takes ~2.5 us per ordinary launch and ~20 us per cooperative one).
  if (!cooperative) {
    cp_select_kernel<T, kSelectBlock, kSelectUnroll><<<dim3(grid), dim3(kSelectBlock), 0, stream>>>(a);
    return hipGetLastError();
  }
  SelectArgs<T> copy = a;
  void *args[] = {&copy};
  return hipLaunchCooperativeKernel((const void *)cp_select_kernel<T, kSelectBlock, kSelectUnroll>,
                                    dim3(grid), dim3(kSelectBlock), args, 0, stream);
}

template <typename T> int select_max_blocks_per_cu() {
  int nb = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(
          &nb, cp_select_kernel<T, kSelectBlock, kSelectUnroll>, kSelectBlock, 0) != hipSuccess)
    return 0;
  return nb;
}

template <typename T>
hipError_t launch_objective(const T *x, int64_t n, int64_t k, const double *ys, int64_t ny,
                            cps_eval *out, double *pd, int64_t *pi, int nb, hipStream_t stream) {
  constexpr int BLOCK = 256;
  objective_partial_kernel<T, BLOCK><<<dim3(nb, (unsigned)ny), dim3(BLOCK), 0, stream>>>(x, n, ys, pd, pi);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  objective_final_kernel<BLOCK><<<dim3((unsigned)ny), dim3(BLOCK), 0, stream>>>(n, k, nb, pd, pi, out);
  return hipGetLastError();
}

template hipError_t launch_select<float>(const SelectArgs<float> &, int, bool, hipStream_t);
template hipError_t launch_select<double>(const SelectArgs<double> &, int, bool, hipStream_t);
template int select_max_blocks_per_cu<float>();
template int select_max_blocks_per_cu<double>();
template hipError_t launch_objective<float>(const float *, int64_t, int64_t, const double *,
                                            int64_t, cps_eval *, double *, int64_t *, int,
                                            hipStream_t);
template hipError_t launch_objective<double>(const double *, int64_t, int64_t, const double *,
                                             int64_t, cps_eval *, double *, int64_t *, int,
                                             hipStream_t);

}  // namespace cps
