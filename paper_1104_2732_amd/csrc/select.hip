// Exact k-th element selection by Kelley's cutting plane, single array, one launch.
//
// One persistent kernel runs every pass of the method (Section 4, Algorithm 1 and the
// hybrid that ends it):
//   pass 0      min, max (with multiplicities), sum and NaN/infinity counts of x in one
//               reduction (step 0), optionally with the two-point check of a proposed
//               bracket;
//   eval passes A(t), B(t), #(w<t), #(w>t), largest w<t and smallest w>t over the working
//               set at the trial point t (the objective and subgradient of Section 3 in
//               one fused reduction); once the bracket is small the same pass splits the
//               bracket's elements at t into a workspace buffer (count-and-compact);
//   final       one workgroup selects the remaining rank exactly (radix select on the
//               ordered keys), in place of the paper's sort of the compacted array.
// Between passes the grid synchronises through an arrival counter; the last workgroup
// to arrive reduces the per-workgroup partials in a fixed order and advances the
// cutting-plane state (cp_state.h), so no pass needs the host.  The kernel is launched
// cooperatively, which guarantees that every workgroup is resident.
#include "cps_device.h"
#include "cps_kernels.h"

namespace cps {

// The scalar cutting-plane update runs in one thread per pass; keeping it out of line
// keeps its registers out of the streaming loops' budget.
__device__ __noinline__ void dev_after_pass0(CpState &s, const Pass0Result &r, const CpConfig &c) {
  cp_after_pass0(s, r, c);
}
__device__ __noinline__ void dev_after_eval(CpState &s, const EvalResult &r, const CpConfig &c) {
  cp_after_eval(s, r, c);
}

// ------------------------------------------------------------------ per-element work

template <typename T> struct EvalAcc {
  double A, B;
  T pred, succ;
  uint64_t L, G;  // wave-uniform
};

template <typename T> __device__ inline T t_inf();
template <> __device__ inline float t_inf<float>() { return __builtin_inff(); }
template <> __device__ inline double t_inf<double>() { return __builtin_inf(); }

template <typename T> __device__ inline T tmin(T a, T b) { return a < b ? a : b; }
template <typename T> __device__ inline T tmax(T a, T b) { return a > b ? a : b; }

// Evaluate one loaded vector at t.  Invalid lanes contribute nothing.
template <typename T, bool CLAMP>
__device__ inline void eval_vec(T (&e)[Traits<T>::kVec], bool valid, T t, T fmin, T fmax,
                                EvalAcc<T> &acc) {
  constexpr int V = Traits<T>::kVec;
  T a_part = 0, b_part = 0;
#pragma unroll
  for (int j = 0; j < V; ++j) {
    T v = e[j];
    if (CLAMP) {
      v = tmin(tmax(v, fmin), fmax);
      e[j] = v;
    }
    const bool l = valid && (v < t);
    const bool g = valid && (v > t);
    const T d = v - t;
    a_part += g ? d : T(0);
    b_part -= l ? d : T(0);
    acc.pred = tmax(acc.pred, l ? v : -t_inf<T>());
    acc.succ = tmin(acc.succ, g ? v : t_inf<T>());
    acc.L += popc(ballot(l));
    acc.G += popc(ballot(g));
  }
  acc.A += (double)a_part;
  acc.B += (double)b_part;
}

template <typename T> struct P0Acc {
  double sum;
  T mn, mx;
  uint32_t cmn, cmx;
  uint64_t nnan, nneg, npos;  // wave-uniform
  uint64_t cle_a, clt_b;      // wave-uniform
  double Aa, Ba, Ab, Bb;
};

template <typename T, bool BRACKET>
__device__ inline void pass0_vec(const T (&e)[Traits<T>::kVec], bool valid, T ba, T bb,
                                 P0Acc<T> &acc) {
  constexpr int V = Traits<T>::kVec;
  T s_part = 0;
  T aa = 0, bA = 0, ab = 0, bB = 0;
#pragma unroll
  for (int j = 0; j < V; ++j) {
    const T v = e[j];
    const bool isnan_ = valid && (v != v);
    const bool ni = valid && (v == -t_inf<T>());
    const bool pi = valid && (v == t_inf<T>());
    const bool fin = valid && !isnan_ && !ni && !pi;
    if (fin && v < acc.mn) { acc.mn = v; acc.cmn = 1u; }
    else if (fin && v == acc.mn) { acc.cmn++; }
    if (fin && v > acc.mx) { acc.mx = v; acc.cmx = 1u; }
    else if (fin && v == acc.mx) { acc.cmx++; }
    s_part += fin ? v : T(0);
    acc.nnan += popc(ballot(isnan_));
    acc.nneg += popc(ballot(ni));
    acc.npos += popc(ballot(pi));
    if (BRACKET) {
      acc.cle_a += popc(ballot(valid && v <= ba));
      acc.clt_b += popc(ballot(valid && v < bb));
      aa += (fin && v > ba) ? v - ba : T(0);
      bA += (fin && v < ba) ? ba - v : T(0);
      ab += (fin && v > bb) ? v - bb : T(0);
      bB += (fin && v < bb) ? bb - v : T(0);
    }
  }
  acc.sum += (double)s_part;
  if (BRACKET) {
    acc.Aa += (double)aa;
    acc.Ba += (double)bA;
    acc.Ab += (double)ab;
    acc.Bb += (double)bB;
  }
}

// ------------------------------------------------------------------ working-set geometry

template <typename T> struct Span {
  const typename Traits<T>::Vec *V;  // aligned body
  const T *W;
  int64_t m, head, nvec, tail_start, nedge;
};

template <typename T> __device__ inline Span<T> make_span(const T *W, int64_t m) {
  Span<T> s;
  s.W = W;
  s.m = m;
  const uintptr_t addr = (uintptr_t)W;
  int64_t head = (int64_t)(((16u - (addr & 15u)) & 15u) / sizeof(T));
  if (head > m) head = m;
  s.head = head;
  s.V = reinterpret_cast<const typename Traits<T>::Vec *>(W + head);
  s.nvec = (m - head) / Traits<T>::kVec;
  s.tail_start = head + s.nvec * Traits<T>::kVec;
  s.nedge = head + (m - s.tail_start);
  return s;
}

// Edge element i (< nedge): the unaligned head, then the tail.
template <typename T> __device__ inline int64_t edge_index(const Span<T> &s, int64_t i) {
  return i < s.head ? i : s.tail_start + (i - s.head);
}

// ------------------------------------------------------------------ kernel

template <typename T, int BLOCK, int UNROLL> struct Shared {
  CpState st;
  double d[8][BLOCK / kWave];
  int64_t i[8][BLOCK / kWave];
  uint64_t wbase[2][BLOCK / kWave];
  uint32_t wcnt[2][BLOCK / kWave];
  uint32_t hist[256];
  int64_t misc[8];
  int last;
};

template <typename T, int BLOCK>
__device__ inline void wave_pair_min(T &m, uint32_t &c) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
    T m2 = __shfl_xor(m, o);
    uint32_t c2 = __shfl_xor(c, o);
    if (m2 < m) { m = m2; c = c2; }
    else if (m2 == m) { c += c2; }
  }
}
template <typename T, int BLOCK>
__device__ inline void wave_pair_max(T &m, uint32_t &c) {
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
    T m2 = __shfl_xor(m, o);
    uint32_t c2 = __shfl_xor(c, o);
    if (m2 > m) { m = m2; c = c2; }
    else if (m2 == m) { c += c2; }
  }
}

// Split the tile's elements: those in (lo_ex, t) go up from the start of zout, those in
// (t, hi_ex) go down from its end (FILTER: the working set is the whole input, so the
// bracket ends are checked too; otherwise every element is inside the bracket).
// Offsets come from one atomic per side per tile; within a wave the elements of one
// slot are written contiguously.
template <typename T, bool FILTER>
__device__ inline bool goes_left(T v, bool valid, T t, T lo_ex) {
  return valid && v < t && (!FILTER || v > lo_ex);
}
template <typename T, bool FILTER>
__device__ inline bool goes_right(T v, bool valid, T t, T hi_ex) {
  return valid && v > t && (!FILTER || v < hi_ex);
}

template <typename T, int BLOCK, int UNROLL, bool FILTER, bool EDGE = false>
__device__ inline void split_tile(T (&e)[UNROLL][Traits<T>::kVec], const bool (&valid)[UNROLL],
                                  T t, T lo_ex, T hi_ex, T *__restrict__ zout, int64_t zcap,
                                  SyncCtl *sync, Shared<T, BLOCK, UNROLL> &sh, int64_t &written) {
  constexpr int V = Traits<T>::kVec;
  const int tid = threadIdx.x, wv = tid / kWave, lane = tid % kWave;
  uint32_t wl = 0, wr = 0;
#pragma unroll
  for (int u = 0; u < UNROLL; ++u)
#pragma unroll
    for (int j = 0; j < V; ++j) {
      if (EDGE && (u > 0 || j > 0)) continue;  // edge tiles hold one element per thread
      wl += popc(ballot(goes_left<T, FILTER>(e[u][j], valid[u], t, lo_ex)));
      wr += popc(ballot(goes_right<T, FILTER>(e[u][j], valid[u], t, hi_ex)));
    }
  if (lane == 0) {
    sh.wcnt[0][wv] = wl;
    sh.wcnt[1][wv] = wr;
  }
  __syncthreads();
  if (tid == 0) {
    uint64_t tl = 0, tr = 0;
    for (int w = 0; w < BLOCK / kWave; ++w) {
      sh.wbase[0][w] = tl;
      tl += sh.wcnt[0][w];
      sh.wbase[1][w] = tr;
      tr += sh.wcnt[1][w];
    }
    const uint64_t bl = tl ? atomic_add_relaxed(&sync->curL, tl) : 0;
    const uint64_t br = tr ? atomic_add_relaxed(&sync->curR, tr) : 0;
    for (int w = 0; w < BLOCK / kWave; ++w) {
      sh.wbase[0][w] += bl;
      sh.wbase[1][w] += br;
    }
    written += (int64_t)(tl + tr);
  }
  __syncthreads();
  // recompute the side tests below instead of keeping 2 x UNROLL x V lane masks alive
#pragma unroll
  for (int u = 0; u < UNROLL; ++u)
#pragma unroll
    for (int j = 0; j < V; ++j) asm volatile("" : "+v"(e[u][j]));
  uint64_t ol = sh.wbase[0][wv], orr = sh.wbase[1][wv];
#pragma unroll
  for (int u = 0; u < UNROLL; ++u)
#pragma unroll
    for (int j = 0; j < V; ++j) {
      if (EDGE && (u > 0 || j > 0)) continue;
      const bool l = goes_left<T, FILTER>(e[u][j], valid[u], t, lo_ex);
      const uint64_t ml = ballot(l);
      if (l) zout[ol + lane_rank(ml)] = e[u][j];
      ol += popc(ml);
      const bool r = goes_right<T, FILTER>(e[u][j], valid[u], t, hi_ex);
      const uint64_t mr = ballot(r);
      if (r) zout[zcap - 1 - (int64_t)(orr + lane_rank(mr))] = e[u][j];
      orr += popc(mr);
    }
  __syncthreads();
}

// One evaluation pass over this workgroup's tiles of the working set.
template <typename T, int BLOCK, int UNROLL, bool CLAMP, bool SPLIT, bool FILTER>
__device__ void eval_pass(const Span<T> &sp, T t, T yL, T yR, T fmin, T fmax, T *zout,
                          int64_t zcap, SyncCtl *sync, Shared<T, BLOCK, UNROLL> &sh,
                          EvalAcc<T> &acc, int64_t &written) {
  constexpr int V = Traits<T>::kVec;
  using Vec = typename Traits<T>::Vec;
  const int tid = threadIdx.x;
  const int G = gridDim.x, bid = blockIdx.x;
  const int64_t tile_vecs = (int64_t)BLOCK * UNROLL;
  const int64_t ntiles = (sp.nvec + tile_vecs - 1) / tile_vecs;
  for (int64_t ti = bid; ti < ntiles; ti += G) {
    const int64_t base = ti * tile_vecs;
    T e[UNROLL][V];
    bool valid[UNROLL];
    Vec raw[UNROLL];
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) {
      const int64_t vi = base + (int64_t)u * BLOCK + tid;
      valid[u] = vi < sp.nvec;
      if (valid[u]) raw[u] = sp.V[vi];
    }
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) {
      vec_to_arr<T>(raw[u], e[u]);
      eval_vec<T, CLAMP>(e[u], valid[u], t, fmin, fmax, acc);
    }
    if (SPLIT) split_tile<T, BLOCK, UNROLL, FILTER>(e, valid, t, yL, yR, zout, zcap, sync, sh, written);
  }
  // unaligned head and tail elements: the last workgroup takes them as one partial tile,
  // one element per thread in slot (0, 0)
  if (sp.nedge > 0 && bid == G - 1) {
    T e[UNROLL][V];
    bool valid[UNROLL];
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) {
      valid[u] = false;
#pragma unroll
      for (int j = 0; j < V; ++j) e[u][j] = T(0);
    }
    const bool have = tid < sp.nedge;
    T v = have ? sp.W[edge_index(sp, tid)] : T(0);
    if (CLAMP) v = tmin(tmax(v, fmin), fmax);
    const bool l = have && v < t, g = have && v > t;
    const T d = v - t;
    acc.A += g ? (double)d : 0.0;
    acc.B += l ? -(double)d : 0.0;
    acc.pred = tmax(acc.pred, l ? v : -t_inf<T>());
    acc.succ = tmin(acc.succ, g ? v : t_inf<T>());
    acc.L += popc(ballot(l));
    acc.G += popc(ballot(g));
    if (SPLIT) {
      e[0][0] = v;
      valid[0] = have;
      split_tile<T, BLOCK, UNROLL, FILTER, true>(e, valid, t, yL, yR, zout, zcap, sync, sh, written);
    }
  }
}

template <typename T, int BLOCK, int UNROLL, bool BRACKET>
__device__ void pass0(const Span<T> &sp, T ba, T bb, P0Acc<T> &acc) {
  constexpr int V = Traits<T>::kVec;
  using Vec = typename Traits<T>::Vec;
  const int tid = threadIdx.x;
  const int G = gridDim.x, bid = blockIdx.x;
  const int64_t tile_vecs = (int64_t)BLOCK * UNROLL;
  const int64_t ntiles = (sp.nvec + tile_vecs - 1) / tile_vecs;
  for (int64_t ti = bid; ti < ntiles; ti += G) {
    const int64_t base = ti * tile_vecs;
    Vec raw[UNROLL];
    bool valid[UNROLL];
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) {
      const int64_t vi = base + (int64_t)u * BLOCK + tid;
      valid[u] = vi < sp.nvec;
      if (valid[u]) raw[u] = sp.V[vi];
    }
#pragma unroll
    for (int u = 0; u < UNROLL; ++u) {
      T e[V];
      vec_to_arr<T>(raw[u], e);
      pass0_vec<T, BRACKET>(e, valid[u], ba, bb, acc);
    }
  }
  if (sp.nedge > 0 && bid == G - 1) {
    // unaligned head and tail elements, one per thread of the last workgroup
    const bool have = tid < sp.nedge;
    const T v = have ? sp.W[edge_index(sp, tid)] : T(0);
    const bool isnan_ = have && (v != v);
    const bool ni = have && (v == -t_inf<T>());
    const bool pi = have && (v == t_inf<T>());
    const bool fin = have && !isnan_ && !ni && !pi;
    if (fin && v < acc.mn) { acc.mn = v; acc.cmn = 1u; }
    else if (fin && v == acc.mn) { acc.cmn++; }
    if (fin && v > acc.mx) { acc.mx = v; acc.cmx = 1u; }
    else if (fin && v == acc.mx) { acc.cmx++; }
    acc.sum += fin ? (double)v : 0.0;
    acc.nnan += popc(ballot(isnan_));
    acc.nneg += popc(ballot(ni));
    acc.npos += popc(ballot(pi));
    if (BRACKET) {
      acc.cle_a += popc(ballot(have && v <= ba));
      acc.clt_b += popc(ballot(have && v < bb));
      acc.Aa += (fin && v > ba) ? (double)(v - ba) : 0.0;
      acc.Ba += (fin && v < ba) ? (double)(ba - v) : 0.0;
      acc.Ab += (fin && v > bb) ? (double)(v - bb) : 0.0;
      acc.Bb += (fin && v < bb) ? (double)(bb - v) : 0.0;
    }
  }
}

// Block reduction of up to 8 double fields (op per field: 0 sum, 1 min, 2 max) and
// 8 int64 sums.  The int fields are either per-thread or wave-uniform (`iuniform`).
// The result is valid in thread 0.  Fixed order, hence deterministic.
template <int BLOCK, int ND, int NI>
__device__ inline void block_reduce(double (&dv)[8], const int (&dop)[8], int64_t (&iv)[8],
                                    bool iuniform, double (&sd)[8][BLOCK / kWave],
                                    int64_t (&si)[8][BLOCK / kWave]) {
  const int tid = threadIdx.x, wv = tid / kWave, lane = tid % kWave;
#pragma unroll
  for (int f = 0; f < ND; ++f) {
    if (dop[f] == 0) dv[f] = wave_sum(dv[f]);
    else if (dop[f] == 1) dv[f] = wave_min(dv[f]);
    else dv[f] = wave_max(dv[f]);
  }
  if (!iuniform) {
#pragma unroll
    for (int f = 0; f < NI; ++f) iv[f] = wave_sum_i64(iv[f]);
  }
  if (lane == 0) {
#pragma unroll
    for (int f = 0; f < ND; ++f) sd[f][wv] = dv[f];
#pragma unroll
    for (int f = 0; f < NI; ++f) si[f][wv] = iv[f];
  }
  __syncthreads();
  if (tid == 0) {
#pragma unroll
    for (int f = 0; f < ND; ++f) {
      double r = sd[f][0];
      for (int w = 1; w < BLOCK / kWave; ++w) {
        const double x = sd[f][w];
        r = dop[f] == 0 ? r + x : (dop[f] == 1 ? fmin(r, x) : fmax(r, x));
      }
      dv[f] = r;
    }
#pragma unroll
    for (int f = 0; f < NI; ++f) {
      int64_t r = 0;
      for (int w = 0; w < BLOCK / kWave; ++w) r += si[f][w];
      iv[f] = r;
    }
  }
  __syncthreads();
}

// Fold (min, multiplicity) and (max, multiplicity) pairs over the workgroup; valid in
// thread 0.
template <int BLOCK>
__device__ inline void block_pair_fold(double &mn, int64_t &cmn, double &mx, int64_t &cmx,
                                       double (&sd)[8][BLOCK / kWave],
                                       int64_t (&si)[8][BLOCK / kWave]) {
  const int tid = threadIdx.x, wv = tid / kWave, lane = tid % kWave;
#pragma unroll
  for (int o = kWave / 2; o > 0; o >>= 1) {
    const double m2 = __shfl_xor(mn, o), x2 = __shfl_xor(mx, o);
    const int64_t c2 = __shfl_xor(cmn, o), d2 = __shfl_xor(cmx, o);
    if (m2 < mn) { mn = m2; cmn = c2; } else if (m2 == mn) cmn += c2;
    if (x2 > mx) { mx = x2; cmx = d2; } else if (x2 == mx) cmx += d2;
  }
  if (lane == 0) {
    sd[0][wv] = mn; si[0][wv] = cmn; sd[1][wv] = mx; si[1][wv] = cmx;
  }
  __syncthreads();
  if (tid == 0) {
    mn = sd[0][0]; cmn = si[0][0]; mx = sd[1][0]; cmx = si[1][0];
    for (int w = 1; w < BLOCK / kWave; ++w) {
      if (sd[0][w] < mn) { mn = sd[0][w]; cmn = si[0][w]; } else if (sd[0][w] == mn) cmn += si[0][w];
      if (sd[1][w] > mx) { mx = sd[1][w]; cmx = si[1][w]; } else if (sd[1][w] == mx) cmx += si[1][w];
    }
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

template <typename T, int BLOCK, int UNROLL>
__global__ __launch_bounds__(BLOCK) void cp_select_kernel(SelectArgs<T> a) {
  __shared__ Shared<T, BLOCK, UNROLL> sh;
  const int tid = threadIdx.x;
  const int G = gridDim.x, bid = blockIdx.x;
  uint32_t gen = 0;
  if (tid == 0) {
    gen = load_acquire(&a.sync->gen);
    if (bid == 0) {
      // a pending record; overwritten on completion, left in place if a wait times out
      cps_result r = {};
      r.status = ST_TIMEOUT;
      *a.out = r;
    }
  }
  const bool use_br = a.cfg.use_bracket != 0;
  const T ba = (T)a.cfg.bracket_lo, bb = (T)a.cfg.bracket_hi;
  int phase = PH_PASS0;
  for (;;) {
    double dv[8];
    int64_t iv[8];
    int dop[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (phase == PH_PASS0) {
      const Span<T> sp = make_span(a.x, a.n);
      P0Acc<T> acc;
      acc.sum = 0;
      acc.mn = t_inf<T>();
      acc.mx = -t_inf<T>();
      acc.cmn = acc.cmx = 0;
      acc.nnan = acc.nneg = acc.npos = acc.cle_a = acc.clt_b = 0;
      acc.Aa = acc.Ba = acc.Ab = acc.Bb = 0;
      if (use_br) pass0<T, BLOCK, UNROLL, true>(sp, ba, bb, acc);
      else pass0<T, BLOCK, UNROLL, false>(sp, ba, bb, acc);
      wave_pair_min<T, BLOCK>(acc.mn, acc.cmn);
      wave_pair_max<T, BLOCK>(acc.mx, acc.cmx);
      // fold the (min, count) pairs across waves through LDS
      const int wv = tid / kWave, lane = tid % kWave;
      if (lane == 0) {
        sh.d[0][wv] = (double)acc.mn;
        sh.i[0][wv] = acc.cmn;
        sh.d[1][wv] = (double)acc.mx;
        sh.i[1][wv] = acc.cmx;
      }
      __syncthreads();
      double mn = 0, mx = 0;
      int64_t cmn = 0, cmx = 0;
      if (tid == 0) {
        mn = sh.d[0][0]; cmn = sh.i[0][0]; mx = sh.d[1][0]; cmx = sh.i[1][0];
        for (int w = 1; w < BLOCK / kWave; ++w) {
          if (sh.d[0][w] < mn) { mn = sh.d[0][w]; cmn = sh.i[0][w]; }
          else if (sh.d[0][w] == mn) cmn += sh.i[0][w];
          if (sh.d[1][w] > mx) { mx = sh.d[1][w]; cmx = sh.i[1][w]; }
          else if (sh.d[1][w] == mx) cmx += sh.i[1][w];
        }
      }
      __syncthreads();
      dv[0] = acc.sum; dv[1] = acc.Aa; dv[2] = acc.Ba; dv[3] = acc.Ab; dv[4] = acc.Bb;
      dv[5] = dv[6] = dv[7] = 0;
      iv[0] = (int64_t)acc.nnan; iv[1] = (int64_t)acc.nneg; iv[2] = (int64_t)acc.npos;
      iv[3] = (int64_t)acc.cle_a; iv[4] = (int64_t)acc.clt_b;
      iv[5] = iv[6] = iv[7] = 0;
      block_reduce<BLOCK, 5, 5>(dv, dop, iv, true, sh.d, sh.i);
      if (tid == 0) {
        dv[5] = mn; dv[6] = mx; iv[5] = cmn; iv[6] = cmx;
      }
    } else {
      const CpState &s = sh.st;
      const T t = (T)s.t, yL = (T)s.yL, yR = (T)s.yR, fmn = (T)s.fmin, fmx = (T)s.fmax;
      const T *W = s.wbuf < 0 ? a.x : (a.z[s.wbuf] + s.woff);
      const Span<T> sp = make_span(W, s.wlen);
      T *zout = a.z[s.zout];
      EvalAcc<T> acc;
      acc.A = acc.B = 0;
      acc.pred = -t_inf<T>();
      acc.succ = t_inf<T>();
      acc.L = acc.G = 0;
      int64_t written = 0;
      const bool clamp = s.has_inf && s.wbuf < 0;
      if (!s.split) {
        if (clamp) eval_pass<T, BLOCK, UNROLL, true, false, false>(sp, t, yL, yR, fmn, fmx, zout, a.cfg.zcap, a.sync, sh, acc, written);
        else eval_pass<T, BLOCK, UNROLL, false, false, false>(sp, t, yL, yR, fmn, fmx, zout, a.cfg.zcap, a.sync, sh, acc, written);
      } else if (s.filter) {
        if (clamp) eval_pass<T, BLOCK, UNROLL, true, true, true>(sp, t, yL, yR, fmn, fmx, zout, a.cfg.zcap, a.sync, sh, acc, written);
        else eval_pass<T, BLOCK, UNROLL, false, true, true>(sp, t, yL, yR, fmn, fmx, zout, a.cfg.zcap, a.sync, sh, acc, written);
      } else {
        eval_pass<T, BLOCK, UNROLL, false, true, false>(sp, t, yL, yR, fmn, fmx, zout, a.cfg.zcap, a.sync, sh, acc, written);
      }
      dv[0] = acc.A; dv[1] = acc.B; dv[2] = (double)acc.pred; dv[3] = (double)acc.succ;
      dop[2] = 2; dop[3] = 1;
      dv[4] = dv[5] = dv[6] = dv[7] = 0;
      iv[0] = (int64_t)acc.L; iv[1] = (int64_t)acc.G;
      iv[2] = iv[3] = iv[4] = iv[5] = iv[6] = iv[7] = 0;
      block_reduce<BLOCK, 4, 2>(dv, dop, iv, true, sh.d, sh.i);
      if (tid == 0) iv[2] = written;  // thread 0 counted the block's writes
    }

    // ---- publish this workgroup's partial and arrive
    const int64_t stride = a.slot_stride;
    if (tid == 0) {
#pragma unroll
      for (int f = 0; f < 8; ++f) {
        a.sd[f * stride + bid] = dv[f];
        a.si[f * stride + bid] = iv[f];
      }
      const uint32_t prev = atomic_add_acq_rel(&a.sync->arrive, 1u);
      sh.last = (prev == (uint32_t)(G - 1));
    }
    __syncthreads();

    if (sh.last) {
      fence_acquire();
      // ---- reduce every workgroup's partial in a fixed order
      double rd[8];
      int64_t ri[8];
      int rop[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      if (phase == PH_PASS0) {
        for (int f = 0; f < 8; ++f) { rd[f] = 0; ri[f] = 0; }
        for (int b = tid; b < G; b += BLOCK) {
          for (int f = 0; f < 5; ++f) rd[f] += a.sd[f * stride + b];
          for (int f = 0; f < 5; ++f) ri[f] += a.si[f * stride + b];
        }
        block_reduce<BLOCK, 5, 5>(rd, rop, ri, false, sh.d, sh.i);
        // (min, count) and (max, count) pairs: strided fold per thread, then a fixed tree
        double mn = __builtin_inf(), mx = -__builtin_inf();
        int64_t cmn = 0, cmx = 0;
        for (int b = tid; b < G; b += BLOCK) {
          const double m2 = a.sd[5 * stride + b], x2 = a.sd[6 * stride + b];
          const int64_t c2 = a.si[5 * stride + b], d2 = a.si[6 * stride + b];
          if (m2 < mn) { mn = m2; cmn = c2; } else if (m2 == mn) cmn += c2;
          if (x2 > mx) { mx = x2; cmx = d2; } else if (x2 == mx) cmx += d2;
        }
        block_pair_fold<BLOCK>(mn, cmn, mx, cmx, sh.d, sh.i);
        if (tid == 0) {
          Pass0Result r;
          r.sum = rd[0]; r.A_a = rd[1]; r.B_a = rd[2]; r.A_b = rd[3]; r.B_b = rd[4];
          r.nnan = ri[0]; r.nneg = ri[1]; r.npos = ri[2]; r.c_le_a = ri[3]; r.c_lt_b = ri[4];
          r.fmin = mn; r.fmax = mx; r.cmin = cmn; r.cmax = cmx;
          CpState &s = sh.st;
          s = CpState{};
          s.n = a.n;
          s.k = a.k;
          s.phase = PH_PASS0;
          dev_after_pass0(s, r, a.cfg);
          if (a.stats) {
            a.stats->population[0] = s.cR - s.cL;
            a.stats->working[0] = a.n;
          }
        }
      } else {
        rop[2] = 2; rop[3] = 1;
        for (int f = 0; f < 8; ++f) { rd[f] = 0; ri[f] = 0; }
        rd[2] = -__builtin_inf();
        rd[3] = __builtin_inf();
        for (int b = tid; b < G; b += BLOCK) {
          rd[0] += a.sd[0 * stride + b];
          rd[1] += a.sd[1 * stride + b];
          rd[2] = fmax(rd[2], a.sd[2 * stride + b]);
          rd[3] = fmin(rd[3], a.sd[3 * stride + b]);
          ri[0] += a.si[0 * stride + b];
          ri[1] += a.si[1 * stride + b];
          ri[2] += a.si[2 * stride + b];
        }
        block_reduce<BLOCK, 4, 3>(rd, rop, ri, false, sh.d, sh.i);
        if (tid == 0) {
          EvalResult r;
          r.A = rd[0]; r.B = rd[1]; r.pred = rd[2]; r.succ = rd[3];
          r.L = ri[0]; r.G = ri[1]; r.written = ri[2];
          CpState &s = sh.st;
          const int64_t wl = s.wlen;
          dev_after_eval(s, r, a.cfg);
          const int p = s.work_passes - 1;
          if (a.stats && p < CPS_STATS_MAX_PASSES) {
            a.stats->population[p] = s.phase == PH_DONE ? 0 : s.cR - s.cL;
            a.stats->working[p] = wl;
          }
        }
      }
      __syncthreads();
      // ---- exact finish in this workgroup when the bracket is small
      if (sh.st.phase == PH_FINAL) {
        const CpState &s = sh.st;
        const T *W = s.wbuf < 0 ? a.x : (a.z[s.wbuf] + s.woff);
        typename Traits<T>::Key key;
        int64_t below, eq;
        block_radix_select<T, BLOCK>(W, s.wlen, !s.on_bracket, (T)s.yL, (T)s.yR, s.k - s.cL,
                                     sh.hist, sh.misc, key, below, eq);
        if (tid == 0) {
          CpState &w = sh.st;
          w.work_passes++;
          w.elements_read += w.wlen;
          if (w.wbuf < 0) w.passes++;
          cp_finish(w, (double)Traits<T>::unkey(key), w.cL + below, eq);
        }
        __syncthreads();
      }
      // publish the new state: every thread copies words, each wave releases its stores
      constexpr int NW = sizeof(CpState) / 8;
      for (int w = tid; w < NW; w += BLOCK)
        reinterpret_cast<uint64_t *>(a.st)[w] = reinterpret_cast<const uint64_t *>(&sh.st)[w];
      if (tid == 0) {
        const CpState &s = sh.st;
        if (s.phase == PH_DONE) write_result<T>(a, s);
        if (s.split) {
          a.sync->curL = 0;
          a.sync->curR = 0;
        }
      }
      fence_release();
      __syncthreads();
      if (tid == 0) {
        store_relaxed(&a.sync->arrive, 0u);
        store_release(&a.sync->gen, gen + 1u);
        gen = gen + 1u;
      }
    } else {
      if (tid == 0) {
        int64_t spins = 0;
        bool timed_out = false;
        while (load_acquire(&a.sync->gen) == gen) {
          __builtin_amdgcn_s_sleep(2);
          if (++spins > a.spin_limit) { timed_out = true; break; }
        }
        sh.misc[7] = timed_out ? 1 : 0;
        if (!timed_out) gen = gen + 1u;
      }
      __syncthreads();
      if (sh.misc[7]) {
        if (tid == 0) {
          sh.st.phase = PH_DONE;
          sh.st.status = ST_TIMEOUT;
        }
      } else {
        // read the state the last workgroup published
        fence_acquire();
        constexpr int NW = sizeof(CpState) / 8;
        for (int w = tid; w < NW; w += BLOCK)
          reinterpret_cast<uint64_t *>(&sh.st)[w] = reinterpret_cast<const uint64_t *>(a.st)[w];
      }
    }
    __syncthreads();
    phase = sh.st.phase;
    if (phase == PH_DONE) break;
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
hipError_t launch_select(const SelectArgs<T> &a, int grid, hipStream_t stream) {
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

template hipError_t launch_select<float>(const SelectArgs<float> &, int, hipStream_t);
template hipError_t launch_select<double>(const SelectArgs<double> &, int, hipStream_t);
template int select_max_blocks_per_cu<float>();
template int select_max_blocks_per_cu<double>();
template hipError_t launch_objective<float>(const float *, int64_t, int64_t, const double *,
                                            int64_t, cps_eval *, double *, int64_t *, int,
                                            hipStream_t);
template hipError_t launch_objective<double>(const double *, int64_t, int64_t, const double *,
                                             int64_t, cps_eval *, double *, int64_t *, int,
                                             hipStream_t);

}  // namespace cps
