// Per-element evaluation, pass-0 reduction, working-set geometry and workgroup
// reductions shared by the single-array and the batched selection kernels.
#pragma once

#include "cps_device.h"

namespace cps {

// ------------------------------------------------------------------ per-element work

template <typename T> __device__ inline T t_inf();
template <> __device__ inline float t_inf<float>() { return __builtin_inff(); }
template <> __device__ inline double t_inf<double>() { return __builtin_inf(); }

template <typename T> __device__ inline T tmin(T a, T b) { return a < b ? a : b; }
template <typename T> __device__ inline T tmax(T a, T b) { return a > b ? a : b; }

// The counters are per lane (one VALU add-with-carry per element, no scalar work in the
// streaming loop); the workgroup reduction sums them.
template <typename T> struct EvalAcc {
  double A, B;
  T pred, succ;
  uint32_t L, G;
};

// Evaluate one element at t.  Invalid lanes contribute nothing.
template <typename T, bool CLAMP>
__device__ inline void eval_one(T &v, bool valid, T t, T fmin, T fmax, T &a_part, T &b_part,
                                EvalAcc<T> &acc) {
  if (CLAMP) v = tmin(tmax(v, fmin), fmax);
  const bool l = valid && (v < t);
  const bool g = valid && (v > t);
  const T d = v - t;
  a_part += g ? d : T(0);
  b_part -= l ? d : T(0);
  acc.pred = tmax(acc.pred, l ? v : -t_inf<T>());
  acc.succ = tmin(acc.succ, g ? v : t_inf<T>());
  acc.L += l ? 1u : 0u;
  acc.G += g ? 1u : 0u;
}

template <typename T> struct P0Acc {
  double sum;
  T mn, mx;
  uint32_t cmn, cmx;
  uint32_t nnan, nneg, npos;  // per lane
  uint32_t cle_a, clt_b;      // per lane
  double Aa, Ba, Ab, Bb;
};

// Pass 0 on one element.  CLASSIFY: count NaN and infinities and keep them out of the
// finite min, max and sum (the slow variant).  Otherwise nothing is classified: NaN makes
// the sum NaN and an infinity shows up as an infinite extreme (or a NaN sum), either of
// which makes the state machine ask for the slow variant.
// Minimum and maximum with their multiplicities, one element (fin: it takes part).
template <typename T> __device__ inline void p0_extremes(T v, bool fin, P0Acc<T> &acc) {
  const bool lt = fin && v < acc.mn, eqn = fin && v == acc.mn;
  acc.cmn = lt ? 1u : acc.cmn + (eqn ? 1u : 0u);
  acc.mn = lt ? v : acc.mn;
  const bool gt = fin && v > acc.mx, eqx = fin && v == acc.mx;
  acc.cmx = gt ? 1u : acc.cmx + (eqx ? 1u : 0u);
  acc.mx = gt ? v : acc.mx;
}

// SKIP_EXTREMES: the caller has established that no lane's element can change the running
// minimum or maximum or their counts (none is <= the minimum or >= the maximum).
// SUMS: with a proposed bracket, also the finite-element parts of A and B at its ends
// (otherwise only the two counts).
template <typename T, bool CLASSIFY, bool BRACKET, bool SKIP_EXTREMES = false, bool SUMS = true>
__device__ inline void pass0_one(T v, bool valid, T ba, T bb, T &aa, T &bA, T &ab,
                                 T &bB, P0Acc<T> &acc) {
  bool fin = valid;
  if (CLASSIFY) {
    const bool isnan_ = valid && (v != v);
    acc.nnan += isnan_ ? 1u : 0u;
    const bool ni = valid && (v == -t_inf<T>());
    const bool pi = valid && (v == t_inf<T>());
    acc.nneg += ni ? 1u : 0u;
    acc.npos += pi ? 1u : 0u;
    fin = valid && !isnan_ && !ni && !pi;
  }
  if (!SKIP_EXTREMES) p0_extremes<T>(v, fin, acc);
  acc.sum += fin ? (double)v : 0.0;  // widened per element: the sum is formed in double
  if (BRACKET) {
    acc.cle_a += (valid && v <= ba) ? 1u : 0u;
    acc.clt_b += (valid && v < bb) ? 1u : 0u;
    if (SUMS) {
      aa += (fin && v > ba) ? v - ba : T(0);
      bA += (fin && v < ba) ? ba - v : T(0);
      ab += (fin && v > bb) ? v - bb : T(0);
      bB += (fin && v < bb) ? bb - v : T(0);
    }
  }
}

// ------------------------------------------------------------------ working-set geometry

template <typename T> struct Span {
  const CPS_GLOBAL typename Traits<T>::Vec *V;  // aligned body
  const CPS_GLOBAL T *W;
  int64_t m, head, nvec, tail_start, nedge;
};

template <typename T> __device__ inline Span<T> make_span(const T *W, int64_t m) {
  Span<T> s;
  s.W = (const CPS_GLOBAL T *)W;
  s.m = m;
  const uintptr_t addr = (uintptr_t)W;
  int64_t head = (int64_t)(((16u - (addr & 15u)) & 15u) / sizeof(T));
  if (head > m) head = m;
  s.head = head;
  s.V = (const CPS_GLOBAL typename Traits<T>::Vec *)(W + head);
  s.nvec = (m - head) / Traits<T>::kVec;
  s.tail_start = head + s.nvec * Traits<T>::kVec;
  s.nedge = head + (m - s.tail_start);
  return s;
}

// Edge element i (< nedge): the unaligned head, then the tail.
template <typename T> __device__ inline int64_t edge_index(const Span<T> &s, int64_t i) {
  return i < s.head ? i : s.tail_start + (i - s.head);
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
  // one thread per field folds the wavefronts' values in wavefront order (fixed order,
  // and the fields in parallel), then thread 0 collects the results
  if (tid < ND) {
    const int f = tid;
    int op = 0;  // dop[f] by selects (an indexed read would move dop to scratch memory)
#pragma unroll
    for (int g = 0; g < ND; ++g) op = g == f ? dop[g] : op;
    double r = sd[f][0];
    for (int w = 1; w < BLOCK / kWave; ++w) {
      const double x = sd[f][w];
      r = op == 0 ? r + x : (op == 1 ? fmin(r, x) : fmax(r, x));
    }
    sd[f][0] = r;
  } else if (tid >= kWave && tid < kWave + NI) {
    const int f = tid - kWave;
    int64_t r = 0;
    for (int w = 0; w < BLOCK / kWave; ++w) r += si[f][w];
    si[f][0] = r;
  }
  __syncthreads();
  if (tid == 0) {
#pragma unroll
    for (int f = 0; f < ND; ++f) dv[f] = sd[f][0];
#pragma unroll
    for (int f = 0; f < NI; ++f) iv[f] = si[f][0];
  }
  __syncthreads();
}

// Fold (min, multiplicity) and (max, multiplicity) pairs over the wavefront: the extreme
// first, then the multiplicities of the lanes that hold it.  Every lane gets the result.
__device__ inline void wave_pair_fold(double &mn, int64_t &cmn, double &mx, int64_t &cmx) {
  const double wm = wave_min(mn), wx = wave_max(mx);
  cmn = wave_sum_i64(mn == wm ? cmn : 0);
  cmx = wave_sum_i64(mx == wx ? cmx : 0);
  mn = wm;
  mx = wx;
}

// Fold (min, multiplicity) and (max, multiplicity) pairs over the workgroup; valid in
// thread 0.
template <int BLOCK>
__device__ inline void block_pair_fold(double &mn, int64_t &cmn, double &mx, int64_t &cmx,
                                       double (&sd)[8][BLOCK / kWave],
                                       int64_t (&si)[8][BLOCK / kWave]) {
  const int tid = threadIdx.x, wv = tid / kWave, lane = tid % kWave;
  wave_pair_fold(mn, cmn, mx, cmx);
  if (lane == 0) {
    sd[0][wv] = mn; si[0][wv] = cmn; sd[1][wv] = mx; si[1][wv] = cmx;
  }
  __syncthreads();
  // the minimum in thread 0 and the maximum in the first thread of wavefront 1, in
  // wavefront order
  if (tid == 0) {
    mn = sd[0][0]; cmn = si[0][0];
    for (int w = 1; w < BLOCK / kWave; ++w) {
      if (sd[0][w] < mn) { mn = sd[0][w]; cmn = si[0][w]; } else if (sd[0][w] == mn) cmn += si[0][w];
    }
  } else if (tid == kWave) {
    double m = sd[1][0];
    int64_t c = si[1][0];
    for (int w = 1; w < BLOCK / kWave; ++w) {
      if (sd[1][w] > m) { m = sd[1][w]; c = si[1][w]; } else if (sd[1][w] == m) c += si[1][w];
    }
    sd[1][0] = m;
    si[1][0] = c;
  }
  __syncthreads();
  if (tid == 0) {
    mx = sd[1][0];
    cmx = si[1][0];
  }
  __syncthreads();
}

}  // namespace cps
