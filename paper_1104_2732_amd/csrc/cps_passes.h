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
  T wmn, wmx;  // the wavefront's running extremes (uniform; see p0_extremes_wave)
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

// The running extremes of a fast pass 0 for one vector of V elements.  An element can be
// the array's minimum (maximum) only if it is at most (at least) the wavefront's running
// minimum wmn (maximum wmx), which are uniform, so the wavefront tests that first; only when
// some lane's element passes do the lanes update their extremes and multiplicities
// (p0_extremes) and the wavefront refold wmn and wmx from them.  Exact for the array's
// extremes: wmn never falls below the final minimum, so every element equal to it passes
// the test when it is read and is counted; an element that does not pass lies above the
// final minimum (below the final maximum), and a lane's extremes over the elements that
// passed are all the fold of the lanes needs.  NaN compares false, as in p0_extremes.
template <typename T, int V>
__device__ inline void p0_extremes_wave(const T (&e)[V], bool valid, P0Acc<T> &acc) {
  bool near = false;
#pragma unroll
  for (int j = 0; j < V; ++j) near |= valid & ((e[j] <= acc.wmn) | (e[j] >= acc.wmx));
  if (ballot(near) != 0) {
#pragma unroll
    for (int j = 0; j < V; ++j) p0_extremes<T>(e[j], valid, acc);
    acc.wmn = (T)wave_min((double)acc.mn);
    acc.wmx = (T)wave_max((double)acc.mx);
  }
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

// Fold (min, multiplicity) and (max, multiplicity) pairs over the wavefront: the extreme
// first, then the multiplicities of the lanes that hold it.  Every lane gets the result.
__device__ inline void wave_pair_fold(double &mn, int64_t &cmn, double &mx, int64_t &cmx) {
  const double wm = wave_min(mn), wx = wave_max(mx);
  cmn = wave_sum_i64(mn == wm ? cmn : 0);
  cmx = wave_sum_i64(mx == wx ? cmx : 0);
  mn = wm;
  mx = wx;
}

// Fold of one value per wavefront (lanes 0 .. NW-1 of wavefront 0 hold them, NW <= 16, the
// other lanes the identity): four row shifts bring the first row's values into lane 15 in a
// fixed order, and lane 15 is read as a scalar, so every lane of the wavefront gets it.
template <int OP> __device__ inline double row_fold16(double v) {
  const double id = OP == 0 ? 0.0 : (OP == 1 ? __builtin_inf() : -__builtin_inf());
  v = dpp_op<OP>(v, dpp_move<0x111, 0xF>(v, id));  // row_shr:1
  v = dpp_op<OP>(v, dpp_move<0x112, 0xF>(v, id));  // row_shr:2
  v = dpp_op<OP>(v, dpp_move<0x114, 0xF>(v, id));  // row_shr:4
  v = dpp_op<OP>(v, dpp_move<0x118, 0xF>(v, id));  // row_shr:8
  const uint64_t b = __builtin_bit_cast(uint64_t, v);
  const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)b, 15);
  const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(b >> 32), 15);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// The wavefronts' values of one field, folded by wavefront 0 (op 0 sum, 1 min, 2 max).
template <int BLOCK>
__device__ inline double fold_waves(const double *row, int op) {
  const int lane = threadIdx.x % kWave;
  const bool in = lane < BLOCK / kWave;
  if (op == 0) return row_fold16<0>(in ? row[lane] : 0.0);
  if (op == 1) return row_fold16<1>(in ? row[lane] : __builtin_inf());
  return row_fold16<2>(in ? row[lane] : -__builtin_inf());
}
template <int BLOCK> __device__ inline int64_t fold_waves_i64(const int64_t *row) {
  const int lane = threadIdx.x % kWave;
  return (int64_t)row_fold16<0>(lane < BLOCK / kWave ? (double)row[lane] : 0.0);
}

// Block reduction of up to 8 double fields (op per field: 0 sum, 1 min, 2 max) and up to
// 8 int64 sums, and with PAIR also the (minimum, multiplicity) and (maximum, multiplicity)
// pairs (the extreme first, then the multiplicities of the lanes that hold it; ND + 2 and
// NI + 2 fields at most then).  The int fields are either per-thread or wave-uniform
// (`iuniform`); integer sums go through double, exact below 2^53.  Each wavefront folds its
// fields with DPP moves, writes one value per field to LDS, and wavefront 0 folds the
// wavefronts' values with row moves: one exchange, two barriers, a fixed order (so the
// results are deterministic).  The results are valid in every lane of wavefront 0.  (Fold
// cost grows with the fields; callers fold only the fields their pass forms.)
template <int BLOCK, int ND, int NI, bool PAIR = false>
__device__ inline void block_reduce_impl(double (&dv)[8], const int (&dop)[8], int64_t (&iv)[8],
                                         bool iuniform, double &mn, int64_t &cmn, double &mx,
                                         int64_t &cmx, double (&sd)[8][BLOCK / kWave],
                                         int64_t (&si)[8][BLOCK / kWave]) {
  static_assert(BLOCK / kWave <= 16, "one row of wavefront 0 folds the wavefronts");
  static_assert(!PAIR || (ND + 2 <= 8 && NI + 2 <= 8), "room for the pairs");
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
  if (PAIR) wave_pair_fold(mn, cmn, mx, cmx);
  if (lane == 0) {
#pragma unroll
    for (int f = 0; f < ND; ++f) sd[f][wv] = dv[f];
#pragma unroll
    for (int f = 0; f < NI; ++f) si[f][wv] = iv[f];
    if (PAIR) {
      sd[ND][wv] = mn;
      sd[ND + 1][wv] = mx;
      si[NI][wv] = cmn;
      si[NI + 1][wv] = cmx;
    }
  }
  __syncthreads();
  if (wv == 0) {
#pragma unroll
    for (int f = 0; f < ND; ++f) dv[f] = fold_waves<BLOCK>(sd[f], dop[f]);
#pragma unroll
    for (int f = 0; f < NI; ++f) iv[f] = fold_waves_i64<BLOCK>(si[f]);
    if (PAIR) {
      const bool in = lane < BLOCK / kWave;
      const double a = in ? sd[ND][lane] : __builtin_inf();
      const double b = in ? sd[ND + 1][lane] : -__builtin_inf();
      mn = row_fold16<1>(a);
      mx = row_fold16<2>(b);
      cmn = (int64_t)row_fold16<0>(in && a == mn ? (double)si[NI][lane] : 0.0);
      cmx = (int64_t)row_fold16<0>(in && b == mx ? (double)si[NI + 1][lane] : 0.0);
    }
  }
  __syncthreads();  // (the exchange rows are free again)
}

template <int BLOCK, int ND, int NI>
__device__ inline void block_reduce(double (&dv)[8], const int (&dop)[8], int64_t (&iv)[8],
                                    bool iuniform, double (&sd)[8][BLOCK / kWave],
                                    int64_t (&si)[8][BLOCK / kWave]) {
  double mn = 0.0, mx = 0.0;
  int64_t cmn = 0, cmx = 0;
  block_reduce_impl<BLOCK, ND, NI, false>(dv, dop, iv, iuniform, mn, cmn, mx, cmx, sd, si);
}

// block_reduce with the extremes' pairs folded in the same exchange: valid in wavefront 0.
template <int BLOCK, int ND, int NI>
__device__ inline void block_reduce_pair(double (&dv)[8], const int (&dop)[8], int64_t (&iv)[8],
                                         double &mn, int64_t &cmn, double &mx, int64_t &cmx,
                                         double (&sd)[8][BLOCK / kWave],
                                         int64_t (&si)[8][BLOCK / kWave]) {
  block_reduce_impl<BLOCK, ND, NI, true>(dv, dop, iv, false, mn, cmn, mx, cmx, sd, si);
}

}  // namespace cps
