// Host-side driver of the cutting-plane state machine (paper_1104_2732_amd/csrc/cp_state.h).
//
// Test infrastructure: it runs the same sequence of passes the GPU kernel runs (pass 0,
// evaluation passes with the optional split of the bracket into a buffer or the count of
// its two sides, histogram passes, final exact select) with plain loops, so that every
// branch of the state machine can be exercised on the CPU.  The final exact select here
// sorts the remaining candidates.
#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

#include "../../paper_1104_2732_amd/csrc/batch_queue.h"
#include "../../paper_1104_2732_amd/csrc/cp_state.h"

using namespace cps;

struct SimResult {
  double value;
  int64_t less, equal;
  int32_t status, passes, work_passes, kelley, bisect, bracket_used;
  int64_t elements_read, elements_written;
};

template <typename T>
static int sim(const T *x, int64_t n, int64_t k, int maxit, int64_t final_threshold,
               double theta, int use_bracket, double blo, double bhi, int p0_split,
               int64_t p0_cap, int hist_bits, int count_first, int hist_compact, int p0_sums,
               int spec_mode, SimResult *out, int side_bits = -1, int transform = 0) {
  CpConfig c{};
  c.transform = transform;
  c.maxit = maxit;
  c.dtype = sizeof(T) == 4 ? 0 : 1;
  c.final_threshold = final_threshold;
  c.final_direct_max = 4 * final_threshold;
  c.theta = theta;
  int64_t zcap = final_threshold;
  if (theta > 0) zcap = std::max<int64_t>(zcap, (int64_t)(theta * (double)n) + 1);
  c.zcap = zcap;
  c.use_bracket = use_bracket;
  c.bracket_lo = blo;
  c.bracket_hi = bhi;
  c.p0_split = p0_split;
  c.hist_bits = hist_bits;
  c.hist_compact = hist_compact;  // 1 as the single-array kernel, 0 as the batched one
  c.count_first = count_first;
  c.spec_min_n = spec_mode ? 1 : 0;
  // one workgroup: a single region per split buffer, as large as the input
  const int64_t R = n + 8;
  std::vector<T> z[2] = {std::vector<T>(R), std::vector<T>(R)};
  std::vector<T> zf(zcap);
  int64_t my_l = 0, my_r = 0;  // this "workgroup's" split counts

  CpState s{};
  s.n = n;
  s.k = k;
  const T ba = (T)blo, bb = (T)bhi;
  for (int attempt = 0; attempt < 2; ++attempt) {
    // pass 0: first without classifying infinities (as the GPU's fast pass), then, if
    // the state asks for it, with the classification
    const bool classify = attempt == 1;
    Pass0Result r{};
    r.classified = classify ? 1 : 0;
    r.sums = p0_sums;  // 0: as a pass 0 that counts the interior (no sums at the ends)
    r.fmin = INFINITY;
    r.fmax = -INFINITY;
    my_l = my_r = 0;
    for (int64_t i = 0; i < n; i++) {
      const T v = x[i];
      if (use_bracket && p0_split && v > ba && v < bb) {
        // the bracket's interior goes to the low part of split buffer 0, while it fits
        if (my_l < p0_cap) z[0][my_l] = v;
        my_l++;
      }
      // the fast pass classifies nothing: NaN reaches the sum (and compares false)
      if (classify && std::isnan(v)) { r.nnan++; continue; }
      const bool fin = !classify || std::isfinite(v);
      if (classify && v == (T)-INFINITY) r.nneg++;
      else if (classify && v == (T)INFINITY) r.npos++;
      if (fin) {
        if (v < r.fmin) { r.fmin = v; r.cmin = 1; } else if (v == r.fmin) r.cmin++;
        if (v > r.fmax) { r.fmax = v; r.cmax = 1; } else if (v == r.fmax) r.cmax++;
        r.sum += v;
        if (use_bracket) {
          if (v > ba) r.A_a += (double)(v - ba);
          if (v < ba) r.B_a += (double)(ba - v);
          if (v > bb) r.A_b += (double)(v - bb);
          if (v < bb) r.B_b += (double)(bb - v);
        }
      }
      if (use_bracket) {
        if (v <= ba) r.c_le_a++;
        if (v < bb) r.c_lt_b++;
      }
    }
    r.split_overflow = (use_bracket && p0_split && my_l > p0_cap) ? 1 : 0;
    if (!p0_sums) r.A_a = r.B_a = r.A_b = r.B_b = 0.0;
    cp_after_pass0(s, r, c);
    if (!(s.phase == PH_PASS0 && s.p0_slow)) break;
  }
  if (s.phase == PH_PASS0) return -15;
  if (s.phase == PH_EVAL && s.counted && c.spec_min_n && n >= c.spec_min_n) {
    // the likely interval of the counting evaluation's copy: quantiles of a strided sample
    // around the rank's fraction of the bracket (spec_mode 2 places it away from the rank,
    // so that the copy is not adopted)
    const int64_t S = n < 4096 ? n : 4096, stride = n / S;
    std::vector<T> smp;
    for (int64_t i = 0; i < S; ++i) {
      const T v = x[i * stride];
      if (v > (T)s.yL && v < (T)s.yR) smp.push_back(v);
    }
    if (smp.size() >= 16) {
      std::sort(smp.begin(), smp.end());
      const double m = (double)smp.size();
      const double p = ((double)(s.k - s.cL) - 0.5) / (double)(s.cR - s.cL);
      const double q = p * m, d = 4.0 * std::sqrt(m * p * (1.0 - p)) + 2.0;
      int64_t rl = (int64_t)std::floor(q - d), rh = (int64_t)std::ceil(q + d);
      if (spec_mode == 2) { rl = (int64_t)m - 2; rh = (int64_t)m - 1; }
      rl = std::max<int64_t>(0, std::min<int64_t>(rl, (int64_t)m - 1));
      rh = std::max<int64_t>(rl, std::min<int64_t>(rh, (int64_t)m - 1));
      s.spec = 1;
      s.spec_a = (double)smp[(size_t)rl];
      s.spec_b = (double)smp[(size_t)rh];
    }
  }
  auto working = [&](int64_t &len) -> const T * {
    if (s.wbuf < 0) { len = s.wlen; return x; }
    if (s.wbuf == 2) { len = s.wlen; return zf.data(); }
    if (s.side == 0) { len = my_l; return z[s.wbuf].data(); }
    len = my_r;
    return z[s.wbuf].data() + (R - my_r);
  };
  while (s.phase == PH_EVAL || s.phase == PH_GATHER || s.phase == PH_HIST) {
    int64_t wl = 0;
    const T *W = working(wl);
    if (s.wbuf >= 0 && s.wbuf < 2 && wl != s.wlen) return -13;
    const T t = (T)s.t, yL = (T)s.yL, yR = (T)s.yR;
    if (s.phase == PH_HIST) {
      // key histogram of the working set's elements inside [lo, hi], then the bin of
      // rank k - cL
      const HistGeom<uint64_t> g = hist_geometry(s.lo, s.hi, c.dtype, c.hist_bits);
      std::vector<int64_t> h((size_t)g.nbins, 0);
      int64_t nc = 0;  // elements copied when the pass also compacts the bracket
      for (int64_t i = 0; i < wl; i++) {
        const uint64_t K = sizeof(T) == 4 ? (uint64_t)key32((float)W[i]) : key64((double)W[i]);
        if (K >= g.klo && K <= g.khi) {
          h[(size_t)((K - g.klo) >> g.shift)]++;
          if (s.compact) z[s.zout][nc++] = W[i];
        }
      }
      if (s.compact) {
        if (nc != s.cR - s.cL) return -19;  // the key range holds exactly the bracket's elements
        my_l = nc;
        my_r = 0;
      }
      const int64_t r = s.k - s.cL;
      int64_t below = 0;
      int32_t b = 0;
      while (b < g.nbins && below + h[(size_t)b] < r) below += h[(size_t)b++];
      if (b >= g.nbins) return -16;
      cp_after_hist(s, b, below, h[(size_t)b], c);
      continue;
    }
    if (s.phase == PH_GATHER) {
      int64_t g = 0;
      for (int64_t i = 0; i < wl; i++) {
        const T v = W[i];
        if (s.filter && !(v > yL && v < yR)) continue;
        if (g >= zcap) return -14;
        zf[g++] = v;
      }
      cp_after_gather(s, g);
      continue;
    }
    const bool clamp = s.has_inf && s.wbuf < 0;
    // a split with the histogram finish also counts each part in key bins; a counting
    // evaluation counts them without writing
    const bool counted = (s.split || s.counted) && c.hist_bits > 0;
    const bool count_only = counted && !s.split;
    const bool spec = count_only && s.spec;
    int64_t nspec = 0;  // elements of [spec_a, spec_b] copied to buffer 0
    HistGeom<uint64_t> pg[2] = {};
    std::vector<int64_t> ph[2];
    // the two sides' bins (the batched kernel's counting evaluation uses fewer per side)
    CpConfig cs = c;
    if (count_only && side_bits >= 0 && side_bits < c.hist_bits) cs.hist_bits = side_bits;
    if (counted)
      for (int p = 0; p < 2; ++p) {
        pg[p] = split_part_geometry(s, p, cs);
        ph[p].assign((size_t)pg[p].nbins, 0);
      }
    EvalResult e{};
    e.pred = -INFINITY;
    e.succ = INFINITY;
    int64_t nl = 0, nr = 0;
    T *zo = z[s.zout].data();
    for (int64_t i = 0; i < wl; i++) {
      T v = W[i];
      if (clamp) v = std::min(std::max(v, (T)s.fmin), (T)s.fmax);
      // (with the transform, the sums are on F(x) = log(1 + x - min x); the counts on x)
      const double dv = s.tf ? cp_F(s, (double)v) - cp_F(s, (double)t) : (double)(v - t);
      if (v < t) { e.L++; e.B -= dv; e.pred = std::max<double>(e.pred, v); }
      if (v > t) { e.G++; e.A += dv; e.succ = std::min<double>(e.succ, v); }
      if (spec && v >= (T)s.spec_a && v <= (T)s.spec_b) z[0][nspec++] = v;
      if (s.split || count_only) {
        const bool inb = !s.filter || (v > yL && v < yR);
        if (s.split && inb && v < t) zo[nl++] = v;
        if (s.split && inb && v > t) zo[R - 1 - nr++] = v;
        if (counted && inb && v != t) {
          const int p = v < t ? 0 : 1;
          const uint64_t K = sizeof(T) == 4 ? (uint64_t)key32((float)v) : key64((double)v);
          if (K < pg[p].klo || K > pg[p].khi) return -17;  // outside its part's range
          ph[p][(size_t)((K - pg[p].klo) >> pg[p].shift)]++;
        }
      }
    }
    e.written = nl + nr;
    if (s.split) { my_l = nl; my_r = nr; }
    if (count_only) {  // as the kernel's counting evaluation: counts and bins only
      e.A = e.B = 0.0;
      e.pred = -INFINITY;
      e.succ = INFINITY;
      e.written = nspec;
    }
    cp_after_eval(s, e, c);
    if (counted && s.phase == PH_HIST && (s.on_bracket || count_only)) {
      // the part that holds x_(k) is counted already: narrow without a histogram pass
      const std::vector<int64_t> &h = ph[s.side];
      const int64_t r = s.k - s.cL;
      int64_t below = 0;
      int32_t b = 0;
      while (b < pg[s.side].nbins && below + h[(size_t)b] < r) below += h[(size_t)b++];
      if (b >= pg[s.side].nbins) return -18;
      cp_hist_narrow(s, pg[s.side], b, below, h[(size_t)b], c);
    }
    if (count_only) {
      cp_adopt_spec(s, nspec, c);
      if (s.wbuf == 0) {
        my_l = nspec;
        my_r = 0;
      }
    }
  }
  if (s.phase == PH_FINAL) {
    int64_t wl = 0;
    const T *W = working(wl);
    std::vector<T> cand;
    for (int64_t i = 0; i < wl; i++) {
      const T v = W[i];
      if (s.on_bracket || (v > (T)s.yL && v < (T)s.yR)) cand.push_back(v);
    }
    const int64_t rr = s.k - s.cL;
    if (rr < 1 || rr > (int64_t)cand.size()) return -11;
    std::sort(cand.begin(), cand.end());
    const T v = cand[rr - 1];
    int64_t below = 0, eq = 0;
    for (T c2 : cand) { if (c2 < v) below++; else if (c2 == v) eq++; }
    cp_after_final(s, (double)v, below, eq);
  }
  if (s.phase != PH_DONE) return -12;
  out->value = (double)((T)s.value + (T)0);
  out->less = s.less;
  out->equal = s.equal;
  out->status = s.status;
  out->passes = s.passes;
  out->work_passes = s.work_passes;
  out->kelley = s.kelley;
  out->bisect = s.bisect;
  out->bracket_used = s.bracket_used;
  out->elements_read = s.elements_read;
  out->elements_written = s.elements_written;
  return 0;
}

// Replay of the batched kernel's work queue on the host: the descriptor checks and the
// largest-first order of the kernel's bitonic network (batch_queue.h, the kernel's own code),
// then every valid array through the state machine with the batched kernel's configuration:
// the counting evaluation with 2^side_bits key bins per side, histogram passes over the array
// itself (no compaction), the gather and the exact select.  addrs: the descriptor pointers as
// the kernel would see them; data[off[i]..] the values of array i (off < 0: not readable).
// order_out: the array taken at each queue position; status_out: 4 (BADARG), the state
// machine's status, or a negative driver error.
template <typename T>
static void replay_batch(const T *data, const uint64_t *addrs, const int64_t *off,
                         const int64_t *sizes, const int64_t *ks, int64_t count, int64_t ft,
                         int hist_bits, int side_bits, int64_t *order_out, int32_t *status_out,
                         double *value_out, int64_t *less_out, int64_t *equal_out,
                         int32_t *passes_out) {
  const bool sorted = count <= kBatchSortMax;
  int64_t m = 1;
  while (m < count) m <<= 1;
  std::vector<uint64_t> order(sorted ? (size_t)m : 0);
  if (sorted) {
    for (int64_t j = 0; j < m; ++j) order[(size_t)j] = j < count ? lpt_key(sizes[j], j) : 0;
    for (int64_t kk = 2; kk <= m; kk <<= 1)
      for (int64_t jj = kk >> 1; jj > 0; jj >>= 1)
        for (int64_t i = 0; i < m; ++i) bitonic_exchange(order.data(), i, jj, kk);
  }
  for (int64_t j = 0; j < count; ++j) {
    const int64_t i = sorted ? lpt_index(order[(size_t)j]) : j;
    order_out[j] = i;
    value_out[i] = 0.0;
    less_out[i] = equal_out[i] = 0;
    passes_out[i] = 0;
    if (!batch_array_valid(addrs[i], sizes[i], ks[i], (uint32_t)sizeof(T))) {
      status_out[i] = ST_BADARG;
      continue;
    }
    if (off[i] < 0) {  // a descriptor the kernel would read but the replay has no data for
      status_out[i] = -100;
      continue;
    }
    SimResult r{};
    const int rc = sim<T>(data + off[i], sizes[i], ks[i], 64, ft, 1.0, 0, 0.0, 0.0, 0, 0,
                          hist_bits, 1, 0, 1, 0, &r, side_bits);
    status_out[i] = rc != 0 ? rc : r.status;
    value_out[i] = r.value;
    less_out[i] = r.less;
    equal_out[i] = r.equal;
    passes_out[i] = r.work_passes;
  }
}

extern "C" {

int replay_batch_f32(const float *data, const uint64_t *addrs, const int64_t *off,
                     const int64_t *sizes, const int64_t *ks, int64_t count, int64_t ft,
                     int hist_bits, int side_bits, int64_t *order_out, int32_t *status_out,
                     double *value_out, int64_t *less_out, int64_t *equal_out,
                     int32_t *passes_out) {
  replay_batch<float>(data, addrs, off, sizes, ks, count, ft, hist_bits, side_bits, order_out,
                      status_out, value_out, less_out, equal_out, passes_out);
  return 0;
}

int sim_select_f32(const float *x, int64_t n, int64_t k, int maxit, int64_t ft, double theta,
                   int ub, double blo, double bhi, int p0_split, int64_t p0_cap, int hist_bits,
                   int count_first, int hist_compact, int p0_sums, int spec_mode,
                   int transform, SimResult *out) {
  return sim<float>(x, n, k, maxit, ft, theta, ub, blo, bhi, p0_split, p0_cap, hist_bits,
                    count_first, hist_compact, p0_sums, spec_mode, out, -1, transform);
}
int sim_select_f64(const double *x, int64_t n, int64_t k, int maxit, int64_t ft, double theta,
                   int ub, double blo, double bhi, int p0_split, int64_t p0_cap, int hist_bits,
                   int count_first, int hist_compact, int p0_sums, int spec_mode,
                   int transform, SimResult *out) {
  return sim<double>(x, n, k, maxit, ft, theta, ub, blo, bhi, p0_split, p0_cap, hist_bits,
                     count_first, hist_compact, p0_sums, spec_mode, out, -1, transform);
}
}
