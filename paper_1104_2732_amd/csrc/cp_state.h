// Cutting-plane state machine for exact k-th element selection.
//
// One instance describes one selection in flight.  It is advanced once per
// reduction pass by a single thread (the last workgroup to finish the pass on
// the GPU; a plain host loop in the CPU unit tests), so everything here is
// scalar code usable from host and device.
//
// Notation (Section 3, Eq. 2, with the orientation whose minimiser is the k-th
// smallest): alpha = k - 1/2, beta = n - k + 1/2,
//   A(y) = sum_{x_i > y} (x_i - y),  B(y) = sum_{x_i < y} (y - x_i),
//   f(y) = alpha A(y) + beta B(y),
//   L = #(x < y), E = #(x = y),  subdifferential [n (L - k + 1/2), n (L + E - k + 1/2)].
//
// Bracket (Section 4, Algorithm 1): x_(k) lies strictly inside (yL, yR) and
//   cL = #(x <= yL) < k <= cR = #(x < yR).
// The cut at yL uses the right derivative gL = n (cL - k + 1/2) < 0 and the cut at
// yR the left derivative gR = n (cR - k + 1/2) > 0; both are subgradients, so the
// two supporting lines meet strictly inside and the update of Algorithm 1 step 1.1
// never divides by zero.  Decisions are made on the integer counts (step 1.4 with
// the set-valued subgradient): L < k <= L + E means the trial point is x_(k).
//
// Working set.  Pass 0 and the first evaluation passes read the whole input.  Once
// the bracket holds few enough elements, a pass also writes the bracket's elements
// below and above the trial point to the two ends of each workgroup's private region
// of a workspace buffer (the count-and-compact of Section 4, done as part of the
// evaluation pass), and the next pass reads only the side that still holds x_(k).
// Once the bracket is small, a gather pass copies its elements into one contiguous
// buffer for the exact select.  Reading only the bracket's
// elements changes f by a positive factor and an affine term on the bracket, so the
// cutting-plane trial points are unchanged: A and B of the full array are rebuilt
// from the bracket-only sums as
//   A(t) = A_W(t) + A(yR) + (n - cR)(yR - t),   B(t) = B_W(t) + B(yL) + cL (t - yL),
// where every term is non-negative.
//
// Termination: an exact hit; one distinct value left inside the bracket (the smallest
// element above yL equals the largest below yR, the exact step at the end of
// Section 4); or few enough elements left for a one-workgroup exact radix select.
// After `maxit` cutting-plane steps the trial point becomes the midpoint of the
// bracket in the ordered bit pattern of T, which bounds the number of passes.
#pragma once

#include <math.h>
#include <stdint.h>

#ifdef __HIPCC__
#define CPS_HD __host__ __device__
#else
#define CPS_HD
#endif

namespace cps {

enum Phase : int32_t {
  PH_PASS0 = 0, PH_EVAL = 1, PH_GATHER = 2, PH_FINAL = 3, PH_DONE = 4, PH_HIST = 5
};

// status values mirror enum cps_status in cpselect.h
enum : int32_t { ST_OK = 0, ST_NAN = 1, ST_TIMEOUT = 2, ST_INTERNAL = 3, ST_BADARG = 4 };

struct CpConfig {
  int32_t maxit;
  int32_t dtype;            // 0 = f32, 1 = f64
  int64_t final_threshold;  // bracket population handled by one workgroup
  int64_t final_direct_max; // largest unsplit input one workgroup may scan directly
  double theta;             // start splitting once population <= theta * n (0 = never)
  int64_t zcap;             // capacity of the gather buffer (elements, >= final_threshold)
  int32_t use_bracket;
  int32_t p0_split;         // pass 0 with a bracket also writes the elements inside it
  double bracket_lo, bracket_hi;
  int64_t split_cap;        // the first split needs population <= split_cap (0 = no limit)
  int32_t hist_bits;        // exact select on the compacted bracket by key histograms of
                            // 2^hist_bits bins (0: cutting-plane passes to the end)
  int32_t hist_compact;     // histogram passes may also compact a narrowed bracket's
                            // elements into the other split buffer (kernels that do so)
  int32_t count_first;      // with hist_bits: where the first split from the input would run,
                            // the evaluation counts both sides in key bins instead and writes
                            // nothing; the bracket narrows to a bin, whose elements the next
                            // pass over the input compacts (hist_compact) or counts
  int32_t transform;        // 1: the cutting plane runs on F(x) = log(1 + x - min x) (see
                            // cp_F); counts, comparisons and the result stay on x
  int64_t spec_min_n;       // inputs of at least this many elements (0: none): the counting
                            // evaluation also copies the elements of a likely interval
                            // [spec_a, spec_b] to split buffer 0 (see cp_adopt_spec)
};

// Results of pass 0 over the whole input (Section 4, step 0: min, max and sum in
// one reduction; here with the multiplicity of min and max, the sum over finite
// values and the counts of NaN and infinities).
struct Pass0Result {
  int32_t classified;   // 1: NaN and infinities were classified (nnan, nneg, npos, finite
                        // min/max); 0: nothing classified (nnan etc. are 0)
  int32_t sums;         // 1: A_a, B_a, A_b, B_b below were formed; 0: only the two counts
                        // (a pass 0 that counts a proposal's interior in key bins)
  double sum;           // sum of finite elements
  double fmin, fmax;    // min and max over finite elements (+inf / -inf if none)
  int64_t cmin, cmax;   // multiplicities of fmin and fmax
  int64_t nnan, nneg, npos;  // counts of NaN, -inf, +inf
  // two-point check of a proposed bracket (a, b): #(x <= a), #(x < b) and the
  // finite-element parts of A and B at a and at b
  int64_t c_le_a, c_lt_b;
  double A_a, B_a, A_b, B_b;
  // pass 0 that also wrote the elements strictly inside (a, b) to split buffer 0: the
  // number of wavefronts whose share did not fit their region (0 = all written)
  int64_t split_overflow;
  // 0: the written elements are exactly those strictly inside (a, b); otherwise how many
  // were written, a superset (whole 16-byte vectors that hold an interior element, and
  // elements equal to a): every extra lies outside the open bracket that pass 0 leaves
  int64_t split_written;
};

// Results of one evaluation pass over the working set W at trial point t.  A counting
// evaluation (CpState::counted) gives only L and G (from its key bins' totals and the
// bracket's counts): A and B are 0, pred and succ -inf and +inf, since the bracket narrows
// by the bins right after it and neither f at the ends nor their neighbours are used again.
struct EvalResult {
  double A, B;          // sums over W of (w - t) for w > t and (t - w) for w < t
  int64_t L, G;         // #(w < t), #(w > t) within W
  double pred, succ;    // largest w < t, smallest w > t in W (-inf / +inf if none)
  int64_t written;      // elements the pass wrote to the split buffer
};

struct CpState {
  int64_t n, k;
  int32_t phase, status;
  double yL, yR;
  double AL, BL, AR, BR;   // A and B of the full array at yL and yR
  int64_t cL, cR;
  double lo, hi;           // a value of T inside (yL, yR) known to be <= / >= every element there
  int32_t lo_data, hi_data;// lo / hi are actual elements of x
  double t;                // trial point of the pass about to run
  int32_t split;           // the pass about to run writes (yL,t) and (t,yR) to buffer zout
  int32_t filter;          // that pass reads x, so the split keeps only elements inside (yL,yR)
  int32_t on_bracket;      // the working set is exactly the elements inside (yL, yR)
  int32_t has_inf;         // evaluate with values clamped into [fmin, fmax]
  double fmin, fmax;
  int32_t wbuf;            // -1: the input; 0/1: split buffer holding the working set;
                           // 2: the gather buffer (contiguous, wlen elements)
  int32_t zout;            // buffer the next split writes
  int32_t side;            // split buffers: 0 = the low part of each region, 1 = the high part
  int32_t narrowed;        // a histogram pass narrowed the bracket: the working set holds
                           // elements outside it, and f at the ends is no longer known
  int64_t wlen;            // elements in the working set
  int32_t passes;          // full reads of the input
  int32_t work_passes;     // all passes
  int32_t kelley, bisect;
  int64_t elements_read, elements_written;
  double value;            // result (as T widened to double)
  int64_t less, equal;
  int64_t final_size;
  int32_t bracket_used;
  int32_t p0_slow;         // pass 0 must classify infinities (the fast pass saw one)
  int32_t compact;         // the histogram pass about to run also copies the bracket's
                           // elements to split buffer zout (low parts)
  int32_t counted;         // the evaluation pass about to run (over the input, no split)
                           // counts the elements on either side of t in key bins
  int32_t spec;            // that counting evaluation also copies every element of
                           // [spec_a, spec_b] to the low parts of split buffer 0
  int32_t tf;              // the objective's values (AL, BL, AR, BR, an evaluation's A and B)
                           // are those of the transformed data F(x) (CpConfig::transform)
  double spec_a, spec_b;
  int32_t fends;           // with tf: F's objective at the bracket ends is not formed yet;
                           // the evaluation about to run at t = yL forms it
  int32_t pad2;
};

static_assert(sizeof(CpState) % 8 == 0, "state is copied in 8-byte words");

// ---------------------------------------------------------------- T helpers

CPS_HD inline uint32_t f32_bits(float v) { return __builtin_bit_cast(uint32_t, v); }
CPS_HD inline uint64_t f64_bits(double v) { return __builtin_bit_cast(uint64_t, v); }
CPS_HD inline float f32_from(uint32_t b) { return __builtin_bit_cast(float, b); }
CPS_HD inline double f64_from(uint64_t b) { return __builtin_bit_cast(double, b); }

// Monotone map from T (no NaN) to unsigned integers: a < b  <=>  key(a) < key(b),
// with -0.0 mapped like +0.0.
// (negative: all bits flipped; otherwise the sign bit set; written without a select: the
// sign bit spread over the word, or'ed with the sign bit, is the mask to flip with)
CPS_HD inline uint32_t key32(float v) {
  uint32_t b = f32_bits(v + 0.0f);
  return b ^ ((uint32_t)((int32_t)b >> 31) | 0x80000000u);
}
CPS_HD inline float unkey32(uint32_t k) {
  uint32_t b = (k & 0x80000000u) ? (k & 0x7fffffffu) : ~k;
  return f32_from(b);
}
CPS_HD inline uint64_t key64(double v) {
  uint64_t b = f64_bits(v + 0.0);
  return b ^ ((uint64_t)((int64_t)b >> 63) | 0x8000000000000000ull);
}
CPS_HD inline double unkey64(uint64_t k) {
  uint64_t b = (k & 0x8000000000000000ull) ? (k & 0x7fffffffffffffffull) : ~k;
  return f64_from(b);
}

// Round a double to the nearest value of T (dtype 0: float), returned widened.
CPS_HD inline double to_T(double v, int32_t dtype) { return dtype == 0 ? (double)(float)v : v; }

// The next representable value of T above / below v (v finite).  The ordered bit
// patterns hold both zeros; a step that lands on the other zero steps once more.
CPS_HD inline double next_up(double v, int32_t dtype) {
  if (dtype == 0) {
    double r = (double)unkey32(key32((float)v) + 1u);
    return r == v ? (double)unkey32(key32((float)v) + 2u) : r;
  }
  double r = unkey64(key64(v) + 1ull);
  return r == v ? unkey64(key64(v) + 2ull) : r;
}
CPS_HD inline double next_down(double v, int32_t dtype) {
  if (dtype == 0) {
    double r = (double)unkey32(key32((float)v) - 1u);
    return r == v ? (double)unkey32(key32((float)v) - 2u) : r;
  }
  double r = unkey64(key64(v) - 1ull);
  return r == v ? unkey64(key64(v) - 2ull) : r;
}

// Midpoint of [a, b] in the ordered bit pattern of T.
CPS_HD inline double key_mid(double a, double b, int32_t dtype) {
  if (dtype == 0) {
    uint32_t ka = key32((float)a), kb = key32((float)b);
    return (double)unkey32(ka + (kb - ka) / 2u);
  }
  uint64_t ka = key64(a), kb = key64(b);
  return unkey64(ka + (kb - ka) / 2ull);
}

CPS_HD inline bool inside(double t, double a, double b) { return t > a && t < b; }

// The monotone transform of the outlier discussion (Section 5.3): F(y) = log(1 + y - min x).
// The k-th smallest is invariant under an increasing F, so the cutting plane may minimise
// the objective of F(x) instead; its sums then stay accurate when a few elements are huge
// (~1e20), where the sums over x lose every other term.  Here only the objective's values
// and the trial points are formed on F(x): the counts, every comparison and the result stay
// on x, so the answer is exact whether F rounds distinct values together or not.
CPS_HD inline double cp_F(const CpState &s, double y) {
  return s.tf ? log1p(y - s.fmin) : y;
}

// ---------------------------------------------------------------- transitions

CPS_HD inline void cp_finish(CpState &s, double value, int64_t less, int64_t equal) {
  s.value = value;
  s.less = less;
  s.equal = equal;
  s.phase = PH_DONE;
}

// Choose the next trial point inside (yL, yR): the intersection of the supporting
// lines at the bracket ends (Algorithm 1, step 1.1), safeguarded, rounded to T and
// clamped to [lo, hi]; or the bit-pattern midpoint once maxit steps are spent.
CPS_HD inline double cp_trial_point(CpState &s, const CpConfig &c) {
  const double n = (double)s.n, k = (double)s.k;
  const double alpha = k - 0.5, beta = n - k + 0.5;
  double t = 0.0;
  bool ok = false;
  if (s.kelley < c.maxit) {
    const double gL = n * ((double)s.cL - k + 0.5);
    const double gR = n * ((double)s.cR - k + 0.5);
    const double fL = alpha * s.AL + beta * s.BL;
    const double fR = alpha * s.AR + beta * s.BR;
    // (with tf, the step is taken on F's scale, y = F(x), and mapped back by F^-1; while F's
    // objective at the ends is not formed, the midpoint on that scale)
    const double uL = cp_F(s, s.yL), uR = cp_F(s, s.yR);
    const double D = uR - uL;
    double u = s.fends ? 0.5 * uL + 0.5 * uR : uL + (fR - fL - gR * D) / (gL - gR);
    if (s.tf && !inside(u, uL, uR)) u = 0.5 * uL + 0.5 * uR;
    t = s.tf ? s.fmin + expm1(u) : u;
    ok = inside(t, s.yL, s.yR);
    if (!ok) {
      t = 0.5 * s.yL + 0.5 * s.yR;
      ok = inside(t, s.yL, s.yR);
    }
    s.kelley++;
  } else {
    s.bisect++;
  }
  if (!ok) t = key_mid(s.lo, s.hi, c.dtype);
  t = to_T(t, c.dtype);
  if (t < s.lo) t = s.lo;
  if (t > s.hi) t = s.hi;
  return t;
}

// Bound on the passes of one selection.  Every kind of pass provably shrinks the bracket
// (a cutting-plane step removes at least one distinct value and the bisection after maxit
// steps halves its key range; a histogram pass keeps one of at least two bins, or finishes;
// a gather is followed by the final select), so this is never reached; it only turns a
// broken invariant into an error instead of an endless loop.
constexpr int32_t kMaxWorkPasses = 4 * 96;

// Decide what the next pass does, given the current bracket.
CPS_HD inline void cp_plan(CpState &s, const CpConfig &c) {
  const int64_t pop = s.cR - s.cL;
  if (pop < 1 || s.work_passes >= kMaxWorkPasses) {
    // the bracket always holds x_(k), and the passes are bounded; anything else is a bug
    s.status = ST_INTERNAL;
    cp_finish(s, 0.0, 0, 0);
    return;
  }
  if (s.lo_data && s.hi_data && s.lo == s.hi) {
    // one distinct value strictly inside the bracket: it is x_(k)
    cp_finish(s, s.lo, s.cL, pop);
    return;
  }
  s.split = 0;
  s.filter = 0;
  s.compact = 0;
  s.counted = 0;  // (spec stays: the caller of a counting evaluation clears it, cp_adopt_spec)
  if (pop <= c.final_threshold) {
    if (s.wbuf < 0 && s.wlen <= c.final_direct_max) {
      s.phase = PH_FINAL;  // small input: select straight from x, keeping (yL, yR) only
      s.final_size = s.wlen;
      return;
    }
    s.phase = PH_GATHER;  // copy the bracket's elements into one contiguous buffer
    s.filter = s.on_bracket ? 0 : 1;
    return;
  }
  if (c.hist_bits > 0 && ((s.on_bracket && s.wbuf >= 0) || s.narrowed)) {
    // the bracket's elements are compacted (or the bracket is one bin of a count): finish
    // with the exact select by key histograms (the paper sorts the compacted elements
    // instead).  When a narrowed bracket holds at most a quarter of the working set, the
    // pass also copies the bracket's elements to a split buffer (the other one, or buffer 0
    // when the pass reads the input), so later passes read only those.
    s.phase = PH_HIST;
    if (c.hist_compact && !s.on_bracket && s.wbuf < 2 && pop * 4 <= s.wlen) {
      s.compact = 1;
      s.zout = s.wbuf < 0 ? 0 : 1 - s.wbuf;
    }
    return;
  }
  if (s.on_bracket) {
    s.split = 1;
    s.zout = 1 - s.wbuf;
  } else if (c.theta > 0.0 && !s.has_inf && (double)pop <= c.theta * (double)s.n) {
    // (inputs holding infinities keep reading x until the gather: no clamped split)
    if (c.count_first && c.hist_bits > 0) {
      s.counted = 1;  // count both sides now (no buffer needed); the bin of x_(k) comes next
      s.filter = 1;
    } else if (c.split_cap == 0 || pop <= c.split_cap) {
      s.split = 1;
      s.filter = 1;
      s.zout = 0;
    }
  }
  s.phase = PH_EVAL;
  if (s.fends && !s.counted && !s.split && s.wbuf < 0) {
    // F's objective at both ends from one evaluation at the left end (F(yL) = 0 there):
    // A_F(yL) = sum F(x), and B_F(yR) = n F(yR) - sum F(x)
    s.filter = 0;
    s.t = s.yL;
    return;
  }
  s.t = cp_trial_point(s, c);
}

// After pass 0 (Section 4, step 0).  Returns with phase DONE when the answer is an
// extreme value (or NaN is present), else with the first trial point planned.
CPS_HD inline void cp_after_pass0(CpState &s, const Pass0Result &r, const CpConfig &c) {
  const int64_t n = s.n, k = s.k;
  s.passes++;
  s.work_passes++;
  s.elements_read += n;
  s.status = ST_OK;
  s.bracket_used = 0;
  s.final_size = 0;
  if (!r.classified &&
      (r.sum != r.sum || r.fmin == -__builtin_inf() || r.fmax == __builtin_inf())) {
    // The fast pass 0 classifies nothing: NaN (a NaN sum) or an infinity (an infinite
    // extreme, or a NaN sum when both signs occur) makes it repeat with the classification;
    // only such inputs pay for the second pass.
    s.phase = PH_PASS0;
    s.p0_slow = 1;
    return;
  }
  if (r.nnan > 0) {
    s.status = ST_NAN;
    cp_finish(s, __builtin_nan(""), 0, 0);
    return;
  }
  const int64_t nf = n - r.nneg - r.npos;
  if (k <= r.nneg) { cp_finish(s, -__builtin_inf(), 0, r.nneg); return; }
  if (k > n - r.npos) { cp_finish(s, __builtin_inf(), n - r.npos, r.npos); return; }
  if (k <= r.nneg + r.cmin) { cp_finish(s, r.fmin, r.nneg, r.cmin); return; }
  if (k > n - r.npos - r.cmax) { cp_finish(s, r.fmax, n - r.npos - r.cmax, r.cmax); return; }
  // x_(k) lies strictly between the finite extremes.
  s.fmin = r.fmin;
  s.fmax = r.fmax;
  s.has_inf = (r.nneg + r.npos) > 0;
  const double span = r.fmax - r.fmin;
  s.yL = r.fmin;
  s.yR = r.fmax;
  s.cL = r.nneg + r.cmin;
  s.cR = n - r.npos - r.cmax;
  // f at the extremes in closed form from the sum (Section 4, step 0); infinities are
  // evaluated as if clamped to the finite extremes, which leaves f' unchanged inside.
  double al = (r.sum - (double)nf * r.fmin) + (double)r.npos * span;
  double br = ((double)nf * r.fmax - r.sum) + (double)r.nneg * span;
  s.AL = al > 0.0 ? al : 0.0;
  s.BL = 0.0;
  s.AR = 0.0;
  s.BR = br > 0.0 ? br : 0.0;
  s.lo = next_up(s.yL, c.dtype);
  s.hi = next_down(s.yR, c.dtype);
  s.lo_data = s.hi_data = 0;
  s.tf = c.transform ? 1 : 0;
  s.fends = s.tf;
  s.wbuf = -1;
  s.side = 0;
  s.wlen = n;
  s.on_bracket = 0;
  // A proposed end replaces the bracket's end only when the counts of the same pass
  // prove it: a is a valid left end when #(x <= a) < k, b a valid right end when
  // k <= #(x < b) (the bracket invariant above); each end is judged on its own, so a
  // proposal that misses on one side still tightens the other.  f at the new ends comes
  // from the two-point sums of the same pass (infinities evaluated as the finite extremes).
  if (c.use_bracket) {
    const double a = to_T(c.bracket_lo, c.dtype), b = to_T(c.bracket_hi, c.dtype);
    if (r.c_le_a < k && a > s.yL) {
      s.bracket_used |= 1;
      s.yL = a;
      s.cL = r.c_le_a;
      s.lo = next_up(a, c.dtype);
      s.lo_data = 0;
      s.AL = r.A_a + (double)r.npos * (r.fmax - a);
      s.BL = r.B_a + (double)r.nneg * (a - r.fmin);
    }
    if (k <= r.c_lt_b && b < s.yR) {
      s.bracket_used |= 2;
      s.yR = b;
      s.cR = r.c_lt_b;
      s.hi = next_down(b, c.dtype);
      s.hi_data = 0;
      s.AR = r.A_b + (double)r.npos * (r.fmax - b);
      s.BR = r.B_b + (double)r.nneg * (b - r.fmin);
    }
    // A pass 0 that formed only the counts at the ends leaves f at an adopted end unknown:
    // the bracket is then finished by key histograms only (its ends are never cut again).
    if (s.bracket_used && !r.sums) s.narrowed = 1;
    // With both ends proven, the elements pass 0 wrote (those strictly inside (a, b))
    // are exactly the bracket's, cR - cL of them: later passes read only those.  With the
    // exact finish by histograms, an end beyond the data (a <= min, b >= max) may stand
    // in for a proven one: the written elements then hold the bracket's and those equal
    // to that extreme, #(a < x < b) of them, and the histogram passes skip the extras.
    const bool left_ok = (s.bracket_used & 1) || a <= r.fmin;
    const bool right_ok = (s.bracket_used & 2) || b >= r.fmax;
    if (c.p0_split && r.split_overflow == 0 && left_ok && right_ok && a < b) {
      if (s.bracket_used == 3 && r.split_written == 0) {
        s.wbuf = 0;
        s.side = 0;
        s.wlen = s.cR - s.cL;
        s.on_bracket = 1;
        s.elements_written += s.wlen;
      } else if (c.hist_bits > 0) {
        // the written elements hold the bracket's and others outside it, which the
        // histogram passes skip
        s.wbuf = 0;
        s.side = 0;
        s.wlen = r.split_written > 0 ? r.split_written : r.c_lt_b - r.c_le_a;
        s.narrowed = 1;
        s.elements_written += s.wlen;
      }
    }
  }
  cp_plan(s, c);
}

// A, B, L and G of the whole array at the trial point s.t, from an evaluation pass over the
// working set: over the bracket's compacted elements the parts outside the bracket are
// added (every term non-negative).
struct FullEval {
  double A, B;
  int64_t L, G;
};

CPS_HD inline FullEval cp_full_eval(const CpState &s, const EvalResult &r) {
  FullEval f;
  f.L = r.L;
  f.G = r.G;
  f.A = r.A;
  f.B = r.B;
  if (s.on_bracket) {
    f.L += s.cL;
    f.G += s.n - s.cR;
    f.A += s.AR + (double)(s.n - s.cR) * (cp_F(s, s.yR) - cp_F(s, s.t));
    f.B += s.BL + (double)s.cL * (cp_F(s, s.t) - cp_F(s, s.yL));
  }
  return f;
}

// After an evaluation pass at s.t over the working set.
CPS_HD inline void cp_after_eval(CpState &s, const EvalResult &r, const CpConfig &c) {
  const int64_t n = s.n, k = s.k;
  const double t = s.t;
  if (s.fends && t == s.yL && s.wbuf < 0 && !s.counted) {
    // the evaluation at the left end (cp_plan): F's objective at both ends
    s.work_passes++;
    s.passes++;
    s.elements_read += s.wlen;
    s.AL = r.A;
    s.BL = 0.0;
    s.AR = 0.0;
    const double br = (double)n * cp_F(s, s.yR) - r.A;
    s.BR = br > 0.0 ? br : 0.0;
    s.fends = 0;
    cp_plan(s, c);
    return;
  }
  const FullEval fe = cp_full_eval(s, r);
  s.work_passes++;
  if (s.wbuf < 0) s.passes++;
  s.elements_read += s.wlen;
  s.elements_written += r.written;
  const int64_t L = fe.L, G = fe.G;
  const double A = fe.A, B = fe.B;
  const int64_t E = n - L - G;
  const bool did_split = s.split != 0;
  const bool did_count = s.counted != 0;
  const int32_t zout = s.zout;
  s.split = 0;
  s.counted = 0;
  if (L < k && k <= L + E) {
    cp_finish(s, t, L, E);
    return;
  }
  if (L + E < k) {  // x_(k) > t: move the left end (Algorithm 1, step 1.4)
    const int64_t nright = s.cR - (L + E);
    s.yL = t;
    s.AL = A;
    s.BL = B;
    s.cL = L + E;
    s.lo = did_count ? next_up(t, c.dtype) : r.succ;
    s.lo_data = did_count ? 0 : 1;
    if (did_split) {
      s.wbuf = zout;
      s.side = 1;
      s.wlen = nright;
      s.on_bracket = 1;
    }
    if (did_count) s.side = 1;
  } else {  // x_(k) < t: move the right end
    const int64_t nleft = L - s.cL;
    s.yR = t;
    s.AR = A;
    s.BR = B;
    s.cR = L;
    s.hi = did_count ? next_down(t, c.dtype) : r.pred;
    s.hi_data = did_count ? 0 : 1;
    if (did_split) {
      s.wbuf = zout;
      s.side = 0;
      s.wlen = nleft;
      s.on_bracket = 1;
    }
    if (did_count) s.side = 0;
  }
  // After a counting evaluation the bracket is one side of t, whose key bins the pass
  // counted: the plan asks for a histogram step, and the caller narrows the bracket with
  // those counts (cp_hist_narrow on split_part_geometry of part `side`) before any pass.
  if (did_count) s.narrowed = 1;
  cp_plan(s, c);
}

// After a counting evaluation that also copied the `written` elements of [spec_a, spec_b]
// to split buffer 0, and after the narrowing by its bins (if any): when every value of the
// bracket lies in that interval, the copied elements hold all of the bracket's (and maybe
// others, which the histogram passes and the gather skip) and become the working set, so
// no further pass reads the input.  Otherwise nothing changes (the copy was only spent).
CPS_HD inline void cp_adopt_spec(CpState &s, int64_t written, const CpConfig &c) {
  const int32_t had = s.spec;
  s.spec = 0;
  if (!had || s.phase == PH_DONE || s.wbuf >= 0) return;
  if (!(s.lo >= s.spec_a && s.hi <= s.spec_b)) return;
  s.wbuf = 0;
  s.side = 0;
  s.wlen = written;
  s.on_bracket = 0;
  s.narrowed = 1;
  cp_plan(s, c);
}

// After the gather pass: the bracket's elements now sit contiguously in the gather
// buffer (`gathered` of them; anything else means the counts and the data disagree).
CPS_HD inline void cp_after_gather(CpState &s, int64_t gathered) {
  s.work_passes++;
  if (s.wbuf < 0) s.passes++;
  s.elements_read += s.wlen;
  s.elements_written += gathered;
  if (gathered != s.cR - s.cL) {
    s.status = ST_INTERNAL;
    cp_finish(s, 0.0, 0, 0);
    return;
  }
  s.wbuf = 2;
  s.wlen = gathered;
  s.on_bracket = 1;
  s.filter = 0;
  s.phase = PH_FINAL;
  s.final_size = gathered;
}

// Key-histogram geometry of the bracket's possible values [lo, hi]: bin of an element
// with ordered key K is (K - klo) >> shift, with at most 2^bits bins.
template <typename K> struct HistGeom {
  K klo, khi;
  int32_t shift;
  int32_t nbins;
};

CPS_HD inline HistGeom<uint64_t> hist_geometry(double lo, double hi, int32_t dtype, int32_t bits) {
  HistGeom<uint64_t> g;
  g.klo = dtype == 0 ? (uint64_t)key32((float)lo) : key64(lo);
  g.khi = dtype == 0 ? (uint64_t)key32((float)hi) : key64(hi);
  const uint64_t span = g.khi - g.klo;
  int32_t sh = 0;
  while ((span >> sh) >= ((uint64_t)1 << bits)) ++sh;
  g.shift = sh;
  g.nbins = (int32_t)(span >> sh) + 1;
  return g;
}

CPS_HD inline double unkey_T(uint64_t k, int32_t dtype) {
  return dtype == 0 ? (double)unkey32((uint32_t)k) : unkey64(k);
}

// Narrow the bracket to bin `b` of the key bins `g`, which hold every element of the bracket:
// rank k - cL has `below` of them in lower bins and `cnt` in bin b.  The bracket becomes the
// values of that bin (an exact step: every element of the bracket lies in exactly one bin),
// the counts follow from the histogram, and one key left means the value is x_(k).
CPS_HD inline void cp_hist_narrow(CpState &s, const HistGeom<uint64_t> &g, int32_t b,
                                  int64_t below, int64_t cnt, const CpConfig &c) {
  const int64_t r = s.k - s.cL;
  if (b < 0 || b >= g.nbins || cnt < 1 || below >= r || below + cnt < r) {
    s.status = ST_INTERNAL;  // the counts and the data disagree
    cp_finish(s, 0.0, 0, 0);
    return;
  }
  const uint64_t nlo = g.klo + ((uint64_t)b << g.shift);
  uint64_t nhi = nlo + (((uint64_t)1 << g.shift) - 1);
  if (nhi > g.khi || nhi < nlo) nhi = g.khi;
  if (nlo == nhi) {
    cp_finish(s, unkey_T(nlo, c.dtype), s.cL + below, cnt);
    return;
  }
  if (nlo > g.klo) {  // everything at or below the bin's predecessor key is below the bin
    // (the key just below +0's is no value's key: it decodes to -0, which equals +0)
    const uint64_t hole = c.dtype == 0 ? 0x7fffffffull : 0x7fffffffffffffffull;
    s.yL = unkey_T(nlo - 1 == hole ? nlo - 2 : nlo - 1, c.dtype);
    s.cL += below;
  }
  if (nhi < g.khi) s.yR = unkey_T(nhi + 1, c.dtype);
  s.cR = s.cL + cnt;
  s.lo = unkey_T(nlo, c.dtype);
  s.hi = unkey_T(nhi, c.dtype);
  s.lo_data = s.hi_data = 0;
  s.on_bracket = 0;
  s.narrowed = 1;
  cp_plan(s, c);
}

// After a histogram pass over the working set, in bins of [lo, hi].
CPS_HD inline void cp_after_hist(CpState &s, int32_t b, int64_t below, int64_t cnt,
                                 const CpConfig &c) {
  s.work_passes++;
  if (s.wbuf < 0) s.passes++;
  s.elements_read += s.wlen;
  const HistGeom<uint64_t> g = hist_geometry(s.lo, s.hi, c.dtype, c.hist_bits);
  if (s.compact) {
    // the pass copied the elements inside the bracket, cR - cL of them, to buffer zout:
    // they are the working set from now on
    s.compact = 0;
    s.wbuf = s.zout;
    s.side = 0;
    s.wlen = s.cR - s.cL;
    s.on_bracket = 1;
    s.elements_written += s.wlen;
  }
  cp_hist_narrow(s, g, b, below, cnt, c);
}

// Key bins of the two parts of a split at the planned trial point t, for a split pass that
// also counts each part's elements: the low part's elements lie in [lo, t^-], the high
// part's in [t^+, hi] (t^- and t^+ the neighbours of t in T).  An empty range has no bins.
// When the state that follows the split asks for a histogram pass over the part that holds
// x_(k), the counts of that part are known already and cp_hist_narrow applies at once,
// which saves that pass.
CPS_HD inline HistGeom<uint64_t> split_part_geometry(const CpState &s, int part,
                                                     const CpConfig &c) {
  const double a = part == 0 ? s.lo : next_up(s.t, c.dtype);
  const double b = part == 0 ? next_down(s.t, c.dtype) : s.hi;
  const uint64_t ka = c.dtype == 0 ? (uint64_t)key32((float)a) : key64(a);
  const uint64_t kb = c.dtype == 0 ? (uint64_t)key32((float)b) : key64(b);
  if (ka > kb) {
    HistGeom<uint64_t> g;
    g.klo = 1;
    g.khi = 0;
    g.shift = 0;
    g.nbins = 0;
    return g;
  }
  return hist_geometry(a, b, c.dtype, c.hist_bits);
}

// After the exact select of rank k - cL among the working set's elements inside the
// bracket: `value` has `below` candidates under it and multiplicity `eq`.
CPS_HD inline void cp_after_final(CpState &s, double value, int64_t below, int64_t eq) {
  s.work_passes++;
  if (s.wbuf < 0) s.passes++;
  s.elements_read += s.wlen;
  cp_finish(s, value, s.cL + below, eq);
}

}  // namespace cps
