/*
 * CPU oracle for exact k-th order statistic selection by convex minimization.
 *
 * TEST INFRASTRUCTURE ONLY.  This library exists to check the GPU library and to
 * time a CPU baseline; only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg may load it.  It shares no code, header or table with the HIP
 * library.  Everything here is the plain definition, written for a reader to check
 * against the paper by eye, not for speed:
 *
 *   - selection (Section 1): x_(k) is the k-th smallest element of x, 1-based k,
 *     ordered by IEEE "<"; the median is x_([(n+1)/2]).  Found by quickselect with a
 *     three-way partition (Section 1 names quickselect as the classical CPU method),
 *     falling back to a library sort of the sub-range when the recursion gets deep.
 *     The counts #(x<m), #(x=m), #(x>m) come from one plain scan of the input.
 *   - objective (Section 3, Eqs. 1-2): f(y) = sum_i max(alpha (x_i - y), beta (y - x_i))
 *     with alpha = k - 1/2 and beta = n - k + 1/2, every term in double precision,
 *     summed with Neumaier's compensated summation.  (The printed weights of Eq. 2 put
 *     n-k+1/2 on x_i - y >= 0, which selects x_(n-k+1); the orientation used here is the
 *     one whose minimiser is x_(k).)  The subdifferential end points follow Section 3:
 *     g-(y) = n (L - k + 1/2), g+(y) = n (L + E - k + 1/2).
 *   - least median of squares (Section 6): r_i = (y_i - sum_j X_ij b_j)^2 with the sum
 *     taken left to right in j, each product and sum rounded (no fused multiply-add:
 *     build with -ffp-contract=off), then the lower median of r.
 *   - least trimmed squares (Section 6): the sum of the h smallest squared residuals, by
 *     its definition (a sorted copy, the first h entries summed with Neumaier's
 *     compensated summation), with the h-th smallest m and the counts #(r < m), #(r = m).
 *   - k nearest neighbours (Section 6, last paragraph): squared Euclidean distances from a
 *     query to every data point, summed left to right over the coordinates without fused
 *     multiply-add, and the mean of the ordinates of the k nearest points, by definition:
 *     the points sorted by distance (ties in index order) and the first k ordinates summed
 *     (Neumaier) and divided by k.
 *
 * NaN is not an ordered value: any NaN in x makes the calls return ORC_ENAN.
 * The returned value is canonicalised as m + 0.0, so -0.0 is reported as +0.0.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_EINVAL (-1)
#define ORC_ENAN (-2)
#define ORC_ENOMEM (-3)

typedef struct {
  uint64_t value_bits; /* raw bits of the selected element, zero-extended */
  double value;        /* the selected element, widened to double */
  int64_t less, equal, greater;
} orc_result;

typedef struct {
  double f;     /* objective at y */
  double A;     /* sum over x_i > y of (x_i - y) */
  double B;     /* sum over x_i < y of (y - x_i) */
  int64_t L, E, G;
  double pred;  /* largest x_i < y, -inf if none */
  double succ;  /* smallest x_i > y, +inf if none */
  double gminus, gplus;
} orc_eval;

/* ---------------------------------------------------------------- helpers */

static void neumaier_add(double *sum, double *comp, double v) {
  double t = *sum + v;
  if (fabs(*sum) >= fabs(v))
    *comp += (*sum - t) + v;
  else
    *comp += (v - t) + *sum;
  *sum = t;
}

static int cmp_double(const void *a, const void *b) {
  double x = *(const double *)a, y = *(const double *)b;
  return (x > y) - (x < y);
}

static int log2_floor(int64_t v) {
  int r = 0;
  while (v > 1) { v >>= 1; r++; }
  return r;
}

/* Median of three values, used as the quickselect pivot. */
static double median3(double a, double b, double c) {
  if (a < b) {
    if (b < c) return b;
    return (a < c) ? c : a;
  }
  if (a < c) return a;
  return (b < c) ? c : b;
}

/*
 * Quickselect on w[0..n): on return the element of rank r (0-based) is known and
 * returned.  Each round partitions the live range [lo,hi) three ways around a pivot:
 * [lo,lt) < p, [lt,gt) == p, [gt,hi) > p.  The rank then lies in exactly one part.
 */
static double quickselect(double *w, int64_t n, int64_t r) {
  int64_t lo = 0, hi = n;
  int depth = 0, max_depth = 2 * log2_floor(n) + 8;
  while (hi - lo > 1) {
    if (depth++ > max_depth) {
      qsort(w + lo, (size_t)(hi - lo), sizeof(double), cmp_double);
      return w[r];
    }
    int64_t mid = lo + (hi - lo) / 2;
    double p = median3(w[lo], w[mid], w[hi - 1]);
    int64_t lt = lo, i = lo, gt = hi;
    while (i < gt) {
      double v = w[i];
      if (v < p) {
        w[i] = w[lt]; w[lt] = v; lt++; i++;
      } else if (v > p) {
        gt--; w[i] = w[gt]; w[gt] = v;
      } else {
        i++;
      }
    }
    if (r < lt)
      hi = lt;
    else if (r >= gt)
      lo = gt;
    else
      return p;
  }
  return w[lo];
}

/* ---------------------------------------------------------------- selection */

#define DEFINE_SELECT(NAME, T, BITS_T)                                              \
  int NAME(const T *x, int64_t n, int64_t k, orc_result *out) {                     \
    if (!x || !out || n < 1 || k < 1 || k > n) return ORC_EINVAL;                   \
    double *w = (double *)malloc((size_t)n * sizeof(double));                       \
    if (!w) return ORC_ENOMEM;                                                      \
    for (int64_t i = 0; i < n; i++) {                                               \
      if (isnan(x[i])) { free(w); return ORC_ENAN; }                                \
      w[i] = (double)x[i];                                                          \
    }                                                                               \
    double m = quickselect(w, n, k - 1);                                            \
    free(w);                                                                        \
    T mt = (T)m + (T)0.0; /* canonical zero */                                      \
    int64_t less = 0, equal = 0;                                                    \
    for (int64_t i = 0; i < n; i++) {                                               \
      if (x[i] < mt) less++;                                                        \
      else if (x[i] == mt) equal++;                                                 \
    }                                                                               \
    BITS_T bits;                                                                    \
    memcpy(&bits, &mt, sizeof(bits));                                               \
    out->value_bits = (uint64_t)bits;                                               \
    out->value = (double)mt;                                                        \
    out->less = less;                                                               \
    out->equal = equal;                                                             \
    out->greater = n - less - equal;                                                \
    return ORC_OK;                                                                  \
  }

DEFINE_SELECT(orc_select_f32, float, uint32_t)
DEFINE_SELECT(orc_select_f64, double, uint64_t)

/* Time only the selection itself on a caller-provided working copy (benchmark use). */
int orc_quickselect_inplace(double *w, int64_t n, int64_t k, double *value) {
  if (!w || !value || n < 1 || k < 1 || k > n) return ORC_EINVAL;
  *value = quickselect(w, n, k - 1);
  return ORC_OK;
}

/* ---------------------------------------------------------------- objective */

#define DEFINE_OBJECTIVE(NAME, T)                                                    \
  int NAME(const T *x, int64_t n, int64_t k, const double *ys, int64_t ny,          \
           orc_eval *out) {                                                          \
    if (!x || !ys || !out || n < 1 || k < 1 || k > n || ny < 0) return ORC_EINVAL;  \
    for (int64_t i = 0; i < n; i++)                                                  \
      if (isnan(x[i])) return ORC_ENAN;                                              \
    const double alpha = (double)k - 0.5, beta = (double)n - (double)k + 0.5;        \
    for (int64_t j = 0; j < ny; j++) {                                               \
      const double y = ys[j];                                                        \
      double fs = 0, fc = 0, as = 0, ac = 0, bs = 0, bc = 0;                         \
      int64_t L = 0, E = 0, G = 0;                                                   \
      double pred = -INFINITY, succ = INFINITY;                                      \
      for (int64_t i = 0; i < n; i++) {                                              \
        const double xi = (double)x[i];                                              \
        const double d = xi - y;                                                     \
        const double up = alpha * d, down = beta * (-d);                             \
        neumaier_add(&fs, &fc, up > down ? up : down);                               \
        if (xi > y) {                                                                \
          G++;                                                                       \
          neumaier_add(&as, &ac, d);                                                 \
          if (xi < succ) succ = xi;                                                  \
        } else if (xi < y) {                                                         \
          L++;                                                                       \
          neumaier_add(&bs, &bc, -d);                                                \
          if (xi > pred) pred = xi;                                                  \
        } else {                                                                     \
          E++;                                                                       \
        }                                                                            \
      }                                                                              \
      out[j].f = fs + fc;                                                            \
      out[j].A = as + ac;                                                            \
      out[j].B = bs + bc;                                                            \
      out[j].L = L;                                                                  \
      out[j].E = E;                                                                  \
      out[j].G = G;                                                                  \
      out[j].pred = pred;                                                            \
      out[j].succ = succ;                                                            \
      out[j].gminus = (double)n * ((double)L - (double)k + 0.5);                     \
      out[j].gplus = (double)n * ((double)(L + E) - (double)k + 0.5);                \
    }                                                                                \
    return ORC_OK;                                                                   \
  }

DEFINE_OBJECTIVE(orc_objective_f32, float)
DEFINE_OBJECTIVE(orc_objective_f64, double)

/* ---------------------------------------------------------------- least median of squares */

/* r_i = (y_i - sum_j X_ij b_j)^2, X row-major n x p, left-to-right sum, every step rounded. */
int orc_lms_residuals(const double *X, const double *y, const double *b, int64_t n, int32_t p,
                      double *r) {
  if (!X || !y || !b || !r || n < 1 || p < 1) return ORC_EINVAL;
  for (int64_t i = 0; i < n; i++) {
    const double *row = X + i * (int64_t)p;
    double s = row[0] * b[0];
    for (int32_t j = 1; j < p; j++) {
      double prod = row[j] * b[j];
      s = s + prod;
    }
    double d = y[i] - s;
    r[i] = d * d;
  }
  return ORC_OK;
}

/* For each of the m candidates (rows of betas, m x p): the lower median of its squared residuals. */
int orc_lms_median_sq(const double *X, const double *y, const double *betas, int64_t n, int32_t p,
                      int64_t m, orc_result *out) {
  if (!X || !y || !betas || !out || n < 1 || p < 1 || m < 0) return ORC_EINVAL;
  double *r = (double *)malloc((size_t)n * sizeof(double));
  if (!r) return ORC_ENOMEM;
  const int64_t k = (n + 1) / 2;
  int rc = ORC_OK;
  for (int64_t c = 0; c < m && rc == ORC_OK; c++) {
    rc = orc_lms_residuals(X, y, betas + c * (int64_t)p, n, p, r);
    if (rc == ORC_OK) rc = orc_select_f64(r, n, k, &out[c]);
  }
  free(r);
  return rc;
}

/* ---------------------------------------------------------------- least trimmed squares */

typedef struct {
  double F;        /* sum of the h smallest values */
  double m;        /* the h-th smallest value */
  int64_t below;   /* #(r < m) */
  int64_t a;       /* h - #(r < m): how many copies of m the sum takes */
  int64_t b;       /* #(r = m) */
} orc_trim;

/* The sum of the h smallest of r[0..n) (1 <= h <= n): sort a copy and add its first h
 * entries in ascending order with compensation. */
int orc_trimmed_sum_f64(const double *r, int64_t n, int64_t h, orc_trim *out) {
  if (!r || !out || n < 1 || h < 1 || h > n) return ORC_EINVAL;
  for (int64_t i = 0; i < n; i++)
    if (isnan(r[i])) return ORC_ENAN;
  double *w = (double *)malloc((size_t)n * sizeof(double));
  if (!w) return ORC_ENOMEM;
  memcpy(w, r, (size_t)n * sizeof(double));
  qsort(w, (size_t)n, sizeof(double), cmp_double);
  double s = 0, c = 0;
  for (int64_t i = 0; i < h; i++) neumaier_add(&s, &c, w[i]);
  const double m = w[h - 1] + 0.0;
  int64_t below = 0, eq = 0;
  for (int64_t i = 0; i < n; i++) {
    below += r[i] < m;
    eq += r[i] == m;
  }
  out->F = s + c;
  out->m = m;
  out->below = below;
  out->a = h - below;
  out->b = eq;
  free(w);
  return ORC_OK;
}

/* For each of the m candidates: the least-trimmed-squares objective of its squared
 * residuals (as orc_lms_residuals) with h kept. */
int orc_lts_objective(const double *X, const double *y, const double *betas, int64_t n, int32_t p,
                      int64_t m, int64_t h, orc_trim *out) {
  if (!X || !y || !betas || !out || n < 1 || p < 1 || m < 0 || h < 1 || h > n) return ORC_EINVAL;
  double *r = (double *)malloc((size_t)n * sizeof(double));
  if (!r) return ORC_ENOMEM;
  int rc = ORC_OK;
  for (int64_t c = 0; c < m && rc == ORC_OK; c++) {
    rc = orc_lms_residuals(X, y, betas + c * (int64_t)p, n, p, r);
    if (rc == ORC_OK) rc = orc_trimmed_sum_f64(r, n, h, &out[c]);
  }
  free(r);
  return rc;
}

/* ---------------------------------------------------------------- k nearest neighbours */

/* d_i = sum_j (P_ij - q_j)^2 over j = 0..dim-1 left to right, every difference, square and
 * sum rounded to float (float arithmetic, no fused multiply-add). */
int orc_knn_distances(const float *P, const float *q, int64_t n, int32_t dim, float *d) {
  if (!P || !q || !d || n < 1 || dim < 1) return ORC_EINVAL;
  for (int64_t i = 0; i < n; i++) {
    const float *row = P + i * (int64_t)dim;
    float s = 0.0f;
    for (int32_t j = 0; j < dim; j++) {
      const float e = row[j] - q[j];
      const float sq = e * e;
      s = j == 0 ? sq : s + sq;
    }
    d[i] = s;
  }
  return ORC_OK;
}

static int cmp_float(const void *a, const void *b) {
  const float x = *(const float *)a, y = *(const float *)b;
  return (x > y) - (x < y);
}

typedef struct {
  double mean;     /* mean ordinate of the k nearest points */
  float dk;        /* the k-th smallest distance */
  int32_t pad;
  int64_t below;   /* #(d < dk) */
  int64_t equal;   /* #(d = dk) */
} orc_knn;

/* For each of the nq queries (rows of Q): the k-th smallest squared Euclidean distance dk
 * to the n points (rows of P), found by sorting, and the mean ordinate of the k nearest
 * points: (sum of f over d < dk + (a / b) * sum of f over d = dk) / k with b = #(d = dk) and
 * a = k - #(d < dk), the weight of Section 6 for the points at the k-th distance (exactly k
 * points' worth; with no tie it is the plain mean of the k nearest). */
int orc_knn_mean(const float *P, const float *f, const float *Q, int64_t n, int32_t dim, int64_t nq,
                 int64_t k, orc_knn *out) {
  if (!P || !f || !Q || !out || n < 1 || dim < 1 || nq < 0 || k < 1 || k > n) return ORC_EINVAL;
  float *d = (float *)malloc((size_t)n * sizeof(float));
  float *w = (float *)malloc((size_t)n * sizeof(float));
  if (!d || !w) {
    free(d);
    free(w);
    return ORC_ENOMEM;
  }
  for (int64_t c = 0; c < nq; c++) {
    orc_knn_distances(P, Q + c * (int64_t)dim, n, dim, d);
    for (int64_t i = 0; i < n; i++)
      if (isnan(d[i])) {
        free(d);
        free(w);
        return ORC_ENAN;
      }
    memcpy(w, d, (size_t)n * sizeof(float));
    qsort(w, (size_t)n, sizeof(float), cmp_float);
    const float dk = w[k - 1] + 0.0f;
    int64_t below = 0, eq = 0;
    double sb = 0, cb = 0, se = 0, ce = 0;
    for (int64_t i = 0; i < n; i++) {
      if (d[i] < dk) {
        below++;
        neumaier_add(&sb, &cb, (double)f[i]);
      } else if (d[i] == dk) {
        eq++;
        neumaier_add(&se, &ce, (double)f[i]);
      }
    }
    const double a = (double)(k - below);
    out[c].mean = ((sb + cb) + a * (se + ce) / (double)eq) / (double)k;
    out[c].dk = dk;
    out[c].pad = 0;
    out[c].below = below;
    out[c].equal = eq;
  }
  free(d);
  free(w);
  return ORC_OK;
}
