/*
 * Oracle helper (test infrastructure only: tests, the smoke check and the
 * benchmark's CPU-baseline leg load it; the HIP product path never does).
 *
 * Correctly rounded FP64 reductions.  The paper runs its experiments in plain
 * double precision and fixes no summation order (Section 5: MATLAB, unit
 * round-off 2^-53).  This oracle reads every row sum and inner product of the
 * method as the double nearest to the EXACT sum of its terms, where each term
 * a*b enters exactly as the pair (fl(a*b), fma(a,b,-fl(a*b))).  That value is
 * unique, so it does not depend on the order of the terms, which lets a
 * parallel device implementation agree with it bit for bit.
 *
 * The exact sum is kept as Shewchuk's non-overlapping expansion ("Adaptive
 * precision floating-point arithmetic", 1997), and the final rounding uses the
 * half-way correction of the same published msum/fsum procedure.
 *
 * Gram matrices are the exception (ord_gram below): they are read as plain
 * FP64 fused multiply-add chains in a stated order, which a device reproduces
 * bit for bit with its FP64 matrix instructions.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fopenmp -shared -fPIC
 * (no fast-math: every + - * must be an IEEE double operation; fma() is the
 * C library's correctly rounded fused multiply-add).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define CR_MAXP 64 /* a double expansion never needs more than ~40 parts */

typedef struct {
  double p[CR_MAXP];
  int n;
  double special; /* running plain sum of non-finite terms */
  int has_special;
} cr_acc;

static void acc_init(cr_acc* a) {
  a->n = 0;
  a->special = 0.0;
  a->has_special = 0;
}

/* Add one double exactly to the expansion. */
static void acc_add(cr_acc* a, double x) {
  if (!isfinite(x)) {
    a->special += x;
    a->has_special = 1;
    return;
  }
  int i = 0;
  for (int j = 0; j < a->n; ++j) {
    double y = a->p[j];
    if (fabs(x) < fabs(y)) {
      double t = x;
      x = y;
      y = t;
    }
    double hi = x + y;
    double lo = y - (hi - x);
    if (lo != 0.0) a->p[i++] = lo;
    x = hi;
  }
  if (!isfinite(x)) { /* exact sum overflowed: report it like a plain sum */
    a->special += x;
    a->has_special = 1;
    a->n = i;
    return;
  }
  a->p[i] = x;
  a->n = i + 1;
}

/* Add the exact product a*b (two doubles, error-free by fma). */
static void acc_add_prod(cr_acc* acc, double a, double b) {
  double p = a * b;
  if (!isfinite(p)) {
    acc_add(acc, p);
    return;
  }
  double e = fma(a, b, -p);
  acc_add(acc, p);
  if (e != 0.0) acc_add(acc, e);
}

/* Round the exact sum held in the expansion to the nearest double
 * (ties to even), as the msum/fsum procedure does. */
static double acc_round(const cr_acc* a) {
  if (a->has_special) {
    double s = a->special;
    for (int j = 0; j < a->n; ++j) s += a->p[j];
    return s;
  }
  int n = a->n;
  if (n == 0) return 0.0;
  double hi = a->p[--n];
  double lo = 0.0;
  while (n > 0) {
    double x = hi;
    double y = a->p[--n];
    hi = x + y;
    double yr = hi - x;
    lo = y - yr;
    if (lo != 0.0) break;
  }
  if (n > 0 && ((lo < 0.0 && a->p[n - 1] < 0.0) || (lo > 0.0 && a->p[n - 1] > 0.0))) {
    double y = lo * 2.0;
    double x = hi + y;
    double yr = x - hi;
    if (y == yr) hi = x;
  }
  return hi;
}

/* ---------------------------------------------------------------- exports */

/* Correctly rounded sum of t[0..n). */
double cr_sum(const double* t, int64_t n) {
  cr_acc a;
  acc_init(&a);
  for (int64_t i = 0; i < n; ++i) acc_add(&a, t[i]);
  return acc_round(&a);
}

/* Correctly rounded inner product sum_i x[i]*y[i]. */
double cr_dot(const double* x, const double* y, int64_t n) {
  cr_acc a;
  acc_init(&a);
  for (int64_t i = 0; i < n; ++i) acc_add_prod(&a, x[i], y[i]);
  return acc_round(&a);
}

/*
 * Row sums of a CSR matrix times a vector, plus diagonal extra terms:
 *   out[i] = RN( sum_k val[k]*u[col[k]]  +  sum_e coef[e]*vec[e][i] )
 * for rows i in [0,n).  rowptr has n+1 entries; vec is an array of nextra
 * pointers to length-n vectors.  Used for A*u (nextra=0), for the three-term
 * polynomial-basis numerator A*u - theta*u - sigma*w, and for b - A*x.
 */
void cr_csr_rowsum(int64_t n, const int32_t* rowptr, const int32_t* col, const double* val,
                   const double* u, int32_t nextra, const double* coef, const double* const* vec,
                   double* out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    cr_acc a;
    acc_init(&a);
    for (int32_t k = rowptr[i]; k < rowptr[i + 1]; ++k) acc_add_prod(&a, val[k], u[col[k]]);
    for (int32_t e = 0; e < nextra; ++e) acc_add_prod(&a, coef[e], vec[e][i]);
    out[i] = acc_round(&a);
  }
}

/*
 * Row-wise linear combination of d column vectors (column-major, leading
 * dimension ld), with an optional base vector entering with weight 1:
 *   out[i] = RN( base[i] + sum_a Y[a*ld+i]*c[a] ).
 */
void cr_rows_comb(int64_t n, int32_t d, const double* Y, int64_t ld, const double* c,
                  const double* base, double* out) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    cr_acc a;
    acc_init(&a);
    if (base) acc_add(&a, base[i]);
    for (int32_t k = 0; k < d; ++k) acc_add_prod(&a, Y[(int64_t)k * ld + i], c[k]);
    out[i] = acc_round(&a);
  }
}

/*
 * Gram matrix G = Y^T Y of d columns of length n (column-major, leading
 * dimension ld): every entry is the correctly rounded inner product, written
 * to both G[a*d+b] and G[b*d+a].
 */
void cr_gram(int64_t n, int32_t d, const double* Y, int64_t ld, double* G) {
  int32_t npair = d * (d + 1) / 2;
#pragma omp parallel for schedule(dynamic, 1)
  for (int32_t q = 0; q < npair; ++q) {
    int32_t a = 0, rem = q;
    while (rem >= d - a) {
      rem -= d - a;
      ++a;
    }
    int32_t b = a + rem;
    double g = cr_dot(Y + (int64_t)a * ld, Y + (int64_t)b * ld, n);
    G[a * d + b] = g;
    G[b * d + a] = g;
  }
}

/*
 * Gram matrix in the oracle's order for Gram matrices (reading R9, Gram
 * part): the rows, zero-padded to a multiple of ORD_GROUP, fall into groups of
 * ORD_GROUP consecutive rows; a group's partial is the chain of IEEE fused
 * multiply-adds s <- fma(y_ra, y_rb, s) over its rows in order, from s = +0;
 * the partials of the groups, zero-padded to the next power of two P, are
 * added by pairwise summation: PT(v[0..P)) = PT(v[0..P/2)) + PT(v[P/2..P)),
 * PT of one value = that value.  Written to G[a*d+b] and G[b*d+a].
 */
#define ORD_GROUP 1024

static double ord_pt(const double* v, int64_t lo, int64_t len, int64_t count) {
  if (len == 1) return lo < count ? v[lo] : 0.0;
  const int64_t h = len / 2;
  const double left = ord_pt(v, lo, h, count);
  const double right = ord_pt(v, lo + h, h, count);
  return left + right;
}

void ord_gram(int64_t n, int32_t d, const double* Y, int64_t ld, double* G) {
  const int64_t ng = (n + ORD_GROUP - 1) / ORD_GROUP;
  int64_t P = 1;
  while (P < ng) P <<= 1;
  int32_t npair = d * (d + 1) / 2;
#pragma omp parallel for schedule(dynamic, 1)
  for (int32_t q = 0; q < npair; ++q) {
    int32_t a = 0, rem = q;
    while (rem >= d - a) {
      rem -= d - a;
      ++a;
    }
    int32_t b = a + rem;
    const double* ya = Y + (int64_t)a * ld;
    const double* yb = Y + (int64_t)b * ld;
    double* part = (double*)malloc(sizeof(double) * (size_t)(ng > 0 ? ng : 1));
    for (int64_t g = 0; g < ng; ++g) {
      double s = 0.0;
      for (int64_t r = g * ORD_GROUP; r < (g + 1) * ORD_GROUP; ++r)
        s = r < n ? fma(ya[r], yb[r], s) : fma(0.0, 0.0, s);
      part[g] = s;
    }
    double gab = ng > 0 ? ord_pt(part, 0, P, ng) : 0.0;
    free(part);
    G[a * d + b] = gab;
    G[b * d + a] = gab;
  }
}

/* Threads the row loops above will use (for reporting). */
int cr_num_threads(void) {
#ifdef _OPENMP
  extern int omp_get_max_threads(void);
  return omp_get_max_threads();
#else
  return 1;
#endif
}
