/*
 * Reference permanents -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, slow CPU code used by the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark to check the HIP library.  The library never
 * includes, links or calls anything in this directory, and this file shares no
 * code with it.
 *
 * What is computed (Masschelein, Richer & Ayers, "Optimizing and benchmarking
 * the computation of the permanent of general matrices"):
 *
 *   per(A) = sum over injective maps s:[m]->[n] of prod_i a[i][s(i)]    (m <= n)
 *   per(A) = per(A^T)                                                   (m >  n)
 *
 * (Sec. 1.1, Eq. permanent_definition and Eq. rectangular_permanent_definition).
 * The empty product convention gives per = 1 for m = 0.
 *
 * Four evaluators:
 *   brute    -- the definition written out: every injective map, one product
 *               each, one running sum.                       (Sec. 1.1)
 *   laplace  -- the same sum grouped by distributivity (memoised Laplace
 *               expansion).  Row form: f_i(S) = sum_{j in S} a[i-1][j] *
 *               f_{i-1}(S\{j}) over column sets S; column form: g_j(R) =
 *               g_{j-1}(R) + sum_{i in R} a[i][j] g_{j-1}(R\{i}) over row sets
 *               R.  Each term of the definition is visited exactly once.
 *   glynn    -- Glynn's formula, Sec. 1.2 Eq. glynn, and for m < n the padded
 *               form Eq. glynn_filled_matrix / Eq. glynn_rectangle, summed in
 *               reflected-Gray-code order over the 2^(n-1) sign vectors with
 *               delta_1 = +1.  Double-double throughout.  Used where the
 *               definition is out of reach (n >= 31).
 *   ryser    -- Ryser's formula, Sec. 1.2 Eq. ryser_square (m = n) and
 *               Eq. ryser_rectangle read over column *subsets* (m < n),
 *               Gray-code order over all 2^n column subsets, double-double.
 *
 * Arithmetic:
 *   integer input (int64)  -> products and sums modulo 2^128 (unsigned wrap);
 *                             exact whenever the true value fits in int128.
 *   real input (double)    -> products rounded in binary64 (brute) or
 *                             double-double (others); sums in double-double.
 *   complex input          -> the same per component, interleaved re,im.
 *
 * Every entry point returns 0 on success, -1 on bad arguments, -2 when the
 * request exceeds the evaluator's size limit, -3 on allocation failure.
 * Built with -ffp-contract=off and without -ffast-math so that TwoSum and
 * TwoProd are exact.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>
#include <pthread.h>
#include <unistd.h>

typedef unsigned __int128 u128;

/* ------------------------------------------------------------------ */
/* double-double arithmetic (Dekker / Knuth error-free transformations) */
/* ------------------------------------------------------------------ */
typedef struct { double hi, lo; } dd;
typedef struct { dd re, im; } cdd;

static inline dd fast_two_sum(double a, double b) {      /* |a| >= |b| */
  double s = a + b;
  double e = b - (s - a);
  dd r = {s, e};
  return r;
}
static inline dd two_sum(double a, double b) {
  double s = a + b;
  double bb = s - a;
  double e = (a - (s - bb)) + (b - bb);
  dd r = {s, e};
  return r;
}
static inline dd two_prod(double a, double b) {
  double p = a * b;
  double e = fma(a, b, -p);
  dd r = {p, e};
  return r;
}
static inline dd dd_from(double a) { dd r = {a, 0.0}; return r; }
static inline dd dd_add(dd x, dd y) {
  dd s = two_sum(x.hi, y.hi);
  dd t = two_sum(x.lo, y.lo);
  s.lo += t.hi;
  s = fast_two_sum(s.hi, s.lo);
  s.lo += t.lo;
  return fast_two_sum(s.hi, s.lo);
}
static inline dd dd_neg(dd x) { dd r = {-x.hi, -x.lo}; return r; }
static inline dd dd_sub(dd x, dd y) { return dd_add(x, dd_neg(y)); }
static inline dd dd_mul(dd x, dd y) {
  dd p = two_prod(x.hi, y.hi);
  p.lo += x.hi * y.lo;
  p.lo += x.lo * y.hi;
  return fast_two_sum(p.hi, p.lo);
}
static inline dd dd_mul_d(dd x, double b) { return dd_mul(x, dd_from(b)); }

static inline cdd cdd_zero(void) { cdd r = {{0, 0}, {0, 0}}; return r; }
static inline cdd cdd_add(cdd x, cdd y) { cdd r = {dd_add(x.re, y.re), dd_add(x.im, y.im)}; return r; }
static inline cdd cdd_neg(cdd x) { cdd r = {dd_neg(x.re), dd_neg(x.im)}; return r; }
static inline cdd cdd_mul(cdd x, cdd y) {
  cdd r = {dd_sub(dd_mul(x.re, y.re), dd_mul(x.im, y.im)),
           dd_add(dd_mul(x.re, y.im), dd_mul(x.im, y.re))};
  return r;
}
static inline cdd cdd_scale(cdd x, double s) {  /* s exact power of two or small */
  cdd r = {dd_mul_d(x.re, s), dd_mul_d(x.im, s)};
  return r;
}

/* ------------------------------------------------------------------ */
/* matrix access: logical m x n with m <= n; `tr` reads the transpose    */
/* ------------------------------------------------------------------ */
typedef struct {
  int m, n;          /* logical shape after orientation, m <= n */
  int tr;            /* 1: logical (i,j) is stored at (j,i) */
  int64_t lda;       /* leading dimension in elements of the stored matrix */
  const void *a;
} mat;

static int orient(int m, int n, const void *a, int64_t lda, mat *out) {
  if (m < 0 || n < 0) return -1;
  if (m > 0 && a == NULL) return -1;
  if (m > 0 && lda < n) return -1;
  out->a = a; out->lda = lda;
  if (m <= n) { out->m = m; out->n = n; out->tr = 0; }
  else        { out->m = n; out->n = m; out->tr = 1; }
  return 0;
}
static inline int64_t off(const mat *A, int i, int j) {
  return A->tr ? (int64_t)j * A->lda + i : (int64_t)i * A->lda + j;
}
static inline int64_t geti(const mat *A, int i, int j) { return ((const int64_t *)A->a)[off(A, i, j)]; }
static inline double getr(const mat *A, int i, int j) { return ((const double *)A->a)[off(A, i, j)]; }
static inline double getc_re(const mat *A, int i, int j) { return ((const double *)A->a)[2 * off(A, i, j)]; }
static inline double getc_im(const mat *A, int i, int j) { return ((const double *)A->a)[2 * off(A, i, j) + 1]; }

/* ------------------------------------------------------------------ */
/* a tiny pthread task pool: tasks 0..ntasks-1 pulled from a counter;  */
/* each task writes its own slot, slots are combined in task order.    */
/* ------------------------------------------------------------------ */
typedef void (*task_fn)(void *ctx, int64_t task);
typedef struct {
  task_fn fn; void *ctx; int64_t ntasks;
  int64_t next; pthread_mutex_t mu;
} pool;

static void *pool_worker(void *p_) {
  pool *p = (pool *)p_;
  for (;;) {
    pthread_mutex_lock(&p->mu);
    int64_t t = p->next++;
    pthread_mutex_unlock(&p->mu);
    if (t >= p->ntasks) break;
    p->fn(p->ctx, t);
  }
  return NULL;
}

static int resolve_threads(int nthreads) {
  if (nthreads > 0) return nthreads;
  long c = sysconf(_SC_NPROCESSORS_ONLN);
  return c > 0 ? (int)c : 1;
}

static void run_tasks(task_fn fn, void *ctx, int64_t ntasks, int nthreads) {
  pool p; p.fn = fn; p.ctx = ctx; p.ntasks = ntasks; p.next = 0;
  pthread_mutex_init(&p.mu, NULL);
  nthreads = resolve_threads(nthreads);
  if (nthreads > ntasks) nthreads = (int)(ntasks > 0 ? ntasks : 1);
  if (nthreads <= 1) { pool_worker(&p); pthread_mutex_destroy(&p.mu); return; }
  pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nthreads);
  int started = 0;
  for (int t = 0; t < nthreads; ++t)
    if (pthread_create(&th[t], NULL, pool_worker, &p) == 0) ++started;
  if (started == 0) pool_worker(&p);
  for (int t = 0; t < started; ++t) pthread_join(th[t], NULL);
  free(th);
  pthread_mutex_destroy(&p.mu);
}

int oracle_hardware_threads(void) { return resolve_threads(0); }

/* ================================================================== */
/* 1. brute force: the definition                                       */
/* ================================================================== */
/* A task fixes the images of the first one or two rows; the remaining rows
 * are enumerated depth-first over unused columns.  The running product is the
 * left-to-right product prod_{i<k} a[i][s(i)], extended by one factor per
 * level, so each leaf holds exactly prod_i a[i][s(i)] for one injective s. */

typedef struct {
  const mat *A; int fixed;  /* rows whose images a task fixes (1 or 2) */
  int kind;                 /* 0 int, 1 real, 2 complex */
  u128 *ires; dd *rres; cdd *cres;
} brute_ctx;

static void brute_int_rec(const mat *A, int i, uint64_t used, u128 prod, u128 *acc) {
  if (i == A->m) { *acc += prod; return; }
  for (int j = 0; j < A->n; ++j) {
    if (used >> j & 1) continue;
    u128 f = (u128)(__int128)geti(A, i, j);
    brute_int_rec(A, i + 1, used | (1ull << j), prod * f, acc);
  }
}
static void brute_real_rec(const mat *A, int i, uint64_t used, double prod, dd *acc) {
  if (i == A->m) { *acc = dd_add(*acc, dd_from(prod)); return; }
  for (int j = 0; j < A->n; ++j) {
    if (used >> j & 1) continue;
    brute_real_rec(A, i + 1, used | (1ull << j), prod * getr(A, i, j), acc);
  }
}
static void brute_cplx_rec(const mat *A, int i, uint64_t used, double pr, double pi, cdd *acc) {
  if (i == A->m) {
    acc->re = dd_add(acc->re, dd_from(pr));
    acc->im = dd_add(acc->im, dd_from(pi));
    return;
  }
  for (int j = 0; j < A->n; ++j) {
    if (used >> j & 1) continue;
    double ar = getc_re(A, i, j), ai = getc_im(A, i, j);
    double qr = pr * ar - pi * ai;
    double qi = pr * ai + pi * ar;
    brute_cplx_rec(A, i + 1, used | (1ull << j), qr, qi, acc);
  }
}

static void brute_task(void *c_, int64_t t) {
  brute_ctx *c = (brute_ctx *)c_;
  const mat *A = c->A;
  int n = A->n;
  int j0 = (int)(t / (c->fixed == 2 ? n : 1));
  int j1 = (int)(t % n);
  if (c->fixed == 1) j0 = (int)t;
  if (c->fixed == 2 && j0 == j1) return;           /* not injective: slot stays 0 */
  uint64_t used = 1ull << j0;
  if (c->kind == 0) {
    u128 prod = (u128)(__int128)geti(A, 0, j0), acc = 0;
    if (c->fixed == 2) { prod *= (u128)(__int128)geti(A, 1, j1); used |= 1ull << j1; }
    brute_int_rec(A, c->fixed, used, prod, &acc);
    c->ires[t] = acc;
  } else if (c->kind == 1) {
    double prod = getr(A, 0, j0); dd acc = {0, 0};
    if (c->fixed == 2) { prod *= getr(A, 1, j1); used |= 1ull << j1; }
    brute_real_rec(A, c->fixed, used, prod, &acc);
    c->rres[t] = acc;
  } else {
    double pr = getc_re(A, 0, j0), pi = getc_im(A, 0, j0); cdd acc = cdd_zero();
    if (c->fixed == 2) {
      double ar = getc_re(A, 1, j1), ai = getc_im(A, 1, j1);
      double qr = pr * ar - pi * ai, qi = pr * ai + pi * ar;
      pr = qr; pi = qi; used |= 1ull << j1;
    }
    brute_cplx_rec(A, c->fixed, used, pr, pi, &acc);
    c->cres[t] = acc;
  }
}

static int brute_common(int kind, int m, int n, const void *a, int64_t lda, int nthreads,
                        void *out) {
  mat A;
  if (orient(m, n, a, lda, &A)) return -1;
  if (A.n > 63) return -2;
  if (A.m == 0) {
    if (kind == 0) { ((uint64_t *)out)[0] = 1; ((uint64_t *)out)[1] = 0; }
    else if (kind == 1) { ((double *)out)[0] = 1; ((double *)out)[1] = 0; }
    else { double *o = (double *)out; o[0] = 1; o[1] = 0; o[2] = 0; o[3] = 0; }
    return 0;
  }
  brute_ctx c; memset(&c, 0, sizeof c);
  c.A = &A; c.kind = kind; c.fixed = A.m >= 2 ? 2 : 1;
  int64_t ntasks = c.fixed == 2 ? (int64_t)A.n * A.n : A.n;
  if (kind == 0) c.ires = (u128 *)calloc((size_t)ntasks, sizeof(u128));
  if (kind == 1) c.rres = (dd *)calloc((size_t)ntasks, sizeof(dd));
  if (kind == 2) c.cres = (cdd *)calloc((size_t)ntasks, sizeof(cdd));
  if (!c.ires && !c.rres && !c.cres) return -3;
  run_tasks(brute_task, &c, ntasks, nthreads);
  if (kind == 0) {
    u128 s = 0;
    for (int64_t t = 0; t < ntasks; ++t) s += c.ires[t];
    ((uint64_t *)out)[0] = (uint64_t)s; ((uint64_t *)out)[1] = (uint64_t)(s >> 64);
    free(c.ires);
  } else if (kind == 1) {
    dd s = {0, 0};
    for (int64_t t = 0; t < ntasks; ++t) s = dd_add(s, c.rres[t]);
    ((double *)out)[0] = s.hi; ((double *)out)[1] = s.lo;
    free(c.rres);
  } else {
    cdd s = cdd_zero();
    for (int64_t t = 0; t < ntasks; ++t) s = cdd_add(s, c.cres[t]);
    double *o = (double *)out; o[0] = s.re.hi; o[1] = s.re.lo; o[2] = s.im.hi; o[3] = s.im.lo;
    free(c.cres);
  }
  return 0;
}

/* out: {lo, hi} 64-bit words of the value modulo 2^128 */
int oracle_brute_i64(int m, int n, const int64_t *a, int64_t lda, int nthreads, uint64_t *out) {
  return brute_common(0, m, n, a, lda, nthreads, out);
}
/* out: {hi, lo} double-double */
int oracle_brute_f64(int m, int n, const double *a, int64_t lda, int nthreads, double *out) {
  return brute_common(1, m, n, a, lda, nthreads, out);
}
/* a: interleaved (re, im); lda in complex elements; out: {re.hi, re.lo, im.hi, im.lo} */
int oracle_brute_c128(int m, int n, const double *a, int64_t lda, int nthreads, double *out) {
  return brute_common(2, m, n, a, lda, nthreads, out);
}

/* ================================================================== */
/* 2. memoised Laplace expansion                                       */
/* ================================================================== */
/* Row form (used when the column count n <= 30): table f over column sets S.
 * Layer i (rows 0..i-1 placed, |S| = i):  f(S) = sum_{j in S} a[i-1][j] f(S\{j}).
 * Layers only read the previous layer's entries, so one table indexed by the
 * bit mask of S holds all of them.  per(A) = sum_{|S| = m} f(S).
 *
 * Column form (used when the row count m <= 30 and it is cheaper): table g
 * over row sets R.  After column j:  g(R) += sum_{i in R} a[i][j] g_old(R\{i}),
 * i.e. rows R are matched into columns 0..j, and column j is either unused or
 * taken by one row i of R.  Entries with |R| = k are updated in order of
 * decreasing k so that g(R\{i}) still holds the value before column j.
 * per(A) = g([m]). */

typedef struct {
  const mat *A; int kind; int layer; int nbits;
  void *tab; int64_t chunk; int col;
} lap_ctx;

static void lap_row_task(void *c_, int64_t t) {
  lap_ctx *c = (lap_ctx *)c_;
  const mat *A = c->A;
  int i = c->layer;                      /* placing row i-1, sets of size i */
  uint64_t lo = (uint64_t)t * (uint64_t)c->chunk;
  uint64_t hi = lo + (uint64_t)c->chunk;
  uint64_t lim = 1ull << c->nbits;
  if (hi > lim) hi = lim;
  for (uint64_t S = lo; S < hi; ++S) {
    if (__builtin_popcountll(S) != i) continue;
    if (c->kind == 0) {
      u128 *f = (u128 *)c->tab, acc = 0;
      for (uint64_t R = S; R; R &= R - 1) {
        int j = __builtin_ctzll(R);
        acc += (u128)(__int128)geti(A, i - 1, j) * f[S & ~(1ull << j)];
      }
      f[S] = acc;
    } else if (c->kind == 1) {
      dd *f = (dd *)c->tab, acc = {0, 0};
      for (uint64_t R = S; R; R &= R - 1) {
        int j = __builtin_ctzll(R);
        acc = dd_add(acc, dd_mul_d(f[S & ~(1ull << j)], getr(A, i - 1, j)));
      }
      f[S] = acc;
    } else {
      cdd *f = (cdd *)c->tab, acc = cdd_zero();
      for (uint64_t R = S; R; R &= R - 1) {
        int j = __builtin_ctzll(R);
        cdd a = {dd_from(getc_re(A, i - 1, j)), dd_from(getc_im(A, i - 1, j))};
        acc = cdd_add(acc, cdd_mul(a, f[S & ~(1ull << j)]));
      }
      f[S] = acc;
    }
  }
}

static void lap_col_task(void *c_, int64_t t) {
  lap_ctx *c = (lap_ctx *)c_;
  const mat *A = c->A;
  int k = c->layer, j = c->col;          /* update sets of size k with column j */
  uint64_t lo = (uint64_t)t * (uint64_t)c->chunk;
  uint64_t hi = lo + (uint64_t)c->chunk;
  uint64_t lim = 1ull << c->nbits;
  if (hi > lim) hi = lim;
  for (uint64_t R = lo; R < hi; ++R) {
    if (__builtin_popcountll(R) != k) continue;
    if (c->kind == 0) {
      u128 *g = (u128 *)c->tab, acc = g[R];
      for (uint64_t Q = R; Q; Q &= Q - 1) {
        int i = __builtin_ctzll(Q);
        acc += (u128)(__int128)geti(A, i, j) * g[R & ~(1ull << i)];
      }
      g[R] = acc;
    } else if (c->kind == 1) {
      dd *g = (dd *)c->tab, acc = g[R];
      for (uint64_t Q = R; Q; Q &= Q - 1) {
        int i = __builtin_ctzll(Q);
        acc = dd_add(acc, dd_mul_d(g[R & ~(1ull << i)], getr(A, i, j)));
      }
      g[R] = acc;
    } else {
      cdd *g = (cdd *)c->tab, acc = g[R];
      for (uint64_t Q = R; Q; Q &= Q - 1) {
        int i = __builtin_ctzll(Q);
        cdd a = {dd_from(getc_re(A, i, j)), dd_from(getc_im(A, i, j))};
        acc = cdd_add(acc, cdd_mul(a, g[R & ~(1ull << i)]));
      }
      g[R] = acc;
    }
  }
}

static int laplace_common(int kind, int m, int n, const void *a, int64_t lda, int nthreads,
                          int form, void *out) {
  mat A;
  if (orient(m, n, a, lda, &A)) return -1;
  size_t esz = kind == 0 ? sizeof(u128) : kind == 1 ? sizeof(dd) : sizeof(cdd);
  if (A.m == 0) return brute_common(kind, m, n, a, lda, nthreads, out);
  /* form: 0 = choose, 1 = row form over column sets, 2 = column form over row sets */
  if (form == 0) form = (A.m + 0 <= A.n && A.m < A.n - 2) ? 2 : 1;
  int nbits = form == 1 ? A.n : A.m;
  if (nbits > 30) return -2;
  uint64_t size = 1ull << nbits;
  void *tab = calloc((size_t)size, esz);
  if (!tab) return -3;
  lap_ctx c; memset(&c, 0, sizeof c);
  c.A = &A; c.kind = kind; c.nbits = nbits; c.tab = tab;
  c.chunk = size >= (1u << 16) ? (int64_t)(size >> 10) : (int64_t)size;
  int64_t ntasks = (int64_t)((size + (uint64_t)c.chunk - 1) / (uint64_t)c.chunk);
  /* empty set / empty matching has value 1 */
  if (kind == 0) ((u128 *)tab)[0] = 1;
  else if (kind == 1) ((dd *)tab)[0] = dd_from(1.0);
  else { cdd one = {dd_from(1.0), dd_from(0.0)}; ((cdd *)tab)[0] = one; }

  if (form == 1) {
    for (int i = 1; i <= A.m; ++i) { c.layer = i; run_tasks(lap_row_task, &c, ntasks, nthreads); }
    /* sum over |S| = m in increasing mask order */
    u128 is = 0; dd rs = {0, 0}; cdd cs = cdd_zero();
    for (uint64_t S = 0; S < size; ++S) {
      if (__builtin_popcountll(S) != A.m) continue;
      if (kind == 0) is += ((u128 *)tab)[S];
      else if (kind == 1) rs = dd_add(rs, ((dd *)tab)[S]);
      else cs = cdd_add(cs, ((cdd *)tab)[S]);
    }
    if (kind == 0) { ((uint64_t *)out)[0] = (uint64_t)is; ((uint64_t *)out)[1] = (uint64_t)(is >> 64); }
    else if (kind == 1) { ((double *)out)[0] = rs.hi; ((double *)out)[1] = rs.lo; }
    else { double *o = (double *)out; o[0] = cs.re.hi; o[1] = cs.re.lo; o[2] = cs.im.hi; o[3] = cs.im.lo; }
  } else {
    for (int j = 0; j < A.n; ++j) {
      c.col = j;
      for (int k = A.m; k >= 1; --k) { c.layer = k; run_tasks(lap_col_task, &c, ntasks, nthreads); }
    }
    uint64_t full = size - 1;
    if (kind == 0) { u128 v = ((u128 *)tab)[full]; ((uint64_t *)out)[0] = (uint64_t)v; ((uint64_t *)out)[1] = (uint64_t)(v >> 64); }
    else if (kind == 1) { dd v = ((dd *)tab)[full]; ((double *)out)[0] = v.hi; ((double *)out)[1] = v.lo; }
    else { cdd v = ((cdd *)tab)[full]; double *o = (double *)out; o[0] = v.re.hi; o[1] = v.re.lo; o[2] = v.im.hi; o[3] = v.im.lo; }
  }
  free(tab);
  return 0;
}

int oracle_laplace_i64(int m, int n, const int64_t *a, int64_t lda, int nthreads, int form, uint64_t *out) {
  return laplace_common(0, m, n, a, lda, nthreads, form, out);
}
int oracle_laplace_f64(int m, int n, const double *a, int64_t lda, int nthreads, int form, double *out) {
  return laplace_common(1, m, n, a, lda, nthreads, form, out);
}
int oracle_laplace_c128(int m, int n, const double *a, int64_t lda, int nthreads, int form, double *out) {
  return laplace_common(2, m, n, a, lda, nthreads, form, out);
}

/* ================================================================== */
/* 3. Glynn's formula in double-double, Gray-code order                */
/* ================================================================== */
/* Square (Eq. glynn):
 *   per(A) = 2^-(n-1) sum_{delta in {+-1}^n, delta_1 = +1} (prod_k delta_k)
 *                                     prod_j sum_i delta_i a_ij
 * (the sum over all 2^n sign vectors counts each term twice, since flipping
 * every sign leaves the summand unchanged; fixing delta_1 and dividing by
 * 2^(n-1) counts it once).  Rectangular m < n (Eq. glynn_filled_matrix,
 * Eq. glynn_rectangle): rows m..n-1 of the padded matrix are all ones and the
 * sum is further divided by (n-m)!.
 *
 * Sign vectors are indexed by k in [0, 2^(n-1)); the reflected Gray code
 * g = k xor (k >> 1) gives delta_{r} = -1 exactly when bit (r-1) of g is set
 * (rows r = 1..n-1; row 0 keeps +1).  Consecutive k differ in one sign and
 * (prod delta) = (-1)^popcount(g) = (-1)^k.  A task covers a contiguous range
 * of k: it computes its first vector's column sums directly, then applies one
 * signed row per step. */

typedef struct {
  const mat *A; int kind; int n; int m;
  uint64_t k0, k1, per_task;
  dd *rres; cdd *cres;
} glynn_ctx;

static void glynn_task(void *c_, int64_t t) {
  glynn_ctx *c = (glynn_ctx *)c_;
  const mat *A = c->A;
  int n = c->n, m = c->m;
  uint64_t lo = c->k0 + (uint64_t)t * c->per_task;
  uint64_t hi = lo + c->per_task;
  if (hi > c->k1) hi = c->k1;
  if (lo >= hi) return;
  /* delta for index lo */
  int delta[64];
  uint64_t g = lo ^ (lo >> 1);
  delta[0] = 1;
  for (int r = 1; r < n; ++r) delta[r] = (g >> (r - 1) & 1) ? -1 : 1;
  if (c->kind == 1) {
    dd s[64];
    for (int j = 0; j < n; ++j) {
      dd acc = {0, 0};
      for (int r = 0; r < n; ++r) {
        double a = r < m ? getr(A, r, j) : 1.0;
        acc = dd_add(acc, dd_from(delta[r] > 0 ? a : -a));
      }
      s[j] = acc;
    }
    dd sum = {0, 0};
    for (uint64_t k = lo;; ) {
      dd p = s[0];
      for (int j = 1; j < n; ++j) p = dd_mul(p, s[j]);
      sum = (k & 1) ? dd_sub(sum, p) : dd_add(sum, p);
      if (++k >= hi) break;
      int r = __builtin_ctzll(k) + 1;          /* the row whose sign changes */
      delta[r] = -delta[r];
      for (int j = 0; j < n; ++j) {
        double a = r < m ? getr(A, r, j) : 1.0;
        double d = 2.0 * a;                   /* exact */
        s[j] = dd_add(s[j], dd_from(delta[r] > 0 ? d : -d));
      }
    }
    c->rres[t] = sum;
  } else {
    cdd s[64];
    for (int j = 0; j < n; ++j) {
      cdd acc = cdd_zero();
      for (int r = 0; r < n; ++r) {
        double ar = r < m ? getc_re(A, r, j) : 1.0;
        double ai = r < m ? getc_im(A, r, j) : 0.0;
        if (delta[r] < 0) { ar = -ar; ai = -ai; }
        acc.re = dd_add(acc.re, dd_from(ar));
        acc.im = dd_add(acc.im, dd_from(ai));
      }
      s[j] = acc;
    }
    cdd sum = cdd_zero();
    for (uint64_t k = lo;; ) {
      cdd p = s[0];
      for (int j = 1; j < n; ++j) p = cdd_mul(p, s[j]);
      sum = (k & 1) ? cdd_add(sum, cdd_neg(p)) : cdd_add(sum, p);
      if (++k >= hi) break;
      int r = __builtin_ctzll(k) + 1;
      delta[r] = -delta[r];
      for (int j = 0; j < n; ++j) {
        double ar = r < m ? getc_re(A, r, j) : 1.0;
        double ai = r < m ? getc_im(A, r, j) : 0.0;
        double dr = 2.0 * ar, di = 2.0 * ai;
        if (delta[r] < 0) { dr = -dr; di = -di; }
        s[j].re = dd_add(s[j].re, dd_from(dr));
        s[j].im = dd_add(s[j].im, dd_from(di));
      }
    }
    c->cres[t] = sum;
  }
}

/* Sums the terms with index k in [k0, k1) (k1 = 0 means all 2^(n-1)) and,
 * when the whole range is summed, applies the normalisation.  `partial`
 * non-zero returns the raw signed partial sum without normalisation. */
static int glynn_common(int kind, int m, int n, const double *a, int64_t lda, int nthreads,
                        uint64_t k0, uint64_t k1, int partial, double *out) {
  mat A;
  if (orient(m, n, a, lda, &A)) return -1;
  if (A.m == 0) {
    if (kind == 1) { out[0] = 1; out[1] = 0; } else { out[0] = 1; out[1] = out[2] = out[3] = 0; }
    return 0;
  }
  if (A.n > 63) return -2;
  uint64_t total = 1ull << (A.n - 1);
  if (k1 == 0 || k1 > total) k1 = total;
  if (k0 > k1) return -1;
  glynn_ctx c; memset(&c, 0, sizeof c);
  c.A = &A; c.kind = kind; c.n = A.n; c.m = A.m; c.k0 = k0; c.k1 = k1;
  int th = resolve_threads(nthreads);
  uint64_t range = k1 - k0;
  int64_t ntasks = range == 0 ? 0 : (int64_t)(th * 16);
  if ((uint64_t)ntasks > range) ntasks = (int64_t)range;
  if (ntasks == 0) ntasks = 1;
  c.per_task = (range + (uint64_t)ntasks - 1) / (uint64_t)ntasks;
  if (kind == 1) c.rres = (dd *)calloc((size_t)ntasks, sizeof(dd));
  else c.cres = (cdd *)calloc((size_t)ntasks, sizeof(cdd));
  if (!c.rres && !c.cres) return -3;
  run_tasks(glynn_task, &c, ntasks, th);
  /* normalisation: 2^-(n-1) exactly, then / (n-m)! in double-double */
  double scale = ldexp(1.0, -(A.n - 1));
  dd fact = dd_from(1.0);
  for (int q = 2; q <= A.n - A.m; ++q) fact = dd_mul_d(fact, (double)q);
  if (kind == 1) {
    dd s = {0, 0};
    for (int64_t t = 0; t < ntasks; ++t) s = dd_add(s, c.rres[t]);
    if (!partial) {
      s = dd_mul_d(s, scale);
      /* s / fact, one Newton step on the double quotient */
      double q1 = s.hi / fact.hi;
      dd r = dd_sub(s, dd_mul_d(fact, q1));
      double q2 = r.hi / fact.hi;
      s = fast_two_sum(q1, q2);
    }
    out[0] = s.hi; out[1] = s.lo;
    free(c.rres);
  } else {
    cdd s = cdd_zero();
    for (int64_t t = 0; t < ntasks; ++t) s = cdd_add(s, c.cres[t]);
    if (!partial) {
      s = cdd_scale(s, scale);
      dd *parts[2] = {&s.re, &s.im};
      for (int p = 0; p < 2; ++p) {
        dd v = *parts[p];
        double q1 = v.hi / fact.hi;
        dd r = dd_sub(v, dd_mul_d(fact, q1));
        double q2 = r.hi / fact.hi;
        *parts[p] = fast_two_sum(q1, q2);
      }
    }
    out[0] = s.re.hi; out[1] = s.re.lo; out[2] = s.im.hi; out[3] = s.im.lo;
    free(c.cres);
  }
  return 0;
}

int oracle_glynn_f64(int m, int n, const double *a, int64_t lda, int nthreads,
                     uint64_t k0, uint64_t k1, int partial, double *out) {
  return glynn_common(1, m, n, a, lda, nthreads, k0, k1, partial, out);
}
int oracle_glynn_c128(int m, int n, const double *a, int64_t lda, int nthreads,
                      uint64_t k0, uint64_t k1, int partial, double *out) {
  return glynn_common(2, m, n, a, lda, nthreads, k0, k1, partial, out);
}

/* ================================================================== */
/* 4. Ryser's formula in double-double, Gray-code order                */
/* ================================================================== */
/* With f(S) = prod_i sum_{j in S} a_ij over column sets S:
 *   square  (Eq. ryser_square):    per = (-1)^n sum_{S} (-1)^|S| f(S)
 *   m < n   (Eq. ryser_rectangle, read over column subsets of size m-k):
 *           per = sum_{k=0}^{m-1} (-1)^k C(n-m+k, k) sum_{|S| = m-k} f(S)
 * Both are one weighted sum over all column sets, weight w(|S|), with
 * w(s) = (-1)^(n-s) for m = n and w(s) = (-1)^(m-s) C(n-s, m-s) for s <= m,
 * 0 for s > m, when m < n.  Sets are visited in reflected Gray-code order
 * (column j is in S exactly when bit j of g(k) is set).  Exact integer
 * binomials are formed in double (exact below 2^53). */

typedef struct {
  const mat *A; int kind; int n; int m;
  uint64_t per_task, total;
  double w[65];
  dd *rres; cdd *cres;
} ryser_ctx;

static void ryser_task(void *c_, int64_t t) {
  ryser_ctx *c = (ryser_ctx *)c_;
  const mat *A = c->A;
  int n = c->n, m = c->m;
  uint64_t lo = (uint64_t)t * c->per_task;
  uint64_t hi = lo + c->per_task;
  if (hi > c->total) hi = c->total;
  if (lo >= hi) return;
  uint64_t g = lo ^ (lo >> 1);
  int size = __builtin_popcountll(g);
  if (c->kind == 1) {
    dd r[64];
    for (int i = 0; i < m; ++i) {
      dd acc = {0, 0};
      for (int j = 0; j < n; ++j) if (g >> j & 1) acc = dd_add(acc, dd_from(getr(A, i, j)));
      r[i] = acc;
    }
    dd sum = {0, 0};
    for (uint64_t k = lo;; ) {
      if (c->w[size] != 0.0) {
        dd p = r[0];
        for (int i = 1; i < m; ++i) p = dd_mul(p, r[i]);
        sum = dd_add(sum, dd_mul_d(p, c->w[size]));
      }
      if (++k >= hi) break;
      int j = __builtin_ctzll(k);
      g ^= 1ull << j;
      int in = (int)(g >> j & 1);
      size += in ? 1 : -1;
      for (int i = 0; i < m; ++i) {
        double v = getr(A, i, j);
        r[i] = dd_add(r[i], dd_from(in ? v : -v));
      }
    }
    c->rres[t] = sum;
  } else {
    cdd r[64];
    for (int i = 0; i < m; ++i) {
      cdd acc = cdd_zero();
      for (int j = 0; j < n; ++j)
        if (g >> j & 1) {
          acc.re = dd_add(acc.re, dd_from(getc_re(A, i, j)));
          acc.im = dd_add(acc.im, dd_from(getc_im(A, i, j)));
        }
      r[i] = acc;
    }
    cdd sum = cdd_zero();
    for (uint64_t k = lo;; ) {
      if (c->w[size] != 0.0) {
        cdd p = r[0];
        for (int i = 1; i < m; ++i) p = cdd_mul(p, r[i]);
        sum = cdd_add(sum, cdd_scale(p, c->w[size]));
      }
      if (++k >= hi) break;
      int j = __builtin_ctzll(k);
      g ^= 1ull << j;
      int in = (int)(g >> j & 1);
      size += in ? 1 : -1;
      for (int i = 0; i < m; ++i) {
        double vr = getc_re(A, i, j), vi = getc_im(A, i, j);
        r[i].re = dd_add(r[i].re, dd_from(in ? vr : -vr));
        r[i].im = dd_add(r[i].im, dd_from(in ? vi : -vi));
      }
    }
    c->cres[t] = sum;
  }
}

static int ryser_common(int kind, int m, int n, const double *a, int64_t lda, int nthreads,
                        double *out) {
  mat A;
  if (orient(m, n, a, lda, &A)) return -1;
  if (A.m == 0) {
    if (kind == 1) { out[0] = 1; out[1] = 0; } else { out[0] = 1; out[1] = out[2] = out[3] = 0; }
    return 0;
  }
  if (A.n > 62) return -2;
  ryser_ctx c; memset(&c, 0, sizeof c);
  c.A = &A; c.kind = kind; c.n = A.n; c.m = A.m; c.total = 1ull << A.n;
  for (int s = 0; s <= A.n; ++s) {
    if (s > A.m) { c.w[s] = 0.0; continue; }
    /* C(n-s, m-s), exact in double for the sizes allowed here */
    double b = 1.0;
    for (int q = 1; q <= A.m - s; ++q) b = b * (double)(A.n - s - (A.m - s) + q) / (double)q;
    double sg = ((A.m - s) & 1) ? -1.0 : 1.0;
    c.w[s] = sg * b;
  }
  int th = resolve_threads(nthreads);
  int64_t ntasks = (int64_t)th * 16;
  if ((uint64_t)ntasks > c.total) ntasks = (int64_t)c.total;
  c.per_task = (c.total + (uint64_t)ntasks - 1) / (uint64_t)ntasks;
  if (kind == 1) c.rres = (dd *)calloc((size_t)ntasks, sizeof(dd));
  else c.cres = (cdd *)calloc((size_t)ntasks, sizeof(cdd));
  if (!c.rres && !c.cres) return -3;
  run_tasks(ryser_task, &c, ntasks, th);
  if (kind == 1) {
    dd s = {0, 0};
    for (int64_t t = 0; t < ntasks; ++t) s = dd_add(s, c.rres[t]);
    out[0] = s.hi; out[1] = s.lo;
    free(c.rres);
  } else {
    cdd s = cdd_zero();
    for (int64_t t = 0; t < ntasks; ++t) s = cdd_add(s, c.cres[t]);
    out[0] = s.re.hi; out[1] = s.re.lo; out[2] = s.im.hi; out[3] = s.im.lo;
    free(c.cres);
  }
  return 0;
}

int oracle_ryser_f64(int m, int n, const double *a, int64_t lda, int nthreads, double *out) {
  return ryser_common(1, m, n, a, lda, nthreads, out);
}
int oracle_ryser_c128(int m, int n, const double *a, int64_t lda, int nthreads, double *out) {
  return ryser_common(2, m, n, a, lda, nthreads, out);
}
