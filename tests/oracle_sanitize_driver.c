/* Test infrastructure: runs every evaluator of the CPU oracle on small
 * shapes (square, rectangular, transposed, padded leading dimension, m = 0,
 * several threads) and checks that they agree, so that a build with
 * -fsanitize=address,undefined exercises all of its code paths.  Exit code 0
 * when every comparison holds; the sanitizers abort on any error. */
#include "../oracle/perm_oracle.c"

#include <stdio.h>
#include <stdlib.h>

static double u01(uint64_t *s) {
  *s = *s * 6364136223846793005ull + 1442695040888963407ull;
  return (double)(*s >> 11) * (1.0 / 9007199254740992.0);
}

static int close_enough(double a, double b, double scale) { return fabs(a - b) <= 1e-12 * scale; }

int main(void) {
  uint64_t seed = 12345;
  int bad = 0;
  const int shapes[][2] = {{0, 3}, {1, 1}, {1, 5}, {2, 2}, {3, 3}, {2, 6}, {4, 4}, {3, 7},
                           {5, 5}, {4, 8}, {6, 6}, {5, 9}, {6, 4}, {7, 3}};
  for (size_t s = 0; s < sizeof shapes / sizeof shapes[0]; ++s) {
    const int m = shapes[s][0], n = shapes[s][1];
    const int64_t lda = n + 2;  /* padded rows */
    const size_t cnt = (size_t)(m > 0 ? m : 1) * (size_t)lda;
    double *a = calloc(cnt, sizeof(double)), *z = calloc(2 * cnt, sizeof(double));
    int64_t *ai = calloc(cnt, sizeof(int64_t));
    double *absa = calloc(cnt, sizeof(double));
    for (int i = 0; i < m; ++i)
      for (int j = 0; j < n; ++j) {
        const size_t o = (size_t)i * lda + j;
        a[o] = 2.0 * u01(&seed) - 1.0;
        absa[o] = fabs(a[o]);
        z[2 * o] = 2.0 * u01(&seed) - 1.0;
        z[2 * o + 1] = 2.0 * u01(&seed) - 1.0;
        ai[o] = (int64_t)(u01(&seed) * 7.0) - 3;
      }
    for (int threads = 1; threads <= 4; threads += 3) {
      double b[2], l[2], g[2], r[2], sc[2];
      double bz[4], lz[4], gz[4], rz[4];
      uint64_t bi[2], li[2];
      int rc = oracle_brute_f64(m, n, a, lda, threads, b) | oracle_laplace_f64(m, n, a, lda, threads, 0, l) |
               oracle_glynn_f64(m, n, a, lda, threads, 0, 0, 0, g) | oracle_ryser_f64(m, n, a, lda, threads, r) |
               oracle_brute_f64(m, n, absa, lda, threads, sc) |
               oracle_brute_c128(m, n, z, lda, threads, bz) | oracle_laplace_c128(m, n, z, lda, threads, 0, lz) |
               oracle_glynn_c128(m, n, z, lda, threads, 0, 0, 0, gz) | oracle_ryser_c128(m, n, z, lda, threads, rz) |
               oracle_brute_i64(m, n, ai, lda, threads, bi) | oracle_laplace_i64(m, n, ai, lda, threads, 0, li);
      if (m > 0) {
        double l1[2], l2[2];
        rc |= oracle_laplace_f64(m, n, a, lda, threads, 1, l1) | oracle_laplace_f64(m, n, a, lda, threads, 2, l2);
        if (!close_enough(l1[0] + l1[1], b[0] + b[1], sc[0] + 1.0) ||
            !close_enough(l2[0] + l2[1], b[0] + b[1], sc[0] + 1.0))
          bad = 1;
      }
      if (rc) bad = 1;
      const double ref = b[0] + b[1], scale = sc[0] + 1.0;
      if (!close_enough(l[0] + l[1], ref, scale) || !close_enough(g[0] + g[1], ref, scale) ||
          !close_enough(r[0] + r[1], ref, scale))
        bad = 1;
      const double zs = 1e3 * (scale + 1.0);
      if (!close_enough(lz[0] + lz[1], bz[0] + bz[1], zs) || !close_enough(gz[0] + gz[1], bz[0] + bz[1], zs) ||
          !close_enough(rz[0] + rz[1], bz[0] + bz[1], zs) || !close_enough(lz[2] + lz[3], bz[2] + bz[3], zs))
        bad = 1;
      if (bi[0] != li[0] || bi[1] != li[1]) bad = 1;
      if (bad) {
        fprintf(stderr, "mismatch at %d x %d, %d threads\n", m, n, threads);
        return 1;
      }
    }
    free(a);
    free(z);
    free(ai);
    free(absa);
  }
  printf("oracle sanitize driver: all evaluators agree\n");
  return 0;
}
