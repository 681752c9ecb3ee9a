/*
 * O-num: the paper's column-by-column left-looking sparse Cholesky
 * (Section 2.1.1, Algorithm 1), in plain C and IEEE binary64.
 *
 * TEST INFRASTRUCTURE. Only tests/, __graft_entry__.smoke() and the
 * cpu_baseline leg of bench.py may load this library. It shares no code with
 * the device path.
 *
 * Build with contraction off (-ffp-contract=off) and without fast-math so
 * every multiply and subtract is rounded on its own.
 *
 * For every column j in ascending order:
 *   1. scatter the lower part of column j of A into the dense work vector t,
 *      through the column's structure glbind(j);
 *   2. for every column k < j whose structure holds row j (k ascending, or
 *      descending when `reverse` is set, to measure the rounding-order noise
 *      floor), subtract L_{i,k} * L_{j,k} from t_i for every i in glbind(k)
 *      with i >= j -- the containment of eq. (1) guarantees i is in glbind(j);
 *   3. gather t back through glbind(j);
 *   4. cdiv(j): stop with info = j+1 when the pivot is not positive, else
 *      take its square root and divide the rest of the column by it.
 *
 * Because column j depends only on columns k < j, factoring a prefix of
 * `ncols` columns gives exactly those columns of the full factor.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

/* Returns 0 on success, j+1 for the first non-positive pivot, -1 on a bad
 * argument or allocation failure.
 *   a_cp/a_ri/a_x : lower CSC (incl. diagonal) of the ordered matrix, n cols
 *   l_cp/l_ri     : exact structure of L, glbind(j) ascending, first = j
 *   l_x           : output values (length l_cp[ncols])
 */
int64_t oracle_alg1(int64_t n, const int64_t *a_cp, const int64_t *a_ri,
                    const double *a_x, const int64_t *l_cp, const int64_t *l_ri,
                    double *l_x, int64_t ncols, int32_t reverse) {
  if (n < 0 || ncols < 0 || ncols > n) return -1;
  if (ncols == 0) return 0;
  double *t = (double *)calloc((size_t)n, sizeof(double));
  int64_t *pos = (int64_t *)malloc(sizeof(int64_t) * (size_t)ncols);
  int64_t *rcount = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
  if (!t || !pos || !rcount) {
    free(t); free(pos); free(rcount);
    return -1;
  }
  /* row lists: for each row j, the columns k < j with j in glbind(k) */
  for (int64_t k = 0; k < ncols; ++k)
    for (int64_t q = l_cp[k] + 1; q < l_cp[k + 1]; ++q) rcount[l_ri[q] + 1]++;
  for (int64_t j = 0; j < n; ++j) rcount[j + 1] += rcount[j];
  int64_t *rcols = (int64_t *)malloc(sizeof(int64_t) * (size_t)(rcount[n] + 1));
  int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
  if (!rcols || !fill) {
    free(t); free(pos); free(rcount); free(rcols); free(fill);
    return -1;
  }
  for (int64_t j = 0; j <= n; ++j) fill[j] = rcount[j];
  for (int64_t k = 0; k < ncols; ++k) {
    pos[k] = l_cp[k] + 1; /* next entry of column k below its diagonal */
    for (int64_t q = l_cp[k] + 1; q < l_cp[k + 1]; ++q) rcols[fill[l_ri[q]]++] = k;
  }

  int64_t info = 0;
  for (int64_t j = 0; j < ncols; ++j) {
    /* 1. scatter A_{*,j} */
    for (int64_t q = l_cp[j]; q < l_cp[j + 1]; ++q) t[l_ri[q]] = 0.0;
    for (int64_t e = a_cp[j]; e < a_cp[j + 1]; ++e) t[a_ri[e]] = a_x[e];
    /* 2. updates from the left */
    int64_t cnt = rcount[j + 1] - rcount[j];
    for (int64_t r = 0; r < cnt; ++r) {
      int64_t k = reverse ? rcols[rcount[j + 1] - 1 - r] : rcols[rcount[j] + r];
      int64_t p = pos[k];
      double ljk = l_x[p];
      for (int64_t q = p; q < l_cp[k + 1]; ++q) {
        double prod = l_x[q] * ljk;
        t[l_ri[q]] = t[l_ri[q]] - prod;
      }
    }
    for (int64_t r = 0; r < cnt; ++r) pos[rcols[rcount[j] + r]]++;
    /* 3. gather */
    for (int64_t q = l_cp[j]; q < l_cp[j + 1]; ++q) l_x[q] = t[l_ri[q]];
    /* 4. cdiv(j) */
    double d = l_x[l_cp[j]];
    if (!(d > 0.0)) {
      info = j + 1;
      break;
    }
    d = sqrt(d);
    l_x[l_cp[j]] = d;
    for (int64_t q = l_cp[j] + 1; q < l_cp[j + 1]; ++q) l_x[q] = l_x[q] / d;
  }
  free(t); free(pos); free(rcount); free(rcols); free(fill);
  return info;
}
