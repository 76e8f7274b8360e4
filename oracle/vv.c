/*
 * vv.c -- velocity cross-correlation of the blobs against their separation
 * (Results section: the correlation of the velocities of two chains,
 * normalised by the mean square velocity, as a function of |R_cc'|, which
 * grows longer-ranged with the pair strength alpha).
 *
 * TEST INFRASTRUCTURE ONLY, like the rest of this directory.
 *
 * Definition (plain FP64, pairs in (i, j) order, i < j):
 *   u_c      = v_c, or with the flow flag v_c - kappa (y_c - Ly/2) x
 *              (the velocity relative to the imposed Couette flow of
 *              Eq. 6c; it is the same for every Lees-Edwards image)
 *   pair     {i, j} with r^2 < r_max^2 under the Lees-Edwards minimum
 *              image (orc_separation, r^2 = (dx^2 + dy^2) + dz^2)
 *   bin      k = the largest integer with k^2 <= t, t = r^2 * c,
 *              c = (nbins * nbins) / (r_max * r_max), capped at nbins - 1
 *              (bin k holds k <= r / (r_max / nbins) < k + 1)
 *   sum[k]   = sum over pairs of bin k of u_i . u_j
 *   count[k] = number of pairs of bin k
 *   u2       = sum_c |u_c|^2
 * so the normalised correlation of bin k is (sum[k] / count[k]) / (u2 / n).
 * The per-bin sums are the exact sums of the FP64 products, evaluated with
 * compensated (Neumaier) summation: within about two units in the last place
 * of the result, however many pairs a bin holds.
 */
#include <math.h>
#include <omp.h>
#include <stdlib.h>

#include "oracle.h"

/* the bin of t >= 0: the largest k with k*k <= t, found from a start value
 * and corrected with exact integer squares                                 */
static int64_t orc_floor_sqrt(double t) {
  int64_t k = (int64_t)sqrt(t);
  while ((double)(k + 1) * (double)(k + 1) <= t) ++k;
  while (k > 0 && (double)k * (double)k > t) --k;
  return k;
}

/* s + x with the rounding error kept in *c (Neumaier's compensated sum) */
static void neumaier_add(double* s, double* c, double x) {
  const double t = *s + x;
  if (fabs(*s) >= fabs(x)) *c += (*s - t) + x;
  else *c += (x - t) + *s;
  *s = t;
}

int orc_velocity_correlation(const orc_params* p, double delta, const double* pos,
                             const double* vel, double r_max, int32_t nbins, int32_t flow,
                             int32_t use_cells, double* sum, int64_t* count, double* u2) {
  if (nbins < 1 || !(r_max > 0.0)) return -1;
  const int64_t n = p->n;
  double* u = (double*)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
  if (!u) return -2;
  double s2 = 0.0;
  for (int64_t c = 0; c < n; ++c) {
    double ux = vel[3 * c];
    if (flow) ux = ux - p->shear_rate * (pos[3 * c + 1] - 0.5 * p->box[1]);
    u[3 * c] = ux;
    u[3 * c + 1] = vel[3 * c + 1];
    u[3 * c + 2] = vel[3 * c + 2];
    s2 += (u[3 * c] * u[3 * c] + u[3 * c + 1] * u[3 * c + 1]) + u[3 * c + 2] * u[3 * c + 2];
  }
  *u2 = s2;
  double* comp = (double*)malloc(sizeof(double) * (size_t)nbins);
  if (!comp) {
    free(u);
    return -2;
  }
  for (int32_t k = 0; k < nbins; ++k) {
    sum[k] = 0.0;
    comp[k] = 0.0;
    count[k] = 0;
  }
  const double rmax2 = r_max * r_max;
  const double cscale = ((double)nbins * (double)nbins) / (r_max * r_max);
  double d[3];
  /* pairs in (i, j) order: every pair tested (brute force, no storage), or
   * the cell-list pair set at cut-off r_max (same set, same order)        */
  int64_t* pr = NULL;
  int64_t np = 0;
  if (use_cells) {
    orc_params q = *p;
    q.rc = r_max;
    np = orc_pairs_cells(&q, delta, pos, 0, NULL);
    pr = np < 0 ? NULL : (int64_t*)malloc(sizeof(int64_t) * 2 * (size_t)(np > 0 ? np : 1));
    if (!pr) {
      free(comp);
      free(u);
      return -2;
    }
    orc_pairs_cells(&q, delta, pos, np, pr);
  }
  if (use_cells) {
    for (int64_t m = 0; m < np; ++m) {
      const int64_t i = pr[2 * m], j = pr[2 * m + 1];
      orc_separation(p, delta, pos + 3 * i, pos + 3 * j, d);
      const double r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
      int64_t k = orc_floor_sqrt(r2 * cscale);
      if (k > nbins - 1) k = nbins - 1;
      neumaier_add(&sum[k], &comp[k],
                   (u[3 * i] * u[3 * j] + u[3 * i + 1] * u[3 * j + 1]) + u[3 * i + 2] * u[3 * j + 2]);
      count[k] += 1;
    }
  } else {
    /* every pair tested; rows i are dealt to the threads in fixed chunks,
     * each thread keeps its own compensated sums, added in thread order   */
    int nt = 1;
#pragma omp parallel
    {
#pragma omp single
      nt = omp_get_num_threads();
    }
    double* ts = (double*)calloc((size_t)nt * 2 * nbins, sizeof(double));
    int64_t* tc = (int64_t*)calloc((size_t)nt * nbins, sizeof(int64_t));
    if (!ts || !tc) {
      free(ts);
      free(tc);
      free(comp);
      free(u);
      return -2;
    }
#pragma omp parallel num_threads(nt)
    {
      const int th = omp_get_thread_num();
      double* s_t = ts + (size_t)th * 2 * nbins;
      double* c_t = s_t + nbins;
      int64_t* n_t = tc + (size_t)th * nbins;
      double dd[3];
#pragma omp for schedule(static, 16)
      for (int64_t i = 0; i < n; ++i)
        for (int64_t j = i + 1; j < n; ++j) {
          orc_separation(p, delta, pos + 3 * i, pos + 3 * j, dd);
          const double r2 = (dd[0] * dd[0] + dd[1] * dd[1]) + dd[2] * dd[2];
          if (!(r2 < rmax2)) continue;
          int64_t k = orc_floor_sqrt(r2 * cscale);
          if (k > nbins - 1) k = nbins - 1;
          neumaier_add(&s_t[k], &c_t[k],
                       (u[3 * i] * u[3 * j] + u[3 * i + 1] * u[3 * j + 1]) + u[3 * i + 2] * u[3 * j + 2]);
          n_t[k] += 1;
        }
    }
    for (int t = 0; t < nt; ++t)
      for (int32_t k = 0; k < nbins; ++k) {
        neumaier_add(&sum[k], &comp[k], ts[(size_t)t * 2 * nbins + k]);
        neumaier_add(&sum[k], &comp[k], ts[(size_t)t * 2 * nbins + nbins + k]);
        count[k] += tc[(size_t)t * nbins + k];
      }
    free(ts);
    free(tc);
  }
  for (int32_t k = 0; k < nbins; ++k) sum[k] += comp[k];
  free(pr);
  free(comp);
  free(u);
  return 0;
}
