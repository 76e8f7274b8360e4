/*
 * block.c -- the friction system with anisotropic pair friction (Discussion:
 * elongated particles as the way to move the small-q peak; this is the
 * friction side of it): the pair coefficient of Eq. 7 becomes a tensor
 *   W_ij = alpha w_ij (a_perp I + (a_par - a_perp) P_ij),  P_ij = d d^T / r^2,
 * so A (Eq. 9) has genuine 3 x 3 blocks.  a_par = a_perp = 1 gives exactly
 * the isotropic system A (x) I_3 of oracle.c.
 *
 * TEST INFRASTRUCTURE ONLY, like the rest of this directory.
 */
#include <math.h>
#include <stdlib.h>

#include "oracle.h"

/* the pairs of the configuration at `step`, (i, j) sorted; caller frees */
static int64_t block_pairs(const orc_params* p, int64_t step, const double* pos, int64_t** out) {
  const double delta = orc_le_offset(p, step);
  const int brute = p->n <= 2048;
  int64_t np = brute ? orc_pairs_brute(p, delta, pos, 0, NULL) : orc_pairs_cells(p, delta, pos, 0, NULL);
  if (np < 0) return -1;
  int64_t* pr = (int64_t*)malloc(sizeof(int64_t) * 2 * (size_t)(np > 0 ? np : 1));
  if (!pr) return -1;
  if (brute) orc_pairs_brute(p, delta, pos, np, pr);
  else orc_pairs_cells(p, delta, pos, np, pr);
  *out = pr;
  return np;
}

/* W of one pair (row-major 3 x 3) and P (the projector on the line of
 * centres); g = alpha w                                                    */
static void block_tensor(double g, double a_par, double a_perp, const double d[3], double r2,
                         double W[9], double P[9]) {
  const double c = a_par - a_perp;
  for (int k = 0; k < 3; ++k)
    for (int l = 0; l < 3; ++l) {
      P[3 * k + l] = r2 > 0.0 ? (d[k] * d[l]) / r2 : 0.0;
      W[3 * k + l] = k == l ? g * (a_perp + c * P[3 * k + l]) : g * (c * P[3 * k + l]);
    }
}

int64_t orc_build_block_system(const orc_params* p, double a_par, double a_perp, int64_t step,
                               const double* pos, int64_t cap, int64_t* rowptr, int64_t* col,
                               double* bval, double* bdiag, double* rhs) {
  const int64_t n = p->n;
  const double Ly = p->box[1];
  const double delta = orc_le_offset(p, step);
  int64_t* pairs = NULL;
  const int64_t np = block_pairs(p, step, pos, &pairs);
  if (np < 0) return -1;
  if (2 * np > cap) {
    free(pairs);
    return -1;
  }
  int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
  if (!fill) {
    free(pairs);
    return -1;
  }
  for (int64_t i = 0; i <= n; ++i) rowptr[i] = 0;
  for (int64_t k = 0; k < np; ++k) {
    rowptr[pairs[2 * k] + 1]++;
    rowptr[pairs[2 * k + 1] + 1]++;
  }
  for (int64_t i = 0; i < n; ++i) rowptr[i + 1] += rowptr[i];
  for (int64_t i = 0; i < n; ++i) fill[i] = rowptr[i];

  /* node terms: background friction, Couette drive, node noise (Eq. 6a, 6c) */
  double amp_node = 0.0, amp_pair = 0.0;
  if (p->noise_mode == ORC_NOISE_FDT) {
    const double c = sqrt(2.0 * p->kT / p->dt);
    amp_node = c * sqrt(p->gamma0);
    amp_pair = c;
  } else if (p->noise_mode == ORC_NOISE_PAPER) {
    amp_node = sqrt(2.0 * p->gamma0 * p->kT / p->dt);
  }
  for (int64_t i = 0; i < n; ++i) {
    for (int k = 0; k < 9; ++k) bdiag[9 * i + k] = 0.0;
    double g[4] = {0.0, 0.0, 0.0, 0.0};
    if (amp_node != 0.0) orc_gauss4(p, (uint64_t)step, 0, (uint64_t)i, 0, g);
    rhs[3 * i + 0] = p->gamma0 * p->shear_rate * (pos[3 * i + 1] - 0.5 * Ly) + amp_node * g[0];
    rhs[3 * i + 1] = amp_node * g[1];
    rhs[3 * i + 2] = amp_node * g[2];
  }
  const double sq_par = sqrt(a_par), sq_perp = sqrt(a_perp);
  double d[3], f[3], W[9], P[9];
  for (int64_t k = 0; k < np; ++k) {
    const int64_t i = pairs[2 * k], j = pairs[2 * k + 1];
    const int s = orc_separation(p, delta, pos + 3 * i, pos + 3 * j, d);
    const double r2 = (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2];
    const double w = orc_weight(p, r2);
    const double gw = p->alpha * w;
    block_tensor(gw, a_par, a_perp, d, r2, W, P);
    orc_pair_force(p, d, r2, f);
    col[fill[i]] = j;
    col[fill[j]] = i;
    for (int m = 0; m < 9; ++m) {
      bval[9 * fill[i] + m] = -W[m];
      bval[9 * fill[j] + m] = -W[m];
      bdiag[9 * i + m] += W[m];
      bdiag[9 * j + m] += W[m];
    }
    fill[i]++;
    fill[j]++;
    /* conservative force and boundary drag W_ij V_ij, V_ij = kappa Ly s_ij x */
    const double v = p->shear_rate * Ly * (double)s;
    for (int c = 0; c < 3; ++c) {
      const double t = f[c] + W[3 * c] * v;
      rhs[3 * i + c] += t;
      rhs[3 * j + c] -= t;
    }
    /* pair thermal force sqrt(2kT/dt) W^(1/2) eta, sigma = +1 on the smaller id */
    if (amp_pair != 0.0 && p->alpha != 0.0) {
      double g[4];
      orc_gauss4(p, (uint64_t)step, 1, (uint64_t)i, (uint64_t)j, g);
      const double a = amp_pair * sqrt(gw);
      const double t = (d[0] * g[0] + d[1] * g[1]) + d[2] * g[2];
      for (int c = 0; c < 3; ++c) {
        const double q = r2 > 0.0 ? (d[c] * t) / r2 : 0.0;
        const double e = a * (sq_perp * g[c] + (sq_par - sq_perp) * q);
        rhs[3 * i + c] += e;
        rhs[3 * j + c] -= e;
      }
    }
  }
  for (int64_t i = 0; i < n; ++i)
    for (int c = 0; c < 3; ++c) bdiag[9 * i + 4 * c] += p->gamma0;
  free(fill);
  free(pairs);
  return 2 * np;
}

/* y = A x on the stacked 3n vector */
static void block_spmv(int64_t n, const int64_t* rowptr, const int64_t* col, const double* bval,
                       const double* bdiag, const double* x, double* y) {
  for (int64_t i = 0; i < n; ++i)
    for (int k = 0; k < 3; ++k) {
      double acc = 0.0;
      for (int l = 0; l < 3; ++l) acc += bdiag[9 * i + 3 * k + l] * x[3 * i + l];
      for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e)
        for (int l = 0; l < 3; ++l) acc += bval[9 * e + 3 * k + l] * x[3 * col[e] + l];
      y[3 * i + k] = acc;
    }
}

static double dot(int64_t m, const double* a, const double* b) {
  double s = 0.0;
  for (int64_t i = 0; i < m; ++i) s += a[i] * b[i];
  return s;
}

int orc_block_pcg(int64_t n, const int64_t* rowptr, const int64_t* col, const double* bval,
                  const double* bdiag, const double* rhs, double* x, double tol, int maxit,
                  int* iters) {
  const int64_t m = 3 * n;
  double* r = (double*)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
  double* z = (double*)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
  double* pv = (double*)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
  double* q = (double*)malloc(sizeof(double) * (size_t)(m > 0 ? m : 1));
  if (!r || !z || !pv || !q) {
    free(r); free(z); free(pv); free(q);
    return -2;
  }
  const double bb = dot(m, rhs, rhs);
  int it = 0, status = -4;
  for (int64_t i = 0; i < m; ++i) x[i] = 0.0;
  if (bb == 0.0) status = 0;
  for (int restart = 0; status != 0 && restart < 20 && it < maxit; ++restart) {
    /* true residual, Jacobi on the scalar diagonal of A */
    block_spmv(n, rowptr, col, bval, bdiag, x, q);
    for (int64_t i = 0; i < m; ++i) r[i] = rhs[i] - q[i];
    if (dot(m, r, r) <= tol * tol * bb) {
      status = 0;
      break;
    }
    for (int64_t i = 0; i < m; ++i) {
      z[i] = r[i] / bdiag[9 * (i / 3) + 4 * (i % 3)];
      pv[i] = z[i];
    }
    double rz = dot(m, r, z);
    while (it < maxit) {
      block_spmv(n, rowptr, col, bval, bdiag, pv, q);
      const double a = rz / dot(m, pv, q);
      for (int64_t i = 0; i < m; ++i) {
        x[i] += a * pv[i];
        r[i] -= a * q[i];
      }
      ++it;
      if (dot(m, r, r) <= tol * tol * bb) break;
      for (int64_t i = 0; i < m; ++i) z[i] = r[i] / bdiag[9 * (i / 3) + 4 * (i % 3)];
      const double rz2 = dot(m, r, z);
      const double beta = rz2 / rz;
      rz = rz2;
      for (int64_t i = 0; i < m; ++i) pv[i] = z[i] + beta * pv[i];
    }
  }
  if (iters) *iters = it;
  free(r); free(z); free(pv); free(q);
  return status;
}

int orc_step_block(const orc_params* p, double a_par, double a_perp, int64_t step, double* pos,
                   double* vel, double tol, int maxit, int* iters) {
  const int64_t n = p->n;
  int64_t* pr = NULL;
  const int64_t np = block_pairs(p, step, pos, &pr);
  if (np < 0) return -2;
  free(pr);
  const int64_t cap = 2 * np > 0 ? 2 * np : 1;
  int64_t* rowptr = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
  int64_t* col = (int64_t*)malloc(sizeof(int64_t) * (size_t)cap);
  double* bval = (double*)malloc(sizeof(double) * 9 * (size_t)cap);
  double* bdiag = (double*)malloc(sizeof(double) * 9 * (size_t)(n > 0 ? n : 1));
  double* rhs = (double*)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
  int status = 0;
  if (!rowptr || !col || !bval || !bdiag || !rhs ||
      orc_build_block_system(p, a_par, a_perp, step, pos, cap, rowptr, col, bval, bdiag, rhs) < 0) {
    status = -2;
  } else {
    status = orc_block_pcg(n, rowptr, col, bval, bdiag, rhs, vel, tol, maxit, iters);
    if (status == 0) {
      for (int64_t i = 0; i < 3 * n; ++i) pos[i] += vel[i] * p->dt;
      orc_wrap(p, step + 1, pos);
    }
  }
  free(rowptr); free(col); free(bval); free(bdiag); free(rhs);
  return status;
}
