/*
 * oracle.c -- plain FP64 CPU oracle of one time step of the sheared mesoscale
 * blob simulation of Korolkovas, arXiv 1808.06381 (Method section).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark; never by the product path.  It shares no
 * code with the GPU library.  Slow on purpose, written so a reader can check
 * each function against the paper by eye.  The row loops of the products and
 * the element-wise vector updates of the solve run on OpenMP threads (all
 * cores unless orc_set_threads or OMP_NUM_THREADS say otherwise; the CPU
 * timing baseline measures 1 and all): each output is written by one thread
 * in the sequential order of operations and every sum stays sequential, so
 * no result bit depends on the thread count:
 *
 *   orc_separation    Lees-Edwards minimum image (Method: "standard
 *                     Lees-Edwards boundary conditions"; image index of Eq. 8)
 *   orc_pairs_*       the truncated pair set (Method: weights below the
 *                     threshold are dropped before the sparse solve)
 *   orc_build_system  Eq. 9: matrix gamma0*I + alpha*L(w), right-hand side
 *                     F_c + gamma0*kappa*(y_c - Ly/2) x + alpha*sum V_cc' w_cc'
 *                     (Eq. 6a-6c, Eq. 8), plus the thermal force of Eq. 6a
 *   orc_pcg           the sparse solve of Eq. 9 (conjugate gradients)
 *   orc_step          one overdamped first-order step of Eq. 7, R += v dt
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math (no FMA contraction, so the
 * pair decision r^2 < rc^2 is the IEEE result of the written operations).
 */
#include "oracle.h"

#include <math.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_ENOMEM -2
#define ORC_ENOCONV -4
#define ORC_EBREAKDOWN -5

/* ===================================================================== */
/* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC'11): ten rounds of two 64x64->128 multiplies with the
 * published multipliers and Weyl key increments.                          */
/* ===================================================================== */
void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
  const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
  uint64_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint64_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    unsigned __int128 p0 = (unsigned __int128)M0 * c0;
    unsigned __int128 p1 = (unsigned __int128)M1 * c2;
    uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
    uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
    uint64_t n0 = hi1 ^ c1 ^ k0;
    uint64_t n2 = hi0 ^ c3 ^ k1;
    c0 = n0; c1 = lo1; c2 = n2; c3 = lo0;
    k0 += W0; k1 += W1;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* 53-bit uniform on the open interval (0, 1): ((bits >> 11) + 1/2) * 2^-53 */
static double orc_uniform(uint64_t bits) {
  return ((double)(bits >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

/* Box & Muller (1958): two uniforms -> two independent standard normals.
 * The thermal force of Eq. 6a is a Wiener increment; per component its
 * discrete form is a standard normal scaled by the amplitude.             */
void orc_gauss4(const orc_params* p, uint64_t step, uint64_t tag, uint64_t a,
                uint64_t b, double g[4]) {
  const double two_pi = 6.283185307179586;
  uint64_t ctr[4] = {step, tag, a, b};
  uint64_t key[2] = {p->seed, p->stream};
  uint64_t bits[4];
  orc_philox4x64_10(ctr, key, bits);
  double u0 = orc_uniform(bits[0]), u1 = orc_uniform(bits[1]);
  double u2 = orc_uniform(bits[2]), u3 = orc_uniform(bits[3]);
  double rad0 = sqrt(-2.0 * log(u0));
  double rad1 = sqrt(-2.0 * log(u2));
  g[0] = rad0 * cos(two_pi * u1);
  g[1] = rad0 * sin(two_pi * u1);
  g[2] = rad1 * cos(two_pi * u3);
  g[3] = rad1 * sin(two_pi * u3);
}

/* ===================================================================== */
/* Geometry                                                               */
/* ===================================================================== */

/* Lees-Edwards offset at step n: the periodic image above the box is moved
 * along x by kappa*Ly*t (mod Lx), t = n*dt.                               */
double orc_le_offset(const orc_params* p, int64_t step) {
  double t = (double)step * p->dt;
  return fmod((p->shear_rate * p->box[1]) * t, p->box[0]);
}

/* Minimum-image separation d = R_i - R_j(image) under Lees-Edwards
 * boundaries with offset delta.  Returns the image index s = round(y_ij/Ly)
 * of Eq. 8 (+1: the nearest image of j lies one box above, and is displaced
 * by +delta in x).  Only add, subtract, multiply by +-1 and compares are
 * used, so d_ji == -d_ij bit for bit.                                      */
int orc_separation(const orc_params* p, double delta, const double* ri,
                   const double* rj, double d[3]) {
  const double Lx = p->box[0], Ly = p->box[1], Lz = p->box[2];
  double dy = ri[1] - rj[1];
  int s = 0;
  if (dy > 0.5 * Ly) s = 1;
  else if (dy < -0.5 * Ly) s = -1;
  dy = dy - (double)s * Ly;
  double dx = (ri[0] - rj[0]) - (double)s * delta;
  /* |dx| < 2.5 Lx here; at most two periods to remove on either side */
  for (int k = 0; k < 2; ++k)
    if (dx > 0.5 * Lx) dx = dx - Lx;
  for (int k = 0; k < 2; ++k)
    if (dx < -0.5 * Lx) dx = dx + Lx;
  double dz = ri[2] - rj[2];
  if (dz > 0.5 * Lz) dz = dz - Lz;
  if (dz < -0.5 * Lz) dz = dz + Lz;
  d[0] = dx;
  d[1] = dy;
  d[2] = dz;
  return s;
}

static double orc_r2(const double d[3]) { return (d[0] * d[0] + d[1] * d[1]) + d[2] * d[2]; }

/* All unordered pairs {i<j} with r^2 < rc^2, by testing every pair.
 * Writes min(count, cap) pairs as (i, j) into pairs[2k], pairs[2k+1];
 * returns the full count.                                                 */
int64_t orc_pairs_brute(const orc_params* p, double delta, const double* pos,
                        int64_t cap, int64_t* pairs) {
  const double rc2 = p->rc * p->rc;
  int64_t count = 0;
  double d[3];
  for (int64_t i = 0; i < p->n; ++i)
    for (int64_t j = i + 1; j < p->n; ++j) {
      orc_separation(p, delta, pos + 3 * i, pos + 3 * j, d);
      if (orc_r2(d) < rc2) {
        if (count < cap) {
          pairs[2 * count] = i;
          pairs[2 * count + 1] = j;
        }
        ++count;
      }
    }
  return count;
}

static int orc_cmp_i64(const void* a, const void* b) {
  int64_t x = *(const int64_t*)a, y = *(const int64_t*)b;
  return (x > y) - (x < y);
}

/* Same pair set as orc_pairs_brute, found with a cell list.  Cells are at
 * least rc wide; for a row of cells across the y boundary every x cell of
 * the wrapped row is a candidate (any Lees-Edwards offset is covered), and
 * a dimension with fewer than three cells is one cell.  Every candidate is
 * tested once with orc_separation, so the result is the brute-force set.  */
int64_t orc_pairs_cells(const orc_params* p, double delta, const double* pos,
                        int64_t cap, int64_t* pairs) {
  const int64_t n = p->n;
  const double rc2 = p->rc * p->rc;
  int64_t nc[3];
  double len[3];
  for (int k = 0; k < 3; ++k) {
    nc[k] = (int64_t)floor(p->box[k] / (p->rc * (1.0 + 1e-12)));
    if (nc[k] < 3) nc[k] = 1;
    len[k] = p->box[k] / (double)nc[k];
  }
  const int64_t ncell = nc[0] * nc[1] * nc[2];
  int64_t* head = (int64_t*)malloc(sizeof(int64_t) * (size_t)ncell);
  int64_t* next = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  int64_t* cell = (int64_t*)malloc(sizeof(int64_t) * 3 * (size_t)(n > 0 ? n : 1));
  int64_t* stamp = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  int64_t* row = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n > 0 ? n : 1));
  if (!head || !next || !cell || !stamp || !row) {
    free(head); free(next); free(cell); free(stamp); free(row);
    return -1;
  }
  for (int64_t c = 0; c < ncell; ++c) head[c] = -1;
  for (int64_t i = n - 1; i >= 0; --i) {
    int64_t flat = 0;
    for (int k = 2; k >= 0; --k) {
      int64_t ci = (int64_t)floor(pos[3 * i + k] / len[k]);
      if (ci < 0) ci = 0;
      if (ci > nc[k] - 1) ci = nc[k] - 1;
      cell[3 * i + k] = ci;
      flat = flat * nc[k] + ci;
    }
    next[i] = head[flat];
    head[flat] = i;
    stamp[i] = -1;
  }
  int64_t count = 0;
  double d[3];
  for (int64_t i = 0; i < n; ++i) {
    int64_t nrow = 0;
    const int64_t cx = cell[3 * i], cy = cell[3 * i + 1], cz = cell[3 * i + 2];
    const int zlo = nc[2] == 1 ? 0 : -1, zhi = nc[2] == 1 ? 0 : 1;
    const int ylo = nc[1] == 1 ? 0 : -1, yhi = nc[1] == 1 ? 0 : 1;
    for (int dz = zlo; dz <= zhi; ++dz)
      for (int dy = ylo; dy <= yhi; ++dy) {
        int64_t z2 = ((cz + dz) % nc[2] + nc[2]) % nc[2];
        int64_t y2raw = cy + dy;
        int wrapped = nc[1] == 1 || y2raw < 0 || y2raw >= nc[1];
        int64_t y2 = (y2raw % nc[1] + nc[1]) % nc[1];
        int64_t xlo, xhi;
        if (wrapped || nc[0] == 1) { xlo = 0; xhi = nc[0] - 1; }
        else { xlo = cx - 1; xhi = cx + 1; }
        for (int64_t xr = xlo; xr <= xhi; ++xr) {
          int64_t x2 = (xr % nc[0] + nc[0]) % nc[0];
          for (int64_t j = head[(z2 * nc[1] + y2) * nc[0] + x2]; j >= 0; j = next[j]) {
            if (j <= i || stamp[j] == i) continue;
            stamp[j] = i;
            orc_separation(p, delta, pos + 3 * i, pos + 3 * j, d);
            if (orc_r2(d) < rc2) row[nrow++] = j;
          }
        }
      }
    qsort(row, (size_t)nrow, sizeof(int64_t), orc_cmp_i64);
    for (int64_t k = 0; k < nrow; ++k) {
      if (count < cap) {
        pairs[2 * count] = i;
        pairs[2 * count + 1] = row[k];
      }
      ++count;
    }
  }
  free(head); free(next); free(cell); free(stamp); free(row);
  return count;
}

/* pair list of the configuration at step `step`; caller frees *out */
static int64_t orc_pairs_alloc(const orc_params* p, int64_t step, const double* pos,
                               int64_t** out) {
  double delta = orc_le_offset(p, step);
  int use_brute = p->n <= 2048;
  int64_t np = use_brute ? orc_pairs_brute(p, delta, pos, 0, NULL)
                         : orc_pairs_cells(p, delta, pos, 0, NULL);
  if (np < 0) return -1;
  int64_t* pairs = (int64_t*)malloc(sizeof(int64_t) * 2 * (size_t)(np > 0 ? np : 1));
  if (!pairs) return -1;
  if (use_brute) orc_pairs_brute(p, delta, pos, np, pairs);
  else orc_pairs_cells(p, delta, pos, np, pairs);
  *out = pairs;
  return np;
}

int64_t orc_count_pairs(const orc_params* p, int64_t step, const double* pos) {
  int64_t* pairs = NULL;
  int64_t np = orc_pairs_alloc(p, step, pos, &pairs);
  free(pairs);
  return np;
}

/* ===================================================================== */
/* Pair terms and the linear system (Eq. 6-9)                            */
/* ===================================================================== */

/* entanglement weight w(r): Gaussian of width lambda (Method, after Eq. 7)
 * or the polynomial envelope (1 - r/rc)^2 (another "reasonable shape")   */
double orc_weight(const orc_params* p, double r2) {
  if (p->weight_law == ORC_W_GAUSS) return exp(-0.5 * r2 / (p->lambda * p->lambda));
  double t = 1.0 - sqrt(r2) / p->rc;
  return t * t;
}

/* conservative pair force on i from j, F = -dU/dr * d/r.
 * Gaussian core, Eq. 6b: U = kT*u_amp*exp(-r^2/(2 lambda^2)), u_amp = v/lambda^3,
 *   so F = (kT*u_amp/lambda^2) * exp(-r^2/(2 lambda^2)) * d.
 * Soft: U = u_amp*(1 - r/rc)^2, so F = (2*u_amp/rc)*(1 - r/rc) * d/r (0 at r = 0). */
void orc_pair_force(const orc_params* p, const double d[3], double r2, double f[3]) {
  double coef = 0.0;
  if (p->potential == ORC_U_GAUSS_CORE) {
    double l2 = p->lambda * p->lambda;
    coef = (p->kT * p->u_amp / l2) * exp(-0.5 * r2 / l2);
  } else if (p->potential == ORC_U_SOFT) {
    double r = sqrt(r2);
    coef = r > 0.0 ? (2.0 * p->u_amp / p->rc) * (1.0 - r / p->rc) / r : 0.0;
  }
  f[0] = coef * d[0];
  f[1] = coef * d[1];
  f[2] = coef * d[2];
}

/* Build the friction system of step `step` at positions pos.
 *   matrix (Eq. 9): A_ii = gamma0 + alpha*sum_j w_ij, A_ij = -alpha*w_ij;
 *   rhs b_i = sum_j F_ij                               (Eq. 6b)
 *           + gamma0*kappa*(y_i - Ly/2) x              (Eq. 6c)
 *           + alpha*sum_j w_ij * kappa*Ly*s_ij x        (Eq. 8 in Eq. 9)
 *           + f_i (thermal force).
 * Thermal force: PAPER mode is Eq. 6a, sqrt(2*gamma0*kT/dt)*xi_i per
 * component.  FDT mode adds one Gaussian vector per pair, with the
 * weighted-incidence amplitude: f_i = sqrt(2kT/dt)*(sqrt(gamma0)*xi_i +
 * sum_j sigma_ij*sqrt(alpha*w_ij)*eta_ij), sigma = +1 for the smaller id, so
 * that the covariance of f is (2kT/dt)*A.  xi (n x 3) and eta (pairs x 3,
 * pair order) replace the generator when given.  fcons (n x 3, optional)
 * receives sum_j F_ij alone.  Returns the number of off-diagonal entries
 * (2 * pairs), or -1 if that exceeds cap / on allocation failure.         */
int64_t orc_build_system(const orc_params* p, int64_t step, const double* pos,
                         const double* xi, const double* eta, int64_t cap,
                         int64_t* rowptr, int64_t* col, double* val,
                         double* diag, double* rhs, double* fcons) {
  const int64_t n = p->n;
  const double Ly = p->box[1];
  const double delta = orc_le_offset(p, step);
  int64_t* pairs = NULL;
  int64_t np = orc_pairs_alloc(p, step, pos, &pairs);
  if (np < 0) return -1;
  if (2 * np > cap) { free(pairs); return -1; }
  int64_t* fill = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
  if (!fill) { free(pairs); return -1; }

  /* row pointers: each pair appears in both rows */
  for (int64_t i = 0; i <= n; ++i) rowptr[i] = 0;
  for (int64_t k = 0; k < np; ++k) {
    rowptr[pairs[2 * k] + 1]++;
    rowptr[pairs[2 * k + 1] + 1]++;
  }
  for (int64_t i = 0; i < n; ++i) rowptr[i + 1] += rowptr[i];
  for (int64_t i = 0; i < n; ++i) fill[i] = rowptr[i];

  /* node terms */
  double amp_node = 0.0, amp_pair = 0.0;
  if (p->noise_mode == ORC_NOISE_FDT) {
    double c = sqrt(2.0 * p->kT / p->dt);
    amp_node = c * sqrt(p->gamma0);
    amp_pair = c;
  } else if (p->noise_mode == ORC_NOISE_PAPER) {
    amp_node = sqrt(2.0 * p->gamma0 * p->kT / p->dt);
  }
  for (int64_t i = 0; i < n; ++i) {
    diag[i] = p->gamma0;
    double g[4] = {0.0, 0.0, 0.0, 0.0};
    if (xi) { g[0] = xi[3 * i]; g[1] = xi[3 * i + 1]; g[2] = xi[3 * i + 2]; }
    else if (amp_node != 0.0) orc_gauss4(p, (uint64_t)step, 0, (uint64_t)i, 0, g);
    rhs[3 * i + 0] = p->gamma0 * p->shear_rate * (pos[3 * i + 1] - 0.5 * Ly) + amp_node * g[0];
    rhs[3 * i + 1] = amp_node * g[1];
    rhs[3 * i + 2] = amp_node * g[2];
    if (fcons) fcons[3 * i] = fcons[3 * i + 1] = fcons[3 * i + 2] = 0.0;
  }

  /* pair terms */
  double d[3], f[3];
  for (int64_t k = 0; k < np; ++k) {
    const int64_t i = pairs[2 * k], j = pairs[2 * k + 1];
    const int s = orc_separation(p, delta, pos + 3 * i, pos + 3 * j, d);
    const double r2 = orc_r2(d);
    const double w = orc_weight(p, r2);
    orc_pair_force(p, d, r2, f);
    /* matrix */
    col[fill[i]] = j; val[fill[i]] = -p->alpha * w; fill[i]++;
    col[fill[j]] = i; val[fill[j]] = -p->alpha * w; fill[j]++;
    diag[i] += p->alpha * w;
    diag[j] += p->alpha * w;
    /* conservative force, antisymmetric */
    for (int c = 0; c < 3; ++c) {
      rhs[3 * i + c] += f[c];
      rhs[3 * j + c] -= f[c];
      if (fcons) { fcons[3 * i + c] += f[c]; fcons[3 * j + c] -= f[c]; }
    }
    /* boundary velocity V_ij = kappa*Ly*s_ij x, weighted by alpha*w; s_ji = -s_ij */
    double drag = p->alpha * w * (p->shear_rate * Ly * (double)s);
    rhs[3 * i] += drag;
    rhs[3 * j] -= drag;
    /* pair thermal force (weighted incidence times a Gaussian vector) */
    if (amp_pair != 0.0 && p->alpha != 0.0) {
      double g[4] = {0.0, 0.0, 0.0, 0.0};
      if (eta) { g[0] = eta[3 * k]; g[1] = eta[3 * k + 1]; g[2] = eta[3 * k + 2]; }
      else orc_gauss4(p, (uint64_t)step, 1, (uint64_t)i, (uint64_t)j, g);
      double a = amp_pair * sqrt(p->alpha * w);
      for (int c = 0; c < 3; ++c) {
        rhs[3 * i + c] += a * g[c];
        rhs[3 * j + c] -= a * g[c];
      }
    }
  }
  free(fill);
  free(pairs);
  return 2 * np;
}

/* ===================================================================== */
/* Conjugate gradients on (A (x) I_3) x = b                               */
/* ===================================================================== */

/* y = A x, x and y n x 3 */
void orc_spmv3(int64_t n, const int64_t* rowptr, const int64_t* col,
               const double* val, const double* diag, const double* x, double* y) {
  /* rows are independent and each is summed in entry order by one thread:
     the same bits with any thread count */
#pragma omp parallel for schedule(static) if (n > 20000)
  for (int64_t i = 0; i < n; ++i) {
    for (int c = 0; c < 3; ++c) {
      double acc = diag[i] * x[3 * i + c];
      for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) acc += val[k] * x[3 * col[k] + c];
      y[3 * i + c] = acc;
    }
  }
}

typedef struct {
  int kind;
  int64_t n;
  const double* diag;
  /* IC(0) factor L (lower, CSR rows with the diagonal last) */
  int64_t* lrow;
  int64_t* lcol;
  double* lval;
  /* given explicit preconditioner M (applied as z = M r) */
  const int64_t *mrow, *mcol;
  const double *mval, *mdiag;
} orc_precond;

/* IC(0): L has the sparsity of the lower triangle of A (original order) and
 * satisfies (L L^T)_ij = A_ij on that pattern (Meijerink & van der Vorst
 * 1977; exists without breakdown for a symmetric M-matrix such as A).     */
static int orc_ic0_factor(orc_precond* pc, int64_t n, const int64_t* rowptr,
                          const int64_t* col, const double* val, const double* diag) {
  int64_t nnz = n;
  for (int64_t i = 0; i < n; ++i)
    for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
      if (col[k] < i) ++nnz;
  pc->lrow = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
  pc->lcol = (int64_t*)malloc(sizeof(int64_t) * (size_t)nnz);
  pc->lval = (double*)malloc(sizeof(double) * (size_t)nnz);
  if (!pc->lrow || !pc->lcol || !pc->lval) return ORC_ENOMEM;
  int64_t pos = 0;
  for (int64_t i = 0; i < n; ++i) {
    pc->lrow[i] = pos;
    for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
      if (col[k] < i) { pc->lcol[pos] = col[k]; pc->lval[pos] = val[k]; ++pos; }
    pc->lcol[pos] = i; pc->lval[pos] = diag[i]; ++pos;
  }
  pc->lrow[n] = pos;
  for (int64_t i = 0; i < n; ++i) {
    const int64_t a = pc->lrow[i], e = pc->lrow[i + 1] - 1; /* e: diagonal slot */
    for (int64_t q = a; q < e; ++q) {
      const int64_t k = pc->lcol[q];
      /* L_ik = (A_ik - sum_{m<k} L_im L_km) / L_kk, m over both patterns */
      double s = pc->lval[q];
      int64_t u = a, v = pc->lrow[k];
      const int64_t vend = pc->lrow[k + 1] - 1;
      while (u < q && v < vend) {
        if (pc->lcol[u] == pc->lcol[v]) { s -= pc->lval[u] * pc->lval[v]; ++u; ++v; }
        else if (pc->lcol[u] < pc->lcol[v]) ++u;
        else ++v;
      }
      pc->lval[q] = s / pc->lval[pc->lrow[k + 1] - 1];
    }
    double s = pc->lval[e];
    for (int64_t q = a; q < e; ++q) s -= pc->lval[q] * pc->lval[q];
    if (!(s > 0.0)) return ORC_EBREAKDOWN;
    pc->lval[e] = sqrt(s);
  }
  return ORC_OK;
}

/* The IC(0) factor of A in the given row order: lrow[n+1], per row the
 * strictly lower entries in ascending column then the diagonal; lcol/lval
 * hold at most nnz_lower + n entries (cap).  Returns the entry count, or a
 * negative ORC_ status.                                                    */
int64_t orc_ic0(int64_t n, const int64_t* rowptr, const int64_t* col, const double* val,
                const double* diag, int64_t cap, int64_t* lrow, int64_t* lcol, double* lval) {
  orc_precond pc;
  memset(&pc, 0, sizeof(pc));
  pc.n = n;
  const int st = orc_ic0_factor(&pc, n, rowptr, col, val, diag);
  int64_t cnt = st == ORC_OK ? pc.lrow[n] : st;
  if (st == ORC_OK && cnt <= cap) {
    memcpy(lrow, pc.lrow, sizeof(int64_t) * (size_t)(n + 1));
    memcpy(lcol, pc.lcol, sizeof(int64_t) * (size_t)cnt);
    memcpy(lval, pc.lval, sizeof(double) * (size_t)cnt);
  }
  free(pc.lrow);
  free(pc.lcol);
  free(pc.lval);
  return cnt;
}

/* z = M^{-1} r for one component c of n x 3 arrays */
static void orc_apply_precond(const orc_precond* pc, const double* r, double* z, int c) {
  const int64_t n = pc->n;
  if (pc->kind == ORC_PC_JACOBI) {
    for (int64_t i = 0; i < n; ++i) z[3 * i + c] = r[3 * i + c] / pc->diag[i];
  } else if (pc->kind == ORC_PC_NONE) {
    for (int64_t i = 0; i < n; ++i) z[3 * i + c] = r[3 * i + c];
  } else if (pc->kind == ORC_PC_IC0) {
    /* forward solve L y = r, then backward L^T z = y */
    for (int64_t i = 0; i < n; ++i) {
      const int64_t e = pc->lrow[i + 1] - 1;
      double s = r[3 * i + c];
      for (int64_t q = pc->lrow[i]; q < e; ++q) s -= pc->lval[q] * z[3 * pc->lcol[q] + c];
      z[3 * i + c] = s / pc->lval[e];
    }
    for (int64_t i = n - 1; i >= 0; --i) {
      const int64_t e = pc->lrow[i + 1] - 1;
      z[3 * i + c] /= pc->lval[e];
      const double zi = z[3 * i + c];
      for (int64_t q = pc->lrow[i]; q < e; ++q) z[3 * pc->lcol[q] + c] -= pc->lval[q] * zi;
    }
  } else { /* ORC_PC_GIVEN: explicit symmetric M, z = M r */
    for (int64_t i = 0; i < n; ++i) {
      double acc = pc->mdiag[i] * r[3 * i + c];
      for (int64_t k = pc->mrow[i]; k < pc->mrow[i + 1]; ++k) acc += pc->mval[k] * r[3 * pc->mcol[k] + c];
      z[3 * i + c] = acc;
    }
  }
}

/* Threads of the element-wise loops and products (OpenMP; 1 = the plain
   sequential oracle).  Every parallel loop writes disjoint outputs in the
   sequential order of operations, and every sum stays sequential, so
   results do not depend on the thread count. */
void orc_set_threads(int n) {
#ifdef _OPENMP
  omp_set_num_threads(n > 0 ? n : 1);
#else
  (void)n;
#endif
}

int orc_get_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

static double orc_dot(int64_t n, const double* a, const double* b, int c) {
  double s = 0.0;
  for (int64_t i = 0; i < n; ++i) s += a[3 * i + c] * b[3 * i + c];
  return s;
}

/* Preconditioned conjugate gradients (Hestenes & Stiefel 1952; Saad,
 * "Iterative Methods for Sparse Linear Systems", Alg. 9.1), one recurrence
 * per component.  x holds the initial guess on entry.  A component stops
 * when its true residual satisfies ||b - A x|| <= tol*||b||: the recursive
 * residual triggers the check, and a failed check restarts from the true
 * residual.  b = 0 gives x = 0 after 0 iterations.  Returns 0, ORC_ENOCONV
 * (maxit reached) or ORC_EBREAKDOWN (p.Ap <= 0).                          */
int orc_pcg(int64_t n, const int64_t* rowptr, const int64_t* col,
            const double* val, const double* diag, const double* rhs,
            double* x, double tol, int maxit, int precond,
            const int64_t* mrowptr, const int64_t* mcol, const double* mval,
            const double* mdiag, int iters[3], double relres[3]) {
  int status = ORC_OK;
  orc_precond pc;
  memset(&pc, 0, sizeof(pc));
  pc.kind = precond;
  pc.n = n;
  pc.diag = diag;
  pc.mrow = mrowptr; pc.mcol = mcol; pc.mval = mval; pc.mdiag = mdiag;
  double* r = (double*)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
  double* z = (double*)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
  double* pv = (double*)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
  double* q = (double*)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
  if (!r || !z || !pv || !q) { status = ORC_ENOMEM; goto done; }
  if (precond == ORC_PC_IC0) {
    status = orc_ic0_factor(&pc, n, rowptr, col, val, diag);
    if (status != ORC_OK) goto done;
  }
  for (int c = 0; c < 3; ++c) {
    iters[c] = 0;
    relres[c] = 0.0;
    const double bnorm = sqrt(orc_dot(n, rhs, rhs, c));
    if (bnorm == 0.0) {
      for (int64_t i = 0; i < n; ++i) x[3 * i + c] = 0.0;
      continue;
    }
    int converged = 0;
    int restart = 1;
    double rz = 0.0;
    while (!converged) {
      if (restart) {
        /* r = b - A x */
        orc_spmv3(n, rowptr, col, val, diag, x, q);
        for (int64_t i = 0; i < n; ++i) r[3 * i + c] = rhs[3 * i + c] - q[3 * i + c];
        double rn = sqrt(orc_dot(n, r, r, c));
        if (rn <= tol * bnorm) { relres[c] = rn / bnorm; converged = 1; break; }
        orc_apply_precond(&pc, r, z, c);
        for (int64_t i = 0; i < n; ++i) pv[3 * i + c] = z[3 * i + c];
        rz = orc_dot(n, r, z, c);
        restart = 0;
      }
      if (iters[c] >= maxit) { status = ORC_ENOCONV; break; }
      orc_spmv3(n, rowptr, col, val, diag, pv, q);
      const double pq = orc_dot(n, pv, q, c);
      if (!(pq > 0.0)) { status = ORC_EBREAKDOWN; break; }
      const double a = rz / pq;
#pragma omp parallel for schedule(static) if (n > 20000)
      for (int64_t i = 0; i < n; ++i) {
        x[3 * i + c] += a * pv[3 * i + c];
        r[3 * i + c] -= a * q[3 * i + c];
      }
      iters[c]++;
      const double rn = sqrt(orc_dot(n, r, r, c));
      relres[c] = rn / bnorm;
      if (rn <= tol * bnorm) { restart = 1; continue; } /* verified at loop top */
      orc_apply_precond(&pc, r, z, c);
      const double rz_new = orc_dot(n, r, z, c);
      const double beta = rz_new / rz;
      rz = rz_new;
#pragma omp parallel for schedule(static) if (n > 20000)
      for (int64_t i = 0; i < n; ++i) pv[3 * i + c] = z[3 * i + c] + beta * pv[3 * i + c];
    }
    if (status != ORC_OK) break;
  }
done:
  free(r); free(z); free(pv); free(q);
  free(pc.lrow); free(pc.lcol); free(pc.lval);
  return status;
}

/* ===================================================================== */
/* Time step                                                              */
/* ===================================================================== */

/* Bring positions back into the box after a move that ends at step
 * `step_after`: a particle leaving through y = Ly re-enters at y - Ly with
 * x shifted by -delta (the image above is displaced by +delta), and the
 * reverse through y = 0; then x and z are wrapped periodically.  The result
 * lies in [0, L] per axis (L itself only through rounding of y + Ly).     */
void orc_wrap(const orc_params* p, int64_t step_after, double* pos) {
  const double Lx = p->box[0], Ly = p->box[1], Lz = p->box[2];
  const double delta = orc_le_offset(p, step_after);
  for (int64_t i = 0; i < p->n; ++i) {
    double x = pos[3 * i], y = pos[3 * i + 1], z = pos[3 * i + 2];
    if (y >= Ly) { y = y - Ly; x = x - delta; }
    else if (y < 0.0) { y = y + Ly; x = x + delta; }
    for (int k = 0; k < 3; ++k)
      if (x >= Lx) x = x - Lx;
    for (int k = 0; k < 3; ++k)
      if (x < 0.0) x = x + Lx;
    if (z >= Lz) z = z - Lz;
    else if (z < 0.0) z = z + Lz;
    pos[3 * i] = x; pos[3 * i + 1] = y; pos[3 * i + 2] = z;
  }
}

/* One step of Eq. 7 from step n to n+1: solve Eq. 9 at the positions of
 * step n (x0 = 0), then R += v*dt (first-order, Euler-Maruyama) and wrap.
 * vel receives v (n x 3).  On a failed solve the positions are unchanged. */
int orc_step(const orc_params* p, int64_t step, double* pos, double* vel,
             double tol, int maxit, int precond, int iters[3]) {
  const int64_t n = p->n;
  int64_t np = orc_count_pairs(p, step, pos);
  if (np < 0) return ORC_ENOMEM;
  int64_t cap = 2 * np;
  int64_t* rowptr = (int64_t*)malloc(sizeof(int64_t) * (size_t)(n + 1));
  int64_t* col = (int64_t*)malloc(sizeof(int64_t) * (size_t)(cap > 0 ? cap : 1));
  double* val = (double*)malloc(sizeof(double) * (size_t)(cap > 0 ? cap : 1));
  double* diag = (double*)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
  double* rhs = (double*)malloc(sizeof(double) * 3 * (size_t)(n > 0 ? n : 1));
  int status = ORC_OK;
  double relres[3];
  if (!rowptr || !col || !val || !diag || !rhs) { status = ORC_ENOMEM; goto done; }
  if (orc_build_system(p, step, pos, NULL, NULL, cap, rowptr, col, val, diag, rhs, NULL) < 0) {
    status = ORC_ENOMEM;
    goto done;
  }
  for (int64_t i = 0; i < 3 * n; ++i) vel[i] = 0.0;
  status = orc_pcg(n, rowptr, col, val, diag, rhs, vel, tol, maxit, precond,
                   NULL, NULL, NULL, NULL, iters, relres);
  if (status != ORC_OK) goto done;
  for (int64_t i = 0; i < 3 * n; ++i) pos[i] += vel[i] * p->dt;
  orc_wrap(p, step + 1, pos);
done:
  free(rowptr); free(col); free(val); free(diag); free(rhs);
  return status;
}
