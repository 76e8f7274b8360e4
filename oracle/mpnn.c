/*
 * mpnn.c -- plain FP64 oracle of the learned preconditioner: a 3-layer
 * message-passing network on the pair graph of the friction matrix A
 * (Method section, Eq. 9) that outputs a symmetric approximate inverse M^-1
 * with the sparsity of A, and the training loss with its gradient.
 *
 * TEST INFRASTRUCTURE ONLY (see oracle.h).  Written from the network's
 * definition below with straightforward loops; the gradient is analytic
 * backpropagation (pinned by finite differences in the tests).
 *
 * Inputs (A in original order, CSR of the off-diagonal part, val = -alpha*w):
 *   node features x_i = (t_i, a_i, deg_i / 8):
 *       t_i = -sum_j val_ij / D_i      (the pair share of the diagonal)
 *       a_i = sum_j What_ij, What_ij = -val_ij / sqrt(D_i D_j)
 *   edge features e_ij = (r_ij / rc, w_ij, What_ij), w_ij = -val_ij / alpha
 * Network (hidden H = 32, three layers):
 *   h0_i = relu(W0 x_i + b0)
 *   layer l:  y_j = P_l h_j;   m_i = (1/8) sum_j relu(y_j + Q_l e_ij + c_l)
 *             h_i <- h_i + relu(U_l h_i + V_l m_i + d_l)
 *   heads:    lam_i = softplus(v . h_i + v0) + eps              (eps = 0.3)
 *             S_ij  = z . (h_i * h_j) + ze . e_ij + z0          (symmetric)
 * Preconditioner:
 *   M^-1 = D^-1/2 (diag(lam) + S) D^-1/2:  mdiag_i = lam_i / D_i,
 *   moff_ij = S_ij / sqrt(D_i D_j).
 *   Symmetric with a positive diagonal; not positive definite for every
 *   parameter value (the best sparse approximate inverses of A are not
 *   diagonally dominant).  lam = 1, S = What is the two-term Neumann series
 *   D^-1 + D^-1 (D - A) D^-1, which is positive definite because
 *   D^-1/2 (D - A) D^-1/2 has spectral radius below 1 (A strictly
 *   diagonally dominant).
 * Loss on a system (A, b, x*): L = ||M^-1 b - x*||_A^2 / ||x*||_A^2, summed
 * over the three components.
 * Weights enter in bfloat16 (round to nearest even of the FP32 master
 * values); everything else is FP64 here.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

#define H 32
#define FN 3
#define FE 3
#define NL 3
#define EPS_LAM 0.3
#define MSG_SCALE 0.125

/* parameter offsets (floats) */
#define OFF_W0 0
#define OFF_B0 (OFF_W0 + H * FN)
#define OFF_L0 (OFF_B0 + H)
#define L_P 0
#define L_Q (L_P + H * H)
#define L_C (L_Q + H * FE)
#define L_U (L_C + H)
#define L_V (L_U + H * H)
#define L_D (L_V + H * H)
#define L_SIZE (L_D + H)
#define OFF_HEAD (OFF_L0 + NL * L_SIZE)
#define H_V 0
#define H_V0 (H_V + H)
#define H_Z (H_V0 + 1)
#define H_ZE (H_Z + H)
#define H_Z0 (H_ZE + FE)
#define NPARAMS (OFF_HEAD + H_Z0 + 1)

int64_t orc_mpnn_nparams(void) { return NPARAMS; }

/* weights enter rounded to bfloat16 unless switched off (finite-difference
 * tests perturb FP32 weights by amounts below the bfloat16 spacing) */
static int g_use_bf16 = 1;
void orc_mpnn_set_bf16(int on) { g_use_bf16 = on; }

/* bfloat16 value of an FP32 number: keep the top 16 bits after rounding the
 * discarded 16 to nearest, ties to even (NaN kept as NaN) */
double orc_bf16(float f) {
  uint32_t u;
  memcpy(&u, &f, 4);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) {
    u |= 0x00400000u;
  } else {
    const uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
  }
  u &= 0xffff0000u;
  float r;
  memcpy(&r, &u, 4);
  return (double)r;
}

static double relu(double a) { return a > 0.0 ? a : 0.0; }
static double sigm(double a) { return 1.0 / (1.0 + exp(-a)); }
static double softplus(double a) { return a > 30.0 ? a : log1p(exp(a)); }

typedef struct {
  int64_t n, nnz;
  const int64_t *rowptr, *col;
  const double *val, *diag, *edge_r;
  double alpha;
  double th[NPARAMS];    /* bf16-valued weights */
  double *x;             /* n x FN */
  double *e;             /* nnz x FE */
  double *hs;            /* (NL+1) x n x H : h^0..h^3 */
  double *ys;            /* NL x n x H     : y^l = P_l h^{l-1} */
  double *ms;            /* NL x n x H     : m^l */
  double *as;            /* NL x n x H     : pre-activation of the update */
  double *tau;           /* n   : node head pre-activation */
  double *tg;            /* nnz : edge head pre-activation */
  double *what;          /* nnz */
} net_t;

static void net_free(net_t* t) {
  free(t->x); free(t->e); free(t->hs); free(t->ys); free(t->ms); free(t->as);
  free(t->tau); free(t->tg); free(t->what);
}

/* features, encoder and message-passing layers (h^0 .. h^NL) */
static int net_trunk(net_t* t, const float* theta) {
  const int64_t n = t->n, nnz = t->nnz;
  for (int k = 0; k < NPARAMS; ++k) t->th[k] = g_use_bf16 ? orc_bf16(theta[k]) : (double)theta[k];
  t->x = (double*)calloc((size_t)(n * FN + 1), sizeof(double));
  t->e = (double*)calloc((size_t)(nnz * FE + 1), sizeof(double));
  t->hs = (double*)calloc((size_t)((NL + 1) * n * H + 1), sizeof(double));
  t->ys = (double*)calloc((size_t)(NL * n * H + 1), sizeof(double));
  t->ms = (double*)calloc((size_t)(NL * n * H + 1), sizeof(double));
  t->as = (double*)calloc((size_t)(NL * n * H + 1), sizeof(double));
  t->tau = (double*)calloc((size_t)(n + 1), sizeof(double));
  t->tg = (double*)calloc((size_t)(nnz + 1), sizeof(double));
  t->what = (double*)calloc((size_t)(nnz + 1), sizeof(double));
  if (!t->x || !t->e || !t->hs || !t->ys || !t->ms || !t->as || !t->tau || !t->tg ||
      !t->what)
    return -2;
  const double* th = t->th;
  /* features */
  for (int64_t i = 0; i < n; ++i) {
    double s = 0.0, a = 0.0;
    for (int64_t q = t->rowptr[i]; q < t->rowptr[i + 1]; ++q) {
      const int64_t j = t->col[q];
      t->what[q] = -t->val[q] / sqrt(t->diag[i] * t->diag[j]);
      s += -t->val[q];
      a += t->what[q];
      t->e[FE * q + 0] = t->edge_r[q];
      t->e[FE * q + 1] = -t->val[q] / t->alpha;
      t->e[FE * q + 2] = t->what[q];
    }
    t->x[FN * i + 0] = s / t->diag[i];
    t->x[FN * i + 1] = a;
    t->x[FN * i + 2] = (double)(t->rowptr[i + 1] - t->rowptr[i]) / 8.0;
  }
  /* encoder */
  for (int64_t i = 0; i < n; ++i)
    for (int k = 0; k < H; ++k) {
      double acc = th[OFF_B0 + k];
      for (int f = 0; f < FN; ++f) acc += th[OFF_W0 + k * FN + f] * t->x[FN * i + f];
      t->hs[i * H + k] = relu(acc);
    }
  /* layers */
  for (int l = 0; l < NL; ++l) {
    const double* L = th + OFF_L0 + l * L_SIZE;
    const double* hin = t->hs + (int64_t)l * n * H;
    double* hout = t->hs + (int64_t)(l + 1) * n * H;
    double* y = t->ys + (int64_t)l * n * H;
    double* m = t->ms + (int64_t)l * n * H;
    double* a = t->as + (int64_t)l * n * H;
    for (int64_t i = 0; i < n; ++i)
      for (int k = 0; k < H; ++k) {
        double acc = 0.0;
        for (int q = 0; q < H; ++q) acc += L[L_P + k * H + q] * hin[i * H + q];
        y[i * H + k] = acc;
      }
    for (int64_t i = 0; i < n; ++i) {
      for (int k = 0; k < H; ++k) m[i * H + k] = 0.0;
      for (int64_t q = t->rowptr[i]; q < t->rowptr[i + 1]; ++q) {
        const int64_t j = t->col[q];
        for (int k = 0; k < H; ++k) {
          double s = y[j * H + k] + L[L_C + k];
          for (int f = 0; f < FE; ++f) s += L[L_Q + k * FE + f] * t->e[FE * q + f];
          m[i * H + k] += MSG_SCALE * relu(s);
        }
      }
      for (int k = 0; k < H; ++k) {
        double acc = L[L_D + k];
        for (int q = 0; q < H; ++q)
          acc += L[L_U + k * H + q] * hin[i * H + q] + L[L_V + k * H + q] * m[i * H + q];
        a[i * H + k] = acc;
        hout[i * H + k] = hin[i * H + k] + relu(acc);
      }
    }
  }
  return 0;
}

/* scalar heads: tau (node), tg = S (edge) and, if asked, the scalar M^-1 */
static void net_heads(net_t* t, double* mdiag, double* moff) {
  const int64_t n = t->n;
  const double* hd = t->th + OFF_HEAD;
  const double* hf = t->hs + (int64_t)NL * n * H;
  for (int64_t i = 0; i < n; ++i) {
    double acc = hd[H_V0];
    for (int k = 0; k < H; ++k) acc += hd[H_V + k] * hf[i * H + k];
    t->tau[i] = acc;
  }
  for (int64_t i = 0; i < n; ++i) {
    for (int64_t q = t->rowptr[i]; q < t->rowptr[i + 1]; ++q) {
      const int64_t j = t->col[q];
      double acc = hd[H_Z0];
      for (int k = 0; k < H; ++k) acc += hd[H_Z + k] * (hf[i * H + k] * hf[j * H + k]);
      for (int f = 0; f < FE; ++f) acc += hd[H_ZE + f] * t->e[FE * q + f];
      t->tg[q] = acc;  /* S_ij */
      if (moff) moff[q] = acc / sqrt(t->diag[i] * t->diag[j]);
    }
    if (mdiag) mdiag[i] = (softplus(t->tau[i]) + EPS_LAM) / t->diag[i];
  }
}

static int net_forward(net_t* t, const float* theta, double* mdiag, double* moff) {
  if (net_trunk(t, theta) != 0) return -2;
  net_heads(t, mdiag, moff);
  return 0;
}

/* backward through the layers and the encoder: dh holds dL/dh^NL on entry
 * (it is overwritten); dm and da are n x H work arrays */
static void net_trunk_backward(const net_t* t, double* dh, double* dm, double* da,
                               double* grad) {
  const int64_t n = t->n;
  const int64_t* rowptr = t->rowptr;
  const int64_t* col = t->col;
  const double* th = t->th;
  /* layers, last to first; dh holds dL/dh^{l+1} on entry to layer l */
  for (int l = NL - 1; l >= 0; --l) {
    const double* L = th + OFF_L0 + l * L_SIZE;
    double* G = grad + OFF_L0 + l * L_SIZE;
    const double* hin = t->hs + (int64_t)l * n * H;
    const double* y = t->ys + (int64_t)l * n * H;
    const double* m = t->ms + (int64_t)l * n * H;
    const double* a = t->as + (int64_t)l * n * H;
    for (int64_t i = 0; i < n; ++i)
      for (int k = 0; k < H; ++k) da[i * H + k] = a[i * H + k] > 0.0 ? dh[i * H + k] : 0.0;
    /* h_out = h_in + relu(U h_in + V m + d): dh_in = dh_out + U^T da, dm = V^T da */
    for (int64_t i = 0; i < n; ++i)
      for (int k = 0; k < H; ++k) {
        const double dak = da[i * H + k];
        G[L_D + k] += dak;
        for (int q = 0; q < H; ++q) {
          G[L_U + k * H + q] += dak * hin[i * H + q];
          G[L_V + k * H + q] += dak * m[i * H + q];
        }
      }
    for (int64_t i = 0; i < n; ++i)
      for (int q = 0; q < H; ++q) {
        double su = 0.0, sv = 0.0;
        for (int k = 0; k < H; ++k) {
          su += L[L_U + k * H + q] * da[i * H + k];
          sv += L[L_V + k * H + q] * da[i * H + k];
        }
        dh[i * H + q] += su;   /* dh_in = dh_out + U^T da (dh_out already in dh) */
        dm[i * H + q] = sv;
      }
    /* m_i = (1/8) sum_j relu(y_j + Q e_ij + c): dy_j, dQ, dc; dh_in += P^T dy */
    double* dy = da; /* reuse: da is no longer needed */
    for (int64_t i = 0; i < n * H; ++i) dy[i] = 0.0;
    for (int64_t i = 0; i < n; ++i)
      for (int64_t q = rowptr[i]; q < rowptr[i + 1]; ++q) {
        const int64_t j = col[q];
        for (int k = 0; k < H; ++k) {
          double s = y[j * H + k] + L[L_C + k];
          for (int f = 0; f < FE; ++f) s += L[L_Q + k * FE + f] * t->e[FE * q + f];
          if (!(s > 0.0)) continue;
          const double dq = MSG_SCALE * dm[i * H + k];
          G[L_C + k] += dq;
          for (int f = 0; f < FE; ++f) G[L_Q + k * FE + f] += dq * t->e[FE * q + f];
          dy[j * H + k] += dq;
        }
      }
    for (int64_t i = 0; i < n; ++i)
      for (int k = 0; k < H; ++k)
        for (int q = 0; q < H; ++q) G[L_P + k * H + q] += dy[i * H + k] * hin[i * H + q];
    for (int64_t i = 0; i < n; ++i)
      for (int q = 0; q < H; ++q) {
        double s = 0.0;
        for (int k = 0; k < H; ++k) s += L[L_P + k * H + q] * dy[i * H + k];
        dh[i * H + q] += s;
      }
  }
  /* encoder: h0 = relu(W0 x + b0) */
  for (int64_t i = 0; i < n; ++i)
    for (int k = 0; k < H; ++k) {
      double acc = th[OFF_B0 + k];
      for (int f = 0; f < FN; ++f) acc += th[OFF_W0 + k * FN + f] * t->x[FN * i + f];
      if (!(acc > 0.0)) continue;
      grad[OFF_B0 + k] += dh[i * H + k];
      for (int f = 0; f < FN; ++f) grad[OFF_W0 + k * FN + f] += dh[i * H + k] * t->x[FN * i + f];
    }
}

/* M^-1 (mdiag, moff) for the system (rowptr, col, val, diag) */
int orc_mpnn_forward(int64_t n, const int64_t* rowptr, const int64_t* col, const double* val,
                     const double* diag, const double* edge_r, double alpha, const float* theta,
                     double* mdiag, double* moff) {
  net_t t;
  memset(&t, 0, sizeof(t));
  t.n = n; t.nnz = rowptr[n]; t.rowptr = rowptr; t.col = col; t.val = val; t.diag = diag;
  t.edge_r = edge_r; t.alpha = alpha;
  int rc = net_forward(&t, theta, mdiag, moff);
  net_free(&t);
  return rc;
}

/* Loss L = ||M^-1 b - x*||^2 / ||x*||^2 (three components) in the A-norm
 * (euclid = 0) or the Euclidean norm (euclid = 1) and, if grad is given,
 * dL/dtheta (with respect to the bf16-rounded weights).                     */
double orc_mpnn_loss_grad_norm(int64_t n, const int64_t* rowptr, const int64_t* col,
                               const double* val, const double* diag, const double* edge_r,
                               double alpha, const float* theta, const double* b,
                               const double* xstar, int euclid, double* grad) {
  net_t t;
  memset(&t, 0, sizeof(t));
  t.n = n; t.nnz = rowptr[n]; t.rowptr = rowptr; t.col = col; t.val = val; t.diag = diag;
  t.edge_r = edge_r; t.alpha = alpha;
  const int64_t nnz = t.nnz;
  double* mdiag = (double*)malloc(sizeof(double) * (size_t)(n + 1));
  double* moff = (double*)malloc(sizeof(double) * (size_t)(nnz + 1));
  double* z = (double*)malloc(sizeof(double) * 3 * (size_t)(n + 1));
  double* ae = (double*)malloc(sizeof(double) * 3 * (size_t)(n + 1));
  double* ax = (double*)malloc(sizeof(double) * 3 * (size_t)(n + 1));
  double loss = NAN;
  if (!mdiag || !moff || !z || !ae || !ax || net_forward(&t, theta, mdiag, moff) != 0) goto out;
  /* z = M^-1 b, e = z - x*, A e, A x* */
  orc_spmv3(n, rowptr, col, moff, mdiag, b, z);
  for (int64_t i = 0; i < 3 * n; ++i) z[i] -= xstar[i];
  if (euclid) {
    /* the identity in place of A */
    memcpy(ae, z, sizeof(double) * 3 * (size_t)n);
    memcpy(ax, xstar, sizeof(double) * 3 * (size_t)n);
  } else {
    orc_spmv3(n, rowptr, col, val, diag, z, ae);
    orc_spmv3(n, rowptr, col, val, diag, xstar, ax);
  }
  double num = 0.0, den = 0.0;
  for (int64_t i = 0; i < 3 * n; ++i) {
    num += z[i] * ae[i];
    den += xstar[i] * ax[i];
  }
  loss = num / den;
  if (!grad) goto out;
  {
    for (int k = 0; k < NPARAMS; ++k) grad[k] = 0.0;
    const double* th = t.th;
    const double* hd = th + OFF_HEAD;
    double* gh = grad + OFF_HEAD;
    /* dL/dz = 2 A e / den (2 e / den Euclidean); dL/dmdiag_i = sum_c G_ic b_ic;
     * dL/dmoff_ij = sum_c G_ic b_jc */
    double* gl = (double*)calloc((size_t)(n + 1), sizeof(double));     /* dL/dlam */
    double* gt = (double*)calloc((size_t)(n + 1), sizeof(double));     /* dL/dtau */
    double* dh = (double*)calloc((size_t)(n * H + 1), sizeof(double)); /* dL/dh */
    double* dm = (double*)calloc((size_t)(n * H + 1), sizeof(double));
    double* da = (double*)calloc((size_t)(n * H + 1), sizeof(double));
    if (!gl || !gt || !dh || !dm || !da) { free(gl); free(gt); free(dh); free(dm); free(da); loss = NAN; goto out; }
    for (int64_t i = 0; i < n; ++i) {
      double gd = 0.0;
      for (int c = 0; c < 3; ++c) gd += 2.0 * ae[3 * i + c] / den * b[3 * i + c];
      gl[i] = gd / diag[i];                      /* mdiag = lam / D */
      gt[i] = gl[i] * sigm(t.tau[i]);            /* lam = softplus(tau) + eps */
    }
    const double* hf = t.hs + (int64_t)NL * n * H;
    for (int64_t i = 0; i < n; ++i) {
      /* node head */
      gh[H_V0] += gt[i];
      for (int k = 0; k < H; ++k) {
        gh[H_V + k] += gt[i] * hf[i * H + k];
        dh[i * H + k] += gt[i] * hd[H_V + k];
      }
      /* edge head: each directed entry evaluates S_ij for its own moff_ij
       * (the reverse entry evaluates the same value for moff_ji) */
      for (int64_t q = rowptr[i]; q < rowptr[i + 1]; ++q) {
        const int64_t j = col[q];
        double gm = 0.0;
        for (int c = 0; c < 3; ++c) gm += 2.0 * ae[3 * i + c] / den * b[3 * j + c];
        const double dtg = gm / sqrt(diag[i] * diag[j]);
        gh[H_Z0] += dtg;
        for (int f = 0; f < FE; ++f) gh[H_ZE + f] += dtg * t.e[FE * q + f];
        for (int k = 0; k < H; ++k) {
          gh[H_Z + k] += dtg * (hf[i * H + k] * hf[j * H + k]);
          dh[i * H + k] += dtg * hd[H_Z + k] * hf[j * H + k];
          dh[j * H + k] += dtg * hd[H_Z + k] * hf[i * H + k];
        }
      }
    }
    net_trunk_backward(&t, dh, dm, da, grad);
    free(gl); free(gt); free(dh); free(dm); free(da);
  }
out:
  free(mdiag); free(moff); free(z); free(ae); free(ax);
  net_free(&t);
  return loss;
}

double orc_mpnn_loss_grad(int64_t n, const int64_t* rowptr, const int64_t* col, const double* val,
                          const double* diag, const double* edge_r, double alpha,
                          const float* theta, const double* b, const double* xstar, double* grad) {
  return orc_mpnn_loss_grad_norm(n, rowptr, col, val, diag, edge_r, alpha, theta, b, xstar, 0,
                                 grad);
}

/* ===========================================================================
 * The learned preconditioner for the anisotropic friction system (block.c:
 * genuine 3 x 3 blocks, A_ij = -W_ij, A_ii = gamma0 I + sum_j W_ij).
 *
 * The trunk above runs unchanged on the scalar shadow of A, the traces
 *   d_i = tr(A_ii) / 3,  omega_ij = tr(W_ij) / 3,
 * in place of (diag, -val): its features are rotation invariant and equal
 * those of the isotropic system when every block is a multiple of I_3
 * (What_ij = omega_ij / sqrt(d_i d_j)).  The heads give four numbers per
 * node / entry:
 *   lam_i  = softplus(v . h_i + v0) + eps          (the scalar node head)
 *   S_ij   = z . (h_i * h_j) + ze . e_ij + z0      (the scalar edge head)
 *   mu_i   = u . h_i + u0                          (node anisotropy)
 *   sig_ij = s . (h_i * h_j) + se . e_ij + s0      (edge anisotropy)
 * and the preconditioner is built in the frame where every diagonal block
 * of A is the identity, R = blockdiag(A_ii^-1/2) (symmetric roots), the
 * block analogue of the scalar network's D^-1/2 (Lambda + S) D^-1/2:
 *   Nh_ij = R_i W_ij R_j                           (normalised pair block)
 *   Xh_ii = lam_i I + mu_i (d_i A_ii^-1 - I),
 *   Xh_ij = S_ij I + sig_ij (Nh_ij - What_ij I),
 *   M^-1 = R Xh R.
 * Built from I and A's own blocks only, M^-1 turns with the system under a
 * rotation; it is symmetric (Xh_ji = Xh_ij^T); when every block of A is a
 * multiple of I_3 both anisotropy terms vanish and M^-1 is the scalar
 * network's preconditioner times I_3.  lam = 1, mu = 0, S = What, sig = 1
 * give Xh = I + Nh, i.e. M^-1 = D^-1 + D^-1 (D - A) D^-1, D = blockdiag(A_ii):
 * the two-term Neumann series of the block-Jacobi splitting, positive
 * definite since each pair adds the positive semidefinite [[W, W], [W, W]]
 * to 2D - A = gamma0 I + ...
 * Parameters: the scalar network's, then u[32], u0, s[32], se[3], s0.
 * =========================================================================== */
#define NPHI (H + 1 + H + FE + 1)
#define PHI_U 0
#define PHI_U0 (PHI_U + H)
#define PHI_S (PHI_U0 + 1)
#define PHI_SE (PHI_S + H)
#define PHI_S0 (PHI_SE + FE)

int64_t orc_mpnn_block_nparams(void) { return NPARAMS + NPHI; }

/* out = a b c (3 x 3, row-major) */
static void mul33(const double* a, const double* b, const double* c, double* out) {
  double ab[9];
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k) {
      double s = 0.0;
      for (int l = 0; l < 3; ++l) s += a[3 * r + l] * b[3 * l + k];
      ab[3 * r + k] = s;
    }
  for (int r = 0; r < 3; ++r)
    for (int k = 0; k < 3; ++k) {
      double s = 0.0;
      for (int l = 0; l < 3; ++l) s += ab[3 * r + l] * c[3 * l + k];
      out[3 * r + k] = s;
    }
}

/* eigenvalues w and orthonormal eigenvectors (columns of V) of a symmetric
 * 3 x 3 matrix by the cyclic Jacobi method (Golub & Van Loan, sec. 8.5):
 * rotations that zero one off-diagonal entry at a time, sweeps until the
 * off-diagonal part is negligible */
static void eig_sym3(const double* a, double* w, double* V) {
  double m[3][3];
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      m[r][c] = a[3 * r + c];
      V[3 * r + c] = r == c ? 1.0 : 0.0;
    }
  for (int sweep = 0; sweep < 50; ++sweep) {
    const double off = m[0][1] * m[0][1] + m[0][2] * m[0][2] + m[1][2] * m[1][2];
    const double dia = m[0][0] * m[0][0] + m[1][1] * m[1][1] + m[2][2] * m[2][2];
    if (off <= 1e-34 * dia) break;
    for (int p = 0; p < 2; ++p)
      for (int q = p + 1; q < 3; ++q) {
        if (m[p][q] == 0.0) continue;
        /* c, s of the rotation that zeroes m[p][q] (the smaller angle) */
        const double theta = (m[q][q] - m[p][p]) / (2.0 * m[p][q]);
        const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
        const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
        /* m <- J^T m J, V <- V J, J the rotation in the (p, q) plane */
        for (int k = 0; k < 3; ++k) {
          const double mkp = m[k][p], mkq = m[k][q];
          m[k][p] = c * mkp - s * mkq;
          m[k][q] = s * mkp + c * mkq;
        }
        for (int k = 0; k < 3; ++k) {
          const double mpk = m[p][k], mqk = m[q][k];
          m[p][k] = c * mpk - s * mqk;
          m[q][k] = s * mpk + c * mqk;
        }
        for (int k = 0; k < 3; ++k) {
          const double vkp = V[3 * k + p], vkq = V[3 * k + q];
          V[3 * k + p] = c * vkp - s * vkq;
          V[3 * k + q] = s * vkp + c * vkq;
        }
      }
  }
  for (int k = 0; k < 3; ++k) w[k] = m[k][k];
}

/* f(a) = V diag(f(w)) V^T for symmetric positive definite a: power -1/2
 * (inverse square root) or -1 (inverse); -1 if not positive definite */
static int sym3_power(const double* a, double power, double* out) {
  double w[3], V[9];
  eig_sym3(a, w, V);
  double fw[3];
  for (int k = 0; k < 3; ++k) {
    if (!(w[k] > 0.0)) return -1;
    fw[k] = power == -1.0 ? 1.0 / w[k] : 1.0 / sqrt(w[k]);
  }
  for (int r = 0; r < 3; ++r)
    for (int c = 0; c < 3; ++c) {
      double s = 0.0;
      for (int k = 0; k < 3; ++k) s += V[3 * r + k] * fw[k] * V[3 * c + k];
      out[3 * r + c] = s;
    }
  return 0;
}

typedef struct {
  net_t t;
  double phi[NPHI];     /* anisotropy head weights (bf16-valued) */
  double *val, *diag;   /* scalar shadow: -omega per entry, d per node */
  double *rt, *binv;    /* n x 9: A_ii^-1/2 and A_ii^-1 */
  double *nh;           /* nnz x 9: Nh_ij = R_i W_ij R_j */
  double *md, *mo;      /* M^-1 blocks: n x 9, nnz x 9 */
} bnet_t;

static void bnet_free(bnet_t* B) {
  free(B->val); free(B->diag); free(B->rt); free(B->binv); free(B->nh); free(B->md);
  free(B->mo);
  net_free(&B->t);
}

static int bnet_forward(bnet_t* B, int64_t n, const int64_t* rowptr, const int64_t* col,
                        const double* bval, const double* bdiag, const double* edge_r,
                        double alpha, const float* theta) {
  const int64_t nnz = rowptr[n];
  B->val = (double*)calloc((size_t)(nnz + 1), sizeof(double));
  B->diag = (double*)calloc((size_t)(n + 1), sizeof(double));
  B->rt = (double*)calloc((size_t)(9 * n + 1), sizeof(double));
  B->binv = (double*)calloc((size_t)(9 * n + 1), sizeof(double));
  B->nh = (double*)calloc((size_t)(9 * nnz + 1), sizeof(double));
  B->md = (double*)calloc((size_t)(9 * n + 1), sizeof(double));
  B->mo = (double*)calloc((size_t)(9 * nnz + 1), sizeof(double));
  if (!B->val || !B->diag || !B->rt || !B->binv || !B->nh || !B->md || !B->mo) return -2;
  for (int64_t q = 0; q < nnz; ++q)
    B->val[q] = ((bval[9 * q] + bval[9 * q + 4]) + bval[9 * q + 8]) / 3.0;
  for (int64_t i = 0; i < n; ++i) {
    B->diag[i] = ((bdiag[9 * i] + bdiag[9 * i + 4]) + bdiag[9 * i + 8]) / 3.0;
    if (sym3_power(bdiag + 9 * i, -0.5, B->rt + 9 * i) != 0) return -1;
    if (sym3_power(bdiag + 9 * i, -1.0, B->binv + 9 * i) != 0) return -1;
  }
  for (int64_t i = 0; i < n; ++i)
    for (int64_t q = rowptr[i]; q < rowptr[i + 1]; ++q) {
      double W[9];
      for (int m = 0; m < 9; ++m) W[m] = -bval[9 * q + m];
      mul33(B->rt + 9 * i, W, B->rt + 9 * col[q], B->nh + 9 * q);
    }
  net_t* t = &B->t;
  t->n = n; t->nnz = nnz; t->rowptr = rowptr; t->col = col; t->val = B->val;
  t->diag = B->diag; t->edge_r = edge_r; t->alpha = alpha;
  if (net_trunk(t, theta) != 0) return -2;
  net_heads(t, NULL, NULL);
  for (int k = 0; k < NPHI; ++k)
    B->phi[k] = g_use_bf16 ? orc_bf16(theta[NPARAMS + k]) : (double)theta[NPARAMS + k];
  const double* ph = B->phi;
  const double* hf = t->hs + (int64_t)NL * n * H;
  for (int64_t i = 0; i < n; ++i) {
    const double* Ri = B->rt + 9 * i;
    const double di = B->diag[i];
    double mu = ph[PHI_U0];
    for (int k = 0; k < H; ++k) mu += ph[PHI_U + k] * hf[i * H + k];
    const double lam = softplus(t->tau[i]) + EPS_LAM;
    double X[9];
    for (int m = 0; m < 9; ++m) {
      const double id = m % 4 == 0 ? 1.0 : 0.0;
      X[m] = lam * id + mu * (di * B->binv[9 * i + m] - id);
    }
    mul33(Ri, X, Ri, B->md + 9 * i);
    for (int64_t q = rowptr[i]; q < rowptr[i + 1]; ++q) {
      const int64_t j = col[q];
      double sg = ph[PHI_S0];
      for (int k = 0; k < H; ++k) sg += ph[PHI_S + k] * (hf[i * H + k] * hf[j * H + k]);
      for (int f = 0; f < FE; ++f) sg += ph[PHI_SE + f] * t->e[FE * q + f];
      const double what = t->what[q];
      for (int m = 0; m < 9; ++m) {
        const double id = m % 4 == 0 ? 1.0 : 0.0;
        X[m] = t->tg[q] * id + sg * (B->nh[9 * q + m] - what * id);
      }
      mul33(Ri, X, B->rt + 9 * j, B->mo + 9 * q);
    }
  }
  return 0;
}

/* M^-1 blocks (row-major 3 x 3: mdiag n x 9, moff nnz x 9) for the block
 * system (rowptr, col, bval, bdiag) of block.c in original order */
int orc_mpnn_block_forward(int64_t n, const int64_t* rowptr, const int64_t* col,
                           const double* bval, const double* bdiag, const double* edge_r,
                           double alpha, const float* theta, double* mdiag, double* moff) {
  bnet_t B;
  memset(&B, 0, sizeof(B));
  int rc = bnet_forward(&B, n, rowptr, col, bval, bdiag, edge_r, alpha, theta);
  if (rc == 0) {
    memcpy(mdiag, B.md, sizeof(double) * 9 * (size_t)n);
    memcpy(moff, B.mo, sizeof(double) * 9 * (size_t)rowptr[n]);
  }
  bnet_free(&B);
  return rc;
}

/* y = A x (block system, stacked 3n vectors) */
static void bsys_mul(int64_t n, const int64_t* rowptr, const int64_t* col, const double* offd,
                     const double* dg, const double* x, double* y) {
  for (int64_t i = 0; i < n; ++i)
    for (int c = 0; c < 3; ++c) {
      double s = 0.0;
      for (int l = 0; l < 3; ++l) s += dg[9 * i + 3 * c + l] * x[3 * i + l];
      for (int64_t q = rowptr[i]; q < rowptr[i + 1]; ++q)
        for (int l = 0; l < 3; ++l) s += offd[9 * q + 3 * c + l] * x[3 * col[q] + l];
      y[3 * i + c] = s;
    }
}

/* Loss L = ||M^-1 b - x*||^2 / ||x*||^2 on the block system, in the A-norm
 * (euclid = 0) or the Euclidean norm (euclid = 1), and, if grad is given,
 * dL/dtheta (NPARAMS + NPHI values).  dL/dM_ij = G_i b_j^T with
 * G = 2 W (M^-1 b - x*) / ||x*||_W^2; through M^-1 = R Xh R,
 * dL/dXh_ij = R_i dL/dM_ij R_j, and the heads enter Xh linearly:
 *   dL/dlam_i = tr dXh_ii, dL/dmu_i = <dXh_ii, d_i A_ii^-1 - I>,
 *   dL/dS_ij = tr dXh_ij, dL/dsig_ij = <dXh_ij, Nh_ij - What_ij I>
 * (<., .> the Frobenius product).                                          */
double orc_mpnn_block_loss_grad(int64_t n, const int64_t* rowptr, const int64_t* col,
                                const double* bval, const double* bdiag, const double* edge_r,
                                double alpha, const float* theta, const double* b,
                                const double* xstar, int euclid, double* grad) {
  bnet_t B;
  memset(&B, 0, sizeof(B));
  double* z = (double*)calloc((size_t)(3 * n + 1), sizeof(double));
  double* ae = (double*)calloc((size_t)(3 * n + 1), sizeof(double));
  double* ax = (double*)calloc((size_t)(3 * n + 1), sizeof(double));
  double loss = NAN;
  if (!z || !ae || !ax ||
      bnet_forward(&B, n, rowptr, col, bval, bdiag, edge_r, alpha, theta) != 0)
    goto out;
  /* z = M^-1 b - x* */
  bsys_mul(n, rowptr, col, B.mo, B.md, b, z);
  for (int64_t i = 0; i < 3 * n; ++i) z[i] -= xstar[i];
  if (euclid) {
    memcpy(ae, z, sizeof(double) * 3 * (size_t)n);
    memcpy(ax, xstar, sizeof(double) * 3 * (size_t)n);
  } else {
    bsys_mul(n, rowptr, col, bval, bdiag, z, ae);
    bsys_mul(n, rowptr, col, bval, bdiag, xstar, ax);
  }
  {
    double num = 0.0, den = 0.0;
    for (int64_t i = 0; i < 3 * n; ++i) {
      num += z[i] * ae[i];
      den += xstar[i] * ax[i];
    }
    loss = num / den;
    if (!grad) goto out;
    for (int k = 0; k < NPARAMS + NPHI; ++k) grad[k] = 0.0;
    const net_t* t = &B.t;
    const double* hd = t->th + OFF_HEAD;
    const double* ph = B.phi;
    double* gh = grad + OFF_HEAD;
    double* gp = grad + NPARAMS;
    const double* hf = t->hs + (int64_t)NL * n * H;
    double* dh = (double*)calloc((size_t)(n * H + 1), sizeof(double));
    double* dm = (double*)calloc((size_t)(n * H + 1), sizeof(double));
    double* da = (double*)calloc((size_t)(n * H + 1), sizeof(double));
    if (!dh || !dm || !da) {
      free(dh); free(dm); free(da);
      loss = NAN;
      goto out;
    }
    for (int64_t i = 0; i < n; ++i) {
      const double* Ri = B.rt + 9 * i;
      const double di = B.diag[i];
      double gi[3];
      for (int c = 0; c < 3; ++c) gi[c] = 2.0 * ae[3 * i + c] / den;
      /* node block */
      double dM[9], dX[9];
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) dM[3 * r + c] = gi[r] * b[3 * i + c];
      mul33(Ri, dM, Ri, dX);
      double dlam = 0.0, dmu = 0.0;
      for (int m = 0; m < 9; ++m) {
        const double id = m % 4 == 0 ? 1.0 : 0.0;
        dlam += dX[m] * id;
        dmu += dX[m] * (di * B.binv[9 * i + m] - id);
      }
      const double gt = dlam * sigm(t->tau[i]);
      gh[H_V0] += gt;
      gp[PHI_U0] += dmu;
      for (int k = 0; k < H; ++k) {
        gh[H_V + k] += gt * hf[i * H + k];
        gp[PHI_U + k] += dmu * hf[i * H + k];
        dh[i * H + k] += gt * hd[H_V + k] + dmu * ph[PHI_U + k];
      }
      /* edge blocks: each directed entry evaluates its own S_ij and sig_ij */
      for (int64_t q = rowptr[i]; q < rowptr[i + 1]; ++q) {
        const int64_t j = col[q];
        for (int r = 0; r < 3; ++r)
          for (int c = 0; c < 3; ++c) dM[3 * r + c] = gi[r] * b[3 * j + c];
        mul33(Ri, dM, B.rt + 9 * j, dX);
        const double what = t->what[q];
        double dS = 0.0, dsg = 0.0;
        for (int m = 0; m < 9; ++m) {
          const double id = m % 4 == 0 ? 1.0 : 0.0;
          dS += dX[m] * id;
          dsg += dX[m] * (B.nh[9 * q + m] - what * id);
        }
        gh[H_Z0] += dS;
        gp[PHI_S0] += dsg;
        for (int f = 0; f < FE; ++f) {
          gh[H_ZE + f] += dS * t->e[FE * q + f];
          gp[PHI_SE + f] += dsg * t->e[FE * q + f];
        }
        for (int k = 0; k < H; ++k) {
          gh[H_Z + k] += dS * (hf[i * H + k] * hf[j * H + k]);
          gp[PHI_S + k] += dsg * (hf[i * H + k] * hf[j * H + k]);
          const double wk = dS * hd[H_Z + k] + dsg * ph[PHI_S + k];
          dh[i * H + k] += wk * hf[j * H + k];
          dh[j * H + k] += wk * hf[i * H + k];
        }
      }
    }
    net_trunk_backward(t, dh, dm, da, grad);
    free(dh); free(dm); free(da);
  }
out:
  free(z); free(ae); free(ax);
  bnet_free(&B);
  return loss;
}
