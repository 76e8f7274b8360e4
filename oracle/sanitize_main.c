/*
 * sanitize_main.c -- runs every oracle entry point once on small inputs, to
 * be built with AddressSanitizer and UndefinedBehaviorSanitizer (gcc, host
 * code only): a memory or undefined-behaviour error anywhere in the oracle
 * aborts the run.  TEST INFRASTRUCTURE ONLY.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "oracle.h"

static uint64_t st = 0x9E3779B97F4A7C15ull;
static double uni(void) { /* xorshift64 */
  st ^= st << 13; st ^= st >> 7; st ^= st << 17;
  return (double)(st >> 11) / 9007199254740992.0;
}

static void check(int ok, const char* what) {
  if (!ok) {
    printf("FAIL %s\n", what);
    exit(1);
  }
}

int main(void) {
  const int64_t n = 600;
  orc_params p;
  memset(&p, 0, sizeof(p));
  p.n = n;
  p.box[0] = 9.0; p.box[1] = 8.0; p.box[2] = 8.5;
  p.kT = 1.0; p.gamma0 = 0.1; p.alpha = 1.0; p.shear_rate = 0.4; p.dt = 0.01;
  p.rc = 1.0; p.lambda = 1.0; p.u_amp = 1.0;
  p.weight_law = ORC_W_POLY2; p.potential = ORC_U_SOFT; p.noise_mode = ORC_NOISE_FDT;
  p.seed = 3;
  double* pos = malloc(sizeof(double) * 3 * n);
  double* vel = malloc(sizeof(double) * 3 * n);
  for (int64_t i = 0; i < n; ++i)
    for (int k = 0; k < 3; ++k) pos[3 * i + k] = p.box[k] * uni();
  const double delta = orc_le_offset(&p, 7);
  /* pairs, both searches */
  const int64_t m = orc_pairs_brute(&p, delta, pos, 0, NULL);
  int64_t* pa = malloc(sizeof(int64_t) * 2 * (m + 1));
  int64_t* pb = malloc(sizeof(int64_t) * 2 * (m + 1));
  check(orc_pairs_brute(&p, delta, pos, m, pa) == m, "pairs brute");
  check(orc_pairs_cells(&p, delta, pos, m, pb) == m, "pairs cells");
  check(memcmp(pa, pb, sizeof(int64_t) * 2 * m) == 0, "pairs equal");
  /* system, solves, IC(0) */
  const int64_t np = orc_count_pairs(&p, 7, pos);
  const int64_t cap = 2 * np + 1;
  int64_t* rowptr = malloc(sizeof(int64_t) * (n + 1));
  int64_t* col = malloc(sizeof(int64_t) * cap);
  double* val = malloc(sizeof(double) * cap);
  double* diag = malloc(sizeof(double) * n);
  double* rhs = malloc(sizeof(double) * 3 * n);
  double* fcons = malloc(sizeof(double) * 3 * n);
  check(orc_build_system(&p, 7, pos, NULL, NULL, cap, rowptr, col, val, diag, rhs, fcons) == 2 * np,
        "build system");
  int iters[3];
  double relres[3];
  for (int pc = 0; pc <= 2; ++pc) {
    check(orc_pcg(n, rowptr, col, val, diag, rhs, vel, 1e-10, 5000, pc, NULL, NULL, NULL, NULL,
                  iters, relres) == 0, "pcg");
  }
  int64_t* lrow = malloc(sizeof(int64_t) * (n + 1));
  int64_t* lcol = malloc(sizeof(int64_t) * (np + n));
  double* lval = malloc(sizeof(double) * (np + n));
  check(orc_ic0(n, rowptr, col, val, diag, np + n, lrow, lcol, lval) > 0, "ic0");
  /* learned preconditioner: forward, loss and gradient */
  const int64_t nw = orc_mpnn_nparams();
  float* theta = malloc(sizeof(float) * nw);
  double* grad = malloc(sizeof(double) * nw);
  for (int64_t k = 0; k < nw; ++k) theta[k] = (float)(0.2 * (uni() - 0.5));
  double* er = malloc(sizeof(double) * cap);
  for (int64_t e = 0; e < 2 * np; ++e) er[e] = uni();
  double* mdiag = malloc(sizeof(double) * n);
  double* moff = malloc(sizeof(double) * cap);
  check(orc_mpnn_forward(n, rowptr, col, val, diag, er, p.alpha, theta, mdiag, moff) == 0,
        "mpnn forward");
  const double l1 = orc_mpnn_loss_grad(n, rowptr, col, val, diag, er, p.alpha, theta, rhs, vel, grad);
  const double l2 = orc_mpnn_loss_grad_norm(n, rowptr, col, val, diag, er, p.alpha, theta, rhs, vel,
                                            1, grad);
  check(isfinite(l1) && isfinite(l2), "mpnn loss");
  /* steps, velocity correlation, anisotropic friction */
  check(orc_step(&p, 7, pos, vel, 1e-10, 5000, 0, iters) == 0, "step");
  double sum[12], u2;
  int64_t cnt[12];
  check(orc_velocity_correlation(&p, delta, pos, vel, 3.0, 12, 1, 0, sum, cnt, &u2) == 0, "vv brute");
  check(orc_velocity_correlation(&p, delta, pos, vel, 3.0, 12, 1, 1, sum, cnt, &u2) == 0, "vv cells");
  int bit;
  check(orc_step_block(&p, 2.5, 0.4, 8, pos, vel, 1e-10, 5000, &bit) == 0, "block step");
  printf("oracle sanitized run ok (%lld pairs)\n", (long long)m);
  free(pos); free(vel); free(pa); free(pb); free(rowptr); free(col); free(val); free(diag);
  free(rhs); free(fcons); free(lrow); free(lcol); free(lval); free(theta); free(grad); free(er);
  free(mdiag); free(moff);
  return 0;
}
