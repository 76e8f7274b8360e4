/* A caller of libsim.so through the C ABI alone (include/sim.h): create a
 * box, step it, read the state back, solve A v = b for a given b, and check
 * properties that hold whatever the data:
 *   - every position stays inside the box, the step counter advances;
 *   - 1^T A = gamma0 1^T (the pair part of A has zero column sums), so the
 *     solution of A v = b has sum_i v_i = sum_i b_i / gamma0 per component,
 *     to the solve's tolerance;
 *   - invalid parameters are rejected with SIM_EINVAL and a message;
 *   - step graphs, S(q) (S(0) = N), the velocity correlation, a batch of two
 *     replicas, and anisotropic friction (the same sum rule) run cleanly.
 * Exit status 0 and "c abi ok" on success.                                 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "sim.h"

#define N 1000

static int fail(const char* what, int rc) {
  printf("FAIL %s: %d (%s)\n", what, rc, sim_strerror(rc));
  return 1;
}

int main(void) {
  static double pos[3 * N], vel[3 * N], b[3 * N], v[3 * N];
  uint64_t s = 88172645463325252ull;  /* xorshift64 (Marsaglia 2003) */
  for (int i = 0; i < 3 * N; ++i) {
    s ^= s << 13;
    s ^= s >> 7;
    s ^= s << 17;
    pos[i] = 10.0 * (double)(s >> 11) / 9007199254740992.0;
  }
  sim_params p;
  memset(&p, 0, sizeof(p));
  p.n = N;
  p.box[0] = p.box[1] = p.box[2] = 10.0;
  p.kT = 1.0;
  p.gamma0 = 0.1;
  p.alpha = 1.0;
  p.shear_rate = 0.05;
  p.dt = 0.01;
  p.rc = 1.0;
  p.lambda = 1.0;
  p.u_amp = 1.0;
  p.weight_law = SIM_W_POLY2;
  p.potential = SIM_U_SOFT;
  p.noise_mode = SIM_NOISE_FDT;
  p.precond = SIM_PC_JACOBI;
  p.cg_tol = 1e-10;
  p.cg_maxit = 10000;
  p.seed = 1;

  sim_params bad = p;
  bad.gamma0 = 0.0;
  sim_t* h = NULL;
  int rc = sim_create(&bad, pos, &h);
  if (rc != SIM_EINVAL || h) return fail("gamma0 = 0 not rejected", rc);

  rc = sim_create(&p, pos, &h);
  if (rc) return fail("sim_create", rc);
  sim_stats st;
  rc = sim_step(h, 5, &st);
  if (rc) return fail("sim_step", rc);
  sim_meta meta;
  rc = sim_state(h, pos, vel, &meta, 0);
  if (rc) return fail("sim_state", rc);
  if (meta.step != 5 || meta.n_total != N) return fail("meta", (int)meta.step);
  for (int i = 0; i < 3 * N; ++i)
    if (!(pos[i] >= 0.0 && pos[i] <= 10.0)) return fail("position outside the box", i);

  for (int i = 0; i < 3 * N; ++i) b[i] = sin(0.37 * i) + 0.25;
  rc = sim_solve(h, b, v, 1e-12, 0, &st);
  if (rc) return fail("sim_solve", rc);
  for (int k = 0; k < 3; ++k) {
    double sv = 0.0, sb = 0.0, nb = 0.0;
    for (int i = 0; i < N; ++i) {
      sv += v[3 * i + k];
      sb += b[3 * i + k];
      nb += fabs(b[3 * i + k]);
    }
    /* |1^T (A v - b)| <= sqrt(n) ||A v - b|| <= sqrt(n) tol ||b||, plus rounding */
    const double err = fabs(p.gamma0 * sv - sb);
    if (err > 1e-9 * nb) return fail("sum_i v_i != sum_i b_i / gamma0", k);
  }
  /* step graphs, the structure factor (S(0) = N exactly) and the velocity
   * correlation of the last step (pairs exist, finite sums) */
  rc = sim_graph_mode(h, 1);
  if (rc) return fail("sim_graph_mode", rc);
  rc = sim_step(h, 4, &st);
  if (rc) return fail("sim_step (graphs)", rc);
  static double sq[8 * 9];
  rc = sim_structure_factor(h, 8, 4, 0, sq, NULL);
  if (rc) return fail("sim_structure_factor", rc);
  if (fabs(sq[4] - (double)N) > 1e-9 * N) return fail("S(0) != N", 0);
  double vs[20], vu2;
  int64_t vc[20];
  rc = sim_velocity_correlation(h, 3.0, 20, 1, vs, vc, &vu2, NULL);
  if (rc) return fail("sim_velocity_correlation", rc);
  int64_t pairs = 0;
  for (int k = 0; k < 20; ++k) {
    pairs += vc[k];
    if (!isfinite(vs[k])) return fail("velocity correlation not finite", k);
  }
  if (pairs <= 0 || !(vu2 > 0.0)) return fail("velocity correlation empty", (int)pairs);
  sim_destroy(h);

  /* two replicas in one handle, then anisotropic friction: the uniform
   * translation is still an eigenvector of A with eigenvalue gamma0 */
  sim_params pr[2] = {p, p};
  pr[1].shear_rate = 0.5;
  pr[1].stream = 1;
  static double pos2[6 * N];
  memcpy(pos2, pos, sizeof(double) * 3 * N);
  memcpy(pos2 + 3 * N, pos, sizeof(double) * 3 * N);
  rc = sim_create_batch(pr, 2, pos2, &h);
  if (rc) return fail("sim_create_batch", rc);
  rc = sim_step(h, 2, &st);
  if (rc) return fail("sim_step (batch)", rc);
  sim_destroy(h);
  sim_params pa = p;
  pa.friction_par = 3.0;
  pa.friction_perp = 0.5;
  rc = sim_create(&pa, pos, &h);
  if (rc) return fail("sim_create (anisotropic)", rc);
  rc = sim_step(h, 2, &st);
  if (rc) return fail("sim_step (anisotropic)", rc);
  rc = sim_solve(h, b, v, 1e-12, 0, &st);
  if (rc) return fail("sim_solve (anisotropic)", rc);
  for (int k = 0; k < 3; ++k) {
    double sv = 0.0, sb = 0.0, nb = 0.0;
    for (int i = 0; i < N; ++i) {
      sv += v[3 * i + k];
      sb += b[3 * i + k];
      nb += fabs(b[3 * i + k]);
    }
    if (fabs(p.gamma0 * sv - sb) > 1e-9 * nb) return fail("anisotropic: sum v != sum b / gamma0", k);
  }
  sim_destroy(h);
  printf("c abi ok: %d steps, last solve %d iterations\n", (int)meta.step, st.iters[0]);
  return 0;
}
