/*
 * oracle.h -- plain FP64 CPU oracle for one time step of the sheared
 * mesoscale blob simulation (Korolkovas, "Giant fluctuations in sheared
 * viscoelastic fluids emerging in a mesoscale simulation", arXiv 1808.06381).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path includes, links or
 * calls this code: only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark load it.  It shares no code, header, table or helper
 * with the GPU library; the two are written independently and agree only
 * because both follow the paper.
 *
 * Conventions (all arrays row-major, particles in ORIGINAL id order):
 *   pos, vel, rhs:  n x 3 doubles (x, y, z) per particle
 *   pairs:          unordered pairs {i, j} with i < j, sorted by (i, j)
 *   A:              A = gamma0*I + alpha*L(w), L the weighted graph Laplacian
 *                   (Method section, Eq. 9 with the pair strength alpha of
 *                   Eq. 7 made explicit); stored as CSR of the off-diagonal
 *                   part (both directions, columns ascending) plus diag[n].
 *   The 3n x 3n system of Eq. 7 is A (x) I_3: the friction acts on the full
 *   relative velocity vector, so x, y and z are three solves with one A.
 */
#ifndef ORACLE_H
#define ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum { ORC_W_GAUSS = 0, ORC_W_POLY2 = 1 };
enum { ORC_U_GAUSS_CORE = 0, ORC_U_SOFT = 1, ORC_U_NONE = 2 };
enum { ORC_NOISE_FDT = 0, ORC_NOISE_PAPER = 1, ORC_NOISE_OFF = 2 };
enum { ORC_PC_JACOBI = 0, ORC_PC_NONE = 1, ORC_PC_IC0 = 2, ORC_PC_GIVEN = 3 };

typedef struct orc_params {
  int64_t n;            /* particles */
  double box[3];        /* Lx, Ly, Lz; shear flow along x, gradient along y */
  double kT;            /* temperature (energy unit) */
  double gamma0;        /* background friction (zeta of Eq. 6a/6c/7) */
  double alpha;         /* pair-friction strength (alpha of Eq. 7) */
  double shear_rate;    /* kappa of Eq. 6c and Eq. 8 */
  double dt;            /* time step */
  double rc;            /* pair cut-off: a pair interacts iff r^2 < rc^2 */
  double lambda;        /* Gaussian width (weight law 0 and core potential 0) */
  double u_amp;         /* potential amplitude: v/lambda^3 (core) or epsilon (soft) */
  int32_t weight_law;   /* ORC_W_* */
  int32_t potential;    /* ORC_U_* */
  int32_t noise_mode;   /* ORC_NOISE_* */
  int32_t pad0;
  uint64_t seed;        /* Philox key word 0 */
  uint64_t stream;      /* Philox key word 1 (replica id) */
} orc_params;

/* ---- random numbers (counter-based; Salmon et al., SC'11) ---------------- */
void orc_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);
/* four standard normals from one Philox block, counter (step, tag, a, b) */
void orc_gauss4(const orc_params* p, uint64_t step, uint64_t tag, uint64_t a,
                uint64_t b, double g[4]);

/* ---- geometry ------------------------------------------------------------- */
double orc_le_offset(const orc_params* p, int64_t step);
int orc_separation(const orc_params* p, double delta, const double* ri,
                   const double* rj, double d[3]);
int64_t orc_pairs_brute(const orc_params* p, double delta, const double* pos,
                        int64_t cap, int64_t* pairs);
int64_t orc_pairs_cells(const orc_params* p, double delta, const double* pos,
                        int64_t cap, int64_t* pairs);

/* ---- velocity cross-correlation (vv.c) ------------------------------------- */
/* Pairs with r < r_max binned by r into nbins equal bins; per bin the sum of
 * u_i . u_j and the pair count over unordered pairs, and u2 = sum |u|^2;
 * u = v, or v minus the Couette flow when `flow` is set.  use_cells picks
 * the cell-list pair search (same set as brute force).  Returns 0, -1 for
 * bad arguments, -2 when out of memory.                                     */
int orc_velocity_correlation(const orc_params* p, double delta, const double* pos,
                             const double* vel, double r_max, int32_t nbins, int32_t flow,
                             int32_t use_cells, double* sum, int64_t* count, double* u2);

/* pair weight w(r^2) and conservative force F_ij on i (used by block.c) */
double orc_weight(const orc_params* p, double r2);
void orc_pair_force(const orc_params* p, const double d[3], double r2, double f[3]);

/* ---- anisotropic pair friction (block.c) ----------------------------------- */
/* Pair friction tensor W_ij = alpha w_ij (a_perp I + (a_par - a_perp) P_ij),
 * P_ij = d d^T / r^2 (0 at r = 0): friction a_par along the line of centres,
 * a_perp across it; a_par = a_perp = 1 is the isotropic system A (x) I_3.
 * The 3n x 3n system: A_ii = gamma0 I + sum_j W_ij, A_ij = -W_ij (3 x 3
 * blocks, 9 doubles row-major per entry / per row), rhs as orc_build_system
 * with the boundary drag W_ij V_ij and, in FDT mode, the pair noise
 * sqrt(2kT/dt) sigma_ij W_ij^(1/2) eta_ij, W^(1/2) = sqrt(alpha w)
 * (sqrt(a_perp) I + (sqrt(a_par) - sqrt(a_perp)) P).  Returns the entries
 * (2 x pairs) or -1.                                                       */
int64_t orc_build_block_system(const orc_params* p, double a_par, double a_perp, int64_t step,
                               const double* pos, int64_t cap, int64_t* rowptr, int64_t* col,
                               double* bval, double* bdiag, double* rhs);
/* plain CG (Jacobi on the scalar diagonal) on the 3n stacked unknowns;
 * stops when ||b - A x|| <= tol ||b|| (true residual).  0, -4 no convergence. */
int orc_block_pcg(int64_t n, const int64_t* rowptr, const int64_t* col, const double* bval,
                  const double* bdiag, const double* rhs, double* x, double tol, int maxit,
                  int* iters);
/* one step with the block system: build, solve to tol, R += v dt, wrap */
int orc_step_block(const orc_params* p, double a_par, double a_perp, int64_t step, double* pos,
                   double* vel, double tol, int maxit, int* iters);

/* ---- friction system ------------------------------------------------------ */
int64_t orc_count_pairs(const orc_params* p, int64_t step, const double* pos);
int64_t orc_build_system(const orc_params* p, int64_t step, const double* pos,
                         const double* xi, const double* eta, int64_t cap,
                         int64_t* rowptr, int64_t* col, double* val,
                         double* diag, double* rhs, double* fcons);

/* ---- threads --------------------------------------------------------------- */
/* OpenMP threads of the row-parallel loops (CPU timing only; results do not
   depend on it); orc_get_threads reports the count in force */
void orc_set_threads(int n);
int orc_get_threads(void);

/* ---- linear solve ---------------------------------------------------------- */
void orc_spmv3(int64_t n, const int64_t* rowptr, const int64_t* col,
               const double* val, const double* diag, const double* x, double* y);
int orc_pcg(int64_t n, const int64_t* rowptr, const int64_t* col,
            const double* val, const double* diag, const double* rhs,
            double* x, double tol, int maxit, int precond,
            const int64_t* mrowptr, const int64_t* mcol, const double* mval,
            const double* mdiag, int iters[3], double relres[3]);

int64_t orc_ic0(int64_t n, const int64_t* rowptr, const int64_t* col, const double* val,
                const double* diag, int64_t cap, int64_t* lrow, int64_t* lcol, double* lval);

/* ---- time step ------------------------------------------------------------- */
int orc_step(const orc_params* p, int64_t step, double* pos, double* vel,
             double tol, int maxit, int precond, int iters[3]);
void orc_wrap(const orc_params* p, int64_t step_after, double* pos);

/* ---- learned preconditioner (mpnn.c) --------------------------------------- */
int64_t orc_mpnn_nparams(void);
double orc_bf16(float f);
void orc_mpnn_set_bf16(int on);
int orc_mpnn_forward(int64_t n, const int64_t* rowptr, const int64_t* col, const double* val,
                     const double* diag, const double* edge_r, double alpha, const float* theta,
                     double* mdiag, double* moff);
double orc_mpnn_loss_grad_norm(int64_t n, const int64_t* rowptr, const int64_t* col,
                               const double* val, const double* diag, const double* edge_r,
                               double alpha, const float* theta, const double* b,
                               const double* xstar, int euclid, double* grad);
double orc_mpnn_loss_grad(int64_t n, const int64_t* rowptr, const int64_t* col, const double* val,
                          const double* diag, const double* edge_r, double alpha,
                          const float* theta, const double* b, const double* xstar, double* grad);
/* the same network with 3 x 3 heads on the anisotropic block system
 * (block.c layout, original order): M^-1 blocks row-major, mdiag n x 9,
 * moff nnz x 9; theta holds orc_mpnn_block_nparams() values (the scalar
 * network's, then the anisotropy heads u[32], u0, s[32], se[3], s0) */
int64_t orc_mpnn_block_nparams(void);
int orc_mpnn_block_forward(int64_t n, const int64_t* rowptr, const int64_t* col,
                           const double* bval, const double* bdiag, const double* edge_r,
                           double alpha, const float* theta, double* mdiag, double* moff);
double orc_mpnn_block_loss_grad(int64_t n, const int64_t* rowptr, const int64_t* col,
                                const double* bval, const double* bdiag, const double* edge_r,
                                double alpha, const float* theta, const double* b,
                                const double* xstar, int euclid, double* grad);

#ifdef __cplusplus
}
#endif
#endif
