/*
 * sim.h -- C ABI of libsim, the MI355X (gfx950) implementation of the time
 * step of the sheared mesoscale blob simulation of Korolkovas,
 * arXiv 1808.06381 (Method section).
 *
 * One step advances every particle c by R_c += v_c*dt, where the velocities
 * solve the coupled overdamped equation of motion (Eq. 7), rewritten as the
 * sparse linear system of Eq. 9:
 *
 *     (gamma0*I + alpha*L(w)) v = F + gamma0*kappa*(y - Ly/2) x
 *                                   + alpha*sum_c' w_cc' V_cc' + f_thermal
 *
 * L(w) is the weighted graph Laplacian of the pairs closer than rc (weights
 * below the threshold dropped, Method section), V_cc' the Lees-Edwards
 * boundary velocity of Eq. 8, F the conservative pair force (Eq. 6b), and
 * gamma0*kappa*(y - Ly/2) the Couette drive (Eq. 6c).  The friction acts on
 * the full relative velocity vector, so the 3N x 3N system is A (x) I_3 and
 * the library solves three right-hand sides against one scalar matrix A.
 *
 * Conventions of every entry point:
 *  - Arrays are row-major n x 3 doubles (x, y, z per particle) in ORIGINAL
 *    particle id order, for a batch the replicas one after another.
 *  - Pointers are host pointers unless a flags argument carries
 *    SIM_DEVICE_PTR; then they are device pointers on the library's device.
 *  - The caller owns every buffer it passes; the library copies inputs and
 *    writes outputs, and owns all device memory behind a handle.
 *  - Every call returns SIM_OK (0) or a negative error code; sim_strerror
 *    names it.  A failed sim_step leaves the state at the last committed step.
 *  - Calls on one handle must not overlap; different handles are independent.
 */
#ifndef SIM_H
#define SIM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- error codes --------------------------------------------------------- */
#define SIM_OK 0
#define SIM_EINVAL -1      /* invalid argument or parameter (see sim_create) */
#define SIM_ENOMEM -2      /* host or device allocation failed */
#define SIM_EDEVICE -3     /* a HIP runtime call failed */
#define SIM_ENOCONV -4     /* CG hit cg_maxit: the step is not committed */
#define SIM_EBREAKDOWN -5  /* CG breakdown (p.Ap <= 0) with a plain preconditioner */
#define SIM_ECAPACITY -6   /* an output buffer given by the caller is too small */
#define SIM_ENUMERIC -7    /* a position became non-finite: step not committed */
#define SIM_ENOTSUP -8     /* option not available in this build */

/* ---- flags --------------------------------------------------------------- */
#define SIM_DEVICE_PTR 1u  /* array arguments are device pointers */

/* ---- enumerations -------------------------------------------------------- */
enum sim_weight_law { SIM_W_GAUSS = 0, SIM_W_POLY2 = 1 };
enum sim_potential { SIM_U_GAUSS_CORE = 0, SIM_U_SOFT = 1, SIM_U_NONE = 2 };
enum sim_noise { SIM_NOISE_FDT = 0, SIM_NOISE_PAPER = 1, SIM_NOISE_OFF = 2 };
enum sim_precond { SIM_PC_JACOBI = 0, SIM_PC_NONE = 1, SIM_PC_IC0 = 2, SIM_PC_LEARNED = 3 };

/* Physical and solver parameters of one box (one replica).
 *  n           particles, >= 1
 *  box         Lx, Ly, Lz > 0: flow along x, velocity gradient along y,
 *              Lees-Edwards images along y, periodic in x and z
 *  kT          temperature >= 0 (the thermal force of Eq. 6a scales with it)
 *  gamma0      background friction > 0 (zeta of Eq. 6 and 7); it is the
 *              smallest eigenvalue of A, so it must be positive
 *  alpha       pair-friction strength >= 0 (alpha of Eq. 7)
 *  shear_rate  kappa of Eq. 6c and Eq. 8 (any sign)
 *  dt          time step > 0
 *  rc          pair cut-off, 0 < rc < min(L)/2: a pair interacts iff r < rc
 *  lambda      Gaussian width > 0 for SIM_W_GAUSS / SIM_U_GAUSS_CORE
 *  u_amp       potential amplitude: v/lambda^3 of Eq. 6b (Gaussian core,
 *              force (kT*u_amp/lambda^2) d exp(-r^2/2lambda^2)) or epsilon of
 *              U = epsilon*(1 - r/rc)^2 (soft)
 *  weight_law  pair friction envelope w(r): exp(-r^2/(2 lambda^2)) (paper)
 *              or (1 - r/rc)^2
 *  noise_mode  SIM_NOISE_FDT: f_i = sqrt(2kT/dt)*(sqrt(gamma0)*xi_i
 *              + sum_j sigma_ij*sqrt(alpha*w_ij)*eta_ij), covariance
 *              (2kT/dt)*A; SIM_NOISE_PAPER: sqrt(2*gamma0*kT/dt)*xi_i only
 *              (Eq. 6a); SIM_NOISE_OFF.  Gaussians come from Philox4x64-10
 *              keyed (seed, stream) with counter (step, 0, id, 0) for xi and
 *              (step, 1, min id, max id) for eta, via Box-Muller.
 *  precond     CG preconditioner, the same for every replica:
 *              SIM_PC_JACOBI (u = D^-1 r), SIM_PC_NONE (u = r),
 *              SIM_PC_IC0 (incomplete Cholesky with A's lower pattern in
 *              multicolour order: cells coloured by the parity of their
 *              coordinates -- a third colour for the last cell of an odd
 *              axis -- rows ordered by (colour, cell, particle id); exact
 *              IC(0) of that ordering, Meijerink & van der Vorst 1977),
 *              SIM_PC_LEARNED (see below; needs alpha > 0)
 *  spmv_fp32   0: FP64 matrix values; 1: FP32 matrix values in the CG
 *              matrix products with FP64 vectors, dots and true-residual
 *              recompute (agreement with FP64 about 1e-5 relative)
 *  warm_start  0: every solve of sim_step starts from v = 0; 1: from the
 *              previous step's velocities (zero before the first step), a
 *              restart whose answer differs from the cold start's only
 *              within cg_tol; sim_solve always starts from 0.  The same
 *              value for every replica of a batch.
 *  cg_maxit    iteration limit per solve (> 0)
 *  cg_tol      stop when ||b_k - A v_k||_2 <= cg_tol*||b_k||_2 for each
 *              component k (true residual, checked at exit)
 *  seed,stream Philox key */
typedef struct sim_params {
  int64_t n;
  double box[3];
  double kT;
  double gamma0;
  double alpha;
  double shear_rate;
  double dt;
  double rc;
  double lambda;
  double u_amp;
  int32_t weight_law;
  int32_t potential;
  int32_t noise_mode;
  int32_t precond;
  int32_t spmv_fp32;
  int32_t warm_start;
  int32_t cg_maxit;
  int32_t reserved0;
  double cg_tol;
  uint64_t seed;
  uint64_t stream;
  /* Anisotropic pair friction (the paper's elongated-particle remedy,
   * Discussion): the pair coefficient of Eq. 7 becomes the tensor
   * W_ij = alpha w_ij (friction_perp I + (friction_par - friction_perp)
   * d d^T / r^2), friction_par along the line of centres and friction_perp
   * across it, so A has 3 x 3 blocks and the pair noise is
   * sqrt(2kT/dt) W^(1/2) eta.  0 stands for 1; both 1 (or 0) is the
   * isotropic method.  When any replica has a value other than 1 the handle
   * solves the block system: block-Jacobi CG over the 3n coupled unknowns,
   * one true-residual tolerance per replica on the stacked vector; steps run
   * eagerly (no step graphs); precond must be Jacobi, none or learned (the
   * 3 x 3 heads below), else SIM_ENOTSUP; spmv_fp32 = 1 rounds the six
   * values of every off-diagonal block to FP32 for the iteration products
   * (diagonal blocks, residual rounds in FP64); warm_start = 1 starts each
   * step's solve from the previous step's velocities, as for the scalar
   * system.                                                                 */
  double friction_par;
  double friction_perp;
} sim_params;

/* Statistics of the last sim_step / sim_solve call (max over replicas). */
typedef struct sim_stats {
  int32_t iters[3];      /* CG iterations per component of the last solve */
  int32_t restarts;      /* true-residual restarts in the last solve */
  double relres[3];      /* true relative residual per component at exit */
  int64_t nnz;           /* off-diagonal entries of A (= 2 x pairs), all replicas */
  int32_t max_row;       /* longest off-diagonal row */
  int32_t fallback;      /* 1 if a learned solve fell back to Jacobi */
  int64_t steps_done;    /* steps committed by the call */
  int64_t cg_iters_total;/* sum over the call's solves of max-component iterations */
} sim_stats;

/* Metadata returned by sim_state. */
typedef struct sim_meta {
  int64_t step;          /* committed steps since creation */
  double time;           /* step * dt of replica 0 */
  double le_offset;      /* Lees-Edwards offset of replica 0 at `step` */
  int32_t replicas;
  int32_t reserved0;
  int64_t n_total;       /* particles over all replicas */
} sim_meta;

typedef struct sim_t sim_t;

/* Create a single-box simulation (Method section: particles R_c, parameters
 * of Eq. 6-9).  pos0: n x 3 initial positions, each in [0, L] per axis.
 * Validates: n >= 1, box > 0, gamma0 > 0 (A = gamma0*I + alpha*L is then
 * SPD), alpha >= 0, kT >= 0, dt > 0, 0 < rc < min(box)/2, lambda > 0 where
 * used, cg_tol > 0, cg_maxit > 0, enum ranges, finite positions inside the
 * box; else SIM_EINVAL.  Copies pos0; *out receives the handle.           */
int sim_create(const sim_params* params, const double* pos0, sim_t** out);

/* Create R independent boxes advanced together (a block-diagonal system;
 * each replica has its own n, box, shear rate and key).  pos0_concat holds
 * the replicas' n_r x 3 blocks one after another.  Same validation.       */
int sim_create_batch(const sim_params* params, int32_t replicas, const double* pos0_concat,
                     sim_t** out);

/* Advance every replica by nsteps steps (Eq. 7 integrated as R += v dt with
 * Lees-Edwards re-entry).  Each step: cell binning, neighbour search under
 * the Lees-Edwards minimum image, pair terms, assembly of A and b, PCG solve
 * to cg_tol (x0 = 0), position update.  Stops at the first failing step
 * (SIM_ENOCONV, SIM_EBREAKDOWN, SIM_ENUMERIC), which is not committed.
 * st (nullable) receives the statistics.                                 */
int sim_step(sim_t* sim, int32_t nsteps, sim_stats* st);

/* Solve A v = b for the matrix of the current positions and step (Eq. 9,
 * left-hand side), to tolerance tol (<= 0: the params' cg_tol) with the
 * params' preconditioner.  b, v: n_total x 3.  flags: SIM_DEVICE_PTR.
 * Does not change the state.                                              */
int sim_solve(sim_t* sim, const double* b, double* v, double tol, uint32_t flags,
              sim_stats* st);

/* Copy out positions and the velocities of the last committed step (zeros
 * before the first), n_total x 3 in original id order; any pointer may be
 * NULL.  flags: SIM_DEVICE_PTR for pos/vel.                               */
int sim_state(sim_t* sim, double* pos, double* vel, sim_meta* meta, uint32_t flags);

/* Structure factor of the blob centres (Results section, Eq. Sfactor) of
 * every replica at the current positions: S(q) = |sum_c exp(-i q.R_c)|^2 / C
 * for one configuration (averaging over configurations is the caller's),
 * on the wavevectors that the Lees-Edwards images of the box leave
 * invariant,
 *   q = (2 pi mx / Lx, 2 pi my / Ly - 2 pi mx delta / (Lx Ly), 2 pi mz / Lz)
 * with delta the current offset, for mx = 0 .. nx-1, my = -my_max ..
 * my_max and the given mz (S(-q) = S(q): mx >= 0 covers the plane).
 * out (host): replicas x nx x (2 my_max + 1) doubles, row-major.  FP64
 * throughout, deterministic.  kernel_ms (optional) receives the duration
 * of the contraction kernel, measured with HIP events bracketing its
 * launch.  1 <= nx <= 256, 0 <= my_max <= 128, |mz| <= 256, else
 * SIM_EINVAL.  Device scratch of the handle grows on demand.              */
int sim_structure_factor(sim_t* sim, int32_t nx, int32_t my_max, int32_t mz, double* out,
                         double* kernel_ms);

/* sim_structure_factor for callers that cannot allocate device memory
 * (code under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same kernels and the same result bits, with every
 * intermediate (chunk table, chunk offsets, partial sums) in one static
 * device array of SIM_NOALLOC_SCRATCH_MAX bytes that the library holds on
 * each GPU it runs on until the process ends.  out is a DEVICE pointer on
 * the handle's device: replicas x nx x (2 my_max + 1) doubles, row-major,
 * written by the call (the caller owns it).  The call allocates nothing and
 * copies nothing from the host; it returns after the result is written.
 * Every call on one GPU shares the one array, so calls that overlap on a GPU
 * (several host threads or streams) race and must be serialised by the
 * caller.  Arguments as sim_structure_factor (SIM_EINVAL); SIM_ECAPACITY
 * when the scratch would exceed SIM_NOALLOC_SCRATCH_MAX: it needs about
 * 1 KiB x W x ceil(N_r / 4096) summed over replicas x ceil(nx / 64) x
 * ceil(ny / W), ny = 2 my_max + 1, W = ny rounded up to a multiple of 16,
 * at most 160 (e.g. N = 10^6 with nx = 64, my_max = 64 uses 35 MiB).      */
#define SIM_NOALLOC_SCRATCH_MAX (48u << 20)
int sim_structure_factor_noalloc(sim_t* sim, int32_t nx, int32_t my_max, int32_t mz,
                                 double* out);

/* Velocity cross-correlation against separation (Results section: the
 * velocity correlation of two chains, normalised by the mean square
 * velocity, against |R_cc'|, longer-ranged as alpha grows), of every
 * replica's last committed step: the configuration R_n of that step and
 * the velocities v_n solved at it (sim_state reports R_{n+1} = R_n + v_n dt
 * and v_n).  With u = v_n, or with `flow` != 0 u = v_n - kappa (y - Ly/2) x
 * (relative to the imposed Couette flow of Eq. 6c, the same for every
 * Lees-Edwards image):
 *   sum[r][k]   = sum of u_i . u_j over unordered pairs of replica r in bin k
 *   count[r][k] = number of those pairs
 *   u2[r]       = sum_c |u_c|^2
 * Pairs: r^2 < r_max^2 under the Lees-Edwards minimum image of step n (the
 * neighbour search's separation, rounding included); bin k = the largest
 * integer with k^2 <= r^2 * (nbins^2 / r_max^2), capped at nbins - 1.  The
 * normalised correlation is (sum / count) / (u2 / n); sums and counts of
 * several calls add up for averages over configurations.
 * sum and u2 are FP64; each pair product is rounded to a fixed-point
 * integer of step 2^-S with S = 61 - ceil(log2(64 n_r)) - e_r, where
 * max_c |u_c|^2 < 2^e_r, and the integers are added exactly, so sum[r][k]
 * is within count * 2^-(S+1) (plus one rounding) of the exact pair sum and
 * is bitwise reproducible.  sum, count: replicas x nbins (host); u2:
 * replicas (host).  kernel_ms (optional) receives the duration of the pair
 * kernel.  SIM_EINVAL when no step has been committed since the handle was
 * created or since the last sim_solve / debug export (they overwrite the
 * step's buffers), for nbins outside 1..1024, r_max <= 0 or r_max larger
 * than half the smallest box side of any replica, or a replica of 2^26
 * particles or more.  Device scratch of the
 * handle grows on demand.                                                 */
int sim_velocity_correlation(sim_t* sim, double r_max, int32_t nbins, int32_t flow, double* sum,
                             int64_t* count, double* u2, double* kernel_ms);

/* Run the library's work on this HIP stream (hipStream_t as void*; NULL is
 * the default stream).  The caller keeps the stream alive.                 */
int sim_set_stream(sim_t* sim, void* hip_stream);

/* Load learned-preconditioner weights from a file: 8 bytes "SIMPC001", an
 * int64 count (SIM_MPNN_NPARAMS or SIM_MPNN_NPARAMS_BLOCK), then the FP32
 * weights, little-endian, set as sim_precond_weights sets them.
 * SIM_EINVAL for a malformed file.                                        */
int sim_load_precond(sim_t* sim, const char* path);

/* Parity export: the unordered pairs {i < j} (original ids, per replica)
 * of the current positions, as (replica, i, j) int64 triples in any order.
 * cap is the triple capacity of ijr; *count receives the number of pairs.
 * Returns SIM_ECAPACITY (with *count set) when cap is too small.          */
int sim_debug_pairs(sim_t* sim, int64_t* ijr, int64_t cap, int64_t* count);

/* Parity export of the system of the current positions and step, original
 * ids: off-diagonal entries as triples (row, col, value) with global row and
 * column numbers (replica offset + id), diag[n_total], rhs[n_total x 3]
 * (including the thermal force of this step).  Same capacity rule.        */
int sim_debug_system(sim_t* sim, int64_t* rows, int64_t* cols, double* vals, int64_t cap,
                     int64_t* count, double* diag, double* rhs);

/* The block system (handles with anisotropic friction) of the current
 * positions and step, in original ids: rows/cols (cap entries, *count set
 * to the number of off-diagonal blocks), vals (9 doubles per entry,
 * row-major -W_ij), diag (9 per particle, nullable), rhs (n_total x 3,
 * nullable); host pointers.  SIM_ENOTSUP on an isotropic handle,
 * SIM_ECAPACITY when cap is too small.  For parity tests.                  */
int sim_debug_block_system(sim_t* sim, int64_t* rows, int64_t* cols, double* vals, int64_t cap,
                           int64_t* count, double* diag, double* rhs);

/* Replace the generated Gaussians of the thermal force (testing only,
 * single-replica handles with n <= 1024): xi is n x 3 (particle i at row
 * i), eta is n x n x 3 with the Gaussian vector of the unordered pair
 * {a < b} at [(a*n + b)*3 + k].  Both NULL return to the generator.  The
 * library copies the tables; they apply to subsequent builds.
 * SIM_ENOTSUP for batches or larger n.                                    */
int sim_debug_set_gaussians(sim_t* sim, const double* xi, const double* eta);

/* ---- learned preconditioner (precond = SIM_PC_LEARNED) --------------------
 * A three-layer message-passing network on the pair graph of A (hidden 32)
 * maps node features (t_i, a_i, deg_i/8) and edge features (r_ij/rc, w_ij,
 * What_ij) to M^-1 = D^-1/2 (diag(lam) + S) D^-1/2 in A's sparsity, with
 * S_ij = z.(h_i*h_j) + ze.e_ij + z0 symmetric and lam_i = softplus(.) +
 * floor (sim_precond_floor, 0.3 unless set; D = diag A,
 * What_ij = alpha w_ij / sqrt(D_i D_j)).  M^-1 is symmetric
 * with a positive diagonal but positive definite only for suitable weights
 * (the best sparse approximate inverses of A are not diagonally dominant);
 * lam = 1, S = What is the two-term Neumann series of A^-1, which is.  It
 * replaces the Jacobi step u = D^-1 r of the CG solve of Eq. 9; the stopping
 * rule (true residual) is unchanged, so it changes iteration counts, not
 * answers.  A solve that stalls (residual not 10 % lower over 10 iterations
 * after 20) or breaks down -- what an indefinite M^-1 leads to -- is redone
 * with Jacobi and flagged in sim_stats.fallback.
 * The weights are SIM_MPNN_NPARAMS FP32 values (bfloat16 in the kernels),
 * in this order: W0[32][3], b0[32], then per layer P[32][32], Q[32][3],
 * c[32], U[32][32], V[32][32], d[32], then v[32], v0, z[32], ze[3], z0.
 * A new handle starts with all weights zero: S = 0, lam = ln 2 + floor, a
 * scaled Jacobi preconditioner.
 *
 * Anisotropic friction (the block system, friction_par / friction_perp;
 * Discussion): the same network runs on the traces of A's 3 x 3 blocks,
 * d_i = tr A_ii / 3 and omega_ij = tr W_ij / 3 (A_ij = -W_ij), in place of
 * (D_i, alpha w_ij), and two more heads, mu_i = u.h_i + u0 and
 * sig_ij = s.(h_i*h_j) + se.e_ij + s0, give 3 x 3 blocks in the frame
 * where every diagonal block of A is the identity, R = blockdiag(A_ii^-1/2)
 * (the block analogue of D^-1/2 above; symmetric roots):
 *   Xh_ii = lam_i I + mu_i (d_i A_ii^-1 - I),
 *   Xh_ij = S_ij I + sig_ij (R_i W_ij R_j - What_ij I),
 *   M^-1 = R Xh R,
 * stored block by block and applied as one more block product per CG
 * iteration.  M^-1 is symmetric, turns with the system under rotations, and
 * is the scalar network's times I_3 when every block of A is a multiple of
 * I_3; lam = 1, mu = 0, S = What, sig = 1 give D^-1 + D^-1 (D - A) D^-1,
 * D = blockdiag(A_ii), the two-term Neumann series of the block-Jacobi
 * splitting (positive definite).  Weights trained on the scalar system
 * carry over (in that frame their S_ij acts as on a scalar system).  A
 * stalled or broken-down solve is redone with block-Jacobi.  The weights are
 * SIM_MPNN_NPARAMS_BLOCK values: the SIM_MPNN_NPARAMS above, then u[32],
 * u0, s[32], se[3], s0.                                                    */
#define SIM_MPNN_NPARAMS 9893
#define SIM_MPNN_NPARAMS_BLOCK 9962
/* Copy the FP32 master weights in (set = 1) or out (set = 0): count =
 * SIM_MPNN_NPARAMS (the anisotropy heads, used by block handles only, keep
 * their values) or SIM_MPNN_NPARAMS_BLOCK.  Setting clears the Adam state. */
int sim_precond_weights(sim_t* sim, float* theta, int64_t count, int32_t set);
/* Activations entering the network's products are rounded to bfloat16
 * (round_act = 1, default) or kept in FP32 (0, for parity tests).
 * learned_maxit > 0 bounds the iterations of a learned-preconditioned
 * solve before it falls back to Jacobi (0: the params' cg_maxit).         */
int sim_precond_config(sim_t* sim, int32_t round_act, int32_t learned_maxit);
/* Floor added to the diagonal head: lam_i = softplus(v.h_i + v0) + lam_floor
 * (default 0.3, >= 0).  It adds lam_floor D^-1 to M^-1: a margin of positive
 * definiteness for the rare strongly coupled clusters where the trained
 * M^-1 is weak, at the price of a slightly weaker preconditioner elsewhere
 * (measured on pre-sheared boxes at shear 0.5: N = 8e6 32.2 / 29.3 / 28.6 /
 * 29.6 mean CG iterations at floors 0.1 / 0.2 / 0.3 / 0.5, N = 1e6 25.8 /
 * 25.9 / 26.5 / 27.8).                                                     */
int sim_precond_floor(sim_t* sim, double lam_floor);
/* One training step on the system of the last successful solve of this
 * single-box handle (A, b and its solution x* from sim_step or sim_solve):
 * network forward, loss L = ||M^-1 b - x*||_A^2 / ||x*||_A^2 (three
 * components), backward and one Adam step (beta 0.9 / 0.999) with learning
 * rate lr; lr = 0 evaluates the loss and gradient only.  *loss receives L
 * at the weights before the update.  SIM_EINVAL without a solved system,
 * or when that system was built before the first preconditioner call on
 * the handle (sim_precond_weights, sim_precond_config, sim_load_precond,
 * sim_precond_floor; a Jacobi handle writes the network's edge input only
 * from then on); SIM_ENOTSUP for batches.  Block handles train all
 * SIM_MPNN_NPARAMS_BLOCK weights on the block system (A-norm of A's blocks). */
int sim_train_step(sim_t* sim, double lr, double* loss);
/* One training step on a white-noise probe of the current system (any
 * number of replicas; needs a successful solve): x* = z with z_ik ~ N(0, 1)
 * (Philox4x64-10, key (seed, replica stream), counter (index, 3, particle
 * id, 0), Box-Muller as for the thermal force) and b = A z, so that
 * L = ||(M^-1 A - I) z||^2 / ||z||^2 (summed over components and replicas)
 * samples the Frobenius distance of M^-1 A from the identity, weighted by A
 * (euclid = 0) or unweighted (euclid = 1, which gives the smooth modes that
 * bound the CG convergence rate their full weight) -- every mode counts,
 * where the solution of Eq. 9 is dominated by smooth ones.  Otherwise as
 * sim_train_step; the solve's b and x are left as they were.              */
int sim_train_probe(sim_t* sim, double lr, uint64_t seed, uint64_t index, int32_t euclid,
                    double* loss);
/* Adam state of the training steps: first and second moments (count =
 * SIM_MPNN_NPARAMS or SIM_MPNN_NPARAMS_BLOCK each) and the step count t,
 * copied out (set = 0) or in (set = 1), so that training can move between
 * handles.  Setting weights with sim_precond_weights clears it.           */
int sim_precond_optimizer(sim_t* sim, float* m1, float* m2, int64_t count, int32_t* t,
                          int32_t set);
/* The gradient dL/dtheta of the last training step (with respect to the
 * bfloat16 weights), count = SIM_MPNN_NPARAMS or SIM_MPNN_NPARAMS_BLOCK
 * (zero beyond the weights the handle trains).                           */
int sim_precond_grad(sim_t* sim, float* grad, int64_t count);
/* Parity export of the preconditioner of the current positions and step.
 * Learned: M^-1 in the form of sim_debug_system (off-diagonal triples,
 * diagonal); block handles write 9 values per entry (the row-major 3 x 3
 * block M_ij) into vals and 9 per particle into mdiag.  IC(0): the strictly lower triangle of L (in the IC order) as
 * (row, col, L_row,col) triples at the positions of A's off-diagonal
 * entries, row = col = -1 in the slots of upper entries, and L's diagonal.
 * SIM_ENOTSUP for Jacobi and no preconditioner.                           */
int sim_debug_precond(sim_t* sim, int64_t* rows, int64_t* cols, double* vals, int64_t cap,
                      int64_t* count, double* mdiag);

/* Kernel timing probe (measurement, not part of the method).  With
 * sample_every > 0, later eager solves (with step graphs on, every
 * sample_every-th step runs eagerly) alternate two forms.  Kernel form:
 * every sample_every-th CG iteration has its three kernels (k_cg_vec,
 * k_cg_spmv, k_cg_apply) bracketed by HIP events on the library's stream
 * (the sampled residue of the iteration index advances by one per such
 * solve, so every position in a solve is sampled alike).  Iteration form
 * ("cg_iteration"): one event pair around the first chunk's iterations
 * except its last two -- every kernel, the finisher and the gaps between
 * launches -- counted as that many launches, each priced at the solve's
 * algorithmic bytes per iteration: 12(nnz + N) + 4N (the matrix: value 8 +
 * column 4 per entry, the diagonal as one more entry, a row pointer; 8
 * instead of 12 with FP32 values) + 200N (the CG vectors) for N particles
 * and nnz off-diagonal entries, plus 12(nnz + N) + 4N for the learned
 * preconditioner's product.  Only iterations in which every component of
 * every replica was still iterating are kept, so each kept record did the
 * full work of its iterations.  sample_every = 0 switches the probe off.   */
typedef struct sim_kernel_prof {
  char name[32];         /* kernel name */
  int64_t launches;      /* timed launches kept */
  double ms;             /* summed event-measured duration of those launches */
  double bytes;          /* summed algorithmic HBM bytes of those launches */
} sim_kernel_prof;
int sim_profile_enable(sim_t* sim, int32_t sample_every);
/* Copy up to cap kernel records into out (*count receives the number of
 * kernels); reset != 0 clears the accumulated records afterwards.         */
int sim_profile_read(sim_t* sim, sim_kernel_prof* out, int32_t cap, int32_t* count,
                     int32_t reset);

/* Plain device copy of `bytes` (a multiple of 16) from src to dst, device
 * pointers, repeated reps times on `hip_stream` between HIP events;
 * *ms_avg receives the mean duration of one copy.  Measurement reference
 * (achievable HBM bandwidth, counter calibration), not part of the method. */
int sim_copy_probe(const void* src, void* dst, int64_t bytes, int32_t reps, void* hip_stream,
                   double* ms_avg);

/* What timing one launch with events adds (measurement reference).  The
 * copy of sim_copy_probe runs reps times back to back between one event
 * pair (*ms_chain: mean per copy, the pair's own cost spread over reps) and
 * reps times more, each after an untimed copy and between the launch-bound
 * event pair the kernel timing probe uses (*ms_each: mean per copy).
 * *ms_each - *ms_chain is the time the probe's events add to each timed
 * launch.  1 <= reps <= 256; device pointers as sim_copy_probe.           */
int sim_event_probe(const void* src, void* dst, int64_t bytes, int32_t reps, void* hip_stream,
                    double* ms_chain, double* ms_each);

/* Whole steps as HIP graphs (batched replicas, many short launches).
 * on != 0: from the second step on, sim_step records one graph per step
 * configuration -- sort, neighbour list, pair terms, the learned forward
 * pass, CG start, the first K CG iterations (K >= the previous solve's
 * count + 1, kept while within 12 of it) and a true-residual check, then the
 * position update and velocity export, which run on the device only if
 * every component of every replica has converged -- and replays it with
 * one host synchronisation per step.  Solves that need more iterations
 * continue with host-queued chunks, so graph and eager steps give identical
 * bits.  With no stream set (NULL), the handle creates a stream of its own
 * that synchronises with the default stream.  With the timing probe on
 * (sim_profile_enable), every sample_every-th step runs eagerly so that its
 * kernels can be timed.  on = 0 releases the graphs.
 * *captures / *replays (optional) receive the counts so far.              */
int sim_graph_mode(sim_t* sim, int32_t on);
int sim_graph_info(sim_t* sim, int64_t* captures, int64_t* replays);

/* Tuning of the CSR products (rows of ~5 entries) w = A u and the learned
 * u = M^-1 r.  A variant is a group of `lanes` lanes per row and a number
 * of entries per lane whose columns and values are loaded one pass of rows
 * ahead of the gathers (0: one entry at a time, no look-ahead), or, with
 * lanes 0, the entry-parallel form: the 256-row sub-tile's entries striped
 * over its threads (`entries` per thread and pass), the products staged in
 * LDS and each row summed by one thread in entry order; index:
 * (lanes, entries)
 *   0: (1, 0)  1: (2, 0)  2: (4, 0)  3: (8, 0)
 *   4: (2, 2)  5: (4, 1)  6: (4, 2)  7: (4, 3)
 *   8: (0, 2)  9: (0, 3)
 * The lane count fixes the summation order of a row; variants with the same
 * lanes give the same bits (the entry-parallel ones those of variant 0),
 * others agree to rounding.  A fixed choice is
 * bitwise reproducible.  Default 8 and 8.                                */
#define SIM_CSR_VARIANTS 10
typedef struct sim_tuning {
  int32_t spmv_variant;  /* 0 .. SIM_CSR_VARIANTS - 1 */
  int32_t apply_variant;
  float spmv_us[SIM_CSR_VARIANTS];  /* sim_autotune: mean duration per variant */
  float apply_us[SIM_CSR_VARIANTS]; /* (0 where not measured) */
  /* CG vector kernel: 0 ordinary loads and stores, 1 nontemporal (streaming)
   * for the vectors not read again within the iteration (faster on a working
   * set larger than the last-level cache); the same bits either way         */
  int32_t vec_variant;
  float vec_us[2];
} sim_tuning;
/* Time every variant `reps` times on the system at the current positions
 * (built for the purpose; the state is unchanged) and keep the fastest.
 * The choice depends on timing, so runs that must be bitwise reproducible
 * should fix it with sim_set_tuning.  out (optional) receives the choice
 * and the timings.                                                        */
int sim_autotune(sim_t* sim, int32_t reps, sim_tuning* out);
/* Use the given variants (timings ignored); SIM_EINVAL for other values. */
int sim_set_tuning(sim_t* sim, const sim_tuning* tuning);

/* Free the handle and all its device memory. NULL is a no-op.             */
void sim_destroy(sim_t* sim);

/* Static string for an error code.                                        */
const char* sim_strerror(int code);

#ifdef __cplusplus
}
#endif
#endif /* SIM_H */
