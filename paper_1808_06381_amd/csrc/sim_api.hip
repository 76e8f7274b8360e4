// sim_api.hip -- host implementation of the C ABI declared in include/sim.h.
//
// The handle owns every device buffer (hipMalloc at creation, grown only
// when the neighbour list outgrows its capacity).  One step queues:
//   ctrl reset, binning, cell scan, scatter, per-cell id sort,
//   neighbour count, row scan, neighbour list, pair terms (A and b),
//   CG start, chunks of CG iterations + true-residual check,
// reads the small control block back once per chunk, then queues the
// position update and reads the control block once more before it commits.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <climits>
#include <mutex>
#include <new>
#include <vector>

#include "launch.h"
#include "mpnn.h"
#include "sim.h"
#include "sim_dev.h"

#define SIM_EOVERFLOW_INTERNAL 1  // capacity of the CSR arrays exceeded: grow and refill
#define SIM_ESTALL_INTERNAL 2     // learned-preconditioned solve stalled: redo with Jacobi
#define SIM_MAX_DEVICES 64

#define HIPCHK(expr)                                   \
  do {                                                 \
    hipError_t e_ = (expr);                            \
    if (e_ != hipSuccess) {                            \
      sim_note_error(e_, #expr, __LINE__);             \
      return SIM_EDEVICE;                              \
    }                                                  \
  } while (0)

static thread_local char g_last_error[512];

static void sim_note_error(hipError_t e, const char* what, int line) {
  snprintf(g_last_error, sizeof(g_last_error), "%s failed (%s) at sim_api.hip:%d", what,
           hipGetErrorString(e), line);
}

struct sim_t {
  int device = 0;
  hipStream_t stream = nullptr;
  int32_t R = 0;
  std::vector<sim_params> prm;
  std::vector<RepDev> reph;
  std::vector<int32_t> blk_rep_h;
  std::vector<int64_t> id_off_h;
  int64_t rows = 0, n_total = 0;
  int64_t step = 0;
  int32_t last_iters = 0;
  DevPtrs d{};
  RepDev* rep_d = nullptr;
  int32_t* scan_tmp = nullptr;
  int32_t* nbr_slots = nullptr;  // [NBR_SLOTS][rows] neighbours kept by the count pass
  int32_t* bsum = nullptr;
  int64_t* id_off_d = nullptr;
  double* io = nullptr;  // n_total x 3 staging for the boundary
  unsigned long long* counter_d = nullptr;
  Ctrl* ctrl_h = nullptr;
  CgRep* cg_h = nullptr;
  double* inj_xi = nullptr;
  double* inj_eta = nullptr;
  std::vector<void*> allocs;
  int32_t restarts_last = 0;
  // kernel timing probe
  int32_t prof_every = 0;
  int32_t prof_phase = 0;               // sampled residue of the iteration index
  std::vector<hipEvent_t> prof_ev;      // pool of event pairs
  struct Sample { int kernel; int iter; int ev; float ms; };
  std::vector<Sample> prof_pending;     // recorded in the current solve
  sim_kernel_prof prof_acc[4] = {};
  int64_t prof_solves = 0;              // probed solves so far (alternate the two forms)
  std::vector<hipEvent_t> prof_run_ev;  // iteration form: before iteration 0, after each
  int32_t prof_run_n = 0;               // iterations recorded in the current solve
  // learned preconditioner
  bool learned = false;      // precond == SIM_PC_LEARNED
  MpPtrs mp{};
  bool mp_ready = false;     // node buffers and weights allocated
  bool mp_train = false;     // training buffers allocated
  int64_t mp_nnz_cap = 0;    // capacity of the per-entry buffers
  int32_t mp_adam_t = 0;
  int32_t learned_maxit = 0;  // 0: cg_maxit
  bool system_valid = false; // A, b, x of a successful solve are in place
  bool er_built = false;     // the last build wrote er (the network's edge input)
  // whole steps replayed as HIP graphs (sim_graph_mode)
  struct StepGraph {
    hipGraphExec_t exec;
    DevPtrs d;   // device state the graph was captured from
    MpPtrs m;
    int K;       // CG iterations recorded before the check round
    bool learned;
  };
  int32_t graph_mode = 0;
  hipStream_t own_stream = nullptr;  // created when graphs need a capturable stream
  std::vector<StepGraph> graphs;
  int64_t graph_captures = 0, graph_replays = 0;
  int32_t graph_K = 0;
  // IC(0) preconditioner
  bool ic0 = false;
  bool warm = false;         // step solves start from the previous velocities
  void* sq_scratch = nullptr;  // structure-factor scratch (grown on demand)
  size_t sq_bytes = 0;
  void* vv_scratch = nullptr;  // velocity-correlation scratch (grown on demand)
  size_t vv_bytes = 0;
  void* vv_scratch2 = nullptr;
  size_t vv_bytes2 = 0;
  // pos_alt and x hold the last committed step's configuration R_n (cell
  // order) and the velocities solved at it; cleared by anything that
  // rebuilds the system or starts a solve
  bool vv_valid = false;
  // anisotropic friction: the block system and its CG
  bool block = false;
  BlockPtrs bp{};
  BlockRep* brep_d = nullptr;
  BcgRep* bcg_h = nullptr;   // pinned host copy of the per-replica solve state
  std::vector<int32_t> ic_color_off;  // offsets of the colours in d.ic_cells (host copy)
  sim_tuning tune{};
};

// The probe's records: three CG kernels (every prof_every-th iteration of a
// probed solve bracketed launch by launch) and the CG iteration as a whole
// (in every other probed solve, one event pair around a run of whole
// iterations of the first chunk: every kernel, the finisher and the gaps
// between launches), priced at the solve's algorithmic bytes per iteration.
static const int kProfKernels = 4;
static const int kProfIteration = 3;
static const char* kProfNames[kProfKernels] = {"k_cg_vec", "k_cg_spmv", "k_cg_apply",
                                               "cg_iteration"};

// ---------------------------------------------------------------------------
// helpers
// ---------------------------------------------------------------------------
static void drop_graphs(sim_t* s) {
  for (auto& g : s->graphs) (void)hipGraphExecDestroy(g.exec);
  s->graphs.clear();
}

static int dalloc(sim_t* s, void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) bytes = 8;
  if (hipMalloc(p, bytes) != hipSuccess) {
    *p = nullptr;
    return SIM_ENOMEM;
  }
  s->allocs.push_back(*p);
  return SIM_OK;
}

static void dfree(sim_t* s, void* p) {
  if (!p) return;
  auto it = std::find(s->allocs.begin(), s->allocs.end(), p);
  if (it != s->allocs.end()) s->allocs.erase(it);
  (void)hipFree(p);
}

// device scratch *p of at least `need` bytes (kept between calls)
static int grow_scratch(sim_t* s, void** p, size_t* have, size_t need) {
  if (need <= *have) return SIM_OK;
  dfree(s, *p);
  *p = nullptr;
  *have = 0;
  int rc = dalloc(s, p, need);
  if (rc) return rc;
  *have = need;
  return SIM_OK;
}

static int validate(const sim_params& p) {
  if (p.n < 1 || p.n > (int64_t)1 << 30) return SIM_EINVAL;
  for (int k = 0; k < 3; ++k)
    if (!(p.box[k] > 0.0) || !std::isfinite(p.box[k])) return SIM_EINVAL;
  if (!(p.gamma0 > 0.0) || !std::isfinite(p.gamma0)) return SIM_EINVAL;
  if (!(p.alpha >= 0.0) || !std::isfinite(p.alpha)) return SIM_EINVAL;
  if (!(p.kT >= 0.0) || !std::isfinite(p.kT)) return SIM_EINVAL;
  if (!(p.dt > 0.0) || !std::isfinite(p.dt)) return SIM_EINVAL;
  if (!std::isfinite(p.shear_rate)) return SIM_EINVAL;
  const double lmin = std::min(p.box[0], std::min(p.box[1], p.box[2]));
  if (!(p.rc > 0.0) || !(p.rc < 0.5 * lmin)) return SIM_EINVAL;
  if (p.weight_law != SIM_W_GAUSS && p.weight_law != SIM_W_POLY2) return SIM_EINVAL;
  if (p.potential < SIM_U_GAUSS_CORE || p.potential > SIM_U_NONE) return SIM_EINVAL;
  if (p.noise_mode < SIM_NOISE_FDT || p.noise_mode > SIM_NOISE_OFF) return SIM_EINVAL;
  if (p.precond < SIM_PC_JACOBI || p.precond > SIM_PC_LEARNED) return SIM_EINVAL;
  if ((p.weight_law == SIM_W_GAUSS || p.potential == SIM_U_GAUSS_CORE) && !(p.lambda > 0.0))
    return SIM_EINVAL;
  if (!std::isfinite(p.u_amp)) return SIM_EINVAL;
  if (!(p.cg_tol > 0.0) || p.cg_maxit < 1) return SIM_EINVAL;
  if (p.warm_start != 0 && p.warm_start != 1) return SIM_EINVAL;
  if (p.spmv_fp32 != 0 && p.spmv_fp32 != 1) return SIM_EINVAL;
  if (p.precond == SIM_PC_LEARNED && !(p.alpha > 0.0)) return SIM_EINVAL;
  if (!(p.friction_par >= 0.0) || !std::isfinite(p.friction_par) || !(p.friction_perp >= 0.0) ||
      !std::isfinite(p.friction_perp))
    return SIM_EINVAL;
  return SIM_OK;
}

// off-diagonal entries of a box with uniform density: n times the mean
// number of neighbours (4/3) pi rc^3 n / V
static double expected_entries(const sim_params& p) {
  const double vol = p.box[0] * p.box[1] * p.box[2];
  return (double)p.n * (4.18879020478639 * p.rc * p.rc * p.rc * (double)p.n / vol);
}

// friction along / across the line of centres (0 stands for 1)
static double fric(double v) { return v == 0.0 ? 1.0 : v; }
static bool anisotropic(const sim_params& p) {
  return fric(p.friction_par) != 1.0 || fric(p.friction_perp) != 1.0;
}

static RepDev make_rep(const sim_params& p) {
  RepDev R;
  std::memset(&R, 0, sizeof(R));
  for (int k = 0; k < 3; ++k) {
    R.L[k] = p.box[k];
    R.hL[k] = 0.5 * p.box[k];
    int nc = (int)std::floor(p.box[k] / (p.rc * (1.0 + 1e-9)));
    if (nc < 3) nc = 1;
    // IC(0) colours cells by coordinate parity, with a third colour for the
    // last cell of an odd axis: an even count (one fewer, larger cells)
    // keeps two colours per axis, 8 launches per triangular sweep, not 27
    if (p.precond == SIM_PC_IC0 && nc >= 5 && nc % 2 == 1) nc -= 1;
    R.nc[k] = nc;
    R.brick = std::max(R.brick, nc);
    R.cell_len[k] = p.box[k] / (double)nc;
    R.inv_cell[k] = (double)nc / p.box[k];
  }
  // bricks of 8^3 cells for boxes of 32 or more cells per axis (the IC(0)
  // form keeps the z-major order its colour lists are built in)
  if (p.precond != SIM_PC_IC0 && R.nc[0] >= 32 && R.nc[1] >= 32 && R.nc[2] >= 32) R.brick = 8;
  R.n = (int32_t)p.n;
  R.kT = p.kT;
  R.gamma0 = p.gamma0;
  R.alpha = p.alpha;
  R.shear = p.shear_rate;
  R.dt = p.dt;
  R.rc = p.rc;
  R.rc2 = p.rc * p.rc;
  R.lam = p.lambda > 0.0 ? p.lambda : 1.0;
  R.inv_lam2 = 1.0 / (R.lam * R.lam);
  R.u_amp = p.u_amp;
  if (p.noise_mode == SIM_NOISE_FDT) {
    const double c = std::sqrt(2.0 * p.kT / p.dt);
    R.amp_node = c * std::sqrt(p.gamma0);
    R.amp_pair = c;
  } else if (p.noise_mode == SIM_NOISE_PAPER) {
    R.amp_node = std::sqrt(2.0 * p.gamma0 * p.kT / p.dt);
    R.amp_pair = 0.0;
  }
  R.force_gc = (p.kT * p.u_amp) / (R.lam * R.lam);
  R.force_soft = 2.0 * p.u_amp / p.rc;
  R.tol2 = p.cg_tol * p.cg_tol;
  R.weight_law = p.weight_law;
  R.potential = p.potential;
  R.noise_mode = p.noise_mode;
  R.precond = p.precond;
  R.seed = p.seed;
  R.stream = p.stream;
  return R;
}

static double host_le_offset(const sim_params& p, int64_t step) {
  const double t = (double)step * p.dt;
  return std::fmod((p.shear_rate * p.box[1]) * t, p.box[0]);
}

static int alloc_csr(sim_t* s, int64_t cap) {
  drop_graphs(s);
  dfree(s, s->d.col);
  dfree(s, s->d.val);
  dfree(s, s->d.valf);
  dfree(s, s->d.er);
  dfree(s, s->d.lcol);
  dfree(s, s->d.lval);
  s->d.lcol = nullptr;
  s->d.lval = nullptr;
  s->d.col = nullptr;
  s->d.val = nullptr;
  s->d.valf = nullptr;
  s->d.er = nullptr;
  if (cap > (int64_t)INT32_MAX) cap = INT32_MAX;
  int rc;
  if ((rc = dalloc(s, (void**)&s->d.col, sizeof(int32_t) * (size_t)cap))) return rc;
  if ((rc = dalloc(s, (void**)&s->d.val, sizeof(double) * (size_t)cap))) return rc;
  if ((rc = dalloc(s, (void**)&s->d.valf, sizeof(float) * (size_t)cap))) return rc;
  if ((rc = dalloc(s, (void**)&s->d.er, sizeof(float) * (size_t)cap))) return rc;
  if (s->block) {
    dfree(s, s->bp.bval);
    dfree(s, s->bp.bvalf);
    s->bp.bval = nullptr;
    s->bp.bvalf = nullptr;
    if ((rc = dalloc(s, (void**)&s->bp.bval, sizeof(double) * 6 * (size_t)cap))) return rc;
    if (s->bp.fp32 && (rc = dalloc(s, (void**)&s->bp.bvalf, sizeof(float) * 6 * (size_t)cap)))
      return rc;
  }
  if (s->ic0) {
    if ((rc = dalloc(s, (void**)&s->d.lcol, sizeof(int32_t) * (size_t)cap))) return rc;
    if ((rc = dalloc(s, (void**)&s->d.lval, sizeof(double) * (size_t)cap))) return rc;
    HIPCHK(hipMemset(s->d.lcol, 0, sizeof(int32_t) * (size_t)cap));
  }
  s->d.nnz_cap = cap;
  return SIM_OK;
}

// Buffers of the learned preconditioner: node arrays and weights once,
// per-entry arrays whenever the CSR capacity changed, training arrays on the
// first training step.  Weights start at zero (a valid SPD preconditioner).
static int ensure_mp(sim_t* s, bool training) {
  MpPtrs& m = s->mp;
  const size_t rows = (size_t)s->rows, H = MP_H;
  int rc;
#define MPALLOC(ptr, bytes) \
  if ((rc = dalloc(s, (void**)&(ptr), (bytes))) != SIM_OK) return rc;
  if (!s->mp_ready) {
    MPALLOC(m.w16, sizeof(uint16_t) * MP_NPARAMS_ALL);
    MPALLOC(m.th32, sizeof(float) * MP_NPARAMS_ALL);
    MPALLOC(m.am, sizeof(float) * MP_NPARAMS_ALL);
    MPALLOC(m.av, sizeof(float) * MP_NPARAMS_ALL);
    MPALLOC(m.grad, sizeof(float) * MP_NPARAMS_ALL);
    MPALLOC(m.x, sizeof(float) * 3 * rows);
    MPALLOC(m.h, sizeof(float) * (MP_NL + 1) * rows * H);
    MPALLOC(m.y, sizeof(float) * MP_NL * rows * H);
    MPALLOC(m.hb, sizeof(uint16_t) * rows * H);
    MPALLOC(m.hb2, sizeof(uint16_t) * rows * H);
    MPALLOC(m.tau, sizeof(float) * rows);
    MPALLOC(m.mdiag, sizeof(double) * rows);
    MPALLOC(m.lpart, sizeof(double) * 2 * (rows / 256 + 1));
    MPALLOC(m.loss, sizeof(double) * 2);
    HIPCHK(hipMemset(m.w16, 0, sizeof(uint16_t) * MP_NPARAMS_ALL));
    HIPCHK(hipMemset(m.th32, 0, sizeof(float) * MP_NPARAMS_ALL));
    HIPCHK(hipMemset(m.am, 0, sizeof(float) * MP_NPARAMS_ALL));
    HIPCHK(hipMemset(m.av, 0, sizeof(float) * MP_NPARAMS_ALL));
    HIPCHK(hipMemset(m.grad, 0, sizeof(float) * MP_NPARAMS_ALL));
    m.rows = s->rows;
    m.round_act = 1;
    m.lam_floor = MP_EPS_LAM;
    m.nparams = s->block ? MP_NPARAMS_ALL : MP_NPARAMS;
    if (s->block) {  // the 3 x 3 heads: A_ii^-1/2 and the node blocks of M^-1
      MPALLOC(s->bp.rsq, sizeof(double) * 6 * rows);
      MPALLOC(s->bp.xd, sizeof(double) * 6 * rows);
    }
    s->mp_ready = true;
  }
  if (s->mp_nnz_cap != s->d.nnz_cap) {
    drop_graphs(s);
    dfree(s, m.ef);
    dfree(s, m.efh);
    dfree(s, m.tg);
    dfree(s, m.moff);
    dfree(s, s->bp.xo);
    m.ef = m.tg = m.moff = nullptr;
    m.efh = nullptr;
    s->bp.xo = nullptr;
    const size_t cap = (size_t)s->d.nnz_cap;
    MPALLOC(m.ef, sizeof(float) * 3 * cap);
    MPALLOC(m.efh, sizeof(uint16_t) * 4 * cap);
    MPALLOC(m.tg, sizeof(float) * cap);
    MPALLOC(m.moff, sizeof(float) * cap);
    if (s->block) MPALLOC(s->bp.xo, sizeof(float) * 9 * cap);
    s->mp_nnz_cap = s->d.nnz_cap;
  }
  if (training && !s->mp_train) {
    MPALLOC(m.m, sizeof(float) * MP_NL * rows * H);
    MPALLOC(m.a, sizeof(float) * MP_NL * rows * H);
    MPALLOC(m.zb, sizeof(double) * 3 * rows);
    MPALLOC(m.G, sizeof(double) * 3 * rows);
    MPALLOC(m.dh, sizeof(float) * rows * H);
    MPALLOC(m.dh2, sizeof(float) * rows * H);
    MPALLOC(m.dm, sizeof(float) * rows * H);
    MPALLOC(m.gpart, sizeof(float) * (rows / MP_ROWS) * MP_NPARAMS_ALL);
    MPALLOC(m.pz, sizeof(double) * 3 * rows);
    MPALLOC(m.pb, sizeof(double) * 3 * rows);
    if (s->block) {  // R G, A_ii^-1 G, R b, A_ii^-1 b
      MPALLOC(s->bp.gt, sizeof(double) * 3 * rows);
      MPALLOC(s->bp.gh, sizeof(double) * 3 * rows);
      MPALLOC(s->bp.t, sizeof(double) * 3 * rows);
      MPALLOC(s->bp.bh, sizeof(double) * 3 * rows);
    }
    s->mp_train = true;
  }
#undef MPALLOC
  m.er = s->d.er;
  s->d.want_er = 1;  // later builds write the network's edge input
  s->d.mdiag = m.mdiag;
  s->d.moff = m.moff;
  return SIM_OK;
}

// ---------------------------------------------------------------------------
// the step's phases
// ---------------------------------------------------------------------------

// a1-a5: sort, neighbour list, A and b at `step`.  The capacity check of the
// fill is read back later (with the first CG chunk).
static int build_system(sim_t* s) {
  DevPtrs& d = s->d;
  s->system_valid = false;
  s->vv_valid = false;
  hipStream_t st = s->stream;
  HIPCHK(launch_ctrl_zero(d, st));
  HIPCHK(launch_fill_i32(d.cell_count, 0, d.ncell_entries, st));
  HIPCHK(launch_bin(d, st));
  HIPCHK(launch_scan(d.cell_count, s->scan_tmp, d.ncell_entries, s->bsum, st));
  HIPCHK(launch_cell_rows(d, s->scan_tmp, st));
  HIPCHK(launch_scatter(d, st));
  std::swap(d.pos, d.pos_alt);
  std::swap(d.cellidx, d.cellidx_alt);
  HIPCHK(launch_cell_sort(d, st));
  HIPCHK(launch_nbr_count(d, s->nbr_slots, st));
  HIPCHK(launch_scan(d.rowlen, d.rowptr, s->rows + 1, s->bsum, st, &d.ctrl->too_many));
  HIPCHK(launch_nbr_list(d, s->nbr_slots, st));
  if (s->block) HIPCHK(launch_pair_block(d, s->bp, st));
  else HIPCHK(launch_pair_terms(d, st));
  s->er_built = d.want_er != 0;
  return SIM_OK;
}

static int read_ctrl(sim_t* s, bool with_cg) {
  HIPCHK(hipMemcpyAsync(s->ctrl_h, s->d.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s->stream));
  if (with_cg)
    HIPCHK(hipMemcpyAsync(s->cg_h, s->d.cg, sizeof(CgRep) * (size_t)s->R, hipMemcpyDeviceToHost,
                          s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  return SIM_OK;
}

static int grow_and_refill(sim_t* s) {
  if (s->ctrl_h->too_many) {
    snprintf(g_last_error, sizeof(g_last_error),
             "the neighbour list holds more than INT32_MAX entries (32-bit CSR offsets)");
    return SIM_ENOMEM;
  }
  int64_t need = s->ctrl_h->nnz;
  int rc = alloc_csr(s, need + need / 4 + 1024);
  if (rc) return rc;
  if (need > s->d.nnz_cap) return SIM_ENOMEM;
  HIPCHK(launch_ctrl_zero(s->d, s->stream));
  HIPCHK(launch_nbr_list(s->d, s->nbr_slots, s->stream));
  if (s->block) HIPCHK(launch_pair_block(s->d, s->bp, s->stream));
  else HIPCHK(launch_pair_terms(s->d, s->stream));
  return SIM_OK;
}

// a6: CG on the current system (b in d.b), x0 = 0, in three host pieces:
// cg_queue_start (reset, fresh start), cg_queue_chunk (n iterations and a
// true-residual check round; finished replicas' blocks return at once) and
// cg_poll_loop (reads the control block after each chunk and queues the
// next one).  A step graph records the start and the first chunk; the host
// loop then continues from the replayed state.
static int cg_maxit(const sim_t* s) {
  int maxit = 1;
  for (auto& p : s->prm) maxit = std::max(maxit, p.cg_maxit);
  if (s->d.learned && s->learned_maxit > 0) maxit = std::min(maxit, (int)s->learned_maxit);
  return maxit;
}

// u = M^-1 r by the learned product or the IC(0) triangular solves (with
// the (r, u) partials), for the components selected by mode
static int queue_apply(sim_t* s, int mode, hipEvent_t e0, hipEvent_t e1, int rev = 0) {
  DevPtrs d = s->d;
  d.rev = rev;
  if (d.ic0) {
    HIPCHK(launch_ic_apply(d, s->ic_color_off.data(), (int)s->ic_color_off.size() - 1, s->stream));
    HIPCHK(launch_cg_dot_ru(d, mode, s->stream));
  } else {
    HIPCHK(launch_cg_apply(d, mode, s->stream, e0, e1));
  }
  return SIM_OK;
}

// the preconditioner of the system just built: learned forward pass or
// IC(0) factorisation
static int prepare_precond(sim_t* s) {
  if (s->learned) {
    int rc = ensure_mp(s, false);
    if (rc) return rc;
    s->mp.store_train = 0;
    if (s->block) {
      HIPCHK(launch_mp_trunk(s->d, s->mp, s->stream));
      HIPCHK(launch_mpb_heads(s->d, s->mp, s->bp, s->stream));
    } else {
      HIPCHK(launch_mp_forward(s->d, s->mp, s->stream));
    }
    s->d.learned = 1;
  }
  if (s->ic0)
    HIPCHK(launch_ic_factor(s->d, s->ic_color_off.data(), (int)s->ic_color_off.size() - 1,
                            s->stream));
  return SIM_OK;
}

// tol > 0 overrides the replicas' own tolerances
// Fresh start from x = 0 (which also takes ||b||^2); with `warm`, the
// iterating components then restart from the previous step's velocities:
// x = v_prev, r = b - A x, done if r passes, else the restart path.
static int cg_queue_start(sim_t* s, double tol, bool warm) {
  s->vv_valid = false;
  const DevPtrs& d = s->d;
  const bool ext = d.learned || d.ic0;
  HIPCHK(launch_cg_reset(d, tol, s->stream));
  HIPCHK(launch_cg_vec(d, 0, s->stream));
  if (ext) {
    int rc = queue_apply(s, 0, nullptr, nullptr);
    if (rc) return rc;
  }
  HIPCHK(launch_cg_spmv(d, 0, 0, s->stream));
  HIPCHK(launch_cg_finish(d, 0, s->stream));
  if (warm) {
    HIPCHK(launch_cg_warm(d, s->id_off_d, s->stream));
    HIPCHK(launch_cg_spmv(d, 2, 0, s->stream));
    HIPCHK(launch_cg_finish(d, 4, s->stream));
    HIPCHK(launch_cg_vec(d, 1, s->stream));
    if (ext) {
      int rc = queue_apply(s, 1, nullptr, nullptr);
      if (rc) return rc;
    }
    HIPCHK(launch_cg_spmv(d, 0, 1, s->stream));
    HIPCHK(launch_cg_finish(d, 1, s->stream));
  }
  return SIM_OK;
}

// n iterations (iteration numbers first..first+n-1 for the timing probe,
// which is off when probes is false), then the check round: true residuals
// of replicas whose components all passed, restarts of those that failed
static int cg_queue_chunk(sim_t* s, int n, int first, bool probes) {
  const DevPtrs& d = s->d;
  hipStream_t stream = s->stream;
  const bool ext = d.learned || d.ic0;  // a separate preconditioner pass
  // iteration form of the probe: an event before iteration 0 of the first
  // chunk and one after each of its iterations; the poll keeps the longest
  // run of iterations that every component went through
  const bool run_form = probes && s->prof_every > 0 && (s->prof_solves & 1) && first == 0 &&
                        n + 1 <= (int)s->prof_run_ev.size();
  if (run_form) {
    s->prof_run_n = n;
    HIPCHK(hipEventRecord(s->prof_run_ev[0], stream));
  }
  int nstream = 0;  // streaming CG launches queued so far in this chunk
  for (int k = 0; k < n; ++k) {
    const int g = first + k;
    const bool probe = probes && !(s->prof_solves & 1) && s->prof_every > 0 &&
                       g % s->prof_every == s->prof_phase &&
                       (int)s->prof_pending.size() + kProfKernels <= (int)s->prof_ev.size() / 2;
    // vector update, then (learned) u = M^-1 r, then w = A u; consecutive
    // streaming launches walk their sub-tiles in opposite directions
    const int order[3] = {0, 2, 1};
    for (int oi = 0; oi < 3; ++oi) {
      const int kern = order[oi];
      if (kern == 2 && !ext) continue;
      DevPtrs dk = d;
      dk.rev = nstream++ & 1;
      hipEvent_t e0 = nullptr, e1 = nullptr;
      if (probe && !(kern == 2 && d.ic0)) {  // the IC(0) pass is many launches: not probed
        const int ev = (int)s->prof_pending.size();
        s->prof_pending.push_back({kern, g, ev, 0.0f});
        e0 = s->prof_ev[2 * ev];
        e1 = s->prof_ev[2 * ev + 1];
      }
      if (kern == 0) HIPCHK(launch_cg_vec(dk, 2, stream, e0, e1));
      else if (kern == 1) HIPCHK(launch_cg_spmv(dk, 0, 2, stream, e0, e1));
      else {
        int rc = queue_apply(s, 2, e0, e1, dk.rev);
        if (rc) return rc;
      }
    }
    HIPCHK(launch_cg_finish(d, 2, stream));
    if (run_form) HIPCHK(hipEventRecord(s->prof_run_ev[k + 1], stream));
  }
  HIPCHK(launch_cg_flush(d, stream));  // x complete where a check is pending
  HIPCHK(launch_cg_spmv(d, 1, 0, stream));
  HIPCHK(launch_cg_finish(d, 3, stream));
  HIPCHK(launch_cg_vec(d, 1, stream));
  if (ext) {
    int rc = queue_apply(s, 1, nullptr, nullptr);
    if (rc) return rc;
  }
  HIPCHK(launch_cg_spmv(d, 0, 1, stream));
  HIPCHK(launch_cg_finish(d, 1, stream));
  return SIM_OK;
}

// Host loop after `launched` iterations have been queued (the last chunk not
// yet polled).  *first_final (optional) tells whether the first poll already
// found the solve finished.  Returns SIM_EOVERFLOW_INTERNAL if the fill
// overflowed (nothing solved), SIM_ESTALL_INTERNAL on a learned stall.
static int cg_poll_loop(sim_t* s, int launched, sim_stats* st, bool* first_final) {
  DevPtrs& d = s->d;
  const int maxit = cg_maxit(s);
  const bool learned = d.learned != 0;
  std::vector<std::pair<int, double>> hist;  // (iterations, worst relative residual^2)
  int status = SIM_OK;
  for (int poll = 0;; ++poll) {
    int rc = read_ctrl(s, true);
    if (rc) return rc;
    if (first_final && poll == 0)
      *first_final = s->ctrl_h->overflow == 0 && s->ctrl_h->n_notdone == 0;
    if (s->ctrl_h->overflow) { status = SIM_EOVERFLOW_INTERNAL; break; }
    if (s->ctrl_h->n_notdone == 0) break;
    if (launched > maxit) { status = SIM_ENOCONV; break; }
    if (learned) {
      // stall: the worst relative residual of an unfinished component has
      // not dropped by 10 % over the last 10 or more iterations (after 20)
      double worst = 0.0;
      for (int r = 0; r < s->R; ++r)
        for (int k = 0; k < 3; ++k) {
          const CgRep& c = s->cg_h[r];
          if (c.state[k] != 2 && c.bb[k] > 0.0) worst = std::max(worst, c.rr[k] / c.bb[k]);
        }
      hist.push_back({launched, worst});
      if (launched >= 20) {
        for (auto it = hist.rbegin(); it != hist.rend(); ++it)
          if (launched - it->first >= 10) {
            if (!(worst < 0.81 * it->second)) status = SIM_ESTALL_INTERNAL;  // 0.9^2 on squares
            break;
          }
        if (status) break;
      }
    }
    const int n = std::max(1, std::min(2, maxit + 1 - launched));
    if ((rc = cg_queue_chunk(s, n, launched, true))) return rc;
    launched += n;
  }
  if (status == SIM_EOVERFLOW_INTERNAL || status == SIM_ESTALL_INTERNAL) {
    s->prof_pending.clear();
    s->prof_run_n = 0;
    return status;
  }
  int itmax = 0, restarts = 0, breakdown = 0;
  int iters[3] = {0, 0, 0};
  double relres[3] = {0, 0, 0};
  for (int r = 0; r < s->R; ++r) {
    const CgRep& c = s->cg_h[r];
    for (int k = 0; k < 3; ++k) {
      iters[k] = std::max(iters[k], c.it[k]);
      itmax = std::max(itmax, c.it[k]);
      const double rel = c.bb[k] > 0.0 ? std::sqrt(c.rr[k] / c.bb[k]) : 0.0;
      relres[k] = std::max(relres[k], rel);
    }
    restarts = std::max(restarts, c.restarts);
    breakdown |= c.breakdown;
  }
  s->last_iters = itmax;
  if (!s->prof_pending.empty() || s->prof_run_n > 0) {
    // keep launches in which every component of every replica iterated
    int itmin = INT32_MAX;
    for (int r = 0; r < s->R; ++r)
      for (int k = 0; k < 3; ++k)
        if (s->cg_h[r].bb[k] > 0.0) itmin = std::min(itmin, s->cg_h[r].it[k]);
    const double rows = (double)s->rows, nnz = (double)s->ctrl_h->nnz;
    const double ntile = (double)(SUBS_PER_TILE * d.nblk);  // partial slots written
    const double per_launch[kProfKernels] = {
        // vector kernel: r, p, w, s, x read (120 B/row), 1/diag (8), p, s, x, r, u written
        // (120); with the learned preconditioner u is read instead of 1/diag and not written;
        // x (48 of these bytes) only in odd iterations (see below)
        (learned ? rows * 240.0 : rows * 248.0) + ntile * 6.0 * 8.0,
        // product: row pointers (4), u (24), diag (8), w written (24), CSR col + value
        rows * 60.0 + 4.0 + nnz * (4.0 + (s->d.spmv_fp32 ? 4.0 : 8.0)) + ntile * 3.0 * 8.0,
        // learned apply: row pointers (4), r (24), M^-1 diagonal (8), u written (24),
        // column + FP32 value per entry
        rows * 60.0 + 4.0 + nnz * 8.0 + ntile * 3.0 * 8.0};
    // one CG iteration's algorithmic bytes over the real particles N with
    // nnz off-diagonal entries (k = nnz / N per row): the matrix 12(k + 1) + 4
    // (value 8 + column 4 per entry, the diagonal as one more entry, a row
    // pointer 4; values 4 bytes with the FP32 product) and 200 vector bytes
    // per row (p read 24, q written and read 48, x and r read and written
    // 96, 1/diag 8, p written 24); the learned form adds one matrix pass for
    // its M^-1 product
    double npart = 0.0;
    for (const RepDev& R : s->reph) npart += (double)R.n;
    const double vb = s->d.spmv_fp32 ? 8.0 : 12.0;
    const double mat = vb * (nnz + npart) + 4.0 * npart;
    const double per_iter = mat + 200.0 * npart + (learned ? 12.0 * (nnz + npart) + 4.0 * npart : 0.0);
    if (s->prof_run_n > 0) {
      // iterations 0 .. m-1, which every component went through in full
      const int m = itmin == INT32_MAX ? 0 : std::min(s->prof_run_n, itmin - 1);
      if (m >= 2) {
        float ms = 0.0f;
        HIPCHK(hipEventElapsedTime(&ms, s->prof_run_ev[0], s->prof_run_ev[m]));
        sim_kernel_prof& acc = s->prof_acc[kProfIteration];
        acc.launches += m;
        acc.ms += ms;
        acc.bytes += per_iter * m;
      }
      s->prof_run_n = 0;
    }
    for (auto& smp : s->prof_pending) {
      float ms = 0.0f;
      HIPCHK(hipEventElapsedTime(&ms, s->prof_ev[2 * smp.ev], s->prof_ev[2 * smp.ev + 1]));
      sim_kernel_prof& acc = s->prof_acc[smp.kernel];
      if (smp.iter >= itmin - 1) continue;
      acc.launches += 1;
      acc.ms += ms;
      // the vector kernel updates x every other iteration: in an even one
      // (iteration number = every component's count here) x is not touched
      acc.bytes += per_launch[smp.kernel] - (smp.kernel == 0 && smp.iter % 2 == 0 ? 48.0 * rows : 0.0);
    }
    s->prof_pending.clear();
    // the next solve samples the next residue, so that every position in a
    // solve is sampled alike (its first iterations run with colder caches)
    if (!(s->prof_solves & 1)) s->prof_phase = (s->prof_phase + 1) % s->prof_every;
  }
  if (st) {
    for (int k = 0; k < 3; ++k) {
      st->iters[k] = std::max(st->iters[k], iters[k]);
      st->relres[k] = std::max(st->relres[k], relres[k]);
    }
    st->restarts = std::max(st->restarts, restarts);
    st->nnz = s->ctrl_h->nnz;
    st->max_row = s->ctrl_h->max_row;
    st->cg_iters_total += itmax;
  }
  if (status) return status;
  if (breakdown) return SIM_EBREAKDOWN;
  return SIM_OK;
}

// the block system's CG (anisotropic friction): residual round (with a warm
// start, a second one from the previous step's velocities), then chunks of
// iterations each closed by a residual round, the host reading the
// per-replica states after each chunk
static int bcg_solve(sim_t* s, double tol, bool warm, sim_stats* st) {
  s->vv_valid = false;
  s->bp.learned = s->learned && s->d.learned ? 1 : 0;
  HIPCHK(hipMemcpyAsync(s->ctrl_h, s->d.ctrl, sizeof(Ctrl), hipMemcpyDeviceToHost, s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  if (s->ctrl_h->overflow) return SIM_EOVERFLOW_INTERNAL;
  HIPCHK(launch_bcg_reset(s->d, s->bp, tol, s->stream));
  HIPCHK(launch_bcg_residual(s->d, s->bp, s->stream));
  if (warm) {
    HIPCHK(launch_bcg_warm(s->d, s->bp, s->id_off_d, s->stream));
    HIPCHK(launch_bcg_residual(s->d, s->bp, s->stream));
  }
  const int maxit = cg_maxit(s);
  int chunk = std::max(4, std::min(32, s->last_iters > 0 ? s->last_iters : 8));
  int status = SIM_OK;
  std::vector<std::pair<int, double>> hist;  // (iterations, worst relative residual^2)
  for (;;) {
    HIPCHK(hipMemcpyAsync(s->bcg_h, s->bp.bcg, sizeof(BcgRep) * (size_t)s->R,
                          hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
    bool all_done = true, broke = false;
    int itmax = 0;
    double worst = 0.0;
    for (int r = 0; r < s->R; ++r) {
      const BcgRep& B = s->bcg_h[r];
      all_done = all_done && B.state == 2;
      broke = broke || B.breakdown;
      itmax = std::max(itmax, (int)B.it);
      if (B.state != 2 && B.bb > 0.0) worst = std::max(worst, B.rr / B.bb);
    }
    if (broke) { status = SIM_EBREAKDOWN; break; }
    if (all_done) break;
    if (itmax >= maxit) { status = SIM_ENOCONV; break; }
    if (s->bp.learned) {
      // stall (as the scalar solve): the worst residual of an unfinished
      // replica not 10 % lower over the last 10 or more iterations (after 20)
      hist.push_back({itmax, worst});
      if (itmax >= 20) {
        for (auto it = hist.rbegin(); it != hist.rend(); ++it)
          if (itmax - it->first >= 10) {
            if (!(worst < 0.81 * it->second)) status = SIM_ESTALL_INTERNAL;
            break;
          }
        if (status) break;
      }
    }
    const int k = std::min(chunk, maxit - itmax);
    for (int q = 0; q < k; ++q) HIPCHK(launch_bcg_iteration(s->d, s->bp, s->stream));
    HIPCHK(launch_bcg_residual(s->d, s->bp, s->stream));
    chunk = 8;
  }
  int itmax = 0, restarts = 0;
  double rel = 0.0;
  for (int r = 0; r < s->R; ++r) {
    const BcgRep& B = s->bcg_h[r];
    itmax = std::max(itmax, (int)B.it);
    restarts = std::max(restarts, (int)B.restarts);
    if (B.bb > 0.0) rel = std::max(rel, std::sqrt(B.rr / B.bb));
  }
  s->last_iters = itmax;
  if (st) {
    for (int k = 0; k < 3; ++k) {
      st->iters[k] = itmax;
      st->relres[k] = rel;
    }
    st->restarts = restarts;
    st->nnz = s->ctrl_h->nnz;
    st->max_row = s->ctrl_h->max_row;
    st->cg_iters_total += itmax;
  }
  return status;
}

static int cg_solve(sim_t* s, double tol, bool warm, sim_stats* st) {
  if (s->block) return bcg_solve(s, tol, warm, st);
  int rc = cg_queue_start(s, tol, warm);
  if (rc) return rc;
  const int n = std::max(1, std::min(s->last_iters > 2 ? s->last_iters - 1 : 8, cg_maxit(s) + 1));
  if ((rc = cg_queue_chunk(s, n, 0, true))) return rc;
  rc = cg_poll_loop(s, n, st, nullptr);
  if (s->prof_every > 0) s->prof_solves += 1;  // the probe alternates its two forms
  return rc;
}

static int build_and_solve(sim_t* s, bool replace_rhs, double tol, sim_stats* st) {
  int rc = build_system(s);
  if (rc) return rc;
  for (int attempt = 0; attempt < 4; ++attempt) {
    if ((rc = prepare_precond(s))) return rc;
    if (replace_rhs) HIPCHK(launch_permute(s->d, s->id_off_d, 1, s->io, nullptr, s->stream));
    rc = cg_solve(s, tol, s->warm && !replace_rhs, st);
    if (s->learned && (rc == SIM_ESTALL_INTERNAL || rc == SIM_EBREAKDOWN || rc == SIM_ENOCONV)) {
      // the learned solve did not make progress: redo it with Jacobi
      s->d.learned = 0;
      rc = cg_solve(s, tol, s->warm && !replace_rhs, st);
      s->d.learned = 1;
      if (st) st->fallback = 1;
    }
    if (rc != SIM_EOVERFLOW_INTERNAL) {
      if (rc == SIM_OK) s->system_valid = true;
      return rc;
    }
    rc = grow_and_refill(s);
    if (rc) return rc;
  }
  return SIM_ENOMEM;
}

// build + capacity check without a solve (parity exports)
static int build_checked(sim_t* s) {
  int rc = build_system(s);
  if (rc) return rc;
  for (int attempt = 0; attempt < 4; ++attempt) {
    rc = read_ctrl(s, false);
    if (rc) return rc;
    if (!s->ctrl_h->overflow) return SIM_OK;
    rc = grow_and_refill(s);
    if (rc) return rc;
  }
  return SIM_ENOMEM;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------
extern "C" {

const char* sim_strerror(int code) {
  switch (code) {
    case SIM_OK: return "ok";
    case SIM_EINVAL: return "invalid argument";
    case SIM_ENOMEM: return "out of memory";
    case SIM_EDEVICE: return g_last_error[0] ? g_last_error : "HIP runtime error";
    case SIM_ENOCONV: return "conjugate gradients did not converge within cg_maxit";
    case SIM_EBREAKDOWN: return "conjugate gradients broke down (p.Ap <= 0)";
    case SIM_ECAPACITY: return "output buffer too small";
    case SIM_ENUMERIC: return "non-finite or escaped position";
    case SIM_ENOTSUP: return "not supported";
    default: return "unknown error";
  }
}

void sim_destroy(sim_t* s) {
  if (!s) return;
  (void)hipSetDevice(s->device);
  drop_graphs(s);
  if (s->own_stream) (void)hipStreamDestroy(s->own_stream);
  for (void* p : s->allocs) (void)hipFree(p);
  for (hipEvent_t e : s->prof_ev) (void)hipEventDestroy(e);
  for (hipEvent_t e : s->prof_run_ev) (void)hipEventDestroy(e);
  if (s->ctrl_h) (void)hipHostFree(s->ctrl_h);
  if (s->cg_h) (void)hipHostFree(s->cg_h);
  if (s->bcg_h) (void)hipHostFree(s->bcg_h);
  delete s;
}

int sim_create_batch(const sim_params* params, int32_t replicas, const double* pos0,
                     sim_t** out) {
  if (!params || !pos0 || !out || replicas < 1) return SIM_EINVAL;
  *out = nullptr;
  for (int r = 0; r < replicas; ++r) {
    int rc = validate(params[r]);
    if (rc) return rc;
  }
  // The CSR offsets are 32-bit: refuse a handle whose uniform-density
  // neighbour list alone would fill half that range (clustering adds about
  // a third to it; the row scan still raises SIM_ENOMEM if a state passes it)
  {
    double expect = 0.0;
    for (int r = 0; r < replicas; ++r) expect += expected_entries(params[r]);
    if (expect > 0.5 * (double)INT32_MAX) return SIM_EINVAL;
  }
  sim_t* s = new (std::nothrow) sim_t();
  if (!s) return SIM_ENOMEM;
  if (hipGetDevice(&s->device) != hipSuccess) { delete s; return SIM_EDEVICE; }
  s->R = replicas;
  s->prm.assign(params, params + replicas);
  s->learned = params[0].precond == SIM_PC_LEARNED;
  s->ic0 = params[0].precond == SIM_PC_IC0;
  for (int r = 0; r < replicas; ++r) s->block = s->block || anisotropic(params[r]);
  if (s->block)
    for (int r = 0; r < replicas; ++r)
      if (params[r].precond == SIM_PC_IC0) {
        delete s;
        return SIM_ENOTSUP;
      }
  for (int r = 1; r < replicas; ++r)
    if ((params[r].precond == SIM_PC_LEARNED) != s->learned ||
        (params[r].precond == SIM_PC_IC0) != s->ic0) {
      delete s;
      return SIM_EINVAL;
    }
  // layout
  int64_t row_off = 0, seg_off = 0, n_total = 0;
  int32_t blk_off = 0;
  for (int r = 0; r < replicas; ++r) {
    RepDev R = make_rep(params[r]);
    const int64_t npad = (params[r].n + ROWS_PER_BLOCK - 1) / ROWS_PER_BLOCK * ROWS_PER_BLOCK;
    const int64_t ncell = (int64_t)R.nc[0] * R.nc[1] * R.nc[2];
    R.row_off = row_off;
    R.npad = (int32_t)npad;
    R.blk_off = blk_off;
    R.nblk = (int32_t)(npad / ROWS_PER_BLOCK);
    R.seg_off = (int32_t)seg_off;
    if (seg_off + ncell + 1 > INT32_MAX || row_off + npad > INT32_MAX / 2) {
      delete s;
      return SIM_EINVAL;
    }
    s->reph.push_back(R);
    for (int b = 0; b < R.nblk; ++b) s->blk_rep_h.push_back(r);
    s->id_off_h.push_back(n_total);
    row_off += npad;
    seg_off += ncell + 1;
    blk_off += R.nblk;
    n_total += params[r].n;
  }
  s->rows = row_off;
  s->n_total = n_total;
  // positions: validate and lay out
  std::vector<double4> ph((size_t)s->rows);
  for (int r = 0; r < replicas; ++r) {
    const RepDev& R = s->reph[r];
    const double* src = pos0 + 3 * s->id_off_h[r];
    for (int64_t i = 0; i < R.npad; ++i) {
      double4 v = make_double4(0.0, 0.0, 0.0, -1.0);
      if (i < R.n) {
        v = make_double4(src[3 * i], src[3 * i + 1], src[3 * i + 2], (double)i);
        const double c[3] = {v.x, v.y, v.z};
        for (int k = 0; k < 3; ++k)
          if (!std::isfinite(c[k]) || c[k] < 0.0 || c[k] > R.L[k]) { delete s; return SIM_EINVAL; }
      }
      ph[(size_t)(R.row_off + i)] = v;
    }
  }
  DevPtrs& d = s->d;
  d.rows = s->rows;
  d.nblk = blk_off;
  d.want_er = s->learned ? 1 : 0;
  // two-level reduction of the CG partials for replicas of many sub-tiles
  std::vector<int32_t> l1_rep_h;
  for (int r = 0; r < replicas; ++r) {
    RepDev& R = s->reph[r];
    const int nsub = SUBS_PER_TILE * R.nblk;
    R.l1_off = (int32_t)l1_rep_h.size();
    R.l1_cnt = nsub > L1_MIN_SUBS ? (nsub + L1_SUBS - 1) / L1_SUBS : 0;
    for (int b = 0; b < R.l1_cnt; ++b) l1_rep_h.push_back(r);
  }
  d.l1_total = (int32_t)l1_rep_h.size();
  d.nrep = replicas;
  d.ncell_entries = (int32_t)seg_off;
  d.spmv_fp32 = params[0].spmv_fp32;
  d.spmv_var = CSR_VARIANT_DEFAULT;
  d.apply_var = CSR_VARIANT_DEFAULT;
  d.ic0 = s->ic0 ? 1 : 0;
  d.pc_none = params[0].precond == SIM_PC_NONE ? 1 : 0;
  for (int r = 1; r < replicas; ++r)
    if ((params[r].precond == SIM_PC_NONE) != (d.pc_none != 0)) { sim_destroy(s); return SIM_EINVAL; }
  s->warm = params[0].warm_start != 0;
  for (int r = 1; r < replicas; ++r)
    if ((params[r].warm_start != 0) != s->warm) { sim_destroy(s); return SIM_EINVAL; }
  s->tune.spmv_variant = CSR_VARIANT_DEFAULT;
  s->tune.apply_variant = CSR_VARIANT_DEFAULT;
  const size_t rows = (size_t)s->rows;
  int rc = SIM_OK;
#define ALLOC(ptr, bytes)                                      \
  if ((rc = dalloc(s, (void**)&(ptr), (bytes))) != SIM_OK) {   \
    sim_destroy(s);                                            \
    return rc;                                                 \
  }
  ALLOC(s->rep_d, sizeof(RepDev) * replicas);
  d.rep = s->rep_d;
  ALLOC(d.cg, sizeof(CgRep) * replicas);
  ALLOC(d.ctrl, sizeof(Ctrl));
  ALLOC(d.step_d, sizeof(int64_t));
  int32_t* blk_rep_d = nullptr;
  ALLOC(blk_rep_d, sizeof(int32_t) * d.nblk);
  d.blk_rep = blk_rep_d;
  ALLOC(d.partial, sizeof(double) * NPART * SUBS_PER_TILE * d.nblk);
  ALLOC(d.partial2, sizeof(double) * NPART * std::max(d.l1_total, 1));
  int32_t* l1_rep_d = nullptr;
  ALLOC(l1_rep_d, sizeof(int32_t) * std::max<size_t>(l1_rep_h.size(), 1));
  d.l1_rep = l1_rep_d;
  ALLOC(d.pos, sizeof(double4) * rows);
  ALLOC(d.pos_alt, sizeof(double4) * rows);
  ALLOC(d.cellidx, sizeof(int32_t) * rows);
  ALLOC(d.cellidx_alt, sizeof(int32_t) * rows);
  ALLOC(d.slot, sizeof(int32_t) * rows);
  ALLOC(d.cell_count, sizeof(int32_t) * d.ncell_entries);
  ALLOC(d.cell_row, sizeof(int32_t) * d.ncell_entries);
  ALLOC(s->scan_tmp, sizeof(int32_t) * d.ncell_entries);
  ALLOC(s->nbr_slots, sizeof(int32_t) * NBR_SLOTS * rows);
  ALLOC(d.rowlen, sizeof(int32_t) * (rows + 1));
  ALLOC(d.rowptr, sizeof(int32_t) * (rows + 1));
  ALLOC(d.diag, sizeof(double) * rows);
  ALLOC(d.dinv, sizeof(double) * rows);
  ALLOC(d.b, sizeof(double) * 3 * rows);
  ALLOC(d.x, sizeof(double) * 3 * rows);
  ALLOC(d.p, sizeof(double) * 3 * rows);
  ALLOC(d.r, sizeof(double) * 3 * rows);
  ALLOC(d.s, sizeof(double) * 3 * rows);
  ALLOC(d.w, sizeof(double) * 3 * rows);
  ALLOC(d.u, sizeof(double) * 3 * rows);
  ALLOC(d.vel_orig, sizeof(double) * 3 * (size_t)n_total);
  ALLOC(s->io, sizeof(double) * 3 * (size_t)n_total);
  ALLOC(s->id_off_d, sizeof(int64_t) * replicas);
  std::vector<int32_t> ccolor_h, iccells_h;
  if (s->ic0) {
    // IC(0) colours: per axis the parity of the cell coordinate, 2 for the
    // last cell of an odd axis (its neighbours on both sides have 0 and 1)
    auto axc = [](int c, int nc) { return (nc > 1 && (nc & 1) && c == nc - 1) ? 2 : (c & 1); };
    ccolor_h.assign((size_t)d.ncell_entries, -1);
    std::vector<std::vector<int32_t>> by_color(27);
    for (int r = 0; r < replicas; ++r) {
      const RepDev& R = s->reph[r];
      const int nx = R.nc[0], ny = R.nc[1], nz = R.nc[2];
      for (int c = 0; c < nx * ny * nz; ++c) {
        const int cx = c % nx, cy = (c / nx) % ny, cz = c / (nx * ny);
        const int col = axc(cx, nx) + 3 * (axc(cy, ny) + 3 * axc(cz, nz));
        const int key = R.seg_off + cell_key(R, cx, cy, cz);
        ccolor_h[(size_t)key] = col;
        by_color[col].push_back(key);
      }
    }
    s->ic_color_off.assign(1, 0);
    for (auto& v : by_color) {
      iccells_h.insert(iccells_h.end(), v.begin(), v.end());
      s->ic_color_off.push_back((int32_t)iccells_h.size());
    }
    int32_t *cc = nullptr, *ic = nullptr;
    ALLOC(cc, sizeof(int32_t) * ccolor_h.size());
    ALLOC(ic, sizeof(int32_t) * std::max<size_t>(iccells_h.size(), 1));
    d.cell_color = cc;
    d.ic_cells = ic;
    ALLOC(d.ldiag, sizeof(double) * rows);
    ALLOC(d.lnlow, sizeof(int32_t) * rows);
  }
  ALLOC(s->counter_d, sizeof(unsigned long long));
  if (s->block) {
    ALLOC(s->brep_d, sizeof(BlockRep) * replicas);
    ALLOC(s->bp.bcg, sizeof(BcgRep) * replicas);
    ALLOC(s->bp.bdiag, sizeof(double) * 6 * rows);
    ALLOC(s->bp.binv, sizeof(double) * 6 * rows);
    s->bp.brep = s->brep_d;
    s->bp.fp32 = params[0].spmv_fp32 ? 1 : 0;
  }
  {
    const int64_t m = std::max<int64_t>(s->rows + 1, d.ncell_entries);
    ALLOC(s->bsum, sizeof(int32_t) * (size_t)(scan_bsum_len(m) + 1));
  }
#undef ALLOC
  // neighbour-list capacity: twice the mean row of a uniform box, + slack
  int64_t cap = 0;
  for (int r = 0; r < replicas; ++r) {
    const double kmean = expected_entries(params[r]) / (double)params[r].n;
    cap += s->reph[r].npad * (int64_t)std::ceil(2.0 * kmean + 16.0);
  }
  if ((rc = alloc_csr(s, cap)) != SIM_OK) { sim_destroy(s); return rc; }
  if (hipHostMalloc((void**)&s->ctrl_h, sizeof(Ctrl), 0) != hipSuccess ||
      hipHostMalloc((void**)&s->cg_h, sizeof(CgRep) * replicas, 0) != hipSuccess ||
      (s->block && hipHostMalloc((void**)&s->bcg_h, sizeof(BcgRep) * replicas, 0) != hipSuccess)) {
    sim_destroy(s);
    return SIM_ENOMEM;
  }
  // uploads (synchronous: creation is not on the hot path)
  auto fail = [&](hipError_t e, const char* what) {
    sim_note_error(e, what, __LINE__);
    sim_destroy(s);
    return SIM_EDEVICE;
  };
  hipError_t e;
  if ((e = hipMemcpy(s->rep_d, s->reph.data(), sizeof(RepDev) * replicas, hipMemcpyHostToDevice)))
    return fail(e, "upload replicas");
  if ((e = hipMemcpy(blk_rep_d, s->blk_rep_h.data(), sizeof(int32_t) * d.nblk, hipMemcpyHostToDevice)))
    return fail(e, "upload block table");
  if (!l1_rep_h.empty() &&
      (e = hipMemcpy(l1_rep_d, l1_rep_h.data(), sizeof(int32_t) * l1_rep_h.size(),
                     hipMemcpyHostToDevice)))
    return fail(e, "upload reduction table");
  if (s->block) {
    std::vector<BlockRep> br((size_t)replicas);
    for (int r = 0; r < replicas; ++r) {
      br[r].a_par = fric(params[r].friction_par);
      br[r].a_perp = fric(params[r].friction_perp);
      br[r].sq_par = std::sqrt(br[r].a_par);
      br[r].sq_perp = std::sqrt(br[r].a_perp);
    }
    if ((e = hipMemcpy(s->brep_d, br.data(), sizeof(BlockRep) * replicas, hipMemcpyHostToDevice)))
      return fail(e, "upload friction tensors");
  }
  if ((e = hipMemcpy(s->id_off_d, s->id_off_h.data(), sizeof(int64_t) * replicas, hipMemcpyHostToDevice)))
    return fail(e, "upload id offsets");
  if ((e = hipMemcpy(d.pos, ph.data(), sizeof(double4) * rows, hipMemcpyHostToDevice)))
    return fail(e, "upload positions");
  if ((e = hipMemset(d.rowlen, 0, sizeof(int32_t) * (rows + 1)))) return fail(e, "clear rowlen");
  if ((e = hipMemset(d.rowptr, 0, sizeof(int32_t) * (rows + 1)))) return fail(e, "clear rowptr");
  if ((e = hipMemset(d.x, 0, sizeof(double) * 3 * rows))) return fail(e, "clear x");
  // padding rows never receive a cell: keep their cell index a valid entry
  if ((e = hipMemset(d.cellidx, 0, sizeof(int32_t) * rows))) return fail(e, "clear cells");
  if ((e = hipMemset(d.cellidx_alt, 0, sizeof(int32_t) * rows))) return fail(e, "clear cells");
  // padding rows keep u = 0 (the IC(0) and learned passes write real rows only)
  if ((e = hipMemset(d.u, 0, sizeof(double) * 3 * rows))) return fail(e, "clear u");
  if (s->ic0) {
    if ((e = hipMemcpy((void*)d.cell_color, ccolor_h.data(), sizeof(int32_t) * ccolor_h.size(),
                       hipMemcpyHostToDevice)))
      return fail(e, "upload cell colours");
    if (!iccells_h.empty() &&
        (e = hipMemcpy((void*)d.ic_cells, iccells_h.data(), sizeof(int32_t) * iccells_h.size(),
                       hipMemcpyHostToDevice)))
      return fail(e, "upload colour lists");
    if ((e = hipMemset(d.lnlow, 0, sizeof(int32_t) * rows))) return fail(e, "clear L");
    if ((e = hipMemset(d.ldiag, 0, sizeof(double) * rows))) return fail(e, "clear L");
  }
  if ((e = hipMemset(d.vel_orig, 0, sizeof(double) * 3 * n_total))) return fail(e, "clear vel");
  if ((e = hipMemset(d.ctrl, 0, sizeof(Ctrl)))) return fail(e, "clear ctrl");
  if ((e = hipMemset(d.step_d, 0, sizeof(int64_t)))) return fail(e, "clear step");
  if ((e = hipMemset(d.cg, 0, sizeof(CgRep) * replicas))) return fail(e, "clear cg");
  // padding rows of the second position buffer stay inert too
  if ((e = hipMemcpy(d.pos_alt, ph.data(), sizeof(double4) * rows, hipMemcpyHostToDevice)))
    return fail(e, "upload positions");
  if ((e = hipDeviceSynchronize())) return fail(e, "synchronize");
  *out = s;
  return SIM_OK;
}

int sim_create(const sim_params* params, const double* pos0, sim_t** out) {
  return sim_create_batch(params, 1, pos0, out);
}

int sim_set_stream(sim_t* s, void* stream) {
  if (!s) return SIM_EINVAL;
  s->stream = (hipStream_t)stream;
  if (!s->stream && s->graph_mode) s->stream = s->own_stream;  // graphs need a capturable stream
  return SIM_OK;
}

int sim_graph_mode(sim_t* s, int32_t on) {
  if (!s || (on != 0 && on != 1)) return SIM_EINVAL;
  if (hipSetDevice(s->device) != hipSuccess) return SIM_EDEVICE;
  if (on && !s->stream) {
    if (!s->own_stream) HIPCHK(hipStreamCreateWithFlags(&s->own_stream, hipStreamDefault));
    s->stream = s->own_stream;
  }
  if (!on) {
    HIPCHK(hipStreamSynchronize(s->stream));
    drop_graphs(s);
  }
  s->graph_mode = on;
  return SIM_OK;
}

int sim_graph_info(sim_t* s, int64_t* captures, int64_t* replays) {
  if (!s) return SIM_EINVAL;
  if (captures) *captures = s->graph_captures;
  if (replays) *replays = s->graph_replays;
  return SIM_OK;
}

static bool valid_variant(int32_t v) { return v >= 0 && v < CSR_VARIANTS; }

int sim_set_tuning(sim_t* s, const sim_tuning* t) {
  if (!s || !t || !valid_variant(t->spmv_variant) || !valid_variant(t->apply_variant) ||
      (t->vec_variant != 0 && t->vec_variant != 1))
    return SIM_EINVAL;
  s->tune.spmv_variant = t->spmv_variant;
  s->tune.apply_variant = t->apply_variant;
  s->tune.vec_variant = t->vec_variant;
  s->d.spmv_var = t->spmv_variant;
  s->d.apply_var = t->apply_variant;
  s->d.vec_nt = t->vec_variant;
  drop_graphs(s);
  return SIM_OK;
}

int sim_autotune(sim_t* s, int32_t reps, sim_tuning* out) {
  if (!s || reps < 1) return SIM_EINVAL;
  if (s->block) return SIM_ENOTSUP;  // the variants tune the scalar CSR products
  if (hipSetDevice(s->device) != hipSuccess) return SIM_EDEVICE;
  int rc = build_checked(s);
  if (rc) return rc;
  DevPtrs& d = s->d;
  if (s->learned) {
    if ((rc = ensure_mp(s, false))) return rc;
    s->mp.store_train = 0;
    HIPCHK(launch_mp_forward(d, s->mp, s->stream));
  }
  s->system_valid = false;
  // u = M^-1 b for every component (a fresh CG start), then time the products
  d.learned = s->learned ? 1 : 0;
  HIPCHK(launch_cg_reset(d, 0.0, s->stream));
  HIPCHK(launch_cg_vec(d, 0, s->stream));
  if (d.learned) HIPCHK(launch_cg_apply(d, 0, s->stream));
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreateWithFlags(&e0, hipEventDisableSystemFence));
  HIPCHK(hipEventCreateWithFlags(&e1, hipEventDisableSystemFence));
  sim_tuning t{};
  int kinds = d.learned ? 2 : 1;
  hipError_t err = hipSuccess;
  for (int kind = 0; kind < kinds && err == hipSuccess; ++kind) {
    float best = 0.0f;
    int pick = CSR_VARIANT_DEFAULT;
    for (int v = 0; v < CSR_VARIANTS && err == hipSuccess; ++v) {
      if (kind == 0) d.spmv_var = v;
      else d.apply_var = v;
      auto once = [&]() {
        return kind == 0 ? launch_cg_spmv(d, 0, 0, s->stream) : launch_cg_apply(d, 0, s->stream);
      };
      if ((err = once())) break;  // untimed warm-up
      if ((err = hipEventRecord(e0, s->stream))) break;
      for (int k = 0; k < reps && err == hipSuccess; ++k) err = once();
      if (err || (err = hipEventRecord(e1, s->stream)) || (err = hipEventSynchronize(e1))) break;
      float ms = 0.0f;
      if ((err = hipEventElapsedTime(&ms, e0, e1))) break;
      const float us = 1000.0f * ms / (float)reps;
      (kind == 0 ? t.spmv_us : t.apply_us)[v] = us;
      if (v == 0 || us < best) { best = us; pick = v; }
    }
    if (kind == 0) t.spmv_variant = pick;
    else t.apply_variant = pick;
  }
  // the vector kernel with ordinary and with nontemporal accesses (its
  // iteration form; the values it leaves do not matter here)
  for (int v = 0; v < 2 && err == hipSuccess; ++v) {
    d.vec_nt = v;
    if ((err = launch_cg_vec(d, 2, s->stream))) break;  // untimed warm-up
    if ((err = hipEventRecord(e0, s->stream))) break;
    for (int k = 0; k < reps && err == hipSuccess; ++k) err = launch_cg_vec(d, 2, s->stream);
    if (err || (err = hipEventRecord(e1, s->stream)) || (err = hipEventSynchronize(e1))) break;
    float ms = 0.0f;
    if ((err = hipEventElapsedTime(&ms, e0, e1))) break;
    t.vec_us[v] = 1000.0f * ms / (float)reps;
  }
  t.vec_variant = t.vec_us[1] < t.vec_us[0] ? 1 : 0;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  d.learned = 0;
  if (err != hipSuccess) {
    d.spmv_var = s->tune.spmv_variant;
    d.apply_var = s->tune.apply_variant;
    d.vec_nt = s->tune.vec_variant;
    sim_note_error(err, "autotune", __LINE__);
    return SIM_EDEVICE;
  }
  if (!s->learned) t.apply_variant = s->tune.apply_variant;
  s->tune = t;
  d.spmv_var = t.spmv_variant;
  d.apply_var = t.apply_variant;
  d.vec_nt = t.vec_variant;
  drop_graphs(s);
  if (out) *out = t;
  return SIM_OK;
}

// parameter counts the weight calls take: the scalar network, or it and the
// 3 x 3 heads of the block system
static bool weight_count_ok(int64_t count) {
  return count == MP_NPARAMS || count == MP_NPARAMS_ALL;
}

int sim_precond_weights(sim_t* s, float* theta, int64_t count, int32_t set) {
  if (!s || !theta || !weight_count_ok(count)) return SIM_EINVAL;
  if (hipSetDevice(s->device) != hipSuccess) return SIM_EDEVICE;
  int rc = ensure_mp(s, false);
  if (rc) return rc;
  if (set) {
    HIPCHK(hipMemcpy(s->mp.th32, theta, sizeof(float) * (size_t)count, hipMemcpyHostToDevice));
    HIPCHK(hipMemset(s->mp.am, 0, sizeof(float) * MP_NPARAMS_ALL));
    HIPCHK(hipMemset(s->mp.av, 0, sizeof(float) * MP_NPARAMS_ALL));
    s->mp_adam_t = 0;
    HIPCHK(launch_mp_cast(s->mp, s->stream));
    HIPCHK(hipStreamSynchronize(s->stream));
  } else {
    HIPCHK(hipMemcpy(theta, s->mp.th32, sizeof(float) * (size_t)count, hipMemcpyDeviceToHost));
  }
  return SIM_OK;
}

int sim_precond_config(sim_t* s, int32_t round_act, int32_t learned_maxit) {
  if (!s || (round_act != 0 && round_act != 1) || learned_maxit < 0) return SIM_EINVAL;
  if (hipSetDevice(s->device) != hipSuccess) return SIM_EDEVICE;
  int rc = ensure_mp(s, false);
  if (rc) return rc;
  s->mp.round_act = round_act;
  s->learned_maxit = learned_maxit;
  return SIM_OK;
}

int sim_precond_floor(sim_t* s, double lam_floor) {
  if (!s || !(lam_floor >= 0.0) || !std::isfinite(lam_floor)) return SIM_EINVAL;
  if (hipSetDevice(s->device) != hipSuccess) return SIM_EDEVICE;
  int rc = ensure_mp(s, false);
  if (rc) return rc;
  s->mp.lam_floor = lam_floor;
  return SIM_OK;
}

int sim_load_precond(sim_t* s, const char* path) {
  if (!s || !path) return SIM_EINVAL;
  FILE* f = std::fopen(path, "rb");
  if (!f) return SIM_EINVAL;
  char magic[8];
  int64_t count = 0;
  std::vector<float> th(MP_NPARAMS_ALL);
  const bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, "SIMPC001", 8) == 0 &&
                  std::fread(&count, sizeof(count), 1, f) == 1 && weight_count_ok(count) &&
                  std::fread(th.data(), sizeof(float), (size_t)count, f) == (size_t)count;
  std::fclose(f);
  if (!ok) return SIM_EINVAL;
  return sim_precond_weights(s, th.data(), count, 1);
}

// training on a system built before the handle had network buffers: the
// pair terms did not write the edge input then
static int no_edge_input() {
  snprintf(g_last_error, sizeof(g_last_error),
           "the system was built before any preconditioner call on this handle: set the "
           "weights (or configure the network) before the step or solve that training uses");
  return SIM_EINVAL;
}

// network forward, loss and backward on the system (b, x*) of dp
static int train_pass(sim_t* s, const DevPtrs& dp, const MpPtrs& mq) {
  if (s->block) {
    HIPCHK(launch_mp_trunk(dp, mq, s->stream));
    HIPCHK(launch_mpb_heads(dp, mq, s->bp, s->stream));
    HIPCHK(launch_mpb_loss(dp, mq, s->bp, s->stream));
    HIPCHK(launch_mpb_backward(dp, mq, s->bp, s->stream));
  } else {
    HIPCHK(launch_mp_forward(dp, mq, s->stream));
    HIPCHK(launch_mp_loss(dp, mq, s->stream));
    HIPCHK(launch_mp_backward(dp, mq, s->stream));
  }
  return SIM_OK;
}

int sim_train_step(sim_t* s, double lr, double* loss) {
  if (!s || !(lr >= 0.0)) return SIM_EINVAL;
  if (s->R != 1) return SIM_ENOTSUP;  // one system: the solution loss of one replica
  if (!s->system_valid) return SIM_EINVAL;
  if (!s->er_built) return no_edge_input();
  if (hipSetDevice(s->device) != hipSuccess) return SIM_EDEVICE;
  int rc = ensure_mp(s, true);
  if (rc) return rc;
  s->mp.store_train = 1;
  if ((rc = train_pass(s, s->d, s->mp))) return rc;
  if (lr > 0.0) HIPCHK(launch_mp_adam(s->mp, (float)lr, ++s->mp_adam_t, s->stream));
  double l[2] = {0.0, 0.0};
  HIPCHK(hipMemcpyAsync(l, s->mp.loss, sizeof(l), hipMemcpyDeviceToHost, s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  if (loss) *loss = l[0];
  return std::isfinite(l[0]) ? SIM_OK : SIM_ENUMERIC;
}

int sim_train_probe(sim_t* s, double lr, uint64_t seed, uint64_t index, int32_t euclid,
                    double* loss) {
  if (!s || !(lr >= 0.0) || (euclid != 0 && euclid != 1)) return SIM_EINVAL;
  if (!s->system_valid) return SIM_EINVAL;
  if (!s->er_built) return no_edge_input();
  if (hipSetDevice(s->device) != hipSuccess) return SIM_EDEVICE;
  int rc = ensure_mp(s, true);
  if (rc) return rc;
  s->mp.store_train = 1;
  // the loss kernels read b and x* through the device-pointer block: point
  // them at the probe (the solve's b and x stay untouched)
  DevPtrs dp = s->d;
  dp.x = s->mp.pz;
  dp.b = s->mp.pb;
  MpPtrs mq = s->mp;
  mq.loss_euclid = euclid;
  if (s->block)
    HIPCHK(launch_mpb_probe(dp, s->bp, s->mp.pz, s->mp.pb, seed, index, s->stream));
  else
    HIPCHK(launch_mp_probe(dp, s->mp.pz, s->mp.pb, seed, index, s->stream));
  if ((rc = train_pass(s, dp, mq))) return rc;
  if (lr > 0.0) HIPCHK(launch_mp_adam(s->mp, (float)lr, ++s->mp_adam_t, s->stream));
  double l[2] = {0.0, 0.0};
  HIPCHK(hipMemcpyAsync(l, s->mp.loss, sizeof(l), hipMemcpyDeviceToHost, s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  if (loss) *loss = l[0];
  return std::isfinite(l[0]) ? SIM_OK : SIM_ENUMERIC;
}

int sim_precond_optimizer(sim_t* s, float* m1, float* m2, int64_t count, int32_t* t, int32_t set) {
  if (!s || !m1 || !m2 || !t || !weight_count_ok(count) || (set && *t < 0)) return SIM_EINVAL;
  if (hipSetDevice(s->device) != hipSuccess) return SIM_EDEVICE;
  int rc = ensure_mp(s, false);
  if (rc) return rc;
  const size_t bytes = sizeof(float) * (size_t)count;
  if (set) {
    HIPCHK(hipMemcpy(s->mp.am, m1, bytes, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(s->mp.av, m2, bytes, hipMemcpyHostToDevice));
    s->mp_adam_t = *t;
  } else {
    HIPCHK(hipMemcpy(m1, s->mp.am, bytes, hipMemcpyDeviceToHost));
    HIPCHK(hipMemcpy(m2, s->mp.av, bytes, hipMemcpyDeviceToHost));
    *t = s->mp_adam_t;
  }
  return SIM_OK;
}

int sim_precond_grad(sim_t* s, float* grad, int64_t count) {
  if (!s || !grad || !weight_count_ok(count) || !s->mp_ready) return SIM_EINVAL;
  if (hipSetDevice(s->device) != hipSuccess) return SIM_EDEVICE;
  HIPCHK(hipMemcpy(grad, s->mp.grad, sizeof(float) * (size_t)count, hipMemcpyDeviceToHost));
  return SIM_OK;
}

int sim_debug_precond(sim_t* s, int64_t* rows, int64_t* cols, double* vals, int64_t cap,
                      int64_t* count, double* mdiag) {
  if (!s || !count || cap < 0) return SIM_EINVAL;
  if (cap > 0 && (!rows || !cols || !vals)) return SIM_EINVAL;
  if (hipSetDevice(s->device) != hipSuccess) return SIM_EDEVICE;
  if (!s->learned && !s->ic0) return SIM_ENOTSUP;
  int rc = build_checked(s);
  if (rc) return rc;
  if (s->learned) {
    if ((rc = ensure_mp(s, false))) return rc;
    s->mp.store_train = 0;
    if (s->block) {
      HIPCHK(launch_mp_trunk(s->d, s->mp, s->stream));
      HIPCHK(launch_mpb_heads(s->d, s->mp, s->bp, s->stream));
    } else {
      HIPCHK(launch_mp_forward(s->d, s->mp, s->stream));
    }
  } else {
    HIPCHK(launch_ic_factor(s->d, s->ic_color_off.data(), (int)s->ic_color_off.size() - 1,
                            s->stream));
  }
  const int64_t nnz = s->ctrl_h->nnz;
  *count = nnz;
  if (nnz > cap) return SIM_ECAPACITY;
  const size_t per = s->block ? 9 : 1;  // values per entry and per particle
  int64_t *r_d = nullptr, *c_d = nullptr;
  double *v_d = nullptr, *dg_d = nullptr;
  const size_t m = (size_t)std::max<int64_t>(nnz, 1);
  if ((rc = dalloc(s, (void**)&r_d, sizeof(int64_t) * m))) return rc;
  if ((rc = dalloc(s, (void**)&c_d, sizeof(int64_t) * m))) return rc;
  if ((rc = dalloc(s, (void**)&v_d, sizeof(double) * per * m))) return rc;
  if ((rc = dalloc(s, (void**)&dg_d, sizeof(double) * per * (size_t)s->n_total))) return rc;
  if (s->learned && s->block)
    HIPCHK(launch_mpb_export(s->d, s->bp, s->id_off_d, r_d, c_d, v_d, nnz, dg_d, s->stream));
  else if (s->learned)
    HIPCHK(launch_mp_export(s->d, s->mp, s->id_off_d, r_d, c_d, v_d, nnz, dg_d, s->stream));
  else
    HIPCHK(launch_ic_export(s->d, s->id_off_d, r_d, c_d, v_d, dg_d, s->stream));
  if (nnz > 0) {
    HIPCHK(hipMemcpyAsync(rows, r_d, sizeof(int64_t) * nnz, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipMemcpyAsync(cols, c_d, sizeof(int64_t) * nnz, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipMemcpyAsync(vals, v_d, sizeof(double) * per * nnz, hipMemcpyDeviceToHost,
                          s->stream));
  }
  if (mdiag)
    HIPCHK(hipMemcpyAsync(mdiag, dg_d, sizeof(double) * per * s->n_total, hipMemcpyDeviceToHost,
                          s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  dfree(s, r_d);
  dfree(s, c_d);
  dfree(s, v_d);
  dfree(s, dg_d);
  return SIM_OK;
}

// a7 on the host's word: update, numeric check, velocities, n -> n + 1
static int commit_step(sim_t* s, sim_stats* st) {
  HIPCHK(launch_update(s->d, 0, s->stream));
  int rc = read_ctrl(s, false);
  if (rc) return rc;
  if (s->ctrl_h->numeric) return SIM_ENUMERIC;
  HIPCHK(launch_save_vel(s->d, s->id_off_d, 0, s->stream));
  HIPCHK(launch_step_commit(s->d, 0, s->stream));
  std::swap(s->d.pos, s->d.pos_alt);
  s->step += 1;
  s->vv_valid = true;
  if (st) st->steps_done += 1;
  return SIM_OK;
}

// ---------------------------------------------------------------------------
// step graphs: one HIP graph holds a whole step -- build, learned forward,
// CG start, the first K iterations and a check round, then the update, the
// velocity export and n -> n + 1, the last three conditional on the device
// (they do nothing unless every component converged).  The host then polls
// once; a solve that needs more iterations continues with host-queued chunks
// and an eager commit, exactly as without graphs, so both paths give the
// same bits.  A graph is keyed by the device pointers and configuration it
// was captured from; the two position/cell buffers alternate, so at most
// two graphs are live per configuration.
// ---------------------------------------------------------------------------
// iterations recorded before the check: at least the last solve's count + 1;
// kept while it stays within 12 of that (the excess iterations of converged
// replicas return at once), else reset to the count + 4 rounded up to a
// multiple of 4, so that the usual step-to-step changes need no new capture
static int graph_iters(sim_t* s) {
  const int need = s->last_iters + 1;
  if (s->graph_K < need || s->graph_K > need + 12) s->graph_K = ((need + 4 + 3) / 4) * 4;
  return s->graph_K;
}

static bool same_bytes(const void* a, const void* b, size_t n) { return std::memcmp(a, b, n) == 0; }

static int queue_graph_step(sim_t* s, int K) {
  int rc = build_system(s);
  if (rc) return rc;
  if (s->learned) HIPCHK(launch_mp_forward(s->d, s->mp, s->stream));
  if (s->ic0)
    HIPCHK(launch_ic_factor(s->d, s->ic_color_off.data(), (int)s->ic_color_off.size() - 1,
                            s->stream));
  if ((rc = cg_queue_start(s, 0.0, s->warm))) return rc;
  if ((rc = cg_queue_chunk(s, K, 0, false))) return rc;
  HIPCHK(launch_update(s->d, 1, s->stream));
  HIPCHK(launch_save_vel(s->d, s->id_off_d, 1, s->stream));
  HIPCHK(launch_step_commit(s->d, 1, s->stream));
  return SIM_OK;
}

static int step_graph(sim_t* s, sim_stats* st) {
  int rc;
  if (s->learned) {
    if ((rc = ensure_mp(s, false))) return rc;
    s->mp.store_train = 0;
    s->d.learned = 1;
  }
  const int K = graph_iters(s);
  const DevPtrs key_d = s->d;
  const MpPtrs key_m = s->mp;
  sim_t::StepGraph* g = nullptr;
  for (auto& c : s->graphs)
    if (c.K == K && c.learned == s->learned && same_bytes(&c.d, &key_d, sizeof(DevPtrs)) &&
        same_bytes(&c.m, &key_m, sizeof(MpPtrs)))
      g = &c;
  if (!g) {
    HIPCHK(hipStreamBeginCapture(s->stream, hipStreamCaptureModeThreadLocal));
    rc = queue_graph_step(s, K);
    hipGraph_t graph = nullptr;
    const hipError_t e = hipStreamEndCapture(s->stream, &graph);
    hipGraphExec_t exec = nullptr;
    hipError_t ei = hipSuccess;
    if (!rc && e == hipSuccess) ei = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    if (graph) (void)hipGraphDestroy(graph);
    if (rc || e != hipSuccess || ei != hipSuccess) {
      s->d = key_d;  // nothing ran: undo the host-side buffer swaps of the capture
      if (rc) return rc;
      sim_note_error(e != hipSuccess ? e : ei, "step graph capture", __LINE__);
      return SIM_EDEVICE;
    }
    if (s->graphs.size() >= 4) {
      (void)hipGraphExecDestroy(s->graphs.front().exec);
      s->graphs.erase(s->graphs.begin());
    }
    s->graphs.push_back({exec, key_d, key_m, K, s->learned});
    g = &s->graphs.back();
    s->graph_captures += 1;
  } else {
    // the host-side effects of build_system
    std::swap(s->d.pos, s->d.pos_alt);
    std::swap(s->d.cellidx, s->d.cellidx_alt);
  }
  s->system_valid = false;
  HIPCHK(hipGraphLaunch(g->exec, s->stream));
  s->graph_replays += 1;
  bool committed = false;
  rc = cg_poll_loop(s, K, st, &committed);
  if (rc == SIM_OK && committed) {
    // update, velocities and n -> n + 1 already ran inside the graph
    if (s->ctrl_h->numeric) return SIM_ENUMERIC;
    s->system_valid = true;
    std::swap(s->d.pos, s->d.pos_alt);
    s->step += 1;
    s->vv_valid = true;
    if (st) st->steps_done += 1;
    return SIM_OK;
  }
  if (s->learned && (rc == SIM_ESTALL_INTERNAL || rc == SIM_EBREAKDOWN || rc == SIM_ENOCONV)) {
    s->d.learned = 0;
    rc = cg_solve(s, 0.0, s->warm, st);
    s->d.learned = 1;
    if (st) st->fallback = 1;
  }
  if (rc == SIM_EOVERFLOW_INTERNAL) {
    // grow the neighbour list and solve eagerly (the graphs are stale)
    drop_graphs(s);
    for (int attempt = 0; attempt < 4 && rc == SIM_EOVERFLOW_INTERNAL; ++attempt) {
      if ((rc = grow_and_refill(s))) return rc;
      if ((rc = prepare_precond(s))) return rc;
      rc = cg_solve(s, 0.0, s->warm, st);
      if (s->learned && (rc == SIM_ESTALL_INTERNAL || rc == SIM_EBREAKDOWN || rc == SIM_ENOCONV)) {
        s->d.learned = 0;
        rc = cg_solve(s, 0.0, s->warm, st);
        s->d.learned = 1;
        if (st) st->fallback = 1;
      }
    }
    if (rc == SIM_EOVERFLOW_INTERNAL) return SIM_ENOMEM;
  }
  if (rc) return rc;
  s->system_valid = true;
  return commit_step(s, st);
}

int sim_step(sim_t* s, int32_t nsteps, sim_stats* st) {
  if (!s || nsteps < 0) return SIM_EINVAL;
  if (hipSetDevice(s->device) != hipSuccess) return SIM_EDEVICE;
  if (st) std::memset(st, 0, sizeof(*st));
  for (int32_t k = 0; k < nsteps; ++k) {
    // graphs need a solve count to size the first chunk; with the timing
    // probe on, every prof_every-th step runs eagerly so its kernels are timed
    const bool probe_step = s->prof_every > 0 && s->step % s->prof_every == 0;
    if (s->graph_mode && s->last_iters > 0 && !probe_step && !s->block) {
      int rc = step_graph(s, st);
      if (rc) return rc;
      continue;
    }
    int rc = build_and_solve(s, false, 0.0, st);
    if (rc) return rc;
    if ((rc = commit_step(s, st))) return rc;
  }
  return SIM_OK;
}

int sim_solve(sim_t* s, const double* b, double* v, double tol, uint32_t flags, sim_stats* st) {
  if (!s || !b || !v) return SIM_EINVAL;
  if (hipSetDevice(s->device) != hipSuccess) return SIM_EDEVICE;
  if (st) std::memset(st, 0, sizeof(*st));
  const size_t bytes = sizeof(double) * 3 * (size_t)s->n_total;
  const bool dev = flags & SIM_DEVICE_PTR;
  HIPCHK(hipMemcpyAsync(s->io, b, bytes, dev ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                        s->stream));
  int rc = build_and_solve(s, true, tol, st);
  if (rc) return rc;
  HIPCHK(launch_permute(s->d, s->id_off_d, 2, nullptr, s->io, s->stream));
  HIPCHK(hipMemcpyAsync(v, s->io, bytes, dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                        s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  return SIM_OK;
}

int sim_state(sim_t* s, double* pos, double* vel, sim_meta* meta, uint32_t flags) {
  if (!s) return SIM_EINVAL;
  if (hipSetDevice(s->device) != hipSuccess) return SIM_EDEVICE;
  const size_t bytes = sizeof(double) * 3 * (size_t)s->n_total;
  const bool dev = flags & SIM_DEVICE_PTR;
  if (pos) {
    HIPCHK(launch_permute(s->d, s->id_off_d, 0, nullptr, s->io, s->stream));
    HIPCHK(hipMemcpyAsync(pos, s->io, bytes, dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost,
                          s->stream));
  }
  if (vel)
    HIPCHK(hipMemcpyAsync(vel, s->d.vel_orig, bytes,
                          dev ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  if (meta) {
    meta->step = s->step;
    meta->time = (double)s->step * s->prm[0].dt;
    meta->le_offset = host_le_offset(s->prm[0], s->step);
    meta->replicas = s->R;
    meta->reserved0 = 0;
    meta->n_total = s->n_total;
  }
  return SIM_OK;
}

int sim_debug_pairs(sim_t* s, int64_t* ijr, int64_t cap, int64_t* count) {
  if (!s || !count || cap < 0 || (cap > 0 && !ijr)) return SIM_EINVAL;
  if (hipSetDevice(s->device) != hipSuccess) return SIM_EDEVICE;
  int rc = build_checked(s);
  if (rc) return rc;
  const int64_t npairs = s->ctrl_h->nnz / 2;
  *count = npairs;
  if (npairs > cap) return SIM_ECAPACITY;
  int64_t* buf = nullptr;
  if ((rc = dalloc(s, (void**)&buf, sizeof(int64_t) * 3 * (size_t)std::max<int64_t>(npairs, 1))))
    return rc;
  HIPCHK(hipMemsetAsync(s->counter_d, 0, sizeof(unsigned long long), s->stream));
  HIPCHK(launch_export_pairs(s->d, buf, npairs, s->counter_d, s->stream));
  HIPCHK(hipMemcpyAsync(ijr, buf, sizeof(int64_t) * 3 * (size_t)npairs, hipMemcpyDeviceToHost,
                        s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  dfree(s, buf);
  return SIM_OK;
}

int sim_debug_block_system(sim_t* s, int64_t* rows, int64_t* cols, double* vals, int64_t cap,
                           int64_t* count, double* diag, double* rhs) {
  if (!s || !count || cap < 0) return SIM_EINVAL;
  if (cap > 0 && (!rows || !cols || !vals)) return SIM_EINVAL;
  if (!s->block) return SIM_ENOTSUP;
  if (hipSetDevice(s->device) != hipSuccess) return SIM_EDEVICE;
  int rc = build_checked(s);
  if (rc) return rc;
  const int64_t nnz = s->ctrl_h->nnz;
  *count = nnz;
  if (nnz > cap) return SIM_ECAPACITY;
  int64_t *r_d = nullptr, *c_d = nullptr;
  double *v_d = nullptr, *dg_d = nullptr, *b_d = nullptr;
  const size_t m = (size_t)std::max<int64_t>(nnz, 1);
  if ((rc = dalloc(s, (void**)&r_d, sizeof(int64_t) * m))) return rc;
  if ((rc = dalloc(s, (void**)&c_d, sizeof(int64_t) * m))) return rc;
  if ((rc = dalloc(s, (void**)&v_d, sizeof(double) * 9 * m))) return rc;
  if ((rc = dalloc(s, (void**)&dg_d, sizeof(double) * 9 * (size_t)s->n_total))) return rc;
  if ((rc = dalloc(s, (void**)&b_d, sizeof(double) * 3 * (size_t)s->n_total))) return rc;
  HIPCHK(launch_block_export(s->d, s->bp, s->id_off_d, r_d, c_d, v_d, dg_d, b_d, s->stream));
  if (nnz > 0) {
    HIPCHK(hipMemcpyAsync(rows, r_d, sizeof(int64_t) * nnz, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipMemcpyAsync(cols, c_d, sizeof(int64_t) * nnz, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipMemcpyAsync(vals, v_d, sizeof(double) * 9 * nnz, hipMemcpyDeviceToHost, s->stream));
  }
  if (diag)
    HIPCHK(hipMemcpyAsync(diag, dg_d, sizeof(double) * 9 * s->n_total, hipMemcpyDeviceToHost,
                          s->stream));
  if (rhs)
    HIPCHK(hipMemcpyAsync(rhs, b_d, sizeof(double) * 3 * s->n_total, hipMemcpyDeviceToHost, s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  dfree(s, r_d);
  dfree(s, c_d);
  dfree(s, v_d);
  dfree(s, dg_d);
  dfree(s, b_d);
  return SIM_OK;
}

int sim_debug_system(sim_t* s, int64_t* rows, int64_t* cols, double* vals, int64_t cap,
                     int64_t* count, double* diag, double* rhs) {
  if (!s || !count || cap < 0) return SIM_EINVAL;
  if (s->block) return SIM_ENOTSUP;
  if (cap > 0 && (!rows || !cols || !vals)) return SIM_EINVAL;
  if (hipSetDevice(s->device) != hipSuccess) return SIM_EDEVICE;
  int rc = build_checked(s);
  if (rc) return rc;
  const int64_t nnz = s->ctrl_h->nnz;
  *count = nnz;
  if (nnz > cap) return SIM_ECAPACITY;
  int64_t *r_d = nullptr, *c_d = nullptr;
  double *v_d = nullptr, *dg_d = nullptr, *b_d = nullptr;
  const size_t m = (size_t)std::max<int64_t>(nnz, 1);
  if ((rc = dalloc(s, (void**)&r_d, sizeof(int64_t) * m))) return rc;
  if ((rc = dalloc(s, (void**)&c_d, sizeof(int64_t) * m))) return rc;
  if ((rc = dalloc(s, (void**)&v_d, sizeof(double) * m))) return rc;
  if ((rc = dalloc(s, (void**)&dg_d, sizeof(double) * (size_t)s->n_total))) return rc;
  if ((rc = dalloc(s, (void**)&b_d, sizeof(double) * 3 * (size_t)s->n_total))) return rc;
  HIPCHK(launch_export_system(s->d, s->id_off_d, r_d, c_d, v_d, nnz, dg_d, b_d, s->stream));
  if (nnz > 0) {
    HIPCHK(hipMemcpyAsync(rows, r_d, sizeof(int64_t) * nnz, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipMemcpyAsync(cols, c_d, sizeof(int64_t) * nnz, hipMemcpyDeviceToHost, s->stream));
    HIPCHK(hipMemcpyAsync(vals, v_d, sizeof(double) * nnz, hipMemcpyDeviceToHost, s->stream));
  }
  if (diag)
    HIPCHK(hipMemcpyAsync(diag, dg_d, sizeof(double) * s->n_total, hipMemcpyDeviceToHost, s->stream));
  if (rhs)
    HIPCHK(hipMemcpyAsync(rhs, b_d, sizeof(double) * 3 * s->n_total, hipMemcpyDeviceToHost, s->stream));
  HIPCHK(hipStreamSynchronize(s->stream));
  dfree(s, r_d);
  dfree(s, c_d);
  dfree(s, v_d);
  dfree(s, dg_d);
  dfree(s, b_d);
  return SIM_OK;
}

int sim_profile_enable(sim_t* s, int32_t sample_every) {
  if (!s || sample_every < 0) return SIM_EINVAL;
  if (hipSetDevice(s->device) != hipSuccess) return SIM_EDEVICE;
  if (sample_every > 0 && s->prof_ev.empty()) {
    s->prof_ev.resize(2 * kProfKernels * 256);
    // timing-only events: no system-scope fence (cache write-back and
    // invalidation) when they complete, which would lengthen and perturb
    // the bracketed kernel; they are read after the solve's own sync
    for (auto& e : s->prof_ev) HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
    s->prof_run_ev.resize(1025);
    for (auto& e : s->prof_run_ev)
      HIPCHK(hipEventCreateWithFlags(&e, hipEventDisableSystemFence));
  }
  s->prof_every = sample_every;
  s->prof_phase = 0;
  s->prof_solves = 0;
  return SIM_OK;
}

int sim_profile_read(sim_t* s, sim_kernel_prof* out, int32_t cap, int32_t* count, int32_t reset) {
  if (!s || !count || cap < 0 || (cap > 0 && !out)) return SIM_EINVAL;
  *count = kProfKernels;
  for (int k = 0; k < kProfKernels && k < cap; ++k) {
    out[k] = s->prof_acc[k];
    std::snprintf(out[k].name, sizeof(out[k].name), "%s", kProfNames[k]);
  }
  if (reset) std::memset(s->prof_acc, 0, sizeof(s->prof_acc));
  return cap < kProfKernels ? SIM_ECAPACITY : SIM_OK;
}

int sim_copy_probe(const void* src, void* dst, int64_t bytes, int32_t reps, void* stream,
                   double* ms_avg) {
  if (!src || !dst || bytes <= 0 || bytes % 16 || reps < 1 || !ms_avg) return SIM_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  hipEvent_t e0, e1;
  HIPCHK(hipEventCreateWithFlags(&e0, hipEventDisableSystemFence));
  HIPCHK(hipEventCreateWithFlags(&e1, hipEventDisableSystemFence));
  HIPCHK(launch_copy16(src, dst, bytes, st));  // untimed first touch
  HIPCHK(hipEventRecord(e0, st));
  for (int k = 0; k < reps; ++k) HIPCHK(launch_copy16(src, dst, bytes, st));
  HIPCHK(hipEventRecord(e1, st));
  HIPCHK(hipEventSynchronize(e1));
  float ms = 0.0f;
  HIPCHK(hipEventElapsedTime(&ms, e0, e1));
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  *ms_avg = (double)ms / reps;
  return SIM_OK;
}

int sim_event_probe(const void* src, void* dst, int64_t bytes, int32_t reps, void* stream,
                    double* ms_chain, double* ms_each) {
  if (!src || !dst || bytes <= 0 || bytes % 16 || reps < 1 || reps > 256 || !ms_chain || !ms_each)
    return SIM_EINVAL;
  hipStream_t st = (hipStream_t)stream;
  std::vector<hipEvent_t> ev(2 * (size_t)reps + 2, nullptr);
  hipError_t err = hipSuccess;
  for (auto& e : ev)
    if ((err = hipEventCreateWithFlags(&e, hipEventDisableSystemFence))) break;
  float chain = 0.0f, each = 0.0f;
  if (!err) err = launch_copy16(src, dst, bytes, st);  // untimed first touch
  // a chain of reps copies between one event pair
  if (!err) err = hipEventRecord(ev[0], st);
  for (int k = 0; k < reps && !err; ++k) err = launch_copy16(src, dst, bytes, st);
  if (!err) err = hipEventRecord(ev[1], st);
  // reps copies, each after an untimed one and between its own launch-bound
  // pair, as the kernel timing probe times the CG kernels
  for (int k = 0; k < reps && !err; ++k) {
    err = launch_copy16(src, dst, bytes, st);
    if (!err) err = launch_copy16(src, dst, bytes, st, ev[2 + 2 * k], ev[3 + 2 * k]);
  }
  if (!err) err = hipStreamSynchronize(st);
  if (!err) err = hipEventElapsedTime(&chain, ev[0], ev[1]);
  for (int k = 0; k < reps && !err; ++k) {
    float ms = 0.0f;
    err = hipEventElapsedTime(&ms, ev[2 + 2 * k], ev[3 + 2 * k]);
    each += ms;
  }
  for (auto& e : ev)
    if (e) (void)hipEventDestroy(e);
  if (err) {
    sim_note_error(err, "event probe", __LINE__);
    return SIM_EDEVICE;
  }
  *ms_chain = (double)chain / reps;
  *ms_each = (double)each / reps;
  return SIM_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free structure factor: the chunk table and partial sums live in
// one file-scope device array, `scratch`, shared by every call on a GPU.  In
// host code the array's name is not a device address: its address on each
// device is taken once with hipGetSymbolAddress (with that device current)
// and only that pointer is passed to kernels.
// ---------------------------------------------------------------------------
#define SIM_NOALLOC_SCRATCH_BYTES ((size_t)SIM_NOALLOC_SCRATCH_MAX)
static __device__ __align__(256) unsigned char scratch[SIM_NOALLOC_SCRATCH_BYTES];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[SIM_MAX_DEVICES] = {};

// device address of `scratch` on the current device (taken on first use)
static int noalloc_scratch(int device, void** ptr) {
  if (device < 0 || device >= SIM_MAX_DEVICES) return SIM_EDEVICE;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      sim_note_error(e, "hipGetSymbolAddress(scratch)", __LINE__);
      return SIM_EDEVICE;
    }
    g_scratch_ptr[device] = p;
  }
  *ptr = g_scratch_ptr[device];
  return SIM_OK;
}

int sim_structure_factor_noalloc(sim_t* s, int32_t nx, int32_t my_max, int32_t mz, double* out) {
  if (!s || !out || nx < 1 || nx > 256 || my_max < 0 || my_max > 128 || mz < -256 || mz > 256)
    return SIM_EINVAL;
  if (hipSetDevice(s->device) != hipSuccess) return SIM_EDEVICE;
  int64_t nchunk = 0;
  for (const RepDev& R : s->reph) nchunk += ((int64_t)R.n + 4095) / 4096;
  const size_t need = sq_scratch_bytes(nchunk, s->R, nx, my_max);
  if (need > SIM_NOALLOC_SCRATCH_BYTES) {
    snprintf(g_last_error, sizeof(g_last_error),
             "structure factor needs %zu bytes of scratch, the allocation-free call has %zu",
             need, SIM_NOALLOC_SCRATCH_BYTES);
    return SIM_ECAPACITY;
  }
  void* base = nullptr;
  int rc = noalloc_scratch(s->device, &base);
  if (rc) return rc;
  hipError_t err = launch_sq_scratch(s->d, nchunk, nx, my_max, mz, base, out, s->stream);
  if (!err) err = hipStreamSynchronize(s->stream);
  if (err) {
    sim_note_error(err, "structure factor (scratch)", __LINE__);
    return SIM_EDEVICE;
  }
  return SIM_OK;
}

int sim_structure_factor(sim_t* s, int32_t nx, int32_t my_max, int32_t mz, double* out,
                         double* kernel_ms) {
  if (!s || !out || nx < 1 || nx > 256 || my_max < 0 || my_max > 128 || mz < -256 || mz > 256)
    return SIM_EINVAL;
  if (hipSetDevice(s->device) != hipSuccess) return SIM_EDEVICE;
  std::vector<int64_t> row0, rows;
  for (const RepDev& R : s->reph) {
    row0.push_back(R.row_off);
    rows.push_back(R.n);
  }
  const int64_t nchunk = sq_chunk_count(rows);
  const int ny = 2 * my_max + 1;
  // scratch: chunk table | chunk offsets | partial sums | output
  auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  const size_t b_ch = up(sq_chunk_bytes() * (size_t)std::max<int64_t>(nchunk, 1));
  const size_t b_c0 = up(sizeof(int32_t) * (s->reph.size() + 1));
  const size_t b_pa = up(sq_partial_bytes(std::max<int64_t>(nchunk, 1), nx, my_max));
  const size_t b_out = up(sizeof(double) * s->reph.size() * (size_t)nx * ny);
  const size_t need = b_ch + b_c0 + b_pa + b_out;
  if (need > s->sq_bytes) {
    dfree(s, s->sq_scratch);
    s->sq_scratch = nullptr;
    s->sq_bytes = 0;
    int rc = dalloc(s, &s->sq_scratch, need);
    if (rc) return rc;
    s->sq_bytes = need;
  }
  char* base = (char*)s->sq_scratch;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (kernel_ms) {
    HIPCHK(hipEventCreateWithFlags(&e0, hipEventDisableSystemFence));
    HIPCHK(hipEventCreateWithFlags(&e1, hipEventDisableSystemFence));
  }
  hipError_t err = launch_sq(s->d, row0, rows, nx, my_max, mz, base, (int32_t*)(base + b_ch),
                             (double2*)(base + b_ch + b_c0), (double*)(base + b_ch + b_c0 + b_pa),
                             s->stream, e0, e1);
  if (!err)
    err = hipMemcpyAsync(out, base + b_ch + b_c0 + b_pa, sizeof(double) * s->reph.size() * nx * ny,
                         hipMemcpyDeviceToHost, s->stream);
  if (!err) err = hipStreamSynchronize(s->stream);
  if (!err && kernel_ms) {
    float ms = 0.0f;
    err = hipEventElapsedTime(&ms, e0, e1);
    *kernel_ms = ms;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (err) {
    sim_note_error(err, "structure factor", __LINE__);
    return SIM_EDEVICE;
  }
  return SIM_OK;
}

// coarse grid of reach M for one replica (cells, edges, culling margin)
static VvRep vv_grid(const RepDev& R, double r_max, int M) {
  const double vol = R.L[0] * R.L[1] * R.L[2];
  const double ell = std::max(r_max / M * (1.0 + 1e-12), std::cbrt(vol / (2.0 * std::max(R.n, 1))));
  VvRep V{};
  V.M = M;
  for (int k = 0; k < 3; ++k)
    V.nc[k] = (int32_t)std::max(1.0, std::min(std::floor(R.L[k] / ell), 4096.0));
  if (V.nc[1] < 2 * M + 1) { V.nc[1] = 1; V.nc[0] = 1; }
  if (V.nc[2] < 2 * M + 1) V.nc[2] = 1;
  if (V.nc[0] < 2 * M + 2) V.nc[0] = 1;
  double lmin = R.L[0];
  for (int k = 0; k < 3; ++k) {
    V.len[k] = R.L[k] / V.nc[k];
    V.inv_len[k] = 1.0 / V.len[k];
    lmin = std::min(lmin, V.len[k]);
  }
  V.margin = 1e-9 * lmin;
  return V;
}

int sim_velocity_correlation(sim_t* s, double r_max, int32_t nbins, int32_t flow, double* sum,
                             int64_t* count, double* u2, double* kernel_ms) {
  if (!s || !sum || !count || !u2 || nbins < 1 || nbins > 1024 || !(r_max > 0.0) ||
      !std::isfinite(r_max))
    return SIM_EINVAL;
  if (!s->vv_valid) return SIM_EINVAL;
  if (hipSetDevice(s->device) != hipSuccess) return SIM_EDEVICE;
  const int nrep = (int)s->reph.size();
  const int home = vv_home();
  // coarse grid per replica: cells of at least r_max / M per axis (at most
  // ~2 cells per particle); an axis too short for the 2M+1 stencil is one
  // cell (and a one-cell y axis makes x one cell too: the image shift is
  // then per pair).  M is the largest reach (<= 8) whose cells hold at least
  // 8 particles on average and that makes no axis one cell that reach 1
  // splits: smaller cells cull more of the stencil, but
  // below that the per-run overhead of the pair kernel dominates (measured
  // at N = 1e6 and 6.6e4 over r_max = 5 .. 16).
  std::vector<VvRep> vr(nrep);
  int64_t ncell = 0;
  for (int r = 0; r < nrep; ++r) {
    const RepDev& R = s->reph[r];
    if (r_max > 0.5 * std::min(R.L[0], std::min(R.L[1], R.L[2]))) return SIM_EINVAL;
    if (R.n >= (1 << 26)) return SIM_EINVAL;  // 32-bit pair counts of one block
    VvRep& V = vr[r];
    V = vv_grid(R, r_max, 1);
    for (int M = 8; M > 1; --M) {
      const VvRep c = vv_grid(R, r_max, M);
      bool keeps = true;  // no axis made one cell that reach 1 splits
      for (int k = 0; k < 3; ++k) keeps = keeps && !(V.nc[k] > 1 && c.nc[k] == 1);
      if (keeps && (double)R.n >= 8.0 * ((double)c.nc[0] * c.nc[1] * c.nc[2])) {
        V = c;
        break;
      }
    }
    V.rmax2 = r_max * r_max;
    V.cscale = ((double)nbins * (double)nbins) / (r_max * r_max);
    V.cell0 = (int32_t)ncell;
    const uint64_t pb = (uint64_t)home * (uint64_t)std::max(R.n, 1);
    int lg = 0;
    while ((1ull << lg) < pb) ++lg;
    V.log2p = lg;
    ncell += (int64_t)V.nc[0] * V.nc[1] * V.nc[2];
    if (ncell > (int64_t)1 << 30) return SIM_EINVAL;
  }
  const int64_t rows = s->rows;
  auto up = [](size_t b) { return (b + 255) / 256 * 256; };
  // scratch: the grid, binning and sorted copies first; the block table and
  // the blocks' partial sums once the cell populations are known
  size_t off = 0;
  auto take = [&](size_t b) { const size_t o = off; off += up(std::max<size_t>(b, 8)); return o; };
  const size_t o_vr = take(sizeof(VvRep) * nrep);
  const size_t o_cnt = take(sizeof(int32_t) * (ncell + 1));
  const size_t o_cstart = take(sizeof(int32_t) * (ncell + 1));
  const size_t o_vcell = take(sizeof(int32_t) * rows);
  const size_t o_slot = take(sizeof(int32_t) * rows);
  const size_t o_spos = take(sizeof(double4) * s->n_total);
  const size_t o_su = take(sizeof(double4) * s->n_total);
  const size_t o_umax = take(sizeof(unsigned long long) * nrep);
  const size_t o_u2p = take(sizeof(double) * s->d.nblk);
  const size_t o_rb = take(sizeof(int32_t) * (nrep + 1));
  const size_t o_osum = take(sizeof(double) * nrep * nbins);
  const size_t o_ocnt = take(sizeof(long long) * nrep * nbins);
  const size_t o_ou2 = take(sizeof(double) * nrep);
  int rc;
  if ((rc = grow_scratch(s, &s->vv_scratch, &s->vv_bytes, off))) return rc;
  char* base = (char*)s->vv_scratch;
  VvRep* vr_d = (VvRep*)(base + o_vr);
  int32_t* cnt_d = (int32_t*)(base + o_cnt);
  int32_t* cstart_d = (int32_t*)(base + o_cstart);
  unsigned long long* umax_d = (unsigned long long*)(base + o_umax);
  hipStream_t st = s->stream;
  HIPCHK(hipMemcpyAsync(vr_d, vr.data(), sizeof(VvRep) * nrep, hipMemcpyHostToDevice, st));
  HIPCHK(hipMemsetAsync(cnt_d, 0, sizeof(int32_t) * (ncell + 1), st));
  HIPCHK(hipMemsetAsync(umax_d, 0, sizeof(unsigned long long) * nrep, st));
  HIPCHK(launch_vv_bin(s->d, vr_d, flow ? 1 : 0, cnt_d, (int32_t*)(base + o_vcell),
                       (int32_t*)(base + o_slot), umax_d, (double*)(base + o_u2p), st));
  std::vector<int32_t> cnt_h(ncell + 1);
  HIPCHK(hipMemcpyAsync(cnt_h.data(), cnt_d, sizeof(int32_t) * (ncell + 1), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  // cell starts and the block table (chunks of home particles per cell)
  std::vector<int32_t> cstart_h(ncell + 1);
  std::vector<VvBlock> blk;
  std::vector<int32_t> rb(nrep + 1);
  int64_t acc = 0;
  for (int r = 0; r < nrep; ++r) {
    rb[r] = (int32_t)blk.size();
    const VvRep& V = vr[r];
    const int64_t nc = (int64_t)V.nc[0] * V.nc[1] * V.nc[2];
    for (int64_t c = V.cell0; c < V.cell0 + nc; ++c) {
      cstart_h[c] = (int32_t)acc;
      for (int32_t a = 0; a < cnt_h[c]; a += home)
        blk.push_back({r, (int32_t)c, (int32_t)(acc + a), std::min(home, cnt_h[c] - a)});
      acc += cnt_h[c];
    }
  }
  rb[nrep] = (int32_t)blk.size();
  cstart_h[ncell] = (int32_t)acc;
  if (acc != s->n_total) {
    snprintf(g_last_error, sizeof(g_last_error), "velocity correlation: binned %lld of %lld rows",
             (long long)acc, (long long)s->n_total);
    return SIM_EDEVICE;
  }
  HIPCHK(hipMemcpyAsync(cstart_d, cstart_h.data(), sizeof(int32_t) * (ncell + 1),
                        hipMemcpyHostToDevice, st));
  size_t off2 = 0;
  auto take2 = [&](size_t b) { const size_t o = off2; off2 += up(std::max<size_t>(b, 8)); return o; };
  // chunks of table blocks for the first reduce stage (never across replicas)
  std::vector<int2> chunks;
  std::vector<int32_t> rc0(nrep + 1);
  for (int r = 0; r < nrep; ++r) {
    rc0[r] = (int32_t)chunks.size();
    for (int32_t b0 = rb[r]; b0 < rb[r + 1]; b0 += vv_fold())
      chunks.push_back(make_int2(b0, std::min(b0 + vv_fold(), rb[r + 1])));
  }
  rc0[nrep] = (int32_t)chunks.size();
  const size_t nch = chunks.size();
  const size_t o_blk = take2(sizeof(VvBlock) * blk.size());
  const size_t o_psum = take2(sizeof(long long) * blk.size() * nbins);
  const size_t o_pcnt = take2(sizeof(unsigned long long) * blk.size() * nbins);
  const size_t o_ch = take2(sizeof(int2) * nch);
  const size_t o_flo = take2(sizeof(unsigned long long) * nch * nbins);
  const size_t o_fhi = take2(sizeof(long long) * nch * nbins);
  const size_t o_fcnt = take2(sizeof(unsigned long long) * nch * nbins);
  if ((rc = grow_scratch(s, &s->vv_scratch2, &s->vv_bytes2, off2))) return rc;
  char* base2 = (char*)s->vv_scratch2;
  VvBlock* blk_d = (VvBlock*)(base2 + o_blk);
  int32_t* rb_d = (int32_t*)(base + o_rb);
  if (!chunks.empty())
    HIPCHK(hipMemcpyAsync(base2 + o_ch, chunks.data(), sizeof(int2) * nch, hipMemcpyHostToDevice, st));
  if (!blk.empty())
    HIPCHK(hipMemcpyAsync(blk_d, blk.data(), sizeof(VvBlock) * blk.size(), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemcpyAsync(rb_d, rc0.data(), sizeof(int32_t) * (nrep + 1), hipMemcpyHostToDevice, st));
  double4* spos_d = (double4*)(base + o_spos);
  double4* su_d = (double4*)(base + o_su);
  HIPCHK(launch_vv_scatter(s->d, flow ? 1 : 0, cstart_d, (int32_t*)(base + o_vcell),
                           (int32_t*)(base + o_slot), spos_d, su_d, st));
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (kernel_ms) {
    HIPCHK(hipEventCreateWithFlags(&e0, hipEventDisableSystemFence));
    HIPCHK(hipEventCreateWithFlags(&e1, hipEventDisableSystemFence));
  }
  long long* psum_d = (long long*)(base2 + o_psum);
  unsigned long long* pcnt_d = (unsigned long long*)(base2 + o_pcnt);
  hipError_t err = launch_vv_pairs(s->d, vr_d, blk_d, (int)blk.size(), cstart_d, spos_d, su_d,
                                   umax_d, nbins, psum_d, pcnt_d, st, e0, e1);
  if (!err)
    err = launch_vv_reduce(s->d, vr_d, (const int2*)(base2 + o_ch), (int)nch, rb_d, nrep, nbins,
                           psum_d, pcnt_d, (unsigned long long*)(base2 + o_flo),
                           (long long*)(base2 + o_fhi), (unsigned long long*)(base2 + o_fcnt),
                           umax_d, (double*)(base + o_u2p), (double*)(base + o_osum),
                           (long long*)(base + o_ocnt), (double*)(base + o_ou2), st);
  if (!err)
    err = hipMemcpyAsync(sum, base + o_osum, sizeof(double) * nrep * nbins, hipMemcpyDeviceToHost, st);
  if (!err)
    err = hipMemcpyAsync(count, base + o_ocnt, sizeof(int64_t) * nrep * nbins,
                         hipMemcpyDeviceToHost, st);
  if (!err) err = hipMemcpyAsync(u2, base + o_ou2, sizeof(double) * nrep, hipMemcpyDeviceToHost, st);
  if (!err) err = hipStreamSynchronize(st);
  if (!err && kernel_ms) {
    float ms = 0.0f;
    err = blk.empty() ? hipSuccess : hipEventElapsedTime(&ms, e0, e1);
    *kernel_ms = ms;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (err) {
    sim_note_error(err, "velocity correlation", __LINE__);
    return SIM_EDEVICE;
  }
  return SIM_OK;
}

int sim_debug_set_gaussians(sim_t* s, const double* xi, const double* eta) {
  if (!s) return SIM_EINVAL;
  if (hipSetDevice(s->device) != hipSuccess) return SIM_EDEVICE;
  if (!xi && !eta) {
    dfree(s, s->inj_xi);
    dfree(s, s->inj_eta);
    s->inj_xi = s->inj_eta = nullptr;
    s->d.inj_xi = s->d.inj_eta = nullptr;
    return SIM_OK;
  }
  if (!xi || !eta) return SIM_EINVAL;
  if (s->R != 1 || s->n_total > 1024) return SIM_ENOTSUP;
  const int64_t n = s->n_total;
  int rc;
  if (!s->inj_xi && (rc = dalloc(s, (void**)&s->inj_xi, sizeof(double) * 3 * n))) return rc;
  if (!s->inj_eta && (rc = dalloc(s, (void**)&s->inj_eta, sizeof(double) * 3 * n * n))) return rc;
  HIPCHK(hipMemcpy(s->inj_xi, xi, sizeof(double) * 3 * n, hipMemcpyHostToDevice));
  HIPCHK(hipMemcpy(s->inj_eta, eta, sizeof(double) * 3 * n * n, hipMemcpyHostToDevice));
  s->d.inj_xi = s->inj_xi;
  s->d.inj_eta = s->inj_eta;
  return SIM_OK;
}

}  // extern "C"
