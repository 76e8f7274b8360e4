// sim_dev.h -- device-side data layout and helpers of libsim (gfx950).
//
// Layout in HBM (all replicas concatenated, rows padded per replica to a
// multiple of ROWS_PER_BLOCK so that every thread block belongs to exactly one
// replica; padding rows are inert: diag 1, no neighbours, zero rhs):
//   pos      double4[rows]   x, y, z, original id (as an exact double)
//                            in cell-sorted order (re-sorted every step)
//   cellidx  int32[rows]     global cell of each particle
//   rowptr   int32[rows+1]   CSR of the off-diagonal part of A, full rows
//   col/val  int32/double    -alpha*w_ij per directed pair (valf: FP32 copy)
//   diag     double[rows]    gamma0 + alpha*sum_j w_ij (dinv = 1/diag)
//   b, x, p, r, s, w, u   double[3*rows]  right-hand sides and the CG vectors
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define ROWS_PER_BLOCK 1024
#define BLOCK_THREADS 1024
#define NPART 16  // doubles per partial slot (9 used)
// The CG kernels work on sub-tiles of SUB_ROWS rows with SUB_THREADS threads
// and leave one partial slot per sub-tile: blocks of four waves wait less at
// their closing reduction than blocks of sixteen (measured on the CSR product
// at N = 8e6: 386 -> 332 us)
#define SUB_ROWS 256
#define SUB_THREADS 256
#define SUBS_PER_TILE (ROWS_PER_BLOCK / SUB_ROWS)

// ---------------------------------------------------------------------------
// Per-replica constants (device copy built at creation)
// ---------------------------------------------------------------------------
struct RepDev {
  double L[3];        // box
  double hL[3];       // L/2
  double cell_len[3]; // cell edge >= rc*(1+1e-9)
  double inv_cell[3];
  int32_t nc[3];      // cells per axis: >= 3, or 1 (whole axis one cell)
  int32_t seg_off;    // first entry of this replica's cell segment (ncell+1 entries)
  int64_t row_off;    // first row
  int32_t n;          // real particles
  int32_t npad;       // rows incl. padding (multiple of ROWS_PER_BLOCK)
  int32_t blk_off;    // first block
  int32_t nblk;       // blocks
  double kT, gamma0, alpha, shear, dt, rc, rc2, lam, inv_lam2, u_amp;
  double amp_node, amp_pair;  // thermal-force amplitudes
  double force_gc;            // kT*u_amp/lambda^2 (Gaussian core)
  double force_soft;          // 2*u_amp/rc (soft)
  double tol2;                // cg_tol^2
  int32_t weight_law, potential, noise_mode, precond;
  int32_t brick;              // brick edge of the cell order, in cells (>= every nc: z-major)
  int32_t l1_cnt;             // first-level reduction blocks of the CG partials (0: none)
  int32_t l1_off;             // the first of them
  int32_t pad0;
  uint64_t seed, stream;
};

// Cell order.  Cells are numbered brick by brick: bricks of brick^3 cells
// (smaller at the high end of an axis) in z-major order, and z-major cells
// (x fastest) inside a brick, so the numbering is dense and a cell's 26
// neighbours are mostly a few hundred cells away instead of one cell plane
// (the row of the gathered neighbour data stays within an XCD's L2).
// brick >= nc on every axis gives the plain z-major order.
__host__ __device__ __forceinline__ int cell_key(const RepDev& R, int cx, int cy, int cz) {
  const int B = R.brick, nx = R.nc[0], ny = R.nc[1], nz = R.nc[2];
  const int bx = cx / B, by = cy / B, bz = cz / B;
  const int wx = cx - bx * B, wy = cy - by * B, wz = cz - bz * B;
  const int sx = nx - bx * B < B ? nx - bx * B : B;
  const int sy = ny - by * B < B ? ny - by * B : B;
  const int sz = nz - bz * B < B ? nz - bz * B : B;
  return bz * B * ny * nx + sz * (by * B) * nx + sz * sy * (bx * B) + (wz * sy + wy) * sx + wx;
}

// Per-replica conjugate-gradient scalars (three components), written only by
// the finishing kernel and read by the row kernels that follow it.
struct CgRep {
  double bb[3];     // ||b||^2
  double rr[3];     // ||r||^2 (recursive while iterating, true after a check)
  double gamma[3];  // (r, M^-1 r) of the current iterate
  double alpha[3];
  double alpha_prev[3];  // the previous iteration's alpha (0 after a start or restart)
  double beta[3];
  double tol2;      // tolerance^2 of this solve
  int32_t state[3]; // 0 iterating, 1 check pending, 2 done, 3 restart pending
  int32_t it[3];
  int32_t run;      // some component iterating
  int32_t check;    // none iterating and some check pending
  int32_t restart;  // some restart pending
  int32_t restarts;
  int32_t breakdown;
  int32_t pad;
};

// Global control words (one per handle)
struct Ctrl {
  int32_t n_notdone;    // (replica, component) pairs not finished
  int32_t overflow;     // CSR capacity exceeded in the last fill
  int32_t numeric;      // non-finite or escaped position after an update
  int32_t max_row;      // longest off-diagonal row of the last build
  int64_t nnz;          // off-diagonal entries of the last build
  int32_t breakdown;    // a component of the current solve broke down
  int32_t too_many;     // the row scan passed INT32_MAX entries (32-bit CSR indices)
};

// A step may be committed on the device (graph replay) only when every
// component converged and nothing overflowed or broke down.
__device__ __forceinline__ bool ctrl_commit_ok(const Ctrl* c) {
  return c->n_notdone == 0 && c->overflow == 0 && c->breakdown == 0;
}

struct DevPtrs {
  const RepDev* rep;
  CgRep* cg;
  Ctrl* ctrl;
  const int32_t* blk_rep;   // block -> replica
  double* partial;          // [sub-tiles][NPART] (the block CG: [tiles][NPART])
  double* partial2;         // [first-level blocks][NPART]
  const int32_t* l1_rep;    // first-level block -> replica
  double4* pos;             // current positions (sorted order)
  double4* pos_alt;         // scatter target
  int32_t* cellidx;
  int32_t* cellidx_alt;
  int32_t* slot;
  int32_t* cell_count;      // [cell entries]
  int32_t* cell_row;        // first row of each cell (segmented, absolute)
  int32_t* rowlen;          // [rows+1]
  int32_t* rowptr;          // [rows+1]
  int32_t* col;
  double* val;
  float* valf;
  double* diag;
  double* dinv;
  double* b;
  double* x;
  double* p;
  double* r;
  double* s;
  double* w;
  double* u;
  double* vel_orig;         // velocities of the last step, original order
  float* er;                // r_ij / rc per CSR entry (learned preconditioner input)
  const double* mdiag;      // learned M^-1 diagonal, or null (Jacobi)
  const float* moff;        // learned M^-1 off-diagonal (A's pattern)
  const double* inj_xi;     // injected Gaussians (testing), or null
  const double* inj_eta;
  // IC(0) in multicolour order (precond = IC0): L in A's row pointers, per
  // row its lower entries (ascending IC order) then its upper entries
  // (descending IC order, holding L_ji); diagonal of L; lower-entry count
  int32_t* lcol;
  double* lval;
  double* ldiag;
  int32_t* lnlow;
  const int32_t* ic_cells;  // cell entries grouped by colour
  const int32_t* cell_color;// colour of every cell entry (-1 for terminal entries)
  int64_t* step_d;          // current step index n (device copy of the host's counter)
  int64_t nnz_cap;
  int64_t rows;
  int32_t nblk;             // blocks over all replicas
  int32_t nrep;
  int32_t ncell_entries;
  int32_t spmv_fp32;
  int32_t learned;          // 1: u = M^-1 r by the learned preconditioner
  int32_t spmv_var;         // CSR product variants (CSR_VARIANT_LIST index)
  int32_t apply_var;
  int32_t ic0;              // 1: u = M^-1 r by the IC(0) triangular solves
  int32_t pc_none;          // 1: no preconditioner, u = r
  int32_t l1_total;         // first-level reduction blocks over all replicas
  int32_t want_er;          // 1: the pair terms write er (the network's edge input)
  int32_t vec_nt;           // 1: the CG vector kernel streams with nontemporal accesses
  int32_t rev;              // 1: each XCD walks its CG sub-tiles from the last
};
static_assert(sizeof(DevPtrs) % 8 == 0, "DevPtrs must have no implicit tail padding");

// CSR product variants: X(index, lanes per row, entries per lane loaded
// one pass ahead of the gathers; 0 = one entry at a time), or (0, entries per
// thread and pass) for the entry-parallel form.  The order is the public one
// of sim_tuning.
#define CSR_VARIANTS 10
#define CSR_VARIANT_DEFAULT 8
#define CSR_VARIANT_LIST(X) \
  X(0, 1, 0) X(1, 2, 0) X(2, 4, 0) X(3, 8, 0) X(4, 2, 2) X(5, 4, 1) X(6, 4, 2) X(7, 4, 3) \
  X(8, 0, 2) X(9, 0, 3)

// The per-replica CG finisher sums the replica's sub-tile partials with
// FINISH_THREADS threads.  A replica of more than L1_MIN_SUBS sub-tiles has
// them summed first by blocks of L1_SUBS sub-tiles each (in parallel, one
// launch) and the finisher adds those blocks' sums: a single block reading
// every partial of an N = 8e6 box (31,252 slots, 4 MB) took about 60 us per
// iteration.  Both are functions of the replica alone, so its totals do not
// depend on the rest of a batch.
#define FINISH_THREADS 256
#define L1_SUBS 256
#define L1_MIN_SUBS 2048

// ---------------------------------------------------------------------------
// Block -> tile mapping: hardware dispatches workgroups round-robin over the
// 8 XCDs; give each XCD a contiguous range of row blocks so that the CSR
// gathers of neighbouring rows hit that XCD's own L2.
// ---------------------------------------------------------------------------
__device__ __forceinline__ int xcd_block(int hw, int nblk) {
  const int per = (nblk + 7) >> 3;
  return (hw & 7) * per + (hw >> 3);
}
__host__ __forceinline__ int xcd_grid(int nblk) { return ((nblk + 7) >> 3) << 3; }

// ---------------------------------------------------------------------------
// Philox4x64-10 (Salmon, Moraes, Dror, Shaw, SC'11) and Box-Muller Gaussians
// ---------------------------------------------------------------------------
__device__ __forceinline__ void philox4x64(uint64_t c[4], uint64_t k0, uint64_t k1) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    const uint64_t m0 = 0xD2E7470EE14C6C93ULL, m1 = 0xCA5A826395121157ULL;
    uint64_t lo0 = m0 * c[0], hi0 = __umul64hi(m0, c[0]);
    uint64_t lo1 = m1 * c[2], hi1 = __umul64hi(m1, c[2]);
    uint64_t n0 = hi1 ^ c[1] ^ k0;
    uint64_t n2 = hi0 ^ c[3] ^ k1;
    c[0] = n0;
    c[1] = lo1;
    c[2] = n2;
    c[3] = lo0;
    k0 += 0x9E3779B97F4A7C15ULL;
    k1 += 0xBB67AE8584CAA73BULL;
  }
}

__device__ __forceinline__ double u01_open(uint64_t bits) {
  return ((double)(bits >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

// three standard normals from counter (step, tag, a, b), key (seed, stream)
__device__ __forceinline__ void gauss3(uint64_t seed, uint64_t stream, uint64_t step,
                                       uint64_t tag, uint64_t a, uint64_t b, double g[3]) {
  uint64_t c[4] = {step, tag, a, b};
  philox4x64(c, seed, stream);
  const double two_pi = 6.283185307179586;
  const double u0 = u01_open(c[0]), u1 = u01_open(c[1]);
  const double u2 = u01_open(c[2]), u3 = u01_open(c[3]);
  const double rad0 = sqrt(-2.0 * log(u0));
  const double rad1 = sqrt(-2.0 * log(u2));
  g[0] = rad0 * cos(two_pi * u1);
  g[1] = rad0 * sin(two_pi * u1);
  g[2] = rad1 * cos(two_pi * u3);
}

// ---------------------------------------------------------------------------
// Lees-Edwards geometry.  Offset of the image above at step n:
// fmod(kappa*Ly*(n*dt), Lx).  Separation d = R_i - R_j(nearest image) with
// the image index s (Eq. 8: s = round(y_ij/Ly)); explicit round-to-nearest
// operations (no contraction) so the pair decision is reproducible.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double le_offset(const RepDev& R, int64_t step) {
  const double t = __dmul_rn((double)step, R.dt);
  return fmod(__dmul_rn(__dmul_rn(R.shear, R.L[1]), t), R.L[0]);
}

__device__ __forceinline__ int le_sep(const RepDev& R, double delta, double xi, double yi, double zi,
                                      double xj, double yj, double zj, double& dx, double& dy,
                                      double& dz) {
  double ty = __dsub_rn(yi, yj);
  int s = 0;
  if (ty > R.hL[1]) s = 1;
  else if (ty < -R.hL[1]) s = -1;
  dy = __dsub_rn(ty, __dmul_rn((double)s, R.L[1]));
  double tx = __dsub_rn(__dsub_rn(xi, xj), __dmul_rn((double)s, delta));
  if (tx > R.hL[0]) tx = __dsub_rn(tx, R.L[0]);
  if (tx > R.hL[0]) tx = __dsub_rn(tx, R.L[0]);
  if (tx < -R.hL[0]) tx = __dadd_rn(tx, R.L[0]);
  if (tx < -R.hL[0]) tx = __dadd_rn(tx, R.L[0]);
  dx = tx;
  double tz = __dsub_rn(zi, zj);
  if (tz > R.hL[2]) tz = __dsub_rn(tz, R.L[2]);
  if (tz < -R.hL[2]) tz = __dadd_rn(tz, R.L[2]);
  dz = tz;
  return s;
}

__device__ __forceinline__ double dist2(double dx, double dy, double dz) {
  return __dadd_rn(__dadd_rn(__dmul_rn(dx, dx), __dmul_rn(dy, dy)), __dmul_rn(dz, dz));
}

__device__ __forceinline__ int cell_axis(double v, const RepDev& R, int k) {
  int c = (int)floor(v * R.inv_cell[k]);
  c = c < 0 ? 0 : c;
  return c > R.nc[k] - 1 ? R.nc[k] - 1 : c;
}

__device__ __forceinline__ int imod(int a, int m) {
  int r = a % m;
  return r < 0 ? r + m : r;
}

// Enumerate every candidate row j of particle (xi, yi, zi) in replica R:
// 3 x 3 rows of cells (z, y) and, per row, a run of x cells: the three
// around cx for rows inside the box, or for a row across the y boundary
// the cells covering x - s*delta +- rc (the Lees-Edwards-shifted images).
// Consecutive x cells of one brick are contiguous in the sorted order, so
// each run is a few row ranges.  f(j) is called for every candidate j != i
// in a fixed order.
template <typename F>
__device__ __forceinline__ void for_candidates(const RepDev& R, const int32_t* cell_row,
                                               double delta, double xi, double yi, double zi,
                                               int64_t self, F&& f) {
  const int cx = cell_axis(xi, R, 0), cy = cell_axis(yi, R, 1), cz = cell_axis(zi, R, 2);
  const int ncx = R.nc[0], ncy = R.nc[1], ncz = R.nc[2];
  const int zlo = ncz == 1 ? 0 : -1, zhi = ncz == 1 ? 0 : 1;
  const int ylo = ncy == 1 ? 0 : -1, yhi = ncy == 1 ? 0 : 1;
  const double eps = 1e-9 * R.cell_len[0];
  for (int dz = zlo; dz <= zhi; ++dz) {
    const int cz2 = imod(cz + dz, ncz);
    for (int dyc = ylo; dyc <= yhi; ++dyc) {
      const int cyr = cy + dyc;
      int cy2, lo, hi;
      if (ncy == 1) {
        cy2 = 0; lo = 0; hi = ncx - 1;
      } else if (cyr >= 0 && cyr < ncy) {
        cy2 = cyr;
        if (ncx == 1) { lo = 0; hi = 0; }
        else { lo = cx - 1; hi = cx + 1; }
      } else {
        // across the y boundary: j's image is shifted by s*delta in x, with
        // s = +1 going up (j in row 0) and -1 going down (j in the top row)
        const double sd = cyr >= ncy ? delta : -delta;
        cy2 = cyr >= ncy ? 0 : ncy - 1;
        const double c0 = xi - sd;
        lo = (int)floor((c0 - R.rc - eps) * R.inv_cell[0]);
        hi = (int)floor((c0 + R.rc + eps) * R.inv_cell[0]);
        if (hi - lo + 1 >= ncx) { lo = 0; hi = ncx - 1; }
      }
      // split [lo, hi] at the periodic x edge and at brick edges into runs
      // of consecutive cells (consecutive keys)
      int a = imod(lo, ncx);
      int len = hi - lo + 1;
      while (len > 0) {
        int run = (a + len <= ncx) ? len : (ncx - a);
        const int bend = (a / R.brick + 1) * R.brick - a;
        run = run < bend ? run : bend;
        const int c0 = R.seg_off + cell_key(R, a, cy2, cz2);
        const int j0 = cell_row[c0], j1 = cell_row[c0 + run];
        for (int j = j0; j < j1; ++j)
          if (j != self) f(j);
        len -= run;
        a = a + run == ncx ? 0 : a + run;
      }
    }
  }
}

// ---------------------------------------------------------------------------
// Deterministic reductions: wave (64 lanes, fixed xor tree, lane 0 result),
// then block (waves in order) -- no floating-point atomics anywhere.
// ---------------------------------------------------------------------------
// Butterfly over the 64 lanes: lane ^ 1 and lane ^ 2 by quad permutes, then
// the mirrored lane of the other half-row (8 lanes) and of the other half of
// the row (16 lanes) -- which hold those groups' sums after the earlier
// steps -- all on registers (DPP); the last two steps cross rows through
// the LDS permute network.  Each step adds the same two operands on both
// partners, so every lane ends with the same bits.
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const int lo = __builtin_amdgcn_mov_dpp(__double2loint(v), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_mov_dpp(__double2hiint(v), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}
constexpr int DPP_XOR1 = 0xB1;         // quad_perm [1, 0, 3, 2]
constexpr int DPP_XOR2 = 0x4E;         // quad_perm [2, 3, 0, 1]
constexpr int DPP_HALF_MIRROR = 0x141; // lane i <- lane 7 - i within 8
constexpr int DPP_MIRROR = 0x140;      // lane i <- lane 15 - i within 16

__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_move<DPP_XOR1>(v);
  v += dpp_move<DPP_XOR2>(v);
  v += dpp_move<DPP_HALF_MIRROR>(v);
  v += dpp_move<DPP_MIRROR>(v);
  v += __shfl_xor(v, 16, 64);
  v += __shfl_xor(v, 32, 64);
  return v;
}

// sums K values over the block; result valid in thread 0
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double (*lds)[K]) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) lds[wave][k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      double s = 0.0;
      for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += lds[w][k];
      v[k] = s;
    }
  }
}
