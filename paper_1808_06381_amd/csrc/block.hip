// block.hip -- the friction system with anisotropic pair friction on gfx950:
// the pair coefficient of Eq. 7 becomes a tensor
//   W_ij = alpha w_ij (a_perp I + (a_par - a_perp) P_ij),  P_ij = d d^T / r^2
// (friction a_par along the line of centres, a_perp across it; P = 0 at
// r = 0), so A of Eq. 9 has genuine 3 x 3 blocks:
//   A_ii = gamma0 I + sum_j W_ij,  A_ij = -W_ij,
//   b_i  = sum_j F_ij + gamma0 kappa (y_i - Ly/2) x + sum_j W_ij V_ij + f_i,
// with the fluctuation-dissipation pair noise
//   sqrt(2kT/dt) sigma_ij W_ij^(1/2) eta_ij,
//   W^(1/2) = sqrt(alpha w) (sqrt(a_perp) I + (sqrt(a_par) - sqrt(a_perp)) P),
// eta_ij the same Philox pair Gaussians as the isotropic system.
//
// Layout: the neighbour list (CSR, cell order) of the isotropic path; per
// entry the six values of -W_ij (xx, xy, xz, yy, yz, zz), per row the six
// values of the diagonal block and of its inverse (block-Jacobi).
//
// Solve: block-Jacobi preconditioned CG with one recurrence over the 3n
// stacked unknowns of each replica (the three components are coupled), in
// the single-reduction form of Chronopoulos & Gear (as the scalar solve),
// stopping on the true residual ||b - A x|| <= tol ||b||.  Per iteration
// three launches: w = A u with tile partials of (w, u); a per-replica
// finisher that reduces (w, u), (r, u) and (r, r) together (convergence of
// the recursive residual, then beta = gamma / gamma_old and
// alpha = gamma / (delta - beta gamma / alpha_old)); and the vector pass
// p = u + beta p, s = w + beta s, x += alpha p, r -= alpha s, u = M^-1 r with
// partials of (r, u), (r, r).  Residual rounds (start, and after the
// recursive residual meets the tolerance): r = b - A x, u = M^-1 r,
// p = s = 0 (so the next pass starts with p = u, s = w).  All reductions in
// a fixed order: deterministic.
#include <hip/hip_runtime.h>

#include "launch.h"
#include "sim_dev.h"

namespace {

// 3 x 3 symmetric, stored xx, xy, xz, yy, yz, zz
__device__ __forceinline__ void sym_mul(const double* m, const double v[3], double out[3]) {
  out[0] = (m[0] * v[0] + m[1] * v[1]) + m[2] * v[2];
  out[1] = (m[1] * v[0] + m[3] * v[1]) + m[4] * v[2];
  out[2] = (m[2] * v[0] + m[4] * v[1]) + m[5] * v[2];
}

// the same with the six values rounded to FP32 (products and sums in FP64)
__device__ __forceinline__ void sym_mul_f(const float* mf, const double v[3], double out[3]) {
  const double m[6] = {mf[0], mf[1], mf[2], mf[3], mf[4], mf[5]};
  sym_mul(m, v, out);
}

// row-major 3 x 3 in FP32 (the learned preconditioner's M_ij) times a vector
__device__ __forceinline__ void full_mul(const float* a, const double v[3], double out[3]) {
#pragma unroll
  for (int r = 0; r < 3; ++r)
    out[r] = ((double)a[3 * r] * v[0] + (double)a[3 * r + 1] * v[1]) + (double)a[3 * r + 2] * v[2];
}

__device__ __forceinline__ void sym_inverse(const double* m, double* inv) {
  const double a = m[0], b = m[1], c = m[2], d = m[3], e = m[4], f = m[5];
  const double c00 = d * f - e * e, c01 = c * e - b * f, c02 = b * e - c * d;
  const double c11 = a * f - c * c, c12 = b * c - a * e, c22 = a * d - b * b;
  const double det = (a * c00 + b * c01) + c * c02;
  const double id = 1.0 / det;
  inv[0] = c00 * id; inv[1] = c01 * id; inv[2] = c02 * id;
  inv[3] = c11 * id; inv[4] = c12 * id; inv[5] = c22 * id;
}

__device__ __forceinline__ double pweight(const RepDev& R, double r2, double r) {
  if (R.weight_law == 0) return exp(-0.5 * r2 * R.inv_lam2);
  const double t = 1.0 - r / R.rc;
  return t * t;
}

__device__ __forceinline__ double pforce(const RepDev& R, double r2, double r) {
  if (R.potential == 0) return R.force_gc * exp(-0.5 * r2 * R.inv_lam2);
  if (R.potential == 1) return r > 0.0 ? R.force_soft * (1.0 - r / R.rc) / r : 0.0;
  return 0.0;
}

// the tile's partial slots 0..2 from every thread's values (fixed order)
// tile partial sums [(w, u), (r, u), (r, r)]: slots first .. first + N - 1
template <int N>
__device__ __forceinline__ void tile_partials(const DevPtrs& d, int tile, int first,
                                              double (&v)[N]) {
  __shared__ double lds[BLOCK_THREADS / 64][N];
  block_sum<N>(v, lds);
  if (threadIdx.x == 0) {
    double* dst = d.partial + (int64_t)tile * NPART + first;
#pragma unroll
    for (int k = 0; k < N; ++k) dst[k] = v[k];
  }
}

}  // namespace

// Pair terms and assembly of the block system.  A block owns a tile of
// PB_THREADS rows and walks the tile's contiguous CSR entries in chunks of
// PB_THREADS, one entry per lane: every entry's block is formed from the
// separation d_ij of the row's particle (the mirror entry gets the same
// block and the negated contribution, bit for bit) and written out, and its
// twelve row contributions (the block, the force and drag term, the noise
// term) go to LDS; each thread then adds its row's in entry order, with the
// same operations a walk of the row would make, and assembles the row.
constexpr int PB_THREADS = 256;
constexpr int PB_TILES = ROWS_PER_BLOCK / PB_THREADS;  // tiles per row block
__global__ __launch_bounds__(PB_THREADS) void k_pair_block(DevPtrs d, BlockPtrs bp) {
  const int tile = xcd_block(blockIdx.x, PB_TILES * d.nblk);  // rows in this XCD's L2
  if (tile >= PB_TILES * d.nblk) return;
  if (d.ctrl->overflow) return;
  const int blk = tile / PB_TILES;
  const int rid = d.blk_rep[blk];
  const RepDev& R = d.rep[rid];
  const BlockRep& Q = bp.brep[rid];
  __shared__ int rp[PB_THREADS + 1];
  __shared__ int16_t erow[PB_THREADS];
  __shared__ double contrib[12][PB_THREADS];  // W (6), force and drag (3), noise (3)
  const int t = threadIdx.x;
  const int64_t row0 = (int64_t)blk * ROWS_PER_BLOCK + (tile % PB_TILES) * PB_THREADS;
  for (int r = t; r <= PB_THREADS; r += PB_THREADS) rp[r] = d.rowptr[row0 + r];
  __syncthreads();
  const int64_t step = *d.step_d;
  const double delta = le_offset(R, step);
  const bool noise = R.amp_pair != 0.0 && R.alpha != 0.0;
  const double c = Q.a_par - Q.a_perp, cs = Q.sq_par - Q.sq_perp;
  const double vunit = R.shear * R.L[1];
  double D[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  double acc[3] = {0.0, 0.0, 0.0};
  const int E0 = rp[0], E1 = rp[PB_THREADS];
  for (int cb = E0; cb < E1; cb += PB_THREADS) {
    {
      const int lo = max(rp[t], cb), hi = min(rp[t + 1], cb + PB_THREADS);
      for (int e = lo; e < hi; ++e) erow[e - cb] = (int16_t)t;
    }
    __syncthreads();
    const int e = cb + t;
    if (e < E1) {
      const int64_t i = row0 + erow[t];
      const double4 pi = d.pos[i];
      const int j = d.col[e];
      const double4 pj = d.pos[j];
      double dv[3];
      const int s = le_sep(R, delta, pi.x, pi.y, pi.z, pj.x, pj.y, pj.z, dv[0], dv[1], dv[2]);
      const double r2 = dist2(dv[0], dv[1], dv[2]);
      const double r = sqrt(r2);
      const double g = R.alpha * pweight(R, r2, r);
      double P[6];
      P[0] = r2 > 0.0 ? (dv[0] * dv[0]) / r2 : 0.0;
      P[1] = r2 > 0.0 ? (dv[0] * dv[1]) / r2 : 0.0;
      P[2] = r2 > 0.0 ? (dv[0] * dv[2]) / r2 : 0.0;
      P[3] = r2 > 0.0 ? (dv[1] * dv[1]) / r2 : 0.0;
      P[4] = r2 > 0.0 ? (dv[1] * dv[2]) / r2 : 0.0;
      P[5] = r2 > 0.0 ? (dv[2] * dv[2]) / r2 : 0.0;
      double W[6];
      W[0] = g * (Q.a_perp + c * P[0]);
      W[1] = g * (c * P[1]);
      W[2] = g * (c * P[2]);
      W[3] = g * (Q.a_perp + c * P[3]);
      W[4] = g * (c * P[4]);
      W[5] = g * (Q.a_perp + c * P[5]);
      double* out = bp.bval + 6 * (int64_t)e;
#pragma unroll
      for (int m = 0; m < 6; ++m) {
        out[m] = -W[m];
        contrib[m][t] = W[m];
      }
      if (bp.fp32) {
        float* outf = bp.bvalf + 6 * (int64_t)e;
#pragma unroll
        for (int m = 0; m < 6; ++m) outf[m] = (float)(-W[m]);
      }
      if (d.want_er) {  // the learned preconditioner's input: traces, r / rc
        d.val[e] = -((W[0] + W[3]) + W[5]) / 3.0;
        d.er[e] = (float)(r / R.rc);
      }
      // conservative force and boundary drag W V, V = kappa Ly s x (column 0)
      const double fc = pforce(R, r2, r);
      const double v = vunit * (double)s;
      contrib[6][t] = fc * dv[0] + W[0] * v;
      contrib[7][t] = fc * dv[1] + W[1] * v;
      contrib[8][t] = fc * dv[2] + W[2] * v;
      if (noise) {
        const int64_t idi = (int64_t)pi.w, idj = (int64_t)pj.w;
        const int64_t a = idi < idj ? idi : idj, bb = idi < idj ? idj : idi;
        double gz[3];
        gauss3(R.seed, R.stream, (uint64_t)step, 1, (uint64_t)a, (uint64_t)bb, gz);
        const double amp = (idi < idj ? 1.0 : -1.0) * (R.amp_pair * sqrt(g));
        const double tt = (dv[0] * gz[0] + dv[1] * gz[1]) + dv[2] * gz[2];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
          const double q = r2 > 0.0 ? (dv[k] * tt) / r2 : 0.0;
          contrib[9 + k][t] = amp * (Q.sq_perp * gz[k] + cs * q);
        }
      }
    }
    __syncthreads();
    {
      const int lo = max(rp[t], cb), hi = min(rp[t + 1], cb + PB_THREADS);
      for (int e2 = lo; e2 < hi; ++e2) {
        const int q = e2 - cb;
#pragma unroll
        for (int m = 0; m < 6; ++m) D[m] += contrib[m][q];
#pragma unroll
        for (int k = 0; k < 3; ++k) acc[k] += contrib[6 + k][q];
        if (noise) {
#pragma unroll
          for (int k = 0; k < 3; ++k) acc[k] += contrib[9 + k][q];
        }
      }
    }
    __syncthreads();  // erow and contrib are rewritten for the next chunk
  }
  const int64_t i = row0 + t;
  if (i - R.row_off >= R.n) {  // padding row: identity, no right-hand side
    double* Dp = bp.bdiag + 6 * i;
    double* Ip = bp.binv + 6 * i;
    Dp[0] = Dp[3] = Dp[5] = Ip[0] = Ip[3] = Ip[5] = 1.0;
    Dp[1] = Dp[2] = Dp[4] = Ip[1] = Ip[2] = Ip[4] = 0.0;
    d.b[3 * i] = d.b[3 * i + 1] = d.b[3 * i + 2] = 0.0;
    if (d.want_er) d.diag[i] = 1.0;
    return;
  }
  const double4 pi = d.pos[i];
  const int64_t idi = (int64_t)pi.w;
  double gn[3] = {0.0, 0.0, 0.0};
  if (R.amp_node != 0.0) gauss3(R.seed, R.stream, (uint64_t)step, 0, (uint64_t)idi, 0, gn);
  D[0] += R.gamma0;
  D[3] += R.gamma0;
  D[5] += R.gamma0;
  double* Dout = bp.bdiag + 6 * i;
#pragma unroll
  for (int m = 0; m < 6; ++m) Dout[m] = D[m];
  sym_inverse(D, bp.binv + 6 * i);
  if (d.want_er) d.diag[i] = ((D[0] + D[3]) + D[5]) / 3.0;
  d.b[3 * i] = R.gamma0 * R.shear * (pi.y - R.hL[1]) + R.amp_node * gn[0] + acc[0];
  d.b[3 * i + 1] = R.amp_node * gn[1] + acc[1];
  d.b[3 * i + 2] = R.amp_node * gn[2] + acc[2];
}

// per replica: fresh solve state (x = 0 is written by k_bcg_zero)
__global__ void k_bcg_reset(DevPtrs d, BlockPtrs bp, double tol) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= d.nrep) return;
  BcgRep& B = bp.bcg[r];
  B.bb = -1.0;
  B.rz = B.alpha = B.beta = B.rr = 0.0;
  B.tol2 = tol > 0.0 ? tol * tol : d.rep[r].tol2;
  B.state = 1;
  B.it = B.restarts = B.breakdown = 0;
  B.first = 1;
}

// Warm start, after the first residual round (which set ||b||^2 from x = 0
// and finished the replicas with b = 0): x = the previous step's velocity
// of each row's particle (kept in original order) for the replicas still
// iterating.  Padding rows keep x = 0.
__global__ __launch_bounds__(BLOCK_THREADS) void k_bcg_warm(DevPtrs d, BlockPtrs bp,
                                                            const int64_t* __restrict__ id_off) {
  static_assert(ROWS_PER_BLOCK == BLOCK_THREADS, "one row per thread");
  const int blk = blockIdx.x;
  const int rid = d.blk_rep[blk];
  if (bp.bcg[rid].state != 0) return;
  const RepDev& R = d.rep[rid];
  const int64_t i = (int64_t)blk * ROWS_PER_BLOCK + threadIdx.x;
  if (i - R.row_off >= R.n) return;
  const int64_t g = id_off[rid] + (int64_t)d.pos[i].w;
  d.x[3 * i] = d.vel_orig[3 * g];
  d.x[3 * i + 1] = d.vel_orig[3 * g + 1];
  d.x[3 * i + 2] = d.vel_orig[3 * g + 2];
}

// the replicas still iterating take one more residual round (r = b - A x
// from the warm x; no iteration has run, so it counts as no restart)
__global__ void k_bcg_rearm(DevPtrs d, BlockPtrs bp) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= d.nrep) return;
  BcgRep& B = bp.bcg[r];
  if (B.state == 0) B.state = 1;
}

__global__ __launch_bounds__(BLOCK_THREADS) void k_bcg_zero(DevPtrs d) {
  const int64_t i = (int64_t)blockIdx.x * BLOCK_THREADS + threadIdx.x;
  if (i >= d.rows) return;
  d.x[3 * i] = d.x[3 * i + 1] = d.x[3 * i + 2] = 0.0;
}

// Entry-parallel 3 x 3 block product over a 1024-row tile (the scalar CG's
// entry-parallel form with a block per entry): the tile's entries, one
// contiguous CSR range, are striped over the block's threads, BEP per thread
// and pass, so the column and block loads are coalesced and none waits on
// its own row's pointers; each thread forms W_e src_j for its entries into
// LDS, and after a barrier the thread of row i adds its row's products in
// entry order.  The tile's own rows of src come in through LDS as
// contiguous runs.  acc = sum_j W_ij src_j, si = src_i.  (Four lanes per row
// walking interleaved entries took 82.5 against 74.4 us at N = 1e6.)
constexpr int BEP = 2;
constexpr int BCAP = BLOCK_THREADS * BEP;
template <class Mul>
__device__ __forceinline__ void bep_tile(const DevPtrs& d, int tile, const double* __restrict__ src,
                                         Mul mul, double (*prod)[BCAP], double* io,
                                         double (&acc)[3], double (&si)[3]) {
  static_assert(ROWS_PER_BLOCK == BLOCK_THREADS, "one thread per row of the tile");
  const int t = threadIdx.x;
  const int64_t base = (int64_t)tile * ROWS_PER_BLOCK;
  // clamped: after an overflowing fill the row pointers may pass the
  // capacity (the host discards that solve; the reads stay in bounds)
  const int cap = (int)d.nnz_cap;
  const int E0 = min(d.rowptr[base], cap);
  const int ne = min(d.rowptr[base + ROWS_PER_BLOCK], cap) - E0;
  const int64_t i = base + t;
  const int r0 = min(d.rowptr[i], cap) - E0, r1 = min(d.rowptr[i + 1], cap) - E0;
#pragma unroll
  for (int q = 0; q < 3; ++q) io[t + q * BLOCK_THREADS] = src[3 * base + t + q * BLOCK_THREADS];
  acc[0] = acc[1] = acc[2] = 0.0;
  for (int c0 = 0; c0 < ne; c0 += BCAP) {
    int c[BEP];
#pragma unroll
    for (int k = 0; k < BEP; ++k) {
      const int e = c0 + t + k * BLOCK_THREADS;
      c[k] = e < ne ? d.col[E0 + e] : -1;
    }
#pragma unroll
    for (int k = 0; k < BEP; ++k) {
      if (c[k] >= 0) {
        const int64_t j = c[k];
        const double g[3] = {src[3 * j], src[3 * j + 1], src[3 * j + 2]};
        double o[3];
        mul((int64_t)E0 + c0 + t + k * BLOCK_THREADS, g, o);
        const int slot = t + k * BLOCK_THREADS;
        prod[0][slot] = o[0];
        prod[1][slot] = o[1];
        prod[2][slot] = o[2];
      }
    }
    __syncthreads();
    const int lo = r0 > c0 ? r0 : c0, hi = r1 < c0 + BCAP ? r1 : c0 + BCAP;
    for (int e = lo; e < hi; ++e) {
      acc[0] += prod[0][e - c0];
      acc[1] += prod[1][e - c0];
      acc[2] += prod[2][e - c0];
    }
    __syncthreads();
  }
  if (ne == 0) __syncthreads();  // the own rows in io, as after a pass
  si[0] = io[3 * t];
  si[1] = io[3 * t + 1];
  si[2] = io[3 * t + 2];
}

// three values per row of the tile to out[3 * (base + row) + k], through LDS
// as contiguous runs (io free: every thread has read its own row)
__device__ __forceinline__ void tile_store3(double* io, int64_t base, const double (&v)[3],
                                            double* __restrict__ out) {
  const int t = threadIdx.x;
  __syncthreads();
  io[3 * t] = v[0];
  io[3 * t + 1] = v[1];
  io[3 * t + 2] = v[2];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 3; ++q) out[3 * base + t + q * BLOCK_THREADS] = io[t + q * BLOCK_THREADS];
}

// mode 0: w = A u, partial (w, u)                        [iterating replicas]
// mode 1: r = b - A x, u = M^-1 r, p = s = 0, partials (r, u), (r, r)
//                                                          [residual round]
// FP32: the off-diagonal blocks of mode 0 from their FP32 copies (the
// residual round always takes the FP64 blocks, so the stopping test is the
// FP64 residual)
template <bool FP32>
__global__ __launch_bounds__(BLOCK_THREADS) void k_bcg_spmv(DevPtrs d, BlockPtrs bp, int mode) {
  const int tile = xcd_block(blockIdx.x, d.nblk);
  if (tile >= d.nblk) return;
  const BcgRep& B = bp.bcg[d.blk_rep[tile]];
  if (B.state != (mode == 0 ? 0 : 1)) return;
  __shared__ double prod[3][BCAP];
  __shared__ double io[3 * ROWS_PER_BLOCK];
  const double* src = mode == 0 ? d.u : d.x;
  double acc[3], si[3];
  bep_tile(d, tile, src,
           [&](int64_t e, const double (&g)[3], double (&o)[3]) {
             if constexpr (FP32)
               sym_mul_f(bp.bvalf + 6 * e, g, o);
             else
               sym_mul(bp.bval + 6 * e, g, o);
           },
           prod, io, acc, si);
  const int64_t base = (int64_t)tile * ROWS_PER_BLOCK;
  const int64_t i = base + threadIdx.x;
  double dg[3];
  sym_mul(bp.bdiag + 6 * i, si, dg);
  double own[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) own[k] = dg[k] + acc[k];
  if (mode == 0) {
    double v[1] = {(si[0] * own[0] + si[1] * own[1]) + si[2] * own[2]};
    tile_store3(io, base, own, d.w);
    tile_partials<1>(d, tile, 0, v);
  } else {
    const double r[3] = {d.b[3 * i] - own[0], d.b[3 * i + 1] - own[1], d.b[3 * i + 2] - own[2]};
    double z[3];
    sym_mul(bp.binv + 6 * i, r, z);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      d.r[3 * i + k] = r[k];
      if (!bp.learned) d.u[3 * i + k] = z[k];  // learned: k_bcg_apply forms u
      d.p[3 * i + k] = 0.0;
      d.s[3 * i + k] = 0.0;
    }
    double v[2] = {(r[0] * z[0] + r[1] * z[1]) + r[2] * z[2], (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2]};
    tile_partials<2>(d, tile, 1, v);
  }
}

// p = u + beta p, s = w + beta s, x += alpha p, r -= alpha s, u = M^-1 r,
// partials (r, u), (r, r).  The vector updates run element-parallel over
// the tile's 3 * 1024 consecutive doubles (coalesced); the new r goes
// through LDS to one thread per row for the 3 x 3 block product, and u
// back through LDS to coalesced stores.
__global__ __launch_bounds__(BLOCK_THREADS) void k_bcg_vec(DevPtrs d, BlockPtrs bp) {
  const int tile = xcd_block(blockIdx.x, d.nblk);
  if (tile >= d.nblk) return;
  const BcgRep& B = bp.bcg[d.blk_rep[tile]];
  if (B.state != 0) return;
  __shared__ double rs[3 * ROWS_PER_BLOCK];
  static_assert(ROWS_PER_BLOCK == BLOCK_THREADS, "one row per thread in the block product");
  const double a = B.alpha, be = B.beta;
  const int64_t base = (int64_t)tile * 3 * ROWS_PER_BLOCK;
  const int t = threadIdx.x;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const int le = q * BLOCK_THREADS + t;
    const int64_t e = base + le;
    const double pk = d.u[e] + be * d.p[e];
    const double sk = d.w[e] + be * d.s[e];
    d.p[e] = pk;
    d.s[e] = sk;
    d.x[e] += a * pk;
    const double rk = d.r[e] - a * sk;
    d.r[e] = rk;
    rs[le] = rk;
  }
  __syncthreads();
  const int64_t i = (int64_t)tile * ROWS_PER_BLOCK + t;
  const double r[3] = {rs[3 * t], rs[3 * t + 1], rs[3 * t + 2]};
  double z[3];
  sym_mul(bp.binv + 6 * i, r, z);
  double v[2] = {(r[0] * z[0] + r[1] * z[1]) + r[2] * z[2], (r[0] * r[0] + r[1] * r[1]) + r[2] * r[2]};
  __syncthreads();  // every row has read its r: rs now takes u
  rs[3 * t] = z[0];
  rs[3 * t + 1] = z[1];
  rs[3 * t + 2] = z[2];
  __syncthreads();
  if (!bp.learned)  // learned: k_bcg_apply forms u
#pragma unroll
    for (int q = 0; q < 3; ++q) d.u[base + q * BLOCK_THREADS + t] = rs[q * BLOCK_THREADS + t];
  tile_partials<2>(d, tile, 1, v);
}

// the learned preconditioner: u = M^-1 r with the stored blocks (M_ii
// symmetric FP64, M_ij row-major FP32), partial (r, u) into slot 1 (over the
// (r, B r) the vector pass or residual round left there).  mode 0 after a
// vector pass, 1 in a residual round.  Entry-parallel as k_bcg_spmv.
__global__ __launch_bounds__(BLOCK_THREADS) void k_bcg_apply(DevPtrs d, BlockPtrs bp, int mode) {
  const int tile = xcd_block(blockIdx.x, d.nblk);
  if (tile >= d.nblk) return;
  const BcgRep& B = bp.bcg[d.blk_rep[tile]];
  if (B.state != (mode == 0 ? 0 : 1)) return;
  __shared__ double prod[3][BCAP];
  __shared__ double io[3 * ROWS_PER_BLOCK];
  double acc[3], ri[3];
  bep_tile(d, tile, d.r,
           [&](int64_t e, const double (&g)[3], double (&o)[3]) { full_mul(bp.xo + 9 * e, g, o); },
           prod, io, acc, ri);
  const int64_t base = (int64_t)tile * ROWS_PER_BLOCK;
  const int64_t i = base + threadIdx.x;
  double dg[3];
  sym_mul(bp.xd + 6 * i, ri, dg);
  double u[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) u[k] = dg[k] + acc[k];
  double v[1] = {(ri[0] * u[0] + ri[1] * u[1]) + ri[2] * u[2]};
  tile_store3(io, base, u, d.u);
  tile_partials<1>(d, tile, 1, v);
}

// one block per replica: the tile partials [(w, u), (r, u), (r, r)] in tile
// order, then
//   mode 0 (after w = A u):   convergence of the recursive residual (-> a
//                             residual round), else beta and alpha of the
//                             next vector pass
//   mode 2 (residual round):  ||b||^2 on the first round; done if the true
//                             residual meets the tolerance, else (re)start
__global__ __launch_bounds__(256) void k_bcg_finish(DevPtrs d, BlockPtrs bp, int mode) {
  const int rid = blockIdx.x;
  BcgRep& B = bp.bcg[rid];
  if (B.state != (mode == 2 ? 1 : 0)) return;
  const RepDev& R = d.rep[rid];
  __shared__ double lds[4][3];
  double acc[3] = {0.0, 0.0, 0.0};
  for (int t = threadIdx.x; t < R.nblk; t += blockDim.x) {
    const double* src = d.partial + (int64_t)(R.blk_off + t) * NPART;
    acc[0] += src[0];
    acc[1] += src[1];
    acc[2] += src[2];
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 3; ++k) acc[k] = wave_sum(acc[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < 3; ++k) lds[wave][k] = acc[k];
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  double tot[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) tot[k] = ((lds[0][k] + lds[1][k]) + lds[2][k]) + lds[3][k];
  const double delta = tot[0], gamma = tot[1];
  if (mode == 0) {
    B.rr = tot[2];
    if (tot[2] <= B.tol2 * B.bb) {
      B.state = 1;
      return;
    }
    double beta = 0.0, den = delta;
    if (!B.first) {
      beta = gamma / B.rz;
      den = delta - beta * gamma / B.alpha;
    }
    if (!(den > 0.0) || !(gamma > 0.0)) {
      B.breakdown = 1;
      B.state = 2;
      return;
    }
    B.beta = beta;
    B.alpha = gamma / den;
    B.rz = gamma;
    B.first = 0;
    B.it += 1;
  } else {
    if (B.bb < 0.0) B.bb = tot[2];
    B.rr = tot[2];
    if (tot[2] <= B.tol2 * B.bb) {
      B.state = 2;
    } else {
      if (B.it > 0) B.restarts += 1;
      B.first = 1;
      B.state = 0;
    }
  }
}

// the block system in original ids: entries (row, col, 9 values row-major),
// diagonal blocks (9 values per particle) and right-hand sides
__global__ __launch_bounds__(BLOCK_THREADS) void k_block_export(DevPtrs d, BlockPtrs bp,
                                                                const int64_t* __restrict__ id_off,
                                                                int64_t* rows, int64_t* cols,
                                                                double* vals, double* diag,
                                                                double* rhs) {
  const int blk = blockIdx.x;
  const int rid = d.blk_rep[blk];
  const RepDev& R = d.rep[rid];
  const int64_t i = (int64_t)blk * ROWS_PER_BLOCK + threadIdx.x;
  if (i - R.row_off >= R.n) return;
  const int64_t g = id_off[rid] + (int64_t)d.pos[i].w;
  const int map[9] = {0, 1, 2, 1, 3, 4, 2, 4, 5};
  for (int64_t e = d.rowptr[i]; e < d.rowptr[i + 1]; ++e) {
    rows[e] = g;
    cols[e] = id_off[rid] + (int64_t)d.pos[d.col[e]].w;
    for (int m = 0; m < 9; ++m) vals[9 * e + m] = bp.bval[6 * e + map[m]];
  }
  for (int m = 0; m < 9; ++m) diag[9 * g + m] = bp.bdiag[6 * i + map[m]];
  for (int k = 0; k < 3; ++k) rhs[3 * g + k] = d.b[3 * i + k];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_pair_block(const DevPtrs& d, const BlockPtrs& bp, hipStream_t s) {
  hipLaunchKernelGGL(k_pair_block, dim3(xcd_grid(PB_TILES * d.nblk)), dim3(PB_THREADS), 0, s, d,
                     bp);
  return hipGetLastError();
}

hipError_t launch_bcg_reset(const DevPtrs& d, const BlockPtrs& bp, double tol, hipStream_t s) {
  hipLaunchKernelGGL(k_bcg_reset, dim3((d.nrep + 63) / 64), dim3(64), 0, s, d, bp, tol);
  hipLaunchKernelGGL(k_bcg_zero, dim3(d.nblk), dim3(BLOCK_THREADS), 0, s, d);
  return hipGetLastError();
}

hipError_t launch_bcg_warm(const DevPtrs& d, const BlockPtrs& bp, const int64_t* id_off,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_bcg_warm, dim3(d.nblk), dim3(BLOCK_THREADS), 0, s, d, bp, id_off);
  hipLaunchKernelGGL(k_bcg_rearm, dim3((d.nrep + 255) / 256), dim3(256), 0, s, d, bp);
  return hipGetLastError();
}
hipError_t launch_bcg_residual(const DevPtrs& d, const BlockPtrs& bp, hipStream_t s) {
  hipLaunchKernelGGL(k_bcg_spmv<false>, dim3(xcd_grid(d.nblk)), dim3(BLOCK_THREADS), 0, s, d, bp, 1);
  if (bp.learned)
    hipLaunchKernelGGL(k_bcg_apply, dim3(xcd_grid(d.nblk)), dim3(BLOCK_THREADS), 0, s, d, bp, 1);
  hipLaunchKernelGGL(k_bcg_finish, dim3(d.nrep), dim3(256), 0, s, d, bp, 2);
  return hipGetLastError();
}

hipError_t launch_bcg_iteration(const DevPtrs& d, const BlockPtrs& bp, hipStream_t s) {
  if (bp.fp32)
    hipLaunchKernelGGL(k_bcg_spmv<true>, dim3(xcd_grid(d.nblk)), dim3(BLOCK_THREADS), 0, s, d, bp, 0);
  else
    hipLaunchKernelGGL(k_bcg_spmv<false>, dim3(xcd_grid(d.nblk)), dim3(BLOCK_THREADS), 0, s, d, bp, 0);
  hipLaunchKernelGGL(k_bcg_finish, dim3(d.nrep), dim3(256), 0, s, d, bp, 0);
  hipLaunchKernelGGL(k_bcg_vec, dim3(xcd_grid(d.nblk)), dim3(BLOCK_THREADS), 0, s, d, bp);
  if (bp.learned)
    hipLaunchKernelGGL(k_bcg_apply, dim3(xcd_grid(d.nblk)), dim3(BLOCK_THREADS), 0, s, d, bp, 0);
  return hipGetLastError();
}

hipError_t launch_block_export(const DevPtrs& d, const BlockPtrs& bp, const int64_t* id_off,
                               int64_t* rows, int64_t* cols, double* vals, double* diag,
                               double* rhs, hipStream_t s) {
  hipLaunchKernelGGL(k_block_export, dim3(d.nblk), dim3(BLOCK_THREADS), 0, s, d, bp, id_off, rows,
                     cols, vals, diag, rhs);
  return hipGetLastError();
}
