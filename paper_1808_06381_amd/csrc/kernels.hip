// kernels.hip -- gfx950 kernels of one time step of the sheared mesoscale
// blob simulation (Korolkovas, arXiv 1808.06381, Method section):
//   binning + stable cell sort -> Lees-Edwards neighbour search ->
//   pair terms, assembly of A = gamma0 I + alpha L(w) and the rhs (Eq. 6-9)
//   -> preconditioned CG on (A (x) I3) v = b -> R += v dt with LE re-entry.
// Every kernel is row-parallel over the padded, cell-sorted row layout of
// sim_dev.h; reductions are deterministic (fixed trees, per-replica "last
// block finishes" with integer arrival counters, no float atomics).
#include "sim_dev.h"

#include <hip/hip_ext.h>
#include "launch.h"

#include <algorithm>

// ===========================================================================
// small utilities
// ===========================================================================
__global__ void k_fill_i32(int32_t* __restrict__ p, int32_t v, int64_t n) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// ---------------------------------------------------------------------------
// exclusive scan of int32 (3 passes: block sums, scan of block sums, down)
// ---------------------------------------------------------------------------
#define SCAN_ITEMS 8
#define SCAN_TILE (BLOCK_THREADS * SCAN_ITEMS)

__global__ __launch_bounds__(BLOCK_THREADS) void k_scan_reduce(const int32_t* __restrict__ in,
                                                               int64_t m,
                                                               int32_t* __restrict__ bsum) {
  __shared__ int32_t lds[BLOCK_THREADS / 64];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
  int32_t s = 0;
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    const int64_t i = base + (int64_t)k * BLOCK_THREADS + threadIdx.x;
    if (i < m) s += in[i];
  }
  for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    int32_t t = 0;
    for (int w = 0; w < BLOCK_THREADS / 64; ++w) t += lds[w];
    bsum[blockIdx.x] = t;
  }
}

// inclusive scan of one value per thread over the block (Hillis-Steele in LDS)
__device__ __forceinline__ int32_t block_incl_scan(int32_t v, int32_t* lds) {
  lds[threadIdx.x] = v;
  __syncthreads();
  for (int o = 1; o < (int)blockDim.x; o <<= 1) {
    const int32_t add = threadIdx.x >= (unsigned)o ? lds[threadIdx.x - o] : 0;
    __syncthreads();
    lds[threadIdx.x] += add;
    __syncthreads();
  }
  return lds[threadIdx.x];
}

// The block sums are scanned in 64 bits: if the total passes INT32_MAX the
// 32-bit offsets below would wrap, so *too_many (optional) is raised and the
// consumers of the offsets (the neighbour list) write nothing.
__device__ __forceinline__ int64_t block_incl_scan64(int64_t v, int64_t* lds) {
  lds[threadIdx.x] = v;
  __syncthreads();
  for (int o = 1; o < (int)blockDim.x; o <<= 1) {
    const int64_t add = threadIdx.x >= (unsigned)o ? lds[threadIdx.x - o] : 0;
    __syncthreads();
    lds[threadIdx.x] += add;
    __syncthreads();
  }
  return lds[threadIdx.x];
}

__global__ __launch_bounds__(1024) void k_scan_top(int32_t* __restrict__ bsum, int64_t nb,
                                                   int32_t* __restrict__ too_many) {
  __shared__ int64_t lds[1024];
  __shared__ int64_t carry;
  if (threadIdx.x == 0) carry = 0;
  __syncthreads();
  for (int64_t base = 0; base < nb; base += 1024) {
    const int64_t i = base + threadIdx.x;
    const int64_t v = i < nb ? bsum[i] : 0;
    const int64_t inc = block_incl_scan64(v, lds);
    const int64_t c = carry;
    if (i < nb) bsum[i] = (int32_t)(c + inc - v);
    __syncthreads();
    if (threadIdx.x == 1023) carry = c + inc;
    __syncthreads();
  }
  if (threadIdx.x == 0 && too_many && carry > (int64_t)INT32_MAX) *too_many = 1;
}

__global__ __launch_bounds__(BLOCK_THREADS) void k_scan_down(const int32_t* __restrict__ in,
                                                             int64_t m,
                                                             const int32_t* __restrict__ bsum,
                                                             int32_t* __restrict__ out) {
  __shared__ int32_t lds[BLOCK_THREADS];
  const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)threadIdx.x * SCAN_ITEMS;
  int32_t v[SCAN_ITEMS];
  int32_t tot = 0;
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    v[k] = base + k < m ? in[base + k] : 0;
    tot += v[k];
  }
  const int32_t inc = block_incl_scan(tot, lds);
  int32_t run = bsum[blockIdx.x] + inc - tot;
  for (int k = 0; k < SCAN_ITEMS; ++k) {
    if (base + k < m) out[base + k] = run;
    run += v[k];
  }
}

// ===========================================================================
// a1: binning and the stable cell sort
// ===========================================================================
__device__ __forceinline__ int rep_of_entry(const RepDev* rep, int nrep, int e) {
  int lo = 0, hi = nrep - 1;
  while (lo < hi) {  // last replica with seg_off <= e
    const int mid = (lo + hi + 1) >> 1;
    if (rep[mid].seg_off <= e) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

// cell of every real particle; slot inside the cell by an integer atomic
__global__ __launch_bounds__(BLOCK_THREADS) void k_bin(DevPtrs d) {
  const int blk = blockIdx.x;
  const RepDev& R = d.rep[d.blk_rep[blk]];
  for (int u = 0; u < ROWS_PER_BLOCK / BLOCK_THREADS; ++u) {
    const int64_t i = (int64_t)blk * ROWS_PER_BLOCK + u * BLOCK_THREADS + threadIdx.x;
    if (i - R.row_off >= R.n) continue;
    const double4 pp = d.pos[i];
    const int cx = cell_axis(pp.x, R, 0), cy = cell_axis(pp.y, R, 1), cz = cell_axis(pp.z, R, 2);
    const int c = R.seg_off + cell_key(R, cx, cy, cz);
    d.cellidx[i] = c;
    d.slot[i] = atomicAdd(&d.cell_count[c], 1);
  }
}

// scanned counts -> absolute first row of every cell entry of each segment
__global__ void k_cell_rows(DevPtrs d, const int32_t* __restrict__ scan) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= d.ncell_entries) return;
  const int r = rep_of_entry(d.rep, d.nrep, e);
  const RepDev& R = d.rep[r];
  d.cell_row[e] = (int32_t)(scan[e] - scan[R.seg_off] + R.row_off);
}

__global__ __launch_bounds__(BLOCK_THREADS) void k_scatter(DevPtrs d) {
  const int blk = blockIdx.x;
  const RepDev& R = d.rep[d.blk_rep[blk]];
  for (int u = 0; u < ROWS_PER_BLOCK / BLOCK_THREADS; ++u) {
    const int64_t i = (int64_t)blk * ROWS_PER_BLOCK + u * BLOCK_THREADS + threadIdx.x;
    if (i - R.row_off >= R.n) continue;
    const int c = d.cellidx[i];
    const int64_t dst = (int64_t)d.cell_row[c] + d.slot[i];
    d.pos_alt[dst] = d.pos[i];
    d.cellidx_alt[dst] = c;
  }
}

// order each cell by original id (cells hold a handful of particles), so the
// layout does not depend on the order the atomics were served in
__global__ void k_cell_sort(DevPtrs d) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= d.ncell_entries) return;
  const int r = rep_of_entry(d.rep, d.nrep, e);
  const RepDev& R = d.rep[r];
  const int ncell = R.nc[0] * R.nc[1] * R.nc[2];
  if (e - R.seg_off >= ncell) return;  // terminal entry of the segment
  const int a = d.cell_row[e], b = d.cell_row[e + 1];
  const int n = b - a;
  if (n <= 1) return;
  if (n <= 8) {
    // in registers: Batcher's odd-even merge network on 8 (19 compare-
    // exchanges, checked against every permutation), absent slots keyed +inf
    constexpr int NET[19][2] = {{0, 1}, {2, 3}, {4, 5}, {6, 7}, {0, 2}, {1, 3}, {4, 6},
                                {5, 7}, {1, 2}, {5, 6}, {0, 4}, {1, 5}, {2, 6}, {3, 7},
                                {2, 4}, {3, 5}, {1, 2}, {3, 4}, {5, 6}};
    double4 v[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) v[k] = k < n ? d.pos[a + k] : make_double4(0.0, 0.0, 0.0, INFINITY);
#pragma unroll
    for (int c = 0; c < 19; ++c) {
      const double4 lo = v[NET[c][0]], hi = v[NET[c][1]];
      const bool sw = lo.w > hi.w;
      v[NET[c][0]] = sw ? hi : lo;
      v[NET[c][1]] = sw ? lo : hi;
    }
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (k < n) d.pos[a + k] = v[k];
    return;
  }
  for (int i = a + 1; i < b; ++i) {
    const double4 key = d.pos[i];
    int j = i - 1;
    while (j >= a && d.pos[j].w > key.w) {
      d.pos[j + 1] = d.pos[j];
      --j;
    }
    d.pos[j + 1] = key;
  }
}

// ===========================================================================
// a2-a5: neighbour search, pair terms, assembly of A and b
// ===========================================================================
// Neighbour count.  The first NBR_SLOTS accepted candidates of each row are
// also kept, slot-major (slots[k * rows + i]), so that the list pass copies
// them instead of searching the stencil again.
__global__ __launch_bounds__(BLOCK_THREADS) void k_nbr_count(DevPtrs d, int32_t* __restrict__ slots) {
  const int blk = xcd_block(blockIdx.x, d.nblk);  // neighbour rows in this XCD's L2
  if (blk >= d.nblk) return;
  // a copy: the box constants stay in registers across the candidate loop
  // (through the reference they were reloaded after every slot store: 1619
  // -> 1580 us at N = 8e6)
  const RepDev R = d.rep[d.blk_rep[blk]];
  const int64_t step = *d.step_d;
  const double delta = le_offset(R, step);
  int mx = 0;
  for (int u = 0; u < ROWS_PER_BLOCK / BLOCK_THREADS; ++u) {
    const int64_t i = (int64_t)blk * ROWS_PER_BLOCK + u * BLOCK_THREADS + threadIdx.x;
    int cnt = 0;
    if (i - R.row_off < R.n) {
      const double4 pi = d.pos[i];
      for_candidates(R, d.cell_row, delta, pi.x, pi.y, pi.z, i, [&](int j) {
        const double4 pj = d.pos[j];
        double dx, dy, dz;
        le_sep(R, delta, pi.x, pi.y, pi.z, pj.x, pj.y, pj.z, dx, dy, dz);
        if (dist2(dx, dy, dz) < R.rc2) {
          if (cnt < NBR_SLOTS) slots[(int64_t)cnt * d.rows + i] = j;
          ++cnt;
        }
      });
    }
    d.rowlen[i] = cnt;
    mx = cnt > mx ? cnt : mx;
  }
  // longest row: one atomic per block (atomics on one address serialise
  // across the chip)
  __shared__ int wmax[BLOCK_THREADS / 64];
  for (int o = 32; o > 0; o >>= 1) {
    const int t = __shfl_xor(mx, o, 64);
    mx = t > mx ? t : mx;
  }
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < BLOCK_THREADS / 64; ++w) mx = wmax[w] > mx ? wmax[w] : mx;
    if (mx > 0) atomicMax(&d.ctrl->max_row, mx);
  }
}

__device__ __forceinline__ double pair_weight(const RepDev& R, double r2, double r) {
  if (R.weight_law == 0) return exp(-0.5 * r2 * R.inv_lam2);
  const double t = 1.0 - r / R.rc;
  return t * t;
}

__device__ __forceinline__ double force_coef(const RepDev& R, double r2, double r) {
  if (R.potential == 0) return R.force_gc * exp(-0.5 * r2 * R.inv_lam2);
  if (R.potential == 1) return r > 0.0 ? R.force_soft * (1.0 - r / R.rc) / r : 0.0;
  return 0.0;
}

// Neighbour list: each passing candidate's sorted row index goes to
// col[rowptr[i] + k], in k_nbr_count's candidate order: copied from the
// count pass's slots, or searched again for a row longer than NBR_SLOTS.
__global__ __launch_bounds__(BLOCK_THREADS) void k_nbr_list(DevPtrs d,
                                                            const int32_t* __restrict__ slots) {
  const int blk = xcd_block(blockIdx.x, d.nblk);  // neighbour rows in this XCD's L2
  if (blk >= d.nblk) return;
  const RepDev& R = d.rep[d.blk_rep[blk]];
  const int64_t step = *d.step_d;
  const double delta = le_offset(R, step);
  for (int u = 0; u < ROWS_PER_BLOCK / BLOCK_THREADS; ++u) {
    const int64_t i = (int64_t)blk * ROWS_PER_BLOCK + u * BLOCK_THREADS + threadIdx.x;
    if (i - R.row_off >= R.n) continue;
    if (d.ctrl->too_many) {  // offsets wrapped: nothing is written, the fill fails
      atomicOr(&d.ctrl->overflow, 1);
      continue;
    }
    const int64_t e1 = d.rowptr[i + 1];
    if (e1 > d.nnz_cap) {
      atomicOr(&d.ctrl->overflow, 1);
      continue;
    }
    int64_t e = d.rowptr[i];
    if (e1 - e <= NBR_SLOTS) {
      for (int k = 0; e < e1; ++k, ++e) d.col[e] = slots[(int64_t)k * d.rows + i];
      continue;
    }
    const double4 pi = d.pos[i];
    for_candidates(R, d.cell_row, delta, pi.x, pi.y, pi.z, i, [&](int j) {
      const double4 pj = d.pos[j];
      double dx, dy, dz;
      le_sep(R, delta, pi.x, pi.y, pi.z, pj.x, pj.y, pj.z, dx, dy, dz);
      if (dist2(dx, dy, dz) < R.rc2) d.col[e++] = j;
    });
  }
  if (blockIdx.x == 0 && threadIdx.x == 0 && !d.ctrl->too_many) d.ctrl->nnz = d.rowptr[d.rows];
}

// Pair terms and assembly: -alpha*w_ij into val, diag = gamma0 + alpha*sum w,
// 1/diag, and the three right-hand sides: Couette drive (Eq. 6c),
// conservative force (Eq. 6b), boundary velocity term of Eq. 8, thermal
// force.  A block owns a tile of PAIR_THREADS rows (a quarter of a row
// block, so that the grid holds enough waves to hide the gathers) and walks
// the tile's CSR entries (contiguous) in chunks of PAIR_THREADS, one entry
// per lane, so every lane has an entry to work on whatever the row lengths;
// each entry leaves its five row contributions (w, w s, and the three force
// components with the pair noise) in LDS, and each thread then adds those of
// its row in entry order.  The node noise and the assembly run once per row.
#define PAIR_THREADS 256
#define PAIR_TILES (ROWS_PER_BLOCK / PAIR_THREADS)   // tiles per row block
__global__ __launch_bounds__(PAIR_THREADS) void k_pair_terms(DevPtrs d) {
  const int tile = xcd_block(blockIdx.x, PAIR_TILES * d.nblk);  // rows in this XCD's L2
  if (tile >= PAIR_TILES * d.nblk) return;
  const int blk = tile / PAIR_TILES;
  const RepDev R = d.rep[d.blk_rep[blk]];  // a copy: no reloads after the entry stores
  if (d.ctrl->overflow) return;
  __shared__ int rp[PAIR_THREADS + 1];        // row pointers of the tile
  __shared__ int16_t erow[PAIR_THREADS];      // tile row of each entry of the chunk
  __shared__ double contrib[5][PAIR_THREADS]; // w, w s, fx, fy, fz of each entry
  const int t = threadIdx.x;
  const int64_t row0 = (int64_t)blk * ROWS_PER_BLOCK + (tile % PAIR_TILES) * PAIR_THREADS;
  for (int r = t; r <= PAIR_THREADS; r += PAIR_THREADS) rp[r] = d.rowptr[row0 + r];
  __syncthreads();
  const int64_t step = *d.step_d;
  const double delta = le_offset(R, step);
  const bool noise = R.amp_pair != 0.0 && R.alpha != 0.0;
  // this thread's row: t (tile-local)
  double acc[5];
#pragma unroll
  for (int k = 0; k < 5; ++k) acc[k] = 0.0;
  const int E0 = rp[0], E1 = rp[PAIR_THREADS];
  for (int cb = E0; cb < E1; cb += PAIR_THREADS) {
    // the tile row of each entry of this chunk
    {
      const int lo = max(rp[t], cb), hi = min(rp[t + 1], cb + PAIR_THREADS);
      for (int e = lo; e < hi; ++e) erow[e - cb] = (int16_t)t;
    }
    __syncthreads();
    const int e = cb + t;
    if (e < E1) {
      const int64_t i = row0 + erow[t];
      const double4 pi = d.pos[i];
      const int j = d.col[e];
      const double4 pj = d.pos[j];
      double dx, dy, dz;
      const int s = le_sep(R, delta, pi.x, pi.y, pi.z, pj.x, pj.y, pj.z, dx, dy, dz);
      const double r2 = dist2(dx, dy, dz);
      const double r = sqrt(r2);
      const double w = pair_weight(R, r2, r);
      d.val[e] = -R.alpha * w;
      // the FP32 copy and the network's edge input only where they are read
      if (d.spmv_fp32) d.valf[e] = (float)(-R.alpha * w);
      if (d.want_er) d.er[e] = (float)(r / R.rc);
      const double fc = force_coef(R, r2, r);
      double fx = fc * dx, fy = fc * dy, fz = fc * dz;
      if (noise) {
        const int64_t idi = (int64_t)pi.w, idj = (int64_t)pj.w;
        const int64_t a = idi < idj ? idi : idj, bb = idi < idj ? idj : idi;
        double g[3];
        if (d.inj_eta) {
          const double* src = d.inj_eta + 3 * (a * (int64_t)R.n + bb);
          g[0] = src[0]; g[1] = src[1]; g[2] = src[2];
        } else {
          gauss3(R.seed, R.stream, (uint64_t)step, 1, (uint64_t)a, (uint64_t)bb, g);
        }
        const double amp = (idi < idj ? 1.0 : -1.0) * R.amp_pair * sqrt(R.alpha * w);
        fx += amp * g[0];
        fy += amp * g[1];
        fz += amp * g[2];
      }
      contrib[0][t] = w;
      contrib[1][t] = w * (double)s;
      contrib[2][t] = fx;
      contrib[3][t] = fy;
      contrib[4][t] = fz;
    }
    __syncthreads();
    {
      const int lo = max(rp[t], cb), hi = min(rp[t + 1], cb + PAIR_THREADS);
      for (int e2 = lo; e2 < hi; ++e2)
#pragma unroll
        for (int k = 0; k < 5; ++k) acc[k] += contrib[k][e2 - cb];
    }
    __syncthreads();  // erow and contrib are rewritten for the next chunk
  }
  const double drag_unit = R.alpha * (R.shear * R.L[1]);
  {
    const int64_t i = row0 + t;
    if (i - R.row_off >= R.n) {  // padding row: identity, no right-hand side
      d.diag[i] = 1.0;
      d.dinv[i] = 1.0;
      d.b[3 * i] = d.b[3 * i + 1] = d.b[3 * i + 2] = 0.0;
      return;
    }
    const double4 pi = d.pos[i];
    const int64_t idi = (int64_t)pi.w;
    double g[3] = {0.0, 0.0, 0.0};
    if (R.amp_node != 0.0) {
      if (d.inj_xi) {
        g[0] = d.inj_xi[3 * idi]; g[1] = d.inj_xi[3 * idi + 1]; g[2] = d.inj_xi[3 * idi + 2];
      } else {
        gauss3(R.seed, R.stream, (uint64_t)step, 0, (uint64_t)idi, 0, g);
      }
    }
    const double dg = R.gamma0 + R.alpha * acc[0];
    d.diag[i] = dg;
    d.dinv[i] = 1.0 / dg;
    d.b[3 * i] = R.gamma0 * R.shear * (pi.y - R.hL[1]) + R.amp_node * g[0] + acc[2] +
                 drag_unit * acc[1];
    d.b[3 * i + 1] = R.amp_node * g[1] + acc[3];
    d.b[3 * i + 2] = R.amp_node * g[2] + acc[4];
  }
}

__global__ void k_ctrl_zero(Ctrl* c) {
  if (threadIdx.x == 0) {
    c->overflow = 0;
    c->numeric = 0;
    c->max_row = 0;
    c->nnz = 0;
    c->breakdown = 0;
    c->too_many = 0;
  }
}

// ===========================================================================
// a7: position update with Lees-Edwards re-entry
// ===========================================================================
// cond = 1 (graph replay): only if the solve finished (ctrl_commit_ok)
__global__ __launch_bounds__(BLOCK_THREADS) void k_update(DevPtrs d, int cond) {
  if (cond && !ctrl_commit_ok(d.ctrl)) return;
  const int blk = blockIdx.x;
  const RepDev& R = d.rep[d.blk_rep[blk]];
  const double delta = le_offset(R, *d.step_d + 1);
  for (int u = 0; u < ROWS_PER_BLOCK / BLOCK_THREADS; ++u) {
    const int64_t i = (int64_t)blk * ROWS_PER_BLOCK + u * BLOCK_THREADS + threadIdx.x;
    if (i - R.row_off >= R.n) continue;
    double4 pp = d.pos[i];
    const double vx = d.x[3 * i], vy = d.x[3 * i + 1], vz = d.x[3 * i + 2];
    double x = pp.x + vx * R.dt, y = pp.y + vy * R.dt, z = pp.z + vz * R.dt;
    if (y >= R.L[1]) { y = y - R.L[1]; x = x - delta; }
    else if (y < 0.0) { y = y + R.L[1]; x = x + delta; }
    for (int k = 0; k < 3; ++k)
      if (x >= R.L[0]) x = x - R.L[0];
    for (int k = 0; k < 3; ++k)
      if (x < 0.0) x = x + R.L[0];
    if (z >= R.L[2]) z = z - R.L[2];
    else if (z < 0.0) z = z + R.L[2];
    const bool ok = x >= 0.0 && x <= R.L[0] && y >= 0.0 && y <= R.L[1] && z >= 0.0 && z <= R.L[2];
    if (!ok) atomicOr(&d.ctrl->numeric, 1);
    pp.x = x; pp.y = y; pp.z = z;
    d.pos_alt[i] = pp;
  }
}

// velocities of the step in original order: vel_orig[3*(off + id) + k]
__global__ __launch_bounds__(BLOCK_THREADS) void k_save_vel(DevPtrs d, const int64_t* __restrict__ id_off,
                                                            int cond) {
  if (cond && !(ctrl_commit_ok(d.ctrl) && d.ctrl->numeric == 0)) return;
  const int blk = blockIdx.x;
  const int rid = d.blk_rep[blk];
  const RepDev& R = d.rep[rid];
  for (int u = 0; u < ROWS_PER_BLOCK / BLOCK_THREADS; ++u) {
    const int64_t i = (int64_t)blk * ROWS_PER_BLOCK + u * BLOCK_THREADS + threadIdx.x;
    if (i - R.row_off >= R.n) continue;
    const int64_t g = id_off[rid] + (int64_t)d.pos[i].w;
    for (int k = 0; k < 3; ++k) d.vel_orig[3 * g + k] = d.x[3 * i + k];
  }
}

// n -> n + 1 on the device (cond = 1: only for a committed step)
__global__ void k_step_commit(DevPtrs d, int cond) {
  if (threadIdx.x != 0) return;
  if (cond && !(ctrl_commit_ok(d.ctrl) && d.ctrl->numeric == 0)) return;
  *d.step_d += 1;
}

// ===========================================================================
// boundary helpers: original-order <-> sorted-order gathers
// ===========================================================================
// mode 0: out[g] = pos.xyz; mode 1: b[i] = in[g]; mode 2: out[g] = x[i]
__global__ __launch_bounds__(BLOCK_THREADS) void k_permute(DevPtrs d, const int64_t* __restrict__ id_off,
                                                           int mode, const double* __restrict__ in,
                                                           double* __restrict__ out) {
  const int blk = blockIdx.x;
  const int rid = d.blk_rep[blk];
  const RepDev& R = d.rep[rid];
  for (int u = 0; u < ROWS_PER_BLOCK / BLOCK_THREADS; ++u) {
    const int64_t i = (int64_t)blk * ROWS_PER_BLOCK + u * BLOCK_THREADS + threadIdx.x;
    if (i - R.row_off >= R.n) continue;
    const double4 pp = d.pos[i];
    const int64_t g = id_off[rid] + (int64_t)pp.w;
    if (mode == 0) {
      out[3 * g] = pp.x; out[3 * g + 1] = pp.y; out[3 * g + 2] = pp.z;
    } else if (mode == 1) {
      for (int k = 0; k < 3; ++k) d.b[3 * i + k] = in[3 * g + k];
    } else {
      for (int k = 0; k < 3; ++k) out[3 * g + k] = d.x[3 * i + k];
    }
  }
}

// parity export of pairs (replica, i, j), i < j original ids; atomic slot
__global__ __launch_bounds__(BLOCK_THREADS) void k_export_pairs(DevPtrs d, int64_t* __restrict__ out,
                                                                int64_t cap,
                                                                unsigned long long* __restrict__ cnt) {
  const int blk = blockIdx.x;
  const int rid = d.blk_rep[blk];
  const RepDev& R = d.rep[rid];
  for (int u = 0; u < ROWS_PER_BLOCK / BLOCK_THREADS; ++u) {
    const int64_t i = (int64_t)blk * ROWS_PER_BLOCK + u * BLOCK_THREADS + threadIdx.x;
    if (i - R.row_off >= R.n) continue;
    const int64_t idi = (int64_t)d.pos[i].w;
    for (int e = d.rowptr[i]; e < d.rowptr[i + 1]; ++e) {
      const int64_t idj = (int64_t)d.pos[d.col[e]].w;
      if (idj <= idi) continue;
      const unsigned long long k = atomicAdd(cnt, 1ULL);
      if ((int64_t)k < cap) {
        out[3 * k] = rid; out[3 * k + 1] = idi; out[3 * k + 2] = idj;
      }
    }
  }
}

// parity export of A (row, col, val in global original numbering), diag, rhs
__global__ __launch_bounds__(BLOCK_THREADS) void k_export_system(DevPtrs d, const int64_t* __restrict__ id_off,
                                                                 int64_t* __restrict__ rows, int64_t* __restrict__ cols,
                                                                 double* __restrict__ vals, int64_t cap,
                                                                 double* __restrict__ diag_out,
                                                                 double* __restrict__ rhs_out) {
  const int blk = blockIdx.x;
  const int rid = d.blk_rep[blk];
  const RepDev& R = d.rep[rid];
  for (int u = 0; u < ROWS_PER_BLOCK / BLOCK_THREADS; ++u) {
    const int64_t i = (int64_t)blk * ROWS_PER_BLOCK + u * BLOCK_THREADS + threadIdx.x;
    if (i - R.row_off >= R.n) continue;
    const int64_t gi = id_off[rid] + (int64_t)d.pos[i].w;
    diag_out[gi] = d.diag[i];
    for (int k = 0; k < 3; ++k) rhs_out[3 * gi + k] = d.b[3 * i + k];
    // entries are packed by sorted row: offset = rowptr - rowptr of replica start
    for (int e = d.rowptr[i]; e < d.rowptr[i + 1]; ++e) {
      if (e >= cap) break;
      rows[e] = gi;
      cols[e] = id_off[rid] + (int64_t)d.pos[d.col[e]].w;
      vals[e] = d.val[e];
    }
  }
}

// plain 16-byte-per-lane copy (bandwidth reference)
__global__ __launch_bounds__(BLOCK_THREADS) void k_copy16(const uint4* __restrict__ src,
                                                          uint4* __restrict__ dst, int64_t n16) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride)
    dst[i] = src[i];
}

// ===========================================================================
// host launchers (C++ linkage, used by sim_api.hip)
// ===========================================================================
static inline unsigned nb_of(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

// ev0/ev1 (optional): the launch-bound event pair of the kernel timing probe
hipError_t launch_copy16(const void* src, void* dst, int64_t bytes, hipStream_t s,
                         hipEvent_t ev0, hipEvent_t ev1) {
  const int64_t n16 = bytes / 16;
  const int64_t want = (n16 + BLOCK_THREADS * 4 - 1) / (BLOCK_THREADS * 4);
  const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>(want, 256 * 16));
  if (ev0 || ev1)
    hipExtLaunchKernelGGL(k_copy16, dim3(grid), dim3(BLOCK_THREADS), 0, s, ev0, ev1, 0,
                          (const uint4*)src, (uint4*)dst, n16);
  else
    hipLaunchKernelGGL(k_copy16, dim3(grid), dim3(BLOCK_THREADS), 0, s, (const uint4*)src,
                       (uint4*)dst, n16);
  return hipGetLastError();
}

hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_i32, dim3(nb_of(n, 256)), dim3(256), 0, s, p, v, n);
  return hipGetLastError();
}

hipError_t launch_scan(const int32_t* in, int32_t* out, int64_t m, int32_t* bsum, hipStream_t s,
                       int32_t* too_many) {
  const int64_t nb = (m + SCAN_TILE - 1) / SCAN_TILE;
  hipLaunchKernelGGL(k_scan_reduce, dim3((unsigned)nb), dim3(BLOCK_THREADS), 0, s, in, m, bsum);
  hipLaunchKernelGGL(k_scan_top, dim3(1), dim3(1024), 0, s, bsum, nb, too_many);
  hipLaunchKernelGGL(k_scan_down, dim3((unsigned)nb), dim3(BLOCK_THREADS), 0, s, in, m, bsum, out);
  return hipGetLastError();
}

int64_t scan_bsum_len(int64_t m) { return (m + SCAN_TILE - 1) / SCAN_TILE; }

hipError_t launch_bin(const DevPtrs& d, hipStream_t s) {
  hipLaunchKernelGGL(k_bin, dim3(d.nblk), dim3(BLOCK_THREADS), 0, s, d);
  return hipGetLastError();
}
hipError_t launch_cell_rows(const DevPtrs& d, const int32_t* scan, hipStream_t s) {
  hipLaunchKernelGGL(k_cell_rows, dim3(nb_of(d.ncell_entries, 256)), dim3(256), 0, s, d, scan);
  return hipGetLastError();
}
hipError_t launch_scatter(const DevPtrs& d, hipStream_t s) {
  hipLaunchKernelGGL(k_scatter, dim3(d.nblk), dim3(BLOCK_THREADS), 0, s, d);
  return hipGetLastError();
}
hipError_t launch_cell_sort(const DevPtrs& d, hipStream_t s) {
  hipLaunchKernelGGL(k_cell_sort, dim3(nb_of(d.ncell_entries, 256)), dim3(256), 0, s, d);
  return hipGetLastError();
}
hipError_t launch_nbr_count(const DevPtrs& d, int32_t* slots, hipStream_t s) {
  hipLaunchKernelGGL(k_nbr_count, dim3(xcd_grid(d.nblk)), dim3(BLOCK_THREADS), 0, s, d, slots);
  return hipGetLastError();
}
hipError_t launch_nbr_list(const DevPtrs& d, const int32_t* slots, hipStream_t s) {
  hipLaunchKernelGGL(k_nbr_list, dim3(xcd_grid(d.nblk)), dim3(BLOCK_THREADS), 0, s, d, slots);
  return hipGetLastError();
}
hipError_t launch_pair_terms(const DevPtrs& d, hipStream_t s) {
  hipLaunchKernelGGL(k_pair_terms, dim3(xcd_grid(PAIR_TILES * d.nblk)), dim3(PAIR_THREADS), 0, s,
                     d);
  return hipGetLastError();
}
hipError_t launch_ctrl_zero(const DevPtrs& d, hipStream_t s) {
  hipLaunchKernelGGL(k_ctrl_zero, dim3(1), dim3(64), 0, s, d.ctrl);
  return hipGetLastError();
}
hipError_t launch_update(const DevPtrs& d, int cond, hipStream_t s) {
  hipLaunchKernelGGL(k_update, dim3(d.nblk), dim3(BLOCK_THREADS), 0, s, d, cond);
  return hipGetLastError();
}
hipError_t launch_save_vel(const DevPtrs& d, const int64_t* id_off, int cond, hipStream_t s) {
  hipLaunchKernelGGL(k_save_vel, dim3(d.nblk), dim3(BLOCK_THREADS), 0, s, d, id_off, cond);
  return hipGetLastError();
}
hipError_t launch_step_commit(const DevPtrs& d, int cond, hipStream_t s) {
  hipLaunchKernelGGL(k_step_commit, dim3(1), dim3(64), 0, s, d, cond);
  return hipGetLastError();
}
hipError_t launch_permute(const DevPtrs& d, const int64_t* id_off, int mode, const double* in,
                          double* out, hipStream_t s) {
  hipLaunchKernelGGL(k_permute, dim3(d.nblk), dim3(BLOCK_THREADS), 0, s, d, id_off, mode, in, out);
  return hipGetLastError();
}
hipError_t launch_export_pairs(const DevPtrs& d, int64_t* out, int64_t cap,
                               unsigned long long* cnt, hipStream_t s) {
  hipLaunchKernelGGL(k_export_pairs, dim3(d.nblk), dim3(BLOCK_THREADS), 0, s, d, out, cap, cnt);
  return hipGetLastError();
}
hipError_t launch_export_system(const DevPtrs& d, const int64_t* id_off, int64_t* rows,
                                int64_t* cols, double* vals, int64_t cap, double* diag,
                                double* rhs, hipStream_t s) {
  hipLaunchKernelGGL(k_export_system, dim3(d.nblk), dim3(BLOCK_THREADS), 0, s, d, id_off, rows,
                     cols, vals, cap, diag, rhs);
  return hipGetLastError();
}
