// ic0.hip -- incomplete Cholesky IC(0) preconditioner for the CG solve of
// Eq. 9 (Method section) in multicolour order (Meijerink & van der Vorst,
// Math. Comp. 31, 1977: IC(0) of a symmetric M-matrix exists without
// breakdown; A = gamma0 I + alpha L(w) is one).
//
// Ordering.  Cells are coloured by the parity of their coordinates, a third
// colour for the last cell of an odd axis: cells of one colour are two or
// more cells apart on some axis, so their particles are never pairs (cell
// side >= r_c), also across the sheared y boundary, where the y colours of
// the two sides always differ.  IC(0) is taken in the order (colour, row):
// rows of one colour depend only on earlier colours and on earlier rows of
// their own cell.  One launch per colour; the factorisation takes one
// thread per cell walking its rows in order, the triangular solves four
// lanes per cell; 2 x colours launches per application (forward, backward).
//
// Storage: L in A's row pointers.  Row i holds its lower entries
// (rank(j) < rank(i)) in ascending rank, then its upper entries in
// descending rank with the mirrored values L_ji, so that both triangular
// solves subtract in the order of the plain sequential algorithm.
#include <hip/hip_runtime.h>

#include "launch.h"
#include "sim_dev.h"

namespace {

__device__ __forceinline__ int row_color(const DevPtrs& d, int64_t i) {
  return d.cell_color[d.cellidx[i]];
}

// rank key of row j: (colour, row)
__device__ __forceinline__ int64_t rank_key(const DevPtrs& d, int64_t j) {
  return ((int64_t)row_color(d, j) << 32) | (int64_t)j;
}

__device__ __forceinline__ void cell_rows(const DevPtrs& d, int cell, int& a, int& b) {
  a = d.cell_row[cell];
  b = d.cell_row[cell + 1];
}

}  // namespace

// Factor the rows of the cells cells[0..count): for each row in order, its
// lower entries by increasing rank:
//   L_ij = (A_ij - sum_{k lower than j} L_ik L_jk) / L_jj,
//   L_ii = sqrt(A_ii - sum_j L_ij^2)
// (the sums over the common lower neighbours in increasing rank).
// Rows of up to IC_REG entries keep their columns and rank keys in
// registers (loaded once; constant-index loops), so the rank selection
// reads no memory; longer rows search the CSR entries directly.
constexpr int IC_REG = 16;

__device__ __forceinline__ void ic_load_row(const DevPtrs& d, int e0, int n, int (&cc)[IC_REG],
                                            int64_t (&kk)[IC_REG]) {
#pragma unroll
  for (int q = 0; q < IC_REG; ++q) {
    cc[q] = q < n ? d.col[e0 + q] : 0;
    kk[q] = q < n ? rank_key(d, cc[q]) : 0;
  }
}

// the entry of smallest rank in (lo, hi) (register form); -1 if none
__device__ __forceinline__ int ic_pick_up(const int64_t (&kk)[IC_REG], int n, int64_t lo,
                                          int64_t hi, int64_t& best) {
  int pick = -1;
  best = hi;
#pragma unroll
  for (int q = 0; q < IC_REG; ++q)
    if (q < n && kk[q] > lo && kk[q] < best) {
      best = kk[q];
      pick = q;
    }
  return pick;
}

// the entry of largest rank in (lo, hi) (register form); -1 if none
__device__ __forceinline__ int ic_pick_down(const int64_t (&kk)[IC_REG], int n, int64_t lo,
                                            int64_t hi, int64_t& best) {
  int pick = -1;
  best = lo;
#pragma unroll
  for (int q = 0; q < IC_REG; ++q)
    if (q < n && kk[q] < hi && kk[q] > best) {
      best = kk[q];
      pick = q;
    }
  return pick;
}

__device__ __forceinline__ int ic_col_at(const int (&cc)[IC_REG], int pick) {
  int j = 0;
#pragma unroll
  for (int q = 0; q < IC_REG; ++q)
    if (q == pick) j = cc[q];
  return j;
}

// Factor the rows of the cells cells[0..count): for each row in order, its
// lower entries by increasing rank:
//   L_ij = (A_ij - sum_{k lower than j} L_ik L_jk) / L_jj,
//   L_ii = sqrt(A_ii - sum_j L_ij^2)
// (the sums over the common lower neighbours in increasing rank).
__global__ __launch_bounds__(256) void k_ic_factor(DevPtrs d, const int32_t* __restrict__ cells,
                                                   int count) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= count || d.ctrl->overflow) return;
  int a, b;
  cell_rows(d, cells[t], a, b);
  const int cap = (int)d.nnz_cap;
  for (int64_t i = a; i < b; ++i) {
    const int e0 = min(d.rowptr[i], cap), e1 = min(d.rowptr[i + 1], cap);
    const int n = e1 - e0;
    const bool reg = n <= IC_REG;
    int cc[IC_REG];
    int64_t kk[IC_REG];
    if (reg) ic_load_row(d, e0, n, cc, kk);
    const int64_t ki = rank_key(d, i);
    int64_t prev = -1;
    int nlow = 0;
    for (;;) {
      // next lower entry by rank
      int pick = -1, j = 0;
      int64_t best = ki;
      if (reg) {
        const int q = ic_pick_up(kk, n, prev, ki, best);
        if (q >= 0) {
          pick = e0 + q;
          j = ic_col_at(cc, q);
        }
      } else {
        for (int e = e0; e < e1; ++e) {
          const int64_t kj = rank_key(d, d.col[e]);
          if (kj > prev && kj < best) { best = kj; pick = e; }
        }
        if (pick >= 0) j = d.col[pick];
      }
      if (pick < 0) break;
      prev = best;
      double s = d.val[pick];
      const int g0 = d.rowptr[j], g1 = g0 + d.lnlow[j];
      for (int q = e0; q < e0 + nlow; ++q) {
        const int k = d.lcol[q];
        for (int g = g0; g < g1; ++g)
          if (d.lcol[g] == k) { s -= d.lval[q] * d.lval[g]; break; }
      }
      d.lcol[e0 + nlow] = j;
      d.lval[e0 + nlow] = s / d.ldiag[j];
      ++nlow;
    }
    double s = d.diag[i];
    for (int q = e0; q < e0 + nlow; ++q) s -= d.lval[q] * d.lval[q];
    if (!(s > 0.0)) {  // cannot happen for an M-matrix; keep the solve finite
      atomicOr(&d.ctrl->numeric, 2);
      s = d.diag[i];
    }
    d.ldiag[i] = sqrt(s);
    d.lnlow[i] = nlow;
  }
}

// Upper entries of every row: columns of higher rank in decreasing rank,
// value L_ji from row j's lower part.
__global__ __launch_bounds__(256) void k_ic_mirror(DevPtrs d) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.rows || d.ctrl->overflow) return;
  const RepDev& R = d.rep[d.blk_rep[i / ROWS_PER_BLOCK]];
  if (i - R.row_off >= R.n) return;  // padding rows have no cell
  const int cap = (int)d.nnz_cap;
  const int e0 = min(d.rowptr[i], cap), e1 = min(d.rowptr[i + 1], cap);
  const int64_t ki = rank_key(d, i);
  int pos = e0 + d.lnlow[i];
  const int n = e1 - e0;
  const bool reg = n <= IC_REG;
  int cc[IC_REG];
  int64_t kk[IC_REG];
  if (reg) ic_load_row(d, e0, n, cc, kk);
  int64_t prev = INT64_MAX;
  for (;;) {
    int pick = -1, j = 0;
    int64_t best = ki;
    if (reg) {
      const int q = ic_pick_down(kk, n, ki, prev, best);
      if (q >= 0) {
        pick = e0 + q;
        j = ic_col_at(cc, q);
      }
    } else {
      for (int e = e0; e < e1; ++e) {
        const int64_t kj = rank_key(d, d.col[e]);
        if (kj < prev && kj > best) { best = kj; pick = e; }
      }
      if (pick >= 0) j = d.col[pick];
    }
    if (pick < 0) break;
    prev = best;
    double v = 0.0;
    const int g0 = d.rowptr[j], g1 = g0 + d.lnlow[j];
    for (int g = g0; g < g1; ++g)
      if (d.lcol[g] == (int)i) { v = d.lval[g]; break; }
    d.lcol[pos] = j;
    d.lval[pos] = v;
    ++pos;
  }
}

// Triangular solves: four lanes per cell.  A cell's rows go in order (a row
// may depend on earlier rows of its cell); a row's entries are spread over
// the four lanes, whose sums meet by shuffles within the group (fixed order:
// deterministic), and lane k < 3 writes component k.  The workgroup fence
// makes the row's result visible before the next row of the cell gathers it.
constexpr int IC_LANES = 4;

__device__ __forceinline__ void ic_group_sum(double& s0, double& s1, double& s2) {
#pragma unroll
  for (int o = 1; o < IC_LANES; o <<= 1) {
    s0 += __shfl_xor(s0, o, 64);
    s1 += __shfl_xor(s1, o, 64);
    s2 += __shfl_xor(s2, o, 64);
  }
}

// Forward solve L y = r for the rows of one colour (y into u)
__global__ __launch_bounds__(256) void k_ic_fwd(DevPtrs d, const int32_t* __restrict__ cells,
                                                int count) {
  const int g = (blockIdx.x * blockDim.x + threadIdx.x) / IC_LANES;
  const int lane = threadIdx.x & (IC_LANES - 1);
  if (g >= count || d.ctrl->overflow) return;  // whole groups: L was not built, or past the end
  int a, b;
  cell_rows(d, cells[g], a, b);
  const int cap = (int)d.nnz_cap;
  for (int64_t i = a; i < b; ++i) {
    const int e0 = min(d.rowptr[i], cap);
    const int e1 = min(e0 + d.lnlow[i], cap);
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int q = e0 + lane; q < e1; q += IC_LANES) {
      const int64_t j = d.lcol[q];
      const double l = d.lval[q];
      s0 += l * d.u[3 * j];
      s1 += l * d.u[3 * j + 1];
      s2 += l * d.u[3 * j + 2];
    }
    ic_group_sum(s0, s1, s2);
    if (lane < 3) {
      const double s = lane == 0 ? s0 : (lane == 1 ? s1 : s2);
      d.u[3 * i + lane] = (d.r[3 * i + lane] - s) / d.ldiag[i];
    }
    if (i + 1 < b) __threadfence_block();
  }
}

// Backward solve L^T z = y for the rows of one colour, in place in u
__global__ __launch_bounds__(256) void k_ic_bwd(DevPtrs d, const int32_t* __restrict__ cells,
                                                int count) {
  const int g = (blockIdx.x * blockDim.x + threadIdx.x) / IC_LANES;
  const int lane = threadIdx.x & (IC_LANES - 1);
  if (g >= count || d.ctrl->overflow) return;
  int a, b;
  cell_rows(d, cells[g], a, b);
  const int cap = (int)d.nnz_cap;
  for (int64_t i = (int64_t)b - 1; i >= a; --i) {
    const int r0 = min(d.rowptr[i], cap), r1 = min(d.rowptr[i + 1], cap);
    const int e0 = min(r0 + d.lnlow[i], r1);
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int q = e0 + lane; q < r1; q += IC_LANES) {
      const int64_t j = d.lcol[q];
      const double l = d.lval[q];
      s0 += l * d.u[3 * j];
      s1 += l * d.u[3 * j + 1];
      s2 += l * d.u[3 * j + 2];
    }
    ic_group_sum(s0, s1, s2);
    if (lane < 3) {
      const double s = lane == 0 ? s0 : (lane == 1 ? s1 : s2);
      d.u[3 * i + lane] = (d.u[3 * i + lane] - s) / d.ldiag[i];
    }
    if (i > a) __threadfence_block();
  }
}

// parity export of L's lower triangle in global original numbering, at the
// positions of A's CSR entries: (row, col, L_ij) for lower entries, row -1
// for the other slots; diag_out[g] = L_ii
__global__ __launch_bounds__(256) void k_ic_export(DevPtrs d, const int64_t* __restrict__ id_off,
                                                   int64_t* __restrict__ rows,
                                                   int64_t* __restrict__ cols,
                                                   double* __restrict__ vals,
                                                   double* __restrict__ diag_out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.rows) return;
  const int rid = d.blk_rep[i / ROWS_PER_BLOCK];
  const RepDev& R = d.rep[rid];
  if (i - R.row_off >= R.n) return;
  const int64_t gi = id_off[rid] + (int64_t)d.pos[i].w;
  diag_out[gi] = d.ldiag[i];
  const int e0 = d.rowptr[i], e1 = d.rowptr[i + 1];
  for (int e = e0; e < e1; ++e) {
    const bool low = e - e0 < d.lnlow[i];
    rows[e] = low ? gi : -1;
    cols[e] = low ? id_off[rid] + (int64_t)d.pos[d.lcol[e]].w : -1;
    vals[e] = low ? d.lval[e] : 0.0;
  }
}

// ---------------------------------------------------------------------------
// launchers; colours are given as (offset, count) ranges of ic_cells
// ---------------------------------------------------------------------------
static inline unsigned nb256(int64_t n) { return (unsigned)((n + 255) / 256); }

hipError_t launch_ic_factor(const DevPtrs& d, const int32_t* color_off, int ncolors,
                            hipStream_t s) {
  for (int c = 0; c < ncolors; ++c) {
    const int cnt = color_off[c + 1] - color_off[c];
    if (cnt == 0) continue;
    hipLaunchKernelGGL(k_ic_factor, dim3(nb256(cnt)), dim3(256), 0, s, d,
                       d.ic_cells + color_off[c], cnt);
  }
  hipLaunchKernelGGL(k_ic_mirror, dim3(nb256(d.rows)), dim3(256), 0, s, d);
  return hipGetLastError();
}

hipError_t launch_ic_apply(const DevPtrs& d, const int32_t* color_off, int ncolors,
                           hipStream_t s) {
  for (int c = 0; c < ncolors; ++c) {
    const int cnt = color_off[c + 1] - color_off[c];
    if (cnt == 0) continue;
    hipLaunchKernelGGL(k_ic_fwd, dim3(nb256((int64_t)IC_LANES * cnt)), dim3(256), 0, s, d,
                       d.ic_cells + color_off[c], cnt);
  }
  for (int c = ncolors - 1; c >= 0; --c) {
    const int cnt = color_off[c + 1] - color_off[c];
    if (cnt == 0) continue;
    hipLaunchKernelGGL(k_ic_bwd, dim3(nb256((int64_t)IC_LANES * cnt)), dim3(256), 0, s, d,
                       d.ic_cells + color_off[c], cnt);
  }
  return hipGetLastError();
}

hipError_t launch_ic_export(const DevPtrs& d, const int64_t* id_off, int64_t* rows, int64_t* cols,
                            double* vals, double* diag, hipStream_t s) {
  hipLaunchKernelGGL(k_ic_export, dim3(nb256(d.rows)), dim3(256), 0, s, d, id_off, rows, cols, vals,
                     diag);
  return hipGetLastError();
}
