// cg.hip -- the sparse solve of Eq. 9 (Method section) on gfx950:
// (A (x) I3) v = b, A = gamma0*I + alpha*L(w), three right-hand sides sharing
// one scalar matrix, Jacobi-preconditioned conjugate gradients in the
// single-reduction form of Chronopoulos & Gear (J. Comput. Appl. Math. 25,
// 1989), which in exact arithmetic produces the iterates of standard PCG:
//
//   p = u + beta p, s = w + beta s, x += alpha p, r -= alpha s, u = M^-1 r
//   w = A u;  gamma = (r, u), delta = (w, u)
//   beta' = gamma' / gamma, alpha' = gamma' / (delta' - beta' gamma' / alpha)
//
// Per iteration three launches (four with the learned M^-1 product,
// k_cg_apply), none with a cache write-back fence:
//   k_cg_vec   every vector update, element-parallel (fully coalesced; x
//              every other iteration), and the partial sums of (r, u) and
//              (r, r) per sub-tile of 256 rows;
//   k_cg_spmv  w = A u, by default entry-parallel (the sub-tile's entries
//              striped over its threads, the products summed per row from
//              LDS), or with a group of 1, 2, 4 or 8 lanes per CSR row (the
//              tuning variants); partial sums of (w, u);
//   k_cg_finish one block per replica: the sub-tile partials in a fixed order,
//              then the scalar recurrences and the convergence state.
// Sums are deterministic (fixed trees, no floating-point atomics).
#include "sim_dev.h"
#include "launch.h"

#include <hip/hip_ext.h>

#define VEC_ELEMS (3 * SUB_ROWS)  // elements (row, component) per sub-tile

// sum over the LANES lanes of a row's group, on registers (DPP): lanes
// exchange with lane ^ 1, then lane ^ 2 (quad permutes), then, for 8 lanes,
// with the mirrored lane of the other quad, which after the quad steps holds
// that quad's sum.  Every lane ends with the same bits, since each step adds
// the same two operands.
template <int LANES>
__device__ __forceinline__ void lane_group_sum(double (&a)[3]) {
  static_assert(LANES == 1 || LANES == 2 || LANES == 4 || LANES == 8, "lanes per row");
  if constexpr (LANES >= 2) {
#pragma unroll
    for (int k = 0; k < 3; ++k) a[k] += dpp_move<DPP_XOR1>(a[k]);
  }
  if constexpr (LANES >= 4) {
#pragma unroll
    for (int k = 0; k < 3; ++k) a[k] += dpp_move<DPP_XOR2>(a[k]);
  }
  if constexpr (LANES >= 8) {
#pragma unroll
    for (int k = 0; k < 3; ++k) a[k] += dpp_move<DPP_HALF_MIRROR>(a[k]);
  }
}

// Components per row are finished by lanes 0..2 of the row's group; with
// LANES < 3 a lane takes TURNS turns (component t * LANES + lane in turn t).
// Register arrays are only indexed with compile-time indices here.
// The entry-parallel form (LANES == 0) gives each thread one whole row: three
// turns, turn k being component k.
template <int LANES>
constexpr int TURNS = LANES == 0 ? 3 : (LANES >= 3 ? 1 : (3 + LANES - 1) / LANES);

__device__ __forceinline__ double pick3(const double (&a)[3], int k) {
  return k == 0 ? a[0] : (k == 1 ? a[1] : a[2]);
}
__device__ __forceinline__ bool on_k(const bool (&on)[3], int k) {
  return k == 0 ? on[0] : (k == 1 ? on[1] : on[2]);
}
// v[k] = the turn sum that belongs to component k (0 where this lane has none)
template <int LANES>
__device__ __forceinline__ void turns_to_components(const double (&vt)[TURNS<LANES>], int lane,
                                                    double (&v)[3]) {
  if constexpr (LANES == 0) {
    v[0] = vt[0];
    v[1] = vt[1];
    v[2] = vt[2];
    return;
  }
#pragma unroll
  for (int t = 0; t < TURNS<LANES>; ++t) {
    const int k = t * LANES + lane;
    v[0] = k == 0 ? vt[t] : v[0];
    v[1] = k == 1 ? vt[t] : v[1];
    v[2] = k == 2 ? vt[t] : v[2];
  }
}

// sub-tile partial sums: [gamma0..2, delta0..2, rr0..2]; `first`..`first+n`
// written (blocks of SUB_THREADS threads)
template <int N>
__device__ __forceinline__ void write_partials(const DevPtrs& d, int sub, int first,
                                               double (&v)[N]) {
  __shared__ double lds[SUB_THREADS / 64][9];
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < N; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < N; ++k) lds[wave][k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x < N) {
    double s = 0.0;
    for (int w = 0; w < SUB_THREADS / 64; ++w) s += lds[w][threadIdx.x];
    d.partial[(int64_t)sub * NPART + first + threadIdx.x] = s;
  }
}

// XCD-contiguous sub-tile of this block (or -1 past the end).  With d.rev
// each XCD takes its range from the last sub-tile down: a kernel launched
// right after one that walked forward starts on the rows that one touched
// last, the most likely to be still in the Infinity Cache.  Partials go to
// their sub-tile's slot either way, so the order changes no bits.
__device__ __forceinline__ int sub_of_block(const DevPtrs& d) {
  const int nsub = SUBS_PER_TILE * d.nblk;
  const int per = (nsub + 7) >> 3;
  const int hw = blockIdx.x;
  const int sub = d.rev ? (hw & 7) * per + (per - 1 - (hw >> 3)) : xcd_block(hw, nsub);
  return sub < nsub ? sub : -1;
}

__global__ void k_cg_reset(DevPtrs d, double tol_override) {
  for (int r = threadIdx.x; r < d.nrep; r += blockDim.x) {
    CgRep& c = d.cg[r];
    for (int k = 0; k < 3; ++k) {
      c.bb[k] = c.rr[k] = c.gamma[k] = c.alpha[k] = c.alpha_prev[k] = c.beta[k] = 0.0;
      c.state[k] = 0;
      c.it[k] = 0;
    }
    c.tol2 = tol_override > 0.0 ? tol_override * tol_override : d.rep[r].tol2;
    c.run = 1;
    c.check = 0;
    c.restart = 0;
    c.restarts = 0;
    c.breakdown = 0;
  }
  if (threadIdx.x == 0) {
    d.ctrl->n_notdone = 3 * d.nrep;
    d.ctrl->breakdown = 0;
  }
}

// nontemporal (streaming) loads and stores, or ordinary ones
template <bool NT, class T>
__device__ __forceinline__ T ldv(const T* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p);
  else return *p;
}
template <bool NT, class T>
__device__ __forceinline__ void stv(T* p, T v) {
  if constexpr (NT) __builtin_nontemporal_store(v, p);
  else *p = v;
}

// Element-parallel vector work of one sub-tile (3 * 256 consecutive doubles
// of the AoS arrays; element e is row e/3, component e%3).  NT: the streams
// that are not read again within the iteration (r, p, w, s, x, 1/diag) are
// loaded and stored as nontemporal, u (gathered by the product next) as
// usual: on a working set larger than the last-level cache this streams
// faster (measured at N = 8e6), below it the ordinary form keeps the
// vectors cached; the autotuner picks.  Same bits either way.
//   mode 0 (fresh start):   x = 0, r = b, p = s = 0, u = M^-1 r
//   mode 1 (restart, r already = b - A x):   p = s = 0, u = M^-1 r
//   mode 2 (iteration):     p = u + beta p, s = w + beta s, x += alpha p,
//                           r -= alpha s, u = M^-1 r
// Partials (r, u) and (r, r) of the components touched.
// x is updated every other iteration: in iteration j (j = it, counted per
// component from the start) with j even the term alpha_j p_j is left
// pending, with j odd x += alpha_{j-1} p_{j-1} + alpha_j p_j, p_{j-1} being
// the p this iteration reads anyway; the x stream (48 bytes per row) is
// touched in half the iterations.  k_cg_flush adds a pending term before
// a true-residual check reads x; a start or restart zeroes p, so no pending
// term outlives one.
template <bool NT>
__global__ __launch_bounds__(SUB_THREADS) void k_cg_vec(DevPtrs d, int mode) {
  const int sub = sub_of_block(d);
  if (sub < 0) return;
  const int rid = d.blk_rep[sub / SUBS_PER_TILE];
  const CgRep& cr = d.cg[rid];
  if ((mode == 1 && !cr.restart) || (mode == 2 && !cr.run)) return;
  bool on[3], xodd[3];
  double al[3], ap[3], be[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    on[k] = mode == 0 ? true : (mode == 1 ? cr.state[k] == 3 : cr.state[k] == 0);
    al[k] = cr.alpha[k];
    ap[k] = cr.alpha_prev[k];
    be[k] = cr.beta[k];
    xodd[k] = (cr.it[k] & 1) != 0;
  }
  double v[6] = {0, 0, 0, 0, 0, 0};  // (r,u)[3], (r,r)[3]
  const int64_t base = (int64_t)sub * VEC_ELEMS;
  const bool ext = d.learned || d.ic0;  // u = M^-1 r comes from a separate pass
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const int le = q * SUB_THREADS + threadIdx.x;
    const int k = le % 3;
    if (!on[k]) continue;
    const int64_t e = base + le;
    // 1/diag only where this kernel applies Jacobi itself
    const double di =
        (ext || d.pc_none) ? 1.0 : ldv<NT>(d.dinv + (int64_t)sub * SUB_ROWS + le / 3);
    double rk;
    if (mode == 0) {
      rk = d.b[e];
      d.x[e] = 0.0;
      d.r[e] = rk;
      d.p[e] = 0.0;
      d.s[e] = 0.0;
    } else if (mode == 1) {
      rk = d.r[e];
      d.p[e] = 0.0;
      d.s[e] = 0.0;
    } else {
      const double r0 = ldv<NT>(d.r + e);
      const double uk0 = ext ? ldv<NT>(d.u + e) : di * r0;
      const double pold = ldv<NT>(d.p + e);
      const double pk = uk0 + be[k] * pold;
      const double sk = ldv<NT>(d.w + e) + be[k] * ldv<NT>(d.s + e);
      stv<NT>(d.p + e, pk);
      stv<NT>(d.s + e, sk);
      if (on_k(xodd, k)) stv<NT>(d.x + e, ldv<NT>(d.x + e) + (ap[k] * pold + al[k] * pk));
      rk = r0 - al[k] * sk;
      stv<NT>(d.r + e, rk);
    }
    if (!ext) {
      const double uk = di * rk;
      d.u[e] = uk;
      v[k] += rk * uk;
    }
    v[3 + k] += rk * rk;
  }
  double g[3] = {v[0], v[1], v[2]}, rr[3] = {v[3], v[4], v[5]};
  if (!ext) {
    write_partials<3>(d, sub, 0, g);
    __syncthreads();
  }
  write_partials<3>(d, sub, 6, rr);
}

// Partials (r, u) per sub-tile after an external preconditioner pass (IC(0)),
// component selection as k_cg_vec's mode.
// Pending x terms before a true-residual check: x += alpha p for the
// components whose check is pending and whose last iteration (it - 1) was
// even (see k_cg_vec); replicas without a pending check return at once.
__global__ __launch_bounds__(SUB_THREADS) void k_cg_flush(DevPtrs d) {
  const int sub = sub_of_block(d);
  if (sub < 0) return;
  const CgRep& cr = d.cg[d.blk_rep[sub / SUBS_PER_TILE]];
  if (!cr.check) return;
  bool on[3];
  double al[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    on[k] = cr.state[k] == 1 && (cr.it[k] & 1) != 0;
    al[k] = cr.alpha[k];
  }
  if (!on[0] && !on[1] && !on[2]) return;
  const int64_t base = (int64_t)sub * VEC_ELEMS;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const int le = q * SUB_THREADS + threadIdx.x;
    const int k = le % 3;
    if (!on_k(on, k)) continue;
    const int64_t e = base + le;
    d.x[e] += pick3(al, k) * d.p[e];
  }
}

__global__ __launch_bounds__(SUB_THREADS) void k_cg_dot_ru(DevPtrs d, int mode) {
  const int sub = sub_of_block(d);
  if (sub < 0) return;
  const CgRep& cr = d.cg[d.blk_rep[sub / SUBS_PER_TILE]];
  if ((mode == 1 && !cr.restart) || (mode == 2 && !cr.run)) return;
  bool on[3];
#pragma unroll
  for (int k = 0; k < 3; ++k)
    on[k] = mode == 0 ? true : (mode == 1 ? cr.state[k] == 3 : cr.state[k] == 0);
  double v[3] = {0, 0, 0};
  const int64_t base = (int64_t)sub * VEC_ELEMS;
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    const int le = q * SUB_THREADS + threadIdx.x;
    const int k = le % 3;
    if (!on_k(on, k)) continue;
    const double add = d.r[base + le] * d.u[base + le];
    v[0] += k == 0 ? add : 0.0;
    v[1] += k == 1 ? add : 0.0;
    v[2] += k == 2 ? add : 0.0;
  }
  write_partials<3>(d, sub, 0, v);
}

// Entry-parallel product over a sub-tile (the (0, EPT) variants).  The
// sub-tile's off-diagonal entries are one contiguous CSR range [E0, E1); it is
// striped over the block's threads in passes of SUB_THREADS * EPT entries
// (entry E0 + c0 + t + k * SUB_THREADS to thread t), so the column and value
// loads are coalesced, all of a thread's are in flight together, and none
// waits on the row pointers of its own row; the next pass's are loaded while
// this pass's gathers are summed.  Each thread gathers its entries' rows of
// src and leaves the three products in LDS; after a barrier the thread of row
// i adds its row's products in entry order (the same order for every EPT: the
// variants give the same bits, and those of the one-lane loop form).  A row
// that spans passes continues its sum in the next one.  The sub-tile's own
// rows of src come in, and its results go out, through LDS as contiguous runs
// of 3 * SUB_ROWS doubles.  Measured at N = 8e6 (brick order, k = 5.5): the
// product 227 against 304 us for four lanes per row (learned CG iterations of
// the evolved box), the loads no longer waiting on a row-pointer load of
// their own and every lane carrying an entry.
template <int EPT, class Val, class Fin>
__device__ __forceinline__ void ep_tile(const DevPtrs& d, int sub, const double* __restrict__ src,
                                        const double* __restrict__ dg, Val val, const bool (&on)[3],
                                        double* __restrict__ out, Fin fin) {
  static_assert(SUB_THREADS == SUB_ROWS, "one thread per row of the sub-tile");
  static_assert(SUB_THREADS % 3 == 1, "component of an io element");
  constexpr int CAP = SUB_THREADS * EPT;
  __shared__ double prod[3][CAP];
  __shared__ double io[3 * SUB_ROWS];
  const int cap = (int)d.nnz_cap;  // clamped as in lane_tile
  const int t = threadIdx.x;
  const int64_t base = (int64_t)sub * SUB_ROWS;
  const int E0 = min(d.rowptr[base], cap);
  const int ne = min(d.rowptr[base + SUB_ROWS], cap) - E0;
  const int64_t i = base + t;
  const int r0 = min(d.rowptr[i], cap) - E0, r1 = min(d.rowptr[i + 1], cap) - E0;
  const double dgi = dg[i];
#pragma unroll
  for (int q = 0; q < 3; ++q) io[t + q * SUB_THREADS] = src[3 * base + t + q * SUB_THREADS];
  // values kept in their stored type until the multiply: a conversion next
  // to the load would wait for it, and with it for every gather in flight
  using VT = decltype(val(0));
  int c[EPT];
  VT m[EPT];
  auto load = [&](int c0, int (&cl)[EPT], VT (&ml)[EPT]) {
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      const int e = c0 + t + k * SUB_THREADS;
      cl[k] = -1;
      ml[k] = VT(0);
      if (e < ne) {
        cl[k] = d.col[E0 + e];
        ml[k] = val(E0 + e);
      }
    }
  };
  load(0, c, m);
  double a[3] = {0.0, 0.0, 0.0};
  for (int c0 = 0; c0 < ne; c0 += CAP) {
    double g[EPT][3];
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      g[k][0] = g[k][1] = g[k][2] = 0.0;
      if (c[k] >= 0) {
        const double* gp = src + 3 * (int64_t)c[k];
        g[k][0] = gp[0];
        g[k][1] = gp[1];
        g[k][2] = gp[2];
      }
    }
    int cn[EPT];
    VT mn[EPT];
    if (c0 + CAP < ne) {
      load(c0 + CAP, cn, mn);
    } else {
#pragma unroll
      for (int k = 0; k < EPT; ++k) {
        cn[k] = -1;
        mn[k] = VT(0);
      }
    }
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      if (c[k] >= 0) {
        const int slot = t + k * SUB_THREADS;
        const double mk = m[k];
        prod[0][slot] = mk * g[k][0];
        prod[1][slot] = mk * g[k][1];
        prod[2][slot] = mk * g[k][2];
      }
    }
    __syncthreads();
    const int lo = r0 > c0 ? r0 : c0, hi = r1 < c0 + CAP ? r1 : c0 + CAP;
    for (int e = lo; e < hi; ++e) {
      a[0] += prod[0][e - c0];
      a[1] += prod[1][e - c0];
      a[2] += prod[2][e - c0];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < EPT; ++k) {
      c[k] = cn[k];
      m[k] = mn[k];
    }
  }
  if (ne == 0) __syncthreads();  // the own rows in io, as after a pass
  double v[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const double sk = io[3 * t + k];
    v[k] = on_k(on, k) ? fin(i, k, k, sk, dgi * sk + a[k]) : 0.0;
  }
  __syncthreads();  // every own row read
#pragma unroll
  for (int k = 0; k < 3; ++k) io[3 * t + k] = v[k];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 3; ++q) {
    int k = t % 3 + q;  // component of element t + q * SUB_THREADS (SUB_THREADS = 1 mod 3)
    k = k >= 3 ? k - 3 : k;
    if (on_k(on, k)) out[3 * base + t + q * SUB_THREADS] = io[t + q * SUB_THREADS];
  }
}

// Products sum_j M_ij src_j (three components) of the sub-tile's 256 rows
// with a group of LANES lanes per row, LANES passes over 256 / LANES rows
// each.
// Lane l of a group takes the row's entries l, l + LANES, l + 2 LANES, ...,
// adds them in that order, then the group adds its lanes; both forms below
// therefore give the same bits.
//   ENT = 0: each lane walks its entries, loading column, value and the
//            gathered row in turn.
//   ENT > 0: software-pipelined over the passes.  The row pointers and the
//            diagonal terms of every pass load first; then the columns and
//            values of the first ENT entries per lane of pass p + 1 load
//            while pass p gathers, so each pass waits for one gather instead
//            of a column load followed by a gather.  Entries past LANES * ENT
//            in a row follow in the loop form.  Loads of missing entries are
//            masked, not issued.  (Loading further ahead was measured slower:
//            the extra data in flight no longer fits the L1 cache.)
// val(e) is the off-diagonal value of CSR entry e (in its stored type, FP32
// or FP64; the products are formed in FP64), dg the diagonal; for the
// components finished by this lane (component k = t * LANES + lane, turn t)
// that are on, out[3i+k] = fin(i, k, t, src_ik, own) with
// own = dg_i src_ik + sum_j M_ij src_jk.
template <int LANES, int ENT, class Val, class Fin>
__device__ __forceinline__ void lane_tile(const DevPtrs& d, int sub, const double* __restrict__ src,
                                          const double* __restrict__ dg, Val val, const bool (&on)[3],
                                          double* __restrict__ out, Fin fin) {
  constexpr int GROUPS = SUB_THREADS / LANES;
  constexpr int PASSES = SUB_ROWS / GROUPS;
  constexpr int T = TURNS<LANES>;
  const int lane = threadIdx.x & (LANES - 1);
  const int grp = threadIdx.x / LANES;
  // clamped: after an overflowing fill the row pointers may pass the
  // capacity (the host discards that solve; the reads stay in bounds)
  const int cap = (int)d.nnz_cap;
  if constexpr (ENT == 0) {
    for (int pass = 0; pass < PASSES; ++pass) {
      const int64_t i = (int64_t)sub * SUB_ROWS + pass * GROUPS + grp;
      const int e0 = min(d.rowptr[i], cap), e1 = min(d.rowptr[i + 1], cap);
      double a[3] = {0.0, 0.0, 0.0};
      for (int e = e0 + lane; e < e1; e += LANES) {
        const int64_t j = d.col[e];
        const double m = val(e);
        a[0] += m * src[3 * j];
        a[1] += m * src[3 * j + 1];
        a[2] += m * src[3 * j + 2];
      }
      lane_group_sum<LANES>(a);
#pragma unroll
      for (int t = 0; t < T; ++t) {
        const int k = t * LANES + lane;
        if (k >= 3) continue;
        if (!on_k(on, k)) continue;
        const double sk = src[3 * i + k];
        out[3 * i + k] = fin(i, k, t, sk, dg[i] * sk + pick3(a, k));
      }
    }
  } else {
    int e0[PASSES], e1[PASSES];
    double dv[PASSES], sv[PASSES][T];
#pragma unroll
    for (int p = 0; p < PASSES; ++p) {
      const int64_t i = (int64_t)sub * SUB_ROWS + p * GROUPS + grp;
      e0[p] = min(d.rowptr[i], cap);
      e1[p] = min(d.rowptr[i + 1], cap);
      dv[p] = lane < 3 ? dg[i] : 0.0;
#pragma unroll
      for (int t = 0; t < T; ++t) {
        const int k = t * LANES + lane;
        sv[p][t] = k < 3 ? src[3 * i + k] : 0.0;
      }
    }
    int c[2][ENT];      // columns of the current / next pass (-1: no entry)
    decltype(val(0)) m[2][ENT];  // values in their stored type (as in ep_tile)
    auto load_entries = [&](int p, int buf) {
#pragma unroll
      for (int q = 0; q < ENT; ++q) {
        const int e = e0[p] + lane + q * LANES;
        c[buf][q] = -1;
        m[buf][q] = 0;
        if (e < e1[p]) {
          c[buf][q] = d.col[e];
          m[buf][q] = val(e);
        }
      }
    };
    load_entries(0, 0);
#pragma unroll
    for (int p = 0; p < PASSES; ++p) {
      const int cur = p & 1;
      if (p + 1 < PASSES) load_entries(p + 1, cur ^ 1);
      double g[ENT][3];
#pragma unroll
      for (int q = 0; q < ENT; ++q) {
        g[q][0] = g[q][1] = g[q][2] = 0.0;
        const int64_t j = c[cur][q];
        if (j >= 0) {
          g[q][0] = src[3 * j];
          g[q][1] = src[3 * j + 1];
          g[q][2] = src[3 * j + 2];
        }
      }
      double a[3];
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        a[k] = 0.0;
#pragma unroll
        for (int q = 0; q < ENT; ++q) {
          const double prod = (double)m[cur][q] * g[q][k];
          a[k] += c[cur][q] >= 0 ? prod : 0.0;  // adding +0 leaves the bits
        }
      }
      for (int e = e0[p] + lane + ENT * LANES; e < e1[p]; e += LANES) {
        const int64_t j = d.col[e];
        const double mv = val(e);
        a[0] += mv * src[3 * j];
        a[1] += mv * src[3 * j + 1];
        a[2] += mv * src[3 * j + 2];
      }
      lane_group_sum<LANES>(a);
      const int64_t i = (int64_t)sub * SUB_ROWS + p * GROUPS + grp;
#pragma unroll
      for (int t = 0; t < T; ++t) {
        const int k = t * LANES + lane;
        if (k >= 3 || !on_k(on, k)) continue;
        out[3 * i + k] = fin(i, k, t, sv[p][t], dv[p] * sv[p][t] + pick3(a, k));
      }
    }
  }
}

// The product of one sub-tile in the form of variant (LANES, ENT): for every
// row i and component k with on[k], out[3i+k] = fin(i, k, t, src_ik, own)
// with own = dg_i src_ik + sum_j M_ij src_jk (fin also takes the partial sums;
// t is the turn of the calling lane)
template <int LANES, int ENT, class Val, class Fin>
__device__ __forceinline__ void csr_tile(const DevPtrs& d, int sub, const double* __restrict__ src,
                                         const double* __restrict__ dg, Val val, const bool (&on)[3],
                                         double* __restrict__ out, Fin fin) {
  if constexpr (LANES == 0)
    ep_tile<ENT>(d, sub, src, dg, val, on, out, fin);
  else
    lane_tile<LANES, ENT>(d, sub, src, dg, val, on, out, fin);
}

// Learned preconditioner: u = M^-1 r with M^-1 in A's pattern, partial
// (r, u).  Same component selection as k_cg_vec's mode.
template <int LANES, int ENT>
__global__ __launch_bounds__(SUB_THREADS) void k_cg_apply(DevPtrs d, int mode) {
  const int sub = sub_of_block(d);
  if (sub < 0) return;
  const int rid = d.blk_rep[sub / SUBS_PER_TILE];
  const CgRep& cr = d.cg[rid];
  if ((mode == 1 && !cr.restart) || (mode == 2 && !cr.run)) return;
  bool on[3];
#pragma unroll
  for (int k = 0; k < 3; ++k)
    on[k] = mode == 0 ? true : (mode == 1 ? cr.state[k] == 3 : cr.state[k] == 0);
  const float* __restrict__ moff = d.moff;
  double vt[TURNS<LANES>] = {};  // this lane's sums, one per turn
  csr_tile<LANES, ENT>(
      d, sub, d.r, d.mdiag, [&](int e) { return moff[e]; }, on, d.u,
      [&](int64_t, int, int t, double rk, double uk) {
        vt[t] += rk * uk;
        return uk;
      });
  double v[3] = {0, 0, 0};
  turns_to_components<LANES>(vt, threadIdx.x & (LANES - 1), v);
  write_partials<3>(d, sub, 0, v);
}

// Advance the recurrences of one replica from its totals
// tot = [gamma0..2, delta0..2, rr0..2].  mode 0: after a fresh start, 1: after
// a restart, 2: after an iteration, 3: after a true-residual check, 4: after
// the residual of a warm-start guess.
__device__ void cg_advance(const DevPtrs& d, CgRep& c, int mode, const double (&tot)[9]) {
  int finished = 0;
  for (int k = 0; k < 3; ++k) {
    const double gam = tot[k], del = tot[3 + k], rr = tot[6 + k];
    if (mode == 0 || (mode == 1 && c.state[k] == 3)) {
      if (mode == 0) c.bb[k] = rr;
      c.rr[k] = rr;
      if (c.bb[k] == 0.0) {  // b = 0: x = 0 is exact
        c.state[k] = 2;
        ++finished;
      } else if (rr <= c.tol2 * c.bb[k]) {
        c.state[k] = 1;
      } else if (!(del > 0.0)) {
        c.state[k] = 2;
        c.breakdown = 1;
        atomicOr(&d.ctrl->breakdown, 1);
        ++finished;
      } else {
        c.state[k] = 0;
        c.gamma[k] = gam;
        c.alpha[k] = gam / del;
        c.alpha_prev[k] = 0.0;
        c.beta[k] = 0.0;
      }
    } else if (mode == 2 && c.state[k] == 0) {
      c.it[k] += 1;
      c.rr[k] = rr;
      if (rr <= c.tol2 * c.bb[k]) {
        c.state[k] = 1;
      } else {
        const double beta = gam / c.gamma[k];
        const double den = del - beta * gam / c.alpha[k];
        if (!(den > 0.0)) {
          c.state[k] = 2;
          c.breakdown = 1;
        atomicOr(&d.ctrl->breakdown, 1);
          ++finished;
        } else {
          c.beta[k] = beta;
          c.alpha_prev[k] = c.alpha[k];
          c.alpha[k] = gam / den;
          c.gamma[k] = gam;
        }
      }
    } else if (mode == 4 && c.state[k] == 0) {
      // residual of the warm-start guess: done if it passes, else restart
      // from it (no restart is counted)
      c.rr[k] = rr;
      c.state[k] = rr <= c.tol2 * c.bb[k] ? 1 : 3;
    } else if (mode == 3 && c.state[k] == 1) {
      c.rr[k] = rr;
      if (rr <= c.tol2 * c.bb[k]) {
        c.state[k] = 2;
        ++finished;
      } else {
        c.state[k] = 3;
        c.restarts += 1;
      }
    }
  }
  int run = 0, pend = 0, rst = 0;
  for (int k = 0; k < 3; ++k) {
    run |= c.state[k] == 0;
    pend |= c.state[k] == 1;
    rst |= c.state[k] == 3;
  }
  c.run = run;
  c.check = !run && pend;
  c.restart = rst;
  if (finished) atomicSub(&d.ctrl->n_notdone, finished);
}

// Sum `count` partial slots starting at `first` in a fixed order (thread t
// takes slots t, t + blockDim, ...; then the wave and block trees).  Totals
// valid in thread 0.
__device__ __forceinline__ void sum_slots(const double* __restrict__ first, int count,
                                          double (&tot)[9]) {
  __shared__ double lds[FINISH_THREADS / 64][9];
  double acc[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) acc[k] = 0.0;
  for (int t = threadIdx.x; t < count; t += blockDim.x) {
    const double* src = first + (int64_t)t * NPART;
#pragma unroll
    for (int k = 0; k < 9; ++k)
      acc[k] += src[k];
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < 9; ++k) acc[k] = wave_sum(acc[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < 9; ++k) lds[wave][k] = acc[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int k = 0; k < 9; ++k) {
      double s = 0.0;
      for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += lds[w][k];
      tot[k] = s;
    }
  }
}

// CSR product over the sub-tile's 256 rows.
//   mode 0: w = A u, partial (w, u)  (components iterating / restarting / fresh)
//   mode 1: r = b - A x, partial (r, r)  (components whose check is pending)
//   mode 2: r = b - A x, partial (r, r)  (iterating components: the residual
//           of a warm-start guess)
// Lane k of a row's group finishes component k (coalesced stores); with
// fewer than three lanes, lane l takes components l, l + LANES, ...
template <bool FP32, int LANES, int ENT>
__global__ __launch_bounds__(SUB_THREADS) void k_cg_spmv(DevPtrs d, int mode, int start_mode) {
  const int sub = sub_of_block(d);
  if (sub < 0) return;
  const int rid = d.blk_rep[sub / SUBS_PER_TILE];
  const CgRep& cr = d.cg[rid];
  bool on[3];
  if (mode == 0) {
    // start_mode: 0 fresh start, 1 restart, 2 iteration (as in k_cg_vec)
    if ((start_mode == 1 && !cr.restart) || (start_mode == 2 && !cr.run)) return;
#pragma unroll
    for (int k = 0; k < 3; ++k)
      on[k] = start_mode == 0 ? true : (start_mode == 1 ? cr.state[k] == 3 : cr.state[k] == 0);
  } else if (mode == 1) {
    if (!cr.check) return;
#pragma unroll
    for (int k = 0; k < 3; ++k) on[k] = cr.state[k] == 1;
  } else {
    if (!cr.run) return;
#pragma unroll
    for (int k = 0; k < 3; ++k) on[k] = cr.state[k] == 0;
  }
  const double* __restrict__ src = mode == 0 ? d.u : d.x;
  const double* __restrict__ val = d.val;
  const float* __restrict__ valf = d.valf;
  double vt[TURNS<LANES>] = {};  // this lane's sums, one per turn
  csr_tile<LANES, ENT>(
      d, sub, src, d.diag, [&](int e) {
        if constexpr (FP32)
          return valf[e];
        else
          return val[e];
      }, on,
      mode == 0 ? d.w : d.r,
      [&](int64_t i, int k, int t, double sk, double own) {
        if (mode == 0) {
          vt[t] += own * sk;
          return own;
        }
        const double rk = d.b[3 * i + k] - own;
        vt[t] += rk * rk;
        return rk;
      });
  double v[3] = {0, 0, 0};
  turns_to_components<LANES>(vt, threadIdx.x & (LANES - 1), v);
  write_partials<3>(d, sub, mode == 0 ? 3 : 6, v);
}

// Warm start: x = the previous step's velocity of each row's particle (kept
// in original order) for the components still iterating after the fresh
// start, which has set ||b||^2 and finished the components with b = 0.
__global__ __launch_bounds__(BLOCK_THREADS) void k_cg_warm(DevPtrs d, const int64_t* __restrict__ id_off) {
  const int tile = xcd_block(blockIdx.x, d.nblk);
  if (tile >= d.nblk) return;
  const int rid = d.blk_rep[tile];
  const CgRep& cr = d.cg[rid];
  if (!cr.run) return;
  const RepDev& R = d.rep[rid];
  const int64_t i = (int64_t)tile * ROWS_PER_BLOCK + threadIdx.x;
  if (i - R.row_off >= R.n) return;  // padding rows keep x = 0
  const int64_t g = id_off[rid] + (int64_t)d.pos[i].w;
#pragma unroll
  for (int k = 0; k < 3; ++k)
    if (cr.state[k] == 0) d.x[3 * i + k] = d.vel_orig[3 * g + k];
}

__device__ __forceinline__ bool finish_work(const CgRep& c, int mode) {
  return (mode == 0) || (mode == 1 && c.restart) || (mode == 2 && c.run) ||
         (mode == 3 && c.check) || (mode == 4 && c.run);
}

// First level of a large replica's reduction: block b sums L1_SUBS of the
// replica's sub-tile partials into partial2[b].
__global__ __launch_bounds__(FINISH_THREADS) void k_cg_reduce1(DevPtrs d, int mode) {
  const int b = blockIdx.x;
  const int rid = d.l1_rep[b];
  const RepDev& R = d.rep[rid];
  if (!finish_work(d.cg[rid], mode)) return;
  const int s0 = (b - R.l1_off) * L1_SUBS;
  const int nsub = SUBS_PER_TILE * R.nblk;
  const int cnt = nsub - s0 < L1_SUBS ? nsub - s0 : L1_SUBS;
  double tot[9];
  sum_slots(d.partial + (int64_t)(SUBS_PER_TILE * R.blk_off + s0) * NPART, cnt, tot);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int k = 0; k < 9; ++k) d.partial2[(int64_t)b * NPART + k] = tot[k];
  }
}

// One block per replica: its sub-tile partials (or, for a large replica,
// the first-level sums) in a fixed order, then the recurrences.
__global__ __launch_bounds__(FINISH_THREADS) void k_cg_finish(DevPtrs d, int mode) {
  const int rid = blockIdx.x;
  const RepDev& R = d.rep[rid];
  CgRep& c = d.cg[rid];
  if (!finish_work(c, mode)) return;
  double tot[9];
  if (R.l1_cnt > 0)
    sum_slots(d.partial2 + (int64_t)R.l1_off * NPART, R.l1_cnt, tot);
  else
    sum_slots(d.partial + (int64_t)(SUBS_PER_TILE * R.blk_off) * NPART, SUBS_PER_TILE * R.nblk,
              tot);
  if (threadIdx.x == 0) cg_advance(d, c, mode, tot);
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
// With events, the extended launch records the kernel's own start and end;
// without, a plain launch (the form that stream capture records).
#define LAUNCH_EV(K, G, B, S, E0, E1, ...)                              \
  do {                                                                  \
    if ((E0) || (E1))                                                   \
      hipExtLaunchKernelGGL(K, G, B, 0, S, E0, E1, 0, __VA_ARGS__);     \
    else                                                                \
      hipLaunchKernelGGL(K, G, B, 0, S, __VA_ARGS__);                   \
  } while (0)

hipError_t launch_cg_reset(const DevPtrs& d, double tol_override, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_reset, dim3(1), dim3(256), 0, s, d, tol_override);
  return hipGetLastError();
}

// ev0/ev1 (optional) take the kernel's own start and end timestamps
hipError_t launch_cg_vec(const DevPtrs& d, int mode, hipStream_t s, hipEvent_t ev0,
                         hipEvent_t ev1) {
  const dim3 g(xcd_grid(SUBS_PER_TILE * d.nblk)), b(SUB_THREADS);
  if (d.vec_nt && mode == 2)
    LAUNCH_EV(k_cg_vec<true>, g, b, s, ev0, ev1, d, mode);
  else
    LAUNCH_EV(k_cg_vec<false>, g, b, s, ev0, ev1, d, mode);
  return hipGetLastError();
}

hipError_t launch_cg_spmv(const DevPtrs& d, int mode, int start_mode, hipStream_t s,
                          hipEvent_t ev0, hipEvent_t ev1) {
  const dim3 g(xcd_grid(SUBS_PER_TILE * d.nblk)), b(SUB_THREADS);
  const bool f32 = d.spmv_fp32 && mode == 0;
  switch (d.spmv_var * 2 + (f32 ? 1 : 0)) {
#define SPMV_CASE(V, L, E)                                                                  \
    case 2 * V:                                                                            \
      LAUNCH_EV((k_cg_spmv<false, L, E>), g, b, s, ev0, ev1, d, mode, start_mode);          \
      break;                                                                               \
    case 2 * V + 1:                                                                        \
      LAUNCH_EV((k_cg_spmv<true, L, E>), g, b, s, ev0, ev1, d, mode, start_mode);           \
      break;
    CSR_VARIANT_LIST(SPMV_CASE)
#undef SPMV_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_cg_dot_ru(const DevPtrs& d, int mode, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_dot_ru, dim3(xcd_grid(SUBS_PER_TILE * d.nblk)), dim3(SUB_THREADS), 0, s,
                     d, mode);
  return hipGetLastError();
}

hipError_t launch_cg_apply(const DevPtrs& d, int mode, hipStream_t s, hipEvent_t ev0,
                           hipEvent_t ev1) {
  const dim3 g(xcd_grid(SUBS_PER_TILE * d.nblk)), b(SUB_THREADS);
  switch (d.apply_var) {
#define APPLY_CASE(V, L, E) \
    case V: LAUNCH_EV((k_cg_apply<L, E>), g, b, s, ev0, ev1, d, mode); break;
    CSR_VARIANT_LIST(APPLY_CASE)
#undef APPLY_CASE
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t launch_cg_warm(const DevPtrs& d, const int64_t* id_off, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_warm, dim3(xcd_grid(d.nblk)), dim3(BLOCK_THREADS), 0, s, d, id_off);
  return hipGetLastError();
}

hipError_t launch_cg_flush(const DevPtrs& d, hipStream_t s) {
  hipLaunchKernelGGL(k_cg_flush, dim3(xcd_grid(SUBS_PER_TILE * d.nblk)), dim3(SUB_THREADS), 0, s, d);
  return hipGetLastError();
}

hipError_t launch_cg_finish(const DevPtrs& d, int mode, hipStream_t s) {
  if (d.l1_total > 0)
    hipLaunchKernelGGL(k_cg_reduce1, dim3(d.l1_total), dim3(FINISH_THREADS), 0, s, d, mode);
  hipLaunchKernelGGL(k_cg_finish, dim3(d.nrep), dim3(FINISH_THREADS), 0, s, d, mode);
  return hipGetLastError();
}
