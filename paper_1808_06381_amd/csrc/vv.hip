// vv.hip -- velocity cross-correlation of the blobs against their
// separation (Results section: the correlation of two chains' velocities,
// normalised by the mean square velocity, as a function of |R_cc'|).
//
// Input: the configuration R_n of the last committed step and the
// velocities v_n solved at it (the step's previous-position buffer and its
// CG solution, both in the cell order of that step).  Per replica and
// distance bin the library returns the sum of u_i . u_j and the count over
// unordered pairs with r < r_max under the Lees-Edwards minimum image, and
// sum_c |u_c|^2; u = v, or v minus the Couette flow kappa (y - Ly/2) x of
// Eq. 6c (the same for every image of a particle).
//
// Pair and bin decisions: r^2 from the same explicitly rounded separation
// as the neighbour search; pair iff r^2 < r_max^2; bin = the largest k with
// k^2 <= r^2 c, c = nbins^2 / r_max^2, capped at nbins - 1.
//
// Layout.  A coarse Lees-Edwards cell grid with cells of at least r_max / M
// per axis (the host picks the largest reach M <= 8 whose cells hold at
// least 8 particles on average); the particles are copied into coarse-cell
// order with their relative velocities.  k_vv_pairs: one block (one wave) per chunk of up to VV_HOME
// particles of one cell; it walks the (2M+1)^2 rows of candidate cells
// (rows across the y boundary cover the x range shifted by the offset;
// cells farther than r_max from the home cell are skipped), stages each run
// of cells through LDS and lets every home particle test every staged
// candidate (lanes of a small cell split into groups that take every G-th
// candidate).  Each unordered pair is counted once, by the home particle
// with the lower coarse-order index: the separation, r^2 and u_i . u_j come
// out with the same bits from either end, so the other end would add the
// same integer; staged runs that lie wholly before the home chunk are
// skipped.
//
// Determinism.  Each product u_i . u_j is rounded to a fixed-point integer
// with a per-replica power-of-two scale 2^S (S from the largest |u|^2 and a
// bound on the pairs of one block, so that a block's int64 sums cannot
// overflow); blocks add the integers in LDS with integer atomics, the
// reduce kernel adds the blocks' integers exactly in 128 bits.  Integer
// sums do not depend on the order of the additions, so neither the cell
// order inside a coarse cell nor the scheduling changes a bit of the
// result.  The error against the exact pair sum is at most 2^-(S+1) per
// pair plus the final conversion to FP64.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "launch.h"
#include "sim_dev.h"

namespace {

constexpr int VV_HOME = 64;       // home particles (threads, one wave) per block
constexpr int VV_STAGE = 64;      // candidates staged in LDS at a time (4 KB: a one-wave
                                  // block with 256 staged, 16 KB, left two waves per SIMD)
constexpr int VV_THREADS = 1024;  // threads of the binning kernels
constexpr int VV_FOLD = 256;      // table blocks folded per first-stage reduce block

}  // namespace

// bin of t >= 0: the largest k with k^2 <= t, capped at nb - 1
// (t < nb^2 (1 + eps) <= 2^20 (1 + eps) for an accepted pair, so the
// single-precision root is within one of the answer: one correction each way)
__device__ __forceinline__ int vv_bin(double t, int nb) {
  int k = (int)sqrtf((float)t);
  k += ((double)(k + 1) * (double)(k + 1) <= t) ? 1 : 0;
  k -= ((double)k * (double)k > t) ? 1 : 0;
  return k < nb - 1 ? k : nb - 1;
}

// fixed-point scale exponent of a replica: 61 - log2p - E with |u|^2 < 2^E
__device__ __forceinline__ int vv_scale_exp(unsigned long long umax_bits, int log2p) {
  const double m = __longlong_as_double((long long)umax_bits);
  if (!(m > 0.0)) return 0;
  int e;
  (void)frexp(m, &e);
  return 61 - log2p - e;
}

// relative velocity of row i (the flow term with the oracle's rounding)
__device__ __forceinline__ double4 vv_u(const DevPtrs& d, const RepDev& R, int64_t i, int flow,
                                        double y) {
  double ux = d.x[3 * i];
  if (flow)
    ux = __dsub_rn(ux, __dmul_rn(R.shear, __dsub_rn(y, __dmul_rn(0.5, R.L[1]))));
  return make_double4(ux, d.x[3 * i + 1], d.x[3 * i + 2], 0.0);
}

__device__ __forceinline__ int vv_axis(double v, double inv_len, int nc) {
  int c = (int)floor(v * inv_len);
  c = c < 0 ? 0 : c;
  return c > nc - 1 ? nc - 1 : c;
}

// coarse cell of every real row (slot in the cell by an integer atomic),
// per block the sum of |u|^2 (fixed order) and per replica the largest
// |u|^2 (integer maximum of the non-negative doubles' bits)
__global__ __launch_bounds__(VV_THREADS) void k_vv_bin(DevPtrs d, const VvRep* __restrict__ vr,
                                                       int flow, int32_t* __restrict__ cnt,
                                                       int32_t* __restrict__ vcell,
                                                       int32_t* __restrict__ slot,
                                                       unsigned long long* __restrict__ umax,
                                                       double* __restrict__ u2_part) {
  __shared__ double lds[VV_THREADS / 64][1];
  const int blk = blockIdx.x;
  const int rid = d.blk_rep[blk];
  const RepDev& R = d.rep[rid];
  const VvRep& V = vr[rid];
  double acc[1] = {0.0};
  double um = 0.0;
  for (int k = 0; k < ROWS_PER_BLOCK / VV_THREADS; ++k) {
    const int64_t i = (int64_t)blk * ROWS_PER_BLOCK + k * VV_THREADS + threadIdx.x;
    if (i - R.row_off >= R.n) continue;
    const double4 p = d.pos_alt[i];
    const double4 u = vv_u(d, R, i, flow, p.y);
    const double u2 = __dadd_rn(__dadd_rn(__dmul_rn(u.x, u.x), __dmul_rn(u.y, u.y)),
                                __dmul_rn(u.z, u.z));
    acc[0] += u2;
    um = fmax(um, u2);
    const int cx = vv_axis(p.x, V.inv_len[0], V.nc[0]);
    const int cy = vv_axis(p.y, V.inv_len[1], V.nc[1]);
    const int cz = vv_axis(p.z, V.inv_len[2], V.nc[2]);
    const int c = V.cell0 + (cz * V.nc[1] + cy) * V.nc[0] + cx;
    vcell[i] = c;
    slot[i] = atomicAdd(&cnt[c], 1);
  }
  block_sum(acc, lds);
  if (threadIdx.x == 0) u2_part[blk] = acc[0];
  // largest |u|^2: one atomic per block (atomics on one address serialise
  // across the chip)
  __shared__ double wmax[VV_THREADS / 64];
  for (int o = 32; o > 0; o >>= 1) um = fmax(um, __shfl_xor(um, o, 64));
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = um;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < VV_THREADS / 64; ++w) um = fmax(um, wmax[w]);
    atomicMax(&umax[rid], (unsigned long long)__double_as_longlong(um));
  }
}

// copy of every real row into coarse-cell order: position and velocity
__global__ __launch_bounds__(VV_THREADS) void k_vv_scatter(DevPtrs d, int flow,
                                                           const int32_t* __restrict__ cstart,
                                                           const int32_t* __restrict__ vcell,
                                                           const int32_t* __restrict__ slot,
                                                           double4* __restrict__ spos,
                                                           double4* __restrict__ su) {
  const int blk = blockIdx.x;
  const RepDev& R = d.rep[d.blk_rep[blk]];
  for (int k = 0; k < ROWS_PER_BLOCK / VV_THREADS; ++k) {
    const int64_t i = (int64_t)blk * ROWS_PER_BLOCK + k * VV_THREADS + threadIdx.x;
    if (i - R.row_off >= R.n) continue;
    const double4 p = d.pos_alt[i];
    const int64_t dst = (int64_t)cstart[vcell[i]] + slot[i];
    spos[dst] = p;
    su[dst] = vv_u(d, R, i, flow, p.y);
  }
}

// one accepted pair: its bin, and the fixed-point product added to the
// block's histogram (integer LDS atomics: order-independent)
__device__ __forceinline__ void vv_accept(double r2, const double4& hu, const double4& w,
                                          double cscale, double scale, int nb,
                                          unsigned long long* hs, unsigned int* hc) {
  const int k = vv_bin(__dmul_rn(r2, cscale), nb);
  const double p = __dadd_rn(__dadd_rn(__dmul_rn(hu.x, w.x), __dmul_rn(hu.y, w.y)),
                             __dmul_rn(hu.z, w.z));
  const long long qv = (long long)rint(p * scale);
  atomicAdd(&hs[k], (unsigned long long)qv);
  atomicAdd(&hc[k], 1u);
}

// pairs of one chunk of home particles with every candidate of its stencil.
// Rows of cells inside the box (0 <= row < ncy, every axis split into cells)
// take a fast path: the image of a whole run of cells is known (no y image,
// x and z periodic shifts fixed per run), so d = R_i - R_j is formed with
// the same rounded operations the neighbour search applies to every pair it
// accepts (a shift of L in x or z only where the search would apply it, and
// where the two disagree -- |d| exactly L/2 -- only the sign differs), and
// r^2 is the same bits.  Rows across the y boundary and one-cell axes use
// the full per-pair separation.
__global__ __launch_bounds__(VV_HOME) void k_vv_pairs(DevPtrs d, const VvRep* __restrict__ vr,
                                                      const VvBlock* __restrict__ blocks, int nblk,
                                                      const int32_t* __restrict__ cstart,
                                                      const double4* __restrict__ spos,
                                                      const double4* __restrict__ su,
                                                      const unsigned long long* __restrict__ umax,
                                                      int nb, long long* __restrict__ psum,
                                                      unsigned long long* __restrict__ pcnt) {
  extern __shared__ unsigned long long vv_hist[];  // [nb] sums, then [nb] 32-bit counts
  __shared__ double4 cp[VV_STAGE], cu[VV_STAGE];
  const int b = xcd_block(blockIdx.x, nblk);
  if (b >= nblk) return;
  const VvBlock B = blocks[b];
  const RepDev& R = d.rep[B.rep];
  const VvRep& V = vr[B.rep];
  const int t = threadIdx.x;
  unsigned long long* hs = vv_hist;
  unsigned int* hc = (unsigned int*)(vv_hist + nb);
  for (int k = t; k < nb; k += VV_HOME) {
    hs[k] = 0ull;
    hc[k] = 0u;
  }
  const double delta = le_offset(R, *d.step_d - 1);
  const double scale = ldexp(1.0, vv_scale_exp(umax[B.rep], V.log2p));
  const double rmax2 = V.rmax2, cscale = V.cscale;
  // lanes: G = 64 / P groups of P = the home count lanes share the wave (the
  // lanes past the last whole group idle), group g testing candidates g,
  // g + G, g + 2G, ...  (Groups of the next power of two >= the count left
  // up to half the lanes idle.)
  const int P = B.count > 0 ? B.count : 1;
  const int G = VV_HOME / P, g = t / P, hl = t - g * P;
  const bool home = g < G && hl < B.count;
  const int64_t self = (int64_t)B.start + hl;
  double4 hp = make_double4(0.0, 0.0, 0.0, 0.0), hu = hp;
  if (home) {
    hp = spos[self];
    hu = su[self];
  }
  const int cl = B.cell - V.cell0;
  const int ncx = V.nc[0], ncy = V.nc[1], ncz = V.nc[2];
  const int cx = cl % ncx, cy = (cl / ncx) % ncy, cz = cl / (ncx * ncy);
  const int M = V.M;
  const int zr = ncz == 1 ? 0 : M, yr = ncy == 1 ? 0 : M;
  const bool split = ncx > 1 && ncy > 1 && ncz > 1;
  __syncthreads();
  for (int dz = -zr; dz <= zr; ++dz) {
    const double gz = fmax((double)(abs(dz) - 1) * V.len[2] - V.margin, 0.0);
    const int czu = cz + dz;
    const int cz2 = imod(czu, ncz);
    const int kz = czu < 0 ? -1 : (czu >= ncz ? 1 : 0);  // z image of the row
    for (int dy = -yr; dy <= yr; ++dy) {
      const double gy = fmax((double)(abs(dy) - 1) * V.len[1] - V.margin, 0.0);
      const double rem = rmax2 - gy * gy - gz * gz;
      if (rem < 0.0) continue;  // the whole row of cells is beyond r_max
      const double reach = sqrt(rem) + V.margin;
      const int cyr = cy + dy;
      int cy2, lo, hi;
      bool fast = false;
      if (ncy == 1) {
        cy2 = 0; lo = 0; hi = ncx - 1;
      } else if (cyr >= 0 && cyr < ncy) {
        cy2 = cyr;
        fast = split;
        if (ncx == 1) {
          lo = 0; hi = 0;
        } else {
          const int rx = min(M, 1 + (int)floor(reach * V.inv_len[0]));
          lo = cx - rx; hi = cx + rx;
        }
      } else {
        // the row across the y boundary: images shifted by +-delta in x
        const double sd = cyr >= ncy ? delta : -delta;
        cy2 = cyr >= ncy ? cyr - ncy : cyr + ncy;
        const double x0 = (double)cx * V.len[0] - sd, x1 = (double)(cx + 1) * V.len[0] - sd;
        lo = (int)floor((x0 - reach) * V.inv_len[0]);
        hi = (int)floor((x1 + reach) * V.inv_len[0]);
        if (hi - lo + 1 >= ncx) { lo = 0; hi = ncx - 1; }
      }
      const int rowbase = V.cell0 + (cz2 * ncy + cy2) * ncx;
      int u0 = lo;            // unwrapped first cell of the next segment
      int len = hi - lo + 1;
      while (len > 0) {
        const int a = imod(u0, ncx);
        const int kx = u0 < 0 ? -1 : (u0 >= ncx ? 1 : 0);  // x image of the segment
        const int run = (a + len <= ncx) ? len : (ncx - a);
        const int j0 = cstart[rowbase + a], j1 = cstart[rowbase + a + run];
        // candidates before the home chunk are skipped: their pairs are
        // counted from the other end
        for (int c0 = max(j0, B.start); c0 < j1; c0 += VV_STAGE) {
          const int m = min(VV_STAGE, j1 - c0);
          for (int q = t; q < m; q += VV_HOME) {
            cp[q] = spos[c0 + q];
            cu[q] = su[c0 + q];
          }
          __syncthreads();
          if (home && fast) {
            for (int jj = g; jj < m; jj += G) {
              const double4 q = cp[jj];
              double dx = __dsub_rn(hp.x, q.x);
              if (kx < 0) dx = __dadd_rn(dx, R.L[0]);        // j's image one box below in x
              else if (kx > 0) dx = __dsub_rn(dx, R.L[0]);   // one box above
              const double dyy = __dsub_rn(hp.y, q.y);
              double dzz = __dsub_rn(hp.z, q.z);
              if (kz < 0) dzz = __dadd_rn(dzz, R.L[2]);
              else if (kz > 0) dzz = __dsub_rn(dzz, R.L[2]);
              const double r2 = dist2(dx, dyy, dzz);
              if (r2 < rmax2 && (int64_t)(c0 + jj) > self)
                vv_accept(r2, hu, cu[jj], cscale, scale, nb, hs, hc);
            }
          } else if (home) {
            for (int jj = g; jj < m; jj += G) {
              const double4 q = cp[jj];
              double dx, dyy, dzz;
              le_sep(R, delta, hp.x, hp.y, hp.z, q.x, q.y, q.z, dx, dyy, dzz);
              const double r2 = dist2(dx, dyy, dzz);
              if (r2 < rmax2 && (int64_t)(c0 + jj) > self)
                vv_accept(r2, hu, cu[jj], cscale, scale, nb, hs, hc);
            }
          }
          __syncthreads();
        }
        u0 += run;
        len -= run;
      }
    }
  }
  __syncthreads();
  for (int k = t; k < nb; k += VV_HOME) {
    psum[(int64_t)b * nb + k] = (long long)hs[k];
    pcnt[(int64_t)b * nb + k] = hc[k];
  }
}

// first reduce stage: per chunk of up to VV_FOLD table blocks of one
// replica and per bin, the blocks' integers added exactly in 128 bits
__device__ __forceinline__ void add128(unsigned long long& lo, long long& hi,
                                       unsigned long long vlo, long long vhi) {
  const unsigned long long nlo = lo + vlo;
  hi += vhi + (nlo < lo ? 1 : 0);
  lo = nlo;
}

__global__ __launch_bounds__(256) void k_vv_fold(const int2* __restrict__ chunks, int nb,
                                                 const long long* __restrict__ psum,
                                                 const unsigned long long* __restrict__ pcnt,
                                                 unsigned long long* __restrict__ f_lo,
                                                 long long* __restrict__ f_hi,
                                                 unsigned long long* __restrict__ f_cnt) {
  const int2 c = chunks[blockIdx.x];
  for (int k = threadIdx.x; k < nb; k += blockDim.x) {
    unsigned long long lo = 0ull, cnt = 0ull;
    long long hi = 0;
    for (int bb = c.x; bb < c.y; ++bb) {
      const long long v = psum[(int64_t)bb * nb + k];
      add128(lo, hi, (unsigned long long)v, v < 0 ? -1 : 0);
      cnt += pcnt[(int64_t)bb * nb + k];
    }
    const int64_t o = (int64_t)blockIdx.x * nb + k;
    f_lo[o] = lo;
    f_hi[o] = hi;
    f_cnt[o] = cnt;
  }
}

// second stage, per replica and bin: the chunks' 128-bit integers added
// exactly (chunk order), halved (each pair was counted from both ends) and
// scaled back; per replica the blocks' |u|^2 sums in block order
__global__ __launch_bounds__(256) void k_vv_reduce(DevPtrs d, const VvRep* __restrict__ vr,
                                                   const int32_t* __restrict__ rep_chunk0,
                                                   int nrep, int nb,
                                                   const unsigned long long* __restrict__ f_lo,
                                                   const long long* __restrict__ f_hi,
                                                   const unsigned long long* __restrict__ f_cnt,
                                                   const unsigned long long* __restrict__ umax,
                                                   const double* __restrict__ u2_part,
                                                   double* __restrict__ out_sum,
                                                   long long* __restrict__ out_cnt,
                                                   double* __restrict__ out_u2) {
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o < (int64_t)nrep * nb) {
    const int rep = (int)(o / nb), k = (int)(o % nb);
    unsigned long long lo = 0ull, c = 0ull;
    long long hi = 0;
    for (int ch = rep_chunk0[rep]; ch < rep_chunk0[rep + 1]; ++ch) {
      const int64_t q = (int64_t)ch * nb + k;
      add128(lo, hi, f_lo[q], f_hi[q]);
      c += f_cnt[q];
    }
    // to FP64 through the magnitude (a small negative total has hi = -1 and
    // lo near 2^64: converting those parts separately would cancel)
    const bool neg = hi < 0;
    unsigned long long mlo = lo, mhi = (unsigned long long)hi;
    if (neg) {
      mlo = ~lo + 1ull;
      mhi = ~mhi + (mlo == 0ull ? 1ull : 0ull);
    }
    const double mag = (double)mhi * 18446744073709551616.0 + (double)mlo;
    const double val = neg ? -mag : mag;
    const int S = vv_scale_exp(umax[rep], vr[rep].log2p);
    out_sum[o] = ldexp(val, -S);
    out_cnt[o] = (long long)c;
  }
  if (o < nrep) {
    const RepDev& R = d.rep[o];
    double s = 0.0;
    for (int bb = 0; bb < R.nblk; ++bb) s += u2_part[R.blk_off + bb];
    out_u2[o] = s;
  }
}

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------
int vv_home() { return VV_HOME; }

hipError_t launch_vv_bin(const DevPtrs& d, const VvRep* vr, int flow, int32_t* cnt,
                         int32_t* vcell, int32_t* slot, unsigned long long* umax, double* u2_part,
                         hipStream_t s) {
  hipLaunchKernelGGL(k_vv_bin, dim3(d.nblk), dim3(VV_THREADS), 0, s, d, vr, flow, cnt, vcell, slot,
                     umax, u2_part);
  return hipGetLastError();
}

hipError_t launch_vv_scatter(const DevPtrs& d, int flow, const int32_t* cstart,
                             const int32_t* vcell, const int32_t* slot, double4* spos,
                             double4* su, hipStream_t s) {
  hipLaunchKernelGGL(k_vv_scatter, dim3(d.nblk), dim3(VV_THREADS), 0, s, d, flow, cstart, vcell,
                     slot, spos, su);
  return hipGetLastError();
}

hipError_t launch_vv_pairs(const DevPtrs& d, const VvRep* vr, const VvBlock* blocks, int nblk,
                           const int32_t* cstart, const double4* spos, const double4* su,
                           const unsigned long long* umax, int nb, long long* psum,
                           unsigned long long* pcnt, hipStream_t s, hipEvent_t ev0,
                           hipEvent_t ev1) {
  if (nblk <= 0) return hipSuccess;
  const dim3 g(xcd_grid(nblk)), bl(VV_HOME);
  const size_t lds = (sizeof(unsigned long long) + sizeof(unsigned int)) * (size_t)nb;
  if (ev0 || ev1)
    hipExtLaunchKernelGGL(k_vv_pairs, g, bl, lds, s, ev0, ev1, 0, d, vr, blocks, nblk, cstart,
                          spos, su, umax, nb, psum, pcnt);
  else
    hipLaunchKernelGGL(k_vv_pairs, g, bl, lds, s, d, vr, blocks, nblk, cstart, spos, su, umax, nb,
                       psum, pcnt);
  return hipGetLastError();
}

int vv_fold() { return VV_FOLD; }

hipError_t launch_vv_reduce(const DevPtrs& d, const VvRep* vr, const int2* chunks, int nchunk,
                            const int32_t* rep_chunk0, int nrep, int nb, const long long* psum,
                            const unsigned long long* pcnt, unsigned long long* f_lo,
                            long long* f_hi, unsigned long long* f_cnt,
                            const unsigned long long* umax, const double* u2_part,
                            double* out_sum, long long* out_cnt, double* out_u2, hipStream_t s) {
  if (nchunk > 0)
    hipLaunchKernelGGL(k_vv_fold, dim3((unsigned)nchunk), dim3(256), 0, s, chunks, nb, psum, pcnt,
                       f_lo, f_hi, f_cnt);
  const int64_t n = std::max<int64_t>((int64_t)nrep * nb, nrep);
  hipLaunchKernelGGL(k_vv_reduce, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, d, vr,
                     rep_chunk0, nrep, nb, f_lo, f_hi, f_cnt, umax, u2_part, out_sum, out_cnt,
                     out_u2);
  return hipGetLastError();
}
