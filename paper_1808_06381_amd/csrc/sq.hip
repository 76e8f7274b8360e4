// sq.hip -- structure factor of the blob centres (Results section, Eq.
// Sfactor) on gfx950: S(q) = |rho(q)|^2 / C, rho(q) = sum_c exp(-i q . R_c),
// for one configuration of each replica.
//
// Wavevectors.  A Lees-Edwards box with offset delta has its images at
// R + a Lx x + b (Ly y + delta x) + c Lz z; the wavevectors that give every
// image the same phase are
//   q = (2 pi mx / Lx, 2 pi my / Ly - 2 pi mx delta / (Lx Ly), 2 pi mz / Lz)
// for integer (mx, my, mz), so that q . R = 2 pi (mx sx + my sy + mz sz) in
// the sheared fractional coordinates sx = x / Lx - delta y / (Lx Ly),
// sy = y / Ly, sz = z / Lz.  The phase factorises,
//   exp(-i q . R_c) = A_c(mx) B_c(my),  A_c(mx) = exp(-2 pi i mx sx),
//   B_c(my) = exp(-2 pi i (my sy + mz sz)),
// so on an (mx, my) grid rho = sum_c A_c(mx) B_c(my) is a complex dense
// contraction over particles whose operands are generated on the fly: the
// work is FP64 arithmetic, not memory traffic (a particle's 24 bytes feed
// nx * ny complex products).
//
// Layout.  k_sq_partial: a block of eight waves takes one tile of 64 mx x W
// my values (W = the grid's my count rounded up to 16, at most 160) and one
// chunk of one replica's rows.  Per group of 16 particles it first forms each
// particle's sheared fractional coordinates and its two unit steps
// exp(-2 pi i sx), exp(-2 pi i sy) (two sincospi per particle), then writes
// the A and B tables to LDS in runs of 8 entries (a sincospi for the run's
// first entry, complex multiplication by the particle's step for the
// others), then the contraction runs on the matrix cores: FP64 16 x 16 x 4
// MFMA, wave w owning mx rows 16(w mod 4).. and the 16-wide my tiles of
// parity w / 4, four particles per step, Re += Ar Br - Ai Bi and
// Im += Ar Bi + Ai Br as four real products.  One block covers every my
// value of its mx rows (up to 160), so a particle's A table is built once,
// not once per my tile; my tiles entirely past the grid are skipped.  The
// vector units only generate the tables.  k_sq_reduce: per replica and q,
// the chunks' partial sums in chunk order, then |rho|^2 / C.  No
// floating-point atomics: the result is deterministic.
// Operand layout of v_mfma_f64_16x16x4f64 (checked on the device): lane l
// supplies A[l%16][l/16] and B[l/16][l%16] and receives D[4r + l/16][l%16]
// in accumulator register r.
#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "launch.h"
#include "sim_dev.h"

namespace {

constexpr int SQ_THREADS = 512;
constexpr int SQ_TX = 64;        // mx per tile
constexpr int SQ_TT = 10;        // 16-wide my tiles per block at most
constexpr int SQ_TYMAX = 16 * SQ_TT;
constexpr int SQ_P = 16;         // particles per LDS group (a multiple of 4)
constexpr int SQ_RUN = 8;        // table entries per sincospi (complex recurrence)
static_assert(SQ_TX == 16 * 4 && SQ_THREADS == 8 * 64 && SQ_TT <= 10,
              "16 mx rows and up to five my tiles per wave");
static_assert(SQ_TX % SQ_RUN == 0 && 16 % SQ_RUN == 0, "runs inside a tile");

typedef double f64x4 __attribute__((ext_vector_type(4)));

struct SqChunk {
  int32_t rep;     // replica
  int32_t pad;
  int64_t row0;    // first row
  int64_t rows;    // rows of the chunk (all real particles)
};

}  // namespace

// my columns of a tile: the grid's, rounded up to 16, at most SQ_TYMAX
__host__ __device__ __forceinline__ int sq_tile_w(int ny) {
  const int w = (ny + 15) / 16 * 16;
  return w < SQ_TYMAX ? w : SQ_TYMAX;
}

// partial[(chunk * ntile + tile) * SQ_TX * tile_w + o] = sum over the chunk's
// particles of A(mx) B(my), o = (mx - mx0) * tile_w + (my - my0); complex as
// double2 (re, im)
__global__ __launch_bounds__(SQ_THREADS) void k_sq_partial(DevPtrs d, const SqChunk* __restrict__ chunks,
                                                           int nx, int my_max, int mz, int tiles_y,
                                                           int tile_w, double2* __restrict__ partial) {
  // rows padded by one entry: the table writes (16 particles of one run per
  // 16 lanes) and the MFMA operand reads fall on distinct banks
  __shared__ double2 A[SQ_P][SQ_TX + 1];
  __shared__ double2 B[SQ_P][SQ_TYMAX + 1];
  __shared__ double2 stA[SQ_P], stB[SQ_P];  // unit steps exp(-2 pi i sx), exp(-2 pi i sy)
  __shared__ double fs[3][SQ_P];            // sx, sy, sz
  const int tile = blockIdx.x, ci = blockIdx.y;
  const SqChunk ch = chunks[ci];
  const RepDev& R = d.rep[ch.rep];
  const int mx0 = (tile / tiles_y) * SQ_TX;
  const int my0 = -my_max + (tile % tiles_y) * tile_w;
  const int ntt = tile_w / 16;
  const double delta = le_offset(R, *d.step_d);
  const double ilx = 1.0 / R.L[0], ily = 1.0 / R.L[1], ilz = 1.0 / R.L[2];
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
  const int wm = wave & 3, wh = wave >> 2;   // mx rows 16 wm.., my tiles tt = 2u + wh
  const int li = lane & 15, lk = lane >> 4;  // operand row / column, particle of the step
  f64x4 re[5], im[5];
#pragma unroll
  for (int u = 0; u < 5; ++u) {
    re[u] = f64x4{0.0, 0.0, 0.0, 0.0};
    im[u] = f64x4{0.0, 0.0, 0.0, 0.0};
  }
  const int runs_a = SQ_TX / SQ_RUN, runs = runs_a + tile_w / SQ_RUN;
  // the particle step of a group (coordinates and unit steps, threads
  // t < SQ_P) runs while the previous group is contracted, its positions
  // loaded one group earlier still
  auto particles = [&](int64_t g, const double4& r) {
    if (t < SQ_P && g + t < ch.rows) {
      const double sx = r.x * ilx - delta * r.y * (ilx * ily);
      const double sy = r.y * ily;
      fs[0][t] = sx;
      fs[1][t] = sy;
      fs[2][t] = r.z * ilz;
      double ss, cs;
      sincospi(2.0 * sx, &ss, &cs);
      stA[t] = make_double2(cs, -ss);
      sincospi(2.0 * sy, &ss, &cs);
      stB[t] = make_double2(cs, -ss);
    }
  };
  auto load_pos = [&](int64_t g) {
    return t < SQ_P && g + t < ch.rows ? d.pos[ch.row0 + g + t] : make_double4(0.0, 0.0, 0.0, 0.0);
  };
  particles(0, load_pos(0));
  double4 rnext = load_pos(SQ_P);
  __syncthreads();
  for (int64_t g = 0; g < ch.rows; g += SQ_P) {
    const int np = (int)min<int64_t>(SQ_P, ch.rows - g);
    // phase tables of this group: A[p][mx - mx0], B[p][my - my0], in runs
    // of SQ_RUN consecutive entries: the first by sincospi, the others by
    // complex multiplication with the unit step (error <= 2 (SQ_RUN - 1)
    // ulp, against one sincospi per entry)
    for (int w = t; w < SQ_P * runs; w += SQ_THREADS) {
      const int p = w % SQ_P, run = w / SQ_P;
      const bool isA = run < runs_a;
      const int k0 = (isA ? run : run - runs_a) * SQ_RUN;
      double2* dst = isA ? &A[p][k0] : &B[p][k0];
      if (p >= np) {  // rows past the group's particles: exact zeros
#pragma unroll
        for (int j = 0; j < SQ_RUN; ++j) dst[j] = make_double2(0.0, 0.0);
        continue;
      }
      double s0, c0;
      if (isA) sincospi(2.0 * (double)(mx0 + k0) * fs[0][p], &s0, &c0);
      else sincospi(2.0 * ((double)(my0 + k0) * fs[1][p] + (double)mz * fs[2][p]), &s0, &c0);
      // z = exp(-i phase) = (c, -s); step u
      double zr = c0, zi = -s0;
      const double2 st = isA ? stA[p] : stB[p];
      const double ur = st.x, ui = st.y;
      dst[0] = make_double2(zr, zi);
#pragma unroll
      for (int j = 1; j < SQ_RUN; ++j) {
        const double nr = fma(zr, ur, -zi * ui);
        const double ni = fma(zr, ui, zi * ur);
        zr = nr;
        zi = ni;
        dst[j] = make_double2(zr, zi);
      }
    }
    __syncthreads();
    // the next group's particle step (the tables of this one are built)
    if (g + SQ_P < ch.rows) {
      particles(g + SQ_P, rnext);
      rnext = load_pos(g + 2 * SQ_P);
    }
    // the contraction over this group's particles, four per MFMA step
    for (int p0 = 0; p0 < np; p0 += 4) {
      const double2 a = A[p0 + lk][16 * wm + li];
#pragma unroll
      for (int u = 0; u < 5; ++u) {
        const int tt = 2 * u + wh;
        if (tt < ntt) {
          const double2 b = B[p0 + lk][16 * tt + li];
          re[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.x, re[u], 0, 0, 0);
          re[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(-a.y, b.y, re[u], 0, 0, 0);
          im[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.x, b.y, im[u], 0, 0, 0);
          im[u] = __builtin_amdgcn_mfma_f64_16x16x4f64(a.y, b.x, im[u], 0, 0, 0);
        }
      }
    }
    __syncthreads();  // the tables are rewritten for the next group, whose
                      // particle step is now visible
  }
  const int64_t base = ((int64_t)ci * gridDim.x + tile) * ((int64_t)SQ_TX * tile_w);
#pragma unroll
  for (int u = 0; u < 5; ++u) {
    const int tt = 2 * u + wh;
    if (tt >= ntt) continue;
#pragma unroll
    for (int r = 0; r < 4; ++r)
      partial[base + (16 * wm + 4 * r + lk) * tile_w + 16 * tt + li] =
          make_double2(re[u][r], im[u][r]);
  }
  (void)nx;
}

// out[(rep * nx + mx) * ny + (my + my_max)] = |sum of the replica's chunk
// partials in chunk order|^2 / C
__global__ __launch_bounds__(256) void k_sq_reduce(DevPtrs d, const int32_t* __restrict__ rep_chunk0,
                                                   int nrep, int nx, int my_max, int tiles_y,
                                                   int tile_w, int ntile,
                                                   const double2* __restrict__ partial,
                                                   double* __restrict__ out) {
  const int ny = 2 * my_max + 1;
  const int64_t o = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= (int64_t)nrep * nx * ny) return;
  const int rep = (int)(o / ((int64_t)nx * ny));
  const int q = (int)(o % ((int64_t)nx * ny));
  const int mx = q / ny, myi = q % ny;
  const int tile = (mx / SQ_TX) * tiles_y + myi / tile_w;
  const int off = (mx % SQ_TX) * tile_w + myi % tile_w;
  double re = 0.0, im = 0.0;
  for (int c = rep_chunk0[rep]; c < rep_chunk0[rep + 1]; ++c) {
    const double2 v = partial[((int64_t)c * ntile + tile) * ((int64_t)SQ_TX * tile_w) + off];
    re += v.x;
    im += v.y;
  }
  const int n = d.rep[rep].n;
  out[o] = n > 0 ? (re * re + im * im) / (double)n : 0.0;
}

// ---------------------------------------------------------------------------
// host side: chunking and launches (device scratch from the caller)
// ---------------------------------------------------------------------------
namespace {
constexpr int64_t SQ_CHUNK = 4096;  // rows per block
}

int64_t sq_chunk_count(const std::vector<int64_t>& rep_rows) {
  int64_t c = 0;
  for (int64_t n : rep_rows) c += (n + SQ_CHUNK - 1) / SQ_CHUNK;
  return c;
}

int64_t sq_tile_count(int nx, int my_max) {
  const int ny = 2 * my_max + 1, w = sq_tile_w(ny);
  return (int64_t)((nx + SQ_TX - 1) / SQ_TX) * ((ny + w - 1) / w);
}

size_t sq_chunk_bytes() { return sizeof(SqChunk); }
size_t sq_partial_bytes(int64_t nchunk, int nx, int my_max) {
  return (size_t)nchunk * (size_t)sq_tile_count(nx, my_max) * SQ_TX *
         (size_t)sq_tile_w(2 * my_max + 1) * sizeof(double2);
}

// The chunk table of every replica built on the device (one thread walks the
// replicas: a handful of stores per chunk), so that a caller's scratch can
// be filled without a host table.
__global__ void k_sq_chunks(DevPtrs d, SqChunk* __restrict__ chunks, int32_t* __restrict__ rep_chunk0) {
  if (blockIdx.x != 0 || threadIdx.x != 0) return;
  int32_t c = 0;
  for (int r = 0; r < d.nrep; ++r) {
    rep_chunk0[r] = c;
    const RepDev& R = d.rep[r];
    for (int64_t a = 0; a < R.n; a += SQ_CHUNK)
      chunks[c++] = SqChunk{r, 0, R.row_off + a, min<int64_t>(SQ_CHUNK, (int64_t)R.n - a)};
  }
  rep_chunk0[d.nrep] = c;
}

namespace {
size_t up256(size_t b) { return (b + 255) / 256 * 256; }
}

// Bytes of caller scratch that launch_sq_scratch needs: chunk table, chunk
// offsets, partial sums (256-byte aligned pieces).
size_t sq_scratch_bytes(int64_t nchunk, int nrep, int nx, int my_max) {
  return up256(sizeof(SqChunk) * (size_t)std::max<int64_t>(nchunk, 1)) +
         up256(sizeof(int32_t) * (size_t)(nrep + 1)) +
         up256(sq_partial_bytes(std::max<int64_t>(nchunk, 1), nx, my_max));
}

// The same kernels as launch_sq with every table on the device: `scratch`
// (sq_scratch_bytes() bytes, 256-byte aligned) holds the chunk table, the
// chunk offsets and the partial sums, out_d receives replicas x nx x ny.
// Nothing is allocated and nothing is copied from the host; the launches
// are asynchronous on stream s.
hipError_t launch_sq_scratch(const DevPtrs& d, int64_t nchunk, int nx, int my_max, int mz,
                             void* scratch, double* out_d, hipStream_t s) {
  char* base = (char*)scratch;
  SqChunk* chunks = (SqChunk*)base;
  const size_t b_ch = up256(sizeof(SqChunk) * (size_t)std::max<int64_t>(nchunk, 1));
  int32_t* c0 = (int32_t*)(base + b_ch);
  const size_t b_c0 = up256(sizeof(int32_t) * (size_t)(d.nrep + 1));
  double2* partial = (double2*)(base + b_ch + b_c0);
  hipLaunchKernelGGL(k_sq_chunks, dim3(1), dim3(64), 0, s, d, chunks, c0);
  const int ny = 2 * my_max + 1;
  const int tile_w = sq_tile_w(ny);
  const int tiles_y = (ny + tile_w - 1) / tile_w;
  const int ntile = (int)sq_tile_count(nx, my_max);
  if (nchunk > 0)
    hipLaunchKernelGGL(k_sq_partial, dim3(ntile, (unsigned)nchunk), dim3(SQ_THREADS), 0, s, d,
                       (const SqChunk*)chunks, nx, my_max, mz, tiles_y, tile_w, partial);
  const int64_t nout = (int64_t)d.nrep * nx * ny;
  hipLaunchKernelGGL(k_sq_reduce, dim3((unsigned)((nout + 255) / 256)), dim3(256), 0, s, d, c0,
                     d.nrep, nx, my_max, tiles_y, tile_w, ntile, partial, out_d);
  return hipGetLastError();
}

// rep_row0 / rep_rows: first row and real particles of each replica;
// chunks_d (sq_chunk_bytes() x count) and rep_chunk0_d (nrep + 1 int32)
// are device scratch, filled here from the host tables; ev0/ev1 (optional)
// bracket the contraction kernel's launch
hipError_t launch_sq(const DevPtrs& d, const std::vector<int64_t>& rep_row0,
                     const std::vector<int64_t>& rep_rows, int nx, int my_max, int mz,
                     void* chunks_d, int32_t* rep_chunk0_d, double2* partial_d, double* out_d,
                     hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
  std::vector<SqChunk> ch;
  std::vector<int32_t> c0;
  for (size_t r = 0; r < rep_rows.size(); ++r) {
    c0.push_back((int32_t)ch.size());
    for (int64_t a = 0; a < rep_rows[r]; a += SQ_CHUNK)
      ch.push_back({(int32_t)r, 0, rep_row0[r] + a, std::min<int64_t>(SQ_CHUNK, rep_rows[r] - a)});
  }
  c0.push_back((int32_t)ch.size());
  hipError_t e;
  if (!ch.empty() &&
      (e = hipMemcpyAsync(chunks_d, ch.data(), ch.size() * sizeof(SqChunk), hipMemcpyHostToDevice, s)))
    return e;
  if ((e = hipMemcpyAsync(rep_chunk0_d, c0.data(), c0.size() * sizeof(int32_t),
                          hipMemcpyHostToDevice, s)))
    return e;
  const int ny = 2 * my_max + 1;
  const int tile_w = sq_tile_w(ny);
  const int tiles_y = (ny + tile_w - 1) / tile_w;
  const int ntile = (int)sq_tile_count(nx, my_max);
  if (!ch.empty()) {
    const dim3 g(ntile, (unsigned)ch.size()), b(SQ_THREADS);
    if (ev0 || ev1)
      hipExtLaunchKernelGGL(k_sq_partial, g, b, 0, s, ev0, ev1, 0, d, (const SqChunk*)chunks_d,
                            nx, my_max, mz, tiles_y, tile_w, partial_d);
    else
      hipLaunchKernelGGL(k_sq_partial, g, b, 0, s, d, (const SqChunk*)chunks_d, nx, my_max, mz,
                         tiles_y, tile_w, partial_d);
  }
  const int64_t nout = (int64_t)rep_rows.size() * nx * ny;
  hipLaunchKernelGGL(k_sq_reduce, dim3((unsigned)((nout + 255) / 256)), dim3(256), 0, s, d,
                     rep_chunk0_d, (int)rep_rows.size(), nx, my_max, tiles_y, tile_w, ntile,
                     partial_d, out_d);
  // host tables must outlive the asynchronous copies
  if ((e = hipStreamSynchronize(s))) return e;
  return hipGetLastError();
}
