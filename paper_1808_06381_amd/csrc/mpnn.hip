// mpnn.hip -- learned preconditioner on gfx950: a three-layer message-passing
// network on the pair graph of the friction matrix A (Method section, Eq. 9)
// that produces an SPD approximate inverse with the sparsity of A, its
// training loss and gradient, and Adam.
//
// Network (hidden 32; weights enter as bfloat16, products accumulate in FP32;
// with bfloat16 activations, the default, the products see bf16 inputs and
// the residual stream h is stored in bf16 between layers):
//   x_i = (t_i, a_i, deg_i/8), t_i = alpha sum_j w_ij / D_i, a_i = sum_j What_ij,
//   What_ij = alpha w_ij / sqrt(D_i D_j); e_ij = (r_ij/rc, w_ij, What_ij)
//   h0 = relu(W0 x + b0)
//   layer: y_j = P h_j, m_i = 1/8 sum_j relu(y_j + Q e_ij + c),
//          h_i <- h_i + relu(U h_i + V m_i + d)
//   heads: lam_i = softplus(v.h_i + v0) + floor (0.3 unless set),
//          S_ij = z.(h_i*h_j) + ze.e_ij + z0
//   M^-1 = D^-1/2 (diag(lam) + S) D^-1/2: symmetric, positive diagonal (the
//   solver's true-residual test and Jacobi fallback cover a non-definite M^-1;
//   the initial heads give the positive definite two-term Neumann series).
// Loss on the last solved system (A, b, x*): ||M^-1 b - x*||_A^2 / ||x*||_A^2.
//
// Layout: one half-wave (32 lanes) per node, lane k = hidden feature k, so a
// neighbour's feature row (32 floats) is one coalesced 128-byte load.
// Blocks of 256 threads own 64 consecutive rows; the parameter gradients are
// per-block partial sums reduced in a fixed order (deterministic).
#include <hip/hip_runtime.h>

#include "launch.h"
#include "mpnn.h"
#include "sim_dev.h"

namespace {

constexpr int NODES = MP_THREADS / MP_H;     // nodes per pass (8)
constexpr int PASSES = MP_ROWS / NODES;      // passes per block (8)

__device__ __forceinline__ float bf16_value(uint16_t b) {
  return __uint_as_float(((uint32_t)b) << 16);
}

// round an FP32 value to the nearest bfloat16 (ties to even), as FP32
__device__ __forceinline__ float bf16_round(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return f;
  u += 0x7fffu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xffff0000u);
}

__device__ __forceinline__ uint16_t bf16_bits(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return (uint16_t)((u >> 16) | 0x40u);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ float act_in(const MpPtrs& m, float v) {
  return m.round_act ? bf16_round(v) : v;
}

// sum over the 32 lanes of a half-wave, the same tree in every lane
__device__ __forceinline__ float half_sum(float v) {
#pragma unroll
  for (int o = 16; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ float sigmoidf_(float t) { return 1.0f / (1.0f + expf(-t)); }
__device__ __forceinline__ float softplusf_(float t) { return t > 20.0f ? t : log1pf(expf(t)); }

// copy n bf16 weights starting at off into LDS as FP32
__device__ __forceinline__ void load_w(const MpPtrs& m, float* dst, int off, int n) {
  for (int k = threadIdx.x; k < n; k += blockDim.x) dst[k] = bf16_value(m.w16[off + k]);
}

// copy a 32 x 32 weight matrix W[k][q] into LDS transposed, dst[q][k]: lane k
// then reads consecutive words for a fixed q (no bank conflicts)
__device__ __forceinline__ void load_wt(const MpPtrs& m, float* dst, int off) {
  for (int idx = threadIdx.x; idx < MP_H * MP_H; idx += blockDim.x) {
    const int k = idx / MP_H, q = idx % MP_H;
    dst[q * MP_H + k] = bf16_value(m.w16[off + idx]);
  }
}

}  // namespace

// ---------------------------------------------------------------------------
// forward
// ---------------------------------------------------------------------------

// node and edge features (one thread per row)
__global__ __launch_bounds__(256) void k_mp_features(DevPtrs d, MpPtrs m) {
  if (d.ctrl->overflow) return;  // row pointers may exceed the capacity
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.rows) return;
  const double di = d.diag[i];
  const double alpha = d.rep[d.blk_rep[i / ROWS_PER_BLOCK]].alpha;
  const int e0 = d.rowptr[i], e1 = d.rowptr[i + 1];
  double s = 0.0, a = 0.0;
  for (int e = e0; e < e1; ++e) {
    const int j = d.col[e];
    const double v = -d.val[e];
    const double what = v / sqrt(di * d.diag[j]);
    s += v;
    a += what;
    m.ef[3 * (int64_t)e + 0] = m.er[e];
    m.ef[3 * (int64_t)e + 1] = (float)(v / alpha);
    m.ef[3 * (int64_t)e + 2] = (float)what;
  }
  m.x[3 * i + 0] = (float)(s / di);
  m.x[3 * i + 1] = (float)a;
  m.x[3 * i + 2] = (float)(e1 - e0) * 0.125f;
}

// h0 = relu(W0 x + b0) and y^0 = P_0 h0
__global__ __launch_bounds__(MP_THREADS) void k_mp_encode(DevPtrs d, MpPtrs m) {
  if (d.ctrl->overflow) return;  // row pointers may exceed the capacity
  __shared__ float w0[MP_H * MP_FN], b0[MP_H], P[MP_H * MP_H];
  __shared__ float sh[NODES][MP_H];
  load_w(m, w0, MP_OFF_W0, MP_H * MP_FN);
  load_w(m, b0, MP_OFF_B0, MP_H);
  load_wt(m, P, MP_OFF_L0 + MP_L_P);
  __syncthreads();
  const int slot = threadIdx.x / MP_H, k = threadIdx.x % MP_H;
  for (int pass = 0; pass < PASSES; ++pass) {
    const int64_t i = (int64_t)blockIdx.x * MP_ROWS + pass * NODES + slot;
    float acc = b0[k];
#pragma unroll
    for (int f = 0; f < MP_FN; ++f) acc += w0[k * MP_FN + f] * act_in(m, m.x[3 * i + f]);
    const float h = acc > 0.0f ? acc : 0.0f;
    m.h[i * MP_H + k] = h;
    sh[slot][k] = act_in(m, h);
    __syncthreads();
    float y = 0.0f;
#pragma unroll 8
    for (int q = 0; q < MP_H; ++q) y += P[q * MP_H + k] * sh[slot][q];
    m.y[i * MP_H + k] = y;
    __syncthreads();
  }
}

// one message-passing layer l: m, a (stored for training), h^{l+1}, y^{l+1}
__global__ __launch_bounds__(MP_THREADS) void k_mp_layer(DevPtrs d, MpPtrs m, int l) {
  if (d.ctrl->overflow) return;  // row pointers may exceed the capacity
  __shared__ float Q[MP_H * MP_FE], c[MP_H], U[MP_H * MP_H], V[MP_H * MP_H], dd[MP_H],
      Pn[MP_H * MP_H];
  __shared__ float sh[NODES][MP_H], sm[NODES][MP_H];
  const int base = MP_OFF_L0 + l * MP_L_SIZE;
  load_w(m, Q, base + MP_L_Q, MP_H * MP_FE);
  load_w(m, c, base + MP_L_C, MP_H);
  load_wt(m, U, base + MP_L_U);
  load_wt(m, V, base + MP_L_V);
  load_w(m, dd, base + MP_L_D, MP_H);
  const bool next = l + 1 < MP_NL;
  if (next) load_wt(m, Pn, base + MP_L_SIZE + MP_L_P);
  __syncthreads();
  const int slot = threadIdx.x / MP_H, k = threadIdx.x % MP_H;
  const float* __restrict__ hin = m.h + (int64_t)l * m.rows * MP_H;
  float* __restrict__ hout = m.h + (int64_t)(l + 1) * m.rows * MP_H;
  const float* __restrict__ y = m.y + (int64_t)l * m.rows * MP_H;
  for (int pass = 0; pass < PASSES; ++pass) {
    const int64_t i = (int64_t)blockIdx.x * MP_ROWS + pass * NODES + slot;
    const int e0 = d.rowptr[i], e1 = d.rowptr[i + 1];
    float msg = 0.0f;
    for (int e = e0; e < e1; ++e) {
      const int64_t j = d.col[e];
      float s = y[j * MP_H + k] + c[k];
#pragma unroll
      for (int f = 0; f < MP_FE; ++f) s += Q[k * MP_FE + f] * act_in(m, m.ef[3 * (int64_t)e + f]);
      msg += s > 0.0f ? s : 0.0f;
    }
    msg *= MP_MSG;
    const float h = hin[i * MP_H + k];
    sh[slot][k] = act_in(m, h);
    sm[slot][k] = act_in(m, msg);
    __syncthreads();
    float a = dd[k];
#pragma unroll 8
    for (int q = 0; q < MP_H; ++q) a += U[q * MP_H + k] * sh[slot][q] + V[q * MP_H + k] * sm[slot][q];
    const float hn = h + (a > 0.0f ? a : 0.0f);
    hout[i * MP_H + k] = hn;
    if (m.store_train) {
      m.m[((int64_t)l * m.rows + i) * MP_H + k] = msg;
      m.a[((int64_t)l * m.rows + i) * MP_H + k] = a;
    }
    __syncthreads();
    if (next) {
      sh[slot][k] = act_in(m, hn);
      __syncthreads();
      float yn = 0.0f;
#pragma unroll 8
      for (int q = 0; q < MP_H; ++q) yn += Pn[q * MP_H + k] * sh[slot][q];
      m.y[((int64_t)(l + 1) * m.rows + i) * MP_H + k] = yn;
      __syncthreads();
    }
  }
}

// heads: M^-1 diagonal and off-diagonal values, head pre-activations
__global__ __launch_bounds__(MP_THREADS) void k_mp_heads(DevPtrs d, MpPtrs m) {
  if (d.ctrl->overflow) return;  // row pointers may exceed the capacity
  __shared__ float hv[MP_H + 1], hz[MP_H], hze[MP_FE + 1];
  load_w(m, hv, MP_OFF_HEAD + MP_H_V, MP_H + 1);
  load_w(m, hz, MP_OFF_HEAD + MP_H_Z, MP_H);
  load_w(m, hze, MP_OFF_HEAD + MP_H_ZE, MP_FE + 1);
  __syncthreads();
  const int slot = threadIdx.x / MP_H, k = threadIdx.x % MP_H;
  const float* __restrict__ hf = m.h + (int64_t)MP_NL * m.rows * MP_H;
  for (int pass = 0; pass < PASSES; ++pass) {
    const int64_t i = (int64_t)blockIdx.x * MP_ROWS + pass * NODES + slot;
    const float hk = act_in(m, hf[i * MP_H + k]);
    const float tau = half_sum(hv[k] * hk) + hv[MP_H];
    const double di = d.diag[i];
    const int e0 = d.rowptr[i], e1 = d.rowptr[i + 1];
    for (int e = e0; e < e1; ++e) {
      const int64_t j = d.col[e];
      const float hj = act_in(m, hf[j * MP_H + k]);
      float t = half_sum(hz[k] * (hk * hj));
#pragma unroll
      for (int f = 0; f < MP_FE; ++f) t += hze[f] * act_in(m, m.ef[3 * (int64_t)e + f]);
      t += hze[MP_FE];
      if (k == 0) {
        m.tg[e] = t;
        m.moff[e] = (float)((double)t / sqrt(di * d.diag[j]));
      }
    }
    if (k == 0) {
      m.tau[i] = tau;
      m.mdiag[i] = ((double)softplusf_(tau) + m.lam_floor) / di;
    }
  }
}

// ---------------------------------------------------------------------------
// forward with bf16 activations on the matrix cores.  A block owns MP_ROWS
// consecutive rows; their CSR entries form one contiguous range that is
// walked in chunks of MX_EC entries, four threads per entry (eight features
// each).  Every product consumes h rounded to bf16, so each layer gathers the
// 64-byte bf16 row of h_j per entry (one 16-byte load per thread) and forms
// y_j = P h_j of the chunk on the matrix cores, rather than gathering a stored
// FP32 y_j (twice the bytes); the product is the one that writes y for the
// backward pass, operand for operand, so both give the same bits.  The dense
// node products (32 x 64 and 32 x 32 per node) run as 16 x 16 x 16 bf16 MFMA
// tiles, FP32 accumulate: wave w owns rows 16w..16w+15 of a tile.
// Operand layout of v_mfma_f32_16x16x16_bf16: lane l supplies
// A[l%16][4(l/16)+i] and B[4(l/16)+i][l%16], i < 4, and receives
// D[4(l/16)+r][l%16] in accumulator register r.
// ---------------------------------------------------------------------------
namespace {

typedef short s16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int MX_EC = 64;                  // CSR entries per chunk
constexpr int MX_AS = 2 * MP_H + 8;        // row stride (bf16) of the [h | m] tile
constexpr int MX_HS = MP_H + 8;            // row stride (bf16) of an h tile
constexpr int MX_FS = MP_H + 4;            // row stride (float) of message / h rows

// B operand of a 32-output product whose weight W[n][q] (n output, q input,
// row-major 32 x 32 bf16) starts at off: step s covers inputs 16s..16s+15,
// tile nt covers outputs 16nt..16nt+15.
__device__ __forceinline__ s16x4 mx_bw(const uint16_t* __restrict__ w16, int off, int s, int nt) {
  const int lane = threadIdx.x & 63;
  const int n = 16 * nt + (lane & 15), q = 16 * s + 4 * (lane >> 4);
  s16x4 b;
#pragma unroll
  for (int i = 0; i < 4; ++i) b[i] = (short)w16[off + n * MP_H + q + i];
  return b;
}

// A operand from an LDS bf16 tile (row stride `stride`), rows of wave w
__device__ __forceinline__ s16x4 mx_a(const uint16_t* tile, int stride, int s) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int row = 16 * w + (lane & 15), q = 16 * s + 4 * (lane >> 4);
  return *reinterpret_cast<const s16x4*>(tile + row * stride + q);
}

__device__ __forceinline__ f32x4 mx_mma(s16x4 a, s16x4 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(a, b, c, 0, 0, 0);
}

// B operands of P (at w16[off]) for mx_py
__device__ __forceinline__ void mx_load_p(const uint16_t* __restrict__ w16, int off,
                                          s16x4 (&pw)[2][2]) {
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) pw[s][nt] = mx_bw(w16, off, s, nt);
}

// y = P h for the 16 rows of wave w: P as loaded by mx_load_p, h the bf16
// tile xh (row stride `stride`).  Lane l holds y[16w + 4(l/16) + r][16nt + l%16]
// in acc[nt][r].
__device__ __forceinline__ void mx_py(const s16x4 (&pw)[2][2], const uint16_t* xh, int stride,
                                      f32x4 (&acc)[2]) {
#pragma unroll
  for (int nt = 0; nt < 2; ++nt) acc[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const s16x4 a = mx_a(xh, stride, s);
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) acc[nt] = mx_mma(a, pw[s][nt], acc[nt]);
  }
}

// P (at w16[off]) in LDS, row n (output) at n * MX_PS: the B operand of a
// 16-input step is one 8-byte read per lane, the 16 rows of a tile on
// distinct bank pairs
constexpr int MX_PS = MP_H + 4;
__device__ __forceinline__ void mx_stage_p(const uint16_t* __restrict__ w16, int off, uint16_t* ps) {
  for (int idx = threadIdx.x; idx < MP_H * MP_H; idx += blockDim.x)
    ps[(idx / MP_H) * MX_PS + idx % MP_H] = w16[off + idx];
}

// y = P h as mx_py, the B operands read from the LDS copy of P
__device__ __forceinline__ void mx_py_lds(const uint16_t* ps, const uint16_t* xh, int stride,
                                          f32x4 (&acc)[2]) {
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int nt = 0; nt < 2; ++nt) acc[nt] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const s16x4 a = mx_a(xh, stride, s);
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) {
      const int n = 16 * nt + (lane & 15), q = 16 * s + 4 * (lane >> 4);
      const s16x4 b = *reinterpret_cast<const s16x4*>(ps + n * MX_PS + q);
      acc[nt] = mx_mma(a, b, acc[nt]);
    }
  }
}

// bf16 copy of h^l: layer l gathers it, layer l - 1 (or the encoder) writes it
__device__ __forceinline__ uint16_t* mx_hb(const MpPtrs& m, int l) {
  return ((l ^ MP_NL) & 1) ? m.hb2 : m.hb;
}

// y = P h as FP32 rows of dst (tile origin i0), kept for the backward pass
__device__ __forceinline__ void mx_store_py(const uint16_t* __restrict__ w16, int off,
                                            const uint16_t* xh, int stride,
                                            float* __restrict__ dst, int64_t i0) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  s16x4 pw[2][2];
  mx_load_p(w16, off, pw);
  f32x4 acc[2];
  mx_py(pw, xh, stride, acc);
#pragma unroll
  for (int nt = 0; nt < 2; ++nt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * w + 4 * (lane >> 4) + r;
      dst[(i0 + row) * MP_H + 16 * nt + (lane & 15)] = acc[nt][r];
    }
}

}  // namespace

// features and h0 = relu(W0 x + b0) (FP32 and bf16; y^0 = P_0 h0 when
// training); four lanes per row
__global__ __launch_bounds__(MP_THREADS) void k_mp_encode_mx(DevPtrs d, MpPtrs m) {
  if (d.ctrl->overflow) return;  // row pointers may exceed the capacity
  __shared__ float w0[MP_H * MP_FN], b0[MP_H];
  __shared__ float xs[MP_ROWS][MP_FN];
  __shared__ __align__(16) uint16_t xh[MP_ROWS * MX_HS];
  const int t = threadIdx.x;
  // tiles of MP_ROWS rows in XCD-contiguous ranges: the neighbour rows a
  // tile reads are in its own XCD's L2
  const int ntiles = (int)(m.rows / MP_ROWS);
  const int tile = xcd_block(blockIdx.x, ntiles);
  if (tile >= ntiles) return;
  load_w(m, w0, MP_OFF_W0, MP_H * MP_FN);
  load_w(m, b0, MP_OFF_B0, MP_H);
  const int64_t i0 = (int64_t)tile * MP_ROWS;
  const int n = t >> 2, q = t & 3;
  const int64_t i = i0 + n;
  {
    const double di = d.diag[i];
    const double alpha = d.rep[d.blk_rep[i / ROWS_PER_BLOCK]].alpha;
    const int e0 = d.rowptr[i], e1 = d.rowptr[i + 1];
    double s = 0.0, a = 0.0;
    for (int e = e0 + q; e < e1; e += 4) {
      const int j = d.col[e];
      const double v = -d.val[e];
      const double what = v / sqrt(di * d.diag[j]);
      s += v;
      a += what;
      const float f0 = m.er[e], f1 = (float)(v / alpha), f2 = (float)what;
      if (m.store_train) {  // the backward pass reads the FP32 features
        m.ef[3 * (int64_t)e + 0] = f0;
        m.ef[3 * (int64_t)e + 1] = f1;
        m.ef[3 * (int64_t)e + 2] = f2;
      }
      // the forward kernels round the features to bf16 before every use
      *reinterpret_cast<ushort4*>(m.efh + 4 * (int64_t)e) =
          make_ushort4(bf16_bits(f0), bf16_bits(f1), bf16_bits(f2), 0);
    }
    s += __shfl_xor(s, 1, 64);
    a += __shfl_xor(a, 1, 64);
    s += __shfl_xor(s, 2, 64);
    a += __shfl_xor(a, 2, 64);
    if (q == 0) {
      const float x0 = (float)(s / di), x1 = (float)a, x2 = (float)(e1 - e0) * 0.125f;
      m.x[3 * i + 0] = x0;
      m.x[3 * i + 1] = x1;
      m.x[3 * i + 2] = x2;
      xs[n][0] = bf16_round(x0);
      xs[n][1] = bf16_round(x1);
      xs[n][2] = bf16_round(x2);
    }
  }
  __syncthreads();
  float hv[8];
#pragma unroll
  for (int kk = 0; kk < 8; ++kk) {
    const int k = 8 * q + kk;
    float acc = b0[k];
#pragma unroll
    for (int f = 0; f < MP_FN; ++f) acc += w0[k * MP_FN + f] * xs[n][f];
    hv[kk] = acc > 0.0f ? acc : 0.0f;
    xh[n * MX_HS + k] = bf16_bits(hv[kk]);
  }
  if (m.store_train) {  // FP32 h0 for the backward pass (which rounds it to bf16)
    float4* hp = reinterpret_cast<float4*>(m.h + i * MP_H + 8 * q);
    hp[0] = make_float4(hv[0], hv[1], hv[2], hv[3]);
    hp[1] = make_float4(hv[4], hv[5], hv[6], hv[7]);
  }
  __syncthreads();
  *reinterpret_cast<uint4*>(mx_hb(m, 0) + i * MP_H + 8 * q) =
      *reinterpret_cast<const uint4*>(xh + n * MX_HS + 8 * q);
  if (m.store_train) mx_store_py(m.w16, MP_OFF_L0 + MP_L_P, xh, MX_HS, m.y, i0);
}

// one message-passing layer l (bf16 activations): m, a and y^{l+1} (training),
// h^{l+1} in FP32 and bf16
// (seven waves per SIMD: P is read from LDS rather than held in registers,
// which leaves room for seven without spills; measured at N = 8e6 against
// six: 1184 against 1201 us.  Neither more entries per chunk (128, four
// waves: 1722 us) nor a gather two chunks ahead (1276-1318 us) was faster.)
__global__ __launch_bounds__(MP_THREADS) __attribute__((amdgpu_waves_per_eu(7, 8)))
void k_mp_layer_mx(DevPtrs d, MpPtrs m, int l) {
  if (d.ctrl->overflow) return;  // row pointers may exceed the capacity
  __shared__ float Q[MP_H * MP_FE], c[MP_H], dd[MP_H];
  __shared__ __align__(16) uint16_t ps[MP_H * MX_PS];
  __shared__ int rp[MP_ROWS + 1];
  // msg holds one chunk's messages during the gather, then the tile's FP32 h
  __shared__ __align__(16) float msg[MX_EC * MX_FS];
  static_assert(MX_EC == MP_ROWS, "the h tile reuses the message buffer");
  float* const hs = msg;
  // xa holds, in turn: one chunk's bf16 h_j (stride MX_HS) and bf16 edge
  // features during the gather; the tile's [bf16 h | bf16 m] (stride MX_AS);
  // bf16 h^{l+1} in the h half, each wave overwriting only its own 16 rows
  // once its products have read them
  __shared__ __align__(16) uint16_t xa[MP_ROWS * MX_AS];
  static_assert(MX_EC * (MX_HS + 4) <= MP_ROWS * MX_AS, "gather tile exceeds xa");
  uint16_t* const xg = xa;
  uint16_t* const es = xa + MX_EC * MX_HS;
  const int t = threadIdx.x, lane = t & 63, w = t >> 6;
  // tiles in XCD-contiguous ranges: the gathered h_j rows of neighbouring
  // tiles stay in one XCD's L2
  const int ntiles = (int)(m.rows / MP_ROWS);
  const int tile = xcd_block(blockIdx.x, ntiles);
  if (tile >= ntiles) return;
  const int base = MP_OFF_L0 + l * MP_L_SIZE;
  load_w(m, Q, base + MP_L_Q, MP_H * MP_FE);
  load_w(m, c, base + MP_L_C, MP_H);
  load_w(m, dd, base + MP_L_D, MP_H);
  mx_stage_p(m.w16, base + MP_L_P, ps);
  const int64_t i0 = (int64_t)tile * MP_ROWS;
  if (t <= MP_ROWS) rp[t] = d.rowptr[i0 + t];
  __syncthreads();
  const int n = t >> 2, q = t & 3;
  const int64_t rows = m.rows;
  const uint16_t* __restrict__ hbl = mx_hb(m, l);
  // messages: relu(y_j + Q e_ij + c) of every entry, summed per row in entry order
  float acc[8];
#pragma unroll
  for (int kk = 0; kk < 8; ++kk) acc[kk] = 0.0f;
  const int E0 = rp[0], E1 = rp[MP_ROWS];
  // software pipeline: while a chunk is processed, the gather of the next one
  // is in flight and the column indices of the one after are being read
  // (bf16 h_j and edge features are zero past the range)
  uint4 hq = make_uint4(0u, 0u, 0u, 0u);
  ushort4 eq = make_ushort4(0, 0, 0, 0);
  if (E0 + n < E1) {
    hq = *reinterpret_cast<const uint4*>(hbl + (int64_t)d.col[E0 + n] * MP_H + 8 * q);
    if (q == 0) eq = *reinterpret_cast<const ushort4*>(m.efh + 4 * (int64_t)(E0 + n));
  }
  int jn = E0 + MX_EC + n < E1 ? d.col[E0 + MX_EC + n] : 0;
  for (int cb = E0; cb < E1; cb += MX_EC) {
    *reinterpret_cast<uint4*>(xg + n * MX_HS + 8 * q) = hq;
    if (q == 0) *reinterpret_cast<ushort4*>(es + 4 * n) = eq;
    __syncthreads();
    {
      const int e = cb + MX_EC + n;   // entry n of the next chunk (column jn)
      hq = make_uint4(0u, 0u, 0u, 0u);
      eq = make_ushort4(0, 0, 0, 0);
      if (e < E1) {
        hq = *reinterpret_cast<const uint4*>(hbl + (int64_t)jn * MP_H + 8 * q);
        if (q == 0) eq = *reinterpret_cast<const ushort4*>(m.efh + 4 * (int64_t)e);
      }
      jn = e + MX_EC < E1 ? d.col[e + MX_EC] : 0;
    }
    // y_j = P h_j on the matrix cores, then the message of each entry
    {
      f32x4 yv[2];
      mx_py_lds(ps, xg, MX_HS, yv);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int en = 16 * w + 4 * (lane >> 4) + r;
        const ushort4 eq = *reinterpret_cast<const ushort4*>(es + 4 * en);
        const float ef[MP_FE] = {bf16_value(eq.x), bf16_value(eq.y), bf16_value(eq.z)};
#pragma unroll
        for (int nt = 0; nt < 2; ++nt) {
          const int k = 16 * nt + (lane & 15);
          float s = yv[nt][r] + c[k];
#pragma unroll
          for (int f = 0; f < MP_FE; ++f) s += Q[k * MP_FE + f] * ef[f];
          msg[en * MX_FS + k] = s > 0.0f ? s : 0.0f;
        }
      }
    }
    __syncthreads();
    const int lo = max(rp[n], cb), hi = min(rp[n + 1], cb + MX_EC);
    for (int e2 = lo; e2 < hi; ++e2) {
      const float4* mp = reinterpret_cast<const float4*>(msg + (e2 - cb) * MX_FS + 8 * q);
      const float4 m0 = mp[0], m1 = mp[1];
      acc[0] += m0.x; acc[1] += m0.y; acc[2] += m0.z; acc[3] += m0.w;
      acc[4] += m1.x; acc[5] += m1.y; acc[6] += m1.z; acc[7] += m1.w;
    }
    // no barrier here: xg and es were last read before the one above, and
    // msg is next written after the next chunk's first barrier
  }
  __syncthreads();   // every row has summed its messages: msg and xa are restaged
  // stage [bf16(h) | bf16(m)] and the residual h of the tile: the residual
  // stream is kept in bf16 (the copy this layer gathers), so no FP32 h is
  // read or, outside training, written
  {
    const int64_t i = i0 + n;
    const uint4 hq8 = *reinterpret_cast<const uint4*>(hbl + i * MP_H + 8 * q);
    const uint32_t hw[4] = {hq8.x, hq8.y, hq8.z, hq8.w};
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
      const int k = 8 * q + kk;
      const uint16_t hb16 = (uint16_t)((kk & 1) ? (hw[kk >> 1] >> 16) : (hw[kk >> 1] & 0xffffu));
      acc[kk] *= MP_MSG;
      hs[n * MX_FS + k] = bf16_value(hb16);
      xa[n * MX_AS + k] = hb16;
      xa[n * MX_AS + MP_H + k] = bf16_bits(acc[kk]);
    }
    if (m.store_train) {
      float4* mo = reinterpret_cast<float4*>(m.m + ((int64_t)l * rows + i) * MP_H + 8 * q);
      mo[0] = make_float4(acc[0], acc[1], acc[2], acc[3]);
      mo[1] = make_float4(acc[4], acc[5], acc[6], acc[7]);
    }
  }
  __syncthreads();
  // a = d + U h + V m
  f32x4 av[2];
#pragma unroll
  for (int nt = 0; nt < 2; ++nt) {
    const float bias = dd[16 * nt + (lane & 15)];
    av[nt] = f32x4{bias, bias, bias, bias};
  }
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const s16x4 a = mx_a(xa, MX_AS, s);
    const int off = base + (s < 2 ? MP_L_U : MP_L_V - 2 * 16);
#pragma unroll
    for (int nt = 0; nt < 2; ++nt) av[nt] = mx_mma(a, mx_bw(m.w16, off, s, nt), av[nt]);
  }
  float* __restrict__ hout = m.h + (int64_t)(l + 1) * rows * MP_H;
#pragma unroll
  for (int nt = 0; nt < 2; ++nt)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = 16 * w + 4 * (lane >> 4) + r, k = 16 * nt + (lane & 15);
      const float a = av[nt][r];
      const float hn = hs[row * MX_FS + k] + (a > 0.0f ? a : 0.0f);
      const uint16_t hnb = bf16_bits(hn);
      // h^{l+1} is stored rounded to bf16 (the next layer's residual and
      // product input, the heads' input); its FP32 copy, the same value, is
      // for the backward pass only
      if (m.store_train) hout[(i0 + row) * MP_H + k] = bf16_value(hnb);
      if (m.store_train) m.a[((int64_t)l * rows + i0 + row) * MP_H + k] = a;
      xa[row * MX_AS + k] = hnb;
    }
  __syncthreads();
  // bf16 h^{l+1}: gathered by the next layer, read by the heads after the last
  *reinterpret_cast<uint4*>(mx_hb(m, l + 1) + (i0 + n) * MP_H + 8 * q) =
      *reinterpret_cast<const uint4*>(xa + n * MX_AS + 8 * q);
  if (l + 1 < MP_NL && m.store_train)
    mx_store_py(m.w16, base + MP_L_SIZE + MP_L_P, xa, MX_AS,
                m.y + (int64_t)(l + 1) * rows * MP_H, i0);
}

// heads (bf16 activations): M^-1 values, four lanes per CSR entry.  After
// the tile's h and a table of every entry's row are staged, every quad walks
// its entries on its own (the owning row read from the table: a binary
// search of the row pointers per entry took 816 against 787 us at N = 8e6),
// the next entry's column index read one entry ahead.
__global__ __launch_bounds__(MP_THREADS) void k_mp_heads_mx(DevPtrs d, MpPtrs m) {
  if (d.ctrl->overflow) return;  // row pointers may exceed the capacity
  __shared__ float hv[MP_H + 1], hz[MP_H], hze[MP_FE + 1];
  __shared__ int rp[MP_ROWS + 1];
  __shared__ double dg[MP_ROWS];
  __shared__ __align__(16) float hi_s[MP_ROWS * MX_FS];
  constexpr int HEADS_EMAX = 4096;          // entries of a tile in the row table
  static_assert(MP_ROWS <= 256, "rows fit the table's bytes");
  __shared__ uint8_t erow[HEADS_EMAX];
  const int t = threadIdx.x;
  const int ntiles = (int)(m.rows / MP_ROWS);
  const int tile = xcd_block(blockIdx.x, ntiles);   // XCD-contiguous tiles
  if (tile >= ntiles) return;
  load_w(m, hv, MP_OFF_HEAD + MP_H_V, MP_H + 1);
  load_w(m, hz, MP_OFF_HEAD + MP_H_Z, MP_H);
  load_w(m, hze, MP_OFF_HEAD + MP_H_ZE, MP_FE + 1);
  const int64_t i0 = (int64_t)tile * MP_ROWS;
  if (t <= MP_ROWS) rp[t] = d.rowptr[i0 + t];
  if (t < MP_ROWS) dg[t] = d.diag[i0 + t];
  const int n = t >> 2, q = t & 3;
  // the final h in bf16 (the heads use it rounded): 8 features per thread
  auto hb8 = [&](int64_t row, float (&v)[8]) {
    const uint4 hq = *reinterpret_cast<const uint4*>(m.hb + row * MP_H + 8 * q);
    const uint32_t wv[4] = {hq.x, hq.y, hq.z, hq.w};
#pragma unroll
    for (int h2 = 0; h2 < 4; ++h2) {
      v[2 * h2] = bf16_value((uint16_t)(wv[h2] & 0xffffu));
      v[2 * h2 + 1] = bf16_value((uint16_t)(wv[h2] >> 16));
    }
  };
  {
    float v[8];
    hb8(i0 + n, v);
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) hi_s[n * MX_FS + 8 * q + kk] = v[kk];
  }
  __syncthreads();
  // the tile row of every entry, written by the row's four threads (a
  // binary search of the row pointers per entry, a chain of six dependent
  // LDS reads, where the tile holds more entries than the table)
  const int E0 = rp[0], E1 = rp[MP_ROWS];
  const bool table = E1 - E0 <= HEADS_EMAX;
  if (table)
    for (int e2 = rp[n] + q; e2 < rp[n + 1]; e2 += 4) erow[e2 - E0] = (uint8_t)n;
  __syncthreads();
  // no barrier below: the four lanes of a quad share every entry, so the
  // quad's shuffles see only active lanes
  int e = E0 + n;
  int jn = e < E1 ? d.col[e] : 0;
  for (; e < E1; e += MX_EC) {
    const int64_t j = jn;
    jn = e + MX_EC < E1 ? d.col[e + MX_EC] : 0;
    float hj[8];
    hb8(j, hj);
    const double dj = d.diag[j];
    const ushort4 eq = *reinterpret_cast<const ushort4*>(m.efh + 4 * (int64_t)e);
    static_assert((MP_ROWS & (MP_ROWS - 1)) == 0, "the row search halves a power of two");
    int r = 0;   // the last row whose range starts at or before e
    if (table) {
      r = erow[e - E0];
    } else {
#pragma unroll
      for (int half = MP_ROWS / 2; half > 0; half >>= 1)
        if (rp[r + half] <= e) r += half;
    }
    float p = 0.0f;
#pragma unroll
    for (int kk = 0; kk < 8; ++kk) {
      const int k = 8 * q + kk;
      p += hz[k] * (hi_s[r * MX_FS + k] * hj[kk]);
    }
    p += __shfl_xor(p, 1, 64);
    p += __shfl_xor(p, 2, 64);
    float tt = p;
    const float ef[MP_FE] = {bf16_value(eq.x), bf16_value(eq.y), bf16_value(eq.z)};
#pragma unroll
    for (int f = 0; f < MP_FE; ++f) tt += hze[f] * ef[f];
    tt += hze[MP_FE];
    if (q == 0) {
      m.moff[e] = (float)((double)tt / sqrt(dg[r] * dj));
      if (m.store_train) m.tg[e] = tt;
    }
  }
  float p = 0.0f;
#pragma unroll
  for (int kk = 0; kk < 8; ++kk) p += hv[8 * q + kk] * hi_s[n * MX_FS + 8 * q + kk];
  p += __shfl_xor(p, 1, 64);
  p += __shfl_xor(p, 2, 64);
  if (q == 0) {
    const int64_t i = i0 + n;
    const float tau = p + hv[MP_H];
    m.tau[i] = tau;
    m.mdiag[i] = ((double)softplusf_(tau) + m.lam_floor) / d.diag[i];
  }
}

// ---------------------------------------------------------------------------
// loss: zb = M^-1 b - x*, G = 2 W zb, partials (zb.W zb, x*.W x*), W = A or I
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_mp_resid(DevPtrs d, MpPtrs m) {
  if (d.ctrl->overflow) return;  // row pointers may exceed the capacity
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.rows) return;
  const double md = m.mdiag[i];
  double z[3] = {md * d.b[3 * i], md * d.b[3 * i + 1], md * d.b[3 * i + 2]};
  for (int e = d.rowptr[i]; e < d.rowptr[i + 1]; ++e) {
    const int64_t j = d.col[e];
    const double mv = m.moff[e];
#pragma unroll
    for (int c = 0; c < 3; ++c) z[c] += mv * d.b[3 * j + c];
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) m.zb[3 * i + c] = z[c] - d.x[3 * i + c];
}

__global__ __launch_bounds__(256) void k_mp_aprod(DevPtrs d, MpPtrs m) {
  if (d.ctrl->overflow) return;  // row pointers may exceed the capacity
  __shared__ double lds[4][2];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double num = 0.0, den = 0.0;
  if (i < d.rows) {
    const double dg = d.diag[i];
    double az[3], ax[3];
    if (m.loss_euclid) {  // the identity in place of A
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        az[c] = m.zb[3 * i + c];
        ax[c] = d.x[3 * i + c];
      }
    } else {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        az[c] = dg * m.zb[3 * i + c];
        ax[c] = dg * d.x[3 * i + c];
      }
      for (int e = d.rowptr[i]; e < d.rowptr[i + 1]; ++e) {
        const int64_t j = d.col[e];
        const double a = d.val[e];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          az[c] += a * m.zb[3 * j + c];
          ax[c] += a * d.x[3 * j + c];
        }
      }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      m.G[3 * i + c] = 2.0 * az[c];
      num += m.zb[3 * i + c] * az[c];
      den += d.x[3 * i + c] * ax[c];
    }
  }
  num = wave_sum(num);
  den = wave_sum(den);
  if ((threadIdx.x & 63) == 0) {
    lds[threadIdx.x >> 6][0] = num;
    lds[threadIdx.x >> 6][1] = den;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    double s = 0.0;
    for (int w = 0; w < 4; ++w) s += lds[w][threadIdx.x];
    m.lpart[2 * (int64_t)blockIdx.x + threadIdx.x] = s;
  }
}

// loss = num / den and the gradient scale 1/den (one block, fixed order)
__global__ __launch_bounds__(1024) void k_mp_loss(MpPtrs m, int nblk) {
  __shared__ double lds[16][2];
  double a[2] = {0.0, 0.0};
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) {
    a[0] += m.lpart[2 * (int64_t)b];
    a[1] += m.lpart[2 * (int64_t)b + 1];
  }
  a[0] = wave_sum(a[0]);
  a[1] = wave_sum(a[1]);
  if ((threadIdx.x & 63) == 0) {
    lds[threadIdx.x >> 6][0] = a[0];
    lds[threadIdx.x >> 6][1] = a[1];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    double num = 0.0, den = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
      num += lds[w][0];
      den += lds[w][1];
    }
    m.loss[0] = den > 0.0 ? num / den : 0.0;
    m.loss[1] = den > 0.0 ? 1.0 / den : 0.0;
  }
}

// ---------------------------------------------------------------------------
// backward.  dL/dmdiag_i = sum_c G_ic b_ic, dL/dmoff_ij = sum_c G_ic b_jc
// (unscaled by 1/den: the reduction applies it).  Per-block partial
// gradients go to gpart[block][param] for the block's parameter ranges.
// ---------------------------------------------------------------------------

// reduce an accumulator held by lane k of every node slot into gpart (one
// float per k), fixed order
__device__ __forceinline__ void slot_reduce_store(float v, float* lds, float* dst) {
  const int slot = threadIdx.x / MP_H, k = threadIdx.x % MP_H;
  lds[slot * MP_H + k] = v;
  __syncthreads();
  if (threadIdx.x < MP_H) {
    float s = 0.0f;
    for (int q = 0; q < NODES; ++q) s += lds[q * MP_H + k];
    dst[k] = s;
  }
  __syncthreads();
}

// row-k accumulators acc[0..31] of a 32 x 32 matrix, summed over node slots
__device__ __forceinline__ void slot_reduce_matrix(const float (&acc)[MP_H], float* lds, float* dst) {
  const int slot = threadIdx.x / MP_H, k = threadIdx.x % MP_H;
  for (int q = 0; q < MP_H; ++q) lds[(slot * MP_H + k) * MP_H + q] = acc[q];
  __syncthreads();
  for (int idx = threadIdx.x; idx < MP_H * MP_H; idx += blockDim.x) {
    float s = 0.0f;
    for (int sl = 0; sl < NODES; ++sl) s += lds[sl * MP_H * MP_H + idx];
    dst[idx] = s;
  }
  __syncthreads();
}

// heads: dL/dh^3 (into dh) and the head parameters v, v0, z, ze, z0
__global__ __launch_bounds__(MP_THREADS) void k_mp_heads_bwd(DevPtrs d, MpPtrs m) {
  if (d.ctrl->overflow) return;  // row pointers may exceed the capacity
  __shared__ float hv[MP_H + 1], hz[MP_H], hze[MP_FE + 1];
  __shared__ float red[NODES * MP_H * MP_H];
  load_w(m, hv, MP_OFF_HEAD + MP_H_V, MP_H + 1);
  load_w(m, hz, MP_OFF_HEAD + MP_H_Z, MP_H);
  load_w(m, hze, MP_OFF_HEAD + MP_H_ZE, MP_FE + 1);
  __syncthreads();
  const int slot = threadIdx.x / MP_H, k = threadIdx.x % MP_H;
  const float* __restrict__ hf = m.h + (int64_t)MP_NL * m.rows * MP_H;
  float g_v = 0.0f, g_v0 = 0.0f, g_z = 0.0f, g_z0 = 0.0f, g_ze[MP_FE] = {0.0f, 0.0f, 0.0f};
  for (int pass = 0; pass < PASSES; ++pass) {
    const int64_t i = (int64_t)blockIdx.x * MP_ROWS + pass * NODES + slot;
    const double di = d.diag[i];
    double gd = 0.0;
#pragma unroll
    for (int c = 0; c < 3; ++c) gd += m.G[3 * i + c] * d.b[3 * i + c];
    const double gl = gd / di;  // dL/dlam_i (mdiag = lam / D)
    const float tau = m.tau[i];
    const float gt = (float)gl * sigmoidf_(tau);
    const float hk = act_in(m, hf[i * MP_H + k]);
    float dh = gt * hv[k];
    g_v += gt * hk;
    if (k == 0) g_v0 += gt;
    for (int e = d.rowptr[i]; e < d.rowptr[i + 1]; ++e) {
      const int64_t j = d.col[e];
      const double sq = sqrt(di * d.diag[j]);
      double gm = 0.0, gmr = 0.0;
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        gm += m.G[3 * i + c] * d.b[3 * j + c];    // this entry (i -> j)
        gmr += m.G[3 * j + c] * d.b[3 * i + c];   // the reverse entry (j -> i)
      }
      // moff = S / sqrt(D_i D_j): dL/dS of this entry and of its reverse
      const float dt_own = (float)(gm / sq);
      const float dt_rev = (float)(gmr / sq);
      const float hj = act_in(m, hf[j * MP_H + k]);
      dh += (dt_own + dt_rev) * hz[k] * hj;
      g_z += dt_own * (hk * hj);
      if (k == 0) {
        g_z0 += dt_own;
#pragma unroll
        for (int f = 0; f < MP_FE; ++f) g_ze[f] += dt_own * act_in(m, m.ef[3 * (int64_t)e + f]);
      }
    }
    m.dh[i * MP_H + k] = dh;
  }
  float* dst = m.gpart + (int64_t)blockIdx.x * MP_NPARAMS_ALL + MP_OFF_HEAD;
  slot_reduce_store(g_v, red, dst + MP_H_V);
  slot_reduce_store(g_z, red, dst + MP_H_Z);
  // scalar terms live in lane 0 of each slot
  float sc[2 + MP_FE] = {g_v0, g_z0, g_ze[0], g_ze[1], g_ze[2]};
  for (int q = 0; q < 2 + MP_FE; ++q) {
    red[threadIdx.x] = sc[q];
    __syncthreads();
    if (threadIdx.x == 0) {
      float s = 0.0f;
      for (int sl = 0; sl < NODES; ++sl) s += red[sl * MP_H];
      const int off = q == 0 ? MP_H_V0 : (q == 1 ? MP_H_Z0 : MP_H_ZE + (q - 2));
      dst[off] = s;
    }
    __syncthreads();
  }
}

// layer l backward, part A (per node i): da = dh * [a > 0];
// dU, dV, dd; dh_in = dh + U^T da; dm = V^T da
__global__ __launch_bounds__(MP_THREADS) void k_mp_layer_bwd_a(DevPtrs d, MpPtrs m, int l) {
  __shared__ float U[MP_H * MP_H], V[MP_H * MP_H];
  __shared__ float sda[NODES][MP_H];
  __shared__ float red[NODES * MP_H * MP_H];
  const int base = MP_OFF_L0 + l * MP_L_SIZE;
  load_w(m, U, base + MP_L_U, MP_H * MP_H);
  load_w(m, V, base + MP_L_V, MP_H * MP_H);
  __syncthreads();
  const int slot = threadIdx.x / MP_H, k = threadIdx.x % MP_H;
  const float* __restrict__ hin = m.h + (int64_t)l * m.rows * MP_H;
  const float* __restrict__ mm = m.m + (int64_t)l * m.rows * MP_H;
  const float* __restrict__ aa = m.a + (int64_t)l * m.rows * MP_H;
  float accU[MP_H], accV[MP_H], accd = 0.0f;
#pragma unroll
  for (int q = 0; q < MP_H; ++q) accU[q] = accV[q] = 0.0f;
  for (int pass = 0; pass < PASSES; ++pass) {
    const int64_t i = (int64_t)blockIdx.x * MP_ROWS + pass * NODES + slot;
    const float dh = m.dh[i * MP_H + k];
    const float da = aa[i * MP_H + k] > 0.0f ? dh : 0.0f;
    accd += da;
    for (int q = 0; q < MP_H; ++q) {
      accU[q] += da * act_in(m, hin[i * MP_H + q]);
      accV[q] += da * act_in(m, mm[i * MP_H + q]);
    }
    sda[slot][k] = da;
    __syncthreads();
    float su = 0.0f, sv = 0.0f;
#pragma unroll 8
    for (int q = 0; q < MP_H; ++q) {
      su += U[q * MP_H + k] * sda[slot][q];
      sv += V[q * MP_H + k] * sda[slot][q];
    }
    m.dh2[i * MP_H + k] = dh + su;
    m.dm[i * MP_H + k] = sv;
    __syncthreads();
  }
  float* dst = m.gpart + (int64_t)blockIdx.x * MP_NPARAMS_ALL + base;
  slot_reduce_matrix(accU, red, dst + MP_L_U);
  slot_reduce_matrix(accV, red, dst + MP_L_V);
  slot_reduce_store(accd, red, dst + MP_L_D);
}

// layer l backward, part B (per node j, pulling from its neighbours i):
// dy_j = 1/8 sum_i dm_i [y_j + Q e_ij + c > 0]; dQ, dc, dP; dh_in_j += P^T dy_j
__global__ __launch_bounds__(MP_THREADS) void k_mp_layer_bwd_b(DevPtrs d, MpPtrs m, int l) {
  if (d.ctrl->overflow) return;  // row pointers may exceed the capacity
  __shared__ float P[MP_H * MP_H], Q[MP_H * MP_FE], c[MP_H];
  __shared__ float sdy[NODES][MP_H];
  __shared__ float red[NODES * MP_H * MP_H];
  const int base = MP_OFF_L0 + l * MP_L_SIZE;
  load_w(m, P, base + MP_L_P, MP_H * MP_H);
  load_w(m, Q, base + MP_L_Q, MP_H * MP_FE);
  load_w(m, c, base + MP_L_C, MP_H);
  __syncthreads();
  const int slot = threadIdx.x / MP_H, k = threadIdx.x % MP_H;
  const float* __restrict__ hin = m.h + (int64_t)l * m.rows * MP_H;
  const float* __restrict__ y = m.y + (int64_t)l * m.rows * MP_H;
  float accP[MP_H], accQ[MP_FE] = {0.0f, 0.0f, 0.0f}, accc = 0.0f;
#pragma unroll
  for (int q = 0; q < MP_H; ++q) accP[q] = 0.0f;
  for (int pass = 0; pass < PASSES; ++pass) {
    const int64_t j = (int64_t)blockIdx.x * MP_ROWS + pass * NODES + slot;
    const float yj = y[j * MP_H + k];
    float dy = 0.0f;
    for (int e = d.rowptr[j]; e < d.rowptr[j + 1]; ++e) {
      const int64_t i = d.col[e];
      float s = yj + c[k];
      float ef[MP_FE];
#pragma unroll
      for (int f = 0; f < MP_FE; ++f) {
        ef[f] = act_in(m, m.ef[3 * (int64_t)e + f]);
        s += Q[k * MP_FE + f] * ef[f];
      }
      if (s > 0.0f) {
        const float ds = MP_MSG * m.dm[i * MP_H + k];
        dy += ds;
        accc += ds;
#pragma unroll
        for (int f = 0; f < MP_FE; ++f) accQ[f] += ds * ef[f];
      }
    }
    for (int q = 0; q < MP_H; ++q) accP[q] += dy * act_in(m, hin[j * MP_H + q]);
    sdy[slot][k] = dy;
    __syncthreads();
    float sp = 0.0f;
#pragma unroll 8
    for (int q = 0; q < MP_H; ++q) sp += P[q * MP_H + k] * sdy[slot][q];
    m.dh[j * MP_H + k] = m.dh2[j * MP_H + k] + sp;  // dL/dh^l for the next part A
    __syncthreads();
  }
  float* dst = m.gpart + (int64_t)blockIdx.x * MP_NPARAMS_ALL + base;
  slot_reduce_matrix(accP, red, dst + MP_L_P);
  slot_reduce_store(accc, red, dst + MP_L_C);
  for (int f = 0; f < MP_FE; ++f) {
    red[threadIdx.x] = accQ[f];
    __syncthreads();
    if (threadIdx.x < MP_H) {
      float s = 0.0f;
      for (int sl = 0; sl < NODES; ++sl) s += red[sl * MP_H + threadIdx.x];
      dst[MP_L_Q + threadIdx.x * MP_FE + f] = s;
    }
    __syncthreads();
  }
}

// encoder backward: h0 = relu(W0 x + b0)
__global__ __launch_bounds__(MP_THREADS) void k_mp_encode_bwd(DevPtrs d, MpPtrs m) {
  __shared__ float w0[MP_H * MP_FN], b0[MP_H];
  __shared__ float red[NODES * MP_H];
  load_w(m, w0, MP_OFF_W0, MP_H * MP_FN);
  load_w(m, b0, MP_OFF_B0, MP_H);
  __syncthreads();
  const int slot = threadIdx.x / MP_H, k = threadIdx.x % MP_H;
  float gw[MP_FN] = {0.0f, 0.0f, 0.0f}, gb = 0.0f;
  for (int pass = 0; pass < PASSES; ++pass) {
    const int64_t i = (int64_t)blockIdx.x * MP_ROWS + pass * NODES + slot;
    float x[MP_FN];
    float acc = b0[k];
#pragma unroll
    for (int f = 0; f < MP_FN; ++f) {
      x[f] = act_in(m, m.x[3 * i + f]);
      acc += w0[k * MP_FN + f] * x[f];
    }
    if (acc > 0.0f) {
      const float dh = m.dh[i * MP_H + k];
      gb += dh;
#pragma unroll
      for (int f = 0; f < MP_FN; ++f) gw[f] += dh * x[f];
    }
  }
  float* dst = m.gpart + (int64_t)blockIdx.x * MP_NPARAMS_ALL;
  slot_reduce_store(gb, red, dst + MP_OFF_B0);
  for (int f = 0; f < MP_FN; ++f) {
    red[threadIdx.x] = gw[f];
    __syncthreads();
    if (threadIdx.x < MP_H) {
      float s = 0.0f;
      for (int sl = 0; sl < NODES; ++sl) s += red[sl * MP_H + threadIdx.x];
      dst[MP_OFF_W0 + threadIdx.x * MP_FN + f] = s;
    }
    __syncthreads();
  }
}

// grad[p] = (1/den) sum_b gpart[b][p], blocks in order (zero beyond the
// parameters this handle trains)
__global__ __launch_bounds__(256) void k_mp_grad_reduce(MpPtrs m, int nblk) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= MP_NPARAMS_ALL) return;
  if (p >= m.nparams) {
    m.grad[p] = 0.0f;
    return;
  }
  double s = 0.0;
  for (int b = 0; b < nblk; ++b) s += m.gpart[(int64_t)b * MP_NPARAMS_ALL + p];
  m.grad[p] = (float)(s * m.loss[1]);
}

// Adam (Kingma & Ba 2015) on the FP32 master weights, then the bf16 copy
__global__ __launch_bounds__(256) void k_mp_adam(MpPtrs m, float lr, int t) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= m.nparams) return;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float g = m.grad[p];
  const float mo = b1 * m.am[p] + (1.0f - b1) * g;
  const float vo = b2 * m.av[p] + (1.0f - b2) * g * g;
  m.am[p] = mo;
  m.av[p] = vo;
  const float mh = mo / (1.0f - powf(b1, (float)t));
  const float vh = vo / (1.0f - powf(b2, (float)t));
  const float th = m.th32[p] - lr * mh / (sqrtf(vh) + eps);
  m.th32[p] = th;
  m.w16[p] = bf16_bits(th);
}

// bf16 copy of the master weights
__global__ __launch_bounds__(256) void k_mp_cast(MpPtrs m) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < MP_NPARAMS_ALL) m.w16[p] = bf16_bits(m.th32[p]);
}

// parity export of M^-1 in global original numbering (as k_export_system)
__global__ __launch_bounds__(256) void k_mp_export(DevPtrs d, MpPtrs m, const int64_t* __restrict__ id_off,
                                                   int64_t* __restrict__ rows, int64_t* __restrict__ cols,
                                                   double* __restrict__ vals, int64_t cap,
                                                   double* __restrict__ diag_out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.rows) return;
  const int rid = d.blk_rep[i / ROWS_PER_BLOCK];
  const RepDev& R = d.rep[rid];
  if (i - R.row_off >= R.n) return;
  const int64_t gi = id_off[rid] + (int64_t)d.pos[i].w;
  diag_out[gi] = m.mdiag[i];
  for (int e = d.rowptr[i]; e < d.rowptr[i + 1]; ++e) {
    if (e >= cap) break;
    rows[e] = gi;
    cols[e] = id_off[rid] + (int64_t)d.pos[d.col[e]].w;
    vals[e] = (double)m.moff[e];
  }
}

// ---------------------------------------------------------------------------
// white-noise probe of the current system: z ~ N(0, 1) per (row, component)
// from Philox4x64-10 (key (seed, replica stream), counter (index, 3,
// particle id, 0)), then b = A z; the loss kernels see x* = z, b = A z
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_mp_probe_z(DevPtrs d, double* __restrict__ z, uint64_t seed,
                                                    uint64_t index) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.rows) return;
  const RepDev& R = d.rep[d.blk_rep[i / ROWS_PER_BLOCK]];
  double g[3] = {0.0, 0.0, 0.0};
  if (i - R.row_off < R.n) gauss3(seed, R.stream, index, 3, (uint64_t)d.pos[i].w, 0, g);
#pragma unroll
  for (int c = 0; c < 3; ++c) z[3 * i + c] = g[c];
}

__global__ __launch_bounds__(256) void k_mp_probe_b(DevPtrs d, const double* __restrict__ z,
                                                    double* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.rows || d.ctrl->overflow) return;
  const double dg = d.diag[i];
  double acc[3] = {dg * z[3 * i], dg * z[3 * i + 1], dg * z[3 * i + 2]};
  for (int e = d.rowptr[i]; e < d.rowptr[i + 1]; ++e) {
    const int64_t j = d.col[e];
    const double a = d.val[e];
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[c] += a * z[3 * j + c];
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) b[3 * i + c] = acc[c];
}

// ---------------------------------------------------------------------------
// 3 x 3 heads on the anisotropic block system (A_ii = gamma0 I + sum_j W_ij,
// A_ij = -W_ij).  The trunk above runs on the traces d_i = tr A_ii / 3 and
// -omega_ij = -tr W_ij / 3 (written to d.diag and d.val by the block pair
// pass), so its features are rotation invariant (What_ij = omega_ij /
// sqrt(d_i d_j)); the heads give lam_i, S_ij (the scalar heads) and
// mu_i = u.h_i + u0, sig_ij = s.(h_i*h_j) + se.e_ij + s0.  The blocks live in
// the frame where every diagonal block of A is the identity,
// R = blockdiag(A_ii^-1/2) (the block analogue of the scalar D^-1/2):
//   Nh_ij = R_i W_ij R_j,
//   Xh_ii = lam_i I + mu_i (d_i A_ii^-1 - I),
//   Xh_ij = S_ij I + sig_ij (Nh_ij - What_ij I),
//   M^-1 = R Xh R, i.e. with B = A_ii^-1 = R^2:
//   M_ii = lam_i B_i + mu_i (d_i B_i^2 - B_i),
//   M_ij = (S_ij - sig_ij What_ij) R_i R_j + sig_ij B_i W_ij B_j.
// Symmetric (M_ji = M_ij^T), turning with the system, and the scalar
// network's M^-1 times I_3 when every block of A is a multiple of I_3.  The
// blocks of M^-1 are stored (M_ii in FP64, M_ij in FP32, row-major) and the
// block CG applies them as one more block product per iteration.
// ---------------------------------------------------------------------------
namespace {

// 3 x 3 symmetric (xx, xy, xz, yy, yz, zz) times a vector
__device__ __forceinline__ void bsym_mul(const double* a, const double v[3], double out[3]) {
  out[0] = (a[0] * v[0] + a[1] * v[1]) + a[2] * v[2];
  out[1] = (a[1] * v[0] + a[3] * v[1]) + a[4] * v[2];
  out[2] = (a[2] * v[0] + a[4] * v[1]) + a[5] * v[2];
}

// row-major 3 x 3 (FP32) times a vector
__device__ __forceinline__ void bfull_mul(const float* a, const double v[3], double out[3]) {
#pragma unroll
  for (int r = 0; r < 3; ++r)
    out[r] = ((double)a[3 * r] * v[0] + (double)a[3 * r + 1] * v[1]) + (double)a[3 * r + 2] * v[2];
}

// row-major 3 x 3 of a symmetric 6-value block
__device__ __forceinline__ void bsym_full(const double* a, double out[9]) {
  const int map[9] = {0, 1, 2, 1, 3, 4, 2, 4, 5};
#pragma unroll
  for (int q = 0; q < 9; ++q) out[q] = a[map[q]];
}

// out = a b (row-major 3 x 3)
__device__ __forceinline__ void bmul33(const double a[9], const double b[9], double out[9]) {
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c)
      out[3 * r + c] = (a[3 * r] * b[c] + a[3 * r + 1] * b[3 + c]) + a[3 * r + 2] * b[6 + c];
}

// A^-1/2 of a symmetric positive definite 3 x 3 (six values in and out):
// eigenvectors by cyclic Jacobi rotations (each zeroes one off-diagonal
// entry; sweeps until the off-diagonal part is below 1e-34 of the diagonal,
// at most 12), then V diag(w^-1/2) V^T
__device__ void sym3_inv_sqrt(const double* a6, double* out6) {
  double m[3][3], V[3][3];
  const int map[9] = {0, 1, 2, 1, 3, 4, 2, 4, 5};
#pragma unroll
  for (int r = 0; r < 3; ++r)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      m[r][c] = a6[map[3 * r + c]];
      V[r][c] = r == c ? 1.0 : 0.0;
    }
  for (int sweep = 0; sweep < 12; ++sweep) {
    const double off = (m[0][1] * m[0][1] + m[0][2] * m[0][2]) + m[1][2] * m[1][2];
    const double dia = (m[0][0] * m[0][0] + m[1][1] * m[1][1]) + m[2][2] * m[2][2];
    if (off <= 1e-34 * dia) break;
#pragma unroll
    for (int pq = 0; pq < 3; ++pq) {
      const int p = pq == 2 ? 1 : 0, q = pq == 0 ? 1 : 2;
      const double apq = m[p][q];
      if (apq == 0.0) continue;
      const double theta = (m[q][q] - m[p][p]) / (2.0 * apq);
      const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
      const double c = 1.0 / sqrt(t * t + 1.0), s = t * c;
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const double mkp = m[k][p], mkq = m[k][q];
        m[k][p] = c * mkp - s * mkq;
        m[k][q] = s * mkp + c * mkq;
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const double mpk = m[p][k], mqk = m[q][k];
        m[p][k] = c * mpk - s * mqk;
        m[q][k] = s * mpk + c * mqk;
      }
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const double vkp = V[k][p], vkq = V[k][q];
        V[k][p] = c * vkp - s * vkq;
        V[k][q] = s * vkp + c * vkq;
      }
    }
  }
  const double f[3] = {1.0 / sqrt(m[0][0]), 1.0 / sqrt(m[1][1]), 1.0 / sqrt(m[2][2])};
  const int rr[6] = {0, 0, 0, 1, 1, 2}, cc[6] = {0, 1, 2, 1, 2, 2};
#pragma unroll
  for (int q = 0; q < 6; ++q) {
    const int r = rr[q], c = cc[q];
    out6[q] = (V[r][0] * f[0] * V[c][0] + V[r][1] * f[1] * V[c][1]) + V[r][2] * f[2] * V[c][2];
  }
}

// the final hidden state as the heads consume it (bf16 when activations are
// rounded: the rounded copy the last layer wrote)
__device__ __forceinline__ float head_h(const MpPtrs& m, int64_t i, int k) {
  if (m.round_act) return bf16_value(m.hb[i * MP_H + k]);
  return m.h[((int64_t)MP_NL * m.rows + i) * MP_H + k];
}

__device__ __forceinline__ float head_ef(const MpPtrs& m, int64_t e, int f) {
  if (m.round_act) return bf16_value(m.efh[4 * e + f]);
  return m.ef[3 * e + f];
}

}  // namespace

// R_i = A_ii^-1/2 of every row (padding rows: the identity)
__global__ __launch_bounds__(256) void k_mpb_root(DevPtrs d, BlockPtrs bp) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.rows) return;
  sym3_inv_sqrt(bp.bdiag + 6 * i, bp.rsq + 6 * i);
}

// heads: the blocks M_ii and M_ij; one half-wave per node, lane k = hidden
// feature k
__global__ __launch_bounds__(MP_THREADS) void k_mpb_heads(DevPtrs d, MpPtrs m, BlockPtrs bp) {
  if (d.ctrl->overflow) return;  // row pointers may exceed the capacity
  __shared__ float hv[MP_H + 1], hz[MP_H], hze[MP_FE + 1], hu[MP_H + 1], hs[MP_H], hse[MP_FE + 1];
  load_w(m, hv, MP_OFF_HEAD + MP_H_V, MP_H + 1);
  load_w(m, hz, MP_OFF_HEAD + MP_H_Z, MP_H);
  load_w(m, hze, MP_OFF_HEAD + MP_H_ZE, MP_FE + 1);
  load_w(m, hu, MP_OFF_PHI + MP_PHI_U, MP_H + 1);
  load_w(m, hs, MP_OFF_PHI + MP_PHI_S, MP_H);
  load_w(m, hse, MP_OFF_PHI + MP_PHI_SE, MP_FE + 1);
  __syncthreads();
  const int slot = threadIdx.x / MP_H, k = threadIdx.x % MP_H;
  for (int pass = 0; pass < PASSES; ++pass) {
    const int64_t i = (int64_t)blockIdx.x * MP_ROWS + pass * NODES + slot;
    const float hk = head_h(m, i, k);
    const float tau = half_sum(hv[k] * hk) + hv[MP_H];
    const float mu = half_sum(hu[k] * hk) + hu[MP_H];
    const double di = d.diag[i];
    double Ri[9], Bi[9];
    bsym_full(bp.rsq + 6 * i, Ri);
    bsym_full(bp.binv + 6 * i, Bi);
    const int e0 = d.rowptr[i], e1 = d.rowptr[i + 1];
    for (int e = e0; e < e1; ++e) {
      const int64_t j = d.col[e];
      const float hj = head_h(m, j, k);
      float t = half_sum(hz[k] * (hk * hj));
      float sg = half_sum(hs[k] * (hk * hj));
#pragma unroll
      for (int f = 0; f < MP_FE; ++f) {
        const float ef = head_ef(m, e, f);
        t += hze[f] * ef;
        sg += hse[f] * ef;
      }
      t += hze[MP_FE];
      sg += hse[MP_FE];
      if (k == 0) {
        // M_ij = (S - sig What) R_i R_j + sig B_i W B_j, W = -bval
        double Rj[9], Bj[9], W[9], P[9], T[9], Q[9];
        bsym_full(bp.rsq + 6 * j, Rj);
        bsym_full(bp.binv + 6 * j, Bj);
        bsym_full(bp.bval + 6 * (int64_t)e, W);
        bmul33(Ri, Rj, P);
        bmul33(Bi, W, T);
        bmul33(T, Bj, Q);
        const double what = -d.val[e] / sqrt(di * d.diag[j]);
        const double a = (double)t - (double)sg * what, c = -(double)sg;  // -sig: W = -bval
        float* mo = bp.xo + 9 * (int64_t)e;
#pragma unroll
        for (int q = 0; q < 9; ++q) mo[q] = (float)(a * P[q] + c * Q[q]);
      }
    }
    if (k == 0) {
      if (m.store_train) m.tau[i] = tau;
      const double lam = (double)softplusf_(tau) + m.lam_floor;
      // M_ii = lam B + mu (d B^2 - B)
      double B2[9];
      bmul33(Bi, Bi, B2);
      const double* b6 = bp.binv + 6 * i;
      const int full[6] = {0, 1, 2, 4, 5, 8};
      double* md = bp.xd + 6 * i;
#pragma unroll
      for (int q = 0; q < 6; ++q)
        md[q] = lam * b6[q] + (double)mu * (di * B2[full[q]] - b6[q]);
    }
  }
}

// zb = M^-1 b - x*
__global__ __launch_bounds__(256) void k_mpb_resid(DevPtrs d, MpPtrs m, BlockPtrs bp) {
  if (d.ctrl->overflow) return;  // row pointers may exceed the capacity
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.rows) return;
  const double bi[3] = {d.b[3 * i], d.b[3 * i + 1], d.b[3 * i + 2]};
  double acc[3];
  bsym_mul(bp.xd + 6 * i, bi, acc);
  for (int e = d.rowptr[i]; e < d.rowptr[i + 1]; ++e) {
    const int64_t j = d.col[e];
    const double bj[3] = {d.b[3 * j], d.b[3 * j + 1], d.b[3 * j + 2]};
    double o[3];
    bfull_mul(bp.xo + 9 * (int64_t)e, bj, o);
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[c] += o[c];
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) m.zb[3 * i + c] = acc[c] - d.x[3 * i + c];
}

// G = 2 W zb and partials (zb.W zb, x*.W x*), W = A or I
__global__ __launch_bounds__(256) void k_mpb_aprod(DevPtrs d, MpPtrs m, BlockPtrs bp) {
  if (d.ctrl->overflow) return;  // row pointers may exceed the capacity
  __shared__ double lds[4][2];
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double num = 0.0, den = 0.0;
  if (i < d.rows) {
    const double zi[3] = {m.zb[3 * i], m.zb[3 * i + 1], m.zb[3 * i + 2]};
    const double xi[3] = {d.x[3 * i], d.x[3 * i + 1], d.x[3 * i + 2]};
    double az[3], ax[3];
    if (m.loss_euclid) {
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        az[c] = zi[c];
        ax[c] = xi[c];
      }
    } else {
      bsym_mul(bp.bdiag + 6 * i, zi, az);
      bsym_mul(bp.bdiag + 6 * i, xi, ax);
      for (int e = d.rowptr[i]; e < d.rowptr[i + 1]; ++e) {
        const int64_t j = d.col[e];
        const double zj[3] = {m.zb[3 * j], m.zb[3 * j + 1], m.zb[3 * j + 2]};
        const double xj[3] = {d.x[3 * j], d.x[3 * j + 1], d.x[3 * j + 2]};
        double oz[3], ox[3];
        bsym_mul(bp.bval + 6 * (int64_t)e, zj, oz);
        bsym_mul(bp.bval + 6 * (int64_t)e, xj, ox);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
          az[c] += oz[c];
          ax[c] += ox[c];
        }
      }
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      m.G[3 * i + c] = 2.0 * az[c];
      num += zi[c] * az[c];
      den += xi[c] * ax[c];
    }
  }
  num = wave_sum(num);
  den = wave_sum(den);
  if ((threadIdx.x & 63) == 0) {
    lds[threadIdx.x >> 6][0] = num;
    lds[threadIdx.x >> 6][1] = den;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    double s = 0.0;
    for (int w = 0; w < 4; ++w) s += lds[w][threadIdx.x];
    m.lpart[2 * (int64_t)blockIdx.x + threadIdx.x] = s;
  }
}

// the node-local transforms of G and b the heads' backward reads:
// R G, B G, R b, B b
__global__ __launch_bounds__(256) void k_mpb_pre(DevPtrs d, MpPtrs m, BlockPtrs bp) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.rows) return;
  const double g[3] = {m.G[3 * i], m.G[3 * i + 1], m.G[3 * i + 2]};
  const double b[3] = {d.b[3 * i], d.b[3 * i + 1], d.b[3 * i + 2]};
  double o[4][3];
  bsym_mul(bp.rsq + 6 * i, g, o[0]);
  bsym_mul(bp.binv + 6 * i, g, o[1]);
  bsym_mul(bp.rsq + 6 * i, b, o[2]);
  bsym_mul(bp.binv + 6 * i, b, o[3]);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    bp.gt[3 * i + c] = o[0][c];
    bp.gh[3 * i + c] = o[1][c];
    bp.t[3 * i + c] = o[2][c];
    bp.bh[3 * i + c] = o[3][c];
  }
}

// heads backward.  With g = R G, gh = B G, c = R b, ch = B b (bp.gt, gh, t,
// bh), dL/dXh_ij = g_i c_j^T, so
//   dL/dlam_i = g_i.c_i,  dL/dmu_i = d_i gh_i.ch_i - g_i.c_i,
//   dL/dS_ij = g_i.c_j,   dL/dsig_ij = gh_i.W_ij ch_j - What_ij g_i.c_j
// (unscaled by 1/den: the reduction applies it); dL/dh^3 into dh and the head
// parameters v, v0, z, ze, z0, u, u0, s, se, s0
__global__ __launch_bounds__(MP_THREADS) void k_mpb_heads_bwd(DevPtrs d, MpPtrs m, BlockPtrs bp) {
  if (d.ctrl->overflow) return;  // row pointers may exceed the capacity
  __shared__ float hv[MP_H + 1], hz[MP_H], hu[MP_H + 1], hs[MP_H];
  __shared__ float red[NODES * MP_H];
  load_w(m, hv, MP_OFF_HEAD + MP_H_V, MP_H + 1);
  load_w(m, hz, MP_OFF_HEAD + MP_H_Z, MP_H);
  load_w(m, hu, MP_OFF_PHI + MP_PHI_U, MP_H + 1);
  load_w(m, hs, MP_OFF_PHI + MP_PHI_S, MP_H);
  __syncthreads();
  const int slot = threadIdx.x / MP_H, k = threadIdx.x % MP_H;
  const float* __restrict__ hf = m.h + (int64_t)MP_NL * m.rows * MP_H;
  float g_v = 0.0f, g_z = 0.0f, g_u = 0.0f, g_s = 0.0f;
  // scalar terms (lane 0 of each slot): v0, z0, ze[3], u0, s0, se[3]
  float g_sc[10] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
  auto ld3 = [](const double* p, int64_t r, double (&v)[3]) {
    v[0] = p[3 * r];
    v[1] = p[3 * r + 1];
    v[2] = p[3 * r + 2];
  };
  auto dot3 = [](const double (&a)[3], const double (&b)[3]) {
    return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2];
  };
  for (int pass = 0; pass < PASSES; ++pass) {
    const int64_t i = (int64_t)blockIdx.x * MP_ROWS + pass * NODES + slot;
    const double di = d.diag[i];
    double gi[3], ghi[3], ci[3], chi[3];
    ld3(bp.gt, i, gi);
    ld3(bp.gh, i, ghi);
    ld3(bp.t, i, ci);
    ld3(bp.bh, i, chi);
    const double gc = dot3(gi, ci);
    const double dl = gc, dmu = di * dot3(ghi, chi) - gc;
    const float tau = m.tau[i];
    const float gt = (float)dl * sigmoidf_(tau);
    const float gm = (float)dmu;
    const float hk = act_in(m, hf[i * MP_H + k]);
    float dh = gt * hv[k] + gm * hu[k];
    g_v += gt * hk;
    g_u += gm * hk;
    if (k == 0) {
      g_sc[0] += gt;
      g_sc[5] += gm;
    }
    for (int e = d.rowptr[i]; e < d.rowptr[i + 1]; ++e) {
      const int64_t j = d.col[e];
      double gj[3], ghj[3], cj[3], chj[3];
      ld3(bp.gt, j, gj);
      ld3(bp.gh, j, ghj);
      ld3(bp.t, j, cj);
      ld3(bp.bh, j, chj);
      const double* bv = bp.bval + 6 * (int64_t)e;  // -W
      double wcj[3], wci[3];
      bsym_mul(bv, chj, wcj);
      bsym_mul(bv, chi, wci);
      const double what = -d.val[e] / sqrt(di * d.diag[j]);
      const double s_own = dot3(gi, cj), s_rev = dot3(gj, ci);
      const double q_own = -dot3(ghi, wcj) - what * s_own;
      const double q_rev = -dot3(ghj, wci) - what * s_rev;
      const float dS_own = (float)s_own, dS_rev = (float)s_rev;
      const float dq_own = (float)q_own, dq_rev = (float)q_rev;
      const float hj = act_in(m, hf[j * MP_H + k]);
      dh += ((dS_own + dS_rev) * hz[k] + (dq_own + dq_rev) * hs[k]) * hj;
      g_z += dS_own * (hk * hj);
      g_s += dq_own * (hk * hj);
      if (k == 0) {
        g_sc[1] += dS_own;
        g_sc[6] += dq_own;
#pragma unroll
        for (int f = 0; f < MP_FE; ++f) {
          const float ef = act_in(m, m.ef[3 * (int64_t)e + f]);
          g_sc[2 + f] += dS_own * ef;
          g_sc[7 + f] += dq_own * ef;
        }
      }
    }
    m.dh[i * MP_H + k] = dh;
  }
  float* dst = m.gpart + (int64_t)blockIdx.x * MP_NPARAMS_ALL;
  slot_reduce_store(g_v, red, dst + MP_OFF_HEAD + MP_H_V);
  slot_reduce_store(g_z, red, dst + MP_OFF_HEAD + MP_H_Z);
  slot_reduce_store(g_u, red, dst + MP_OFF_PHI + MP_PHI_U);
  slot_reduce_store(g_s, red, dst + MP_OFF_PHI + MP_PHI_S);
  const int offs[10] = {MP_OFF_HEAD + MP_H_V0, MP_OFF_HEAD + MP_H_Z0, MP_OFF_HEAD + MP_H_ZE,
                        MP_OFF_HEAD + MP_H_ZE + 1, MP_OFF_HEAD + MP_H_ZE + 2,
                        MP_OFF_PHI + MP_PHI_U0, MP_OFF_PHI + MP_PHI_S0, MP_OFF_PHI + MP_PHI_SE,
                        MP_OFF_PHI + MP_PHI_SE + 1, MP_OFF_PHI + MP_PHI_SE + 2};
  for (int q = 0; q < 10; ++q) {
    red[threadIdx.x] = g_sc[q];
    __syncthreads();
    if (threadIdx.x == 0) {
      float s = 0.0f;
      for (int sl = 0; sl < NODES; ++sl) s += red[sl * MP_H];
      dst[offs[q]] = s;
    }
    __syncthreads();
  }
}

// b = A z on the block system (the probe's right-hand side)
__global__ __launch_bounds__(256) void k_mpb_probe_b(DevPtrs d, BlockPtrs bp,
                                                     const double* __restrict__ z,
                                                     double* __restrict__ b) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.rows || d.ctrl->overflow) return;
  const double zi[3] = {z[3 * i], z[3 * i + 1], z[3 * i + 2]};
  double acc[3];
  bsym_mul(bp.bdiag + 6 * i, zi, acc);
  for (int e = d.rowptr[i]; e < d.rowptr[i + 1]; ++e) {
    const int64_t j = d.col[e];
    const double zj[3] = {z[3 * j], z[3 * j + 1], z[3 * j + 2]};
    double o[3];
    bsym_mul(bp.bval + 6 * (int64_t)e, zj, o);
#pragma unroll
    for (int c = 0; c < 3; ++c) acc[c] += o[c];
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) b[3 * i + c] = acc[c];
}

// parity export: the blocks M_ii and M_ij, row-major 3 x 3, in global
// original numbering (as k_block_export)
__global__ __launch_bounds__(256) void k_mpb_export(DevPtrs d, BlockPtrs bp,
                                                    const int64_t* __restrict__ id_off,
                                                    int64_t* __restrict__ rows,
                                                    int64_t* __restrict__ cols,
                                                    double* __restrict__ vals, int64_t cap,
                                                    double* __restrict__ diag_out) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= d.rows) return;
  const int rid = d.blk_rep[i / ROWS_PER_BLOCK];
  const RepDev& R = d.rep[rid];
  if (i - R.row_off >= R.n) return;
  const int64_t gi = id_off[rid] + (int64_t)d.pos[i].w;
  double M[9];
  bsym_full(bp.xd + 6 * i, M);
#pragma unroll
  for (int q = 0; q < 9; ++q) diag_out[9 * gi + q] = M[q];
  for (int e = d.rowptr[i]; e < d.rowptr[i + 1]; ++e) {
    if (e >= cap) break;
    rows[e] = gi;
    cols[e] = id_off[rid] + (int64_t)d.pos[d.col[e]].w;
#pragma unroll
    for (int q = 0; q < 9; ++q) vals[9 * (int64_t)e + q] = (double)bp.xo[9 * (int64_t)e + q];
  }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
static inline unsigned nb(int64_t n, int t) { return (unsigned)((n + t - 1) / t); }

hipError_t launch_mp_trunk(const DevPtrs& d, const MpPtrs& m, hipStream_t s) {
  const unsigned blocks = (unsigned)(d.rows / MP_ROWS);
  if (m.round_act) {
    const dim3 g((unsigned)xcd_grid((int)blocks));
    hipLaunchKernelGGL(k_mp_encode_mx, g, dim3(MP_THREADS), 0, s, d, m);
    for (int l = 0; l < MP_NL; ++l)
      hipLaunchKernelGGL(k_mp_layer_mx, g, dim3(MP_THREADS), 0, s, d, m, l);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(k_mp_features, dim3(nb(d.rows, 256)), dim3(256), 0, s, d, m);
  hipLaunchKernelGGL(k_mp_encode, dim3(blocks), dim3(MP_THREADS), 0, s, d, m);
  for (int l = 0; l < MP_NL; ++l)
    hipLaunchKernelGGL(k_mp_layer, dim3(blocks), dim3(MP_THREADS), 0, s, d, m, l);
  return hipGetLastError();
}

hipError_t launch_mp_forward(const DevPtrs& d, const MpPtrs& m, hipStream_t s) {
  hipError_t e = launch_mp_trunk(d, m, s);
  if (e != hipSuccess) return e;
  const unsigned blocks = (unsigned)(d.rows / MP_ROWS);
  if (m.round_act)
    hipLaunchKernelGGL(k_mp_heads_mx, dim3((unsigned)xcd_grid((int)blocks)), dim3(MP_THREADS), 0,
                       s, d, m);
  else
    hipLaunchKernelGGL(k_mp_heads, dim3(blocks), dim3(MP_THREADS), 0, s, d, m);
  return hipGetLastError();
}

hipError_t launch_mp_loss(const DevPtrs& d, const MpPtrs& m, hipStream_t s) {
  const unsigned b = nb(d.rows, 256);
  hipLaunchKernelGGL(k_mp_resid, dim3(b), dim3(256), 0, s, d, m);
  hipLaunchKernelGGL(k_mp_aprod, dim3(b), dim3(256), 0, s, d, m);
  hipLaunchKernelGGL(k_mp_loss, dim3(1), dim3(1024), 0, s, m, (int)b);
  return hipGetLastError();
}

// the layers' and the encoder's backward from dL/dh^NL in m.dh, then the
// parameter gradient
static hipError_t launch_mp_trunk_backward(const DevPtrs& d, const MpPtrs& m, hipStream_t s) {
  const unsigned blocks = (unsigned)(d.rows / MP_ROWS);
  for (int l = MP_NL - 1; l >= 0; --l) {
    hipLaunchKernelGGL(k_mp_layer_bwd_a, dim3(blocks), dim3(MP_THREADS), 0, s, d, m, l);
    hipLaunchKernelGGL(k_mp_layer_bwd_b, dim3(blocks), dim3(MP_THREADS), 0, s, d, m, l);
  }
  hipLaunchKernelGGL(k_mp_encode_bwd, dim3(blocks), dim3(MP_THREADS), 0, s, d, m);
  hipLaunchKernelGGL(k_mp_grad_reduce, dim3(nb(MP_NPARAMS_ALL, 256)), dim3(256), 0, s, m,
                     (int)blocks);
  return hipGetLastError();
}

hipError_t launch_mp_backward(const DevPtrs& d, const MpPtrs& m, hipStream_t s) {
  const unsigned blocks = (unsigned)(d.rows / MP_ROWS);
  hipLaunchKernelGGL(k_mp_heads_bwd, dim3(blocks), dim3(MP_THREADS), 0, s, d, m);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_mp_trunk_backward(d, m, s);
}

hipError_t launch_mp_adam(const MpPtrs& m, float lr, int t, hipStream_t s) {
  hipLaunchKernelGGL(k_mp_adam, dim3(nb(MP_NPARAMS_ALL, 256)), dim3(256), 0, s, m, lr, t);
  return hipGetLastError();
}

hipError_t launch_mp_export(const DevPtrs& d, const MpPtrs& m, const int64_t* id_off, int64_t* rows,
                            int64_t* cols, double* vals, int64_t cap, double* diag, hipStream_t s) {
  hipLaunchKernelGGL(k_mp_export, dim3(nb(d.rows, 256)), dim3(256), 0, s, d, m, id_off, rows, cols,
                     vals, cap, diag);
  return hipGetLastError();
}

hipError_t launch_mp_probe(const DevPtrs& d, double* z, double* b, uint64_t seed, uint64_t index,
                           hipStream_t s) {
  hipLaunchKernelGGL(k_mp_probe_z, dim3(nb(d.rows, 256)), dim3(256), 0, s, d, z, seed, index);
  hipLaunchKernelGGL(k_mp_probe_b, dim3(nb(d.rows, 256)), dim3(256), 0, s, d, z, b);
  return hipGetLastError();
}

hipError_t launch_mp_cast(const MpPtrs& m, hipStream_t s) {
  hipLaunchKernelGGL(k_mp_cast, dim3(nb(MP_NPARAMS_ALL, 256)), dim3(256), 0, s, m);
  return hipGetLastError();
}

// ---- the 3 x 3 heads on the block system --------------------------------
hipError_t launch_mpb_heads(const DevPtrs& d, const MpPtrs& m, const BlockPtrs& bp, hipStream_t s) {
  hipLaunchKernelGGL(k_mpb_root, dim3(nb(d.rows, 256)), dim3(256), 0, s, d, bp);
  hipLaunchKernelGGL(k_mpb_heads, dim3((unsigned)(d.rows / MP_ROWS)), dim3(MP_THREADS), 0, s, d, m,
                     bp);
  return hipGetLastError();
}

hipError_t launch_mpb_loss(const DevPtrs& d, const MpPtrs& m, const BlockPtrs& bp, hipStream_t s) {
  const unsigned b = nb(d.rows, 256);
  hipLaunchKernelGGL(k_mpb_resid, dim3(b), dim3(256), 0, s, d, m, bp);
  hipLaunchKernelGGL(k_mpb_aprod, dim3(b), dim3(256), 0, s, d, m, bp);
  hipLaunchKernelGGL(k_mp_loss, dim3(1), dim3(1024), 0, s, m, (int)b);
  return hipGetLastError();
}

hipError_t launch_mpb_backward(const DevPtrs& d, const MpPtrs& m, const BlockPtrs& bp,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_mpb_pre, dim3(nb(d.rows, 256)), dim3(256), 0, s, d, m, bp);
  hipLaunchKernelGGL(k_mpb_heads_bwd, dim3((unsigned)(d.rows / MP_ROWS)), dim3(MP_THREADS), 0, s,
                     d, m, bp);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_mp_trunk_backward(d, m, s);
}

hipError_t launch_mpb_probe(const DevPtrs& d, const BlockPtrs& bp, double* z, double* b,
                            uint64_t seed, uint64_t index, hipStream_t s) {
  hipLaunchKernelGGL(k_mp_probe_z, dim3(nb(d.rows, 256)), dim3(256), 0, s, d, z, seed, index);
  hipLaunchKernelGGL(k_mpb_probe_b, dim3(nb(d.rows, 256)), dim3(256), 0, s, d, bp, z, b);
  return hipGetLastError();
}

hipError_t launch_mpb_export(const DevPtrs& d, const BlockPtrs& bp, const int64_t* id_off,
                             int64_t* rows, int64_t* cols, double* vals, int64_t cap, double* diag,
                             hipStream_t s) {
  hipLaunchKernelGGL(k_mpb_export, dim3(nb(d.rows, 256)), dim3(256), 0, s, d, bp, id_off, rows,
                     cols, vals, cap, diag);
  return hipGetLastError();
}
