// mpnn.h -- parameter layout and device pointers of the learned
// preconditioner (internal; the layout is also stated in include/sim.h).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define MP_H 32        // hidden features
#define MP_FN 3        // node input features
#define MP_FE 3        // edge input features
#define MP_NL 3        // message-passing layers
#define MP_THREADS 256 // threads per block (8 nodes x 32 features)
#define MP_ROWS 64     // rows per block
#define MP_MSG 0.125f  // message scale
#define MP_EPS_LAM 0.3 // default floor of the diagonal head lam

#define MP_OFF_W0 0
#define MP_OFF_B0 (MP_OFF_W0 + MP_H * MP_FN)
#define MP_OFF_L0 (MP_OFF_B0 + MP_H)
#define MP_L_P 0
#define MP_L_Q (MP_L_P + MP_H * MP_H)
#define MP_L_C (MP_L_Q + MP_H * MP_FE)
#define MP_L_U (MP_L_C + MP_H)
#define MP_L_V (MP_L_U + MP_H * MP_H)
#define MP_L_D (MP_L_V + MP_H * MP_H)
#define MP_L_SIZE (MP_L_D + MP_H)
#define MP_OFF_HEAD (MP_OFF_L0 + MP_NL * MP_L_SIZE)
#define MP_H_V 0
#define MP_H_V0 (MP_H_V + MP_H)
#define MP_H_Z (MP_H_V0 + 1)
#define MP_H_ZE (MP_H_Z + MP_H)
#define MP_H_Z0 (MP_H_ZE + MP_FE)
#define MP_NPARAMS (MP_OFF_HEAD + MP_H_Z0 + 1)
// the 3 x 3 heads on the anisotropic block system (after the scalar network):
// mu_i = u.h_i + u0, sig_ij = s.(h_i*h_j) + se.e_ij + s0
#define MP_OFF_PHI MP_NPARAMS
#define MP_PHI_U 0
#define MP_PHI_U0 (MP_PHI_U + MP_H)
#define MP_PHI_S (MP_PHI_U0 + 1)
#define MP_PHI_SE (MP_PHI_S + MP_H)
#define MP_PHI_S0 (MP_PHI_SE + MP_FE)
#define MP_NPHI (MP_PHI_S0 + 1)
#define MP_NPARAMS_ALL (MP_NPARAMS + MP_NPHI)

struct MpPtrs {
  uint16_t* w16;   // bf16 weights used by the kernels
  float* th32;     // FP32 master weights
  float* am;       // Adam first moment
  float* av;       // Adam second moment
  float* grad;     // gradient of the last training step
  float* gpart;    // [blocks][MP_NPARAMS_ALL] partial gradients
  float* x;        // [rows][3] node features
  float* ef;       // [nnz][3] edge features
  float* er;       // [nnz] r_ij / rc (written by the pair-terms kernel)
  float* h;        // [NL+1][rows][H]
  float* y;        // [NL][rows][H]
  float* m;        // [NL][rows][H] (training)
  float* a;        // [NL][rows][H] (training)
  float* tau;      // [rows] node-head pre-activation
  float* tg;       // [nnz] edge-head pre-activation
  float* moff;     // [nnz] M^-1 off-diagonal
  double* mdiag;   // [rows] M^-1 diagonal
  double* zb;      // [rows][3] M^-1 b - x*
  double* G;       // [rows][3] 2 A zb
  double* lpart;   // loss partials
  double* loss;    // [2]: loss, 1 / ||x*||_A^2
  double* pz;      // [rows][3] probe vector z (training on probes)
  double* pb;      // [rows][3] A z
  float* dh;       // [rows][H]
  float* dh2;      // [rows][H]
  float* dm;       // [rows][H]
  uint16_t* hb;    // [rows][H] bfloat16 of h^l for l = NL, NL-2, ... (the heads and
                   // the layers round h to bf16 before every product anyway)
  uint16_t* hb2;   // [rows][H] bfloat16 of h^l for l = NL-1, NL-3, ...
  uint16_t* efh;   // [nnz][4] bfloat16 edge features and a zero (likewise)
  int64_t rows;
  int round_act;   // 1: round activations entering products to bf16
  int store_train; // 1: keep m and a for the backward pass
  int loss_euclid; // loss norm: 0 the A-norm, 1 the Euclidean norm
  int nparams;     // parameters trained: MP_NPARAMS (scalar) or MP_NPARAMS_ALL (blocks)
  double lam_floor; // floor added to the diagonal head: lam = softplus(.) + lam_floor
};
static_assert(sizeof(MpPtrs) % 8 == 0, "MpPtrs must have no implicit tail padding");
