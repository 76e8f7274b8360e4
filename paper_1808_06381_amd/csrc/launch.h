// launch.h -- host launchers of the kernels in kernels.hip (internal).
#pragma once
#include <hip/hip_runtime.h>
#include "sim_dev.h"

hipError_t launch_fill_i32(int32_t* p, int32_t v, int64_t n, hipStream_t s);
// exclusive scan of int32; too_many (optional, device) is set to 1 when the
// total passes INT32_MAX (the int32 outputs are then not valid)
hipError_t launch_scan(const int32_t* in, int32_t* out, int64_t m, int32_t* bsum, hipStream_t s,
                       int32_t* too_many = nullptr);
int64_t scan_bsum_len(int64_t m);
hipError_t launch_bin(const DevPtrs& d, hipStream_t s);
hipError_t launch_cell_rows(const DevPtrs& d, const int32_t* scan, hipStream_t s);
hipError_t launch_scatter(const DevPtrs& d, hipStream_t s);
hipError_t launch_cell_sort(const DevPtrs& d, hipStream_t s);
hipError_t launch_ctrl_zero(const DevPtrs& d, hipStream_t s);
// the count pass keeps the first NBR_SLOTS neighbours of every row in
// slots[NBR_SLOTS][rows] (slot-major) for the list pass
#define NBR_SLOTS 16
hipError_t launch_nbr_count(const DevPtrs& d, int32_t* slots, hipStream_t s);
hipError_t launch_nbr_list(const DevPtrs& d, const int32_t* slots, hipStream_t s);
hipError_t launch_pair_terms(const DevPtrs& d, hipStream_t s);
hipError_t launch_update(const DevPtrs& d, int cond, hipStream_t s);
hipError_t launch_save_vel(const DevPtrs& d, const int64_t* id_off, int cond, hipStream_t s);
hipError_t launch_step_commit(const DevPtrs& d, int cond, hipStream_t s);
hipError_t launch_permute(const DevPtrs& d, const int64_t* id_off, int mode, const double* in,
                          double* out, hipStream_t s);
hipError_t launch_export_pairs(const DevPtrs& d, int64_t* out, int64_t cap,
                               unsigned long long* cnt, hipStream_t s);
hipError_t launch_export_system(const DevPtrs& d, const int64_t* id_off, int64_t* rows,
                                int64_t* cols, double* vals, int64_t cap, double* diag,
                                double* rhs, hipStream_t s);
hipError_t launch_copy16(const void* src, void* dst, int64_t bytes, hipStream_t s,
                         hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
hipError_t launch_cg_reset(const DevPtrs& d, double tol_override, hipStream_t s);
hipError_t launch_cg_vec(const DevPtrs& d, int mode, hipStream_t s, hipEvent_t ev0 = nullptr,
                         hipEvent_t ev1 = nullptr);
hipError_t launch_cg_spmv(const DevPtrs& d, int mode, int start_mode, hipStream_t s,
                          hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);
hipError_t launch_cg_finish(const DevPtrs& d, int mode, hipStream_t s);
hipError_t launch_cg_flush(const DevPtrs& d, hipStream_t s);
hipError_t launch_cg_warm(const DevPtrs& d, const int64_t* id_off, hipStream_t s);
hipError_t launch_cg_apply(const DevPtrs& d, int mode, hipStream_t s, hipEvent_t ev0 = nullptr,
                           hipEvent_t ev1 = nullptr);
hipError_t launch_cg_dot_ru(const DevPtrs& d, int mode, hipStream_t s);
hipError_t launch_ic_factor(const DevPtrs& d, const int32_t* color_off, int ncolors, hipStream_t s);
hipError_t launch_ic_apply(const DevPtrs& d, const int32_t* color_off, int ncolors, hipStream_t s);
hipError_t launch_ic_export(const DevPtrs& d, const int64_t* id_off, int64_t* rows, int64_t* cols,
                            double* vals, double* diag, hipStream_t s);
struct MpPtrs;
hipError_t launch_mp_forward(const DevPtrs& d, const MpPtrs& m, hipStream_t s);
hipError_t launch_mp_loss(const DevPtrs& d, const MpPtrs& m, hipStream_t s);
hipError_t launch_mp_backward(const DevPtrs& d, const MpPtrs& m, hipStream_t s);
hipError_t launch_mp_adam(const MpPtrs& m, float lr, int t, hipStream_t s);
hipError_t launch_mp_cast(const MpPtrs& m, hipStream_t s);
hipError_t launch_mp_probe(const DevPtrs& d, double* z, double* b, uint64_t seed, uint64_t index,
                           hipStream_t s);
hipError_t launch_mp_export(const DevPtrs& d, const MpPtrs& m, const int64_t* id_off, int64_t* rows,
                            int64_t* cols, double* vals, int64_t cap, double* diag, hipStream_t s);

// structure factor (sq.hip)
#include <vector>
int64_t sq_chunk_count(const std::vector<int64_t>& rep_rows);
int64_t sq_tile_count(int nx, int my_max);
size_t sq_chunk_bytes();
size_t sq_partial_bytes(int64_t nchunk, int nx, int my_max);
size_t sq_scratch_bytes(int64_t nchunk, int nrep, int nx, int my_max);
hipError_t launch_sq_scratch(const DevPtrs& d, int64_t nchunk, int nx, int my_max, int mz,
                             void* scratch, double* out_d, hipStream_t s);
hipError_t launch_sq(const DevPtrs& d, const std::vector<int64_t>& rep_row0,
                     const std::vector<int64_t>& rep_rows, int nx, int my_max, int mz,
                     void* chunks_d, int32_t* rep_chunk0_d, double2* partial_d, double* out_d,
                     hipStream_t s, hipEvent_t ev0 = nullptr, hipEvent_t ev1 = nullptr);

// velocity cross-correlation (vv.hip)
struct VvRep {          // coarse cell grid of one replica
  double len[3];        // cell edge per axis (>= r_max / M, or the whole axis)
  double inv_len[3];
  double margin;        // slack of the distance culling (rounding of cell indices)
  double rmax2;         // r_max^2: pair iff r^2 < rmax2
  double cscale;        // nbins^2 / r_max^2: bin = floor(sqrt(r^2 cscale))
  int32_t nc[3];        // cells per axis (1: the whole axis is one cell)
  int32_t M;            // stencil reach in cells
  int32_t cell0;        // first global cell of this replica
  int32_t log2p;        // ceil(log2(home particles per block x n)): pair bound of a block
};
struct VvBlock {        // one chunk of home particles of one coarse cell
  int32_t rep, cell, start, count;
};
int vv_home();
hipError_t launch_vv_bin(const DevPtrs& d, const VvRep* vr, int flow, int32_t* cnt,
                         int32_t* vcell, int32_t* slot, unsigned long long* umax, double* u2_part,
                         hipStream_t s);
hipError_t launch_vv_scatter(const DevPtrs& d, int flow, const int32_t* cstart,
                             const int32_t* vcell, const int32_t* slot, double4* spos,
                             double4* su, hipStream_t s);
hipError_t launch_vv_pairs(const DevPtrs& d, const VvRep* vr, const VvBlock* blocks, int nblk,
                           const int32_t* cstart, const double4* spos, const double4* su,
                           const unsigned long long* umax, int nb, long long* psum,
                           unsigned long long* pcnt, hipStream_t s, hipEvent_t ev0 = nullptr,
                           hipEvent_t ev1 = nullptr);
int vv_fold();
hipError_t launch_vv_reduce(const DevPtrs& d, const VvRep* vr, const int2* chunks, int nchunk,
                            const int32_t* rep_chunk0, int nrep, int nb, const long long* psum,
                            const unsigned long long* pcnt, unsigned long long* f_lo,
                            long long* f_hi, unsigned long long* f_cnt,
                            const unsigned long long* umax, const double* u2_part,
                            double* out_sum, long long* out_cnt, double* out_u2, hipStream_t s);

// anisotropic pair friction, block system (block.hip)
struct BlockRep {       // per replica: W = alpha w (a_perp I + (a_par - a_perp) d d^T / r^2)
  double a_par, a_perp;
  double sq_par, sq_perp;  // square roots (the noise amplitude W^(1/2))
};
struct BcgRep {         // per-replica scalars of the block CG (3n stacked unknowns)
  double bb;            // ||b||^2 (negative until the first residual round)
  double rz;            // gamma = (r, u) of the last vector pass (or residual round)
  double alpha, beta;
  double rr;            // ||r||^2 (recursive while iterating, true after a residual round)
  double tol2;          // tolerance^2 of this solve
  int32_t state;        // 0 iterating, 1 residual round pending, 2 done
  int32_t it;
  int32_t restarts;
  int32_t breakdown;
  int32_t first;        // 1: the next vector pass starts the recurrences (beta = 0)
  int32_t pad0;
};
struct BlockPtrs {
  double* bval;         // -W_ij per CSR entry: xx, xy, xz, yy, yz, zz
  float* bvalf;         // the same rounded to FP32 (iteration products when fp32)
  double* bdiag;        // gamma0 I + sum_j W_ij per row (6 values)
  double* binv;         // its inverse (6 values): the block-Jacobi preconditioner
  BcgRep* bcg;          // [replicas]
  const BlockRep* brep; // [replicas]
  // learned preconditioner with 3 x 3 heads: M^-1 = R Xh R, R = blockdiag(A_ii^-1/2)
  double* rsq;          // [rows][6] R_i
  double* xd;           // [rows][6] M_ii
  float* xo;            // [nnz][9] M_ij, row-major
  double* t;            // [rows][3] R b (training)
  double* bh;           // [rows][3] A_ii^-1 b (training)
  double* gt;           // [rows][3] R G (training)
  double* gh;           // [rows][3] A_ii^-1 G (training)
  int32_t learned;      // 1: the block CG applies the learned M^-1
  int32_t fp32;         // 1: w = A u of the iterations with the FP32 blocks
};
hipError_t launch_pair_block(const DevPtrs& d, const BlockPtrs& bp, hipStream_t s);
hipError_t launch_bcg_reset(const DevPtrs& d, const BlockPtrs& bp, double tol, hipStream_t s);
hipError_t launch_bcg_residual(const DevPtrs& d, const BlockPtrs& bp, hipStream_t s);
hipError_t launch_bcg_warm(const DevPtrs& d, const BlockPtrs& bp, const int64_t* id_off,
                           hipStream_t s);
hipError_t launch_bcg_iteration(const DevPtrs& d, const BlockPtrs& bp, hipStream_t s);
hipError_t launch_block_export(const DevPtrs& d, const BlockPtrs& bp, const int64_t* id_off,
                               int64_t* rows, int64_t* cols, double* vals, double* diag,
                               double* rhs, hipStream_t s);
// the learned preconditioner on the block system (mpnn.hip)
hipError_t launch_mp_trunk(const DevPtrs& d, const MpPtrs& m, hipStream_t s);
hipError_t launch_mpb_heads(const DevPtrs& d, const MpPtrs& m, const BlockPtrs& bp, hipStream_t s);
hipError_t launch_mpb_loss(const DevPtrs& d, const MpPtrs& m, const BlockPtrs& bp, hipStream_t s);
hipError_t launch_mpb_backward(const DevPtrs& d, const MpPtrs& m, const BlockPtrs& bp,
                               hipStream_t s);
hipError_t launch_mpb_probe(const DevPtrs& d, const BlockPtrs& bp, double* z, double* b,
                            uint64_t seed, uint64_t index, hipStream_t s);
hipError_t launch_mpb_export(const DevPtrs& d, const BlockPtrs& bp, const int64_t* id_off,
                             int64_t* rows, int64_t* cols, double* vals, int64_t cap, double* diag,
                             hipStream_t s);
