// Kernel argument blocks and launch wrappers of sweep.hip.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "kernels.hpp"

namespace qc {

// Lattice geometry of one segment: its slots are slot0 .. slot0 + max(n, 1) - 1
// and slot t sits at s = (jf + t - half) h along the line u (n > 0), or at
// the segment midpoint smid (n = 0).
struct SegGeo {
  int64_t slot0;
  double u;     // (line - half) h
  double smid;  // (s_min + s_max) / 2
  int32_t jf, n, k, pad;
};

struct InterpArgs {
  int64_t nslot;
  int64_t nseg;
  int64_t ncell;  // nx * ny
  int ncomp, n_theta;
  GridGeom geom;
  const int32_t* slot_angle;
  const double* px;
  const double* py;
  const int32_t* fb;
  const double* aext;   // v_k . A_ext per slot
  const double* eta;    // complex [ncomp][n_theta]
  const double* cosk;
  const double* sink;
  const double* delta;  // complex [ncomp][ny][nx]
  const double* A;      // [2][ny][nx]
  // single-component path: slot positions and A_ext formed on the fly
  const SegGeo* seg_geo;
  double cx, cy, half;     // grid centre and (M - 1) / 2
  int gauge;               // 0 symmetric, 1 Landau, 2 solenoid
  double flux, bfield;     // flux quanta; pi flux / area
};

struct SweepArgs {
  int64_t nseg;
  const int32_t* order;   // launch order of the segments (longest first) or nullptr
  int G, log2g;           // lanes per segment (power of two dividing 64)
  int n_e;                // energies in this launch (stride of gbuf / ebuf)
  int n_e_tot;            // stride of the boundary stores
  int e_off;              // first energy of this launch
  int bc_valid;           // 0: start at the bulk roots
  double h, q, twopi_tt;
  const int64_t* seg_slot0;
  const int32_t* seg_n;
  const double* seg_hfirst;
  const double* seg_hlast;
  const int32_t* tap_start_seg;
  const double* tap_start_w;
  const int32_t* tap_end_seg;
  const double* tap_end_w;
  const double* eps;      // complex energies [n_e_tot]: i eps~_p or e + i delta
  const double* rp;       // pole weights [n_e_tot]
  double* node_out;       // mode 0: [nslot][4] = S_f (re, im), S_g, S_I per node
  int maxn;               // most nodes of any segment (batched spill layout)
  // Matsubara sweeps (mode 0) with an even EPL and 2G <= 64: the first nlong
  // segments of the launch order take 2G lanes and EPL/2 energies per lane,
  // the rest G lanes and EPL; nlong * 2G is a multiple of 64 (0: one shape)
  int64_t nlong;
};

struct SweepBufs {
  const void* nodes;      // node4<T> [nslot]
  const void* bc_g_prev;
  const void* bc_gt_prev;
  void* bc_g_next;
  void* bc_gt_next;
  void* gbuf;             // gamma spill [nslot][n_e] (single-grain launches)
  void* ebuf;
};

// one grain of a batched sweep: its arguments and buffers
struct BatchGrainDev {
  SweepArgs a;
  SweepBufs b;
};

struct BackArgs {
  int64_t ncg;     // grain cells
  int64_t ncell;   // nx * ny
  int ncomp, n_theta;
  const int32_t* grain_cells;
  // [n_theta][ncg] corner slots (-1: not a node; {s, -2, -2, -2}: nearest
  // node s alone); the bilinear weights are formed from the cell position
  const int4* rb4;
  int nx;
  double x0, y0, h, cx, cy, half;
  const double* node_out;
  const double* wk;
  const double* cosk;
  const double* sink;
  const double* eta;
  const double* den;   // gap denominators per component
  const double* logt;  // ln(t / t_c,G)
  double four_q;
  double twopi_rz;     // 2 pi sum_p R_p / z_p
  const double* delta;
  double* delta_new;
  double* j;
  double* omega;       // [ny][nx] or nullptr
  double* omega_cell;  // [ncg] scratch for the total
  // angles k >= pair_k0 read the node sums of their mirror slots on angle
  // k - n_theta/2 (rb4 already points there): S_g changes sign, S_f and
  // S_I do not.  n_theta when angle pairs are off.
  int pair_k0;
  // pair_fold: angle k + pair_k0 has the corners of angle k (the same
  // lattice points), so each gather of a lower angle serves both
  int pair_fold;
};

struct LdosBackArgs {
  int64_t ncg, ncell;
  int n_theta, n_e, e_off;
  const int32_t* grain_cells;
  const int32_t* rb_idx;
  const double* rb_w;
  const double* wk;
  double* out;  // [n_e_total][ny][nx]
  // e_map: output energy index of each energy of the launch order (nullptr:
  // e_off + e).  fold_k0 > 0 (LDOS only): the per-node values exist for the
  // angles k < fold_k0 alone; angle k + fold_k0 has the corners of angle k
  // and takes the values of energy e_partner[e] (both indices of the launch
  // order, partners within the block)
  const int32_t* e_map;
  const int32_t* e_partner;
  int fold_k0;
};

struct DiffNormArgs {
  const double* xnew;
  const double* xold;
  const int32_t* idx;
  int64_t n;
  int nrep;
  int64_t field_stride;
  int stride;
  int p;
  double* part;
  double* update;  // nullptr, or xold itself: then xold += alpha (xnew - xold) in the same pass
  double alpha;
  // Polyak (App. E) when vel is set: vel <- (1 - beta) vel + alpha (xnew - xold),
  // xold += vel, and the norm is taken of the step vel instead of xnew - xold
  double* vel;
  double beta;
};

// ---- reverse mode (adjoint.hip)
using AdjArgs = SweepArgs;  // node_out unused; e_off must be 0

struct AdjBufs {
  const void* nodes;       // node4<double>
  const void* bc_g_prev;   // boundary store read by the differentiated sweep
  const void* bc_gt_prev;
  void* gbuf;              // gamma at nodes  [nslot][n_e]
  void* gtbuf;             // gamma~ at nodes [nslot][n_e]
  void* lgt;               // node-local adjoint of gamma~ [nslot][n_e]
  const void* gS;          // gradients of the per-node sums [nslot][4]
  double* gV;              // out: gradients of the slot values [nslot][3] (Re D, Im D, a)
  // checkpointed variant (ck > 0): gamma and gamma~ kept every ck slots, each
  // block of ck slots recomputed into a per-thread scratch
  int ck = 0;
  const int64_t* ckbase = nullptr;  // first checkpoint block of each segment
  void* ckg = nullptr;              // gamma entering block k: [block][n_e]
  void* ckgt = nullptr;             // gamma~ at the first slot of block k: [block][n_e]
  void* scr = nullptr;              // [2][ck][EPL][nthreads] complex
  int64_t nthr = 0;                 // nseg * G
};

struct BackAdjArgs {
  int64_t ncg, ncell;
  int ncomp, n_theta;
  const int32_t* grain_cells;
  const int32_t* rb_idx;
  const double* rb_w;
  const double* wk;
  const double* cosk;
  const double* sink;
  const double* eta;
  const double* den;
  double four_q, h2, gomega;
  const double* gdn;  // complex gradient of Delta_new or nullptr
  const double* gj;   // gradient of j or nullptr
  double* gS;         // out: [nslot][4]
  // transpose of the rotate-back table by slot: entries [bt_ptr[s], bt_ptr[s+1])
  // hold (grain-cell position, weight)
  int64_t nslot;
  const int32_t* slot_angle;
  const int64_t* bt_ptr;
  const int32_t* bt_c;
  const double* bt_w;
};

struct InterpAdjArgs {
  int64_t nslot, ncell;
  int ncomp, n_theta;
  GridGeom geom;
  const int32_t* slot_angle;
  const double* px;
  const double* py;
  const int32_t* fb;
  const double* eta;
  const double* cosk;
  const double* sink;
  const double* gV;
  double* gdelta;  // out: complex [ncomp][ny][nx]
  double* gA;      // out: [2][ny][nx]
  // transposes of the slot stencils by cell: Delta entries [it_dptr[c],
  // it_dptr[c+1]) and A_ind entries [it_aptr[c], it_aptr[c+1]) hold (slot, weight)
  const int64_t* it_dptr;
  const int32_t* it_ds;
  const double* it_dw;
  const int64_t* it_aptr;
  const int32_t* it_as;
  const double* it_aw;
};

struct OmegaAdjArgs {
  int64_t ncg, ncell;
  int ncomp, n_theta;
  const int32_t* grain_cells;
  const double* delta;
  const double* eta;
  const double* wk;
  const double* logt;
  double twopi_rz, h2, gomega;
  double* gdelta;
};

void launch_adjoint(int epl, const AdjArgs& a, const AdjBufs& b, hipStream_t st);
void launch_back_adjoint(const BackAdjArgs& a, hipStream_t st);
void launch_interp_adjoint(const InterpAdjArgs& a, hipStream_t st);
void launch_omega_delta_adjoint(const OmegaAdjArgs& a, hipStream_t st);
void launch_curl_adjoint(const double* B, double* gA, int nx, int ny, double h, double s, hipStream_t st);

// cells: workspace of ncell cell4<T> records, used when ncomp == 1 (else nullptr)
template <typename T>
void launch_interp(const InterpArgs& a, void* cells, void* nodes, hipStream_t st);
template <typename T>
void launch_sweep(int mode, int epl, const SweepArgs& a, const SweepBufs& b, hipStream_t st);
// wave slots of the whole device for the Matsubara sweep kernel of this
// precision and lane shape (resident waves per CU x CUs)
template <typename T>
int64_t sweep_wave_slots(int epl);
void launch_rotate_back(const BackArgs& a, hipStream_t st);
// End values of the upper angle of each pair from its mirror segment:
// gamma_end(s') = conj(gamma~_end(s)), gamma~_end(s') = conj(gamma_end(s))
// for each (s', s) in pairs, n_e energies per segment (T = float or double)
template <typename T>
// partner: for real energies, the index of -e for each energy e of the
// store (the reversed direction at e mirrors energy -e); nullptr for the
// Matsubara poles (each its own partner)
void launch_mirror_fill(const int2* pairs, int64_t npairs, int n_e, const int32_t* partner, void* bc_g, void* bc_gt,
                        hipStream_t st);
// blocks of 256 lanes, each lane writes out[lane]: out holds nblocks * 256 floats
void launch_valu_rate(int op, float* out, int nblocks, int iters, hipStream_t st);
template <typename T>
void launch_batch_sweep(int epl, const BatchGrainDev* grains, const int2* tiles, int ntiles, int* counter, int nblocks,
                        void* spill, int64_t wave_elems,
                        hipStream_t st);
template <typename T>
void launch_ldos_back(const LdosBackArgs& a, const void* ebuf, hipStream_t st);
// complex counterpart for sweep mode 3: out = -i pi <(1-X)/(1+X)>, interleaved
template <typename T>
void launch_green_back(const LdosBackArgs& a, const void* ebuf, hipStream_t st);
void launch_fill(double* p, int64_t n, double v, hipStream_t st);
void launch_curl(const double* A, double* B, int nx, int ny, double h, hipStream_t st);
// one block-partial sum: nparts partials of x[i] (mode 0) or x[i]^2 (mode 1)
// over i < n, gathered through idx when given
struct BlockSumRow {
  const double* x;
  const int32_t* idx;
  int64_t n;
  int mode;
  double* part;
};
// two independent sums in one launch
void launch_block_sum2(const BlockSumRow& r0, const BlockSumRow& r1, int nparts, hipStream_t st);
void launch_block_sum(const double* x, const int32_t* idx, int64_t n, int mode, double* part, int nparts,
                      hipStream_t st);
void launch_diff_norm(const DiffNormArgs& a, int nparts, hipStream_t st);
// 1 to 3 independent fields in one launch (blockIdx.y picks the field)
void launch_diff_norm_n(const DiffNormArgs* a, int count, int nparts, hipStream_t st);
// CongAcc (App. E): per-component step sizes and weights of one field
constexpr int kCongMaxComp = 8;
struct CongCoef {
  double a[kCongMaxComp], w[kCongMaxComp];
};
// partials [nparts][3] of m.m, m.d, d.d over component c of the elements
// (base + idx[i] or base + i) * stride + c, d = xnew - xold
void launch_congacc_dots(const double* xnew, const double* xold, const int32_t* idx, int64_t n, int64_t base,
                         int stride, int c, const double* m, double* part, int nparts, hipStream_t st);
// m <- w m + (1 - w) d, x += a m with the coefficients of component r * stride + c
void launch_congacc_update(double* x, const double* gx, double* m, const int32_t* idx, int64_t n, int nrep,
                           int64_t field_stride, int stride, const CongCoef& cf, hipStream_t st);
// partials [nparts][3] of dp.dp, dp.(d - dp), (d - dp).(d - dp), d = scale (xnew - xold); dprev <- d
void launch_bb_dots(const double* xnew, const double* xold, const int32_t* idx, int64_t n, int nrep,
                    int64_t field_stride, int stride, double scale, double* dprev, double* part, int nparts,
                    hipStream_t st);
void launch_picard(double* x, const double* gx, const int32_t* idx, int64_t n, int nrep, int64_t field_stride,
                   int stride, double alpha, hipStream_t st);
void launch_means(const double* part, int nparts, double inv_n, double* mean, hipStream_t st);
// Luttinger-Ward free energy: per grain cell c, acc[c] (+)= w * 2 sum_G
// den_G Re(conj(delta_G) delta_new_G) (first: = instead of +=)
void launch_lw_accumulate(const double* delta, const double* delta_new, const int32_t* grain_cells, int64_t ncg,
                          int ncomp, int64_t ncell, const double* den, double w, int first, double* acc,
                          hipStream_t st);
// omega(c) = sum_G |delta_G|^2 logt_G + twopi_rz sum_k w_k |sum_G eta_G(k) delta_G|^2 - acc[c] on grain
// cells: written to omega_cell[c] (grain-cell order) and, when given, omega[cell]
void launch_lw_finish(const double* delta, const int32_t* grain_cells, int64_t ncg, int ncomp, int64_t ncell,
                      int n_theta, const double* eta, const double* wk, const double* logt, double twopi_rz,
                      const double* acc, double* omega_cell, double* omega, hipStream_t st);
void launch_scale(const double* x, double s, int64_t n, double* y, hipStream_t st);
// eigen-truncated A-solve (vecpot.hip): jp [2][n][n] masked current, vk
// [nmodes][n] eigenvectors, lam [nmodes]; y [2][nmodes][n][n] work;
// aout [2][n][n] = alpha sum_k lam_k T_k jp T_k
void launch_eig_vecpot(int n, int nmodes, const double* jp, const double* vk, const double* lam, double* y,
                       double* aout, double alpha, hipStream_t st);
void launch_masked_current(const double* j, const uint8_t* mask, int64_t ncell, const double* mean, double* jp,
                           hipStream_t st);
// per grain cell (x - cx) j_y - (y - cy) j_x, grain-cell order
void launch_torque(const double* j, const int32_t* grain_cells, int64_t ncg, int64_t ncell, int nx, double x0,
                   double y0, double h, double cx, double cy, double* out, hipStream_t st);
void launch_pad_current(const double* j, const uint8_t* mask, int nx, int ny, int px, int py, const double* mean,
                        double2* w, hipStream_t st);
void launch_fft_rows(double2* w, int rows, int logn, const double2* tw, int sign, const double2* pre, hipStream_t st);
void launch_transpose(const double2* in, double2* out, int rows, int cols, hipStream_t st);
void launch_unpad_A(const double2* w, int nx, int ny, int px, double scale, double* A, hipStream_t st);

}  // namespace qc
