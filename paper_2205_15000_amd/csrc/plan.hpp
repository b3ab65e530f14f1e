// Host-side trajectory tables of one grain (Sec. III.A of arXiv:2205.15000).
//
// The reference grid carries Delta_G and A_ind at cell centres.  For every
// Fermi-surface angle phi_k a square lattice of the same spacing h, rotated so
// that its "node" axis is parallel to v_F(phi_k) and centred on the grid
// centre, supplies the trajectories: each lattice line is cut by the exact
// grain boundary into segments [s_min, s_max]; the lattice nodes strictly
// inside a segment are where gamma, gamma~ and the Green's functions live.
// A segment without an interior node gets one value slot at its midpoint.
//
// Everything here is built once per grain on the host and uploaded.
#pragma once

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

namespace qc {

struct Shape {
  int kind = 0;  // 0 disc, 1 convex polygon (regular polygons are converted),
                 // 2 closed polyline from a cell mask (even-odd inside)
  bool add = true;
  double cx = 0, cy = 0, r = 0;
  std::vector<double> vx, vy;  // counter-clockwise
  std::vector<double> ax, ay, bx, by;  // kind 2: contour edges a -> b
};

// Kind-2 component from a cell mask [ny][nx] (nonzero = inside) on the grid
// with cell centres (x0 + (i + 1/2) h, y0 + (j + 1/2) h): the marching-squares
// contour at level 1/2 over the cell centres, cells beyond the array outside,
// diagonal-only squares keeping their two corners apart.
Shape mask_shape(const uint8_t* mask, int nx, int ny, double x0, double y0, double h, bool add);

struct Plan {
  // ---- inputs
  int nx = 0, ny = 0;
  double h = 0, x0 = 0, y0 = 0, cx = 0, cy = 0;
  int n_theta = 0, n_poles = 0, ncomp = 0;
  double t = 0;
  std::vector<double> tc_rel;
  std::vector<std::complex<double>> eta;  // [ncomp][n_theta]
  double kappa = 0, flux = 0;
  int gauge = 0, q = -1, precision = 0;
  std::vector<Shape> shapes;

  // ---- grid and tables
  std::vector<uint8_t> mask;           // [ny][nx]
  std::vector<int32_t> grain_cells;    // flat indices of grain cells, in 16 x 16 tile order
  double area = 0;
  int M = 0;                           // lattice side
  double half = 0;                     // (M-1)/2
  std::vector<double> phi, cosk, sink, wk;  // per angle
  std::vector<double> zp, rp;          // Ozaki poles and residues (ascending z)

  // ---- segments, ordered by (angle, line, s)
  int64_t nseg = 0;
  std::vector<int32_t> seg_angle, seg_line, seg_jfirst, seg_n;
  std::vector<int64_t> seg_slot0;      // first value slot
  std::vector<double> seg_smin, seg_smax, seg_tmin, seg_tmax;
  std::vector<double> seg_hfirst, seg_hlast;  // partial end steps (n>0); hfirst = length if n==0
  std::vector<int64_t> angle_seg0;     // [n_theta+1]
  std::vector<int64_t> line_seg0;      // [n_theta][M+1]

  // ---- value slots, ordered by segment
  int64_t nslot = 0, nnode = 0;
  std::vector<int32_t> slot_angle;
  std::vector<int32_t> slot_seg;
  std::vector<double> slot_px, slot_py; // slot positions; the device forms the
                                       // bilinear weights of Delta (masked) and A_ind
                                       // (clamped) from them
  std::vector<int32_t> slot_fb;        // nearest grain cell where no masked corner
                                       // keeps a positive weight, else -1
  std::vector<double> slot_aext;       // v_k . A_ext(slot)

  // ---- rotate-back stencils of grain cells: [angle][corner][cell]
  std::vector<int32_t> rb_idx;         // global slot index
  std::vector<double> rb_w;
  // compact form [n_theta][ncg][4]: slot of each corner or -1; a cell that
  // takes its nearest node instead holds {slot, -2, -2, -2}
  std::vector<int32_t> rb4;

  // ---- specular boundary taps: [seg][4]
  std::vector<int32_t> tap_start_seg, tap_end_seg;
  std::vector<double> tap_start_w, tap_end_w;

  // ---- angle pairs (k, k + n_theta/2): the same lattice points on reversed
  // lines.  pair_ok when every segment of an angle k >= n_theta/2 has a
  // mirror on angle k - n_theta/2 with the same nodes in reverse order (same
  // slot positions and nearest-cell fallbacks), and the weights and basis
  // values of the two angles agree.  seg_mirror[s] is that mirror for
  // segments of the upper angles (-1 for the lower ones); rb4_pair is rb4
  // with the slots of the upper angles replaced by their mirrors.
  bool pair_ok = false;
  int64_t nseg_pair = 0, nslot_pair = 0;  // segments / slots of the lower angles
  std::vector<int32_t> seg_mirror;
  std::vector<int32_t> rb4_pair;
  // rb_fold: for every grain cell, the corners of each upper angle are the
  // corners of its lower angle (the same lattice points, in reverse order),
  // so the rotate-back may gather once per pair
  bool rb_fold = false;

  int64_t steps_per_sweep() const;
};

// Builds every table; throws std::runtime_error with a message on bad input.
void build_plan(Plan& p);

// Ozaki poles z_p > 0 and residues R_p (ascending z): eigen-decomposition of
// the 2N x 2N tridiagonal continued-fraction matrix, Jacobi rotations.
void ozaki_table(int n_poles, std::vector<double>& z, std::vector<double>& r);

// App. F basis function (qc_basis) at the angle phi from the crystal axis:
// s = 1, d_{x2-y2} = sqrt2 cos 2 phi, d_xy = sqrt2 sin 2 phi, g = sqrt2 sin 4 phi.
std::complex<double> basis_eta(int kind, double phi);

// Normalised periodic Fermi-surface quadrature weights (Sec. III.A).
std::vector<double> fs_weights(int n_theta);

// Eigen-decomposition of a dense symmetric n x n matrix (row-major, taken
// by value): Householder reduction to tridiagonal form, then implicit QR
// sweeps with Wilkinson shifts.  lam[i] with eigenvector column i of
// vec (row-major, vec[r * n + i]).
void sym_eigen(int n, std::vector<double> a, std::vector<double>& lam, std::vector<double>& vec);

}  // namespace qc
