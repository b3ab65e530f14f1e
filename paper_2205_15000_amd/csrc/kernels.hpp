// Device-side building blocks: complex arithmetic and the Riccati step.
//
// Everything here runs in either FP64 or FP32 (the mixed path).  FP32 uses
// the hardware square root, reciprocal square root and reciprocal (1 ulp).
// FP64 refines the hardware reciprocal and reciprocal square root with two
// Newton iterations each (quadratic convergence from the ~2^-23 hardware
// approximation to full double precision).  All of it is branch-free.
#pragma once

#include <hip/hip_runtime.h>

namespace qc {

template <typename T>
struct cpx {
  T x, y;
};

// Workgroups are dispatched round-robin over the 8 XCDs, each with its own
// L2.  Map the hardware block index to a logical one so that every XCD runs
// one contiguous range of logical blocks (a bijection of [0, nb)).
__device__ __forceinline__ int64_t xcd_block(int64_t bid, int64_t nb) {
  const int64_t q = nb / 8, r = nb % 8, x = bid % 8, l = bid / 8;
  return x < r ? x * (q + 1) + l : r * (q + 1) + (x - r) * q + l;
}

// one reference-grid cell for the single-component interpolation:
// Delta (re, im) and A_ind (x, y) side by side
template <typename T>
struct __attribute__((aligned(4 * sizeof(T)))) cell4 {
  T dx, dy, ax, ay;
};

// node value slot: Delta(p_k, slot) and a(slot) = v_k . A(slot)
template <typename T>
struct __attribute__((aligned(4 * sizeof(T)))) node4 {
  T dx, dy, a, pad;
};

template <typename T>
__device__ __forceinline__ cpx<T> mk(T a, T b) {
  cpx<T> r;
  r.x = a;
  r.y = b;
  return r;
}
template <typename T>
__device__ __forceinline__ cpx<T> operator+(cpx<T> a, cpx<T> b) { return mk(a.x + b.x, a.y + b.y); }
template <typename T>
__device__ __forceinline__ cpx<T> operator-(cpx<T> a, cpx<T> b) { return mk(a.x - b.x, a.y - b.y); }
template <typename T>
__device__ __forceinline__ cpx<T> operator*(cpx<T> a, cpx<T> b) {
  return mk(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
template <typename T>
__device__ __forceinline__ cpx<T> operator*(T s, cpx<T> a) { return mk(s * a.x, s * a.y); }

__device__ __forceinline__ double dabs(double v) { return __builtin_fabs(v); }
__device__ __forceinline__ float dabs(float v) { return __builtin_fabsf(v); }
__device__ __forceinline__ double dsign(double m, double s) { return __builtin_copysign(m, s); }
__device__ __forceinline__ float dsign(float m, float s) { return __builtin_copysignf(m, s); }
__device__ __forceinline__ double dmax(double a, double b) { return __builtin_fmax(a, b); }
__device__ __forceinline__ float dmax(float a, float b) { return __builtin_fmaxf(a, b); }

// 1/x
__device__ __forceinline__ float drcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double drcp(double x) {
  double y = __builtin_amdgcn_rcp(x);
  double e = __builtin_fma(-x, y, 1.0);
  y = __builtin_fma(y, e, y);
  e = __builtin_fma(-x, y, 1.0);
  return __builtin_fma(y, e, y);
}
// 1/sqrt(x), x > 0
__device__ __forceinline__ float drsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double drsq(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  double e = __builtin_fma(-h * y, y, 0.5);  // y <- y (3/2 - x y^2 / 2)
  y = __builtin_fma(y, e, y);
  e = __builtin_fma(-h * y, y, 0.5);
  return __builtin_fma(y, e, y);
}
// sqrt(x), x >= 0
__device__ __forceinline__ float dsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double dsqrt(double x) { return x * drsq(dmax(x, 1e-300)); }
template <typename T>
__device__ __forceinline__ T tiny();
template <>
__device__ __forceinline__ float tiny<float>() { return 1e-30f; }
template <>
__device__ __forceinline__ double tiny<double>() { return 1e-300; }

// Principal square root (branch cut on the negative real axis; the sign of
// a zero imaginary part picks the side), from u = (|w| + |x|)/2:
// sqrt(w) = (sqrt u, y / (2 sqrt u)) for x >= 0, else (|y| / (2 sqrt u), +-sqrt u).
template <typename T>
__device__ __forceinline__ cpx<T> csqrt(cpx<T> w) {
  const T r = dsqrt(w.x * w.x + w.y * w.y);
  const T u = T(0.5) * (r + dabs(w.x));
  const T rs = drsq(dmax(u, tiny<T>()));
  const T t = u * rs;
  const T yq = T(0.5) * w.y * rs;
  const bool pos = w.x >= T(0);
  return mk(pos ? t : dabs(yq), pos ? yq : dsign(t, w.y));
}

// Per-node constants of one implicit-midpoint step (App. C) for the half-step
// order parameter dm and step length hs: c2 = (i hs/4) conj(dm) and 4 c2.
template <typename T>
struct StepNode {
  T c2x, c2y, c4x, c4y, hs;
};
template <typename T>
__device__ __forceinline__ StepNode<T> step_node(T dmx, T dmy, T hs) {
  StepNode<T> s;
  const T hq = T(0.25) * hs;
  s.c2x = hq * dmy;
  s.c2y = hq * dmx;
  s.c4x = T(4) * s.c2x;
  s.c4y = T(4) * s.c2y;
  s.hs = hs;
  return s;
}

// One implicit-midpoint step of d gamma/ds = i[D* g^2 + 2 z g + D] (App. C,
// v_F = 1) with z = (zx, zy): g' = 2 c0 / (-c1 + sqrt(c1^2 - 4 c2 c0)) with
// c1 = 2 c2 g + i h z - 1 and c0 = (c1 - c2 g + 2) g - 4 conj(c2); the root is
// flipped if it points away from -c1, so that g' -> g as h -> 0.
template <typename T>
__device__ __forceinline__ cpx<T> riccati_step(cpx<T> g, const StepNode<T>& s, T zx, T zy) {
  const T cgx = s.c2x * g.x - s.c2y * g.y;  // c2 g
  const T cgy = s.c2x * g.y + s.c2y * g.x;
  const T kx = -s.hs * zy - T(1);            // i h z - 1
  const T ky = s.hs * zx;
  const T c1x = T(2) * cgx + kx, c1y = T(2) * cgy + ky;
  const T px = cgx + kx + T(2), py = cgy + ky;  // c1 - c2 g + 2
  const T c0x = px * g.x - py * g.y - s.c4x;
  const T c0y = px * g.y + py * g.x + s.c4y;
  const T dx = c1x * c1x - c1y * c1y - (s.c4x * c0x - s.c4y * c0y);
  const T dy = T(2) * c1x * c1y - (s.c4x * c0y + s.c4y * c0x);
  cpx<T> rt = csqrt(mk(dx, dy));
  const bool flip = rt.x * c1x + rt.y * c1y > T(0);  // Re(rt conj(-c1)) < 0
  rt = mk(flip ? -rt.x : rt.x, flip ? -rt.y : rt.y);
  const T ex = rt.x - c1x, ey = rt.y - c1y;
  const T rn = T(2) * drcp(ex * ex + ey * ey);
  return mk((c0x * ex + c0y * ey) * rn, (c0y * ex - c0x * ey) * rn);
}

__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }

// The same implicit-midpoint step as riccati_step, solved for the midpoint
// value w = (g + g')/2 instead of g'.  With D the half-step order parameter,
// k = i h z - 1 and the step equation g' - g = i h [D* w^2 + 2 z w + D]:
//   (i h D*) w^2 + 2 k w + U = 0,   U = 2 g + i h D.
// With K = k/2 and c2 = (i h/4) conj(D) (so i h D* = 4 c2 and i h D =
// -4 conj(c2)) the stable root is w = -U / (2 e), e = K + s sqrt(disc),
//   disc = K^2 - c2 U,
// the sign s taken so that s sqrt(disc) points along K (|e| is then the
// larger of the two choices and w -> g as h -> 0).  So g' = 2 w - g =
// -U conj(e) / |e|^2 - g.  (disc is a quarter of c1^2 - 4 c2 c0 of
// riccati_step with the terms in g^2 cancelled.)
// The roots of disc = (dx, dy) are +-(a, b) r with v = |disc| + |dx|,
// r = 1/sqrt(2 v) and (a, b) = (v, dy) for dx >= 0, (dy, v) otherwise
// ((a + i b)^2 r^2 = disc in both cases); since r > 0 the sign of
// a Kx + b Ky picks s without forming the principal root.
// Per step (shared by all energies): c2 and U0 = i h D = -4 conj(c2).  Per
// energy: Kx = (-h Im z - 1)/2, its square Kx2, and Ky = h Re z / 2.
template <typename T>
struct StepC {
  T c2x, c2y, U0x, U0y;
};
template <typename T>
__device__ __forceinline__ cpx<T> riccati_step_c(cpx<T> g, const StepC<T>& s, T Kx, T Kx2, T Ky) {
  const T Ux = fmaT(T(2), g.x, s.U0x), Uy = fmaT(T(2), g.y, s.U0y);
  const T dx = fmaT(-s.c2x, Ux, fmaT(s.c2y, Uy, fmaT(-Ky, Ky, Kx2)));
  const T dy = fmaT(-s.c2x, Uy, fmaT(-s.c2y, Ux, (Kx + Kx) * Ky));
  const T v = dsqrt(fmaT(dx, dx, dy * dy)) + dabs(dx);
  const T r = drsq(fmaT(v, T(2), tiny<T>()));
  const bool pos = dx >= T(0);
  const T ra = pos ? v : dy, rb = pos ? dy : v;
  const T rs = fmaT(ra, Kx, rb * Ky) < T(0) ? -r : r;
  const T ex = fmaT(rs, ra, Kx), ey = fmaT(rs, rb, Ky);
  const T rn = drcp(fmaT(ex, ex, ey * ey));
  const T nx = fmaT(Ux, ex, Uy * ey), ny = fmaT(Uy, ex, -(Ux * ey));
  return mk(fmaT(-nx, rn, -g.x), fmaT(-ny, rn, -g.y));
}

// Step constants of riccati_step_c for half-step value dm and length hs
template <typename T>
__device__ __forceinline__ StepC<T> step_consts(T dmx, T dmy, T hs) {
  StepC<T> c;
  const T h4 = T(0.25) * hs;
  c.c2x = h4 * dmy;
  c.c2y = h4 * dmx;
  c.U0x = T(-4) * c.c2x;
  c.U0y = T(4) * c.c2y;
  return c;
}
// riccati_step_c with the per-energy constants formed from z = (zx, zy)
template <typename T>
__device__ __forceinline__ cpx<T> riccati_step_z(cpx<T> g, const StepC<T>& c, T hs, T zx, T zy) {
  const T Kx = fmaT(T(-0.5) * hs, zy, T(-0.5));
  return riccati_step_c(g, c, Kx, Kx * Kx, T(0.5) * hs * zx);
}

// Stable homogeneous root of D* g^2 + 2 z g + D = 0: -D / (z + s) with
// s = sqrt(z^2 - |D|^2) on the branch Im s > 0.
template <typename T>
__device__ __forceinline__ cpx<T> bulk_root(T zx, T zy, T dx, T dy) {
  cpx<T> s = csqrt(mk(zx * zx - zy * zy - (dx * dx + dy * dy), T(2) * zx * zy));
  const bool neg = s.y < T(0);
  const T sx = neg ? -s.x : s.x, sy = neg ? -s.y : s.y;
  const T bx = zx + sx, by = zy + sy;
  const T r = drcp(bx * bx + by * by);
  return mk(-(dx * bx + dy * by) * r, -(dy * bx - dx * by) * r);
}

// Lattice and cell positions rounded operation by operation, in the order
// written, as the host plan forms them (its host code has no fused
// multiply-add): floor() of these values then picks the plan's corners even
// where a coordinate sits exactly on a lattice line.
__device__ __forceinline__ double rn_point(double c0, double u, double eu, double s, double es) {
#pragma clang fp contract(off)
  return c0 + u * eu + s * es;
}
__device__ __forceinline__ double rn_node_s(double j, double half, double h) {
#pragma clang fp contract(off)
  return (j - half) * h;
}
__device__ __forceinline__ double rn_cell_offset(double x0, double i, double h, double c) {
#pragma clang fp contract(off)
  return x0 + (i + 0.5) * h - c;
}
__device__ __forceinline__ double rn_lattice(double rx, double ex, double ry, double ey, double h, double half) {
#pragma clang fp contract(off)
  return (rx * ex + ry * ey) / h + half;
}

// Bilinear weights of the four cell centres around (px, py) on the
// reference grid (Sec. III.A), formed with the same IEEE operations as the
// host tables (the adjoint's transposed tables call them on the host).  Delta: corners off the array or outside the grain are
// dropped and the rest renormalised; fb >= 0 names the nearest grain cell
// used when no corner keeps a positive weight.  A_ind: plain bilinear with
// the point clamped onto the outermost cell centres.
struct GridGeom {
  int nx, ny;
  double x0, y0, h;
  const uint8_t* mask;
};
__host__ __device__ inline void delta_stencil(const GridGeom& gg, double px, double py, int fb, int idx[4],
                                              double w[4]) {
  const double fx = (px - gg.x0) / gg.h - 0.5, fy = (py - gg.y0) / gg.h - 0.5;
  const int i0 = static_cast<int>(__builtin_floor(fx)), j0 = static_cast<int>(__builtin_floor(fy));
  const double wx = fx - i0, wy = fy - j0;
  w[0] = (1 - wx) * (1 - wy);
  w[1] = wx * (1 - wy);
  w[2] = (1 - wx) * wy;
  w[3] = wx * wy;
  double tot = 0.0;
  for (int c = 0; c < 4; ++c) {
    const int ci = i0 + (c & 1), cj = j0 + (c >> 1);
    const bool ok = ci >= 0 && ci < gg.nx && cj >= 0 && cj < gg.ny && gg.mask[cj * gg.nx + ci];
    idx[c] = ok ? cj * gg.nx + ci : 0;
    if (!ok) w[c] = 0.0;
    tot += w[c];
  }
  if (fb >= 0) {
    idx[0] = fb;
    idx[1] = idx[2] = idx[3] = 0;
    w[0] = 1.0;
    w[1] = w[2] = w[3] = 0.0;
  } else if (tot > 0.0) {
    for (int c = 0; c < 4; ++c) w[c] /= tot;
  }
}
__host__ __device__ inline void a_stencil(const GridGeom& gg, double px, double py, int idx[4], double w[4]) {
  const double fx = __builtin_fmin(__builtin_fmax((px - gg.x0) / gg.h - 0.5, 0.0), gg.nx - 1.0);
  const double fy = __builtin_fmin(__builtin_fmax((py - gg.y0) / gg.h - 0.5, 0.0), gg.ny - 1.0);
  const int fi = static_cast<int>(__builtin_floor(fx)), fj = static_cast<int>(__builtin_floor(fy));
  const int i0 = fi < gg.nx - 2 ? fi : gg.nx - 2;
  const int j0 = fj < gg.ny - 2 ? fj : gg.ny - 2;
  const double wx = fx - i0, wy = fy - j0;
  idx[0] = j0 * gg.nx + i0;
  idx[1] = idx[0] + 1;
  idx[2] = idx[0] + gg.nx;
  idx[3] = idx[2] + 1;
  w[0] = (1 - wx) * (1 - wy);
  w[1] = wx * (1 - wy);
  w[2] = (1 - wx) * wy;
  w[3] = wx * wy;
}

// Sum of v over aligned groups of G lanes (G a power of two <= 64); every
// lane of the group ends with the total.  DPP within rows of 16 lanes,
// cross-lane permutes beyond.
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, true);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, true);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ double group_sum(double v, int G) {
  if (G >= 2) v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
  if (G >= 4) v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
  if (G >= 8) v += dpp_f64<0x141>(v);  // row_half_mirror
  if (G >= 16) v += dpp_f64<0x140>(v); // row_mirror
  if (G >= 32) v += __shfl_xor(v, 16);
  if (G >= 64) v += __shfl_xor(v, 32);
  return v;
}

__device__ __forceinline__ double sel(bool c, double a, double b) { return c ? a : b; }
// v + v of the lane 16 (32) apart: the row (half-wave) swap leaves the
// partner's value in one of the two results and the lane's own in the other
__device__ __forceinline__ double xor16_sum(double v) {
  const unsigned lo = static_cast<unsigned>(__double2loint(v)), hi = static_cast<unsigned>(__double2hiint(v));
  const auto l = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
  const auto h = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
  return __hiloint2double(static_cast<int>(h[0]), static_cast<int>(l[0])) +
         __hiloint2double(static_cast<int>(h[1]), static_cast<int>(l[1]));
}
__device__ __forceinline__ double xor32_sum(double v) {
  const unsigned lo = static_cast<unsigned>(__double2loint(v)), hi = static_cast<unsigned>(__double2hiint(v));
  const auto l = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
  const auto h = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
  return __hiloint2double(static_cast<int>(h[0]), static_cast<int>(l[0])) +
         __hiloint2double(static_cast<int>(h[1]), static_cast<int>(l[1]));
}
// xor-4 partner inside a 32-lane half (the LDS crossbar swizzle, bit mode)
__device__ __forceinline__ double swz_xor4(double v) {
  const int lo = __builtin_amdgcn_ds_swizzle(__double2loint(v), 0x101F);
  const int hi = __builtin_amdgcn_ds_swizzle(__double2hiint(v), 0x101F);
  return __hiloint2double(hi, lo);
}

// Sums of four quantities over aligned groups of G >= 4 lanes (G a power of
// two <= 64), scattered: every lane ends with the group total of quantity
// 2 (lane & 1) + ((lane >> 1) & 1), so lanes 0..3 of the group hold all four.
// Two halving steps inside each quad (each lane keeps half of what it has
// and adds the partner's matching half), then plain sums across quads:
// rotations by 4 and 8 inside a 16-lane row, row and half-wave swaps beyond.
__device__ __forceinline__ double group_sum4_scatter(double q0, double q1, double q2, double q3, int G,
                                                    int lane) {
  const bool b0 = lane & 1, b1 = (lane >> 1) & 1;
  double k0 = sel(b0, q2, q0), k1 = sel(b0, q3, q1);
  const double s0 = sel(b0, q0, q2), s1 = sel(b0, q1, q3);
  k0 += dpp_f64<0xB1>(s0);  // quad_perm [1,0,3,2]
  k1 += dpp_f64<0xB1>(s1);
  double k = sel(b1, k1, k0);
  const double s = sel(b1, k0, k1);
  k += dpp_f64<0x4E>(s);  // quad_perm [2,3,0,1]
  if (G == 8) k += swz_xor4(k);
  if (G >= 16) {
    k += dpp_f64<0x124>(k);  // row_ror:4
    k += dpp_f64<0x128>(k);  // row_ror:8
  }
  if (G >= 32) k = xor16_sum(k);
  if (G >= 64) k = xor32_sum(k);
  return k;
}
__device__ __forceinline__ int scatter_index(int lane) { return 2 * (lane & 1) + ((lane >> 1) & 1); }


}  // namespace qc
