// HIP kernels of the Riccati-sweep iteration for gfx950 (arXiv:2205.15000).
//
//   interp_kernel       Delta(p_k, slot), a(slot) = v_k.A(slot) on the rotated
//                       lattices (Sec. III.A bilinear interpolation)
//   sweep_kernel        gamma forward / gamma~ backward along every segment
//                       (App. C), Green's functions (Sec. II.A) and per-node
//                       pole sums; one group of G lanes per segment, EPL
//                       energies per lane, all angles in one launch
//   rotate_back_kernel  rotated lattice -> reference cells, angle sums,
//                       gap update (Eq. gapeq_fixpoint), current
//                       (Eq. current_density), free-energy density
//   ldos_back_kernel    rotate-back of the per-energy LDOS values
//   fft / A-solve / curl / reductions / Picard helpers (App. D, App. E)
#include "kernels.hpp"
#include "sweep.hpp"

namespace qc {

// --------------------------------------------------------------------------
// interpolation pre-pass
// --------------------------------------------------------------------------
template <typename T>
__global__ void __launch_bounds__(256) interp_kernel(InterpArgs a, node4<T>* __restrict__ nodes) {
  const int64_t s = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s >= a.nslot) return;
  const int k = a.slot_angle[s];
  const double px = a.px[s], py = a.py[s];
  int di[4], ai[4];
  double dw[4], aw[4];
  delta_stencil(a.geom, px, py, a.fb[s], di, dw);
  a_stencil(a.geom, px, py, ai, aw);
  double dx = 0.0, dy = 0.0;
  for (int c = 0; c < 4; ++c) {
    const int idx = di[c];
    const double w = dw[c];
    double vx = 0.0, vy = 0.0;
    for (int g = 0; g < a.ncomp; ++g) {
      const double ex = a.eta[2 * (g * a.n_theta + k)], ey = a.eta[2 * (g * a.n_theta + k) + 1];
      const double fx = a.delta[2 * (static_cast<int64_t>(g) * a.ncell + idx)];
      const double fy = a.delta[2 * (static_cast<int64_t>(g) * a.ncell + idx) + 1];
      vx += ex * fx - ey * fy;
      vy += ex * fy + ey * fx;
    }
    dx += vx * w;
    dy += vy * w;
  }
  double ax = 0.0, ay = 0.0;
  for (int c = 0; c < 4; ++c) {
    ax += a.A[ai[c]] * aw[c];
    ay += a.A[a.ncell + ai[c]] * aw[c];
  }
  node4<T> v;
  v.dx = static_cast<T>(dx);
  v.dy = static_cast<T>(dy);
  v.a = static_cast<T>(a.cosk[k] * ax + a.sink[k] * ay + a.aext[s]);
  v.pad = T(0);
  nodes[s] = v;
}

// Single order-parameter component: Delta and A_ind packed per cell in the
// sweep precision, so the gathers of a slot touch one 16 B (FP32) or 32 B
// (FP64) record per corner and the FP32 grid stays resident in L2.  Cells
// outside the grain carry a NaN in Re Delta: the masked interpolation reads
// the mask from the same record instead of a separate dependent load.
template <typename T>
__global__ void __launch_bounds__(256) pack_cells_kernel(const double* __restrict__ delta,
                                                         const double* __restrict__ A,
                                                         const uint8_t* __restrict__ mask, int64_t ncell,
                                                         cell4<T>* __restrict__ cells) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= ncell) return;
  cell4<T> c;
  c.dx = mask[i] ? static_cast<T>(delta[2 * i]) : __builtin_nan("");
  c.dy = static_cast<T>(delta[2 * i + 1]);
  c.ax = static_cast<T>(A[i]);
  c.ay = static_cast<T>(A[ncell + i]);
  cells[i] = c;
}

// Same stencils as interp_kernel (identical floating-point operations for the
// weights): masked bilinear for Delta with the nearest-grain-cell fallback,
// clamped bilinear for A_ind.  Away from the array edge the two stencils
// share their corners, and the four records serve both.
template <typename T>
__global__ void __launch_bounds__(256) interp1_kernel(InterpArgs a, const cell4<T>* __restrict__ cells,
                                                      node4<T>* __restrict__ nodes) {
  // one wave per segment: its record is read once (scalar loads), and each
  // lane takes every 64th slot of the segment
  const int64_t seg = __builtin_amdgcn_readfirstlane(static_cast<int>(blockIdx.x) * 4 + static_cast<int>(threadIdx.x >> 6));
  if (seg >= a.nseg) return;
  const SegGeo sgeo = a.seg_geo[seg];
  const int nsl = sgeo.n > 0 ? sgeo.n : 1;
  const GridGeom& gg = a.geom;
  const int k = sgeo.k;
  const double epx = a.cosk[k], epy = a.sink[k];
  for (int t = static_cast<int>(threadIdx.x & 63); t < nsl; t += 64) {
    const int64_t s = sgeo.slot0 + t;
    const int fb = a.fb[s];
    // the slot position as the plan forms it, so the corner choice below is
    // the one the nearest-cell fallback was decided on
    const double sp = sgeo.n > 0 ? rn_node_s(static_cast<double>(sgeo.jf + t), a.half, gg.h) : sgeo.smid;
    const double px = rn_point(a.cx, sgeo.u, epy, sp, epx);
    const double py = rn_point(a.cy, sgeo.u, -epx, sp, epy);
    const double fx = (px - gg.x0) / gg.h - 0.5, fy = (py - gg.y0) / gg.h - 0.5;
    const int i0 = static_cast<int>(__builtin_floor(fx)), j0 = static_cast<int>(__builtin_floor(fy));
    const double wx = fx - i0, wy = fy - j0;
    double w[4];
    w[0] = (1 - wx) * (1 - wy);
    w[1] = wx * (1 - wy);
    w[2] = (1 - wx) * wy;
    w[3] = wx * wy;
    cell4<T> v[4];
    double tot = 0.0;
    for (int c = 0; c < 4; ++c) {
      const int ci = i0 + (c & 1), cj = j0 + (c >> 1);
      const bool in = ci >= 0 && ci < gg.nx && cj >= 0 && cj < gg.ny;
      const int lc = min(max(ci, 0), gg.nx - 1), lj = min(max(cj, 0), gg.ny - 1);
      v[c] = cells[static_cast<int64_t>(lj) * gg.nx + lc];
      const bool ok = in && v[c].dx == v[c].dx;  // NaN marks cells outside the grain
      if (!ok) w[c] = 0.0;
      tot += w[c];
    }
    const double ex = a.eta[2 * k], ey = a.eta[2 * k + 1];
    double dx = 0.0, dy = 0.0;
    if (fb >= 0) {
      const cell4<T> f = cells[fb];
      const double fx0 = static_cast<double>(f.dx), fy0 = static_cast<double>(f.dy);
      dx = ex * fx0 - ey * fy0;
      dy = ex * fy0 + ey * fx0;
    } else {
      if (tot > 0.0)
        for (int c = 0; c < 4; ++c) w[c] /= tot;
      for (int c = 0; c < 4; ++c) {
        if (w[c] == 0.0) continue;  // a dropped corner may hold the NaN marker
        const double cx = static_cast<double>(v[c].dx), cy = static_cast<double>(v[c].dy);
        dx += (ex * cx - ey * cy) * w[c];
        dy += (ex * cy + ey * cx) * w[c];
      }
    }
    // A_ind: clamped bilinear
    const double fxa = __builtin_fmin(__builtin_fmax(fx, 0.0), gg.nx - 1.0);
    const double fya = __builtin_fmin(__builtin_fmax(fy, 0.0), gg.ny - 1.0);
    const int i0a = min(static_cast<int>(__builtin_floor(fxa)), gg.nx - 2);
    const int j0a = min(static_cast<int>(__builtin_floor(fya)), gg.ny - 2);
    const double wxa = fxa - i0a, wya = fya - j0a;
    double aw[4];
    aw[0] = (1 - wxa) * (1 - wya);
    aw[1] = wxa * (1 - wya);
    aw[2] = (1 - wxa) * wya;
    aw[3] = wxa * wya;
    double ax = 0.0, ay = 0.0;
    if (i0a == i0 && j0a == j0) {
      for (int c = 0; c < 4; ++c) {
        ax += static_cast<double>(v[c].ax) * aw[c];
        ay += static_cast<double>(v[c].ay) * aw[c];
      }
    } else {
      const int64_t b0 = static_cast<int64_t>(j0a) * gg.nx + i0a;
      for (int c = 0; c < 4; ++c) {
        const cell4<T> u = cells[b0 + (c & 1) + (c >> 1) * gg.nx];
        ax += static_cast<double>(u.ax) * aw[c];
        ay += static_cast<double>(u.ay) * aw[c];
      }
    }
    node4<T> o;
    o.dx = static_cast<T>(dx);
    o.dy = static_cast<T>(dy);
    // external field: symmetric, Landau or solenoid gauge (App. B; Eq. solenoid_gauge)
    double ex_x = 0.0, ex_y = 0.0;
    const double rx = px - a.cx, ry = py - a.cy;
    if (a.gauge == 0) {
      ex_x = -0.5 * a.bfield * ry;
      ex_y = 0.5 * a.bfield * rx;
    } else if (a.gauge == 1) {
      ex_x = -a.bfield * ry;
    } else {
      const double r2 = rx * rx + ry * ry;
      if (r2 > 0.0) {
        ex_x = -0.5 * a.flux * ry / r2;
        ex_y = 0.5 * a.flux * rx / r2;
      }
    }
    o.a = static_cast<T>(epx * (ax + ex_x) + epy * (ay + ex_y));
    o.pad = T(0);
    nodes[s] = o;
  }
}

// --------------------------------------------------------------------------
// Riccati sweep
//
// Lane group of G lanes per segment, EPL consecutive energies per lane
// (energy e = lane * EPL + i).  Step t (t = 0..n) joins value slot t-1 and t;
// a boundary point takes the value of the nearest slot (App. C), so the
// half-step value is the mean of the two slot values with V(-1) = V(0) and
// V(n) = V(n-1).  gamma runs t = 0..n, gamma~ t = n..0 with D -> -D*.  The
// partial end steps (t = 0 and t = n) are peeled off the loops, so interior
// steps use per-energy constants formed once for the full step h.
//
// Per node and pole (Sec. II.A): X = gamma gamma~, g = -i pi (1-X)/(1+X),
// f = -2 i pi gamma/(1+X), f~ = 2 i pi gamma~/(1+X); the pole sums are
// formed from 1/(1+X) alone (identities at node_sums below).
// --------------------------------------------------------------------------
template <typename T, int EPL, int MODE>
__device__ __forceinline__ void sweep_segment(const SweepArgs& a, int64_t wseg, int lane, int G, int lg,
                                              const node4<T>* __restrict__ nodes,
                                              const cpx<T>* __restrict__ bc_g_prev,
                                              const cpx<T>* __restrict__ bc_gt_prev,
                                              cpx<T>* __restrict__ bc_g_next, cpx<T>* __restrict__ bc_gt_next,
                                              cpx<T>* __restrict__ gbase, int64_t gmul, T* __restrict__ ebuf,
                                              double* __restrict__ lsum) {
  const int64_t seg = a.order ? static_cast<int64_t>(a.order[wseg]) : wseg;
  const int64_t slot0 = a.seg_slot0[seg];
  const int n = a.seg_n[seg];
  const int last = n > 0 ? n - 1 : 0;
  const T hfirst = static_cast<T>(a.seg_hfirst[seg]), hlast = static_cast<T>(a.seg_hlast[seg]);
  const T hfull = static_cast<T>(a.h);
  const T q = static_cast<T>(a.q);
  const int e0 = lane * EPL;
  // The lane marches the energies es .. es + EPL - 1.  Its own start at e0;
  // a lane at the end of the range (e0 + EPL > n_e) starts early enough that
  // all EPL exist (the host never launches EPL > n_e).  The energies below
  // e0 belong to the lane before it, whose values it reproduces exactly
  // (same constants, same start): its loads and stores then cover EPL
  // consecutive entries, and its duplicates carry no weight and write no
  // end values.
  const int es = min(e0, a.n_e - EPL);
  bool own[EPL];
  for (int i = 0; i < EPL; ++i) own[i] = es + i >= e0;

  T ex[EPL], ey[EPL];
  // interior steps (length h): Kx = (-h Im z - 1)/2 and its square per energy
  T kxi[EPL], kx2i[EPL];
  for (int i = 0; i < EPL; ++i) {
    const int e = es + i;
    ex[i] = static_cast<T>(a.eps[2 * (a.e_off + e)]);
    ey[i] = static_cast<T>(a.eps[2 * (a.e_off + e) + 1]);
    kxi[i] = fmaT(T(-0.5) * hfull, ey[i], T(-0.5));
    kx2i[i] = kxi[i] * kxi[i];
  }
  const T hh = T(0.5) * hfull, hq8 = T(0.125) * hfull, hqa = T(0.25) * q * hfull;

  // Step with the half-step values (mean of two slots; sd = -1 applies
  // D -> -D* for gamma~).  End steps take every constant from their length.
  auto end_step = [&](cpx<T>* gv, const node4<T>& pv, const node4<T>& cv, T hs, T sd) {
    const T h8 = T(0.125) * hs;
    StepC<T> c;
    c.c2x = h8 * (pv.dy + cv.dy);
    c.c2y = h8 * (sd * (pv.dx + cv.dx));
    c.U0x = T(-4) * c.c2x;
    c.U0y = T(4) * c.c2y;
    const T qa = T(0.5) * q * (pv.a + cv.a);
    for (int i = 0; i < EPL; ++i) {
      const T kx = fmaT(T(-0.5) * hs, ey[i], T(-0.5));
      gv[i] = riccati_step_c(gv[i], c, kx, kx * kx, T(0.5) * hs * (qa + ex[i]));
    }
  };
  auto mid_step = [&](cpx<T>* gv, const node4<T>& pv, const node4<T>& cv, T sd) {
    StepC<T> c;
    c.c2x = hq8 * (pv.dy + cv.dy);
    c.c2y = hq8 * (sd * (pv.dx + cv.dx));
    c.U0x = T(-4) * c.c2x;
    c.U0y = T(4) * c.c2y;
    const T hq = hqa * (pv.a + cv.a);
    for (int i = 0; i < EPL; ++i) gv[i] = riccati_step_c(gv[i], c, kxi[i], kx2i[i], fmaT(hh, ex[i], hq));
  };

  // ---- gamma: R_min -> R_max
  cpx<T> g[EPL];
  // the segment's slot values; indexed with unsigned 32-bit offsets, which
  // widen to the 64-bit address without a sign extension
  const node4<T>* const nseg = nodes + slot0;
  node4<T> prev = nseg[0];
  {
    const int64_t tb = seg * 4;
    const double wsum = a.tap_start_w[tb] + a.tap_start_w[tb + 1] + a.tap_start_w[tb + 2] + a.tap_start_w[tb + 3];
    if (a.bc_valid && wsum > 0.0) {
      for (int i = 0; i < EPL; ++i) g[i] = mk(T(0), T(0));
      for (int c = 0; c < 4; ++c) {
        const T w = static_cast<T>(a.tap_start_w[tb + c]);
        const cpx<T>* src = bc_g_prev + static_cast<int64_t>(a.tap_start_seg[tb + c]) * a.n_e_tot + a.e_off;
        for (int i = 0; i < EPL; ++i) {
          const cpx<T> v = src[es + i];
          g[i] = mk(g[i].x + w * v.x, g[i].y + w * v.y);
        }
      }
    } else {
      const T qa = q * prev.a;
      for (int i = 0; i < EPL; ++i) g[i] = bulk_root(qa + ex[i], ey[i], prev.dx, prev.dy);
    }
  }
  // gamma spill of this segment, node t at gseg[t * n_e]: the grain's array
  // (gmul = n_e) or a wave's own scratch (gmul = 0); this lane's entries
  // start at gseg + es
  cpx<T>* const gseg = gbase + slot0 * gmul;
  cpx<T>* const glane = gseg + es;
  // Every lane stores all its EPL entries (a duplicate writes the value its
  // owner writes).  With no conditional stores the compiler knows how many
  // stores were issued after a prefetch and waits for the prefetch alone.
  auto store_g = [&](int t) {
    cpx<T>* dst = glane + static_cast<int64_t>(t) * a.n_e;
    for (int i = 0; i < EPL; ++i) dst[i] = g[i];
  };
  // Slot values are loaded one step ahead, so the load overlaps a step.  A
  // wait for that load must not also wait for a gamma store issued just
  // before it: in FP32 the stores close each step, and the loop is entered
  // as it repeats (prefetch, then two stores), so the compiler waits for the
  // prefetch alone; in FP64, where the compiler sinks the first prefetch
  // below step 0's store, a node's gamma is stored in the next step, right
  // after that step's prefetch.
  constexpr bool late_store = sizeof(T) == 4;
  node4<T> nxt = nseg[static_cast<uint32_t>(min(1, last))];
  // step 0 from R_min (the boundary point takes slot 0's values); a segment
  // with no node still owns one slot, so its store is in range
  end_step(g, prev, prev, hfirst, T(1));
  if (late_store && MODE != 2) store_g(0);
  // (FP32: two steps per loop turn, so the look-ahead registers rotate by
  // renaming instead of moves; in FP64 that would cost a wave per SIMD)
  constexpr int kUnrollG = sizeof(T) == 4 ? 2 : 1;
#pragma unroll kUnrollG
  for (int t = 1; t < n; ++t) {
    const node4<T> cur = nxt;
    nxt = nseg[static_cast<uint32_t>(min(t + 1, last))];
    if (!late_store && MODE != 2) store_g(t - 1);
    mid_step(g, prev, cur, T(1));
    prev = cur;
    if (late_store && MODE != 2) store_g(t);
  }
  if (!late_store && MODE != 2 && n > 0) store_g(n - 1);
  // step n to R_max (the boundary point takes slot n-1's values)
  if (n > 0) end_step(g, prev, prev, hlast, T(1));
  // end values for the next sweep (the LDOS output pass writes them only
  // when iterating to convergence: bc_g_next given)
  if (MODE == 0 || MODE == 2 || (MODE == 1 && bc_g_next)) {
    cpx<T>* dst = bc_g_next + seg * a.n_e_tot + a.e_off + es;
    for (int i = 0; i < EPL; ++i)
      if (own[i]) dst[i] = g[i];
  }

  // ---- gamma~: R_max -> R_min with D -> -D*
  // pole weights R_p of the lane's energies (0 for padding), kept in FP64:
  // the gap denominator holds them exactly, and rounding them to FP32 in
  // the node sums would bias every gap update the same way
  double rw[EPL];
  for (int i = 0; i < EPL; ++i)
    rw[i] = (MODE == 0 && own[i]) ? a.rp[a.e_off + es + i] : 0.0;
  cpx<T> gt[EPL];
  prev = nseg[static_cast<uint32_t>(last)];
  {
    const int64_t tb = seg * 4;
    const double wsum = a.tap_end_w[tb] + a.tap_end_w[tb + 1] + a.tap_end_w[tb + 2] + a.tap_end_w[tb + 3];
    if (a.bc_valid && wsum > 0.0) {
      for (int i = 0; i < EPL; ++i) gt[i] = mk(T(0), T(0));
      for (int c = 0; c < 4; ++c) {
        const T w = static_cast<T>(a.tap_end_w[tb + c]);
        const cpx<T>* src = bc_gt_prev + static_cast<int64_t>(a.tap_end_seg[tb + c]) * a.n_e_tot + a.e_off;
        for (int i = 0; i < EPL; ++i) {
          const cpx<T> v = src[es + i];
          gt[i] = mk(gt[i].x + w * v.x, gt[i].y + w * v.y);
        }
      }
    } else {
      const T qa = q * prev.a;
      for (int i = 0; i < EPL; ++i) gt[i] = bulk_root(qa + ex[i], ey[i], -prev.dx, prev.dy);
    }
  }

  // Per node and pole (Sec. II.A), with X = gamma gamma~ and I = 1/(1+X):
  //   f + conj f~ = -2 i pi [Re((gamma + gamma~) I) + i Im((gamma - gamma~) I)],
  //   Re g = pi Im((1-X)/(1+X)) = 2 pi Im I,
  //   (D* f + D f~) / (pi + i g) = i (D gamma~ - D* gamma)  since pi + i g = 2 pi I,
  // so the Eilenberger free-energy term needs no division.
  // gamma of a node for this lane's energies
  auto load_g = [&](cpx<T>* gv, int t) {
    const cpx<T>* src = glane + static_cast<int64_t>(t) * a.n_e;
    for (int i = 0; i < EPL; ++i) gv[i] = src[i];
  };
  // Node sums through LDS (MODE 0, G >= 8).  The wave's buffer holds two
  // nodes x four components x 64 lanes; slot b of component c of lane l is
  // lsum[b * 256 + c * 64 + l].  Lanes of one wave see each other's LDS
  // writes in issue order; the fences keep the compiler from moving the
  // accesses across each other.  Every lane of a group then takes one
  // (node, component) output and a block of 8 partials, and P = G / 8
  // neighbouring lanes finish it with quad moves.
  auto lds_reduce = [&](int64_t node0, int cnt) {
    const int l64 = threadIdx.x & 63;
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    const int lp = lg - 3;  // log2 P
    const int o = lane >> lp, r = lane & ((1 << lp) - 1);
    const double2* src = reinterpret_cast<const double2*>(lsum + o * 64 + (l64 - lane));
    // partials of lanes 8 r .. 8 r + 7 of the group
    const double2 x0 = src[r << 2];
    double v = x0.x + x0.y;
    for (int j = 1; j < 4; ++j) {
      const double2 x = src[(r << 2) + j];
      v += x.x + x.y;
    }
    if (lp >= 1) v += dpp_f64<0xB1>(v);   // quad_perm [1,0,3,2]
    if (lp >= 2) v += dpp_f64<0x4E>(v);   // quad_perm [2,3,0,1]
    if (lp >= 3) v += dpp_f64<0x141>(v);  // row_half_mirror: lane 0 of 8 adds lane 7
    __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    // slot b = o >> 2 holds node0 - b; component o & 3
    if (r == 0 && (o >> 2) < cnt) a.node_out[(node0 - (o >> 2)) * 4 + (o & 3)] = a.twopi_tt * v;
  };
  // k counts the nodes visited before this one (the same for every group of
  // the wave, since all groups start their march together)
  auto node_sums = [&](int64_t node, const node4<T>& nv, const cpx<T>* gn, int k) {
    if (MODE == 0) {
      double sfx, sfy, sg, si;
      if constexpr (sizeof(T) == 4) {
        // mixed precision: each pole's terms are formed from the FP32
        // marches, weighted by R_p and summed over poles in FP64
        for (int i = 0; i < EPL; ++i) {
          const cpx<T> gg = gn[i];
          const T xx = fmaT(gg.x, gt[i].x, -(gg.y * gt[i].y));
          const T xy = fmaT(gg.x, gt[i].y, gg.y * gt[i].x);
          const T dxr = T(1) + xx;
          // I = 1/(1+X) = (dxr - i xy) u with u = 1 / |1+X|^2
          const T u = drcp(fmaT(dxr, dxr, xy * xy));
          const T ix = dxr * u, iy = xy * u;  // I = ix - i iy
          const T sxs = gg.x + gt[i].x, sys = gg.y + gt[i].y;
          const T dxs = gg.x - gt[i].x, dys = gg.y - gt[i].y;
          const double tfx = static_cast<double>(fmaT(sxs, ix, sys * iy));     // Re((gamma + gamma~) I)
          const double tfy = static_cast<double>(fmaT(dys, ix, -(dxs * iy)));  // Im((gamma - gamma~) I)
          const double tg = static_cast<double>(iy);                           // -Im I
          const double ti = static_cast<double>(fmaT(nv.dx, dys, -(nv.dy * sxs)));  // Im(D* gamma - D gamma~)
          if (i == 0) {
            sfx = rw[0] * tfx;
            sfy = rw[0] * tfy;
            sg = -rw[0] * tg;
            si = rw[0] * ti;
          } else {
            sfx = __builtin_fma(rw[i], tfx, sfx);
            sfy = __builtin_fma(rw[i], tfy, sfy);
            sg = __builtin_fma(-rw[i], tg, sg);
            si = __builtin_fma(rw[i], ti, si);
          }
        }
      } else {
        T pfx = T(0), pfy = T(0), pg = T(0), p1 = T(0), p2 = T(0);
        for (int i = 0; i < EPL; ++i) {
          const cpx<T> gg = gn[i];
          const T xx = fmaT(gg.x, gt[i].x, -(gg.y * gt[i].y));
          const T xy = fmaT(gg.x, gt[i].y, gg.y * gt[i].x);
          const T dxr = T(1) + xx;
          // I = 1/(1+X) = (dxr - i xy) u / R with u = R / |1+X|^2 (R the pole weight)
          const T r = static_cast<T>(rw[i]);
          const T u = r * drcp(fmaT(dxr, dxr, xy * xy));
          const T sxs = gg.x + gt[i].x, sys = gg.y + gt[i].y;
          const T dxs = gg.x - gt[i].x, dys = gg.y - gt[i].y;
          pfx = fmaT(u, fmaT(sxs, dxr, sys * xy), pfx);     // R Re((gamma + gamma~) I)
          pfy = fmaT(u, fmaT(dys, dxr, -(dxs * xy)), pfy);  // R Im((gamma - gamma~) I)
          pg = fmaT(-u, xy, pg);                            // R Im I
          p1 = fmaT(r, dys, p1);
          p2 = fmaT(r, sxs, p2);
        }
        sfx = pfx;
        sfy = pfy;
        sg = pg;
        // Im(D* gamma - D gamma~) summed over the lane's poles
        si = fmaT(nv.dx, p1, -(nv.dy * p2));
      }
      // S_f = -2 i pi t~ (sfx + i sfy), S_g = 2 pi t~ sg, S_I = 2 pi t~ si
      if (G >= 8) {
        // the lane's four partials go to LDS; every second node the group
        // sums the pair (this node and the one before it, node + 1)
        const int b = k & 1;
        double* w = lsum + b * 256 + (threadIdx.x & 63);
        w[0] = sfy;
        w[64] = -sfx;
        w[128] = sg;
        w[192] = si;
        if (b) lds_reduce(node + 1, 2);
      } else if (G >= 4) {
        // lane q of the group (q < 4) ends with component q of the node's sums
        const double v = group_sum4_scatter(sfy, -sfx, sg, si, G, lane);
        if (lane < 4) a.node_out[node * 4 + scatter_index(lane)] = a.twopi_tt * v;
      } else {
        const double ox = group_sum(sfy, G), oy = group_sum(sfx, G);
        const double oz = group_sum(sg, G), ow = group_sum(si, G);
        if (lane == 0) {
          double4 o;
          o.x = a.twopi_tt * ox;
          o.y = -a.twopi_tt * oy;
          o.z = a.twopi_tt * oz;
          o.w = a.twopi_tt * ow;
          reinterpret_cast<double4*>(a.node_out)[node] = o;
        }
      }
    } else if (MODE == 1) {  // N/N_F = -Im g / pi = Re((1-X)/(1+X)) = 2 Re I - 1 per energy
      T* dst = ebuf + node * a.n_e + es;
      for (int i = 0; i < EPL; ++i) {
        if (!own[i]) continue;
        const cpx<T> gg = gn[i];
        const T xx = fmaT(gg.x, gt[i].x, -(gg.y * gt[i].y));
        const T xy = fmaT(gg.x, gt[i].y, gg.y * gt[i].x);
        const T dxr = T(1) + xx;
        const T ri = drcp(fmaT(dxr, dxr, xy * xy));
        dst[i] = fmaT(T(2) * dxr, ri, T(-1));
      }
    } else {  // MODE 3: (1-X)/(1+X) = 2 I - 1 per energy, complex (g = -i pi times it)
      T* dst = ebuf + 2 * (node * a.n_e + es);
      for (int i = 0; i < EPL; ++i) {
        if (!own[i]) continue;
        const cpx<T> gg = gn[i];
        const T xx = fmaT(gg.x, gt[i].x, -(gg.y * gt[i].y));
        const T xy = fmaT(gg.x, gt[i].y, gg.y * gt[i].x);
        const T dxr = T(1) + xx;
        const T ri = drcp(fmaT(dxr, dxr, xy * xy));
        dst[2 * i] = fmaT(T(2) * dxr, ri, T(-1));
        dst[2 * i + 1] = T(-2) * xy * ri;
      }
    }
  };

  // step n from R_max (boundary point = slot n-1; the whole segment if n = 0)
  cpx<T> gn[EPL];
  if (MODE != 2) load_g(gn, last);
  end_step(gt, prev, prev, n > 0 ? hlast : hfirst, T(-1));
  if (MODE != 2 && n > 0) node_sums(slot0 + n - 1, prev, gn, 0);
  // slot values and gamma are loaded one step ahead, so the loads overlap
  // a step (gamma comes back from HBM: it was written a whole march ago)
  // (FP32 only: in FP64 the registers would cost a wave per SIMD)
  constexpr bool gpre = MODE != 2 && sizeof(T) == 4;
  // (the prefetched row, max(t - 2, 0) at step t, is walked down with a
  // pointer rather than formed from t, which costs 64-bit multiplies)
  nxt = nseg[static_cast<uint32_t>(max(n - 2, 0))];
  cpx<T> gnx[EPL];
  const cpx<T>* grow = glane + static_cast<int64_t>(max(n - 2, 0)) * a.n_e;
  auto load_row = [&](cpx<T>* gv, const cpx<T>* row) {
    for (int i = 0; i < EPL; ++i) gv[i] = row[i];
  };
  if (gpre) load_row(gnx, grow);
  for (int t = n - 1; t >= 1; --t) {
    const node4<T> cur = nxt;
    nxt = nseg[static_cast<uint32_t>(max(t - 2, 0))];
    if (gpre) {
      for (int i = 0; i < EPL; ++i) gn[i] = gnx[i];
      if (t >= 2) grow -= a.n_e;
      load_row(gnx, grow);
    } else if (MODE != 2) {
      load_g(gn, t - 1);
    }
    mid_step(gt, prev, cur, T(-1));
    prev = cur;
    if (MODE != 2) node_sums(slot0 + t - 1, cur, gn, n - t);
  }
  // with an odd node count, node 0 is left alone in slot 0
  if (MODE == 0 && G >= 8 && (n & 1)) lds_reduce(slot0, 1);
  // step 0 to R_min (boundary point = slot 0)
  if (n > 0) end_step(gt, prev, prev, hfirst, T(-1));
  if (MODE == 0 || MODE == 2 || (MODE == 1 && bc_gt_next)) {
    cpx<T>* dst = bc_gt_next + seg * a.n_e_tot + a.e_off + es;
    for (int i = 0; i < EPL; ++i)
      if (own[i]) dst[i] = gt[i];
  }
}

// Occupancy floors (waves per SIMD) for the FP32 variants: 7 (<= 72 VGPRs)
// with two energies per lane (the spills, gamma look-ahead included, stay
// outside the loops; 6 waves without spills ran slower); with four,
// 4 (<= 128) for the pole-sum sweep, which spills in its loops at 5, and 5
// for the other modes; the rest keep the compiler's default.
template <typename T, int EPL, int MODE>
constexpr int sweep_min_waves() {
  return (sizeof(T) == 4 && EPL == 4) ? (MODE == 0 ? 4 : 5) : (sizeof(T) == 4 && EPL == 2) ? 7 : 1;
}

template <typename T, int EPL, int MODE>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sweep_min_waves<T, EPL, MODE>())))
sweep_kernel(SweepArgs a, const node4<T>* __restrict__ nodes,
                                                    const cpx<T>* __restrict__ bc_g_prev,
                                                    const cpx<T>* __restrict__ bc_gt_prev,
                                                    cpx<T>* __restrict__ bc_g_next,
                                                    cpx<T>* __restrict__ bc_gt_next,
                                                    cpx<T>* __restrict__ gbuf, T* __restrict__ ebuf) {
  const int64_t gtid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  double* lsum = nullptr;
  if constexpr (MODE == 0) {
    __shared__ double red[4 * 512];  // two nodes x four sums x 64 lanes per wave
    lsum = red + (threadIdx.x >> 6) * 512;
  }
  // The launch order is longest first.  In a launch that fills the device's
  // wave slots about once, the longest segments set its length; the first
  // nlong of them march with twice the lanes and half the energies per lane,
  // so they finish in about half the time.  The split falls on a wave
  // boundary (nlong * 2G is a multiple of 64), so each wave takes one shape.
  int64_t r = gtid, first = 0;
  if constexpr (MODE == 0 && EPL % 2 == 0) {
    first = a.nlong;
    const int64_t nl = a.nlong << (a.log2g + 1);
    if (r < nl) {
      sweep_segment<T, EPL / 2, MODE>(a, r >> (a.log2g + 1), static_cast<int>(r & (2 * a.G - 1)), 2 * a.G,
                                      a.log2g + 1, nodes, bc_g_prev, bc_gt_prev, bc_g_next, bc_gt_next, gbuf, a.n_e,
                                      ebuf, lsum);
      return;
    }
    r -= nl;
  }
  const int64_t wseg = first + (r >> a.log2g);
  const int lane = static_cast<int>(r & (a.G - 1));
  if (wseg >= a.nseg) return;  // whole lane groups leave together (G | 64)
  sweep_segment<T, EPL, MODE>(a, wseg, lane, a.G, a.log2g, nodes, bc_g_prev, bc_gt_prev, bc_g_next, bc_gt_next,
                              gbuf, a.n_e, ebuf, lsum);
}

// Batched grains: one persistent launch.  Every wave pulls tiles (a grain
// and a bundle of 64/G of its segments) from a queue sorted by cost until
// the queue is empty; every wave reaches that exit.  The gamma spill of a
// tile lives only between its two marches, so each wave keeps it in its own
// slice of `spill` (wave_elems records; segment k of the tile at
// k * maxn * n_e), reused tile after tile: the spill memory is set by the
// resident waves, not by the number or size of the grains.
template <typename T, int EPL>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(sweep_min_waves<T, EPL, 0>())))
batch_sweep_kernel(const BatchGrainDev* __restrict__ grains,
                                                          const int2* __restrict__ tiles, int ntiles,
                                                          int* __restrict__ counter, cpx<T>* __restrict__ spill,
                                                          int64_t wave_elems) {
  const int l64 = threadIdx.x & 63;
  cpx<T>* const wspill = spill + (static_cast<int64_t>(blockIdx.x) * 4 + (threadIdx.x >> 6)) * wave_elems;
  __shared__ double red[4 * 512];  // node-sum exchange, two nodes x four sums x 64 lanes per wave
  while (true) {
    int t = 0;
    if (l64 == 0) t = atomicAdd(counter, 1);
    // all 64 lanes are active here, so the first active lane is lane 0; the
    // tile index becomes wave-uniform and the grain's arguments scalar loads
    t = __builtin_amdgcn_readfirstlane(t);
    if (t >= ntiles) break;
    const int2 tile = tiles[t];
    const BatchGrainDev& gd = grains[tile.x];
    const int64_t wseg = static_cast<int64_t>(tile.y) + (l64 >> gd.a.log2g);
    if (wseg < gd.a.nseg)
      sweep_segment<T, EPL, 0>(gd.a, wseg, l64 & (gd.a.G - 1), gd.a.G, gd.a.log2g, static_cast<const node4<T>*>(gd.b.nodes),
                               static_cast<const cpx<T>*>(gd.b.bc_g_prev), static_cast<const cpx<T>*>(gd.b.bc_gt_prev),
                               static_cast<cpx<T>*>(gd.b.bc_g_next), static_cast<cpx<T>*>(gd.b.bc_gt_next),
                               wspill + static_cast<int64_t>(l64 >> gd.a.log2g) * gd.a.maxn * gd.a.n_e, 0, nullptr,
                               red + (threadIdx.x >> 6) * 512);
  }
}

__global__ void reset_counter_kernel(int* counter) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *counter = 0;
}

// --------------------------------------------------------------------------
// rotate back + angle sums + gap / current / free energy
// --------------------------------------------------------------------------
// A block of kBackWaves waves shares 64 grain cells: wave w takes the angles
// k = w, w + kBackWaves, ... for all of them, so each load of a wave gathers
// the lattice corners of 64 neighbouring cells at one angle; the waves'
// partial angle sums meet in LDS.
constexpr int kBackWaves = 4;
constexpr int kBackFields = 12;  // 2 x (up to 4 components) + jx, jy, I, <|Delta|^2>

// NC = 1: one order-parameter component (its arrays in fixed registers);
// NC = 4: a.ncomp <= 4 components
template <int NC>
__global__ void __launch_bounds__(64 * kBackWaves) rotate_back_kernel(BackArgs a) {
  __shared__ double part[kBackWaves - 1][kBackFields][64];
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  // each XCD takes a contiguous band of grain cells: neighbouring cells share
  // lattice corners, which then meet in the same L2
  const int64_t c = xcd_block(blockIdx.x, gridDim.x) * 64 + lane;
  const bool live = c < a.ncg;
  const int cell = live ? a.grain_cells[c] : 0;
  constexpr int MAXC = NC;
  const int ncomp = NC == 1 ? 1 : a.ncomp;
  double nx_[MAXC], ny_[MAXC], dx_[MAXC], dy_[MAXC];
  for (int g = 0; g < ncomp; ++g) {
    nx_[g] = 0.0;
    ny_[g] = 0.0;
    dx_[g] = a.delta[2 * (static_cast<int64_t>(g) * a.ncell + cell)];
    dy_[g] = a.delta[2 * (static_cast<int64_t>(g) * a.ncell + cell) + 1];
  }
  // cell centre relative to the grid centre, as the plan forms it
  const double rx = rn_cell_offset(a.x0, static_cast<double>(cell % a.nx), a.h, a.cx);
  const double ry = rn_cell_offset(a.y0, static_cast<double>(cell / a.nx), a.h, a.cy);
  const double4* nsum = reinterpret_cast<const double4*>(a.node_out);
  double jx = 0.0, jy = 0.0, icell = 0.0, d2avg = 0.0;
  // angle kk's share of the sums from the node sums gathered at its corners
  // (sgn: the sign of S_g, -1 for the reversed direction of a pair)
  auto add_angle = [&](int kk, double cfx, double cfy, double cg, double ci) {
    const double wk = a.wk[kk];
    double dkx = 0.0, dky = 0.0;
    for (int g = 0; g < ncomp; ++g) {
      const double ex = a.eta[2 * (g * a.n_theta + kk)], ey = a.eta[2 * (g * a.n_theta + kk) + 1];
      const double px = wk * ex, py = -wk * ey;  // wk conj(eta)
      nx_[g] += px * cfx - py * cfy;
      ny_[g] += px * cfy + py * cfx;
      dkx += ex * dx_[g] - ey * dy_[g];
      dky += ex * dy_[g] + ey * dx_[g];
    }
    jx += a.four_q * wk * a.cosk[kk] * cg;
    jy += a.four_q * wk * a.sink[kk] * cg;
    icell += wk * ci;
    d2avg += wk * (dkx * dkx + dky * dky);
  };
  // with pair_fold each gather of a lower angle serves its upper angle too
  const int kend = a.pair_fold ? a.pair_k0 : a.n_theta;
  // the corner record of the wave's next angle is loaded one iteration
  // ahead, so only the node-sum gathers wait in each iteration
  int k = live ? wv : kend;
  int4 ixn = make_int4(0, 0, 0, 0);
  if (k < kend) ixn = a.rb4[static_cast<int64_t>(k) * a.ncg + c];
  for (; k < kend; k += kBackWaves) {
    const int4 ix = ixn;
    if (k + kBackWaves < kend) ixn = a.rb4[static_cast<int64_t>(k + kBackWaves) * a.ncg + c];
    const double epx = a.cosk[k], epy = a.sink[k];
    // lattice coordinates (line u, node v) of the cell centre
    const double u = rn_lattice(rx, epy, ry, -epx, a.h, a.half);
    const double v = rn_lattice(rx, epx, ry, epy, a.h, a.half);
    const double wu = u - __builtin_floor(u), wv = v - __builtin_floor(v);
    double w[4] = {(1 - wu) * (1 - wv), wu * (1 - wv), (1 - wu) * wv, wu * wv};
    int sl[4] = {ix.x, ix.y, ix.z, ix.w};
    if (ix.y == -2) {  // no lattice corner is a node: the nearest node alone
      w[0] = 1.0;
      w[1] = w[2] = w[3] = 0.0;
    }
    // corners that are not nodes read slot 0 with weight 0, so the four
    // gathers issue together
    double tot = 0.0;
    for (int qd = 0; qd < 4; ++qd) {
      if (sl[qd] < 0) {
        w[qd] = 0.0;
        sl[qd] = 0;
      }
      tot += w[qd];
    }
    const double rt = (ix.x | ix.y | ix.z | ix.w) < 0 ? 1.0 / tot : 1.0;
    double cfx = 0.0, cfy = 0.0, cg = 0.0, ci = 0.0;
    for (int qd = 0; qd < 4; ++qd) {
      const double4 vv = nsum[sl[qd]];
      const double wq = w[qd] * rt;
      cfx += vv.x * wq;
      cfy += vv.y * wq;
      cg += vv.z * wq;
      ci += vv.w * wq;
    }
    // S_g of the reversed direction changes sign; S_f and S_I do not
    add_angle(k, cfx, cfy, k >= a.pair_k0 ? -cg : cg, ci);
    if (a.pair_fold) add_angle(k + a.pair_k0, cfx, cfy, -cg, ci);
  }
  if (wv > 0) {
    double* p = &part[wv - 1][0][lane];
    for (int g = 0; g < ncomp; ++g) {
      p[64 * (2 * g)] = nx_[g];
      p[64 * (2 * g + 1)] = ny_[g];
    }
    p[64 * 8] = jx;
    p[64 * 9] = jy;
    p[64 * 10] = icell;
    p[64 * 11] = d2avg;
  }
  __syncthreads();
  if (wv > 0 || !live) return;
  for (int w = 0; w < kBackWaves - 1; ++w) {
    const double* p = &part[w][0][lane];
    for (int g = 0; g < ncomp; ++g) {
      nx_[g] += p[64 * (2 * g)];
      ny_[g] += p[64 * (2 * g + 1)];
    }
    jx += p[64 * 8];
    jy += p[64 * 9];
    icell += p[64 * 10];
    d2avg += p[64 * 11];
  }
  double om = 0.0;
  for (int g = 0; g < ncomp; ++g) {
    a.delta_new[2 * (static_cast<int64_t>(g) * a.ncell + cell)] = nx_[g] / a.den[g];
    a.delta_new[2 * (static_cast<int64_t>(g) * a.ncell + cell) + 1] = ny_[g] / a.den[g];
    om += (dx_[g] * dx_[g] + dy_[g] * dy_[g]) * a.logt[g];
  }
  om += a.twopi_rz * d2avg - icell;
  a.j[cell] = jx;
  a.j[a.ncell + cell] = jy;
  if (a.omega) a.omega[cell] = om;
  a.omega_cell[c] = om;
}

// gamma~ along a line is the conjugate of gamma along the reversed line
// (even order parameter): the end values of the upper angle of a pair follow
// from its mirror segment's
template <typename T>
__global__ void __launch_bounds__(256) mirror_fill_kernel(const int2* __restrict__ pairs, int64_t npairs, int n_e,
                                                          const int32_t* __restrict__ partner,
                                                          cpx<T>* __restrict__ bc_g, cpx<T>* __restrict__ bc_gt) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= npairs * n_e) return;
  const int64_t q = t / n_e;
  const int e = static_cast<int>(t - q * n_e);
  const int2 pr = pairs[q];
  // real energies: the reversed direction at e mirrors energy -e (partner)
  const int es = partner ? partner[e] : e;
  const int64_t dst = static_cast<int64_t>(pr.x) * n_e + e, src = static_cast<int64_t>(pr.y) * n_e + es;
  const cpx<T> g = bc_g[src], gt = bc_gt[src];
  bc_g[dst] = mk(gt.x, -gt.y);
  bc_gt[dst] = mk(g.x, -g.y);
}

template <typename T>
__global__ void __launch_bounds__(256) ldos_back_kernel(LdosBackArgs a, const T* __restrict__ ebuf) {
  // thread per (grain cell, energy of the block), energy fastest
  const int64_t tid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t c = tid / a.n_e;
  const int e = static_cast<int>(tid - c * a.n_e);
  if (c >= a.ncg) return;
  // with fold_k0 each lower angle's corners serve its upper angle too, at
  // the partner energy (N of the reversed direction at e is N at -e)
  const bool fold = a.fold_k0 > 0;
  const int kend = fold ? a.fold_k0 : a.n_theta;
  const int ep = fold ? a.e_partner[a.e_off + e] - a.e_off : e;
  double acc = 0.0;
  for (int k = 0; k < kend; ++k) {
    double v = 0.0, vp = 0.0;
    for (int qd = 0; qd < 4; ++qd) {
      const int64_t o = (static_cast<int64_t>(k) * 4 + qd) * a.ncg + c;
      const int64_t row = static_cast<int64_t>(a.rb_idx[o]) * a.n_e;
      const double w = a.rb_w[o];
      v += static_cast<double>(ebuf[row + e]) * w;
      if (fold) vp += static_cast<double>(ebuf[row + ep]) * w;
    }
    acc += a.wk[k] * v;
    if (fold) acc += a.wk[k + a.fold_k0] * vp;
  }
  const int64_t eo = a.e_map ? a.e_map[a.e_off + e] : a.e_off + e;
  a.out[eo * a.ncell + a.grain_cells[c]] = acc;
}

// Fermi-surface average of g = -i pi (1-X)/(1+X) per cell and energy of the
// block: the rotate-back of the complex per-node values of sweep mode 3
template <typename T>
__global__ void __launch_bounds__(256) green_back_kernel(LdosBackArgs a, const T* __restrict__ ebuf) {
  const int64_t tid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t c = tid / a.n_e;
  const int e = static_cast<int>(tid - c * a.n_e);
  if (c >= a.ncg) return;
  double ax = 0.0, ay = 0.0;
  for (int k = 0; k < a.n_theta; ++k) {
    double vx = 0.0, vy = 0.0;
    for (int qd = 0; qd < 4; ++qd) {
      const int64_t o = (static_cast<int64_t>(k) * 4 + qd) * a.ncg + c;
      const int64_t src = 2 * (static_cast<int64_t>(a.rb_idx[o]) * a.n_e + e);
      vx += static_cast<double>(ebuf[src]) * a.rb_w[o];
      vy += static_cast<double>(ebuf[src + 1]) * a.rb_w[o];
    }
    ax += a.wk[k] * vx;
    ay += a.wk[k] * vy;
  }
  const double pi = 3.14159265358979323846;
  double* o = a.out + 2 * (static_cast<int64_t>(a.e_off + e) * a.ncell + a.grain_cells[c]);
  o[0] = pi * ay;   // -i pi (ax + i ay)
  o[1] = -pi * ax;
}

// --------------------------------------------------------------------------
// grid helpers: zero fill, curl + magnetic energy, block reductions
// --------------------------------------------------------------------------
__global__ void fill_kernel(double* __restrict__ p, int64_t n, double v) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ void __launch_bounds__(256) curl_kernel(const double* __restrict__ A, double* __restrict__ B,
                                                   int nx, int ny, double h) {
  const int64_t c = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= static_cast<int64_t>(nx) * ny) return;
  const int i = static_cast<int>(c % nx), j = static_cast<int>(c / nx);
  const double* ax = A;
  const double* ay = A + static_cast<int64_t>(nx) * ny;
  double dyx, dxy;  // d_x A_y, d_y A_x
  if (i == 0)
    dyx = (ay[c + 1] - ay[c]) / h;
  else if (i == nx - 1)
    dyx = (ay[c] - ay[c - 1]) / h;
  else
    dyx = (ay[c + 1] - ay[c - 1]) / (2 * h);
  if (j == 0)
    dxy = (ax[c + nx] - ax[c]) / h;
  else if (j == ny - 1)
    dxy = (ax[c] - ax[c - nx]) / h;
  else
    dxy = (ax[c + nx] - ax[c - nx]) / (2 * h);
  B[c] = dyx - dxy;
}

// Block partial sums of f(x) (x gathered through idx when given): mode 0
// sum x, mode 1 sum x^2.  One partial per block written to part[blockIdx.x];
// the host adds them in order.
// Up to two sums per launch: blockIdx.y picks the row (BlockSumRow r0, r1);
// each row's partials are those a launch of its own would give.
__global__ void __launch_bounds__(256) block_sum_kernel(BlockSumRow r0, BlockSumRow r1) {
  const BlockSumRow& r = blockIdx.y == 0 ? r0 : r1;
  const double* __restrict__ x = r.x;
  const int32_t* __restrict__ idx = r.idx;
  const int64_t n = r.n;
  const int mode = r.mode;
  double* __restrict__ part = r.part;
  __shared__ double sh[256];
  double acc = 0.0;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const double v = x[idx ? idx[i] : i];
    acc += mode == 1 ? v * v : v;
  }
  sh[threadIdx.x] = acc;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) sh[threadIdx.x] += sh[threadIdx.x + s];
    __syncthreads();
  }
  if (threadIdx.x == 0) part[blockIdx.x] = sh[0];
}

// Luttinger-Ward free energy (Sec. II): the propagator term at one
// coupling lambda, 2 sum_G den_G Re(conj(Delta_G) Delta_new_G[lambda Delta])
// with den_G the gap-equation denominator, weighted into acc per grain cell
__global__ void __launch_bounds__(256) lw_accumulate_kernel(const double* __restrict__ delta,
                                                            const double* __restrict__ dnew,
                                                            const int32_t* __restrict__ grain_cells, int64_t ncg,
                                                            int ncomp, int64_t ncell, const double* __restrict__ den,
                                                            double w, int first, double* __restrict__ acc) {
  const int64_t c = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= ncg) return;
  const int64_t cell = grain_cells[c];
  double v = 0.0;
  for (int g = 0; g < ncomp; ++g) {
    const int64_t o = 2 * (static_cast<int64_t>(g) * ncell + cell);
    v += den[g] * (delta[o] * dnew[o] + delta[o + 1] * dnew[o + 1]);
  }
  v *= 2.0 * w;
  acc[c] = first ? v : acc[c] + v;
}

// The terms of the free-energy density before the propagator term,
// sum_G |Delta_G|^2 ln(t / t_c,G) + 2 pi sum_p (R_p / z_p) <|Delta(p)|^2>,
// minus the lambda integral of the propagator term
__global__ void __launch_bounds__(256) lw_finish_kernel(const double* __restrict__ delta,
                                                        const int32_t* __restrict__ grain_cells, int64_t ncg,
                                                        int ncomp, int64_t ncell, int n_theta,
                                                        const double* __restrict__ eta, const double* __restrict__ wk,
                                                        const double* __restrict__ logt, double twopi_rz,
                                                        const double* __restrict__ acc,
                                                        double* __restrict__ omega_cell, double* __restrict__ omega) {
  const int64_t c = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= ncg) return;
  const int64_t cell = grain_cells[c];
  double dx[4], dy[4], base = 0.0;
  for (int g = 0; g < ncomp; ++g) {
    dx[g] = delta[2 * (static_cast<int64_t>(g) * ncell + cell)];
    dy[g] = delta[2 * (static_cast<int64_t>(g) * ncell + cell) + 1];
    base += (dx[g] * dx[g] + dy[g] * dy[g]) * logt[g];
  }
  double d2 = 0.0;
  for (int k = 0; k < n_theta; ++k) {
    double px = 0.0, py = 0.0;
    for (int g = 0; g < ncomp; ++g) {
      const double ex = eta[2 * (g * n_theta + k)], ey = eta[2 * (g * n_theta + k) + 1];
      px += ex * dx[g] - ey * dy[g];
      py += ex * dy[g] + ey * dx[g];
    }
    d2 += wk[k] * (px * px + py * py);
  }
  const double om = base + twopi_rz * d2 - acc[c];
  omega_cell[c] = om;
  if (omega) omega[cell] = om;
}

__global__ void __launch_bounds__(256) scale_kernel(const double* __restrict__ x, double s, int64_t n,
                                                    double* __restrict__ y) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n) y[i] = s * x[i];
}

// Partial p-norms of (new - old) and of old over `n` elements of `stride`
// doubles each (stride 2: complex modulus).  p = 1, 2, or 0 (max).
// Elements may be gathered through idx (grain cells) when idx != nullptr,
// for `nrep` consecutive fields of `field_stride` elements.
// up to three independent fields per launch, picked by blockIdx.y
__global__ void __launch_bounds__(256) diff_norm_kernel(DiffNormArgs a0, DiffNormArgs a1, DiffNormArgs a2) {
  const DiffNormArgs& a = blockIdx.y == 0 ? a0 : (blockIdx.y == 1 ? a1 : a2);
  __shared__ double s0[256], s1[256];
  double acc0 = 0.0, acc1 = 0.0;
  const int64_t total = a.n * a.nrep;
  for (int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < total;
       t += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t r = t / a.n, i = t - r * a.n;
    const int64_t e = r * a.field_stride + (a.idx ? a.idx[i] : i);
    double dn = 0.0, dd = 0.0;
    for (int c = 0; c < a.stride; ++c) {
      const int64_t k = e * a.stride + c;
      const double vn = a.xnew[k], vo = a.xold[k];
      const double d = vn - vo;
      if (a.vel) {  // the heavy-ball step
        const double step = (1.0 - a.beta) * a.vel[k] + a.alpha * d;
        a.vel[k] = step;
        a.update[k] = vo + step;
      } else if (a.update) {
        a.update[k] = vo + a.alpha * d;  // the Picard step
      }
      // the global error is of g(x) - x, before any step (Alg. 1)
      dn += d * d;
      dd += vo * vo;
    }
    if (a.p == 2) {
      acc0 += dn;
      acc1 += dd;
    } else if (a.p == 1) {
      acc0 += __builtin_sqrt(dn);
      acc1 += __builtin_sqrt(dd);
    } else {
      acc0 = fmax(acc0, __builtin_sqrt(dn));
      acc1 = fmax(acc1, __builtin_sqrt(dd));
    }
  }
  s0[threadIdx.x] = acc0;
  s1[threadIdx.x] = acc1;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if (threadIdx.x < s) {
      if (a.p == 0) {
        s0[threadIdx.x] = fmax(s0[threadIdx.x], s0[threadIdx.x + s]);
        s1[threadIdx.x] = fmax(s1[threadIdx.x], s1[threadIdx.x + s]);
      } else {
        s0[threadIdx.x] += s0[threadIdx.x + s];
        s1[threadIdx.x] += s1[threadIdx.x + s];
      }
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    a.part[2 * blockIdx.x] = s0[0];
    a.part[2 * blockIdx.x + 1] = s1[0];
  }
}

// x <- x + alpha (g - x) on n doubles (gathered through idx when given, for
// nrep fields of field_stride elements with `stride` doubles each)
__global__ void __launch_bounds__(256) picard_kernel(double* __restrict__ x, const double* __restrict__ gx,
                                                     const int32_t* __restrict__ idx, int64_t n, int nrep,
                                                     int64_t field_stride, int stride, double alpha) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n * nrep) return;
  const int64_t r = t / n, i = t - r * n;
  const int64_t e = r * field_stride + (idx ? idx[i] : i);
  for (int c = 0; c < stride; ++c) {
    const double v = x[e * stride + c];
    x[e * stride + c] = v + alpha * (gx[e * stride + c] - v);
  }
}

// Barzilai-Borwein dot products (App. E) over one field of the concatenated
// x: with d = scale (xnew - xold) and dp the previous iteration's d, block
// partials of dp.dp, dp.(d - dp) and (d - dp).(d - dp); dp <- d.
__global__ void __launch_bounds__(256) bb_dots_kernel(const double* __restrict__ xnew,
                                                      const double* __restrict__ xold,
                                                      const int32_t* __restrict__ idx, int64_t n, int nrep,
                                                      int64_t field_stride, int stride, double scale,
                                                      double* __restrict__ dprev, double* __restrict__ part) {
  __shared__ double sm[3][256];
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  const int64_t total = n * nrep;
  for (int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; t < total;
       t += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t r = t / n, i = t - r * n;
    const int64_t e = r * field_stride + (idx ? idx[i] : i);
    for (int c = 0; c < stride; ++c) {
      const int64_t k = e * stride + c;
      const double d = scale * (xnew[k] - xold[k]);
      const double pv = dprev[k];
      const double q = d - pv;
      a0 += pv * pv;
      a1 += pv * q;
      a2 += q * q;
      dprev[k] = d;
    }
  }
  sm[0][threadIdx.x] = a0;
  sm[1][threadIdx.x] = a1;
  sm[2][threadIdx.x] = a2;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int c = 0; c < 3; ++c) sm[c][threadIdx.x] += sm[c][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int c = 0; c < 3; ++c) part[3 * blockIdx.x + c] = sm[c][0];
}

// CongAcc (App. E): dot products m.m, m.d, d.d of one component of x, with
// d = xnew - xold and m the component's moving average.
__global__ void __launch_bounds__(256) congacc_dots_kernel(const double* __restrict__ xnew,
                                                           const double* __restrict__ xold,
                                                           const int32_t* __restrict__ idx, int64_t n, int64_t base,
                                                           int stride, int c, const double* __restrict__ m,
                                                           double* __restrict__ part) {
  __shared__ double sm[3][256];
  double a0 = 0.0, a1 = 0.0, a2 = 0.0;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < n;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t k = (base + (idx ? idx[i] : i)) * stride + c;
    const double d = xnew[k] - xold[k], mv = m[k];
    a0 += mv * mv;
    a1 += mv * d;
    a2 += d * d;
  }
  sm[0][threadIdx.x] = a0;
  sm[1][threadIdx.x] = a1;
  sm[2][threadIdx.x] = a2;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (threadIdx.x < w)
      for (int j = 0; j < 3; ++j) sm[j][threadIdx.x] += sm[j][threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0)
    for (int j = 0; j < 3; ++j) part[3 * blockIdx.x + j] = sm[j][0];
}

// CongAcc step: m <- w m + (1 - w) d, x += a m, with d = gx - x and the
// coefficients of component r * stride + c.
__global__ void __launch_bounds__(256) congacc_update_kernel(double* __restrict__ x, const double* __restrict__ gx,
                                                             double* __restrict__ m, const int32_t* __restrict__ idx,
                                                             int64_t n, int nrep, int64_t field_stride, int stride,
                                                             CongCoef cf) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= n * nrep) return;
  const int64_t r = t / n, i = t - r * n;
  const int64_t e = r * field_stride + (idx ? idx[i] : i);
  for (int c = 0; c < stride; ++c) {
    const int comp = static_cast<int>(r) * stride + c;
    const int64_t k = e * stride + c;
    const double w = cf.w[comp];
    const double mn = w * m[k] + (1.0 - w) * (gx[k] - x[k]);
    m[k] = mn;
    x[k] += cf.a[comp] * mn;
  }
}

// --------------------------------------------------------------------------
// A-solve (App. D): zero-padded FFT correlation with the cell-averaged
// Green's function of the 2D Laplacian
// --------------------------------------------------------------------------
// grain means of the two current components from block partials (fixed
// summation order, the same as a host-side sum of the partials)
__global__ void __launch_bounds__(256) means_kernel(const double* __restrict__ part, int nparts, double inv_n,
                                                    double* __restrict__ mean) {
  // one block; fixed-order tree over the partials: deterministic
  __shared__ double sh[2][256];
  for (int c = 0; c < 2; ++c) {
    double v = 0.0;
    for (int i = threadIdx.x; i < nparts; i += blockDim.x) v += part[c * nparts + i];
    sh[c][threadIdx.x] = v;
  }
  __syncthreads();
  for (int st = 128; st > 0; st >>= 1) {
    if (threadIdx.x < st) {
      sh[0][threadIdx.x] += sh[0][threadIdx.x + st];
      sh[1][threadIdx.x] += sh[1][threadIdx.x + st];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    mean[0] = sh[0][0] * inv_n;
    mean[1] = sh[1][0] * inv_n;
  }
}

__global__ void __launch_bounds__(256) pad_current_kernel(const double* __restrict__ j, const uint8_t* __restrict__ mask,
                                                          int nx, int ny, int px, int py,
                                                          const double* __restrict__ mean, double2* __restrict__ w) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (t >= static_cast<int64_t>(px) * py) return;
  const int x = static_cast<int>(t % px), y = static_cast<int>(t / px);
  double2 v = make_double2(0.0, 0.0);
  if (x < nx && y < ny) {
    const int64_t c = static_cast<int64_t>(y) * nx + x;
    if (mask[c]) v = make_double2(j[c] - mean[0], j[static_cast<int64_t>(nx) * ny + c] - mean[1]);
  }
  w[t] = v;
}

// In-place radix-2 FFT of every row (length n = 2^logn) of a [rows][n]
// complex array, one workgroup per row, staged in LDS.  sign = -1 forward.
// pre (optional, same layout): the input is multiplied by it on the way in.
__global__ void __launch_bounds__(256) fft_rows_kernel(double2* __restrict__ w, int logn,
                                                       const double2* __restrict__ tw, int sign,
                                                       const double2* __restrict__ pre) {
  extern __shared__ double2 buf[];
  const int n = 1 << logn;
  double2* row = w + static_cast<int64_t>(blockIdx.x) * n;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const int r = static_cast<int>(__builtin_bitreverse32(static_cast<unsigned>(i)) >> (32 - logn));
    double2 v = row[i];
    if (pre) {
      const double2 b = pre[static_cast<int64_t>(blockIdx.x) * n + i];
      v = make_double2(v.x * b.x - v.y * b.y, v.x * b.y + v.y * b.x);
    }
    buf[r] = v;
  }
  __syncthreads();
  // twiddle exp(-+2 pi i pos / 2^s) of stage s
  auto twiddle = [&](int pos, int s) {
    double2 tf = tw[pos << (logn - s)];
    if (sign > 0) tf.y = -tf.y;
    return tf;
  };
  auto butterfly = [](double2& u, double2& v, double2 tf) {
    const double2 vt = make_double2(v.x * tf.x - v.y * tf.y, v.x * tf.y + v.y * tf.x);
    v = make_double2(u.x - vt.x, u.y - vt.y);
    u = make_double2(u.x + vt.x, u.y + vt.y);
  };
  // two radix-2 stages per pass, the four elements a thread combines held in
  // registers: stage s pairs (i, i + h) and (i + 2h, i + 3h), stage s + 1
  // pairs (i, i + 2h) and (i + h, i + 3h), h = 2^(s-1)
  int s = 1;
  for (; s + 1 <= logn; s += 2) {
    const int h = 1 << (s - 1);
    for (int b = threadIdx.x; b < n / 4; b += blockDim.x) {
      const int grp = b / h, pos = b - grp * h;
      const int i0 = grp * 4 * h + pos;
      double2 x0 = buf[i0], x1 = buf[i0 + h], x2 = buf[i0 + 2 * h], x3 = buf[i0 + 3 * h];
      const double2 t1 = twiddle(pos, s);
      butterfly(x0, x1, t1);
      butterfly(x2, x3, t1);
      butterfly(x0, x2, twiddle(pos, s + 1));
      butterfly(x1, x3, twiddle(pos + h, s + 1));
      buf[i0] = x0;
      buf[i0 + h] = x1;
      buf[i0 + 2 * h] = x2;
      buf[i0 + 3 * h] = x3;
    }
    __syncthreads();
  }
  if (s == logn) {  // odd logn: one radix-2 stage left
    const int h = 1 << (s - 1);
    for (int b = threadIdx.x; b < n / 2; b += blockDim.x) {
      const int grp = b / h, pos = b - grp * h;
      const int i0 = grp * 2 * h + pos;
      double2 u = buf[i0], v = buf[i0 + h];
      butterfly(u, v, twiddle(pos, s));
      buf[i0] = u;
      buf[i0 + h] = v;
    }
    __syncthreads();
  }
  for (int i = threadIdx.x; i < n; i += blockDim.x) row[i] = buf[i];
}

// out[x][y] = in[y][x] for a [rows][cols] complex array, 32x32 LDS tiles
__global__ void __launch_bounds__(256) transpose_kernel(const double2* __restrict__ in, double2* __restrict__ out,
                                                        int rows, int cols) {
  __shared__ double2 tile[32][33];
  const int bx = blockIdx.x * 32, by = blockIdx.y * 32;
  for (int r = threadIdx.y; r < 32; r += 8) {
    const int y = by + r, x = bx + threadIdx.x;
    if (y < rows && x < cols) tile[r][threadIdx.x] = in[static_cast<int64_t>(y) * cols + x];
  }
  __syncthreads();
  for (int r = threadIdx.y; r < 32; r += 8) {
    const int x = bx + r, y = by + threadIdx.x;
    if (x < cols && y < rows) out[static_cast<int64_t>(x) * rows + y] = tile[threadIdx.x][r];
  }
}

__global__ void __launch_bounds__(256) unpad_A_kernel(const double2* __restrict__ w, int nx, int ny, int px,
                                                      double scale, double* __restrict__ A) {
  const int64_t c = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= static_cast<int64_t>(nx) * ny) return;
  const int x = static_cast<int>(c % nx), y = static_cast<int>(c / nx);
  const double2 v = w[static_cast<int64_t>(y) * px + x];
  A[c] = scale * v.x;
  A[static_cast<int64_t>(nx) * ny + c] = scale * v.y;
}

// --------------------------------------------------------------------------
// issue-rate probe: eight independent chains of one FP32 operation per lane
// (op 0 fma, 1 rsq, 2 sqrt, 3 rcp), for the roofline of the sweep kernels
// --------------------------------------------------------------------------
template <int OP>
__device__ __forceinline__ float rate_op(float a, float s) {
  if (OP == 0) return __builtin_fmaf(a, s, 0.5f);
  if (OP == 1) return __builtin_amdgcn_rsqf(a);
  if (OP == 2) return __builtin_amdgcn_sqrtf(a);
  return __builtin_amdgcn_rcpf(a);
}
template <int OP>
__global__ void __launch_bounds__(256) valu_rate_kernel(float* __restrict__ out, int iters, float s) {
  float v[8];
  for (int i = 0; i < 8; ++i) v[i] = 1.0f + 1e-3f * static_cast<float>(threadIdx.x) + 0.1f * static_cast<float>(i);
  for (int k = 0; k < iters; ++k)
    for (int i = 0; i < 8; ++i) v[i] = rate_op<OP>(v[i], s);
  float t = 0.0f;
  for (int i = 0; i < 8; ++i) t += v[i];
  out[static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x] = t;
}

// --------------------------------------------------------------------------
// launch wrappers
// --------------------------------------------------------------------------
static inline unsigned nblk(int64_t n, int b = 256) { return static_cast<unsigned>((n + b - 1) / b); }

template <typename T>
void launch_interp(const InterpArgs& a, void* cells, void* nodes, hipStream_t st) {
  if (a.nslot == 0) return;
  if (cells && a.ncomp == 1) {
    hipLaunchKernelGGL(pack_cells_kernel<T>, dim3(nblk(a.ncell)), dim3(256), 0, st, a.delta, a.A, a.geom.mask,
                       a.ncell, static_cast<cell4<T>*>(cells));
    hipLaunchKernelGGL(interp1_kernel<T>, dim3(static_cast<unsigned>((a.nseg + 3) / 4)), dim3(256), 0, st, a,
                       static_cast<const cell4<T>*>(cells), static_cast<node4<T>*>(nodes));
  } else {
    hipLaunchKernelGGL(interp_kernel<T>, dim3(nblk(a.nslot)), dim3(256), 0, st, a, static_cast<node4<T>*>(nodes));
  }
}
template void launch_interp<double>(const InterpArgs&, void*, void*, hipStream_t);
template void launch_interp<float>(const InterpArgs&, void*, void*, hipStream_t);

template <typename T, int EPL, int MODE>
static void launch_sweep_t(const SweepArgs& a, const SweepBufs& b, hipStream_t st) {
  const bool split = MODE == 0 && EPL % 2 == 0 && a.nlong > 0;
  const int64_t threads = split ? a.nlong * 2 * a.G + (a.nseg - a.nlong) * a.G : a.nseg * a.G;
  hipLaunchKernelGGL((sweep_kernel<T, EPL, MODE>), dim3(nblk(threads)), dim3(256), 0, st, a,
                     static_cast<const node4<T>*>(b.nodes),
                     static_cast<const cpx<T>*>(b.bc_g_prev), static_cast<const cpx<T>*>(b.bc_gt_prev),
                     static_cast<cpx<T>*>(b.bc_g_next), static_cast<cpx<T>*>(b.bc_gt_next),
                     static_cast<cpx<T>*>(b.gbuf), static_cast<T*>(b.ebuf));
}

template <typename T, int MODE>
static void launch_sweep_m(int epl, const SweepArgs& a, const SweepBufs& b, hipStream_t st) {
  switch (epl) {
    case 1: launch_sweep_t<T, 1, MODE>(a, b, st); break;
    case 2: launch_sweep_t<T, 2, MODE>(a, b, st); break;
    case 3: launch_sweep_t<T, 3, MODE>(a, b, st); break;
    case 4: launch_sweep_t<T, 4, MODE>(a, b, st); break;
    default: launch_sweep_t<T, 8, MODE>(a, b, st); break;
  }
}

template <typename T>
void launch_sweep(int mode, int epl, const SweepArgs& a, const SweepBufs& b, hipStream_t st) {
  if (a.nseg == 0) return;
  if (mode == 0)
    launch_sweep_m<T, 0>(epl, a, b, st);
  else if (mode == 1)
    launch_sweep_m<T, 1>(epl, a, b, st);
  else if (mode == 2)
    launch_sweep_m<T, 2>(epl, a, b, st);
  else
    launch_sweep_m<T, 3>(epl, a, b, st);
}
template void launch_sweep<double>(int, int, const SweepArgs&, const SweepBufs&, hipStream_t);
template void launch_sweep<float>(int, int, const SweepArgs&, const SweepBufs&, hipStream_t);

template <typename T, int EPL>
static int64_t wave_slots_t() {
  int dev = 0, blocks = 0, cus = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, sweep_kernel<T, EPL, 0>, 256, 0) != hipSuccess) return 0;
  return static_cast<int64_t>(blocks) * 4 * cus;
}

template <typename T>
int64_t sweep_wave_slots(int epl) {
  switch (epl) {
    case 1: return wave_slots_t<T, 1>();
    case 2: return wave_slots_t<T, 2>();
    case 3: return wave_slots_t<T, 3>();
    case 4: return wave_slots_t<T, 4>();
    default: return wave_slots_t<T, 8>();
  }
}
template int64_t sweep_wave_slots<double>(int);
template int64_t sweep_wave_slots<float>(int);

template <typename T>
void launch_batch_sweep(int epl, const BatchGrainDev* grains, const int2* tiles, int ntiles, int* counter, int nblocks,
                        void* spill, int64_t wave_elems, hipStream_t st) {
  hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(64), 0, st, counter);
  cpx<T>* sp = static_cast<cpx<T>*>(spill);
#define QC_BATCH(E)                                                                                                  \
  hipLaunchKernelGGL((batch_sweep_kernel<T, E>), dim3(nblocks), dim3(256), 0, st, grains, tiles, ntiles, counter, sp, \
                     wave_elems)
  switch (epl) {
    case 1: QC_BATCH(1); break;
    case 2: QC_BATCH(2); break;
    case 3: QC_BATCH(3); break;
    case 4: QC_BATCH(4); break;
    default: QC_BATCH(8); break;
  }
#undef QC_BATCH
}
template void launch_batch_sweep<double>(int, const BatchGrainDev*, const int2*, int, int*, int, void*, int64_t,
                                         hipStream_t);
template void launch_batch_sweep<float>(int, const BatchGrainDev*, const int2*, int, int*, int, void*, int64_t,
                                        hipStream_t);

void launch_valu_rate(int op, float* out, int nblocks, int iters, hipStream_t st) {
  switch (op) {
    case 0: hipLaunchKernelGGL(valu_rate_kernel<0>, dim3(nblocks), dim3(256), 0, st, out, iters, 0.999f); break;
    case 1: hipLaunchKernelGGL(valu_rate_kernel<1>, dim3(nblocks), dim3(256), 0, st, out, iters, 0.999f); break;
    case 2: hipLaunchKernelGGL(valu_rate_kernel<2>, dim3(nblocks), dim3(256), 0, st, out, iters, 0.999f); break;
    default: hipLaunchKernelGGL(valu_rate_kernel<3>, dim3(nblocks), dim3(256), 0, st, out, iters, 0.999f); break;
  }
}

template <typename T>
void launch_mirror_fill(const int2* pairs, int64_t npairs, int n_e, const int32_t* partner, void* bc_g, void* bc_gt,
                        hipStream_t st) {
  if (npairs * n_e > 0)
    hipLaunchKernelGGL(mirror_fill_kernel<T>, dim3(nblk(npairs * n_e)), dim3(256), 0, st, pairs, npairs, n_e, partner,
                       static_cast<cpx<T>*>(bc_g), static_cast<cpx<T>*>(bc_gt));
}
template void launch_mirror_fill<float>(const int2*, int64_t, int, const int32_t*, void*, void*, hipStream_t);
template void launch_mirror_fill<double>(const int2*, int64_t, int, const int32_t*, void*, void*, hipStream_t);

void launch_rotate_back(const BackArgs& a, hipStream_t st) {
  if (a.ncg == 0) return;
  if (a.ncomp == 1)
    hipLaunchKernelGGL(rotate_back_kernel<1>, dim3((a.ncg + 63) / 64), dim3(64 * kBackWaves), 0, st, a);
  else
    hipLaunchKernelGGL(rotate_back_kernel<4>, dim3((a.ncg + 63) / 64), dim3(64 * kBackWaves), 0, st, a);
}

template <typename T>
void launch_ldos_back(const LdosBackArgs& a, const void* ebuf, hipStream_t st) {
  hipLaunchKernelGGL(ldos_back_kernel<T>, dim3(nblk(a.ncg * a.n_e)), dim3(256), 0, st, a,
                     static_cast<const T*>(ebuf));
}
template void launch_ldos_back<double>(const LdosBackArgs&, const void*, hipStream_t);
template void launch_ldos_back<float>(const LdosBackArgs&, const void*, hipStream_t);

template <typename T>
void launch_green_back(const LdosBackArgs& a, const void* ebuf, hipStream_t st) {
  hipLaunchKernelGGL(green_back_kernel<T>, dim3(nblk(a.ncg * a.n_e)), dim3(256), 0, st, a,
                     static_cast<const T*>(ebuf));
}
template void launch_green_back<double>(const LdosBackArgs&, const void*, hipStream_t);
template void launch_green_back<float>(const LdosBackArgs&, const void*, hipStream_t);

void launch_fill(double* p, int64_t n, double v, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(fill_kernel, dim3(nblk(n)), dim3(256), 0, st, p, n, v);
}
void launch_curl(const double* A, double* B, int nx, int ny, double h, hipStream_t st) {
  hipLaunchKernelGGL(curl_kernel, dim3(nblk(static_cast<int64_t>(nx) * ny)), dim3(256), 0, st, A, B, nx, ny, h);
}
void launch_block_sum(const double* x, const int32_t* idx, int64_t n, int mode, double* part, int nparts,
                      hipStream_t st) {
  const BlockSumRow r{x, idx, n, mode, part};
  hipLaunchKernelGGL(block_sum_kernel, dim3(nparts), dim3(256), 0, st, r, r);
}
void launch_block_sum2(const BlockSumRow& r0, const BlockSumRow& r1, int nparts, hipStream_t st) {
  hipLaunchKernelGGL(block_sum_kernel, dim3(nparts, 2), dim3(256), 0, st, r0, r1);
}
void launch_diff_norm(const DiffNormArgs& a, int nparts, hipStream_t st) {
  hipLaunchKernelGGL(diff_norm_kernel, dim3(nparts), dim3(256), 0, st, a, a, a);
}
void launch_diff_norm_n(const DiffNormArgs* a, int count, int nparts, hipStream_t st) {
  if (count < 1 || count > 3) return;
  hipLaunchKernelGGL(diff_norm_kernel, dim3(nparts, count), dim3(256), 0, st, a[0], a[count > 1 ? 1 : 0],
                     a[count > 2 ? 2 : 0]);
}
void launch_congacc_dots(const double* xnew, const double* xold, const int32_t* idx, int64_t n, int64_t base,
                         int stride, int c, const double* m, double* part, int nparts, hipStream_t st) {
  hipLaunchKernelGGL(congacc_dots_kernel, dim3(nparts), dim3(256), 0, st, xnew, xold, idx, n, base, stride, c, m,
                     part);
}
void launch_congacc_update(double* x, const double* gx, double* m, const int32_t* idx, int64_t n, int nrep,
                           int64_t field_stride, int stride, const CongCoef& cf, hipStream_t st) {
  if (n * nrep > 0)
    hipLaunchKernelGGL(congacc_update_kernel, dim3(nblk(n * nrep)), dim3(256), 0, st, x, gx, m, idx, n, nrep,
                       field_stride, stride, cf);
}
void launch_bb_dots(const double* xnew, const double* xold, const int32_t* idx, int64_t n, int nrep,
                    int64_t field_stride, int stride, double scale, double* dprev, double* part, int nparts,
                    hipStream_t st) {
  hipLaunchKernelGGL(bb_dots_kernel, dim3(nparts), dim3(256), 0, st, xnew, xold, idx, n, nrep, field_stride, stride,
                     scale, dprev, part);
}
void launch_picard(double* x, const double* gx, const int32_t* idx, int64_t n, int nrep, int64_t field_stride,
                   int stride, double alpha, hipStream_t st) {
  if (n * nrep > 0)
    hipLaunchKernelGGL(picard_kernel, dim3(nblk(n * nrep)), dim3(256), 0, st, x, gx, idx, n, nrep, field_stride,
                       stride, alpha);
}
void launch_lw_accumulate(const double* delta, const double* delta_new, const int32_t* grain_cells, int64_t ncg,
                          int ncomp, int64_t ncell, const double* den, double w, int first, double* acc,
                          hipStream_t st) {
  if (ncg > 0)
    hipLaunchKernelGGL(lw_accumulate_kernel, dim3(nblk(ncg)), dim3(256), 0, st, delta, delta_new, grain_cells, ncg,
                       ncomp, ncell, den, w, first, acc);
}
void launch_lw_finish(const double* delta, const int32_t* grain_cells, int64_t ncg, int ncomp, int64_t ncell,
                      int n_theta, const double* eta, const double* wk, const double* logt, double twopi_rz,
                      const double* acc, double* omega_cell, double* omega, hipStream_t st) {
  if (ncg > 0)
    hipLaunchKernelGGL(lw_finish_kernel, dim3(nblk(ncg)), dim3(256), 0, st, delta, grain_cells, ncg, ncomp, ncell,
                       n_theta, eta, wk, logt, twopi_rz, acc, omega_cell, omega);
}
void launch_scale(const double* x, double s, int64_t n, double* y, hipStream_t st) {
  if (n > 0) hipLaunchKernelGGL(scale_kernel, dim3(nblk(n)), dim3(256), 0, st, x, s, n, y);
}
void launch_means(const double* part, int nparts, double inv_n, double* mean, hipStream_t st) {
  hipLaunchKernelGGL(means_kernel, dim3(1), dim3(256), 0, st, part, nparts, inv_n, mean);
}
void launch_pad_current(const double* j, const uint8_t* mask, int nx, int ny, int px, int py, const double* mean,
                        double2* w, hipStream_t st) {
  hipLaunchKernelGGL(pad_current_kernel, dim3(nblk(static_cast<int64_t>(px) * py)), dim3(256), 0, st, j, mask, nx,
                     ny, px, py, mean, w);
}
void launch_fft_rows(double2* w, int rows, int logn, const double2* tw, int sign, const double2* pre, hipStream_t st) {
  hipLaunchKernelGGL(fft_rows_kernel, dim3(rows), dim3(256), sizeof(double2) << logn, st, w, logn, tw, sign, pre);
}
void launch_transpose(const double2* in, double2* out, int rows, int cols, hipStream_t st) {
  hipLaunchKernelGGL(transpose_kernel, dim3((cols + 31) / 32, (rows + 31) / 32), dim3(32, 8), 0, st, in, out, rows,
                     cols);
}
void launch_unpad_A(const double2* w, int nx, int ny, int px, double scale, double* A, hipStream_t st) {
  hipLaunchKernelGGL(unpad_A_kernel, dim3(nblk(static_cast<int64_t>(nx) * ny)), dim3(256), 0, st, w, nx, ny, px,
                     scale, A);
}

}  // namespace qc
