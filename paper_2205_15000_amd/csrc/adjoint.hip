// Reverse mode of one iteration map (FP64): gradients of a real loss of
// (Delta_new, j, Omega) with respect to Delta_G(R) and A_ind(R), the
// boundary store held fixed (start values from specular taps are inputs;
// start values that are bulk roots of the end values are differentiated).
//
// Complex gradients follow dL = Re(conj(G_x) dx), i.e. G_x = dL/dRe x +
// i dL/dIm x.  For y = F(x, x*): G_x = conj(dF/dx) G_y + dF/dx* conj(G_y).
//
// Implicit-midpoint step (App. C) y = F(g; D, z, h) solves
//   y - g - h f((g+y)/2) = 0,  f(m) = i (D* m^2 + 2 z m + D),
// so with m = (g+y)/2, f' = i (2 D* m + 2 z) and Q = 1 - h f'/2:
//   dF/dg = (1 + h f'/2)/Q,  dF/dD = i h/Q,  dF/dD* = i h m^2/Q,  dF/dz = 2 i h m/Q.
// Bulk root y = -D/(z+s), s = z + D* y: dy/dD = -1/(2s), dy/dD* = -y^2/(2s),
// dy/dz = -y/s.
#include "kernels.hpp"
#include "sweep.hpp"

namespace qc {

using C = cpx<double>;

__device__ __forceinline__ C cconj(C a) { return mk(a.x, -a.y); }
__device__ __forceinline__ C cdivd(C a, C b) {
  const double r = drcp(b.x * b.x + b.y * b.y);
  return mk((a.x * b.x + a.y * b.y) * r, (a.y * b.x - a.x * b.y) * r);
}
__device__ __forceinline__ C cscale(double s, C a) { return mk(s * a.x, s * a.y); }

// Sums over the segment's lane group of the three slot gradients (Re, Im of
// G_Delta and the gradient of a), written (or added) to o[0..2] by the
// group's first lanes.
__device__ __forceinline__ void put_slot_grad(double* o, double rx, double ry, double ra, int G, int lane,
                                              bool add) {
  if (G >= 4) {
    const double v = group_sum4_scatter(rx, ry, ra, 0.0, G, lane);
    const int qq = scatter_index(lane);
    if (lane < 4 && qq < 3) o[qq] = add ? o[qq] + v : v;
  } else {
    rx = group_sum(rx, G);
    ry = group_sum(ry, G);
    ra = group_sum(ra, G);
    if (lane == 0) {
      o[0] = add ? o[0] + rx : rx;
      o[1] = add ? o[1] + ry : ry;
      o[2] = add ? o[2] + ra : ra;
    }
  }
}

struct StepDer {
  C dg, dd, ddc, dz;
};

// derivatives of y = F(g; d, z, h) given both ends g and y
__device__ __forceinline__ StepDer step_der(C g, C y, C d, C z, double h) {
  const C m = mk(0.5 * (g.x + y.x), 0.5 * (g.y + y.y));
  const C dm = cconj(d) * m;
  const C fp = mk(-2.0 * (dm.y + z.y), 2.0 * (dm.x + z.x));  // i (2 D* m + 2 z)
  const C qd = mk(1.0 - 0.5 * h * fp.x, -0.5 * h * fp.y);
  const C inv = cdivd(mk(1.0, 0.0), qd);
  StepDer r;
  r.dg = mk(2.0 * inv.x - 1.0, 2.0 * inv.y);  // (2 - Q)/Q
  const C ih = mk(0.0, h);
  r.dd = ih * inv;
  r.ddc = ih * (m * m) * inv;
  r.dz = cscale(2.0, ih * m * inv);
  return r;
}

// adjoint of y = bulk root(z, d) (start value) with adjoint gy: adds to
// G_d (complex) and to the real gradient of z's real part
__device__ __forceinline__ void bulk_adj(C y, C z, C d, C gy, C& gd, double& gzr) {
  const C s = z + cconj(d) * y;
  const C i2s = cdivd(mk(-0.5, 0.0), s);   // -1/(2s)
  const C dd = i2s;
  const C ddc = y * y * i2s;
  const C dz = cscale(2.0, y * i2s);       // -y/s
  gd = gd + cconj(dd) * gy + ddc * cconj(gy);
  gzr += (cconj(gy) * dz).x;
}

// Node-local gradients of the per-node sums at one pole (Sec. II.A, Sec. II)
// for gamma = gg, gamma~ = gv, node order parameter dn, sum gradients gs and
// pole weight r: the adjoint of gamma (added to lam), of gamma~ (returned
// in lgt) and of D through S_I (added to acc).
__device__ __forceinline__ void node_adj(C gg, C gv, C dn, const double4& gs, double r, double pt, C& lam, C& lgt,
                                         C& acc) {
  const C gsf = mk(gs.x, gs.y);
  const C x = gg * gv;
  const C inv = cdivd(mk(1.0, 0.0), mk(1.0 + x.x, x.y));
  const C inv2 = inv * inv;
  const C kf = cconj(gsf) * mk(0.0, -pt * r);        // S_f = -i 2pi t~ R (u + conj v)
  const C kg = mk(0.0, -0.5 * pt * r * gs.z);        // S_g = pi t~ R Im((1-X)/(1+X))
  const C ki = mk(0.0, -pt * r * gs.w);              // S_I = 2pi t~ R Im(D* g - D g~)
  const C agam = kf * inv2 - cconj(kf) * (gv * gv) * inv2 - cscale(2.0, kg * gv * inv2) + ki * cconj(dn);
  const C agt = cconj(kf) * inv2 - kf * (gg * gg) * inv2 - cscale(2.0, kg * gg * inv2) - ki * dn;
  lam = lam + cconj(agam);
  lgt = cconj(agt);
  acc = acc + ki * gg - cconj(ki * gv);  // G_D through S_I
}

template <int EPL>
__global__ void __launch_bounds__(256) adjoint_kernel(AdjArgs a, const node4<double>* __restrict__ nodes,
                                                      const C* __restrict__ bc_g_prev,
                                                      const C* __restrict__ bc_gt_prev, C* __restrict__ gbuf,
                                                      C* __restrict__ gtbuf, C* __restrict__ lgt,
                                                      const double4* __restrict__ gS, double* __restrict__ gV) {
  const int64_t gtid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t wseg = gtid >> a.log2g;
  const int lane = static_cast<int>(gtid & (a.G - 1));
  if (wseg >= a.nseg) return;
  const int64_t seg = a.order ? static_cast<int64_t>(a.order[wseg]) : wseg;
  const int64_t slot0 = a.seg_slot0[seg];
  const int n = a.seg_n[seg];
  const int last = n > 0 ? n - 1 : 0;
  const double hfirst = a.seg_hfirst[seg], hlast = a.seg_hlast[seg], hfull = a.h;
  const double q = a.q;
  const int e0 = lane * EPL;
  double ex[EPL], ey[EPL], rw[EPL];
  bool ok[EPL];
  for (int i = 0; i < EPL; ++i) {
    ok[i] = e0 + i < a.n_e;
    const int e = ok[i] ? e0 + i : a.n_e - 1;
    ex[i] = a.eps[2 * e];
    ey[i] = a.eps[2 * e + 1];
    rw[i] = ok[i] ? a.rp[e] : 0.0;
  }
  auto hstep = [&](int t) { return t == 0 ? hfirst : (t == n ? hlast : hfull); };
  auto mid = [&](int t, C& dm, double& am) {
    const node4<double> lo = nodes[slot0 + (t >= 1 ? t - 1 : 0)];
    const node4<double> up = nodes[slot0 + (t < last ? t : last)];
    dm = mk(0.5 * (lo.dx + up.dx), 0.5 * (lo.dy + up.dy));
    am = 0.5 * (lo.a + up.a);
  };

  // ---- pass 1: gamma forward, stored at the nodes
  const int64_t tb = seg * 4;
  const bool staps = a.bc_valid && a.tap_start_w[tb] + a.tap_start_w[tb + 1] + a.tap_start_w[tb + 2] +
                                           a.tap_start_w[tb + 3] > 0.0;
  const bool etaps = a.bc_valid && a.tap_end_w[tb] + a.tap_end_w[tb + 1] + a.tap_end_w[tb + 2] +
                                           a.tap_end_w[tb + 3] > 0.0;
  C g0[EPL], g[EPL];
  {
    const node4<double> v0 = nodes[slot0];
    for (int i = 0; i < EPL; ++i) {
      if (staps) {
        C acc = mk(0.0, 0.0);
        for (int c = 0; c < 4; ++c)
          acc = acc + cscale(a.tap_start_w[tb + c],
                             bc_g_prev[static_cast<int64_t>(a.tap_start_seg[tb + c]) * a.n_e_tot + (ok[i] ? e0 + i : a.n_e - 1)]);
        g0[i] = acc;
      } else {
        g0[i] = bulk_root(q * v0.a + ex[i], ey[i], v0.dx, v0.dy);
      }
      g[i] = g0[i];
    }
  }
  for (int t = 0; t <= n; ++t) {
    C dm;
    double am;
    mid(t, dm, am);
    const double hs = hstep(t);
    const StepC<double> sc = step_consts(dm.x, dm.y, hs);
    for (int i = 0; i < EPL; ++i) g[i] = riccati_step_z(g[i], sc, hs, q * am + ex[i], ey[i]);
    if (t < n)
      for (int i = 0; i < EPL; ++i)
        if (ok[i]) gbuf[(slot0 + t) * a.n_e + e0 + i] = g[i];
  }
  // g[] now holds gamma at R_max

  // ---- pass 2: gamma~ backward; node-local gradients; adjoint of gamma
  C gt0[EPL], gt[EPL], lam[EPL];
  {
    const node4<double> v1 = nodes[slot0 + last];
    for (int i = 0; i < EPL; ++i) {
      if (etaps) {
        C acc = mk(0.0, 0.0);
        for (int c = 0; c < 4; ++c)
          acc = acc + cscale(a.tap_end_w[tb + c],
                             bc_gt_prev[static_cast<int64_t>(a.tap_end_seg[tb + c]) * a.n_e_tot + (ok[i] ? e0 + i : a.n_e - 1)]);
        gt0[i] = acc;
      } else {
        gt0[i] = bulk_root(q * v1.a + ex[i], ey[i], -v1.dx, v1.dy);
      }
      gt[i] = gt0[i];
      lam[i] = mk(0.0, 0.0);
    }
  }
  const double pt = a.twopi_tt;  // 2 pi t~
  // Step t feeds half of its gradient to slot max(t-1,0) and half to slot
  // min(t,last).  Going down, slot t is complete once the local gradient at
  // node t and the upper half of step t are in (plus, for slot 0, the lower
  // half of step 0 and the bulk start); `carry` holds the lower half of the
  // step just processed.
  C carry = mk(0.0, 0.0);
  double carrya = 0.0;
  C gcur[EPL];  // gamma at slot t (at R_max for t = n), loaded once per slot
  for (int i = 0; i < EPL; ++i) gcur[i] = g[i];
  for (int t = n; t >= 0; --t) {
    C acc = carry;
    double acca = carrya;
    if (t < n) {
      // node t: gradients of the per-node sums (Sec. II.A, Sec. II)
      const int64_t node = slot0 + t;
      const node4<double> v = nodes[node];
      const C dn = mk(v.dx, v.dy);
      const double4 gs = gS[node];
      for (int i = 0; i < EPL; ++i) {
        if (!ok[i]) continue;
        C lv;
        node_adj(gcur[i], gt[i], dn, gs, rw[i], pt, lam[i], lv, acc);
        lgt[node * a.n_e + e0 + i] = lv;
        gtbuf[node * a.n_e + e0 + i] = gt[i];
      }
    }
    // step t: adjoint of gamma_{t-1} -> gamma_t; primal gamma~_t -> gamma~_{t-1}
    C dm;
    double am;
    mid(t, dm, am);
    const double hs = hstep(t);
    C stepD = mk(0.0, 0.0);
    double stepa = 0.0;
    const StepC<double> sc = step_consts(-dm.x, dm.y, hs);
    for (int i = 0; i < EPL; ++i) {
      const C z = mk(q * am + ex[i], ey[i]);
      if (ok[i]) {
        const C gl = t >= 1 ? gbuf[(slot0 + t - 1) * a.n_e + e0 + i] : g0[i];
        const C gu = gcur[i];
        gcur[i] = gl;
        const StepDer sd = step_der(gl, gu, dm, z, hs);
        const C l = lam[i];
        stepD = stepD + cconj(sd.dd) * l + sd.ddc * cconj(l);
        stepa += q * (cconj(l) * sd.dz).x;
        lam[i] = cconj(sd.dg) * l;
      }
      gt[i] = riccati_step_z(gt[i], sc, hs, z.x, z.y);
    }
    if (t == n && n >= 1) {  // both halves of the last step go to slot n-1
      carry = stepD;
      carrya = stepa;
      continue;
    }
    acc = acc + cscale(0.5, stepD);
    acca += 0.5 * stepa;
    carry = cscale(0.5, stepD);
    carrya = 0.5 * stepa;
    if (t == 0) {
      acc = acc + carry;  // lower half of step 0 is slot 0 too
      acca += carrya;
      if (!staps) {       // gamma started at the bulk root of slot 0's values
        const node4<double> v0 = nodes[slot0];
        for (int i = 0; i < EPL; ++i) {
          if (!ok[i]) continue;
          double gz = 0.0;
          bulk_adj(g0[i], mk(q * v0.a + ex[i], ey[i]), mk(v0.dx, v0.dy), lam[i], acc, gz);
          acca += q * gz;
        }
      }
    }
    put_slot_grad(gV + (slot0 + t) * 3, acc.x, acc.y, acca, a.G, lane, false);
  }
  // gt[] now holds gamma~ at R_min

  // ---- pass 3: adjoint of gamma~ (forward in t).  Step t maps gamma~_t to
  // gamma~_{t-1}; slot t-1 is complete after step t (slot n-1 also takes
  // both halves of step n and the bulk start at R_max).
  C mu[EPL];
  C gprv[EPL];  // gamma~ at slot t-1 (at R_min for t = 0), loaded once per slot
  for (int i = 0; i < EPL; ++i) {
    mu[i] = mk(0.0, 0.0);
    gprv[i] = gt[i];
  }
  carry = mk(0.0, 0.0);
  carrya = 0.0;
  for (int t = 0; t <= n; ++t) {
    C dm;
    double am;
    mid(t, dm, am);
    const double hs = hstep(t);
    const C dprime = mk(-dm.x, dm.y);  // -conj(dm)
    C stepD = mk(0.0, 0.0);
    double stepa = 0.0;
    for (int i = 0; i < EPL; ++i) {
      if (!ok[i]) continue;
      const C z = mk(q * am + ex[i], ey[i]);
      const C gu = t < n ? gtbuf[(slot0 + t) * a.n_e + e0 + i] : gt0[i];
      const C gl = gprv[i];
      gprv[i] = gu;
      const StepDer sd = step_der(gu, gl, dprime, z, hs);
      const C l = mu[i];
      const C gdp = cconj(sd.dd) * l + sd.ddc * cconj(l);  // gradient of D' = -conj(dm)
      stepD = stepD - cconj(gdp);
      stepa += q * (cconj(l) * sd.dz).x;
      mu[i] = cconj(sd.dg) * l;
      if (t < n) mu[i] = mu[i] + lgt[(slot0 + t) * a.n_e + e0 + i];
    }
    if (t == 0) {
      carry = stepD;  // both halves of step 0 belong to slot 0
      carrya = stepa;
      if (n >= 1) continue;
    }
    C acc;
    double acca;
    int slot;
    if (t == 0) {  // n == 0
      acc = carry;
      acca = carrya;
      slot = 0;
    } else if (t < n) {
      acc = carry + cscale(0.5, stepD);
      acca = carrya + 0.5 * stepa;
      carry = cscale(0.5, stepD);
      carrya = 0.5 * stepa;
      slot = t - 1;
    } else {
      acc = carry + stepD;
      acca = carrya + stepa;
      slot = last;
    }
    if (t == n && !etaps) {  // gamma~ started at the bulk root of the last slot
      const node4<double> v1 = nodes[slot0 + last];
      for (int i = 0; i < EPL; ++i) {
        if (!ok[i]) continue;
        double gz = 0.0;
        C gdp = mk(0.0, 0.0);
        bulk_adj(gt0[i], mk(q * v1.a + ex[i], ey[i]), mk(-v1.dx, v1.dy), mu[i], gdp, gz);
        acc = acc - cconj(gdp);
        acca += q * gz;
      }
    }
    put_slot_grad(gV + (slot0 + slot) * 3, acc.x, acc.y, acca, a.G, lane, true);
  }
}

// The same reverse mode with checkpoints every CK slots instead of gamma,
// gamma~ and the gamma~ adjoint terms at every node: pass 1 keeps gamma
// entering each block; pass 2 (backward) recomputes each block's gamma
// forward from its checkpoint into a per-thread scratch and keeps gamma~ at
// each block's first slot; pass 3 (forward) recomputes a block's gamma
// forward and gamma~ backward (from the next block's checkpoint) and forms
// the node-local gamma~ adjoint terms again.  The recomputation runs the same
// steps on the same inputs as the stored variant.
template <int EPL>
__global__ void __launch_bounds__(256) adjoint_ckpt_kernel(AdjArgs a, const node4<double>* __restrict__ nodes,
                                                           const C* __restrict__ bc_g_prev,
                                                           const C* __restrict__ bc_gt_prev,
                                                           const double4* __restrict__ gS, double* __restrict__ gV,
                                                           int CK, const int64_t* __restrict__ ckbase,
                                                           C* __restrict__ ckg, C* __restrict__ ckgt,
                                                           C* __restrict__ scr, int64_t nthr) {
  const int64_t gtid = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t wseg = gtid >> a.log2g;
  const int lane = static_cast<int>(gtid & (a.G - 1));
  if (wseg >= a.nseg) return;
  const int64_t seg = a.order ? static_cast<int64_t>(a.order[wseg]) : wseg;
  const int64_t slot0 = a.seg_slot0[seg];
  const int n = a.seg_n[seg];
  const int last = n > 0 ? n - 1 : 0;
  const double hfirst = a.seg_hfirst[seg], hlast = a.seg_hlast[seg], hfull = a.h;
  const double q = a.q;
  const int e0 = lane * EPL;
  const int64_t cb = ckbase[seg];
  double ex[EPL], ey[EPL], rw[EPL];
  bool ok[EPL];
  for (int i = 0; i < EPL; ++i) {
    ok[i] = e0 + i < a.n_e;
    const int e = ok[i] ? e0 + i : a.n_e - 1;
    ex[i] = a.eps[2 * e];
    ey[i] = a.eps[2 * e + 1];
    rw[i] = ok[i] ? a.rp[e] : 0.0;
  }
  auto hstep = [&](int t) { return t == 0 ? hfirst : (t == n ? hlast : hfull); };
  auto mid = [&](int t, C& dm, double& am) {
    const node4<double> lo = nodes[slot0 + (t >= 1 ? t - 1 : 0)];
    const node4<double> up = nodes[slot0 + (t < last ? t : last)];
    dm = mk(0.5 * (lo.dx + up.dx), 0.5 * (lo.dy + up.dy));
    am = 0.5 * (lo.a + up.a);
  };
  // scratch: region 0 gamma, region 1 gamma~, lane-interleaved
  auto sc_at = [&](int region, int pos, int i) -> C& {
    return scr[((static_cast<int64_t>(region) * CK + pos) * EPL + i) * nthr + gtid];
  };
  auto ck_at = [&](C* base, int kb, int i) -> C& { return base[(cb + kb) * a.n_e + e0 + i]; };

  const int64_t tb = seg * 4;
  const bool staps = a.bc_valid && a.tap_start_w[tb] + a.tap_start_w[tb + 1] + a.tap_start_w[tb + 2] +
                                           a.tap_start_w[tb + 3] > 0.0;
  const bool etaps = a.bc_valid && a.tap_end_w[tb] + a.tap_end_w[tb + 1] + a.tap_end_w[tb + 2] +
                                           a.tap_end_w[tb + 3] > 0.0;
  C g0[EPL], g[EPL];
  {
    const node4<double> v0 = nodes[slot0];
    for (int i = 0; i < EPL; ++i) {
      if (staps) {
        C acc = mk(0.0, 0.0);
        for (int c = 0; c < 4; ++c)
          acc = acc + cscale(a.tap_start_w[tb + c],
                             bc_g_prev[static_cast<int64_t>(a.tap_start_seg[tb + c]) * a.n_e_tot + (ok[i] ? e0 + i : a.n_e - 1)]);
        g0[i] = acc;
      } else {
        g0[i] = bulk_root(q * v0.a + ex[i], ey[i], v0.dx, v0.dy);
      }
      g[i] = g0[i];
    }
  }
  auto gamma_step = [&](C* gv, int t) {
    C dm;
    double am;
    mid(t, dm, am);
    const double hs = hstep(t);
    const StepC<double> sc = step_consts(dm.x, dm.y, hs);
    for (int i = 0; i < EPL; ++i) gv[i] = riccati_step_z(gv[i], sc, hs, q * am + ex[i], ey[i]);
  };
  auto gammat_step = [&](C* gv, int t) {
    C dm;
    double am;
    mid(t, dm, am);
    const double hs = hstep(t);
    const StepC<double> sc = step_consts(-dm.x, dm.y, hs);
    for (int i = 0; i < EPL; ++i) gv[i] = riccati_step_z(gv[i], sc, hs, q * am + ex[i], ey[i]);
  };
  // gamma at the slots of block kb (slots kb*CK .. min((kb+1)*CK, n) - 1)
  auto recompute_gamma = [&](int kb) {
    C gr[EPL];
    for (int i = 0; i < EPL; ++i) gr[i] = kb == 0 ? g0[i] : (ok[i] ? ck_at(ckg, kb, i) : g0[i]);
    const int s0 = kb * CK, s1 = min(s0 + CK, n);
    for (int s = s0; s < s1; ++s) {
      gamma_step(gr, s);
      for (int i = 0; i < EPL; ++i) sc_at(0, s - s0, i) = gr[i];
    }
  };

  // ---- pass 1: gamma forward, kept entering each block
  for (int t = 0; t <= n; ++t) {
    gamma_step(g, t);
    if (t + 1 < n && (t + 1) % CK == 0)
      for (int i = 0; i < EPL; ++i)
        if (ok[i]) ck_at(ckg, (t + 1) / CK, i) = g[i];
  }

  // ---- pass 2: gamma~ backward; node-local gradients; adjoint of gamma
  C gt0[EPL], gt[EPL], lam[EPL];
  {
    const node4<double> v1 = nodes[slot0 + last];
    for (int i = 0; i < EPL; ++i) {
      if (etaps) {
        C acc = mk(0.0, 0.0);
        for (int c = 0; c < 4; ++c)
          acc = acc + cscale(a.tap_end_w[tb + c],
                             bc_gt_prev[static_cast<int64_t>(a.tap_end_seg[tb + c]) * a.n_e_tot + (ok[i] ? e0 + i : a.n_e - 1)]);
        gt0[i] = acc;
      } else {
        gt0[i] = bulk_root(q * v1.a + ex[i], ey[i], -v1.dx, v1.dy);
      }
      gt[i] = gt0[i];
      lam[i] = mk(0.0, 0.0);
    }
  }
  const double pt = a.twopi_tt;  // 2 pi t~
  C carry = mk(0.0, 0.0);
  double carrya = 0.0;
  C gcur[EPL];  // gamma at slot t (at R_max for t = n)
  for (int i = 0; i < EPL; ++i) gcur[i] = g[i];
  int loaded = -1;
  for (int t = n; t >= 0; --t) {
    C acc = carry;
    double acca = carrya;
    if (t < n) {
      const int64_t node = slot0 + t;
      const node4<double> v = nodes[node];
      const C dn = mk(v.dx, v.dy);
      const double4 gs = gS[node];
      for (int i = 0; i < EPL; ++i) {
        if (!ok[i]) continue;
        C lv;
        node_adj(gcur[i], gt[i], dn, gs, rw[i], pt, lam[i], lv, acc);
        if (t > 0 && t % CK == 0) ck_at(ckgt, t / CK, i) = gt[i];
      }
    }
    if (t >= 1 && (t - 1) / CK != loaded) {
      loaded = (t - 1) / CK;
      recompute_gamma(loaded);
    }
    C dm;
    double am;
    mid(t, dm, am);
    const double hs = hstep(t);
    C stepD = mk(0.0, 0.0);
    double stepa = 0.0;
    const StepC<double> sc = step_consts(-dm.x, dm.y, hs);
    for (int i = 0; i < EPL; ++i) {
      const C z = mk(q * am + ex[i], ey[i]);
      if (ok[i]) {
        const C gl = t >= 1 ? sc_at(0, (t - 1) - loaded * CK, i) : g0[i];
        const C gu = gcur[i];
        gcur[i] = gl;
        const StepDer sd = step_der(gl, gu, dm, z, hs);
        const C l = lam[i];
        stepD = stepD + cconj(sd.dd) * l + sd.ddc * cconj(l);
        stepa += q * (cconj(l) * sd.dz).x;
        lam[i] = cconj(sd.dg) * l;
      }
      gt[i] = riccati_step_z(gt[i], sc, hs, z.x, z.y);
    }
    if (t == n && n >= 1) {
      carry = stepD;
      carrya = stepa;
      continue;
    }
    acc = acc + cscale(0.5, stepD);
    acca += 0.5 * stepa;
    carry = cscale(0.5, stepD);
    carrya = 0.5 * stepa;
    if (t == 0) {
      acc = acc + carry;
      acca += carrya;
      if (!staps) {
        const node4<double> v0 = nodes[slot0];
        for (int i = 0; i < EPL; ++i) {
          if (!ok[i]) continue;
          double gz = 0.0;
          bulk_adj(g0[i], mk(q * v0.a + ex[i], ey[i]), mk(v0.dx, v0.dy), lam[i], acc, gz);
          acca += q * gz;
        }
      }
    }
    put_slot_grad(gV + (slot0 + t) * 3, acc.x, acc.y, acca, a.G, lane, false);
  }

  // ---- pass 3: adjoint of gamma~, forward, block by block
  C mu[EPL];
  C gprv[EPL];
  for (int i = 0; i < EPL; ++i) {
    mu[i] = mk(0.0, 0.0);
    gprv[i] = gt[i];
  }
  carry = mk(0.0, 0.0);
  carrya = 0.0;
  loaded = -1;
  for (int t = 0; t <= n; ++t) {
    if (t < n && t / CK != loaded) {
      loaded = t / CK;
      recompute_gamma(loaded);
      // gamma~ over the block, backward from the next block's first slot
      const int s0 = loaded * CK, s1 = min(s0 + CK, n);
      C gv[EPL];
      for (int i = 0; i < EPL; ++i) gv[i] = s1 == n ? gt0[i] : (ok[i] ? ck_at(ckgt, s1 / CK, i) : gt0[i]);
      for (int s = s1; s > s0; --s) {
        gammat_step(gv, s);
        for (int i = 0; i < EPL; ++i) sc_at(1, s - 1 - s0, i) = gv[i];
      }
    }
    C dm;
    double am;
    mid(t, dm, am);
    const double hs = hstep(t);
    const C dprime = mk(-dm.x, dm.y);
    C stepD = mk(0.0, 0.0);
    double stepa = 0.0;
    node4<double> v;
    double4 gs;
    if (t < n) {
      v = nodes[slot0 + t];
      gs = gS[slot0 + t];
    }
    for (int i = 0; i < EPL; ++i) {
      if (!ok[i]) continue;
      const C z = mk(q * am + ex[i], ey[i]);
      const C gu = t < n ? sc_at(1, t - loaded * CK, i) : gt0[i];
      const C gl = gprv[i];
      gprv[i] = gu;
      const StepDer sd = step_der(gu, gl, dprime, z, hs);
      const C l = mu[i];
      const C gdp = cconj(sd.dd) * l + sd.ddc * cconj(l);
      stepD = stepD - cconj(gdp);
      stepa += q * (cconj(l) * sd.dz).x;
      mu[i] = cconj(sd.dg) * l;
      if (t < n) {
        C lamd = mk(0.0, 0.0), accd = mk(0.0, 0.0), lv;
        node_adj(sc_at(0, t - loaded * CK, i), gu, mk(v.dx, v.dy), gs, rw[i], pt, lamd, lv, accd);
        mu[i] = mu[i] + lv;
      }
    }
    if (t == 0) {
      carry = stepD;
      carrya = stepa;
      if (n >= 1) continue;
    }
    C acc;
    double acca;
    int slot;
    if (t == 0) {
      acc = carry;
      acca = carrya;
      slot = 0;
    } else if (t < n) {
      acc = carry + cscale(0.5, stepD);
      acca = carrya + 0.5 * stepa;
      carry = cscale(0.5, stepD);
      carrya = 0.5 * stepa;
      slot = t - 1;
    } else {
      acc = carry + stepD;
      acca = carrya + stepa;
      slot = last;
    }
    if (t == n && !etaps) {
      const node4<double> v1 = nodes[slot0 + last];
      for (int i = 0; i < EPL; ++i) {
        if (!ok[i]) continue;
        double gz = 0.0;
        C gdp = mk(0.0, 0.0);
        bulk_adj(gt0[i], mk(q * v1.a + ex[i], ey[i]), mk(-v1.dx, v1.dy), mu[i], gdp, gz);
        acc = acc - cconj(gdp);
        acca += q * gz;
      }
    }
    put_slot_grad(gV + (slot0 + slot) * 3, acc.x, acc.y, acca, a.G, lane, true);
  }
}

// Gradients of the per-node sums from the cell gradients: the transpose of
// the rotate-back gather, formed as a gather per slot over the cells whose
// rotate-back stencil uses it (no atomics; each slot written once).
__global__ void __launch_bounds__(256) back_adjoint_kernel(BackAdjArgs a) {
  const int64_t s = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (s >= a.nslot) return;
  const int k = a.slot_angle[s];
  const double wk = a.wk[k], ck = a.cosk[k], sk = a.sink[k];
  double ex[4], ey[4];
  for (int g = 0; g < a.ncomp; ++g) {
    ex[g] = a.eta[2 * (g * a.n_theta + k)];
    ey[g] = a.eta[2 * (g * a.n_theta + k) + 1];
  }
  double sx = 0.0, sy = 0.0, sj = 0.0, sw = 0.0;
  for (int64_t e = a.bt_ptr[s]; e < a.bt_ptr[s + 1]; ++e) {
    const double w = a.bt_w[e];
    const int64_t cell = a.grain_cells[a.bt_c[e]];
    // G_{S_f} = wk sum_G eta_G G_{Num_G}, G_{Num_G} = G_{Delta_new,G} / den_G
    if (a.gdn) {
      double fx = 0.0, fy = 0.0;
      for (int g = 0; g < a.ncomp; ++g) {
        const double nx = a.gdn[2 * (g * a.ncell + cell)] / a.den[g];
        const double ny = a.gdn[2 * (g * a.ncell + cell) + 1] / a.den[g];
        fx += ex[g] * nx - ey[g] * ny;
        fy += ex[g] * ny + ey[g] * nx;
      }
      sx += w * fx;
      sy += w * fy;
    }
    if (a.gj) sj += w * (ck * a.gj[cell] + sk * a.gj[a.ncell + cell]);
    sw += w;
  }
  double4 o;
  o.x = wk * sx;
  o.y = wk * sy;
  o.z = a.four_q * wk * sj;
  o.w = wk * (-a.h2 * a.gomega) * sw;  // omega = ... - I
  reinterpret_cast<double4*>(a.gS)[s] = o;
}

// Gradients on the reference grid from the slot gradients: the transpose of
// the interpolation pre-pass, as a gather per cell over the slots whose
// stencils use it (each cell written once, zero where none does).  Sixteen
// lanes share a cell, lane q taking every 16th entry of its lists; their
// partial sums are combined with DPP moves.
constexpr int kItLanes = 16;
__global__ void __launch_bounds__(256) interp_adjoint_kernel(InterpAdjArgs a) {
  const int64_t t = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  const int64_t cell = t / kItLanes;
  const int q = static_cast<int>(t & (kItLanes - 1));
  if (cell >= a.ncell) return;  // whole groups of sixteen leave together
  double dx[4] = {0.0, 0.0, 0.0, 0.0}, dy[4] = {0.0, 0.0, 0.0, 0.0};
  for (int64_t e = a.it_dptr[cell] + q; e < a.it_dptr[cell + 1]; e += kItLanes) {
    const int64_t s = a.it_ds[e];
    const double w = a.it_dw[e];
    const int k = a.slot_angle[s];
    const double gx = a.gV[s * 3], gy = a.gV[s * 3 + 1];
    for (int g = 0; g < a.ncomp; ++g) {
      // y = eta w x  ->  G_x += conj(eta) w G_y
      const double ex = a.eta[2 * (g * a.n_theta + k)], ey = a.eta[2 * (g * a.n_theta + k) + 1];
      dx[g] += w * (ex * gx + ey * gy);
      dy[g] += w * (ex * gy - ey * gx);
    }
  }
  double ax = 0.0, ay = 0.0;
  for (int64_t e = a.it_aptr[cell] + q; e < a.it_aptr[cell + 1]; e += kItLanes) {
    const int64_t s = a.it_as[e];
    const double wg = a.it_aw[e] * a.gV[s * 3 + 2];
    const int k = a.slot_angle[s];
    ax += wg * a.cosk[k];
    ay += wg * a.sink[k];
  }
  for (int g = 0; g < a.ncomp; ++g) {
    dx[g] = group_sum(dx[g], kItLanes);
    dy[g] = group_sum(dy[g], kItLanes);
  }
  ax = group_sum(ax, kItLanes);
  ay = group_sum(ay, kItLanes);
  if (q != 0) return;
  for (int g = 0; g < a.ncomp; ++g) {
    a.gdelta[2 * (g * a.ncell + cell)] = dx[g];
    a.gdelta[2 * (g * a.ncell + cell) + 1] = dy[g];
  }
  a.gA[cell] = ax;
  a.gA[a.ncell + cell] = ay;
}

// explicit dependence of Omega on Delta at the cells:
// G_{Delta_G} += h^2 gOmega (2 ln(t/t_cG) Delta_G + 2 c sum_k w_k conj(eta_G,k) Delta_k)
__global__ void __launch_bounds__(256) omega_delta_adjoint_kernel(OmegaAdjArgs a) {
  const int64_t c = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= a.ncg) return;
  const int cell = a.grain_cells[c];
  constexpr int MAXC = 4;
  double dx[MAXC], dy[MAXC], ox[MAXC], oy[MAXC];
  for (int g = 0; g < a.ncomp; ++g) {
    dx[g] = a.delta[2 * (static_cast<int64_t>(g) * a.ncell + cell)];
    dy[g] = a.delta[2 * (static_cast<int64_t>(g) * a.ncell + cell) + 1];
    ox[g] = 2.0 * a.logt[g] * dx[g];
    oy[g] = 2.0 * a.logt[g] * dy[g];
  }
  for (int k = 0; k < a.n_theta; ++k) {
    double kx = 0.0, ky = 0.0;
    for (int g = 0; g < a.ncomp; ++g) {
      const double ex = a.eta[2 * (g * a.n_theta + k)], ey = a.eta[2 * (g * a.n_theta + k) + 1];
      kx += ex * dx[g] - ey * dy[g];
      ky += ex * dy[g] + ey * dx[g];
    }
    const double s = 2.0 * a.twopi_rz * a.wk[k];
    for (int g = 0; g < a.ncomp; ++g) {
      const double ex = a.eta[2 * (g * a.n_theta + k)], ey = a.eta[2 * (g * a.n_theta + k) + 1];
      ox[g] += s * (ex * kx + ey * ky);
      oy[g] += s * (ex * ky - ey * kx);
    }
  }
  const double f = a.h2 * a.gomega;
  for (int g = 0; g < a.ncomp; ++g) {
    a.gdelta[2 * (static_cast<int64_t>(g) * a.ncell + cell)] += f * ox[g];
    a.gdelta[2 * (static_cast<int64_t>(g) * a.ncell + cell) + 1] += f * oy[g];
  }
}

// transpose of the curl B = d_x A_y - d_y A_x (central, one-sided at the
// edges): gA += s * D^T B
__global__ void __launch_bounds__(256) curl_adjoint_kernel(const double* __restrict__ B, double* __restrict__ gA,
                                                           int nx, int ny, double h, double s) {
  const int64_t c = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (c >= static_cast<int64_t>(nx) * ny) return;
  const int i = static_cast<int>(c % nx), j = static_cast<int>(c / nx);
  // d_x A_y at column i' uses A_y[i] with weights: collect from B at i' = i-1, i, i+1
  double gy = 0.0;
  for (int ip = i - 1; ip <= i + 1; ++ip) {
    if (ip < 0 || ip >= nx) continue;
    double w = 0.0;
    if (ip == 0) {
      w = (i == 1 ? 1.0 : (i == 0 ? -1.0 : 0.0)) / h;
    } else if (ip == nx - 1) {
      w = (i == nx - 1 ? 1.0 : (i == nx - 2 ? -1.0 : 0.0)) / h;
    } else {
      w = (i == ip + 1 ? 1.0 : (i == ip - 1 ? -1.0 : 0.0)) / (2 * h);
    }
    gy += w * B[static_cast<int64_t>(j) * nx + ip];
  }
  double gx = 0.0;
  for (int jp = j - 1; jp <= j + 1; ++jp) {
    if (jp < 0 || jp >= ny) continue;
    double w = 0.0;
    if (jp == 0) {
      w = (j == 1 ? 1.0 : (j == 0 ? -1.0 : 0.0)) / h;
    } else if (jp == ny - 1) {
      w = (j == ny - 1 ? 1.0 : (j == ny - 2 ? -1.0 : 0.0)) / h;
    } else {
      w = (j == jp + 1 ? 1.0 : (j == jp - 1 ? -1.0 : 0.0)) / (2 * h);
    }
    gx -= w * B[static_cast<int64_t>(jp) * nx + i];
  }
  gA[c] += s * gx;
  gA[static_cast<int64_t>(nx) * ny + c] += s * gy;
}

static inline unsigned nb(int64_t n) { return static_cast<unsigned>((n + 255) / 256); }

void launch_adjoint(int epl, const AdjArgs& a, const AdjBufs& b, hipStream_t st) {
  const int64_t threads = a.nseg * a.G;
  if (b.ck > 0) {
#define QC_ADJC(E)                                                                                        \
  hipLaunchKernelGGL(adjoint_ckpt_kernel<E>, dim3(nb(threads)), dim3(256), 0, st, a,                      \
                     static_cast<const node4<double>*>(b.nodes), static_cast<const C*>(b.bc_g_prev),      \
                     static_cast<const C*>(b.bc_gt_prev), static_cast<const double4*>(b.gS), b.gV, b.ck,   \
                     b.ckbase, static_cast<C*>(b.ckg), static_cast<C*>(b.ckgt), static_cast<C*>(b.scr), b.nthr)
    if (epl == 1)
      QC_ADJC(1);
    else if (epl == 2)
      QC_ADJC(2);
    else if (epl == 3)
      QC_ADJC(3);
    else if (epl == 4)
      QC_ADJC(4);
    else
      QC_ADJC(8);
#undef QC_ADJC
    return;
  }
#define QC_ADJ(E)                                                                                        \
  hipLaunchKernelGGL(adjoint_kernel<E>, dim3(nb(threads)), dim3(256), 0, st, a,                          \
                     static_cast<const node4<double>*>(b.nodes), static_cast<const C*>(b.bc_g_prev),      \
                     static_cast<const C*>(b.bc_gt_prev), static_cast<C*>(b.gbuf), static_cast<C*>(b.gtbuf), \
                     static_cast<C*>(b.lgt), static_cast<const double4*>(b.gS), b.gV)
  if (epl == 1)
    QC_ADJ(1);
  else if (epl == 2)
    QC_ADJ(2);
  else if (epl == 3)
    QC_ADJ(3);
  else if (epl == 4)
    QC_ADJ(4);
  else
    QC_ADJ(8);
#undef QC_ADJ
}
void launch_back_adjoint(const BackAdjArgs& a, hipStream_t st) {
  if (a.nslot > 0) hipLaunchKernelGGL(back_adjoint_kernel, dim3(nb(a.nslot)), dim3(256), 0, st, a);
}
void launch_interp_adjoint(const InterpAdjArgs& a, hipStream_t st) {
  if (a.ncell > 0) hipLaunchKernelGGL(interp_adjoint_kernel, dim3(nb(a.ncell * kItLanes)), dim3(256), 0, st, a);
}
void launch_omega_delta_adjoint(const OmegaAdjArgs& a, hipStream_t st) {
  hipLaunchKernelGGL(omega_delta_adjoint_kernel, dim3(nb(a.ncg)), dim3(256), 0, st, a);
}
void launch_curl_adjoint(const double* B, double* gA, int nx, int ny, double h, double s, hipStream_t st) {
  hipLaunchKernelGGL(curl_adjoint_kernel, dim3(nb(static_cast<int64_t>(nx) * ny)), dim3(256), 0, st, B, gA, nx, ny,
                     h, s);
}

}  // namespace qc
