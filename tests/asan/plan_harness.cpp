// Host-side planner under AddressSanitizer / UndefinedBehaviorSanitizer:
// builds the trajectory tables of several grains (disc, regular polygon,
// convex polygon, cell mask, subtracted holes, odd and even angle counts)
// and the eigen-decomposition of the App. D kernel matrix, and checks a few
// invariants of the tables.  Built and run by tests/test_host_asan.py with
// g++ (host code only; no device code is involved).
#include <cmath>
#include <cstdio>
#include <vector>

#include "plan.hpp"

namespace {

int fails = 0;
void check(bool ok, const char* what) {
  if (!ok) {
    std::printf("FAIL: %s\n", what);
    ++fails;
  }
}

qc::Shape disc(double cx, double cy, double r, bool add) {
  qc::Shape s;
  s.kind = 0;
  s.cx = cx;
  s.cy = cy;
  s.r = r;
  s.add = add;
  return s;
}

qc::Shape polygon(std::vector<double> vx, std::vector<double> vy, bool add) {
  qc::Shape s;
  s.kind = 1;
  s.vx = vx;
  s.vy = vy;
  s.add = add;
  return s;
}

void run(const char* name, int nx, int ny, double h, int n_theta, int n_poles, std::vector<qc::Shape> shapes) {
  qc::Plan p;
  p.nx = nx;
  p.ny = ny;
  p.h = h;
  p.x0 = -0.5 * nx * h;
  p.y0 = -0.5 * ny * h;
  p.n_theta = n_theta;
  p.n_poles = n_poles;
  p.t = 0.4;
  p.ncomp = 1;
  p.tc_rel = {1.0};
  for (int k = 0; k < n_theta; ++k) p.eta.push_back(qc::basis_eta(1, 2.0 * M_PI * k / n_theta));
  p.kappa = 2.0;
  p.flux = 0.7;
  p.shapes = shapes;
  qc::build_plan(p);
  const int64_t nc = static_cast<int64_t>(p.grain_cells.size());
  check(nc > 0, "grain cells");
  check(static_cast<int64_t>(p.rb4.size()) == static_cast<int64_t>(n_theta) * nc * 4, "rotate-back table size");
  for (int64_t s = 0; s < p.nseg; ++s) {
    check(p.seg_smin[s] < p.seg_smax[s], "segment order");
    for (int c = 0; c < 4; ++c) check(p.tap_start_seg[s * 4 + c] >= 0 && p.tap_start_seg[s * 4 + c] < p.nseg, "tap range");
  }
  for (int32_t v : p.rb4) check(v >= -2 && v < p.nslot, "corner slot range");
  if (p.pair_ok)
    for (int64_t s = p.nseg_pair; s < p.nseg; ++s) check(p.seg_mirror[s] >= 0 && p.seg_mirror[s] < p.nseg_pair, "mirror");
  std::printf("%s: %lld segments, %lld slots, pairs %d\n", name, static_cast<long long>(p.nseg),
              static_cast<long long>(p.nslot), p.pair_ok ? 1 : 0);
}

}  // namespace

int main() {
  run("disc", 40, 40, 0.5, 16, 6, {disc(0.0, 0.0, 8.6, true)});
  run("holed", 36, 36, 0.5, 24, 6, {disc(0.0, 0.0, 8.6, true), disc(1.3, 0.4, 2.0, false)});
  run("polygon odd angles", 30, 26, 0.45, 15, 5,
      {polygon({-6.0, 5.5, 6.4, 0.5, -5.8}, {-5.0, -5.4, 1.0, 5.5, 3.0}, true)});
  run("square", 24, 24, 0.5, 32, 4, {polygon({-5.0, 5.0, 5.0, -5.0}, {-5.0, -5.0, 5.0, 5.0}, true)});
  {
    std::vector<uint8_t> m(30 * 34, 0);
    for (int j = 5; j < 25; ++j)
      for (int i = 4; i < 30; ++i)
        if ((i - 17) * (i - 17) + (j - 15) * (j - 15) < 90 && !(i == 20 && j == 15)) m[j * 34 + i] = 1;
    run("mask", 34, 30, 0.5, 16, 6, {qc::mask_shape(m.data(), 34, 30, -8.5, -7.5, 0.5, true)});
  }
  // eigen-decomposition of a symmetric kernel matrix
  const int n = 48;
  std::vector<double> a(n * n);
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) a[i * n + j] = std::log(1.0 + (i - j) * (i - j)) + 0.3 * (i == j);
  std::vector<double> lam, vec;
  qc::sym_eigen(n, a, lam, vec);
  double worst = 0.0;
  for (int k = 0; k < n; ++k)
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      for (int j = 0; j < n; ++j) s += a[i * n + j] * vec[j * n + k];
      worst = std::fmax(worst, std::fabs(s - lam[k] * vec[i * n + k]));
    }
  check(worst < 1e-10, "eigen residual");
  std::printf("eigen residual %.3g\n", worst);
  std::printf(fails ? "FAILED\n" : "OK\n");
  return fails ? 1 : 0;
}
