// Host-side trajectory tables (Sec. III.A of arXiv:2205.15000); see plan.hpp.
#include "plan.hpp"

#include <algorithm>
#include <array>
#include <cmath>
#include <limits>
#include <stdexcept>
#include <utility>

namespace qc {

namespace {

constexpr double kPi = 3.14159265358979323846;

bool inside(const Shape& sh, double x, double y) {
  if (sh.kind == 0) {
    const double dx = x - sh.cx, dy = y - sh.cy;
    return dx * dx + dy * dy <= sh.r * sh.r;
  }
  if (sh.kind == 2) {
    // even-odd rule: crossings of the ray to +x, each edge half-open in y
    bool in = false;
    for (size_t m = 0; m < sh.ax.size(); ++m) {
      if ((sh.ay[m] > y) == (sh.by[m] > y)) continue;
      const double xi = sh.ax[m] + (y - sh.ay[m]) * (sh.bx[m] - sh.ax[m]) / (sh.by[m] - sh.ay[m]);
      if (x < xi) in = !in;
    }
    return in;
  }
  const size_t n = sh.vx.size();
  for (size_t m = 0; m < n; ++m) {
    const double ax = sh.vx[m], ay = sh.vy[m];
    const double bx = sh.vx[(m + 1) % n], by = sh.vy[(m + 1) % n];
    const double cr = (bx - ax) * (y - ay) - (by - ay) * (x - ax);
    if (!(cr >= 0.0)) return false;
  }
  return true;
}

// The grain as the ordered fold of its components (App. B).
bool in_grain(const std::vector<Shape>& shapes, double x, double y) {
  bool d = false;
  for (const Shape& sh : shapes) {
    const bool in = inside(sh, x, y);
    d = sh.add ? (d || in) : (d && !in);
  }
  return d;
}

struct Hit {
  double s;
  double tangent;
};

// Intersections of the line B + s e with every component boundary.
std::vector<Hit> boundary_hits(const std::vector<Shape>& shapes, double bx, double by,
                               double ex, double ey) {
  std::vector<Hit> hits;
  for (const Shape& sh : shapes) {
    if (sh.kind == 0) {
      const double dx = bx - sh.cx, dy = by - sh.cy;
      const double bq = dx * ex + dy * ey;
      const double cq = dx * dx + dy * dy - sh.r * sh.r;
      const double disc = bq * bq - cq;
      if (disc > 0.0) {
        const double rt = std::sqrt(disc);
        const double ss[2] = {-bq - rt, -bq + rt};
        for (double s : ss) {
          const double px = bx + s * ex, py = by + s * ey;
          hits.push_back({s, std::atan2(py - sh.cy, px - sh.cx) + 0.5 * kPi});
        }
      }
    } else if (sh.kind == 2) {
      // the polygon-edge formula, per contour edge
      for (size_t m = 0; m < sh.ax.size(); ++m) {
        const double dx = sh.bx[m] - sh.ax[m], dy = sh.by[m] - sh.ay[m];
        const double den = ex * dy - ey * dx;
        if (den == 0.0) continue;
        const double wx = sh.ax[m] - bx, wy = sh.ay[m] - by;
        const double s = (wx * dy - wy * dx) / den;
        const double tt = (wx * ey - wy * ex) / den;
        if (tt >= 0.0 && tt <= 1.0) hits.push_back({s, std::atan2(dy, dx)});
      }
    } else {
      const size_t n = sh.vx.size();
      for (size_t m = 0; m < n; ++m) {
        const double ax = sh.vx[m], ay = sh.vy[m];
        const double dx = sh.vx[(m + 1) % n] - ax, dy = sh.vy[(m + 1) % n] - ay;
        const double den = ex * dy - ey * dx;
        if (den == 0.0) continue;
        const double wx = ax - bx, wy = ay - by;
        const double s = (wx * dy - wy * dx) / den;
        const double tt = (wx * ey - wy * ex) / den;
        if (tt >= 0.0 && tt <= 1.0) hits.push_back({s, std::atan2(dy, dx)});
      }
    }
  }
  std::stable_sort(hits.begin(), hits.end(), [](const Hit& a, const Hit& b) { return a.s < b.s; });
  return hits;
}

struct Seg {
  double s0, s1, t0, t1;
};

// Maximal D-intervals of a line: the sorted hits cut it into pieces, a piece
// belongs to D when its midpoint does, adjacent D-pieces merge; pieces
// shorter than 1e-9 h are skipped.
std::vector<Seg> line_segments(const std::vector<Shape>& shapes, double bx, double by,
                               double ex, double ey, double h) {
  const std::vector<Hit> hits = boundary_hits(shapes, bx, by, ex, ey);
  std::vector<Seg> out;
  const double tol = 1e-9 * h;
  bool open = false;
  Hit start{0, 0}, end{0, 0};
  for (size_t a = 0; a + 1 < hits.size(); ++a) {
    const Hit& ha = hits[a];
    const Hit& hb = hits[a + 1];
    if (hb.s - ha.s <= tol) continue;
    const double sm = 0.5 * (ha.s + hb.s);
    const bool in = in_grain(shapes, bx + sm * ex, by + sm * ey);
    if (in) {
      if (!open) {
        start = ha;
        open = true;
      }
      end = hb;
    } else if (open) {
      out.push_back({start.s, end.s, start.tangent, end.tangent});
      open = false;
    }
  }
  if (open) out.push_back({start.s, end.s, start.tangent, end.tangent});
  return out;
}

void external_A(const Plan& p, double x, double y, double& ax, double& ay) {
  const double dx = x - p.cx, dy = y - p.cy;
  ax = 0.0;
  ay = 0.0;
  if (p.flux == 0.0) return;
  if (p.gauge == 0) {  // symmetric
    const double b = kPi * p.flux / p.area;
    ax = -0.5 * b * dy;
    ay = 0.5 * b * dx;
  } else if (p.gauge == 1) {  // landau
    const double b = kPi * p.flux / p.area;
    ax = -b * dy;
    ay = 0.0;
  } else {  // solenoid
    const double r2 = dx * dx + dy * dy;
    if (r2 > 0.0) {
      ax = -0.5 * p.flux * dy / r2;
      ay = 0.5 * p.flux * dx / r2;
    }
  }
}

}  // namespace

std::complex<double> basis_eta(int kind, double phi) {
  const double r2 = std::sqrt(2.0);
  switch (kind) {
    case 0: return {1.0, 0.0};
    case 1: return {r2 * std::cos(2.0 * phi), 0.0};
    case 2: return {r2 * std::sin(2.0 * phi), 0.0};
    case 3: return {r2 * std::sin(4.0 * phi), 0.0};
    default: throw std::runtime_error("unknown basis function");
  }
}

std::vector<double> fs_weights(int n) {
  std::vector<double> pat;
  if (n % 4 == 0)
    pat = {14.0, 32.0, 12.0, 32.0};
  else if (n % 3 == 0)
    pat = {2.0, 3.0, 3.0};
  else if (n % 2 == 0)
    pat = {2.0, 4.0};
  else
    pat = {1.0};
  std::vector<double> w(n);
  double tot = 0.0;
  for (int k = 0; k < n; ++k) {
    w[k] = pat[k % pat.size()];
    tot += w[k];
  }
  for (double& v : w) v /= tot;
  return w;
}

void ozaki_table(int n_poles, std::vector<double>& z, std::vector<double>& r) {
  // Continued-fraction matrix of the Fermi function: zero diagonal,
  // off-diagonal b_m = 1/(2 sqrt((2m-1)(2m+1))).  Its positive eigenvalues
  // lam_p give the poles z_p = 1/lam_p and, with the first component v0 of
  // the normalised eigenvector, the residues R_p = v0^2/(4 lam_p^2).
  // Cyclic Jacobi rotations on the dense symmetric matrix; only row 0 of
  // the eigenvector matrix is needed and tracked.
  const int n = 2 * n_poles;
  std::vector<double> a(static_cast<size_t>(n) * n, 0.0);
  for (int m = 1; m < n; ++m) {
    const double b = 1.0 / (2.0 * std::sqrt((2.0 * m - 1.0) * (2.0 * m + 1.0)));
    a[(m - 1) * n + m] = b;
    a[m * n + m - 1] = b;
  }
  std::vector<double> v0(n, 0.0);
  v0[0] = 1.0;
  for (int sweep = 0; sweep < 100; ++sweep) {
    double off = 0.0;
    for (int p = 0; p < n; ++p)
      for (int q = p + 1; q < n; ++q) off += a[p * n + q] * a[p * n + q];
    if (off < 1e-60) break;
    for (int p = 0; p < n; ++p) {
      for (int q = p + 1; q < n; ++q) {
        const double apq = a[p * n + q];
        if (apq == 0.0) continue;
        const double app = a[p * n + p], aqq = a[q * n + q];
        const double theta = (aqq - app) / (2.0 * apq);
        const double tt = (theta >= 0.0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(tt * tt + 1.0);
        const double s = tt * c;
        // A <- J^T A J with J the rotation in the (p, q) plane
        for (int k = 0; k < n; ++k) {
          const double akp = a[k * n + p], akq = a[k * n + q];
          a[k * n + p] = c * akp - s * akq;
          a[k * n + q] = s * akp + c * akq;
        }
        for (int k = 0; k < n; ++k) {
          const double apk = a[p * n + k], aqk = a[q * n + k];
          a[p * n + k] = c * apk - s * aqk;
          a[q * n + k] = s * apk + c * aqk;
        }
        const double vp = v0[p], vq = v0[q];
        v0[p] = c * vp - s * vq;
        v0[q] = s * vp + c * vq;
      }
    }
  }
  std::vector<std::pair<double, double>> ev;  // (lambda, v0)
  for (int k = 0; k < n; ++k)
    if (a[k * n + k] > 0.0) ev.push_back({a[k * n + k], v0[k]});
  std::sort(ev.begin(), ev.end(), [](const auto& x, const auto& y) { return x.first > y.first; });
  z.resize(ev.size());
  r.resize(ev.size());
  for (size_t k = 0; k < ev.size(); ++k) {
    const double lam = ev[k].first;
    z[k] = 1.0 / lam;
    r[k] = ev[k].second * ev[k].second / (4.0 * lam * lam);
  }
}

// T = Q^T A Q by Householder reflections H = I - 2 v v^T, each zeroing one
// column below the subdiagonal (A22 <- A22 - v w^T - w v^T with
// w = 2 (A22 v - (v.A22 v) v)), Q accumulated as H_0 H_1 ...; then implicit
// QR steps on the unreduced trailing block of T: a Wilkinson shift from its
// last 2 x 2, a Givens rotation from the shifted first column, the bulge
// chased down with rotations that zero it, every rotation applied to the
// columns of Q.  Off-diagonals below 1e-16 (|d_i| + |d_i+1|) are dropped.
void sym_eigen(int n, std::vector<double> a, std::vector<double>& lam, std::vector<double>& z) {
  auto A = [&](int r, int c) -> double& { return a[static_cast<size_t>(r) * n + c]; };
  z.assign(static_cast<size_t>(n) * n, 0.0);
  for (int i = 0; i < n; ++i) z[static_cast<size_t>(i) * n + i] = 1.0;
  std::vector<double> v(n), p(n), w(n);
  // ---- Householder: zero column k below the subdiagonal
  for (int k = 0; k + 2 < n; ++k) {
    const int m = n - k - 1;  // length of x = A[k+1:, k]
    double nx = 0.0;
    for (int i = 0; i < m; ++i) nx += A(k + 1 + i, k) * A(k + 1 + i, k);
    nx = std::sqrt(nx);
    if (nx == 0.0) continue;
    const double x0 = A(k + 1, k);
    const double alpha = x0 >= 0.0 ? -nx : nx;
    for (int i = 0; i < m; ++i) v[i] = A(k + 1 + i, k);
    v[0] -= alpha;
    double nv = 0.0;
    for (int i = 0; i < m; ++i) nv += v[i] * v[i];
    nv = std::sqrt(nv);
    if (nv == 0.0) continue;
    for (int i = 0; i < m; ++i) v[i] /= nv;
    // p = A22 v, K = v.p, w = 2 (p - K v); A22 <- A22 - v w^T - w v^T
    double K = 0.0;
    for (int i = 0; i < m; ++i) {
      double s = 0.0;
      const double* row = &a[static_cast<size_t>(k + 1 + i) * n + k + 1];
      for (int j = 0; j < m; ++j) s += row[j] * v[j];
      p[i] = s;
      K += v[i] * s;
    }
    for (int i = 0; i < m; ++i) w[i] = 2.0 * (p[i] - K * v[i]);
    for (int i = 0; i < m; ++i) {
      double* row = &a[static_cast<size_t>(k + 1 + i) * n + k + 1];
      for (int j = 0; j < m; ++j) row[j] -= v[i] * w[j] + w[i] * v[j];
    }
    A(k + 1, k) = alpha;
    A(k, k + 1) = alpha;
    for (int i = 1; i < m; ++i) {
      A(k + 1 + i, k) = 0.0;
      A(k, k + 1 + i) = 0.0;
    }
    // Q <- Q H: columns k+1.. of every row: row <- row - 2 (row . v) v
    for (int r = 0; r < n; ++r) {
      double* row = &z[static_cast<size_t>(r) * n + k + 1];
      double s = 0.0;
      for (int j = 0; j < m; ++j) s += row[j] * v[j];
      s *= 2.0;
      for (int j = 0; j < m; ++j) row[j] -= s * v[j];
    }
  }
  std::vector<double> d(n), e(std::max(n - 1, 1), 0.0);
  for (int i = 0; i < n; ++i) d[i] = A(i, i);
  for (int i = 0; i + 1 < n; ++i) e[i] = A(i + 1, i);
  // ---- implicit QR on the tridiagonal matrix
  int m = n - 1;
  int guard = 0;
  while (m > 0) {
    if (guard > 100 * n) throw std::runtime_error("sym_eigen: the QR iteration did not converge");
    // deflate negligible off-diagonals at the bottom
    if (std::fabs(e[m - 1]) <= 1e-16 * (std::fabs(d[m - 1]) + std::fabs(d[m]))) {
      e[m - 1] = 0.0;
      --m;
      continue;
    }
    int l = m - 1;
    while (l > 0 && std::fabs(e[l - 1]) > 1e-16 * (std::fabs(d[l - 1]) + std::fabs(d[l]))) --l;
    if (l > 0) e[l - 1] = 0.0;
    ++guard;
    // Wilkinson shift from the trailing 2 x 2 block
    const double del = 0.5 * (d[m - 1] - d[m]);
    const double b2 = e[m - 1] * e[m - 1];
    const double mu = d[m] - b2 / (del + (del >= 0.0 ? 1.0 : -1.0) * std::sqrt(del * del + b2));
    double pp = d[l] - mu, qq = e[l];
    for (int k = l; k < m; ++k) {
      const double r = std::hypot(pp, qq);
      const double c = r > 0.0 ? pp / r : 1.0, s = r > 0.0 ? qq / r : 0.0;
      if (k > l) e[k - 1] = r;
      const double Aa = d[k], B = e[k], C = d[k + 1];
      d[k] = c * c * Aa + 2.0 * c * s * B + s * s * C;
      d[k + 1] = s * s * Aa - 2.0 * c * s * B + c * c * C;
      e[k] = c * s * (C - Aa) + (c * c - s * s) * B;
      if (k + 1 < m) {
        const double D = e[k + 1];
        qq = s * D;       // the bulge T[k][k+2]
        e[k + 1] = c * D;
        pp = e[k];
      }
      for (int r2 = 0; r2 < n; ++r2) {
        double* row = &z[static_cast<size_t>(r2) * n];
        const double zk = row[k], zk1 = row[k + 1];
        row[k] = c * zk + s * zk1;
        row[k + 1] = -s * zk + c * zk1;
      }
    }
  }
  lam = d;
}

int64_t Plan::steps_per_sweep() const {
  int64_t s = 0;
  for (int64_t k = 0; k < nseg; ++k) s += seg_n[k] + 1;
  return 2 * static_cast<int64_t>(n_poles) * s;
}

Shape mask_shape(const uint8_t* mask, int nx, int ny, double x0, double y0, double h, bool add) {
  // contour pieces per square by inside corners (1 lower-left, 2 lower-right,
  // 4 upper-right, 8 upper-left); 0..3 = side midpoints B, R, T, L
  static const int kPieces[16][4] = {
      {-1, -1, -1, -1}, {3, 0, -1, -1}, {0, 1, -1, -1}, {3, 1, -1, -1},
      {1, 2, -1, -1},   {3, 0, 1, 2},   {0, 2, -1, -1}, {3, 2, -1, -1},
      {2, 3, -1, -1},   {0, 2, -1, -1}, {0, 1, 2, 3},   {1, 2, -1, -1},
      {3, 1, -1, -1},   {0, 1, -1, -1}, {3, 0, -1, -1}, {-1, -1, -1, -1}};
  auto val = [&](int i, int j) {
    return i >= 0 && i < nx && j >= 0 && j < ny && mask[static_cast<size_t>(j) * nx + i] != 0;
  };
  Shape sh;
  sh.kind = 2;
  sh.add = add;
  for (int j = -1; j < ny; ++j)
    for (int i = -1; i < nx; ++i) {
      const int c = (val(i, j) ? 1 : 0) | (val(i + 1, j) ? 2 : 0) | (val(i + 1, j + 1) ? 4 : 0) |
                    (val(i, j + 1) ? 8 : 0);
      const double px[4] = {x0 + (i + 1) * h, x0 + (i + 1.5) * h, x0 + (i + 1) * h, x0 + (i + 0.5) * h};
      const double py[4] = {y0 + (j + 0.5) * h, y0 + (j + 1) * h, y0 + (j + 1.5) * h, y0 + (j + 1) * h};
      for (int q = 0; q < 4 && kPieces[c][q] >= 0; q += 2) {
        sh.ax.push_back(px[kPieces[c][q]]);
        sh.ay.push_back(py[kPieces[c][q]]);
        sh.bx.push_back(px[kPieces[c][q + 1]]);
        sh.by.push_back(py[kPieces[c][q + 1]]);
      }
    }
  return sh;
}

// Angle k + n_theta/2 has the lattice of angle k with both axes reversed:
// line i, node j there is the point of line M-1-i, node M-1-j of angle k.
// Along such a pair of lines gamma~ of one direction is the complex
// conjugate of gamma of the other for an order parameter that is even in
// the momentum direction (singlet pairing), so one march serves both.  The
// tables of the two angles are built independently; pairing is enabled
// only where they agree: same segments with the same node counts, slot
// positions within 1e-9 h, the same fallback cells, equal weights and
// basis values.
static void build_pairs(Plan& p) {
  p.pair_ok = false;
  p.seg_mirror.assign(static_cast<size_t>(p.nseg), -1);
  p.rb4_pair.clear();
  p.nseg_pair = p.nseg;
  p.nslot_pair = p.nslot;
  const int n = p.n_theta, M = p.M;
  if (n < 2 || n % 2 != 0) return;
  const int n2 = n / 2;
  for (int k = 0; k < n2; ++k) {
    if (std::fabs(p.wk[k + n2] - p.wk[k]) > 1e-14 * p.wk[k]) return;
  }
  double emax = 0.0;
  for (const auto& e : p.eta) emax = std::max(emax, std::abs(e));
  for (int g = 0; g < p.ncomp; ++g)
    for (int k = 0; k < n2; ++k)
      if (std::abs(p.eta[static_cast<size_t>(g) * n + k + n2] - p.eta[static_cast<size_t>(g) * n + k]) >
          1e-14 * emax)
        return;
  std::vector<int64_t> slot_mirror(static_cast<size_t>(p.nslot), -1);
  const double tol = 1e-9 * p.h;
  for (int k = n2; k < n; ++k) {
    for (int i = 0; i < M; ++i) {
      const int64_t a0 = p.line_seg0[static_cast<size_t>(k) * (M + 1) + i];
      const int64_t a1 = p.line_seg0[static_cast<size_t>(k) * (M + 1) + i + 1];
      const int64_t b0 = p.line_seg0[static_cast<size_t>(k - n2) * (M + 1) + (M - 1 - i)];
      const int64_t b1 = p.line_seg0[static_cast<size_t>(k - n2) * (M + 1) + (M - 1 - i) + 1];
      if (a1 - a0 != b1 - b0) return;
      for (int64_t q = 0; q < a1 - a0; ++q) {
        const int64_t sa = a0 + q, sb = b1 - 1 - q;  // segments run the other way
        const int na = p.seg_n[sa];
        if (p.seg_n[sb] != na) return;
        if (na > 0 && p.seg_jfirst[sb] != M - p.seg_jfirst[sa] - na) return;
        const int nsl = std::max(na, 1);
        for (int t = 0; t < nsl; ++t) {
          const int64_t la = p.seg_slot0[sa] + t, lb = p.seg_slot0[sb] + (nsl - 1 - t);
          if (std::fabs(p.slot_px[la] - p.slot_px[lb]) > tol || std::fabs(p.slot_py[la] - p.slot_py[lb]) > tol)
            return;
          if (p.slot_fb[la] != p.slot_fb[lb]) return;
          slot_mirror[la] = lb;
        }
        p.seg_mirror[sa] = static_cast<int32_t>(sb);
      }
    }
  }
  // The boundary taps of an upper segment must be the mirror image of its
  // mirror's (start taps of s' against end taps of s and vice versa: the
  // same weights on mirrored segments), so that its start values are the
  // conjugates of its mirror's.  A line through a corner of the boundary
  // can record a different wall tangent in the two directions; such grains
  // keep every angle.
  std::vector<int32_t> partner(static_cast<size_t>(p.nseg), -1);
  for (int64_t sg = 0; sg < p.nseg; ++sg)
    if (p.seg_mirror[sg] >= 0) {
      partner[sg] = p.seg_mirror[sg];
      partner[p.seg_mirror[sg]] = static_cast<int32_t>(sg);
    }
  for (int64_t sg = 0; sg < p.nseg; ++sg) {
    if (p.seg_mirror[sg] < 0) continue;
    const int64_t mg = p.seg_mirror[sg];
    for (int side = 0; side < 2; ++side) {
      // side 0: start taps of sg vs end taps of mg; side 1: the reverse
      const int32_t* ta = side == 0 ? &p.tap_start_seg[sg * 4] : &p.tap_end_seg[sg * 4];
      const double* wa = side == 0 ? &p.tap_start_w[sg * 4] : &p.tap_end_w[sg * 4];
      const int32_t* tb = side == 0 ? &p.tap_end_seg[mg * 4] : &p.tap_start_seg[mg * 4];
      const double* wb = side == 0 ? &p.tap_end_w[mg * 4] : &p.tap_start_w[mg * 4];
      for (int a = 0; a < 4; ++a) {
        if (wa[a] == 0.0) continue;
        // the mirrored tap must appear on the other side with its weight
        double wsum = 0.0;
        for (int b = 0; b < 4; ++b)
          if (wb[b] != 0.0 && tb[b] == partner[ta[a]]) wsum += wb[b];
        double wself = 0.0;
        for (int c = 0; c < 4; ++c)
          if (wa[c] != 0.0 && ta[c] == ta[a]) wself += wa[c];
        if (std::fabs(wsum - wself) > 1e-12) return;
      }
      double na = 0.0, nb = 0.0;
      for (int a = 0; a < 4; ++a) {
        na += wa[a];
        nb += wb[a];
      }
      if ((na > 0.0) != (nb > 0.0)) return;
    }
  }
  const int64_t nc = static_cast<int64_t>(p.grain_cells.size());
  p.rb4_pair = p.rb4;
  for (size_t i = static_cast<size_t>(n2) * nc * 4; i < p.rb4_pair.size(); ++i) {
    const int32_t v = p.rb4_pair[i];
    if (v >= 0) {
      if (slot_mirror[v] < 0) throw std::runtime_error("angle pairs: rotate-back corner without a mirror");
      p.rb4_pair[i] = static_cast<int32_t>(slot_mirror[v]);
    }
  }
  p.nseg_pair = p.angle_seg0[n2];
  p.nslot_pair = p.seg_slot0[p.nseg_pair];
  p.pair_ok = true;
  // The lattice of angle k + n/2 is that of angle k turned by pi about the
  // grid centre, so a cell's bilinear corners are the same points with the
  // same weights.  Check that the tables agree, to rounding, on every corner
  // of weight above 1e-12 (a cell centre on a lattice line picks its
  // zero-weight corner on opposite sides in the two directions, or gives it
  // a weight of the size of the rounding of cos and sin) and on the
  // nearest-node fallback, whose tie-break could differ.
  p.rb_fold = true;
  for (int k = 0; k < n2 && p.rb_fold; ++k)
    for (int64_t c = 0; c < nc && p.rb_fold; ++c) {
      std::array<std::pair<int32_t, double>, 4> lo, up;
      int nlo = 0, nup = 0;
      for (int q = 0; q < 4; ++q) {
        const double wl = p.rb_w[(static_cast<size_t>(k) * 4 + q) * nc + c];
        const double wh = p.rb_w[(static_cast<size_t>(k + n2) * 4 + q) * nc + c];
        if (wl > 1e-12) lo[nlo++] = {p.rb4_pair[(static_cast<size_t>(k) * nc + c) * 4 + q], wl};
        if (wh > 1e-12) up[nup++] = {p.rb4_pair[(static_cast<size_t>(k + n2) * nc + c) * 4 + q], wh};
      }
      if (nlo != nup) {
        p.rb_fold = false;
        break;
      }
      std::sort(lo.begin(), lo.begin() + nlo);
      std::sort(up.begin(), up.begin() + nup);
      for (int q = 0; q < nlo; ++q)
        if (lo[q].first != up[q].first || std::fabs(lo[q].second - up[q].second) > 1e-12) {
          p.rb_fold = false;
          break;
        }
    }
}

void build_plan(Plan& p) {
  if (p.nx < 2 || p.ny < 2) throw std::runtime_error("grid must be at least 2x2");
  if (!(p.h > 0.0) || !std::isfinite(p.h)) throw std::runtime_error("h must be > 0");
  if (p.n_theta < 1) throw std::runtime_error("n_theta must be >= 1");
  if (p.n_poles < 1) throw std::runtime_error("n_poles must be >= 1");
  if (!(p.t > 0.0)) throw std::runtime_error("t must be > 0");
  if (p.ncomp < 1) throw std::runtime_error("ncomp must be >= 1");
  if (p.shapes.empty()) throw std::runtime_error("no geometry component");

  p.cx = p.x0 + 0.5 * p.nx * p.h;
  p.cy = p.y0 + 0.5 * p.ny * p.h;
  const int nx = p.nx, ny = p.ny;
  const double h = p.h;

  // ---- mask
  p.mask.assign(static_cast<size_t>(nx) * ny, 0);
  p.grain_cells.clear();
  for (int j = 0; j < ny; ++j)
    for (int i = 0; i < nx; ++i) {
      const double x = p.x0 + (i + 0.5) * h, y = p.y0 + (j + 0.5) * h;
      if (in_grain(p.shapes, x, y)) {
        p.mask[static_cast<size_t>(j) * nx + i] = 1;
        p.grain_cells.push_back(j * nx + i);
      }
    }
  if (p.grain_cells.empty()) throw std::runtime_error("the grain covers no cell centre");
  p.area = h * h * static_cast<double>(p.grain_cells.size());

  // ---- lattice, angles, tables
  p.M = static_cast<int>(std::ceil(std::sqrt(static_cast<double>(nx) * nx + static_cast<double>(ny) * ny) + 3.0));
  if ((p.M - nx) % 2 != 0) p.M += 1;
  const int M = p.M;
  p.half = 0.5 * (M - 1);
  const double half = p.half;
  p.phi.resize(p.n_theta);
  p.cosk.resize(p.n_theta);
  p.sink.resize(p.n_theta);
  for (int k = 0; k < p.n_theta; ++k) {
    p.phi[k] = 2.0 * kPi * k / p.n_theta;
    p.cosk[k] = std::cos(p.phi[k]);
    p.sink[k] = std::sin(p.phi[k]);
  }
  p.wk = fs_weights(p.n_theta);
  ozaki_table(p.n_poles, p.zp, p.rp);

  // ---- segments
  p.seg_angle.clear(); p.seg_line.clear(); p.seg_jfirst.clear(); p.seg_n.clear();
  p.seg_smin.clear(); p.seg_smax.clear(); p.seg_tmin.clear(); p.seg_tmax.clear();
  p.angle_seg0.assign(p.n_theta + 1, 0);
  p.line_seg0.assign(static_cast<size_t>(p.n_theta) * (M + 1), 0);
  for (int k = 0; k < p.n_theta; ++k) {
    p.angle_seg0[k] = static_cast<int64_t>(p.seg_angle.size());
    const double epx = p.cosk[k], epy = p.sink[k];
    const double eqx = p.sink[k], eqy = -p.cosk[k];
    for (int i = 0; i < M; ++i) {
      p.line_seg0[static_cast<size_t>(k) * (M + 1) + i] = static_cast<int64_t>(p.seg_angle.size());
      const double u = (i - half) * h;
      const double bx = p.cx + u * eqx, by = p.cy + u * eqy;
      for (const Seg& sg : line_segments(p.shapes, bx, by, epx, epy, h)) {
        const int jf = static_cast<int>(std::floor(sg.s0 / h + half)) + 1;
        const int jl = static_cast<int>(std::ceil(sg.s1 / h + half)) - 1;
        p.seg_angle.push_back(k);
        p.seg_line.push_back(i);
        p.seg_jfirst.push_back(jf);
        p.seg_n.push_back(std::max(0, jl - jf + 1));
        p.seg_smin.push_back(sg.s0);
        p.seg_smax.push_back(sg.s1);
        p.seg_tmin.push_back(sg.t0);
        p.seg_tmax.push_back(sg.t1);
      }
    }
    p.line_seg0[static_cast<size_t>(k) * (M + 1) + M] = static_cast<int64_t>(p.seg_angle.size());
  }
  p.angle_seg0[p.n_theta] = static_cast<int64_t>(p.seg_angle.size());
  p.nseg = static_cast<int64_t>(p.seg_angle.size());
  if (p.nseg == 0) throw std::runtime_error("no trajectory crosses the grain");
  if (p.nseg > std::numeric_limits<int32_t>::max() / 2) throw std::runtime_error("too many segments");

  // ---- value slots
  p.seg_slot0.resize(p.nseg);
  p.seg_hfirst.resize(p.nseg);
  p.seg_hlast.resize(p.nseg);
  int64_t ns = 0, nn = 0;
  for (int64_t g = 0; g < p.nseg; ++g) {
    p.seg_slot0[g] = ns;
    ns += std::max(p.seg_n[g], 1);
    nn += p.seg_n[g];
  }
  if (ns > std::numeric_limits<int32_t>::max()) throw std::runtime_error("too many lattice nodes");
  p.nslot = ns;
  p.nnode = nn;
  p.slot_angle.resize(ns);
  p.slot_seg.resize(ns);
  p.slot_px.assign(ns, 0.0);
  p.slot_py.assign(ns, 0.0);
  p.slot_fb.assign(ns, -1);
  p.slot_aext.assign(ns, 0.0);
  std::vector<double> gx, gy;  // grain cell centres, for the nearest-cell fallback
  for (int32_t c : p.grain_cells) {
    gx.push_back(p.x0 + (c % nx + 0.5) * h);
    gy.push_back(p.y0 + (c / nx + 0.5) * h);
  }
  for (int64_t g = 0; g < p.nseg; ++g) {
    const int k = p.seg_angle[g];
    const double epx = p.cosk[k], epy = p.sink[k];
    const double eqx = p.sink[k], eqy = -p.cosk[k];
    const int n = p.seg_n[g], jf = p.seg_jfirst[g];
    const double u = (p.seg_line[g] - half) * h;
    if (n > 0) {
      p.seg_hfirst[g] = (jf - half) * h - p.seg_smin[g];
      p.seg_hlast[g] = p.seg_smax[g] - (jf + n - 1 - half) * h;
    } else {
      p.seg_hfirst[g] = p.seg_smax[g] - p.seg_smin[g];
      p.seg_hlast[g] = 0.0;
    }
    const int nsl = std::max(n, 1);
    for (int t = 0; t < nsl; ++t) {
      const int64_t sl = p.seg_slot0[g] + t;
      p.slot_angle[sl] = k;
      p.slot_seg[sl] = static_cast<int32_t>(g);
      const double s = n > 0 ? (jf + t - half) * h : 0.5 * (p.seg_smin[g] + p.seg_smax[g]);
      const double px = p.cx + u * eqx + s * epx;
      const double py = p.cy + u * eqy + s * epy;
      p.slot_px[sl] = px;
      p.slot_py[sl] = py;
      // Delta: masked bilinear over the four surrounding cell centres (the
      // device forms the weights); only the fallback is decided here: the
      // nearest grain cell when no masked corner keeps a positive weight
      {
        const double fx = (px - p.x0) / h - 0.5, fy = (py - p.y0) / h - 0.5;
        const int i0 = static_cast<int>(std::floor(fx)), j0 = static_cast<int>(std::floor(fy));
        const double wx = fx - i0, wy = fy - j0;
        const int ci[4] = {i0, i0 + 1, i0, i0 + 1};
        const int cj[4] = {j0, j0, j0 + 1, j0 + 1};
        const double w[4] = {(1 - wx) * (1 - wy), wx * (1 - wy), (1 - wx) * wy, wx * wy};
        double tot = 0.0;
        for (int c = 0; c < 4; ++c) {
          const bool ok = ci[c] >= 0 && ci[c] < nx && cj[c] >= 0 && cj[c] < ny &&
                          p.mask[static_cast<size_t>(cj[c]) * nx + ci[c]];
          if (ok) tot += w[c];
        }
        if (!(tot > 0.0)) {
          size_t best = 0;
          double bd = std::numeric_limits<double>::infinity();
          for (size_t a = 0; a < gx.size(); ++a) {
            const double d2 = (gx[a] - px) * (gx[a] - px) + (gy[a] - py) * (gy[a] - py);
            if (d2 < bd) {
              bd = d2;
              best = a;
            }
          }
          p.slot_fb[sl] = p.grain_cells[best];
        }
      }
      double ax, ay;
      external_A(p, px, py, ax, ay);
      p.slot_aext[sl] = epx * ax + epy * ay;
    }
  }

  // ---- order of the per-cell kernels: 16 x 16 tiles of the grid, row-major
  // inside a tile, so that a block of 256 threads covers a compact patch and
  // neighbouring cells share lattice corners in the rotate-back gathers
  // (the nearest-cell fallback above broke its ties in ascending order)
  std::stable_sort(p.grain_cells.begin(), p.grain_cells.end(), [nx](int32_t a, int32_t b) {
    const int ia = a % nx, ja = a / nx, ib = b % nx, jb = b / nx;
    if ((ja >> 4) != (jb >> 4)) return (ja >> 4) < (jb >> 4);
    if ((ia >> 4) != (ib >> 4)) return (ia >> 4) < (ib >> 4);
    return a < b;
  });

  // ---- rotate-back stencils of the grain cells
  const int64_t nc = static_cast<int64_t>(p.grain_cells.size());
  p.rb_idx.assign(static_cast<size_t>(p.n_theta) * 4 * nc, 0);
  p.rb_w.assign(static_cast<size_t>(p.n_theta) * 4 * nc, 0.0);
  p.rb4.assign(static_cast<size_t>(p.n_theta) * 4 * nc, -1);
  std::vector<int32_t> node(static_cast<size_t>(M) * M);
  for (int k = 0; k < p.n_theta; ++k) {
    std::fill(node.begin(), node.end(), -1);
    for (int64_t g = p.angle_seg0[k]; g < p.angle_seg0[k + 1]; ++g)
      for (int t = 0; t < p.seg_n[g]; ++t)
        node[static_cast<size_t>(p.seg_line[g]) * M + p.seg_jfirst[g] + t] =
            static_cast<int32_t>(p.seg_slot0[g] + t);
    const double epx = p.cosk[k], epy = p.sink[k];
    const double eqx = p.sink[k], eqy = -p.cosk[k];
    for (int64_t a = 0; a < nc; ++a) {
      const int32_t c = p.grain_cells[a];
      const double x = p.x0 + (c % nx + 0.5) * h, y = p.y0 + (c / nx + 0.5) * h;
      const double dx = x - p.cx, dy = y - p.cy;
      const double u = (dx * eqx + dy * eqy) / h + half;
      const double v = (dx * epx + dy * epy) / h + half;
      const int i0 = static_cast<int>(std::floor(u)), j0 = static_cast<int>(std::floor(v));
      const double wu = u - i0, wv = v - j0;
      const int li[4] = {i0, i0 + 1, i0, i0 + 1};
      const int lj[4] = {j0, j0, j0 + 1, j0 + 1};
      double w[4] = {(1 - wu) * (1 - wv), wu * (1 - wv), (1 - wu) * wv, wu * wv};
      int32_t idx[4];
      int32_t* c4 = &p.rb4[(static_cast<size_t>(k) * nc + a) * 4];
      double tot = 0.0;
      for (int q = 0; q < 4; ++q) {
        int32_t s = -1;
        if (li[q] >= 0 && li[q] < M && lj[q] >= 0 && lj[q] < M) s = node[static_cast<size_t>(li[q]) * M + lj[q]];
        c4[q] = s;
        idx[q] = s >= 0 ? s : 0;
        if (s < 0) w[q] = 0.0;
        tot += w[q];
      }
      if (tot > 0.0) {
        for (int q = 0; q < 4; ++q) w[q] /= tot;
      } else {
        // nearest interior node (ties -> smallest (line, node)): grow a box
        // around (u, v) until the best distance is inside the searched box
        int32_t best = -1;
        double bd = std::numeric_limits<double>::infinity();
        for (int R = 1; R <= M; ++R) {
          best = -1;
          bd = std::numeric_limits<double>::infinity();
          for (int i = std::max(0, i0 - R); i <= std::min(M - 1, i0 + 1 + R); ++i)
            for (int j = std::max(0, j0 - R); j <= std::min(M - 1, j0 + 1 + R); ++j) {
              const int32_t s = node[static_cast<size_t>(i) * M + j];
              if (s < 0) continue;
              const double d2 = (i - u) * (i - u) + (j - v) * (j - v);
              if (d2 < bd) {
                bd = d2;
                best = s;
              }
            }
          if (best >= 0 && bd <= static_cast<double>(R) * R) break;
        }
        if (best < 0) throw std::runtime_error("rotate-back: angle without interior node");
        c4[0] = best;
        c4[1] = c4[2] = c4[3] = -2;
        idx[0] = best;
        idx[1] = idx[2] = idx[3] = 0;
        w[0] = 1.0;
        w[1] = w[2] = w[3] = 0.0;
      }
      for (int q = 0; q < 4; ++q) {
        p.rb_idx[(static_cast<size_t>(k) * 4 + q) * nc + a] = idx[q];
        p.rb_w[(static_cast<size_t>(k) * 4 + q) * nc + a] = w[q];
      }
    }
  }

  // ---- specular boundary taps
  p.tap_start_seg.assign(static_cast<size_t>(p.nseg) * 4, 0);
  p.tap_end_seg.assign(static_cast<size_t>(p.nseg) * 4, 0);
  p.tap_start_w.assign(static_cast<size_t>(p.nseg) * 4, 0.0);
  p.tap_end_w.assign(static_cast<size_t>(p.nseg) * 4, 0.0);
  const double dphi = 2.0 * kPi / p.n_theta;
  for (int64_t g = 0; g < p.nseg; ++g) {
    for (int at_start = 1; at_start >= 0; --at_start) {
      const int k = p.seg_angle[g];
      const double u = (p.seg_line[g] - half) * h;
      const double s = at_start ? p.seg_smin[g] : p.seg_smax[g];
      const double px = p.cx + u * p.sink[k] + s * p.cosk[k];
      const double py = p.cy + u * (-p.cosk[k]) + s * p.sink[k];
      const double th = at_start ? p.seg_tmin[g] : p.seg_tmax[g];
      // reflected direction: mirror of phi_k about the wall tangent
      double phr = std::fmod(2.0 * th - p.phi[k], 2.0 * kPi);
      if (phr < 0.0) phr += 2.0 * kPi;
      const double x = phr / dphi;
      const int k0 = static_cast<int>(std::floor(x));
      const double wphi = x - k0;
      int32_t tseg[4];
      double tw[4];
      int nt = 0;
      const int kks[2] = {((k0 % p.n_theta) + p.n_theta) % p.n_theta, (((k0 + 1) % p.n_theta) + p.n_theta) % p.n_theta};
      const double wks[2] = {1.0 - wphi, wphi};
      for (int a = 0; a < 2; ++a) {
        const int kk = kks[a];
        const double eqx = p.sink[kk], eqy = -p.cosk[kk];
        const double uu = ((px - p.cx) * eqx + (py - p.cy) * eqy) / h + half;
        const int i0 = static_cast<int>(std::floor(uu));
        const double wu = uu - i0;
        const double sn = std::fabs(std::sin(p.phi[kk] - th));
        const double dacc = 2.0 * h / std::max(sn, 0.125);
        const int iis[2] = {i0, i0 + 1};
        const double wis[2] = {1.0 - wu, wu};
        for (int b = 0; b < 2; ++b) {
          const int ii = iis[b];
          if (ii < 0 || ii >= M) continue;
          const int64_t g0 = p.line_seg0[static_cast<size_t>(kk) * (M + 1) + ii];
          const int64_t g1 = p.line_seg0[static_cast<size_t>(kk) * (M + 1) + ii + 1];
          if (g1 == g0) continue;
          int64_t bestg = -1;
          double bd = std::numeric_limits<double>::infinity();
          const double uk = (ii - half) * h;
          for (int64_t gg = g0; gg < g1; ++gg) {
            const double se = at_start ? p.seg_smax[gg] : p.seg_smin[gg];
            const double ex = p.cx + uk * p.sink[kk] + se * p.cosk[kk];
            const double ey = p.cy + uk * (-p.cosk[kk]) + se * p.sink[kk];
            const double d = std::hypot(ex - px, ey - py);
            if (d < bd) {
              bd = d;
              bestg = gg;
            }
          }
          if (bd <= dacc) {
            tseg[nt] = static_cast<int32_t>(bestg);
            tw[nt] = wks[a] * wis[b];
            ++nt;
          }
        }
      }
      double tot = 0.0;
      for (int a = 0; a < nt; ++a) tot += tw[a];
      int32_t* os = at_start ? &p.tap_start_seg[g * 4] : &p.tap_end_seg[g * 4];
      double* ow = at_start ? &p.tap_start_w[g * 4] : &p.tap_end_w[g * 4];
      for (int a = 0; a < 4; ++a) {
        os[a] = static_cast<int32_t>(g);
        ow[a] = 0.0;
      }
      if (tot > 0.0)
        for (int a = 0; a < nt; ++a) {
          os[a] = tseg[a];
          ow[a] = tw[a] / tot;
        }
    }
  }

  build_pairs(p);
}

}  // namespace qc
