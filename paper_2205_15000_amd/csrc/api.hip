// C-ABI of the Riccati-sweep library; see include/qcsweep.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <exception>
#include <mutex>
#include <new>
#include <stdexcept>
#include <string>
#include <vector>

#include "plan.hpp"
#include "qcsweep.h"
#include "sweep.hpp"

namespace {

thread_local std::string g_err;

qc_status fail(qc_status s, const std::string& msg) {
  g_err = msg;
  return s;
}

struct HipError : std::runtime_error {
  using std::runtime_error::runtime_error;
};
struct OomError : std::runtime_error {
  using std::runtime_error::runtime_error;
};

void hcheck(hipError_t e, const char* what) {
  if (e == hipErrorOutOfMemory) throw OomError(std::string(what) + ": out of device memory");
  if (e != hipSuccess) throw HipError(std::string(what) + ": " + hipGetErrorString(e));
}

template <typename F>
qc_status guarded(F&& f) {
  try {
    return f();
  } catch (const OomError& e) {
    return fail(QC_ERR_OOM, e.what());
  } catch (const HipError& e) {
    return fail(QC_ERR_HIP, e.what());
  } catch (const std::bad_alloc&) {
    return fail(QC_ERR_OOM, "host allocation failed");
  } catch (const std::invalid_argument& e) {
    return fail(QC_ERR_INVALID, e.what());
  } catch (const std::range_error& e) {
    return fail(QC_ERR_NAN, e.what());
  } catch (const std::exception& e) {
    return fail(QC_ERR_INVALID, e.what());
  }
}

constexpr double kPi = 3.14159265358979323846;

template <typename V>
void* upload(const std::vector<V>& v) {
  void* p = nullptr;
  if (v.empty()) return nullptr;
  hcheck(hipMalloc(&p, v.size() * sizeof(V)), "hipMalloc");
  hcheck(hipMemcpy(p, v.data(), v.size() * sizeof(V), hipMemcpyHostToDevice), "hipMemcpy");
  return p;
}

void* dalloc(size_t bytes) {
  void* p = nullptr;
  if (bytes == 0) return nullptr;
  hcheck(hipMalloc(&p, bytes), "hipMalloc");
  return p;
}

int ilog2(int v) {
  int l = 0;
  while ((1 << l) < v) ++l;
  return l;
}

// Lanes per segment G (a power of two <= 64) for epl energies per lane
int lanes_for(int n_e, int epl) {
  const int need = (n_e + epl - 1) / epl;
  int G = 1;
  while (G < need) G <<= 1;
  return G;
}

// Energies per lane: a forced value (1, 2, 3, 4, 8) if it fits 64 lanes and
// does not exceed the energies, else the shape with the least cost G * epl * f(epl), i.e. energy slots
// (padding included) weighted by the measured relative cost per slot of
// each variant on gfx950 (64- and 48-pole grains).  Two per lane for 64
// poles, three for 48, four for 256-energy blocks (both precisions).
void lane_shape(int n_e, int force, bool fp32, int& G, int& epl) {
  static const int kEpl[5] = {1, 2, 3, 4, 8};
  static const double kCost32[5] = {1.13, 1.0, 1.28, 1.15, 1.55};
  static const double kCost64[5] = {1.07, 1.0, 1.20, 1.12, 1.24};
  const double* kCost = fp32 ? kCost32 : kCost64;
  if ((force == 1 || force == 2 || force == 3 || force == 4 || force == 8) && force <= n_e &&
      lanes_for(n_e, force) <= 64) {
    epl = force;
  } else {
    double best = INFINITY;
    epl = 1;
    for (int i = 0; i < 5; ++i) {
      const int Gi = lanes_for(n_e, kEpl[i]);
      if (Gi > 64 || kEpl[i] > std::max(n_e, 1)) continue;
      const double c = kCost[i] * Gi * kEpl[i];
      if (c < best) {
        best = c;
        epl = kEpl[i];
      }
    }
  }
  G = std::min(lanes_for(n_e, epl), 64);
}

void check_desc(const qc_grain_desc* d) {
  if (!d) throw std::invalid_argument("desc is NULL");
  if (d->nx < 2 || d->ny < 2) throw std::invalid_argument("nx and ny must be >= 2");
  if (static_cast<int64_t>(d->nx) * d->ny > (int64_t(1) << 28)) throw std::invalid_argument("grid too large");
  if (!(d->h > 0.0) || !std::isfinite(d->h)) throw std::invalid_argument("h must be finite and > 0");
  if (!std::isfinite(d->x0) || !std::isfinite(d->y0)) throw std::invalid_argument("x0/y0 must be finite");
  if (!d->shapes || d->n_shapes < 1) throw std::invalid_argument("at least one shape is required");
  if (d->n_theta < 1 || d->n_theta > 4096) throw std::invalid_argument("n_theta must be in [1, 4096]");
  if (d->n_poles < 1 || d->n_poles > 512) throw std::invalid_argument("n_poles must be in [1, 512]");
  if (!(d->t > 0.0) || !std::isfinite(d->t)) throw std::invalid_argument("t must be finite and > 0");
  if (d->ncomp < 1 || d->ncomp > 4) throw std::invalid_argument("ncomp must be in [1, 4]");
  if (!d->tc_rel) throw std::invalid_argument("tc_rel is required");
  if (!d->eta && !d->basis) throw std::invalid_argument("either eta or basis is required");
  if (!d->eta) {
    if (!std::isfinite(d->crystal_rotation)) throw std::invalid_argument("crystal_rotation must be finite");
    for (int c = 0; c < d->ncomp; ++c)
      if (d->basis[c] < QC_BASIS_S || d->basis[c] > QC_BASIS_G) throw std::invalid_argument("unknown basis function");
  }
  for (int g = 0; g < d->ncomp; ++g)
    if (!(d->tc_rel[g] > 0.0) || !std::isfinite(d->tc_rel[g])) throw std::invalid_argument("tc_rel must be > 0");
  if (d->eta)
    for (int64_t i = 0; i < 2LL * d->ncomp * d->n_theta; ++i)
      if (!std::isfinite(d->eta[i])) throw std::invalid_argument("eta must be finite");
  if (!std::isfinite(d->kappa) || !std::isfinite(d->flux_quanta)) throw std::invalid_argument("kappa/flux must be finite");
  if (d->gauge < 0 || d->gauge > 2) throw std::invalid_argument("gauge must be 0, 1 or 2");
  if (d->charge_sign != 1 && d->charge_sign != -1) throw std::invalid_argument("charge_sign must be +1 or -1");
  if (d->precision != QC_FP64 && d->precision != QC_MIXED) throw std::invalid_argument("precision must be 0 or 1");
  for (int s = 0; s < d->n_shapes; ++s) {
    const qc_shape& sh = d->shapes[s];
    if (sh.kind == QC_SHAPE_DISC) {
      if (!(sh.radius > 0.0) || !std::isfinite(sh.radius)) throw std::invalid_argument("disc radius must be > 0");
    } else if (sh.kind == QC_SHAPE_REGULAR_POLYGON) {
      if (sh.n_edges < 3 || !(sh.side > 0.0)) throw std::invalid_argument("regular polygon needs >= 3 edges, side > 0");
    } else if (sh.kind == QC_SHAPE_POLYGON) {
      if (sh.nv < 3 || !sh.vx || !sh.vy) throw std::invalid_argument("polygon needs >= 3 vertices");
    } else if (sh.kind == QC_SHAPE_MASK) {
      if (!sh.mask) throw std::invalid_argument("mask shape needs a mask");
    } else {
      throw std::invalid_argument("unknown shape kind");
    }
  }
}

void fill_plan_inputs(const qc_grain_desc* d, qc::Plan& p) {
  p.nx = d->nx;
  p.ny = d->ny;
  p.h = d->h;
  p.x0 = d->x0;
  p.y0 = d->y0;
  p.n_theta = d->n_theta;
  p.n_poles = d->n_poles;
  p.t = d->t;
  p.ncomp = d->ncomp;
  p.tc_rel.assign(d->tc_rel, d->tc_rel + d->ncomp);
  p.eta.resize(static_cast<size_t>(d->ncomp) * d->n_theta);
  if (d->eta) {
    for (size_t i = 0; i < p.eta.size(); ++i) p.eta[i] = {d->eta[2 * i], d->eta[2 * i + 1]};
  } else {
    for (int c = 0; c < d->ncomp; ++c)
      for (int k = 0; k < d->n_theta; ++k)
        p.eta[static_cast<size_t>(c) * d->n_theta + k] =
            qc::basis_eta(d->basis[c], 2.0 * kPi * k / d->n_theta - 2.0 * kPi * d->crystal_rotation);
  }
  p.kappa = d->kappa;
  p.flux = d->flux_quanta;
  p.gauge = d->gauge;
  p.q = d->charge_sign;
  p.precision = d->precision;
  p.shapes.clear();
  for (int s = 0; s < d->n_shapes; ++s) {
    const qc_shape& in = d->shapes[s];
    qc::Shape sh;
    sh.add = in.add != 0;
    if (in.kind == QC_SHAPE_DISC) {
      sh.kind = 0;
      sh.cx = in.cx;
      sh.cy = in.cy;
      sh.r = in.radius;
    } else if (in.kind == QC_SHAPE_REGULAR_POLYGON) {
      // first edge horizontal at the bottom for rotation 0
      sh.kind = 1;
      const int n = in.n_edges;
      const double rc = in.side / (2.0 * std::sin(kPi / n));
      for (int m = 0; m < n; ++m) {
        const double a = -0.5 * kPi - kPi / n + 2.0 * kPi * m / n + 2.0 * kPi * in.rotation;
        sh.vx.push_back(in.cx + rc * std::cos(a));
        sh.vy.push_back(in.cy + rc * std::sin(a));
      }
    } else if (in.kind == QC_SHAPE_MASK) {
      sh = qc::mask_shape(in.mask, d->nx, d->ny, d->x0, d->y0, d->h, in.add != 0);
    } else {
      sh.kind = 1;
      sh.vx.assign(in.vx, in.vx + in.nv);
      sh.vy.assign(in.vy, in.vy + in.nv);
    }
    p.shapes.push_back(sh);
  }
}

void info_of(const qc::Plan& p, qc_plan_info* o) {
  o->n_segments = p.nseg;
  o->n_slots = p.nslot;
  o->n_nodes = p.nnode;
  o->n_grain_cells = static_cast<int64_t>(p.grain_cells.size());
  o->steps_per_sweep = p.steps_per_sweep();
  o->lattice_m = p.M;
  o->area = p.area;
}

// Cell-averaged Green's function of the 2D Laplacian (App. D closed form).
double green_mn(double m, double n, double h) {
  auto alpha = [](double a, double b) {
    return (1 + 2 * a) * (1 + 2 * b) * std::log(0.5 * (1 + 2 * a) * (1 + 2 * a) + 0.5 * (1 + 2 * b) * (1 + 2 * b));
  };
  auto beta = [](double a, double b) { return (-2 * a * a + 2 * b * b + 4 * b + 1) * std::atan((1 + 2 * a) / (1 + 2 * b)); };
  double tot = 0.0;
  for (int sa = 0; sa < 2; ++sa)
    for (int sb = 0; sb < 2; ++sb) {
      const double a = sa ? -m : m, b = sb ? -n : n;
      tot += alpha(a, b) + beta(a, b) + beta(b, a);
    }
  return h * h / (4.0 * kPi) * (2.0 * std::log(h) - std::log(2.0) - 3.0 + 0.25 * tot);
}

}  // namespace

struct qc_plan {
  qc::Plan p;
};

struct qc_grain {
  int device = 0;
  qc_plan_info info{};
  int nx = 0, ny = 0, ncomp = 0, n_theta = 0, n_poles = 0, precision = 0;
  double h = 0, t = 0, kappa = 0, q = -1, twopi_rz = 0;
  int64_t ncell = 0, ncg = 0, nseg = 0, nslot = 0;
  int maxn = 1;  // most nodes of any segment
  std::vector<double> zp, rp;
  // static tables
  int32_t* slot_angle = nullptr;
  double* slot_px = nullptr;
  double* slot_py = nullptr;
  int32_t* slot_fb = nullptr;
  qc::SegGeo* seg_geo = nullptr;
  double cx = 0, cy = 0, half = 0, flux = 0, bfield = 0;
  int gauge = 0;
  double x0 = 0, y0 = 0;
  double* aext = nullptr;
  double* eta = nullptr;
  double* cosk = nullptr;
  double* sink = nullptr;
  double* wk = nullptr;
  int64_t* seg_slot0 = nullptr;
  int32_t* seg_n = nullptr;
  double* seg_hfirst = nullptr;
  double* seg_hlast = nullptr;
  int32_t* tap_s_seg = nullptr;
  double* tap_s_w = nullptr;
  int32_t* tap_e_seg = nullptr;
  double* tap_e_w = nullptr;
  int32_t* grain_cells = nullptr;
  int32_t* rb_idx = nullptr;
  double* rb_w = nullptr;
  int4* rb4 = nullptr;
  uint8_t* mask = nullptr;
  double* eps = nullptr;
  double* rpd = nullptr;
  double* den = nullptr;
  double* logt = nullptr;
  // work buffers
  void* nodes = nullptr;
  void* cells = nullptr;   // packed Delta / A_ind per cell (single component)
  int32_t* order = nullptr;
  int epl_override = 0;
  // segment node counts in launch order (every segment; lower angles of the
  // pairs), the split fraction of the Matsubara sweep's launch shape and the
  // device's wave slots per (precision, energies per lane), found on first use
  std::vector<int32_t> len_order, len_order_pair;
  double split_frac = 0.8;
  int64_t wave_slots[9] = {-1, -1, -1, -1, -1, -1, -1, -1, -1};
  void* gbuf = nullptr;
  double* node_out = nullptr;
  void* bc[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  int bc_cur = 0;
  int bc_valid = 0;
  int last_bc_valid = -1;  // store validity seen by the latest sweep (-1: no sweep yet)
  // reverse-mode buffers (allocated on first use)
  void* gtbuf = nullptr;
  void* lgt = nullptr;
  double* gS = nullptr;
  double* gV = nullptr;
  // checkpointed reverse mode (adj_ck > 0): offsets and buffers for that ck
  int adj_ck = 32;
  int ck_built = 0;
  int64_t* ckbase = nullptr;
  void* ckg = nullptr;
  void* ckgt = nullptr;
  void* ckscr = nullptr;
  size_t ckscr_bytes = 0;
  // transposed gather tables of the adjoint (built on first use)
  int64_t* bt_ptr = nullptr;
  int32_t* bt_c = nullptr;
  double* bt_w = nullptr;
  int64_t* it_dptr = nullptr;
  int32_t* it_ds = nullptr;
  double* it_dw = nullptr;
  int64_t* it_aptr = nullptr;
  int32_t* it_as = nullptr;
  double* it_aw = nullptr;
  double* omega_cell = nullptr;
  double* dmean = nullptr;
  double* part = nullptr;
  double* part_host = nullptr;
  double* bbuf = nullptr;
  // A-solve
  int px = 0, py = 0, lpx = 0, lpy = 0;
  double2* fw = nullptr;
  double2* fw2 = nullptr;
  double2* ghat = nullptr;
  double2* twx = nullptr;
  double2* twy = nullptr;
  // SCF scratch
  double* dnew = nullptr;
  double* jcur = nullptr;
  double* jold = nullptr;
  double* anew = nullptr;
  // SCF accelerator (App. E): 0 Picard, 1 Polyak with drag beta, 2
  // Barzilai-Borwein; the Polyak velocities (BB: previous differences) of
  // Delta and A
  int accel = 0;
  double beta = 0.5;
  double* vel_d = nullptr;
  double* vel_a = nullptr;
  // CongAcc: per-component dot-product partials [component][kParts][3]
  double* cpart = nullptr;
  double* cpart_host = nullptr;
  // CongAcc weights set by bisection and by the anti-parallel rule
  int64_t cong_bisect = 0, cong_anti = 0;
  // angle pairs (k, k + n_theta/2): the sweep of the Matsubara iteration
  // runs the lower angles only (see build_pairs); pair_ok when the tables
  // allow it, pairing when it is in use
  bool pair_ok = false, pairing = false, rb_fold = false;
  int64_t nseg_pair = 0, nslot_pair = 0, npairs = 0;
  int32_t* order_pair = nullptr;
  int4* rb4_pair = nullptr;
  int2* mirror_pairs = nullptr;
  // transposed rotate-back of the paired reverse mode: the entries of the
  // upper angles moved onto their mirror slots
  int64_t* btp_ptr = nullptr;
  int32_t* btp_c = nullptr;
  double* btp_w = nullptr;
  // eigen-truncated A-solve (App. D): tolerance, kept modes, eigenvalues and
  // eigenvectors [a_nmodes][nx], masked current and per-mode products
  double a_eps = 0.0;
  int a_nmodes = 0;
  double* a_lam = nullptr;
  double* a_vk = nullptr;
  double* a_jp = nullptr;
  double* a_y = nullptr;
  // Luttinger-Ward free energy: per-cell lambda integral, lambda Delta, and
  // the boundary store kept aside while the lambda sweeps run
  double* lw_acc = nullptr;
  double* lw_dl = nullptr;
  void* lw_save = nullptr;
  // profiling
  bool prof = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> ev;
  double prof_ms = 0.0;
  int64_t prof_n = 0;

  size_t real_bytes() const { return precision == QC_MIXED ? sizeof(float) : sizeof(double); }
};

static constexpr int kParts = 256;
// bounds of the Barzilai-Borwein step (App. E's defaults)
static constexpr double kBBStepMin = 1e-3, kBBStepMax = 1e2;
// CongAcc (App. E's defaults): step factor, minimum similarity, step bounds
static constexpr double kCongK = 1.234, kCongSmin = 0.7, kCongStepMin = 1e-3, kCongStepMax = 1e2;
// a similarity at or below -1 + kCongAnti reads as anti-parallel m and d:
// the blend w m + (1 - w) d is then a multiple of d whose similarity with d
// jumps from 1 to -1 where it vanishes, so no weight reaches smin; the
// average restarts from d (w = 0)
static constexpr double kCongAnti = 1e-9;

// The weight w* in [0, 1] at which w m + (1 - w) d has cosine similarity
// smin with d, by bisection from m.m, m.d and d.d (similarity 1 at w = 0).
static double congacc_weight(double mm, double md, double dd, double smin) {
  auto sim = [&](double w) {
    const double uu = w * w * mm + 2.0 * w * (1.0 - w) * md + (1.0 - w) * (1.0 - w) * dd;
    return uu > 0.0 ? (w * md + (1.0 - w) * dd) / std::sqrt(uu * dd) : 1.0;
  };
  double lo = 0.0, hi = 1.0;
  for (int it = 0; it < 60; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (sim(mid) >= smin)
      lo = mid;
    else
      hi = mid;
  }
  return 0.5 * (lo + hi);
}
// regions of the block-partial buffer (kParts doubles each, diffs 2 kParts)
// (BB dot products 3 kParts each)
enum {
  kROmega = 0, kRB2 = 1, kRJx = 2, kRJy = 3, kRDiffD = 4, kRDiffJ = 6, kRDiffA = 8, kRBBD = 10, kRBBA = 13,
  kRegions = 16
};

namespace {

void free_grain(qc_grain* g) {
  void* ptrs[] = {g->slot_angle, g->slot_px, g->slot_py, g->slot_fb, g->seg_geo, g->aext, g->eta, g->cosk,
                  g->sink, g->wk, g->seg_slot0, g->seg_n, g->seg_hfirst, g->seg_hlast, g->tap_s_seg,
                  g->tap_s_w, g->tap_e_seg, g->tap_e_w, g->grain_cells, g->rb_idx, g->rb_w, g->rb4, g->mask,
                  g->eps, g->rpd, g->den, g->logt, g->nodes, g->cells, g->order, g->gbuf, g->node_out, g->bc[0][0],
                  g->bc[0][1], g->bc[1][0], g->bc[1][1], g->omega_cell, g->dmean, g->part, g->bbuf, g->fw, g->fw2,
                  g->ghat, g->twx, g->twy, g->dnew, g->jcur, g->jold, g->anew, g->vel_d, g->vel_a, g->gtbuf, g->lgt, g->gS, g->gV,
                  g->bt_ptr, g->bt_c, g->bt_w, g->it_dptr, g->it_ds, g->it_dw, g->it_aptr, g->it_as, g->it_aw,
                  g->ckbase, g->ckg, g->ckgt, g->ckscr, g->lw_acc, g->lw_dl, g->lw_save, g->order_pair, g->rb4_pair,
                  g->mirror_pairs, g->a_lam, g->a_vk, g->a_jp, g->a_y, g->btp_ptr, g->btp_c, g->btp_w};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  if (g->part_host) (void)hipHostFree(g->part_host);
  if (g->cpart) (void)hipFree(g->cpart);
  if (g->cpart_host) (void)hipHostFree(g->cpart_host);
  for (auto& e : g->ev) {
    (void)hipEventDestroy(e.first);
    (void)hipEventDestroy(e.second);
  }
  delete g;
}

hipStream_t S(void* s) { return static_cast<hipStream_t>(s); }

double* region(qc_grain* g, int r) { return g->part + static_cast<int64_t>(r) * kParts; }

// one copy of every block partial to the host, then wait for the stream
void fetch_parts(qc_grain* g, hipStream_t st) {
  hcheck(hipMemcpyAsync(g->part_host, g->part, sizeof(double) * kRegions * kParts, hipMemcpyDeviceToHost, st),
         "D2H");
  hcheck(hipStreamSynchronize(st), "sync");
}

// host sum of one region (fixed order: deterministic)
double region_sum(const qc_grain* g, int r) {
  double s = 0.0;
  for (int i = 0; i < kParts; ++i) s += g->part_host[static_cast<int64_t>(r) * kParts + i];
  return s;
}

// rows along x, transpose, rows along y (result in fw2, [px][py] layout);
// rows y >= nz_rows of fw are zero and keep a zero transform
void fft_forward_2d(qc_grain* g, hipStream_t st, int sign, int nz_rows) {
  qc::launch_fft_rows(g->fw, nz_rows, g->lpx, g->twx, sign, nullptr, st);
  qc::launch_transpose(g->fw, g->fw2, g->py, g->px, st);
  qc::launch_fft_rows(g->fw2, g->px, g->lpy, g->twy, sign, nullptr, st);
}

// inverse of fw2 times pre (elementwise, [px][py]) into fw; only rows
// y < out_rows of fw are transformed along x
void fft_inverse_2d(qc_grain* g, hipStream_t st, const double2* pre, int out_rows) {
  qc::launch_fft_rows(g->fw2, g->px, g->lpy, g->twy, +1, pre, st);
  qc::launch_transpose(g->fw2, g->fw, g->px, g->py, st);
  qc::launch_fft_rows(g->fw, out_rows, g->lpx, g->twx, +1, nullptr, st);
}

std::vector<double2> twiddles(int n) {
  std::vector<double2> tw(std::max(1, n / 2));
  for (int k = 0; k < n / 2; ++k) tw[k] = make_double2(std::cos(2.0 * kPi * k / n), -std::sin(2.0 * kPi * k / n));
  return tw;
}

qc::GridGeom geom_of(const qc_grain* g) {
  qc::GridGeom gg;
  gg.nx = g->nx;
  gg.ny = g->ny;
  gg.x0 = g->x0;
  gg.y0 = g->y0;
  gg.h = g->h;
  gg.mask = g->mask;
  return gg;
}

// rotate-back of the node sums into Delta_new, j and the free energy
qc::BackArgs back_args(qc_grain* g, const double* delta, double* dnew, double* j, double* omega) {
  qc::BackArgs r;
  r.ncg = g->ncg;
  r.ncell = g->ncell;
  r.ncomp = g->ncomp;
  r.n_theta = g->n_theta;
  r.grain_cells = g->grain_cells;
  r.rb4 = g->pairing ? g->rb4_pair : g->rb4;
  r.pair_k0 = g->pairing ? g->n_theta / 2 : g->n_theta;
  r.pair_fold = g->pairing && g->rb_fold ? 1 : 0;
  r.nx = g->nx;
  r.x0 = g->x0;
  r.y0 = g->y0;
  r.h = g->h;
  r.cx = g->cx;
  r.cy = g->cy;
  r.half = g->half;
  r.node_out = g->node_out;
  r.wk = g->wk;
  r.cosk = g->cosk;
  r.sink = g->sink;
  r.eta = g->eta;
  r.den = g->den;
  r.logt = g->logt;
  r.four_q = 4.0 * g->q;
  r.twopi_rz = g->twopi_rz;
  r.delta = delta;
  r.delta_new = dnew;
  r.j = j;
  r.omega = omega;
  r.omega_cell = g->omega_cell;
  return r;
}

// node values of every slot, or (pair) of the slots of the lower angles of
// the angle pairs only
void do_interp(qc_grain* g, const double* delta, const double* A, hipStream_t st, bool pair = false) {
  qc::InterpArgs a;
  pair = pair && g->pairing;
  a.nslot = pair ? g->nslot_pair : g->nslot;
  a.nseg = pair ? g->nseg_pair : g->nseg;
  a.ncell = g->ncell;
  a.ncomp = g->ncomp;
  a.n_theta = g->n_theta;
  a.slot_angle = g->slot_angle;
  a.geom = geom_of(g);
  a.px = g->slot_px;
  a.py = g->slot_py;
  a.fb = g->slot_fb;
  a.aext = g->aext;
  a.eta = g->eta;
  a.cosk = g->cosk;
  a.sink = g->sink;
  a.delta = delta;
  a.A = A;
  a.seg_geo = g->seg_geo;
  a.cx = g->cx;
  a.cy = g->cy;
  a.half = g->half;
  a.gauge = g->gauge;
  a.flux = g->flux;
  a.bfield = g->bfield;
  if (g->ncomp == 1 && !g->cells) g->cells = dalloc(4 * g->real_bytes() * g->ncell);
  void* cells = g->ncomp == 1 ? g->cells : nullptr;
  if (g->precision == QC_MIXED)
    qc::launch_interp<float>(a, cells, g->nodes, st);
  else
    qc::launch_interp<double>(a, cells, g->nodes, st);
}

// arguments of a sweep over every segment, or (pair) over the segments of
// the lower angles of the angle pairs
qc::SweepArgs sweep_args(qc_grain* g, int n_e, int n_e_tot, int e_off, const double* eps, const double* rp,
                         bool pair = false) {
  qc::SweepArgs a;
  pair = pair && g->pairing;
  a.nseg = pair ? g->nseg_pair : g->nseg;
  a.order = pair ? g->order_pair : g->order;
  int epl;
  lane_shape(n_e, g->epl_override, g->precision == QC_MIXED, a.G, epl);
  a.log2g = ilog2(a.G);
  a.n_e = n_e;
  a.n_e_tot = n_e_tot;
  a.e_off = e_off;
  a.bc_valid = 0;
  a.h = g->h;
  a.q = g->q;
  a.twopi_tt = g->t;
  a.seg_slot0 = g->seg_slot0;
  a.seg_n = g->seg_n;
  a.seg_hfirst = g->seg_hfirst;
  a.seg_hlast = g->seg_hlast;
  a.tap_start_seg = g->tap_s_seg;
  a.tap_start_w = g->tap_s_w;
  a.tap_end_seg = g->tap_e_seg;
  a.tap_end_w = g->tap_e_w;
  a.eps = eps;
  a.rp = rp;
  a.node_out = g->node_out;
  a.maxn = g->maxn;
  a.nlong = 0;
  return a;
}

// Segments of a Matsubara sweep that take the wide lane shape (2G lanes,
// EPL/2 energies per lane; see SweepArgs::nlong): only when the launch
// fills the device's wave slots less than twice, so that its longest
// segments set its length, and then those longer than split_frac x the
// longest, rounded up to whole waves
int64_t split_count(qc_grain* g, const qc::SweepArgs& a, int epl) {
  if (!(g->split_frac > 0.0) || epl % 2 != 0 || 2 * a.G > 64 || a.nseg == 0) return 0;
  const std::vector<int32_t>& len = a.order == g->order_pair && g->order_pair ? g->len_order_pair : g->len_order;
  if (static_cast<int64_t>(len.size()) != a.nseg) return 0;
  int64_t& slots = g->wave_slots[epl];
  if (slots < 0)
    slots = g->precision == QC_MIXED ? qc::sweep_wave_slots<float>(epl) : qc::sweep_wave_slots<double>(epl);
  const int64_t waves = (a.nseg * a.G + 63) / 64;
  if (slots <= 0 || waves >= 2 * slots) return 0;
  const double cut = g->split_frac * len[0];
  int64_t k = 0;
  while (k < a.nseg && len[k] > cut) ++k;
  const int64_t per = 64 / (2 * a.G);
  k = (k + per - 1) / per * per;
  return std::min(k, a.nseg);
}

void launch_sweep_timed(qc_grain* g, int mode, const qc::SweepArgs& a, const qc::SweepBufs& b, hipStream_t st) {
  int G, epl;
  lane_shape(a.n_e, g->epl_override, g->precision == QC_MIXED, G, epl);
  // every lane marches epl existing energies (the kernel's lane layout)
  if (epl > a.n_e || G * epl < a.n_e) throw std::logic_error("sweep lane shape does not fit the energies");
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (g->prof) {
    hcheck(hipEventCreate(&e0), "event");
    hcheck(hipEventCreate(&e1), "event");
    hcheck(hipEventRecord(e0, st), "event");
  }
  if (g->precision == QC_MIXED)
    qc::launch_sweep<float>(mode, epl, a, b, st);
  else
    qc::launch_sweep<double>(mode, epl, a, b, st);
  hcheck(hipGetLastError(), "sweep launch");
  if (g->prof) {
    hcheck(hipEventRecord(e1, st), "event");
    g->ev.push_back({e0, e1});
  }
}

// the end values of the upper angles of the pairs, from their mirrors, so
// that the boundary store is complete for every reader
void mirror_fill(qc_grain* g, void* bc_g, void* bc_gt, hipStream_t st) {
  if (!g->pairing) return;
  if (g->precision == QC_MIXED)
    qc::launch_mirror_fill<float>(g->mirror_pairs, g->npairs, g->n_poles, nullptr, bc_g, bc_gt, st);
  else
    qc::launch_mirror_fill<double>(g->mirror_pairs, g->npairs, g->n_poles, nullptr, bc_g, bc_gt, st);
}

double omega_from_parts(const qc_grain* g) {
  double tot = g->h * g->h * region_sum(g, kROmega);
  if (g->kappa > 0.0) tot += g->h * g->h * 0.5 * g->kappa * g->kappa * region_sum(g, kRB2);
  return tot;
}

// buffers of the iteration map (gamma at nodes, per-node sums, boundary
// store), allocated on first use so that LDOS-only grains do not hold them
// spill: also the gamma spill of single-grain sweeps (batched sweeps keep it
// in per-wave scratch instead)
void ensure_sweep_buffers(qc_grain* g, bool spill = true) {
  // the packed interpolation cells are needed before any graph capture
  if (g->ncomp == 1 && !g->cells) g->cells = dalloc(4 * g->real_bytes() * g->ncell);
  const size_t rb = g->real_bytes();
  if (spill && !g->gbuf) g->gbuf = dalloc(2 * rb * g->nslot * g->n_poles);
  if (g->node_out) return;
  g->node_out = static_cast<double*>(dalloc(4 * sizeof(double) * g->nslot));
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) g->bc[a][b] = dalloc(2 * rb * g->nseg * g->n_poles);
}

// steps 3-8 of one iteration; omega_total (host) optional (synchronises)
// zero_out: clear delta_new, j (and omega) first; the rotate-back writes
// grain cells only, so a caller that keeps the off-grain cells at zero itself
// may skip it
void do_sweep(qc_grain* g, const double* delta, const double* A, double* delta_new, double* j, double* omega,
              double* omega_total, hipStream_t st, bool zero_out = true) {
  ensure_sweep_buffers(g);
  do_interp(g, delta, A, st, true);
  qc::SweepArgs a = sweep_args(g, g->n_poles, g->n_poles, 0, g->eps, g->rpd, true);
  a.bc_valid = g->bc_valid;
  {
    int G, epl;
    lane_shape(a.n_e, g->epl_override, g->precision == QC_MIXED, G, epl);
    a.nlong = split_count(g, a, epl);
  }
  qc::SweepBufs b;
  b.nodes = g->nodes;
  b.bc_g_prev = g->bc[g->bc_cur][0];
  b.bc_gt_prev = g->bc[g->bc_cur][1];
  b.bc_g_next = g->bc[1 - g->bc_cur][0];
  b.bc_gt_next = g->bc[1 - g->bc_cur][1];
  b.gbuf = g->gbuf;
  b.ebuf = nullptr;
  launch_sweep_timed(g, 0, a, b, st);
  mirror_fill(g, b.bc_g_next, b.bc_gt_next, st);
  g->last_bc_valid = g->bc_valid;
  g->bc_cur = 1 - g->bc_cur;
  g->bc_valid = 1;

  if (zero_out) {
    qc::launch_fill(delta_new, 2 * g->ncomp * g->ncell, 0.0, st);
    qc::launch_fill(j, 2 * g->ncell, 0.0, st);
    if (omega) qc::launch_fill(omega, g->ncell, 0.0, st);
  }
  qc::launch_rotate_back(back_args(g, delta, delta_new, j, omega), st);
  hcheck(hipGetLastError(), "rotate-back launch");
  // block partials of the free energy (condensation and magnetic parts)
  if (g->kappa > 0.0) {
    qc::launch_curl(A, g->bbuf, g->nx, g->ny, g->h, st);
    qc::launch_block_sum2({g->omega_cell, nullptr, g->ncg, 0, region(g, kROmega)},
                          {g->bbuf, nullptr, g->ncell, 1, region(g, kRB2)}, kParts, st);
  } else {
    qc::launch_block_sum(g->omega_cell, nullptr, g->ncg, 0, region(g, kROmega), kParts, st);
  }
  if (omega_total) {
    fetch_parts(g, st);
    *omega_total = omega_from_parts(g);
  }
}

void do_solve_A(qc_grain* g, const double* j, double* A_out, double* B_out, hipStream_t st);

}  // namespace

// ------------------------------------------------------------------------
extern "C" {

const char* qc_last_error(void) { return g_err.c_str(); }

int qc_version(void) { return 1; }

qc_status qc_valu_rate(int device, int op, double* lane_ops_per_s) {
  if (!lane_ops_per_s) return fail(QC_ERR_INVALID, "lane_ops_per_s is NULL");
  if (op < 0 || op > 3) return fail(QC_ERR_INVALID, "op must be 0 (fma), 1 (rsq), 2 (sqrt) or 3 (rcp)");
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev)
    return fail(QC_ERR_NO_DEVICE, "no such HIP device");
  float* out = nullptr;
  hipStream_t st = nullptr;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const qc_status rs = guarded([&]() -> qc_status {
    hcheck(hipSetDevice(device), "hipSetDevice");
    hipDeviceProp_t prop;
    hcheck(hipGetDeviceProperties(&prop, device), "properties");
    const int nblocks = prop.multiProcessorCount * 8, iters = 4096;
    out = static_cast<float*>(dalloc(sizeof(float) * 256 * static_cast<size_t>(nblocks)));
    hcheck(hipStreamCreate(&st), "stream");
    hcheck(hipEventCreate(&e0), "event");
    hcheck(hipEventCreate(&e1), "event");
    qc::launch_valu_rate(op, out, nblocks, iters, st);  // warm-up
    hcheck(hipEventRecord(e0, st), "event");
    qc::launch_valu_rate(op, out, nblocks, iters, st);
    hcheck(hipEventRecord(e1, st), "event");
    hcheck(hipEventSynchronize(e1), "event");
    float ms = 0.f;
    hcheck(hipEventElapsedTime(&ms, e0, e1), "event");
    *lane_ops_per_s = 256.0 * nblocks * iters * 8.0 / (1e-3 * ms);
    return QC_OK;
  });
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (st) (void)hipStreamDestroy(st);
  if (out) (void)hipFree(out);
  return rs;
}

qc_status qc_device_count(int* n_out) {
  if (!n_out) return fail(QC_ERR_INVALID, "n_out is NULL");
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess) n = 0;
  *n_out = n;
  return QC_OK;
}

qc_status qc_plan_create(const qc_grain_desc* desc, qc_plan** out) {
  return guarded([&]() -> qc_status {
    if (!out) throw std::invalid_argument("out is NULL");
    *out = nullptr;
    check_desc(desc);
    auto* pl = new qc_plan();
    try {
      fill_plan_inputs(desc, pl->p);
      qc::build_plan(pl->p);
    } catch (...) {
      delete pl;
      throw;
    }
    *out = pl;
    return QC_OK;
  });
}

void qc_plan_destroy(qc_plan* plan) { delete plan; }

qc_status qc_plan_get_info(const qc_plan* plan, qc_plan_info* out) {
  if (!plan || !out) return fail(QC_ERR_INVALID, "NULL argument");
  info_of(plan->p, out);
  return QC_OK;
}

qc_status qc_plan_get_mask(const qc_plan* plan, uint8_t* mask_out) {
  if (!plan || !mask_out) return fail(QC_ERR_INVALID, "NULL argument");
  std::memcpy(mask_out, plan->p.mask.data(), plan->p.mask.size());
  return QC_OK;
}

qc_status qc_plan_get_segments(const qc_plan* plan, double* out) {
  if (!plan || !out) return fail(QC_ERR_INVALID, "NULL argument");
  const qc::Plan& p = plan->p;
  for (int64_t g = 0; g < p.nseg; ++g) {
    double* o = out + g * 8;
    o[0] = p.seg_angle[g];
    o[1] = p.seg_line[g];
    o[2] = p.seg_smin[g];
    o[3] = p.seg_smax[g];
    o[4] = p.seg_jfirst[g];
    o[5] = p.seg_n[g];
    o[6] = p.seg_tmin[g];
    o[7] = p.seg_tmax[g];
  }
  return QC_OK;
}

qc_status qc_plan_get_taps(const qc_plan* plan, int at_start, int32_t* seg_out, double* w_out) {
  if (!plan || !seg_out || !w_out) return fail(QC_ERR_INVALID, "NULL argument");
  const qc::Plan& p = plan->p;
  const auto& s = at_start ? p.tap_start_seg : p.tap_end_seg;
  const auto& w = at_start ? p.tap_start_w : p.tap_end_w;
  std::memcpy(seg_out, s.data(), s.size() * sizeof(int32_t));
  std::memcpy(w_out, w.data(), w.size() * sizeof(double));
  return QC_OK;
}

qc_status qc_plan_get_poles(const qc_plan* plan, double* z_out, double* r_out) {
  if (!plan || !z_out || !r_out) return fail(QC_ERR_INVALID, "NULL argument");
  std::memcpy(z_out, plan->p.zp.data(), plan->p.zp.size() * sizeof(double));
  std::memcpy(r_out, plan->p.rp.data(), plan->p.rp.size() * sizeof(double));
  return QC_OK;
}

qc_status qc_plan_get_eta(const qc_plan* plan, double* eta_out) {
  if (!plan || !eta_out) return fail(QC_ERR_INVALID, "NULL argument");
  const qc::Plan& p = plan->p;
  for (size_t i = 0; i < p.eta.size(); ++i) {
    eta_out[2 * i] = p.eta[i].real();
    eta_out[2 * i + 1] = p.eta[i].imag();
  }
  return QC_OK;
}

qc_status qc_plan_get_pairing(const qc_plan* plan, int* available, int64_t* swept_steps_per_sweep,
                              int32_t* seg_mirror_out) {
  if (!plan) return fail(QC_ERR_INVALID, "plan is NULL");
  const qc::Plan& p = plan->p;
  if (available) *available = p.pair_ok ? (p.rb_fold ? 3 : 1) : 0;
  if (swept_steps_per_sweep) {
    int64_t s = 0;
    const int64_t nsw = p.pair_ok ? p.nseg_pair : p.nseg;
    for (int64_t k = 0; k < nsw; ++k) s += p.seg_n[k] + 1;
    *swept_steps_per_sweep = 2 * static_cast<int64_t>(p.n_poles) * s;
  }
  if (seg_mirror_out)
    for (int64_t k = 0; k < p.nseg; ++k) seg_mirror_out[k] = p.pair_ok ? p.seg_mirror[k] : -1;
  return QC_OK;
}

qc_status qc_grain_create(int device, const qc_grain_desc* desc, qc_grain** out) {
  if (!out) return fail(QC_ERR_INVALID, "out is NULL");
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || ndev == 0) return fail(QC_ERR_NO_DEVICE, "no HIP device");
  if (device < 0 || device >= ndev) return fail(QC_ERR_INVALID, "device index out of range");
  qc_grain* g = new (std::nothrow) qc_grain();
  if (!g) return fail(QC_ERR_OOM, "host allocation failed");
  qc_status st = guarded([&]() -> qc_status {
    check_desc(desc);
    hipDeviceProp_t prop;
    hcheck(hipGetDeviceProperties(&prop, device), "hipGetDeviceProperties");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
      throw HipError(std::string("device is ") + prop.gcnArchName + ", this library is built for gfx950");
    hcheck(hipSetDevice(device), "hipSetDevice");
    g->device = device;
    qc::Plan p;
    fill_plan_inputs(desc, p);
    qc::build_plan(p);
    info_of(p, &g->info);
    g->nx = p.nx;
    g->ny = p.ny;
    g->ncomp = p.ncomp;
    g->n_theta = p.n_theta;
    g->n_poles = p.n_poles;
    g->precision = p.precision;
    g->h = p.h;
    g->t = p.t;
    g->kappa = p.kappa;
    g->q = p.q;
    g->ncell = static_cast<int64_t>(p.nx) * p.ny;
    g->ncg = static_cast<int64_t>(p.grain_cells.size());
    g->nseg = p.nseg;
    g->nslot = p.nslot;
    for (int32_t n : p.seg_n) g->maxn = std::max(g->maxn, static_cast<int>(n));
    g->zp = p.zp;
    g->rp = p.rp;
    double rz = 0.0;
    for (int k = 0; k < p.n_poles; ++k) rz += p.rp[k] / p.zp[k];
    g->twopi_rz = 2.0 * kPi * rz;
    std::vector<double> den(p.ncomp), logt(p.ncomp);
    for (int c = 0; c < p.ncomp; ++c) {
      logt[c] = std::log(p.t / p.tc_rel[c]);
      den[c] = logt[c] + g->twopi_rz;
    }
    std::vector<double> eps(2 * p.n_poles);
    const double tt = p.t / (2.0 * kPi);
    for (int k = 0; k < p.n_poles; ++k) {
      eps[2 * k] = 0.0;
      eps[2 * k + 1] = p.zp[k] * tt;
    }
    std::vector<double> eta(2 * p.eta.size());
    for (size_t i = 0; i < p.eta.size(); ++i) {
      eta[2 * i] = p.eta[i].real();
      eta[2 * i + 1] = p.eta[i].imag();
    }
    g->slot_angle = static_cast<int32_t*>(upload(p.slot_angle));
    g->slot_px = static_cast<double*>(upload(p.slot_px));
    g->slot_py = static_cast<double*>(upload(p.slot_py));
    g->slot_fb = static_cast<int32_t*>(upload(p.slot_fb));
    {
      std::vector<qc::SegGeo> sg(static_cast<size_t>(p.nseg));
      for (int64_t i = 0; i < p.nseg; ++i) {
        sg[i].slot0 = p.seg_slot0[i];
        sg[i].u = (p.seg_line[i] - p.half) * p.h;  // the plan's expression
        sg[i].smid = 0.5 * (p.seg_smin[i] + p.seg_smax[i]);
        sg[i].jf = p.seg_jfirst[i];
        sg[i].n = p.seg_n[i];
        sg[i].k = p.seg_angle[i];
        sg[i].pad = 0;
      }
      g->seg_geo = static_cast<qc::SegGeo*>(upload(sg));
      g->cx = p.cx;
      g->cy = p.cy;
      g->half = p.half;
      g->gauge = p.gauge;
      g->flux = p.flux;
      g->bfield = p.area > 0.0 ? kPi * p.flux / p.area : 0.0;
    }
    g->x0 = p.x0;
    g->y0 = p.y0;
    g->aext = static_cast<double*>(upload(p.slot_aext));
    g->eta = static_cast<double*>(upload(eta));
    g->cosk = static_cast<double*>(upload(p.cosk));
    g->sink = static_cast<double*>(upload(p.sink));
    g->wk = static_cast<double*>(upload(p.wk));
    g->seg_slot0 = static_cast<int64_t*>(upload(p.seg_slot0));
    g->seg_n = static_cast<int32_t*>(upload(p.seg_n));
    g->seg_hfirst = static_cast<double*>(upload(p.seg_hfirst));
    g->seg_hlast = static_cast<double*>(upload(p.seg_hlast));
    g->tap_s_seg = static_cast<int32_t*>(upload(p.tap_start_seg));
    g->tap_s_w = static_cast<double*>(upload(p.tap_start_w));
    g->tap_e_seg = static_cast<int32_t*>(upload(p.tap_end_seg));
    g->tap_e_w = static_cast<double*>(upload(p.tap_end_w));
    g->grain_cells = static_cast<int32_t*>(upload(p.grain_cells));
    g->rb_idx = static_cast<int32_t*>(upload(p.rb_idx));
    g->rb_w = static_cast<double*>(upload(p.rb_w));
    g->rb4 = static_cast<int4*>(upload(p.rb4));
    g->mask = static_cast<uint8_t*>(upload(p.mask));
    g->eps = static_cast<double*>(upload(eps));
    g->rpd = static_cast<double*>(upload(p.rp));
    g->den = static_cast<double*>(upload(den));
    g->logt = static_cast<double*>(upload(logt));
    const size_t rb = g->real_bytes();
    g->nodes = dalloc(4 * rb * g->nslot);
    {
      // launch order: longest segments first (least tail, no lane waste)
      std::vector<int32_t> ord(g->nseg);
      for (int64_t k = 0; k < g->nseg; ++k) ord[k] = static_cast<int32_t>(k);
      std::stable_sort(ord.begin(), ord.end(), [&](int32_t x, int32_t y) { return p.seg_n[x] > p.seg_n[y]; });
      g->order = static_cast<int32_t*>(upload(ord));
      g->len_order.resize(ord.size());
      for (size_t k = 0; k < ord.size(); ++k) g->len_order[k] = p.seg_n[ord[k]];
    }
    if (p.pair_ok) {
      std::vector<int32_t> ord(static_cast<size_t>(p.nseg_pair));
      for (int64_t k = 0; k < p.nseg_pair; ++k) ord[k] = static_cast<int32_t>(k);
      std::stable_sort(ord.begin(), ord.end(), [&](int32_t x, int32_t y) { return p.seg_n[x] > p.seg_n[y]; });
      g->order_pair = static_cast<int32_t*>(upload(ord));
      g->len_order_pair.resize(ord.size());
      for (size_t k = 0; k < ord.size(); ++k) g->len_order_pair[k] = p.seg_n[ord[k]];
      g->rb4_pair = static_cast<int4*>(upload(p.rb4_pair));
      std::vector<int2> mp;
      for (int64_t sg = p.nseg_pair; sg < p.nseg; ++sg) mp.push_back(make_int2(static_cast<int>(sg), p.seg_mirror[sg]));
      g->mirror_pairs = static_cast<int2*>(upload(mp));
      g->npairs = static_cast<int64_t>(mp.size());
      g->nseg_pair = p.nseg_pair;
      g->nslot_pair = p.nslot_pair;
      g->pair_ok = true;
      g->pairing = true;
      g->rb_fold = p.rb_fold;
    }
    // gbuf, node_out and the boundary store are allocated by the first sweep
    g->omega_cell = static_cast<double*>(dalloc(sizeof(double) * g->ncg));
    g->part = static_cast<double*>(dalloc(sizeof(double) * kRegions * kParts));
    g->dmean = static_cast<double*>(dalloc(sizeof(double) * 2));
    hcheck(hipHostMalloc(reinterpret_cast<void**>(&g->part_host), sizeof(double) * kRegions * kParts),
           "hipHostMalloc");
    g->bbuf = static_cast<double*>(dalloc(sizeof(double) * g->ncell));
    g->dnew = static_cast<double*>(dalloc(sizeof(double) * 2 * g->ncomp * g->ncell));
    g->jcur = static_cast<double*>(dalloc(sizeof(double) * 2 * g->ncell));
    g->jold = static_cast<double*>(dalloc(sizeof(double) * 2 * g->ncell));
    g->anew = static_cast<double*>(dalloc(sizeof(double) * 2 * g->ncell));
    if (g->kappa > 0.0) {
      g->px = 1 << ilog2(2 * p.nx);
      g->py = 1 << ilog2(2 * p.ny);
      g->lpx = ilog2(g->px);
      g->lpy = ilog2(g->py);
      if (g->lpx > 12 || g->lpy > 12) throw std::invalid_argument("grid too large for the A-solve (max 2048)");
      const int64_t np = static_cast<int64_t>(g->px) * g->py;
      std::vector<double2> gp(np);
      for (int y = 0; y < g->py; ++y)
        for (int x = 0; x < g->px; ++x) {
          const int m = std::min(x, g->px - x), n = std::min(y, g->py - y);
          const double v = (m <= p.nx - 1 && n <= p.ny - 1) ? green_mn(m, n, p.h) : 0.0;
          gp[static_cast<int64_t>(y) * g->px + x] = make_double2(v, 0.0);
        }
      g->twx = static_cast<double2*>(upload(twiddles(g->px)));
      g->twy = static_cast<double2*>(upload(twiddles(g->py)));
      g->fw = static_cast<double2*>(upload(gp));
      g->fw2 = static_cast<double2*>(dalloc(sizeof(double2) * np));
      g->ghat = static_cast<double2*>(dalloc(sizeof(double2) * np));
      fft_forward_2d(g, nullptr, -1, g->py);
      hcheck(hipMemcpy(g->ghat, g->fw2, sizeof(double2) * np, hipMemcpyDeviceToDevice), "copy");
    }
    hcheck(hipDeviceSynchronize(), "grain setup");
    return QC_OK;
  });
  if (st != QC_OK) {
    free_grain(g);
    return st;
  }
  *out = g;
  return QC_OK;
}

void qc_grain_destroy(qc_grain* grain) {
  if (!grain) return;
  (void)hipSetDevice(grain->device);
  (void)hipDeviceSynchronize();
  free_grain(grain);
}

qc_status qc_grain_get_mask(const qc_grain* grain, uint8_t* mask_out) {
  if (!grain || !mask_out) return fail(QC_ERR_INVALID, "NULL argument");
  return guarded([&]() -> qc_status {
    hcheck(hipSetDevice(grain->device), "hipSetDevice");
    hcheck(hipMemcpy(mask_out, grain->mask, static_cast<size_t>(grain->ncell), hipMemcpyDeviceToHost), "copy");
    return QC_OK;
  });
}

qc_status qc_grain_get_info(const qc_grain* grain, qc_plan_info* out) {
  if (!grain || !out) return fail(QC_ERR_INVALID, "NULL argument");
  *out = grain->info;
  return QC_OK;
}

qc_status qc_grain_reset_bc(qc_grain* grain) {
  if (!grain) return fail(QC_ERR_INVALID, "grain is NULL");
  grain->bc_valid = 0;
  return QC_OK;
}

qc_status qc_sweep(qc_grain* g, const double* delta, const double* A_ind, double* delta_new, double* j,
                   double* omega_density, double* omega_total, void* stream) {
  if (!g) return fail(QC_ERR_INVALID, "grain is NULL");
  if (!delta || !A_ind || !delta_new || !j) return fail(QC_ERR_INVALID, "delta, A_ind, delta_new and j are required");
  return guarded([&]() -> qc_status {
    hcheck(hipSetDevice(g->device), "hipSetDevice");
    do_sweep(g, delta, A_ind, delta_new, j, omega_density, omega_total, S(stream));
    return QC_OK;
  });
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Allocation-free sweep: the per-call work arrays of qc_sweep (slot values,
// the gamma spill, per-node sums, packed interpolation cells) live in one
// file-scope device array instead of grain-owned allocations.  Each device
// holds its own copy of the array until the process ends; its address on a
// device comes from hipGetSymbolAddress with that device current.
namespace {

constexpr size_t kScratchBytes = size_t(64) << 20;  // 64 MiB per device
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// device address of this device's scratch array (device current)
void* scratch_ptr(int device) {
  if (device < 0 || device >= kMaxDevices) throw std::invalid_argument("device index beyond the scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[device]) {
    void* ptr = nullptr;
    hcheck(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)), "hipGetSymbolAddress(scratch)");
    if (!ptr) throw HipError("hipGetSymbolAddress(scratch) returned NULL");
    g_scratch_ptr[device] = ptr;
  }
  return g_scratch_ptr[device];
}

size_t align256(size_t b) { return (b + 255) & ~size_t(255); }

// bytes of scratch one sweep of this grain needs: slot values, gamma spill,
// per-node sums, packed cells (one component)
size_t static_sweep_bytes(const qc_grain* g) {
  const size_t rb = g->real_bytes();
  size_t b = align256(4 * rb * g->nslot) + align256(2 * rb * g->nslot * g->n_poles) +
             align256(4 * sizeof(double) * g->nslot);
  if (g->ncomp == 1) b += align256(4 * rb * g->ncell);
  return b;
}

}  // namespace

extern "C" {

qc_status qc_sweep_static(qc_grain* g, const double* delta, const double* A_ind, double* delta_new, double* j,
                          double* omega_density, double* omega_total, void* stream) {
  if (!g) return fail(QC_ERR_INVALID, "grain is NULL");
  if (!delta || !A_ind || !delta_new || !j) return fail(QC_ERR_INVALID, "delta, A_ind, delta_new and j are required");
  const size_t need = static_sweep_bytes(g);
  if (need > kScratchBytes)
    return fail(QC_ERR_INVALID, "qc_sweep_static: this grain needs " + std::to_string(need) +
                                    " bytes of scratch, more than the " + std::to_string(kScratchBytes) +
                                    " the library holds per device (use qc_sweep)");
  if (!g->bc[0][0] || !g->bc[1][0])
    return fail(QC_ERR_INVALID, "qc_sweep_static: the grain has no boundary store yet (run qc_sweep or "
                                "qc_set_state once first)");
  return guarded([&]() -> qc_status {
    hcheck(hipSetDevice(g->device), "hipSetDevice");
    unsigned char* base = static_cast<unsigned char*>(scratch_ptr(g->device));
    const size_t rb = g->real_bytes();
    // the grain's own work arrays are set aside for the call
    void* own_nodes = g->nodes;
    void* own_gbuf = g->gbuf;
    double* own_out = g->node_out;
    void* own_cells = g->cells;
    size_t off = 0;
    g->nodes = base + off;
    off += align256(4 * rb * g->nslot);
    g->gbuf = base + off;
    off += align256(2 * rb * g->nslot * g->n_poles);
    g->node_out = reinterpret_cast<double*>(base + off);
    off += align256(4 * sizeof(double) * g->nslot);
    if (g->ncomp == 1) g->cells = base + off;
    qc_status st = QC_OK;
    try {
      do_sweep(g, delta, A_ind, delta_new, j, omega_density, omega_total, S(stream));
    } catch (...) {
      g->nodes = own_nodes;
      g->gbuf = own_gbuf;
      g->node_out = own_out;
      g->cells = own_cells;
      throw;
    }
    g->nodes = own_nodes;
    g->gbuf = own_gbuf;
    g->node_out = own_out;
    g->cells = own_cells;
    return st;
  });
}

qc_status qc_sweep_static_bytes(const qc_grain* g, size_t* needed, size_t* available) {
  if (!g) return fail(QC_ERR_INVALID, "grain is NULL");
  if (needed) *needed = static_sweep_bytes(g);
  if (available) *available = kScratchBytes;
  return QC_OK;
}

}  // extern "C"


namespace {

void do_solve_A(qc_grain* g, const double* j, double* A_out, double* B_out, hipStream_t st) {
  if (g->kappa <= 0.0) {
    qc::launch_fill(A_out, 2 * g->ncell, 0.0, st);
    if (B_out) qc::launch_fill(B_out, g->ncell, 0.0, st);
    return;
  }
  // mean current over the grain cells, subtracted before the solve (App. D)
  qc::launch_block_sum2({j, g->grain_cells, g->ncg, 0, region(g, kRJx)},
                        {j + g->ncell, g->grain_cells, g->ncg, 0, region(g, kRJy)}, kParts, st);
  qc::launch_means(region(g, kRJx), kParts, 1.0 / static_cast<double>(g->ncg), g->dmean, st);
  if (g->a_nmodes > 0) {
    // the separable kernel kept to its largest modes: two MFMA contractions
    qc::launch_masked_current(j, g->mask, g->ncell, g->dmean, g->a_jp, st);
    qc::launch_eig_vecpot(g->nx, g->a_nmodes, g->a_jp, g->a_vk, g->a_lam, g->a_y, A_out,
                          -1.0 / (g->kappa * g->kappa), st);
    if (B_out) qc::launch_curl(A_out, B_out, g->nx, g->ny, g->h, st);
    hcheck(hipGetLastError(), "A-solve launch");
    return;
  }
  qc::launch_pad_current(j, g->mask, g->nx, g->ny, g->px, g->py, g->dmean, g->fw, st);
  // the padded current is zero beyond row ny, and only rows < ny of the
  // correlation are kept; the product with the kernel's transform is taken
  // as the inverse pass loads its rows
  fft_forward_2d(g, st, -1, g->ny);
  fft_inverse_2d(g, st, g->ghat, g->ny);
  const double scale = -1.0 / (g->kappa * g->kappa * static_cast<double>(g->px) * g->py);
  qc::launch_unpad_A(g->fw, g->nx, g->ny, g->px, scale, A_out, st);
  if (B_out) qc::launch_curl(A_out, B_out, g->nx, g->ny, g->h, st);
  hcheck(hipGetLastError(), "A-solve launch");
}

// Arguments of the pass that forms the block partials of ||xnew - xold||_p
// and ||xold||_p over n elements of `stride` doubles (gathered through idx
// when given) for nrep fields into region reg; with update, the pass also
// takes the Picard step xold += alpha (xnew - xold)
qc::DiffNormArgs diff_args(qc_grain* g, const double* xnew, double* xold, const int32_t* idx, int64_t n, int nrep,
                           int64_t field_stride, int stride, int p, int reg, bool update = false, double alpha = 1.0,
                           double* vel = nullptr) {
  qc::DiffNormArgs a;
  a.xnew = xnew;
  a.xold = xold;
  a.idx = idx;
  a.n = n;
  a.nrep = nrep;
  a.field_stride = field_stride;
  a.stride = stride;
  a.p = p;
  a.part = region(g, reg);
  a.update = update ? xold : nullptr;
  a.alpha = alpha;
  a.vel = vel;
  a.beta = g->beta;
  return a;
}

// ||new - old||_p / ||old||_p from fetched partials (0/0 = 0, x/0 = inf)
double rel_from_parts(const qc_grain* g, int reg, int p) {
  const double* q = g->part_host + static_cast<int64_t>(reg) * kParts;
  double num = 0.0, den = 0.0;
  for (int i = 0; i < kParts; ++i) {
    if (p == 0) {
      num = std::max(num, q[2 * i]);
      den = std::max(den, q[2 * i + 1]);
    } else {
      num += q[2 * i];
      den += q[2 * i + 1];
    }
  }
  if (p == 2) {
    num = std::sqrt(num);
    den = std::sqrt(den);
  }
  if (den == 0.0) return num == 0.0 ? 0.0 : INFINITY;
  return num / den;
}

}  // namespace

extern "C" {

qc_status qc_solve_A(qc_grain* g, const double* j, double* A_out, double* B_out, void* stream) {
  if (!g) return fail(QC_ERR_INVALID, "grain is NULL");
  if (!j || !A_out) return fail(QC_ERR_INVALID, "j and A_out are required");
  return guarded([&]() -> qc_status {
    hcheck(hipSetDevice(g->device), "hipSetDevice");
    do_solve_A(g, j, A_out, B_out, S(stream));
    return QC_OK;
  });
}

// Nodes and weights of the n-point Gauss-Legendre rule on [0, 1]: the roots
// of P_n by Newton's method from Chebyshev-like starts, weights
// 2 / ((1 - x^2) P_n'(x)^2) on [-1, 1], halved for [0, 1].
static void gauss_legendre01(int n, std::vector<double>& x, std::vector<double>& w) {
  x.assign(n, 0.0);
  w.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    double r = std::cos(kPi * (i + 0.75) / (n + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = r;  // P_0, P_1
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * r * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      const double pn = n == 1 ? r : p1, pm = n == 1 ? 1.0 : p0;  // P_n, P_{n-1}
      dp = n * (r * pn - pm) / (r * r - 1.0);
      const double dr = pn / dp;
      r -= dr;
      if (std::fabs(dr) < 1e-16) break;
    }
    {
      double p0 = 1.0, p1 = r;
      for (int k = 2; k <= n; ++k) {
        const double p2 = ((2.0 * k - 1.0) * r * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      const double pn = n == 1 ? r : p1, pm = n == 1 ? 1.0 : p0;
      dp = n * (r * pn - pm) / (r * r - 1.0);
    }
    x[i] = 0.5 * (1.0 - r);
    w[i] = 1.0 / ((1.0 - r * r) * dp * dp);
  }
}

qc_status qc_free_energy_lw(qc_grain* g, const double* delta, const double* A_ind, int n_lambda, int bc_iters,
                            double* omega_density, double* omega_total, void* stream) {
  if (!g) return fail(QC_ERR_INVALID, "grain is NULL");
  if (!delta || !A_ind || !omega_total) return fail(QC_ERR_INVALID, "delta, A_ind and omega_total are required");
  if (n_lambda < 1 || n_lambda > 64 || bc_iters < 0) return fail(QC_ERR_INVALID, "need 1 <= n_lambda <= 64, bc_iters >= 0");
  return guarded([&]() -> qc_status {
    hipStream_t st = S(stream);
    hcheck(hipSetDevice(g->device), "hipSetDevice");
    ensure_sweep_buffers(g);
    const size_t half = 2 * g->real_bytes() * g->nseg * g->n_poles;
    if (!g->lw_acc) g->lw_acc = static_cast<double*>(dalloc(sizeof(double) * std::max<int64_t>(g->ncg, 1)));
    if (!g->lw_dl) g->lw_dl = static_cast<double*>(dalloc(sizeof(double) * 2 * g->ncomp * g->ncell));
    if (!g->lw_save) g->lw_save = dalloc(2 * half);
    // the grain's boundary store is kept aside and restored at the end
    const int saved_valid = g->bc_valid, saved_cur = g->bc_cur;
    if (saved_valid) {
      hcheck(hipMemcpyAsync(g->lw_save, g->bc[g->bc_cur][0], half, hipMemcpyDeviceToDevice, st), "copy");
      hcheck(hipMemcpyAsync(static_cast<char*>(g->lw_save) + half, g->bc[g->bc_cur][1], half, hipMemcpyDeviceToDevice,
                            st),
             "copy");
    }
    std::vector<double> lam, wl;
    gauss_legendre01(n_lambda, lam, wl);
    for (int l = 0; l < n_lambda; ++l) {
      qc::launch_scale(delta, lam[l], 2 * g->ncomp * g->ncell, g->lw_dl, st);
      g->bc_valid = 0;  // each coupling starts from bulk roots of lambda Delta
      for (int it = 0; it <= bc_iters; ++it)
        do_sweep(g, g->lw_dl, A_ind, g->dnew, g->jcur, nullptr, nullptr, st, false);
      qc::launch_lw_accumulate(delta, g->dnew, g->grain_cells, g->ncg, g->ncomp, g->ncell, g->den, wl[l], l == 0,
                               g->lw_acc, st);
    }
    if (omega_density) qc::launch_fill(omega_density, g->ncell, 0.0, st);
    qc::launch_lw_finish(delta, g->grain_cells, g->ncg, g->ncomp, g->ncell, g->n_theta, g->eta, g->wk, g->logt,
                         g->twopi_rz, g->lw_acc, g->omega_cell, omega_density, st);
    qc::launch_block_sum(g->omega_cell, nullptr, g->ncg, 0, region(g, kROmega), kParts, st);
    if (g->kappa > 0.0) {
      qc::launch_curl(A_ind, g->bbuf, g->nx, g->ny, g->h, st);
      qc::launch_block_sum(g->bbuf, nullptr, g->ncell, 1, region(g, kRB2), kParts, st);
    }
    fetch_parts(g, st);
    *omega_total = omega_from_parts(g);
    // restore the store the caller's next sweep expects
    g->bc_cur = saved_cur;
    g->bc_valid = saved_valid;
    if (saved_valid) {
      hcheck(hipMemcpyAsync(g->bc[g->bc_cur][0], g->lw_save, half, hipMemcpyDeviceToDevice, st), "copy");
      hcheck(hipMemcpyAsync(g->bc[g->bc_cur][1], static_cast<char*>(g->lw_save) + half, half, hipMemcpyDeviceToDevice,
                            st),
             "copy");
    }
    hcheck(hipStreamSynchronize(st), "sync");
    return QC_OK;
  });
}

// N* of App. D: the smallest count of the largest-|lambda| modes whose
// dropped remainder has sqrt(sum lambda^2 (dropped) / sum lambda^2 (all))
// below eps (summed over the dropped modes directly, not as 1 - kept/total)
static int kept_modes(const std::vector<double>& lam_sorted, double eps) {
  const int n = static_cast<int>(lam_sorted.size());
  std::vector<double> tail(n + 1, 0.0);
  for (int k = n - 1; k >= 0; --k) tail[k] = tail[k + 1] + lam_sorted[k] * lam_sorted[k];
  for (int k = 0; k <= n; ++k)
    if (std::sqrt(tail[k] / tail[0]) < eps) return k;
  return n;
}

qc_status qc_grain_set_A_solver(qc_grain* g, double eps) {
  if (!g) return fail(QC_ERR_INVALID, "grain is NULL");
  if (!(eps >= 0.0) || !std::isfinite(eps)) return fail(QC_ERR_INVALID, "eps must be finite and >= 0");
  if (eps > 0.0 && g->nx != g->ny) return fail(QC_ERR_INVALID, "the eigen-truncated A-solve needs a square grid");
  return guarded([&]() -> qc_status {
    hcheck(hipSetDevice(g->device), "hipSetDevice");
    hcheck(hipDeviceSynchronize(), "sync");
    for (double** p : {&g->a_lam, &g->a_vk, &g->a_jp, &g->a_y})
      if (*p) {
        (void)hipFree(*p);
        *p = nullptr;
      }
    g->a_nmodes = 0;
    g->a_eps = eps;
    if (eps == 0.0) return QC_OK;
    const int n = g->nx;
    std::vector<double> G(static_cast<size_t>(n) * n);
    for (int a = 0; a < n; ++a)
      for (int b = 0; b < n; ++b) G[static_cast<size_t>(a) * n + b] = green_mn(a, b, g->h);
    std::vector<double> lam, vec;
    qc::sym_eigen(n, G, lam, vec);
    std::vector<int> ord(n);
    for (int i = 0; i < n; ++i) ord[i] = i;
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return std::fabs(lam[x]) > std::fabs(lam[y]); });
    std::vector<double> ls(n);
    for (int i = 0; i < n; ++i) ls[i] = lam[ord[i]];
    const int nk = std::max(kept_modes(ls, eps), 1);
    std::vector<double> lk(nk), vk(static_cast<size_t>(nk) * n);
    for (int k = 0; k < nk; ++k) {
      lk[k] = ls[k];
      for (int a = 0; a < n; ++a) vk[static_cast<size_t>(k) * n + a] = vec[static_cast<size_t>(a) * n + ord[k]];
    }
    g->a_lam = static_cast<double*>(upload(lk));
    g->a_vk = static_cast<double*>(upload(vk));
    g->a_jp = static_cast<double*>(dalloc(sizeof(double) * 2 * g->ncell));
    g->a_y = static_cast<double*>(dalloc(sizeof(double) * 2 * static_cast<size_t>(nk) * g->ncell));
    g->a_nmodes = nk;
    return QC_OK;
  });
}

qc_status qc_grain_get_A_solver(const qc_grain* g, double* eps, int* n_modes) {
  if (!g) return fail(QC_ERR_INVALID, "grain is NULL");
  if (eps) *eps = g->a_eps;
  if (n_modes) *n_modes = g->a_nmodes;
  return QC_OK;
}

qc_status qc_magnetic_moment(qc_grain* g, const double* j, double* m_out, void* stream) {
  if (!g || !j || !m_out) return fail(QC_ERR_INVALID, "grain, j and m_out are required");
  return guarded([&]() -> qc_status {
    hipStream_t st = S(stream);
    hcheck(hipSetDevice(g->device), "hipSetDevice");
    qc::launch_torque(j, g->grain_cells, g->ncg, g->ncell, g->nx, g->x0, g->y0, g->h, g->cx, g->cy, g->bbuf, st);
    qc::launch_block_sum(g->bbuf, nullptr, g->ncg, 0, region(g, kRJx), kParts, st);
    fetch_parts(g, st);
    *m_out = region_sum(g, kRJx) / (2.0 * static_cast<double>(g->ncg));
    return QC_OK;
  });
}

qc_status qc_scf_run(qc_grain* g, double* delta_io, double* A_io, int max_iter, int min_iter, int burnin,
                     double tol, int norm_p, double alpha, int* iters_done, double* residuals_out, void* stream) {
  if (!g) return fail(QC_ERR_INVALID, "grain is NULL");
  if (!delta_io || !A_io) return fail(QC_ERR_INVALID, "delta_io and A_io are required");
  if (max_iter < 1 || min_iter < 0 || burnin < 0) return fail(QC_ERR_INVALID, "bad iteration counts");
  if (!(tol >= 0.0) || !(alpha > 0.0) || !std::isfinite(alpha)) return fail(QC_ERR_INVALID, "bad tol or alpha");
  if (norm_p != 0 && norm_p != 1 && norm_p != 2) return fail(QC_ERR_INVALID, "norm_p must be 0, 1 or 2");
  return guarded([&]() -> qc_status {
    hipStream_t st = S(stream);
    hcheck(hipSetDevice(g->device), "hipSetDevice");
    // Delta lives on grain cells only
    {
      // zero the off-grain cells of the input once (they stay zero)
      hcheck(hipMemcpyAsync(g->dnew, delta_io, sizeof(double) * 2 * g->ncomp * g->ncell, hipMemcpyDeviceToDevice,
                            st),
             "copy");
      qc::launch_fill(delta_io, 2 * g->ncomp * g->ncell, 0.0, st);
      qc::launch_picard(delta_io, g->dnew, g->grain_cells, g->ncg, g->ncomp, g->ncell, 2, 1.0, st);
    }
    // no screening (kappa <= 0): no induced vector potential, A stays zero
    if (g->kappa <= 0.0) qc::launch_fill(A_io, 2 * g->ncell, 0.0, st);
    // the sweeps write grain cells only: off-grain j stays zero in both
    // current buffers, and off-grain Delta_new is never read here
    ensure_sweep_buffers(g);
    qc::launch_fill(g->jcur, 2 * g->ncell, 0.0, st);
    qc::launch_fill(g->jold, 2 * g->ncell, 0.0, st);
    // Polyak: velocities start at zero in every run; BB keeps the previous
    // iteration's difference in the same arrays
    const bool polyak = g->accel == 1, bb = g->accel == 2, cong = g->accel == 3;
    if (cong && norm_p != 2) throw std::invalid_argument("CongAcc residuals are 2-norms: norm_p must be 2");
    if (polyak || bb || cong) {
      if (!g->vel_d) g->vel_d = static_cast<double*>(dalloc(sizeof(double) * 2 * g->ncomp * g->ncell));
      if (!g->vel_a) g->vel_a = static_cast<double*>(dalloc(sizeof(double) * 2 * g->ncell));
      qc::launch_fill(g->vel_d, 2 * g->ncomp * g->ncell, 0.0, st);
      qc::launch_fill(g->vel_a, 2 * g->ncell, 0.0, st);
    }
    // the global errors are of d = g(x) - x, taken before the accelerator
    // moves x (Alg. 1)
    double a_bb = alpha;  // BB step, alpha for the first iteration
    int i_bb = 0;
    // CongAcc: components 2 G + (0 re, 1 im) of Delta, then A_x, A_y
    const int ncx = 2 * g->ncomp + 2;
    std::vector<double> cg_a(ncx, alpha), cg_w(ncx, 0.0);
    bool cg_first = true;
    if (cong && !g->cpart) {
      g->cpart = static_cast<double*>(dalloc(sizeof(double) * 3 * kParts * ncx));
      hcheck(hipHostMalloc(reinterpret_cast<void**>(&g->cpart_host), sizeof(double) * 3 * kParts * ncx),
             "hipHostMalloc");
    }
    const double ksc = g->kappa > 0.0 ? g->kappa * g->kappa : 1.0;  // x holds kappa^2 A
    double om_old = 0.0;
    bool have_old = false;
    int it = 0;
    bool conv = false;
    for (; it < max_iter; ++it) {
      do_sweep(g, delta_io, A_io, g->dnew, g->jcur, nullptr, nullptr, st, false);
      if (it < burnin) {
        std::swap(g->jold, g->jcur);
        fetch_parts(g, st);
        const double om = omega_from_parts(g);
        const double res[5] = {0.0, 0.0, 0.0, 0.0, om};
        om_old = om;
        have_old = true;
        if (residuals_out) std::memcpy(residuals_out + 5 * it, res, sizeof(res));
        continue;
      }
      do_solve_A(g, g->jcur, g->anew, nullptr, st);
      // residuals of Delta and A with their Picard steps fused in
      // (BB: norms and dot products first; the step follows once its size is known)
      // (the three fields in one launch)
      {
        qc::DiffNormArgs da[3];
        int nd = 0;
        da[nd++] = diff_args(g, g->dnew, delta_io, g->grain_cells, g->ncg, g->ncomp, g->ncell, 2, norm_p, kRDiffD,
                             !bb && !cong, alpha, polyak ? g->vel_d : nullptr);
        if (have_old) da[nd++] = diff_args(g, g->jcur, g->jold, nullptr, 2 * g->ncell, 1, 0, 1, norm_p, kRDiffJ);
        da[nd++] = diff_args(g, g->anew, A_io, nullptr, 2 * g->ncell, 1, 0, 1, norm_p, kRDiffA, !bb && !cong, alpha,
                             polyak ? g->vel_a : nullptr);
        qc::launch_diff_norm_n(da, nd, kParts, st);
      }
      if (cong && !cg_first) {
        for (int c = 0; c < ncx; ++c) {
          double* pc = g->cpart + static_cast<int64_t>(c) * 3 * kParts;
          if (c < 2 * g->ncomp)
            qc::launch_congacc_dots(g->dnew, delta_io, g->grain_cells, g->ncg, static_cast<int64_t>(c / 2) * g->ncell,
                                    2, c % 2, g->vel_d, pc, kParts, st);
          else
            qc::launch_congacc_dots(g->anew, A_io, nullptr, g->ncell,
                                    static_cast<int64_t>(c - 2 * g->ncomp) * g->ncell, 1, 0, g->vel_a, pc, kParts, st);
        }
        hcheck(hipMemcpyAsync(g->cpart_host, g->cpart, sizeof(double) * 3 * kParts * ncx, hipMemcpyDeviceToHost, st),
               "D2H");
      }
      if (bb) {
        qc::launch_bb_dots(g->dnew, delta_io, g->grain_cells, g->ncg, g->ncomp, g->ncell, 2, 1.0, g->vel_d,
                           region(g, kRBBD), kParts, st);
        qc::launch_bb_dots(g->anew, A_io, nullptr, 2 * g->ncell, 1, 0, 1, ksc, g->vel_a, region(g, kRBBA), kParts,
                           st);
      }
      std::swap(g->jold, g->jcur);
      fetch_parts(g, st);
      if (bb) {
        if (i_bb > 0) {
          double pp = 0.0, pd = 0.0, dd = 0.0;
          for (int reg : {kRBBD, kRBBA}) {
            const double* q = g->part_host + static_cast<int64_t>(reg) * kParts;
            for (int b = 0; b < kParts; ++b) {
              pp += q[3 * b];
              pd += q[3 * b + 1];
              dd += q[3 * b + 2];
            }
          }
          pd = std::fabs(pd);
          const double num = (i_bb % 2 == 1) ? pp : pd, den = (i_bb % 2 == 1) ? pd : dd;
          if (den != 0.0) a_bb = std::min(std::max(a_bb * num / den, kBBStepMin), kBBStepMax);
        }
        ++i_bb;
        qc::launch_picard(delta_io, g->dnew, g->grain_cells, g->ncg, g->ncomp, g->ncell, 2, a_bb, st);
        qc::launch_picard(A_io, g->anew, nullptr, 2 * g->ncell, 1, 0, 1, a_bb, st);
      }
      // CongAcc: per-component step sizes and weights, then the step
      if (cong) {
        for (int c = 0; c < ncx; ++c) {
          if (cg_first) continue;
          double mm = 0.0, md = 0.0, dd = 0.0;
          const double* q = g->cpart_host + static_cast<int64_t>(c) * 3 * kParts;
          for (int b = 0; b < kParts; ++b) {
            mm += q[3 * b];
            md += q[3 * b + 1];
            dd += q[3 * b + 2];
          }
          const double sc = (mm > 0.0 && dd > 0.0) ? md / std::sqrt(mm * dd) : 0.0;
          cg_a[c] = std::min(std::max(cg_a[c] * std::pow(kCongK, sc), kCongStepMin), kCongStepMax);
          if (sc < kCongSmin && mm > 0.0 && dd > 0.0) {
            if (sc <= -1.0 + kCongAnti) {
              cg_w[c] = 0.0;
              ++g->cong_anti;
            } else {
              cg_w[c] = congacc_weight(mm, md, dd, kCongSmin);
              ++g->cong_bisect;
            }
          }
        }
        qc::CongCoef cd{}, ca{};
        for (int c = 0; c < 2 * g->ncomp; ++c) {
          cd.a[c] = cg_a[c];
          cd.w[c] = cg_first ? 0.0 : cg_w[c];
        }
        for (int c = 0; c < 2; ++c) {
          ca.a[c] = cg_a[2 * g->ncomp + c];
          ca.w[c] = cg_first ? 0.0 : cg_w[2 * g->ncomp + c];
        }
        qc::launch_congacc_update(delta_io, g->dnew, g->vel_d, g->grain_cells, g->ncg, g->ncomp, g->ncell, 2, cd, st);
        qc::launch_congacc_update(A_io, g->anew, g->vel_a, nullptr, g->ncell, 2, g->ncell, 1, ca, st);
      }
      const double om = omega_from_parts(g);
      double res[5];
      res[0] = rel_from_parts(g, kRDiffD, norm_p);
      res[1] = have_old ? rel_from_parts(g, kRDiffJ, norm_p) : INFINITY;
      res[2] = rel_from_parts(g, kRDiffA, norm_p);
      if (cong) cg_first = false;
      res[3] = (have_old && om_old != 0.0) ? std::fabs(om - om_old) / std::fabs(om_old) : INFINITY;
      res[4] = om;
      if (residuals_out) std::memcpy(residuals_out + 5 * it, res, sizeof(res));
      if (!std::isfinite(res[0]) || !std::isfinite(om) || std::isnan(res[2]))
        throw std::range_error("non-finite residual (Delta and A hold the failed update)");
      om_old = om;
      have_old = true;
      if (it + 1 >= min_iter && res[0] < tol && res[1] < tol && res[2] < tol && res[3] < tol) {
        conv = true;
        ++it;
        break;
      }
    }
    hcheck(hipStreamSynchronize(st), "sync");
    if (iters_done) *iters_done = it;
    return conv ? QC_OK : QC_NOT_CONVERGED;
  });
}

// Partner of each real energy under e -> -e (to 1e-12 of the largest |e|)
// when the set is symmetric about zero (as a multiset); false otherwise
bool energy_partners(const double* en, int n, std::vector<int32_t>& partner) {
  double emax = 0.0;
  for (int i = 0; i < n; ++i) emax = std::max(emax, std::fabs(en[i]));
  const double tol = 1e-12 * std::max(emax, 1e-300);
  std::vector<int32_t> idx(static_cast<size_t>(n));
  for (int i = 0; i < n; ++i) idx[i] = i;
  std::stable_sort(idx.begin(), idx.end(), [&](int32_t x, int32_t y) { return en[x] < en[y]; });
  partner.assign(static_cast<size_t>(n), -1);
  for (int k = 0; k < n; ++k) {
    const int32_t i = idx[k], j = idx[n - 1 - k];
    if (std::fabs(en[i] + en[j]) > tol) return false;
    partner[i] = j;
  }
  return true;
}

qc_status qc_ldos(qc_grain* g, const double* delta, const double* A_ind, const double* energies, int n_e,
                  double broadening, int bc_iters, double* ldos_out, void* stream) {
  if (!g) return fail(QC_ERR_INVALID, "grain is NULL");
  if (!delta || !A_ind || !energies || !ldos_out) return fail(QC_ERR_INVALID, "NULL argument");
  if (n_e < 1 || bc_iters < 0) return fail(QC_ERR_INVALID, "n_e must be >= 1 and bc_iters >= 0");
  if (!(broadening > 0.0) || !std::isfinite(broadening)) return fail(QC_ERR_INVALID, "broadening must be > 0");
  for (int i = 0; i < n_e; ++i)
    if (!std::isfinite(energies[i])) return fail(QC_ERR_INVALID, "energies must be finite");
  void* bcl[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  double* deps = nullptr;
  int32_t* dpart = nullptr;
  int32_t* dmap = nullptr;
  void* lg = nullptr;
  void* le = nullptr;
  qc_status rs = guarded([&]() -> qc_status {
    hipStream_t st = S(stream);
    hcheck(hipSetDevice(g->device), "hipSetDevice");
    const size_t rb = g->real_bytes();
    // Angle pairs: with an energy set symmetric about zero, the reversed
    // direction at e + i delta follows from its mirror at -e + i delta
    // (Sec. II.A symmetry with z -> -z*).  The boundary sweeps then march
    // the lower angle of each pair, and the store of the upper one is filled
    // from its mirror after every iteration.  The energies run in an order
    // of their own, each e beside its -e (self-partners last), so that every
    // even-sized block of the output pass holds whole pairs: the output
    // sweep marches the lower angles too, and the rotate-back reads each
    // lower angle's corners for both angles of the pair (where the planner
    // found them equal).
    std::vector<int32_t> partner;
    const bool pair = g->pairing && energy_partners(energies, n_e, partner);
    std::vector<int32_t> perm(static_cast<size_t>(n_e));  // run order -> caller's index
    for (int i = 0; i < n_e; ++i) perm[i] = i;
    std::vector<int32_t> part_run;  // partner in the run order
    if (pair) {
      std::vector<char> placed(static_cast<size_t>(n_e), 0);
      int k = 0;
      for (int i = 0; i < n_e; ++i)
        if (!placed[i] && partner[i] != i) {
          perm[k++] = i;
          perm[k++] = partner[i];
          placed[i] = placed[partner[i]] = 1;
        }
      for (int i = 0; i < n_e; ++i)
        if (!placed[i]) perm[k++] = i;
      std::vector<int32_t> inv(static_cast<size_t>(n_e));
      for (int j = 0; j < n_e; ++j) inv[perm[j]] = j;
      part_run.resize(static_cast<size_t>(n_e));
      for (int j = 0; j < n_e; ++j) part_run[j] = inv[partner[perm[j]]];
      dpart = static_cast<int32_t*>(upload(part_run));
      dmap = static_cast<int32_t*>(upload(perm));
    }
    std::vector<double> eps(2 * n_e);
    for (int i = 0; i < n_e; ++i) {
      eps[2 * i] = energies[perm[i]];
      eps[2 * i + 1] = broadening;
    }
    deps = static_cast<double*>(upload(eps));
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) bcl[a][b] = dalloc(2 * rb * g->nseg * n_e);
    do_interp(g, delta, A_ind, st);
    const int blk_all = 256;  // energies of one boundary-only launch (64 lanes x 4)
    int cur = 0;
    qc::SweepBufs b;
    b.nodes = g->nodes;
    b.gbuf = nullptr;
    b.ebuf = nullptr;
    for (int it = 0; it < bc_iters; ++it) {
      for (int e0 = 0; e0 < n_e; e0 += blk_all) {
        const int ne = std::min(blk_all, n_e - e0);
        qc::SweepArgs a = sweep_args(g, ne, n_e, e0, deps, nullptr, pair);
        a.bc_valid = it > 0;
        b.bc_g_prev = bcl[cur][0];
        b.bc_gt_prev = bcl[cur][1];
        b.bc_g_next = bcl[1 - cur][0];
        b.bc_gt_next = bcl[1 - cur][1];
        launch_sweep_timed(g, 2, a, b, st);
      }
      if (pair) {
        if (g->precision == QC_MIXED)
          qc::launch_mirror_fill<float>(g->mirror_pairs, g->npairs, n_e, dpart, bcl[1 - cur][0], bcl[1 - cur][1], st);
        else
          qc::launch_mirror_fill<double>(g->mirror_pairs, g->npairs, n_e, dpart, bcl[1 - cur][0], bcl[1 - cur][1], st);
      }
      cur = 1 - cur;
    }
    // output pass in energy blocks of up to 64 (32 lanes of two energies per
    // segment: long contiguous gamma and LDOS rows), bounded by half of the
    // free device memory
    size_t free_b = 0, total_b = 0;
    hcheck(hipMemGetInfo(&free_b, &total_b), "hipMemGetInfo");
    const double budget = std::max(static_cast<double>(1 << 30), 0.5 * static_cast<double>(free_b));
    const double per_e = static_cast<double>(g->nslot) * 3.0 * rb;
    int blk = 64;
    while (blk > 1 && blk * per_e > budget) blk >>= 1;
    blk = std::min(blk, n_e);
    // paired output: blocks of even size hold whole pairs (self-partners,
    // last in the run order, pair with themselves)
    const bool out_pair = pair && g->rb_fold && (blk % 2 == 0 || blk == n_e);
    lg = dalloc(2 * rb * g->nslot * blk);
    le = dalloc(rb * g->nslot * blk);
    qc::launch_fill(ldos_out, static_cast<int64_t>(n_e) * g->ncell, 0.0, st);
    for (int e0 = 0; e0 < n_e; e0 += blk) {
      const int ne = std::min(blk, n_e - e0);
      qc::SweepArgs a = sweep_args(g, ne, n_e, e0, deps, nullptr, out_pair);
      a.bc_valid = bc_iters > 0;
      b.bc_g_prev = bcl[cur][0];
      b.bc_gt_prev = bcl[cur][1];
      b.bc_g_next = nullptr;
      b.bc_gt_next = nullptr;
      b.gbuf = lg;
      b.ebuf = le;
      launch_sweep_timed(g, 1, a, b, st);
      qc::LdosBackArgs la{};
      la.ncg = g->ncg;
      la.ncell = g->ncell;
      la.n_theta = g->n_theta;
      la.n_e = ne;
      la.e_off = e0;
      la.grain_cells = g->grain_cells;
      la.rb_idx = g->rb_idx;
      la.rb_w = g->rb_w;
      la.wk = g->wk;
      la.out = ldos_out;
      la.e_map = dmap;
      la.e_partner = out_pair ? dpart : nullptr;
      la.fold_k0 = out_pair ? g->n_theta / 2 : 0;
      if (g->precision == QC_MIXED)
        qc::launch_ldos_back<float>(la, le, st);
      else
        qc::launch_ldos_back<double>(la, le, st);
      hcheck(hipGetLastError(), "ldos launch");
    }
    hcheck(hipStreamSynchronize(st), "sync");
    return QC_OK;
  });
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      if (bcl[a][b]) (void)hipFree(bcl[a][b]);
  if (deps) (void)hipFree(deps);
  if (dpart) (void)hipFree(dpart);
  if (dmap) (void)hipFree(dmap);
  if (lg) (void)hipFree(lg);
  if (le) (void)hipFree(le);
  return rs;
}

qc_status qc_ldos_converge(qc_grain* g, const double* delta, const double* A_ind, const double* energies, int n_e,
                           double broadening, double tol, int max_iter, int energies_per_block, int* iters_out,
                           double* ldos_out, void* stream) {
  if (!g) return fail(QC_ERR_INVALID, "grain is NULL");
  if (!delta || !A_ind || !energies || !ldos_out) return fail(QC_ERR_INVALID, "NULL argument");
  if (n_e < 1 || max_iter < 1 || energies_per_block < 0) return fail(QC_ERR_INVALID, "bad n_e, max_iter or block");
  if (!(broadening > 0.0) || !std::isfinite(broadening)) return fail(QC_ERR_INVALID, "broadening must be > 0");
  if (!(tol >= 0.0)) return fail(QC_ERR_INVALID, "tol must be >= 0");
  for (int i = 0; i < n_e; ++i)
    if (!std::isfinite(energies[i])) return fail(QC_ERR_INVALID, "energies must be finite");
  void* bcl[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};
  double* deps = nullptr;
  double* prev = nullptr;
  void* lg = nullptr;
  void* le = nullptr;
  qc_status rs = guarded([&]() -> qc_status {
    hipStream_t st = S(stream);
    hcheck(hipSetDevice(g->device), "hipSetDevice");
    const size_t rb = g->real_bytes();
    std::vector<double> eps(2 * n_e);
    for (int i = 0; i < n_e; ++i) {
      eps[2 * i] = energies[i];
      eps[2 * i + 1] = broadening;
    }
    deps = static_cast<double*>(upload(eps));
    do_interp(g, delta, A_ind, st);
    // energy block: the caller's, or the largest power of two up to 64 whose
    // gamma rows fit in half of the free device memory
    int blk = energies_per_block;
    if (blk == 0) {
      size_t free_b = 0, total_b = 0;
      hcheck(hipMemGetInfo(&free_b, &total_b), "hipMemGetInfo");
      const double budget = std::max(static_cast<double>(1 << 30), 0.5 * static_cast<double>(free_b));
      const double per_e = static_cast<double>(g->nslot) * 3.0 * rb + 4.0 * rb * g->nseg;
      blk = 64;
      while (blk > 1 && blk * per_e > budget) blk >>= 1;
    }
    blk = std::min(blk, n_e);
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) bcl[a][b] = dalloc(2 * rb * g->nseg * blk);
    lg = dalloc(2 * rb * g->nslot * blk);
    le = dalloc(rb * g->nslot * blk);
    prev = static_cast<double*>(dalloc(sizeof(double) * blk * g->ncell));
    qc::launch_fill(ldos_out, static_cast<int64_t>(n_e) * g->ncell, 0.0, st);
    int worst = 0;
    for (int e0 = 0; e0 < n_e; e0 += blk) {
      const int ne = std::min(blk, n_e - e0);
      double* out = ldos_out + static_cast<int64_t>(e0) * g->ncell;
      int cur = 0, it = 0;
      for (; it < max_iter; ++it) {
        // one output sweep of the block from the previous end values (bulk
        // roots at the first), which also stores this sweep's end values
        qc::SweepArgs a = sweep_args(g, ne, ne, 0, deps + 2 * e0, nullptr);
        a.bc_valid = it > 0;
        qc::SweepBufs b;
        b.nodes = g->nodes;
        b.bc_g_prev = bcl[cur][0];
        b.bc_gt_prev = bcl[cur][1];
        b.bc_g_next = bcl[1 - cur][0];
        b.bc_gt_next = bcl[1 - cur][1];
        b.gbuf = lg;
        b.ebuf = le;
        launch_sweep_timed(g, 1, a, b, st);
        cur = 1 - cur;
        if (it > 0)
          hcheck(hipMemcpyAsync(prev, out, sizeof(double) * ne * g->ncell, hipMemcpyDeviceToDevice, st), "copy");
        qc::LdosBackArgs la{};
        la.ncg = g->ncg;
        la.ncell = g->ncell;
        la.n_theta = g->n_theta;
        la.n_e = ne;
        la.e_off = 0;
        la.grain_cells = g->grain_cells;
        la.rb_idx = g->rb_idx;
        la.rb_w = g->rb_w;
        la.wk = g->wk;
        la.out = out;
        if (g->precision == QC_MIXED)
          qc::launch_ldos_back<float>(la, le, st);
        else
          qc::launch_ldos_back<double>(la, le, st);
        hcheck(hipGetLastError(), "ldos launch");
        if (it == 0) continue;
        // relative 2-norm change of the block's LDOS (every cell; zero off the grain)
        qc::DiffNormArgs dn;
        dn.xnew = out;
        dn.xold = prev;
        dn.idx = nullptr;
        dn.n = static_cast<int64_t>(ne) * g->ncell;
        dn.nrep = 1;
        dn.field_stride = 0;
        dn.stride = 1;
        dn.p = 2;
        dn.part = region(g, kRDiffD);
        dn.update = nullptr;
        dn.alpha = 1.0;
        dn.vel = nullptr;
        dn.beta = 0.0;
        qc::launch_diff_norm(dn, kParts, st);
        fetch_parts(g, st);
        if (rel_from_parts(g, kRDiffD, 2) < tol) {
          ++it;
          break;
        }
      }
      worst = std::max(worst, it);
    }
    hcheck(hipStreamSynchronize(st), "sync");
    if (iters_out) *iters_out = worst;
    return QC_OK;
  });
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b)
      if (bcl[a][b]) (void)hipFree(bcl[a][b]);
  for (void* p : {static_cast<void*>(deps), static_cast<void*>(prev), lg, le})
    if (p) (void)hipFree(p);
  return rs;
}

qc_status qc_green_average(qc_grain* g, const double* delta, const double* A_ind, double* g_out, void* stream) {
  if (!g) return fail(QC_ERR_INVALID, "grain is NULL");
  if (!delta || !A_ind || !g_out) return fail(QC_ERR_INVALID, "delta, A_ind and g_out are required");
  void* lg = nullptr;
  void* le = nullptr;
  qc_status rs = guarded([&]() -> qc_status {
    hipStream_t st = S(stream);
    hcheck(hipSetDevice(g->device), "hipSetDevice");
    const size_t rb = g->real_bytes();
    do_interp(g, delta, A_ind, st);
    // poles in blocks of up to 64, bounded by half of the free device memory
    size_t free_b = 0, total_b = 0;
    hcheck(hipMemGetInfo(&free_b, &total_b), "hipMemGetInfo");
    const double budget = std::max(static_cast<double>(1 << 30), 0.5 * static_cast<double>(free_b));
    const double per_e = static_cast<double>(g->nslot) * 4.0 * rb;
    int blk = 64;
    while (blk > 1 && blk * per_e > budget) blk >>= 1;
    blk = std::min(blk, g->n_poles);
    lg = dalloc(2 * rb * g->nslot * blk);
    le = dalloc(2 * rb * g->nslot * blk);
    qc::launch_fill(g_out, 2LL * g->n_poles * g->ncell, 0.0, st);
    qc::SweepBufs b;
    b.nodes = g->nodes;
    b.bc_g_prev = g->bc[g->bc_cur][0];
    b.bc_gt_prev = g->bc[g->bc_cur][1];
    b.bc_g_next = nullptr;
    b.bc_gt_next = nullptr;
    b.gbuf = lg;
    b.ebuf = le;
    for (int e0 = 0; e0 < g->n_poles; e0 += blk) {
      const int ne = std::min(blk, g->n_poles - e0);
      qc::SweepArgs a = sweep_args(g, ne, g->n_poles, e0, g->eps, nullptr);
      a.bc_valid = g->bc_valid;  // the start values the next sweep would use
      launch_sweep_timed(g, 3, a, b, st);
      qc::LdosBackArgs la{};
      la.ncg = g->ncg;
      la.ncell = g->ncell;
      la.n_theta = g->n_theta;
      la.n_e = ne;
      la.e_off = e0;
      la.grain_cells = g->grain_cells;
      la.rb_idx = g->rb_idx;
      la.rb_w = g->rb_w;
      la.wk = g->wk;
      la.out = g_out;
      if (g->precision == QC_MIXED)
        qc::launch_green_back<float>(la, le, st);
      else
        qc::launch_green_back<double>(la, le, st);
      hcheck(hipGetLastError(), "green launch");
    }
    hcheck(hipStreamSynchronize(st), "sync");
    return QC_OK;
  });
  if (lg) (void)hipFree(lg);
  if (le) (void)hipFree(le);
  return rs;
}

qc_status qc_get_state(const qc_grain* g, void* state, size_t* bytes, void* stream) {
  if (!g || !bytes) return fail(QC_ERR_INVALID, "NULL argument");
  const size_t half = 2 * g->real_bytes() * g->nseg * g->n_poles;
  if (!state) {
    *bytes = 2 * half;
    return QC_OK;
  }
  if (*bytes < 2 * half) return fail(QC_ERR_INVALID, "state buffer too small");
  if (!g->bc_valid || !g->bc[0][0]) return fail(QC_ERR_INVALID, "no boundary values yet (run a sweep first)");
  return guarded([&]() -> qc_status {
    hcheck(hipSetDevice(g->device), "hipSetDevice");
    hcheck(hipMemcpyAsync(state, g->bc[g->bc_cur][0], half, hipMemcpyDeviceToDevice, S(stream)), "copy");
    hcheck(hipMemcpyAsync(static_cast<char*>(state) + half, g->bc[g->bc_cur][1], half, hipMemcpyDeviceToDevice,
                          S(stream)),
           "copy");
    *bytes = 2 * half;
    return QC_OK;
  });
}

qc_status qc_set_state(qc_grain* g, const void* state, size_t bytes, void* stream) {
  if (!g || !state) return fail(QC_ERR_INVALID, "NULL argument");
  const size_t half = 2 * g->real_bytes() * g->nseg * g->n_poles;
  if (bytes != 2 * half) return fail(QC_ERR_INVALID, "state size does not match this grain");
  return guarded([&]() -> qc_status {
    hcheck(hipSetDevice(g->device), "hipSetDevice");
    ensure_sweep_buffers(g);
    hcheck(hipMemcpyAsync(g->bc[g->bc_cur][0], state, half, hipMemcpyDeviceToDevice, S(stream)), "copy");
    hcheck(hipMemcpyAsync(g->bc[g->bc_cur][1], static_cast<const char*>(state) + half, half, hipMemcpyDeviceToDevice,
                          S(stream)),
           "copy");
    g->bc_valid = 1;
    return QC_OK;
  });
}

}  // extern "C"

namespace {

template <typename T>
std::vector<T> download(const T* d, size_t n) {
  std::vector<T> h(n);
  if (n) hcheck(hipMemcpy(h.data(), d, sizeof(T) * n, hipMemcpyDeviceToHost), "copy");
  return h;
}

// Compressed rows from (row, column, weight) triples given row by row in
// any order: counting sort by row, entries of a row in input order.
struct Csr {
  std::vector<int64_t> ptr;
  std::vector<int32_t> col;
  std::vector<double> w;
};
Csr to_csr(int64_t nrows, const std::vector<int64_t>& row, const std::vector<int32_t>& col,
           const std::vector<double>& w) {
  Csr c;
  c.ptr.assign(nrows + 1, 0);
  for (int64_t r : row) ++c.ptr[r + 1];
  for (int64_t i = 0; i < nrows; ++i) c.ptr[i + 1] += c.ptr[i];
  c.col.resize(row.size());
  c.w.resize(row.size());
  std::vector<int64_t> pos(c.ptr.begin(), c.ptr.end() - 1);
  for (size_t e = 0; e < row.size(); ++e) {
    const int64_t p = pos[row[e]]++;
    c.col[p] = col[e];
    c.w[p] = w[e];
  }
  return c;
}

// The adjoint's transposed tables, built on the host from the device tables
// the forward path uses: rotate-back entries by slot, interpolation entries
// (the same stencil code as the device) by cell.
void ensure_adjoint_tables(qc_grain* g) {
  if (g->bt_ptr) return;
  {
    const size_t n = static_cast<size_t>(g->n_theta) * 4 * g->ncg;
    const std::vector<int32_t> idx = download(g->rb_idx, n);
    const std::vector<double> w = download(g->rb_w, n);
    std::vector<int64_t> row;
    std::vector<int32_t> col;
    std::vector<double> ww;
    for (size_t o = 0; o < n; ++o) {
      if (w[o] == 0.0) continue;
      row.push_back(idx[o]);
      col.push_back(static_cast<int32_t>(o % g->ncg));
      ww.push_back(w[o]);
    }
    const Csr c = to_csr(g->nslot, row, col, ww);
    g->bt_ptr = static_cast<int64_t*>(upload(c.ptr));
    g->bt_c = static_cast<int32_t*>(upload(c.col));
    g->bt_w = static_cast<double*>(upload(c.w));
  }
  const std::vector<double> px = download(g->slot_px, g->nslot), py = download(g->slot_py, g->nslot);
  const std::vector<int32_t> fb = download(g->slot_fb, g->nslot);
  const std::vector<uint8_t> mask = download(g->mask, g->ncell);
  qc::GridGeom gg = geom_of(g);
  gg.mask = mask.data();
  std::vector<int64_t> drow, arow;
  std::vector<int32_t> dcol, acol;
  std::vector<double> dw, aw;
  drow.reserve(4 * g->nslot);
  arow.reserve(4 * g->nslot);
  for (int64_t s = 0; s < g->nslot; ++s) {
    int di[4], ai[4];
    double dwt[4], awt[4];
    qc::delta_stencil(gg, px[s], py[s], fb[s], di, dwt);
    qc::a_stencil(gg, px[s], py[s], ai, awt);
    for (int c = 0; c < 4; ++c) {
      if (dwt[c] != 0.0) {
        drow.push_back(di[c]);
        dcol.push_back(static_cast<int32_t>(s));
        dw.push_back(dwt[c]);
      }
      if (awt[c] != 0.0) {
        arow.push_back(ai[c]);
        acol.push_back(static_cast<int32_t>(s));
        aw.push_back(awt[c]);
      }
    }
  }
  const Csr d = to_csr(g->ncell, drow, dcol, dw);
  const Csr a = to_csr(g->ncell, arow, acol, aw);
  g->it_dptr = static_cast<int64_t*>(upload(d.ptr));
  g->it_ds = static_cast<int32_t*>(upload(d.col));
  g->it_dw = static_cast<double*>(upload(d.w));
  g->it_aptr = static_cast<int64_t*>(upload(a.ptr));
  g->it_as = static_cast<int32_t*>(upload(a.col));
  g->it_aw = static_cast<double*>(upload(a.w));
}

// The transposed rotate-back for the paired reverse mode.  A corner of an
// upper angle k' = k + n_theta/2 reads the node sums of its mirror slot on
// angle k (S_f, S_I equal, S_g of opposite sign); its gradient terms, formed
// with the mirror slot's angle (w, eta equal; v_k' = -v_k cancels the S_g
// sign), are those of a corner of angle k, so the entry moves onto the
// mirror slot with its weight.
void ensure_adjoint_pair_tables(qc_grain* g) {
  if (g->btp_ptr || !g->pair_ok) return;
  const int64_t nc = g->ncg;
  const int n2 = g->n_theta / 2;
  const size_t n = static_cast<size_t>(g->n_theta) * 4 * nc;
  const std::vector<int32_t> idx = download(g->rb_idx, n);
  const std::vector<double> w = download(g->rb_w, n);
  const std::vector<int4> r4 = download(g->rb4, static_cast<size_t>(g->n_theta) * nc);
  const std::vector<int4> r4p = download(g->rb4_pair, static_cast<size_t>(g->n_theta) * nc);
  std::vector<int32_t> mirror(static_cast<size_t>(g->nslot), -1);
  for (size_t e = static_cast<size_t>(n2) * nc; e < r4.size(); ++e) {
    const int32_t a[4] = {r4[e].x, r4[e].y, r4[e].z, r4[e].w};
    const int32_t b[4] = {r4p[e].x, r4p[e].y, r4p[e].z, r4p[e].w};
    for (int q = 0; q < 4; ++q)
      if (a[q] >= 0) mirror[a[q]] = b[q];
  }
  std::vector<int64_t> row;
  std::vector<int32_t> col;
  std::vector<double> ww;
  for (size_t o = 0; o < n; ++o) {
    if (w[o] == 0.0) continue;
    const int k = static_cast<int>(o / (4 * static_cast<size_t>(nc)));
    int32_t sl = idx[o];
    if (k >= n2) {
      sl = mirror[sl];
      if (sl < 0) throw std::runtime_error("paired reverse mode: a corner without a mirror slot");
    }
    row.push_back(sl);
    col.push_back(static_cast<int32_t>(o % nc));
    ww.push_back(w[o]);
  }
  const Csr c = to_csr(g->nslot, row, col, ww);
  g->btp_ptr = static_cast<int64_t*>(upload(c.ptr));
  g->btp_c = static_cast<int32_t*>(upload(c.col));
  g->btp_w = static_cast<double*>(upload(c.w));
}

}  // namespace

extern "C" {

qc_status qc_sweep_adjoint(qc_grain* g, const double* delta, const double* A_ind, const double* g_delta_new,
                           const double* g_j, double g_omega, double* grad_delta, double* grad_A, void* stream) {
  if (!g) return fail(QC_ERR_INVALID, "grain is NULL");
  if (!delta || !A_ind || !grad_delta || !grad_A) return fail(QC_ERR_INVALID, "NULL argument");
  if (g->precision != QC_FP64) return fail(QC_ERR_INVALID, "the adjoint sweep needs a QC_FP64 grain");
  if (g->last_bc_valid < 0) return fail(QC_ERR_INVALID, "run qc_sweep first: the adjoint differentiates it");
  if (!std::isfinite(g_omega)) return fail(QC_ERR_INVALID, "g_omega must be finite");
  return guarded([&]() -> qc_status {
    hipStream_t st = S(stream);
    hcheck(hipSetDevice(g->device), "hipSetDevice");
    const size_t nb = sizeof(double) * 2 * g->nslot * g->n_poles;
    int G, epl;
    lane_shape(g->n_poles, g->epl_override, g->precision == QC_MIXED, G, epl);
    if (g->adj_ck == 0) {
      if (!g->gtbuf) g->gtbuf = dalloc(nb);
      if (!g->lgt) g->lgt = dalloc(nb);
    } else {
      const int ck = g->adj_ck;
      if (g->ck_built != ck) {
        // checkpoint blocks of each segment: ceil(n / ck)
        const std::vector<int32_t> n = download(g->seg_n, g->nseg);
        std::vector<int64_t> base(g->nseg + 1, 0);
        for (int64_t sg = 0; sg < g->nseg; ++sg) base[sg + 1] = base[sg] + (n[sg] + ck - 1) / ck;
        for (void* p : {static_cast<void*>(g->ckbase), g->ckg, g->ckgt})
          if (p) (void)hipFree(p);
        g->ckbase = static_cast<int64_t*>(upload(base));
        const size_t cbytes = sizeof(double) * 2 * std::max<int64_t>(base[g->nseg], 1) * g->n_poles;
        g->ckg = dalloc(cbytes);
        g->ckgt = dalloc(cbytes);
        g->ck_built = ck;
      }
      const size_t sbytes = sizeof(double) * 2 * 2 * static_cast<size_t>(ck) * epl * g->nseg * G;
      if (sbytes > g->ckscr_bytes) {
        if (g->ckscr) (void)hipFree(g->ckscr);
        g->ckscr = nullptr;
        g->ckscr_bytes = 0;
        g->ckscr = dalloc(sbytes);
        g->ckscr_bytes = sbytes;
      }
    }
    if (!g->gS) g->gS = static_cast<double*>(dalloc(sizeof(double) * 4 * g->nslot));
    if (!g->gV) g->gV = static_cast<double*>(dalloc(sizeof(double) * 3 * g->nslot));
    ensure_adjoint_tables(g);
    // with angle pairs the reverse mode marches the lower angles only, as
    // the forward sweep does
    const bool pair = g->pairing;
    if (pair) ensure_adjoint_pair_tables(g);
    do_interp(g, delta, A_ind, st, pair);
    // gradients of the per-node sums
    qc::BackAdjArgs ba;
    ba.ncg = g->ncg;
    ba.ncell = g->ncell;
    ba.ncomp = g->ncomp;
    ba.n_theta = g->n_theta;
    ba.grain_cells = g->grain_cells;
    ba.rb_idx = g->rb_idx;
    ba.rb_w = g->rb_w;
    ba.wk = g->wk;
    ba.cosk = g->cosk;
    ba.sink = g->sink;
    ba.eta = g->eta;
    ba.den = g->den;
    ba.four_q = 4.0 * g->q;
    ba.h2 = g->h * g->h;
    ba.gomega = g_omega;
    ba.gdn = g_delta_new;
    ba.gj = g_j;
    ba.gS = g->gS;
    ba.nslot = pair ? g->nslot_pair : g->nslot;
    ba.slot_angle = g->slot_angle;
    ba.bt_ptr = pair ? g->btp_ptr : g->bt_ptr;
    ba.bt_c = pair ? g->btp_c : g->bt_c;
    ba.bt_w = pair ? g->btp_w : g->bt_w;
    qc::launch_back_adjoint(ba, st);
    // reverse sweep with the store the latest sweep read
    qc::AdjArgs a = sweep_args(g, g->n_poles, g->n_poles, 0, g->eps, g->rpd, pair);
    a.bc_valid = g->last_bc_valid;
    qc::AdjBufs b;
    b.nodes = g->nodes;
    b.bc_g_prev = g->bc[1 - g->bc_cur][0];
    b.bc_gt_prev = g->bc[1 - g->bc_cur][1];
    b.gbuf = g->gbuf;
    b.gtbuf = g->gtbuf;
    b.lgt = g->lgt;
    b.gS = g->gS;
    b.gV = g->gV;
    if (g->adj_ck > 0) {
      b.ck = g->adj_ck;
      b.ckbase = g->ckbase;
      b.ckg = g->ckg;
      b.ckgt = g->ckgt;
      b.scr = g->ckscr;
      b.nthr = a.nseg * G;
    }
    qc::launch_adjoint(epl, a, b, st);
    hcheck(hipGetLastError(), "adjoint launch");
    // the upper angles' slots take no part in the paired map
    if (pair) qc::launch_fill(g->gV + 3 * g->nslot_pair, 3 * (g->nslot - g->nslot_pair), 0.0, st);
    // back to the reference grid (the gather writes every cell)
    qc::InterpAdjArgs ia;
    ia.nslot = g->nslot;
    ia.ncell = g->ncell;
    ia.ncomp = g->ncomp;
    ia.n_theta = g->n_theta;
    ia.slot_angle = g->slot_angle;
    ia.geom = geom_of(g);
    ia.px = g->slot_px;
    ia.py = g->slot_py;
    ia.fb = g->slot_fb;
    ia.eta = g->eta;
    ia.cosk = g->cosk;
    ia.sink = g->sink;
    ia.gV = g->gV;
    ia.gdelta = grad_delta;
    ia.gA = grad_A;
    ia.it_dptr = g->it_dptr;
    ia.it_ds = g->it_ds;
    ia.it_dw = g->it_dw;
    ia.it_aptr = g->it_aptr;
    ia.it_as = g->it_as;
    ia.it_aw = g->it_aw;
    qc::launch_interp_adjoint(ia, st);
    if (g_omega != 0.0) {
      qc::OmegaAdjArgs oa;
      oa.ncg = g->ncg;
      oa.ncell = g->ncell;
      oa.ncomp = g->ncomp;
      oa.n_theta = g->n_theta;
      oa.grain_cells = g->grain_cells;
      oa.delta = delta;
      oa.eta = g->eta;
      oa.wk = g->wk;
      oa.logt = g->logt;
      oa.twopi_rz = g->twopi_rz;
      oa.h2 = g->h * g->h;
      oa.gomega = g_omega;
      oa.gdelta = grad_delta;
      qc::launch_omega_delta_adjoint(oa, st);
      if (g->kappa > 0.0) {
        qc::launch_curl(A_ind, g->bbuf, g->nx, g->ny, g->h, st);
        qc::launch_curl_adjoint(g->bbuf, grad_A, g->nx, g->ny, g->h, g->h * g->h * g->kappa * g->kappa * g_omega, st);
      }
    }
    hcheck(hipGetLastError(), "adjoint launch");
    return QC_OK;
  });
}

qc_status qc_grain_set_accelerator(qc_grain* g, int kind, double beta) {
  if (!g) return fail(QC_ERR_INVALID, "grain is NULL");
  if (kind < 0 || kind > 3)
    return fail(QC_ERR_INVALID, "accelerator must be 0 (Picard), 1 (Polyak), 2 (BB) or 3 (CongAcc)");
  if (kind == 1 && !(beta > 0.0 && beta <= 1.0)) return fail(QC_ERR_INVALID, "Polyak drag must be in (0, 1]");
  g->accel = kind;
  g->beta = kind == 1 ? beta : 0.5;
  return QC_OK;
}

qc_status qc_grain_set_pairing(qc_grain* g, int enable) {
  if (!g) return fail(QC_ERR_INVALID, "grain is NULL");
  if (enable && !g->pair_ok) return fail(QC_ERR_INVALID, "this grain's tables do not allow angle pairs");
  g->pairing = enable != 0;
  return QC_OK;
}

qc_status qc_grain_get_pairing(const qc_grain* g, int* available, int* enabled, int64_t* swept_steps_per_sweep) {
  if (!g) return fail(QC_ERR_INVALID, "grain is NULL");
  if (available) *available = g->pair_ok ? (g->rb_fold ? 3 : 1) : 0;
  if (enabled) *enabled = g->pairing ? 1 : 0;
  if (swept_steps_per_sweep) {
    if (!g->pairing) {
      *swept_steps_per_sweep = g->info.steps_per_sweep;
    } else {
      const std::vector<int32_t> n = download(g->seg_n, g->nseg_pair);
      int64_t s = 0;
      for (int32_t v : n) s += v + 1;
      *swept_steps_per_sweep = 2 * static_cast<int64_t>(g->n_poles) * s;
    }
  }
  return QC_OK;
}

qc_status qc_grain_get_accel_stats(const qc_grain* g, int64_t* bisected, int64_t* anti_parallel) {
  if (!g) return fail(QC_ERR_INVALID, "grain is NULL");
  if (bisected) *bisected = g->cong_bisect;
  if (anti_parallel) *anti_parallel = g->cong_anti;
  return QC_OK;
}

qc_status qc_grain_set_adjoint_checkpoint(qc_grain* g, int every) {
  if (!g) return fail(QC_ERR_INVALID, "grain is NULL");
  if (every < 0 || every > 4096) return fail(QC_ERR_INVALID, "checkpoint interval must be in [0, 4096]");
  g->adj_ck = every;
  return QC_OK;
}

qc_status qc_grain_set_lanes(qc_grain* g, int energies_per_lane) {
  if (!g) return fail(QC_ERR_INVALID, "grain is NULL");
  if (energies_per_lane != 0 && energies_per_lane != 1 && energies_per_lane != 2 && energies_per_lane != 3 &&
      energies_per_lane != 4 && energies_per_lane != 8)
    return fail(QC_ERR_INVALID, "energies_per_lane must be 0 (auto), 1, 2, 3, 4 or 8");
  g->epl_override = energies_per_lane;
  return QC_OK;
}

qc_status qc_grain_set_split(qc_grain* g, double frac) {
  if (!g) return fail(QC_ERR_INVALID, "grain is NULL");
  if (!(frac >= 0.0 && frac <= 1.0)) return fail(QC_ERR_INVALID, "frac must be in [0, 1]");
  g->split_frac = frac;
  return QC_OK;
}

qc_status qc_grain_get_split(qc_grain* g, double* frac, int64_t* n_wide) {
  if (!g) return fail(QC_ERR_INVALID, "grain is NULL");
  return guarded([&]() -> qc_status {
    if (frac) *frac = g->split_frac;
    if (n_wide) {
      hcheck(hipSetDevice(g->device), "hipSetDevice");
      qc::SweepArgs a = sweep_args(g, g->n_poles, g->n_poles, 0, g->eps, g->rpd, true);
      int G, epl;
      lane_shape(a.n_e, g->epl_override, g->precision == QC_MIXED, G, epl);
      *n_wide = split_count(g, a, epl);
    }
    return QC_OK;
  });
}

qc_status qc_grain_get_lanes(const qc_grain* g, int* energies_per_lane, int* lanes_per_segment) {
  if (!g) return fail(QC_ERR_INVALID, "grain is NULL");
  if (!energies_per_lane || !lanes_per_segment) return fail(QC_ERR_INVALID, "output pointers are required");
  int G = 1, epl = 1;
  lane_shape(g->n_poles, g->epl_override, g->precision == QC_MIXED, G, epl);
  *energies_per_lane = epl;
  *lanes_per_segment = G;
  return QC_OK;
}

qc_status qc_profile_enable(qc_grain* g, int enable) {
  if (!g) return fail(QC_ERR_INVALID, "grain is NULL");
  g->prof = enable != 0;
  return QC_OK;
}

qc_status qc_profile_read(qc_grain* g, double* sweep_ms, int64_t* sweep_launches) {
  if (!g || !sweep_ms || !sweep_launches) return fail(QC_ERR_INVALID, "NULL argument");
  return guarded([&]() -> qc_status {
    hcheck(hipSetDevice(g->device), "hipSetDevice");
    double tot = 0.0;
    for (auto& e : g->ev) {
      hcheck(hipEventSynchronize(e.second), "event sync");
      float ms = 0.f;
      hcheck(hipEventElapsedTime(&ms, e.first, e.second), "event time");
      tot += ms;
      (void)hipEventDestroy(e.first);
      (void)hipEventDestroy(e.second);
    }
    *sweep_ms = tot;
    *sweep_launches = static_cast<int64_t>(g->ev.size());
    g->ev.clear();
    return QC_OK;
  });
}

}  // extern "C"

// ------------------------------------------------------------------------
// batched grains
// ------------------------------------------------------------------------
struct qc_batch {
  int device = 0;
  int precision = 0;
  std::vector<qc_grain*> grains;
  std::vector<double*> delta, A;   // per-grain fields owned by the batch
  int epl = 0;  // energies per lane of every grain; 0: each grain's automatic choice
  int nblocks = 0;
  qc::BatchGrainDev* d_args = nullptr;  // [n] for the current launch
  int2* d_tiles = nullptr;
  // gamma spill of the persistent sweep: wave_elems records per resident
  // wave slot (nblocks x 4 slots), sized for the largest tile of any grain
  void* spill = nullptr;
  size_t spill_bytes = 0;
  int64_t wave_elems = 0;
  int ntiles = 0;
  // tiles grouped by the grains' lane shapes: one persistent launch per group
  std::vector<int> grp_epl, grp_off, grp_n;
  int* d_counter = nullptr;  // one tile counter per group
  hipStream_t own = nullptr;
  hipGraphExec_t gexec = nullptr;
  std::vector<int> graph_parity;   // bc_cur of every grain when the graph was captured
  int graph_epl = 0;
  int64_t steps_per_iter = 0;
  double last_ms = 0.0;
  std::vector<qc::BatchGrainDev> host_args;
};

namespace {

// tiles: for every grain, waves of 64/G segments in launch order (longest
// first); all tiles sorted by their longest segment, longest first
// Tiles: for every grain, waves of 64/G segments in launch order (longest
// first).  Grains are grouped by lane shape (energies per lane: the batch's
// setting, or each grain's automatic choice when it is 0); within a group
// the tiles are sorted by their longest segment, longest first.
void drop_graph(qc_batch* b);

void build_tiles(qc_batch* b) {
  struct T3 {
    int g, w0, cost;
  };
  std::vector<std::vector<T3>> groups(9);
  for (size_t gi = 0; gi < b->grains.size(); ++gi) {
    qc_grain* g = b->grains[gi];
    int G, epl;
    lane_shape(g->n_poles, b->epl, g->precision == QC_MIXED, G, epl);
    const int64_t nsw = g->pairing ? g->nseg_pair : g->nseg;
    std::vector<int32_t> ord(nsw), n(g->nseg);
    hcheck(hipMemcpy(ord.data(), g->pairing ? g->order_pair : g->order, sizeof(int32_t) * nsw, hipMemcpyDeviceToHost),
           "copy");
    hcheck(hipMemcpy(n.data(), g->seg_n, sizeof(int32_t) * g->nseg, hipMemcpyDeviceToHost), "copy");
    const int per = 64 / G;
    for (int64_t w = 0; w < nsw; w += per)
      groups[epl].push_back({static_cast<int>(gi), static_cast<int>(w), n[ord[w]] + 1});
  }
  std::vector<int2> t;
  b->grp_epl.clear();
  b->grp_off.clear();
  b->grp_n.clear();
  for (int e = 1; e <= 8; ++e) {
    std::vector<T3>& all = groups[e];
    if (all.empty()) continue;
    std::stable_sort(all.begin(), all.end(), [](const T3& x, const T3& y) { return x.cost > y.cost; });
    b->grp_epl.push_back(e);
    b->grp_off.push_back(static_cast<int>(t.size()));
    b->grp_n.push_back(static_cast<int>(all.size()));
    for (const T3& x : all) t.push_back(make_int2(x.g, x.w0));
  }
  if (b->d_tiles) (void)hipFree(b->d_tiles);
  b->d_tiles = static_cast<int2*>(upload(t));
  b->ntiles = static_cast<int>(t.size());
  // per-wave spill: 64/G segments of up to maxn nodes and n_e poles each
  int64_t we = 1;
  for (qc_grain* g : b->grains) {
    int G, epl;
    lane_shape(g->n_poles, b->epl, g->precision == QC_MIXED, G, epl);
    we = std::max(we, static_cast<int64_t>(64 / G) * g->maxn * g->n_poles);
  }
  b->wave_elems = we;
  const size_t need = static_cast<size_t>(b->nblocks) * 4 * we * 2 * b->grains[0]->real_bytes();
  if (need > b->spill_bytes) {
    drop_graph(b);  // a captured graph holds the old pointer
    if (b->spill) (void)hipFree(b->spill);
    b->spill = nullptr;
    b->spill_bytes = 0;
    b->spill = dalloc(need);
    b->spill_bytes = need;
  }
}

// per-grain arguments of the next sweep (each grain's current store parity)
void upload_args(qc_batch* b, hipStream_t st) {
  std::vector<qc::BatchGrainDev>& v = b->host_args;
  v.resize(b->grains.size());
  for (size_t gi = 0; gi < b->grains.size(); ++gi) {
    qc_grain* g = b->grains[gi];
    int G, epl;
    lane_shape(g->n_poles, b->epl, g->precision == QC_MIXED, G, epl);
    qc::SweepArgs a = sweep_args(g, g->n_poles, g->n_poles, 0, g->eps, g->rpd, true);
    a.G = G;
    a.log2g = ilog2(G);
    a.bc_valid = g->bc_valid;
    v[gi].a = a;
    v[gi].b.nodes = g->nodes;
    v[gi].b.bc_g_prev = g->bc[g->bc_cur][0];
    v[gi].b.bc_gt_prev = g->bc[g->bc_cur][1];
    v[gi].b.bc_g_next = g->bc[1 - g->bc_cur][0];
    v[gi].b.bc_gt_next = g->bc[1 - g->bc_cur][1];
    v[gi].b.gbuf = g->gbuf;
    v[gi].b.ebuf = nullptr;
  }
  hcheck(hipMemcpyAsync(b->d_args, v.data(), sizeof(qc::BatchGrainDev) * v.size(), hipMemcpyHostToDevice, st),
         "H2D");
  hcheck(hipStreamSynchronize(st), "sync");  // the host block is reused by the next upload
}

void rotate_back_grain(qc_grain* g, const double* delta, double* dnew, double* j, hipStream_t st) {
  qc::launch_rotate_back(back_args(g, delta, dnew, j, nullptr), st);
}

// one Picard iteration (alpha = 1) of every grain: per-grain interpolation,
// one persistent sweep over all grains, per-grain rotate-back, A-solve and
// update.  Only kernel launches: it can be captured into a graph.
void batch_iteration(qc_batch* b, hipStream_t st, bool upload) {
  for (size_t gi = 0; gi < b->grains.size(); ++gi) do_interp(b->grains[gi], b->delta[gi], b->A[gi], st, true);
  if (upload) upload_args(b, st);
  for (size_t k = 0; k < b->grp_epl.size(); ++k) {
    if (b->precision == QC_MIXED)
      qc::launch_batch_sweep<float>(b->grp_epl[k], b->d_args, b->d_tiles + b->grp_off[k], b->grp_n[k],
                                    b->d_counter + k, b->nblocks, b->spill, b->wave_elems, st);
    else
      qc::launch_batch_sweep<double>(b->grp_epl[k], b->d_args, b->d_tiles + b->grp_off[k], b->grp_n[k],
                                     b->d_counter + k, b->nblocks, b->spill, b->wave_elems, st);
  }
  for (size_t gi = 0; gi < b->grains.size(); ++gi) {
    qc_grain* g = b->grains[gi];
    mirror_fill(g, g->bc[1 - g->bc_cur][0], g->bc[1 - g->bc_cur][1], st);
    rotate_back_grain(g, b->delta[gi], g->dnew, g->jcur, st);
    // A from the current (zero for an infinite penetration depth), as in the
    // single-grain Picard loop
    do_solve_A(g, g->jcur, g->anew, nullptr, st);
    qc::launch_picard(b->A[gi], g->anew, nullptr, 2 * g->ncell, 1, 0, 1, 1.0, st);
    qc::launch_picard(b->delta[gi], g->dnew, g->grain_cells, g->ncg, g->ncomp, g->ncell, 2, 1.0, st);
    g->bc_cur = 1 - g->bc_cur;
    g->bc_valid = 1;
    g->last_bc_valid = -1;  // batched sweeps are not differentiated
  }
  hcheck(hipGetLastError(), "batch launch");
}

void drop_graph(qc_batch* b) {
  if (b->gexec) (void)hipGraphExecDestroy(b->gexec);
  b->gexec = nullptr;
  b->graph_parity.clear();
}

void free_batch(qc_batch* b) {
  drop_graph(b);
  for (double* p : b->delta)
    if (p) (void)hipFree(p);
  for (double* p : b->A)
    if (p) (void)hipFree(p);
  if (b->d_args) (void)hipFree(b->d_args);
  if (b->d_tiles) (void)hipFree(b->d_tiles);
  if (b->d_counter) (void)hipFree(b->d_counter);
  if (b->spill) (void)hipFree(b->spill);
  if (b->own) (void)hipStreamDestroy(b->own);
  delete b;
}

}  // namespace

extern "C" {

qc_status qc_batch_create(qc_grain* const* grains, int n, qc_batch** out) {
  if (!out || !grains || n < 1) return fail(QC_ERR_INVALID, "need at least one grain");
  *out = nullptr;
  for (int i = 0; i < n; ++i) {
    if (!grains[i]) return fail(QC_ERR_INVALID, "NULL grain in the batch");
    if (grains[i]->device != grains[0]->device || grains[i]->precision != grains[0]->precision)
      return fail(QC_ERR_INVALID, "all grains of a batch need the same device and precision");
    if (grains[i]->n_poles > 512) return fail(QC_ERR_INVALID, "too many poles for a batched sweep");
    for (int k = 0; k < i; ++k)
      if (grains[k] == grains[i]) return fail(QC_ERR_INVALID, "a grain appears twice in the batch");
  }
  qc_batch* b = new (std::nothrow) qc_batch();
  if (!b) return fail(QC_ERR_OOM, "host allocation failed");
  qc_status st = guarded([&]() -> qc_status {
    b->device = grains[0]->device;
    b->precision = grains[0]->precision;
    hcheck(hipSetDevice(b->device), "hipSetDevice");
    hipDeviceProp_t prop;
    hcheck(hipGetDeviceProperties(&prop, b->device), "props");
    b->nblocks = prop.multiProcessorCount * 8;
    for (int i = 0; i < n; ++i) {
      qc_grain* g = grains[i];
      ensure_sweep_buffers(g, false);
      b->grains.push_back(g);
      b->steps_per_iter += g->info.steps_per_sweep;
      double* d = static_cast<double*>(dalloc(sizeof(double) * 2 * g->ncomp * g->ncell));
      double* a = static_cast<double*>(dalloc(sizeof(double) * 2 * g->ncell));
      b->delta.push_back(d);
      b->A.push_back(a);
      qc::launch_fill(d, 2 * g->ncomp * g->ncell, 0.0, nullptr);
      qc::launch_fill(a, 2 * g->ncell, 0.0, nullptr);
      // off-grain cells of delta_new stay zero: rotate-back writes grain cells only
      qc::launch_fill(g->dnew, 2 * g->ncomp * g->ncell, 0.0, nullptr);
    }
    b->d_args = static_cast<qc::BatchGrainDev*>(dalloc(sizeof(qc::BatchGrainDev) * n));
    b->d_counter = static_cast<int*>(dalloc(8 * sizeof(int)));
    hcheck(hipStreamCreate(&b->own), "stream");
    build_tiles(b);
    hcheck(hipDeviceSynchronize(), "batch setup");
    return QC_OK;
  });
  if (st != QC_OK) {
    free_batch(b);
    return st;
  }
  *out = b;
  return QC_OK;
}

void qc_batch_destroy(qc_batch* b) {
  if (!b) return;
  (void)hipSetDevice(b->device);
  (void)hipDeviceSynchronize();
  free_batch(b);
}

qc_status qc_batch_get_info(const qc_batch* b, int64_t* steps_per_iteration, int* energies_per_lane, int* n_tiles) {
  if (!b) return fail(QC_ERR_INVALID, "batch is NULL");
  if (steps_per_iteration) *steps_per_iteration = b->steps_per_iter;
  if (energies_per_lane) *energies_per_lane = b->epl;
  if (n_tiles) *n_tiles = b->ntiles;
  return QC_OK;
}

qc_status qc_batch_set_fields(qc_batch* b, int i, const double* delta, const double* A_ind, void* stream) {
  if (!b || i < 0 || i >= static_cast<int>(b->grains.size())) return fail(QC_ERR_INVALID, "bad batch index");
  if (!delta || !A_ind) return fail(QC_ERR_INVALID, "NULL field");
  return guarded([&]() -> qc_status {
    qc_grain* g = b->grains[i];
    hcheck(hipSetDevice(b->device), "hipSetDevice");
    hcheck(hipMemcpyAsync(g->dnew, delta, sizeof(double) * 2 * g->ncomp * g->ncell, hipMemcpyDeviceToDevice, S(stream)),
           "copy");
    qc::launch_fill(b->delta[i], 2 * g->ncomp * g->ncell, 0.0, S(stream));
    qc::launch_picard(b->delta[i], g->dnew, g->grain_cells, g->ncg, g->ncomp, g->ncell, 2, 1.0, S(stream));
    qc::launch_fill(g->dnew, 2 * g->ncomp * g->ncell, 0.0, S(stream));
    // no screening (kappa <= 0): no induced vector potential, A stays zero
    if (g->kappa <= 0.0)
      qc::launch_fill(b->A[i], 2 * g->ncell, 0.0, S(stream));
    else
      hcheck(hipMemcpyAsync(b->A[i], A_ind, sizeof(double) * 2 * g->ncell, hipMemcpyDeviceToDevice, S(stream)),
             "copy");
    return QC_OK;
  });
}

qc_status qc_batch_get_fields(const qc_batch* b, int i, double* delta_out, double* A_out, void* stream) {
  if (!b || i < 0 || i >= static_cast<int>(b->grains.size())) return fail(QC_ERR_INVALID, "bad batch index");
  return guarded([&]() -> qc_status {
    qc_grain* g = b->grains[i];
    hcheck(hipSetDevice(b->device), "hipSetDevice");
    if (delta_out)
      hcheck(hipMemcpyAsync(delta_out, b->delta[i], sizeof(double) * 2 * g->ncomp * g->ncell, hipMemcpyDeviceToDevice,
                            S(stream)),
             "copy");
    if (A_out)
      hcheck(hipMemcpyAsync(A_out, b->A[i], sizeof(double) * 2 * g->ncell, hipMemcpyDeviceToDevice, S(stream)), "copy");
    return QC_OK;
  });
}

qc_status qc_batch_iterate(qc_batch* b, int n_iter, int use_graph, void* stream) {
  if (!b || n_iter < 0) return fail(QC_ERR_INVALID, "bad arguments");
  return guarded([&]() -> qc_status {
    hcheck(hipSetDevice(b->device), "hipSetDevice");
    hipStream_t st = stream ? S(stream) : b->own;
    hipEvent_t e0, e1;
    hcheck(hipEventCreate(&e0), "event");
    hcheck(hipEventCreate(&e1), "event");
    hcheck(hipEventRecord(e0, st), "event");
    int left = n_iter;
    // the first sweep of a fresh grain starts from bulk roots: run it eagerly
    bool fresh = false;
    for (qc_grain* g : b->grains) fresh = fresh || !g->bc_valid;
    if (fresh && left > 0) {
      batch_iteration(b, st, true);
      --left;
    }
    if (use_graph && left >= 2) {
      std::vector<int> par;
      for (qc_grain* g : b->grains) par.push_back(g->bc_cur);
      if (!b->gexec || par != b->graph_parity || b->graph_epl != b->epl) {
        drop_graph(b);
        // the graph holds two iterations (both store parities); the argument
        // blocks are baked per parity into two device copies
        hcheck(hipStreamSynchronize(st), "sync");
        qc::BatchGrainDev* saved = b->d_args;
        qc::BatchGrainDev* args2 =
            static_cast<qc::BatchGrainDev*>(dalloc(sizeof(qc::BatchGrainDev) * 2 * b->grains.size()));
        b->d_args = args2;
        upload_args(b, st);
        for (qc_grain* g : b->grains) g->bc_cur = 1 - g->bc_cur;
        b->d_args = args2 + b->grains.size();
        upload_args(b, st);
        for (qc_grain* g : b->grains) g->bc_cur = 1 - g->bc_cur;
        hcheck(hipStreamSynchronize(st), "sync");
        hipStream_t cs;
        hcheck(hipStreamCreate(&cs), "stream");
        hipGraph_t graph;
        hcheck(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "capture");
        b->d_args = args2;
        batch_iteration(b, cs, false);
        b->d_args = args2 + b->grains.size();
        batch_iteration(b, cs, false);
        hcheck(hipStreamEndCapture(cs, &graph), "capture");
        // the capture flipped the parities twice: back where it started
        hcheck(hipGraphInstantiate(&b->gexec, graph, nullptr, nullptr, 0), "instantiate");
        (void)hipGraphDestroy(graph);
        (void)hipStreamDestroy(cs);
        if (saved) (void)hipFree(saved);
        b->d_args = args2;  // kept alive for the graph (first half; second half follows)
        b->graph_parity = par;
        b->graph_epl = b->epl;
      }
      while (left >= 2) {
        hcheck(hipGraphLaunch(b->gexec, st), "graph launch");
        left -= 2;
      }
    }
    while (left > 0) {
      if (b->gexec) {
        // eager iterations must not overwrite the graph's argument blocks
        drop_graph(b);
        (void)hipFree(b->d_args);
        b->d_args = static_cast<qc::BatchGrainDev*>(dalloc(sizeof(qc::BatchGrainDev) * b->grains.size()));
      }
      batch_iteration(b, st, true);
      --left;
    }
    hcheck(hipEventRecord(e1, st), "event");
    hcheck(hipEventSynchronize(e1), "event");
    float ms = 0.f;
    hcheck(hipEventElapsedTime(&ms, e0, e1), "event");
    b->last_ms = ms;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return QC_OK;
  });
}

qc_status qc_batch_last_ms(const qc_batch* b, double* ms) {
  if (!b || !ms) return fail(QC_ERR_INVALID, "NULL argument");
  *ms = b->last_ms;
  return QC_OK;
}

qc_status qc_batch_autotune(qc_batch* b, int iters_per_trial, int* best_epl, void* stream) {
  if (!b || iters_per_trial < 1) return fail(QC_ERR_INVALID, "bad arguments");
  int maxp = 0;
  for (qc_grain* g : b->grains) maxp = std::max(maxp, g->n_poles);
  double best = INFINITY;
  int arg = b->epl;
  // 0: every grain its own automatic lane shape (one launch per shape)
  const int cand[6] = {0, 1, 2, 3, 4, 8};
  for (int e : cand) {
    if (e > 0 && (maxp + e - 1) / e > 64) continue;
    b->epl = e;
    qc_status st = guarded([&]() -> qc_status {
      drop_graph(b);
      build_tiles(b);
      return QC_OK;
    });
    if (st != QC_OK) return st;
    st = qc_batch_iterate(b, iters_per_trial, 0, stream);
    if (st != QC_OK) return st;
    if (b->last_ms < best) {
      best = b->last_ms;
      arg = e;
    }
  }
  b->epl = arg;
  qc_status st = guarded([&]() -> qc_status {
    build_tiles(b);
    return QC_OK;
  });
  if (best_epl) *best_epl = arg;
  return st;
}

}  // extern "C"
