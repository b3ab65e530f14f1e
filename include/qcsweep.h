/*
 * qcsweep: Riccati-sweep library for ballistic quasiclassical (Eilenberger)
 * theory of 2D singlet superconducting grains, for AMD MI355X (gfx950).
 *
 * The method (arXiv:2205.15000): for every Fermi-surface angle phi_k and
 * every Ozaki pole (or real energy), the coherence functions gamma and
 * gamma~ are integrated with the implicit midpoint rule (App. C) along the
 * lines of a square lattice rotated so that one axis is parallel to the
 * Fermi velocity (Sec. III.A); Delta(R) and A(R) are interpolated onto the
 * lattice bilinearly; the Green's functions of the Riccati parametrisation
 * (Sec. II.A) are summed over energies, rotated back to the reference grid
 * and averaged over angles into the gap update (Eq. gapeq_fixpoint), the
 * current (Eq. current_density) and the Eilenberger free energy (Sec. II);
 * between iterations the induced vector potential is re-solved with the
 * cell-averaged Green's function of the 2D Laplacian (App. D).
 *
 * Units (App. F): lengths in xi0, energies in 2 pi k_B Tc, t = T/Tc,
 * A in Phi0/(pi xi0), B in Phi0/(pi xi0^2), j in 2 pi k_B Tc |e| v_F N_F,
 * free-energy density in (2 pi k_B Tc)^2 N_F per xi0^2.
 *
 * Layout: grid fields are row-major [..][ny][nx] with x fastest; cell (i,j)
 * has its centre at (x0 + (i+1/2) h, y0 + (j+1/2) h).  Complex values are
 * interleaved (re, im) doubles.
 *
 * Ownership: the caller owns every array argument.  Arguments of compute
 * calls (qc_sweep, qc_solve_A, qc_scf_run, qc_ldos, qc_get_state,
 * qc_set_state) that hold grid fields are DEVICE pointers on the grain's
 * device (e.g. torch tensors' data_ptr); scalar outputs and small tables
 * are host pointers, as stated per argument.  The library owns the
 * handles and everything they hold; *_destroy frees it.
 *
 * Errors: no exception crosses this interface.  Status codes >= 0 are
 * success (QC_NOT_CONVERGED is informational), < 0 are errors; the
 * message of the last error on the calling thread is qc_last_error().
 * Every argument is checked on the host before anything is launched.
 *
 * Streams: `stream` is a hipStream_t (NULL = the default stream).  Calls
 * return after enqueueing unless they return host scalars, in which case
 * they synchronise the stream.  Calls on one grain must not overlap.
 */
#ifndef QCSWEEP_H
#define QCSWEEP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  QC_OK = 0,
  QC_NOT_CONVERGED = 1,   /* scf: max_iter reached above the tolerance */
  QC_ERR_INVALID = -1,    /* bad argument; see qc_last_error() */
  QC_ERR_NO_DEVICE = -2,  /* no usable gfx950 device */
  QC_ERR_OOM = -3,        /* device or host allocation failed */
  QC_ERR_HIP = -4,        /* a HIP runtime call failed */
  QC_ERR_NAN = -5         /* a residual became NaN or Inf */
} qc_status;

typedef enum { QC_FP64 = 0, QC_MIXED = 1 } qc_precision;
/* QC_MIXED: interpolated node values, the Riccati marches, the Green's
 * functions and each lane's sum over its few poles (2 or 3) in complex FP32;
 * the energy sums across lanes, angle sums, gap denominator, free energy,
 * A-solve and residuals in FP64.  The interface is FP64 either way. */

typedef enum {
  QC_SHAPE_DISC = 0,             /* cx, cy, radius */
  QC_SHAPE_REGULAR_POLYGON = 1,  /* cx, cy, n_edges, side, rotation (turns) */
  QC_SHAPE_POLYGON = 2,          /* convex, vertices vx/vy counter-clockwise */
  QC_SHAPE_MASK = 3              /* cells given by mask (grid of the descriptor) */
} qc_shape_kind;

typedef enum {
  QC_GAUGE_SYMMETRIC = 0,  /* A = B/2 (-(y-cy), x-cx), B = pi*flux/area */
  QC_GAUGE_LANDAU = 1,     /* A = (-B (y-cy), 0) */
  QC_GAUGE_SOLENOID = 2    /* A = flux/(2 r) along phi-hat */
} qc_gauge;

/* One geometry component (App. B).  Components are combined in order:
 * add != 0 unites it with the grain, add == 0 removes it.  Points on a
 * boundary count as inside.  A regular polygon with rotation 0 has a
 * horizontal bottom edge.  A mask component takes mask[ny][nx] (nonzero =
 * the cell centre is inside) on the descriptor's grid; its exact boundary
 * is the marching-squares contour of the mask at level 1/2 over the cell
 * centres (cells beyond the array outside; a square with only two diagonal
 * corners inside keeps them apart), and inside is the even-odd rule of
 * that contour, so the cell centres inside are exactly the mask's.
 * vx/vy/mask are host pointers read during the call. */
typedef struct {
  int kind;
  int add;
  double cx, cy;
  double radius;
  int n_edges;
  double side;
  double rotation;
  const double* vx;
  const double* vy;
  int nv;
  const uint8_t* mask;
} qc_shape;

/* Grain description.  All pointers are host pointers read during the call.
 *   nx, ny, h, x0, y0  reference grid (Sec. III.A)
 *   n_theta            Fermi-surface angles phi_k = 2 pi k / n_theta with
 *                      Boole / Simpson 3/8 / Simpson 1/3 / trapezoid
 *                      weights when divisible by 4 / 3 / 2 / otherwise
 *   n_poles            positive Ozaki poles of the energy sums (Sec. III.A)
 *   t                  T/Tc, 0 < t
 *   ncomp, tc_rel      order-parameter components and their T_c,G / Tc
 *   eta                complex [ncomp][n_theta] basis values eta_G(phi_k),
 *                      or NULL: then basis[ncomp] (qc_basis) names each
 *                      component's App. F function and the library
 *                      tabulates eta_G(phi_k) = f_G(phi_k - 2 pi
 *                      crystal_rotation) (rotation in full turns, App. B)
 *   kappa              penetration depth / xi0; <= 0 means infinite (A_ind=0)
 *   flux_quanta, gauge external field (App. B, App. F)
 *   charge_sign        +1 or -1 (sign of the carrier charge; -1 electrons)
 *   precision          qc_precision
 */
/* Basis functions of App. F (circular Fermi surface), phi measured from the
 * crystal a-axis: s = 1, d_{x2-y2} = sqrt2 cos 2 phi, d_xy = sqrt2 sin 2 phi,
 * g_{xy(x2-y2)} = sqrt2 sin 4 phi. */
typedef enum { QC_BASIS_S = 0, QC_BASIS_DX2Y2 = 1, QC_BASIS_DXY = 2, QC_BASIS_G = 3 } qc_basis;

typedef struct {
  int nx, ny;
  double h;
  double x0, y0;
  const qc_shape* shapes;
  int n_shapes;
  int n_theta;
  int n_poles;
  double t;
  int ncomp;
  const double* tc_rel;
  const double* eta;
  double kappa;
  double flux_quanta;
  int gauge;
  int charge_sign;
  int precision;
  const int* basis;
  double crystal_rotation;
} qc_grain_desc;

typedef struct qc_plan qc_plan;    /* host-side trajectory tables */
typedef struct qc_grain qc_grain;  /* a plan resident on one device */

typedef struct {
  int64_t n_segments;       /* trajectory segments over all angles */
  int64_t n_slots;          /* interior lattice nodes + one midpoint slot per
                               segment without interior node */
  int64_t n_nodes;          /* interior lattice nodes over all angles */
  int64_t n_grain_cells;    /* reference cells inside the grain */
  int64_t steps_per_sweep;  /* 2 * n_poles * sum over segments of (n + 1) */
  int lattice_m;            /* side of the rotated lattice */
  double area;              /* h^2 * n_grain_cells, xi0^2 */
} qc_plan_info;

/* ---- library ---------------------------------------------------------- */
/* Message of the last error on this thread ("" if none). */
const char* qc_last_error(void);
/* Interface version, 1 for this header. */
int qc_version(void);
/* Number of visible HIP devices (0 without a GPU; never an error). */
qc_status qc_device_count(int* n_out);

/* ---- host plan (no device needed) --------------------------------------
 * Builds the trajectory tables of Sec. III.A on the host: grain mask,
 * per-angle segments of the rotated lattice lines inside the grain with
 * their exact end points (Fig. 2), interpolation stencils of Delta and
 * A_ind at the lattice nodes, rotate-back stencils of the grain cells,
 * specular boundary-condition taps (Sec. III.A: interpolation in angle and
 * boundary coordinate), the Ozaki poles and the Fermi-surface weights. */
qc_status qc_plan_create(const qc_grain_desc* desc, qc_plan** out);
void qc_plan_destroy(qc_plan* plan);
qc_status qc_plan_get_info(const qc_plan* plan, qc_plan_info* out);
/* mask_out: host uint8 [ny][nx], 1 on grain cells. */
qc_status qc_plan_get_mask(const qc_plan* plan, uint8_t* mask_out);
/* out: host double [n_segments][8] = angle, line, s_min, s_max, first node
 * index, interior node count, wall tangent angle at s_min, at s_max. */
qc_status qc_plan_get_segments(const qc_plan* plan, double* out);
/* Start-value taps of every segment: for gamma at s_min (at_start=1) or
 * gamma~ at s_max (at_start=0).  seg_out: host int32 [n_segments][4]
 * global segment indices, w_out: host double [n_segments][4] weights that
 * sum to one; a row of zero weights means the bulk root is used. */
qc_status qc_plan_get_taps(const qc_plan* plan, int at_start, int32_t* seg_out, double* w_out);
/* z_out, r_out: host double [n_poles] Ozaki poles and residues. */
qc_status qc_plan_get_poles(const qc_plan* plan, double* z_out, double* r_out);
/* basis values eta_G(phi_k) the plan uses: host complex [ncomp][n_theta] */
qc_status qc_plan_get_eta(const qc_plan* plan, double* eta_out);
/* grain cells of a device grain: host uint8 [ny][nx], 1 inside */
qc_status qc_grain_get_mask(const qc_grain* grain, uint8_t* mask_out);
/* Angle pairs of the plan (see qc_grain_set_pairing): whether the tables of
 * phi_k and phi_k + pi mirror each other (*available: 0 no; 1 yes; 3 yes,
 * and every grain cell also has the same four rotate-back corners on both
 * angles, so the paired rotate-back gathers the node sums once per pair),
 * the trajectory steps a paired Matsubara sweep marches, and (optional,
 * host int32 [n_segments]) the mirror segment on phi_k - pi of every
 * segment of an angle phi_k >= pi (-1 for the others and when
 * unavailable). */
qc_status qc_plan_get_pairing(const qc_plan* plan, int* available, int64_t* swept_steps_per_sweep,
                              int32_t* seg_mirror_out);

/* ---- device grain -------------------------------------------------------- */
/* Builds the plan and uploads it to `device`.  The boundary-value store
 * starts empty: the first sweep starts every trajectory at the bulk root of
 * its end values. */
qc_status qc_grain_create(int device, const qc_grain_desc* desc, qc_grain** out);
void qc_grain_destroy(qc_grain* grain);
qc_status qc_grain_get_info(const qc_grain* grain, qc_plan_info* out);
/* Forget the boundary values: the next sweep starts from bulk roots. */
qc_status qc_grain_reset_bc(qc_grain* grain);

/* One iteration map (loop body of Alg. 1) with Delta and A_ind given:
 * interpolate onto the rotated lattices, march gamma and gamma~ for every
 * angle and positive pole, sum g, f, f~ over poles per node, rotate back,
 * accumulate over angles; then Delta_new (Eq. gapeq_fixpoint), j
 * (Eq. current_density) and the Eilenberger free-energy density.
 *   delta       device complex [ncomp][ny][nx] (values off-grain ignored)
 *   A_ind       device double [2][ny][nx] induced vector potential
 *   delta_new   device complex [ncomp][ny][nx] (0 off-grain)
 *   j           device double [2][ny][nx] (0 off-grain)
 *   omega_density device double [ny][nx] condensation part (0 off-grain);
 *               may be NULL
 *   omega_total host double: h^2 sum omega + h^2 sum (kappa^2/2)|curl A_ind|^2;
 *               may be NULL (then the call does not synchronise)
 * Start values come from the boundary-value store (specular taps of the
 * previous sweep's end values, Jacobi update as in Alg. 1); the store is
 * then replaced by this sweep's end values. */
qc_status qc_sweep(qc_grain* grain, const double* delta, const double* A_ind,
                   double* delta_new, double* j, double* omega_density,
                   double* omega_total, void* stream);

/* qc_sweep without allocation, for callers that cannot allocate device
 * memory (code under stream or graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same map, arguments and results as
 * qc_sweep; the per-call work arrays (slot values, the gamma spill between
 * the two marches, per-node sums, packed interpolation cells) live in one
 * 64 MiB array that the library holds on each device it runs on until the
 * process ends, instead of grain-owned allocations.  Calls on one device
 * share that array, so calls that overlap on one GPU race; nothing in it
 * needs clearing between calls (every element a call reads it wrote
 * first).  Needs a grain whose boundary store exists (any earlier qc_sweep
 * or qc_set_state creates it).  Errors: QC_ERR_INVALID when the grain needs
 * more scratch than the array holds (qc_sweep_static_bytes tells) or has no
 * boundary store yet. */
qc_status qc_sweep_static(qc_grain* grain, const double* delta, const double* A_ind,
                          double* delta_new, double* j, double* omega_density,
                          double* omega_total, void* stream);
/* scratch bytes qc_sweep_static needs for this grain and the size of the
 * per-device array; either pointer may be NULL. */
qc_status qc_sweep_static_bytes(const qc_grain* grain, size_t* needed, size_t* available);

/* Induced vector potential from a current (App. D): the grain mean of j is
 * subtracted on grain cells, then A = -kappa^-2 sum G_{|dm|,|dn|} j' over the
 * whole array (zero-padded FFT correlation), B = curl A with central
 * differences (one-sided at the array edge).
 *   j      device double [2][ny][nx]
 *   A_out  device double [2][ny][nx]
 *   B_out  device double [ny][nx], may be NULL
 * With kappa <= 0 both outputs are zero. */
qc_status qc_solve_A(qc_grain* grain, const double* j, double* A_out, double* B_out, void* stream);

/* A-solve with the separable, eigen-truncated kernel of App. D on a square
 * grid: G_{m,n} = sum_k lambda_k V_m^(k) V_n^(k) (eigen-decomposition of
 * the N x N matrix G, done once on the host by Householder reduction and
 * implicit QR), kept to the N* modes of largest |lambda| with N* the
 * smallest count whose dropped remainder has
 * sqrt(sum_dropped lambda^2 / sum_all lambda^2) < eps (the App. D
 * criterion, summed over the dropped modes).  Then every A-solve of the
 * grain (qc_solve_A, qc_scf_run, batches) computes
 *   A = -kappa^-2 sum_k lambda_k T_k J' T_k,  T_k[a][b] = V^(k)_{|a-b|},
 * as two FP64 matrix-core contractions per component (J' the current minus
 * its grain mean on grain cells).  eps = 0 restores the exact zero-padded
 * FFT correlation (the default).  Device memory: 2 (N* + 1) N^2 doubles.
 * Errors: QC_ERR_INVALID for eps < 0 or, with eps > 0, nx != ny. */
qc_status qc_grain_set_A_solver(qc_grain* grain, double eps);
/* the tolerance set and the modes kept (0 for the FFT solve); either
 * pointer may be NULL. */
qc_status qc_grain_get_A_solver(const qc_grain* grain, double* eps, int* n_modes);

/* Magnetic moment of the in-plane current (Sec. V.A,
 * Eq. magnetic_moment_def) along z, per unit thickness, in units of
 * m0 = j0 xi0 V (V = thickness x grain area):
 *   m_z / m0 = (1 / 2A) h^2 sum over grain cells of (x - c_x) j_y - (y - c_y) j_x,
 * about the grid centre (c_x, c_y), A = h^2 x (grain cells).
 *   j     device double [2][ny][nx]
 *   m_out host double
 * Synchronises the stream. */
qc_status qc_magnetic_moment(qc_grain* grain, const double* j, double* m_out, void* stream);

/* Luttinger-Ward form of the free energy (Sec. II, Eqs. qcLWFE and
 * qcLWFE_I), the check on the Eilenberger form that qc_sweep returns: per
 * grain cell
 *   omega = sum_G |Delta_G|^2 ln(t/t_c,G) + 2 pi sum_p (R_p/z_p) <|Delta(p)|^2>
 *           - int_0^1 dlambda 2 sum_G den_G Re[conj(Delta_G) Delta_new,G[lambda Delta]],
 * where Delta_new[lambda Delta] is the gap update (Eq. gapeq_fixpoint) of one
 * sweep with the scaled gap lambda Delta (A unscaled) and den_G its
 * denominator: with f(-e) = f~(e)*, T sum_n <Delta* f + Delta f~> over both
 * signs of the energies equals that expression.  The lambda integral is
 * the n_lambda-point Gauss-Legendre rule on [0, 1]; for every lambda the
 * boundary values start from bulk roots and take bc_iters burn-in sweeps
 * (App. B) before the sweep that is used.  The total adds
 * h^2 sum (kappa^2/2) |B_ind|^2 as the Eilenberger form does.  Costs
 * n_lambda (bc_iters + 1) sweeps.  The grain's boundary store is restored
 * before the call returns.
 *   delta          device complex [ncomp][ny][nx]
 *   A_ind          device double [2][ny][nx]
 *   omega_density  device double [ny][nx] (zero off the grain), may be NULL
 *   omega_total    host double
 * Errors: QC_ERR_INVALID unless 1 <= n_lambda <= 64 and bc_iters >= 0. */
qc_status qc_free_energy_lw(qc_grain* grain, const double* delta, const double* A_ind, int n_lambda,
                            int bc_iters, double* omega_density, double* omega_total, void* stream);

/* Picard self-consistency (App. E) on x = (Re Delta_G, Im Delta_G on grain
 * cells, kappa^2 A_ind): x <- x + alpha (g(x) - x), A from the current of
 * the same iteration.  The first `burnin` iterations keep Delta and A fixed
 * and only update boundary values (App. B).  Stops when every global error
 * (Eq. global_error with norm_p in {1, 2, 0 = infinity}) of Delta, j, A and
 * the free energy is below tol, after at least min_iter iterations, or at
 * max_iter.  The errors of Delta and A are those of d = g(x) - x relative to
 * x, taken after the A-solve and before the accelerator moves x (Alg. 1);
 * those of j and the free energy compare with the previous iteration.
 * With kappa <= 0 (no screening) A_io is set to zero and stays zero.
 *   delta_io   device complex [ncomp][ny][nx], in: start, out: final
 *   A_io       device double [2][ny][nx], in: start, out: final
 *   iters_done host int
 *   residuals_out host double [max_iter][5]: eps_Delta, eps_j, eps_A,
 *              eps_Omega, Omega_total per iteration; may be NULL
 * Returns QC_OK on convergence, QC_NOT_CONVERGED at max_iter. */
qc_status qc_scf_run(qc_grain* grain, double* delta_io, double* A_io, int max_iter,
                     int min_iter, int burnin, double tol, int norm_p, double alpha,
                     int* iters_done, double* residuals_out, void* stream);

/* Accelerator of qc_scf_run (App. E) on the concatenated x = (Re Delta,
 * Im Delta on grain cells, kappa^2 A; kappa^2 read as 1 when kappa <= 0):
 *   kind 0: Picard, x <- x + alpha d with d = g(x) - x (the default);
 *   kind 1: Polyak's heavy ball, v <- (1 - beta) v + alpha d, x <- x + v,
 *           with drag beta in (0, 1] and v = 0 at the start of every run;
 *   kind 2: Barzilai-Borwein, x <- x + a_i d_i with a_0 = alpha and, for
 *           accelerated iteration i >= 1 of the run, a_i = a_{i-1} s_i:
 *           s_i = |d_{i-1}|^2 / |d_{i-1}.(d_i - d_{i-1})| for odd i,
 *           |d_{i-1}.(d_i - d_{i-1})| / |d_i - d_{i-1}|^2 for even i,
 *           a_i clamped to [1e-3, 1e2]; a zero denominator keeps a_{i-1}.
 *           beta is ignored;
 *   kind 3: CongAcc, per component c of x (Re and Im of each Delta
 *           component, A_x, A_y): s = cosine similarity of the moving
 *           average m_c with d_c, a_c <- a_c 1.234^s clamped to [1e-3, 1e2],
 *           the weight w_c kept while s >= 0.7 and otherwise set by
 *           bisection so that w m + (1 - w) d has similarity 0.7 with d,
 *           m_c <- w_c m_c + (1 - w_c) d_c, x_c <- x_c + a_c m_c.  The first
 *           iteration takes w = 0 and a_c = alpha; a similarity with a zero
 *           vector counts as 0.  Anti-parallel m_c and d_c (s <= -1 + 1e-9)
 *           leave no weight with similarity 0.7 (the blend is a multiple of
 *           d_c that flips sign where it vanishes): then w_c = 0, so the
 *           average restarts from d_c.  Needs norm_p = 2 (QC_ERR_INVALID
 *           otherwise).  beta is ignored.
 * alpha is qc_scf_run's argument.  Picard and Polyak are linear in x, so the
 * kappa^2 scale of A drops out of them; it enters BB's dot products.
 * Polyak, BB and CongAcc keep two
 * device arrays of the sizes of Delta and A, allocated at their first run.
 * Errors: QC_ERR_INVALID for an unknown kind or a Polyak drag outside (0, 1]. */
qc_status qc_grain_set_accelerator(qc_grain* grain, int kind, double beta);

/* Angle pairs.  For an order parameter even in the momentum direction
 * (singlet pairing: every basis function of App. F), gamma~ along a
 * trajectory is the complex conjugate of gamma along the reversed one
 * (Sec. II.A: gamma~(p, e_n) = gamma(-p, e_n)*), and the rotated lattice of
 * angle phi_k + pi is that of phi_k with both axes reversed (Sec. III.A).
 * So the Matsubara sweeps of qc_sweep, qc_scf_run, qc_free_energy_lw and the
 * batch march the angles phi_k < pi only: the node sums of phi_k + pi are
 * those of the mirror node (S_f and S_I equal, S_g of opposite sign) and
 * its end values the conjugates of the mirror segment's (stored, so the
 * boundary store stays complete for every reader).  The result is the
 * same map up to rounding, at half the marches.  Available when n_theta is
 * even, the quadrature weights and basis values of phi_k and phi_k + pi
 * agree, and the planner's tables of the two angles mirror each other
 * exactly (same segments, node counts, slot positions within 1e-9 h and
 * fallback cells); enabled by default when available.  The reverse mode
 * marches the lower angles as the sweep does; qc_ldos does so when its
 * energies are symmetric about zero (the reversed direction at e mirrors
 * energy -e): in its boundary iterations, and in its output pass where the
 * pairs share their rotate-back corners (available = 3 below); the
 * converging LDOS and the Green's function average march every angle.  Set
 * it before qc_batch_create for grains of a batch.
 * Errors: QC_ERR_INVALID when enabling on a grain where it is unavailable. */
qc_status qc_grain_set_pairing(qc_grain* grain, int enable);
/* available / enabled flags and the trajectory steps one Matsubara sweep
 * marches (steps_per_sweep of qc_plan_info counts every angle); any output
 * pointer may be NULL.  *available is 3 when, beyond the pairs, every grain
 * cell has the same rotate-back corners on both angles of a pair (see
 * qc_plan_get_pairing), 1 with pairs alone, 0 without. */
qc_status qc_grain_get_pairing(const qc_grain* grain, int* available, int* enabled, int64_t* swept_steps_per_sweep);

/* Counts, over the grain's lifetime, of the CongAcc weights that were set by
 * bisection and by the anti-parallel rule (see qc_grain_set_accelerator).
 * Either pointer may be NULL.  Errors: QC_ERR_INVALID for a NULL grain. */
qc_status qc_grain_get_accel_stats(const qc_grain* grain, int64_t* bisected, int64_t* anti_parallel);

/* Local density of states N(R, e)/N_F = < -Im g^R / pi > (Sec. II) at the
 * real energies e + i*broadening, Delta and A frozen: bc_iters sweeps update
 * only the boundary values (burn-in, App. B), then one sweep produces the
 * output.  The boundary store used starts from bulk roots and is separate
 * from the one of qc_sweep.  With angle pairs on and a set of energies
 * symmetric about zero (to 1e-12 of the largest |e|), the sweeps march half
 * the angles (see qc_grain_set_pairing); the energies may come in any
 * order, and ldos_out keeps the caller's order.
 *   energies host double [n_e]
 *   ldos_out device double [n_e][ny][nx] (0 off-grain) */
qc_status qc_ldos(qc_grain* grain, const double* delta, const double* A_ind,
                  const double* energies, int n_e, double broadening, int bc_iters,
                  double* ldos_out, void* stream);

/* The LDOS as qc_ldos, with the boundary iteration run to convergence (the
 * post-process of Sec. IV and App. B: burn-in until the LDOS settles):
 * every iteration is a full output sweep whose start values are the
 * previous sweep's end values (bulk roots at the first), and a block of
 * energies stops after the sweep whose LDOS changed by less than tol in
 * the relative 2-norm over all cells and the block's energies, or at
 * max_iter.  Energies are processed in blocks of energies_per_block (0:
 * the largest power of two up to 64 that fits half of the free device
 * memory); blocks converge independently (the boundary condition couples
 * angles, not energies).  The block that took the most sweeps gives
 * iters_out; with one block the result equals qc_ldos with
 * bc_iters = iters_out - 1.
 *   ldos_out device double [n_e][ny][nx]; iters_out host int, may be NULL
 * Errors: as qc_ldos, and QC_ERR_INVALID for max_iter < 1 or tol < 0. */
qc_status qc_ldos_converge(qc_grain* grain, const double* delta, const double* A_ind,
                           const double* energies, int n_e, double broadening, double tol,
                           int max_iter, int energies_per_block, int* iters_out,
                           double* ldos_out, void* stream);

/* Reverse mode of the most recent qc_sweep on this grain (the map with the
 * boundary store it read held fixed; start values that are bulk roots of
 * the segment-end values are differentiated).  No qc_sweep may run in
 * between.  QC_FP64 grains only.  For a real loss L with
 *   g_delta_new = dL/dRe Delta_new + i dL/dIm Delta_new  (device complex
 *                 [ncomp][ny][nx], NULL = 0),
 *   g_j         = dL/dj  (device [2][ny][nx], NULL = 0),
 *   g_omega     = dL/dOmega_total (host scalar),
 * writes grad_delta = dL/dRe Delta + i dL/dIm Delta (device complex
 * [ncomp][ny][nx]) and grad_A = dL/dA_ind (device [2][ny][nx]).
 * Derivatives of the implicit-midpoint step (App. C) follow from implicit
 * differentiation of its defining equation.  The transposes of the
 * interpolation and of the rotate-back are gathers over transposed tables
 * (built on the first call), so every output element is written once: no
 * atomics, and repeated calls give identical gradients.  Memory: by default
 * trajectory checkpoints every 32 slots plus a per-thread scratch; see
 * qc_grain_set_adjoint_checkpoint for the fully stored mode. */
qc_status qc_sweep_adjoint(qc_grain* grain, const double* delta, const double* A_ind, const double* g_delta_new,
                           const double* g_j, double g_omega, double* grad_delta, double* grad_A, void* stream);

/* ---- batched grains ----------------------------------------------------
 * Many grains of different shape, size, temperature, field, symmetry,
 * angle and pole counts iterated together: per iteration every grain's
 * interpolation runs, then one persistent sweep launch per lane shape in
 * use (usually one or two) in which each wave pulls tiles (a grain and a
 * bundle of 64/G of its segments) from a queue sorted by cost (longest
 * trajectories first), then every grain's
 * rotate-back, A-solve and Picard update (alpha = 1).  With use_graph the
 * iterations are replayed from a captured hipGraph (two iterations per
 * replay, one per boundary-store parity).  All grains must share device and
 * precision; each appears once; the batch keeps its own Delta and A per
 * grain and uses the grains' buffers (do not sweep them separately while
 * the batch is in use).  The gamma values between a tile's two marches live
 * in one scratch array with a slice per resident wave (reused tile after
 * tile), sized for the largest tile of the batch: the spill memory depends
 * on the longest trajectory and the pole count, not on the number of grains. */
typedef struct qc_batch qc_batch;
qc_status qc_batch_create(qc_grain* const* grains, int n, qc_batch** out);
void qc_batch_destroy(qc_batch* batch);
/* trajectory steps of one iteration over all grains; energies per lane
 * (0: each grain its own automatic choice, the default); number of tiles.
 * Any output pointer may be NULL. */
qc_status qc_batch_get_info(const qc_batch* batch, int64_t* steps_per_iteration, int* energies_per_lane,
                            int* n_tiles);
/* set / read grain i's fields: device complex [ncomp][ny][nx] and device
 * double [2][ny][nx] of that grain (copies; off-grain Delta set to zero;
 * a grain with kappa <= 0 stores A = 0, as qc_scf_run holds it). */
qc_status qc_batch_set_fields(qc_batch* batch, int i, const double* delta, const double* A_ind, void* stream);
qc_status qc_batch_get_fields(const qc_batch* batch, int i, double* delta_out, double* A_out, void* stream);
/* n_iter Picard iterations of every grain (stream NULL: the batch's own
 * stream); returns after they finish.  The first sweep of a grain that has
 * no boundary values yet runs eagerly (bulk starts). */
qc_status qc_batch_iterate(qc_batch* batch, int n_iter, int use_graph, void* stream);
/* wall time of the latest qc_batch_iterate (HIP events on its stream) */
qc_status qc_batch_last_ms(const qc_batch* batch, double* ms);
/* autotuner: times iters_per_trial real iterations for each feasible
 * energies-per-lane choice (0 = per grain, 1, 2, 3, 4, 8) and keeps the
 * fastest; these iterations advance the self-consistency like
 * qc_batch_iterate. */
qc_status qc_batch_autotune(qc_batch* batch, int iters_per_trial, int* best_epl, void* stream);

/* Fermi-surface average of the quasiclassical Green's function at the
 * positive poles of the energy sums (Sec. II.A: g = -i pi (1 - gamma
 * gamma~)/(1 + gamma gamma~) along each trajectory; rotate-back and angle
 * weights as for the gap, Sec. III.A): g_out = <g>(R, i eps~_p), complex
 * interleaved [n_poles][ny][nx] in pole order (ascending eps~_p), zero off
 * the grain.  delta, A_ind, g_out are device pointers as for qc_sweep.  The
 * start values are the ones the next qc_sweep would use (the boundary store
 * left by the latest sweep, bulk roots before the first); the store is not
 * changed.  Works in pole blocks with temporary device buffers (allocates
 * and frees; QC_ERR_OOM when they do not fit).  Synchronises the stream. */
qc_status qc_green_average(qc_grain* grain, const double* delta, const double* A_ind, double* g_out, void* stream);

/* Boundary-value store of qc_sweep (resume without burn-in, App. B).
 * bytes: in/out host size_t; with state == NULL only the size is returned.
 * state: device buffer of that size. */
qc_status qc_get_state(const qc_grain* grain, void* state, size_t* bytes, void* stream);
qc_status qc_set_state(qc_grain* grain, const void* state, size_t bytes, void* stream);

/* Memory mode of qc_sweep_adjoint.  every = C > 0 (default 32):
 * checkpoints every C slots of each trajectory (32 B per C nodes and pole)
 * plus a per-thread scratch of 2 C slots; each block is recomputed from its
 * checkpoint (three extra marches per node) with the same steps on the same
 * inputs.  every = 0: gamma~ and the node-local gamma~ adjoint are stored
 * at every (node, pole) instead (32 B in FP64).  Both modes give the same
 * gradients to rounding. */
qc_status qc_grain_set_adjoint_checkpoint(qc_grain* grain, int every);

/* Launch shape of the sweep kernel: energies handled by each lane (1, 2, 3,
 * 4 or 8; 0 = automatic: the fewest padded energy slots weighted by each
 * variant's measured cost).  The lanes of one trajectory segment share the
 * per-node energy sums, so fewer energies per lane means more lanes per
 * segment (a power of two up to 64; a forced value that would need more, or
 * that exceeds the number of energies of a launch, is replaced by the
 * automatic choice).  Results are identical up to rounding order. */
qc_status qc_grain_set_lanes(qc_grain* grain, int energies_per_lane);
/* The lane shape the next SCF sweep of this grain will use: energies per
 * lane (1, 2, 3, 4 or 8) and lanes per trajectory segment (a power of two
 * <= 64).  Both outputs are host ints written on success. */
qc_status qc_grain_get_lanes(const qc_grain* grain, int* energies_per_lane, int* lanes_per_segment);

/* Split launch shape of the SCF sweep (Matsubara poles).  Segments are
 * launched longest first.  When a launch fills the device's wave slots less
 * than twice, its longest segments set its length; with an even number of
 * energies per lane and twice the lanes still within 64, the segments longer
 * than frac x the longest then march with twice the lanes and half the
 * energies per lane (rounded up to whole waves).  frac in [0, 1]; 0 turns
 * the split off; the default is 0.8.  Results are identical up to the order
 * of the FP64 pole sums.  Errors: QC_ERR_INVALID for frac outside [0, 1]. */
qc_status qc_grain_set_split(qc_grain* grain, double frac);
/* The fraction set and the number of segments the next SCF sweep launches
 * with the wide shape (0 when the split does not apply); either pointer may
 * be NULL. */
qc_status qc_grain_get_split(qc_grain* grain, double* frac, int64_t* n_wide);

/* Kernel timing with HIP events on the launch stream (for roofline
 * reports).  Enable, run, then read the summed milliseconds and launch
 * count of the Riccati sweep kernel; reading resets the counters. */
qc_status qc_profile_enable(qc_grain* grain, int enable);
qc_status qc_profile_read(qc_grain* grain, double* sweep_ms, int64_t* sweep_launches);

/* Measurement aid for the roofline of the sweep kernels (not an operation
 * of the method): the sustained rate, in lane operations per second, of one
 * FP32 VALU operation on `device` with every CU busy (8 independent chains
 * per lane, 8 blocks of 256 lanes per CU, timed with HIP events after one
 * warm-up launch).  op: 0 fma, 1 rsq, 2 sqrt, 3 rcp.  Allocates and frees
 * its own small buffer; QC_ERR_NO_DEVICE without the device. */
qc_status qc_valu_rate(int device, int op, double* lane_ops_per_s);

#ifdef __cplusplus
}
#endif

#endif /* QCSWEEP_H */
