"""qcsweep: MI355X-native Riccati sweep for quasiclassical superconducting
grains (arXiv:2205.15000), Python binding of the C-ABI library.

This module only marshals arguments: every step of the method runs in the
HIP library libqcsweep.so (built with paper_2205_15000_amd.build).  PyTorch
supplies device memory and streams.  If the library has not been built the
import fails with an error; there is no CPU fallback.
"""
import ctypes
import math
import os

import numpy as np

__all__ = ["Grain", "Plan", "QcError", "lib", "spec_desc", "PRECISIONS", "sweep_autograd"]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libqcsweep.so")
if not os.path.exists(LIB_PATH):
    raise ImportError("libqcsweep.so is not built: run `python paper_2205_15000_amd/build.py` "
                      "(hipcc for gfx950) before importing paper_2205_15000_amd")
lib = ctypes.CDLL(LIB_PATH)

QC_OK, QC_NOT_CONVERGED = 0, 1
PRECISIONS = {"fp64": 0, "mixed": 1}
_SHAPES = {"disc": 0, "regular_polygon": 1, "polygon": 2, "mask": 3}
_GAUGES = {"symmetric": 0, "landau": 1, "solenoid": 2}
_BASIS = {"s": 0, "dx2y2": 1, "dxy": 2, "g": 3}


class QcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("qcsweep error %d: %s" % (status, msg))
        self.status = status


class _Shape(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int), ("add", ctypes.c_int), ("cx", ctypes.c_double),
                ("cy", ctypes.c_double), ("radius", ctypes.c_double), ("n_edges", ctypes.c_int),
                ("side", ctypes.c_double), ("rotation", ctypes.c_double),
                ("vx", ctypes.POINTER(ctypes.c_double)), ("vy", ctypes.POINTER(ctypes.c_double)),
                ("nv", ctypes.c_int), ("mask", ctypes.POINTER(ctypes.c_uint8))]


class _Desc(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int), ("ny", ctypes.c_int), ("h", ctypes.c_double),
                ("x0", ctypes.c_double), ("y0", ctypes.c_double),
                ("shapes", ctypes.POINTER(_Shape)), ("n_shapes", ctypes.c_int),
                ("n_theta", ctypes.c_int), ("n_poles", ctypes.c_int), ("t", ctypes.c_double),
                ("ncomp", ctypes.c_int), ("tc_rel", ctypes.POINTER(ctypes.c_double)),
                ("eta", ctypes.POINTER(ctypes.c_double)), ("kappa", ctypes.c_double),
                ("flux_quanta", ctypes.c_double), ("gauge", ctypes.c_int),
                ("charge_sign", ctypes.c_int), ("precision", ctypes.c_int),
                ("basis", ctypes.POINTER(ctypes.c_int)), ("crystal_rotation", ctypes.c_double)]


class _Info(ctypes.Structure):
    _fields_ = [("n_segments", ctypes.c_int64), ("n_slots", ctypes.c_int64),
                ("n_nodes", ctypes.c_int64), ("n_grain_cells", ctypes.c_int64),
                ("steps_per_sweep", ctypes.c_int64), ("lattice_m", ctypes.c_int),
                ("area", ctypes.c_double)]


_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)


def _sig(name, res, args):
    try:
        f = getattr(lib, name)
    except AttributeError as e:
        raise ImportError("libqcsweep.so is stale (missing %s): rebuild it with "
                          "`python paper_2205_15000_amd/build.py`" % name) from e
    f.restype = res
    f.argtypes = args
    return f


_sig("qc_last_error", ctypes.c_char_p, [])
_sig("qc_version", ctypes.c_int, [])
_sig("qc_device_count", ctypes.c_int, [ctypes.POINTER(ctypes.c_int)])
_sig("qc_valu_rate", ctypes.c_int, [ctypes.c_int, ctypes.c_int, ctypes.POINTER(ctypes.c_double)])
_sig("qc_plan_create", ctypes.c_int, [ctypes.POINTER(_Desc), ctypes.POINTER(_P)])
_sig("qc_plan_destroy", None, [_P])
_sig("qc_plan_get_info", ctypes.c_int, [_P, ctypes.POINTER(_Info)])
_sig("qc_plan_get_mask", ctypes.c_int, [_P, _P])
_sig("qc_plan_get_segments", ctypes.c_int, [_P, _P])
_sig("qc_plan_get_taps", ctypes.c_int, [_P, ctypes.c_int, _P, _P])
_sig("qc_plan_get_poles", ctypes.c_int, [_P, _P, _P])
_sig("qc_plan_get_eta", ctypes.c_int, [_P, _P])
_sig("qc_plan_get_pairing", ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int64), _P])
_sig("qc_grain_create", ctypes.c_int, [ctypes.c_int, ctypes.POINTER(_Desc), ctypes.POINTER(_P)])
_sig("qc_grain_destroy", None, [_P])
_sig("qc_grain_get_info", ctypes.c_int, [_P, ctypes.POINTER(_Info)])
_sig("qc_grain_get_mask", ctypes.c_int, [_P, _P])
_sig("qc_grain_reset_bc", ctypes.c_int, [_P])
_sig("qc_grain_get_lanes", ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)])
_sig("qc_sweep", ctypes.c_int, [_P, _P, _P, _P, _P, _P, _D, _P])
_sig("qc_sweep_static", ctypes.c_int, [_P, _P, _P, _P, _P, _P, _D, _P])
_sig("qc_sweep_static_bytes", ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_size_t), ctypes.POINTER(ctypes.c_size_t)])
_sig("qc_solve_A", ctypes.c_int, [_P, _P, _P, _P, _P])
_sig("qc_grain_set_A_solver", ctypes.c_int, [_P, ctypes.c_double])
_sig("qc_grain_get_A_solver", ctypes.c_int, [_P, _D, ctypes.POINTER(ctypes.c_int)])
_sig("qc_magnetic_moment", ctypes.c_int, [_P, _P, _D, _P])
_sig("qc_scf_run", ctypes.c_int, [_P, _P, _P, ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double,
                                   ctypes.c_int, ctypes.c_double, ctypes.POINTER(ctypes.c_int), _P, _P])
_sig("qc_ldos", ctypes.c_int, [_P, _P, _P, _P, ctypes.c_int, ctypes.c_double, ctypes.c_int, _P, _P])
_sig("qc_ldos_converge", ctypes.c_int, [_P, _P, _P, _P, ctypes.c_int, ctypes.c_double, ctypes.c_double, ctypes.c_int,
                                        ctypes.c_int, ctypes.POINTER(ctypes.c_int), _P, _P])
_sig("qc_sweep_adjoint", ctypes.c_int, [_P, _P, _P, _P, _P, ctypes.c_double, _P, _P, _P])
_sig("qc_green_average", ctypes.c_int, [_P, _P, _P, _P, _P])
_sig("qc_free_energy_lw", ctypes.c_int, [_P, _P, _P, ctypes.c_int, ctypes.c_int, _P, _D, _P])
_sig("qc_grain_set_adjoint_checkpoint", ctypes.c_int, [_P, ctypes.c_int])
_sig("qc_grain_set_accelerator", ctypes.c_int, [_P, ctypes.c_int, ctypes.c_double])
_sig("qc_grain_set_pairing", ctypes.c_int, [_P, ctypes.c_int])
_sig("qc_grain_get_pairing", ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int),
                                            ctypes.POINTER(ctypes.c_int64)])
_sig("qc_grain_get_accel_stats", ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64)])
_sig("qc_get_state", ctypes.c_int, [_P, _P, ctypes.POINTER(ctypes.c_size_t), _P])
_sig("qc_batch_create", ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int, ctypes.POINTER(_P)])
_sig("qc_batch_destroy", None, [_P])
_sig("qc_batch_get_info", ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int),
                                         ctypes.POINTER(ctypes.c_int)])
_sig("qc_batch_set_fields", ctypes.c_int, [_P, ctypes.c_int, _P, _P, _P])
_sig("qc_batch_get_fields", ctypes.c_int, [_P, ctypes.c_int, _P, _P, _P])
_sig("qc_batch_iterate", ctypes.c_int, [_P, ctypes.c_int, ctypes.c_int, _P])
_sig("qc_batch_last_ms", ctypes.c_int, [_P, _D])
_sig("qc_batch_autotune", ctypes.c_int, [_P, ctypes.c_int, ctypes.POINTER(ctypes.c_int), _P])
_sig("qc_set_state", ctypes.c_int, [_P, _P, ctypes.c_size_t, _P])
_sig("qc_profile_enable", ctypes.c_int, [_P, ctypes.c_int])
_sig("qc_grain_set_lanes", ctypes.c_int, [_P, ctypes.c_int])
_sig("qc_grain_set_split", ctypes.c_int, [_P, ctypes.c_double])
_sig("qc_grain_get_split", ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)])
_sig("qc_profile_read", ctypes.c_int, [_P, _D, ctypes.POINTER(ctypes.c_int64)])


def _check(st):
    if st < 0:
        raise QcError(st, lib.qc_last_error().decode())
    return st


def device_count():
    n = ctypes.c_int(0)
    _check(lib.qc_device_count(ctypes.byref(n)))
    return n.value


def valu_rate(op, device=0):
    """Sustained lane operations per second of one FP32 VALU operation
    (op: "fma", "rsq", "sqrt" or "rcp") with every CU busy."""
    v = ctypes.c_double()
    _check(lib.qc_valu_rate(int(device), ["fma", "rsq", "sqrt", "rcp"].index(op), ctypes.byref(v)))
    return v.value


class _DescHolder:
    """Keeps the ctypes descriptor and every array it points to alive."""

    def __init__(self, spec, precision):
        nx, ny, h = int(spec["nx"]), int(spec["ny"]), float(spec["h"])
        x0 = spec.get("x0")
        y0 = spec.get("y0")
        x0 = -0.5 * nx * h if x0 is None else float(x0)
        y0 = -0.5 * ny * h if y0 is None else float(y0)
        comps = spec.get("components", [("s", 1.0)])
        self.keep = []
        shapes = (_Shape * len(spec["shapes"]))()
        for i, sh in enumerate(spec["shapes"]):
            s = shapes[i]
            s.kind = _SHAPES[sh["kind"]]
            s.add = 1 if sh.get("add", True) else 0
            s.cx = float(sh.get("cx", 0.0))
            s.cy = float(sh.get("cy", 0.0))
            s.radius = float(sh.get("radius", 0.0))
            s.n_edges = int(sh.get("n_edges", 0))
            s.side = float(sh.get("side", 0.0))
            s.rotation = float(sh.get("rotation", 0.0))
            if sh["kind"] == "polygon":
                vx = np.ascontiguousarray(sh["vx"], dtype=np.float64)
                vy = np.ascontiguousarray(sh["vy"], dtype=np.float64)
                self.keep += [vx, vy]
                s.vx = vx.ctypes.data_as(_D)
                s.vy = vy.ctypes.data_as(_D)
                s.nv = len(vx)
            elif sh["kind"] == "mask":
                mk = np.ascontiguousarray(np.asarray(sh["mask"]) != 0, dtype=np.uint8)
                if mk.shape != (ny, nx):
                    raise ValueError("mask shape %s does not match the grid (%d, %d)" % (mk.shape, ny, nx))
                self.keep.append(mk)
                s.mask = mk.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8))
        self.keep.append(shapes)
        n_theta = int(spec["n_theta"])
        # the basis functions by name (the library tabulates them), or an
        # explicit eta table when the spec gives one
        eta = spec.get("eta")
        if eta is not None:
            eta = np.ascontiguousarray(np.asarray(eta, dtype=np.complex128).reshape(len(comps), n_theta))
        basis = np.ascontiguousarray([_BASIS[c[0]] for c in comps], dtype=np.int32)
        tc = np.ascontiguousarray([float(c[1]) for c in comps], dtype=np.float64)
        self.keep += [eta, basis, tc]
        d = _Desc()
        d.nx, d.ny, d.h, d.x0, d.y0 = nx, ny, h, x0, y0
        d.shapes = shapes
        d.n_shapes = len(spec["shapes"])
        d.n_theta = n_theta
        d.n_poles = int(spec["n_poles"])
        d.t = float(spec["t"])
        d.ncomp = len(comps)
        d.tc_rel = tc.ctypes.data_as(_D)
        d.eta = eta.ctypes.data_as(_D) if eta is not None else None
        d.basis = basis.ctypes.data_as(ctypes.POINTER(ctypes.c_int))
        d.crystal_rotation = float(spec.get("crystal_rotation", 0.0))
        d.kappa = float(spec.get("kappa", 0.0))
        d.flux_quanta = float(spec.get("flux_quanta", 0.0))
        d.gauge = _GAUGES[spec.get("gauge", "symmetric")]
        d.charge_sign = int(spec.get("charge_sign", -1))
        d.precision = PRECISIONS[precision]
        self.desc = d


def spec_desc(spec, precision="fp64"):
    return _DescHolder(spec, precision)


def _info_dict(info):
    return {f: getattr(info, f) for f, _ in _Info._fields_}


class Plan:
    """Host-side trajectory tables (no device needed)."""

    def __init__(self, spec, precision="fp64"):
        self._h = _DescHolder(spec, precision)
        p = _P()
        _check(lib.qc_plan_create(ctypes.byref(self._h.desc), ctypes.byref(p)))
        self._p = p
        inf = _Info()
        _check(lib.qc_plan_get_info(self._p, ctypes.byref(inf)))
        self.info = _info_dict(inf)
        self.nx, self.ny = int(spec["nx"]), int(spec["ny"])

    def __del__(self, _destroy=lib.qc_plan_destroy):
        # the destroy function is bound at definition: module globals may
        # already be cleared when the interpreter finalises objects
        if getattr(self, "_p", None):
            _destroy(self._p)
            self._p = None

    def mask(self):
        m = np.zeros((self.ny, self.nx), dtype=np.uint8)
        _check(lib.qc_plan_get_mask(self._p, m.ctypes.data))
        return m.astype(bool)

    def segments(self):
        out = np.zeros((self.info["n_segments"], 8))
        _check(lib.qc_plan_get_segments(self._p, out.ctypes.data))
        return out

    def taps(self, at_start):
        n = self.info["n_segments"]
        s = np.zeros((n, 4), dtype=np.int32)
        w = np.zeros((n, 4))
        _check(lib.qc_plan_get_taps(self._p, 1 if at_start else 0, s.ctypes.data, w.ctypes.data))
        return s, w

    def poles(self):
        n = self._h.desc.n_poles
        z = np.zeros(n)
        r = np.zeros(n)
        _check(lib.qc_plan_get_poles(self._p, z.ctypes.data, r.ctypes.data))
        return z, r

    def eta(self):
        """Basis values eta_G(phi_k) of the plan, complex [ncomp, n_theta]."""
        out = np.zeros((self._h.desc.ncomp, self._h.desc.n_theta), dtype=np.complex128)
        _check(lib.qc_plan_get_eta(self._p, out.ctypes.data))
        return out

    def pairing(self):
        """(available, swept steps per paired sweep, mirror segment per segment)."""
        a = ctypes.c_int(0)
        n = ctypes.c_int64(0)
        mir = np.zeros(self.info["n_segments"], dtype=np.int32)
        _check(lib.qc_plan_get_pairing(self._p, ctypes.byref(a), ctypes.byref(n), mir.ctypes.data))
        return bool(a.value), n.value, mir

    def rotate_fold(self):
        """Whether every grain cell has the same rotate-back corners on both
        angles of each pair (the paired rotate-back then gathers once)."""
        a = ctypes.c_int(0)
        _check(lib.qc_plan_get_pairing(self._p, ctypes.byref(a), None, None))
        return bool(a.value & 2)


def _torch():
    import torch
    return torch


def _stream(stream):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dptr(t, dtype, shape, name):
    torch = _torch()
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError("%s must be a CUDA (HIP) torch tensor" % name)
    if t.dtype != dtype or tuple(t.shape) != tuple(shape) or not t.is_contiguous():
        raise ValueError("%s must be a contiguous %s tensor of shape %s (got %s %s)"
                         % (name, dtype, tuple(shape), t.dtype, tuple(t.shape)))
    return ctypes.c_void_p(t.data_ptr())


def _sweep_function():
    torch = _torch()

    class SweepFn(torch.autograd.Function):
        """(delta, A) -> (delta_new, j, omega_total) through qc_sweep, with the
        hand-written adjoint sweep as backward.  The boundary store read by
        the forward is held fixed; call backward before the next sweep on the
        same grain."""

        @staticmethod
        def forward(ctx, delta, A, grain):
            dn, j, om = grain.sweep(delta.detach().contiguous(), A.detach().contiguous())
            ctx.grain = grain
            ctx.count = grain._count
            ctx.save_for_backward(delta.detach().contiguous(), A.detach().contiguous())
            return dn, j, torch.tensor(om, dtype=torch.float64, device=delta.device)

        @staticmethod
        def backward(ctx, g_dn, g_j, g_om):
            grain = ctx.grain
            if grain._count != ctx.count:
                raise RuntimeError("another sweep ran on this grain since the forward: backward needs its store")
            delta, A = ctx.saved_tensors
            gd, ga = grain.sweep_adjoint(
                delta, A,
                g_dn.contiguous() if g_dn is not None else None,
                g_j.contiguous() if g_j is not None else None,
                float(g_om) if g_om is not None else 0.0)
            return gd, ga, None

    return SweepFn


_SWEEP_FN = None


def sweep_autograd(grain, delta, A):
    """Differentiable iteration map: returns (delta_new, j, omega_total)."""
    global _SWEEP_FN
    if _SWEEP_FN is None:
        _SWEEP_FN = _sweep_function()
    return _SWEEP_FN.apply(delta, A, grain)


class Grain:
    """A grain resident on one GPU.  spec: grain description dict (see
    paper_2205_15000_amd.workloads); precision "fp64" or "mixed"."""

    def __init__(self, spec, precision="fp64", device=0):
        self._h = _DescHolder(spec, precision)
        self.spec = spec
        self.precision = precision
        self.device = device
        self.nx, self.ny = int(spec["nx"]), int(spec["ny"])
        self.ncomp = len(spec.get("components", [("s", 1.0)]))
        self.n_poles = int(spec["n_poles"])
        p = _P()
        _check(lib.qc_grain_create(int(device), ctypes.byref(self._h.desc), ctypes.byref(p)))
        self._g = p
        inf = _Info()
        _check(lib.qc_grain_get_info(self._g, ctypes.byref(inf)))
        self.info = _info_dict(inf)
        self._count = 0

    def close(self, _destroy=lib.qc_grain_destroy):
        if getattr(self, "_g", None):
            _destroy(self._g)
            self._g = None

    def __del__(self):
        self.close()

    @property
    def steps_per_sweep(self):
        return self.info["steps_per_sweep"]

    def _dev(self):
        return _torch().device("cuda", self.device)

    def mask(self):
        """Grain cells, bool [ny, nx]."""
        m = np.zeros((self.ny, self.nx), dtype=np.uint8)
        _check(lib.qc_grain_get_mask(self._g, m.ctypes.data))
        return m.astype(bool)

    def reset_bc(self):
        _check(lib.qc_grain_reset_bc(self._g))

    def sweep(self, delta, A, omega_density=False, total=True, stream=None, out=None):
        """One iteration map: returns (delta_new, j, omega_total[, omega_density])."""
        torch = _torch()
        shp_d = (self.ncomp, self.ny, self.nx)
        dp = _dptr(delta, torch.complex128, shp_d, "delta")
        ap = _dptr(A, torch.float64, (2, self.ny, self.nx), "A")
        if out is None:
            dn = torch.empty(shp_d, dtype=torch.complex128, device=self._dev())
            j = torch.empty((2, self.ny, self.nx), dtype=torch.float64, device=self._dev())
        else:
            dn, j = out
        od = torch.empty((self.ny, self.nx), dtype=torch.float64, device=self._dev()) if omega_density else None
        tot = ctypes.c_double(0.0)
        self._count += 1
        _check(lib.qc_sweep(self._g, dp, ap, ctypes.c_void_p(dn.data_ptr()), ctypes.c_void_p(j.data_ptr()),
                            ctypes.c_void_p(od.data_ptr()) if od is not None else None,
                            ctypes.byref(tot) if total else None, _stream(stream)))
        res = (dn, j, tot.value if total else None)
        return res + ((od,) if omega_density else ())

    def solve_A(self, j, B=True, stream=None):
        torch = _torch()
        jp = _dptr(j, torch.float64, (2, self.ny, self.nx), "j")
        A = torch.empty((2, self.ny, self.nx), dtype=torch.float64, device=self._dev())
        Bt = torch.empty((self.ny, self.nx), dtype=torch.float64, device=self._dev()) if B else None
        _check(lib.qc_solve_A(self._g, jp, ctypes.c_void_p(A.data_ptr()),
                              ctypes.c_void_p(Bt.data_ptr()) if Bt is not None else None, _stream(stream)))
        return A, Bt

    def set_A_solver(self, eps):
        """eps > 0: eigen-truncated separable A-solve (square grids); 0: FFT."""
        _check(lib.qc_grain_set_A_solver(self._g, float(eps)))

    def A_solver(self):
        """(eps, modes kept)."""
        e = ctypes.c_double(0.0)
        n = ctypes.c_int(0)
        _check(lib.qc_grain_get_A_solver(self._g, ctypes.byref(e), ctypes.byref(n)))
        return e.value, n.value

    def magnetic_moment(self, j, stream=None):
        """m_z / m0 of the current j [2, ny, nx] about the grid centre."""
        torch = _torch()
        jp = _dptr(j, torch.float64, (2, self.ny, self.nx), "j")
        m = ctypes.c_double(0.0)
        _check(lib.qc_magnetic_moment(self._g, jp, ctypes.byref(m), _stream(stream)))
        return m.value

    def scf(self, delta, A, max_iter, min_iter=0, burnin=0, tol=0.0, norm_p=2, alpha=1.0, stream=None):
        """SCF in place on (delta, A) with the grain's accelerator (Picard
        unless set_accelerator chose Polyak); returns (iters,
        residuals[iters,5], converged)."""
        torch = _torch()
        dp = _dptr(delta, torch.complex128, (self.ncomp, self.ny, self.nx), "delta")
        ap = _dptr(A, torch.float64, (2, self.ny, self.nx), "A")
        res = np.zeros((max_iter, 5))
        it = ctypes.c_int(0)
        st = _check(lib.qc_scf_run(self._g, dp, ap, int(max_iter), int(min_iter), int(burnin), float(tol),
                                   int(norm_p), float(alpha), ctypes.byref(it), res.ctypes.data, _stream(stream)))
        return it.value, res[:it.value], st == QC_OK

    def ldos(self, delta, A, energies, broadening, bc_iters, stream=None):
        torch = _torch()
        dp = _dptr(delta, torch.complex128, (self.ncomp, self.ny, self.nx), "delta")
        ap = _dptr(A, torch.float64, (2, self.ny, self.nx), "A")
        e = np.ascontiguousarray(energies, dtype=np.float64)
        out = torch.empty((len(e), self.ny, self.nx), dtype=torch.float64, device=self._dev())
        _check(lib.qc_ldos(self._g, dp, ap, e.ctypes.data, len(e), float(broadening), int(bc_iters),
                           ctypes.c_void_p(out.data_ptr()), _stream(stream)))
        return out

    def ldos_converge(self, delta, A, energies, broadening, tol, max_iter, energies_per_block=0, stream=None):
        """LDOS with the boundary iteration run until it changes by less than
        tol; returns (ldos [E, ny, nx], sweeps of the slowest block)."""
        torch = _torch()
        dp = _dptr(delta, torch.complex128, (self.ncomp, self.ny, self.nx), "delta")
        ap = _dptr(A, torch.float64, (2, self.ny, self.nx), "A")
        e = np.ascontiguousarray(energies, dtype=np.float64)
        out = torch.empty((len(e), self.ny, self.nx), dtype=torch.float64, device=self._dev())
        it = ctypes.c_int(0)
        _check(lib.qc_ldos_converge(self._g, dp, ap, e.ctypes.data, len(e), float(broadening), float(tol),
                                    int(max_iter), int(energies_per_block), ctypes.byref(it),
                                    ctypes.c_void_p(out.data_ptr()), _stream(stream)))
        return out, it.value

    def sweep_adjoint(self, delta, A, g_delta_new=None, g_j=None, g_omega=0.0, stream=None):
        """Reverse mode of the most recent sweep: returns (grad_delta, grad_A)
        for a real loss with the given output gradients."""
        torch = _torch()
        shp_d = (self.ncomp, self.ny, self.nx)
        dp = _dptr(delta, torch.complex128, shp_d, "delta")
        ap = _dptr(A, torch.float64, (2, self.ny, self.nx), "A")
        gdn = _dptr(g_delta_new, torch.complex128, shp_d, "g_delta_new") if g_delta_new is not None else None
        gj = _dptr(g_j, torch.float64, (2, self.ny, self.nx), "g_j") if g_j is not None else None
        gd = torch.empty(shp_d, dtype=torch.complex128, device=self._dev())
        ga = torch.empty((2, self.ny, self.nx), dtype=torch.float64, device=self._dev())
        _check(lib.qc_sweep_adjoint(self._g, dp, ap, gdn, gj, float(g_omega), ctypes.c_void_p(gd.data_ptr()),
                                    ctypes.c_void_p(ga.data_ptr()), _stream(stream)))
        return gd, ga

    def green_average(self, delta, A, stream=None):
        """<g>(R, i eps_p) at the positive poles, complex [n_poles, ny, nx],
        with the start values the next sweep would use."""
        torch = _torch()
        shp_d = (self.ncomp, self.ny, self.nx)
        dp = _dptr(delta, torch.complex128, shp_d, "delta")
        ap = _dptr(A, torch.float64, (2, self.ny, self.nx), "A")
        out = torch.empty((self.n_poles, self.ny, self.nx), dtype=torch.complex128, device=self._dev())
        _check(lib.qc_green_average(self._g, dp, ap, ctypes.c_void_p(out.data_ptr()), _stream(stream)))
        return out

    def free_energy_lw(self, delta, A, n_lambda, bc_iters, density=False, stream=None):
        """Luttinger-Ward free energy: returns omega_total (and the density
        [ny, nx] when density is set)."""
        torch = _torch()
        shp_d = (self.ncomp, self.ny, self.nx)
        dp = _dptr(delta, torch.complex128, shp_d, "delta")
        ap = _dptr(A, torch.float64, (2, self.ny, self.nx), "A")
        od = torch.empty((self.ny, self.nx), dtype=torch.float64, device=self._dev()) if density else None
        tot = ctypes.c_double(0.0)
        _check(lib.qc_free_energy_lw(self._g, dp, ap, int(n_lambda), int(bc_iters),
                                     ctypes.c_void_p(od.data_ptr()) if od is not None else None,
                                     ctypes.byref(tot), _stream(stream)))
        return (tot.value, od) if density else tot.value

    def get_state(self, stream=None):
        torch = _torch()
        n = ctypes.c_size_t(0)
        _check(lib.qc_get_state(self._g, None, ctypes.byref(n), None))
        buf = torch.empty(n.value, dtype=torch.uint8, device=self._dev())
        _check(lib.qc_get_state(self._g, ctypes.c_void_p(buf.data_ptr()), ctypes.byref(n), _stream(stream)))
        return buf

    def set_state(self, buf, stream=None):
        _check(lib.qc_set_state(self._g, ctypes.c_void_p(buf.data_ptr()), ctypes.c_size_t(buf.numel()),
                                _stream(stream)))

    def set_accelerator(self, kind, beta=0.5):
        """SCF accelerator of scf(): "picard", "polyak" (heavy ball with
        drag beta; the step size is scf's alpha) or "bb" (Barzilai-Borwein
        step sizes, scf's alpha the first) or "congacc" (per-component steps,
        scf's alpha the first; 2-norm residuals)."""
        k = {"picard": 0, "polyak": 1, "bb": 2, "congacc": 3}[kind]
        _check(lib.qc_grain_set_accelerator(self._g, k, float(beta)))

    def set_pairing(self, enable):
        """Angle pairs (phi_k, phi_k + pi) in the Matsubara sweeps: one march
        serves both directions (on by default where the tables allow it)."""
        _check(lib.qc_grain_set_pairing(self._g, 1 if enable else 0))

    def pairing(self):
        """(available, enabled, trajectory steps one Matsubara sweep marches)."""
        a = ctypes.c_int(0)
        e = ctypes.c_int(0)
        n = ctypes.c_int64(0)
        _check(lib.qc_grain_get_pairing(self._g, ctypes.byref(a), ctypes.byref(e), ctypes.byref(n)))
        return bool(a.value), bool(e.value), n.value

    def rotate_fold(self):
        """Whether each pair of angles shares its rotate-back corners (the
        paired rotate-back and the paired LDOS output gather once per pair)."""
        a = ctypes.c_int(0)
        _check(lib.qc_grain_get_pairing(self._g, ctypes.byref(a), None, None))
        return bool(a.value & 2)

    def accel_stats(self):
        """(bisected, anti_parallel): CongAcc weights set by bisection and by
        the anti-parallel rule over the grain's lifetime."""
        b = ctypes.c_int64(0)
        a = ctypes.c_int64(0)
        _check(lib.qc_grain_get_accel_stats(self._g, ctypes.byref(b), ctypes.byref(a)))
        return b.value, a.value

    def set_adjoint_checkpoint(self, every):
        """Reverse mode with checkpoints every `every` slots (default 32;
        0 stores gamma~ and its adjoint terms at every node)."""
        _check(lib.qc_grain_set_adjoint_checkpoint(self._g, int(every)))

    def set_lanes(self, energies_per_lane):
        """Energies per lane of the sweep kernel (1, 2, 3, 4, 8; 0 = automatic)."""
        _check(lib.qc_grain_set_lanes(self._g, int(energies_per_lane)))

    def lanes(self):
        """(energies per lane, lanes per segment) of the next SCF sweep."""
        e = ctypes.c_int(0)
        G = ctypes.c_int(0)
        _check(lib.qc_grain_get_lanes(self._g, ctypes.byref(e), ctypes.byref(G)))
        return e.value, G.value

    def set_split(self, frac):
        """Split launch shape of the SCF sweep: segments longer than frac x
        the longest march with twice the lanes when the launch is short
        (0 turns it off; default 0.8)."""
        _check(lib.qc_grain_set_split(self._g, float(frac)))

    def split(self):
        """(fraction, segments the next SCF sweep launches with the wide shape)."""
        f = ctypes.c_double(0.0)
        n = ctypes.c_int64(0)
        _check(lib.qc_grain_get_split(self._g, ctypes.byref(f), ctypes.byref(n)))
        return f.value, n.value

    def profile(self, enable=True):
        _check(lib.qc_profile_enable(self._g, 1 if enable else 0))

    def profile_read(self):
        ms = ctypes.c_double(0.0)
        n = ctypes.c_int64(0)
        _check(lib.qc_profile_read(self._g, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value


class Batch:
    """Several grains iterated together: one persistent sweep launch per
    iteration, optionally replayed from a hipGraph."""

    def __init__(self, grains):
        self.grains = list(grains)
        arr = (_P * len(self.grains))(*[g._g for g in self.grains])
        p = _P()
        _check(lib.qc_batch_create(arr, len(self.grains), ctypes.byref(p)))
        self._b = p

    def close(self, _destroy=lib.qc_batch_destroy):
        if getattr(self, "_b", None):
            _destroy(self._b)
            self._b = None

    def __del__(self):
        self.close()

    def info(self):
        st = ctypes.c_int64(0)
        e = ctypes.c_int(0)
        t = ctypes.c_int(0)
        _check(lib.qc_batch_get_info(self._b, ctypes.byref(st), ctypes.byref(e), ctypes.byref(t)))
        return {"steps_per_iteration": st.value, "energies_per_lane": e.value, "tiles": t.value}

    def set_fields(self, i, delta, A, stream=None):
        torch = _torch()
        g = self.grains[i]
        dp = _dptr(delta, torch.complex128, (g.ncomp, g.ny, g.nx), "delta")
        ap = _dptr(A, torch.float64, (2, g.ny, g.nx), "A")
        _check(lib.qc_batch_set_fields(self._b, int(i), dp, ap, _stream(stream)))

    def get_fields(self, i, stream=None):
        torch = _torch()
        g = self.grains[i]
        d = torch.empty((g.ncomp, g.ny, g.nx), dtype=torch.complex128, device=g._dev())
        a = torch.empty((2, g.ny, g.nx), dtype=torch.float64, device=g._dev())
        _check(lib.qc_batch_get_fields(self._b, int(i), ctypes.c_void_p(d.data_ptr()), ctypes.c_void_p(a.data_ptr()),
                                       _stream(stream)))
        return d, a

    def iterate(self, n_iter, graph=True, stream=None):
        """Runs n_iter Picard iterations of every grain; returns milliseconds."""
        _check(lib.qc_batch_iterate(self._b, int(n_iter), 1 if graph else 0,
                                    _stream(stream) if stream is not None else None))
        ms = ctypes.c_double(0.0)
        _check(lib.qc_batch_last_ms(self._b, ctypes.byref(ms)))
        return ms.value

    def autotune(self, iters_per_trial=2):
        e = ctypes.c_int(0)
        _check(lib.qc_batch_autotune(self._b, int(iters_per_trial), ctypes.byref(e), None))
        return e.value
