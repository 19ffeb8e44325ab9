"""Thin ctypes binding of libsis.so (include/sis.h).

Argument marshalling only: every step of the hot path runs in the library's
HIP kernels.  PyTorch provides device memory and the current stream.  If the
library has not been built this module raises on import of the library
(no fallback of any kind).
"""
import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsis.so")

SIS_OK = 0
SIS_E_INVALID = -1
SIS_E_SHAPE = -2
SIS_E_DEVICE = -3
SIS_E_OOM = -4
SIS_E_NOT_CONVERGED = -5
SIS_E_NUMERIC = -6
SIS_E_UNSUPPORTED = -7

KERNEL_HARD_SPHERE = 0
KERNEL_IPL = 1
PREC_FP64, PREC_FP32, PREC_BF16X3, PREC_BF16 = 0, 1, 2, 3
PRECISIONS = {"fp64": PREC_FP64, "fp32": PREC_FP32, "bf16x3": PREC_BF16X3, "bf16": PREC_BF16}
FLOW_NONE, FLOW_POISEUILLE, FLOW_TRANSPIRATION = 0, 1, 2
SCHEME_CIS, SCHEME_SIS = 0, 1
GEOM_PLANAR_HALF, GEOM_DUCT_QUARTER, GEOM_PERIODIC_2D, GEOM_TUBE = 0, 1, 2, 3
GRID_CARTESIAN, GRID_POLAR = 0, 1
DIFFUSION_CG, DIFFUSION_INVERSE = 0, 1


class SisError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"sis error {code}: {msg}")
        self.code = code


class VelocityDesc(ctypes.Structure):
    _fields_ = [("n_v", ctypes.c_int32), ("l_v", ctypes.c_double), ("n_pad", ctypes.c_int32),
                ("m_angle", ctypes.c_int32), ("r_trunc", ctypes.c_double),
                ("kernel", ctypes.c_int32), ("visc_index", ctypes.c_double),
                ("n_threads", ctypes.c_int32), ("n_species", ctypes.c_int32),
                ("mass", ctypes.c_double * 2), ("diam", ctypes.c_double * 2),
                ("chi", ctypes.c_double * 2), ("m_rho", ctypes.c_int32), ("parity", ctypes.c_int32),
                ("grid", ctypes.c_int32), ("n_vr", ctypes.c_int32), ("vr_max", ctypes.c_double),
                ("n_th", ctypes.c_int32), ("n_vz", ctypes.c_int32), ("l_pad", ctypes.c_double)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("n_v", ctypes.c_int32), ("n3", ctypes.c_int32), ("n_pad", ctypes.c_int32),
                ("m_angle", ctypes.c_int32), ("n_dir", ctypes.c_int32),
                ("l_v", ctypes.c_double), ("dv", ctypes.c_double), ("b0", ctypes.c_double),
                ("r_trunc", ctypes.c_double), ("nubar", ctypes.c_double),
                ("alpha", ctypes.c_double), ("gamma", ctypes.c_double),
                ("operator_bytes", ctypes.c_int64), ("plan_seconds_host", ctypes.c_double),
                ("plan_seconds_device", ctypes.c_double), ("n_species", ctypes.c_int32),
                ("n_dof", ctypes.c_int32), ("nubar_b", ctypes.c_double),
                ("viscosity_ratio", ctypes.c_double), ("flow_factor", ctypes.c_double),
                ("parity", ctypes.c_int32), ("n_vel", ctypes.c_int32)]


class GeometryDesc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n_cases", ctypes.c_int32),
                ("node_offset", ctypes.POINTER(ctypes.c_int64)),
                ("x1", ctypes.POINTER(ctypes.c_double)),
                ("delta", ctypes.POINTER(ctypes.c_double)),
                ("flow", ctypes.POINTER(ctypes.c_int32)),
                ("n1", ctypes.POINTER(ctypes.c_int32)),
                ("n2", ctypes.POINTER(ctypes.c_int32)),
                ("face1", ctypes.POINTER(ctypes.c_double)),
                ("face2", ctypes.POINTER(ctypes.c_double)),
                ("solid", ctypes.POINTER(ctypes.c_uint8))]


class SolveOpts(ctypes.Structure):
    _fields_ = [("scheme", ctypes.c_int32), ("N", ctypes.c_double), ("eps", ctypes.c_double),
                ("max_it", ctypes.c_int32), ("project", ctypes.c_int32),
                ("check_every", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("refresh_every", ctypes.c_int32), ("persistent", ctypes.c_int32)]


class SolveResult(ctypes.Structure):
    _fields_ = [("M", ctypes.POINTER(ctypes.c_double)), ("Q", ctypes.POINTER(ctypes.c_double)),
                ("iters", ctypes.POINTER(ctypes.c_int32)),
                ("residual", ctypes.POINTER(ctypes.c_double)),
                ("U", ctypes.POINTER(ctypes.c_double)), ("q", ctypes.POINTER(ctypes.c_double)),
                ("seconds", ctypes.c_double), ("total_iters", ctypes.c_int32)]


_P = ctypes.c_void_p
_D = ctypes.POINTER(ctypes.c_double)
_SIGS = {
    "sis_last_error": (ctypes.c_char_p, []),
    "sis_version": (ctypes.c_int32, []),
    "sis_plan_create": (ctypes.c_int32, [ctypes.POINTER(VelocityDesc), _P, ctypes.POINTER(_P)]),
    "sis_plan_destroy": (ctypes.c_int32, [_P]),
    "sis_plan_query": (ctypes.c_int32, [_P, ctypes.POINTER(PlanInfo)]),
    "sis_plan_tables": (ctypes.c_int32, [_P, _P, _P, _P, _P]),
    "sis_host_tables": (ctypes.c_int32, [ctypes.POINTER(VelocityDesc), _P, _P, _P, _P, _D, _D]),
    "sis_plan_set_precision": (ctypes.c_int32, [_P, ctypes.c_int32, _P]),
    "sis_geometry_create": (ctypes.c_int32, [_P, ctypes.POINTER(GeometryDesc), _P, ctypes.POINTER(_P)]),
    "sis_geometry_destroy": (ctypes.c_int32, [_P]),
    "sis_geometry_cells": (ctypes.c_int64, [_P]),
    "sis_geometry_moment_stride": (ctypes.c_int32, [_P]),
    "sis_geometry_sweep_form": (ctypes.c_int32, [_P]),
    "sis_geometry_diffusion_solver": (ctypes.c_int32, [_P, ctypes.c_int32, _P]),
    "sis_geometry_diffusion_info": (ctypes.c_int32, [_P, ctypes.POINTER(ctypes.c_int32),
                                                     ctypes.POINTER(ctypes.c_int32), _D]),
    "sis_collide": (ctypes.c_int32, [_P, ctypes.c_int64, _P, _P, _P, _P, ctypes.c_int32, _P, _P, _P, _P]),
    "sis_collide_noalloc": (ctypes.c_int32, [_P, ctypes.c_int64, _P, _P, _P, _P, ctypes.c_int32, _P, _P, _P, _P]),
    "sis_collide_fsm": (ctypes.c_int32, [_P, ctypes.c_int64, _P, _P, _P, _P, ctypes.c_int32, _P, _P, _P, _P]),
    "sis_plan_fsm_info": (ctypes.c_int32, [_P, _D, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int64)]),
    "sis_plan_set_fsm_slab": (ctypes.c_int32, [_P, ctypes.c_int32]),
    "sis_plan_fsm_timing_read": (ctypes.c_int32, [_P, _D, ctypes.POINTER(ctypes.c_int64)]),
    "sis_transport_sweep": (ctypes.c_int32, [_P, _P, _P, _P, _P, _P]),
    "sis_moments": (ctypes.c_int32, [_P, ctypes.c_int64, _P, _P, _P]),
    "sis_diffusion_correct": (ctypes.c_int32, [_P, _P, _P, _P, ctypes.c_double, _P, _P, _P]),
    "sis_solve": (ctypes.c_int32, [_P, _P, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveResult), _P]),
    "sis_state_create": (ctypes.c_int32, [_P, _P, ctypes.POINTER(SolveOpts), _P, ctypes.POINTER(_P)]),
    "sis_state_reset": (ctypes.c_int32, [_P, _P]),
    "sis_state_step": (ctypes.c_int32, [_P, ctypes.c_int32, _P]),
    "sis_state_poll": (ctypes.c_int32, [_P, ctypes.POINTER(ctypes.c_int32), _P]),
    "sis_state_results": (ctypes.c_int32, [_P, ctypes.POINTER(SolveResult), _P]),
    "sis_state_destroy": (ctypes.c_int32, [_P]),
    "sis_plan_set_contraction_config": (ctypes.c_int32, [_P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                                         ctypes.c_int32, ctypes.c_int32]),
    "sis_plan_contraction_config": (ctypes.c_int32, [_P, ctypes.c_int64, ctypes.c_int32,
                                                     ctypes.POINTER(ctypes.c_int32),
                                                     ctypes.POINTER(ctypes.c_int32),
                                                     ctypes.POINTER(ctypes.c_int32),
                                                     ctypes.POINTER(ctypes.c_int32)]),
    "sis_plan_timing": (ctypes.c_int32, [_P, ctypes.c_int32]),
    "sis_plan_timing_read": (ctypes.c_int32, [_P, _D, ctypes.POINTER(ctypes.c_int64)]),
}

_lib = None


def lib():
    """Load libsis.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_1612_04488_amd.build`")
        # PyTorch brings its own HIP runtime: load it first so that the library
        # binds to the same runtime instance as the tensors it is handed.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(code):
    if code != SIS_OK:
        raise SisError(code, lib().sis_last_error().decode())
    return code


def _ptr(t):
    """Device pointer of a tensor (or None)."""
    if t is None:
        return None
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    if stream is not None:
        return ctypes.c_void_p(stream)
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def velocity_desc(n_v, l_v=6.0, n_pad=0, m_angle=6, kernel="hs", visc_index=0.81,
                  r_trunc=0.0, n_threads=0, mixture=None, parity=0, polar=None):
    """mixture: None (one gas) or dict(masses=(m_A, m_B), diameters=(d_A, d_B),
    chi=(chi_A, chi_B), m_rho=16) for a binary hard-sphere mixture.
    parity: 0 full grid, 1 store v3 > 0 (odd in v3), 2 store v2, v3 > 0 (planar).
    polar: None (Cartesian n_v^3 grid) or dict(n_vr, vr_max, n_th, n_vz, l_pad=0) for
    the tube's polar grid (v_z on [0, l_v]; n_v and parity ignored)."""
    k = KERNEL_HARD_SPHERE if kernel == "hs" else KERNEL_IPL
    d = VelocityDesc(n_v, l_v, n_pad, m_angle, r_trunc, k, visc_index, n_threads)
    d.parity = int(parity)
    if polar is not None:
        d.grid = GRID_POLAR
        d.n_vr = int(polar["n_vr"])
        d.vr_max = float(polar["vr_max"])
        d.n_th = int(polar["n_th"])
        d.n_vz = int(polar["n_vz"])
        d.l_pad = float(polar.get("l_pad", 0.0))
    if mixture is not None:
        d.n_species = 2
        d.mass[:] = [float(x) for x in mixture["masses"]]
        d.diam[:] = [float(x) for x in mixture["diameters"]]
        d.chi[:] = [float(x) for x in mixture["chi"]]
        d.m_rho = int(mixture.get("m_rho", 0))
    return d


def host_tables(desc):
    """Host-only tables (no GPU): dict with feq, nu, A, B (numpy), b0, nubar.
    Mixtures: feq, nu of shape (2, n3), nubar of shape (2,), no A, B."""
    import numpy as np
    n3 = desc.n_v ** 3
    if desc.n_species == 2:
        feq, nu = np.zeros((2, n3)), np.zeros((2, n3))
        b0, nubar = ctypes.c_double(), (ctypes.c_double * 2)()
        check(lib().sis_host_tables(ctypes.byref(desc), feq.ctypes.data_as(_P), nu.ctypes.data_as(_P),
                                    None, None, ctypes.byref(b0), ctypes.cast(nubar, _D)))
        return dict(feq=feq, nu=nu, b0=b0.value, nubar=np.array(nubar[:]))
    D = desc.m_angle ** 2
    feq, nu = np.zeros(n3), np.zeros(n3)
    A, B = np.zeros((D, n3)), np.zeros((D, n3))
    b0, nubar = ctypes.c_double(), ctypes.c_double()
    check(lib().sis_host_tables(ctypes.byref(desc), feq.ctypes.data_as(_P), nu.ctypes.data_as(_P),
                                A.ctypes.data_as(_P), B.ctypes.data_as(_P),
                                ctypes.byref(b0), ctypes.byref(nubar)))
    return dict(feq=feq, nu=nu, A=A, B=B, b0=b0.value, nubar=nubar.value)


class Plan:
    """Velocity grid + assembled fast-spectral operator on the current device."""

    def __init__(self, n_v, l_v=6.0, n_pad=0, m_angle=6, kernel="hs", visc_index=0.81,
                 r_trunc=0.0, n_threads=0, stream=None, mixture=None, parity=0, polar=None):
        self.desc = velocity_desc(n_v, l_v, n_pad, m_angle, kernel, visc_index, r_trunc, n_threads,
                                  mixture, parity, polar)
        h = ctypes.c_void_p()
        check(lib().sis_plan_create(ctypes.byref(self.desc), _stream(stream), ctypes.byref(h)))
        self.handle = h
        self.polar = polar is not None
        self.n_species = 2 if mixture is not None else 1
        if self.polar:
            self.n_v = 0
            self.parity = 0
            self.n_vel = int(polar["n_vr"]) * int(polar["n_th"]) * int(polar["n_vz"])
            self.n3 = self.n_vel
        else:
            self.n_v = n_v
            self.n3 = n_v ** 3
            self.parity = int(parity)
            self.n_vel = n_v * (n_v // 2 if parity == 2 else n_v) * (n_v // 2 if parity else n_v)
        self.n_dof = self.n_species * self.n_vel

    def close(self):
        if getattr(self, "handle", None):
            lib().sis_plan_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def info(self):
        i = PlanInfo()
        check(lib().sis_plan_query(self.handle, ctypes.byref(i)))
        return {f: getattr(i, f) for f, _ in PlanInfo._fields_}

    def tables(self, operator=False):
        import numpy as np
        ns = self.n_species
        v1d, feq, nu = np.zeros(self.n_v), np.zeros(ns * self.n_vel), np.zeros(ns * self.n_vel)
        op = np.zeros((self.n_dof, self.n_dof)) if operator else None
        check(lib().sis_plan_tables(self.handle, v1d.ctypes.data_as(_P), feq.ctypes.data_as(_P),
                                    nu.ctypes.data_as(_P),
                                    op.ctypes.data_as(_P) if operator else None))
        if ns > 1:
            feq, nu = feq.reshape(ns, self.n_vel), nu.reshape(ns, self.n_vel)
        return dict(v1d=v1d, feq=feq, nu=nu, op=op)

    def set_precision(self, precision, stream=None):
        p = PRECISIONS.get(precision, precision)
        check(lib().sis_plan_set_precision(self.handle, p, _stream(stream)))

    def collide(self, h, delta, rhs_out, dU=None, flow=None, project=False, lh_out=None,
                amom_out=None, stream=None):
        n_cells = h.shape[0]
        check(lib().sis_collide(self.handle, n_cells, _ptr(h), _ptr(dU), _ptr(delta), _ptr(flow),
                                1 if project else 0, _ptr(rhs_out), _ptr(lh_out), _ptr(amom_out),
                                _stream(stream)))

    def collide_noalloc(self, h, delta, rhs_out, dU=None, flow=None, project=False, lh_out=None,
                        amom_out=None, stream=None):
        """sis_collide with the library's fixed device workspace (no allocation)."""
        n_cells = h.shape[0]
        check(lib().sis_collide_noalloc(self.handle, n_cells, _ptr(h), _ptr(dU), _ptr(delta), _ptr(flow),
                                        1 if project else 0, _ptr(rhs_out), _ptr(lh_out), _ptr(amom_out),
                                        _stream(stream)))

    def collide_fsm(self, h, delta, rhs_out, dU=None, flow=None, project=False, lh_out=None,
                    amom_out=None, stream=None):
        """sis_collide with L+ from the per-cell transforms of the fast spectral method."""
        n_cells = h.shape[0]
        check(lib().sis_collide_fsm(self.handle, n_cells, _ptr(h), _ptr(dU), _ptr(delta), _ptr(flow),
                                    1 if project else 0, _ptr(rhs_out), _ptr(lh_out), _ptr(amom_out),
                                    _stream(stream)))

    def fsm_info(self):
        """Executed flops per cell update, l1-slab width and table bytes of the transform path."""
        f, s, b = ctypes.c_double(), ctypes.c_int32(), ctypes.c_int64()
        check(lib().sis_plan_fsm_info(self.handle, ctypes.byref(f), ctypes.byref(s), ctypes.byref(b)))
        return {"flops_per_cell": f.value, "slab_l1": s.value, "table_bytes": b.value}

    def set_fsm_slab(self, slab_l1):
        check(lib().sis_plan_set_fsm_slab(self.handle, int(slab_l1)))

    def set_contraction_config(self, n_cells, tile_rows, k_stage, splits, precision="fp64"):
        """Fix the contraction configuration for n_cells cells instead of tuning it."""
        check(lib().sis_plan_set_contraction_config(self.handle, int(n_cells), PRECISIONS.get(precision, precision),
                                                    int(tile_rows), int(k_stage), int(splits)))

    def contraction_config(self, n_cells, precision="fp64", with_depth=False):
        """(tile rows, split-K, tuned[, k-stage depth]) of the contraction for n_cells cells."""
        t, s, u, k = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        check(lib().sis_plan_contraction_config(self.handle, int(n_cells), PRECISIONS.get(precision, precision),
                                                ctypes.byref(t), ctypes.byref(s), ctypes.byref(u), ctypes.byref(k)))
        if with_depth:
            return t.value, s.value, bool(u.value), k.value
        return t.value, s.value, bool(u.value)

    def timing(self, enable):
        check(lib().sis_plan_timing(self.handle, 1 if enable else 0))

    def timing_read(self, fsm=False):
        """(summed ms, launches) of the timed contractions, or with fsm=True of the
        timed sis_collide_fsm calls."""
        ms, n = ctypes.c_double(), ctypes.c_int64()
        fn = lib().sis_plan_fsm_timing_read if fsm else lib().sis_plan_timing_read
        check(fn(self.handle, ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def moments(self, h, mom_out, stream=None):
        check(lib().sis_moments(self.handle, h.shape[0], _ptr(h), _ptr(mom_out), _stream(stream)))


class Geometry:
    """Planar half-channel geometry for a batch of cases (host arrays copied); with
    kind="tube" (plans on the polar grid) the cases are tubes and xs their radial
    nodes (r > 0 increasing to the wall r = 1)."""

    def __init__(self, plan, xs, deltas, flows, stream=None, kind="planar"):
        import numpy as np
        self.plan = plan
        off = np.zeros(len(xs) + 1, dtype=np.int64)
        off[1:] = np.cumsum([len(x) for x in xs])
        self.offsets = off
        self._x = np.ascontiguousarray(np.concatenate([np.asarray(x, np.float64) for x in xs]))
        self._d = np.ascontiguousarray(np.asarray(deltas, np.float64))
        self._f = np.ascontiguousarray(np.asarray(flows, np.int32))
        d = GeometryDesc(GEOM_TUBE if kind == "tube" else GEOM_PLANAR_HALF, len(xs),
                         self.offsets.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                         self._x.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                         self._d.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                         self._f.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)))
        self.mom_stride = 8 if kind == "tube" else 4
        h = ctypes.c_void_p()
        check(lib().sis_geometry_create(plan.handle, ctypes.byref(d), _stream(stream), ctypes.byref(h)))
        self.handle = h
        self.n_cells = int(off[-1])
        self.n_cases = len(xs)

    def close(self):
        if getattr(self, "handle", None):
            lib().sis_geometry_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Geometry2D:
    """Quarter ducts (kind "duct") or periodic porous cells (kind "periodic").

    cases: list of (face1, face2, solid-or-None); solid is an (n1, n2) bool
    array (True = solid).  Fluid cells are numbered per case in row-major
    (i, j) order.
    """

    def __init__(self, plan, kind, cases, deltas, flows, stream=None):
        import numpy as np
        self.plan = plan
        k = GEOM_DUCT_QUARTER if kind == "duct" else GEOM_PERIODIC_2D
        n1 = np.array([len(c[0]) - 1 for c in cases], np.int32)
        n2 = np.array([len(c[1]) - 1 for c in cases], np.int32)
        f1 = np.ascontiguousarray(np.concatenate([np.asarray(c[0], np.float64) for c in cases]))
        f2 = np.ascontiguousarray(np.concatenate([np.asarray(c[1], np.float64) for c in cases]))
        has_solid = any(c[2] is not None for c in cases)
        solid = None
        if has_solid:
            solid = np.ascontiguousarray(np.concatenate([
                (np.zeros((a, b), np.uint8) if c[2] is None else np.asarray(c[2], np.uint8)).ravel()
                for a, b, c in zip(n1, n2, cases)]))
        self._keep = (n1, n2, f1, f2, solid)
        self._d = np.ascontiguousarray(np.asarray(deltas, np.float64))
        self._f = np.ascontiguousarray(np.asarray(flows, np.int32))
        I32 = ctypes.POINTER(ctypes.c_int32)
        D = ctypes.POINTER(ctypes.c_double)
        d = GeometryDesc(k, len(cases), None, None, self._d.ctypes.data_as(D), self._f.ctypes.data_as(I32),
                         n1.ctypes.data_as(I32), n2.ctypes.data_as(I32), f1.ctypes.data_as(D),
                         f2.ctypes.data_as(D),
                         solid.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)) if has_solid else None)
        h = ctypes.c_void_p()
        check(lib().sis_geometry_create(plan.handle, ctypes.byref(d), _stream(stream), ctypes.byref(h)))
        self.handle = h
        self.n_cells = int(lib().sis_geometry_cells(h))
        self.n_cases = len(cases)
        fl = [int(np.sum(1 - (np.zeros((a, b)) if c[2] is None else np.asarray(c[2], int))))
              for a, b, c in zip(n1, n2, cases)]
        self.offsets = np.concatenate([[0], np.cumsum(fl)]).astype(np.int64)
        self.mom_stride = 8

    def sweep_form(self):
        """Kernel form of the 2-D sweep: 1 row-blocked (every case at most 128
        cells along axis 2, distributions under 2 GiB), 2 pipelined anti-diagonal,
        3 plain anti-diagonal."""
        return int(lib().sis_geometry_sweep_form(self.handle))

    def diffusion_solver(self, mode, stream=None):
        """"inverse" (default: precomputed per-case inverse where it applies) or "cg"."""
        m = {"cg": DIFFUSION_CG, "inverse": DIFFUSION_INVERSE}[mode]
        check(lib().sis_geometry_diffusion_solver(self.handle, m, _stream(stream)))

    def diffusion_info(self):
        """(cases solved with the inverse, distinct inverses held, largest Frobenius residual)."""
        n, d = ctypes.c_int32(), ctypes.c_int32()
        r = ctypes.c_double()
        check(lib().sis_geometry_diffusion_info(self.handle, ctypes.byref(n), ctypes.byref(d), ctypes.byref(r)))
        return int(n.value), int(d.value), float(r.value)

    def close(self):
        if getattr(self, "handle", None):
            lib().sis_geometry_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def transport_sweep(plan, geom, rhs, h_half_out, mom_out=None, stream=None):
    check(lib().sis_transport_sweep(plan.handle, geom.handle, _ptr(rhs), _ptr(h_half_out),
                                    _ptr(mom_out), _stream(stream)))


def diffusion_correct(plan, geom, mom_half, amom, N, U_out=None, dU_out=None, stream=None):
    check(lib().sis_diffusion_correct(plan.handle, geom.handle, _ptr(mom_half), _ptr(amom),
                                      float(N), _ptr(U_out), _ptr(dU_out), _stream(stream)))


def solve(plan, geom, scheme="SIS", N=0.0, eps=1e-8, max_it=10000, project=False,
          check_every=4, use_graph=True, stream=None, raise_not_converged=True, refresh_every=0,
          persistent=0):
    """Run sis_solve; returns a dict of numpy arrays (M, Q, iters, residual, U, q).
    persistent: 1 (or a workgroup count) runs the iterations between polls as one
    cooperative launch (planar one-gas FP64 solves)."""
    import numpy as np
    nc, ns, sp = geom.n_cells, geom.n_cases, plan.n_species
    M, Q, res = np.zeros((ns, sp)), np.zeros((ns, sp)), np.zeros(ns)
    it = np.zeros(ns, dtype=np.int32)
    U, q = np.zeros((nc, sp)), np.zeros((nc, sp))
    r = SolveResult(M.ctypes.data_as(_D), Q.ctypes.data_as(_D),
                    it.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), res.ctypes.data_as(_D),
                    U.ctypes.data_as(_D), q.ctypes.data_as(_D), 0.0, 0)
    o = SolveOpts(SCHEME_SIS if scheme == "SIS" else SCHEME_CIS, float(N), float(eps), int(max_it),
                  1 if project else 0, int(check_every), 1 if use_graph else 0, int(refresh_every),
                  int(persistent))
    code = lib().sis_solve(plan.handle, geom.handle, ctypes.byref(o), ctypes.byref(r), _stream(stream))
    if code != SIS_OK and not (code == SIS_E_NOT_CONVERGED and not raise_not_converged):
        check(code)
    if sp == 1:
        M, Q, U, q = M[:, 0], Q[:, 0], U[:, 0], q[:, 0]
    return dict(M=M, Q=Q, iters=it, residual=res, U=U, q=q, seconds=r.seconds,
                total_iters=r.total_iters, status=code)


def _opts(scheme, N, eps, max_it, project, check_every, use_graph, refresh_every=0, persistent=0):
    return SolveOpts(SCHEME_SIS if scheme == "SIS" else SCHEME_CIS, float(N), float(eps),
                     int(max_it), 1 if project else 0, int(check_every), 1 if use_graph else 0,
                     int(refresh_every), int(persistent))


class State:
    """Persistent iteration state of sis_solve (sis_state_* entry points)."""

    def __init__(self, plan, geom, scheme="SIS", N=0.0, eps=1e-8, max_it=10000, project=False,
                 use_graph=True, stream=None, refresh_every=0, persistent=0):
        self.plan, self.geom = plan, geom
        o = _opts(scheme, N, eps, max_it, project, 4, use_graph, refresh_every, persistent)
        h = ctypes.c_void_p()
        check(lib().sis_state_create(plan.handle, geom.handle, ctypes.byref(o), _stream(stream),
                                     ctypes.byref(h)))
        self.handle = h

    def reset(self, stream=None):
        check(lib().sis_state_reset(self.handle, _stream(stream)))

    def step(self, n_iters=1, stream=None):
        check(lib().sis_state_step(self.handle, int(n_iters), _stream(stream)))

    def poll(self, stream=None):
        n = ctypes.c_int32()
        check(lib().sis_state_poll(self.handle, ctypes.byref(n), _stream(stream)))
        return n.value

    def results(self, stream=None, raise_not_converged=False):
        import numpy as np
        nc, ns, sp = self.geom.n_cells, self.geom.n_cases, self.plan.n_species
        M, Q, res = np.zeros((ns, sp)), np.zeros((ns, sp)), np.zeros(ns)
        it = np.zeros(ns, dtype=np.int32)
        U, q = np.zeros((nc, sp)), np.zeros((nc, sp))
        r = SolveResult(M.ctypes.data_as(_D), Q.ctypes.data_as(_D),
                        it.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), res.ctypes.data_as(_D),
                        U.ctypes.data_as(_D), q.ctypes.data_as(_D), 0.0, 0)
        code = lib().sis_state_results(self.handle, ctypes.byref(r), _stream(stream))
        if code not in (SIS_OK, SIS_E_NOT_CONVERGED) or (code != SIS_OK and raise_not_converged):
            check(code)
        if sp == 1:
            M, Q, U, q = M[:, 0], Q[:, 0], U[:, 0], q[:, 0]
        return dict(M=M, Q=Q, iters=it, residual=res, U=U, q=q, total_iters=r.total_iters,
                    status=code)

    def close(self):
        if getattr(self, "handle", None):
            lib().sis_state_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
