"""Host-side checks of libsis.so that need no GPU: the library loads and
exports every entry point of include/sis.h, the host planner's tables equal
the oracle's, and argument validation fails before any device work."""
import ctypes
import os
import re

import numpy as np
import pytest

from oracle import collision
from oracle.velocity import VelocityGrid
from paper_1612_04488_amd import sis

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "sis.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sis_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = sis.lib()
    names = declared_symbols()
    assert len(names) >= 14
    for n in names:
        assert hasattr(L, n), n
    assert L.sis_version() == 100


@pytest.mark.parametrize("n_v,l_v,m,kernel", [(8, 4.0, 4, "hs"), (16, 6.0, 6, "hs"),
                                               (12, 4.0, 4, "ipl")])
def test_host_tables_equal_oracle(n_v, l_v, m, kernel):
    """T1: planner feq, nu_eq, A_p, B_p, b0, nubar == oracle to ~1e-14."""
    d = sis.velocity_desc(n_v, l_v, m_angle=m, kernel=kernel, visc_index=0.81)
    t = sis.host_tables(d)
    alpha = 1.0 if kernel == "hs" else collision.ipl_alpha(0.81)
    f = collision.FSM(VelocityGrid(n_v, l_v), m_angle=m, alpha=alpha)
    D = m * m
    assert abs(t["b0"] - f.b0) < 1e-15 * f.b0
    assert abs(t["nubar"] - f.nubar()) < 1e-13
    assert np.max(np.abs(t["feq"] - f.grid.feq.ravel())) < 1e-16
    tol = 2e-14 if kernel == "hs" else 5e-13
    assert np.max(np.abs(t["nu"] - f.nu.ravel())) < tol * np.max(np.abs(f.nu))
    assert np.max(np.abs(t["A"] - f.A.reshape(D, -1))) < tol * np.max(np.abs(f.A))
    assert np.max(np.abs(t["B"] - f.B.reshape(D, -1))) < tol * np.max(np.abs(f.B))


@pytest.mark.parametrize("kw,msg", [
    (dict(n_v=7), "n_v"), (dict(n_v=16, l_v=-1.0), "l_v"), (dict(n_v=16, n_pad=10), "n_pad"),
    (dict(n_v=16, m_angle=0), "m_angle"), (dict(n_v=16, kernel="ipl", visc_index=2.0), "viscosity"),
])
def test_plan_validation_happens_before_device_work(kw, msg):
    """T2: invalid descriptors are rejected on the host with a message."""
    d = sis.velocity_desc(**kw)
    h = ctypes.c_void_p()
    code = sis.lib().sis_plan_create(ctypes.byref(d), None, ctypes.byref(h))
    assert code == sis.SIS_E_INVALID
    assert msg in sis.lib().sis_last_error().decode()
    assert not h.value


def test_null_handles_rejected():
    L = sis.lib()
    assert L.sis_collide(None, 1, None, None, None, None, 0, None, None, None, None) == sis.SIS_E_INVALID
    assert L.sis_plan_destroy(None) == sis.SIS_E_INVALID
    assert L.sis_geometry_cells(None) == -1
    assert "null" in L.sis_last_error().decode()


def test_inputs_module_is_seeded():
    from paper_1612_04488_amd import inputs
    a = inputs.smooth_h(8, 4.0, 3)
    b = inputs.smooth_h(8, 4.0, 3)
    assert np.array_equal(a, b) and a.shape == (3, 8, 8, 8)
    # odd in v3 by construction
    assert np.allclose(a, -a[..., ::-1], atol=0.0)
    assert np.array_equal(inputs.nodes_tanh(100), inputs.nodes_tanh(100))


@pytest.mark.parametrize("n_v,l_v,m,chi", [(8, 4.0, 4, (0.5, 0.5)), (12, 4.5, 6, (0.1, 0.9))])
def test_mixture_host_tables_equal_oracle(n_v, l_v, m, chi):
    """Mixture planner: f_a, nu_a (scaled by the mixture viscosity) and N_a == oracle."""
    from oracle import mixture
    mx = dict(masses=(20.18, 39.95), diameters=(0.72, 1.0), chi=chi, m_rho=4)
    t = sis.host_tables(sis.velocity_desc(n_v, l_v, m_angle=m, mixture=mx))
    o = mixture.MixtureFSM(VelocityGrid(n_v, l_v), mx["masses"], mx["diameters"], chi, m_angle=m, m_rho=4)
    assert np.max(np.abs(t["feq"] - o.feq.reshape(2, -1))) < 1e-16
    assert np.max(np.abs(t["nu"] - o.nu.reshape(2, -1))) < 2e-14 * np.max(np.abs(o.nu))
    assert np.allclose(t["nubar"], o.nubar(), rtol=1e-13, atol=0)


@pytest.mark.parametrize("mx,msg", [
    (dict(masses=(1.0, -1.0), diameters=(1.0, 1.0), chi=(0.5, 0.5)), "mass"),
    (dict(masses=(1.0, 2.0), diameters=(1.0, 1.0), chi=(0.5, 0.6)), "chi"),
    (dict(masses=(1.0, 2.0), diameters=(0.0, 1.0), chi=(0.5, 0.5)), "diam"),
])
def test_mixture_validation(mx, msg):
    d = sis.velocity_desc(8, 4.0, m_angle=4, mixture=mx)
    h = ctypes.c_void_p()
    assert sis.lib().sis_plan_create(ctypes.byref(d), None, ctypes.byref(h)) == sis.SIS_E_INVALID
    assert msg in sis.lib().sis_last_error().decode()
    d = sis.velocity_desc(8, 4.0, m_angle=4, kernel="ipl",
                          mixture=dict(masses=(1.0, 2.0), diameters=(1.0, 1.0), chi=(0.5, 0.5)))
    assert sis.lib().sis_plan_create(ctypes.byref(d), None, ctypes.byref(h)) == sis.SIS_E_UNSUPPORTED
