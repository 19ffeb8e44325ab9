"""Pins of the polar-coordinate tube oracle (Sec. 4) against what the
mathematics fixes: the free-molecular flow rate of a tube, the hard-sphere
collision frequency, the momentum invariant, the plain collision integral,
and the SIS/CIS fixed point."""
import functools
import math

import numpy as np
from scipy import special

from oracle import direct, polar

FM_TUBE = 4.0 / (3.0 * math.sqrt(math.pi))      # free-molecular tube, lengths in radii


@functools.lru_cache(maxsize=None)
def fsm(nvr, nth, nvz, V, Z, m):
    """Polar FSM with the default box (lattice spacing 1/2)."""
    return polar.PolarFSM(polar.PolarGrid(nvr, V, nth, nvz, Z), m_angle=m)


def test_PT1_free_molecular_tube():
    """delta = 0: the flow rate converges to 4/(3 sqrt pi) = 0.75225 under
    refinement of r and th (the paper's Table 3 prints 0.752); -Q/M equals
    the velocity-quadrature ratio exactly (h factors into a v_r, v_z part
    and a geometric part at delta = 0), which is 1/2 up to quadrature error."""
    errs = []
    for nr, nth in [(20, 16), (40, 32), (80, 64)]:
        g = polar.PolarGrid(16, 4.0, nth, 8, 6.0)
        r = (np.arange(nr) + 1.0) / nr
        M, Q = polar.free_molecular_tube(g, r)
        errs.append(abs(M - FM_TUBE))
        w = g.wvr[:, None] * g.vz[None, :] ** 2 * np.exp(-(g.vr[:, None] ** 2 + g.vz[None, :] ** 2)) / g.vr[:, None]
        ratio = -np.sum(w * (g.vr[:, None] ** 2 + g.vz[None, :] ** 2 - 2.5)) / np.sum(w)
        assert abs(-Q / M - ratio) < 1e-12
        assert abs(ratio - 0.5) < 1e-4
    assert errs[1] < 0.5 * errs[0] and errs[2] < 0.5 * errs[1] and errs[2] < 5e-4


def test_PT2_operator_converges_to_the_boltzmann_operator():
    """The polar FSM (transforms between the polar nodes and the Cartesian
    modes): nubar = 1.25 delta (Sec. 2.5), the hard-sphere closed form of
    nu_eq, the momentum invariant L(v_z f_eq) = 0 and the plain
    sigma-representation integral at three nodes, all improving from the
    coarse to the finer grid (small velocity boxes keep the oracle cheap; the
    production box, |v_r| < 4 and |v_z| < 6, is checked on the GPU against
    the paper's Table 3)."""
    coarse, fine = fsm(6, 8, 4, 3.0, 3.0, 3), fsm(8, 12, 6, 3.0, 3.0, 4)
    out = []
    for f in (coarse, fine):
        g = f.grid
        v = np.sqrt(g.vsq)
        ref = 4 * math.pi * f.b0 * (np.exp(-v ** 2) / math.sqrt(math.pi) + (v + 1 / (2 * v)) * special.erf(v))
        sel = v < 2
        e_nu = np.max(np.abs(f.nu - ref)[sel]) / ref[sel].max()
        e_inv = np.max(np.abs(f.apply(g.VZ * g.feq))) / np.max(np.abs(f.nu * g.VZ * g.feq))
        poly = lambda V: V[..., 2] * (0.3 + 0.5 * V[..., 0] + 0.2 * V[..., 0] ** 2 - 0.1 * V[..., 1] ** 2
                                      + 0.1 * np.sum(V * V, axis=-1))
        V = np.stack([g.V1, g.V2, g.VZ], axis=-1)
        L = f.apply(g.feq * poly(V))
        sc = np.max(np.abs(L))
        e_dir = max(abs(direct.sigma_quadrature_L(V[idx], poly, f.b0, nr=64, nu_ang=(16, 32), ns=(8, 16)) - L[idx]) / sc
                    for idx in [(1, 1, 0), (3, 3, 1), (4, 5, 2)])
        out.append((abs(f.nubar() - 1.25), e_nu, e_inv, e_dir))
    (n0, nu0, i0, d0), (n1, nu1, i1, d1) = out
    assert n1 < 1e-3 and nu1 < 0.04 and i1 < 0.04 and d1 < 0.06
    assert n1 < 0.5 * n0 and nu1 < 0.5 * nu0 and i1 < 0.2 * i0 and d1 < 0.5 * d0


def test_PT3_sis_and_cis_share_the_fixed_point():
    """The polar velocity equation is a moment of the kinetic equation, so SIS
    and CIS converge to the same flow rates up to discretisation error (within
    3% on eight radial nodes), SIS in fewer iterations (delta = 1)."""
    f = fsm(8, 12, 6, 3.0, 3.0, 4)
    r = (np.arange(8) + 1.0) / 8
    rs = polar.solve_tube(f, r, 1.0, "SIS", eps=1e-9, max_it=300)
    rc = polar.solve_tube(f, r, 1.0, "CIS", eps=1e-9, max_it=300)
    assert rs["converged"] and rc["converged"]
    assert rs["iters"] < 0.8 * rc["iters"]
    assert abs(rs["M"] - rc["M"]) < 0.03 * rc["M"]
    assert abs(rs["Q"] - rc["Q"]) < 0.03 * abs(rc["Q"])
