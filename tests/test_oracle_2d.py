"""Pins of the 2-D oracle (quarter ducts, periodic porous cells)."""
import json
import math
import os

import numpy as np
import pytest

from oracle import collision, duct
from oracle.velocity import POISEUILLE, TRANSPIRATION, VelocityGrid
from paper_1612_04488_amd import inputs

GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


class FreeMolecular:
    """delta = 0: the collision term vanishes; only nu and the grid are used."""

    def __init__(self, grid):
        self.grid = grid
        self.nu = np.ones_like(grid.feq)

    def lplus(self, h):
        return np.zeros_like(h)

    def nubar(self):
        return 1.0


def test_free_molecular_square_duct_reproduces_table2():
    """delta = 0, square duct: the scheme's flow rates converge like 1/N in the
    velocity grid; extrapolating N = 32, 48 gives Table 2's M_P = 0.419,
    -Q_P = 0.210 and Q_T = 9/4 M_P (closed form 0.41936); M_T = Q_P exactly."""
    g = duct.duct_quarter(8, 8, ratio=1.0)
    res = {}
    for N in (32, 48):
        op = FreeMolecular(VelocityGrid(N, 4.0))
        rP = duct.solve_2d(op, g, 0.0, POISEUILLE, "CIS", eps=1e-12, max_it=3)
        rT = duct.solve_2d(op, g, 0.0, TRANSPIRATION, "CIS", eps=1e-12, max_it=3)
        assert abs(rT["M"] - rP["Q"]) < 1e-14
        res[N] = (rP["M"], rP["Q"], rT["Q"])
    ext = [(48 * a - 32 * b) / 16 for a, b in zip(res[48], res[32])]
    t2 = GOLDEN["table2_square_duct_free_molecular"]
    assert abs(ext[0] - 0.41936) < 1e-3 * 0.41936
    assert abs(ext[0] - t2["M_P"]) < 1e-3
    assert abs(-ext[1] - t2["minus_Q_P"]) < 1e-3
    assert abs(ext[2] / ext[0] - 2.25) < 2e-3


def test_periodic_sweep_preserves_uniform_state():
    """Periodic cell without solids: a spatially uniform right side and the
    matching uniform previous iterate are a fixed point of the sweep (every
    upwind difference of a constant vanishes, across the wrapped edge too)."""
    vg = VelocityGrid(6, 4.0)
    g = duct.periodic_cell(np.zeros((5, 7), bool))
    nu = 1.0 + 0.1 * vg.vsq
    rng = np.random.default_rng(3)
    r1 = rng.standard_normal(vg.feq.shape)
    rhs = np.broadcast_to(r1, (35,) + r1.shape).copy()
    h0 = rhs / nu
    h = duct.sweep_2d(rhs, nu, g, vg, h0)
    assert np.max(np.abs(h - h0)) < 1e-14


def test_duct_sweep_zero_right_side_gives_zero():
    vg = VelocityGrid(6, 4.0)
    g = duct.duct_quarter(4, 5)
    h = duct.sweep_2d(np.zeros((20,) + vg.feq.shape), np.ones_like(vg.feq), g, vg,
                      np.ones((20,) + vg.feq.shape))
    assert np.max(np.abs(h)) == 0.0


def ns_square_mean_velocity():
    """Mean of U with lap U = -1, U = 0 on the unit square (Fourier series)."""
    s = sum(math.tanh(n * math.pi / 2) / n ** 5 for n in range(1, 200, 2))
    return (1.0 - 192.0 / math.pi ** 5 * s) / 12.0


def test_duct_sis_matches_cis_and_ns_limit():
    """SIS and CIS agree up to discretisation error in the square duct, and
    kappa = M/delta approaches the Navier-Stokes value 0.03514 from above."""
    f = collision.ProjectedFSM(collision.FSM(VelocityGrid(8, 4.0), m_angle=4))
    g = duct.duct_quarter(6, 6)
    rs = duct.solve_2d(f, g, 1.0, POISEUILLE, "SIS", eps=1e-8)
    rc = duct.solve_2d(f, g, 1.0, POISEUILLE, "CIS", eps=1e-8)
    assert rs["converged"] and rc["converged"]
    assert abs(rs["M"] - rc["M"]) < 0.02 * abs(rc["M"])
    # the Navier-Stokes limit is a property of any operator with this viscosity:
    # the (cheaper) BGK form with collision frequency delta
    from oracle import modes
    r100 = duct.solve_2d(modes.BGKOperator(VelocityGrid(8, 4.0)), g, 100.0, POISEUILLE, "SIS", eps=1e-8,
                         max_it=400)
    kap = r100["M"] / 100.0
    ref = ns_square_mean_velocity()
    assert abs(ref - 0.035144) < 2e-6
    assert ref < kap < 1.15 * ref


def test_duct_sis_iterations_at_resolution():
    """With the Dirichlet layer thin (32 x 32 geometric cells) SIS converges at
    delta = 100 in a few tens of iterations (Table 2: 40 at 50 x 50), CIS not."""
    from oracle import modes
    b = modes.BGKOperator(VelocityGrid(8, 4.0))
    g = duct.duct_quarter(32, 32)
    r = duct.solve_2d(b, g, 100.0, POISEUILLE, "SIS", eps=1e-8, max_it=200)
    assert r["converged"] and r["iters"] < 60
    rc = duct.solve_2d(b, g, 100.0, POISEUILLE, "CIS", eps=1e-8, max_it=60)
    assert not rc["converged"]


def test_porous_generator():
    mask, discs = inputs.porous_discs(128)
    assert abs(mask.mean() - 0.4) < 2e-3
    rs = [r for _, r in discs]
    assert max(rs) <= 0.1 + 1e-12 and min(rs) >= 0.01 - 1e-12
    for a in range(len(discs)):
        for b in range(a + 1, len(discs)):
            d = np.abs(discs[a][0] - discs[b][0])
            d = np.minimum(d, 1 - d)
            assert np.hypot(*d) >= discs[a][1] + discs[b][1]
    m2, _ = inputs.porous_discs(128)
    assert np.array_equal(mask, m2)


def test_sierpinski_carpet_geometry():
    """Sec. 3.1 carpets: porosity (8/9)^level exactly, each level keeps the
    solids of the previous one, and the quarter is symmetric about its diagonal."""
    for level, cells in inputs.SIERPINSKI_CELLS.items():
        f1, f2, s = inputs.sierpinski_quarter(level, cells)
        assert len(f1) == cells + 1 and f1[0] == -0.5 and f1[-1] == 0.0
        assert abs((1.0 - s.mean()) - (8.0 / 9.0) ** level) < 1e-14
        assert np.array_equal(s, s.T)
        if level > 0:
            prev = inputs.sierpinski_quarter(level - 1, cells)[2]
            assert np.all(s[prev])
    # level 1: the central square of side 1/3 is the corner [-1/6, 0]^2 of the quarter
    s = inputs.sierpinski_quarter(1, 6)[2]
    assert s[4:, 4:].all() and s.sum() == 4
    with pytest.raises(ValueError):
        inputs.sierpinski_quarter(2, 10)


def test_free_molecular_sierpinski_ratios():
    """delta = 0 on the level-1 carpet: M_T = Q_P exactly (the scheme keeps
    Onsager's reciprocity), and the geometry-independent ratios of the
    free-molecular limit, -Q_P/M_P = 1/2 and Q_T/M_P = 9/4 (the velocity
    integrals factor out of the path-length integral), hold after
    extrapolating N = 32, 48; the carpet passes less gas than the plain duct."""
    f1, f2, s = inputs.sierpinski_quarter(1, 6)
    bc = (duct.WALL, duct.SYM, duct.WALL, duct.SYM)
    g = duct.Grid2D(f1, f2, bc, s)
    g0 = duct.Grid2D(f1, f2, bc)
    res = {}
    for N in (32, 48):
        op = FreeMolecular(VelocityGrid(N, 4.0))
        rP = duct.solve_2d(op, g, 0.0, POISEUILLE, "CIS", eps=1e-12, max_it=3)
        rT = duct.solve_2d(op, g, 0.0, TRANSPIRATION, "CIS", eps=1e-12, max_it=3)
        assert abs(rT["M"] - rP["Q"]) < 1e-14
        res[N] = (rP["M"], rP["Q"], rT["Q"])
        if N == 32:
            r0 = duct.solve_2d(op, g0, 0.0, POISEUILLE, "CIS", eps=1e-12, max_it=3)
            assert rP["M"] < 0.7 * r0["M"]
    M, Q, QT = [(48 * a - 32 * b) / 16 for a, b in zip(res[48], res[32])]
    assert abs(-Q / M - 0.5) < 5e-3
    assert abs(QT / M - 2.25) < 1e-2
