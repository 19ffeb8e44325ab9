"""Pins of the binary-mixture oracle (Sec. 5) against what the mathematics fixes.

The paper prints neither the mixture FSM nor the viscosity used for delta;
these tests pin the oracle's reading against exact reductions, detailed
balance, conservation, textbook closed forms and a brute-force collision
integral, none of which share the FSM's construction.
"""
import math

import numpy as np
import pytest
from scipy import special

from oracle import collision, direct, mixture, solver
from oracle import transport as tr
from oracle.velocity import VelocityGrid

NEAR = mixture.NE_AR
_cache = {}


def mix(n, lv, m, mr, chi=(0.5, 0.5), masses=NEAR["masses"], diameters=NEAR["diameters"]):
    key = (n, lv, m, mr, tuple(chi), tuple(masses), tuple(diameters))
    if key not in _cache:
        _cache[key] = mixture.MixtureFSM(VelocityGrid(n, lv), masses, diameters, chi, m_angle=m, m_rho=mr)
    return _cache[key]


def test_M1_identical_species_reduce_to_one_gas():
    """Equal masses and diameters: L_a(chi_A h, chi_B h) = chi_a L(h) of the one-gas
    operator exactly, nu_a and N_a equal the one-gas values, the viscosity factor
    is 1, and the CIS fixed point gives M_A = M_B = M and Q_a = chi_a Q."""
    g = VelocityGrid(8, 4.0)
    op = mixture.MixtureFSM(g, (4.0, 4.0), (1.0, 1.0), (0.3, 0.7), m_angle=4, m_rho=4)
    one = collision.FSM(g, m_angle=4)
    assert abs(op.scale - 1.0) < 1e-15
    h = np.random.default_rng(0).standard_normal(g.feq.shape) * g.feq
    L2 = op.apply(np.stack([0.3 * h, 0.7 * h]))
    L1 = one.apply(h)
    sc = np.abs(L1).max()
    assert np.abs(L2[0] - 0.3 * L1).max() < 1e-13 * sc
    assert np.abs(L2[1] - 0.7 * L1).max() < 1e-13 * sc
    assert np.allclose(op.nubar(), one.nubar(), rtol=1e-13, atol=0)
    x = tr.nodes_uniform(4)
    r2 = mixture.solve_mixture_1d(op, x, 1.0, scheme="CIS", eps=1e-11, max_it=400)
    r1 = solver.solve_1d(one, x, 1.0, scheme="CIS", eps=1e-11)
    assert np.allclose(r2["M"], r1.M, rtol=1e-9, atol=0)
    assert np.allclose(r2["Q"], [0.3 * r1.Q, 0.7 * r1.Q], rtol=1e-9, atol=0)


def test_M2_free_molecular_planar_exact():
    """delta = 0: the upwind scheme solves v1 dh_a/dx1 = v3 f_a exactly, so the
    solver must return the discrete closed form of every species' flow rates."""
    op = mix(8, 4.0, 4, 4)
    r = mixture.solve_mixture_1d(op, tr.nodes_tanh(10), 0.0, eps=1e-13, max_it=5)
    M, Q = mixture.free_molecular_1d(op)
    assert np.allclose(r["M"], M, rtol=1e-12, atol=0)
    assert np.allclose(r["Q"], Q, rtol=1e-12, atol=0)
    assert M[0] > M[1] > 0          # the lighter species flows faster


def _balance_and_invariants(op):
    g = op.grid
    errs = []
    for a in range(2):
        for b in range(2):
            gain = op.gain(a, b, op.Fhat[a], op.Fhat[b])       # Q+_ab(f_a, f_b)
            loss = op.feq[a] * op.nu_ab[a, b]
            errs.append(np.abs(gain - loss).max() / np.abs(loss).max())
    # collision invariants: per-species number, common velocity, common temperature
    h = np.stack([op.feq[s] * (0.3 * (s + 1) + op.a[s] * (0.2 * g.V1 - 0.1 * g.V3)
                               + 0.15 * op.a[s] * g.vsq) for s in range(2)])
    inv = np.abs(op.apply(h)).max() / np.abs(op.nu * h).max()
    return max(errs), inv


def test_M3_detailed_balance_and_collision_invariants():
    """Q+_ab(f_a, f_b) = f_a nu_ab pointwise (detailed balance of Maxwellians at a
    common temperature) and L annihilates f_a (c_a + a_a u.v + a_a T |v|^2): both
    exact for the Boltzmann operator; the FSM error must fall under refinement.
    A wrong Carleman shift, Jacobian or mass factor breaks both at O(1)."""
    b12, i12 = _balance_and_invariants(mix(12, 4.5, 6, 12))
    b16, i16 = _balance_and_invariants(mix(16, 5.0, 6, 16))
    assert b16 < 1e-2 and i16 < 1e-2
    assert b16 < 0.5 * b12 and i16 < 0.5 * i12


def test_M4_collision_frequency_closed_form():
    """Hard spheres: nu_ab(v) = 4 pi b_ab chi_b [e^{-a v^2}/sqrt(pi a) +
    (|v| + 1/(2 a |v|)) erf(sqrt(a) |v|)], a = m_b/m_A (mean relative speed
    against a Maxwellian); the error falls under velocity refinement."""
    errs = []
    for n, m in [(16, 6), (24, 8)]:
        op = mix(n, 5.0, m, 4)
        g = op.grid
        v = np.sqrt(g.vsq)
        sel = v < 3.0
        e = 0.0
        for a in range(2):
            for b in range(2):
                ab = op.a[b]
                cf = op.chi[b] * (np.exp(-ab * v ** 2) / np.sqrt(math.pi * ab)
                                  + (v + 1.0 / (2.0 * ab * v)) * special.erf(np.sqrt(ab) * v))
                cf *= math.pi * op.C[a, b]          # 4 pi b_ab
                e = max(e, np.abs(op.nu_ab[a, b] - cf)[sel].max() / cf[sel].max())
        errs.append(e)
    assert errs[1] < 5e-3
    assert errs[1] < 0.5 * errs[0]


def test_M5_viscosity_closed_form_matches_operator():
    """The delta normalisation uses the textbook first Chapman-Enskog viscosity
    of a hard-sphere mixture; the Galerkin shear bracket of the discrete
    operator must reproduce it (plausible slips in the closed form -- the sign or
    factor 2 of the cross term, the reduced mass -- move it by > 15%)."""
    op = mix(20, 5.0, 6, 12)
    vr, _ = op.shear_bracket()
    ref = mixture.viscosity_ratio(op.m, op.d, op.chi)
    assert abs(vr - ref) < 1.5e-2 * ref
    assert abs(mixture.viscosity_ratio((3.0, 3.0), (1.0, 1.0), (0.2, 0.8)) - 1.0) < 1e-14


def _pA(V):
    v1, v2, v3 = V[..., 0], V[..., 1], V[..., 2]
    return v1 * v2 + 0.3 * v3 * (np.sum(V * V, axis=-1) - 2.5) + 0.2 * v1 ** 2


def _pB(V):
    v1, v2, v3 = V[..., 0], V[..., 1], V[..., 2]
    return 0.5 * v1 * v3 - 0.2 * v2 + 0.1 * np.sum(V * V, axis=-1) * v3


def test_M6_fsm_matches_direct_collision_integral():
    """Mixture FSM L_a(f p) vs the plain sigma-representation integral of the
    linearized operator (unequal-mass post-collision velocities, no Carleman
    form, no truncation, no FFT)."""
    op = mix(16, 5.0, 6, 16)
    g = op.grid
    V = np.stack([g.V1, g.V2, g.V3], axis=-1)
    L = op.apply(np.stack([op.feq[0] * _pA(V), op.feq[1] * _pB(V)]))
    for a in range(2):
        sc = np.abs(L[a]).max()
        for idx in [(7, 8, 9), (9, 5, 8), (10, 10, 7)]:
            v = np.array([g.v1d[i] for i in idx])
            ref = direct.sigma_quadrature_mix_L(v, a, (_pA, _pB), op.m, op.d, op.chi, op.b0, op.scale,
                                                nr=64, nu_ang=(16, 32), ns=(8, 16))
            assert abs(ref - L[a][idx]) < 2e-2 * sc, (a, idx, ref, L[a][idx])


def test_M7_sis_and_cis_share_the_fixed_point_up_to_discretisation():
    """The SIS velocity equations (B: own shear stress; A: total stress x1 minus
    B's) are moments of the kinetic equation, so SIS and CIS converge to the same
    flow rates up to discretisation error, which must shrink under velocity
    refinement (species of equal mass, so the solves stay cheap; a wrong sign of
    P_B13 or of the penalty moves the SIS fixed point at O(1))."""
    gaps = []
    for n, lv in [(8, 4.0), (12, 4.5)]:
        op = mixture.MixtureFSM(VelocityGrid(n, lv), (4.0, 4.0), (1.0, 1.0), (0.3, 0.7), m_angle=4, m_rho=4)
        x = tr.nodes_uniform(4)
        rs = mixture.solve_mixture_1d(op, x, 1.0, eps=1e-10, max_it=300)
        rc = mixture.solve_mixture_1d(op, x, 1.0, scheme="CIS", eps=1e-10, max_it=300)
        assert rs["converged"] and rc["converged"]
        assert rs["iters"] < rc["iters"]
        gaps.append(np.max(np.abs(rs["M"] - rc["M"]) / rc["M"]))
    assert gaps[1] < 3e-2
    assert gaps[1] < 0.3 * gaps[0]


# ------------------------------------------------------------------ rectangular ducts (Table 5)
def test_MD1_identical_species_in_a_duct_reduce_to_one_gas():
    """Cross-section CIS of a mixture of identical species: M_A = M_B = M and
    Q_a = chi_a Q of the one-gas 2-D solve, exactly (collide, 2-D sweep and
    moments of each species, flow rates)."""
    from oracle import duct
    from oracle.velocity import POISEUILLE
    g = duct.duct_quarter(3, 4, ratio=1.0)
    vg = VelocityGrid(8, 4.0)
    op = mixture.MixtureFSM(vg, (4.0, 4.0), (1.0, 1.0), (0.3, 0.7), m_angle=4, m_rho=4)
    r2 = mixture.solve_mixture_2d(op, g, 1.0, scheme="CIS", eps=1e-9, max_it=200)
    r1 = duct.solve_2d(collision.FSM(vg, m_angle=4), g, 1.0, POISEUILLE, "CIS", eps=1e-9, max_it=200)
    assert r2["iters"] == r1["iters"]
    assert np.allclose(r2["M"], r1["M"], rtol=1e-12, atol=0)
    assert np.allclose(r2["Q"], [0.3 * r1["Q"], 0.7 * r1["Q"]], rtol=1e-12, atol=0)


def test_MD2_species_velocity_equations_sum_to_the_mixture_equation():
    """With N_A = N_B m_A/m_B the pressure-gradient terms of species B cancel
    between eqs. LBE2_true2 and LBE2_true1, so chi_A U_A + chi_B U_B solves the
    single-gas velocity equation with the summed moments (G, A) and wall
    values U3_A + U3_B: an exact identity of the discrete (linear) solves that
    fixes the sign and scale of every div P_B term, the source of A and the
    placement of chi."""
    from oracle import duct
    op = mix(8, 4.0, 4, 3)
    solid = np.zeros((5, 6), bool)
    solid[2, 3] = True
    g = duct.Grid2D(duct.geometric_faces(5, 0.5, 1.1), duct.geometric_faces(6, 0.5, 1.0),
                    (duct.WALL, duct.SYM, duct.WALL, duct.SYM), solid)
    nf = len(g.cells)
    rng = np.random.default_rng(17)
    mom = rng.standard_normal((nf, 2, 7))
    amom = rng.standard_normal((nf, 2, 4))
    delta, NB = 2.5, 1.3
    N = (NB / op.a[1], NB)
    U = mixture.velocity_2d(op, g, mom, amom, delta, N)
    msum = np.zeros((nf, 7))
    msum[:, 0] = mom[:, 0, 0] + mom[:, 1, 0]
    msum[:, 2:5] = mom[:, 0, 2:5] + mom[:, 1, 2:5]
    asum = np.zeros((nf, 4))
    for s in range(2):
        asum[:, 0] += amom[:, s, 0] + N[s] * delta * amom[:, s, 1]
        asum[:, 2] += amom[:, s, 2] + N[s] * delta * amom[:, s, 3]
    ref = duct.diffusion_2d(g, msum, asum, delta, N[0], duct.POISEUILLE)
    lhs = op.chi[0] * U[:, 0] + op.chi[1] * U[:, 1]
    assert np.max(np.abs(lhs - ref)) < 1e-11 * np.max(np.abs(ref))
