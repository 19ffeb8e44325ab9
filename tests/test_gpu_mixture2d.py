"""GPU parity of the binary mixture on 2-D cross sections (Sec. 5.3, Table 5)
against the CPU oracle, through the C ABI.

Same seeded inputs on both sides: sweep and moments of both species <= 1e-12
relative, the two velocity equations <= 1e-10, full SIS/CIS solves with
identical iteration counts and flow rates <= 1e-10; parity storage equals the
full grid; the SIS and CIS fixed points approach each other under velocity
refinement; the production resolution against the paper's Table 5.
"""
import functools
import json
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import duct, mixture
from oracle.velocity import VelocityGrid
from paper_1612_04488_amd import inputs, sis

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
NEAR = inputs.MIX_NEAR["mixture"]
GOLDEN = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def say(*a):
    print("[gpu-mix2d]", *a, flush=True)
    sys.stdout.flush()


def dev(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


CFG = (8, 4.0, 3, 3, (0.5, 0.5))


@functools.lru_cache(maxsize=None)
def oracle_mix(n, lv, m, mr, chi):
    return mixture.MixtureFSM(VelocityGrid(n, lv), NEAR["masses"], NEAR["diameters"], chi, m_angle=m, m_rho=mr)


@functools.lru_cache(maxsize=None)
def gpu_mix(n, lv, m, mr, chi, parity=1):
    say("mixture plan", n, lv, m, mr, chi, parity)
    return sis.Plan(n, lv, m_angle=m, parity=parity,
                    mixture=dict(masses=NEAR["masses"], diameters=NEAR["diameters"], chi=chi, m_rho=mr))


def small_cases(kind):
    if kind == "duct":
        return [(inputs.duct_faces(4, 0.5), inputs.duct_faces(5, 1.0), None),
                (inputs.duct_faces(3, 0.5), inputs.duct_faces(3, 0.5), None)]
    m = np.zeros((6, 5), bool)
    m[2:4, 1:3] = True
    return [(np.linspace(0, 1, 7), np.linspace(0, 1, 6), m)]


def oracle_grid(kind, c):
    if kind == "duct":
        return duct.Grid2D(c[0], c[1], (duct.WALL, duct.SYM, duct.WALL, duct.SYM))
    return duct.Grid2D(c[0], c[1], (duct.PERIODIC,) * 4, c[2])


def full_h(n, h_stored):
    """Stored (v3 > 0) half of a field odd in v3 -> the full grid."""
    return np.concatenate([-h_stored[..., ::-1], h_stored], axis=-1)


@pytest.mark.parametrize("kind", ["duct", "periodic"])
def test_mix2d_sweep_moments_velocity_parity(kind):
    say("sweep/moments/velocity", kind)
    p, o = gpu_mix(*CFG), oracle_mix(*CFG)
    n = CFG[0]
    cases = small_cases(kind)
    deltas = [0.4, 3.0][:len(cases)]
    geom = sis.Geometry2D(p, kind, cases, deltas, [1] * len(cases))
    assert geom.diffusion_info()[0] == len(cases)
    nc = geom.n_cells
    rng = np.random.default_rng(31)
    odd = lambda x: 0.5 * (x - x[..., ::-1])                   # the part odd in v3
    rhs = odd(inputs.mixture_h(n, CFG[1], nc, rough=True))
    hprev = odd(inputs.mixture_h(n, CFG[1], nc, rough=True, seed=77))
    hv = n // 2
    hd = dev(hprev[..., hv:].reshape(nc, -1))
    mom = torch.empty((nc, 2, 8), dtype=torch.float64, device=DEV)
    sis.transport_sweep(p, geom, dev(rhs[..., hv:].reshape(nc, -1)), hd, mom)
    amom = rng.standard_normal((nc, 2, 4)) * 0.1
    U = torch.empty((nc, 2), dtype=torch.float64, device=DEV)
    dU = torch.empty((nc, 2), dtype=torch.float64, device=DEV)
    Npen = 1.4
    sis.diffusion_correct(p, geom, mom, dev(amom), Npen, U, dU)
    torch.cuda.synchronize()
    h_g = full_h(n, hd.cpu().numpy().reshape(nc, 2, n, n, hv))
    mom, U, dU = mom.cpu().numpy(), U.cpu().numpy(), dU.cpu().numpy()
    for c, case in enumerate(cases):
        g = oracle_grid(kind, case)
        a, b = geom.offsets[c], geom.offsets[c + 1]
        h_o = mixture.sweep_2d(o, rhs[a:b], g, deltas[c], hprev[a:b])
        assert rel(h_g[a:b], h_o) < 1e-12, c
        m_o = mixture.moments_2d(o, h_o)
        for k in range(7):
            assert rel(mom[a:b, :, k], m_o[:, :, k]) < 1e-12, (c, k)
        U_o = mixture.velocity_2d(o, g, m_o, amom[a:b], deltas[c], (Npen, Npen))
        assert rel(U[a:b], U_o) < 1e-10, c
        assert rel(dU[a:b], U_o - m_o[:, :, 0] / o.chi) < 1e-9, c


@pytest.mark.parametrize("scheme", ["SIS", "CIS"])
def test_mix2d_solve_matches_oracle(scheme):
    p, o = gpu_mix(*CFG), oracle_mix(*CFG)
    case = small_cases("duct")[1]
    for delta in (0.5, 2.0):
        geom = sis.Geometry2D(p, "duct", [case], [delta], [1])
        r = sis.solve(p, geom, scheme=scheme, eps=1e-10, max_it=400)
        ro = mixture.solve_mixture_2d(o, oracle_grid("duct", case), delta, scheme=scheme, eps=1e-10, max_it=400)
        say(scheme, delta, r["M"][0], ro["M"], r["iters"][0], ro["iters"])
        assert ro["converged"]
        assert int(r["iters"][0]) == ro["iters"]
        assert rel(r["M"][0], ro["M"]) < 1e-10 and rel(r["Q"][0], ro["Q"]) < 1e-10
        assert rel(r["U"], ro["U"]) < 1e-10


def test_mix2d_parity_storage_equals_full_grid_and_graph():
    cases = small_cases("duct")
    out = []
    for parity in (0, 1):
        p = gpu_mix(*CFG, parity=parity)
        geom = sis.Geometry2D(p, "duct", cases, [0.3, 4.0], [1, 1])
        out.append(sis.solve(p, geom, eps=1e-10, max_it=400))
        if parity == 1:
            eager = sis.solve(p, geom, eps=1e-10, max_it=400, use_graph=False)
            assert np.array_equal(eager["M"], out[-1]["M"]) and np.array_equal(eager["iters"], out[-1]["iters"])
    assert np.array_equal(out[0]["iters"], out[1]["iters"])
    assert rel(out[1]["M"], out[0]["M"]) < 1e-12 and rel(out[1]["Q"], out[0]["Q"]) < 1e-12


def test_mix2d_rejects_cg():
    p = gpu_mix(*CFG)
    geom = sis.Geometry2D(p, "duct", small_cases("duct")[:1], [1.0], [1])
    with pytest.raises(sis.SisError):
        geom.diffusion_solver("cg")
    with pytest.raises(sis.SisError):
        sis.Geometry2D(p, "duct", small_cases("duct")[:1], [1.0], [2])     # transpiration


def test_mix2d_sis_and_cis_fixed_points_converge():
    """The SIS velocity equations are moments of the kinetic equation, so the
    SIS and CIS fixed points differ only by discretisation error, which falls
    as the velocity grid is refined (Ne-Ar, square duct, delta = 2)."""
    case = (inputs.duct_faces(8, 0.5), inputs.duct_faces(8, 0.5), None)
    gaps = []
    for n, lv, m, mr in [(8, 4.0, 4, 4), (12, 4.5, 6, 8), (16, 5.0, 6, 8)]:
        p = gpu_mix(n, lv, m, mr, (0.5, 0.5))
        geom = sis.Geometry2D(p, "duct", [case], [2.0], [1])
        rs = sis.solve(p, geom, eps=1e-10, max_it=2000)
        rc = sis.solve(p, geom, scheme="CIS", eps=1e-10, max_it=2000)
        gap = float(np.max(np.abs(rs["M"][0] - rc["M"][0]) / rc["M"][0]))
        say("n", n, "SIS", rs["M"][0], rs["iters"][0], "CIS", rc["M"][0], rc["iters"][0], "gap", gap)
        gaps.append(gap)
    assert gaps[2] < 0.5 * gaps[0] and gaps[2] < 2e-2


def test_mix2d_table5_square_duct():
    """Production resolution (24^3 velocities on [-5, 5]^3 with v3 > 0 stored,
    M = 8, 16 rho nodes; 64^2 quarter cells growing by 1.05 from the wall),
    N_a = 1.5 and eps = 1e-7 as in Table 5, aspect ratio 1.  Near the
    continuum (delta = 10) both species flow like the single gas on the same
    grid (within 3%), as the paper states for the planar mixture; against
    Table 5 the flow rates agree within 4% at delta = 1 and 6% at delta = 10
    (the table's near-continuum values sit 2-9% below the paper's own
    single-gas Table 2, which the single-gas path reproduces within 0.5% at
    delta = 10) and within 15% at delta = 0.1 (the uniform 24-point velocity
    grid under-resolves the grazing molecules there, for one gas as well);
    iteration counts within twice the paper's."""
    w = inputs.MIX_NEAR
    say("Table 5")
    p = sis.Plan(w["n_v"], w["l_v"], n_pad=w["n_pad"], m_angle=w["m_angle"], mixture=w["mixture"], parity=1)
    rows = [r for r in GOLDEN["table5_duct_near_chi05"]["aspect_1"] if r[0] in (0.1, 1.0, 10.0)]
    case = (inputs.duct_faces(64, 0.5), inputs.duct_faces(64, 0.5), None)
    geom = sis.Geometry2D(p, "duct", [case] * len(rows), [r[0] for r in rows], [1] * len(rows))
    assert geom.diffusion_info()[:2] == (len(rows), 1)
    r = sis.solve(p, geom, N=1.5, eps=1e-7, max_it=300)
    p1 = sis.Plan(w["n_v"], w["l_v"], n_pad=w["n_pad"], m_angle=w["m_angle"], parity=1)
    one = sis.solve(p1, sis.Geometry2D(p1, "duct", [case], [10.0], [1]), eps=1e-9, max_it=300)
    say("single gas, delta 10:", one["M"][0])
    for c, row in enumerate(rows):
        say("delta", row[0], "iters", r["iters"][c], "paper", row[1], "M", r["M"][c], "paper", row[2:4],
            "-2Q", -2 * r["Q"][c], "paper", row[4:6])
    for c, row in enumerate(rows):
        tol = {0.1: 0.15, 1.0: 0.04, 10.0: 0.06}[row[0]]
        assert abs(r["M"][c][0] - row[2]) < tol * row[2]
        assert abs(r["M"][c][1] - row[3]) < tol * row[3]
        assert r["iters"][c] <= 2 * row[1]
        if row[0] == 10.0:
            assert np.all(np.abs(r["M"][c] - one["M"][0]) < 0.03 * one["M"][0])
