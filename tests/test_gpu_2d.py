"""GPU parity of the 2-D cross-section path (quarter ducts, periodic porous
cells) against the oracle, through the C ABI."""
import functools
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import collision, duct
from oracle.velocity import POISEUILLE, TRANSPIRATION, VelocityGrid
from paper_1612_04488_amd import inputs, sis

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(*a):
    print("[gpu-2d]", *a, flush=True)


@functools.lru_cache(maxsize=None)
def plan(n_v, l_v, m, kernel="hs"):
    return sis.Plan(n_v, l_v, m_angle=m, kernel=kernel, visc_index=0.81)


@functools.lru_cache(maxsize=None)
def fsm(n_v, l_v, m, alpha=1.0):
    return collision.FSM(VelocityGrid(n_v, l_v), m_angle=m, alpha=alpha)


def dev(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def small_porous(n, seed):
    rng = np.random.default_rng(seed)
    m = np.zeros((n, n), bool)
    for _ in range(3):
        i, j = rng.integers(0, n, 2)
        m[i:i + 2, j:j + 3] = True
    return m


def oracle_grids(kind, cases):
    if kind == "duct":
        return [duct.Grid2D(c[0], c[1], (duct.WALL, duct.SYM, duct.WALL, duct.SYM), c[2]) for c in cases]
    return [duct.Grid2D(c[0], c[1], (duct.PERIODIC,) * 4, c[2]) for c in cases]


CASES = {
    "duct": [(inputs.duct_faces(7, 0.5), inputs.duct_faces(7, 0.5), None),
             (inputs.duct_faces(5, 0.5), inputs.duct_faces(9, 1.0), None)],
    "periodic": [(np.linspace(0, 1, 11), np.linspace(0, 1, 9), small_porous(10, 1)[:, :8]),
                 (np.linspace(0, 1, 9), np.linspace(0, 1, 9), small_porous(8, 2))],
}


@pytest.mark.parametrize("kind", ["duct", "periodic"])
def test_sweep2d_and_moments_parity(kind):
    n_v, l_v, m = 8, 4.0, 3
    say("sweep2d", kind)
    p = plan(n_v, l_v, m)
    cases = CASES[kind]
    deltas, flows = [1.0, 7.0], [1, 2]
    geom = sis.Geometry2D(p, kind, cases, deltas, flows)
    f = fsm(n_v, l_v, m)
    vg = f.grid
    grids = oracle_grids(kind, cases)
    nc = geom.n_cells
    assert nc == sum(len(g.cells) for g in grids)
    rhs = inputs.rough_h(n_v, l_v, nc) + inputs.smooth_h(n_v, l_v, nc, seed=5)
    hprev = inputs.rough_h(n_v, l_v, nc, seed=9)
    hd = dev(hprev.reshape(nc, -1))
    mom = torch.empty((nc, 8), dtype=torch.float64, device=DEV)
    sis.transport_sweep(p, geom, dev(rhs.reshape(nc, -1)), hd, mom)
    torch.cuda.synchronize()
    hd, mom = hd.cpu().numpy(), mom.cpu().numpy()
    o = geom.offsets
    for c, g in enumerate(grids):
        s = slice(o[c], o[c + 1])
        ref = duct.sweep_2d(rhs[s], deltas[c] * f.nu, g, vg, hprev[s])
        assert rel(hd[s].reshape(ref.shape), ref) < 1e-12, c
        mref = duct.moments_2d(vg, ref)
        assert np.max(np.abs(mom[s, :7] - mref)) < 1e-12 * np.max(np.abs(mref)), c


@pytest.mark.parametrize("solver", ["inverse", "cg"])
@pytest.mark.parametrize("kind", ["duct", "periodic"])
def test_diffusion2d_parity(kind, solver):
    n_v, l_v, m = 8, 4.0, 3
    say("diffusion2d", kind, solver)
    p = plan(n_v, l_v, m)
    cases = CASES[kind]
    deltas, flows = [2.0, 30.0], [1, 2]
    geom = sis.Geometry2D(p, kind, cases, deltas, flows)
    geom.diffusion_solver(solver)
    n_inv, n_dist, res = geom.diffusion_info()
    assert n_inv == (len(cases) if solver == "inverse" else 0)
    assert n_dist == (len(cases) if solver == "inverse" else 0)
    assert res < 1e-8
    grids = oracle_grids(kind, cases)
    nc = geom.n_cells
    rng = np.random.default_rng(4)
    mom = rng.standard_normal((nc, 8))
    amom = rng.standard_normal((nc, 4))
    N = 1.25
    U = torch.empty(nc, dtype=torch.float64, device=DEV)
    dU = torch.empty_like(U)
    sis.diffusion_correct(p, geom, dev(mom), dev(amom), N, U, dU)
    torch.cuda.synchronize()
    U, dU = U.cpu().numpy(), dU.cpu().numpy()
    o = geom.offsets
    for c, g in enumerate(grids):
        s = slice(o[c], o[c + 1])
        ref = duct.diffusion_2d(g, mom[s], amom[s], deltas[c], N, flows[c])
        assert rel(U[s], ref) < 1e-10, c
        assert rel(dU[s], ref - mom[s, 0]) < 1e-9, c


@pytest.mark.parametrize("kind,scheme,solver", [("duct", "SIS", "inverse"), ("duct", "SIS", "cg"),
                                                 ("duct", "CIS", "inverse"), ("periodic", "SIS", "inverse"),
                                                 ("periodic", "SIS", "cg")])
def test_solve2d_matches_oracle(kind, scheme, solver):
    n_v, l_v, m = 8, 4.0, 3
    say("solve2d", kind, scheme, solver)
    p = plan(n_v, l_v, m)
    cases = CASES[kind][:1]
    deltas, flows = [1.0], [1]
    geom = sis.Geometry2D(p, kind, cases, deltas, flows)
    geom.diffusion_solver(solver)
    r = sis.solve(p, geom, scheme=scheme, eps=1e-9, max_it=300)
    f = fsm(n_v, l_v, m)
    g = oracle_grids(kind, cases)[0]
    ref = duct.solve_2d(f, g, 1.0, POISEUILLE, scheme, N=f.nubar(), eps=1e-9, max_it=300)
    say("gpu", r["M"], r["Q"], r["iters"], "oracle", ref["M"], ref["Q"], ref["iters"])
    assert int(r["iters"][0]) == ref["iters"]
    assert abs(r["M"][0] - ref["M"]) < 1e-10 * abs(ref["M"])
    assert abs(r["Q"][0] - ref["Q"]) < 1e-10 * abs(ref["Q"])


@pytest.mark.parametrize("kind", ["duct", "periodic"])
def test_diffusion2d_inverse_at_full_size(kind):
    """The velocity equation of the full-size cross sections (64^2 quarter
    ducts of aspect 1 and 2; the 128^2 porous cell with its disc packing):
    the precomputed inverse agrees with the oracle's sparse direct solve and
    with the conjugate-gradient path.  The operator depends on the geometry
    only, so a small velocity plan serves."""
    say("diffusion2d full size", kind)
    p = plan(8, 4.0, 3)
    if kind == "duct":
        w = inputs.DUCT_IPL
        cases = inputs.duct_cases(w)[2:4]
    else:
        w = inputs.POROUS_HS
        cases = inputs.porous_cases(w)[:1]
    deltas, flows = [5.0] * len(cases), [1] * len(cases)
    geom = sis.Geometry2D(p, kind, cases, deltas, flows)
    n_inv, n_dist, res = geom.diffusion_info()
    say("inverse cases", n_inv, "distinct", n_dist, "residual", res)
    assert n_inv == len(cases) and n_dist == len(cases) and res < 1e-8
    nc = geom.n_cells
    rng = np.random.default_rng(12)
    mom = rng.standard_normal((nc, 8)) * 0.1
    mom[:, 0] += 1.0
    amom = rng.standard_normal((nc, 4)) * 0.1
    N = 1.1
    out = {}
    for solver in ("inverse", "cg"):
        geom.diffusion_solver(solver)
        U = torch.empty(nc, dtype=torch.float64, device=DEV)
        sis.diffusion_correct(p, geom, dev(mom), dev(amom), N, U, None)
        torch.cuda.synchronize()
        out[solver] = U.cpu().numpy()
    grids = oracle_grids(kind, cases)
    o = geom.offsets
    for c, g in enumerate(grids):
        s = slice(o[c], o[c + 1])
        ref = duct.diffusion_2d(g, mom[s], amom[s], deltas[c], N, flows[c])
        say(c, rel(out["inverse"][s], ref), rel(out["cg"][s], ref))
        assert rel(out["inverse"][s], ref) < 1e-10, c
        assert rel(out["cg"][s], ref) < 1e-8, c


def test_inverse_falls_back_on_singular_cases():
    """A periodic cell without solids has no Dirichlet cell: its operator is
    singular, so that case keeps the conjugate-gradient solve."""
    p = plan(8, 4.0, 3)
    f = np.linspace(0, 1, 7)
    cases = [(f, f, np.zeros((6, 6), bool)), CASES["periodic"][1]]
    geom = sis.Geometry2D(p, "periodic", cases, [1.0, 1.0], [0, 1])
    assert geom.diffusion_info()[:2] == (1, 1)


def test_shared_inverse_for_equal_cross_sections():
    """Cases with the same cross section share one inverse (applied to up to
    eight right sides per read): eleven cases over two cross sections (one of
    them nine times, so split over two reads) hold two inverses, and every
    case's velocity matches the oracle."""
    say("shared inverse")
    p = plan(8, 4.0, 3)
    base = CASES["periodic"]
    order = [0, 1, 1, 0, 1, 1, 1, 1, 1, 1, 1]
    cases = [base[i] for i in order]
    deltas = [0.5 + 0.7 * k for k in range(len(cases))]
    flows = [1, 2] * 5 + [1]
    geom = sis.Geometry2D(p, "periodic", cases, deltas, flows)
    n_inv, n_dist, res = geom.diffusion_info()
    assert n_inv == len(cases) and n_dist == 2 and res < 1e-8
    nc = geom.n_cells
    rng = np.random.default_rng(6)
    mom = rng.standard_normal((nc, 8))
    amom = rng.standard_normal((nc, 4))
    U = torch.empty(nc, dtype=torch.float64, device=DEV)
    sis.diffusion_correct(p, geom, dev(mom), dev(amom), 1.3, U, None)
    torch.cuda.synchronize()
    U = U.cpu().numpy()
    grids = oracle_grids("periodic", cases)
    o = geom.offsets
    for c, g in enumerate(grids):
        s = slice(o[c], o[c + 1])
        ref = duct.diffusion_2d(g, mom[s], amom[s], deltas[c], 1.3, flows[c])
        assert rel(U[s], ref) < 1e-10, c


def test_sweep2d_at_benchmark_size():
    """The 2-D sweep and moments at the duct benchmark's size and storage: 64 x 64
    quarter cross sections of aspect ratio 1 and 2, IPL 24^3 velocities with
    v3 > 0 stored, the launch configuration bench.py times.  The sweep couples no
    velocities, so the oracle's full-grid sweep restricted to v3 > 0 is the
    reference; inputs odd in v3 (as the solver's state) make the stored-half
    moments equal the full-grid ones."""
    w = inputs.DUCT_IPL
    say("sweep2d benchmark size")
    p = sis.Plan(w["n_v"], w["l_v"], n_pad=w["n_pad"], m_angle=w["m_angle"], kernel=w["kernel"],
                 visc_index=w["visc_index"], parity=1)
    all_cases = inputs.duct_cases(w)
    cases = [all_cases[0], all_cases[3]]
    deltas, flows = [1.0, 50.0], [1, 1]
    geom = sis.Geometry2D(p, "duct", cases, deltas, flows)
    f = collision.FSM(VelocityGrid(w["n_v"], w["l_v"]), n_pad=w["n_pad"], m_angle=w["m_angle"],
                      alpha=2.0 * (1.0 - w["visc_index"]))
    vg = f.grid
    grids = oracle_grids("duct", cases)
    nc = geom.n_cells
    assert nc == 2 * w["cells"] ** 2
    rhs = inputs.smooth_h(w["n_v"], w["l_v"], nc, seed=5)
    hprev = inputs.smooth_h(w["n_v"], w["l_v"], nc, seed=9)
    half = w["n_v"] // 2
    hd = dev(np.ascontiguousarray(hprev[..., half:]).reshape(nc, -1))
    mom = torch.empty((nc, 8), dtype=torch.float64, device=DEV)
    sis.transport_sweep(p, geom, dev(np.ascontiguousarray(rhs[..., half:]).reshape(nc, -1)), hd, mom)
    torch.cuda.synchronize()
    hd, mom = hd.cpu().numpy(), mom.cpu().numpy()
    o = geom.offsets
    for c, g in enumerate(grids):
        s = slice(o[c], o[c + 1])
        ref = duct.sweep_2d(rhs[s], deltas[c] * f.nu, g, vg, hprev[s])
        assert rel(hd[s], ref[..., half:].reshape(o[c + 1] - o[c], -1)) < 1e-12, c
        mref = duct.moments_2d(vg, ref)
        assert np.max(np.abs(mom[s, :7] - mref)) < 1e-12 * np.max(np.abs(mref)), c


def _large_sweep_case(name):
    """Cross sections that select each form of the 2-D sweep.  Row-blocked with
    4 columns per wave (at most 64 cells along axis 2): a 64^2 periodic disc mask
    (Sec. 3.2; solids, periodic wraps at rows and columns 0 and 1), the level-3
    Sierpinski quarter on 54^2 cells (Sec. 3.1; solids, mirror ghosts) and a
    ragged batch of quarter ducts of 64 x 64, 12 x 10 and 9 x 3 cells (blocks of
    one column and empty blocks); with 8 columns per wave: the porous benchmark's
    128^2 disc mask.  Pipelined anti-diagonal (more than 128 cells along axis 2):
    the level-3 Sierpinski quarter on 135^2 cells (three cells per slot).  Plain
    anti-diagonal: a 200^2 quarter duct (Sec. 2.4; anti-diagonals over 192
    cells)."""
    if name == "porous64":
        mask, _ = inputs.porous_discs(64)
        f = np.linspace(0.0, 1.0, 65)
        return "periodic", [(f, f, mask)], 1
    if name == "carpet54":
        return "duct", [inputs.sierpinski_quarter(3, 54)], 1
    if name == "ragged":
        return "duct", [(inputs.duct_faces(64, 0.5), inputs.duct_faces(64, 0.5), None),
                        (inputs.duct_faces(12, 0.5), inputs.duct_faces(10, 1.0), None),
                        (inputs.duct_faces(9, 0.5), inputs.duct_faces(3, 0.25), None)], 1
    if name == "porous128":
        f, _, mask = inputs.porous_cases(inputs.POROUS_HS)[0]
        return "periodic", [(f, f, mask)], 1
    if name == "carpet135":
        return "duct", [inputs.sierpinski_quarter(3, 135)], 2
    f = inputs.duct_faces(200, 0.5)
    return "duct", [(f, f, None)], 3


@pytest.mark.parametrize("name", ["porous64", "carpet54", "ragged", "porous128", "carpet135", "duct200"])
def test_sweep2d_forms_parity(name):
    """Every form of the 2-D sweep, element by element over all cells against
    the oracle's sweep, on a small velocity grid (8^3) so that the oracle stays
    cheap; the geometry reports which form it launches."""
    n_v, l_v, m = 8, 4.0, 3
    kind, cases, form = _large_sweep_case(name)
    say("sweep2d form", name)
    p = plan(n_v, l_v, m)
    deltas, flows = [3.0, 0.0, 0.5][:len(cases)], [1] * len(cases)
    geom = sis.Geometry2D(p, kind, cases, deltas, flows)
    assert geom.sweep_form() == form
    f = fsm(n_v, l_v, m)
    vg = f.grid
    grids = oracle_grids(kind, cases)
    nc = geom.n_cells
    assert nc == sum(len(g.cells) for g in grids)
    rhs = inputs.smooth_h(n_v, l_v, nc, seed=5) + 0.1 * inputs.rough_h(n_v, l_v, nc, seed=3)
    hprev = inputs.rough_h(n_v, l_v, nc, seed=9)
    hd = dev(hprev.reshape(nc, -1))
    mom = torch.empty((nc, 8), dtype=torch.float64, device=DEV)
    sis.transport_sweep(p, geom, dev(rhs.reshape(nc, -1)), hd, mom)
    torch.cuda.synchronize()
    hd, mom = hd.cpu().numpy(), mom.cpu().numpy()
    o = geom.offsets
    for c, g in enumerate(grids):
        s = slice(o[c], o[c + 1])
        ref = duct.sweep_2d(rhs[s], deltas[c] * f.nu, g, vg, hprev[s])
        assert rel(hd[s].reshape(ref.shape), ref) < 1e-12, c
        mref = duct.moments_2d(vg, ref)
        assert np.max(np.abs(mom[s, :7] - mref)) < 1e-12 * np.max(np.abs(mref)), c
