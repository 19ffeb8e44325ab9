"""Parity storage (distributions odd in v3, and even in v2 for planar flows).

The plan restricted to the symmetry class must reproduce the full-grid
operator (oracle) on symmetric inputs, and solves must reproduce the
full-grid GPU solves, which are themselves pinned to the oracle.
"""
import functools
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import collision, mixture
from oracle import transport as tr
from oracle.velocity import VelocityGrid
from paper_1612_04488_amd import inputs, sis

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
NEAR = inputs.MIX_NEAR["mixture"]


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


def dev(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def symmetrize(h, parity):
    """Full-grid field -> its odd-in-v3 (and even-in-v2) part (last three axes v1, v2, v3)."""
    h = 0.5 * (h - h[..., ::-1])
    if parity == 2:
        h = 0.5 * (h + h[..., ::-1, :])
    return h


def stored(h, parity):
    n = h.shape[-1]
    h = h[..., n // 2:]
    if parity == 2:
        h = h[..., n // 2:, :]
    return h


@functools.lru_cache(maxsize=None)
def plan(n, lv, m, parity, mix=False):
    say("plan", n, lv, m, parity, mix)
    mx = dict(masses=NEAR["masses"], diameters=NEAR["diameters"], chi=(0.5, 0.5), m_rho=4) if mix else None
    return sis.Plan(n, lv, m_angle=m, mixture=mx, parity=parity)


@pytest.mark.parametrize("parity", [1, 2])
def test_restricted_operator_matches_oracle(parity):
    n, lv, m = 8, 4.0, 4
    p = plan(n, lv, m, parity)
    f = collision.FSM(VelocityGrid(n, lv), m_angle=m)
    t = p.tables(operator=True)
    assert t["op"].shape == (p.n_vel, p.n_vel)
    assert rel(t["feq"], stored(f.grid.feq, parity).ravel()) < 1e-15
    assert rel(t["nu"], stored(f.nu, parity).ravel()) < 1e-13
    h = symmetrize(inputs.rough_h(n, lv, 3), parity)
    for c in range(3):
        ref = stored(f.lplus(h[c]), parity).ravel()
        assert rel(t["op"] @ stored(h[c], parity).ravel(), ref) < 1e-13, c


@pytest.mark.parametrize("project", [False, True])
def test_restricted_collide_matches_oracle(project):
    n, lv, m, parity = 8, 4.0, 4, 2
    p = plan(n, lv, m, parity)
    f = collision.FSM(VelocityGrid(n, lv), m_angle=m)
    op = collision.ProjectedFSM(f) if project else f
    g = f.grid
    nc = 29
    rng = np.random.default_rng(4)
    h = symmetrize(inputs.rough_h(n, lv, nc), parity)
    delta = rng.choice([0.1, 2.0, 50.0], size=nc)
    flow = rng.integers(0, 3, size=nc).astype(np.int32)
    dU = rng.uniform(-1, 1, size=nc)
    hs = dev(stored(h, parity).reshape(nc, -1))
    rhs, lh = torch.empty_like(hs), torch.empty_like(hs)
    amom = torch.empty((nc, 4), dtype=torch.float64, device=DEV)
    p.collide(hs, dev(delta), rhs, dU=dev(dU), flow=dev(flow, torch.int32), project=project, lh_out=lh,
              amom_out=amom)
    torch.cuda.synchronize()
    rhs, lh, amom = rhs.cpu().numpy(), lh.cpu().numpy(), amom.cpu().numpy()
    for c in range(nc):
        hk = h[c] + dU[c] * 2.0 * g.V3 * g.feq
        lp = delta[c] * op.lplus(hk)
        L = lp - delta[c] * f.nu * hk
        S = g.source(flow[c]) if flow[c] else 0.0
        assert rel(rhs[c], stored(lp + S, parity).ravel()) < 1e-12, c
        assert rel(lh[c], stored(L, parity).ravel()) < 1e-12, c
        ref = [g.integrate(2 * g.V1 * g.V3 * L), g.integrate(2 * g.V1 * g.V3 * hk), 0.0, 0.0]
        sc = g.integrate(np.abs(2 * g.V1 * g.V3 * L)) + abs(ref[1])
        assert np.max(np.abs(amom[c] - ref)) < 1e-12 * sc, c


def _planar_solve(p, sections, deltas, flows, **kw):
    xs = [tr.nodes_tanh(s) for s in sections]
    geom = sis.Geometry(p, xs, deltas, flows)
    return sis.solve(p, geom, **kw)


@pytest.mark.parametrize("n,lv,m", [(8, 4.0, 4), (16, 6.0, 6)])
def test_planar_solves_equal_full_grid(n, lv, m):
    kw = dict(eps=1e-10, max_it=300)
    args = ([12, 7, 9, 12], [0.3, 4.0, 0.3, 30.0], [1, 1, 2, 2])
    full = _planar_solve(plan(n, lv, m, 0), *args, **kw)
    for parity in (1, 2):
        r = _planar_solve(plan(n, lv, m, parity), *args, **kw)
        say("parity", parity, r["iters"], full["iters"], rel(r["M"], full["M"]))
        assert np.array_equal(r["iters"], full["iters"])
        assert rel(r["M"], full["M"]) < 1e-12 and rel(r["Q"], full["Q"]) < 1e-12
        assert rel(r["U"], full["U"]) < 1e-12


def test_duct_solve_parity1_equals_full_grid():
    n, lv, m = 8, 4.0, 4
    cases = [(inputs.duct_faces(6, 0.5), inputs.duct_faces(9, 1.0), None)]
    out = []
    for parity in (0, 1):
        p = plan(n, lv, m, parity)
        g = sis.Geometry2D(p, "duct", cases, [2.0], [1])
        out.append(sis.solve(p, g, eps=1e-10, max_it=300))
    assert np.array_equal(out[0]["iters"], out[1]["iters"])
    assert rel(out[1]["M"], out[0]["M"]) < 1e-12 and rel(out[1]["Q"], out[0]["Q"]) < 1e-12
    with pytest.raises(sis.SisError):
        sis.Geometry2D(plan(n, lv, m, 2), "duct", cases, [2.0], [1])


def test_mixture_parity2_equals_full_grid():
    n, lv, m = 8, 4.0, 4
    out = []
    for parity in (0, 2):
        out.append(_planar_solve(plan(n, lv, m, parity, True), [9, 6], [0.2, 2.0], [1, 1], eps=1e-10, max_it=300))
    assert np.array_equal(out[0]["iters"], out[1]["iters"])
    assert rel(out[1]["M"], out[0]["M"]) < 1e-12 and rel(out[1]["Q"], out[0]["Q"]) < 1e-12
    o = mixture.MixtureFSM(VelocityGrid(n, lv), NEAR["masses"], NEAR["diameters"], (0.5, 0.5), m_angle=m, m_rho=4)
    t = plan(n, lv, m, 2, True).tables(operator=True)
    H = inputs.mixture_h(n, lv, 1, rough=True)[0]
    H = symmetrize(H, 2)
    assert rel(t["op"] @ stored(H, 2).ravel(), stored(o.lplus(H), 2).ravel()) < 1e-13


def test_mixed_precision_with_parity():
    p = plan(16, 6.0, 6, 2)
    args = ([12, 9], [0.5, 20.0], [1, 2])
    p.set_precision("fp64")
    ref = _planar_solve(p, *args, eps=1e-10, max_it=300)
    for prec in ("fp32", "bf16x3"):
        p.set_precision(prec)
        r = _planar_solve(p, *args, eps=1e-10, max_it=300)
        assert rel(r["M"], ref["M"]) < 1e-5 and rel(r["Q"], ref["Q"]) < 1e-5, prec
    p.set_precision("fp64")


@pytest.mark.parametrize("precision,tol", [("fp64", 1e-12), ("bf16x3", 5e-4)])
@pytest.mark.parametrize("workload", ["planar-batch", "duct"])
def test_benchmark_size_collide_matches_oracle_on_sampled_cells(workload, precision, tol):
    """The contraction at the benchmark's full size and launch configuration
    (planar batch: 32^3 velocities padded to 64^3, M = 12, 808 cells, v2, v3 > 0
    stored; duct: IPL 24^3 padded to 48^3, M = 8, 6 x 64^2 cells, v3 > 0 stored;
    the tuned tile and split-K, as bench.py times it), checked against the
    oracle's FFT form of L+ on sampled cells: FP64 to rounding, the plain
    3xBF16 contraction within the error bound it meets at small sizes."""
    w = inputs.PLANAR_BATCH if workload == "planar-batch" else inputs.DUCT_IPL
    parity = 2 if workload == "planar-batch" else 1
    nc = (sum(len(x) for x in inputs.workload_nodes(w)) if workload == "planar-batch"
          else w["cells"] ** 2 * len(w["aspect"]))
    say("benchmark-size collide", workload, precision, nc)
    p = sis.Plan(w["n_v"], w["l_v"], n_pad=w["n_pad"], m_angle=w["m_angle"], kernel=w["kernel"],
                 visc_index=w.get("visc_index", 0.81), parity=parity)
    h = inputs.smooth_h(w["n_v"], w["l_v"], nc)   # odd in v3, even in v2
    delta = np.resize(np.asarray(w["deltas"], dtype=np.float64), nc)
    hs = dev(stored(h, parity).reshape(nc, -1))
    rhs = torch.empty_like(hs)
    p.set_precision(precision)
    p.collide(hs, dev(delta), rhs)
    torch.cuda.synchronize()
    rows, splits, tuned, depth = p.contraction_config(nc, precision, with_depth=True)
    say("configuration", rows, splits, tuned, depth)
    assert tuned
    alpha = 2.0 * (1.0 - w.get("visc_index", 0.81)) if w["kernel"] == "ipl" else 1.0
    f = collision.FSM(VelocityGrid(w["n_v"], w["l_v"]), n_pad=w["n_pad"], m_angle=w["m_angle"], alpha=alpha)
    for c in (0, nc // 2 + 1, nc - 1):
        ref = stored(delta[c] * f.lplus(h[c]), parity).ravel()
        got = rhs[c].cpu().numpy()
        assert rel(got, ref) < tol, (workload, precision, c, rel(got, ref))
