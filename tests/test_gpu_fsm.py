"""GPU parity of the per-cell fast-spectral transform path (sis_collide_fsm).

The transform path evaluates L+ of every cell from its own forward and inverse
DFTs (the fast spectral method the paper cites for eq. LBE_collision); it must
equal the oracle's FFT form of the same discrete operator to rounding, and the
assembled-operator path (sis_collide) on every output, through the C ABI.
"""
import functools
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import collision
from oracle.velocity import VelocityGrid
from paper_1612_04488_amd import inputs, sis

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def say(*a):
    print("[gpu-fsm]", *a, flush=True)
    sys.stdout.flush()


def dev(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def rel(a, b):
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def symmetrize(h, parity):
    """Full-grid field -> its odd-in-v3 (parity >= 1) and even-in-v2 (parity 2) part."""
    if parity >= 1:
        h = 0.5 * (h - h[..., ::-1])
    if parity == 2:
        h = 0.5 * (h + h[..., ::-1, :])
    return h


def stored(h, parity):
    n = h.shape[-1]
    if parity >= 1:
        h = h[..., n // 2:]
    if parity == 2:
        h = h[..., n // 2:, :]
    return h


@functools.lru_cache(maxsize=None)
def gpu_plan(n, lv, m, parity, kernel):
    say("plan", n, lv, m, parity, kernel)
    return sis.Plan(n, lv, m_angle=m, kernel=kernel, visc_index=0.81, parity=parity)


@functools.lru_cache(maxsize=None)
def oracle_fsm(n, lv, m, kernel):
    alpha = 2.0 * (1.0 - 0.81) if kernel == "ipl" else 1.0
    return collision.FSM(VelocityGrid(n, lv), m_angle=m, alpha=alpha)


CASES = [(6, 4.0, 3, 0, "hs"), (8, 4.0, 4, 0, "ipl"), (8, 4.0, 4, 1, "hs"), (12, 5.0, 4, 2, "hs"),
         (12, 5.0, 5, 1, "ipl"), (16, 6.0, 6, 2, "hs"), (16, 6.0, 3, 0, "hs")]


@pytest.mark.parametrize("case", CASES, ids=lambda c: "n%d-m%d-p%d-%s" % (c[0], c[2], c[3], c[4]))
def test_fsm_collide_matches_oracle_and_operator_path(case):
    """Every output of sis_collide_fsm (right side with random delta, flow codes and
    the pending correction; L; the A1/A2 moments; with and without the invariant
    projection) against the oracle's FFT form and against sis_collide, on a
    ragged batch of rough and smooth cells in the plan's parity class."""
    n, lv, m, parity, kernel = case
    say("fsm collide", case)
    p = gpu_plan(n, lv, m, parity, kernel)
    f = oracle_fsm(n, lv, m, kernel)
    g = f.grid
    nc = 37
    h = np.concatenate([inputs.rough_h(n, lv, 20, seed=11), inputs.smooth_h(n, lv, 17, seed=12)])
    h = symmetrize(h, parity)
    rng = np.random.default_rng(7)
    delta = rng.uniform(0.1, 20.0, nc)
    flow = rng.integers(0, 3, nc).astype(np.int32)
    dU = rng.standard_normal(nc) * 0.1
    hs = dev(stored(h, parity).reshape(nc, -1))
    nv = hs.shape[1]
    for project in (False, True):
        outs = {}
        for mode in ("fsm", "operator"):
            rhs = torch.empty_like(hs)
            lh = torch.empty_like(hs)
            amom = torch.empty((nc, 4), dtype=torch.float64, device=DEV)
            fn = p.collide_fsm if mode == "fsm" else p.collide
            fn(hs, dev(delta), rhs, dU=dev(dU), flow=dev(flow, torch.int32), project=project,
               lh_out=lh, amom_out=amom)
            torch.cuda.synchronize()
            outs[mode] = (rhs.cpu().numpy(), lh.cpu().numpy(), amom.cpu().numpy())
        for k in range(3):
            assert rel(outs["fsm"][k], outs["operator"][k]) < 1e-12, (case, project, k)
        if not project:
            # right side from the oracle: delta L+(h + dU 2 v3 f_eq) + S(flow)
            corr = 2.0 * g.V3 * g.feq
            for c in (0, 19, 20, nc - 1):
                hk = h[c] + dU[c] * corr
                ref = delta[c] * f.lplus(hk) + (g.source(int(flow[c])) if flow[c] else 0.0)
                got = outs["fsm"][0][c].reshape(stored(h[c], parity).shape)
                assert rel(got, stored(ref, parity)) < 1e-12, (case, c)
    assert nv == stored(h[0], parity).size


@pytest.mark.parametrize("slab", [1, 2, 3, 5])
def test_fsm_slab_width_does_not_change_results(slab):
    """The l1-slab width of the inverse-transform workgroups (including a ragged
    last slab) only reorders the sum over l1."""
    p = gpu_plan(12, 5.0, 4, 2, "hs")
    h = symmetrize(inputs.rough_h(12, 5.0, 9, seed=3), 2)
    hs = dev(stored(h, 2).reshape(9, -1))
    delta = dev(np.linspace(0.5, 3.0, 9))
    ref = torch.empty_like(hs)
    p.collide(hs, delta, ref)
    p.set_fsm_slab(slab)
    out = torch.empty_like(hs)
    p.collide_fsm(hs, delta, out)
    torch.cuda.synchronize()
    p.set_fsm_slab(2)
    assert rel(out.cpu().numpy(), ref.cpu().numpy()) < 1e-12


def test_fsm_empty_batch_and_rejections():
    p = gpu_plan(8, 4.0, 4, 1, "hs")
    h = torch.zeros((0, p.n_dof), dtype=torch.float64, device=DEV)
    p.collide_fsm(h, torch.zeros(0, dtype=torch.float64, device=DEV), torch.zeros_like(h))
    mix = sis.Plan(8, 4.0, m_angle=3, mixture=dict(masses=(20.18, 39.95), diameters=(0.72, 1.0),
                                                   chi=(0.5, 0.5), m_rho=4))
    hm = torch.zeros((2, mix.n_dof), dtype=torch.float64, device=DEV)
    with pytest.raises(sis.SisError) as e:
        mix.collide_fsm(hm, torch.ones(2, dtype=torch.float64, device=DEV), torch.zeros_like(hm))
    assert e.value.code == sis.SIS_E_UNSUPPORTED
    with pytest.raises(sis.SisError) as e:
        p.set_fsm_slab(0)
    assert e.value.code == sis.SIS_E_INVALID


@pytest.mark.parametrize("workload", ["planar-batch", "duct"])
def test_fsm_at_benchmark_size(workload):
    """The transform path over the whole benchmark batch (planar: 32^3 padded to
    64^3, M = 12, 808 cells, v2, v3 > 0 stored; duct: IPL 24^3 padded to 48^3,
    M = 8, 24 576 cells in chunks, v3 > 0 stored): sampled cells against the
    oracle's FFT form, every cell against the assembled-operator path."""
    w = inputs.PLANAR_BATCH if workload == "planar-batch" else inputs.DUCT_IPL
    parity = 2 if workload == "planar-batch" else 1
    nc = (sum(len(x) for x in inputs.workload_nodes(w)) if workload == "planar-batch"
          else w["cells"] ** 2 * len(w["aspect"]))
    say("fsm benchmark size", workload, nc)
    p = sis.Plan(w["n_v"], w["l_v"], n_pad=w["n_pad"], m_angle=w["m_angle"], kernel=w["kernel"],
                 visc_index=w.get("visc_index", 0.81), parity=parity)
    h = inputs.smooth_h(w["n_v"], w["l_v"], nc)
    delta = np.resize(np.asarray(w["deltas"], dtype=np.float64), nc)
    hs = dev(stored(h, parity).reshape(nc, -1))
    out = torch.empty_like(hs)
    ref = torch.empty_like(hs)
    p.collide_fsm(hs, dev(delta), out)
    p.collide(hs, dev(delta), ref)
    torch.cuda.synchronize()
    say("fsm info", p.fsm_info())
    assert rel(out.cpu().numpy(), ref.cpu().numpy()) < 1e-12
    alpha = 2.0 * (1.0 - w.get("visc_index", 0.81)) if w["kernel"] == "ipl" else 1.0
    f = collision.FSM(VelocityGrid(w["n_v"], w["l_v"]), n_pad=w["n_pad"], m_angle=w["m_angle"], alpha=alpha)
    got = out.cpu().numpy()
    for c in (0, nc // 2 + 1, nc - 1):
        r = stored(delta[c] * f.lplus(h[c]), parity).ravel()
        assert rel(got[c], r) < 1e-12, (workload, c, rel(got[c], r))
