"""Persistent launch of the planar iteration (sis_solve_opts.persistent): the iterations
between polls run as one cooperative launch with grid barriers between the steps of the
iteration (Sec. 2.2: collision, sweep, velocity equation, correction; Sec. 2.4: the stop
rule).  Compared with the launched path and with the oracle's solve.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import collision, solver
from oracle.velocity import POISEUILLE, VelocityGrid
from paper_1612_04488_amd import inputs, sis

pytestmark = pytest.mark.gpu

_plans = {}


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


def plan(n_v, l_v, m, parity=0):
    key = (n_v, l_v, m, parity)
    if key not in _plans:
        say("plan", *key)
        _plans[key] = sis.Plan(n_v, l_v, m_angle=m, parity=parity)
    return _plans[key]


def rel(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / max(np.max(np.abs(b)), 1e-300))


@pytest.mark.parametrize("scheme", ["SIS", "CIS"])
def test_persistent_small_planar_matches_launched_and_oracle(scheme):
    """The 17-node coarse-grid case (16^3 velocities, HS, delta = 1): same iteration count as
    the launched path and the oracle, flow rates within rounding of both."""
    w = inputs.PLANAR_SMALL
    p = plan(w["n_v"], w["l_v"], w["m_angle"])
    x = inputs.nodes_uniform(w["sections"])
    geom = sis.Geometry(p, [x], [1.0], [1])
    say("launched", scheme)
    rl = sis.solve(p, geom, scheme=scheme, eps=1e-8, max_it=500)
    say("persistent", scheme)
    rp = sis.solve(p, geom, scheme=scheme, eps=1e-8, max_it=500, persistent=1)
    say("iters", rl["iters"], rp["iters"], "M", rl["M"], rp["M"])
    assert np.array_equal(rl["iters"], rp["iters"])
    assert rel(rp["M"], rl["M"]) < 1e-12 and rel(rp["Q"], rl["Q"]) < 1e-12
    assert rel(rp["U"], rl["U"]) < 1e-11
    f = collision.FSM(VelocityGrid(w["n_v"], w["l_v"]), m_angle=w["m_angle"])
    ref = solver.solve_1d(f, x, 1.0, POISEUILLE, scheme, eps=1e-8)
    assert int(rp["iters"][0]) == ref.iters
    assert abs(rp["M"][0] - ref.M) < 1e-10 * abs(ref.M)
    assert abs(rp["Q"][0] - ref.Q) < 1e-10 * abs(ref.Q)


@pytest.mark.parametrize("parity", [0, 2])
def test_persistent_ragged_batch_any_workgroup_count(parity):
    """Four cases of 2 to 33 nodes (uniform, tanh, smoothstep; Poiseuille and thermal
    transpiration; delta 0.5 to 30), frozen one by one as they converge: the persistent launch
    with the default workgroup count, with fewer workgroups than contraction tiles (8) and
    with fewer than cells (3) gives bit-identical results (the same split-K slicing), equal
    iteration counts to the launched path and flow rates within rounding of it."""
    xs = [inputs.nodes_tanh(10), inputs.nodes_uniform(1), inputs.nodes_smoothstep(32),
          inputs.nodes_uniform(6)]
    deltas, flows = [0.5, 3.0, 30.0, 10.0], [1, 1, 2, 1]
    p = plan(8, 4.0, 4, parity)
    geom = sis.Geometry(p, xs, deltas, flows)
    say("launched parity", parity, "cells", geom.n_cells)
    rl = sis.solve(p, geom, scheme="SIS", eps=1e-9, max_it=400)
    outs = []
    for blocks in (1, 8, 3):
        say("persistent blocks", blocks)
        outs.append(sis.solve(p, geom, scheme="SIS", eps=1e-9, max_it=400, persistent=blocks, check_every=3))
    for r in outs[1:]:
        assert np.array_equal(r["iters"], outs[0]["iters"])
        assert np.array_equal(r["M"], outs[0]["M"]) and np.array_equal(r["Q"], outs[0]["Q"])
        assert np.array_equal(r["U"], outs[0]["U"])
    rp = outs[0]
    say("iters", rl["iters"], rp["iters"])
    assert np.array_equal(rl["iters"], rp["iters"])
    assert rel(rp["M"], rl["M"]) < 1e-12 and rel(rp["Q"], rl["Q"]) < 1e-12
    assert rel(rp["U"], rl["U"]) < 1e-11


def test_persistent_projection_and_not_converged():
    """The invariant projection runs inside the persistent finish step as in the launched
    one; a max_it cap is reported as not converged after exactly max_it iterations."""
    p = plan(8, 4.0, 4)
    xs = [inputs.nodes_uniform(12)]
    geom = sis.Geometry(p, xs, [5.0], [1])
    rl = sis.solve(p, geom, scheme="SIS", eps=1e-9, max_it=400, project=True)
    rp = sis.solve(p, geom, scheme="SIS", eps=1e-9, max_it=400, project=True, persistent=1)
    assert np.array_equal(rl["iters"], rp["iters"])
    assert rel(rp["M"], rl["M"]) < 1e-12
    r = sis.solve(p, geom, scheme="CIS", eps=1e-14, max_it=5, persistent=1, raise_not_converged=False,
                  check_every=2)
    assert r["status"] == sis.SIS_E_NOT_CONVERGED
    assert r["iters"][0] == 5


def test_persistent_rejects_other_solves():
    """Only planar one-gas FP64 solves take the persistent launch."""
    p = sis.Plan(8, 4.0, m_angle=4)
    geom = sis.Geometry(p, [inputs.nodes_uniform(6)], [1.0], [1])
    p.set_precision("bf16x3")
    with pytest.raises(sis.SisError):
        sis.solve(p, geom, scheme="SIS", eps=1e-8, max_it=10, persistent=1)
    p.set_precision("fp64")
    r = sis.solve(p, geom, scheme="SIS", eps=1e-8, max_it=200, persistent=1)
    assert r["status"] == 0
    f = inputs.duct_faces(4, 0.5)
    g2 = sis.Geometry2D(p, "duct", [(f, f, None)], [1.0], [1])
    with pytest.raises(sis.SisError):
        sis.solve(p, g2, scheme="SIS", eps=1e-8, max_it=10, persistent=1)
