"""Seeded synthetic inputs shared by the tests, the benchmark and the smoke
check.  Holds no arithmetic of the method itself: only workload recipes
(node sets of the paper's geometries, smooth seeded velocity distributions,
the benchmark configurations).
"""
import math

import numpy as np

SEED = 1612


def velocity_nodes(n_v, l_v):
    """Cell-centred nodes -l_v + (j + 1/2) 2 l_v / n_v of one velocity axis."""
    return -l_v + (np.arange(n_v) + 0.5) * (2.0 * l_v / n_v)


def smooth_h(n_v, l_v, n_cells, seed=SEED, scale=1.0):
    """h_c(v) = f(v) v3 [a + b v1 + c (|v|^2 - 5/2) + d (2 v1^2 - 1)], (a,b,c,d) ~ U(-1, 1).

    f(v) = pi^-3/2 exp(-|v|^2); Poiseuille-like smooth fields (odd in v3).
    Returns an (n_cells, n_v, n_v, n_v) float64 array.
    """
    rng = np.random.default_rng(seed)
    co = rng.uniform(-1.0, 1.0, size=(n_cells, 4)) * scale
    v = velocity_nodes(n_v, l_v)
    V1, V2, V3 = np.meshgrid(v, v, v, indexing="ij")
    vsq = V1 ** 2 + V2 ** 2 + V3 ** 2
    f = np.exp(-vsq) / math.pi ** 1.5
    basis = np.stack([np.ones_like(vsq), V1, vsq - 2.5, 2 * V1 ** 2 - 1]) * (V3 * f)
    return np.einsum("ck,kxyz->cxyz", co, basis)


def rough_h(n_v, l_v, n_cells, seed=SEED):
    """Gaussian-weighted white noise (no symmetry): exercises every operator entry."""
    rng = np.random.default_rng(seed + 1)
    v = velocity_nodes(n_v, l_v)
    V1, V2, V3 = np.meshgrid(v, v, v, indexing="ij")
    f = np.exp(-(V1 ** 2 + V2 ** 2 + V3 ** 2) / 2.0)
    return rng.standard_normal((n_cells, n_v, n_v, n_v)) * f


# --------------------------------------------------------------- node sets
def nodes_uniform(n_s):
    return -0.5 + 0.5 * np.arange(n_s + 1) / n_s


def nodes_tanh(n_s, beta=3.0):
    """Wall-clustered: x_i = -1/2 + 1/2 [1 - tanh(beta (1 - i/N_s)) / tanh(beta)]."""
    t = np.arange(n_s + 1) / n_s
    return -0.5 + 0.5 * (1.0 - np.tanh(beta * (1.0 - t)) / math.tanh(beta))


def nodes_smoothstep(n_s):
    s = np.arange(n_s + 1) / (2.0 * n_s)
    return (10.0 - 15.0 * s + 6.0 * s ** 2) * s ** 3 - 0.5


# --------------------------------------------------------------- workloads
# Planar Poiseuille, hard spheres, delta = 1, 16 uniform sections, 16^3 on
# [-6, 6]^3 padded to 32^3, M = 6 (36 directions).
PLANAR_SMALL = dict(name="planar-hs-16v-16cells", n_v=16, l_v=6.0, n_pad=32, m_angle=6,
                    kernel="hs", sections=16, grid="uniform", deltas=[1.0], flows=[1])
# Planar Poiseuille + thermal transpiration, hard spheres, 100 tanh(3)
# sections, 32^3 padded to 64^3, M = 12 (144 directions), 4 deltas x 2 flows.
PLANAR_BATCH = dict(name="planar-hs-32v-100cells-8cases", n_v=32, l_v=6.0, n_pad=64,
                    m_angle=12, kernel="hs", sections=100, grid="tanh",
                    deltas=[0.1, 1.0, 10.0, 100.0] * 2, flows=[1] * 4 + [2] * 4)


def workload_nodes(w):
    f = {"uniform": nodes_uniform, "tanh": nodes_tanh, "smoothstep": nodes_smoothstep}[w["grid"]]
    return [f(w["sections"]) for _ in w["deltas"]]
