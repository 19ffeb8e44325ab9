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


def mixture_h(n_v, l_v, n_cells, widths=(1.0, 2.0), seed=SEED, rough=False):
    """Two-species fields, shape (n_cells, 2, n_v, n_v, n_v): species s carries
    the envelope exp(-widths[s] |v|^2) times either the smooth seeded basis of
    `smooth_h` or (rough=True) white noise."""
    rng = np.random.default_rng(seed + 7)
    v = velocity_nodes(n_v, l_v)
    V1, V2, V3 = np.meshgrid(v, v, v, indexing="ij")
    vsq = V1 ** 2 + V2 ** 2 + V3 ** 2
    out = np.empty((n_cells, 2, n_v, n_v, n_v))
    for s, w in enumerate(widths):
        env = np.exp(-w * vsq)
        if rough:
            out[:, s] = rng.standard_normal((n_cells, n_v, n_v, n_v)) * env
        else:
            co = rng.uniform(-1.0, 1.0, size=(n_cells, 4))
            basis = np.stack([np.ones_like(vsq), V1, vsq - 2.5, 2 * V1 ** 2 - 1]) * (V3 * env)
            out[:, s] = np.einsum("ck,kxyz->cxyz", co, basis)
    return out


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


# Binary Ne-Ar hard-sphere mixture (masses 20.18 : 39.95, diameters 0.72 : 1,
# equimolar), planar Poiseuille, 200 tanh(3) sections per case, 24^3 velocities
# on [-5, 5]^3 padded to 48^3, M = 8, 16 rho nodes, 16 deltas log-spaced in
# [0.01, 100]: 16 cases x 201 nodes x 2 species.
MIX_NEAR = dict(name="mixture-near-hs-24v-201nodes-16cases", n_v=24, l_v=5.0, n_pad=48, m_angle=8,
                kernel="hs", mixture=dict(masses=(20.18, 39.95), diameters=(0.72, 1.0), chi=(0.5, 0.5),
                                          m_rho=16),
                sections=200, grid="tanh", deltas=[10.0 ** (-2.0 + 4.0 * j / 15.0) for j in range(16)],
                flows=[1] * 16)


# The mixture batch with uneven per-case grids (Sec. 5, Table 4 setting): the same
# gas and 16 deltas, 100 + round(100 j / 15) tanh(3) sections for case j (101 to
# 201 nodes), all cases in one batch.
MIX_RAGGED = dict(MIX_NEAR, name="mixture-near-hs-24v-101to201nodes-16cases",
                  sections=[100 + round(100 * j / 15) for j in range(16)])


def workload_nodes(w):
    f = {"uniform": nodes_uniform, "tanh": nodes_tanh, "smoothstep": nodes_smoothstep}[w["grid"]]
    sec = w["sections"]
    return [f(sec[i] if isinstance(sec, (list, tuple)) else sec) for i in range(len(w["deltas"]))]


# --------------------------------------------------------------- 2-D cross sections
def duct_faces(n, length, ratio=1.05):
    """n cells from the wall (-length) to the centre (0), sides growing by `ratio`."""
    w0 = length * (ratio - 1.0) / (ratio ** n - 1.0) if ratio != 1.0 else length / n
    f = np.concatenate([[0.0], np.cumsum(w0 * ratio ** np.arange(n))]) - length
    f[-1] = 0.0
    return f


def porous_discs(n=128, solid_fraction=0.4, r_max=0.1, r_ratio=10.0, seed=SEED, max_tries=200000):
    """Periodic unit cell with non-overlapping discs (random sequential addition,
    radii log-uniform in [r_max / r_ratio, r_max]) until the staircase solid
    fraction on an n x n grid reaches `solid_fraction`.  Returns (mask, discs)."""
    rng = np.random.default_rng(seed)
    xc = (np.arange(n) + 0.5) / n
    X, Y = np.meshgrid(xc, xc, indexing="ij")
    mask = np.zeros((n, n), bool)
    discs = []
    for _ in range(max_tries):
        r = r_max * r_ratio ** (-rng.uniform(0.0, 1.0))
        p = rng.uniform(0.0, 1.0, size=2)
        ok = True
        for (q, s) in discs:
            d = np.abs(p - q)
            d = np.minimum(d, 1.0 - d)
            if np.hypot(d[0], d[1]) < r + s:
                ok = False
                break
        if not ok:
            continue
        discs.append((p, r))
        dx = np.abs(X - p[0])
        dx = np.minimum(dx, 1.0 - dx)
        dy = np.abs(Y - p[1])
        dy = np.minimum(dy, 1.0 - dy)
        mask |= dx * dx + dy * dy <= r * r
        if mask.mean() >= solid_fraction:
            break
    return mask, discs


# Quarter rectangular ducts of aspect ratio 1 and 2 (shorter side = 1), 64 x 64
# geometric (1.05) cells, inverse-power-law gas (viscosity index 0.81), 24^3
# velocities padded to 48^3, M = 8, delta in {1, 10, 50}: 6 cases.
DUCT_IPL = dict(name="duct-ipl081-24v-64x64-6cases", n_v=24, l_v=6.0, n_pad=48, m_angle=8,
                kernel="ipl", visc_index=0.81, cells=64, aspect=[1, 1, 1, 2, 2, 2],
                deltas=[1.0, 10.0, 50.0] * 2, flows=[1] * 6)
# Equimolar Ne-Ar mixture in quarter ducts of aspect ratio 1 and 2 (Table 5):
# 64 x 64 cells growing by 1.05 from the walls, 24^3 velocities on [-5, 5]^3
# (v3 > 0 stored), M = 8, 16 rho nodes, N_a = 1.5, delta in {1, 10} per aspect ratio.
MIX_DUCT = dict(name="mixture-duct-near-hs-24v-64x64-4cases", n_v=24, l_v=5.0, n_pad=48, m_angle=8,
                kernel="hs", mixture=MIX_NEAR["mixture"], cells=64, aspect=[1, 1, 2, 2],
                deltas=[1.0, 10.0, 1.0, 10.0], flows=[1] * 4)
# Periodic porous unit cell, 128^2 staircase discs (porosity 0.6), hard spheres,
# 24^3 velocities padded to 48^3, M = 8, delta in {1, 10}.
POROUS_HS = dict(name="porous-hs-24v-128sq-2cases", n_v=24, l_v=6.0, n_pad=48, m_angle=8,
                 kernel="hs", cells=128, deltas=[1.0, 10.0], flows=[1, 1])


def duct_cases(w):
    out = []
    for ar in w["aspect"]:
        out.append((duct_faces(w["cells"], 0.5), duct_faces(w["cells"], 0.5 * ar), None))
    return out


def porous_cases(w):
    mask, _ = porous_discs(w["cells"])
    f = np.linspace(0.0, 1.0, w["cells"] + 1)
    return [(f, f, mask) for _ in w["deltas"]]


# --------------------------------------------------------------- Sierpinski carpets (Sec. 3.1)
def sierpinski_quarter(level, cells):
    """Quarter [-1/2, 0]^2 of the Sierpinski carpet of recursion `level` on the
    square [-1/2, 1/2]^2 (walls on its sides), `cells` uniform cells per side
    of the quarter.  Level r removes, inside every remaining square of side
    3^(1-r), the central square of side 3^-r; removed squares are solid.
    Returns (face1, face2, solid) for the quarter-duct geometry (symmetry
    planes at x1 = 0 and x2 = 0); 2 * cells must be a multiple of 3^level."""
    n = 2 * cells
    if n % 3 ** level:
        raise ValueError("2 * cells must be a multiple of 3**level")
    s = n // 3 ** level                       # cells per finest square
    m = np.arange(cells) // s                 # finest-square index of each quarter cell
    solid = np.zeros((cells, cells), bool)
    for r in range(1, level + 1):
        d = (m // 3 ** (level - r)) % 3 == 1  # r-th ternary digit is the middle one
        solid |= d[:, None] & d[None, :]
    f = np.linspace(-0.5, 0.0, cells + 1)
    return f, f.copy(), solid


# Sierpinski carpets as in the paper's Sec. 3.1: levels 1-3 on 60^2, 90^2, 135^2
# uniform quarter cells; hard spheres, 24^3 velocities (v3 > 0 stored), N = 1.5,
# delta in {0.1, 1, 10, 100}; the benchmark line runs level 3.
SIERPINSKI_CELLS = {0: 45, 1: 60, 2: 90, 3: 135}
SIERPINSKI_HS = dict(name="sierpinski-l3-hs-24v-135sq-4cases", n_v=24, l_v=6.0, n_pad=48, m_angle=8,
                     kernel="hs", level=3, cells=135, deltas=[0.1, 1.0, 10.0, 100.0], flows=[1] * 4)


def sierpinski_cases(w):
    c = sierpinski_quarter(w["level"], w["cells"])
    return [c for _ in w["deltas"]]


# Tube (Sec. 4, Table 3): the paper's polar grid (22 v_r nodes on (0, 4), 40 th on
# [0, pi], 12 v_z on (0, 6); FSM on the 48^3 lattice of spacing 1/2, M = 8), 150
# radial nodes clustered at the wall, hard spheres, N = 1, ten delta of Table 3.
TUBE_HS = dict(name="tube-hs-polar-22x40x12-150r-10cases", n_v=0, l_v=6.0, n_pad=0, m_angle=8, kernel="hs",
               polar=dict(n_vr=22, vr_max=4.0, n_th=40, n_vz=12), radial=150,
               deltas=[0.01, 0.1, 0.5, 1.0, 5.0, 10.0, 20.0, 30.0, 50.0, 100.0], flows=[1] * 10)


def tube_radial(n):
    """Radial nodes r_i = sin(pi (i + 1) / (2 n)): clustered at the wall r = 1."""
    return np.sin(0.5 * np.pi * (np.arange(n) + 1.0) / n)


def tube_h(nv, n_cells, seed=SEED):
    """Seeded smooth-magnitude fields on a polar grid row (the values do not
    change throughput)."""
    rng = np.random.default_rng(seed + 11)
    return rng.uniform(-1.0, 1.0, size=(n_cells, nv)) * 1e-2
