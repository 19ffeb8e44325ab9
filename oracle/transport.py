"""Spatial grids, upwind transport sweeps, the diffusion correction and flow
rates for the planar (1-D) problem.

Paper:
* eq. LBE_iteration / eq. syn_LBE (Sec. 2, 2.2): nu h^{k+1} + v.grad h^{k+1} = RHS,
  spatial derivative by second-order upwind differences (first order next to
  a boundary, Sec. 2.4).
* Sec. 2.4: half channel -1/2 <= x1 <= 0, diffuse wall at x1 = -1/2
  (reflected perturbation zero; the printed "h(v_2>0)=0" is read as v1 > 0),
  specular reflection at x1 = 0; smoothstep node formula.
* eq. first_order (Sec. 2.4) with the tuning parameter N of eq. BGK_penlty2
  (Sec. 2.5): d(U3 + G1)/dx1 = -N delta x1 [Poiseuille] + A1,
  A1 = 2 int v1 v3 (L + N delta h); marched from the wall with the same
  upwind stencil, U3 at the wall taken from the VDF.
* Flow rates M = 2 int U3 dx1, Q = 2 int q3 dx1 (Sec. 2.4), trapezoid rule on
  the nodes.
"""
import math

import numpy as np

from .velocity import POISEUILLE


# --------------------------------------------------------------------------
# 1-D node sets on [-1/2, 0]
# --------------------------------------------------------------------------
def nodes_uniform(n_s):
    return -0.5 + 0.5 * np.arange(n_s + 1) / n_s


def nodes_smoothstep(n_s):
    """Sec. 2.4: x1 = (10 - 15 s + 6 s^2) s^3 - 1/2, s = i / (2 N_s)."""
    s = np.arange(n_s + 1) / (2.0 * n_s)
    return (10.0 - 15.0 * s + 6.0 * s ** 2) * s ** 3 - 0.5


def nodes_tanh(n_s, beta=3.0):
    """Wall-clustered nodes x_i = -1/2 + 1/2 [1 - tanh(beta (1 - i/N_s)) / tanh beta]."""
    t = np.arange(n_s + 1) / n_s
    return -0.5 + 0.5 * (1.0 - np.tanh(beta * (1.0 - t)) / math.tanh(beta))


# --------------------------------------------------------------------------
# upwind stencils
# --------------------------------------------------------------------------
def backward_coeffs(x, i):
    """(a, b, c) with dy/dx at x_i ~ a y_i + b y_{i-1} + c y_{i-2}.

    First order at i = 1 (first step from the wall), three-point non-uniform
    second order otherwise.
    """
    d1 = x[i] - x[i - 1]
    if i == 1:
        return 1.0 / d1, -1.0 / d1, 0.0
    d2 = x[i - 1] - x[i - 2]
    return ((2.0 * d1 + d2) / (d1 * (d1 + d2)), -(d1 + d2) / (d1 * d2),
            d1 / (d2 * (d1 + d2)))


def forward_coeffs(x, i):
    """(a, b, c) with -dy/dx at x_i ~ a y_i + b y_{i+1} + c y_{i+2}.

    First order at i = n-1 (first step from the symmetry plane).
    """
    n = len(x) - 1
    d1 = x[i + 1] - x[i]
    if i == n - 1:
        return 1.0 / d1, -1.0 / d1, 0.0
    d2 = x[i + 2] - x[i + 1]
    return ((2.0 * d1 + d2) / (d1 * (d1 + d2)), -(d1 + d2) / (d1 * d2),
            d1 / (d2 * (d1 + d2)))


# --------------------------------------------------------------------------
# transport sweep
# --------------------------------------------------------------------------
def sweep_1d(rhs, nu_d, x, grid):
    """Solve nu_d h + v1 dh/dx1 = rhs on the half channel.

    rhs: (n+1, N, N, N) at the nodes x (x[0] = -1/2 wall, x[n] = 0 symmetry).
    nu_d: (N, N, N) collision frequency times delta.
    v1 > 0: h = 0 at the wall, march towards x = 0.
    v1 < 0: specular reflection h(x=0, v1) = h(x=0, -v1), march to the wall.
    """
    n = len(x) - 1
    v1 = grid.V1
    pos = v1 > 0
    neg = ~pos
    av = np.abs(v1)
    h = np.zeros_like(rhs)
    for i in range(1, n + 1):
        a, b, c = backward_coeffs(x, i)
        prev2 = h[i - 2] if i >= 2 else 0.0
        val = (rhs[i] - v1 * (b * h[i - 1] + c * prev2)) / (nu_d + v1 * a)
        h[i][pos] = val[pos]
    mirror = h[n][::-1, :, :]            # v1 index j <-> N-1-j is v1 -> -v1
    h[n][neg] = mirror[neg]
    for i in range(n - 1, -1, -1):
        a, b, c = forward_coeffs(x, i)
        nxt2 = h[i + 2] if i + 2 <= n else 0.0
        val = (rhs[i] - av * (b * h[i + 1] + c * nxt2)) / (nu_d + av * a)
        h[i][neg] = val[neg]
    return h


# --------------------------------------------------------------------------
# diffusion correction (eq. first_order with N)
# --------------------------------------------------------------------------
def diffusion_1d(x, U_wall, G1, A1, delta, N, flow):
    """March D(U + G1) = -N delta x [Poiseuille] + A1 from the wall.

    Returns U at every node; U[0] = U_wall (value from the VDF).
    """
    n = len(x) - 1
    y = np.zeros(n + 1)
    y[0] = U_wall + G1[0]
    src = A1.copy()
    if flow == POISEUILLE:
        src = src - N * delta * x
    for i in range(1, n + 1):
        a, b, c = backward_coeffs(x, i)
        prev2 = y[i - 2] if i >= 2 else 0.0
        y[i] = (src[i] - b * y[i - 1] - c * prev2) / a
    return y - G1


def flow_rate_1d(x, u):
    """2 int_{-1/2}^0 u dx1 (trapezoid on the nodes)."""
    return 2.0 * float(np.sum(0.5 * (u[1:] + u[:-1]) * np.diff(x)))


def free_molecular_1d(grid, flow):
    """delta = 0 planar flow rates on the discrete grid (exact for the scheme).

    h is linear in x1 for each velocity, so U3 and q3 are constant:
    M = 1/2 sum w v3 S / |v1|,  Q = 1/2 sum w (|v|^2 - 5/2) v3 S / |v1|.
    """
    S = grid.source(flow)
    av = np.abs(grid.V1)
    M = 0.5 * grid.integrate(grid.V3 * S / av)
    Q = 0.5 * grid.integrate((grid.vsq - 2.5) * grid.V3 * S / av)
    return float(M), float(Q)
