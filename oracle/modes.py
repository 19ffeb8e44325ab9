"""Fourier-mode convergence analysis of CIS and SIS (Sec. 2.3).

The system is periodic in x1 with period 1 (wavenumber 2 pi) and homogeneous
in x2; h and U3 stand for their x1-Fourier coefficients.

* CIS, eq. conv_iteration:  h^{k+1} = (L+ h^k + S) / (nu + 2 pi i v1).
* SIS, eq. acceleratred_iteration: h^{k+1/2} from the same formula, then
  U^{k+1} = (N delta [Poiseuille] - 2 pi i A1 - 4 pi^2 A2) / (4 pi^2) with
  A1 = 2 int v1 v3 (L + N delta h^k), A2 = int (2 v1^2 - 1) v3 h^{k+1/2},
  and the correction of eq. guided.  (The paper prints delta in place of
  N delta; with N = 1 they coincide.)
* omega: the paper fits U3(k) = U_inf + C exp(-lambda k), omega = exp(-lambda).
  `fitted_omega` estimates it from the ratio of successive U3 differences;
  `spectral_radius` is the modulus of the dominant eigenvalue of the linear
  part of the iteration on the flow's symmetry subspace (odd in v3, even in v2).

Closed forms for the BGK operator (L+ h = 2 delta U3(h) v3 f_eq, nu = delta),
obtained by integrating the mode iteration over v2, v3:
  CIS: omega = sqrt(pi) z exp(z^2) erfc(z), z = delta / (2 pi);
  SIS (N = 1): omega = | delta int (2v^2 - 1) e^{-v^2} / (sqrt(pi)(delta + 2 pi i v)) dv |.
"""
import math

import numpy as np
from scipy import integrate, special


def lplus_matrix(op):
    """Dense (N^3 x N^3) matrix of L+ at delta = 1, column j = L+(e_j)."""
    g = op.grid
    n3 = g.n ** 3
    K = np.empty((n3, n3))
    e = np.zeros(n3)
    for j in range(n3):
        e[j] = 1.0
        K[:, j] = op.lplus(e.reshape(g.feq.shape)).ravel()
        e[j] = 0.0
    return K


def symmetry_projector(grid):
    """Projector onto functions odd in v3 and even in v2 (flattened grid)."""
    n = grid.n
    idx = np.arange(n ** 3).reshape(n, n, n)
    m2 = idx[:, ::-1, :].ravel()
    m3 = idx[:, :, ::-1].ravel()
    m23 = idx[:, ::-1, ::-1].ravel()
    P = np.zeros((n ** 3, n ** 3))
    r = np.arange(n ** 3)
    P[r, r] += 0.25
    P[r, m2] += 0.25
    P[r, m3] -= 0.25
    P[r, m23] -= 0.25
    return P


def cis_map(K, nu, grid, delta):
    """Linear part of the CIS mode iteration."""
    den = (delta * nu + 2j * math.pi * grid.V1).ravel()
    return (delta * K) / den[:, None]


def sis_map(K, nu, grid, delta, N):
    """Linear part of the SIS mode iteration (source dropped)."""
    C = cis_map(K, nu, grid, delta)
    w = grid.w
    v1, v3 = grid.V1.ravel(), grid.V3.ravel()
    n3 = v1.size
    Lmat = delta * (K - np.diag(nu.ravel()))
    a1 = 2.0 * w * (v1 * v3) @ (Lmat + N * delta * np.eye(n3))
    a2 = w * ((2.0 * v1 ** 2 - 1.0) * v3) @ C
    u = w * v3 @ C
    corr = 2.0 * (v3 * grid.feq.ravel())
    row = (-2j * math.pi * a1 - 4.0 * math.pi ** 2 * a2) / (4.0 * math.pi ** 2) - u
    return C + np.outer(corr, row)


def symmetry_basis(grid):
    """Orthonormal basis Q (columns) of the range of `symmetry_projector`:
    one column (e_i + e_m2(i) - e_m3(i) - e_m23(i)) / 2 per node i with
    v2 > 0, v3 > 0, so that Q Q^T is the projector (even n: no node on the
    mirror planes)."""
    n = grid.n
    if n % 2:
        raise ValueError("symmetry_basis needs an even number of nodes per axis")
    idx = np.arange(n ** 3).reshape(n, n, n)
    h = n // 2
    i = idx[:, h:, h:].ravel()
    m2 = idx[:, h - 1::-1, h:].ravel()
    m3 = idx[:, h:, h - 1::-1].ravel()
    m23 = idx[:, h - 1::-1, h - 1::-1].ravel()
    Q = np.zeros((n ** 3, i.size))
    c = np.arange(i.size)
    Q[i, c] = 0.5
    Q[m2, c] = 0.5
    Q[m3, c] = -0.5
    Q[m23, c] = -0.5
    return Q


def spectral_radius(T, Q=None):
    """Largest |eigenvalue| of T, or of T restricted to the span of the
    orthonormal columns Q (the nonzero spectrum of Q Q^T T Q Q^T)."""
    if Q is not None:
        T = Q.T @ T @ Q
    return float(np.max(np.abs(np.linalg.eigvals(T))))


def iterate(T, s, n_it, grid):
    """Run h <- T h + s from h = 0; return the U3 history."""
    h = np.zeros(T.shape[0], dtype=complex)
    w = grid.w
    v3 = grid.V3.ravel()
    hist = []
    for _ in range(n_it):
        h = T @ h + s
        hist.append(w * np.dot(v3, h))
    return np.array(hist)


def fitted_omega(U, tail=12, floor=1e-11):
    """exp(-lambda) of U(k) = U_inf + C exp(-lambda k): least-squares slope of
    log|U(k+1) - U(k)| over the last `tail` differences still above the
    rounding floor (relative to max |U|)."""
    d = np.abs(np.diff(U))
    k = np.nonzero(d > floor * np.max(np.abs(U)))[0]
    k = k[-tail:]
    slope = np.polyfit(k.astype(float), np.log(d[k]), 1)[0]
    return float(np.exp(slope))


def sis_source(grid, delta, N, S, den):
    """Constant part of the SIS mode iteration for source S (Poiseuille)."""
    h_half = S.ravel() / den
    w = grid.w
    v1, v3 = grid.V1.ravel(), grid.V3.ravel()
    a2 = w * np.dot((2.0 * v1 ** 2 - 1.0) * v3, h_half)
    u = w * np.dot(v3, h_half)
    U = (N * delta - 4.0 * math.pi ** 2 * a2) / (4.0 * math.pi ** 2)
    return h_half + 2.0 * (U - u) * (v3 * grid.feq.ravel())


# ---------------------------------------------------------------- BGK forms
def bgk_cis_omega(delta):
    z = delta / (2.0 * math.pi)
    return math.sqrt(math.pi) * z * special.erfcx(z)


def bgk_sis_omega(delta):
    def re(v):
        return ((2 * v * v - 1) * math.exp(-v * v) * delta
                / (math.sqrt(math.pi) * (delta ** 2 + 4 * math.pi ** 2 * v * v)) * delta)

    def im(v):
        return (-(2 * v * v - 1) * math.exp(-v * v) * 2 * math.pi * v
                / (math.sqrt(math.pi) * (delta ** 2 + 4 * math.pi ** 2 * v * v)) * delta)

    r = integrate.quad(re, -np.inf, np.inf, epsabs=1e-14, epsrel=1e-13, limit=400)[0]
    i = integrate.quad(im, -np.inf, np.inf, epsabs=1e-14, epsrel=1e-13, limit=400)[0]
    return math.hypot(r, i)


class BGKOperator:
    """Linearized BGK operator of eq. BGK at delta = 1: L+ h = 2 U3(h) v3 f_eq, nu = 1."""

    def __init__(self, grid):
        self.grid = grid
        self.nu = np.ones_like(grid.feq)

    def lplus(self, h):
        return 2.0 * self.grid.U3(h) * self.grid.V3 * self.grid.feq

    def nubar(self):
        return 1.0


# ------------------------------------------------ BGK forms on the grid itself
def bgk_factors_discrete(grid, delta):
    """Exact grid versions of the BGK mode factors (velocity sums, not integrals).

    Returns (F_cis, F_sis, c) where F_cis = U'/U, F_sis = U^{k+1}/U (N = 1) and
    c = sum w 2 v3^2 f_eq; the SIS eigenvalue is (1 - c) F_cis + c F_sis.
    """
    den = delta + 2j * math.pi * grid.V1
    base = grid.w * 2.0 * delta * grid.V3 ** 2 * grid.feq / den
    F_cis = base.sum()
    F_sis = -((2.0 * grid.V1 ** 2 - 1.0) * base).sum()
    c = grid.integrate(2.0 * grid.V3 ** 2 * grid.feq)
    return complex(F_cis), complex(F_sis), float(c)
