"""Poiseuille flow through a tube in polar coordinates (oracle; test infrastructure).

Paper, Sec. 4 (SIS in the polar coordinate): the cross section is the unit
disc (lengths in units of the radius); by axial symmetry h depends on the
position only through r, and at the point (r, 0) the velocity is written
v = (v_r cos th, v_r sin th, v_z) with th the angle of the in-plane velocity
from the radial direction.  Eq. polar is the kinetic equation in these
variables, eq. polar_final the SIS velocity equation.

Readings:
* velocity nodes (the paper gives counts and ranges, not the node formulas):
  v_r = V t^2 with t the n_vr-point Gauss-Legendre nodes on [0, 1] (most
  nodes near v_r = 0), weight 2 V^2 t^3 w_t for int g v_r dv_r; th midpoints
  of n_th uniform cells on [0, pi]; v_z midpoints of n_vz cells on [0, Z].
  h is even in th (mirror of the tube about the radial line) and odd in v_z;
  the stored nodes are the th, v_z > 0 halves, and an integral of an even-even
  integrand over all velocities is 4 sum w (.) over them;
* collision operator: the single-gas fast spectral method of `collision.py`
  (same kernel, truncation, directions and multipliers on the modes
  xi = pi l / L_p of an N_p^3 periodic box; by default L_p = 2 max(V, Z) and
  N_p = 4 L_p, i.e. the lattice spacing 2 L_p / N_p = 1/2 of the Cartesian
  24^3 grids, which resolves the spectrum of f_eq; a spacing of 1 or more
  truncates it, and the resulting operator is not dissipative: the CIS
  diverges at delta = 5) with its transforms taken between
  the polar nodes and the Cartesian modes, as the paper describes: the
  spectrum F h (l) = sum over all nodes (both mirrors) of (w / dv_c^3) h
  e^{-i xi.v}, dv_c = 2 L_p / N_p (on a Cartesian lattice this is the DFT of
  the Cartesian operator), and F^-1 c (v) = N_p^-3 sum_l c(l) e^{i xi.v}
  evaluated at the stored nodes; f_eq is transformed with the same nodes;
* transport (eq. polar): v_r cos th dh/dr - (v_r sin th / r) dh/dth; the th
  derivative is taken upwind from larger th (the in-plane velocity turns
  towards the radial direction along a trajectory), three-point second order
  with the mirror ghost h(pi + e) = h(pi - e), first order at the node next to
  pi; r derivatives are the three-point non-uniform upwind differences of the
  planar sweep.  Inward molecules (th > pi/2) are swept from the wall (h = 0
  for molecules leaving a diffuse wall) to the centre; the centre passes a
  molecule from (r, th) to the opposite side, so the outward sweep (th < pi/2)
  starts with ghosts at -r_0, -r_1 holding h(r_0, pi - th), h(r_1, pi - th);
* velocity equation (eq. polar_final with the penalty of eq. BGK_penlty2 as
  in the planar reading): d(U + G)/dr = -N delta r / 2 - S2 / r + A with
  G = int v_z (2 v1^2 - 1) h, S2 = int 2 v_z (v1^2 - v2^2) h of h^{k+1/2},
  A = 2 int v1 v_z (L + N delta h) of h^k, v1 = v_r cos th, v2 = v_r sin th;
  marched from the wall (U there from the distribution) to the centre with
  the upwind differences (first order at the first step);
* flow rates M = 2 int_0^1 U3 r dr, Q = 2 int_0^1 q3 r dr (the area mean over
  the disc; trapezoid on the nodes and the centre, where the integrand is 0).
"""
import math

import numpy as np

from .collision import b0_unit, directions, phi_factor, psi_factor


class PolarGrid:
    """Stored velocity nodes (v_r, th, v_z) with v_z fastest."""

    def __init__(self, n_vr=22, vr_max=4.0, n_th=40, n_vz=12, vz_max=6.0):
        self.n_vr, self.n_th, self.n_vz = n_vr, n_th, n_vz
        self.vr_max, self.vz_max = float(vr_max), float(vz_max)
        x, w = np.polynomial.legendre.leggauss(n_vr)
        t = 0.5 * (x + 1.0)
        wt = 0.5 * w
        self.vr = vr_max * t ** 2
        self.wvr = 2.0 * vr_max ** 2 * t ** 3 * wt          # int g(v_r) v_r dv_r
        self.dth = math.pi / n_th
        self.th = (np.arange(n_th) + 0.5) * self.dth
        self.dz = vz_max / n_vz
        self.vz = (np.arange(n_vz) + 0.5) * self.dz
        VR, TH, VZ = np.meshgrid(self.vr, self.th, self.vz, indexing="ij")
        self.VR, self.TH, self.VZ = VR, TH, VZ
        self.V1 = VR * np.cos(TH)
        self.V2 = VR * np.sin(TH)
        self.vsq = VR ** 2 + VZ ** 2
        self.w = (self.wvr[:, None, None] * self.dth * self.dz) * np.ones_like(VR)
        self.feq = math.pi ** -1.5 * np.exp(-self.vsq)
        self.shape = VR.shape

    def integrate(self, f):
        """Integral over all velocities of an integrand even in th and in v_z."""
        return 4.0 * np.sum(self.w * f, axis=(-3, -2, -1))

    def U3(self, h):
        return self.integrate(self.VZ * h)

    def q3(self, h):
        return self.integrate((self.vsq - 2.5) * self.VZ * h)


class PolarFSM:
    """Fast-spectral L on the polar nodes (delta = 1)."""

    def __init__(self, grid: PolarGrid, n_pad=None, l_pad=None, m_angle=4, alpha=1.0, gamma=0.0):
        self.grid = g = grid
        self.L_p = float(l_pad) if l_pad else 2.0 * max(g.vr_max, g.vz_max)
        Np = self.n_pad = int(n_pad) if n_pad else 2 * int(round(2.0 * self.L_p))
        self.dvc = 2.0 * self.L_p / Np
        self.R = 4.0 * self.L_p / (3.0 + math.sqrt(2.0))
        self.b0 = b0_unit(alpha, gamma)
        dirs, W = directions(m_angle)
        self.W = W
        lf = np.arange(-Np // 2, Np // 2, dtype=np.float64)
        L0, L1, L2 = np.meshgrid(lf, lf, lf, indexing="ij")
        l = np.stack([L0.ravel(), L1.ravel(), L2.ravel()], axis=1)
        nyq = np.any(l == -Np // 2, axis=1)
        xi = math.pi * l / self.L_p
        self.phi = np.empty((len(W), len(l)))
        self.psi = np.empty((len(W), len(l)))
        for p, e in enumerate(dirs):
            s = l @ e
            perp = np.sqrt(np.maximum(np.sum((l - s[:, None] * e[None, :]) ** 2, axis=1), 0.0))
            self.phi[p] = phi_factor(s, self.R, self.L_p, alpha, gamma)
            self.psi[p] = psi_factor(perp, self.R, self.L_p, gamma)
        self.phi[:, nyq] = 0.0
        self.psi[:, nyq] = 0.0
        self.beta = 4.0 * self.b0 * np.einsum("p,pl,pl->l", W, self.phi, self.psi)
        # all nodes: the stored ones and their mirrors th -> -th, v_z -> -v_z
        v = np.stack([g.V1.ravel(), g.V2.ravel(), g.VZ.ravel()], axis=1)
        imgs = [(1.0, 1.0, 1.0, 1.0), (1.0, -1.0, 1.0, 1.0), (1.0, 1.0, -1.0, -1.0), (1.0, -1.0, -1.0, -1.0)]
        self.fwd = np.zeros((len(l), v.shape[0]), complex)   # h (stored, odd in v_z) -> F h
        self.fwd_even = np.zeros((len(l), v.shape[0]), complex)   # same for a field even in v_z
        wn = g.w.ravel() / self.dvc ** 3
        for s1, s2, s3, sg in imgs:
            ph = np.exp(-1j * (xi @ (v * np.array([s1, s2, s3])).T)) * wn[None, :]
            self.fwd += sg * ph
            self.fwd_even += ph
        self.inv = np.exp(1j * (v @ xi.T)) / Np ** 3          # F^-1 at the stored nodes
        fh = self.fwd_even @ g.feq.ravel()
        self.A = np.real(self.inv @ (self.psi * fh).T).T.reshape((len(W),) + g.shape)   # F^-1[psi_p F f_eq]
        self.B = np.real(self.inv @ (self.phi * fh).T).T.reshape((len(W),) + g.shape)   # F^-1[phi_p F f_eq]
        self.nu = np.real(self.inv @ (self.beta * fh)).reshape(g.shape)

    def lplus(self, h):
        """L+(h) at delta = 1 for one radial node, h of shape (n_vr, n_th, n_vz)."""
        g = self.grid
        H = self.fwd @ h.ravel()
        acc = np.zeros(g.shape)
        for p in range(len(self.W)):
            gp = np.real(self.inv @ (self.psi[p] * H)).reshape(g.shape)
            gf = np.real(self.inv @ (self.phi[p] * H)).reshape(g.shape)
            acc += self.W[p] * (self.B[p] * gp + gf * self.A[p])
        loss = g.feq * np.real(self.inv @ (self.beta * H)).reshape(g.shape)
        return 4.0 * self.b0 * acc - loss

    def apply(self, h):
        return self.lplus(h) - self.nu * h

    def nubar(self):
        return self.grid.integrate(self.nu * self.grid.feq)


# ------------------------------------------------------------------ transport
def _upwind_coeffs(x, i, j, k):
    """(a, b, c) with dy/dx at x[i] ~ a y_i + b y_j + c y_k for the nodes
    x[i], x[j], x[k] (j, k the two upwind neighbours; k None: two-point)."""
    d1 = x[i] - x[j]
    if k is None:
        return 1.0 / d1, -1.0 / d1, 0.0
    d2 = x[j] - x[k]
    return ((2.0 * d1 + d2) / (d1 * (d1 + d2)), -(d1 + d2) / (d1 * d2), d1 / (d2 * (d1 + d2)))


def sweep_tube(rhs, nu_d, r, grid):
    """Solve nu_d h + v_r cos th dh/dr - (v_r sin th / r) dh/dth = rhs on the
    radial nodes r (r[-1] = 1 the wall).  rhs: (n, n_vr, n_th, n_vz)."""
    g = grid
    n = len(r)
    nth = g.n_th
    half = nth // 2
    h = np.zeros_like(rhs)
    vr = g.vr[:, None]
    th_c = 3.0 / (2.0 * g.dth)
    # extended coordinates: ghosts -r_1, -r_0 before the nodes
    xe = np.concatenate([[-r[1], -r[0]], r])
    for k in range(nth - 1, half - 1, -1):             # inward: wall -> centre
        c1 = vr * math.cos(g.th[k])                    # < 0
        for i in range(n - 2, -1, -1):
            ct = vr * math.sin(g.th[k]) / r[i]         # > 0
            if i == n - 2:
                a, b, c = _upwind_coeffs(r, i, i + 1, None)
                up = b * h[i + 1, :, k]
            else:
                a, b, c = _upwind_coeffs(r, i, i + 1, i + 2)
                up = b * h[i + 1, :, k] + c * h[i + 2, :, k]
            diag = nu_d[:, k, :] + c1 * a
            src = rhs[i, :, k] - c1 * up
            if k < nth - 1:
                k2 = k + 2 if k + 2 < nth else nth - 1     # mirror ghost about pi
                diag = diag + ct * th_c
                src = src + ct * (4.0 * h[i, :, k + 1] - h[i, :, k2]) / (2.0 * g.dth)
            h[i, :, k] = src / diag
    for k in range(half - 1, -1, -1):                  # outward: centre -> wall
        c1 = vr * math.cos(g.th[k])                    # > 0
        km = nth - 1 - k                               # pi - th
        for i in range(n):
            ct = vr * math.sin(g.th[k]) / r[i]
            ie = i + 2
            a, b, c = _upwind_coeffs(xe, ie, ie - 1, ie - 2)
            y1 = h[i - 1, :, k] if i >= 1 else h[0, :, km]
            y2 = h[i - 2, :, k] if i >= 2 else h[1 - i, :, km]
            diag = nu_d[:, k, :] + c1 * a + ct * th_c
            src = (rhs[i, :, k] - c1 * (b * y1 + c * y2)
                   + ct * (4.0 * h[i, :, k + 1] - h[i, :, k + 2]) / (2.0 * g.dth))
            h[i, :, k] = src / diag
    return h


def moments_tube(grid, h):
    """(n, 5): U3, q3, G = int v_z (2 v1^2 - 1) h, S2 = int 2 v_z (v1^2 - v2^2) h,
    P_rz = int 2 v1 v_z h."""
    g = grid
    return np.stack([g.U3(h), g.q3(h), g.integrate(g.VZ * (2.0 * g.V1 ** 2 - 1.0) * h),
                     g.integrate(2.0 * g.VZ * (g.V1 ** 2 - g.V2 ** 2) * h),
                     g.integrate(2.0 * g.V1 * g.VZ * h)], axis=1)


def velocity_tube(r, mom, amom, delta, N, poiseuille=True):
    """d(U + G)/dr = -N delta r / 2 [Poiseuille] - S2 / r + A, A = amom[:, 0] +
    N delta amom[:, 1]; y = U + G from the wall value inwards."""
    n = len(r)
    A = amom[:, 0] + N * delta * amom[:, 1]
    src = A - mom[:, 3] / r - (N * delta * r / 2.0 if poiseuille else 0.0)
    y = np.zeros(n)
    y[n - 1] = mom[n - 1, 0] + mom[n - 1, 2]
    for i in range(n - 2, -1, -1):
        if i == n - 2:
            a, b, c = _upwind_coeffs(r, i, i + 1, None)
            y[i] = (src[i] - b * y[i + 1]) / a
        else:
            a, b, c = _upwind_coeffs(r, i, i + 1, i + 2)
            y[i] = (src[i] - b * y[i + 1] - c * y[i + 2]) / a
    return y - mom[:, 2]


def flow_rate_tube(r, f):
    """2 int_0^1 f r dr (trapezoid on the centre and the nodes)."""
    x = np.concatenate([[0.0], r])
    y = np.concatenate([[0.0], f * r])
    return 2.0 * float(np.sum(0.5 * (y[1:] + y[:-1]) * np.diff(x)))


def collide_tube(fsm, h, dU, delta, poiseuille=True):
    """h^k = h + dU 2 v_z f_eq, L+ = delta L+_1, L = L+ - delta nu h^k, rhs = L+ + S,
    amom = {2 int v1 v_z L, 2 int v1 v_z h^k}."""
    g = fsm.grid
    corr = 2.0 * g.VZ * g.feq
    hk = h + dU[:, None, None, None] * corr
    Lp = delta * np.stack([fsm.lplus(c) for c in hk]) if delta != 0 else np.zeros_like(hk)
    L = Lp - delta * fsm.nu * hk
    S = g.VZ * g.feq if poiseuille else 0.0
    amom = np.stack([g.integrate(2.0 * g.V1 * g.VZ * L), g.integrate(2.0 * g.V1 * g.VZ * hk)], axis=1)
    return Lp + S, L, amom


def solve_tube(fsm, r, delta, scheme="SIS", N=None, eps=1e-8, max_it=5000):
    """CIS / SIS outer iterations for Poiseuille flow through the tube (h^0 = 0)."""
    g = fsm.grid
    r = np.asarray(r, float)
    if N is None:
        N = fsm.nubar()
    n = len(r)
    corr = 2.0 * g.VZ * g.feq
    cU, cq = g.U3(corr), g.q3(corr)
    h = np.zeros((n,) + g.shape)
    dU = np.zeros(n)
    M_old = Q_old = 0.0
    converged = False
    it = 0
    for it in range(1, max_it + 1):
        rhs, L, amom = collide_tube(fsm, h, dU, delta)
        h = sweep_tube(rhs, delta * fsm.nu, r, g)
        mom = moments_tube(g, h)
        if scheme == "SIS":
            dU = velocity_tube(r, mom, amom, delta, N) - mom[:, 0]
        elif scheme == "CIS":
            dU = np.zeros(n)
        else:
            raise ValueError(scheme)
        Un = mom[:, 0] + dU * cU
        qn = mom[:, 1] + dU * cq
        M, Q = flow_rate_tube(r, Un), flow_rate_tube(r, qn)
        res = max(abs(M - M_old) / max(abs(M), 1e-300), abs(Q - Q_old) / max(abs(Q), 1e-300))
        M_old, Q_old = M, Q
        if res < eps:
            converged = True
            break
    return dict(M=M, Q=Q, iters=it, converged=converged, residual=res, U=Un, q=qn, h=h, dU=dU)


def free_molecular_tube(grid, r):
    """delta = 0: one sweep of the source v_z f_eq (nu_d = 0); returns (M, Q)."""
    g = grid
    rhs = np.broadcast_to(g.VZ * g.feq, (len(r),) + g.shape).copy()
    h = sweep_tube(rhs, np.zeros(g.shape), np.asarray(r, float), g)
    mom = moments_tube(g, h)
    return flow_rate_tube(r, mom[:, 0]), flow_rate_tube(r, mom[:, 1])
