"""Binary gas mixture: linearized collision operator and planar SIS (oracle).

Paper, Sec. 5 (SIS for the LBE of gas mixtures): velocities in units of the
most probable speed of species A; eq. Maxwell gives the equilibria, eq.
Boltzmann_lin the operators L_a = sum_b Q_ab(f_a, h_b) + Q_ab(h_a, f_b), the
moments U_a, P_a13, q_a and the flow rates M_a, Q_a follow the definitions
printed after it; the SIS velocity equations are eqs. LBE2_true2 (species B)
and LBE2_true1 (species A) with the penalty of eq. LBE_penlty and N_a from the
equilibrium collision frequency.

Readings (the paper cites, but does not print, the mixture FSM):
* equilibrium: f_a = chi_a (a/pi)^{3/2} exp(-a |v|^2), a = m_a / m_A (the
  printed exponent carries an extra factor 1/2 that contradicts the printed
  normalisation; the Maxwellian of species a in these units has none);
* hard spheres, B_ab = b0 (d_ab/d_A)^2 |u|, d_ab = (d_a + d_b)/2, b0 the
  single-gas hard-sphere amplitude;
* Carleman form for unequal masses (derived here): with mu = m_b/(m_a + m_b),
  x = v' - v = mu (|u| sigma - u) and y the part of v*' - v normal to x,
    v*' = v + y - c x,  c = (m_a - m_b) / (2 m_b),  v* = v + y + x / (2 mu),
  and the change of variables from (v*, sigma) costs a factor (2 mu)^-2:
    Q+_ab(g, h)(v) = 4 b_ab (2 mu)^-2 iint delta(x.y) g(v + x) h(v + y - c x) dx dy;
* truncation: |y| <= R and |x| <= 2 mu R (x is the fraction 2 mu of a
  relative-velocity chord, so the partner v* stays within the single-gas
  range); R = 4 L_p / (3 + sqrt 2) with zero extension to N_p^3 as for one gas.
  With x = 2 mu rho e (e on the half sphere, M x M directions), kappa = 2 mu c
  = (m_a - m_b)/(m_a + m_b) and psi_p the y-integral of one gas,
    Q+_ab = 4 b_ab sum_p W_p int_{-R}^{R} |rho| g(v + 2 mu rho e_p) (psi_p h)(v - kappa rho e_p) drho,
  i.e. in Fourier modes l (Nyquist zeroed)
    Q+_ab = 4 b_ab sum_p W_p sum_r w_r |rho_r| F^-1[e^{i pi 2mu rho_r l.e_p/L_p} g^]
                                              F^-1[psi_p e^{-i pi kappa rho_r l.e_p/L_p} h^]
  with an M_rho-point Gauss-Legendre rule on [0, R] and its mirror; for equal
  masses (kappa = 0, 2 mu = 1) the rho integral is the closed-form phi(l.e_p)
  of one gas;
* loss Q-_ab(g, h) = g F^-1[beta_ab h^], beta_ab = 4 b_ab sum_p W_p phi_p psi_p
  (the single-gas multiplier: with |x| <= 2 mu R the partner offset
  x/(2 mu) + y has the single-gas range);
* delta is normalised by the mixture's first Chapman-Enskog viscosity (hard
  spheres, one Sonine term, the textbook closed form in `viscosity_ratio`) and
  the mixture's most probable speed, so the operator at delta carries the
  factor delta sqrt(m_A/m) mu_mix/mu_A; `shear_bracket` computes the same
  viscosity from the discrete operator (pinned against the closed form).
"""
import math

import numpy as np

from .collision import _phi_hs, b0_unit, directions, psi_factor
from .velocity import VelocityGrid

NE_AR = dict(masses=(20.18, 39.95), diameters=(0.72, 1.0))


def viscosity_ratio(masses, diameters, chi):
    """First-approximation viscosity of a binary hard-sphere mixture divided by
    that of pure species A (same number density, diameter d_A).

    Textbook closed form (Chapman-Enskog, one Sonine term):
    mu = x^T H^-1 x with x the molar fractions and, in units of 1/mu_A,
      H_aa = x_a^2/mu_a + 2 x_a x_b/mu_ab * m_a m_b/(m_a+m_b)^2 * (5/(3A) + m_b/m_a),
      H_ab = -2 x_a x_b/mu_ab * m_a m_b/(m_a+m_b)^2 * (5/(3A) - 1),
    A = Omega22/Omega11 = 1 for hard spheres, mu_a ~ sqrt(m_a)/d_a^2 and the
    interaction viscosity mu_ab ~ sqrt(2 m_a m_b/(m_a+m_b))/d_ab^2.
    """
    m = np.asarray(masses, float)
    d = np.asarray(diameters, float)
    x = np.asarray(chi, float)
    mu = np.sqrt(m / m[0]) * (d[0] / d) ** 2
    dab = 0.5 * (d[0] + d[1])
    mu12 = math.sqrt(2.0 * m[0] * m[1] / (m[0] + m[1]) / m[0]) * (d[0] / dab) ** 2
    red = m[0] * m[1] / (m[0] + m[1]) ** 2
    k = 2.0 * x[0] * x[1] / mu12 * red
    H = np.array([[x[0] ** 2 / mu[0] + k * (5.0 / 3.0 + m[1] / m[0]), -k * (5.0 / 3.0 - 1.0)],
                  [-k * (5.0 / 3.0 - 1.0), x[1] ** 2 / mu[1] + k * (5.0 / 3.0 + m[0] / m[1])]])
    return float(x @ np.linalg.solve(H, x))


class MixtureFSM:
    """Fast-spectral L_A, L_B of a binary hard-sphere mixture at delta = 1.

    Arrays: h of shape (2, N, N, N), species A first.
    """

    def __init__(self, grid: VelocityGrid, masses, diameters, chi, n_pad=None, m_angle=6,
                 m_rho=8, r_trunc=None):
        self.grid = grid
        N = grid.n
        self.m = np.asarray(masses, float)
        self.d = np.asarray(diameters, float)
        self.chi = np.asarray(chi, float)
        if self.chi.shape != (2,) or abs(self.chi.sum() - 1.0) > 1e-12 or np.any(self.chi <= 0):
            raise ValueError("chi must be two positive molar fractions summing to 1")
        self.a = self.m / self.m[0]
        self.mbar = float(np.sum(self.chi * self.m))
        self.n_pad = Np = int(n_pad or 2 * N)
        self.L_p = Np * grid.dv / 2.0
        self.R = float(r_trunc) if r_trunc else 4.0 * self.L_p / (3.0 + math.sqrt(2.0))
        self.off = (Np - N) // 2
        self.dirs, self.W = directions(m_angle)
        self.D = len(self.W)
        self.m_rho = int(m_rho)
        x, w = np.polynomial.legendre.leggauss(self.m_rho)
        rho = 0.5 * self.R * (x + 1.0)
        wr = 0.5 * self.R * w
        self.rho = np.concatenate([rho, -rho])
        self.wr = np.concatenate([wr, wr])
        self.feq = np.stack([self.chi[s] * (self.a[s] / math.pi) ** 1.5 * np.exp(-self.a[s] * grid.vsq)
                             for s in range(2)])
        self.shp = (Np,) * 3
        lf = np.fft.fftfreq(Np, 1.0 / Np)
        lh = np.arange(Np // 2 + 1, dtype=float)
        l0, l1, l2 = np.meshgrid(lf, lf, lh, indexing="ij")
        self.nyq = (l0 == -Np // 2) | (l1 == -Np // 2) | (l2 == Np // 2)
        self.s = np.empty((self.D,) + l0.shape)      # l.e_p
        self.psi = np.empty_like(self.s)
        for p, e in enumerate(self.dirs):
            s = l0 * e[0] + l1 * e[1] + l2 * e[2]
            perp = np.sqrt(np.maximum((l0 - s * e[0]) ** 2 + (l1 - s * e[1]) ** 2
                                      + (l2 - s * e[2]) ** 2, 0.0))
            ps = psi_factor(perp, self.R, self.L_p, 0.0)
            ps[self.nyq] = 0.0
            self.s[p] = s
            self.psi[p] = ps
        self.b0 = b0_unit(1.0, 0.0)
        self.Fhat = [np.fft.rfftn(self.pad(f)) for f in self.feq]
        self.two_mu = np.zeros((2, 2))     # 2 m_b / (m_a + m_b)
        self.kappa = np.zeros((2, 2))      # (m_a - m_b) / (m_a + m_b)
        self.C = np.zeros((2, 2))          # 4 b_ab
        beta = np.zeros(l0.shape)
        for p in range(self.D):
            ph = _phi_hs(math.pi * self.s[p] / self.L_p, self.R)
            ph[self.nyq] = 0.0
            beta += self.W[p] * ph * self.psi[p]
        self.beta = {}
        self.nu_ab = np.zeros((2, 2) + grid.feq.shape)
        for a_ in range(2):
            for b_ in range(2):
                dab = 0.5 * (self.d[a_] + self.d[b_]) / self.d[0]
                self.two_mu[a_, b_] = 2.0 * self.m[b_] / (self.m[a_] + self.m[b_])
                self.kappa[a_, b_] = (self.m[a_] - self.m[b_]) / (self.m[a_] + self.m[b_])
                self.C[a_, b_] = 4.0 * self.b0 * dab ** 2
                self.beta[a_, b_] = self.C[a_, b_] * beta
                self.nu_ab[a_, b_] = self.crop(self._irf(self.beta[a_, b_] * self.Fhat[b_]))
        self.scale = math.sqrt(self.m[0] / self.mbar) * viscosity_ratio(self.m, self.d, self.chi)
        self._fcache = {}

    # ---------------------------------------------------------------- plumbing
    def pad(self, h):
        Np, o, N = self.n_pad, self.off, self.grid.n
        out = np.zeros(h.shape[:-3] + (Np,) * 3)
        out[..., o:o + N, o:o + N, o:o + N] = h
        return out

    def crop(self, hp):
        o, N = self.off, self.grid.n
        return hp[..., o:o + N, o:o + N, o:o + N]

    def _irf(self, X):
        return np.fft.irfftn(X, s=self.shp, axes=(-3, -2, -1))

    def _terms(self, a_, b_):
        """(weight, multiplier on the x-slot spectrum, multiplier on the y-slot
        spectrum) of every separable term of Q+_ab (unit amplitude)."""
        kap, tm = self.kappa[a_, b_], self.two_mu[a_, b_]
        k = math.pi / self.L_p
        if abs(kap) < 1e-14:
            for p in range(self.D):
                ph = _phi_hs(k * self.s[p], self.R)
                ph[self.nyq] = 0.0
                yield self.W[p], ph, self.psi[p]
        else:
            for p in range(self.D):
                for rho, wr in zip(self.rho, self.wr):
                    gx = np.exp(1j * k * tm * rho * self.s[p])
                    gx[self.nyq] = 0.0
                    yield self.W[p] * wr * abs(rho), gx, self.psi[p] * np.exp(-1j * k * kap * rho * self.s[p])

    # ---------------------------------------------------------------- the operator
    def gain(self, a_, b_, G, H):
        """Q+_ab(g, h) (unit amplitude) from the half spectra G, H of the
        zero-extended g (argument v + 2 mu rho e) and h (argument v + y - kappa rho e)."""
        acc = np.zeros(self.shp)
        for w, mx, my in self._terms(a_, b_):
            acc += w * self._irf(mx * G) * self._irf(my * H)
        return self.C[a_, b_] * self.crop(acc)

    def _feq_factors(self, a_, b_):
        """Cropped equilibrium factors of both gain terms of pair (a, b), cached:
        x-slot F^-1[mx f_a^] for Q+(f_a, h_b), y-slot F^-1[my f_b^] for Q+(h_a, f_b)."""
        key = (a_, b_)
        if key not in self._fcache:
            fx, fy = [], []
            for w, mx, my in self._terms(a_, b_):
                fx.append(self.crop(self._irf(mx * self.Fhat[a_])))
                fy.append(self.crop(self._irf(my * self.Fhat[b_])))
            self._fcache[key] = (np.array(fx), np.array(fy))
        return self._fcache[key]

    def lplus(self, h):
        """L+_a = sum_b Q+_ab(f_a, h_b) + Q+_ab(h_a, f_b) - f_a F^-1[beta_ab h_b^]
        at delta = 1, h of shape (2, N, N, N)."""
        Hh = [np.fft.rfftn(self.pad(h[s])) for s in range(2)]
        out = np.zeros_like(h, dtype=float)
        for a_ in range(2):
            for b_ in range(2):
                fx, fy = self._feq_factors(a_, b_)
                acc = np.zeros(self.grid.feq.shape)
                for t, (w, mx, my) in enumerate(self._terms(a_, b_)):
                    acc += w * (fx[t] * self.crop(self._irf(my * Hh[b_]))
                                + self.crop(self._irf(mx * Hh[a_])) * fy[t])
                out[a_] += self.C[a_, b_] * acc
                out[a_] -= self.feq[a_] * self.crop(self._irf(self.beta[a_, b_] * Hh[b_]))
        return self.scale * out

    @property
    def nu(self):
        """Equilibrium collision frequency of each species at delta = 1, (2, N, N, N)."""
        return self.scale * self.nu_ab.sum(axis=1)

    def apply(self, h):
        return self.lplus(h) - self.nu * h

    def nubar(self):
        """N_a delta at delta = 1: int nu_a f_a / chi_a."""
        return np.array([self.grid.integrate(self.nu[s] * self.feq[s]) / self.chi[s] for s in range(2)])

    # ---------------------------------------------------------------- normalisation check
    def shear_bracket(self):
        """mu_mix / mu_A from the discrete operator: Galerkin solution of the
        first Chapman-Enskog shear problem with trial functions v1 v2 f_a.

        H_ab = -int v1 v2 L_a(v1 v2 f_b), s_a = 2 a_a int (v1 v2)^2 f_a; the
        total shear stress gives mu_mix/mu_A = s^T H^-1 s for the unit-amplitude
        operator (pure A gas: 1).
        """
        g = self.grid
        H = np.zeros((2, 2))
        for b_ in range(2):
            ph = np.zeros((2,) + g.feq.shape)
            ph[b_] = g.V1 * g.V2 * self.feq[b_]
            L = self.apply(ph) / self.scale
            for a_ in range(2):
                H[a_, b_] = -g.integrate(g.V1 * g.V2 * L[a_])
        s = np.array([2.0 * self.a[k] * g.integrate((g.V1 * g.V2) ** 2 * self.feq[k]) for k in range(2)])
        return float(s @ np.linalg.solve(H, s)), H


# ---------------------------------------------------------------------- planar SIS
def correction_shapes(op):
    """2 (m_a/m_A) v3 f_a: the correction of species a per unit change of U_a."""
    g = op.grid
    return np.stack([2.0 * op.a[s] * g.V3 * op.feq[s] for s in range(2)])


def collide_1d(op, h, dU, delta, poiseuille=True):
    """Collision step per node: h^k = h + dU_a corr_a, L+ = delta L+_1(h^k),
    L = L+ - delta nu h^k, rhs = L+ + S (S_a = v3 f_a for Poiseuille) and the
    amom moments {2 int v1 v3 L_a, 2 int v1 v3 h_a^k}.  h: (n, 2, N, N, N)."""
    g = op.grid
    hk = h + np.asarray(dU)[:, :, None, None, None] * correction_shapes(op)
    delta = np.broadcast_to(np.asarray(delta, float), (h.shape[0],))
    Lp = np.stack([d * op.lplus(c) for d, c in zip(delta, hk)])
    L = Lp - delta[:, None, None, None, None] * op.nu * hk
    S = np.stack([g.V3 * op.feq[s] for s in range(2)]) if poiseuille else 0.0
    amom = np.stack([2.0 * g.integrate(g.V1 * g.V3 * L), 2.0 * g.integrate(g.V1 * g.V3 * hk)], axis=-1)
    return Lp + S, L, amom


def sweep_1d(op, rhs, x, delta):
    """Each species swept with its own delta nu_a (the single-gas sweep)."""
    from . import transport as tr
    return np.stack([tr.sweep_1d(rhs[:, s], delta * op.nu[s], x, op.grid) for s in range(2)], axis=1)


def moments_1d(op, h):
    """(n, 2, 4): int v3 h_a, q_a = int (a v^2 - 5/2) v3 h_a, G1_a, P_a13 = 2 a int v1 v3 h_a."""
    g = op.grid
    out = np.zeros(h.shape[:2] + (4,))
    for s in range(2):
        hs = h[:, s]
        out[:, s, 0] = g.integrate(g.V3 * hs)
        out[:, s, 1] = g.integrate((op.a[s] * g.vsq - 2.5) * g.V3 * hs)
        out[:, s, 2] = g.G1(hs)
        out[:, s, 3] = 2.0 * op.a[s] * g.integrate(g.V1 * g.V3 * hs)
    return out


def velocity_1d(op, x, mom, amom, delta, N, poiseuille=True):
    """SIS velocity equations, eqs. LBE2_true2 (B) and LBE2_true1 (A), in
    the planar half channel.  Integrated once from the symmetry plane (every
    term is odd there) they read
      chi_B D(U_B) + D(G1_B) = -N_B delta (m_A/m_B) P_B13 + A_B,
      chi_A D(U_A) + D(G1_A) = -N_A delta (x1 - P_B13) + A_A,
    with A_a = 2 int v1 v3 (L_a + N_a delta h_a^k) (eq. LBE_penlty) and P_B13
    of h^{k+1/2}; marched from the wall with the sweep's upwind stencil, U_a
    at the wall from the distribution.  Returns U (n, 2), per unit molar
    fraction (U_a = int v3 h_a / chi_a)."""
    from . import transport as tr
    x = np.asarray(x, float)
    n = len(x)
    N = np.broadcast_to(np.asarray(N, float), (2,))
    PB = mom[:, 1, 3]
    U = np.zeros((n, 2))
    for s in range(2):
        Nd = N[s] * delta
        A = amom[:, s, 0] + Nd * amom[:, s, 1]
        if s == 1:
            src = A - Nd * PB / op.a[1]
        else:
            src = A - Nd * ((x if poiseuille else 0.0) - PB)
        G = mom[:, s, 2]
        y = np.zeros(n)
        y[0] = mom[0, s, 0] + G[0]
        for i in range(1, n):
            ca, cb, cc = tr.backward_coeffs(x, i)
            y2 = y[i - 2] if i >= 2 else 0.0
            y[i] = (src[i] - cb * y[i - 1] - cc * y2) / ca
        U[:, s] = (y - G) / op.chi[s]
    return U


def solve_mixture_1d(op, x, delta, scheme="SIS", Npen=None, eps=1e-8, max_it=5000):
    """Planar Poiseuille flow of the binary mixture from h^0 = 0.

    One iteration: `collide_1d`, `sweep_1d`, `moments_1d`; SIS: `velocity_1d`
    and the correction h_a^{k+1} = h_a^{k+1/2} + 2 a_a (U_a - U_a^{k+1/2}) v3 f_a
    (the analogue of eq. guided).  Flow rates M_a = sqrt(m/m_A) 2 int U_a dx1,
    Q_a likewise with q_a (trapezoid rule); stop when the relative change of
    all four is below eps.  Npen: N_a (default int nu_a f_a / chi_a).
    """
    from . import transport as tr
    g = op.grid
    N = op.nubar() if Npen is None else np.broadcast_to(np.asarray(Npen, float), (2,))
    x = np.asarray(x, float)
    n = len(x)
    corr = correction_shapes(op)
    cU = np.array([g.U3(corr[s]) / op.chi[s] for s in range(2)])
    cq = np.array([g.integrate((op.a[s] * g.vsq - 2.5) * g.V3 * corr[s]) for s in range(2)])
    fac = math.sqrt(op.mbar / op.m[0])
    h = np.zeros((n, 2) + g.feq.shape)
    dU = np.zeros((n, 2))
    M_old = np.zeros(2)
    Q_old = np.zeros(2)
    converged = False
    it = 0
    for it in range(1, max_it + 1):
        rhs, L, amom = collide_1d(op, h, dU, delta)
        h = sweep_1d(op, rhs, x, delta)
        mom = moments_1d(op, h)
        U_half = mom[:, :, 0] / op.chi
        if scheme == "SIS":
            dU = velocity_1d(op, x, mom, amom, delta, N) - U_half
        elif scheme == "CIS":
            dU = np.zeros((n, 2))
        else:
            raise ValueError(scheme)
        Un = U_half + dU * cU
        qn = mom[:, :, 1] + dU * cq
        M = np.array([fac * tr.flow_rate_1d(x, Un[:, s]) for s in range(2)])
        Q = np.array([fac * tr.flow_rate_1d(x, qn[:, s]) for s in range(2)])
        res = float(np.max(np.concatenate([np.abs(M - M_old) / np.maximum(np.abs(M), 1e-300),
                                           np.abs(Q - Q_old) / np.maximum(np.abs(Q), 1e-300)])))
        M_old, Q_old = M, Q
        if res < eps:
            converged = True
            break
    return dict(M=M, Q=Q, iters=it, converged=converged, residual=res, U=Un, q=qn, dU=dU,
                h_half=h, N=N)


def free_molecular_1d(op):
    """delta = 0: per species v1 dh_a/dx1 = v3 f_a is solved exactly by the
    upwind scheme (h linear in x1), so U_a and q_a are uniform:
    M_a = sqrt(m/m_A) (1/chi_a) 1/2 sum w v3^2 f_a / |v1|, Q_a likewise."""
    g = op.grid
    fac = math.sqrt(op.mbar / op.m[0])
    av = np.abs(g.V1)
    M = np.array([fac * 0.5 * g.integrate(g.V3 ** 2 * op.feq[s] / av) / op.chi[s] for s in range(2)])
    Q = np.array([fac * 0.5 * g.integrate((op.a[s] * g.vsq - 2.5) * g.V3 ** 2 * op.feq[s] / av)
                  for s in range(2)])
    return M, Q


# ------------------------------------------------------------------ rectangular ducts (Sec. 5.3, Table 5)
def sweep_2d(op, rhs, g, delta, h_prev):
    """Each species swept over the cross section with its own delta nu_a (the
    single-gas 2-D sweep).  rhs, h_prev: (n_fluid, 2, N, N, N)."""
    from . import duct
    return np.stack([duct.sweep_2d(rhs[:, s], delta * op.nu[s], g, op.grid, h_prev[:, s])
                     for s in range(2)], axis=1)


def moments_2d(op, h):
    """(n, 2, 7): U3_a = int v3 h_a, q_a = int (a v^2 - 5/2) v3 h_a, G1_a, G12_a, G2_a
    (F^a_{201}/4, F^a_{111}/4, F^a_{021}/4) and P_a13, P_a23 = 2 a int v1,2 v3 h_a."""
    g = op.grid
    out = np.zeros(h.shape[:2] + (7,))
    for s in range(2):
        hs = h[:, s]
        out[:, s, 0] = g.U3(hs)
        out[:, s, 1] = g.integrate((op.a[s] * g.vsq - 2.5) * g.V3 * hs)
        out[:, s, 2] = g.G1(hs)
        out[:, s, 3] = g.G12(hs)
        out[:, s, 4] = g.G2(hs)
        out[:, s, 5] = op.a[s] * g.P13(hs)
        out[:, s, 6] = op.a[s] * g.P23(hs)
    return out


def velocity_2d(op, g, mom, amom, delta, N, poiseuille=True):
    """SIS velocity equations on a cross section, eqs. LBE2_true2 (B) and
    LBE2_true1 (A) as printed (two Poisson problems, one per species):
      chi_B lap U_B = -N_B delta (m_A/m_B) div P_B - (d11 G1_B + 2 d12 G12_B + d22 G2_B) + d1 A1_B + d2 A2_B,
      chi_A lap U_A = N_A delta (div P_B - 1) - (d11 G1_A + ...) + d1 A1_A + d2 A2_A,
    with A1_a, A2_a = 2 int v1,2 v3 (L_a + N_a delta h_a^k), div P_B of h^{k+1/2},
    U_a = U3_a / chi_a at the cells next to a wall or solid; the single-gas
    finite-volume discretisation.  mom (n, 2, 7), amom (n, 2, 4); returns U (n, 2)."""
    from . import duct
    N = np.broadcast_to(np.asarray(N, float), (2,))
    PB = (mom[:, 1, 5], mom[:, 1, 6])
    U = np.zeros((mom.shape[0], 2))
    for s in range(2):
        Nd = N[s] * delta
        if s == 1:
            src, coef = 0.0, -Nd / op.a[1]
        else:
            src, coef = (-Nd if poiseuille else 0.0), Nd
        U[:, s] = duct.diffusion_2d(g, mom[:, s], amom[:, s], delta, N[s], duct.POISEUILLE if poiseuille else 0,
                                    chi=op.chi[s], source=src, div_p=PB, div_coef=coef)
    return U


def collide_2d(op, h, dU, delta, poiseuille=True):
    """`collide_1d` with the v2 v3 moments too: amom (n, 2, 4) = {2 int v1 v3 L_a,
    2 int v1 v3 h_a^k, 2 int v2 v3 L_a, 2 int v2 v3 h_a^k}."""
    g = op.grid
    rhs, L, _ = collide_1d(op, h, dU, delta, poiseuille)
    hk = h + np.asarray(dU)[:, :, None, None, None] * correction_shapes(op)
    amom = np.stack([2.0 * g.integrate(g.V1 * g.V3 * L), 2.0 * g.integrate(g.V1 * g.V3 * hk),
                     2.0 * g.integrate(g.V2 * g.V3 * L), 2.0 * g.integrate(g.V2 * g.V3 * hk)], axis=-1)
    return rhs, L, amom


def solve_mixture_2d(op, g, delta, scheme="SIS", Npen=None, eps=1e-8, max_it=5000):
    """Poiseuille flow of the binary mixture through a cross section from h^0 = 0:
    `collide_2d`, `sweep_2d`, `moments_2d`; SIS: `velocity_2d` and the
    correction h_a += 2 a_a (U_a - U_a^{k+1/2}) v3 f_a.  Flow rates
    M_a = sqrt(m/m_A) (1/A) sum U_a dA, Q_a = sqrt(m/m_A) (1/A) sum q_a dA;
    stop when the relative change of all four is below eps."""
    from . import duct
    vg = op.grid
    N = op.nubar() if Npen is None else np.broadcast_to(np.asarray(Npen, float), (2,))
    nf = len(g.cells)
    corr = correction_shapes(op)
    cU = np.array([vg.U3(corr[s]) / op.chi[s] for s in range(2)])
    cq = np.array([vg.integrate((op.a[s] * vg.vsq - 2.5) * vg.V3 * corr[s]) for s in range(2)])
    fac = math.sqrt(op.mbar / op.m[0])
    h = np.zeros((nf, 2) + vg.feq.shape)
    dU = np.zeros((nf, 2))
    M_old = np.zeros(2)
    Q_old = np.zeros(2)
    converged = False
    it = 0
    for it in range(1, max_it + 1):
        rhs, L, amom = collide_2d(op, h, dU, delta)
        h = sweep_2d(op, rhs, g, delta, h)
        mom = moments_2d(op, h)
        U_half = mom[:, :, 0] / op.chi
        if scheme == "SIS":
            dU = velocity_2d(op, g, mom, amom, delta, N) - U_half
        elif scheme == "CIS":
            dU = np.zeros((nf, 2))
        else:
            raise ValueError(scheme)
        Un = U_half + dU * cU
        qn = mom[:, :, 1] + dU * cq
        MQ = [duct.flow_rates_2d(g, Un[:, s], qn[:, s]) for s in range(2)]
        M = fac * np.array([m[0] for m in MQ])
        Q = fac * np.array([m[1] for m in MQ])
        res = float(np.max(np.concatenate([np.abs(M - M_old) / np.maximum(np.abs(M), 1e-300),
                                           np.abs(Q - Q_old) / np.maximum(np.abs(Q), 1e-300)])))
        M_old, Q_old = M, Q
        if res < eps:
            converged = True
            break
    return dict(M=M, Q=Q, iters=it, converged=converged, residual=res, U=Un, q=qn, dU=dU, h_half=h, N=N)
