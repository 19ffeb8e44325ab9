"""Fast-spectral linearized Boltzmann collision operator (oracle).

Paper: eq. LBE_collision (Sec. 2) defines L = L+ - nu_eq h with
L+ = iint B [f_eq(v') h(v*') + f_eq(v*') h(v') - f_eq(v) h(v*)] dOmega dv*
and nu_eq = iint B f_eq(v*) dOmega dv*.  The paper evaluates it with the fast
spectral method (FSM) of its cited reference, whose formulas it does not print.

Reading taken here (written out from the Carleman form of the gain term, not
copied from anywhere):

* Kernel, sigma representation with deflection angle theta:
  B(|u|, theta) = b0 |u|^alpha sin^(alpha+gamma-1)(theta/2) cos^(-gamma)(theta/2).
  Hard spheres: alpha = 1, gamma = 0.  Inverse power law with viscosity index
  w: alpha = 2(1 - w), gamma = 0.
* b0 is fixed so that the first Chapman-Enskog shear viscosity gives the
  rarefaction parameter delta = p0 l / (mu v_m) of eq. delta (Sec. 2.1), i.e.
  the shear Rayleigh quotient -<v1v2 f, L(v1v2 f)>/<v1v2 f, v1v2 f> in
  L2(1/f_eq) equals delta.  The operator is linear in delta; tables are built
  for delta = 1.
* Carleman form: with x = v' - v, y = v*' - v (x perpendicular to y) the gain is
  Q+(g, h)(v) = iint Bt(x, y) delta(x.y) g(v + x) h(v + y) dx dy,
  Bt = 4 B / |x + y| = 4 b0 |x|^(alpha+gamma-1) |y|^(-gamma) (separable).
* h is zero-extended from the N^3 grid to an N_p^3 periodic box of half-width
  L_p = N_p dv / 2; |x|, |y| are truncated at R = 4 L_p / (3 + sqrt 2).
  x = rho e with e on the half sphere, rho in [-R, R]; (theta, phi) of e are
  M-point Gauss-Legendre nodes on [0, pi] each, weight w_a w_b sin(theta_a).
* Mode l has frequency xi_l = pi l / L_p.  With
  phi(s) = int_{-R}^{R} |rho|^(alpha+gamma) cos(pi rho s / L_p) d rho,
  psi(t) = 2 pi int_0^R rho^(1-gamma) J0(pi rho t / L_p) d rho,
  phi_p(l) = phi(l.e_p), psi_p(l) = psi(|l - (l.e_p) e_p|), both zeroed on
  Nyquist modes:
  Q+(g, h) = 4 b0 sum_p W_p  F^-1[phi_p F g] * F^-1[psi_p F h],
  loss     = f_eq * F^-1[beta F h],  beta = 4 b0 sum_p W_p phi_p psi_p,
  nu_eq    = F^-1[beta F f_eq]  (f_eq zero-extended like h),
  L+(h)    = Q+(f_eq, h) + Q+(h, f_eq) - loss,   L(h) = L+(h) - nu_eq h,
  all restricted to the central N^3 grid.
"""
import math

import numpy as np
from scipy import special

from .velocity import VelocityGrid


# --------------------------------------------------------------------------
# kernel normalisation
# --------------------------------------------------------------------------
def angular_integral(alpha, gamma):
    """I = int_0^pi sin^3(t) sin^(alpha+gamma-1)(t/2) cos^(-gamma)(t/2) dt.

    With t = 2s: sin t = 2 sin s cos s, so the integrand is
    16 sin^(alpha+gamma+2)(s) cos^(3-gamma)(s) over s in [0, pi/2], a Beta
    integral: 8 B((alpha+gamma+3)/2, (4-gamma)/2).
    """
    a = (alpha + gamma + 3.0) / 2.0
    b = (4.0 - gamma) / 2.0
    return 8.0 * math.exp(math.lgamma(a) + math.lgamma(b) - math.lgamma(a + b))


def b0_unit(alpha, gamma):
    """Kernel amplitude b0 for delta = 1.

    First Chapman-Enskog viscosity of B = b0 |u|^alpha Theta(theta): the shear
    bracket evaluates to
    delta = b0 * I * Gamma((7+alpha)/2) * 2^((2+alpha)/2) * 2 sqrt(pi) / 5.
    (Centre-of-mass reduction of -(1/4) iiint B f f* (Delta v1v2)^2, divided by
    int (v1 v2)^2 f_eq = 1/4.)
    """
    g = math.gamma((7.0 + alpha) / 2.0)
    return 1.0 / (angular_integral(alpha, gamma) * g * 2.0 ** ((2.0 + alpha) / 2.0)
                  * 2.0 * math.sqrt(math.pi) / 5.0)


def ipl_alpha(visc_index):
    """Inverse power law: mu ~ T^w gives alpha = 2 (1 - w) (gamma = 0 reading)."""
    return 2.0 * (1.0 - visc_index)


# --------------------------------------------------------------------------
# radial spectral factors phi(s), psi(t)
# --------------------------------------------------------------------------
def _phi_hs(b, R):
    """2 int_0^R rho cos(b rho) d rho (closed form; series for small bR)."""
    b = np.abs(np.asarray(b, dtype=np.float64))
    out = np.empty_like(b)
    x = b * R
    small = x < 0.5
    bs = b[~small]
    out[~small] = 2.0 * (R * np.sin(bs * R) / bs + (np.cos(bs * R) - 1.0) / bs ** 2)
    # 2 R^2 sum_k (-1)^k x^(2k) / ((2k)! (2k+2))
    xs = x[small]
    term = np.ones_like(xs)
    acc = term / 2.0
    for k in range(1, 12):
        term = term * (-(xs ** 2)) / ((2 * k - 1) * (2 * k))
        acc = acc + term / (2 * k + 2)
    out[small] = 2.0 * R ** 2 * acc
    return out


def _jacobi_nodes(a, n, R):
    """Nodes/weights for int_0^R rho^a f(rho) d rho (Gauss-Jacobi, mapped)."""
    x, w = special.roots_jacobi(n, 0.0, a)
    rho = 0.5 * R * (x + 1.0)
    return rho, w * (0.5 * R) ** (a + 1.0)


def phi_factor(s, R, L_p, alpha, gamma, nquad=None):
    """phi(s) = int_{-R}^{R} |rho|^(alpha+gamma) cos(pi rho s / L_p) d rho."""
    s = np.asarray(s, dtype=np.float64)
    b = math.pi * s / L_p
    a = alpha + gamma
    if abs(a - 1.0) < 1e-15:
        return _phi_hs(b, R)
    bmax = float(np.max(np.abs(b))) * R if b.size else 0.0
    n = nquad or int(48 + 0.8 * bmax)
    rho, w = _jacobi_nodes(a, n, R)
    flat = b.reshape(-1)
    out = np.empty_like(flat)
    step = max(1, 2_000_000 // n)
    for i in range(0, flat.size, step):
        out[i:i + step] = 2.0 * np.cos(np.outer(flat[i:i + step], rho)) @ w
    return out.reshape(b.shape)


def psi_factor(t, R, L_p, gamma, nquad=None):
    """psi(t) = 2 pi int_0^R rho^(1-gamma) J0(pi rho t / L_p) d rho."""
    t = np.asarray(t, dtype=np.float64)
    c = math.pi * R * t / L_p
    if gamma == 0.0:
        out = np.empty_like(c)
        nz = c > 0.0
        out[nz] = 2.0 * math.pi * R ** 2 * special.j1(c[nz]) / c[nz]
        out[~nz] = math.pi * R ** 2
        return out
    cmax = float(np.max(c)) if c.size else 0.0
    n = nquad or int(48 + 0.8 * cmax)
    rho, w = _jacobi_nodes(1.0 - gamma, n, R)
    flat = (math.pi * t / L_p).reshape(-1)
    out = np.empty_like(flat)
    step = max(1, 2_000_000 // n)
    for i in range(0, flat.size, step):
        out[i:i + step] = 2.0 * math.pi * special.j0(np.outer(flat[i:i + step], rho)) @ w
    return out.reshape(t.shape)


# --------------------------------------------------------------------------
# directions on the half sphere
# --------------------------------------------------------------------------
def directions(m_angle):
    """M x M Gauss-Legendre directions on [0, pi]^2 and weights w_a w_b sin(theta_a)."""
    x, w = np.polynomial.legendre.leggauss(m_angle)
    t = 0.5 * math.pi * (x + 1.0)
    wt = 0.5 * math.pi * w
    th, ph = np.meshgrid(t, t, indexing="ij")
    wth, wph = np.meshgrid(wt, wt, indexing="ij")
    e = np.stack([np.sin(th) * np.cos(ph), np.sin(th) * np.sin(ph), np.cos(th)], axis=-1)
    W = wth * wph * np.sin(th)
    return e.reshape(-1, 3), W.reshape(-1)


# --------------------------------------------------------------------------
# the operator
# --------------------------------------------------------------------------
class FSM:
    """Fast-spectral L for one gas on a VelocityGrid (delta = 1).

    Arrays on the velocity grid have shape (..., N, N, N).
    """

    def __init__(self, grid: VelocityGrid, n_pad=None, m_angle=6, alpha=1.0,
                 gamma=0.0, r_trunc=None):
        self.grid = grid
        N = grid.n
        self.n_pad = Np = int(n_pad or 2 * N)
        if Np < N or Np % 2:
            raise ValueError("n_pad must be even and >= n_v")
        self.alpha, self.gamma = float(alpha), float(gamma)
        self.L_p = Np * grid.dv / 2.0
        self.R = float(r_trunc) if r_trunc else 4.0 * self.L_p / (3.0 + math.sqrt(2.0))
        self.b0 = b0_unit(alpha, gamma)
        self.off = (Np - N) // 2
        self.dirs, self.W = directions(m_angle)
        self.D = len(self.W)

        # signed integer modes on the half spectrum used by rfftn
        lf = np.fft.fftfreq(Np, 1.0 / Np)            # 0..Np/2-1, -Np/2..-1
        lh = np.arange(Np // 2 + 1, dtype=np.float64)  # 0..Np/2 (Np/2 is Nyquist)
        l0, l1, l2 = np.meshgrid(lf, lf, lh, indexing="ij")
        nyq = (l0 == -Np // 2) | (l1 == -Np // 2) | (l2 == Np // 2)
        lsq = l0 ** 2 + l1 ** 2 + l2 ** 2
        self.phi = np.empty((self.D,) + l0.shape)
        self.psi = np.empty((self.D,) + l0.shape)
        for p, e in enumerate(self.dirs):
            s = l0 * e[0] + l1 * e[1] + l2 * e[2]
            perp = np.sqrt(np.maximum(
                (l0 - s * e[0]) ** 2 + (l1 - s * e[1]) ** 2 + (l2 - s * e[2]) ** 2, 0.0))
            ph = phi_factor(s, self.R, self.L_p, alpha, gamma)
            ps = psi_factor(perp, self.R, self.L_p, gamma)
            ph[nyq] = 0.0
            ps[nyq] = 0.0
            self.phi[p] = ph
            self.psi[p] = ps
        del lsq
        self.beta = 4.0 * self.b0 * np.einsum("p,pijk,pijk->ijk", self.W, self.phi, self.psi)

        F = np.fft.rfftn(self.pad(grid.feq))
        shp = (Np, Np, Np)
        self.A = np.empty((self.D, N, N, N))   # F^-1[psi_p F f_eq]
        self.B = np.empty((self.D, N, N, N))   # F^-1[phi_p F f_eq]
        for p in range(self.D):
            self.A[p] = self.crop(np.fft.irfftn(self.psi[p] * F, s=shp, axes=(-3, -2, -1)))
            self.B[p] = self.crop(np.fft.irfftn(self.phi[p] * F, s=shp, axes=(-3, -2, -1)))
        self.nu = self.crop(np.fft.irfftn(self.beta * F, s=shp, axes=(-3, -2, -1)))

    # zero extension to / restriction from the padded box
    def pad(self, h):
        Np, o, N = self.n_pad, self.off, self.grid.n
        out = np.zeros(h.shape[:-3] + (Np, Np, Np))
        out[..., o:o + N, o:o + N, o:o + N] = h
        return out

    def crop(self, hp):
        o, N = self.off, self.grid.n
        return hp[..., o:o + N, o:o + N, o:o + N]

    def gain(self, g_hat, h_hat):
        """Q+(g, h) from the half spectra of the zero-extended g and h."""
        shp = (self.n_pad,) * 3
        acc = 0.0
        for p in range(self.D):
            acc = acc + self.W[p] * (np.fft.irfftn(self.phi[p] * g_hat, s=shp)
                                     * np.fft.irfftn(self.psi[p] * h_hat, s=shp, axes=(-3, -2, -1)))
        return 4.0 * self.b0 * self.crop(acc)

    def lplus(self, h):
        """L+(h) at delta = 1 for a single cell h of shape (N, N, N)."""
        shp = (self.n_pad,) * 3
        H = np.fft.rfftn(self.pad(h))
        acc = np.zeros_like(h)
        for p in range(self.D):
            acc += self.W[p] * (self.B[p] * self.crop(np.fft.irfftn(self.psi[p] * H, s=shp, axes=(-3, -2, -1)))
                                + self.crop(np.fft.irfftn(self.phi[p] * H, s=shp, axes=(-3, -2, -1))) * self.A[p])
        loss = self.grid.feq * self.crop(np.fft.irfftn(self.beta * H, s=shp, axes=(-3, -2, -1)))
        return 4.0 * self.b0 * acc - loss

    def apply(self, h):
        """L(h) = L+(h) - nu_eq h at delta = 1 (single cell)."""
        return self.lplus(h) - self.nu * h

    def lplus_cells(self, h):
        """L+ for a stack of cells, shape (n_cells, N, N, N)."""
        return np.stack([self.lplus(hc) for hc in h])

    def nubar(self):
        """Average collision frequency int nu_eq f_eq (Sec. 2.5)."""
        return self.grid.integrate(self.nu * self.grid.feq)


def invariants(grid):
    """Collision invariants psi_i in {1, v1, v2, v3, |v|^2} on the grid, shape (5, N, N, N)."""
    return np.stack([np.ones_like(grid.vsq), grid.V1, grid.V2, grid.V3, grid.vsq])


class ProjectedFSM:
    """FSM with the minimum-norm invariant projection of L.

    L <- L - f_eq sum_i c_i psi_i with c = Gram^-1 m, m_i = sum_v w psi_i L,
    Gram_ij = sum_v w psi_i psi_j f_eq: afterwards sum_v w psi_i L = 0 (mass,
    momentum and energy conservation of the discrete operator).  The same
    correction applies to L+ since nu_eq h is unchanged.
    """

    def __init__(self, fsm):
        self.fsm = fsm
        self.grid = fsm.grid
        self.nu = fsm.nu
        self.psi = invariants(fsm.grid)
        g = fsm.grid
        self.gram = g.w * np.einsum("iabc,jabc,abc->ij", self.psi, self.psi, g.feq)

    def project(self, L):
        g = self.grid
        m = g.w * np.einsum("iabc,abc->i", self.psi, L)
        c = np.linalg.solve(self.gram, m)
        return g.feq * np.einsum("i,iabc->abc", c, self.psi)

    def lplus(self, h):
        lp = self.fsm.lplus(h)
        return lp - self.project(lp - self.nu * h)

    def apply(self, h):
        L = self.fsm.apply(h)
        return L - self.project(L)

    def nubar(self):
        return self.fsm.nubar()
