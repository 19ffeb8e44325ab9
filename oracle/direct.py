"""Slow, non-FFT references for the collision operator (oracle pins only).

* `mode_sum_lplus`: the FSM of `collision` written as the explicit spectral
  convolution  (Q+)^_k = N_p^-3 sum_{l + m = k (mod N_p)} beta(l, m) g^_l h^_m,
  beta(l, m) = 4 b0 sum_p W_p phi_p(l) psi_p(m), evaluated in O(N_p^6).  The FFT
  form must equal it to rounding: this pins the pointwise-product /
  convolution bookkeeping, the zero extension, the Nyquist handling and the
  normalisation of the FFT implementation.
* `sigma_quadrature_L` (hard spheres) and `sigma_quadrature_L_ipl` (inverse
  power law, any alpha with gamma = 0): L(h)(v) from the plain definition eq. LBE_collision
  (sigma representation, hard spheres B = b0 |u|) for h = f_eq p(v) with p a
  polynomial: with f(v') f(v*') = f(v) f(v*),
  L(h)(v) = b0 f(v) int dv* f(v*) |u| int dsigma [p(v') + p(v*') - p(v) - p(v*)],
  v', v*' = (v + v*)/2 +- |u| sigma / 2.  Computed by product Gauss quadrature
  in u = v - v* (spherical coordinates) and sigma.  Independent of every FSM
  choice (truncation, directions, padding), so it checks the whole reading.
"""
import math

import numpy as np

from .collision import phi_factor, psi_factor


def full_tables(fsm):
    """phi_p, psi_p on the full N_p^3 spectrum (FFT index order)."""
    Np = fsm.n_pad
    lf = np.fft.fftfreq(Np, 1.0 / Np)
    l0, l1, l2 = np.meshgrid(lf, lf, lf, indexing="ij")
    nyq = (l0 == -Np // 2) | (l1 == -Np // 2) | (l2 == -Np // 2)
    ph = np.empty((fsm.D,) + l0.shape)
    ps = np.empty_like(ph)
    for p, e in enumerate(fsm.dirs):
        s = l0 * e[0] + l1 * e[1] + l2 * e[2]
        perp = np.sqrt(np.maximum((l0 - s * e[0]) ** 2 + (l1 - s * e[1]) ** 2
                                  + (l2 - s * e[2]) ** 2, 0.0))
        a = phi_factor(s, fsm.R, fsm.L_p, fsm.alpha, fsm.gamma)
        b = psi_factor(perp, fsm.R, fsm.L_p, fsm.gamma)
        a[nyq] = 0.0
        b[nyq] = 0.0
        ph[p], ps[p] = a, b
    return ph, ps


def _gain_mode_sum(fsm, ph, ps, g, h):
    Np = fsm.n_pad
    n = Np ** 3
    G = np.fft.fftn(fsm.pad(g)).ravel()
    H = np.fft.fftn(fsm.pad(h)).ravel()
    phf = ph.reshape(fsm.D, n)
    psf = ps.reshape(fsm.D, n)
    beta = 4.0 * fsm.b0 * np.einsum("p,pl,pm->lm", fsm.W, phf, psf)
    k = np.stack(np.unravel_index(np.arange(n), (Np,) * 3), axis=-1)
    out = np.zeros(n, dtype=complex)
    for kk in range(n):
        m = np.ravel_multi_index(((k[kk][:, None] - k.T) % Np), (Np,) * 3)
        out[kk] = np.sum(beta[np.arange(n), m] * G * H[m])
    q = np.fft.ifftn(out.reshape((Np,) * 3) / n)
    return fsm.crop(q), beta


def mode_sum_lplus(fsm, h):
    """L+(h) by explicit spectral convolutions (tiny grids only)."""
    ph, ps = full_tables(fsm)
    feq = fsm.grid.feq
    q1, beta = _gain_mode_sum(fsm, ph, ps, feq, h)
    q2, _ = _gain_mode_sum(fsm, ph, ps, h, feq)
    Np = fsm.n_pad
    H = np.fft.fftn(fsm.pad(h))
    bd = np.diag(beta).reshape((Np,) * 3)
    loss = feq * fsm.crop(np.fft.ifftn(bd * H))
    return (q1 + q2 - loss).real, np.abs(q1.imag).max() + np.abs(q2.imag).max()


def _gauss(a, b, n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (b - a) * x + 0.5 * (b + a), 0.5 * (b - a) * w


def sphere_rule(nt, nph):
    """Product Gauss rule on the unit sphere: points (n, 3), weights (n,)."""
    ct, wt = _gauss(-1.0, 1.0, nt)
    ph, wp = _gauss(0.0, 2.0 * math.pi, nph)
    st = np.sqrt(1.0 - ct ** 2)
    pts = np.stack([np.outer(st, np.cos(ph)), np.outer(st, np.sin(ph)),
                    np.outer(ct, np.ones_like(ph))], axis=-1).reshape(-1, 3)
    return pts, np.outer(wt, wp).ravel()


def sigma_quadrature_L(v, poly, b0, nr=96, nu_ang=(24, 48), ns=(8, 16), rmax=None):
    """Hard-sphere L(f_eq p)(v) at one point v from eq. LBE_collision.

    poly: callable mapping an (..., 3) array of velocities to p(v).
    """
    v = np.asarray(v, dtype=np.float64)
    rmax = rmax or (np.linalg.norm(v) + 8.0)
    r, wr = _gauss(0.0, rmax, nr)
    om, wom = sphere_rule(*nu_ang)
    sg, wsg = sphere_rule(*ns)
    f = lambda x: np.exp(-np.sum(x * x, axis=-1)) / math.pi ** 1.5
    pv = poly(v)
    total = 0.0
    for ri, wri in zip(r, wr):
        u = ri * om                           # (nu, 3), u = v - v*
        vs = v - u
        G = 0.5 * (v + vs)                    # (nu, 3)
        vp = G[:, None, :] + 0.5 * ri * sg[None, :, :]
        vsp = G[:, None, :] - 0.5 * ri * sg[None, :, :]
        br = (poly(vp) + poly(vsp)) @ wsg - 4.0 * math.pi * (pv + poly(vs))
        total += wri * ri ** 2 * ri * np.sum(wom * f(vs) * br)
    return b0 * f(v) * total


def _jacobi_gauss(n, a):
    """Nodes and weights of int_{-1}^{1} (1 - x)^a g(x) dx (Gauss-Jacobi)."""
    from scipy import special
    return special.roots_jacobi(n, a, 0.0)


def sigma_quadrature_L_ipl(v, poly, b0, alpha, nr=96, nu_ang=(24, 48), nx=32, nphi=48, rmax=None):
    """L(f_eq p)(v) at one point v from eq. LBE_collision for the kernel
    B = b0 |u|^alpha sin^(alpha-1)(theta/2) (sigma representation, gamma = 0;
    hard spheres at alpha = 1):
      L(h)(v) = f(v) int dv* f(v*) int dsigma B [p(v') + p(v*') - p(v) - p(v*)],
      v', v*' = (v + v*)/2 +- |u| sigma / 2,  cos theta = sigma . u/|u|.
    sigma is parametrised about u: x = cos theta by a Gauss-Jacobi rule whose
    weight (1 - x)^((alpha-1)/2) carries the grazing-angle factor
    sin^(alpha-1)(theta/2) = ((1 - x)/2)^((alpha-1)/2), and the azimuth by the
    periodic trapezoid rule; u = v - v* by Gauss rules in |u| and direction.
    No FSM choice (truncation, directions, padding, spectral step) enters."""
    v = np.asarray(v, dtype=np.float64)
    rmax = rmax or (np.linalg.norm(v) + 8.0)
    r, wr = _gauss(0.0, rmax, nr)
    om, wom = sphere_rule(*nu_ang)
    a = 0.5 * (alpha - 1.0)
    x, wx = _jacobi_gauss(nx, a)
    wx = wx * 2.0 ** (-a)                         # ((1 - x)/2)^a = 2^-a (1 - x)^a
    ph = 2.0 * math.pi * np.arange(nphi) / nphi
    wsig = np.outer(wx, np.full(nphi, 2.0 * math.pi / nphi)).ravel()   # over (x, phi)
    sx = np.sqrt(np.maximum(1.0 - x * x, 0.0))
    f = lambda y: np.exp(-np.sum(y * y, axis=-1)) / math.pi ** 1.5
    pv = poly(v)
    # orthonormal frame (om, e1, e2) for every direction of u
    t = np.where(np.abs(om[:, 2:3]) < 0.9, np.array([[0.0, 0.0, 1.0]]), np.array([[1.0, 0.0, 0.0]]))
    e1 = np.cross(om, t)
    e1 /= np.linalg.norm(e1, axis=1, keepdims=True)
    e2 = np.cross(om, e1)
    # sigma[u-direction, (x, phi), 3]
    sig = (x[None, :, None, None] * om[:, None, None, :]
           + (sx[:, None] * np.cos(ph)[None, :])[None, :, :, None] * e1[:, None, None, :]
           + (sx[:, None] * np.sin(ph)[None, :])[None, :, :, None] * e2[:, None, None, :])
    sig = sig.reshape(len(om), -1, 3)
    total = 0.0
    for ri, wri in zip(r, wr):
        u = ri * om
        vs = v - u
        G = 0.5 * (v + vs)
        vp = G[:, None, :] + 0.5 * ri * sig
        vsp = G[:, None, :] - 0.5 * ri * sig
        br = (poly(vp) + poly(vsp)) @ wsig - np.sum(wsig) * (pv + poly(vs))
        total += wri * ri ** 2 * ri ** alpha * np.sum(wom * f(vs) * br)
    return b0 * f(v) * total


def sigma_quadrature_mix_L(v, a_, polys, masses, diameters, chi, b0, scale,
                           nr=96, nu_ang=(24, 48), ns=(8, 16)):
    """Binary hard-sphere mixture: L_a(h)(v) at one point v for h_s = f_s p_s.

    Plain sigma representation of the linearized operator of eq. Boltzmann_lin
    (no Carleman form, no truncation, no spectral step): with m_a |v'|^2 +
    m_b |v*'|^2 = m_a |v|^2 + m_b |v*|^2 the Maxwellians factor out,
      L_a = scale sum_b b_ab f_a(v) int dv* f_b(v*) |u| int dsigma
            [p_a(v') + p_b(v*') - p_a(v) - p_b(v*)],
      v' = v - mu_b u + mu_b |u| sigma,  v*' = v* + mu_a u - mu_a |u| sigma,
    u = v - v*, mu_b = m_b/(m_a + m_b), mu_a = 1 - mu_b, b_ab = b0 (d_ab/d_A)^2.
    polys: two callables (species A, B) mapping (..., 3) velocities to p_s.
    """
    v = np.asarray(v, dtype=np.float64)
    m = np.asarray(masses, float)
    d = np.asarray(diameters, float)
    x = np.asarray(chi, float)
    av = m / m[0]
    f = [lambda w, s=s: x[s] * (av[s] / math.pi) ** 1.5 * np.exp(-av[s] * np.sum(w * w, axis=-1))
         for s in range(2)]
    om, wom = sphere_rule(*nu_ang)
    sg, wsg = sphere_rule(*ns)
    pa_v = polys[a_](v)
    out = 0.0
    for b_ in range(2):
        mub = m[b_] / (m[a_] + m[b_])
        mua = 1.0 - mub
        bab = b0 * (0.5 * (d[a_] + d[b_]) / d[0]) ** 2
        rmax = np.linalg.norm(v) + 9.0 / math.sqrt(av[b_])
        r, wr = _gauss(0.0, rmax, nr)
        total = 0.0
        for ri, wri in zip(r, wr):
            u = ri * om
            vs = v - u
            vp = (v - mub * u)[:, None, :] + mub * ri * sg[None, :, :]
            vsp = (vs + mua * u)[:, None, :] - mua * ri * sg[None, :, :]
            br = (polys[a_](vp) + polys[b_](vsp)) @ wsg - 4.0 * math.pi * (pa_v + polys[b_](vs))
            total += wri * ri ** 2 * ri * np.sum(wom * f[b_](vs) * br)
        out += bab * total
    return scale * f[a_](v) * out
