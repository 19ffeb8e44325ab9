"""Conventional (CIS) and synthetic (SIS) iterative schemes, planar flow.

Paper:
* CIS, eq. LBE_iteration (Sec. 2): nu h^{k+1} + v1 dh^{k+1}/dx1 = L+(h^k) + S.
* SIS, Sec. 2.2 with the tuning parameter N of Sec. 2.5:
  1. from h^k compute A1 = 2 int v1 v3 (L(h^k) + N delta h^k) and solve
     eq. syn_LBE for h^{k+1/2};
  2. moments U3, q3, G1 = F_{2,0,1}/4 of h^{k+1/2};
  3. U^{k+1}: wall node from the VDF, bulk from eq. first_order;
  4. eq. guided: h^{k+1} = h^{k+1/2} + 2 (U^{k+1} - U3^{k+1/2}) v3 f_eq.
* Stop when the relative changes of M and Q between consecutive iterations are
  both below eps (Sec. 2.4).  Start from h^0 = 0 (silent in the paper).
* Default N = nubar / delta (Sec. 2.5), i.e. the delta = 1 nubar.

The collision operator enters only through L+(h) and nu_eq (both linear in
delta), so `fsm` may be any object with `lplus(h)`, `nu`, `grid`, `nubar()`.
"""
import numpy as np

from . import transport as tr
from .velocity import POISEUILLE


class Result:
    def __init__(self, **kw):
        self.__dict__.update(kw)


def solve_1d(fsm, x, delta, flow=POISEUILLE, scheme="SIS", N=None, eps=1e-8,
             max_it=10000, history=False):
    grid = fsm.grid
    if N is None:
        N = fsm.nubar()
    x = np.asarray(x, dtype=np.float64)
    n = len(x)
    S = grid.source(flow)
    nu_d = delta * fsm.nu
    corr = 2.0 * grid.V3 * grid.feq               # eq. guided correction shape
    cU, cq = grid.U3(corr), grid.q3(corr)
    h = np.zeros((n,) + grid.feq.shape)            # h^{k-1/2}
    dU = np.zeros(n)
    M_old = Q_old = 0.0
    res_hist, M_hist, Q_hist = [], [], []
    converged = False
    it = 0
    for it in range(1, max_it + 1):
        hk = h + dU[:, None, None, None] * corr    # h^k
        if delta != 0.0:
            Lp = delta * np.stack([fsm.lplus(c) for c in hk])
        else:
            Lp = np.zeros_like(hk)
        L = Lp - nu_d * hk
        A1 = 2.0 * grid.integrate(grid.V1 * grid.V3 * (L + N * delta * hk))
        h = tr.sweep_1d(Lp + S, nu_d, x, grid)       # h^{k+1/2}
        U_half, q_half, G1 = grid.U3(h), grid.q3(h), grid.G1(h)
        if scheme == "SIS":
            U = tr.diffusion_1d(x, U_half[0], G1, A1, delta, N, flow)
            dU = U - U_half
        elif scheme == "CIS":
            dU = np.zeros(n)
        else:
            raise ValueError(scheme)
        U_new = U_half + dU * cU                   # moments of h^{k+1}
        q_new = q_half + dU * cq
        M = tr.flow_rate_1d(x, U_new)
        Q = tr.flow_rate_1d(x, q_new)
        res = max(abs(M - M_old) / max(abs(M), 1e-300),
                  abs(Q - Q_old) / max(abs(Q), 1e-300))
        res_hist.append(res)
        M_hist.append(M)
        Q_hist.append(Q)
        M_old, Q_old = M, Q
        if res < eps:
            converged = True
            break
    return Result(M=M, Q=Q, iters=it, converged=converged, residual=res,
                  U=U_new, q=q_new, h_half=h, dU=dU, res_hist=np.array(res_hist),
                  M_hist=np.array(M_hist), Q_hist=np.array(Q_hist), N=N)
