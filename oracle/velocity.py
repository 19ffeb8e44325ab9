"""Discrete velocity space, equilibrium and source terms.

Paper: Sec. 2 (equilibrium f_eq = pi^{-3/2} exp(-|v|^2); sources for Poiseuille
and thermal-transpiration flow with X_P = X_T = -1).

Reading (the paper defers the velocity grid to its cited FSM reference):
a uniform, cell-centred, mirror-symmetric grid on [-L_v, L_v]^3,
v_j = -L_v + (j + 1/2) dv, dv = 2 L_v / N, quadrature weight dv^3 (midpoint
rule).  There is no v = 0 node on any axis.
"""
import numpy as np

POISEUILLE = 1
TRANSPIRATION = 2


class VelocityGrid:
    """Uniform N^3 velocity grid on [-l_v, l_v]^3 (array axes: v1, v2, v3)."""

    def __init__(self, n_v, l_v=6.0):
        if n_v % 2:
            raise ValueError("n_v must be even (no v = 0 node)")
        self.n = int(n_v)
        self.l_v = float(l_v)
        self.dv = 2.0 * self.l_v / self.n
        self.v1d = -self.l_v + (np.arange(self.n) + 0.5) * self.dv
        self.V1, self.V2, self.V3 = np.meshgrid(self.v1d, self.v1d, self.v1d,
                                                indexing="ij")
        self.vsq = self.V1 ** 2 + self.V2 ** 2 + self.V3 ** 2
        self.w = self.dv ** 3
        self.feq = np.exp(-self.vsq) / np.pi ** 1.5

    def integrate(self, f):
        """Midpoint rule over velocity space; f has the grid as its last 3 axes."""
        return self.w * f.sum(axis=(-3, -2, -1))

    def source(self, flow):
        """S of Sec. 2 with X_P = X_T = -1."""
        if flow == POISEUILLE:
            return self.V3 * self.feq
        if flow == TRANSPIRATION:
            return self.V3 * (self.vsq - 2.5) * self.feq
        raise ValueError(flow)

    # macroscopic moments of Sec. 2 and the Hermite moment F_{2,0,1}/4 of Sec. 2.1
    def U3(self, h):
        return self.integrate(self.V3 * h)

    def q3(self, h):
        return self.integrate((self.vsq - 2.5) * self.V3 * h)

    def P13(self, h):
        return self.integrate(2.0 * self.V1 * self.V3 * h)

    def P23(self, h):
        return self.integrate(2.0 * self.V2 * self.V3 * h)

    def G1(self, h):
        """F_{2,0,1}/4 = int v3 (2 v1^2 - 1) h  (H_2(v) = 4v^2 - 2, H_1(v) = 2v)."""
        return self.integrate(self.V3 * (2.0 * self.V1 ** 2 - 1.0) * h)

    def G12(self, h):
        """F_{1,1,1}/4 = int 2 v1 v2 v3 h."""
        return self.integrate(2.0 * self.V1 * self.V2 * self.V3 * h)

    def G2(self, h):
        """F_{0,2,1}/4 = int v3 (2 v2^2 - 1) h."""
        return self.integrate(self.V3 * (2.0 * self.V2 ** 2 - 1.0) * h)
