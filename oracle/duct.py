"""Two-dimensional cross sections: quarter rectangular ducts and periodic
porous unit cells (oracle).

Paper:
* eq. LBE / eq. syn_LBE with both spatial derivatives (Sec. 2), second-order
  upwind differences; square duct with one quarter simulated and cell sides
  in geometric progression (ratio 1.05) from the wall to the centre
  (Sec. 2.4); rectangular ducts of aspect ratio 2 with the shorter side as
  the length scale (Sec. 5.3); random porous media of staircase discs on a
  uniform grid (Sec. 3.2).
* eq. diffusion_LBE with the tuning parameter N (Sec. 2.2, 2.5):
  lap U = -N delta [Poiseuille] - (d11 G1 + 2 d12 G12 + d22 G2) + d1 A1 + d2 A2,
  G1 = F_201/4, G12 = F_111/4, G2 = F_021/4, Ai = 2 int vi v3 (L + N delta h),
  discretised by a five-point difference; U3 near the boundary taken from the
  VDF.  Flow rates M = (1/A) sum U3 dA, Q = (1/A) sum q3 dA.

Readings (silent in the paper):
* cell-centred grid; a wall or solid face is an upwind node carrying h = 0
  for the velocities leaving it (diffuse reflection of a zero perturbation);
  a symmetry plane is handled by mirror ghost cells (h of the mirrored
  velocity); periodic edges use the previous iterate's values across the
  edge (one-iteration lag);
* upwind stencil along each axis: three-point non-uniform second order from
  the two upwind points, first order when only one upwind point exists;
* quadrant order (+,+), (-,+), (+,-), (-,-) so every mirrored inflow is
  already computed;
* diffusion equation in finite-volume form (symmetric): face fluxes
  (U_N - U_P)/d_PN times the face length, the same second differences for
  G1 and G2, central first differences for A1, A2 and for the cross term;
  moments of solid cells are zero; Dirichlet U = U3(h^{k+1/2}) on fluid cells
  with a wall or solid 4-neighbour; solved exactly (sparse LU).
"""
import numpy as np
from scipy.sparse import coo_matrix
from scipy.sparse.linalg import spsolve

from .velocity import POISEUILLE

WALL, SYM, PERIODIC = 0, 1, 2


class Grid2D:
    """Cell-centred tensor grid with boundary kinds (x1-, x1+, x2-, x2+) and solids."""

    def __init__(self, f1, f2, bc, solid=None):
        self.f1 = np.asarray(f1, float)
        self.f2 = np.asarray(f2, float)
        self.n1, self.n2 = len(f1) - 1, len(f2) - 1
        self.c1 = 0.5 * (self.f1[1:] + self.f1[:-1])
        self.c2 = 0.5 * (self.f2[1:] + self.f2[:-1])
        self.w1 = np.diff(self.f1)
        self.w2 = np.diff(self.f2)
        self.bc = tuple(bc)
        self.solid = np.zeros((self.n1, self.n2), bool) if solid is None else np.asarray(solid, bool)
        self.index = -np.ones((self.n1, self.n2), int)
        fl = np.argwhere(~self.solid)
        self.cells = fl                                  # fluid cells in row-major (i, j) order
        self.index[fl[:, 0], fl[:, 1]] = np.arange(len(fl))
        self.area = (self.f1[-1] - self.f1[0]) * (self.f2[-1] - self.f2[0])
        self.dA = np.outer(self.w1, self.w2)
        self.dirichlet = np.zeros((self.n1, self.n2), bool)
        for i, j in fl:
            for (ii, jj) in ((i - 1, j), (i + 1, j), (i, j - 1), (i, j + 1)):
                kind, q = self._neighbor(ii, jj)
                if kind == "wall" or (kind == "cell" and self.solid[q]):
                    self.dirichlet[i, j] = True

    def _neighbor(self, i, j):
        """Classify cell (i, j), possibly outside the grid: ('cell', (i, j)),
        ('wall', None) or ('mirror', (i', j', axis))."""
        if i < 0 or i >= self.n1:
            side = self.bc[0] if i < 0 else self.bc[1]
            if side == WALL:
                return "wall", None
            if side == PERIODIC:
                return "cell", (i % self.n1, j)
            return "mirror", (-i - 1 if i < 0 else 2 * self.n1 - 1 - i, j, 1)
        if j < 0 or j >= self.n2:
            side = self.bc[2] if j < 0 else self.bc[3]
            if side == WALL:
                return "wall", None
            if side == PERIODIC:
                return "cell", (i, j % self.n2)
            return "mirror", (i, -j - 1 if j < 0 else 2 * self.n2 - 1 - j, 2)
        return "cell", (i, j)


def geometric_faces(n, length, ratio):
    """n cells from the wall (coordinate -length) to the centre (0), sides
    growing by `ratio` towards the centre."""
    w0 = length * (ratio - 1.0) / (ratio ** n - 1.0) if ratio != 1.0 else length / n
    w = w0 * ratio ** np.arange(n)
    f = np.concatenate([[0.0], np.cumsum(w)]) - length
    f[-1] = 0.0
    return f


def duct_quarter(n1, n2, a=0.5, b=0.5, ratio=1.05):
    """Quarter of the duct [-a, a] x [-b, b]: walls at x1 = -a, x2 = -b, symmetry at 0."""
    return Grid2D(geometric_faces(n1, a, ratio), geometric_faces(n2, b, ratio),
                  (WALL, SYM, WALL, SYM))


def periodic_cell(solid):
    """Periodic unit square with a staircase solid mask (uniform cells)."""
    n1, n2 = solid.shape
    return Grid2D(np.linspace(0.0, 1.0, n1 + 1), np.linspace(0.0, 1.0, n2 + 1),
                  (PERIODIC, PERIODIC, PERIODIC, PERIODIC), solid)


def _coeffs(x0, x1, x2):
    """Upwind stencil for s dh/dx at x0 from points x1 (and x2, or None)."""
    d1 = abs(x0 - x1)
    if x2 is None:
        return 1.0 / d1, -1.0 / d1, 0.0
    d2 = abs(x1 - x2)
    return (2 * d1 + d2) / (d1 * (d1 + d2)), -(d1 + d2) / (d1 * d2), d1 / (d2 * (d1 + d2))


def _virtual(g, axis, vi, other):
    """Map a virtual cell index along `axis` (row/column `other`) to
    ('cell', (i, j), position) for a real (possibly periodic-wrapped) fluid
    cell, ('mirror', (i, j), position) for a mirror ghost of a real cell, or
    ('wall', None, None) for a wall side or a solid cell."""
    n = g.n1 if axis == 1 else g.n2
    f = g.f1 if axis == 1 else g.f2
    c = g.c1 if axis == 1 else g.c2
    if 0 <= vi < n:
        real, pos, kind = vi, c[vi], "cell"
    else:
        side = g.bc[(0 if vi < 0 else 1) + (0 if axis == 1 else 2)]
        if side == WALL:
            return "wall", None, None
        if side == PERIODIC:
            real = vi % n
            pos = c[real] + (f[-1] - f[0]) * (1 if vi >= n else -1)
            kind = "cell"
        else:
            plane = f[0] if vi < 0 else f[-1]
            real = -vi - 1 if vi < 0 else 2 * n - 1 - vi
            pos = 2.0 * plane - c[real]
            kind = "mirror"
    ij = (real, other) if axis == 1 else (other, real)
    if g.solid[ij]:
        return "wall", None, None
    return kind, ij, pos


def _axis_points(g, i, j, axis, s):
    """Position of cell (i, j) along `axis` and its (at most two) upwind points
    for velocity sign s: [(position, (kind, (i', j')))], a wall/solid face
    ending the list with kind 'wall'."""
    idx, other = (i, j) if axis == 1 else (j, i)
    w = g.w1 if axis == 1 else g.w2
    pos0 = g.c1[i] if axis == 1 else g.c2[j]
    prev_pos, prev_w = pos0, w[idx]
    pts = []
    for k in (1, 2):
        kind, ij, pos = _virtual(g, axis, idx - s * k, other)
        if kind == "wall":
            pts.append((prev_pos - s * prev_w / 2.0, ("wall", None)))
            break
        pts.append((pos, (kind, ij)))
        prev_pos, prev_w = pos, w[ij[0] if axis == 1 else ij[1]]
    return pos0, pts


def sweep_2d(rhs, nu_d, g, vg, h_prev):
    """Solve nu_d h + v1 dh/dx1 + v2 dh/dx2 = rhs on the fluid cells.

    rhs, h_prev: (n_fluid, N, N, N).  Returns h (same shape).
    Quadrants (+,+), (-,+), (+,-), (-,-); within a quadrant cells are visited
    in upwind order (row-major with the sweep directions).
    """
    N = vg.n
    h = h_prev.copy()
    half = N // 2
    for s1, s2 in ((1, 1), (-1, 1), (1, -1), (-1, -1)):
        j1 = np.arange(half, N) if s1 > 0 else np.arange(0, half)
        j2 = np.arange(half, N) if s2 > 0 else np.arange(0, half)
        sl = np.ix_(j1, j2, np.arange(N))
        av1 = np.abs(vg.V1[sl])
        av2 = np.abs(vg.V2[sl])
        mir1 = np.ix_(N - 1 - j1, j2, np.arange(N))     # velocity mirrored in v1
        mir2 = np.ix_(j1, N - 1 - j2, np.arange(N))
        I = range(g.n1) if s1 > 0 else range(g.n1 - 1, -1, -1)
        J = range(g.n2) if s2 > 0 else range(g.n2 - 1, -1, -1)
        for j in J:
            for i in I:
                if g.solid[i, j]:
                    continue
                k = g.index[i, j]
                acc = rhs[k][sl].copy()
                diag = nu_d[sl].copy()
                for axis, s, av in ((1, s1, av1), (2, s2, av2)):
                    pos0, pts = _axis_points(g, i, j, axis, s)
                    x1p = pts[0][0]
                    x2p = pts[1][0] if len(pts) > 1 else None
                    a, b, c = _coeffs(pos0, x1p, x2p)
                    diag = diag + av * a
                    for coef, (pos, ref) in zip((b, c), pts):
                        if ref[0] == "wall":
                            continue
                        if ref[0] == "mirror":
                            mi, mj = ref[1]
                            src = h[g.index[mi, mj]][mir1 if axis == 1 else mir2]
                        else:
                            ii, jj = ref[1]
                            src = h[g.index[ii, jj]][sl]   # current sweep if done, else lagged
                        acc = acc - av * coef * src
                h[k][sl] = acc / diag
    return h


def moments_2d(vg, h):
    """Per fluid cell: U3, q3, G1, G12, G2, P13, P23."""
    return np.stack([vg.U3(h), vg.q3(h), vg.G1(h), vg.G12(h), vg.G2(h), vg.P13(h), vg.P23(h)], axis=1)


def _field(g, vals):
    f = np.zeros((g.n1, g.n2))
    f[g.cells[:, 0], g.cells[:, 1]] = vals
    return f


def _val(g, F, i, j, parity):
    """Value of field F at (i, j) with mirror ghosts (parity (p1, p2)) and periodic wrap."""
    s = 1.0
    if i < 0 or i >= g.n1:
        if g.bc[0 if i < 0 else 1] == PERIODIC:
            i %= g.n1
        elif g.bc[0 if i < 0 else 1] == SYM:
            i = -i - 1 if i < 0 else 2 * g.n1 - 1 - i
            s *= parity[0]
        else:
            return 0.0
    if j < 0 or j >= g.n2:
        if g.bc[2 if j < 0 else 3] == PERIODIC:
            j %= g.n2
        elif g.bc[2 if j < 0 else 3] == SYM:
            j = -j - 1 if j < 0 else 2 * g.n2 - 1 - j
            s *= parity[1]
        else:
            return 0.0
    return s * F[i, j]


def _pos1(g, i):
    if 0 <= i < g.n1:
        return g.c1[i]
    L = g.f1[-1] - g.f1[0]
    if g.bc[0 if i < 0 else 1] == PERIODIC:
        return g.c1[i % g.n1] + (L if i >= g.n1 else -L)
    plane = g.f1[0] if i < 0 else g.f1[-1]
    return 2 * plane - g.c1[-i - 1 if i < 0 else 2 * g.n1 - 1 - i]


def _pos2(g, j):
    if 0 <= j < g.n2:
        return g.c2[j]
    L = g.f2[-1] - g.f2[0]
    if g.bc[2 if j < 0 else 3] == PERIODIC:
        return g.c2[j % g.n2] + (L if j >= g.n2 else -L)
    plane = g.f2[0] if j < 0 else g.f2[-1]
    return 2 * plane - g.c2[-j - 1 if j < 0 else 2 * g.n2 - 1 - j]


def diffusion_2d(g, mom, amom, delta, N, flow, chi=1.0, source=None, div_p=None, div_coef=0.0):
    """Solve the discrete eq. diffusion_LBE; returns U on the fluid cells.

    mom: (n_fluid, >= 5) with U3, q3, G1, G12, G2 of h^{k+1/2};
    amom: (n_fluid, 4) {2 sum w v1 v3 L, 2 sum w v1 v3 h, 2 sum w v2 v3 L, 2 sum w v2 v3 h}.
    Species form (eqs. LBE2_true2, LBE2_true1): chi lap U = source + div_coef
    (d1 P13 + d2 P23) - (...) + d1 A1 + d2 A2 with U = U3 / chi, div_p =
    (P13, P23) per fluid cell; source None -> -N delta for Poiseuille flow.
    """
    Uh = _field(g, mom[:, 0] / chi)
    if div_p is not None:
        P13, P23 = _field(g, div_p[0]), _field(g, div_p[1])
    G1, G12, G2 = _field(g, mom[:, 2]), _field(g, mom[:, 3]), _field(g, mom[:, 4])
    A1 = _field(g, amom[:, 0] + N * delta * amom[:, 1])
    A2 = _field(g, amom[:, 2] + N * delta * amom[:, 3])
    # parities under the x1- and x2-mirrors
    EV, O1, O2, O12 = (1, 1), (-1, 1), (1, -1), (-1, -1)
    unk = (~g.solid) & (~g.dirichlet)
    uid = -np.ones((g.n1, g.n2), int)
    cells = np.argwhere(unk)
    uid[cells[:, 0], cells[:, 1]] = np.arange(len(cells))
    rows, cols, vals = [], [], []
    b = np.zeros(len(cells))

    def d1(F, par, i, j):
        return (_val(g, F, i + 1, j, par) - _val(g, F, i - 1, j, par)) / (_pos1(g, i + 1) - _pos1(g, i - 1))

    def d2(F, par, i, j):
        return (_val(g, F, i, j + 1, par) - _val(g, F, i, j - 1, par)) / (_pos2(g, j + 1) - _pos2(g, j - 1))

    def d11(F, par, i, j):
        fe, fw, fp = _val(g, F, i + 1, j, par), _val(g, F, i - 1, j, par), F[i, j]
        de, dw = _pos1(g, i + 1) - g.c1[i], g.c1[i] - _pos1(g, i - 1)
        return ((fe - fp) / de - (fp - fw) / dw) / g.w1[i]

    def d22(F, par, i, j):
        fn, fs, fp = _val(g, F, i, j + 1, par), _val(g, F, i, j - 1, par), F[i, j]
        dn, ds = _pos2(g, j + 1) - g.c2[j], g.c2[j] - _pos2(g, j - 1)
        return ((fn - fp) / dn - (fp - fs) / ds) / g.w2[j]

    for r, (i, j) in enumerate(cells):
        rhs = 0.0
        if source is not None:
            rhs += source
        elif flow == POISEUILLE:
            rhs -= N * delta
        if div_p is not None:
            rhs += div_coef * (d1(P13, O1, i, j) + d2(P23, O2, i, j))
        cross = (_d2_at(g, G12, O12, i + 1, j) - _d2_at(g, G12, O12, i - 1, j)) / (_pos1(g, i + 1) - _pos1(g, i - 1))
        rhs -= d11(G1, EV, i, j) + 2.0 * cross + d22(G2, EV, i, j)
        rhs += d1(A1, O1, i, j) + d2(A2, O2, i, j)
        # -lap U * dA = sum_faces (U_P - U_N) len / dist
        bi = -(rhs / chi) * g.dA[i, j]
        diag = 0.0
        for (ii, jj, L, dist) in ((i + 1, j, g.w2[j], _pos1(g, i + 1) - g.c1[i]),
                                  (i - 1, j, g.w2[j], g.c1[i] - _pos1(g, i - 1)),
                                  (i, j + 1, g.w1[i], _pos2(g, j + 1) - g.c2[j]),
                                  (i, j - 1, g.w1[i], g.c2[j] - _pos2(g, j - 1))):
            wgt = L / dist
            kind, q = g._neighbor(ii, jj)
            if kind == "mirror":
                continue                      # zero flux through a symmetry plane (U even)
            qi, qj = q
            diag += wgt
            if unk[qi, qj]:
                rows.append(r)
                cols.append(uid[qi, qj])
                vals.append(-wgt)
            else:
                bi += wgt * Uh[qi, qj]        # Dirichlet neighbour
        rows.append(r)
        cols.append(r)
        vals.append(diag)
        b[r] = bi
    A = coo_matrix((vals, (rows, cols)), shape=(len(cells), len(cells))).tocsr()
    x = spsolve(A, b) if len(cells) else np.zeros(0)
    U = Uh.copy()
    U[cells[:, 0], cells[:, 1]] = x
    return U[g.cells[:, 0], g.cells[:, 1]]


def _d2_at(g, F, par, i, j):
    """Central x2-difference of F at (i, j) (i may be a ghost/wrapped index)."""
    def val(ii, jj):
        return _val(g, F, ii, jj, par)
    return (val(i, j + 1) - val(i, j - 1)) / (_pos2(g, j + 1) - _pos2(g, j - 1))


def flow_rates_2d(g, U, q):
    dA = g.dA[g.cells[:, 0], g.cells[:, 1]]
    return float(np.sum(U * dA) / g.area), float(np.sum(q * dA) / g.area)


def solve_2d(fsm, g, delta, flow=POISEUILLE, scheme="SIS", N=None, eps=1e-8, max_it=5000):
    """CIS / SIS outer iterations on a 2-D cross section (h^0 = 0)."""
    vg = fsm.grid
    if N is None:
        N = fsm.nubar()
    nf = len(g.cells)
    S = vg.source(flow)
    nu_d = delta * fsm.nu
    corr = 2.0 * vg.V3 * vg.feq
    cU, cq = vg.U3(corr), vg.q3(corr)
    h = np.zeros((nf,) + vg.feq.shape)
    dU = np.zeros(nf)
    M_old = Q_old = 0.0
    it = 0
    converged = False
    for it in range(1, max_it + 1):
        hk = h + dU[:, None, None, None] * corr
        Lp = delta * np.stack([fsm.lplus(c) for c in hk]) if delta != 0 else np.zeros_like(hk)
        L = Lp - nu_d * hk
        w2 = lambda f: vg.integrate(f)
        amom = np.stack([w2(2 * vg.V1 * vg.V3 * L), w2(2 * vg.V1 * vg.V3 * hk),
                         w2(2 * vg.V2 * vg.V3 * L), w2(2 * vg.V2 * vg.V3 * hk)], axis=1)
        h = sweep_2d(Lp + S, nu_d, g, vg, h)
        mom = moments_2d(vg, h)
        if scheme == "SIS":
            U = diffusion_2d(g, mom, amom, delta, N, flow)
            dU = U - mom[:, 0]
        else:
            dU = np.zeros(nf)
        Un = mom[:, 0] + dU * cU
        qn = mom[:, 1] + dU * cq
        M, Q = flow_rates_2d(g, Un, qn)
        res = max(abs(M - M_old) / max(abs(M), 1e-300), abs(Q - Q_old) / max(abs(Q), 1e-300))
        M_old, Q_old = M, Q
        if res < eps:
            converged = True
            break
    return dict(M=M, Q=Q, iters=it, converged=converged, residual=res, U=Un, q=qn, h=h, dU=dU)
