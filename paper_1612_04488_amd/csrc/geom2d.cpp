// Host tables of 2-D cross sections (see geom2d.h).
//
// Discretisation (cell-centred tensor grid):
//  * transport: along each axis the upwind derivative at a cell uses its two
//    upwind points with the three-point non-uniform second-order formula, or
//    first order when only one exists.  Upwind points are fluid cells
//    (periodic edges wrap; the value across the edge is whatever the sweep
//    buffer holds, i.e. the previous iterate), mirror ghosts across a
//    symmetry plane (value of the mirrored velocity at the real cell), or a
//    wall / solid face, which ends the list and carries h = 0.
//  * diffusion: finite-volume five-point operator, flux weight = face length
//    / centre distance, zero flux through symmetry planes; Dirichlet cells are
//    the fluid cells with a wall or solid 4-neighbour.
#include "geom2d.h"

#include <cmath>

namespace sis {

namespace {

struct Virt {
  int kind;     // 0 wall/solid, 1 cell, 2 mirror
  int i, j;     // real cell
  double pos;   // coordinate along the axis
};

Virt resolve(const Case2D& c, const std::vector<double>& c1, const std::vector<double>& c2, int axis,
             int vi, int other) {
  const int n = axis == 0 ? c.n1 : c.n2;
  const std::vector<double>& f = axis == 0 ? c.f1 : c.f2;
  const std::vector<double>& cc = axis == 0 ? c1 : c2;
  int real;
  double pos;
  int kind;
  if (vi >= 0 && vi < n) {
    real = vi;
    pos = cc[vi];
    kind = 1;
  } else {
    const int side = c.bc[(vi < 0 ? 0 : 1) + (axis == 0 ? 0 : 2)];
    if (side == kWall) return {0, -1, -1, 0.0};
    if (side == kPeriodic) {
      real = ((vi % n) + n) % n;
      pos = cc[real] + (f[n] - f[0]) * (vi >= n ? 1.0 : -1.0);
      kind = 1;
    } else {
      const double plane = vi < 0 ? f[0] : f[n];
      real = vi < 0 ? -vi - 1 : 2 * n - 1 - vi;
      pos = 2.0 * plane - cc[real];
      kind = 2;
    }
  }
  const int i = axis == 0 ? real : other;
  const int j = axis == 0 ? other : real;
  if (c.solid.size() && c.solid[static_cast<size_t>(i) * c.n2 + j]) return {0, -1, -1, 0.0};
  return {kind, i, j, pos};
}

// Full 2-D resolution of (i, j) possibly outside the grid: grid cell + mirror bits, or wall.
bool resolve2(const Case2D& c, int i, int j, int* ri, int* rj, int* bits) {
  *bits = 0;
  if (i < 0 || i >= c.n1) {
    const int side = c.bc[i < 0 ? 0 : 1];
    if (side == kWall) return false;
    if (side == kPeriodic) i = ((i % c.n1) + c.n1) % c.n1;
    else { i = i < 0 ? -i - 1 : 2 * c.n1 - 1 - i; *bits |= 1; }
  }
  if (j < 0 || j >= c.n2) {
    const int side = c.bc[j < 0 ? 2 : 3];
    if (side == kWall) return false;
    if (side == kPeriodic) j = ((j % c.n2) + c.n2) % c.n2;
    else { j = j < 0 ? -j - 1 : 2 * c.n2 - 1 - j; *bits |= 2; }
  }
  if (c.solid.size() && c.solid[static_cast<size_t>(i) * c.n2 + j]) return false;
  *ri = i;
  *rj = j;
  return true;
}

double pos_along(const Case2D& c, const std::vector<double>& cc, int axis, int vi) {
  const int n = axis == 0 ? c.n1 : c.n2;
  const std::vector<double>& f = axis == 0 ? c.f1 : c.f2;
  if (vi >= 0 && vi < n) return cc[vi];
  const int side = c.bc[(vi < 0 ? 0 : 1) + (axis == 0 ? 0 : 2)];
  if (side == kPeriodic) return cc[((vi % n) + n) % n] + (f[n] - f[0]) * (vi >= n ? 1.0 : -1.0);
  const double plane = vi < 0 ? f[0] : f[n];
  return 2.0 * plane - cc[vi < 0 ? -vi - 1 : 2 * n - 1 - vi];
}

}  // namespace

bool build_tables_2d(const std::vector<Case2D>& cases, Tables2D& t, std::string& err) {
  t = Tables2D();
  t.n_cases = static_cast<int>(cases.size());
  t.cell_off.assign(t.n_cases + 1, 0);
  t.grid_off.assign(t.n_cases + 1, 0);
  for (int k = 0; k < t.n_cases; ++k) {
    const Case2D& c = cases[k];
    if (c.n1 < 2 || c.n2 < 2) { err = "2-D case needs at least 2 x 2 cells"; return false; }
    if (static_cast<int>(c.f1.size()) != c.n1 + 1 || static_cast<int>(c.f2.size()) != c.n2 + 1) {
      err = "face arrays must have n + 1 entries";
      return false;
    }
    for (int i = 0; i < c.n1; ++i)
      if (!(c.f1[i + 1] > c.f1[i])) { err = "x1 faces must increase"; return false; }
    for (int j = 0; j < c.n2; ++j)
      if (!(c.f2[j + 1] > c.f2[j])) { err = "x2 faces must increase"; return false; }
    if (!c.solid.empty() && c.solid.size() != static_cast<size_t>(c.n1) * c.n2) {
      err = "solid mask size mismatch";
      return false;
    }
    int64_t nf = 0;
    for (int i = 0; i < c.n1 * c.n2; ++i) nf += (c.solid.empty() || !c.solid[i]) ? 1 : 0;
    if (nf == 0) { err = "case has no fluid cell"; return false; }
    t.n1.push_back(c.n1);
    t.n2.push_back(c.n2);
    t.cell_off[k + 1] = t.cell_off[k] + nf;
    t.grid_off[k + 1] = t.grid_off[k] + static_cast<int64_t>(c.n1) * c.n2;
    t.area.push_back((c.f1[c.n1] - c.f1[0]) * (c.f2[c.n2] - c.f2[0]));
  }
  t.n_cells = t.cell_off.back();
  t.n_grid = t.grid_off.back();
  t.cell_grid.resize(t.n_cells);
  t.cell_case.resize(t.n_cells);
  t.st_coef.assign(t.n_cells * 12, 0.0);
  t.st_ref.assign(t.n_cells * 8, -1);
  t.st_kind.assign(t.n_cells * 8, 0);
  t.dflag.assign(t.n_grid, 0);
  t.gcell.assign(t.n_grid, -1);
  t.nb.assign(t.n_grid * 8, -1);
  t.nbm.assign(t.n_grid * 8, 0);
  t.npos.assign(t.n_grid * 4, 0.0);
  t.fw.assign(t.n_grid * 4, 0.0);
  t.width.assign(t.n_grid * 2, 0.0);
  t.cpos.assign(t.n_grid * 2, 0.0);
  t.dA.assign(t.n_grid, 0.0);

  for (int k = 0; k < t.n_cases; ++k) {
    const Case2D& c = cases[k];
    std::vector<double> c1(c.n1), c2(c.n2), w1(c.n1), w2(c.n2);
    for (int i = 0; i < c.n1; ++i) { c1[i] = 0.5 * (c.f1[i] + c.f1[i + 1]); w1[i] = c.f1[i + 1] - c.f1[i]; }
    for (int j = 0; j < c.n2; ++j) { c2[j] = 0.5 * (c.f2[j] + c.f2[j + 1]); w2[j] = c.f2[j + 1] - c.f2[j]; }
    auto solid = [&](int i, int j) { return !c.solid.empty() && c.solid[static_cast<size_t>(i) * c.n2 + j]; };
    std::vector<int32_t> gidx(static_cast<size_t>(c.n1) * c.n2, -1);
    int64_t next = t.cell_off[k];
    for (int i = 0; i < c.n1; ++i)
      for (int j = 0; j < c.n2; ++j)
        if (!solid(i, j)) {
          gidx[static_cast<size_t>(i) * c.n2 + j] = static_cast<int32_t>(next);
          t.cell_grid[next] = i * c.n2 + j;
          t.cell_case[next] = k;
          ++next;
        }
    // sweep stencils
    for (int i = 0; i < c.n1; ++i)
      for (int j = 0; j < c.n2; ++j) {
        if (solid(i, j)) continue;
        const int64_t cell = gidx[static_cast<size_t>(i) * c.n2 + j];
        for (int axis = 0; axis < 2; ++axis)
          for (int sg = 0; sg < 2; ++sg) {
            const int s = sg == 0 ? 1 : -1;
            const int idx = axis == 0 ? i : j, other = axis == 0 ? j : i;
            const std::vector<double>& w = axis == 0 ? w1 : w2;
            const double pos0 = axis == 0 ? c1[i] : c2[j];
            double prev_pos = pos0, prev_w = w[idx];
            double pts[2];
            int np = 0;
            int32_t ref[2] = {-1, -1};
            int8_t kind[2] = {0, 0};
            for (int st = 1; st <= 2; ++st) {
              Virt v = resolve(c, c1, c2, axis, idx - s * st, other);
              if (v.kind == 0) {
                pts[np++] = prev_pos - s * prev_w / 2.0;   // wall / solid face, h = 0
                break;
              }
              pts[np] = v.pos;
              ref[np] = gidx[static_cast<size_t>(v.i) * c.n2 + v.j];
              kind[np] = static_cast<int8_t>(v.kind);
              ++np;
              prev_pos = v.pos;
              prev_w = w[axis == 0 ? v.i : v.j];
            }
            double a, b, cc;
            const double d1 = std::fabs(pos0 - pts[0]);
            if (np == 1) {
              a = 1.0 / d1; b = -1.0 / d1; cc = 0.0;
            } else {
              const double d2 = std::fabs(pts[0] - pts[1]);
              a = (2.0 * d1 + d2) / (d1 * (d1 + d2));
              b = -(d1 + d2) / (d1 * d2);
              cc = d1 / (d2 * (d1 + d2));
            }
            const int64_t o = (cell * 2 + axis) * 2 + sg;
            t.st_coef[o * 3 + 0] = a;
            t.st_coef[o * 3 + 1] = b;
            t.st_coef[o * 3 + 2] = cc;
            for (int q = 0; q < 2; ++q) {
              t.st_ref[o * 2 + q] = ref[q];
              t.st_kind[o * 2 + q] = kind[q];
            }
          }
      }
    // diffusion tables
    const int di[8] = {1, -1, 0, 0, 1, -1, 1, -1};
    const int dj[8] = {0, 0, 1, -1, 1, 1, -1, -1};
    for (int i = 0; i < c.n1; ++i)
      for (int j = 0; j < c.n2; ++j) {
        const int64_t g = t.grid_off[k] + static_cast<int64_t>(i) * c.n2 + j;
        t.width[g * 2 + 0] = w1[i];
        t.width[g * 2 + 1] = w2[j];
        t.cpos[g * 2 + 0] = c1[i];
        t.cpos[g * 2 + 1] = c2[j];
        t.dA[g] = w1[i] * w2[j];
        if (solid(i, j)) { t.dflag[g] = 0; continue; }
        t.gcell[g] = gidx[static_cast<size_t>(i) * c.n2 + j];
        bool dir = false;
        for (int q = 0; q < 8; ++q) {
          int ri, rj, bits;
          if (resolve2(c, i + di[q], j + dj[q], &ri, &rj, &bits)) {
            t.nb[g * 8 + q] = ri * c.n2 + rj;
            t.nbm[g * 8 + q] = static_cast<int8_t>(bits);
          } else if (q < 4) {
            dir = true;
          }
        }
        t.dflag[g] = dir ? 1 : 2;
        t.npos[g * 4 + 0] = pos_along(c, c1, 0, i + 1);
        t.npos[g * 4 + 1] = pos_along(c, c1, 0, i - 1);
        t.npos[g * 4 + 2] = pos_along(c, c2, 1, j + 1);
        t.npos[g * 4 + 3] = pos_along(c, c2, 1, j - 1);
        for (int q = 0; q < 4; ++q) {
          if (t.nb[g * 8 + q] < 0) continue;
          const bool mirror = (q < 2 && (t.nbm[g * 8 + q] & 1)) || (q >= 2 && (t.nbm[g * 8 + q] & 2));
          if (mirror) continue;   // zero flux through a symmetry plane
          const double len = q < 2 ? w2[j] : w1[i];
          const double dist = q == 0 ? t.npos[g * 4 + 0] - c1[i]
                            : q == 1 ? c1[i] - t.npos[g * 4 + 1]
                            : q == 2 ? t.npos[g * 4 + 2] - c2[j]
                                     : c2[j] - t.npos[g * 4 + 3];
          t.fw[g * 4 + q] = len / dist;
        }
      }
  }
  return true;
}

}  // namespace sis
