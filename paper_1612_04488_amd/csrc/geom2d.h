// Host construction of the device tables of a 2-D cross-section batch
// (quarter ducts, periodic porous cells): fluid-cell numbering, upwind
// stencils of the transport sweep and the finite-volume diffusion operator.
#pragma once
#include <stdint.h>

#include <string>
#include <vector>

namespace sis {

enum Side { kWall = 0, kSym = 1, kPeriodic = 2 };

struct Case2D {
  int n1 = 0, n2 = 0;
  std::vector<double> f1, f2;        // faces
  int bc[4] = {kWall, kSym, kWall, kSym};   // x1-, x1+, x2-, x2+
  std::vector<uint8_t> solid;        // [n1 * n2], i major
};

struct Tables2D {
  int n_cases = 0;
  int64_t n_cells = 0;               // fluid cells, all cases
  int64_t n_grid = 0;                // grid cells, all cases
  std::vector<int32_t> n1, n2;
  std::vector<int64_t> cell_off;     // [n_cases + 1]
  std::vector<int64_t> grid_off;     // [n_cases + 1]
  std::vector<double> area;          // [n_cases]
  // per fluid cell (global index)
  std::vector<int32_t> cell_grid;    // grid index within its case
  std::vector<int32_t> cell_case;
  // sweep stencil per fluid cell, axis a (0: x1, 1: x2), sign s (0: v > 0, 1: v < 0):
  // coefficients a, b, c of |v| dh/dx ~ a h + b h1 + c h2 and the upwind references
  std::vector<double> st_coef;       // [cell][2][2][3]
  std::vector<int32_t> st_ref;       // [cell][2][2][2] global fluid cell index (or -1)
  std::vector<int8_t> st_kind;       // [cell][2][2][2] 0 none/wall, 1 cell, 2 mirror
  // diffusion tables per grid cell (index within case + grid_off)
  std::vector<int8_t> dflag;         // 0 solid, 1 Dirichlet, 2 unknown
  std::vector<int32_t> gcell;        // global fluid cell index or -1
  std::vector<int32_t> nb;           // [grid][8] E W N S NE NW SE SW: grid index in case or -1
  std::vector<int8_t> nbm;           // [grid][8] mirror bits: 1 = across an x1 plane, 2 = x2 plane
  std::vector<double> npos;          // [grid][4] positions xE, xW, yN, yS
  std::vector<double> fw;            // [grid][4] flux weights E W N S (0: symmetry plane)
  std::vector<double> width;         // [grid][2] w1, w2
  std::vector<double> cpos;          // [grid][2] c1, c2
  std::vector<double> dA;            // [grid]
};

bool build_tables_2d(const std::vector<Case2D>& cases, Tables2D& t, std::string& err);

}  // namespace sis
