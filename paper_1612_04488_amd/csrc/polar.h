// Host tables of the polar-coordinate velocity grid (tube flows, Sec. 4) and of
// the fast spectral method taken between its nodes and the Cartesian modes.
#pragma once
#include <string>
#include <vector>

namespace sis {

struct PolarDesc {
  int n_vr = 22, n_th = 40, n_vz = 12;
  double vr_max = 4.0, vz_max = 6.0;
  int n_pad = 0;          // lattice points per axis (0 -> 4 l_pad, rounded to even)
  double l_pad = 0.0;     // half-width of the periodic box (0 -> 2 max(vr_max, vz_max))
  int m_angle = 8;
  int n_threads = 0;
};

struct PolarTables {
  int n_vr = 0, n_th = 0, n_vz = 0, nv = 0;
  std::vector<double> vr, wvr, th, vz;   // nodes per axis; wvr: weights of int g v_r dv_r
  std::vector<double> vnode;             // [3][nv] v1 = v_r cos th, v2 = v_r sin th, v3 = v_z
  std::vector<double> wbase;             // [nv] w_vr dth dvz (one image)
  std::vector<double> feq;               // [nv]
  int np = 0, D = 0;
  double lp = 0, dvc = 0, R = 0, b0 = 0;
  std::vector<double> W;                 // [D]
  // half-space modes without Nyquist components (l and -l share one entry), padded to
  // an even count with a zero-weight mode: xi[3][nm], pair = 2 (1 for l = 0, 0 for the pad)
  int nm = 0, T = 0, Tp = 0;             // T = 2D + 1 multipliers (psi_p, phi_p, beta), Tp even
  std::vector<double> xi, pair;
  std::vector<double> mt_tm;             // [Tp][nm] multipliers, term-major
  std::vector<double> mt_mm;             // [nm][Tp] multipliers, mode-major
};

bool build_polar_tables(const PolarDesc& d, PolarTables& t, std::string& err);

}  // namespace sis
