// Host-side construction of the velocity grid and of the fast-spectral
// collision tables (no device code).  See planner.cpp for the definitions.
#pragma once
#include <string>
#include <vector>

namespace sis {

struct Quadrature {
  std::vector<double> x, w;
};

// Gauss quadrature for the weight (1-x)^a (1+x)^b on [-1, 1] (Golub-Welsch).
bool gauss_jacobi(int n, double a, double b, Quadrature& q);

// Kernel amplitude b0 for delta = 1 (first Chapman-Enskog viscosity).
double b0_unit(double alpha, double gamma);

// Hard-sphere radial factors of the fast spectral method (closed forms):
// phi(s) = 2 int_0^R rho cos(pi rho s / Lp) d rho, psi(t) = 2 pi int_0^R rho J0(pi rho t / Lp) d rho.
double phi_hs(double s, double R, double Lp);
double psi_hs(double t, double R, double Lp);

// M x M Gauss-Legendre directions on [0, pi]^2 (theta, phi) of the half
// sphere with weights w_a w_b sin(theta_a); D = M^2.
bool half_sphere_directions(int M, std::vector<double>& ex, std::vector<double>& ey, std::vector<double>& ez,
                            std::vector<double>& W);

struct TableDesc {
  int n_v = 16;
  double l_v = 6.0;
  int n_pad = 0;
  int m_angle = 6;
  double r_trunc = 0.0;
  double alpha = 1.0, gamma = 0.0;
  int n_threads = 0;
};

struct HostTables {
  int n = 0, n3 = 0, np = 0, nd = 0, nd3 = 0, D = 0;
  double lv = 0, dv = 0, Lp = 0, R = 0, b0 = 0, nubar = 0, alpha = 1, gamma = 0;
  std::vector<double> v1d;          // [n]
  std::vector<double> feq, nu;      // [n3], nu at delta = 1
  std::vector<double> W;            // [D] direction weights
  std::vector<double> A, B;         // [D][n3]  F^-1[psi_p F f_eq], F^-1[phi_p F f_eq]
  std::vector<double> Psi, Phi;     // [D][nd3] real-space kernels on d in [-(n-1), n-1]^3
  std::vector<double> beta_r;       // [nd3]    real-space loss kernel F^-1[beta]
};

// Radial factors phi(s), psi(t) as the planner evaluates them: closed forms for
// alpha + gamma = 1 (phi) and gamma = 0 (psi), else Gauss-Jacobi rules mapped to
// [0, R] with the weight rho^(alpha+gamma) (phi) or rho^(1-gamma) (psi):
//   phi(s) = 2 sum_k w_k cos(|pi s / Lp| x_k),  psi(t) = 2 pi sum_k w_k J0(pi t x_k / Lp).
struct RadialRule {
  double R = 0, Lp = 0;
  bool phi_closed = true, psi_closed = true;
  std::vector<double> phi_x, phi_w, psi_x, psi_w;
};
bool radial_rule(const TableDesc& d, RadialRule& r, std::string& err);

// Grid, equilibrium, b0, Lp, R and direction weights only (no transforms): fills
// n, n3, np, nd, nd3, lv, dv, Lp, R, alpha, gamma, b0, D, v1d, feq, W.
bool build_grid_tables(const TableDesc& d, HostTables& t, std::string& err);

// Build all tables.  want_kernels = false skips Psi/Phi/beta_r (cheaper).
bool build_host_tables(const TableDesc& d, bool want_kernels, HostTables& t, std::string& err);

}  // namespace sis
