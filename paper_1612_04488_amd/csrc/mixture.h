// Host construction of the fast-spectral tables of a binary hard-sphere
// mixture (species A, B; velocities in units of A's most probable speed).
//
// Operator (eq. Boltzmann_lin of the paper, Sec. 5), unknowns h = (h_A, h_B):
//   L+_a(h) = sum_b Q+_ab(f_a, h_b) + Q+_ab(h_a, f_b) - f_a F^-1[beta_ab F h_b],
//   nu_a = sum_b F^-1[beta_ab F f_b],   L_a = L+_a - nu_a h_a,
// with the Carleman form of unequal masses (2mu = 2 m_b/(m_a+m_b),
// kappa = (m_a - m_b)/(m_a + m_b), |x| <= 2mu R, |y| <= R):
//   Q+_ab(g, h) = 4 b_ab sum_p W_p int_{-R}^{R} |rho| g(v + 2mu rho e_p) (psi_p h)(v - kappa rho e_p) drho,
// evaluated spectrally; for kappa = 0 the rho integral is phi_p in closed
// form, otherwise an m_rho-point Gauss-Legendre rule on [0, R] and its mirror.
// beta_ab = 4 b_ab sum_p W_p phi_p psi_p.  Every table is scaled by the
// viscosity normalisation (delta of the mixture, eq. delta with the mixture
// viscosity and most probable speed).
//
// Each term of L+ is a field X_t(i) times a difference kernel Y_t(i - j) of
// the operator matrix; the tables here are those X and Y per operator block.
#pragma once
#include <string>
#include <vector>

namespace sis {

struct MixDesc {
  int n_v = 16;
  double l_v = 6.0;
  int n_pad = 0;
  int m_angle = 6;
  int m_rho = 8;
  double r_trunc = 0.0;
  double mass[2] = {1.0, 1.0}, diam[2] = {1.0, 1.0}, chi[2] = {0.5, 0.5};
  int n_threads = 0;
};

struct MixTables {
  int n = 0, n3 = 0, np = 0, nd = 0, nd3 = 0, D = 0, m_rho = 0;
  double lv = 0, dv = 0, Lp = 0, R = 0, b0 = 0, scale = 0, mbar_over_mA = 1;
  double a[2] = {1, 1}, chi[2] = {0.5, 0.5};
  double two_mu[2][2] = {{1, 1}, {1, 1}}, kappa[2][2] = {{0, 0}, {0, 0}}, C[2][2] = {{0, 0}, {0, 0}};
  std::vector<double> v1d;                 // [n]
  std::vector<double> prof[2];             // [n] separable profile: f_s = prod of prof_s over axes
  std::vector<double> feq, nu;             // [2][n3]; nu scaled (delta = 1)
  double nubar[2] = {0, 0};                // int nu_s f_s / chi_s
  std::vector<double> ex, ey, ez, W;       // [D]
  std::vector<double> rho, wr;             // [m_rho] Gauss-Legendre on [0, R]
  // kappa = 0 terms: kernels Psi_p = F^-1[psi_p], Phi_p = F^-1[phi_p] ([D][nd3]) and per
  // species fields Fphi_s = F^-1[phi_p F f_s], Fpsi_s = F^-1[psi_p F f_s] ([D][n3], unscaled)
  std::vector<double> Psi, Phi, Fphi[2], Fpsi[2];
  std::vector<double> beta_r;              // [nd3] F^-1[sum_p W_p phi_p psi_p] (unscaled)
};

// Velocity grid, equilibria, directions, rho nodes and the pair constants only (no
// transforms: Psi, Phi, Fphi, Fpsi, beta_r, nu and nubar are left empty).
bool build_mix_grid(const MixDesc& d, MixTables& t, std::string& err);

// Velocity grid, equilibria, collision frequencies, kappa = 0 tables.
bool build_mix_base(const MixDesc& d, MixTables& t, std::string& err);

// Mixture viscosity / viscosity of pure A (first Chapman-Enskog approximation,
// hard spheres, equal number density).
double mix_viscosity_ratio(const double mass[2], const double diam[2], const double chi[2]);

// Term tables of the kappa != 0 gain of pair (a, b) for the direction/node
// items q in [q0, q1), q = p * m_rho + r (p direction, r positive rho node);
// each item yields two terms (+rho_r, -rho_r), written in order at
// X[2 (q - q0) + {0, 1}][n3], Y[...][nd3], fully scaled.
//   kind 0: Q+_ab(f_a, h_b) -> block (a, b): X = F^-1[e^{+} F f_a], Y = F^-1[psi_p e^{-}]
//   kind 1: Q+_ab(h_a, f_b) -> block (a, a): X = F^-1[psi_p e^{-} F f_b], Y = F^-1[e^{+}]
// with e^{+} = e^{i pi 2mu rho l.e_p / Lp}, e^{-} = e^{-i pi kappa rho l.e_p / Lp}.
void build_mix_cross_terms(const MixTables& t, int a, int b, int kind, int q0, int q1, double* X, double* Y,
                           int n_threads);

}  // namespace sis
