// Host construction of the fast-spectral collision tables.
//
// Operator (eq. LBE_collision of the paper, evaluated with the cited fast
// spectral method in Carleman form): h lives on n^3 velocity points, is
// zero-extended to an np^3 periodic box (half-width Lp = np dv / 2), and
//   L+(h) = Q+(f_eq, h) + Q+(h, f_eq) - f_eq F^-1[beta F h],
//   Q+(g, h) = 4 b0 sum_p W_p F^-1[phi_p F g] F^-1[psi_p F h],
//   phi_p(l) = phi(l.e_p), psi_p(l) = psi(|l - (l.e_p) e_p|),
//   phi(s) = int_{-R}^{R} |rho|^(alpha+gamma) cos(pi rho s / Lp) d rho,
//   psi(t) = 2 pi int_0^R rho^(1-gamma) J0(pi rho t / Lp) d rho,
//   beta = 4 b0 sum_p W_p phi_p psi_p, Nyquist modes zeroed.
// Because a pointwise product in v of two inverse transforms is a
// convolution, every term of L+ is a product of an n^3 field with a discrete
// convolution of h:
//   F^-1[psi_p F h](i) = sum_j Psi_p(i - j) h(j),  Psi_p = F^-1[psi_p],
// and likewise Phi_p, beta_r = F^-1[beta].  The tables built here are those
// real-space kernels on the difference grid d in [-(n-1), n-1]^3 and the
// f_eq fields A_p = F^-1[psi_p F f_eq], B_p = F^-1[phi_p F f_eq],
// nu = F^-1[beta F f_eq] on the n^3 grid, all by pruned separable inverse
// DFTs (only the needed outputs are formed).
#include "planner.h"

#include "pruned_dft.h"

#include <algorithm>
#include <cmath>
#include <complex>
#include <thread>

namespace sis {

namespace {

const double kPi = 3.14159265358979323846;

// Implicit symmetric QL iteration on a tridiagonal matrix (diagonal d,
// sub-diagonal e[i] coupling i and i+1).  On return d holds the eigenvalues;
// z, initialised to the first unit vector, holds the first components of
// the eigenvectors.
bool tridiagonal_ql(std::vector<double>& d, std::vector<double>& e, std::vector<double>& z) {
  const int n = static_cast<int>(d.size());
  e.resize(n, 0.0);
  e[n - 1] = 0.0;
  for (int l = 0; l < n; ++l) {
    for (int iter = 0;; ++iter) {
      int m = l;
      for (; m < n - 1; ++m) {
        const double dd = std::fabs(d[m]) + std::fabs(d[m + 1]);
        if (std::fabs(e[m]) <= 2.2e-16 * dd) break;
      }
      if (m == l) break;
      if (iter > 100) return false;
      double g = (d[l + 1] - d[l]) / (2.0 * e[l]);
      double r = std::hypot(g, 1.0);
      g = d[m] - d[l] + e[l] / (g + std::copysign(r, g));
      double s = 1.0, c = 1.0, p = 0.0;
      bool split = false;
      for (int i = m - 1; i >= l; --i) {
        const double f = s * e[i];
        const double b = c * e[i];
        r = std::hypot(f, g);
        e[i + 1] = r;
        if (r == 0.0) {
          d[i + 1] -= p;
          e[m] = 0.0;
          split = true;
          break;
        }
        s = f / r;
        c = g / r;
        g = d[i + 1] - p;
        r = (d[i] - g) * s + 2.0 * c * b;
        p = s * r;
        d[i + 1] = g + p;
        g = c * r - b;
        const double zf = z[i + 1];
        z[i + 1] = s * z[i] + c * zf;
        z[i] = c * z[i] - s * zf;
      }
      if (split) continue;
      d[l] -= p;
      e[l] = g;
      e[m] = 0.0;
    }
  }
  return true;
}

// Recurrence coefficients of the monic Jacobi polynomials for the weight
// (1-x)^a (1+x)^b: p_{k+1} = (x - al_k) p_k - be_k p_{k-1}.
void jacobi_recurrence(int n, double a, double b, std::vector<double>& al, std::vector<double>& be) {
  al.assign(n, 0.0);
  be.assign(n, 0.0);
  for (int k = 0; k < n; ++k) {
    const double s = 2.0 * k + a + b;
    if (k == 0)
      al[k] = (b - a) / (a + b + 2.0);
    else
      al[k] = (b * b - a * a) / (s * (s + 2.0));
    if (k >= 1) {
      if (k == 1)
        be[k] = 4.0 * (1.0 + a) * (1.0 + b) / ((2.0 + a + b) * (2.0 + a + b) * (3.0 + a + b));
      else
        be[k] = 4.0 * k * (k + a) * (k + b) * (k + a + b) / (s * s * (s + 1.0) * (s - 1.0));
    }
  }
}

}  // namespace

bool gauss_jacobi(int n, double a, double b, Quadrature& q) {
  if (n < 1) return false;
  std::vector<double> al, be;
  jacobi_recurrence(n, a, b, al, be);
  std::vector<double> d(al), e(n, 0.0), z(n, 0.0);
  for (int k = 0; k + 1 < n; ++k) e[k] = std::sqrt(be[k + 1]);
  z[0] = 1.0;
  if (!tridiagonal_ql(d, e, z)) return false;
  std::sort(d.begin(), d.end());
  const double mu0 = std::exp((a + b + 1.0) * std::log(2.0) + std::lgamma(a + 1.0) +
                              std::lgamma(b + 1.0) - std::lgamma(a + b + 2.0));
  // h_k = int p_k^2 w = mu0 * be_1 * ... * be_k
  std::vector<double> h(n);
  h[0] = mu0;
  for (int k = 1; k < n; ++k) h[k] = h[k - 1] * be[k];
  q.x.resize(n);
  q.w.resize(n);
  for (int i = 0; i < n; ++i) {
    double x = d[i];
    // Newton polish of the eigenvalue as a root of p_n
    for (int it = 0; it < 3; ++it) {
      double p0 = 1.0, p1 = x - al[0], dp0 = 0.0, dp1 = 1.0;
      for (int k = 1; k < n; ++k) {
        const double p2 = (x - al[k]) * p1 - be[k] * p0;
        const double dp2 = p1 + (x - al[k]) * dp1 - be[k] * dp0;
        p0 = p1; p1 = p2; dp0 = dp1; dp1 = dp2;
      }
      if (n == 1) { p1 = x - al[0]; dp1 = 1.0; }
      if (dp1 == 0.0) break;
      x -= p1 / dp1;
    }
    // Christoffel weight 1 / sum_k p_k(x)^2 / h_k
    double p0 = 1.0, p1 = x - al[0], s = 1.0 / h[0];
    if (n > 1) s += p1 * p1 / h[1];
    for (int k = 1; k + 1 < n; ++k) {
      const double p2 = (x - al[k]) * p1 - be[k] * p0;
      p0 = p1;
      p1 = p2;
      s += p2 * p2 / h[k + 1];
    }
    q.x[i] = x;
    q.w[i] = 1.0 / s;
  }
  return true;
}

double b0_unit(double alpha, double gamma) {
  // int_0^pi sin^3 t sin^(alpha+gamma-1)(t/2) cos^-gamma(t/2) dt = 8 B((alpha+gamma+3)/2, (4-gamma)/2)
  const double x = 0.5 * (alpha + gamma + 3.0), y = 0.5 * (4.0 - gamma);
  const double I = 8.0 * std::exp(std::lgamma(x) + std::lgamma(y) - std::lgamma(x + y));
  // delta = b0 I Gamma((7+alpha)/2) 2^((2+alpha)/2) (2 sqrt(pi) / 5)
  const double k = I * std::tgamma(0.5 * (7.0 + alpha)) * std::pow(2.0, 0.5 * (2.0 + alpha)) *
                   2.0 * std::sqrt(kPi) / 5.0;
  return 1.0 / k;
}

double phi_hs(double s, double R, double Lp) {
  // 2 int_0^R rho cos(b rho) d rho, b = pi s / Lp; power series for small b R
  const double b = std::fabs(kPi * s / Lp);
  const double x = b * R;
  if (x < 0.5) {
    double term = 1.0, acc = 0.5;
    for (int k = 1; k < 12; ++k) {
      term *= -(x * x) / ((2.0 * k - 1.0) * (2.0 * k));
      acc += term / (2.0 * k + 2.0);
    }
    return 2.0 * R * R * acc;
  }
  return 2.0 * (R * std::sin(x) / b + (std::cos(x) - 1.0) / (b * b));
}

double psi_hs(double t, double R, double Lp) {
  // 2 pi int_0^R rho J0(pi rho t / Lp) d rho = 2 pi R^2 J1(c) / c
  const double c = kPi * R * t / Lp;
  if (c == 0.0) return kPi * R * R;
  return 2.0 * kPi * R * R * ::j1(c) / c;
}

bool half_sphere_directions(int M, std::vector<double>& ex, std::vector<double>& ey, std::vector<double>& ez,
                            std::vector<double>& W) {
  Quadrature gl;
  if (!gauss_jacobi(M, 0.0, 0.0, gl)) return false;
  const int D = M * M;
  ex.resize(D);
  ey.resize(D);
  ez.resize(D);
  W.resize(D);
  for (int a = 0; a < M; ++a)
    for (int b = 0; b < M; ++b) {
      const double th = 0.5 * kPi * (gl.x[a] + 1.0), ph = 0.5 * kPi * (gl.x[b] + 1.0);
      const int p = a * M + b;
      ex[p] = std::sin(th) * std::cos(ph);
      ey[p] = std::sin(th) * std::sin(ph);
      ez[p] = std::cos(th);
      W[p] = (0.5 * kPi * gl.w[a]) * (0.5 * kPi * gl.w[b]) * std::sin(th);
    }
  return true;
}

namespace {

struct Radial {
  double R, Lp, a_phi, gamma;
  Quadrature qphi, qpsi;  // mapped to [0, R]: nodes rho, weights incl. rho^a factor
  bool phi_closed, psi_closed;

  double phi(double s) const {
    const double b = std::fabs(kPi * s / Lp);
    if (phi_closed) return phi_hs(s, R, Lp);
    double acc = 0.0;
    for (size_t k = 0; k < qphi.x.size(); ++k) acc += qphi.w[k] * std::cos(b * qphi.x[k]);
    return 2.0 * acc;
  }

  double psi(double t) const {
    if (psi_closed) return psi_hs(t, R, Lp);
    const double b = kPi * t / Lp;
    double acc = 0.0;
    for (size_t k = 0; k < qpsi.x.size(); ++k) acc += qpsi.w[k] * ::j0(b * qpsi.x[k]);
    return 2.0 * kPi * acc;
  }
};

bool mapped_rule(int n, double a, double R, Quadrature& q) {
  Quadrature g;
  if (!gauss_jacobi(n, 0.0, a, g)) return false;
  q.x.resize(n);
  q.w.resize(n);
  const double sc = std::pow(0.5 * R, a + 1.0);
  for (int k = 0; k < n; ++k) {
    q.x[k] = 0.5 * R * (g.x[k] + 1.0);
    q.w[k] = g.w[k] * sc;
  }
  return true;
}

bool radial_setup(const TableDesc& d, Radial& rad, std::string& err) {
  const int n = d.n_v;
  const int np = d.n_pad > 0 ? d.n_pad : 2 * n;
  const double dv = 2.0 * d.l_v / n;
  rad.Lp = np * dv / 2.0;
  rad.R = d.r_trunc > 0.0 ? d.r_trunc : 4.0 * rad.Lp / (3.0 + std::sqrt(2.0));
  rad.a_phi = d.alpha + d.gamma;
  rad.gamma = d.gamma;
  rad.phi_closed = std::fabs(rad.a_phi - 1.0) < 1e-15;
  rad.psi_closed = d.gamma == 0.0;
  const double smax = std::sqrt(3.0) * 0.5 * np + 1.0;
  const int nq = 48 + static_cast<int>(0.8 * kPi * smax * rad.R / rad.Lp);
  if (!rad.phi_closed && !mapped_rule(nq, rad.a_phi, rad.R, rad.qphi)) { err = "Gauss-Jacobi failed"; return false; }
  if (!rad.psi_closed && !mapped_rule(nq, 1.0 - d.gamma, rad.R, rad.qpsi)) { err = "Gauss-Jacobi failed"; return false; }
  return true;
}

}  // namespace

bool radial_rule(const TableDesc& d, RadialRule& r, std::string& err) {
  Radial rad;
  if (!radial_setup(d, rad, err)) return false;
  r.R = rad.R;
  r.Lp = rad.Lp;
  r.phi_closed = rad.phi_closed;
  r.psi_closed = rad.psi_closed;
  r.phi_x = rad.qphi.x;
  r.phi_w = rad.qphi.w;
  r.psi_x = rad.qpsi.x;
  r.psi_w = rad.qpsi.w;
  return true;
}

bool build_grid_tables(const TableDesc& d, HostTables& t, std::string& err) {
  const int n = d.n_v;
  const int np = d.n_pad > 0 ? d.n_pad : 2 * n;
  t.n = n;
  t.n3 = n * n * n;
  t.np = np;
  t.nd = 2 * n - 1;
  t.nd3 = t.nd * t.nd * t.nd;
  t.lv = d.l_v;
  t.dv = 2.0 * d.l_v / n;
  t.Lp = np * t.dv / 2.0;
  t.R = d.r_trunc > 0.0 ? d.r_trunc : 4.0 * t.Lp / (3.0 + std::sqrt(2.0));
  t.alpha = d.alpha;
  t.gamma = d.gamma;
  t.b0 = b0_unit(d.alpha, d.gamma);
  t.v1d.resize(n);
  std::vector<double> g1(n);
  for (int j = 0; j < n; ++j) {
    t.v1d[j] = -d.l_v + (j + 0.5) * t.dv;
    g1[j] = std::exp(-t.v1d[j] * t.v1d[j]) / std::sqrt(kPi);
  }
  t.feq.resize(t.n3);
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b)
      for (int c = 0; c < n; ++c) t.feq[(a * n + b) * n + c] = g1[a] * g1[b] * g1[c];
  std::vector<double> ex, ey, ez;
  if (!half_sphere_directions(d.m_angle, ex, ey, ez, t.W)) { err = "Gauss-Legendre failed"; return false; }
  t.D = static_cast<int>(t.W.size());
  return true;
}

bool build_host_tables(const TableDesc& d, bool want_kernels, HostTables& t, std::string& err) {
  const int n = d.n_v;
  const int np = d.n_pad > 0 ? d.n_pad : 2 * n;
  t.n = n;
  t.n3 = n * n * n;
  t.np = np;
  t.nd = 2 * n - 1;
  t.nd3 = t.nd * t.nd * t.nd;
  t.lv = d.l_v;
  t.dv = 2.0 * d.l_v / n;
  t.Lp = np * t.dv / 2.0;
  t.R = d.r_trunc > 0.0 ? d.r_trunc : 4.0 * t.Lp / (3.0 + std::sqrt(2.0));
  t.alpha = d.alpha;
  t.gamma = d.gamma;
  t.b0 = b0_unit(d.alpha, d.gamma);
  const int off = (np - n) / 2;

  t.v1d.resize(n);
  std::vector<double> g1(n);
  for (int j = 0; j < n; ++j) {
    t.v1d[j] = -d.l_v + (j + 0.5) * t.dv;
    g1[j] = std::exp(-t.v1d[j] * t.v1d[j]) / std::sqrt(kPi);
  }
  t.feq.resize(t.n3);
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b)
      for (int c = 0; c < n; ++c) t.feq[(a * n + b) * n + c] = g1[a] * g1[b] * g1[c];

  // directions
  std::vector<double> ex, ey, ez;
  if (!half_sphere_directions(d.m_angle, ex, ey, ez, t.W)) { err = "Gauss-Legendre failed"; return false; }
  t.D = static_cast<int>(t.W.size());

  // radial factors
  Radial rad;
  if (!radial_setup(d, rad, err)) return false;

  // signed modes per index; Nyquist flag
  std::vector<int> lsig(np);
  for (int k = 0; k < np; ++k) lsig[k] = k < np / 2 ? k : k - np;

  // DFT factor matrices: kernels (difference grid) and f_eq fields (n grid)
  PrunedDFT protoK, protoF;
  for (int ax = 0; ax < 3; ++ax) {
    if (want_kernels) protoK.set_kernel_axis(ax, np, n, 0.0);
    protoF.set_field_axis(ax, np, g1, 0.0);
  }

  const size_t np3 = static_cast<size_t>(np) * np * np;
  t.A.assign(static_cast<size_t>(t.D) * t.n3, 0.0);
  t.B.assign(static_cast<size_t>(t.D) * t.n3, 0.0);
  if (want_kernels) {
    t.Psi.assign(static_cast<size_t>(t.D) * t.nd3, 0.0);
    t.Phi.assign(static_cast<size_t>(t.D) * t.nd3, 0.0);
  }

  int nthreads = d.n_threads > 0 ? d.n_threads : static_cast<int>(std::thread::hardware_concurrency());
  nthreads = std::max(1, std::min(nthreads, t.D));
  std::vector<std::vector<double>> beta_part(nthreads, std::vector<double>(np3, 0.0));

  auto worker = [&](int tid) {
    PrunedDFT pk = protoK, pf = protoF;
    std::vector<double> ph(np3), ps(np3);
    std::vector<double>& beta = beta_part[tid];
    for (int p = tid; p < t.D; p += nthreads) {
      for (int k0 = 0; k0 < np; ++k0)
        for (int k1 = 0; k1 < np; ++k1)
          for (int k2 = 0; k2 < np; ++k2) {
            const size_t idx = (static_cast<size_t>(k0) * np + k1) * np + k2;
            const int l0 = lsig[k0], l1 = lsig[k1], l2 = lsig[k2];
            if (l0 == -np / 2 || l1 == -np / 2 || l2 == -np / 2) {
              ph[idx] = 0.0;
              ps[idx] = 0.0;
              continue;
            }
            const double s = l0 * ex[p] + l1 * ey[p] + l2 * ez[p];
            const double q0 = l0 - s * ex[p], q1 = l1 - s * ey[p], q2 = l2 - s * ez[p];
            const double perp = std::sqrt(q0 * q0 + q1 * q1 + q2 * q2);
            ph[idx] = rad.phi(s);
            ps[idx] = rad.psi(perp);
            beta[idx] += t.W[p] * ph[idx] * ps[idx];
          }
      pf.run(ps.data(), &t.A[static_cast<size_t>(p) * t.n3]);
      pf.run(ph.data(), &t.B[static_cast<size_t>(p) * t.n3]);
      if (want_kernels) {
        pk.run(ps.data(), &t.Psi[static_cast<size_t>(p) * t.nd3]);
        pk.run(ph.data(), &t.Phi[static_cast<size_t>(p) * t.nd3]);
      }
    }
  };
  std::vector<std::thread> pool;
  for (int i = 1; i < nthreads; ++i) pool.emplace_back(worker, i);
  worker(0);
  for (auto& th : pool) th.join();

  std::vector<double> beta(np3, 0.0);
  for (int i = 0; i < nthreads; ++i)
    for (size_t j = 0; j < np3; ++j) beta[j] += beta_part[i][j];
  for (size_t j = 0; j < np3; ++j) beta[j] *= 4.0 * t.b0;
  t.nu.assign(t.n3, 0.0);
  {
    PrunedDFT pf = protoF;
    pf.run(beta.data(), t.nu.data());
  }
  if (want_kernels) {
    t.beta_r.assign(t.nd3, 0.0);
    PrunedDFT pk = protoK;
    pk.run(beta.data(), t.beta_r.data());
  }
  const double w = t.dv * t.dv * t.dv;
  double nb = 0.0;
  for (int i = 0; i < t.n3; ++i) nb += w * t.nu[i] * t.feq[i];
  t.nubar = nb;
  (void)off;
  return true;
}

}  // namespace sis
