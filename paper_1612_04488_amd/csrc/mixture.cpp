// Host tables of the binary-mixture fast-spectral operator (see mixture.h).
#include "mixture.h"

#include <algorithm>
#include <cmath>
#include <thread>

#include "planner.h"
#include "pruned_dft.h"

namespace sis {

namespace {

const double kPi = 3.14159265358979323846;

// (1/np) sum over the non-Nyquist modes l of e^{2 pi i l w / np} (real, even in w)
double dirichlet(double w, int np) {
  double s = 1.0;
  for (int l = 1; l < np / 2; ++l) s += 2.0 * std::cos(2.0 * kPi * l * w / np);
  return s / np;
}

template <class F>
void parallel_for(int count, int n_threads, F&& body) {
  int nt = n_threads > 0 ? n_threads : static_cast<int>(std::thread::hardware_concurrency());
  nt = std::max(1, std::min(nt, count));
  auto worker = [&](int tid) {
    for (int i = tid; i < count; i += nt) body(i, tid);
  };
  std::vector<std::thread> pool;
  for (int i = 1; i < nt; ++i) pool.emplace_back(worker, i);
  worker(0);
  for (auto& th : pool) th.join();
}

// psi_p on the full np^3 spectrum (FFT index order), Nyquist zeroed
void psi_spectrum(const MixTables& t, int p, std::vector<double>& ps) {
  const int np = t.np;
  ps.resize(static_cast<size_t>(np) * np * np);
  for (int k0 = 0; k0 < np; ++k0)
    for (int k1 = 0; k1 < np; ++k1)
      for (int k2 = 0; k2 < np; ++k2) {
        const size_t idx = (static_cast<size_t>(k0) * np + k1) * np + k2;
        const int l0 = PrunedDFT::signed_mode(k0, np), l1 = PrunedDFT::signed_mode(k1, np),
                  l2 = PrunedDFT::signed_mode(k2, np);
        if (l0 == -np / 2 || l1 == -np / 2 || l2 == -np / 2) {
          ps[idx] = 0.0;
          continue;
        }
        const double s = l0 * t.ex[p] + l1 * t.ey[p] + l2 * t.ez[p];
        const double q0 = l0 - s * t.ex[p], q1 = l1 - s * t.ey[p], q2 = l2 - s * t.ez[p];
        ps[idx] = psi_hs(std::sqrt(q0 * q0 + q1 * q1 + q2 * q2), t.R, t.Lp);
      }
}

}  // namespace

double mix_viscosity_ratio(const double mass[2], const double diam[2], const double chi[2]) {
  // mu = x^T H^-1 x (units of the pure-A viscosity), one Sonine term, A* = 1 (hard spheres)
  const double m0 = mass[0], m1 = mass[1];
  const double mu0 = 1.0, mu1 = std::sqrt(m1 / m0) * (diam[0] / diam[1]) * (diam[0] / diam[1]);
  const double dab = 0.5 * (diam[0] + diam[1]);
  const double mu01 = std::sqrt(2.0 * m0 * m1 / (m0 + m1) / m0) * (diam[0] / dab) * (diam[0] / dab);
  const double red = m0 * m1 / ((m0 + m1) * (m0 + m1));
  const double k = 2.0 * chi[0] * chi[1] / mu01 * red;
  const double H00 = chi[0] * chi[0] / mu0 + k * (5.0 / 3.0 + m1 / m0);
  const double H11 = chi[1] * chi[1] / mu1 + k * (5.0 / 3.0 + m0 / m1);
  const double H01 = -k * (5.0 / 3.0 - 1.0);
  const double det = H00 * H11 - H01 * H01;
  const double y0 = (H11 * chi[0] - H01 * chi[1]) / det, y1 = (H00 * chi[1] - H01 * chi[0]) / det;
  return chi[0] * y0 + chi[1] * y1;
}

bool build_mix_grid(const MixDesc& d, MixTables& t, std::string& err) {
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
  t.b0 = b0_unit(1.0, 0.0);
  t.m_rho = d.m_rho;
  const double mbar = d.chi[0] * d.mass[0] + d.chi[1] * d.mass[1];
  t.mbar_over_mA = mbar / d.mass[0];
  t.scale = std::sqrt(d.mass[0] / mbar) * mix_viscosity_ratio(d.mass, d.diam, d.chi);
  for (int s = 0; s < 2; ++s) {
    t.a[s] = d.mass[s] / d.mass[0];
    t.chi[s] = d.chi[s];
  }
  for (int a = 0; a < 2; ++a)
    for (int b = 0; b < 2; ++b) {
      t.two_mu[a][b] = 2.0 * d.mass[b] / (d.mass[a] + d.mass[b]);
      t.kappa[a][b] = (d.mass[a] - d.mass[b]) / (d.mass[a] + d.mass[b]);
      const double dab = 0.5 * (d.diam[a] + d.diam[b]) / d.diam[0];
      t.C[a][b] = 4.0 * t.b0 * dab * dab;
    }
  t.v1d.resize(n);
  for (int j = 0; j < n; ++j) t.v1d[j] = -d.l_v + (j + 0.5) * t.dv;
  t.feq.assign(2 * static_cast<size_t>(t.n3), 0.0);
  for (int s = 0; s < 2; ++s) {
    t.prof[s].resize(n);
    const double c = std::cbrt(t.chi[s]) * std::sqrt(t.a[s] / kPi);
    for (int j = 0; j < n; ++j) t.prof[s][j] = c * std::exp(-t.a[s] * t.v1d[j] * t.v1d[j]);
    for (int i0 = 0; i0 < n; ++i0)
      for (int i1 = 0; i1 < n; ++i1)
        for (int i2 = 0; i2 < n; ++i2)
          t.feq[s * static_cast<size_t>(t.n3) + (i0 * n + i1) * n + i2] =
              t.prof[s][i0] * t.prof[s][i1] * t.prof[s][i2];
  }
  if (!half_sphere_directions(d.m_angle, t.ex, t.ey, t.ez, t.W)) { err = "Gauss-Legendre failed"; return false; }
  t.D = static_cast<int>(t.W.size());
  {
    Quadrature gl;
    if (!gauss_jacobi(d.m_rho, 0.0, 0.0, gl)) { err = "Gauss-Legendre failed"; return false; }
    t.rho.resize(d.m_rho);
    t.wr.resize(d.m_rho);
    for (int r = 0; r < d.m_rho; ++r) {
      t.rho[r] = 0.5 * t.R * (gl.x[r] + 1.0);
      t.wr[r] = 0.5 * t.R * gl.w[r];
    }
  }

  return true;
}

bool build_mix_base(const MixDesc& d, MixTables& t, std::string& err) {
  if (!build_mix_grid(d, t, err)) return false;
  const int n = t.n, np = t.np;
  PrunedDFT protoK, protoF[2];
  for (int ax = 0; ax < 3; ++ax) {
    protoK.set_kernel_axis(ax, np, n, 0.0);
    for (int s = 0; s < 2; ++s) protoF[s].set_field_axis(ax, np, t.prof[s], 0.0);
  }
  const size_t np3 = static_cast<size_t>(np) * np * np;
  const size_t tabK = static_cast<size_t>(t.D) * t.nd3, tabF = static_cast<size_t>(t.D) * t.n3;
  t.Psi.assign(tabK, 0.0);
  t.Phi.assign(tabK, 0.0);
  for (int s = 0; s < 2; ++s) {
    t.Fphi[s].assign(tabF, 0.0);
    t.Fpsi[s].assign(tabF, 0.0);
  }
  int nthreads = d.n_threads > 0 ? d.n_threads : static_cast<int>(std::thread::hardware_concurrency());
  nthreads = std::max(1, std::min(nthreads, t.D));
  std::vector<std::vector<double>> beta_part(nthreads, std::vector<double>(np3, 0.0));
  parallel_for(t.D, nthreads, [&](int p, int tid) {
    PrunedDFT pk = protoK, pf0 = protoF[0], pf1 = protoF[1];
    std::vector<double> ph(np3), ps;
    psi_spectrum(t, p, ps);
    std::vector<double>& beta = beta_part[tid];
    for (int k0 = 0; k0 < np; ++k0)
      for (int k1 = 0; k1 < np; ++k1)
        for (int k2 = 0; k2 < np; ++k2) {
          const size_t idx = (static_cast<size_t>(k0) * np + k1) * np + k2;
          const int l0 = PrunedDFT::signed_mode(k0, np), l1 = PrunedDFT::signed_mode(k1, np),
                    l2 = PrunedDFT::signed_mode(k2, np);
          if (l0 == -np / 2 || l1 == -np / 2 || l2 == -np / 2) {
            ph[idx] = 0.0;
            continue;
          }
          ph[idx] = phi_hs(l0 * t.ex[p] + l1 * t.ey[p] + l2 * t.ez[p], t.R, t.Lp);
          beta[idx] += t.W[p] * ph[idx] * ps[idx];
        }
    pk.run(ps.data(), &t.Psi[static_cast<size_t>(p) * t.nd3]);
    pk.run(ph.data(), &t.Phi[static_cast<size_t>(p) * t.nd3]);
    pf0.run(ph.data(), &t.Fphi[0][static_cast<size_t>(p) * t.n3]);
    pf0.run(ps.data(), &t.Fpsi[0][static_cast<size_t>(p) * t.n3]);
    pf1.run(ph.data(), &t.Fphi[1][static_cast<size_t>(p) * t.n3]);
    pf1.run(ps.data(), &t.Fpsi[1][static_cast<size_t>(p) * t.n3]);
  });
  std::vector<double> beta(np3, 0.0);
  for (int i = 0; i < nthreads; ++i)
    for (size_t j = 0; j < np3; ++j) beta[j] += beta_part[i][j];
  t.beta_r.assign(t.nd3, 0.0);
  protoK.run(beta.data(), t.beta_r.data());
  std::vector<double> nuu[2];
  for (int s = 0; s < 2; ++s) {
    nuu[s].assign(t.n3, 0.0);
    PrunedDFT pf = protoF[s];
    pf.run(beta.data(), nuu[s].data());
  }
  t.nu.assign(2 * static_cast<size_t>(t.n3), 0.0);
  const double w = t.dv * t.dv * t.dv;
  for (int a = 0; a < 2; ++a) {
    double nb = 0.0;
    for (int i = 0; i < t.n3; ++i) {
      const double v = t.scale * (t.C[a][0] * nuu[0][i] + t.C[a][1] * nuu[1][i]);
      t.nu[a * static_cast<size_t>(t.n3) + i] = v;
      nb += w * v * t.feq[a * static_cast<size_t>(t.n3) + i];
    }
    t.nubar[a] = nb / t.chi[a];
  }
  return true;
}

void build_mix_cross_terms(const MixTables& t, int a, int b, int kind, int q0, int q1, double* X, double* Y,
                           int n_threads) {
  const int n = t.n, np = t.np, nd = t.nd;
  const size_t n3 = t.n3, nd3 = t.nd3;
  const double tm = t.two_mu[a][b], kap = t.kappa[a][b];
  parallel_for(q1 - q0, n_threads, [&](int it, int) {
    const int q = q0 + it;
    const int p = q / t.m_rho, r = q % t.m_rho;
    const double rho = t.rho[r];
    const double wt = t.scale * t.C[a][b] * t.W[p] * t.wr[r] * rho;
    const double e[3] = {t.ex[p], t.ey[p], t.ez[p]};
    double zp[3], zm[3];  // shifts in grid units of e^{+} and e^{-}
    for (int k = 0; k < 3; ++k) {
      zp[k] = tm * rho * e[k] / t.dv;
      zm[k] = -kap * rho * e[k] / t.dv;
    }
    double* Xp = X + static_cast<size_t>(2 * it) * n3;
    double* Xm = Xp + n3;
    double* Yp = Y + static_cast<size_t>(2 * it) * nd3;
    double* Ym = Yp + nd3;
    std::vector<double> ps;
    psi_spectrum(t, p, ps);
    PrunedDFT P;
    if (kind == 0) {
      // X = shifted band-limited f_a (separable), Y = F^-1[psi_p e^-]
      const std::vector<double>& g = t.prof[a];
      double gs[3][64];
      for (int k = 0; k < 3; ++k)
        for (int i = 0; i < n; ++i) {
          double s = 0.0;
          for (int j = 0; j < n; ++j) s += g[j] * dirichlet(i - j + zp[k], np);
          gs[k][i] = s;
        }
      for (int i0 = 0; i0 < n; ++i0)
        for (int i1 = 0; i1 < n; ++i1)
          for (int i2 = 0; i2 < n; ++i2) Xp[(i0 * n + i1) * n + i2] = wt * gs[0][i0] * gs[1][i1] * gs[2][i2];
      for (int ax = 0; ax < 3; ++ax) P.set_kernel_axis(ax, np, n, zm[ax]);
      P.run(ps.data(), Yp);
    } else {
      // X = F^-1[psi_p e^- F f_b] (field, shifted), Y = shifted band-limited delta (separable)
      for (int ax = 0; ax < 3; ++ax) P.set_field_axis(ax, np, t.prof[b], zm[ax]);
      P.run(ps.data(), Xp);
      for (size_t i = 0; i < n3; ++i) Xp[i] *= wt;
      double ds[3][128];
      for (int k = 0; k < 3; ++k)
        for (int c = 0; c < nd; ++c) ds[k][c] = dirichlet((c - (n - 1)) + zp[k], np);
      for (int c0 = 0; c0 < nd; ++c0)
        for (int c1 = 0; c1 < nd; ++c1)
          for (int c2 = 0; c2 < nd; ++c2) Yp[(static_cast<size_t>(c0) * nd + c1) * nd + c2] = ds[0][c0] * ds[1][c1] * ds[2][c2];
    }
    // -rho: mirror (profiles and kernels are even)
    for (size_t i = 0; i < n3; ++i) Xm[i] = Xp[n3 - 1 - i];
    for (size_t i = 0; i < nd3; ++i) Ym[i] = Yp[nd3 - 1 - i];
  });
}

}  // namespace sis
