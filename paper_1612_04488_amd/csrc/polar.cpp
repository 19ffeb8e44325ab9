// Polar-coordinate velocity grid (v_r, th, v_z) and fast-spectral multipliers on the
// Cartesian modes (Sec. 4): the tube's distributions are even in th and odd in v_z,
// so the stored nodes are the th, v_z > 0 halves (v_z fastest).
#include "polar.h"

#include <algorithm>
#include <cmath>
#include <thread>

#include "planner.h"

namespace sis {

namespace {
constexpr double kPi = 3.14159265358979323846;
}

bool build_polar_tables(const PolarDesc& d, PolarTables& t, std::string& err) {
  if (d.n_vr < 2 || d.n_vr > 64 || d.n_th < 4 || d.n_th > 256 || d.n_th % 2 || d.n_vz < 2 || d.n_vz > 64) {
    err = "polar grid: n_vr in [2, 64], n_th even in [4, 256], n_vz in [2, 64]";
    return false;
  }
  if (!(d.vr_max > 0.0) || !(d.vz_max > 0.0)) {
    err = "polar grid: vr_max and the v_z range must be positive";
    return false;
  }
  t.n_vr = d.n_vr;
  t.n_th = d.n_th;
  t.n_vz = d.n_vz;
  t.nv = d.n_vr * d.n_th * d.n_vz;
  // v_r = V s^2, s the Gauss-Legendre nodes on [0, 1]: int_0^V g v_r dv_r = 2 V^2 int_0^1 g s^3 ds
  Quadrature gl;
  if (!gauss_jacobi(d.n_vr, 0.0, 0.0, gl)) { err = "Gauss-Legendre nodes"; return false; }
  t.vr.resize(d.n_vr);
  t.wvr.resize(d.n_vr);
  for (int i = 0; i < d.n_vr; ++i) {
    const double s = 0.5 * (gl.x[i] + 1.0), ws = 0.5 * gl.w[i];
    t.vr[i] = d.vr_max * s * s;
    t.wvr[i] = 2.0 * d.vr_max * d.vr_max * s * s * s * ws;
  }
  const double dth = kPi / d.n_th, dz = d.vz_max / d.n_vz;
  t.th.resize(d.n_th);
  t.vz.resize(d.n_vz);
  for (int k = 0; k < d.n_th; ++k) t.th[k] = (k + 0.5) * dth;
  for (int k = 0; k < d.n_vz; ++k) t.vz[k] = (k + 0.5) * dz;
  const int nv = t.nv;
  t.vnode.resize(3 * static_cast<size_t>(nv));
  t.wbase.resize(nv);
  t.feq.resize(nv);
  for (int a = 0; a < d.n_vr; ++a)
    for (int b = 0; b < d.n_th; ++b)
      for (int c = 0; c < d.n_vz; ++c) {
        const int j = (a * d.n_th + b) * d.n_vz + c;
        t.vnode[j] = t.vr[a] * std::cos(t.th[b]);
        t.vnode[nv + j] = t.vr[a] * std::sin(t.th[b]);
        t.vnode[2 * nv + j] = t.vz[c];
        t.wbase[j] = t.wvr[a] * dth * dz;
        t.feq[j] = std::pow(kPi, -1.5) * std::exp(-(t.vr[a] * t.vr[a] + t.vz[c] * t.vz[c]));
      }
  // periodic box of the fast spectral method (hard spheres)
  t.lp = d.l_pad > 0.0 ? d.l_pad : 2.0 * std::max(d.vr_max, d.vz_max);
  t.np = d.n_pad > 0 ? d.n_pad : 2 * static_cast<int>(std::lround(2.0 * t.lp));
  if (t.np < 4 || t.np % 2 || t.np > 128) { err = "polar grid: n_pad must be even in [4, 128]"; return false; }
  t.dvc = 2.0 * t.lp / t.np;
  t.R = 4.0 * t.lp / (3.0 + std::sqrt(2.0));
  t.b0 = b0_unit(1.0, 0.0);
  std::vector<double> ex, ey, ez;
  if (!half_sphere_directions(d.m_angle, ex, ey, ez, t.W)) { err = "directions"; return false; }
  t.D = static_cast<int>(t.W.size());
  // modes l in (-np/2, np/2)^3, one of each pair {l, -l}
  const int h = t.np / 2;
  std::vector<int> L;
  for (int a = -h + 1; a < h; ++a)
    for (int b = -h + 1; b < h; ++b)
      for (int c = -h + 1; c < h; ++c) {
        const bool first = a > 0 || (a == 0 && (b > 0 || (b == 0 && c >= 0)));
        if (!first) continue;
        L.push_back(a);
        L.push_back(b);
        L.push_back(c);
      }
  const int nreal = static_cast<int>(L.size() / 3);
  t.nm = nreal + (nreal % 2);
  t.T = 2 * t.D + 1;
  t.Tp = t.T + (t.T % 2);
  t.xi.assign(3 * static_cast<size_t>(t.nm), 0.0);
  t.pair.assign(t.nm, 0.0);
  t.mt_tm.assign(static_cast<size_t>(t.Tp) * t.nm, 0.0);
  t.mt_mm.assign(static_cast<size_t>(t.nm) * t.Tp, 0.0);
  const int D = t.D, nm = t.nm, Tp = t.Tp;
  auto work = [&](int m0, int m1) {
    for (int m = m0; m < m1; ++m) {
      const double l0 = L[3 * m], l1 = L[3 * m + 1], l2 = L[3 * m + 2];
      t.xi[m] = kPi * l0 / t.lp;
      t.xi[nm + m] = kPi * l1 / t.lp;
      t.xi[2 * nm + m] = kPi * l2 / t.lp;
      t.pair[m] = (l0 == 0 && l1 == 0 && l2 == 0) ? 1.0 : 2.0;
      double beta = 0.0;
      for (int p = 0; p < D; ++p) {
        const double s = l0 * ex[p] + l1 * ey[p] + l2 * ez[p];
        const double q0 = l0 - s * ex[p], q1 = l1 - s * ey[p], q2 = l2 - s * ez[p];
        const double ph = phi_hs(s, t.R, t.lp), ps = psi_hs(std::sqrt(q0 * q0 + q1 * q1 + q2 * q2), t.R, t.lp);
        t.mt_tm[static_cast<size_t>(p) * nm + m] = ps;
        t.mt_tm[static_cast<size_t>(D + p) * nm + m] = ph;
        t.mt_mm[static_cast<size_t>(m) * Tp + p] = ps;
        t.mt_mm[static_cast<size_t>(m) * Tp + D + p] = ph;
        beta += t.W[p] * ph * ps;
      }
      beta *= 4.0 * t.b0;
      t.mt_tm[static_cast<size_t>(2 * D) * nm + m] = beta;
      t.mt_mm[static_cast<size_t>(m) * Tp + 2 * D] = beta;
    }
  };
  int nth = d.n_threads > 0 ? d.n_threads : static_cast<int>(std::thread::hardware_concurrency());
  nth = std::max(1, std::min(nth, 64));
  std::vector<std::thread> pool;
  const int chunk = (nreal + nth - 1) / nth;
  for (int k = 0; k < nth; ++k) {
    const int m0 = k * chunk, m1 = std::min(nreal, m0 + chunk);
    if (m0 < m1) pool.emplace_back(work, m0, m1);
  }
  for (auto& th : pool) th.join();
  return true;
}

}  // namespace sis
