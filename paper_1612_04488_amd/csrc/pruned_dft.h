// Pruned separable inverse DFT on the host (plan-time table construction).
//
//   out[a0][a1][a2] = Re sum_k T[k0][k1][k2] E0[k0][a0] E1[k1][a1] E2[k2][a2]
//
// for a real spectrum T on the np^3 modes and complex factor matrices E_x of
// shape [np][m] (one per axis; m outputs per axis).  The three passes cost
// O(np^3 m + np^2 m^2 + np m^3) instead of a full np^3 transform per output.
//
// Factor matrices used by the collision tables (l_k the signed mode of FFT
// index k, shifts z in units of the grid spacing):
//   kernel:  E[k][a] = e^{2 pi i l_k (a - (n-1) + z) / np} / np
//            (real-space kernel K(d + z) on the difference grid d = a - (n-1));
//   field:   E[k][i] = sum_j g_j e^{2 pi i l_k (i - j + z) / np} / np
//            (discrete convolution of the separable profile g with K, shifted).
#pragma once
#include <cmath>
#include <vector>

namespace sis {

struct PrunedDFT {
  int np = 0, m = 0;
  std::vector<double> er[3], ei[3];  // per axis, [np][m]
  std::vector<double> x1r, x1i, x2r, x2i;

  static int signed_mode(int k, int np) { return k < np / 2 ? k : k - np; }

  // Axis factor of a real-space kernel on the difference grid, shifted by z.
  void set_kernel_axis(int ax, int np_, int n, double z) {
    np = np_;
    m = 2 * n - 1;
    er[ax].resize(static_cast<size_t>(np) * m);
    ei[ax].resize(static_cast<size_t>(np) * m);
    const double tp = 2.0 * 3.14159265358979323846 / np;
    for (int k = 0; k < np; ++k) {
      const double l = signed_mode(k, np);
      for (int a = 0; a < m; ++a) {
        const double d = (a - (n - 1)) + z;
        double ang = l * d;
        ang -= np * std::floor(ang / np);  // reduce mod np (exact for integer l*d)
        er[ax][static_cast<size_t>(k) * m + a] = std::cos(tp * ang) / np;
        ei[ax][static_cast<size_t>(k) * m + a] = std::sin(tp * ang) / np;
      }
    }
  }

  // Axis factor of a field: convolution of profile g (length n) with the kernel, shifted by z.
  void set_field_axis(int ax, int np_, const std::vector<double>& g, double z) {
    np = np_;
    const int n = static_cast<int>(g.size());
    m = n;
    er[ax].assign(static_cast<size_t>(np) * n, 0.0);
    ei[ax].assign(static_cast<size_t>(np) * n, 0.0);
    const double tp = 2.0 * 3.14159265358979323846 / np;
    for (int k = 0; k < np; ++k) {
      const double l = signed_mode(k, np);
      for (int i = 0; i < n; ++i) {
        double sr = 0.0, si = 0.0;
        for (int j = 0; j < n; ++j) {
          double ang = l * ((i - j) + z);
          ang -= np * std::floor(ang / np);
          sr += g[j] * std::cos(tp * ang);
          si += g[j] * std::sin(tp * ang);
        }
        er[ax][static_cast<size_t>(k) * n + i] = sr / np;
        ei[ax][static_cast<size_t>(k) * n + i] = si / np;
      }
    }
  }

  void copy_axis(int dst, int src) {
    er[dst] = er[src];
    ei[dst] = ei[src];
  }

  void run(const double* T, double* out) {
    const int n2 = np * np;
    const std::vector<double>&e0r = er[0], &e0i = ei[0], &e1r = er[1], &e1i = ei[1], &e2r = er[2],
                                   &e2i = ei[2];
    x1r.assign(static_cast<size_t>(n2) * m, 0.0);
    x1i.assign(static_cast<size_t>(n2) * m, 0.0);
    for (int q = 0; q < n2; ++q) {
      const double* t = T + static_cast<size_t>(q) * np;
      double* r = &x1r[static_cast<size_t>(q) * m];
      double* im = &x1i[static_cast<size_t>(q) * m];
      for (int k2 = 0; k2 < np; ++k2) {
        const double tv = t[k2];
        if (tv == 0.0) continue;
        const double* a = &e2r[static_cast<size_t>(k2) * m];
        const double* b = &e2i[static_cast<size_t>(k2) * m];
        for (int j = 0; j < m; ++j) {
          r[j] += tv * a[j];
          im[j] += tv * b[j];
        }
      }
    }
    const size_t mm = static_cast<size_t>(m) * m;
    x2r.assign(np * mm, 0.0);
    x2i.assign(np * mm, 0.0);
    for (int k0 = 0; k0 < np; ++k0) {
      for (int k1 = 0; k1 < np; ++k1) {
        const double* ar = &x1r[(static_cast<size_t>(k0) * np + k1) * m];
        const double* ai = &x1i[(static_cast<size_t>(k0) * np + k1) * m];
        for (int a1 = 0; a1 < m; ++a1) {
          const double cr = e1r[static_cast<size_t>(k1) * m + a1], ci = e1i[static_cast<size_t>(k1) * m + a1];
          double* yr = &x2r[k0 * mm + static_cast<size_t>(a1) * m];
          double* yi = &x2i[k0 * mm + static_cast<size_t>(a1) * m];
          for (int a2 = 0; a2 < m; ++a2) {
            yr[a2] += ar[a2] * cr - ai[a2] * ci;
            yi[a2] += ar[a2] * ci + ai[a2] * cr;
          }
        }
      }
    }
    std::fill(out, out + static_cast<size_t>(m) * mm, 0.0);
    for (int k0 = 0; k0 < np; ++k0) {
      const double* yr = &x2r[k0 * mm];
      const double* yi = &x2i[k0 * mm];
      for (int a0 = 0; a0 < m; ++a0) {
        const double cr = e0r[static_cast<size_t>(k0) * m + a0], ci = e0i[static_cast<size_t>(k0) * m + a0];
        double* o = out + a0 * mm;
        for (size_t j = 0; j < mm; ++j) o[j] += yr[j] * cr - yi[j] * ci;
      }
    }
  }
};

}  // namespace sis
