// The fast spectral method (the collision evaluation the paper cites for eq.
// LBE_collision) applied per cell on the device: a pruned forward DFT of each
// cell's distribution, then for every one of the 2D + 1 terms its multiplier,
// a pruned inverse DFT back to the stored velocities and the product with the
// term's f_eq field, summed over the terms.  Every DFT is separable: each axis
// is a small dense complex GEMM against a factor matrix, run on the FP64 MFMA
// (v_mfma_f64_16x16x4) with the operands staged in LDS.  Declarations in fsm.h.
#include "fsm.h"

#include <algorithm>

namespace sis {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) void gbl_void_t;
constexpr int kThreads = 256;   // four wave64s

__device__ inline v4d mfma(double a, double b, v4d c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// C(m, n) = sum_{k < K} A(m, k) B(k, n) for the 16 x 16 NT block at (m0, n0),
// complex planar: la(m, k, re, im), lb(k, n, re, im) fetch the operands (zero
// outside the matrices).  Lane l holds, for tile j and element r, the entry
// (m0 + l/16 + 4r, n0 + 16 j + l%16) (the 16x16x4 FP64 layout: A from lane
// (row l%16, k l/16), B from lane (k l/16, column l%16)).
template <int NT, class LA, class LB>
__device__ inline void cgemm_block(int K, int m0, int n0, LA la, LB lb, v4d (&cr)[NT], v4d (&ci)[NT]) {
  const int lane = threadIdx.x & 63, kr = lane >> 4, cc = lane & 15;
#pragma unroll
  for (int j = 0; j < NT; ++j) {
    cr[j] = v4d{0.0, 0.0, 0.0, 0.0};
    ci[j] = v4d{0.0, 0.0, 0.0, 0.0};
  }
  for (int k0 = 0; k0 < K; k0 += 4) {
    double ar, ai;
    la(m0 + cc, k0 + kr, ar, ai);
    const double nai = -ai;
#pragma unroll
    for (int j = 0; j < NT; ++j) {
      double br, bi;
      lb(k0 + kr, n0 + 16 * j + cc, br, bi);
      cr[j] = mfma(ar, br, cr[j]);
      ci[j] = mfma(ar, bi, ci[j]);
      cr[j] = mfma(nai, bi, cr[j]);
      ci[j] = mfma(ai, br, ci[j]);
    }
  }
}

// Every (16 x 16 NT) block of an M x N complex product, blocks dealt round-robin
// to the four waves; st(m, n, re, im) stores the entries inside the matrix.
template <int NT, class LA, class LB, class ST>
__device__ inline void cgemm(int M, int N, int K, LA la, LB lb, ST st) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63, kr = lane >> 4, cc = lane & 15;
  const int mb = (M + 15) / 16, nbk = (N + 16 * NT - 1) / (16 * NT);
  for (int blk = wave; blk < mb * nbk; blk += 4) {
    const int m0 = (blk / nbk) * 16, n0 = (blk % nbk) * 16 * NT;
    v4d cr[NT], ci[NT];
    cgemm_block<NT>(K, m0, n0, la, lb, cr, ci);
#pragma unroll
    for (int j = 0; j < NT; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + kr + 4 * r, n = n0 + 16 * j + cc;
        if (m < M && n < N) st(m, n, cr[j][r], ci[j][r]);
      }
  }
}

// ---------------------------------------------------------------- multipliers
__device__ double phi_closed(double s, double R, double Lp) {
  // 2 int_0^R rho cos(b rho) d rho, b = |pi s / Lp|; power series for small b R
  const double b = fabs(M_PI * s / Lp);
  const double x = b * R;
  if (x < 0.5) {
    double term = 1.0, acc = 0.5;
    for (int k = 1; k < 12; ++k) {
      term *= -(x * x) / ((2.0 * k - 1.0) * (2.0 * k));
      acc += term / (2.0 * k + 2.0);
    }
    return 2.0 * R * R * acc;
  }
  return 2.0 * (R * sin(x) / b + (cos(x) - 1.0) / (b * b));
}

__global__ __launch_bounds__(256) void fsm_mult_kernel(FsmMultArgs a) {
  const FsmDims d = a.d;
  const int64_t qll = static_cast<int64_t>(d.Q) * d.L * d.L;
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= qll) return;
  const int l2i = static_cast<int>(idx % d.L);
  const int l1i = static_cast<int>((idx / d.L) % d.L);
  const int l3 = static_cast<int>(idx / (static_cast<int64_t>(d.L) * d.L));
  const double l1 = l1i - (d.P / 2 - 1), l2 = l2i - (d.P / 2 - 1), l3d = l3;
  double beta = 0.0;
  for (int p = 0; p < a.D; ++p) {
    const double ex = a.dirs[3 * p], ey = a.dirs[3 * p + 1], ez = a.dirs[3 * p + 2];
    const double s = l1 * ex + l2 * ey + l3d * ez;
    const double q0 = l1 - s * ex, q1 = l2 - s * ey, q2 = l3d - s * ez;
    const double perp = sqrt(fmax(q0 * q0 + q1 * q1 + q2 * q2, 0.0));
    double ph, ps;
    if (a.phi_closed) {
      ph = phi_closed(s, a.R, a.Lp);
    } else {
      const double b = fabs(M_PI * s / a.Lp);
      double acc = 0.0;
      for (int k = 0; k < a.n_phi; ++k) acc += a.phi_w[k] * cos(b * a.phi_x[k]);
      ph = 2.0 * acc;
    }
    if (a.psi_closed) {
      const double c = M_PI * a.R * perp / a.Lp;
      ps = c == 0.0 ? M_PI * a.R * a.R : 2.0 * M_PI * a.R * a.R * j1(c) / c;
    } else {
      const double b = M_PI * perp / a.Lp;
      double acc = 0.0;
      for (int k = 0; k < a.n_psi; ++k) acc += a.psi_w[k] * j0(b * a.psi_x[k]);
      ps = 2.0 * M_PI * acc;
    }
    a.mult[static_cast<int64_t>(2 * p) * qll + idx] = ps;
    a.mult[static_cast<int64_t>(2 * p + 1) * qll + idx] = ph;
    beta += a.W[p] * ph * ps;
  }
  a.mult[static_cast<int64_t>(2 * a.D) * qll + idx] = 4.0 * a.b0 * beta;
}

// ---------------------------------------------------------------- forward
// One workgroup per (cell, chunk of B3 l3 modes):
//   T1(l3, j1, s2) = sum_s3 F3(l3, s3) h(j1, s2, s3)
//   T2(l3, l2, j1) = sum_s2 F2(l2, s2) T1(l3, j1, s2)
//   S(l1, l3, l2)  = sum_j1 F1(l1, j1) T2(l3, l2, j1)
__global__ __launch_bounds__(kThreads) void fsm_forward_kernel(FsmDims d, FsmFactors f, int B3,
                                                               const double* __restrict__ h,
                                                               double* __restrict__ S) {
  extern __shared__ double sm[];
  const int64_t cell = blockIdx.y;
  const int q0 = blockIdx.x * B3;
  const int nq = min(B3, d.Q - q0);
  const int n = d.n, n2 = d.n2, n3 = d.n3, L = d.L, Q = d.Q;
  double* T1r = sm;                      // [B3][n][n2]
  double* T1i = T1r + B3 * n * n2;
  double* T2r = T1i + B3 * n * n2;       // [B3][L][n]
  double* T2i = T2r + B3 * L * n;
  const double* hc = h + cell * d.nv;
  {
    const int M = nq, K = n3, N = n * n2;
    auto la = [&](int m, int k, double& re, double& im) {
      const bool ok = m < M && k < K;
      re = ok ? f.f3r[(q0 + m) * n3 + k] : 0.0;
      im = ok ? f.f3i[(q0 + m) * n3 + k] : 0.0;
    };
    auto lb = [&](int k, int c, double& re, double& im) {
      re = (k < K && c < N) ? hc[static_cast<int64_t>(c) * n3 + k] : 0.0;
      im = 0.0;
    };
    auto st = [&](int m, int c, double re, double im) {
      T1r[m * N + c] = re;
      T1i[m * N + c] = im;
    };
    cgemm<2>(M, N, K, la, lb, st);
  }
  __syncthreads();
  {
    const int M = L, K = n2, N = nq * n;   // column c = (l3c, j1)
    auto la = [&](int m, int k, double& re, double& im) {
      const bool ok = m < M && k < K;
      re = ok ? f.f2r[m * n2 + k] : 0.0;
      im = ok ? f.f2i[m * n2 + k] : 0.0;
    };
    auto lb = [&](int k, int c, double& re, double& im) {
      const bool ok = k < K && c < N;
      re = ok ? T1r[c * n2 + k] : 0.0;
      im = ok ? T1i[c * n2 + k] : 0.0;
    };
    auto st = [&](int m, int c, double re, double im) {
      const int l3c = c / n, j1 = c - l3c * n;
      T2r[(l3c * L + m) * n + j1] = re;
      T2i[(l3c * L + m) * n + j1] = im;
    };
    cgemm<2>(M, N, K, la, lb, st);
  }
  __syncthreads();
  {
    const int M = L, K = n, N = nq * L;    // column c = (l3c, l2)
    auto la = [&](int m, int k, double& re, double& im) {
      const bool ok = m < M && k < K;
      re = ok ? f.f1r[m * n + k] : 0.0;
      im = ok ? f.f1i[m * n + k] : 0.0;
    };
    auto lb = [&](int k, int c, double& re, double& im) {
      const bool ok = k < K && c < N;
      re = ok ? T2r[c * n + k] : 0.0;
      im = ok ? T2i[c * n + k] : 0.0;
    };
    double* Sc = S + cell * static_cast<int64_t>(L) * 2 * Q * L;
    auto st = [&](int m, int c, double re, double im) {
      const int l3c = c / L, l2 = c - l3c * L;
      const int64_t o = (static_cast<int64_t>(m) * 2 * Q + (q0 + l3c)) * L + l2;
      Sc[o] = re;
      Sc[o + static_cast<int64_t>(Q) * L] = im;
    };
    cgemm<2>(M, N, K, la, lb, st);
  }
}

// ---------------------------------------------------------------- inverse
// One workgroup per (cell, slab of B1 l1 modes).  The slab of the spectrum and the
// factor matrices stay in LDS for all terms; per term t:
//   stage 1  Y1(s3, b, l2) = sum_l3 E3(s3, l3) m_t(l3, l1, l2) S(l1, l3, l2)
//   stage 2  Y2(b, s2, s3) = sum_l2 Y1(s3, b, l2) E2(s2, l2)      (rows (s3, b))
//   stage 3  G(j1, s2, s3) += field_t(j1, s2, s3) Re sum_b E1(j1, l1) Y2(b, s2, s3)
// (l1 = l10 + b).  Each block's operands for all its k-steps (stage 1) or four
// k-steps at a time (stage 2) are loaded before its MFMAs, so one load latency is
// paid per block or chunk, not per k-step.  G stays in registers: stage-3 tile q
// of wave w is tile w + 8q.
constexpr int kKs1 = 8;   // stage-1 k-steps held in registers: Q <= 32 (n_pad <= 64)

constexpr int kInvWaves = 8;
constexpr int kInvThreads = 64 * kInvWaves;

template <int MAXG>
__global__ __launch_bounds__(kInvThreads) void fsm_inverse_kernel(FsmDims d, FsmFactors f, int B1,
                                                               const double* __restrict__ S,
                                                               const double* __restrict__ mult,
                                                               const double* __restrict__ field,
                                                               double* __restrict__ accp, int64_t n_cells) {
  extern __shared__ double sm[];
  const int slab = blockIdx.x;
  const int64_t cell = blockIdx.y;
  const int n = d.n, n2 = d.n2, n3 = d.n3, L = d.L, Q = d.Q;
  const int l10 = slab * B1, nb = min(B1, L - l10);
  const int NB = B1 * L;
  const int N3c = n2 * n3;
  double* Sr = sm;                 // [Q][B1][L]
  double* Si = Sr + Q * NB;
  double* Y1r = Si + Q * NB;       // [n3][B1][L]
  double* Y1i = Y1r + n3 * NB;
  // Rows padded by one double where 16 lanes read (or write) down a column: E3 (stride Q, 32 at
  // n_pad 64), Y2 (stride n3) and E1 (stride B1) would otherwise put those lanes on a few banks.
  const int Qp = Q + 1, n3p = n3 + 1, B1p = B1 + 1;
  const int N3p = n2 * n3p;
  double* Y2r = Y1i + n3 * NB;     // [B1][n2][n3 + 1]
  double* Y2i = Y2r + B1 * N3p;
  double* E3r = Y2i + B1 * N3p;    // [n3][Q + 1]
  double* E3i = E3r + n3 * Qp;
  double* E2r = E3i + n3 * Qp;     // [n2][L]
  double* E2i = E2r + n2 * L;
  double* E1r = E2i + n2 * L;      // [n][B1 + 1] (the slab's columns)
  double* E1i = E1r + n * B1p;
  double* pf = E1i + n * B1p;      // 256 B that the multiplier prefetch writes and nothing reads
  // wave index as a scalar: the per-wave block and tile loops below branch uniformly
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int lane = threadIdx.x & 63, kr = lane >> 4, cc = lane & 15;

  const double* Sc = S + (cell * L + l10) * 2 * static_cast<int64_t>(Q) * L;
  for (int i = threadIdx.x; i < nb * 2 * Q * L; i += kInvThreads) {
    const int l2 = i % L;
    int r = i / L;
    const int l3 = r % Q;
    r /= Q;
    const int ri = r & 1, b = r >> 1;
    (ri ? Si : Sr)[l3 * NB + b * L + l2] = Sc[i];
  }
  for (int i = threadIdx.x; i < n3 * Q; i += kInvThreads) {
    const int o = (i / Q) * Qp + i % Q;
    E3r[o] = f.e3r[i];
    E3i[o] = f.e3i[i];
  }
  for (int i = threadIdx.x; i < n2 * L; i += kInvThreads) {
    E2r[i] = f.e2r[i];
    E2i[i] = f.e2i[i];
  }
  for (int i = threadIdx.x; i < n * B1; i += kInvThreads) {
    const int j1 = i / B1, b = i - j1 * B1;
    E1r[j1 * B1p + b] = b < nb ? f.e1r[j1 * L + l10 + b] : 0.0;
    E1i[j1 * B1p + b] = b < nb ? f.e1i[j1 * L + l10 + b] : 0.0;
  }
  __syncthreads();

  const int nb3 = (N3c + 15) / 16;
  const int tiles3 = ((n + 15) / 16) * nb3;
  v4d G[MAXG];
#pragma unroll
  for (int q = 0; q < MAXG; ++q) G[q] = v4d{0.0, 0.0, 0.0, 0.0};
  const int64_t LL = static_cast<int64_t>(L) * L;
  const int64_t qll = static_cast<int64_t>(Q) * LL;
  const int nks1 = (Q + 3) / 4, nks2 = (L + 3) / 4;
  // Stage 2 has few 16 x 16 tiles (2 for 32^3 velocities on the v2, v3 > 0 quarter).  When two
  // per tile fit in the waves, each tile's k-steps are split in two halves taken by different
  // waves, which evens out the four SIMDs' work: both halves add into the zeroed Y2, and
  // 0 + x + y rounds the same in either order, so the result does not depend on which wave adds
  // first.  The split costs a zeroing pass and a barrier per term, so it is used only then.
  const int mb2 = (n3 * B1 + 15) / 16, nbk2 = (n2 + 15) / 16;
  const bool ksplit = 2 * mb2 * nbk2 <= kInvWaves;

  for (int t = 0; t < d.T; ++t) {
    const double* mt = mult + t * qll + static_cast<int64_t>(l10) * L;
    // with the split, Y2 is accumulated by stage 2; nothing reads or writes it during stage 1
    if (ksplit)
      for (int i = threadIdx.x; i < 2 * B1 * N3p; i += kInvThreads) Y2r[i] = 0.0;
    {
      // stage 1: M = n3, N = nb L, K = Q
      const int M = n3, N = nb * L;
      const int mb = (M + 15) / 16, nbk = (N + 15) / 16;
      for (int blk = wave; blk < mb * nbk; blk += kInvWaves) {
        const int m0 = (blk / nbk) * 16, n0 = (blk % nbk) * 16;
        const int m = m0 + cc, c = n0 + cc;
        // Loads from clamped (in-bounds) addresses, masked after the load: no lane-divergent
        // branch between them, so all of a block's loads are in flight together.
        const int mcl = min(m, M - 1), ccl = min(c, N - 1);
        // All loads first, nothing computed from them until every one is issued (one latency per block).
        double ar[kKs1], ai[kKs1], mv[kKs1], br[kKs1], bi[kKs1];
#pragma unroll
        for (int ks = 0; ks < kKs1; ++ks) {
          ar[ks] = ai[ks] = mv[ks] = br[ks] = bi[ks] = 0.0;
          if (ks < nks1) {
            const int kcl = min(ks * 4 + kr, Q - 1);
            ar[ks] = E3r[mcl * Qp + kcl];
            ai[ks] = E3i[mcl * Qp + kcl];
            mv[ks] = mt[kcl * LL + ccl];
            br[ks] = Sr[kcl * NB + ccl];
            bi[ks] = Si[kcl * NB + ccl];
          }
        }
        v4d cr = v4d{0.0, 0.0, 0.0, 0.0}, ci = cr;
#pragma unroll
        for (int ks = 0; ks < kKs1; ++ks)
          if (ks < nks1) {
            const int k = ks * 4 + kr;
            const bool oka = k < Q && m < M, okb = k < Q && c < N;
            const double xr = oka ? ar[ks] : 0.0;
            const double xi = oka ? -ai[ks] : 0.0;   // negated: the imaginary product enters cr with a minus
            const double yr = okb ? mv[ks] * br[ks] : 0.0;
            const double yi = okb ? mv[ks] * bi[ks] : 0.0;
            cr = mfma(xr, yr, cr);
            ci = mfma(xr, yi, ci);
            cr = mfma(xi, yi, cr);
            ci = mfma(-xi, yr, ci);
          }
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = m0 + kr + 4 * r;
          if (row < M && c < N) {
            Y1r[row * NB + c] = cr[r];
            Y1i[row * NB + c] = ci[r];
          }
        }
      }
    }
    __syncthreads();
    if (t + 1 < d.T) {
      // Prefetch into L2 the multiplier lines that the stage-1 blocks read in the next term
      // (otherwise each block's first loads wait on a table of 55 MB to 0.3 GB in MALL or HBM):
      // one dword per line, lanes 0..31 the first and lanes 32..63 the last line of each row's
      // 16 columns.  The dwords land in pf through the LDS DMA path, so no register holds them.
      // The waves that stage 2 leaves idle issue it, so it does not delay stage 2.
      const double* mn = mult + (t + 1) * qll + static_cast<int64_t>(l10) * L;
      const int N1 = nb * L, nbk1 = (N1 + 15) / 16;
      const int kp = min(lane & 31, Q - 1);
      const int items2 = (ksplit ? 2 : 1) * mb2 * nbk2, nidle = kInvWaves - items2;
      const int first = nidle > 0 ? wave - items2 : wave, step = nidle > 0 ? nidle : kInvWaves;
      for (int blk = first; blk >= 0 && blk < ((n3 + 15) / 16) * nbk1; blk += step) {
        const int n0 = (blk % nbk1) * 16;
        const int c = lane < 32 ? n0 : min(n0 + 15, N1 - 1);
        __builtin_amdgcn_global_load_lds((gbl_void_t*)(mn + kp * LL + c), (lds_void_t*)pf, 4, 0, 0);
      }
    }
    {
      // stage 2: rows r = (s3, b) (M = n3 B1), columns s2 (N = n2), K = L
      const int M = n3 * B1, N = n2, nbk = nbk2;
      const int kh = ksplit ? (nks2 + 1) / 2 : nks2;
      for (int it = wave; it < (ksplit ? 2 : 1) * mb2 * nbk2; it += kInvWaves) {
        const int blk = ksplit ? it >> 1 : it;
        const int kb = ksplit && (it & 1) ? kh : 0, ke = ksplit && !(it & 1) ? kh : nks2;
        const int m0 = (blk / nbk) * 16, n0 = (blk % nbk) * 16;
        const int r = m0 + cc, s2 = n0 + cc;
        const bool rowok = r < M && (r % B1) < nb, colok = s2 < N;
        const int rcl = min(r, M - 1), s2cl = min(s2, N - 1);
        v4d cr = v4d{0.0, 0.0, 0.0, 0.0}, ci = cr;
        for (int kc = kb; kc < ke; kc += 4) {
          double ar[4], ai[4], br[4], bi[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            const int k = (kc + u) * 4 + kr, kcl = min(k, L - 1);
            const bool ok = kc + u < ke && k < L;
            const double yr = Y1r[rcl * L + kcl], yi = Y1i[rcl * L + kcl];
            const double er = E2r[s2cl * L + kcl], ei = E2i[s2cl * L + kcl];
            ar[u] = ok && rowok ? yr : 0.0;
            ai[u] = ok && rowok ? yi : 0.0;
            br[u] = ok && colok ? er : 0.0;
            bi[u] = ok && colok ? ei : 0.0;
          }
#pragma unroll
          for (int u = 0; u < 4; ++u)
            if (kc + u < ke) {
              cr = mfma(ar[u], br[u], cr);
              ci = mfma(ar[u], bi[u], ci);
              cr = mfma(-ai[u], bi[u], cr);
              ci = mfma(ai[u], br[u], ci);
            }
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const int row = m0 + kr + 4 * q, col = n0 + cc;
          const int s3 = row / B1, b = row - s3 * B1;
          if (row < M && b < nb && col < N) {
            const int o = (b * n2 + col) * n3p + s3;
            if (ksplit) {
              __hip_atomic_fetch_add(&Y2r[o], cr[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
              __hip_atomic_fetch_add(&Y2i[o], ci[q], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            } else {
              Y2r[o] = cr[q];
              Y2i[o] = ci[q];
            }
          }
        }
      }
    }
    __syncthreads();
    {
      const double* ft = field + static_cast<int64_t>(t) * d.nv;
#pragma unroll
      for (int q = 0; q < MAXG; ++q) {
        const int tile = wave + kInvWaves * q;
        if (tile < tiles3) {
          const int m0 = (tile / nb3) * 16, n0 = (tile % nb3) * 16;
          const int col = n0 + cc, ccl = min(col, N3c - 1);
          // Unmasked loads from clamped addresses (finite values): rows or columns outside the grid
          // accumulate into entries of G that are never stored, and a masked load would be turned
          // into a branch with its own wait.
          double fv[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) fv[r] = ft[min(m0 + kr + 4 * r, n - 1) * N3c + ccl];
          v4d o = v4d{0.0, 0.0, 0.0, 0.0};
          // the lane's column s2 n3 + s3 of the tile in the padded Y2 rows
          const int s2c = ccl / n3, colp = s2c * n3p + (ccl - s2c * n3);
          const int mcl = min(m0 + cc, n - 1);
          for (int k0 = 0; k0 < 2 * B1; k0 += 4) {
            const int kk = min(k0 + kr, 2 * B1 - 1);
            const int ri = kk / B1, b = kk - ri * B1;
            const bool okk = k0 + kr < 2 * B1 && b < nb;
            const double e = (ri ? E1i : E1r)[mcl * B1p + b];
            const double y = (ri ? Y2i : Y2r)[b * N3p + colp];
            const double av = okk && m0 + cc < n ? (ri ? -e : e) : 0.0;
            const double bv = okk && col < N3c ? y : 0.0;
            o = mfma(av, bv, o);
          }
#pragma unroll
          for (int r = 0; r < 4; ++r) G[q][r] += fv[r] * o[r];
        }
      }
    }
    if (ksplit) __syncthreads();   // every read of Y2 done before the next term zeroes it
  }
  // no prefetch into pf may still be in flight when the workgroup's LDS is released
  __builtin_amdgcn_s_waitcnt(0x0f70);   // vmcnt(0)
  double* out = accp + (static_cast<int64_t>(slab) * n_cells + cell) * d.nv;
#pragma unroll
  for (int q = 0; q < MAXG; ++q) {
    const int tile = wave + kInvWaves * q;
    if (tile < tiles3) {
      const int m0 = (tile / nb3) * 16, n0 = (tile % nb3) * 16;
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int j1 = m0 + kr + 4 * r, c = n0 + cc;
        if (j1 < n && c < N3c) out[j1 * N3c + c] = G[q][r];
      }
    }
  }
}

// ---------------------------------------------------------------- plan tables
// One workgroup per (term, slab of K1 output rows a1):
//   Z(a1, l3, l2)  = sum_l1 E1(a1, l1) m_t(l3, l1, l2) X(l1, l3, l2)
//   W(a1, l3, a2)  = sum_l2 Z(a1, l3, l2) E2(a2, l2)
//   O(a1, a2, a3)  = Re sum_l3 W(a1, l3, a2) E3(a3, l3)
__global__ __launch_bounds__(kThreads) void fsm_table_kernel(FsmTableArgs a, int K1) {
  extern __shared__ double sm[];
  const FsmDims d = a.d;
  const int t = a.t0 + blockIdx.y;
  const int slot = a.slot[t];
  if (slot < 0) return;
  const int L = d.L, Q = d.Q, m2 = a.m2, m3 = a.m3;
  const double* e1r = a.e1r + t * a.e1_ts;
  const double* e1i = a.e1i + t * a.e1_ts;
  const double* e2r = a.e2r + t * a.e2_ts;
  const double* e2i = a.e2i + t * a.e2_ts;
  const double* e3r = a.e3r + t * a.e3_ts;
  const double* e3i = a.e3i + t * a.e3_ts;
  const int r0 = blockIdx.x * K1, kr1 = min(K1, a.m1 - r0);
  double* Zr = sm;                    // [K1][Q][L]
  double* Zi = Zr + K1 * Q * L;
  double* Wr = Zi + K1 * Q * L;       // [K1][Q][m2]
  double* Wi = Wr + K1 * Q * m2;
  const int64_t LL = static_cast<int64_t>(L) * L;
  const double* mt = a.mult + static_cast<int64_t>(a.mrow ? a.mrow[t] : t) * Q * LL;
  const int64_t sQL = static_cast<int64_t>(Q) * L;
  {
    const int M = kr1, K = L, N = Q * L;   // column c = (l3, l2)
    auto la = [&](int m, int k, double& re, double& im) {
      const bool ok = m < M && k < K;
      re = ok ? e1r[(r0 + m) * L + k] : 0.0;
      im = ok ? e1i[(r0 + m) * L + k] : 0.0;
    };
    auto lb = [&](int k, int c, double& re, double& im) {
      if (k < K && c < N) {
        const int l3 = c / L, l2 = c - l3 * L;
        const double mv = mt[l3 * LL + static_cast<int64_t>(k) * L + l2];
        if (a.X) {
          const int64_t o = (static_cast<int64_t>(k) * 2 * Q + l3) * L + l2;
          re = mv * a.X[o];
          im = mv * a.X[o + sQL];
        } else {
          re = mv;
          im = 0.0;
        }
      } else {
        re = im = 0.0;
      }
    };
    auto st = [&](int m, int c, double re, double im) {
      Zr[m * N + c] = re;
      Zi[m * N + c] = im;
    };
    cgemm<2>(M, N, K, la, lb, st);
  }
  __syncthreads();
  {
    const int M = kr1 * Q, K = L, N = m2;  // row r = (a1, l3)
    auto la = [&](int m, int k, double& re, double& im) {
      const bool ok = m < M && k < K;
      re = ok ? Zr[m * L + k] : 0.0;
      im = ok ? Zi[m * L + k] : 0.0;
    };
    auto lb = [&](int k, int c, double& re, double& im) {
      const bool ok = k < K && c < N;
      re = ok ? e2r[c * L + k] : 0.0;
      im = ok ? e2i[c * L + k] : 0.0;
    };
    auto st = [&](int m, int c, double re, double im) {
      Wr[m * m2 + c] = re;
      Wi[m * m2 + c] = im;
    };
    cgemm<2>(M, N, K, la, lb, st);
  }
  __syncthreads();
  {
    const int M = kr1 * m2, K = Q, N = m3;  // row r = (a1, a2)
    auto la = [&](int m, int k, double& re, double& im) {
      const bool ok = m < M && k < K;
      const int a1 = ok ? m / m2 : 0, a2 = m - a1 * m2;
      re = ok ? Wr[(a1 * Q + k) * m2 + a2] : 0.0;
      im = ok ? Wi[(a1 * Q + k) * m2 + a2] : 0.0;
    };
    auto lb = [&](int k, int c, double& re, double& im) {
      const bool ok = k < K && c < N;
      re = ok ? e3r[c * Q + k] : 0.0;
      im = ok ? e3i[c * Q + k] : 0.0;
    };
    const double sc = a.scale[t];
    double* out = a.out + static_cast<int64_t>(slot) * a.m1 * m2 * m3;
    auto st = [&](int m, int c, double re, double) {
      out[(static_cast<int64_t>(r0) * m2 + m) * m3 + c] = sc * re;
    };
    cgemm<2>(M, N, K, la, lb, st);
  }
}

__global__ void fsm_gather_kernel(FsmDims d, int nrows, const double* __restrict__ in, const int* __restrict__ src,
                                  const double* __restrict__ feq, double scale, double* __restrict__ out) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= static_cast<int64_t>(nrows) * d.nv) return;
  const int t = static_cast<int>(i / d.nv), v = static_cast<int>(i - static_cast<int64_t>(t) * d.nv);
  const int s3 = v % d.n3, s2 = (v / d.n3) % d.n2, j1 = v / (d.n3 * d.n2);
  const int n = d.n;
  const int64_t full = (static_cast<int64_t>(j1) * n + s2 + (n - d.n2)) * n + s3 + (n - d.n3);
  const int r = src[t];
  out[i] = scale * (r >= 0 ? in[static_cast<int64_t>(r) * n * n * n + full] : -feq[full]);
}

__global__ void fsm_shift_factor_kernel(int nt, int m, int nl, int lmin, int doubled, const int* __restrict__ base,
                                        const double* __restrict__ shift, int shift_stride, int P,
                                        double* __restrict__ er, double* __restrict__ ei) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= static_cast<int64_t>(nt) * m * nl) return;
  const int k = static_cast<int>(i % nl), a = static_cast<int>((i / nl) % m), t = static_cast<int>(i / (static_cast<int64_t>(nl) * m));
  const int l = lmin + k;
  // the angle pi q / P with q = l (base + 2 z) reduced mod 2P before the sine and cosine
  double q = l * (base[a] + 2.0 * shift[static_cast<int64_t>(t) * shift_stride]);
  q -= 2.0 * P * floor(q / (2.0 * P));
  const double ang = M_PI * q / P;
  const double w = (doubled && l > 0) ? 2.0 : 1.0;
  er[i] = w * cos(ang);
  ei[i] = w * sin(ang);
}

__global__ void band_profile_kernel(int nt, int m, int off, const double* __restrict__ g, int ng,
                                    const double* __restrict__ z, int P, double* __restrict__ S) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= static_cast<int64_t>(nt) * 3 * m) return;
  const int a = static_cast<int>(i % m), k = static_cast<int>((i / m) % 3), t = static_cast<int>(i / (3 * m));
  const double zz = z[3 * t + k];
  auto dirichlet = [&](double w) {
    double s = 1.0;
    for (int l = 1; l < P / 2; ++l) s += 2.0 * cos(2.0 * M_PI * l * w / P);
    return s / P;
  };
  double acc = 0.0;
  if (ng == 0) {
    acc = dirichlet(off + a + zz);
  } else {
    for (int j = 0; j < ng; ++j) acc += g[j] * dirichlet(off + a - j + zz);
  }
  S[i] = acc;
}

__global__ void separable_kernel(int nt, int m, const double* __restrict__ S, const double* __restrict__ w,
                                 double* __restrict__ out) {
  const int64_t m3 = static_cast<int64_t>(m) * m * m;
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nt * m3) return;
  const int t = static_cast<int>(i / m3);
  const int64_t r = i - t * m3;
  const int a0 = static_cast<int>(r / (m * m)), a1 = static_cast<int>((r / m) % m), a2 = static_cast<int>(r % m);
  const double* St = S + static_cast<int64_t>(t) * 3 * m;
  out[i] = w[t] * St[a0] * St[m + a1] * St[2 * m + a2];
}

__global__ void scale_rows_kernel(int nt, int64_t len, const double* __restrict__ in, const int* __restrict__ src,
                                  const double* __restrict__ sc, double* __restrict__ out) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= nt * len) return;
  const int t = static_cast<int>(i / len);
  out[i] = sc[t] * in[static_cast<int64_t>(src[t]) * len + (i - t * len)];
}

size_t table_lds_bytes(const FsmDims& d, int m2, int K1) {
  return static_cast<size_t>(2 * K1 * d.Q * d.L + 2 * K1 * d.Q * m2) * sizeof(double);
}

int stage3_tiles_per_wave(const FsmDims& d) {
  const int tiles = ((d.n + 15) / 16) * ((d.n2 * d.n3 + 15) / 16);
  return (tiles + kInvWaves - 1) / kInvWaves;
}

size_t forward_lds_bytes(const FsmDims& d, int B3) {
  return static_cast<size_t>(2 * B3 * d.n * d.n2 + 2 * B3 * d.L * d.n) * sizeof(double);
}

// l3 modes per forward workgroup: the most (up to 4) whose LDS fits two workgroups per CU
int forward_chunk(const FsmDims& d) {
  int B3 = 4;
  while (B3 > 1 && forward_lds_bytes(d, B3) > 80 * 1024) --B3;
  return B3;
}

size_t inverse_lds_bytes(const FsmDims& d, int B1) {
  const size_t NB = static_cast<size_t>(B1) * d.L;
  // Y2, E3 and E1 rows padded by one double (bank spread of the column-wise lane accesses)
  // (+ 32 doubles written by the multiplier prefetch)
  return (2 * d.Q * NB + 2 * d.n3 * NB + 2 * static_cast<size_t>(B1) * d.n2 * (d.n3 + 1) +
          2 * static_cast<size_t>(d.n3) * (d.Q + 1) + 2 * static_cast<size_t>(d.n2) * d.L +
          2 * static_cast<size_t>(d.n) * (B1 + 1) + 32) *
         sizeof(double);
}

constexpr size_t kLdsMax = 160 * 1024;

}  // namespace

hipError_t launch_fsm_multipliers(const FsmMultArgs& a, hipStream_t s) {
  const int64_t qll = static_cast<int64_t>(a.d.Q) * a.d.L * a.d.L;
  hipLaunchKernelGGL(fsm_mult_kernel, dim3(static_cast<unsigned>((qll + 255) / 256)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_fsm_forward(const FsmDims& d, const FsmFactors& f, int64_t n_cells, const double* h, double* S,
                              hipStream_t s) {
  if (n_cells <= 0) return hipSuccess;
  const int B3 = forward_chunk(d);
  const size_t lds = forward_lds_bytes(d, B3);
  if (lds > kLdsMax) return hipErrorInvalidValue;
  dim3 grid((d.Q + B3 - 1) / B3, static_cast<unsigned>(n_cells));
  hipLaunchKernelGGL(fsm_forward_kernel, grid, dim3(kThreads), lds, s, d, f, B3, h, S);
  return hipGetLastError();
}

hipError_t launch_fsm_gather(const FsmDims& d, int nrows, const double* in, const int* src, const double* feq,
                             double scale, double* out, hipStream_t s) {
  const int64_t total = static_cast<int64_t>(nrows) * d.nv;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(fsm_gather_kernel, dim3(static_cast<unsigned>((total + 255) / 256)), dim3(256), 0, s, d, nrows,
                     in, src, feq, scale, out);
  return hipGetLastError();
}

hipError_t launch_fsm_shift_factors(int nt, int m, int nl, int lmin, int doubled, const int* base, const double* shift,
                                    int shift_stride, int P, double* er, double* ei, hipStream_t s) {
  const int64_t total = static_cast<int64_t>(nt) * m * nl;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(fsm_shift_factor_kernel, dim3(static_cast<unsigned>((total + 255) / 256)), dim3(256), 0, s, nt, m,
                     nl, lmin, doubled, base, shift, shift_stride, P, er, ei);
  return hipGetLastError();
}

hipError_t launch_band_profiles(int nt, int m, int off, const double* g, int ng, const double* z, int P, double* S,
                                hipStream_t s) {
  const int64_t total = static_cast<int64_t>(nt) * 3 * m;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(band_profile_kernel, dim3(static_cast<unsigned>((total + 255) / 256)), dim3(256), 0, s, nt, m, off,
                     g, ng, z, P, S);
  return hipGetLastError();
}

hipError_t launch_separable(int nt, int m, const double* S, const double* w, double* out, hipStream_t s) {
  const int64_t total = static_cast<int64_t>(nt) * m * m * m;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(separable_kernel, dim3(static_cast<unsigned>((total + 255) / 256)), dim3(256), 0, s, nt, m, S, w,
                     out);
  return hipGetLastError();
}

hipError_t launch_scale_rows(int nt, int64_t len, const double* in, const int* src, const double* sc, double* out,
                             hipStream_t s) {
  const int64_t total = static_cast<int64_t>(nt) * len;
  if (total <= 0) return hipSuccess;
  hipLaunchKernelGGL(scale_rows_kernel, dim3(static_cast<unsigned>((total + 255) / 256)), dim3(256), 0, s, nt, len, in,
                     src, sc, out);
  return hipGetLastError();
}

bool fsm_tables_fit(const FsmDims& d, int m2) { return table_lds_bytes(d, m2, 1) <= kLdsMax; }

hipError_t launch_fsm_tables(const FsmTableArgs& a, hipStream_t s) {
  if (a.nt <= 0) return hipSuccess;
  int K1 = 4;
  while (K1 > 1 && table_lds_bytes(a.d, a.m2, K1) > kLdsMax) --K1;
  const size_t lds = table_lds_bytes(a.d, a.m2, K1);
  if (lds > kLdsMax) return hipErrorInvalidValue;
  dim3 grid((a.m1 + K1 - 1) / K1, a.nt);
  hipLaunchKernelGGL(fsm_table_kernel, grid, dim3(kThreads), lds, s, a, K1);
  return hipGetLastError();
}

int fsm_slab_count(const FsmDims& d, int slab_l1) { return (d.L + slab_l1 - 1) / slab_l1; }

int fsm_default_slab(const FsmDims& d) {
  int B1 = 4;
  while (B1 > 1 && inverse_lds_bytes(d, B1) > kLdsMax) --B1;
  return B1;
}

bool fsm_slab_fits(const FsmDims& d, int slab_l1) {
  return slab_l1 >= 1 && slab_l1 <= d.L && inverse_lds_bytes(d, slab_l1) <= kLdsMax;
}

const char* fsm_unsupported(const FsmDims& d) {
  if (stage3_tiles_per_wave(d) > 8)
    return "the per-cell transform path holds at most 64 x 16 x 16 outputs per cell (use parity storage)";
  if (d.Q > 4 * kKs1) return "the per-cell transform path takes n_pad <= 64";
  if (inverse_lds_bytes(d, 1) > kLdsMax || forward_lds_bytes(d, 1) > kLdsMax)
    return "velocity grid too large for the per-cell transform path";
  return nullptr;
}

hipError_t launch_fsm_inverse(const FsmDims& d, const FsmFactors& f, int slab_l1, int64_t n_cells, const double* S,
                              const double* mult, const double* field, double* acc, hipStream_t s) {
  if (n_cells <= 0) return hipSuccess;
  const size_t lds = inverse_lds_bytes(d, slab_l1);
  if (lds > kLdsMax) return hipErrorInvalidValue;
  dim3 grid(fsm_slab_count(d, slab_l1), static_cast<unsigned>(n_cells));
  const int g = stage3_tiles_per_wave(d);
  if (g <= 2)
    hipLaunchKernelGGL(fsm_inverse_kernel<2>, grid, dim3(kInvThreads), lds, s, d, f, slab_l1, S, mult, field, acc,
                       n_cells);
  else if (g <= 4)
    hipLaunchKernelGGL(fsm_inverse_kernel<4>, grid, dim3(kInvThreads), lds, s, d, f, slab_l1, S, mult, field, acc,
                       n_cells);
  else if (g <= 6)
    hipLaunchKernelGGL(fsm_inverse_kernel<6>, grid, dim3(kInvThreads), lds, s, d, f, slab_l1, S, mult, field, acc,
                       n_cells);
  else if (g <= 8)
    hipLaunchKernelGGL(fsm_inverse_kernel<8>, grid, dim3(kInvThreads), lds, s, d, f, slab_l1, S, mult, field, acc,
                       n_cells);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

double fsm_flops_per_cell(const FsmDims& d, int slab_l1) {
  // MFMAs issued (2048 flops each): forward stages, then per slab and term the three inverse stages
  auto t16 = [](int x) { return static_cast<double>((x + 15) / 16); };
  auto k4 = [](int x) { return static_cast<double>((x + 3) / 4); };
  double fwd = 0.0;
  const int B3 = forward_chunk(d);
  for (int q0 = 0; q0 < d.Q; q0 += B3) {
    const int nq = std::min(B3, d.Q - q0);
    fwd += t16(nq) * t16(d.n * d.n2) * k4(d.n3) * 4.0;
    fwd += t16(d.L) * t16(nq * d.n) * k4(d.n2) * 4.0;
    fwd += t16(d.L) * t16(nq * d.L) * k4(d.n) * 4.0;
  }
  double inv = 0.0;
  const int slabs = fsm_slab_count(d, slab_l1);
  for (int sl = 0; sl < slabs; ++sl) {
    const int nb = std::min(slab_l1, d.L - sl * slab_l1);
    const double s1 = t16(d.n3) * t16(nb * d.L) * k4(d.Q) * 4.0;
    const double s2 = t16(d.n3 * slab_l1) * t16(d.n2) * k4(d.L) * 4.0;
    const double s3 = t16(d.n) * t16(d.n2 * d.n3) * k4(2 * slab_l1);
    inv += d.T * (s1 + s2 + s3);
  }
  return 2048.0 * (fwd + inv);
}

}  // namespace sis
