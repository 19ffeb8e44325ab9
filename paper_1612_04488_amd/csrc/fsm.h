// The fast spectral method evaluated per cell on the device: separable pruned
// DFTs of the velocity grid as small complex GEMMs on the FP64 MFMA, staged in
// LDS (fsm.hip).  All pointers are device pointers.
//
// Modes: l1, l2 take the P - 1 signed values -(P/2 - 1) .. P/2 - 1 (index
// l + P/2 - 1; the Nyquist mode -P/2 carries no multiplier), l3 the Q = P/2
// values 0 .. P/2 - 1 (half spectrum: h is real, so its transform is
// Hermitian).  Frequencies xi_l = pi l / L_p, velocities v_j = (j + 1/2 - n/2) dv.
//
// Stored velocities follow the plan's parity storage: axis 1 all n nodes,
// axis 2 the n2 = n or n/2 nodes with v2 > 0 (even images), axis 3 the n3 = n
// or n/2 nodes with v3 > 0 (odd images).  The forward factors fold the images
// in, so the stored half transforms to the full-grid spectrum.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sis {

struct FsmDims {
  int n;        // velocity nodes per axis
  int P;        // padded DFT size per axis
  int L;        // P - 1 modes on axes 1, 2
  int Q;        // P / 2 modes on axis 3
  int n2, n3;   // stored nodes on axes 2, 3
  int nv;       // n * n2 * n3 stored velocities per cell
  int T;        // terms: 2 D gain terms and the loss
};

// Factor matrices, complex planar (re, im), row-major:
//   forward  F1 [L][n], F2 [L][n2], F3 [Q][n3]   (images folded in)
//   inverse  E1 [n][L], E2 [n2][L], E3 [n3][Q]   (E3 carries 1 for l3 = 0, 2 otherwise)
struct FsmFactors {
  const double *f1r, *f1i, *f2r, *f2i, *f3r, *f3i;
  const double *e1r, *e1i, *e2r, *e2i, *e3r, *e3i;
};

// Multipliers m[T][Q][L][L] (term 2p: psi_p, 2p + 1: phi_p, 2D: beta) of the
// half spectrum, evaluated on the device.  dirs[D][3], W[D]; the radial rule as
// RadialRule (planner.h): phi_closed / psi_closed select the closed forms, else
// the node tables (nodes, weights) are used.
struct FsmMultArgs {
  FsmDims d;
  int D;
  double b0, R, Lp;
  const double* dirs;
  const double* W;
  int phi_closed, psi_closed;
  int n_phi, n_psi;
  const double *phi_x, *phi_w, *psi_x, *psi_w;
  double* mult;
};
hipError_t launch_fsm_multipliers(const FsmMultArgs& a, hipStream_t s);

// Forward transform of n_cells cells: h [cells][nv] (stored layout) ->
// S [cells][L (l1)][2 (re, im)][Q (l3)][L (l2)].
hipError_t launch_fsm_forward(const FsmDims& d, const FsmFactors& f, int64_t n_cells, const double* h, double* S,
                              hipStream_t s);

// Inverse transforms of every term with their field products, summed:
//   acc[slab][cell][i] = sum_t field[t][i] Re sum_{l1 in slab} sum_{l2, l3} E1 E2 E3 mult[t][l] S[cell][l]
// for the l1 slabs of slab_l1 modes each (n_slabs = ceil(L / slab_l1)); the
// slabs' partial sums add up to L+ of each cell at delta = 1.
int fsm_slab_count(const FsmDims& d, int slab_l1);
int fsm_default_slab(const FsmDims& d);
// whether the inverse kernel's LDS holds a slab of slab_l1 modes
bool fsm_slab_fits(const FsmDims& d, int slab_l1);
// 0 if the dimensions are within what the inverse kernel holds in registers
// (stage-3 output tiles per wave), else the reason.
const char* fsm_unsupported(const FsmDims& d);
hipError_t launch_fsm_inverse(const FsmDims& d, const FsmFactors& f, int slab_l1, int64_t n_cells, const double* S,
                              const double* mult, const double* field, double* acc, hipStream_t s);
// Per-term pruned inverse DFTs of the multipliers (plan-time tables), times a
// spectrum X (layout of S, one cell) or X = 1 when X is null:
//   out[slot[t]][a1][a2][a3] = scale[t] Re sum_l E1(a1, l1) E2(a2, l2) E3(a3, l3) m_t(l) X(l)
// for the terms t in [t0, t0 + nt), on output nodes given by the factor matrices
// E1 [m1][L], E2 [m2][L], E3 [m3][Q] (E3 doubled for l3 > 0 as in FsmFactors).
// Terms with slot[t] < 0 are skipped.
struct FsmTableArgs {
  FsmDims d;
  int m1, m2, m3;
  const double *e1r, *e1i, *e2r, *e2i, *e3r, *e3i;
  int64_t e1_ts, e2_ts, e3_ts;  // per-term strides of the factor arrays (0: one set for all terms)
  const double* mult;
  const int* mrow;      // [T] multiplier row of each term, or null (row t)
  const double* X;
  const int* slot;      // [T]
  const double* scale;  // [T]
  double* out;
  int t0, nt;
};
hipError_t launch_fsm_tables(const FsmTableArgs& a, hipStream_t s);
// whether launch_fsm_tables holds the modes of d and m2 output nodes on axis 2 in LDS
bool fsm_tables_fit(const FsmDims& d, int m2);

// Shifted factor matrices of nt terms on m nodes and nl modes l = lmin .. lmin + nl - 1:
//   e[t][a][k] = w(l) e^{i pi l (base[a] + 2 shift[t]) / P},  w = 1, or (doubled != 0) 2 for l > 0,
// re and im parts in er, ei ([nt][m][nl] each); base[a] are integers (2a + 1 - n for the velocity
// nodes, 2(a - (n - 1)) for the difference grid), shift[t] in grid spacings.
hipError_t launch_fsm_shift_factors(int nt, int m, int nl, int lmin, int doubled, const int* base, const double* shift,
                                    int shift_stride, int P, double* er, double* ei, hipStream_t s);

// One-dimensional band-limited profiles of nt terms on three axes:
//   S[t][k][a] = sum_{j < ng} g[j] D_P(off + a - j + z[t][k])   (ng = 0: D_P(off + a + z[t][k])),
// D_P(w) = (1/P) sum over the non-Nyquist modes l of e^{2 pi i l w / P}; and their products
//   out[t][a0][a1][a2] = w[t] S[t][0][a0] S[t][1][a1] S[t][2][a2].
hipError_t launch_band_profiles(int nt, int m, int off, const double* g, int ng, const double* z, int P, double* S,
                                hipStream_t s);
hipError_t launch_separable(int nt, int m, const double* S, const double* w, double* out, hipStream_t s);
// out[t][i] = s[t] in[src[t]][i], i < len
hipError_t launch_scale_rows(int nt, int64_t len, const double* in, const int* src, const double* sc, double* out,
                             hipStream_t s);

// Field table of the per-cell path from full-grid rows: for t < nrows,
//   out[t][v] = scale * (src[t] >= 0 ? in[src[t]][full(v)] : -feq[full(v)])
// over the stored velocities v of d (full(v): index of v on the n^3 grid).
hipError_t launch_fsm_gather(const FsmDims& d, int nrows, const double* in, const int* src, const double* feq,
                             double scale, double* out, hipStream_t s);

// Executed flops of one cell update (every MFMA issued, padding included)
double fsm_flops_per_cell(const FsmDims& d, int slab_l1);

}  // namespace sis
