// Launch wrappers of the device kernels (kernels.hip).  All pointers are
// device pointers; every wrapper enqueues on `s` and returns the launch status.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sis {

// Operator assembly on one n^3 x n^3 block (row stride ldo):
//   op[i][j] = (accumulate ? op[i][j] : 0) + sum_t X_t(i) Y_t(i - j)
//              - loss_coef feq(i) beta_r(i - j)          (loss skipped if feq is null)
// X: [T][n^3] fields, Y: [T][(2n-1)^3] real-space kernels on the difference grid.
hipError_t launch_assemble(int n, int T, const double* X, const double* Y, const double* feq,
                           double loss_coef, const double* beta_r, double* op, int64_t ldo, int accumulate,
                           hipStream_t s);

// Restriction of the operator (row stride ld, nsp species blocks of n^3) to distributions odd in
// v3 (parity 1) or odd in v3 and even in v2 (parity 2): stored velocities v3 > 0 (and v2 > 0),
// red is [nsp*nv][nsp*nv], nv = n * (parity 2 ? n/2 : n) * n/2.
hipError_t launch_reduce_operator(const double* op, int64_t ld, double* red, int nsp, int n, int parity,
                                  hipStream_t s);

// op2 = op (double) rounded to float.
hipError_t launch_convert_f32(const double* op, float* out, int64_t count, hipStream_t s);

// BF16 pair layout of the low-precision contraction operands: rows of K values
// stored with Kp = pair_stride(K) (K rounded up to 64); row r occupies 2 Kp bf16
// at P + 2 Kp r, and each block of 32 k-values holds the 32 hi parts, then their
// 32 lo parts; entries k >= K are zero.  launch_split_pairs writes
// x = X - Xref (Xref may be null) for rows x K doubles: hi = RNE(x),
// lo = RNE(x - hi), or lo = 0 when with_lo is 0.  P holds rows * 2 Kp bf16.
int pair_stride(int K);
hipError_t launch_split_pairs(const double* X, const double* Xref, int64_t rows, int K, uint16_t* P, int with_lo,
                              hipStream_t s);

// Contraction acc[z][m][n] = sum_{k in split z} X[m][k] * op[n][k]  (op stored n x k).
// precision: 0 fp64 (op64), 1 fp32 (op32), 2 bf16x3, 3 bf16 (hi products only)
// (Xp, opp in the pair layout).  Accumulators are written as double for every
// precision.
struct GemmArgs {
  int precision;
  const double* X;         // FP64 cell operand (precision 0, and the FP32 path's source)
  const double* Xref;      // null, or anchor: the contraction is applied to X - Xref
  const uint16_t* Xp;      // precisions 2, 3: X - Xref in the pair layout, M rows (launch_split_pairs)
  const float* X32;        // precision 1: X - Xref rounded to FP32 [M][K] (launch_convert_x_f32)
  const double* op64;
  const float* op32;
  const uint16_t* opp;     // precisions 2, 3: the operator in the pair layout, N rows
  double* acc;
  int64_t M;
  int N, K;
  int splits;        // split-K factor (grid.z)
  int tile;          // tile configuration id: 0 (128 x 128), 2 (64 x 128), 1 (32 x 128) with 16-deep
                     // double-buffered stages (64-deep single-buffered for the bf16 forms; FP64 tile 0:
                     // eight waves, LDS-DMA stages of k pairs, for K <= 2^20); FP64 only:
                     // 3 (128 x 128), 4 (64 x 128) with 32-deep single-buffered stages; BF16X3 only:
                     // 5 (256 x 256, 32-deep LDS-DMA stages in two buffers; gemm_wide_fits).
                     // FP64 needs K even (hipErrorInvalidValue otherwise).
};
int gemm_tile_rows(int tile);
int gemm_tile_depth(int tile, int precision);
// whether the 256 x 256 BF16X3 tile takes M cells against N operator rows of K
// (both pair arrays under 4 GiB: its loads use 32-bit offsets)
bool gemm_wide_fits(int64_t M, int N, int K);
hipError_t launch_gemm(const GemmArgs& a, hipStream_t s);
// x = X - Xref (Xref may be null) -> FP32; count = M * K
hipError_t launch_convert_x_f32(const double* X, const double* Xref, int64_t count, float* out, hipStream_t s);
int gemm_k_per_split(int K, int splits);

// Rows are (cell, species) pairs of n3 values: row = cell * nsp + species.  A row holds the
// velocities (v1, v2, v3) on n x d2 x d3 nodes (v1d, v2d, v3d): the full grid, or v3 > 0 (and
// v2 > 0) when the distribution is stored by parity; w then carries the image count.
struct FinishArgs {
  int n3;                  // stored velocities per (cell, species) row
  int even_v2;             // h stored for v2 > 0 only: the v2 v3 moments are zero
  int nsp;                 // species per cell (1 or 2)
  double mass_ratio[2];    // m_s / m_A (1 for one gas)
  int64_t n_cells;         // rows = cells * nsp
  int splits;              // split-K partial sums in acc (0: the contraction is zero)
  const double* acc;       // [splits][rows][n3]
  const double* h;         // [rows][n3]
  const double* dU;        // [rows] or null
  const double* delta;     // [cells]
  const int32_t* flow;     // [cells] or null
  int project;             // one gas only
  const double* vtab;      // [3][n3] v1, v2, v3 of each stored velocity
  const double* wtab;      // [n3] its quadrature weight (images of unstored half spaces included)
  const double* feq;       // [nsp][n3]
  const double* nu;        // [nsp][n3]
  const double* Kc;        // [nsp][nsp][n3]: L+_1 of the correction 2 (m_q/m_A) v3 f_q of species q
  const double* gram_inv;  // [25]
  const int32_t* active;   // [cells] or null: skip cells with active == 0
  // FP64-anchored defect correction (solver only; mode 0 = off):
  //  mode 1 (refresh):     acc is op*h in FP64; store accref = acc, xref = h
  //  mode 2 (incremental): acc is op~*(h - xref); use accref + acc
  int anchor_mode;
  double* accref;          // [n_cells][n3]
  double* xref;            // [n_cells][n3]
  double* rhs;             // [n_cells][n3]  (may alias acc when splits == 1)
  double* lh;              // [n_cells][n3] or null
  double* amom;            // [n_cells][4] or null
};
hipError_t launch_finish(const FinishArgs& a, hipStream_t s);

struct SweepArgs {
  int n, n3;
  int d2, d3;                // stored v2, v3 nodes per row (see FinishArgs)
  int nsp;                   // species per cell; grid.z runs over species
  int n_cases;
  const int64_t* node_off;   // [n_cases+1]
  const double* coef;        // [cells][6]: backward a,b,c ; forward a,b,c
  const double* delta_case;  // [n_cases]
  const double* v1d;         // [n]
  const double* nu;          // [nsp][n3]
  const double* rhs;         // [cells][nsp][n3], not aliasing h
  double* h;                 // [cells][nsp][n3]
  const int32_t* case_active;// [n_cases] or null
};
hipError_t launch_sweep1d(const SweepArgs& a, hipStream_t s);
// mom[row][4] = {U3, q3, G1, P13} of h[row][n x d2 x d3] directly (rows = cells * nsp;
// q3 and P13 weighted with the mass ratio of the row's species)
hipError_t launch_moments(int n3, int nsp, const double* mass_ratio, int64_t n_rows, const double* vtab,
                          const double* h, double w, double* mom, hipStream_t s);

struct DiffusionArgs {
  int n_cases;
  const int64_t* node_off;
  const double* x;           // [cells]
  const double* coef;        // [cells][6]
  const double* delta_case;  // [n_cases]
  const int32_t* flow_case;  // [n_cases]
  const double* mom;         // [cells][4]
  const double* amom;        // [cells][4] or null
  double N;
  int sis;                   // 1: solve the velocity equation; 0: dU = 0 (CIS)
  double cU, cq;             // moments U3, q3 of the correction shape 2 v3 f_eq
  double* U;                 // [cells] or null
  double* dU;                // [cells] or null
  // solver state (all null outside sis_solve)
  double* state;             // [n_cases][4]: M_prev, Q_prev, residual, M  (+ Q in [n_cases][4]+..)
  int32_t* iters;            // [n_cases]
  int32_t* case_active;      // [n_cases]
  double* qfield;            // [cells] q3 of the new iterate or null
  double* ufield;            // [cells] U3 of the new iterate or null
  int32_t* cell_active;      // [cells] or null: set to the case's flag after its march (1-D cases)
  double eps;
  // binary mixture (nsp == 2): arrays above are per (cell, species) row,
  // state is [n_cases][6] = {M_A, M_B, Q_A, Q_B, residual, iterations}
  int nsp;
  double chi[2], mass_ratio[2], Ns[2], cUs[2], cqs[2];
  double flow_factor;        // sqrt(m / m_A)
};
hipError_t launch_diffusion1d(const DiffusionArgs& a, hipStream_t s);

// Persistent 1-D iteration (one gas, FP64 contraction): n_iters whole SIS/CIS iterations in
// one cooperative launch of `blocks` workgroups (at most persist1d_max_blocks()), the phases
// separated by grid barriers.  The contraction runs on 32 x 128 tiles with split-K slices of
// kps (a multiple of 16) into acc [splits][n_cells][n3]; fin, sw, dif are the launched path's
// arguments for the finish, sweep and velocity-equation steps (fin.acc and fin.splits are set
// per iteration).  first_from_zero: the first iteration starts from h = 0 and skips the
// contraction.  cell_active [n_cells] is rewritten from dif.case_active after each march.
// bar: 4 device words, zeroed by the launcher; bar[2] != 0 after the launch means a barrier
// wait ran out (the results are then invalid).
struct Persist1DArgs {
  const double* h;
  const double* op;
  double* acc;
  int64_t n_cells;
  int n3, kps, splits;
  FinishArgs fin;
  SweepArgs sw;
  const double* vtab;
  double w;
  double* mom;
  DiffusionArgs dif;
  int32_t* cell_active;
  int n_iters, first_from_zero;
  unsigned* bar;
};
int persist1d_max_blocks();
hipError_t launch_persist1d(const Persist1DArgs& a, int blocks, hipStream_t s);

// ---------------------------------------------------------------- 2-D cross sections
struct Sweep2DArgs {
  int n, n3, n_cases;
  int nsp;                   // species per cell: rows cell * nsp + s, nu of species s at nu + s * n3
  int d3;                    // stored v3 nodes (n, or n/2 for distributions odd in v3)
  const double* v3d;
  const int32_t* n1;
  const int32_t* n2;
  const int64_t* grid_off;
  const int32_t* gcell;      // [grid] global fluid cell or -1
  const double* coef;        // [cell][2][2][3]
  const int32_t* ref;        // [cell][2][2][2]
  const int8_t* kind;        // [cell][2][2][2]
  const uint32_t* rec;       // [cell][2][2] 32-byte records: the three coefficients (FP64), then
                             // (ref << 2 | kind) of both references (0 for kind 0)
  const uint32_t* grec;      // [grid + 1][2][2] the records in grid order, coefficients of kind-0
                             // references set to 0; at solid cells a = 1, the rest 0
  const uint32_t* growb;     // [grid + 1] byte offset of the cell's first row (species 0) in h and
                             // rhs, 0xffffffff at solid cells (valid while h is under 2 GiB)
  int64_t grid_none;         // index of the extra solid entry of grec and growb (positions
                             // outside the grid)
  int64_t row_bytes_total;   // bytes of h (all cells and species)
  int quad_split;            // no mirror ghosts: the four quadrants are independent
  const double* delta_case;
  const double* v1d;
  const double* nu;
  const double* rhs;
  double* h;                 // in: previous iterate (lagged periodic values), out: new
  const int32_t* case_active;
  int max_diag;              // largest min(n1, n2) over the cases (cells on an anti-diagonal)
  int max_n2;                // largest n2 over the cases
};
hipError_t launch_sweep2d(const Sweep2DArgs& a, hipStream_t s);
// Kernel form launch_sweep2d takes: 1 sweep2d_rows_kernel (max_n2 <= 128 and h under 2 GiB),
// else for anti-diagonals of up to max_diag cells 2 sweep2d_pipelined_kernel (max_diag <= 192)
// or 3 sweep2d_kernel.
int sweep2d_form(int max_diag, int max_n2, int64_t row_bytes_total);
// mom[cell][species][8] = {U3, q3, G1, G12, G2, P13, P23, 0}; rows of n x n x d3 velocities;
// q3 and P13, P23 carry the species mass ratio (q3 = int (a v^2 - 5/2) v3 h, P = 2 a int v v3 h)
hipError_t launch_moments2d(int n3, int nsp, const double* mass_ratio, int64_t n_cells, const double* vtab,
                            const double* h, double w, const int32_t* cell_active, double* mom, hipStream_t s);

struct Diff2DArgs {
  int n_cases;
  int64_t n_grid;            // grid cells of all cases (species workspace stride)
  const int32_t* n2;
  const int64_t* grid_off;
  const int8_t* dflag;
  const int32_t* gcell;
  const int32_t* nb;
  const int8_t* nbm;
  const double* npos;
  const double* fw;
  const double* width;
  const double* cpos;
  const double* dA;
  const double* area;
  const double* delta_case;
  const int32_t* flow_case;
  const double* mom;         // [cell][species][8]
  const double* amom;        // [cell][species][4] or null
  int sis;
  // species (one gas: nsp 1, chi 1, mass ratio 1, Ns = N, cUs/cqs = the one-gas factors)
  int nsp;
  double chi[2], mass_ratio[2], Ns[2], cUs[2], cqs[2];
  double flow_factor;        // sqrt(m / m_A) (mixtures)
  double* work;              // [species][grid][kDiffWork]
  int32_t* have_x;           // [n_cases]: warm start available
  double tol;
  int max_iter;
  double* U;                 // [cell][species] diffusion solution or null
  double* dU;                // [cell][species] or null
  double* ufield;            // [cell][species] U3 of the new iterate or null
  double* qfield;            // [cell][species] q3 of the new iterate or null
  double* state;             // [n_cases][2 nsp + 2] or null
  int32_t* iters;
  int32_t* case_active;
  double eps;
  int32_t* cg_iters;         // [n_cases] or null
  // inverse form (cases with direct[c] != 0): A^-1 of the case's unknown cells, precomputed
  const int32_t* direct;     // [n_cases] or null (CG for every case; one gas only)
  const int32_t* uidx;       // [grid] compact unknown index within its case, -1 otherwise
  const int64_t* uoff;       // [n_cases] unknowns of the earlier cases; species s of case c
                             // has its right side / solution at nsp * uoff[c] + s * n_unknown[c]
  const int32_t* n_unknown;  // [n_cases]
  int max_unknown;
  // right sides with the same cross section share one inverse: group g holds grp_size[g] <= 8
  // vectors at bvec / yvec + grp_vec[g * 8 + m], its inverse at ainv + grp_aoff[g] (grp_n[g]^2)
  int n_groups;
  const int64_t* grp_aoff;
  const int32_t* grp_n;
  const int32_t* grp_size;
  const int64_t* grp_vec;
  const double* ainv;
  double* bvec;              // [nsp * unknowns]
  double* yvec;              // [nsp * unknowns]
};
constexpr int kInverseGroup = 8;
// workspace per (species, grid cell): Uh G1 G12 G2 A1 A2 | CG: x r p Ap | P_B13 P_B23
constexpr int kDiffWork = 12;
// CG kernel for cases without an inverse, then (if a.direct) right sides, y = A^-1 b, outputs
hipError_t launch_diffusion2d(const Diff2DArgs& a, hipStream_t s);
// Newton-Schulz helpers (plan time): per-block sum of squares of I - P into part[blocks];
// P <- 2I - P; out = diag(sc) X diag(sc) (n x n of X with leading dimension ldx);
// S[rc[2i]][rc[2i+1]] = val[i]; X <- alpha I
hipError_t launch_ns_residual(const double* P, int n, double* part, int blocks, hipStream_t s);
hipError_t launch_ns_two_minus(double* P, int n, hipStream_t s);
hipError_t launch_ns_scale(const double* X, int ldx, int n, const double* sc, double* out, hipStream_t s);
hipError_t launch_ns_scatter(double* S, int n, const int32_t* rc, const double* val, int64_t count, hipStream_t s);
hipError_t launch_ns_init(double* X, int n, double alpha, hipStream_t s);

// cell_active[c] = case_active[case_of_cell[c]]
hipError_t launch_expand_active(const int32_t* case_active, const int32_t* case_of_cell,
                                int64_t n_cells, int32_t* cell_active, hipStream_t s);

// ------------------------------------------------------------------ polar velocity grid (tube)
// Assembly of the fast-spectral operator on polar nodes v_j (stored th, v_z > 0 halves; the
// distribution is even in th and odd in v_z) from nm half-space Cartesian modes xi[3][nm]:
//   fhat[m] = sum_j wf[j] 4 cos(xi0 v1) cos(xi1 v2) cos(xi2 v3)     (f_eq, even-even fold)
//   X[i][m] = cos(xi_m . v_i)
//   Xc[i][2m], Xc[i][2m+1] = C[i][m] s[m] {cos, sin}(xi_m . v_i)
//   Op2[j][2m], Op2[j][2m+1] = 4 wp[j] {-sin a cos b sin c, cos a cos b sin c}  (odd-v_z fold,
//                             a, b, c = xi0 v1_j, xi1 v2_j, xi2 v3_j)
//   out[t][m] = mt[t][m] fhat[m] s[m]
hipError_t launch_polar_fhat(int nm, const double* xi, int nv, const double* vnode, const double* wf, double* fhat,
                             hipStream_t s);
hipError_t launch_polar_cos(int nv, int nm, const double* vnode, const double* xi, double* X, hipStream_t s);
hipError_t launch_polar_scale_terms(int Tp, int nm, const double* mt, const double* fhat, const double* sc,
                                    double* out, hipStream_t s);
// aT[i][t] = c[t] AB[i][src[t]] (src[t] >= 0), -feq[i] (src[t] == -1), 0 (src[t] == -2); nu[i] = AB[i][inu]
hipError_t launch_polar_coef(int nv, int Tp, const double* AB, const int32_t* src, const double* c,
                             const double* feq, int inu, double* aT, double* nu, hipStream_t s);
hipError_t launch_polar_xc(int nv, int nm, const double* vnode, const double* xi, const double* sc,
                           const double* C, double* Xc, hipStream_t s);
hipError_t launch_polar_op2(int nv, int nm, const double* vnode, const double* xi, const double* wp, double* Op2,
                            hipStream_t s);

// Tube (Sec. 4): radial nodes r of each case (r[last] = 1, the wall), velocities of the polar
// grid (n_vr x n_th x n_vz, v_z fastest).
struct TubeSweepArgs {
  int n_vr, n_th, n_vz, nv;
  int n_cases;
  const int64_t* node_off;   // [n_cases + 1]
  const double* r;           // [nodes]
  const double* cin;         // [nodes][3] inward (from larger r) coefficients of d/dr
  const double* cout;        // [nodes][3] outward coefficients (ghosts -r_1, -r_0 at the centre)
  const double* vr;          // [n_vr]
  const double* cth;         // [n_th] cos th
  const double* sth;         // [n_th] sin th
  double dth;
  const double* delta_case;
  const double* nu;          // [nv]
  const double* rhs;         // [nodes][nv]
  double* h;                 // [nodes][nv]
  const int32_t* case_active;
  int max_nodes;
};
hipError_t launch_sweep_tube(const TubeSweepArgs& a, hipStream_t s);
// mom[node][8] = {U3, q3, G = int v3 (2 v1^2 - 1) h, S2 = int 2 v3 (v1^2 - v2^2) h, P_rz = int 2 v1 v3 h, 0, 0, 0}
hipError_t launch_moments_tube(int64_t n_nodes, int nv, const double* vnode, const double* wnode, const double* h,
                               const int32_t* active, double* mom, hipStream_t s);
struct TubeDiffArgs {
  int n_cases;
  const int64_t* node_off;
  const double* r;
  const double* cin;         // inward coefficients (as in the sweep)
  const double* tw;          // [nodes] weights of 2 int_0^1 f r dr
  const double* delta_case;
  const int32_t* flow_case;
  const double* mom;         // [nodes][8]
  const double* amom;        // [nodes][4] or null
  double N;
  int sis;
  double cU, cq;
  double* U;
  double* dU;
  double* ufield;
  double* qfield;
  double* state;             // [n_cases][4] or null
  int32_t* iters;
  int32_t* case_active;
  double eps;
};
hipError_t launch_diffusion_tube(const TubeDiffArgs& a, hipStream_t s);

}  // namespace sis
