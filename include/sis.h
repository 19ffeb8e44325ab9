/*
 * sis.h -- C ABI of libsis.so: the per-iteration hot path of the synthetic
 * iterative scheme (SIS) for the steady linearized Boltzmann equation
 * (Wu, Zhang, Liu, Zhang & Reese, arXiv:1612.04488) on one AMD MI355X (gfx950).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * - Velocity space: a uniform cell-centred grid of n_v points per axis on
 *   [-l_v, l_v]^3 (Sec. 2; grid deferred by the paper to its FSM reference).
 *   A velocity distribution of one spatial cell is n3 = n_v^3 doubles in
 *   C order [v1][v2][v3] (v3 fastest).  Arrays over many cells are
 *   [cell][v1][v2][v3], cells contiguous; the cells of several cases are
 *   concatenated in case order.
 * - All array arguments of the compute calls are caller-owned DEVICE
 *   pointers (FP64 unless stated), borrowed for the duration of the call in
 *   stream order; the library never frees or retains them.  Descriptor
 *   structs are HOST memory and are copied during the call.
 * - Every call validates its arguments on the host before anything is
 *   enqueued and returns a negative sis_status on failure; the message is
 *   available from sis_last_error() on the calling thread.  Asynchronous
 *   device faults surface as SIS_E_DEVICE at the next synchronising call.
 *   No C++ exception crosses this interface.
 * - A plan is used by one stream at a time.  Compute calls are asynchronous
 *   with respect to the host unless stated.
 * - The collision operator is linear in the rarefaction parameter delta
 *   (eq. delta, Sec. 2.1): tables are built once for delta = 1 and every call
 *   takes delta per cell or per case.
 */
#ifndef SIS_H
#define SIS_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t sis_status;
enum {
  SIS_OK = 0,
  SIS_E_INVALID = -1,       /* bad argument value or null pointer             */
  SIS_E_SHAPE = -2,         /* inconsistent sizes                             */
  SIS_E_DEVICE = -3,        /* a HIP runtime call failed                      */
  SIS_E_OOM = -4,           /* device or host allocation failed               */
  SIS_E_NOT_CONVERGED = -5, /* sis_solve hit max_it; results are still filled */
  SIS_E_NUMERIC = -6,       /* NaN/Inf detected in a flow rate                */
  SIS_E_UNSUPPORTED = -7    /* valid request the library does not implement   */
};

/* Collision kernels: B = b0 |u|^alpha sin^(alpha+gamma-1)(theta/2) cos^-gamma(theta/2)
 * (sigma representation, deflection angle theta), b0 set by the first
 * Chapman-Enskog viscosity so that delta = p0 l / (mu v_m).                */
enum { SIS_KERNEL_HARD_SPHERE = 0, SIS_KERNEL_IPL = 1 };
/* Arithmetic of the collision contraction (everything else is FP64).
 * BF16X3: both operands split into bf16 hi + lo, products hi*hi + hi*lo +
 * lo*hi, FP32 accumulation.  BF16: the hi*hi product alone (about 3 decimal
 * digits); meant for sis_solve with FP64 anchors (refresh_every), where the
 * low-precision contraction only acts on the change since the last anchor.
 * Measured worst cases against FP64 at eps = 1e-8: one gas on planar and duct
 * workloads ~1e-7 in the flow rates, the Sierpinski-carpet heat flux 2.8e-5
 * (above the 1e-5 bound of the mixed forms), so BF16 is outside every
 * mixed-precision accuracy claim; BF16X3 is the mixed form.  Two-species plans
 * reject BF16 (SIS_E_UNSUPPORTED: the species blocks deviate by ~1e-3).       */
enum { SIS_PREC_FP64 = 0, SIS_PREC_FP32 = 1, SIS_PREC_BF16X3 = 2, SIS_PREC_BF16 = 3 };
/* Source terms S of Sec. 2 with X_P = X_T = -1.                             */
enum { SIS_FLOW_NONE = 0, SIS_FLOW_POISEUILLE = 1, SIS_FLOW_TRANSPIRATION = 2 };
enum { SIS_SCHEME_CIS = 0, SIS_SCHEME_SIS = 1 };
enum { SIS_GEOM_PLANAR_HALF = 0, SIS_GEOM_DUCT_QUARTER = 1, SIS_GEOM_PERIODIC_2D = 2, SIS_GEOM_TUBE = 3 };
enum { SIS_GRID_CARTESIAN = 0, SIS_GRID_POLAR = 1 };
enum { SIS_DIFFUSION_CG = 0, SIS_DIFFUSION_INVERSE = 1 };

const char* sis_last_error(void);   /* thread-local; valid until the next call on this thread */
int32_t sis_version(void);          /* 100 * major + minor                                    */

/* ------------------------------------------------------------------ plans
 * A plan holds the velocity grid and the fast-spectral collision operator
 * of one gas, assembled on the device at creation.
 *
 * Operator (eq. LBE_collision, evaluated by the fast spectral method that
 * Sec. 2.4 cites; Carleman form): h is zero-extended to an n_pad^3 periodic
 * box, |x|,|y| truncated at r_trunc (0 -> 4 L_p/(3 + sqrt 2)), directions
 * e = (sin t cos p, sin t sin p, cos t) with (t, p) the m_angle-point
 * Gauss-Legendre nodes on [0, pi]^2, weight w_t w_p sin t.  With
 * phi_p(l) = phi(l.e_p), psi_p(l) = psi(|l - (l.e_p) e_p|) (Nyquist modes 0),
 *   L+(h) = Q+(f_eq,h) + Q+(h,f_eq) - f_eq F^-1[beta F h],
 *   Q+(g,h) = 4 b0 sum_p W_p F^-1[phi_p F g] F^-1[psi_p F h],
 *   nu_eq = F^-1[beta F f_eq],  beta = 4 b0 sum_p W_p phi_p psi_p,
 *   L(h) = L+(h) - nu_eq h.
 * The plan stores the n3 x n3 matrix of h -> L+(h) (delta = 1), assembled
 * from these spectral factors, and applies it as a dense contraction.       */
typedef struct sis_plan* sis_plan_t;

typedef struct {
  int32_t n_v;        /* velocity points per axis (even, 4..40)                        */
  double  l_v;        /* velocity half-width (> 0)                                     */
  int32_t n_pad;      /* padded DFT size per axis (even, >= n_v; 0 -> 2 n_v)           */
  int32_t m_angle;    /* Gauss points per angle; directions D = m_angle^2 (1..32)     */
  double  r_trunc;    /* truncation radius (0 -> 4 L_p / (3 + sqrt 2))                 */
  int32_t kernel;     /* SIS_KERNEL_*                                                  */
  double  visc_index; /* IPL viscosity index w: alpha = 2 (1 - w), gamma = 0           */
  int32_t n_threads;  /* host threads for table construction (0 -> hardware count)    */
  /* Binary gas mixture (Sec. 5), hard spheres only.  n_species = 0 or 1: one gas
   * (the fields below are ignored).  n_species = 2: species A, B with masses,
   * diameters (any common unit) and molar fractions chi (> 0, sum 1); velocities
   * in units of A's most probable speed; see "mixtures" below.                   */
  int32_t n_species;
  double  mass[2];
  double  diam[2];
  double  chi[2];
  int32_t m_rho;      /* Gauss nodes on [0, R] of the rho integral of unequal-mass pairs (0 -> 16) */
  /* Parity storage (0, 1, 2).  The discrete operator commutes with v3 -> -v3 and
   * v2 -> -v2 (symmetric grid and direction set), and the Poiseuille and
   * transpiration sources are odd in v3 and even in v2, so their iterates keep
   * that symmetry.  parity 1 stores only v3 > 0 (any geometry); parity 2 stores
   * v2 > 0 and v3 > 0 (planar only).  A distribution of one (cell, species) is
   * then n_vel = n_v * (parity 2 ? n_v/2 : n_v) * n_v/2 doubles, C order
   * [v1][v2][v3] over the stored nodes (the upper halves of the v2, v3 axes);
   * every compute call takes and returns that layout, and moments, flow rates
   * and projections are those of the full-grid distribution it represents.
   * The operator is the full one restricted to the class (4x / 16x fewer
   * entries).  Inputs outside the class are the caller's error.             */
  int32_t parity;
  /* Velocity grid.  SIS_GRID_CARTESIAN (0): n_v^3 nodes on [-l_v, l_v]^3 as above.
   * SIS_GRID_POLAR (1), for the tube (Sec. 4, one gas, hard spheres): at the
   * point (r, 0) of the cross section v = (v_r cos th, v_r sin th, v_z), th the
   * angle of the in-plane velocity from the radial direction; distributions are
   * even in th and odd in v_z, so the stored nodes are v_r = vr_max s^2 (s the
   * n_vr Gauss-Legendre nodes on [0, 1]), th the n_th midpoints on [0, pi] and
   * v_z the n_vz midpoints on [0, l_v]; a row is [v_r][th][v_z] (v_z fastest,
   * n_vel = n_vr n_th n_vz).  The collision operator is the fast spectral
   * method of the Cartesian grids on the modes pi l / l_pad of an n_pad^3 box
   * (l_pad = 0 -> 2 max(vr_max, l_v); n_pad = 0 -> 4 l_pad, a lattice spacing
   * of 1/2), its transforms taken between the polar nodes (weights
   * w_vr dth dv_z over all four mirror images) and those modes.  n_v, parity
   * and the mixture fields are ignored.                                      */
  int32_t grid;
  int32_t n_vr;
  double  vr_max;
  int32_t n_th;
  int32_t n_vz;
  double  l_pad;
} sis_velocity_desc;

typedef struct {
  int32_t n_v, n3, n_pad, m_angle, n_dir;
  double  l_v, dv, b0, r_trunc, nubar;   /* nubar = int nu_eq f_eq at delta = 1 (Sec. 2.5) */
  double  alpha, gamma;
  int64_t operator_bytes;                /* device bytes of the FP64 operator                */
  double  plan_seconds_host, plan_seconds_device;
  int32_t n_species;                     /* 1 or 2                                           */
  int32_t n_dof;                         /* n_species * n3: unknowns per spatial cell        */
  double  nubar_b;                       /* mixture: int nu_B f_B / chi_B (nubar is A's)     */
  double  viscosity_ratio;               /* mixture: mu_mix / mu_A (first Chapman-Enskog)    */
  double  flow_factor;                   /* mixture: sqrt(m / m_A), m = chi_A m_A + chi_B m_B */
  int32_t parity;                        /* 0, 1, 2 (see sis_velocity_desc)                  */
  int32_t n_vel;                         /* stored velocities per (cell, species)            */
} sis_plan_info;

/* Mixtures (n_species = 2).  Unknowns per spatial cell: h = (h_A, h_B),
 * stored [cell][species][n3] (n_dof = 2 n3 doubles per cell).  Operator
 * (eq. Boltzmann_lin; the mixture FSM the paper cites, in a Carleman form
 * for unequal masses with 2mu = 2 m_b/(m_a+m_b), kappa = (m_a-m_b)/(m_a+m_b)):
 *   L+_a = sum_b Q+_ab(f_a, h_b) + Q+_ab(h_a, f_b) - f_a F^-1[beta_ab F h_b],
 *   Q+_ab(g,h) = 4 b_ab sum_p W_p int_{-R}^{R} |rho| g(v + 2mu rho e_p) (psi_p h)(v - kappa rho e_p) drho,
 *   b_ab = b0 ((d_a + d_b)/(2 d_A))^2, beta_ab = 4 b_ab sum_p W_p phi_p psi_p,
 *   nu_a = sum_b F^-1[beta_ab F f_b],  f_a = chi_a (m_a/(pi m_A))^{3/2} e^{-m_a v^2/m_A};
 * the rho integral is phi_p in closed form for equal masses and an m_rho-point
 * Gauss-Legendre rule on [0, R] (mirrored) otherwise.  delta is normalised
 * with the mixture viscosity (first Chapman-Enskog, hard spheres) and the
 * mixture most probable speed: every table carries sqrt(m_A/m) mu_mix/mu_A.
 * Supported: planar and 2-D geometries (2-D: the velocity equations need the
 * precomputed inverse of every case), Poiseuille flow (SIS_FLOW_POISEUILLE or
 * NONE), no invariant projection.  Per-cell arrays of the compute calls
 * become per (cell, species) as stated at each call.                        */

/* Build the tables on the host (threads) and assemble the operator on the
 * current device with `stream`.  Synchronous.  Owns ~8 n_dof^2 bytes of
 * device memory plus tables.                                                 */
sis_status sis_plan_create(const sis_velocity_desc* desc, hipStream_t stream, sis_plan_t* out);
sis_status sis_plan_destroy(sis_plan_t plan);
sis_status sis_plan_query(sis_plan_t plan, sis_plan_info* out);

/* Copy plan tables to HOST arrays (any may be NULL):
 * v1d[n_v], feq[n_species][n3], nu[n_species][n3] (delta = 1),
 * op[n_dof*n_dof] (row-major, row = output (species, velocity); the L+ matrix
 * at delta = 1).  Synchronous.                                             */
sis_status sis_plan_tables(sis_plan_t plan, double* v1d, double* feq, double* nu, double* op);

/* Host-only table construction (no device needed): the delta = 1 collision
 * frequency nu_eq[n3], the equilibrium feq[n3], and optionally the
 * f_eq-fields A_p = F^-1[psi_p F f_eq], B_p = F^-1[phi_p F f_eq] on the n3
 * grid for every direction p ([n_dir][n3] each), as used by the assembly.
 * Arrays are HOST memory, any may be NULL.  Reports b0 and nubar.
 * Mixtures: feq and nu are [2][n3], nubar points to 2 doubles (A, B), A and
 * B must be NULL.                                                           */
sis_status sis_host_tables(const sis_velocity_desc* desc, double* feq, double* nu,
                           double* A, double* B, double* b0, double* nubar);

/* Select the arithmetic of the collision contraction for later sis_collide
 * / sis_solve calls on this plan (builds the low-precision operator copy on
 * first use; synchronous).                                                   */
sis_status sis_plan_set_precision(sis_plan_t plan, int32_t precision, hipStream_t stream);

/* ------------------------------------------------------------------ geometry
 * Device-resident spatial geometry for a batch of independent cases.  One
 * spatial cell per node (planar) or per fluid cell (2-D); cells of all cases
 * are concatenated in case order.  delta[c], flow[c] (SIS_FLOW_*) are per
 * case.  All arrays are HOST memory and are copied.
 *
 * SIS_GEOM_PLANAR_HALF (Sec. 2.4): case c is the half channel
 *   -1/2 <= x1 <= 0 with nodes x1[node_offset[c] .. node_offset[c+1])
 *   (strictly increasing, first -1/2 = diffuse wall, last 0 = specular
 *   symmetry plane, >= 2 nodes).
 * SIS_GEOM_DUCT_QUARTER (Sec. 2.4, 5.3): case c is the quarter of a
 *   rectangular duct, n1[c] x n2[c] cells with faces face1 (n1+1 values,
 *   from the wall to the symmetry plane x1 = 0) and face2 (n2+1 values),
 *   concatenated over cases; walls at the first faces, symmetry planes at
 *   the last.
 * SIS_GEOM_PERIODIC_2D (Sec. 3.2): periodic cell with faces face1/face2 and a
 *   staircase solid mask solid (n1*n2 bytes per case, i major, 1 = solid);
 *   solid faces reflect diffusely.
 * SIS_GEOM_TUBE (Sec. 4; plans with SIS_GRID_POLAR only): case c is the tube
 *   of unit radius, radial nodes x1[node_offset[c] .. node_offset[c+1])
 *   (strictly increasing from r > 0 to r = 1, the diffuse wall; >= 3 nodes);
 *   Poiseuille flow.  Moments have 8 entries per node.
 * 2-D cells are numbered per case in row-major (i, j) order over fluid
 * cells.  Sweep moments have 8 entries per cell in 2-D (4 planar): see
 * sis_geometry_moment_stride.                                               */
typedef struct {
  int32_t kind;                 /* SIS_GEOM_*                                   */
  int32_t n_cases;
  const int64_t* node_offset;   /* planar: [n_cases + 1], node_offset[0] = 0    */
  const double*  x1;            /* planar: [node_offset[n_cases]]               */
  const double*  delta;         /* [n_cases], >= 0                              */
  const int32_t* flow;          /* [n_cases]                                    */
  const int32_t* n1;            /* 2-D: [n_cases] cells along x1 (>= 2)         */
  const int32_t* n2;            /* 2-D: [n_cases] cells along x2 (>= 2)         */
  const double*  face1;         /* 2-D: concatenated faces, n1[c]+1 per case    */
  const double*  face2;         /* 2-D: concatenated faces, n2[c]+1 per case    */
  const uint8_t* solid;         /* 2-D: concatenated masks or NULL (no solids)  */
} sis_geometry_desc;
typedef struct sis_geom* sis_geom_t;

sis_status sis_geometry_create(sis_plan_t plan, const sis_geometry_desc* desc,
                               hipStream_t stream, sis_geom_t* out);
sis_status sis_geometry_destroy(sis_geom_t geom);
int64_t    sis_geometry_cells(sis_geom_t geom);
int32_t    sis_geometry_moment_stride(sis_geom_t geom);   /* 4 planar, 8 in 2-D; -1 if NULL */
/* Form of the 2-D transport sweep this geometry launches (diagnostic; the
 * results do not depend on it): 1 the row-blocked sweep (every case at most 128
 * cells along axis 2 and the distributions under 2 GiB: one velocity quadruple
 * per lane, columns split over up to 16 waves), else anti-diagonal wavefronts:
 * 2 pipelined (anti-diagonals of up to 192 cells), 3 plain.  -1 for planar and
 * tube geometries or NULL.                                                      */
int32_t    sis_geometry_sweep_form(sis_geom_t geom);

/* Solver of the 2-D velocity equation (sis_diffusion_correct; the operator
 * depends on the geometry only).  SIS_DIFFUSION_INVERSE (the default after
 * sis_geometry_create) precomputes, per case, the dense inverse of the
 * finite-volume operator on the case's unknown cells by Newton-Schulz
 * iteration on the GPU (FP64 contractions, about log2(condition) + 5 steps,
 * each 4 nu^3 flops), so that every outer iteration applies it as one
 * matrix-vector product (nu^2 doubles read).  Cases with the same cross
 * section (same faces and solids) share one inverse, which one product per
 * iteration applies to all of them (up to 8 per read).  It holds nu^2 doubles
 * per distinct cross section (at most 16 GiB per geometry, nu <= 16384);
 * cases beyond that, cases whose
 * fluid has a group of unknown cells that reaches no wall or solid (the
 * operator is singular there) and cases whose iteration does not reach a
 * Frobenius residual ||I - S X|| < 1e-8 use the conjugate-gradient solve.
 * SIS_DIFFUSION_CG frees the inverses and uses conjugate gradients for
 * every case.  Planar geometries ignore the call.  Synchronises stream.
 * sis_geometry_diffusion_info: number of cases on the inverse, number of
 * distinct inverses held, and the largest Frobenius residual of the
 * (Jacobi-scaled) inverses; all nullable.                                     */
sis_status sis_geometry_diffusion_solver(sis_geom_t geom, int32_t mode, hipStream_t stream);
sis_status sis_geometry_diffusion_info(sis_geom_t geom, int32_t* n_inverse, int32_t* n_distinct,
                                       double* residual);

/* ------------------------------------------------------------------ compute
 * sis_collide -- collision step of one outer iteration for n_cells cells
 * (eq. LBE_collision applied pointwise in space, eq. syn_LBE right side,
 * correction of eq. guided applied on load):
 *   h^k      = h + dU[c] * 2 v3 f_eq                (dU may be NULL: no correction)
 *   L+       = delta[c] * L+_1(h^k),   L = L+ - delta[c] nu_1 h^k
 *   rhs_out  = L+ + S(flow[c])                       [n_cells][n3]
 *   lh_out   = L                                     [n_cells][n3]  (nullable)
 *   amom_out = { 2 sum w v1 v3 L, 2 sum w v1 v3 h^k,
 *                2 sum w v2 v3 L, 2 sum w v2 v3 h^k }  [n_cells][4] (nullable)
 *   (so A1 = 2 int v1 v3 (L + N delta h) = amom[0] + N delta[c] amom[1]).
 * If project != 0 the minimum-norm invariant projection is applied to L
 * (and L+): L -= f_eq sum_i c_i psi_i, c = Gram^-1 m, m_i = sum w psi_i L,
 * psi in {1, v1, v2, v3, |v|^2}.
 * delta[n_cells] and flow[n_cells] (int32) are DEVICE arrays; flow may be NULL.
 * h and rhs_out must be 16-byte aligned (the contraction reads h in 16-byte
 * vectors; SIS_E_INVALID otherwise); lh_out may have any 8-byte alignment.
 * Arithmetic of the contraction per sis_plan_set_precision; rest FP64.
 * Mixtures: h, rhs_out, lh_out are [n_cells][2][n3], dU is [n_cells][2]
 * (correction h_a += dU_a 2 (m_a/m_A) v3 f_a; the correction of both species
 * enters L+ of each), amom_out is [n_cells][2][4]; S_a = v3 f_a for
 * Poiseuille, 0 otherwise; project must be 0.                               */
sis_status sis_collide(sis_plan_t plan, int64_t n_cells, const double* h, const double* dU,
                       const double* delta, const int32_t* flow, int32_t project,
                       double* rhs_out, double* lh_out, double* amom_out, hipStream_t stream);

/* sis_collide_noalloc -- for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the collision step of sis_collide (same arguments, layouts, outputs and
 * errors) that calls no hipMalloc, hipFree or allocating routine.  Its workspace
 * (the low-precision copy of h for FP32 / BF16X3 / BF16 plans, then the split-K
 * partial sums) is a fixed 64 MiB device array inside the library, one per GPU,
 * held until the process ends.  It runs the plan's contraction configuration for
 * this n_cells and precision (tuned by an earlier sis_collide, else the default
 * heuristic; it never tunes), with the split-K count lowered until the partials
 * fit; a low-precision operand of more than 64 MiB (n_cells * n_dof * 4 bytes
 * for FP32; n_cells * Kp * 4 bytes for BF16X3 / BF16, Kp = n_dof rounded up to
 * 64) is rejected with SIS_E_SHAPE before anything is enqueued.  Every call on a GPU
 * shares that GPU's array: calls that overlap on one GPU (other streams, other
 * threads, other plans) race and must be ordered by the caller.              */
sis_status sis_collide_noalloc(sis_plan_t plan, int64_t n_cells, const double* h, const double* dU,
                               const double* delta, const int32_t* flow, int32_t project,
                               double* rhs_out, double* lh_out, double* amom_out, hipStream_t stream);

/* sis_collide_fsm -- the same collision step as sis_collide (same arguments,
 * layouts, outputs and errors), with L+ evaluated per cell by the fast spectral
 * method's transforms instead of the assembled operator (eq. LBE_collision with
 * the FSM the paper cites in Sec. 2.4; the Carleman form of the plan comment):
 * per cell the pruned forward DFT of h^k onto the n_pad^3 modes (half spectrum,
 * Nyquist modes dropped), then for each of the 2D + 1 terms (psi_p and phi_p of
 * every direction, and the loss multiplier beta) the product with the term's
 * multiplier, the pruned inverse DFT back to the stored velocities and the
 * product with the term's f_eq field (4 b0 W_p F^-1[phi_p F f_eq],
 * 4 b0 W_p F^-1[psi_p F f_eq], -f_eq), summed over the terms.  Every DFT is
 * separable and runs as small complex GEMMs on the FP64 MFMA with LDS-staged
 * operands; FP64 regardless of sis_plan_set_precision.  One-gas Cartesian plans
 * only (SIS_E_UNSUPPORTED otherwise, and for grids whose per-cell outputs exceed
 * 64 x 16 x 16 stored velocities, e.g. n_v = 24 without parity storage).  The
 * first call evaluates the multipliers on the device (T n_pad/2 (n_pad - 1)^2
 * doubles, plan-owned) and allocates scratch (spectra and per-slab partial sums
 * of up to ~2 GiB of cells at a time): not capturable (SIS_E_UNSUPPORTED while
 * the stream is capturing).  Timed by sis_plan_timing like the contraction
 * (read with sis_plan_fsm_timing_read: whole calls).                           */
sis_status sis_collide_fsm(sis_plan_t plan, int64_t n_cells, const double* h, const double* dU,
                           const double* delta, const int32_t* flow, int32_t project,
                           double* rhs_out, double* lh_out, double* amom_out, hipStream_t stream);
/* Executed flops of one cell update of sis_collide_fsm (every MFMA issued,
 * padding included), its l1-slab width (modes per workgroup of the inverse
 * transforms) and the device bytes of its tables; all nullable.             */
sis_status sis_plan_fsm_info(sis_plan_t plan, double* flops_per_cell, int32_t* slab_l1, int64_t* table_bytes);
/* l1 modes per inverse-transform workgroup (1..8, with the workgroup's LDS
 * within 160 KiB; default: the widest up to 4 that fits).  Results do not
 * depend on it beyond rounding order.                                        */
sis_status sis_plan_set_fsm_slab(sis_plan_t plan, int32_t slab_l1);
/* Summed milliseconds and number of sis_collide_fsm calls timed since
 * sis_plan_timing enabled timing (synchronises).                              */
sis_status sis_plan_fsm_timing_read(sis_plan_t plan, double* ms, int64_t* calls);

/* sis_transport_sweep -- solve delta nu h + v . grad h = rhs per velocity
 * (eq. syn_LBE / eq. LBE_iteration) by second-order upwind differences.
 * Planar: first order at the first step from each boundary; v1 > 0: h = 0
 * at the wall, march to x1 = 0; v1 < 0: specular h(0, v1) = h(0, -v1), march
 * to the wall.  mom_out (nullable): [cells][4] = { U3, q3, G1 = F_201/4, P13 }.
 * 2-D: quadrants (+,+), (-,+), (+,-), (-,-); two upwind points per axis
 * (first order when a wall/solid face is the only one; the face carries
 * h = 0), mirror ghosts at symmetry planes.  PERIODIC_2D reads the values
 * across a periodic edge from h_half_out on entry (the previous iterate), so
 * h_half_out is in/out there.  mom_out: [cells][8] =
 * { U3, q3, G1, G12 = F_111/4, G2 = F_021/4, P13, P23, 0 }.
 * rhs, h_half_out: [cells][n3]; moments are midpoint sums with weight dv^3.
 * Mixtures: each species is swept with its own nu_a; rhs, h_half_out
 * [cells][2][n3]; planar mom_out [cells][2][4] = { int v3 h_a, q_a =
 * int (m_a v^2/m_A - 5/2) v3 h_a, G1, P_a13 = 2 (m_a/m_A) int v1 v3 h_a };
 * 2-D mom_out [cells][2][8] = { U3, q_a, G1, G12, G2, P_a13, P_a23, 0 } with
 * the same mass factor in q_a and P_a13, P_a23 = 2 (m_a/m_A) int v2 v3 h_a.    */
sis_status sis_transport_sweep(sis_plan_t plan, sis_geom_t geom, const double* rhs,
                               double* h_half_out, double* mom_out, hipStream_t stream);

/* sis_moments -- macroscopic moments of the perturbation h (midpoint sums with
 * the velocity weight, over the full grid h represents):
 *   U3 = int v3 h (the velocity of Sec. 2), q3 = int (|v|^2 - 5/2) v3 h (the heat
 *   flux of Sec. 2), G1 = int v3 (2 v1^2 - 1) h = F_201 / 4 (the Hermite moment
 *   of Sec. 2.1 that eqs. diffusion_LBE and first_order carry), P13 = 2 int v1 v3 h
 *   (the shear stress of Sec. 2.1);
 * h[n_cells][n_vel] -> mom_out[n_cells][4] = { U3, q3, G1, P13 }.  Mixtures
 * (Sec. 5): h[n_cells][2][n_vel] -> mom_out[n_cells][2][4] with the mass
 * factors of the sweep's moments.  Errors: SIS_E_INVALID for NULL pointers or
 * n_cells < 0; nothing is enqueued then.                                       */
sis_status sis_moments(sis_plan_t plan, int64_t n_cells, const double* h, double* mom_out,
                       hipStream_t stream);

/* sis_diffusion_correct -- the SIS velocity equation.
 * 2-D (eq. diffusion_LBE with N): lap U = -N delta [Poiseuille]
 *   - (d11 G1 + 2 d12 G12 + d22 G2) + d1 A1 + d2 A2 in finite-volume form,
 *   U = U3(h_half) on fluid cells next to a wall or solid, solved with the
 *   precomputed inverse or by Jacobi-preconditioned conjugate gradients to a
 *   relative residual 1e-13 (sis_geometry_diffusion_solver);
 *   mom_half [cells][8], amom [cells][4] (A2 = amom[2] + N delta amom[3]).
 * Planar form (eq. first_order with the tuning parameter N, Sec. 2.5):
 *   d(U + G1)/dx1 = -N delta x1 [Poiseuille] + A1,   A1 = amom[0] + N delta amom[1],
 * marched from the wall with the upwind stencil (first order at the first
 * step), U at the wall = U3 of h_half.  mom_half: [cells][4] from the sweep;
 * amom: [cells][4] from sis_collide (NULL -> A1 = 0).  N <= 0 -> nubar.
 * Outputs U_out[cells] and dU_out[cells] = U - U3(h_half) (the correction
 * amplitude of eq. guided), both nullable.
 * Mixtures (eqs. LBE2_true2, LBE2_true1 integrated once from the symmetry
 * plane, same march; U_a = int v3 h_a / chi_a):
 *   chi_B d(U_B)/dx1 + d(G1_B)/dx1 = -N_B delta (m_A/m_B) P_B13 + A_B,
 *   chi_A d(U_A)/dx1 + d(G1_A)/dx1 = -N_A delta (x1 - P_B13) + A_A,
 * A_a = amom[c][a][0] + N_a delta amom[c][a][1], P_B13 from mom_half;
 * N <= 0 -> N_a = int nu_a f_a / chi_a, else N_A = N_B = N.  mom_half,
 * amom [cells][2][4]; U_out, dU_out [cells][2].
 * 2-D mixtures (eqs. LBE2_true2, LBE2_true1 as printed, one Poisson problem
 * per species on the single-gas finite-volume operator and its inverse):
 *   chi_B lap U_B = -N_B delta (m_A/m_B) div P_B - (d11 G1_B + 2 d12 G12_B + d22 G2_B) + d1 A1_B + d2 A2_B,
 *   chi_A lap U_A = N_A delta (div P_B - 1) - (d11 G1_A + ...) + d1 A1_A + d2 A2_A,
 * div P_B = d1 P_B13 + d2 P_B23 (central differences) of mom_half,
 * A2_a = amom[c][a][2] + N_a delta amom[c][a][3]; U_a = U3_a / chi_a next to
 * a wall or solid.  mom_half [cells][2][8], amom [cells][2][4].              */
sis_status sis_diffusion_correct(sis_plan_t plan, sis_geom_t geom, const double* mom_half,
                                 const double* amom, double N, double* U_out, double* dU_out,
                                 hipStream_t stream);

/* ------------------------------------------------------------------ solver
 * sis_solve -- CIS (the conventional iteration, eq. LBE_iteration of Sec. 2.2)
 * or SIS (eq. syn_LBE of Sec. 2.2 followed by the velocity equation and the
 * correction of eq. guided, with the tuning parameter N of Sec. 2.5) outer
 * iterations from h = 0 for every case of a geometry until the relative change
 * of both flow rates M = 2 int U3 dx1 and Q = 2 int q3 dx1 (the flow rates of
 * Sec. 2) between consecutive iterations is below eps (per case; the stop rule
 * of Sec. 2.4, which uses eps = 1e-10), or max_it.  One iteration = sis_collide + sis_transport_sweep (+
 * sis_diffusion_correct for SIS) + flow rates, launched as a captured HIP
 * graph.  Converged cases are frozen while the others continue.  Results are
 * copied to HOST arrays (each nullable).  Synchronous.  2-D: M = (1/A) sum U3 dA
 * over the fluid cells, A the whole cross-section (solids included).        */
typedef struct {
  int32_t scheme;        /* SIS_SCHEME_*                                   */
  double  N;             /* penalty parameter; <= 0 -> nubar (Sec. 2.5)    */
  double  eps;           /* convergence criterion (>= 0; 0 runs exactly max_it iterations) */
  int32_t max_it;        /* >= 1                                           */
  int32_t project;       /* invariant projection of L in sis_collide       */
  int32_t check_every;   /* host convergence poll period (0 -> 4)          */
  int32_t use_graph;     /* capture one iteration in a HIP graph (0/1)     */
  int32_t refresh_every; /* with a low-precision contraction (FP32/BF16X3/
                            BF16): iterations 0 (h = 0) and R/2, 3R/2, ... for
                            R = refresh_every apply the operator in FP64 and
                            store the anchor (x_a, L+ x_a); the others apply
                            the low-precision operator to x - x_a only:
                            L+ x ~ L+ x_a + L~+ (x - x_a).  0 -> 16; 1 -> every
                            iteration FP64; < 0 -> no anchors (plain
                            low-precision contraction every iteration).
                            Ignored in FP64.                                 */
  int32_t persistent;    /* 0: each iteration as launched kernels (a graph
                            with use_graph).  1: the check_every iterations
                            between polls as ONE cooperative launch whose
                            workgroups stay resident and separate the steps
                            of the iteration (contraction, finish, sweep,
                            moments, velocity equation and stop rule) by
                            grid barriers -- for small batches, where each
                            launched step is a few microseconds of work.
                            > 1: the same with that many workgroups (capped
                            at the co-resident limit; default at most 64).
                            Meant for small batches: its contraction runs
                            on 32 x 128 tiles over those workgroups only.
                            Planar one-gas plans with the FP64 contraction
                            only; any other solve returns
                            SIS_E_UNSUPPORTED at creation.
                            Results match the launched path to rounding
                            (the contraction's split-K slicing differs).
                            A barrier wait that runs out ends the launch
                            early and the next poll returns SIS_E_DEVICE. */
} sis_solve_opts;

/* Mixtures: M, Q are [n_cases][2] (M_a = sqrt(m/m_A) 2 int U_a dx1, Q_a
 * likewise with q_a; 2-D: sqrt(m/m_A) (1/A) sum U_a dA; all four must meet
 * eps), U, q are [cells][2].                                                */
typedef struct {
  double*  M;            /* [n_cases] mass flow rate                                   */
  double*  Q;            /* [n_cases] heat flow rate                                   */
  int32_t* iters;        /* [n_cases] iterations until the criterion held (or max_it) */
  double*  residual;     /* [n_cases] last relative change                            */
  double*  U;            /* [cells] U3 of the final iterate                           */
  double*  q;            /* [cells] q3 of the final iterate                           */
  double   seconds;      /* wall time of the iteration loop (excl. setup)             */
  int32_t  total_iters;  /* outer iterations launched                                 */
} sis_solve_result;

sis_status sis_solve(sis_plan_t plan, sis_geom_t geom, const sis_solve_opts* opts,
                     sis_solve_result* result, hipStream_t stream);

/* Persistent iteration state (what sis_solve runs on): device buffers for
 * h^{k+1/2}, the right side, moments, the pending correction dU and the
 * per-case flow rates / convergence flags, plus the captured graph of one
 * iteration.  Created with h = 0.  Owns ~2 cells*n3*8 bytes.
 * sis_state_step enqueues n_iters iterations on `stream` (asynchronous);
 * converged cases are frozen by the kernels themselves.
 * sis_state_poll synchronises `stream` and returns the number of cases still
 * iterating.  sis_state_results synchronises and fills `result` (seconds =
 * 0, total_iters = iterations enqueued since create/reset).                 */
typedef struct sis_state* sis_state_t;
sis_status sis_state_create(sis_plan_t plan, sis_geom_t geom, const sis_solve_opts* opts,
                            hipStream_t stream, sis_state_t* out);
sis_status sis_state_reset(sis_state_t state, hipStream_t stream);
sis_status sis_state_step(sis_state_t state, int32_t n_iters, hipStream_t stream);
sis_status sis_state_poll(sis_state_t state, int32_t* n_active, hipStream_t stream);
sis_status sis_state_results(sis_state_t state, sis_solve_result* result, hipStream_t stream);
sis_status sis_state_destroy(sis_state_t state);

/* Contraction configuration used for n_cells cells in `precision`: the
 * autotuner (run on the first eager sis_collide of a shape and at
 * sis_state_create, outside stream capture) times every (tile, split-K)
 * candidate on the device (per launch), adds the finish step's cost of
 * reading each split-K partial beyond the first (M x N x 8 bytes at 4 TB/s)
 * and, for the bf16 tiles that read the pair layout, the measured split of
 * the cell operand into it, and keeps,
 * among those within 1% of the fastest, the fewest split-K partials, then
 * the taller tile; tile_rows is the
 * cell-tile height (128, 64 or 32, the operator tile 128; or 256 for the
 * BF16X3 256 x 256 tile), k_stage the k-depth of its LDS stages (FP64 and
 * FP32: 16, or 32 for the FP64 single-buffered variants; BF16X3 and BF16:
 * 64, or 32 for the 256 x 256 tile; nullable), tuned = 0 if the default
 * heuristic is in use.                                                      */
sis_status sis_plan_contraction_config(sis_plan_t plan, int64_t n_cells, int32_t precision,
                                       int32_t* tile_rows, int32_t* splits, int32_t* tuned,
                                       int32_t* k_stage);
/* Fix the configuration for n_cells cells in `precision` instead of tuning it
 * (reproducible runs, tests): tile_rows 128, 64 or 32 with k_stage 16
 * (FP64, FP32) or 64 (BF16X3, BF16), or (FP64 only) 128 or 64 with k_stage
 * 32, or (BF16X3 only) 256 with k_stage 32 (256 cells x 256 operator rows
 * per tile; SIS_E_UNSUPPORTED when a bf16 pair array of the cells or of the
 * operator would reach 4 GiB); splits in 1..32.  Invalid combinations return
 * SIS_E_INVALID.  At equal splits every BF16X3 tile gives bit-identical
 * results.                                                                  */
sis_status sis_plan_set_contraction_config(sis_plan_t plan, int64_t n_cells, int32_t precision,
                                           int32_t tile_rows, int32_t k_stage, int32_t splits);

/* Kernel timing of the collision contraction: while enabled, every eager
 * (non-graph) contraction launch on a plan is bracketed by HIP events on its
 * stream; sis_plan_timing_read synchronises and returns the summed
 * milliseconds and the number of launches since enabling.                   */
sis_status sis_plan_timing(sis_plan_t plan, int32_t enable);
sis_status sis_plan_timing_read(sis_plan_t plan, double* gemm_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif
#endif /* SIS_H */
