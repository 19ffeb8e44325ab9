// C ABI of libsis.so (declarations and contracts in include/sis.h).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <utility>
#include <vector>

#include "fsm.h"
#include "geom2d.h"
#include "kernels.h"
#include "mixture.h"
#include "polar.h"
#include "planner.h"
#include "sis.h"

namespace {

thread_local std::string g_err;

sis_status fail(sis_status code, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return code;
}

#define HIP_TRY(expr)                                                                     \
  do {                                                                                    \
    hipError_t e_ = (expr);                                                               \
    if (e_ != hipSuccess)                                                                 \
      return fail(e_ == hipErrorOutOfMemory ? SIS_E_OOM : SIS_E_DEVICE, "%s: %s (%s:%d)", \
                  #expr, hipGetErrorString(e_), __FILE__, __LINE__);                      \
  } while (0)

template <class T>
hipError_t dmalloc(T** p, size_t count) {
  return hipMalloc(reinterpret_cast<void**>(p), std::max<size_t>(count, 1) * sizeof(T));
}

template <class T>
hipError_t upload(T** dst, const std::vector<T>& src, hipStream_t s) {
  hipError_t e = dmalloc(dst, src.size());
  if (e != hipSuccess) return e;
  if (src.empty()) return hipSuccess;
  return hipMemcpyAsync(*dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, s);
}

// cos, sin of the exact phase pi q / P (q reduced mod 2P in integers).
void phase_q(long q, int P, double& c, double& sn) {
  const double kPi = 3.14159265358979323846;
  q %= 2L * P;
  if (q < 0) q += 2L * P;
  const double ang = kPi * static_cast<double>(q) / P;
  c = std::cos(ang);
  sn = std::sin(ang);
}

// Phase xi_l v_j of the centred DFT: v_j = (j + 1/2 - n/2) dv, xi_l = pi l / L_p, so
// xi_l v_j = pi l (2 j + 1 - n) / P.
void fsm_phase(int l, int j, int n, int P, double& c, double& sn) {
  phase_q(static_cast<long>(l) * (2 * j + 1 - n), P, c, sn);
}

void dfree(void* p) {
  if (p) (void)hipFree(p);
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

// Grow-only device scratch buffer.
struct Scratch {
  void* p = nullptr;
  size_t bytes = 0;
  hipError_t ensure(size_t need) {
    if (need <= bytes) return hipSuccess;
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    hipError_t e = hipMalloc(&p, need);
    if (e == hipSuccess) bytes = need;
    return e;
  }
  // give back what the largest tuning candidate needed beyond `keep` bytes
  hipError_t shrink(size_t keep) {
    if (bytes <= keep) return hipSuccess;
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
    return keep ? ensure(keep) : hipSuccess;
  }
  ~Scratch() { dfree(p); }
};

// Workspace of sis_collide_noalloc: a file-scope device array (one copy per GPU,
// held until the process ends), so that the call allocates nothing.  Host code
// never uses the array's name as an address: static_scratch() returns the device
// address from hipGetSymbolAddress, looked up once per device with that device
// current.
constexpr size_t kStaticScratchBytes = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

hipError_t static_scratch(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace

struct sis_plan {
  int device = 0;
  int n = 0, n3 = 0, np = 0, D = 0, m_angle = 0;
  double lv = 0, dv = 0, w = 0, b0 = 0, R = 0, nubar = 0, alpha = 1, gamma = 0;
  double host_s = 0, dev_s = 0;
  int precision = SIS_PREC_FP64;
  // species: 1 (one gas) or 2 (binary mixture); rows of the operator are (species, velocity)
  int nsp = 1, ndof = 0;
  // parity storage: 0 full grid; 1 odd in v3 (v3 > 0 stored); 2 odd in v3 and even in v2
  // (v2, v3 > 0 stored).  nv velocities per (cell, species) row on n x d2 x d3 nodes; wr is
  // the quadrature weight of a stored velocity times its number of mirror images.
  int parity = 0, d2 = 0, d3 = 0, nv = 0;
  double wr = 0.0;
  double mass_ratio[2] = {1.0, 1.0}, chi[2] = {1.0, 0.0}, nubar_s[2] = {0.0, 0.0};
  double cU_s[2] = {0.0, 0.0}, cq_s[2] = {0.0, 0.0};
  double flow_factor = 1.0, visc_ratio = 1.0;
  double* op = nullptr;         // [ndof][ndof] L+ at delta = 1
  float* op32 = nullptr;
  uint16_t* opp = nullptr;   // the operator in the bf16 pair layout (ndof rows)
  double* v1d = nullptr;        // [n]
  double* feq = nullptr;        // [nsp][n3]
  double* nu = nullptr;         // [nsp][n3]
  double* Kc = nullptr;         // [nsp][ndof] L+ of the correction shape of each species
  double* gram_inv = nullptr;   // [25]
  // polar velocity grid (tube flows): per-node velocity components [3][nv], weights [nv]
  // (both mirror images in th and v_z included), axis tables for the sweep
  bool polar = false;
  int n_vr = 0, n_th = 0, n_vz = 0;
  double dth = 0.0;
  double *vnode = nullptr, *wnode = nullptr, *d_vr = nullptr, *d_cth = nullptr, *d_sth = nullptr;
  // every grid: v1, v2, v3 [3][nv] and quadrature weight [nv] of each stored velocity
  double *vtab = nullptr, *wtab = nullptr;
  double cU = 0, cq = 0;        // U3, q3 of 2 v3 feq
  std::vector<double> h_v1d, h_feq, h_nu;
  // scratch of eager compute calls (a solver state owns its own, fixed at creation,
  // so that the buffers its captured graphs use are never reallocated)
  Scratch ws_acc, ws_x;  // split-K partials, low-precision cell operand
  bool timing = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> events;
  // per-cell transform path (sis_collide_fsm; one gas, Cartesian grid): factor matrices and
  // f_eq fields [T][nv] from plan creation, multipliers and L+ of the correction shape on
  // first use
  bool fsm_ok = false, fsm_ready = false;
  sis::FsmDims fsm_d{};
  sis::FsmFactors fsm_f{};
  int fsm_slab = 0;
  double* fsm_fac = nullptr;    // the 12 planar factor arrays
  double* fsm_field = nullptr;  // [T][nv]
  double* fsm_mult = nullptr;   // [T][Q][L][L]
  double* fsm_Kc = nullptr;     // [nv]
  double* fsm_dirs = nullptr;   // [D][3], then W [D]
  double* fsm_rad = nullptr;    // radial nodes and weights
  sis::RadialRule fsm_rule;
  std::vector<double> fsm_corr; // correction shape 2 v3 f_eq (stored layout)
  Scratch fsm_S, fsm_acc;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> fsm_events;
  // tuned contraction configuration per (cells, precision): tile id, split-K
  std::map<std::pair<int64_t, int>, std::pair<int, int>> gemm_choice;
  ~sis_plan() {
    for (auto& e : events) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
    for (auto& e : fsm_events) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
    dfree(fsm_fac); dfree(fsm_field); dfree(fsm_mult); dfree(fsm_Kc); dfree(fsm_dirs); dfree(fsm_rad);
    dfree(op); dfree(op32); dfree(opp);
    dfree(v1d); dfree(feq); dfree(nu); dfree(Kc); dfree(gram_inv);
    dfree(vnode); dfree(wnode); dfree(d_vr); dfree(d_cth); dfree(d_sth); dfree(vtab); dfree(wtab);
  }
};

struct sis_geom {
  sis_plan* plan = nullptr;
  int kind = 0, n_cases = 0, max_nodes = 0;
  int64_t n_cells = 0;
  std::vector<int64_t> h_off;
  std::vector<double> h_x, h_delta;
  std::vector<int32_t> h_flow;
  int64_t* off = nullptr;
  double* x = nullptr;
  double* coef = nullptr;        // [cells][6]
  double* delta_case = nullptr;
  int32_t* flow_case = nullptr;
  double* delta_cell = nullptr;
  int32_t* flow_cell = nullptr;
  int32_t* case_of_cell = nullptr;
  // 2-D tables (kinds DUCT_QUARTER, PERIODIC_2D)
  bool two_d = false;
  bool tube = false;             // SIS_GEOM_TUBE: radial nodes, polar velocity grid
  int max_diag = 0;              // 2-D: largest min(n1, n2) over the cases
  int max_n2 = 0;                // 2-D: largest n2 over the cases
  bool no_mirror = false;        // 2-D: no stencil reference is a mirror ghost
  double *d_r = nullptr, *d_cin = nullptr, *d_cout = nullptr, *d_tw = nullptr;
  sis::Tables2D t2;
  int32_t *d_n1 = nullptr, *d_n2 = nullptr, *d_gcell = nullptr, *d_sref = nullptr, *d_nb = nullptr;
  uint32_t* d_srec = nullptr;    // packed stencil records of the look-ahead sweep
  uint32_t* d_grec = nullptr;    // the same in grid order, for the row-blocked sweep
  uint32_t* d_growb = nullptr;   // [grid + 1] byte offset of the cell's first row in h, or ~0 (solid)
  int64_t* d_goff = nullptr;
  int8_t *d_skind = nullptr, *d_dflag = nullptr, *d_nbm = nullptr;
  double *d_scoef = nullptr, *d_npos = nullptr, *d_fw = nullptr, *d_width = nullptr, *d_cpos = nullptr,
         *d_dA = nullptr, *d_area = nullptr;
  double* work = nullptr;        // [grid][10] diffusion workspace
  int32_t* have_x = nullptr;     // [n_cases]
  int32_t* cg_iters = nullptr;   // [n_cases]
  // 2-D velocity equation by a precomputed inverse (cases with h_direct[c] != 0)
  std::vector<int32_t> h_direct;
  int32_t *d_direct = nullptr, *d_uidx = nullptr, *d_nunk = nullptr;
  int32_t *d_grp_n = nullptr, *d_grp_size = nullptr;
  int64_t *d_uoff = nullptr, *d_grp_aoff = nullptr, *d_grp_vec = nullptr;
  double *ainv = nullptr, *bvec = nullptr, *yvec = nullptr;
  int max_unknown = 0, n_direct = 0, n_groups = 0, n_inverses = 0;
  double inv_residual = 0.0;     // largest ||I - X S||_F of the scaled inverses
  void free_inverse() {
    dfree(d_direct); dfree(d_uidx); dfree(d_nunk); dfree(d_uoff);
    dfree(d_grp_aoff); dfree(d_grp_n); dfree(d_grp_size); dfree(d_grp_vec);
    dfree(ainv); dfree(bvec); dfree(yvec);
    d_direct = d_uidx = d_nunk = d_grp_n = d_grp_size = nullptr;
    d_uoff = d_grp_aoff = d_grp_vec = nullptr;
    ainv = bvec = yvec = nullptr;
    h_direct.clear();
    max_unknown = n_direct = n_groups = n_inverses = 0;
    inv_residual = 0.0;
  }
  int mom_stride() const { return (two_d || tube) ? 8 : 4; }
  ~sis_geom() {
    free_inverse();
    dfree(d_r); dfree(d_cin); dfree(d_cout); dfree(d_tw);
    dfree(off); dfree(x); dfree(coef); dfree(delta_case); dfree(flow_case);
    dfree(delta_cell); dfree(flow_cell); dfree(case_of_cell);
    dfree(d_n1); dfree(d_n2); dfree(d_gcell); dfree(d_sref); dfree(d_nb); dfree(d_goff); dfree(d_srec); dfree(d_grec); dfree(d_growb);
    dfree(d_skind); dfree(d_dflag); dfree(d_nbm); dfree(d_scoef); dfree(d_npos); dfree(d_fw);
    dfree(d_width); dfree(d_cpos); dfree(d_dA); dfree(d_area); dfree(work); dfree(have_x); dfree(cg_iters);
  }
};

namespace {

bool invert5(const double* a, double* inv) {
  double m[5][10];
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j < 10; ++j) m[i][j] = j < 5 ? a[i * 5 + j] : (j - 5 == i ? 1.0 : 0.0);
  for (int c = 0; c < 5; ++c) {
    int piv = c;
    for (int r = c + 1; r < 5; ++r)
      if (std::fabs(m[r][c]) > std::fabs(m[piv][c])) piv = r;
    if (m[piv][c] == 0.0) return false;
    if (piv != c)
      for (int j = 0; j < 10; ++j) std::swap(m[c][j], m[piv][j]);
    const double d = m[c][c];
    for (int j = 0; j < 10; ++j) m[c][j] /= d;
    for (int r = 0; r < 5; ++r)
      if (r != c) {
        const double f = m[r][c];
        for (int j = 0; j < 10; ++j) m[r][j] -= f * m[c][j];
      }
  }
  for (int i = 0; i < 5; ++i)
    for (int j = 0; j < 5; ++j) inv[i * 5 + j] = m[i][j + 5];
  return true;
}

sis_status validate_desc(const sis_velocity_desc* d) {
  if (!d) return fail(SIS_E_INVALID, "null velocity descriptor");
  if (d->grid != SIS_GRID_CARTESIAN && d->grid != SIS_GRID_POLAR) return fail(SIS_E_INVALID, "unknown velocity grid %d", d->grid);
  if (d->grid == SIS_GRID_POLAR) {
    if (d->kernel != SIS_KERNEL_HARD_SPHERE) return fail(SIS_E_UNSUPPORTED, "the polar grid supports hard spheres only");
    if (d->n_species == 2) return fail(SIS_E_UNSUPPORTED, "the polar grid supports one gas only");
    if (d->m_angle < 1 || d->m_angle > 32) return fail(SIS_E_INVALID, "m_angle must be in [1, 32]");
    if (!(d->l_v > 0.0) || !std::isfinite(d->l_v) || !(d->vr_max > 0.0) || !std::isfinite(d->vr_max))
      return fail(SIS_E_INVALID, "l_v and vr_max must be positive");
    if (d->l_pad < 0.0 || d->n_pad < 0) return fail(SIS_E_INVALID, "l_pad and n_pad must be >= 0");
    return SIS_OK;
  }
  if (d->n_v < 4 || d->n_v > 40 || d->n_v % 2) return fail(SIS_E_INVALID, "n_v must be even in [4, 40] (got %d)", d->n_v);
  if (!(d->l_v > 0.0) || !std::isfinite(d->l_v)) return fail(SIS_E_INVALID, "l_v must be positive");
  const int np = d->n_pad > 0 ? d->n_pad : 2 * d->n_v;
  if (np < d->n_v || np % 2 || np > 128) return fail(SIS_E_INVALID, "n_pad must be even, >= n_v and <= 128 (got %d)", np);
  if (d->m_angle < 1 || d->m_angle > 32) return fail(SIS_E_INVALID, "m_angle must be in [1, 32]");
  if (d->r_trunc < 0.0) return fail(SIS_E_INVALID, "r_trunc must be >= 0");
  if (d->kernel != SIS_KERNEL_HARD_SPHERE && d->kernel != SIS_KERNEL_IPL)
    return fail(SIS_E_UNSUPPORTED, "unknown collision kernel %d", d->kernel);
  if (d->kernel == SIS_KERNEL_IPL && !(d->visc_index >= 0.5 && d->visc_index <= 1.0))
    return fail(SIS_E_INVALID, "IPL viscosity index must be in [0.5, 1]");
  if (d->n_species < 0 || d->n_species > 2) return fail(SIS_E_UNSUPPORTED, "n_species must be 1 or 2");
  if (d->parity < 0 || d->parity > 2) return fail(SIS_E_INVALID, "parity must be 0, 1 or 2");
  if (d->n_species == 2) {
    if (d->kernel != SIS_KERNEL_HARD_SPHERE) return fail(SIS_E_UNSUPPORTED, "mixtures support hard spheres only");
    for (int s = 0; s < 2; ++s) {
      if (!(d->mass[s] > 0.0) || !std::isfinite(d->mass[s])) return fail(SIS_E_INVALID, "mass[%d] must be positive", s);
      if (!(d->diam[s] > 0.0) || !std::isfinite(d->diam[s])) return fail(SIS_E_INVALID, "diam[%d] must be positive", s);
      if (!(d->chi[s] > 0.0 && d->chi[s] < 1.0)) return fail(SIS_E_INVALID, "chi[%d] must be in (0, 1)", s);
    }
    if (std::fabs(d->chi[0] + d->chi[1] - 1.0) > 1e-12) return fail(SIS_E_INVALID, "chi must sum to 1");
    if (d->m_rho < 0 || d->m_rho > 64) return fail(SIS_E_INVALID, "m_rho must be in [0, 64]");
  }
  return SIS_OK;
}

sis::MixDesc mix_desc(const sis_velocity_desc* d) {
  sis::MixDesc m;
  m.n_v = d->n_v;
  m.l_v = d->l_v;
  m.n_pad = d->n_pad;
  m.m_angle = d->m_angle;
  m.m_rho = d->m_rho > 0 ? d->m_rho : 16;
  m.r_trunc = d->r_trunc;
  for (int s = 0; s < 2; ++s) {
    m.mass[s] = d->mass[s];
    m.diam[s] = d->diam[s];
    m.chi[s] = d->chi[s];
  }
  m.n_threads = d->n_threads;
  return m;
}

sis::TableDesc table_desc(const sis_velocity_desc* d) {
  sis::TableDesc t;
  t.n_v = d->n_v;
  t.l_v = d->l_v;
  t.n_pad = d->n_pad;
  t.m_angle = d->m_angle;
  t.r_trunc = d->r_trunc;
  t.alpha = d->kernel == SIS_KERNEL_IPL ? 2.0 * (1.0 - d->visc_index) : 1.0;
  t.gamma = 0.0;
  t.n_threads = d->n_threads;
  return t;
}

// Default tile and split-K for a contraction of M cells against the n3 x n3
// operator: enough workgroups (>= 1024) to fill the chip.
void choose_gemm(int64_t M, int n3, int* tile, int* splits) {
  *tile = M >= 256 ? 0 : 1;
  const int64_t bm = *tile == 0 ? 128 : 32;
  const int64_t blocks = ((n3 + 127) / 128) * ((M + bm - 1) / bm);
  int s = 1;
  while (blocks * s < 1024 && s < 16 && n3 / (s * 2) >= 256) s *= 2;
  *splits = s;
}

// Cell operand of a low-precision contraction (x = X - Xref rounded once per launch).
sis_status prepare_lowp_operand(sis_plan* p, int precision, int64_t n_cells, const double* h, const double* xref,
                                Scratch* ws_x, sis::GemmArgs& g, hipStream_t s) {
  if (precision == SIS_PREC_FP64) return SIS_OK;
  const int64_t cnt = n_cells * static_cast<int64_t>(p->ndof);
  if (precision == SIS_PREC_BF16X3 || precision == SIS_PREC_BF16) {
    // pair layout: 2 Kp bf16 per cell, 4 bytes per padded unknown
    HIP_TRY(ws_x->ensure(static_cast<size_t>(n_cells) * sis::pair_stride(p->ndof) * 4));
    uint16_t* hx = static_cast<uint16_t*>(ws_x->p);
    HIP_TRY(sis::launch_split_pairs(h, xref, n_cells, p->ndof, hx, precision == SIS_PREC_BF16X3, s));
    g.Xp = hx;
  } else {
    HIP_TRY(ws_x->ensure(static_cast<size_t>(cnt) * 4));
    float* fx = static_cast<float*>(ws_x->p);
    HIP_TRY(sis::launch_convert_x_f32(h, xref, cnt, fx, s));
    g.X32 = fx;
  }
  return SIS_OK;
}

// The 32-row BF16 tiles split the FP64 cell operand while staging it (no split_pairs launch):
// the few-cell shapes that pick them are bound by launch latency.
bool fused_split(int precision, int tile) {
  return (precision == SIS_PREC_BF16X3 || precision == SIS_PREC_BF16) && tile == 1;
}

// Autotuner of the contraction: times every (tile, split-K) candidate on the
// actual shape (two launches each after a warm-up, HIP events on `s`) and
// keeps, per (cells, precision), the candidate with the fewest split-K
// partials, then the tallest tile, among those within 1% of the fastest after
// charging each extra partial its read by the finish step (so that timing noise
// does not flip between near-equal configurations).  Not
// callable while `s` is capturing.  Candidates whose split-K partials would
// exceed 4 GiB are skipped.
sis_status tune_gemm(sis_plan* p, int64_t M, int precision, const double* h, Scratch* ws_acc, Scratch* ws_x,
                     hipStream_t s) {
  const auto key = std::make_pair(M, precision);
  if (p->gemm_choice.count(key)) return SIS_OK;
  sis::GemmArgs g{};
  g.precision = precision;
  g.X = h;
  g.op64 = p->op;
  g.op32 = p->op32;
  g.opp = p->opp;
  g.M = M;
  g.N = p->ndof;
  g.K = p->ndof;
  if (sis_status st = prepare_lowp_operand(p, precision, M, h, nullptr, ws_x, g, s)) return st;
  const uint16_t* xp_split = g.Xp;
  int dt, ds;
  choose_gemm(M, p->ndof, &dt, &ds);
  std::vector<std::pair<float, std::pair<int, int>>> timed;
  hipEvent_t e0, e1;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  // the split of the cell operand into the bf16 pair layout, per launch (two timed launches)
  const bool bf16 = precision == SIS_PREC_BF16X3 || precision == SIS_PREC_BF16;
  float split_ms = 0.f;
  if (bf16) {
    uint16_t* xp = const_cast<uint16_t*>(xp_split);
    hipError_t e = hipEventRecord(e0, s);
    for (int r = 0; r < 2 && e == hipSuccess; ++r)
      e = sis::launch_split_pairs(h, nullptr, M, p->ndof, xp, precision == SIS_PREC_BF16X3, s);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(&split_ms, e0, e1);
    if (e != hipSuccess) {
      (void)hipEventDestroy(e0);
      (void)hipEventDestroy(e1);
      return fail(SIS_E_DEVICE, "contraction tuning: %s", hipGetErrorString(e));
    }
    split_ms *= 0.5f;
  }
  // candidates: FP64 tiles 0, 2, 1, 3, 4; FP32 and BF16 tiles 0, 2, 1; BF16X3 tiles 0, 2, 1 and the
  // 256 x 256 tile 5 where its pair arrays take 32-bit offsets
  std::vector<int> tiles = {0, 2, 1};
  if (precision == SIS_PREC_FP64) tiles.insert(tiles.end(), {3, 4});
  if (precision == SIS_PREC_BF16X3 && sis::gemm_wide_fits(M, p->ndof, p->ndof)) tiles.push_back(5);
  // split-K up to 32 (at least 64 k values per split): few cells leave most CUs idle otherwise
  const int splits[10] = {1, 2, 3, 4, 6, 8, 12, 16, 24, 32};
  hipError_t err = hipSuccess;
  for (size_t ti = 0; ti < tiles.size() && err == hipSuccess; ++ti)
    for (int si = 0; si < 10 && err == hipSuccess; ++si) {
      const int sp = splits[si];
      if (sp > 1 && sis::gemm_k_per_split(p->ndof, sp) * (sp - 1) >= p->ndof) continue;   // an empty split
      if (sp > 1 && sis::gemm_k_per_split(p->ndof, sp) < 64) continue;
      const double bytes = static_cast<double>(sp) * M * p->ndof * 8.0;
      if (bytes > 4.0 * (1 << 30)) continue;
      err = ws_acc->ensure(static_cast<size_t>(bytes));
      if (err != hipSuccess) break;
      g.acc = static_cast<double*>(ws_acc->p);
      g.tile = tiles[ti];
      g.splits = sp;
      g.Xp = fused_split(precision, g.tile) ? nullptr : xp_split;
      err = sis::launch_gemm(g, s);
      if (err == hipSuccess) err = hipEventRecord(e0, s);
      for (int r = 0; r < 2 && err == hipSuccess; ++r) err = sis::launch_gemm(g, s);
      if (err == hipSuccess) err = hipEventRecord(e1, s);
      if (err == hipSuccess) err = hipEventSynchronize(e1);
      float ms = 0.f;
      if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
      // per launch; the bf16 tiles that read the pair layout also pay its split launch
      ms *= 0.5f;
      if (bf16 && !fused_split(precision, g.tile)) ms += split_ms;
      if (err == hipSuccess) timed.emplace_back(ms, std::make_pair(g.tile, sp));
    }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (err != hipSuccess) return fail(SIS_E_DEVICE, "contraction tuning: %s", hipGetErrorString(err));
  std::pair<int, int> best(dt, ds);
  if (!timed.empty()) {
    // each split-K partial beyond the first costs the finish step one more FP64 row read per
    // cell (M x N x 8 bytes at the ~4 TB/s that finish_kernel streams): add it to the timing
    for (auto& c : timed)
      c.first += static_cast<float>((c.second.second - 1) * static_cast<double>(M) * p->ndof * 8.0 / 4.0e12 * 1e3);
    float fastest = timed[0].first;
    for (const auto& c : timed) fastest = std::min(fastest, c.first);
    // within 1% of the fastest: fewest split-K partials, then the larger tile, then the faster
    int best_rows = -1, best_splits = 1 << 30;
    float best_ms = 0.f;
    for (const auto& c : timed) {
      if (c.first > 1.01f * fastest) continue;
      const int rows = sis::gemm_tile_rows(c.second.first), sp = c.second.second;
      if (sp < best_splits || (sp == best_splits && rows > best_rows) ||
          (sp == best_splits && rows == best_rows && c.first < best_ms)) {
        best_splits = sp;
        best_rows = rows;
        best_ms = c.first;
        best = c.second;
      }
    }
  }
  p->gemm_choice[key] = best;
  // the split-K partials of the kept configuration, not of the largest candidate
  const size_t keep = best.second > 1 ? static_cast<size_t>(best.second) * M * p->ndof * sizeof(double) : 0;
  if (ws_acc->shrink(keep) != hipSuccess) return fail(SIS_E_DEVICE, "contraction tuning: scratch reallocation failed");
  return SIS_OK;
}

// Arguments of finish_kernel for a contraction of n_cells cells (partial sums set by the caller).
sis::FinishArgs finish_args(const sis_plan* p, int64_t n_cells, const double* h, const double* dU,
                            const double* delta, const int32_t* flow, int project, double* rhs, double* lh,
                            double* amom, const int32_t* cell_active, int anchor_mode, double* xref,
                            double* accref) {
  sis::FinishArgs f{};
  f.n3 = p->nv;
  f.even_v2 = p->parity == 2;
  f.nsp = p->nsp;
  f.mass_ratio[0] = p->mass_ratio[0];
  f.mass_ratio[1] = p->mass_ratio[1];
  f.n_cells = n_cells * p->nsp;
  f.h = h;
  f.dU = dU;
  f.delta = delta;
  f.flow = flow;
  f.project = project;
  f.vtab = p->vtab;
  f.wtab = p->wtab;
  f.feq = p->feq;
  f.nu = p->nu;
  f.Kc = p->Kc;
  f.gram_inv = p->gram_inv;
  f.active = cell_active;
  f.anchor_mode = anchor_mode;
  f.accref = accref;
  f.xref = xref;
  f.rhs = rhs;
  f.lh = lh;
  f.amom = amom;
  return f;
}

sis_status run_collide(sis_plan* p, int64_t n_cells, const double* h, const double* dU,
                       const double* delta, const int32_t* flow, int project, double* rhs,
                       double* lh, double* amom, const int32_t* cell_active, hipStream_t s,
                       int precision = -1, int anchor_mode = 0, double* xref = nullptr,
                       double* accref = nullptr, Scratch* ws_acc = nullptr, Scratch* ws_x = nullptr,
                       bool h_is_zero = false) {
  if (h_is_zero) {
    // L+ h = 0 for h = 0: no contraction; finish_kernel sums no partials (the anchor, if one
    // is being taken, becomes (0, 0))
    sis::FinishArgs f = finish_args(p, n_cells, h, dU, delta, flow, project, rhs, lh, amom, cell_active,
                                    anchor_mode, xref, accref);
    f.splits = 0;
    f.acc = nullptr;
    HIP_TRY(sis::launch_finish(f, s));
    return SIS_OK;
  }
  if (!ws_acc) ws_acc = &p->ws_acc;
  if (!ws_x) ws_x = &p->ws_x;
  if (precision < 0) precision = p->precision;
  int tile, splits;
  const auto tuned = p->gemm_choice.find(std::make_pair(n_cells, precision));
  if (tuned != p->gemm_choice.end()) {
    tile = tuned->second.first;
    splits = tuned->second.second;
  } else {
    choose_gemm(n_cells, p->ndof, &tile, &splits);
  }
  double* acc = rhs;
  if (splits > 1) {
    HIP_TRY(ws_acc->ensure(static_cast<size_t>(splits) * n_cells * p->ndof * sizeof(double)));
    acc = static_cast<double*>(ws_acc->p);
  }
  sis::GemmArgs g{};
  g.precision = precision;
  g.X = h;
  g.Xref = anchor_mode == 2 ? xref : nullptr;
  if (fused_split(precision, tile))
    g.Xp = nullptr;   // the contraction splits h (minus the anchor) itself
  else if (sis_status st = prepare_lowp_operand(p, precision, n_cells, h, g.Xref, ws_x, g, s))
    return st;
  g.op64 = p->op;
  g.op32 = p->op32;
  g.opp = p->opp;
  g.acc = acc;
  g.M = n_cells;
  g.N = p->ndof;
  g.K = p->ndof;
  g.splits = splits;
  g.tile = tile;
  if (p->timing) {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(s, &cs));
    if (cs == hipStreamCaptureStatusNone) {
      hipEvent_t a, b;
      HIP_TRY(hipEventCreate(&a));
      HIP_TRY(hipEventCreate(&b));
      p->events.emplace_back(a, b);
      HIP_TRY(hipEventRecord(a, s));
      HIP_TRY(sis::launch_gemm(g, s));
      HIP_TRY(hipEventRecord(b, s));
    } else {
      HIP_TRY(sis::launch_gemm(g, s));
    }
  } else {
    HIP_TRY(sis::launch_gemm(g, s));
  }
  sis::FinishArgs f = finish_args(p, n_cells, h, dU, delta, flow, project, rhs, lh, amom, cell_active,
                                  anchor_mode, xref, accref);
  f.splits = splits;
  f.acc = acc;
  HIP_TRY(sis::launch_finish(f, s));
  return SIS_OK;
}

// Per-cell transform path: cells in chunks (spectra and per-slab partial sums in the plan's
// scratch, at most ~2 GiB per chunk): forward DFTs, the inverse DFTs of every term with their
// field products, then finish_kernel sums the slabs' partials and applies the epilogue.
sis_status run_fsm_chunks(sis_plan* p, int64_t n_cells, const double* h, const double* dU, const double* delta,
                          const int32_t* flow, int project, double* rhs, double* lh, double* amom,
                          const double* Kc, hipStream_t s) {
  const sis::FsmDims& d = p->fsm_d;
  const int slabs = sis::fsm_slab_count(d, p->fsm_slab);
  const int64_t per_s = static_cast<int64_t>(d.L) * 2 * d.Q * d.L;
  const int64_t per_a = static_cast<int64_t>(slabs) * d.nv;
  // cells per chunk: ~2 GiB of spectra and partials, at most 65535 (the grid's y extent)
  const int64_t chunk = std::max<int64_t>(
      1, std::min<int64_t>({n_cells, int64_t(65535), (int64_t(2) << 30) / (8 * (per_s + per_a))}));
  HIP_TRY(p->fsm_S.ensure(static_cast<size_t>(chunk * per_s) * 8));
  HIP_TRY(p->fsm_acc.ensure(static_cast<size_t>(chunk * per_a) * 8));
  double* S = static_cast<double*>(p->fsm_S.p);
  double* acc = static_cast<double*>(p->fsm_acc.p);
  const int64_t nv = d.nv;
  for (int64_t c0 = 0; c0 < n_cells; c0 += chunk) {
    const int64_t nc = std::min(chunk, n_cells - c0);
    HIP_TRY(sis::launch_fsm_forward(d, p->fsm_f, nc, h + c0 * nv, S, s));
    HIP_TRY(sis::launch_fsm_inverse(d, p->fsm_f, p->fsm_slab, nc, S, p->fsm_mult, p->fsm_field, acc, s));
    sis::FinishArgs f = finish_args(p, nc, h + c0 * nv, dU ? dU + c0 : nullptr, delta + c0, flow ? flow + c0 : nullptr,
                                    project, rhs + c0 * nv, lh ? lh + c0 * nv : nullptr, amom ? amom + c0 * 4 : nullptr,
                                    nullptr, 0, nullptr, nullptr);
    f.Kc = Kc;
    f.splits = slabs;
    f.acc = acc;
    HIP_TRY(sis::launch_finish(f, s));
  }
  return SIS_OK;
}

// L+ of the correction shape by the transform path itself (the multipliers and fields are
// built with the plan).
sis_status ensure_fsm(sis_plan* p, hipStream_t s) {
  if (p->fsm_ready) return SIS_OK;
  const sis::FsmDims& d = p->fsm_d;
  if (!p->fsm_Kc) HIP_TRY(dmalloc(&p->fsm_Kc, d.nv));
  double *dc = nullptr, *one = nullptr;
  auto cleanup = [&]() { dfree(dc); dfree(one); };
  hipError_t e = upload(&dc, p->fsm_corr, s);
  const std::vector<double> v1(1, 1.0);
  if (e == hipSuccess) e = upload(&one, v1, s);
  if (e != hipSuccess) {
    cleanup();
    return fail(SIS_E_DEVICE, "transform path tables: %s", hipGetErrorString(e));
  }
  // rhs of one cell at delta = 1 with no source and no correction is L+ of that cell
  sis_status st = run_fsm_chunks(p, 1, dc, nullptr, one, nullptr, 0, p->fsm_Kc, nullptr, nullptr, p->Kc, s);
  if (st == SIS_OK) {
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) st = fail(SIS_E_DEVICE, "transform path tables: %s", hipGetErrorString(e));
  }
  cleanup();
  if (st == SIS_OK) p->fsm_ready = true;
  return st;
}

sis_status run_sweep(sis_plan* p, sis_geom* g, const double* rhs, double* h, double* mom,
                     const int32_t* case_active, hipStream_t s, const int32_t* cell_active = nullptr) {
  if (g->tube) {
    sis::TubeSweepArgs a{};
    a.n_vr = p->n_vr;
    a.n_th = p->n_th;
    a.n_vz = p->n_vz;
    a.nv = p->nv;
    a.n_cases = g->n_cases;
    a.node_off = g->off;
    a.r = g->d_r;
    a.cin = g->d_cin;
    a.cout = g->d_cout;
    a.vr = p->d_vr;
    a.cth = p->d_cth;
    a.sth = p->d_sth;
    a.dth = p->dth;
    a.delta_case = g->delta_case;
    a.nu = p->nu;
    a.rhs = rhs;
    a.h = h;
    a.case_active = case_active;
    a.max_nodes = g->max_nodes;
    HIP_TRY(sis::launch_sweep_tube(a, s));
    if (mom) HIP_TRY(sis::launch_moments_tube(g->n_cells, p->nv, p->vnode, p->wnode, h, cell_active, mom, s));
    return SIS_OK;
  }
  if (g->two_d) {
    sis::Sweep2DArgs a{};
    a.n = p->n;
    a.n3 = p->nv;
    a.nsp = p->nsp;
    a.d3 = p->d3;
    a.v3d = p->v1d + (p->n - p->d3);
    a.n_cases = g->n_cases;
    a.n1 = g->d_n1;
    a.n2 = g->d_n2;
    a.grid_off = g->d_goff;
    a.gcell = g->d_gcell;
    a.coef = g->d_scoef;
    a.ref = g->d_sref;
    a.kind = g->d_skind;
    a.rec = g->d_srec;
    a.grec = g->d_grec;
    a.growb = g->d_growb;
    a.grid_none = g->t2.n_grid;
    a.row_bytes_total = g->n_cells * static_cast<int64_t>(p->nsp) * p->nv * static_cast<int64_t>(sizeof(double));
    a.quad_split = g->no_mirror ? 1 : 0;
    a.delta_case = g->delta_case;
    a.v1d = p->v1d;
    a.nu = p->nu;
    a.rhs = rhs;
    a.h = h;
    a.case_active = case_active;
    a.max_diag = g->max_diag;
    a.max_n2 = g->max_n2;
    HIP_TRY(sis::launch_sweep2d(a, s));
    if (mom)
      HIP_TRY(sis::launch_moments2d(p->nv, p->nsp, p->mass_ratio, g->n_cells, p->vtab, h, p->wr, cell_active, mom, s));
    return SIS_OK;
  }
  sis::SweepArgs a{};
  a.n = p->n;
  a.n3 = p->nv;
  a.d2 = p->d2;
  a.d3 = p->d3;
  a.nsp = p->nsp;
  a.n_cases = g->n_cases;
  a.node_off = g->off;
  a.coef = g->coef;
  a.delta_case = g->delta_case;
  a.v1d = p->v1d;
  a.nu = p->nu;
  a.rhs = rhs;
  a.h = h;
  a.case_active = case_active;
  HIP_TRY(sis::launch_sweep1d(a, s));
  if (mom)
    HIP_TRY(sis::launch_moments(p->nv, p->nsp, p->mass_ratio, g->n_cells * p->nsp, p->vtab, h, p->wr, mom, s));
  return SIS_OK;
}

sis::TubeDiffArgs tube_diff_args(sis_plan* p, sis_geom* g, const double* mom, const double* amom, double N) {
  sis::TubeDiffArgs a{};
  a.n_cases = g->n_cases;
  a.node_off = g->off;
  a.r = g->d_r;
  a.cin = g->d_cin;
  a.tw = g->d_tw;
  a.delta_case = g->delta_case;
  a.flow_case = g->flow_case;
  a.mom = mom;
  a.amom = amom;
  a.N = N;
  a.sis = 1;
  a.cU = p->cU;
  a.cq = p->cq;
  return a;
}

sis::Diff2DArgs diff2d_args(sis_plan* p, sis_geom* g, const double* mom, const double* amom, double N) {
  sis::Diff2DArgs a{};
  a.n_cases = g->n_cases;
  a.n_grid = g->t2.n_grid;
  a.n2 = g->d_n2;
  a.grid_off = g->d_goff;
  a.dflag = g->d_dflag;
  a.gcell = g->d_gcell;
  a.nb = g->d_nb;
  a.nbm = g->d_nbm;
  a.npos = g->d_npos;
  a.fw = g->d_fw;
  a.width = g->d_width;
  a.cpos = g->d_cpos;
  a.dA = g->d_dA;
  a.area = g->d_area;
  a.delta_case = g->delta_case;
  a.flow_case = g->flow_case;
  a.mom = mom;
  a.amom = amom;
  a.sis = 1;
  // species: N <= 0 -> nubar of each species (one gas: the caller's N)
  a.nsp = p->nsp;
  if (p->nsp == 1) {
    a.chi[0] = 1.0;
    a.mass_ratio[0] = 1.0;
    a.Ns[0] = N;
    a.cUs[0] = p->cU;
    a.cqs[0] = p->cq;
    a.flow_factor = 1.0;
  } else {
    for (int s = 0; s < 2; ++s) {
      a.chi[s] = p->chi[s];
      a.mass_ratio[s] = p->mass_ratio[s];
      a.Ns[s] = N > 0.0 ? N : p->nubar_s[s];
      a.cUs[s] = p->cU_s[s];
      a.cqs[s] = p->cq_s[s];
    }
    a.flow_factor = p->flow_factor;
  }
  a.work = g->work;
  a.have_x = g->have_x;
  a.tol = 1e-13;
  a.max_iter = 20000;
  a.cg_iters = g->cg_iters;
  if (g->d_direct) {
    a.direct = g->d_direct;
    a.uidx = g->d_uidx;
    a.uoff = g->d_uoff;
    a.n_unknown = g->d_nunk;
    a.max_unknown = g->max_unknown;
    a.n_groups = g->n_groups;
    a.grp_aoff = g->d_grp_aoff;
    a.grp_n = g->d_grp_n;
    a.grp_size = g->d_grp_size;
    a.grp_vec = g->d_grp_vec;
    a.ainv = g->ainv;
    a.bvec = g->bvec;
    a.yvec = g->yvec;
  }
  return a;
}

sis_status check_plan(sis_plan_t p) {
  if (!p) return fail(SIS_E_INVALID, "null plan");
  return SIS_OK;
}

// Species fields of the planar velocity equation(s); N <= 0 -> nubar of each species.
void set_species(sis::DiffusionArgs& a, const sis_plan* p, double N) {
  a.nsp = p->nsp;
  for (int s = 0; s < 2; ++s) {
    a.chi[s] = p->chi[s];
    a.mass_ratio[s] = p->mass_ratio[s];
    a.Ns[s] = N > 0.0 ? N : p->nubar_s[s];
    a.cUs[s] = p->cU_s[s];
    a.cqs[s] = p->cq_s[s];
  }
  a.flow_factor = p->flow_factor;
}

}  // namespace


namespace {

// Inverse of the finite-volume velocity operator of each 2-D case, restricted to
// its unknown cells (those with four fluid neighbours).  A = diag(sum fw) -
// (fw to unknown neighbours) is symmetric; it is positive definite when every
// connected group of unknowns reaches a Dirichlet cell.  With D = diag(A) and
// S = D^-1/2 A D^-1/2 the Newton-Schulz iteration X <- X (2I - S X), X0 = I,
// squares I - S X every step; A^-1 = D^-1/2 X D^-1/2.  Cases that are singular,
// too large, or whose iteration stalls keep the conjugate-gradient solve.
constexpr int64_t kInverseMaxUnknowns = 16384;
constexpr double kInverseMaxBytes = 16.0 * 1073741824.0;
constexpr int kNewtonSchulzMaxIter = 64;

// Same velocity operator on the unknown cells of cases k and r (same cross section)?
bool same_operator_2d(const sis::Tables2D& t, int k, int r) {
  const int64_t gk = t.grid_off[k], gr = t.grid_off[r];
  const int64_t n = t.grid_off[k + 1] - gk;
  if (t.grid_off[r + 1] - gr != n) return false;
  for (int64_t i = 0; i < n; ++i) {
    if (t.dflag[gk + i] != t.dflag[gr + i]) return false;
    for (int q = 0; q < 4; ++q)
      if (t.nb[(gk + i) * 8 + q] != t.nb[(gr + i) * 8 + q] || t.fw[(gk + i) * 4 + q] != t.fw[(gr + i) * 4 + q])
        return false;
  }
  return true;
}

sis_status build_inverse_2d(sis_plan* p, sis_geom* g, hipStream_t s) {
  g->free_inverse();
  const sis::Tables2D& t = g->t2;
  const int nc = g->n_cases;
  std::vector<int32_t> uidx(t.n_grid, -1), nunk(nc, 0), direct(nc, 0), rep(nc, -1);
  std::vector<int64_t> uoff(nc + 1, 0), aoff(nc, -1);
  int64_t ainv_size = 0;
  for (int k = 0; k < nc; ++k) {
    const int64_t g0 = t.grid_off[k], g1 = t.grid_off[k + 1];
    for (int64_t G = g0; G < g1; ++G)
      if (t.dflag[G] == 2) uidx[G] = nunk[k]++;
    uoff[k + 1] = uoff[k] + nunk[k];
    if (nunk[k] > kInverseMaxUnknowns) continue;
    for (int r = 0; r < k && rep[k] < 0; ++r)
      if (rep[r] == r && same_operator_2d(t, k, r)) rep[k] = r;
    if (rep[k] >= 0) continue;
    // every connected group of unknowns must touch a Dirichlet cell
    bool ok = true;
    if (nunk[k] > 0) {
      std::vector<char> seen(nunk[k], 0);
      std::vector<int32_t> stack;
      for (int64_t G = g0; G < g1 && ok; ++G) {
        if (t.dflag[G] != 2 || seen[uidx[G]]) continue;
        bool anchor = false;
        seen[uidx[G]] = 1;
        stack.assign(1, static_cast<int32_t>(G - g0));
        while (!stack.empty()) {
          const int64_t H = g0 + stack.back();
          stack.pop_back();
          for (int q = 0; q < 4; ++q) {
            if (t.fw[H * 4 + q] == 0.0) continue;
            const int r = t.nb[H * 8 + q];
            if (t.dflag[g0 + r] != 2) { anchor = true; continue; }
            if (!seen[uidx[g0 + r]]) {
              seen[uidx[g0 + r]] = 1;
              stack.push_back(r);
            }
          }
        }
        ok = anchor;
      }
    }
    const int64_t need = static_cast<int64_t>(nunk[k]) * nunk[k];
    if (ok && (ainv_size + need) * 8.0 <= kInverseMaxBytes) {
      rep[k] = k;
      aoff[k] = ainv_size;
      ainv_size += need;
    }
  }
  int max_np = 0;
  for (int k = 0; k < nc; ++k)
    if (rep[k] == k) max_np = std::max(max_np, (nunk[k] + 1) & ~1);
  // scratch of the iteration: S, X, P, X_next and the residual partials
  const int kBlocks = 1024;
  double *S = nullptr, *X = nullptr, *P = nullptr, *Xn = nullptr, *part = nullptr, *sc = nullptr, *val = nullptr;
  int32_t* rc = nullptr;
  auto cleanup = [&]() {
    dfree(S); dfree(X); dfree(P); dfree(Xn); dfree(part); dfree(sc); dfree(val); dfree(rc);
    S = X = P = Xn = part = sc = val = nullptr;
    rc = nullptr;
  };
#define INV_TRY(expr)                                                                          \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess) {                                                                    \
      cleanup();                                                                               \
      g->free_inverse();                                                                       \
      return fail(e_ == hipErrorOutOfMemory ? SIS_E_OOM : SIS_E_DEVICE, "%s: %s", #expr,        \
                  hipGetErrorString(e_));                                                      \
    }                                                                                          \
  } while (0)
  const size_t mat = static_cast<size_t>(max_np) * max_np;
  if (max_np > 0) {
    INV_TRY(dmalloc(&S, mat));
    INV_TRY(dmalloc(&X, mat));
    INV_TRY(dmalloc(&P, mat));
    INV_TRY(dmalloc(&Xn, mat));
    INV_TRY(dmalloc(&part, kBlocks));
    INV_TRY(dmalloc(&sc, max_np));
    INV_TRY(dmalloc(&val, static_cast<size_t>(max_np) * 5));
    INV_TRY(dmalloc(&rc, static_cast<size_t>(max_np) * 10));
    INV_TRY(dmalloc(&g->ainv, static_cast<size_t>(ainv_size)));
  }
  std::vector<double> h_part(kBlocks);
  std::vector<char> inverted(nc, 0);
  double worst = 0.0;
  for (int k = 0; k < nc; ++k) {
    if (rep[k] != k) continue;
    const int nu = nunk[k], np = (nu + 1) & ~1;
    if (nu == 0) { inverted[k] = 1; continue; }
    const int64_t g0 = t.grid_off[k], g1 = t.grid_off[k + 1];
    // scaled entries: unit diagonal, -fw / sqrt(d_i d_j) to unknown neighbours
    std::vector<double> hs(np, 1.0);
    for (int64_t G = g0; G < g1; ++G) {
      if (t.dflag[G] != 2) continue;
      double d = 0.0;
      for (int q = 0; q < 4; ++q) d += t.fw[G * 4 + q];
      hs[uidx[G]] = 1.0 / std::sqrt(d);
    }
    std::vector<int32_t> h_rc;
    std::vector<double> h_val;
    for (int i = 0; i < np; ++i) {
      h_rc.push_back(i);
      h_rc.push_back(i);
      h_val.push_back(1.0);
    }
    for (int64_t G = g0; G < g1; ++G) {
      if (t.dflag[G] != 2) continue;
      const int i = uidx[G];
      int cols[4];
      double vals[4];
      int m = 0;
      for (int q = 0; q < 4; ++q) {
        const double fw = t.fw[G * 4 + q];
        if (fw == 0.0) continue;
        const int r = t.nb[G * 8 + q];
        if (t.dflag[g0 + r] != 2) continue;
        const int j = uidx[g0 + r];
        const double v = -fw * hs[i] * hs[j];
        int e = 0;
        while (e < m && cols[e] != j) ++e;
        if (e == m) { cols[m] = j; vals[m] = 0.0; ++m; }
        vals[e] += v;
      }
      for (int e = 0; e < m; ++e) {
        h_rc.push_back(i);
        h_rc.push_back(cols[e]);
        h_val.push_back(vals[e]);
      }
    }
    const int64_t ne = static_cast<int64_t>(h_val.size());
    const size_t sq = static_cast<size_t>(np) * np;
    INV_TRY(hipMemsetAsync(S, 0, sq * sizeof(double), s));
    INV_TRY(hipMemcpyAsync(rc, h_rc.data(), h_rc.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    INV_TRY(hipMemcpyAsync(val, h_val.data(), h_val.size() * sizeof(double), hipMemcpyHostToDevice, s));
    INV_TRY(hipMemcpyAsync(sc, hs.data(), np * sizeof(double), hipMemcpyHostToDevice, s));
    INV_TRY(sis::launch_ns_scatter(S, np, rc, val, ne, s));
    // X0 = I: the spectrum of S lies in (0, 2), so |1 - lambda| < 1
    INV_TRY(hipMemsetAsync(X, 0, sq * sizeof(double), s));
    INV_TRY(sis::launch_ns_scatter(X, np, rc, val, np, s));   // the unit diagonal entries come first
    sis::GemmArgs ga{};
    ga.precision = 0;
    ga.M = np;
    ga.N = np;
    ga.K = np;
    ga.splits = 1;
    ga.tile = 0;
    const int blocks = static_cast<int>(std::min<int64_t>(kBlocks, (static_cast<int64_t>(np) * np + 255) / 256));
    int extra = -1;
    double res = 0.0;
    bool ok = false;
    for (int it = 0; it < kNewtonSchulzMaxIter; ++it) {
      ga.X = X;          // P = X S (S symmetric, so X S^T = X S)
      ga.op64 = S;
      ga.acc = P;
      INV_TRY(sis::launch_gemm(ga, s));
      INV_TRY(sis::launch_ns_residual(P, np, part, blocks, s));
      INV_TRY(hipMemcpyAsync(h_part.data(), part, blocks * sizeof(double), hipMemcpyDeviceToHost, s));
      INV_TRY(hipStreamSynchronize(s));
      res = 0.0;
      for (int b = 0; b < blocks; ++b) res += h_part[b];
      res = std::sqrt(res);
      if (!std::isfinite(res)) break;
      if (extra == 0) { ok = res < 1e-8; break; }
      if (extra < 0 && res < 0.25) extra = 4;   // 2-norm < 1/4: four squarings reach rounding level
      if (extra > 0) --extra;
      INV_TRY(sis::launch_ns_two_minus(P, np, s));
      ga.X = X;          // X_next = X (2I - P)^T = X (2I - S X)
      ga.op64 = P;
      ga.acc = Xn;
      INV_TRY(sis::launch_gemm(ga, s));
      std::swap(X, Xn);
    }
    if (!ok) continue;
    inverted[k] = 1;
    worst = std::max(worst, res);
    INV_TRY(sis::launch_ns_scale(X, np, nu, sc, g->ainv + aoff[k], s));
  }
  INV_TRY(hipStreamSynchronize(s));
  cleanup();
  // groups of at most kInverseGroup right sides (case, species) per shared inverse
  const int nsp = p->nsp;
  std::vector<int64_t> grp_aoff, grp_vec;
  std::vector<int32_t> grp_n, grp_size;
  int n_direct = 0, max_unknown = 0;
  for (int r = 0; r < nc; ++r) {
    if (rep[r] != r || !inverted[r]) continue;
    for (int k = r; k < nc; ++k) {
      if (rep[k] != r) continue;
      direct[k] = 1;
      ++n_direct;
      if (nunk[k] == 0) continue;
      for (int s = 0; s < nsp; ++s) {
        const int64_t voff = nsp * uoff[k] + static_cast<int64_t>(s) * nunk[k];
        if (grp_n.empty() || grp_aoff.back() != aoff[r] || grp_size.back() == sis::kInverseGroup) {
          grp_aoff.push_back(aoff[r]);
          grp_n.push_back(nunk[r]);
          grp_size.push_back(0);
          grp_vec.resize(grp_vec.size() + sis::kInverseGroup, voff);
        }
        grp_vec[(grp_size.size() - 1) * sis::kInverseGroup + grp_size.back()] = voff;
        ++grp_size.back();
      }
      max_unknown = std::max(max_unknown, nunk[k]);
    }
  }
  if (nsp == 2 && n_direct < nc) {
    g->free_inverse();
    return fail(SIS_E_UNSUPPORTED,
                "2-D mixtures need the precomputed inverse of every case (a case is singular or too large)");
  }
  if (n_direct == 0) {
    dfree(g->ainv);
    g->ainv = nullptr;
    return SIS_OK;
  }
  INV_TRY(upload(&g->d_direct, direct, s));
  INV_TRY(upload(&g->d_uidx, uidx, s));
  INV_TRY(upload(&g->d_nunk, nunk, s));
  INV_TRY(upload(&g->d_uoff, uoff, s));
  INV_TRY(upload(&g->d_grp_aoff, grp_aoff, s));
  INV_TRY(upload(&g->d_grp_n, grp_n, s));
  INV_TRY(upload(&g->d_grp_size, grp_size, s));
  INV_TRY(upload(&g->d_grp_vec, grp_vec, s));
  INV_TRY(dmalloc(&g->bvec, static_cast<size_t>(nsp * uoff[nc])));
  INV_TRY(dmalloc(&g->yvec, static_cast<size_t>(nsp * uoff[nc])));
  INV_TRY(hipMemsetAsync(g->bvec, 0, std::max<int64_t>(nsp * uoff[nc], 1) * sizeof(double), s));
  INV_TRY(hipStreamSynchronize(s));
#undef INV_TRY
  g->h_direct = direct;
  g->n_direct = n_direct;
  g->n_groups = static_cast<int>(grp_n.size());
  g->n_inverses = 0;
  for (int r = 0; r < nc; ++r) g->n_inverses += (rep[r] == r && inverted[r] && nunk[r] > 0) ? 1 : 0;
  g->max_unknown = max_unknown;
  g->inv_residual = worst;
  return SIS_OK;
}

// Tube (Sec. 4): per case the radial nodes r_0 < ... < r_{n-1} = 1 (the wall), n >= 3.
// Upwind coefficients of d/dr: inward from the nodes i, i+1, i+2 (two-point next to the
// wall), outward from i, i-1, i-2 with the centre ghosts -r_0, -r_1; trapezoid weights of
// 2 int_0^1 f r dr with the centre (f r = 0 there) as the first point.
sis_status create_geometry_tube(sis_plan* p, const sis_geometry_desc* d, hipStream_t stream, sis_geom_t* out) {
  if (!d->node_offset || !d->x1 || !d->delta || !d->flow) return fail(SIS_E_INVALID, "null geometry array");
  if (d->node_offset[0] != 0) return fail(SIS_E_INVALID, "node_offset[0] must be 0");
  auto* g = new sis_geom();
  g->plan = p;
  g->kind = d->kind;
  g->n_cases = d->n_cases;
  g->tube = true;
  g->h_off.assign(d->node_offset, d->node_offset + d->n_cases + 1);
  g->n_cells = g->h_off.back();
  for (int c = 0; c < d->n_cases; ++c) {
    const int64_t a = g->h_off[c], b = g->h_off[c + 1];
    if (b - a < 3) { delete g; return fail(SIS_E_SHAPE, "case %d has fewer than 3 radial nodes", c); }
    g->max_nodes = std::max<int>(g->max_nodes, static_cast<int>(b - a));
    if (!(d->x1[a] > 0.0) || d->x1[b - 1] != 1.0) { delete g; return fail(SIS_E_INVALID, "case %d radial nodes must run from r > 0 to 1", c); }
    for (int64_t i = a + 1; i < b; ++i)
      if (!(d->x1[i] > d->x1[i - 1])) { delete g; return fail(SIS_E_INVALID, "case %d nodes not increasing", c); }
    if (!(d->delta[c] >= 0.0) || !std::isfinite(d->delta[c])) { delete g; return fail(SIS_E_INVALID, "case %d delta must be >= 0", c); }
    if (d->flow[c] != SIS_FLOW_NONE && d->flow[c] != SIS_FLOW_POISEUILLE) { delete g; return fail(SIS_E_UNSUPPORTED, "the tube supports Poiseuille flow only (case %d)", c); }
  }
  g->h_x.assign(d->x1, d->x1 + g->n_cells);
  g->h_delta.assign(d->delta, d->delta + d->n_cases);
  g->h_flow.assign(d->flow, d->flow + d->n_cases);
  const int64_t nc = g->n_cells;
  std::vector<double> cin(nc * 3, 0.0), cout(nc * 3, 0.0), tw(nc, 0.0), dcell(nc);
  std::vector<int32_t> fcell(nc), ccell(nc);
  auto coeffs = [](double d1, double d2, double* q) {
    q[0] = (2.0 * d1 + d2) / (d1 * (d1 + d2));
    q[1] = -(d1 + d2) / (d1 * d2);
    q[2] = d1 / (d2 * (d1 + d2));
  };
  for (int c = 0; c < d->n_cases; ++c) {
    const int64_t a = g->h_off[c];
    const int n = static_cast<int>(g->h_off[c + 1] - a);
    const double* r = d->x1 + a;
    std::vector<double> xe(n + 2);
    xe[0] = -r[1];
    xe[1] = -r[0];
    for (int i = 0; i < n; ++i) xe[i + 2] = r[i];
    for (int i = 0; i < n; ++i) {
      double* qi = &cin[(a + i) * 3];
      if (i == n - 2) {
        const double d1 = r[i] - r[i + 1];
        qi[0] = 1.0 / d1;
        qi[1] = -1.0 / d1;
        qi[2] = 0.0;
      } else if (i < n - 2) {
        coeffs(r[i] - r[i + 1], r[i + 1] - r[i + 2], qi);
      }
      coeffs(xe[i + 2] - xe[i + 1], xe[i + 1] - xe[i], &cout[(a + i) * 3]);
      const double lo = i == 0 ? 0.0 : r[i - 1], hi = i == n - 1 ? r[i] : r[i + 1];
      tw[a + i] = r[i] * (hi - lo);
      dcell[a + i] = d->delta[c];
      fcell[a + i] = d->flow[c];
      ccell[a + i] = c;
    }
  }
#define TUBE_TRY(expr)                                                                         \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess) {                                                                    \
      delete g;                                                                                \
      return fail(e_ == hipErrorOutOfMemory ? SIS_E_OOM : SIS_E_DEVICE, "%s: %s", #expr,        \
                  hipGetErrorString(e_));                                                      \
    }                                                                                          \
  } while (0)
  TUBE_TRY(upload(&g->off, g->h_off, stream));
  TUBE_TRY(upload(&g->d_r, g->h_x, stream));
  TUBE_TRY(upload(&g->d_cin, cin, stream));
  TUBE_TRY(upload(&g->d_cout, cout, stream));
  TUBE_TRY(upload(&g->d_tw, tw, stream));
  TUBE_TRY(upload(&g->delta_case, g->h_delta, stream));
  TUBE_TRY(upload(&g->flow_case, g->h_flow, stream));
  TUBE_TRY(upload(&g->delta_cell, dcell, stream));
  TUBE_TRY(upload(&g->flow_cell, fcell, stream));
  TUBE_TRY(upload(&g->case_of_cell, ccell, stream));
  TUBE_TRY(hipStreamSynchronize(stream));
#undef TUBE_TRY
  *out = g;
  g_err.clear();
  return SIS_OK;
}

sis_status create_geometry_2d(sis_plan* p, const sis_geometry_desc* d, hipStream_t stream, sis_geom_t* out) {
  if (!d->n1 || !d->n2 || !d->face1 || !d->face2 || !d->delta || !d->flow)
    return fail(SIS_E_INVALID, "null 2-D geometry array");
  std::vector<sis::Case2D> cases(d->n_cases);
  int64_t f1o = 0, f2o = 0, so = 0;
  int max_diag = 0, max_n2 = 0;
  for (int c = 0; c < d->n_cases; ++c) {
    sis::Case2D& k = cases[c];
    k.n1 = d->n1[c];
    k.n2 = d->n2[c];
    max_diag = std::max(max_diag, std::min(k.n1, k.n2));
    max_n2 = std::max(max_n2, k.n2);
    if (k.n1 < 2 || k.n2 < 2 || k.n1 > 4096 || k.n2 > 4096)
      return fail(SIS_E_SHAPE, "case %d: n1, n2 must be in [2, 4096]", c);
    k.f1.assign(d->face1 + f1o, d->face1 + f1o + k.n1 + 1);
    k.f2.assign(d->face2 + f2o, d->face2 + f2o + k.n2 + 1);
    f1o += k.n1 + 1;
    f2o += k.n2 + 1;
    if (d->kind == SIS_GEOM_DUCT_QUARTER) {
      k.bc[0] = sis::kWall; k.bc[1] = sis::kSym; k.bc[2] = sis::kWall; k.bc[3] = sis::kSym;
    } else {
      for (int q = 0; q < 4; ++q) k.bc[q] = sis::kPeriodic;
    }
    if (d->solid) {
      k.solid.assign(d->solid + so, d->solid + so + static_cast<int64_t>(k.n1) * k.n2);
      so += static_cast<int64_t>(k.n1) * k.n2;
    }
    if (!(d->delta[c] >= 0.0) || !std::isfinite(d->delta[c])) return fail(SIS_E_INVALID, "case %d delta must be >= 0", c);
    if (d->flow[c] < 0 || d->flow[c] > 2) return fail(SIS_E_INVALID, "case %d flow code %d", c, d->flow[c]);
  }
  auto* g = new sis_geom();
  g->plan = p;
  g->kind = d->kind;
  g->n_cases = d->n_cases;
  g->two_d = true;
  g->max_diag = max_diag;
  g->max_n2 = max_n2;
  std::string err;
  if (!sis::build_tables_2d(cases, g->t2, err)) { delete g; return fail(SIS_E_INVALID, "%s", err.c_str()); }
  const sis::Tables2D& t = g->t2;
  g->n_cells = t.n_cells;
  g->h_off = t.cell_off;
  g->h_delta.assign(d->delta, d->delta + d->n_cases);
  g->h_flow.assign(d->flow, d->flow + d->n_cases);
  std::vector<double> dcell(t.n_cells);
  std::vector<int32_t> fcell(t.n_cells);
  for (int64_t i = 0; i < t.n_cells; ++i) {
    dcell[i] = d->delta[t.cell_case[i]];
    fcell[i] = d->flow[t.cell_case[i]];
  }
#define G2_TRY(expr)                                                                           \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess) {                                                                    \
      delete g;                                                                                \
      return fail(e_ == hipErrorOutOfMemory ? SIS_E_OOM : SIS_E_DEVICE, "%s: %s", #expr,        \
                  hipGetErrorString(e_));                                                      \
    }                                                                                          \
  } while (0)
  G2_TRY(upload(&g->off, t.cell_off, stream));
  G2_TRY(upload(&g->d_n1, t.n1, stream));
  G2_TRY(upload(&g->d_n2, t.n2, stream));
  G2_TRY(upload(&g->d_goff, t.grid_off, stream));
  G2_TRY(upload(&g->d_gcell, t.gcell, stream));
  G2_TRY(upload(&g->d_scoef, t.st_coef, stream));
  G2_TRY(upload(&g->d_sref, t.st_ref, stream));
  G2_TRY(upload(&g->d_skind, t.st_kind, stream));
  // one 32-byte record per (cell, axis, sign): coefficients a, b, c, then the two references
  // as (ref << 2 | kind); at least one record so that masked lanes can load a valid address.
  // The row-blocked sweep reads the same records in grid order, with the coefficient of a
  // reference of kind 0 (wall or solid face, h = 0) set to 0 and zero records at solid cells.
  const size_t nrec = t.st_coef.size() / 3;
  if (nrec / 4 >= (size_t(1) << 30)) { delete g; return fail(SIS_E_SHAPE, "more than 2^30 fluid cells"); }
  std::vector<uint32_t> rec(std::max<size_t>(nrec, 1) * 8, 0u);
  for (size_t o = 0; o < nrec; ++o) {
    std::memcpy(&rec[o * 8], &t.st_coef[o * 3], 3 * sizeof(double));
    for (int k = 0; k < 2; ++k) {
      const int kind = t.st_kind[o * 2 + k];
      rec[o * 8 + 6 + k] = kind == 0 ? 0u : (static_cast<uint32_t>(t.st_ref[o * 2 + k]) << 2) | static_cast<uint32_t>(kind);
    }
  }
  G2_TRY(upload(&g->d_srec, rec, stream));
  g->no_mirror = true;
  for (int8_t kind : t.st_kind) g->no_mirror = g->no_mirror && kind != 2;
  // (solid cells: a = 1, so that the placeholder update the sweep computes there stays finite;
  // one more solid entry at index n_grid stands for positions outside the grid)
  std::vector<uint32_t> grec(static_cast<size_t>(t.n_grid + 1) * 4 * 8, 0u);
  std::vector<uint32_t> growb(t.n_grid + 1, 0xffffffffu);
  for (int64_t gi = 0; gi <= t.n_grid; ++gi) {
    const int32_t cell = gi < t.n_grid ? t.gcell[gi] : -1;
    for (int o = 0; o < 4; ++o) {
      uint32_t* dst = &grec[(static_cast<size_t>(gi) * 4 + o) * 8];
      if (cell < 0) {
        const double one = 1.0;
        std::memcpy(dst, &one, sizeof(double));
        continue;
      }
      const uint32_t* src = &rec[(static_cast<size_t>(cell) * 4 + o) * 8];
      std::memcpy(dst, src, 8 * sizeof(uint32_t));
      for (int k = 0; k < 2; ++k)
        if (src[6 + k] == 0u) { dst[2 + 2 * k] = 0u; dst[3 + 2 * k] = 0u; }
    }
    const int64_t off = static_cast<int64_t>(cell) * p->nsp * p->nv * static_cast<int64_t>(sizeof(double));
    if (cell >= 0 && off < (int64_t(1) << 31)) growb[gi] = static_cast<uint32_t>(off);
  }
  G2_TRY(upload(&g->d_grec, grec, stream));
  G2_TRY(upload(&g->d_growb, growb, stream));
  G2_TRY(upload(&g->d_dflag, t.dflag, stream));
  G2_TRY(upload(&g->d_nb, t.nb, stream));
  G2_TRY(upload(&g->d_nbm, t.nbm, stream));
  G2_TRY(upload(&g->d_npos, t.npos, stream));
  G2_TRY(upload(&g->d_fw, t.fw, stream));
  G2_TRY(upload(&g->d_width, t.width, stream));
  G2_TRY(upload(&g->d_cpos, t.cpos, stream));
  G2_TRY(upload(&g->d_dA, t.dA, stream));
  G2_TRY(upload(&g->d_area, t.area, stream));
  G2_TRY(upload(&g->delta_case, g->h_delta, stream));
  G2_TRY(upload(&g->flow_case, g->h_flow, stream));
  G2_TRY(upload(&g->delta_cell, dcell, stream));
  G2_TRY(upload(&g->flow_cell, fcell, stream));
  G2_TRY(upload(&g->case_of_cell, t.cell_case, stream));
  G2_TRY(dmalloc(&g->work, static_cast<size_t>(t.n_grid) * sis::kDiffWork * p->nsp));
  G2_TRY(upload(&g->have_x, std::vector<int32_t>(d->n_cases, 0), stream));
  G2_TRY(upload(&g->cg_iters, std::vector<int32_t>(d->n_cases, 0), stream));
  G2_TRY(hipStreamSynchronize(stream));
#undef G2_TRY
  if (sis_status st = build_inverse_2d(p, g, stream)) {
    delete g;
    return st;
  }
  *out = g;
  g_err.clear();
  return SIS_OK;
}


// Stored velocity layout of a plan (see sis_plan::parity).
void set_layout(sis_plan* p, int parity) {
  const int n = p->n;
  p->parity = parity;
  p->d2 = parity == 2 ? n / 2 : n;
  p->d3 = parity >= 1 ? n / 2 : n;
  p->nv = n * p->d2 * p->d3;
  p->ndof = p->nsp * p->nv;
  p->wr = p->w * (parity == 2 ? 4.0 : parity == 1 ? 2.0 : 1.0);
}

// Per-velocity tables of a Cartesian plan in its stored layout: the components of each stored
// velocity and its weight (the images of the unstored half spaces included).
sis_status build_velocity_tables(sis_plan* p, hipStream_t stream) {
  const int n = p->n, d2 = p->d2, d3 = p->d3;
  const size_t nv = static_cast<size_t>(p->nv);
  std::vector<double> vt(3 * nv), wt(nv, p->wr);
  for (int j1 = 0; j1 < n; ++j1)
    for (int j2 = 0; j2 < d2; ++j2)
      for (int j3 = 0; j3 < d3; ++j3) {
        const size_t v = (static_cast<size_t>(j1) * d2 + j2) * d3 + j3;
        vt[v] = p->h_v1d[j1];
        vt[nv + v] = p->h_v1d[j2 + (n - d2)];
        vt[2 * nv + v] = p->h_v1d[j3 + (n - d3)];
      }
  dfree(p->vtab);
  dfree(p->wtab);
  p->vtab = p->wtab = nullptr;
  HIP_TRY(upload(&p->vtab, vt, stream));
  HIP_TRY(upload(&p->wtab, wt, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  return SIS_OK;
}

// Full-grid [species][n^3] array -> stored [species][nv] (v2, v3 of the upper halves).
std::vector<double> restrict_rows(const sis_plan* p, const double* full, int rows) {
  const int n = p->n, n3 = n * n * n;
  std::vector<double> out(static_cast<size_t>(rows) * p->nv);
  for (int s = 0; s < rows; ++s)
    for (int j1 = 0; j1 < n; ++j1)
      for (int j2 = 0; j2 < p->d2; ++j2)
        for (int j3 = 0; j3 < p->d3; ++j3)
          out[static_cast<size_t>(s) * p->nv + (j1 * p->d2 + j2) * p->d3 + j3] =
              full[static_cast<size_t>(s) * n3 + (j1 * n + j2 + (n - p->d2)) * n + j3 + (n - p->d3)];
  return out;
}

// Replace the assembled full-grid operator by its restriction to the stored
// parity class and restrict the equilibrium / collision-frequency tables.
sis_status apply_parity(sis_plan* p, hipStream_t stream) {
  if (!p->parity) return SIS_OK;
  const int64_t ld_full = static_cast<int64_t>(p->nsp) * p->n3;
  double* red = nullptr;
  HIP_TRY(dmalloc(&red, static_cast<size_t>(p->ndof) * p->ndof));
  hipError_t e = sis::launch_reduce_operator(p->op, ld_full, red, p->nsp, p->n, p->parity, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  if (e != hipSuccess) {
    dfree(red);
    return fail(SIS_E_DEVICE, "operator restriction: %s", hipGetErrorString(e));
  }
  dfree(p->op);
  p->op = red;
  p->h_feq = restrict_rows(p, p->h_feq.data(), p->nsp);
  p->h_nu = restrict_rows(p, p->h_nu.data(), p->nsp);
  HIP_TRY(hipMemcpyAsync(p->feq, p->h_feq.data(), p->h_feq.size() * 8, hipMemcpyHostToDevice, stream));
  HIP_TRY(hipMemcpyAsync(p->nu, p->h_nu.data(), p->h_nu.size() * 8, hipMemcpyHostToDevice, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  return SIS_OK;
}

// Binary-mixture plan: 2 x 2 blocks of n3 x n3, each assembled from the
// equal-mass (closed-form phi) terms or the rho-quadrature terms of the
// unequal-mass gain, plus the loss.  Cross terms are built on the host in
// chunks and accumulated on the device while the next chunk is built.
// Inverse factor matrices (re block then im block) of the velocity nodes (diff = false, m = n)
// or the difference grid (diff = true, m = 2n - 1) over the modes of an n_pad = P box:
// e1 [m][L] for axes 1, 2 and e3 [m][Q] (doubled for l3 > 0) for axis 3.
void inverse_factors(int n, int P, int m, bool diff, std::vector<double>& e1, std::vector<double>& e3) {
  const int L = P - 1, Q = P / 2, half = P / 2 - 1;
  e1.assign(2 * static_cast<size_t>(m) * L, 0.0);
  e3.assign(2 * static_cast<size_t>(m) * Q, 0.0);
  double c, sn;
  for (int a = 0; a < m; ++a) {
    for (int li = 0; li < L; ++li) {
      const int l = li - half;
      if (diff) phase_q(2L * l * (a - (n - 1)), P, c, sn);
      else fsm_phase(l, a, n, P, c, sn);
      e1[static_cast<size_t>(a) * L + li] = c;
      e1[static_cast<size_t>(m) * L + static_cast<size_t>(a) * L + li] = sn;
    }
    for (int l3 = 0; l3 < Q; ++l3) {
      if (diff) phase_q(2L * l3 * (a - (n - 1)), P, c, sn);
      else fsm_phase(l3, a, n, P, c, sn);
      const double w = l3 == 0 ? 1.0 : 2.0;
      e3[static_cast<size_t>(a) * Q + l3] = w * c;
      e3[static_cast<size_t>(m) * Q + static_cast<size_t>(a) * Q + l3] = w * sn;
    }
  }
}

// Spectrum of a zero-extended separable even profile, prod_k ghat(l_k), in the layout of a
// transform-path spectrum ([L][re, im][Q][L]; real).
std::vector<double> separable_spectrum(const std::vector<double>& g, int n, int P) {
  const int L = P - 1, Q = P / 2, half = P / 2 - 1;
  std::vector<double> gl(L);
  double c, sn;
  for (int li = 0; li < L; ++li) {
    double acc = 0.0;
    for (int j = 0; j < n; ++j) {
      fsm_phase(li - half, j, n, P, c, sn);
      acc += g[j] * c;
    }
    gl[li] = acc;
  }
  std::vector<double> X(static_cast<size_t>(L) * 2 * Q * L, 0.0);
  for (int l1 = 0; l1 < L; ++l1)
    for (int l3 = 0; l3 < Q; ++l3)
      for (int l2 = 0; l2 < L; ++l2) X[(static_cast<size_t>(l1) * 2 * Q + l3) * L + l2] = gl[l1] * gl[l3 + half] * gl[l2];
  return X;
}

// The binary-mixture operator assembled from term tables built on the device: the hard-sphere
// multipliers, pruned inverse DFTs for the unshifted kernels Psi_p, Phi_p, beta_r and the
// species fields, and for every (direction, rho node, sign) of the unequal-mass pairs the
// shifted kernel or field (per-term factor matrices) with the separable band-limited factor.
// Fills p->op (full grid, zeroed by the caller), the host nu tables and nubar of t.
sis_status mix_tables_device(sis_plan* p, sis::MixTables& t, hipStream_t stream) {
  const int n = t.n, P = t.np, L = P - 1, Q = P / 2, D = t.D, nd = t.nd, T1 = 2 * D + 1;
  const int64_t n3 = t.n3, nd3 = t.nd3, ndof = p->ndof;
  std::vector<void*> owned;
  auto cleanup = [&]() { for (void* q : owned) dfree(q); owned.clear(); };
  auto ua = [&](auto** dst, const auto& v) -> hipError_t {
    hipError_t e = upload(dst, v, stream);
    if (e == hipSuccess) owned.push_back(*dst);
    return e;
  };
  auto al = [&](double** dst, size_t count) -> hipError_t {
    hipError_t e = dmalloc(dst, count);
    if (e == hipSuccess) owned.push_back(*dst);
    return e;
  };
#define MT_TRY(expr)                                                                          \
  do {                                                                                        \
    hipError_t e_ = (expr);                                                                   \
    if (e_ != hipSuccess) {                                                                   \
      (void)hipStreamSynchronize(stream);                                                     \
      cleanup();                                                                              \
      return fail(e_ == hipErrorOutOfMemory ? SIS_E_OOM : SIS_E_DEVICE, "mixture tables: %s: %s", #expr, \
                  hipGetErrorString(e_));                                                     \
    }                                                                                         \
  } while (0)
  sis::FsmDims d{};
  d.n = n;
  d.P = P;
  d.L = L;
  d.Q = Q;
  d.n2 = d.n3 = n;
  d.nv = static_cast<int>(n3);
  d.T = T1;
  // hard-sphere multipliers psi_p, phi_p, beta = 4 b0 sum_p W_p phi_p psi_p
  std::vector<double> dw(4 * D);
  for (int q = 0; q < D; ++q) {
    dw[3 * q] = t.ex[q];
    dw[3 * q + 1] = t.ey[q];
    dw[3 * q + 2] = t.ez[q];
    dw[3 * D + q] = t.W[q];
  }
  double *ddir = nullptr, *dmult = nullptr;
  MT_TRY(ua(&ddir, dw));
  const int64_t qll = static_cast<int64_t>(Q) * L * L;
  MT_TRY(al(&dmult, static_cast<size_t>(T1) * qll));
  {
    sis::FsmMultArgs m{};
    m.d = d;
    m.D = D;
    m.b0 = t.b0;
    m.R = t.R;
    m.Lp = t.Lp;
    m.dirs = ddir;
    m.W = ddir + 3 * D;
    m.phi_closed = m.psi_closed = 1;
    m.mult = dmult;
    MT_TRY(sis::launch_fsm_multipliers(m, stream));
  }
  // unshifted kernels and the species fields
  std::vector<double> ev1, ev3, ed1, ed3;
  inverse_factors(n, P, n, false, ev1, ev3);
  inverse_factors(n, P, nd, true, ed1, ed3);
  double *dv1 = nullptr, *dv3 = nullptr, *dd1 = nullptr, *dd3 = nullptr, *dK = nullptr, *dF[2] = {nullptr, nullptr};
  double *dS[2] = {nullptr, nullptr}, *dsc = nullptr;
  int *dslK = nullptr, *dslF = nullptr;
  MT_TRY(ua(&dv1, ev1));
  MT_TRY(ua(&dv3, ev3));
  MT_TRY(ua(&dd1, ed1));
  MT_TRY(ua(&dd3, ed3));
  std::vector<int> slK(T1), slF(T1);
  for (int q = 0; q < D; ++q) {
    slK[2 * q] = q;           // Psi_p
    slK[2 * q + 1] = D + q;   // Phi_p
    slF[2 * q] = D + q;       // Fpsi_s
    slF[2 * q + 1] = q;       // Fphi_s
  }
  slK[2 * D] = slF[2 * D] = 2 * D;   // beta_r, 4 b0 F^-1[sum W phi psi F f_s]
  MT_TRY(ua(&dslK, slK));
  MT_TRY(ua(&dslF, slF));
  const std::vector<double> scT(T1, 1.0 / (static_cast<double>(P) * P * P));
  MT_TRY(ua(&dsc, scT));
  MT_TRY(al(&dK, static_cast<size_t>(T1) * nd3));
  std::vector<double> spec[2];
  for (int s = 0; s < 2; ++s) {
    spec[s] = separable_spectrum(t.prof[s], n, P);
    MT_TRY(ua(&dS[s], spec[s]));
    MT_TRY(al(&dF[s], static_cast<size_t>(T1) * n3));
  }
  sis::FsmTableArgs a{};
  a.d = d;
  a.mult = dmult;
  a.scale = dsc;
  a.t0 = 0;
  a.nt = T1;
  a.m1 = a.m2 = a.m3 = nd;
  a.e1r = a.e2r = dd1;
  a.e1i = a.e2i = dd1 + static_cast<size_t>(nd) * L;
  a.e3r = dd3;
  a.e3i = dd3 + static_cast<size_t>(nd) * Q;
  a.slot = dslK;
  a.out = dK;
  MT_TRY(sis::launch_fsm_tables(a, stream));
  a.m1 = a.m2 = a.m3 = n;
  a.e1r = a.e2r = dv1;
  a.e1i = a.e2i = dv1 + static_cast<size_t>(n) * L;
  a.e3r = dv3;
  a.e3i = dv3 + static_cast<size_t>(n) * Q;
  a.slot = dslF;
  for (int s = 0; s < 2; ++s) {
    a.X = dS[s];
    a.out = dF[s];
    MT_TRY(sis::launch_fsm_tables(a, stream));
  }
  // collision frequencies nu_a = scale sum_b (C_ab / 4 b0) (4 b0 F^-1[beta F f_b]) and nubar
  std::vector<double> nuu(2 * n3);
  MT_TRY(hipStreamSynchronize(stream));
  for (int s = 0; s < 2; ++s)
    MT_TRY(hipMemcpy(nuu.data() + s * n3, dF[s] + 2 * D * n3, n3 * 8, hipMemcpyDeviceToHost));
  const double inv4b0 = 1.0 / (4.0 * t.b0);
  t.nu.assign(2 * n3, 0.0);
  for (int s = 0; s < 2; ++s) {
    double nb = 0.0;
    for (int64_t i = 0; i < n3; ++i) {
      const double v = t.scale * inv4b0 * (t.C[s][0] * nuu[i] + t.C[s][1] * nuu[n3 + i]);
      t.nu[s * n3 + i] = v;
      nb += p->w * v * t.feq[s * n3 + i];
    }
    t.nubar[s] = nb / t.chi[s];
  }
  auto block = [&](int ra, int cb) { return p->op + static_cast<size_t>(ra) * n3 * ndof + static_cast<size_t>(cb) * n3; };
  // loss terms: block (a, b) -= scale C_ab f_a(i) beta_r(i - j)
  for (int ra = 0; ra < 2; ++ra)
    for (int cb = 0; cb < 2; ++cb)
      MT_TRY(sis::launch_assemble(n, 0, nullptr, nullptr, p->feq + static_cast<size_t>(ra) * n3,
                                  t.scale * t.C[ra][cb] * inv4b0, dK + 2 * D * nd3, block(ra, cb), ndof, 1, stream));
  // equal-mass pairs: closed-form phi terms with the shared kernels Psi_p, Phi_p
  double* dXw = nullptr;
  int* dsrc = nullptr;
  double* dsw = nullptr;
  MT_TRY(al(&dXw, static_cast<size_t>(D) * n3));
  std::vector<int> srcv(D);
  std::vector<double> swv(D);
  int* dsrcbuf = nullptr;
  double* dswbuf = nullptr;
  MT_TRY(dmalloc(&dsrcbuf, D));
  owned.push_back(dsrcbuf);
  MT_TRY(al(&dswbuf, D));
  dsrc = dsrcbuf;
  dsw = dswbuf;
  for (int ra = 0; ra < 2; ++ra)
    for (int cb = 0; cb < 2; ++cb) {
      if (t.kappa[ra][cb] != 0.0) continue;
      for (int kind = 0; kind < 2; ++kind) {
        // kind 0: Q+_ab(f_a, h_b) -> block (a, b), X = phi-field of f_a, Y = Psi_p
        // kind 1: Q+_ab(h_a, f_b) -> block (a, a), X = psi-field of f_b, Y = Phi_p
        for (int q = 0; q < D; ++q) {
          srcv[q] = kind == 0 ? q : D + q;
          swv[q] = t.scale * t.C[ra][cb] * t.W[q];
        }
        MT_TRY(hipStreamSynchronize(stream));   // the previous round has consumed dXw, dsrc, dsw
        MT_TRY(hipMemcpyAsync(dsrc, srcv.data(), D * sizeof(int), hipMemcpyHostToDevice, stream));
        MT_TRY(hipMemcpyAsync(dsw, swv.data(), D * sizeof(double), hipMemcpyHostToDevice, stream));
        MT_TRY(sis::launch_scale_rows(D, n3, kind == 0 ? dF[ra] : dF[cb], dsrc, dsw, dXw, stream));
        MT_TRY(sis::launch_assemble(n, D, dXw, dK + (kind == 0 ? 0 : static_cast<size_t>(D) * nd3), nullptr, 0.0,
                                    nullptr, kind == 0 ? block(ra, cb) : block(ra, ra), ndof, 1, stream));
      }
    }
  // unequal-mass pairs: every (direction p, rho node r, sign) is a term with shifts
  // zp = 2mu rho e_p / dv (of the f-argument) and zm = -kappa rho e_p / dv (of the psi-argument)
  const int items = D * t.m_rho * 2;
  const int CH = std::min(items, 512);
  double *dXc = nullptr, *dYc = nullptr, *dE1 = nullptr, *dE2 = nullptr, *dE3 = nullptr, *dSp = nullptr;
  double *dz = nullptr, *dzp = nullptr, *dwt = nullptr, *dscl = nullptr, *dones = nullptr;
  int *dmrow = nullptr, *dslot = nullptr, *dbv = nullptr, *dbd = nullptr;
  bool any_cross = false;
  for (int ra = 0; ra < 2; ++ra)
    for (int cb = 0; cb < 2; ++cb) any_cross = any_cross || t.kappa[ra][cb] != 0.0;
  if (any_cross) {
    MT_TRY(al(&dXc, static_cast<size_t>(CH) * n3));
    MT_TRY(al(&dYc, static_cast<size_t>(CH) * nd3));
    MT_TRY(al(&dE1, 2 * static_cast<size_t>(CH) * nd * L));
    MT_TRY(al(&dE2, 2 * static_cast<size_t>(CH) * nd * L));
    MT_TRY(al(&dE3, 2 * static_cast<size_t>(CH) * nd * Q));
    MT_TRY(al(&dSp, static_cast<size_t>(CH) * 3 * nd));
    MT_TRY(al(&dz, 6 * static_cast<size_t>(CH)));
    MT_TRY(al(&dzp, 3 * static_cast<size_t>(CH)));
    MT_TRY(al(&dwt, static_cast<size_t>(CH)));
    MT_TRY(al(&dscl, static_cast<size_t>(CH)));
    int* tmp = nullptr;
    MT_TRY(dmalloc(&tmp, CH));
    owned.push_back(tmp);
    dmrow = tmp;
    MT_TRY(dmalloc(&tmp, CH));
    owned.push_back(tmp);
    dslot = tmp;
    std::vector<int> bv(n), bd(nd), sl(CH);
    for (int i = 0; i < n; ++i) bv[i] = 2 * i + 1 - n;
    for (int i = 0; i < nd; ++i) bd[i] = 2 * (i - (n - 1));
    for (int i = 0; i < CH; ++i) sl[i] = i;
    MT_TRY(upload(&dbv, bv, stream));
    owned.push_back(dbv);
    MT_TRY(upload(&dbd, bd, stream));
    owned.push_back(dbd);
    MT_TRY(hipMemcpyAsync(dslot, sl.data(), CH * sizeof(int), hipMemcpyHostToDevice, stream));
  }
  double* dprof[2] = {nullptr, nullptr};
  for (int s = 0; s < 2 && any_cross; ++s) MT_TRY(ua(&dprof[s], t.prof[s]));
  const std::vector<double> ones(CH, 1.0);
  if (any_cross) MT_TRY(ua(&dones, ones));
  std::vector<double> zv(6 * static_cast<size_t>(CH)), zp(3 * static_cast<size_t>(CH)), wv(CH), scv(CH);
  std::vector<int> mr(CH);
  const double invP3 = 1.0 / (static_cast<double>(P) * P * P);
  for (int ra = 0; ra < 2; ++ra)
    for (int cb = 0; cb < 2; ++cb) {
      if (t.kappa[ra][cb] == 0.0) continue;
      const double tm = t.two_mu[ra][cb], kap = t.kappa[ra][cb];
      for (int kind = 0; kind < 2; ++kind)
        for (int q0 = 0; q0 < items; q0 += CH) {
          const int nt = std::min(CH, items - q0);
          MT_TRY(hipStreamSynchronize(stream));   // the previous chunk (and its copies) are done
          for (int i = 0; i < nt; ++i) {
            const int q = q0 + i;                  // q = (p m_rho + r) 2 + sign
            const int sgn = (q & 1) ? -1 : 1, pr = q >> 1, pp = pr / t.m_rho, r = pr % t.m_rho;
            const double rho = sgn * t.rho[r];
            const double e[3] = {t.ex[pp], t.ey[pp], t.ez[pp]};
            for (int k = 0; k < 3; ++k) {
              zv[6 * i + k] = tm * rho * e[k] / t.dv;        // zp
              zv[6 * i + 3 + k] = -kap * rho * e[k] / t.dv;  // zm
            }
            wv[i] = t.scale * t.C[ra][cb] * t.W[pp] * t.wr[r] * t.rho[r];
            mr[i] = 2 * pp;                        // psi_p
            scv[i] = kind == 0 ? invP3 : wv[i] * invP3;
            for (int k = 0; k < 3; ++k) zp[3 * i + k] = zv[6 * i + k];
          }
          MT_TRY(hipMemcpyAsync(dz, zv.data(), 6 * nt * 8, hipMemcpyHostToDevice, stream));
          MT_TRY(hipMemcpyAsync(dwt, wv.data(), nt * 8, hipMemcpyHostToDevice, stream));
          MT_TRY(hipMemcpyAsync(dscl, scv.data(), nt * 8, hipMemcpyHostToDevice, stream));
          MT_TRY(hipMemcpyAsync(dmrow, mr.data(), nt * sizeof(int), hipMemcpyHostToDevice, stream));
          const bool kern = kind == 0;               // shifted transform on the difference grid
          const int m = kern ? nd : n;
          const int* base = kern ? dbd : dbv;
          // per-term factor matrices with the psi-argument shift zm (axes 1, 2, 3)
          MT_TRY(sis::launch_fsm_shift_factors(nt, m, L, -(P / 2 - 1), 0, base, dz + 3, 6, P, dE1,
                                               dE1 + static_cast<size_t>(nt) * m * L, stream));
          MT_TRY(sis::launch_fsm_shift_factors(nt, m, L, -(P / 2 - 1), 0, base, dz + 4, 6, P, dE2,
                                               dE2 + static_cast<size_t>(nt) * m * L, stream));
          MT_TRY(sis::launch_fsm_shift_factors(nt, m, Q, 0, 1, base, dz + 5, 6, P, dE3,
                                               dE3 + static_cast<size_t>(nt) * m * Q, stream));
          sis::FsmTableArgs b{};
          b.d = d;
          b.m1 = b.m2 = b.m3 = m;
          b.e1r = dE1;
          b.e1i = dE1 + static_cast<size_t>(nt) * m * L;
          b.e2r = dE2;
          b.e2i = dE2 + static_cast<size_t>(nt) * m * L;
          b.e3r = dE3;
          b.e3i = dE3 + static_cast<size_t>(nt) * m * Q;
          b.e1_ts = b.e2_ts = static_cast<int64_t>(m) * L;
          b.e3_ts = static_cast<int64_t>(m) * Q;
          b.mult = dmult;
          b.mrow = dmrow;
          b.X = kern ? nullptr : dS[cb];
          b.slot = dslot;
          b.scale = dscl;
          b.out = kern ? dYc : dXc;
          b.t0 = 0;
          b.nt = nt;
          MT_TRY(sis::launch_fsm_tables(b, stream));
          // the separable factor: kind 0 the shifted band-limited f_a on the nodes (x w), kind 1
          // the shifted band-limited delta on the difference grid
          MT_TRY(hipMemcpyAsync(dzp, zp.data(), 3 * nt * 8, hipMemcpyHostToDevice, stream));
          if (kern) {
            MT_TRY(sis::launch_band_profiles(nt, n, 0, dprof[ra], n, dzp, P, dSp, stream));
            MT_TRY(sis::launch_separable(nt, n, dSp, dwt, dXc, stream));
          } else {
            MT_TRY(sis::launch_band_profiles(nt, nd, -(n - 1), nullptr, 0, dzp, P, dSp, stream));
            MT_TRY(sis::launch_separable(nt, nd, dSp, dones, dYc, stream));
          }
          MT_TRY(sis::launch_assemble(n, nt, dXc, dYc, nullptr, 0.0, nullptr,
                                      kind == 0 ? block(ra, cb) : block(ra, ra), ndof, 1, stream));
        }
    }
  MT_TRY(hipStreamSynchronize(stream));
  cleanup();
#undef MT_TRY
  return SIS_OK;
}

sis_status create_mix_plan(const sis_velocity_desc* desc, hipStream_t stream, sis_plan_t* out) {
  auto t0 = std::chrono::steady_clock::now();
  const sis::MixDesc md = mix_desc(desc);
  sis::MixTables t;
  std::string err;
  // the transforms of the tables run on the device when the table kernel's LDS holds the
  // modes; otherwise the host planner builds them
  bool device_tables;
  {
    const int nn = md.n_v, np = md.n_pad > 0 ? md.n_pad : 2 * md.n_v;
    sis::FsmDims dd{};
    dd.n = nn;
    dd.P = np;
    dd.L = np - 1;
    dd.Q = np / 2;
    device_tables = sis::fsm_tables_fit(dd, 2 * nn - 1);
  }
  if (!(device_tables ? sis::build_mix_grid(md, t, err) : sis::build_mix_base(md, t, err)))
    return fail(SIS_E_INVALID, "%s", err.c_str());
  sis_plan* p = new sis_plan();
  HIP_TRY(hipGetDevice(&p->device));
  const int n = t.n, n3 = t.n3, D = t.D, nd3 = t.nd3;
  p->n = n;
  p->n3 = n3;
  p->np = t.np;
  p->D = D;
  p->m_angle = desc->m_angle;
  p->lv = t.lv;
  p->dv = t.dv;
  p->w = t.dv * t.dv * t.dv;
  p->b0 = t.b0;
  p->R = t.R;
  p->alpha = 1.0;
  p->gamma = 0.0;
  p->nsp = 2;
  p->ndof = 2 * n3;
  set_layout(p, 0);
  for (int s = 0; s < 2; ++s) {
    p->mass_ratio[s] = t.a[s];
    p->chi[s] = t.chi[s];
  }
  p->flow_factor = std::sqrt(t.mbar_over_mA);
  p->visc_ratio = sis::mix_viscosity_ratio(md.mass, md.diam, md.chi);
  p->h_v1d = t.v1d;
  p->h_feq = t.feq;
  const int64_t ndof = p->ndof;
  const int chunk = 64;  // (direction, rho) items per host/device round
  const size_t tabX = static_cast<size_t>(std::max(2 * chunk, D)) * n3;
  const size_t tabY = static_cast<size_t>(std::max(2 * chunk, 2 * D)) * nd3;
  double *dX = nullptr, *dY = nullptr, *dbr = nullptr;
  auto cleanup = [&]() { dfree(dX); dfree(dY); dfree(dbr); };
#define MIX_TRY(expr)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) {                                                                  \
      (void)hipStreamSynchronize(stream);                                                    \
      cleanup();                                                                             \
      delete p;                                                                              \
      return fail(e_ == hipErrorOutOfMemory ? SIS_E_OOM : SIS_E_DEVICE, "%s: %s", #expr,      \
                  hipGetErrorString(e_));                                                    \
    }                                                                                        \
  } while (0)
  MIX_TRY(dmalloc(&p->op, static_cast<size_t>(ndof) * ndof));
  MIX_TRY(dmalloc(&p->v1d, n));
  MIX_TRY(dmalloc(&p->feq, 2 * n3));
  MIX_TRY(dmalloc(&p->nu, 2 * n3));
  MIX_TRY(dmalloc(&p->Kc, 2 * ndof));
  MIX_TRY(dmalloc(&p->gram_inv, 25));
  MIX_TRY(hipMemcpyAsync(p->v1d, t.v1d.data(), n * 8, hipMemcpyHostToDevice, stream));
  MIX_TRY(hipMemcpyAsync(p->feq, t.feq.data(), 2 * n3 * 8, hipMemcpyHostToDevice, stream));
  MIX_TRY(hipMemsetAsync(p->op, 0, static_cast<size_t>(ndof) * ndof * 8, stream));
  if (device_tables) {
    if (sis_status st = mix_tables_device(p, t, stream)) {
      cleanup();
      delete p;
      return st;
    }
  } else {
    MIX_TRY(dmalloc(&dX, tabX));
    MIX_TRY(dmalloc(&dY, tabY));
    MIX_TRY(dmalloc(&dbr, nd3));
    MIX_TRY(hipMemcpyAsync(dbr, t.beta_r.data(), nd3 * 8, hipMemcpyHostToDevice, stream));
    auto block = [&](int a, int b) { return p->op + static_cast<size_t>(a) * n3 * ndof + static_cast<size_t>(b) * n3; };
    // loss terms: block (a, b) -= scale C_ab f_a(i) beta_r(i - j)
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b)
        MIX_TRY(sis::launch_assemble(n, 0, nullptr, nullptr, p->feq + static_cast<size_t>(a) * n3,
                                     t.scale * t.C[a][b], dbr, block(a, b), ndof, 1, stream));
    // equal-mass pairs: closed-form phi terms with the shared kernels Psi_p, Phi_p
    MIX_TRY(hipMemcpyAsync(dY, t.Psi.data(), static_cast<size_t>(D) * nd3 * 8, hipMemcpyHostToDevice, stream));
    MIX_TRY(hipMemcpyAsync(dY + static_cast<size_t>(D) * nd3, t.Phi.data(), static_cast<size_t>(D) * nd3 * 8,
                           hipMemcpyHostToDevice, stream));
    std::vector<double> hx(tabX), hy;
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) {
        if (t.kappa[a][b] != 0.0) continue;
        for (int kind = 0; kind < 2; ++kind) {
          // kind 0: Q+_ab(f_a, h_b) -> block (a, b), X = phi-field of f_a, Y = Psi
          // kind 1: Q+_ab(h_a, f_b) -> block (a, a), X = psi-field of f_b, Y = Phi
          const std::vector<double>& F = kind == 0 ? t.Fphi[a] : t.Fpsi[b];
          MIX_TRY(hipStreamSynchronize(stream));
          for (int q = 0; q < D; ++q) {
            const double sc = t.scale * t.C[a][b] * t.W[q];
            for (int i = 0; i < n3; ++i) hx[static_cast<size_t>(q) * n3 + i] = sc * F[static_cast<size_t>(q) * n3 + i];
          }
          MIX_TRY(hipMemcpyAsync(dX, hx.data(), static_cast<size_t>(D) * n3 * 8, hipMemcpyHostToDevice, stream));
          MIX_TRY(sis::launch_assemble(n, D, dX, dY + (kind == 0 ? 0 : static_cast<size_t>(D) * nd3), nullptr, 0.0,
                                       nullptr, kind == 0 ? block(a, b) : block(a, a), ndof, 1, stream));
        }
      }
    // unequal-mass pairs: rho-quadrature terms, in chunks
    hy.resize(static_cast<size_t>(2 * chunk) * nd3);
    for (int a = 0; a < 2; ++a)
      for (int b = 0; b < 2; ++b) {
        if (t.kappa[a][b] == 0.0) continue;
        const int items = D * t.m_rho;
        for (int kind = 0; kind < 2; ++kind)
          for (int q0 = 0; q0 < items; q0 += chunk) {
            const int q1 = std::min(items, q0 + chunk);
            sis::build_mix_cross_terms(t, a, b, kind, q0, q1, hx.data(), hy.data(), md.n_threads);
            MIX_TRY(hipStreamSynchronize(stream));  // previous chunk has consumed dX, dY
            const size_t T = 2 * static_cast<size_t>(q1 - q0);
            MIX_TRY(hipMemcpyAsync(dX, hx.data(), T * n3 * 8, hipMemcpyHostToDevice, stream));
            MIX_TRY(hipMemcpyAsync(dY, hy.data(), T * nd3 * 8, hipMemcpyHostToDevice, stream));
            MIX_TRY(sis::launch_assemble(n, static_cast<int>(T), dX, dY, nullptr, 0.0, nullptr,
                                         kind == 0 ? block(a, b) : block(a, a), ndof, 1, stream));
          }
      }
  }
  for (int s = 0; s < 2; ++s) p->nubar_s[s] = t.nubar[s];
  p->nubar = t.nubar[0];
  p->h_nu = t.nu;
  MIX_TRY(hipMemcpyAsync(p->nu, t.nu.data(), 2 * n3 * 8, hipMemcpyHostToDevice, stream));
  // restriction to the stored parity class (odd in v3 / even in v2)
  MIX_TRY(hipStreamSynchronize(stream));
  set_layout(p, desc->parity);
  if (sis_status st = apply_parity(p, stream)) {
    cleanup();
    delete p;
    return st;
  }
  if (sis_status st = build_velocity_tables(p, stream)) {
    cleanup();
    delete p;
    return st;
  }
  // correction shapes 2 (m_s/m_A) v3 f_s and their L+ (two-row contraction)
  std::vector<double> corr(2 * static_cast<size_t>(ndof), 0.0);
  for (int s = 0; s < 2; ++s) {
    double cu = 0.0, cq = 0.0;
    for (int i0 = 0; i0 < n; ++i0)
      for (int i1 = 0; i1 < n; ++i1)
        for (int i2 = 0; i2 < n; ++i2) {
          const int i = (i0 * n + i1) * n + i2;
          const double v1 = t.v1d[i0], v2 = t.v1d[i1], v3 = t.v1d[i2];
          const double c = 2.0 * t.a[s] * v3 * t.feq[static_cast<size_t>(s) * n3 + i];
          corr[static_cast<size_t>(s) * ndof + static_cast<size_t>(s) * n3 + i] = c;
          cu += p->w * v3 * c;
          cq += p->w * (t.a[s] * (v1 * v1 + v2 * v2 + v3 * v3) - 2.5) * v3 * c;
        }
    p->cU_s[s] = cu / t.chi[s];
    p->cq_s[s] = cq;
  }
  p->cU = p->cU_s[0];
  p->cq = p->cq_s[0];
  if (p->parity) corr = restrict_rows(p, corr.data(), 4);  // [2 shapes][2 species] -> stored rows
  MIX_TRY(hipStreamSynchronize(stream));
  if (!dX) MIX_TRY(dmalloc(&dX, corr.size()));
  MIX_TRY(hipMemcpyAsync(dX, corr.data(), corr.size() * 8, hipMemcpyHostToDevice, stream));
  {
    sis::GemmArgs g{};
    g.precision = 0;
    g.X = dX;
    g.op64 = p->op;
    g.acc = p->Kc;
    g.M = 2;
    g.N = static_cast<int>(p->ndof);
    g.K = static_cast<int>(p->ndof);
    g.splits = 1;
    g.tile = 1;
    MIX_TRY(sis::launch_gemm(g, stream));
  }
  MIX_TRY(hipStreamSynchronize(stream));
  cleanup();
#undef MIX_TRY
  auto t1 = std::chrono::steady_clock::now();
  p->host_s = 0.0;
  p->dev_s = std::chrono::duration<double>(t1 - t0).count();
  *out = p;
  g_err.clear();
  return SIS_OK;
}

}  // namespace

extern "C" {

const char* sis_last_error(void) { return g_err.c_str(); }
int32_t sis_version(void) { return 100; }

sis_status sis_host_tables(const sis_velocity_desc* desc, double* feq, double* nu, double* A,
                           double* B, double* b0, double* nubar) {
  sis_status st = validate_desc(desc);
  if (st) return st;
  if (desc->grid == SIS_GRID_POLAR) return fail(SIS_E_UNSUPPORTED, "host tables are for the Cartesian grids");
  std::string err;
  if (desc->n_species == 2) {
    if (A || B) return fail(SIS_E_UNSUPPORTED, "A/B fields are not reported for mixtures");
    sis::MixTables mt;
    if (!sis::build_mix_base(mix_desc(desc), mt, err)) return fail(SIS_E_INVALID, "%s", err.c_str());
    if (feq) std::memcpy(feq, mt.feq.data(), mt.feq.size() * sizeof(double));
    if (nu) std::memcpy(nu, mt.nu.data(), mt.nu.size() * sizeof(double));
    if (b0) *b0 = mt.b0;
    if (nubar) { nubar[0] = mt.nubar[0]; nubar[1] = mt.nubar[1]; }
    g_err.clear();
    return SIS_OK;
  }
  sis::HostTables t;
  if (!sis::build_host_tables(table_desc(desc), false, t, err)) return fail(SIS_E_INVALID, "%s", err.c_str());
  if (feq) std::memcpy(feq, t.feq.data(), t.n3 * sizeof(double));
  if (nu) std::memcpy(nu, t.nu.data(), t.n3 * sizeof(double));
  if (A) std::memcpy(A, t.A.data(), t.A.size() * sizeof(double));
  if (B) std::memcpy(B, t.B.data(), t.B.size() * sizeof(double));
  if (b0) *b0 = t.b0;
  if (nubar) *nubar = t.nubar;
  g_err.clear();
  return SIS_OK;
}

}  // extern "C"

namespace {

// Polar velocity grid (tube): host tables, then the operator assembled on the device from
// the half-space Cartesian modes l (pair weight s_l = 2, 1 for l = 0, over n_pad^3):
//   fhat_l = sum_j w'_j f_eq 4 cos cos cos            (w' = w_base / dv_c^3)
//   AB[i][t] = sum_l cos(xi_l . v_i) m_t(l) fhat_l s_l     (F^-1 of m_t F f_eq at the nodes)
//   a_t(i): 4 b0 W_p B_p(i) with psi_p, 4 b0 W_p A_p(i) with phi_p, -f_eq(i) with beta
//   C[i][l] = sum_t a_t(i) m_t(l);  op = sum_l C[i][l] s_l [cos_i c_j(l) + sin_i s_j(l)]
// where c_j, s_j are the cos / sin parts of sum over the four mirror images of node j of
// sign w'_j e^{i xi.v} (sign -1 for v_z -> -v_z).  Three FP64 MFMA contractions.
sis_status create_polar_plan(const sis_velocity_desc* desc, hipStream_t stream, sis_plan_t* out) {
  auto t0 = std::chrono::steady_clock::now();
  sis::PolarDesc pd;
  pd.n_vr = desc->n_vr;
  pd.n_th = desc->n_th;
  pd.n_vz = desc->n_vz;
  pd.vr_max = desc->vr_max;
  pd.vz_max = desc->l_v;
  pd.n_pad = desc->n_pad;
  pd.l_pad = desc->l_pad;
  pd.m_angle = desc->m_angle;
  pd.n_threads = desc->n_threads;
  sis::PolarTables t;
  std::string err;
  if (!sis::build_polar_tables(pd, t, err)) return fail(SIS_E_INVALID, "%s", err.c_str());
  auto t1 = std::chrono::steady_clock::now();
  sis_plan* p = new sis_plan();
  HIP_TRY(hipGetDevice(&p->device));
  const int nv = t.nv, nm = t.nm, Tp = t.Tp, D = t.D;
  p->polar = true;
  p->n = 0;
  p->n3 = nv;
  p->nv = nv;
  p->ndof = nv;
  p->nsp = 1;
  p->np = t.np;
  p->D = D;
  p->m_angle = desc->m_angle;
  p->lv = desc->l_v;
  p->dv = t.dvc;
  p->b0 = t.b0;
  p->R = t.R;
  p->n_vr = t.n_vr;
  p->n_th = t.n_th;
  p->n_vz = t.n_vz;
  p->dth = 3.14159265358979323846 / t.n_th;
  p->alpha = 1.0;
  p->gamma = 0.0;
  std::vector<double> wn(nv), wf(nv), wp(nv), cth(t.n_th), sth(t.n_th);
  const double dvc3 = t.dvc * t.dvc * t.dvc;
  for (int j = 0; j < nv; ++j) {
    wn[j] = 4.0 * t.wbase[j];
    wp[j] = t.wbase[j] / dvc3;
    wf[j] = wp[j] * t.feq[j];
  }
  for (int k = 0; k < t.n_th; ++k) {
    cth[k] = std::cos(t.th[k]);
    sth[k] = std::sin(t.th[k]);
  }
  // coefficient sources: psi_p terms take B_p = column D + p, phi_p terms take A_p = column p
  std::vector<int32_t> srcT(Tp, -2);
  std::vector<double> cT(Tp, 0.0), sc(nm);
  for (int q = 0; q < D; ++q) {
    srcT[q] = D + q;
    cT[q] = 4.0 * t.b0 * t.W[q];
    srcT[D + q] = q;
    cT[D + q] = 4.0 * t.b0 * t.W[q];
  }
  srcT[2 * D] = -1;
  const double inp3 = 1.0 / (static_cast<double>(t.np) * t.np * t.np);
  for (int m = 0; m < nm; ++m) sc[m] = t.pair[m] * inp3;
  double *dxi = nullptr, *dsc = nullptr, *dwf = nullptr, *dwp = nullptr, *dfh = nullptr, *dmt = nullptr,
         *dterm = nullptr, *dAB = nullptr, *daT = nullptr, *dcT = nullptr, *bufA = nullptr, *bufB = nullptr,
         *bufC = nullptr, *dcorr = nullptr;
  int32_t* dsrc = nullptr;
  auto cleanup = [&]() {
    dfree(dxi); dfree(dsc); dfree(dwf); dfree(dwp); dfree(dfh); dfree(dmt); dfree(dterm); dfree(dAB);
    dfree(daT); dfree(dcT); dfree(bufA); dfree(bufB); dfree(bufC); dfree(dcorr); dfree(dsrc);
  };
#define POL_TRY(expr)                                                                          \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess) {                                                                    \
      cleanup();                                                                               \
      delete p;                                                                                \
      return fail(e_ == hipErrorOutOfMemory ? SIS_E_OOM : SIS_E_DEVICE, "%s: %s", #expr,        \
                  hipGetErrorString(e_));                                                      \
    }                                                                                          \
  } while (0)
  POL_TRY(upload(&p->vnode, t.vnode, stream));
  POL_TRY(upload(&p->wnode, wn, stream));
  POL_TRY(upload(&p->vtab, t.vnode, stream));
  POL_TRY(upload(&p->wtab, wn, stream));
  POL_TRY(upload(&p->feq, t.feq, stream));
  POL_TRY(upload(&p->d_vr, t.vr, stream));
  POL_TRY(upload(&p->d_cth, cth, stream));
  POL_TRY(upload(&p->d_sth, sth, stream));
  POL_TRY(dmalloc(&p->nu, nv));
  POL_TRY(dmalloc(&p->op, static_cast<size_t>(nv) * nv));
  POL_TRY(dmalloc(&p->Kc, nv));
  POL_TRY(dmalloc(&p->gram_inv, 25));
  POL_TRY(dmalloc(&p->v1d, 1));
  POL_TRY(upload(&dxi, t.xi, stream));
  POL_TRY(upload(&dsc, sc, stream));
  POL_TRY(upload(&dwf, wf, stream));
  POL_TRY(upload(&dwp, wp, stream));
  POL_TRY(upload(&dsrc, srcT, stream));
  POL_TRY(upload(&dcT, cT, stream));
  POL_TRY(dmalloc(&dfh, nm));
  POL_TRY(sis::launch_polar_fhat(nm, dxi, nv, p->vnode, dwf, dfh, stream));
  // fields A_p, B_p, nu at the nodes
  POL_TRY(upload(&dmt, t.mt_tm, stream));
  POL_TRY(dmalloc(&dterm, static_cast<size_t>(Tp) * nm));
  POL_TRY(sis::launch_polar_scale_terms(Tp, nm, dmt, dfh, dsc, dterm, stream));
  POL_TRY(dmalloc(&bufA, static_cast<size_t>(nv) * nm));
  POL_TRY(sis::launch_polar_cos(nv, nm, p->vnode, dxi, bufA, stream));
  POL_TRY(dmalloc(&dAB, static_cast<size_t>(nv) * Tp));
  sis::GemmArgs g{};
  g.precision = 0;
  g.splits = 1;
  g.tile = 0;
  g.X = bufA;
  g.op64 = dterm;
  g.acc = dAB;
  g.M = nv;
  g.N = Tp;
  g.K = nm;
  POL_TRY(sis::launch_gemm(g, stream));
  POL_TRY(dmalloc(&daT, static_cast<size_t>(nv) * Tp));
  POL_TRY(sis::launch_polar_coef(nv, Tp, dAB, dsrc, dcT, p->feq, 2 * D, daT, p->nu, stream));
  // C = a m^T into bufA, then the cos / sin factors of both sides and the contraction over modes
  POL_TRY(hipStreamSynchronize(stream));
  dfree(dmt);
  dmt = nullptr;
  POL_TRY(upload(&dmt, t.mt_mm, stream));
  g.X = daT;
  g.op64 = dmt;
  g.acc = bufA;
  g.M = nv;
  g.N = nm;
  g.K = Tp;
  POL_TRY(sis::launch_gemm(g, stream));
  POL_TRY(dmalloc(&bufB, static_cast<size_t>(nv) * 2 * nm));
  POL_TRY(dmalloc(&bufC, static_cast<size_t>(nv) * 2 * nm));
  POL_TRY(sis::launch_polar_xc(nv, nm, p->vnode, dxi, dsc, bufA, bufB, stream));
  POL_TRY(sis::launch_polar_op2(nv, nm, p->vnode, dxi, dwp, bufC, stream));
  g.X = bufB;
  g.op64 = bufC;
  g.acc = p->op;
  g.M = nv;
  g.N = nv;
  g.K = 2 * nm;
  POL_TRY(sis::launch_gemm(g, stream));
  // host copies of f_eq and nu; nubar, correction moments, Kc = L+(2 v_z f_eq)
  p->h_feq = t.feq;
  p->h_nu.assign(nv, 0.0);
  POL_TRY(hipMemcpyAsync(p->h_nu.data(), p->nu, nv * 8, hipMemcpyDeviceToHost, stream));
  POL_TRY(hipStreamSynchronize(stream));
  std::vector<double> corr(nv);
  for (int j = 0; j < nv; ++j) {
    const double v1 = t.vnode[j], v2 = t.vnode[nv + j], v3 = t.vnode[2 * nv + j];
    corr[j] = 2.0 * v3 * t.feq[j];
    p->nubar += wn[j] * p->h_nu[j] * t.feq[j];
    p->cU += wn[j] * v3 * corr[j];
    p->cq += wn[j] * (v1 * v1 + v2 * v2 + v3 * v3 - 2.5) * v3 * corr[j];
  }
  p->nubar_s[0] = p->nubar;
  p->cU_s[0] = p->cU;
  p->cq_s[0] = p->cq;
  POL_TRY(upload(&dcorr, corr, stream));
  g.X = dcorr;
  g.op64 = p->op;
  g.acc = p->Kc;
  g.M = 1;
  g.N = nv;
  g.K = nv;
  g.tile = 1;
  if (nv % 2) {
    cleanup();
    delete p;
    return fail(SIS_E_INVALID, "polar grid: n_vr n_th n_vz must be even");
  }
  POL_TRY(sis::launch_gemm(g, stream));
  POL_TRY(hipStreamSynchronize(stream));
  cleanup();
#undef POL_TRY
  auto t2 = std::chrono::steady_clock::now();
  p->host_s = std::chrono::duration<double>(t1 - t0).count();
  p->dev_s = std::chrono::duration<double>(t2 - t1).count();
  *out = p;
  g_err.clear();
  return SIS_OK;
}

// Factor matrices and f_eq fields of the per-cell transform path (one-gas Cartesian plan
// with the given parity storage).  dX holds the full-grid fields of the assembly,
// [B_p; A_p] already scaled by 4 b0 W_p; dfeq the full-grid f_eq.
sis_status build_fsm_static(sis_plan* p, int parity, const double* dX, const double* dfeq, hipStream_t stream) {
  sis::FsmDims d{};
  d.n = p->n;
  d.P = p->np;
  d.L = p->np - 1;
  d.Q = p->np / 2;
  d.n2 = parity == 2 ? p->n / 2 : p->n;
  d.n3 = parity >= 1 ? p->n / 2 : p->n;
  d.nv = d.n * d.n2 * d.n3;
  d.T = 2 * p->D + 1;
  p->fsm_d = d;
  if (sis::fsm_unsupported(d)) return SIS_OK;   // sis_collide_fsm reports it
  const int n = d.n, P = d.P, L = d.L, Q = d.Q, half = P / 2 - 1;
  const int o2 = n - d.n2, o3 = n - d.n3;        // first stored node on axes 2, 3
  const size_t sz[6] = {static_cast<size_t>(L) * n, static_cast<size_t>(L) * d.n2, static_cast<size_t>(Q) * d.n3,
                        static_cast<size_t>(n) * L, static_cast<size_t>(d.n2) * L, static_cast<size_t>(d.n3) * Q};
  size_t total = 0;
  for (size_t k : sz) total += 2 * k;
  std::vector<double> fac(total);
  double* a[12];
  {
    size_t off = 0;
    for (int k = 0; k < 6; ++k) {
      a[2 * k] = fac.data() + off;
      a[2 * k + 1] = fac.data() + off + sz[k];
      off += 2 * sz[k];
    }
  }
  double c, sn;
  // forward: F1 [L][n], F2 [L][n2], F3 [Q][n3] with the images folded in
  for (int li = 0; li < L; ++li)
    for (int j = 0; j < n; ++j) {
      fsm_phase(li - half, j, n, P, c, sn);
      a[0][li * n + j] = c;
      a[1][li * n + j] = -sn;
    }
  for (int li = 0; li < L; ++li)
    for (int s2 = 0; s2 < d.n2; ++s2) {
      fsm_phase(li - half, s2 + o2, n, P, c, sn);
      const bool even = parity == 2;      // images v2 -> -v2 with sign +1
      a[2][li * d.n2 + s2] = even ? 2.0 * c : c;
      a[3][li * d.n2 + s2] = even ? 0.0 : -sn;
    }
  for (int l3 = 0; l3 < Q; ++l3)
    for (int s3 = 0; s3 < d.n3; ++s3) {
      fsm_phase(l3, s3 + o3, n, P, c, sn);
      const bool odd = parity >= 1;       // images v3 -> -v3 with sign -1
      a[4][l3 * d.n3 + s3] = odd ? 0.0 : c;
      a[5][l3 * d.n3 + s3] = odd ? -2.0 * sn : -sn;
    }
  // inverse: E1 [n][L], E2 [n2][L], E3 [n3][Q] (2 for l3 > 0: the conjugate half)
  for (int j = 0; j < n; ++j)
    for (int li = 0; li < L; ++li) {
      fsm_phase(li - half, j, n, P, c, sn);
      a[6][j * L + li] = c;
      a[7][j * L + li] = sn;
    }
  for (int s2 = 0; s2 < d.n2; ++s2)
    for (int li = 0; li < L; ++li) {
      fsm_phase(li - half, s2 + o2, n, P, c, sn);
      a[8][s2 * L + li] = c;
      a[9][s2 * L + li] = sn;
    }
  for (int s3 = 0; s3 < d.n3; ++s3)
    for (int l3 = 0; l3 < Q; ++l3) {
      fsm_phase(l3, s3 + o3, n, P, c, sn);
      const double w = l3 == 0 ? 1.0 : 2.0;
      a[10][s3 * Q + l3] = w * c;
      a[11][s3 * Q + l3] = w * sn;
    }
  HIP_TRY(upload(&p->fsm_fac, fac, stream));
  const double* dev[12];
  for (int k = 0; k < 12; ++k) dev[k] = p->fsm_fac + (a[k] - fac.data());
  p->fsm_f = sis::FsmFactors{dev[0], dev[1], dev[2], dev[3], dev[4], dev[5],
                             dev[6], dev[7], dev[8], dev[9], dev[10], dev[11]};
  // fields [T][nv] of the stored velocities: term 2p (multiplier psi_p) carries B_p, term
  // 2p + 1 (phi_p) carries A_p, the loss term -f_eq; all / P^3 (the inverse DFT's scale)
  std::vector<int> src(d.T);
  for (int q = 0; q < p->D; ++q) {
    src[2 * q] = q;
    src[2 * q + 1] = p->D + q;
  }
  src[2 * p->D] = -1;
  int* dsrc = nullptr;
  HIP_TRY(upload(&dsrc, src, stream));
  hipError_t e = dmalloc(&p->fsm_field, static_cast<size_t>(d.T) * d.nv);
  if (e == hipSuccess)
    e = sis::launch_fsm_gather(d, d.T, dX, dsrc, dfeq, 1.0 / (static_cast<double>(P) * P * P), p->fsm_field, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  dfree(dsrc);
  if (e != hipSuccess) return fail(SIS_E_DEVICE, "transform path tables: %s", hipGetErrorString(e));
  p->fsm_slab = sis::fsm_default_slab(d);
  p->fsm_ok = true;
  return SIS_OK;
}

// Directions, weights, the radial rule and the multipliers [T][Q][L][L] on the device.
sis_status build_fsm_multipliers(sis_plan* p, const sis_velocity_desc* desc, hipStream_t stream) {
  std::vector<double> ex, ey, ez, W;
  if (!sis::half_sphere_directions(desc->m_angle, ex, ey, ez, W)) return fail(SIS_E_NUMERIC, "directions");
  std::vector<double> dw(4 * p->D);
  for (int q = 0; q < p->D; ++q) {
    dw[3 * q] = ex[q];
    dw[3 * q + 1] = ey[q];
    dw[3 * q + 2] = ez[q];
    dw[3 * p->D + q] = W[q];
  }
  HIP_TRY(upload(&p->fsm_dirs, dw, stream));
  std::string err;
  if (!sis::radial_rule(table_desc(desc), p->fsm_rule, err)) return fail(SIS_E_NUMERIC, "%s", err.c_str());
  std::vector<double> rad;
  for (double x : p->fsm_rule.phi_x) rad.push_back(x);
  for (double x : p->fsm_rule.phi_w) rad.push_back(x);
  for (double x : p->fsm_rule.psi_x) rad.push_back(x);
  for (double x : p->fsm_rule.psi_w) rad.push_back(x);
  if (rad.empty()) rad.push_back(0.0);
  HIP_TRY(upload(&p->fsm_rad, rad, stream));
  sis::FsmDims d{};
  d.n = p->n;
  d.P = p->np;
  d.L = p->np - 1;
  d.Q = p->np / 2;
  d.n2 = d.n3 = p->n;
  d.nv = p->n3;
  d.T = 2 * p->D + 1;
  const int64_t qll = static_cast<int64_t>(d.Q) * d.L * d.L;
  HIP_TRY(dmalloc(&p->fsm_mult, static_cast<size_t>(d.T) * qll));
  sis::FsmMultArgs m{};
  m.d = d;
  m.D = p->D;
  m.b0 = p->b0;
  m.R = p->fsm_rule.R;
  m.Lp = p->fsm_rule.Lp;
  m.dirs = p->fsm_dirs;
  m.W = p->fsm_dirs + 3 * p->D;
  m.phi_closed = p->fsm_rule.phi_closed;
  m.psi_closed = p->fsm_rule.psi_closed;
  m.n_phi = static_cast<int>(p->fsm_rule.phi_x.size());
  m.n_psi = static_cast<int>(p->fsm_rule.psi_x.size());
  m.phi_x = p->fsm_rad;
  m.phi_w = p->fsm_rad + m.n_phi;
  m.psi_x = p->fsm_rad + 2 * m.n_phi;
  m.psi_w = p->fsm_rad + 2 * m.n_phi + m.n_psi;
  m.mult = p->fsm_mult;
  HIP_TRY(sis::launch_fsm_multipliers(m, stream));
  return SIS_OK;
}

// Tables of the assembly by the fast spectral method's own transforms on the device: with
// the multipliers m_t, the spectrum fhat of the zero-extended f_eq (separable, on the host)
// and pruned inverse DFTs onto the velocity nodes and the difference grid,
//   dX = [B_p; A_p] x 4 b0 W_p and nu  (fields F^-1[m_t fhat] on the n^3 nodes),
//   dY = [Psi_p; Phi_p] and beta_r     (kernels F^-1[m_t] on d in [-(n-1), n-1]^3).
sis_status build_tables_device(sis_plan* p, const sis::HostTables& t, double* dX, double* dY, hipStream_t stream) {
  const int n = t.n, P = t.np, L = P - 1, Q = P / 2, half = P / 2 - 1, D = t.D, T = 2 * D + 1, nd = t.nd;
  sis::FsmDims d{};
  d.n = n;
  d.P = P;
  d.L = L;
  d.Q = Q;
  d.n2 = d.n3 = n;
  d.nv = t.n3;
  d.T = T;
  // spectrum of the zero-extended f_eq: g(l) = sum_j e^{-v_j^2}/sqrt(pi) cos(xi_l v_j) per axis
  std::vector<double> gl(L), gq(Q);
  const double spi = std::sqrt(3.14159265358979323846);
  double c, sn;
  for (int li = 0; li < L; ++li) {
    double acc = 0.0;
    for (int j = 0; j < n; ++j) {
      fsm_phase(li - half, j, n, P, c, sn);
      acc += std::exp(-t.v1d[j] * t.v1d[j]) / spi * c;
    }
    gl[li] = acc;
  }
  for (int l3 = 0; l3 < Q; ++l3) gq[l3] = gl[l3 + half];
  std::vector<double> X(static_cast<size_t>(L) * 2 * Q * L, 0.0);
  for (int l1 = 0; l1 < L; ++l1)
    for (int l3 = 0; l3 < Q; ++l3)
      for (int l2 = 0; l2 < L; ++l2) X[(static_cast<size_t>(l1) * 2 * Q + l3) * L + l2] = gl[l1] * gq[l3] * gl[l2];
  // inverse factor matrices: velocity nodes (n) and the difference grid (2n - 1)
  auto factors = [&](int m, bool diff, std::vector<double>& e1, std::vector<double>& e3) {
    e1.assign(2 * static_cast<size_t>(m) * L, 0.0);
    e3.assign(2 * static_cast<size_t>(m) * Q, 0.0);
    for (int a = 0; a < m; ++a) {
      for (int li = 0; li < L; ++li) {
        const int l = li - half;
        if (diff) phase_q(2L * l * (a - (n - 1)), P, c, sn);
        else fsm_phase(l, a, n, P, c, sn);
        e1[static_cast<size_t>(a) * L + li] = c;
        e1[static_cast<size_t>(m) * L + static_cast<size_t>(a) * L + li] = sn;
      }
      for (int l3 = 0; l3 < Q; ++l3) {
        if (diff) phase_q(2L * l3 * (a - (n - 1)), P, c, sn);
        else fsm_phase(l3, a, n, P, c, sn);
        const double w = l3 == 0 ? 1.0 : 2.0;
        e3[static_cast<size_t>(a) * Q + l3] = w * c;
        e3[static_cast<size_t>(m) * Q + static_cast<size_t>(a) * Q + l3] = w * sn;
      }
    }
  };
  std::vector<double> ev1, ev3, ed1, ed3;
  factors(n, false, ev1, ev3);
  factors(nd, true, ed1, ed3);
  const double inv = 1.0 / (static_cast<double>(P) * P * P);
  std::vector<int> slotF(T), slotK(T);
  std::vector<double> scF(T), scK(T, inv);
  for (int q = 0; q < D; ++q) {
    slotF[2 * q + 1] = q;       // B_p = F^-1[phi_p fhat]
    slotF[2 * q] = D + q;       // A_p = F^-1[psi_p fhat]
    scF[2 * q] = scF[2 * q + 1] = 4.0 * t.b0 * t.W[q] * inv;
    slotK[2 * q] = q;           // Psi_p
    slotK[2 * q + 1] = D + q;   // Phi_p
  }
  slotF[2 * D] = slotK[2 * D] = 2 * D;   // nu, beta_r
  scF[2 * D] = inv;
  double *dXf = nullptr, *dv1 = nullptr, *dv3 = nullptr, *dd1 = nullptr, *dd3 = nullptr, *dsc = nullptr;
  int* dsl = nullptr;
  auto cleanup = [&]() { dfree(dXf); dfree(dv1); dfree(dv3); dfree(dd1); dfree(dd3); dfree(dsc); dfree(dsl); };
  std::vector<double> sc(scF);
  sc.insert(sc.end(), scK.begin(), scK.end());
  std::vector<int> sl(slotF);
  sl.insert(sl.end(), slotK.begin(), slotK.end());
  hipError_t e = upload(&dXf, X, stream);
  if (e == hipSuccess) e = upload(&dv1, ev1, stream);
  if (e == hipSuccess) e = upload(&dv3, ev3, stream);
  if (e == hipSuccess) e = upload(&dd1, ed1, stream);
  if (e == hipSuccess) e = upload(&dd3, ed3, stream);
  if (e == hipSuccess) e = upload(&dsc, sc, stream);
  if (e == hipSuccess) e = upload(&dsl, sl, stream);
  if (e == hipSuccess) {
    sis::FsmTableArgs a{};
    a.d = d;
    a.mult = p->fsm_mult;
    a.t0 = 0;
    a.nt = T;
    // fields on the velocity nodes
    a.m1 = a.m2 = a.m3 = n;
    a.e1r = a.e2r = dv1;
    a.e1i = a.e2i = dv1 + static_cast<size_t>(n) * L;
    a.e3r = dv3;
    a.e3i = dv3 + static_cast<size_t>(n) * Q;
    a.X = dXf;
    a.slot = dsl;
    a.scale = dsc;
    a.out = dX;
    e = sis::launch_fsm_tables(a, stream);
    // kernels on the difference grid
    a.m1 = a.m2 = a.m3 = nd;
    a.e1r = a.e2r = dd1;
    a.e1i = a.e2i = dd1 + static_cast<size_t>(nd) * L;
    a.e3r = dd3;
    a.e3i = dd3 + static_cast<size_t>(nd) * Q;
    a.X = nullptr;
    a.slot = dsl + T;
    a.scale = dsc + T;
    a.out = dY;
    if (e == hipSuccess) e = sis::launch_fsm_tables(a, stream);
  }
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  cleanup();
  if (e != hipSuccess) return fail(SIS_E_DEVICE, "device tables: %s", hipGetErrorString(e));
  return SIS_OK;
}

}  // namespace

extern "C" {

sis_status sis_plan_create(const sis_velocity_desc* desc, hipStream_t stream, sis_plan_t* out) {
  if (!out) return fail(SIS_E_INVALID, "null output handle");
  *out = nullptr;
  sis_status st = validate_desc(desc);
  if (st) return st;
  if (desc->grid == SIS_GRID_POLAR) return create_polar_plan(desc, stream, out);
  if (desc->n_species == 2) return create_mix_plan(desc, stream, out);
  auto t0 = std::chrono::steady_clock::now();
  sis::HostTables t;
  std::string err;
  const sis::TableDesc td = table_desc(desc);
  if (!sis::build_grid_tables(td, t, err)) return fail(SIS_E_INVALID, "%s", err.c_str());
  // the transforms of the tables run on the device when the table kernel's LDS holds the
  // modes (n_pad <= 100 or so); otherwise the host planner builds them
  bool device_tables;
  {
    sis::FsmDims dd{};
    dd.n = t.n;
    dd.P = t.np;
    dd.L = t.np - 1;
    dd.Q = t.np / 2;
    device_tables = sis::fsm_tables_fit(dd, t.nd);
  }
  if (!device_tables && !sis::build_host_tables(td, true, t, err)) return fail(SIS_E_INVALID, "%s", err.c_str());
  auto t1 = std::chrono::steady_clock::now();

  sis_plan* p = new sis_plan();
  HIP_TRY(hipGetDevice(&p->device));
  p->n = t.n;
  p->n3 = t.n3;
  p->np = t.np;
  p->D = t.D;
  p->m_angle = desc->m_angle;
  p->lv = t.lv;
  p->dv = t.dv;
  p->w = t.dv * t.dv * t.dv;
  p->b0 = t.b0;
  p->R = t.R;
  p->nsp = 1;
  p->ndof = t.n3;
  set_layout(p, 0);
  p->alpha = t.alpha;
  p->gamma = t.gamma;
  p->h_v1d = t.v1d;
  p->h_feq = t.feq;
  const int n = t.n, n3 = t.n3, D = t.D;

  // term tables of the assembly: X = [B_p; A_p] (scaled by 4 b0 W_p) and nu, Y = [Psi_p; Phi_p]
  // and beta_r
  double *dX = nullptr, *dY = nullptr;
  auto cleanup = [&]() { dfree(dX); dfree(dY); };
#define PLAN_TRY(expr)                                                                       \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) {                                                                  \
      cleanup();                                                                             \
      delete p;                                                                              \
      return fail(e_ == hipErrorOutOfMemory ? SIS_E_OOM : SIS_E_DEVICE, "%s: %s", #expr,      \
                  hipGetErrorString(e_));                                                    \
    }                                                                                        \
  } while (0)
#define PLAN_ST(expr)          \
  do {                         \
    sis_status st_ = (expr);   \
    if (st_ != SIS_OK) {       \
      cleanup();               \
      delete p;                \
      return st_;              \
    }                          \
  } while (0)
  const size_t tabX = static_cast<size_t>(D) * n3, tabY = static_cast<size_t>(D) * t.nd3;
  PLAN_TRY(dmalloc(&dX, 2 * tabX + n3));
  PLAN_TRY(dmalloc(&dY, 2 * tabY + t.nd3));
  PLAN_TRY(dmalloc(&p->op, static_cast<size_t>(n3) * n3));
  PLAN_TRY(dmalloc(&p->v1d, n));
  PLAN_TRY(dmalloc(&p->feq, n3));
  PLAN_TRY(dmalloc(&p->nu, n3));
  PLAN_TRY(dmalloc(&p->Kc, n3));
  PLAN_TRY(dmalloc(&p->gram_inv, 25));
  PLAN_TRY(hipMemcpyAsync(p->v1d, t.v1d.data(), n * 8, hipMemcpyHostToDevice, stream));
  PLAN_TRY(hipMemcpyAsync(p->feq, t.feq.data(), n3 * 8, hipMemcpyHostToDevice, stream));
  if (device_tables) {
    PLAN_ST(build_fsm_multipliers(p, desc, stream));
    PLAN_ST(build_tables_device(p, t, dX, dY, stream));
    t.nu.resize(n3);
    PLAN_TRY(hipMemcpy(t.nu.data(), dX + 2 * tabX, n3 * 8, hipMemcpyDeviceToHost));
    double nb = 0.0;
    for (int i = 0; i < n3; ++i) nb += p->w * t.nu[i] * t.feq[i];
    t.nubar = nb;
  } else {
    for (int d = 0; d < D; ++d) {
      const double sc = 4.0 * t.b0 * t.W[d];
      for (int i = 0; i < n3; ++i) {
        t.A[static_cast<size_t>(d) * n3 + i] *= sc;
        t.B[static_cast<size_t>(d) * n3 + i] *= sc;
      }
    }
    PLAN_TRY(hipMemcpyAsync(dY, t.Psi.data(), tabY * 8, hipMemcpyHostToDevice, stream));
    PLAN_TRY(hipMemcpyAsync(dY + tabY, t.Phi.data(), tabY * 8, hipMemcpyHostToDevice, stream));
    PLAN_TRY(hipMemcpyAsync(dY + 2 * tabY, t.beta_r.data(), t.beta_r.size() * 8, hipMemcpyHostToDevice, stream));
    PLAN_TRY(hipMemcpyAsync(dX, t.B.data(), tabX * 8, hipMemcpyHostToDevice, stream));
    PLAN_TRY(hipMemcpyAsync(dX + tabX, t.A.data(), tabX * 8, hipMemcpyHostToDevice, stream));
  }
  p->nubar = t.nubar;
  p->nubar_s[0] = t.nubar;
  p->h_nu = t.nu;
  PLAN_TRY(hipMemcpyAsync(p->nu, t.nu.data(), n3 * 8, hipMemcpyHostToDevice, stream));
  if (device_tables) PLAN_ST(build_fsm_static(p, desc->parity, dX, p->feq, stream));
  const double* dbr = dY + 2 * tabY;

  // Gram matrix of the invariants {1, v1, v2, v3, |v|^2} with weight w f_eq
  double G[25] = {0}, Gi[25];
  std::vector<double> corr(n3);
  for (int a = 0; a < n; ++a)
    for (int b = 0; b < n; ++b)
      for (int c = 0; c < n; ++c) {
        const int i = (a * n + b) * n + c;
        const double v1 = t.v1d[a], v2 = t.v1d[b], v3 = t.v1d[c];
        const double psi[5] = {1.0, v1, v2, v3, v1 * v1 + v2 * v2 + v3 * v3};
        for (int r = 0; r < 5; ++r)
          for (int q = 0; q < 5; ++q) G[r * 5 + q] += p->w * psi[r] * psi[q] * t.feq[i];
        corr[i] = 2.0 * v3 * t.feq[i];
        p->cU += p->w * v3 * corr[i];
        p->cq += p->w * (psi[4] - 2.5) * v3 * corr[i];
      }
  p->cU_s[0] = p->cU;
  p->cq_s[0] = p->cq;
  if (desc->parity) {
    // stored by parity the projection keeps only its v3 (x3-momentum) component: the
    // Gram matrix is block diagonal in v3-parity and L is odd in v3
    for (int k = 0; k < 25; ++k) Gi[k] = 0.0;
    Gi[3 * 5 + 3] = 1.0 / G[3 * 5 + 3];
  } else if (!invert5(G, Gi)) {
    cleanup();
    delete p;
    return fail(SIS_E_NUMERIC, "singular invariant Gram matrix");
  }
  PLAN_TRY(hipMemcpyAsync(p->gram_inv, Gi, 25 * 8, hipMemcpyHostToDevice, stream));

  PLAN_TRY(sis::launch_assemble(n, 2 * D, dX, dY, p->feq, 1.0, dbr, p->op, n3, 0, stream));
  // restriction to the stored parity class, then Kc = L+(2 v3 feq): one-row contraction
  PLAN_TRY(hipStreamSynchronize(stream));
  set_layout(p, desc->parity);
  if (sis_status st = apply_parity(p, stream)) {
    cleanup();
    delete p;
    return st;
  }
  if (sis_status st = build_velocity_tables(p, stream)) {
    cleanup();
    delete p;
    return st;
  }
  if (p->parity) corr = restrict_rows(p, corr.data(), 1);
  p->fsm_corr = corr;
  double* dcorr = dX;  // reuse (large enough)
  PLAN_TRY(hipMemcpyAsync(dcorr, corr.data(), corr.size() * 8, hipMemcpyHostToDevice, stream));
  {
    sis::GemmArgs g{};
    g.precision = 0;
    g.X = dcorr;
    g.op64 = p->op;
    g.acc = p->Kc;
    g.M = 1;
    g.N = p->ndof;
    g.K = p->ndof;
    g.splits = 1;
    g.tile = 1;
    PLAN_TRY(sis::launch_gemm(g, stream));
  }
  PLAN_TRY(hipStreamSynchronize(stream));
  cleanup();
#undef PLAN_TRY
#undef PLAN_ST
  auto t2 = std::chrono::steady_clock::now();
  p->host_s = std::chrono::duration<double>(t1 - t0).count();
  p->dev_s = std::chrono::duration<double>(t2 - t1).count();
  *out = p;
  g_err.clear();
  return SIS_OK;
}

sis_status sis_plan_destroy(sis_plan_t plan) {
  if (!plan) return fail(SIS_E_INVALID, "null plan");
  delete plan;
  return SIS_OK;
}

sis_status sis_plan_query(sis_plan_t p, sis_plan_info* out) {
  if (sis_status st = check_plan(p)) return st;
  if (!out) return fail(SIS_E_INVALID, "null output");
  out->n_v = p->n;
  out->n3 = p->n3;
  out->n_pad = p->np;
  out->m_angle = p->m_angle;
  out->n_dir = p->D;
  out->l_v = p->lv;
  out->dv = p->dv;
  out->b0 = p->b0;
  out->r_trunc = p->R;
  out->nubar = p->nubar;
  out->alpha = p->alpha;
  out->gamma = p->gamma;
  out->operator_bytes = static_cast<int64_t>(p->ndof) * p->ndof * 8;
  out->n_species = p->nsp;
  out->n_dof = p->ndof;
  out->nubar_b = p->nsp == 2 ? p->nubar_s[1] : 0.0;
  out->viscosity_ratio = p->visc_ratio;
  out->flow_factor = p->flow_factor;
  out->parity = p->parity;
  out->n_vel = p->nv;
  out->plan_seconds_host = p->host_s;
  out->plan_seconds_device = p->dev_s;
  return SIS_OK;
}

sis_status sis_plan_tables(sis_plan_t p, double* v1d, double* feq, double* nu, double* op) {
  if (sis_status st = check_plan(p)) return st;
  if (v1d) std::memcpy(v1d, p->h_v1d.data(), p->n * 8);
  if (feq) std::memcpy(feq, p->h_feq.data(), static_cast<size_t>(p->nsp) * p->nv * 8);
  if (nu) std::memcpy(nu, p->h_nu.data(), static_cast<size_t>(p->nsp) * p->nv * 8);
  if (op) HIP_TRY(hipMemcpy(op, p->op, static_cast<size_t>(p->ndof) * p->ndof * 8, hipMemcpyDeviceToHost));
  return SIS_OK;
}

sis_status sis_plan_set_precision(sis_plan_t p, int32_t precision, hipStream_t stream) {
  if (sis_status st = check_plan(p)) return st;
  const int64_t cnt = static_cast<int64_t>(p->ndof) * p->ndof;
  if (precision == SIS_PREC_FP64) {
  } else if (precision == SIS_PREC_FP32) {
    if (!p->op32) {
      HIP_TRY(dmalloc(&p->op32, cnt));
      HIP_TRY(sis::launch_convert_f32(p->op, p->op32, cnt, stream));
      HIP_TRY(hipStreamSynchronize(stream));
    }
  } else if (precision == SIS_PREC_BF16X3 || precision == SIS_PREC_BF16) {
    if (p->ndof % 8) return fail(SIS_E_UNSUPPORTED, "the BF16 contractions need the unknowns per cell divisible by 8");
    if (precision == SIS_PREC_BF16 && p->nsp == 2)
      return fail(SIS_E_UNSUPPORTED, "the one-product BF16 contraction is not offered for two-species plans "
                                     "(the species blocks deviate by ~1e-3 in the heat flux); use BF16X3");
    if (!p->opp) {
      HIP_TRY(dmalloc(&p->opp, static_cast<int64_t>(p->ndof) * 2 * sis::pair_stride(p->ndof)));
      HIP_TRY(sis::launch_split_pairs(p->op, nullptr, p->ndof, p->ndof, p->opp, 1, stream));
      HIP_TRY(hipStreamSynchronize(stream));
    }
  } else {
    return fail(SIS_E_UNSUPPORTED, "unknown precision %d", precision);
  }
  p->precision = precision;
  return SIS_OK;
}

sis_status sis_geometry_create(sis_plan_t p, const sis_geometry_desc* d, hipStream_t stream,
                               sis_geom_t* out) {
  if (sis_status st = check_plan(p)) return st;
  if (!d || !out) return fail(SIS_E_INVALID, "null argument");
  *out = nullptr;
  if (d->n_cases < 1) return fail(SIS_E_INVALID, "n_cases must be >= 1");
  if (p->parity == 2 && d->kind != SIS_GEOM_PLANAR_HALF)
    return fail(SIS_E_UNSUPPORTED, "parity 2 (even in v2) needs the planar geometry");
  if (p->nsp == 2) {
    for (int c = 0; c < d->n_cases; ++c)
      if (d->flow && d->flow[c] != SIS_FLOW_NONE && d->flow[c] != SIS_FLOW_POISEUILLE)
        return fail(SIS_E_UNSUPPORTED, "mixtures support Poiseuille flow only (case %d)", c);
  }
  if ((d->kind == SIS_GEOM_TUBE) != p->polar)
    return fail(SIS_E_UNSUPPORTED, "the tube geometry and the polar velocity grid go together");
  if (d->kind == SIS_GEOM_TUBE) return create_geometry_tube(p, d, stream, out);
  if (d->kind == SIS_GEOM_DUCT_QUARTER || d->kind == SIS_GEOM_PERIODIC_2D)
    return create_geometry_2d(p, d, stream, out);
  if (d->kind != SIS_GEOM_PLANAR_HALF) return fail(SIS_E_UNSUPPORTED, "geometry kind %d not supported", d->kind);
  if (!d->node_offset || !d->x1 || !d->delta || !d->flow) return fail(SIS_E_INVALID, "null geometry array");
  if (d->node_offset[0] != 0) return fail(SIS_E_INVALID, "node_offset[0] must be 0");
  auto* g = new sis_geom();
  g->plan = p;
  g->kind = d->kind;
  g->n_cases = d->n_cases;
  g->h_off.assign(d->node_offset, d->node_offset + d->n_cases + 1);
  g->n_cells = g->h_off.back();
  for (int c = 0; c < d->n_cases; ++c) {
    const int64_t a = g->h_off[c], b = g->h_off[c + 1];
    if (b - a < 2) { delete g; return fail(SIS_E_SHAPE, "case %d has fewer than 2 nodes", c); }
    g->max_nodes = std::max<int>(g->max_nodes, static_cast<int>(b - a));
    if (d->x1[a] != -0.5 || d->x1[b - 1] != 0.0) { delete g; return fail(SIS_E_INVALID, "case %d nodes must run from -0.5 to 0", c); }
    for (int64_t i = a + 1; i < b; ++i)
      if (!(d->x1[i] > d->x1[i - 1])) { delete g; return fail(SIS_E_INVALID, "case %d nodes not increasing", c); }
    if (!(d->delta[c] >= 0.0) || !std::isfinite(d->delta[c])) { delete g; return fail(SIS_E_INVALID, "case %d delta must be >= 0", c); }
    if (d->flow[c] < 0 || d->flow[c] > 2) { delete g; return fail(SIS_E_INVALID, "case %d flow code %d", c, d->flow[c]); }
  }
  g->h_x.assign(d->x1, d->x1 + g->n_cells);
  g->h_delta.assign(d->delta, d->delta + d->n_cases);
  g->h_flow.assign(d->flow, d->flow + d->n_cases);
  // upwind stencil coefficients per node (first order at the first step from a boundary)
  std::vector<double> coef(static_cast<size_t>(g->n_cells) * 6, 0.0);
  std::vector<double> dcell(g->n_cells);
  std::vector<int32_t> fcell(g->n_cells), ccell(g->n_cells);
  for (int c = 0; c < d->n_cases; ++c) {
    const int64_t a = g->h_off[c], b = g->h_off[c + 1];
    const int nn = static_cast<int>(b - a);
    const double* x = d->x1 + a;
    for (int i = 0; i < nn; ++i) {
      double* q = &coef[(a + i) * 6];
      if (i >= 1) {
        const double d1 = x[i] - x[i - 1];
        if (i == 1) { q[0] = 1.0 / d1; q[1] = -1.0 / d1; q[2] = 0.0; }
        else {
          const double d2 = x[i - 1] - x[i - 2];
          q[0] = (2.0 * d1 + d2) / (d1 * (d1 + d2));
          q[1] = -(d1 + d2) / (d1 * d2);
          q[2] = d1 / (d2 * (d1 + d2));
        }
      }
      if (i <= nn - 2) {
        const double d1 = x[i + 1] - x[i];
        if (i == nn - 2) { q[3] = 1.0 / d1; q[4] = -1.0 / d1; q[5] = 0.0; }
        else {
          const double d2 = x[i + 2] - x[i + 1];
          q[3] = (2.0 * d1 + d2) / (d1 * (d1 + d2));
          q[4] = -(d1 + d2) / (d1 * d2);
          q[5] = d1 / (d2 * (d1 + d2));
        }
      }
      dcell[a + i] = d->delta[c];
      fcell[a + i] = d->flow[c];
      ccell[a + i] = c;
    }
  }
#define GEOM_TRY(expr)                                                                         \
  do {                                                                                         \
    hipError_t e_ = (expr);                                                                    \
    if (e_ != hipSuccess) {                                                                    \
      delete g;                                                                                \
      return fail(e_ == hipErrorOutOfMemory ? SIS_E_OOM : SIS_E_DEVICE, "%s: %s", #expr,        \
                  hipGetErrorString(e_));                                                      \
    }                                                                                          \
  } while (0)
  const int64_t nc = g->n_cells;
  GEOM_TRY(dmalloc(&g->off, d->n_cases + 1));
  GEOM_TRY(dmalloc(&g->x, nc));
  GEOM_TRY(dmalloc(&g->coef, nc * 6));
  GEOM_TRY(dmalloc(&g->delta_case, d->n_cases));
  GEOM_TRY(dmalloc(&g->flow_case, d->n_cases));
  GEOM_TRY(dmalloc(&g->delta_cell, nc));
  GEOM_TRY(dmalloc(&g->flow_cell, nc));
  GEOM_TRY(dmalloc(&g->case_of_cell, nc));
  GEOM_TRY(hipMemcpyAsync(g->off, g->h_off.data(), (d->n_cases + 1) * 8, hipMemcpyHostToDevice, stream));
  GEOM_TRY(hipMemcpyAsync(g->x, d->x1, nc * 8, hipMemcpyHostToDevice, stream));
  GEOM_TRY(hipMemcpyAsync(g->coef, coef.data(), nc * 6 * 8, hipMemcpyHostToDevice, stream));
  GEOM_TRY(hipMemcpyAsync(g->delta_case, d->delta, d->n_cases * 8, hipMemcpyHostToDevice, stream));
  GEOM_TRY(hipMemcpyAsync(g->flow_case, d->flow, d->n_cases * 4, hipMemcpyHostToDevice, stream));
  GEOM_TRY(hipMemcpyAsync(g->delta_cell, dcell.data(), nc * 8, hipMemcpyHostToDevice, stream));
  GEOM_TRY(hipMemcpyAsync(g->flow_cell, fcell.data(), nc * 4, hipMemcpyHostToDevice, stream));
  GEOM_TRY(hipMemcpyAsync(g->case_of_cell, ccell.data(), nc * 4, hipMemcpyHostToDevice, stream));
  GEOM_TRY(hipStreamSynchronize(stream));
#undef GEOM_TRY
  *out = g;
  g_err.clear();
  return SIS_OK;
}

sis_status sis_geometry_destroy(sis_geom_t g) {
  if (!g) return fail(SIS_E_INVALID, "null geometry");
  delete g;
  return SIS_OK;
}

int64_t sis_geometry_cells(sis_geom_t g) { return g ? g->n_cells : -1; }

sis_status sis_geometry_diffusion_solver(sis_geom_t g, int32_t mode, hipStream_t stream) {
  if (!g) return fail(SIS_E_INVALID, "null geometry");
  if (mode != SIS_DIFFUSION_CG && mode != SIS_DIFFUSION_INVERSE)
    return fail(SIS_E_INVALID, "diffusion solver mode %d", mode);
  if (!g->two_d) return SIS_OK;
  if (mode == SIS_DIFFUSION_CG) {
    if (g->plan->nsp == 2) return fail(SIS_E_UNSUPPORTED, "2-D mixtures use the precomputed inverse only");
    HIP_TRY(hipStreamSynchronize(stream));
    g->free_inverse();
    g_err.clear();
    return SIS_OK;
  }
  if (g->d_direct) return SIS_OK;
  return build_inverse_2d(g->plan, g, stream);
}

sis_status sis_geometry_diffusion_info(sis_geom_t g, int32_t* n_inverse, int32_t* n_distinct, double* residual) {
  if (!g) return fail(SIS_E_INVALID, "null geometry");
  if (n_inverse) *n_inverse = g->n_direct;
  if (n_distinct) *n_distinct = g->n_inverses;
  if (residual) *residual = g->inv_residual;
  return SIS_OK;
}
int32_t sis_geometry_moment_stride(sis_geom_t g) { return g ? g->mom_stride() : -1; }

int32_t sis_geometry_sweep_form(sis_geom_t g) {
  if (!g || !g->two_d) return -1;
  return sis::sweep2d_form(g->max_diag, g->max_n2, g->n_cells * static_cast<int64_t>(g->plan->nsp) * g->plan->nv * 8);
}

sis_status sis_collide(sis_plan_t p, int64_t n_cells, const double* h, const double* dU,
                       const double* delta, const int32_t* flow, int32_t project, double* rhs_out,
                       double* lh_out, double* amom_out, hipStream_t stream) {
  if (sis_status st = check_plan(p)) return st;
  if (n_cells < 0) return fail(SIS_E_SHAPE, "n_cells must be >= 0");
  if (n_cells == 0) return SIS_OK;
  if (n_cells > (int64_t(1) << 31) / 1) return fail(SIS_E_SHAPE, "n_cells too large");
  if (!h || !delta || !rhs_out) return fail(SIS_E_INVALID, "h, delta and rhs_out must be non-null");
  if (!aligned16(h) || !aligned16(rhs_out)) return fail(SIS_E_INVALID, "h and rhs_out must be 16-byte aligned");
  if (h == rhs_out) return fail(SIS_E_INVALID, "rhs_out must not alias h");
  if (project && p->nsp != 1) return fail(SIS_E_UNSUPPORTED, "invariant projection is for one gas only");
  if (project && p->polar) return fail(SIS_E_UNSUPPORTED, "invariant projection is for the Cartesian grids");
  {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(stream, &cs));
    if (cs == hipStreamCaptureStatusNone)
      if (sis_status st = tune_gemm(p, n_cells, p->precision, h, &p->ws_acc, &p->ws_x, stream)) return st;
  }
  return run_collide(p, n_cells, h, dU, delta, flow, project, rhs_out, lh_out, amom_out, nullptr, stream);
}

sis_status sis_collide_noalloc(sis_plan_t p, int64_t n_cells, const double* h, const double* dU,
                               const double* delta, const int32_t* flow, int32_t project, double* rhs_out,
                               double* lh_out, double* amom_out, hipStream_t stream) {
  if (sis_status st = check_plan(p)) return st;
  if (n_cells < 0) return fail(SIS_E_SHAPE, "n_cells must be >= 0");
  if (n_cells == 0) return SIS_OK;
  if (n_cells > (int64_t(1) << 31)) return fail(SIS_E_SHAPE, "n_cells too large");
  if (!h || !delta || !rhs_out) return fail(SIS_E_INVALID, "h, delta and rhs_out must be non-null");
  if (!aligned16(h) || !aligned16(rhs_out)) return fail(SIS_E_INVALID, "h and rhs_out must be 16-byte aligned");
  if (h == rhs_out) return fail(SIS_E_INVALID, "rhs_out must not alias h");
  if (project && p->nsp != 1) return fail(SIS_E_UNSUPPORTED, "invariant projection is for one gas only");
  if (project && p->polar) return fail(SIS_E_UNSUPPORTED, "invariant projection is for the Cartesian grids");
  // the plan's configuration for this shape (tuned by earlier sis_collide calls, else the
  // default heuristic); no tuning here, since tuning allocates
  const int precision = p->precision;
  int tile, splits;
  const auto tuned = p->gemm_choice.find(std::make_pair(n_cells, precision));
  if (tuned != p->gemm_choice.end()) {
    tile = tuned->second.first;
    splits = tuned->second.second;
  } else {
    choose_gemm(n_cells, p->ndof, &tile, &splits);
  }
  const int64_t cnt = n_cells * static_cast<int64_t>(p->ndof);
  // low-precision cell operand first in the scratch (4 bytes per unknown), then the split-K
  // partials; the split count is lowered until the partials fit (one split needs none)
  // FP32: 4 bytes per unknown; the bf16 forms: 4 bytes per padded unknown (pair layout)
  const int64_t xcnt = precision == SIS_PREC_FP32 ? cnt : n_cells * static_cast<int64_t>(sis::pair_stride(p->ndof));
  const size_t xbytes = precision == SIS_PREC_FP64 ? 0 : ((static_cast<size_t>(xcnt) * 4 + 255) / 256) * 256;
  if (xbytes > kStaticScratchBytes)
    return fail(SIS_E_SHAPE, "sis_collide_noalloc: the low-precision cell operand needs %zu bytes, more than its "
                             "%zu-byte workspace (use fewer cells per call)", xbytes, kStaticScratchBytes);
  while (splits > 1 && xbytes + static_cast<size_t>(splits) * cnt * sizeof(double) > kStaticScratchBytes) --splits;
  void* base = nullptr;
  {
    const hipError_t e = static_scratch(&base);
    if (e != hipSuccess) return fail(SIS_E_DEVICE, "workspace address: %s", hipGetErrorString(e));
  }
  unsigned char* ws = static_cast<unsigned char*>(base);
  sis::GemmArgs g{};
  g.precision = precision;
  g.X = h;
  if (precision == SIS_PREC_BF16X3 || precision == SIS_PREC_BF16) {
    uint16_t* hx = reinterpret_cast<uint16_t*>(ws);
    HIP_TRY(sis::launch_split_pairs(h, nullptr, n_cells, p->ndof, hx, precision == SIS_PREC_BF16X3, stream));
    g.Xp = hx;
  } else if (precision == SIS_PREC_FP32) {
    float* fx = reinterpret_cast<float*>(ws);
    HIP_TRY(sis::launch_convert_x_f32(h, nullptr, cnt, fx, stream));
    g.X32 = fx;
  }
  double* acc = splits > 1 ? reinterpret_cast<double*>(ws + xbytes) : rhs_out;
  g.op64 = p->op;
  g.op32 = p->op32;
  g.opp = p->opp;
  g.acc = acc;
  g.M = n_cells;
  g.N = p->ndof;
  g.K = p->ndof;
  g.splits = splits;
  g.tile = tile;
  HIP_TRY(sis::launch_gemm(g, stream));
  sis::FinishArgs f = finish_args(p, n_cells, h, dU, delta, flow, project, rhs_out, lh_out, amom_out, nullptr, 0,
                                  nullptr, nullptr);
  f.splits = splits;
  f.acc = acc;
  HIP_TRY(sis::launch_finish(f, stream));
  return SIS_OK;
}

sis_status sis_collide_fsm(sis_plan_t p, int64_t n_cells, const double* h, const double* dU,
                           const double* delta, const int32_t* flow, int32_t project, double* rhs_out,
                           double* lh_out, double* amom_out, hipStream_t stream) {
  if (sis_status st = check_plan(p)) return st;
  if (p->nsp != 1 || p->polar) return fail(SIS_E_UNSUPPORTED, "the per-cell transform path serves one-gas Cartesian plans");
  if (!p->fsm_ok) {
    const char* why = sis::fsm_unsupported(p->fsm_d);
    return fail(SIS_E_UNSUPPORTED, "%s", why ? why : "per-cell transform path unavailable");
  }
  if (n_cells < 0) return fail(SIS_E_SHAPE, "n_cells must be >= 0");
  if (n_cells == 0) return SIS_OK;
  if (n_cells > (int64_t(1) << 31)) return fail(SIS_E_SHAPE, "n_cells too large");
  if (!h || !delta || !rhs_out) return fail(SIS_E_INVALID, "h, delta and rhs_out must be non-null");
  if (h == rhs_out) return fail(SIS_E_INVALID, "rhs_out must not alias h");
  {
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    HIP_TRY(hipStreamIsCapturing(stream, &cs));
    if (cs != hipStreamCaptureStatusNone)
      return fail(SIS_E_UNSUPPORTED, "sis_collide_fsm allocates its scratch on first use: not capturable");
  }
  if (sis_status st = ensure_fsm(p, stream)) return st;
  hipEvent_t a = nullptr, b = nullptr;
  if (p->timing) {
    HIP_TRY(hipEventCreate(&a));
    HIP_TRY(hipEventCreate(&b));
    p->fsm_events.emplace_back(a, b);
    HIP_TRY(hipEventRecord(a, stream));
  }
  if (sis_status st = run_fsm_chunks(p, n_cells, h, dU, delta, flow, project, rhs_out, lh_out, amom_out, p->fsm_Kc,
                                     stream))
    return st;
  if (p->timing) HIP_TRY(hipEventRecord(b, stream));
  return SIS_OK;
}

sis_status sis_plan_fsm_info(sis_plan_t p, double* flops_per_cell, int32_t* slab_l1, int64_t* table_bytes) {
  if (sis_status st = check_plan(p)) return st;
  if (!p->fsm_ok) return fail(SIS_E_UNSUPPORTED, "no per-cell transform path on this plan");
  const sis::FsmDims& d = p->fsm_d;
  if (flops_per_cell) *flops_per_cell = sis::fsm_flops_per_cell(d, p->fsm_slab);
  if (slab_l1) *slab_l1 = p->fsm_slab;
  if (table_bytes)
    *table_bytes = 8 * (static_cast<int64_t>(d.T) * d.Q * d.L * d.L + static_cast<int64_t>(d.T) * d.nv);
  return SIS_OK;
}

sis_status sis_plan_set_fsm_slab(sis_plan_t p, int32_t slab_l1) {
  if (sis_status st = check_plan(p)) return st;
  if (!p->fsm_ok) return fail(SIS_E_UNSUPPORTED, "no per-cell transform path on this plan");
  if (slab_l1 < 1 || slab_l1 > 8 || !sis::fsm_slab_fits(p->fsm_d, slab_l1))
    return fail(SIS_E_INVALID, "slab_l1 must be in 1..8 with the inverse transforms' LDS within 160 KiB");
  p->fsm_slab = slab_l1;
  return SIS_OK;
}

sis_status sis_plan_fsm_timing_read(sis_plan_t p, double* ms, int64_t* calls) {
  if (sis_status st = check_plan(p)) return st;
  double tot = 0.0;
  for (auto& e : p->fsm_events) {
    HIP_TRY(hipEventSynchronize(e.second));
    float m = 0.f;
    HIP_TRY(hipEventElapsedTime(&m, e.first, e.second));
    tot += m;
  }
  if (ms) *ms = tot;
  if (calls) *calls = static_cast<int64_t>(p->fsm_events.size());
  return SIS_OK;
}

sis_status sis_transport_sweep(sis_plan_t p, sis_geom_t g, const double* rhs, double* h_half_out,
                               double* mom_out, hipStream_t stream) {
  if (sis_status st = check_plan(p)) return st;
  if (!g || g->plan != p) return fail(SIS_E_INVALID, "geometry does not belong to this plan");
  if (!rhs || !h_half_out) return fail(SIS_E_INVALID, "rhs and h_half_out must be non-null");
  if (rhs == h_half_out) return fail(SIS_E_INVALID, "h_half_out must not alias rhs");
  return run_sweep(p, g, rhs, h_half_out, mom_out, nullptr, stream);
}

sis_status sis_moments(sis_plan_t p, int64_t n_cells, const double* h, double* mom_out, hipStream_t stream) {
  if (sis_status st = check_plan(p)) return st;
  if (n_cells < 0) return fail(SIS_E_SHAPE, "n_cells must be >= 0");
  if (n_cells == 0) return SIS_OK;
  if (!h || !mom_out) return fail(SIS_E_INVALID, "null array");
  if (p->polar) {
    HIP_TRY(sis::launch_moments_tube(n_cells, p->nv, p->vnode, p->wnode, h, nullptr, mom_out, stream));
    return SIS_OK;
  }
  HIP_TRY(sis::launch_moments(p->nv, p->nsp, p->mass_ratio, n_cells * p->nsp, p->vtab, h, p->wr, mom_out, stream));
  return SIS_OK;
}

sis_status sis_diffusion_correct(sis_plan_t p, sis_geom_t g, const double* mom_half,
                                 const double* amom, double N, double* U_out, double* dU_out,
                                 hipStream_t stream) {
  if (sis_status st = check_plan(p)) return st;
  if (!g || g->plan != p) return fail(SIS_E_INVALID, "geometry does not belong to this plan");
  if (!mom_half) return fail(SIS_E_INVALID, "mom_half must be non-null");
  if (!std::isfinite(N)) return fail(SIS_E_INVALID, "N must be finite");
  if (g->tube) {
    sis::TubeDiffArgs a = tube_diff_args(p, g, mom_half, amom, N > 0.0 ? N : p->nubar);
    a.U = U_out;
    a.dU = dU_out;
    HIP_TRY(sis::launch_diffusion_tube(a, stream));
    return SIS_OK;
  }
  if (g->two_d) {
    sis::Diff2DArgs a = diff2d_args(p, g, mom_half, amom, p->nsp == 2 ? N : (N > 0.0 ? N : p->nubar));
    a.U = U_out;
    a.dU = dU_out;
    HIP_TRY(sis::launch_diffusion2d(a, stream));
    return SIS_OK;
  }
  sis::DiffusionArgs a{};
  a.n_cases = g->n_cases;
  a.node_off = g->off;
  a.x = g->x;
  a.coef = g->coef;
  a.delta_case = g->delta_case;
  a.flow_case = g->flow_case;
  a.mom = mom_half;
  a.amom = amom;
  a.N = N > 0.0 ? N : p->nubar;
  a.sis = 1;
  a.cU = p->cU;
  a.cq = p->cq;
  a.U = U_out;
  a.dU = dU_out;
  set_species(a, p, N);
  HIP_TRY(sis::launch_diffusion1d(a, stream));
  return SIS_OK;
}

}  // extern "C"

struct sis_state {
  sis_plan* p = nullptr;
  sis_geom* g = nullptr;
  sis_solve_opts o{};
  double Npen = 0.0;
  double *h = nullptr, *rhs = nullptr, *amom = nullptr, *mom = nullptr, *dU = nullptr, *U = nullptr,
         *q = nullptr, *state = nullptr;
  int32_t *iters = nullptr, *cact = nullptr, *lact = nullptr;
  double *xref = nullptr, *accref = nullptr;   // FP64 anchor of the defect correction
  Scratch ws_acc, ws_x;                        // sized at creation, used by the captured graphs
  int precision = 0, refresh = 1;
  hipStream_t cap = nullptr;
  hipGraph_t graph[2] = {nullptr, nullptr};    // [0] refresh / plain, [1] incremental
  hipGraphExec_t exec[2] = {nullptr, nullptr};
  int total = 0;
  // persistent launch (planar one-gas FP64 solves): workgroups, split-K slices of the
  // contraction and their depth, the grid-barrier words
  bool persistent = false;
  int p_blocks = 0, p_splits = 1, p_kps = 0;
  unsigned* bar = nullptr;
  ~sis_state() {
    for (int i = 0; i < 2; ++i) {
      if (exec[i]) (void)hipGraphExecDestroy(exec[i]);
      if (graph[i]) (void)hipGraphDestroy(graph[i]);
    }
    dfree(xref); dfree(accref);
    dfree(h); dfree(rhs); dfree(amom); dfree(mom); dfree(dU); dfree(U); dfree(q); dfree(state);
    dfree(iters); dfree(cact); dfree(lact); dfree(bar);
    if (cap) (void)hipStreamDestroy(cap);
  }
};

namespace {

// kind 0: plain (FP64) or refresh iteration; kind 1: incremental low-precision iteration
sis_status state_iteration(sis_state* b, hipStream_t s, int kind, bool h_is_zero = false) {
  sis_plan* p = b->p;
  sis_geom* g = b->g;
  const bool sis = b->o.scheme == SIS_SCHEME_SIS;
  const bool mixed = b->precision != SIS_PREC_FP64;
  int prec = b->precision, mode = 0;
  if (mixed && b->refresh == 1) {
    prec = SIS_PREC_FP64;
  } else if (mixed && b->refresh > 1) {
    prec = kind == 0 ? SIS_PREC_FP64 : b->precision;
    mode = kind == 0 ? 1 : 2;
  }
  if (sis_status st = run_collide(p, g->n_cells, b->h, sis ? b->dU : nullptr, g->delta_cell,
                                  g->flow_cell, b->o.project, b->rhs, nullptr, b->amom, b->lact, s,
                                  prec, mode, b->xref, b->accref, &b->ws_acc, &b->ws_x, h_is_zero))
    return st;
  if (sis_status st = run_sweep(p, g, b->rhs, b->h, b->mom, b->cact, s, b->lact)) return st;
  if (g->tube) {
    sis::TubeDiffArgs a = tube_diff_args(p, g, b->mom, b->amom, b->Npen);
    a.sis = sis ? 1 : 0;
    a.U = nullptr;
    a.ufield = b->U;
    a.dU = b->dU;
    a.qfield = b->q;
    a.state = b->state;
    a.iters = b->iters;
    a.case_active = b->cact;
    a.eps = b->o.eps;
    HIP_TRY(sis::launch_diffusion_tube(a, s));
    HIP_TRY(sis::launch_expand_active(b->cact, g->case_of_cell, g->n_cells, b->lact, s));
    return SIS_OK;
  }
  if (g->two_d) {
    sis::Diff2DArgs a = diff2d_args(p, g, b->mom, b->amom, p->nsp == 2 ? b->o.N : b->Npen);
    a.sis = sis ? 1 : 0;
    a.U = nullptr;
    a.ufield = b->U;
    a.dU = b->dU;
    a.qfield = b->q;
    a.state = b->state;
    a.iters = b->iters;
    a.case_active = b->cact;
    a.eps = b->o.eps;
    HIP_TRY(sis::launch_diffusion2d(a, s));
    HIP_TRY(sis::launch_expand_active(b->cact, g->case_of_cell, g->n_cells, b->lact, s));
    return SIS_OK;
  }
  sis::DiffusionArgs a{};
  a.n_cases = g->n_cases;
  a.node_off = g->off;
  a.x = g->x;
  a.coef = g->coef;
  a.delta_case = g->delta_case;
  a.flow_case = g->flow_case;
  a.mom = b->mom;
  a.amom = b->amom;
  a.N = b->Npen;
  a.sis = sis ? 1 : 0;
  a.cU = p->cU;
  a.cq = p->cq;
  a.U = nullptr;
  a.ufield = b->U;
  a.dU = b->dU;
  a.state = b->state;
  a.iters = b->iters;
  a.case_active = b->cact;
  a.qfield = b->q;
  a.eps = b->o.eps;
  a.cell_active = b->lact;   // the march writes its cells' flags (no expansion launch)
  set_species(a, p, b->o.N);
  HIP_TRY(sis::launch_diffusion1d(a, s));
  return SIS_OK;
}

// n_iters iterations as one persistent cooperative launch (planar one-gas FP64 solves): the
// arguments of the launched path's finish, sweep, moment and velocity-equation steps.
sis_status persistent_iterations(sis_state* b, int n_iters, hipStream_t s) {
  sis_plan* p = b->p;
  sis_geom* g = b->g;
  const bool sis = b->o.scheme == SIS_SCHEME_SIS;
  sis::Persist1DArgs a{};
  a.h = b->h;
  a.op = p->op;
  a.acc = static_cast<double*>(b->ws_acc.p);
  a.n_cells = g->n_cells;
  a.n3 = p->ndof;
  a.kps = b->p_kps;
  a.splits = b->p_splits;
  a.fin = finish_args(p, g->n_cells, b->h, sis ? b->dU : nullptr, g->delta_cell, g->flow_cell, b->o.project, b->rhs,
                      nullptr, b->amom, b->lact, 0, nullptr, nullptr);
  a.sw.n = p->n;
  a.sw.n3 = p->nv;
  a.sw.d2 = p->d2;
  a.sw.d3 = p->d3;
  a.sw.nsp = p->nsp;
  a.sw.n_cases = g->n_cases;
  a.sw.node_off = g->off;
  a.sw.coef = g->coef;
  a.sw.delta_case = g->delta_case;
  a.sw.v1d = p->v1d;
  a.sw.nu = p->nu;
  a.sw.rhs = b->rhs;
  a.sw.h = b->h;
  a.sw.case_active = b->cact;
  a.vtab = p->vtab;
  a.w = p->wr;
  a.mom = b->mom;
  a.dif.n_cases = g->n_cases;
  a.dif.node_off = g->off;
  a.dif.x = g->x;
  a.dif.coef = g->coef;
  a.dif.delta_case = g->delta_case;
  a.dif.flow_case = g->flow_case;
  a.dif.mom = b->mom;
  a.dif.amom = b->amom;
  a.dif.N = b->Npen;
  a.dif.sis = sis ? 1 : 0;
  a.dif.cU = p->cU;
  a.dif.cq = p->cq;
  a.dif.U = nullptr;
  a.dif.ufield = b->U;
  a.dif.dU = b->dU;
  a.dif.state = b->state;
  a.dif.iters = b->iters;
  a.dif.case_active = b->cact;
  a.dif.qfield = b->q;
  a.dif.eps = b->o.eps;
  set_species(a.dif, p, b->o.N);
  a.cell_active = b->lact;
  a.n_iters = n_iters;
  a.first_from_zero = b->total == 0 ? 1 : 0;
  a.bar = b->bar;
  HIP_TRY(sis::launch_persist1d(a, b->p_blocks, s));
  return SIS_OK;
}

sis_status state_init(sis_state* b, hipStream_t s) {
  const int64_t nc = b->g->n_cells;
  const int ncase = b->g->n_cases;
  const int nsp = b->p->nsp;
  HIP_TRY(hipMemsetAsync(b->h, 0, static_cast<size_t>(nc) * b->p->ndof * 8, s));
  HIP_TRY(hipMemsetAsync(b->dU, 0, nc * nsp * 8, s));
  HIP_TRY(hipMemsetAsync(b->U, 0, nc * nsp * 8, s));
  HIP_TRY(hipMemsetAsync(b->q, 0, nc * nsp * 8, s));
  HIP_TRY(hipMemsetAsync(b->state, 0, ncase * (2 * nsp + 2) * 8, s));
  HIP_TRY(hipMemsetAsync(b->iters, 0, ncase * 4, s));
  if (b->g->two_d) HIP_TRY(hipMemsetAsync(b->g->have_x, 0, ncase * 4, s));
  std::vector<int32_t> ones(std::max<int64_t>(nc, ncase), 1);
  HIP_TRY(hipMemcpyAsync(b->cact, ones.data(), ncase * 4, hipMemcpyHostToDevice, s));
  HIP_TRY(hipMemcpyAsync(b->lact, ones.data(), nc * 4, hipMemcpyHostToDevice, s));
  HIP_TRY(hipStreamSynchronize(s));
  b->total = 0;
  return SIS_OK;
}

}  // namespace

extern "C" {

sis_status sis_state_create(sis_plan_t p, sis_geom_t g, const sis_solve_opts* o, hipStream_t stream,
                            sis_state_t* out) {
  if (sis_status st = check_plan(p)) return st;
  if (!out) return fail(SIS_E_INVALID, "null output handle");
  *out = nullptr;
  if (!g || g->plan != p) return fail(SIS_E_INVALID, "geometry does not belong to this plan");
  if (!o) return fail(SIS_E_INVALID, "null options");
  if (o->scheme != SIS_SCHEME_CIS && o->scheme != SIS_SCHEME_SIS) return fail(SIS_E_INVALID, "unknown scheme");
  if (!(o->eps >= 0.0)) return fail(SIS_E_INVALID, "eps must be >= 0");
  if (o->max_it < 1) return fail(SIS_E_INVALID, "max_it must be >= 1");
  auto* b = new sis_state();
  b->p = p;
  b->g = g;
  b->o = *o;
  b->precision = p->precision;
  // refresh: 0 = plain contraction in the plan precision every iteration,
  //          1 = FP64 every iteration, R > 1 = FP64 anchors at iterations 0, R/2, 3R/2, ...
  b->refresh = p->precision == SIS_PREC_FP64 ? 0
               : (o->refresh_every < 0 ? 0 : (o->refresh_every == 0 ? 16 : o->refresh_every));
  b->Npen = o->N > 0.0 ? o->N : p->nubar;
  const int64_t nc = g->n_cells;
  const int ncase = g->n_cases;
  const int n3 = p->ndof;  // unknowns per cell
  const int nsp = p->nsp;
  if (nsp == 2 && o->project) { delete b; return fail(SIS_E_UNSUPPORTED, "invariant projection is for one gas only"); }
  if (p->polar && o->project) { delete b; return fail(SIS_E_UNSUPPORTED, "invariant projection is for the Cartesian grids"); }
#define ST_TRY(expr)                                                                            \
  do {                                                                                          \
    hipError_t e_ = (expr);                                                                     \
    if (e_ != hipSuccess) {                                                                     \
      delete b;                                                                                 \
      return fail(e_ == hipErrorOutOfMemory ? SIS_E_OOM : SIS_E_DEVICE, "%s: %s", #expr,         \
                  hipGetErrorString(e_));                                                       \
    }                                                                                           \
  } while (0)
  ST_TRY(dmalloc(&b->h, static_cast<size_t>(nc) * n3));
  ST_TRY(dmalloc(&b->rhs, static_cast<size_t>(nc) * n3));
  ST_TRY(dmalloc(&b->amom, nc * 4 * nsp));
  ST_TRY(dmalloc(&b->mom, nc * g->mom_stride() * nsp));
  ST_TRY(dmalloc(&b->dU, nc * nsp));
  ST_TRY(dmalloc(&b->U, nc * nsp));
  ST_TRY(dmalloc(&b->q, nc * nsp));
  ST_TRY(dmalloc(&b->state, ncase * (2 * nsp + 2)));
  ST_TRY(dmalloc(&b->iters, ncase));
  ST_TRY(dmalloc(&b->cact, ncase));
  ST_TRY(dmalloc(&b->lact, nc));
  if (b->refresh > 1) {
    ST_TRY(dmalloc(&b->xref, static_cast<size_t>(nc) * n3));
    ST_TRY(dmalloc(&b->accref, static_cast<size_t>(nc) * n3));
  }
  if (o->persistent) {
    if (g->two_d || g->tube || p->polar || nsp != 1 || p->precision != SIS_PREC_FP64) {
      delete b;
      return fail(SIS_E_UNSUPPORTED, "the persistent launch runs planar one-gas solves with the FP64 contraction");
    }
    const int maxb = sis::persist1d_max_blocks();
    if (maxb < 1) { delete b; return fail(SIS_E_DEVICE, "persistent launch: no co-resident workgroups"); }
    // split-K slices (multiples of 16 deep, at least 32) so that the contraction has about
    // 64 tiles; as many workgroups as the largest phase needs, at most 64 (each grid barrier
    // costs more with more workgroups: 32-64 measured fastest on 2- and 17-cell batches)
    // and within the co-resident limit, or the count the caller asked for
    const int tiles = ((n3 + 127) / 128) * static_cast<int>((nc + 31) / 32);
    int sp = std::max(1, std::min(64 / std::max(1, tiles), n3 / 32));
    int kps = ((n3 + sp - 1) / sp + 15) / 16 * 16;
    sp = (n3 + kps - 1) / kps;
    int64_t want = std::min<int64_t>(64, std::max<int64_t>({static_cast<int64_t>(tiles) * sp, nc,
                                                            static_cast<int64_t>(ncase)}));
    if (o->persistent > 1) want = o->persistent;
    b->persistent = true;
    b->p_splits = sp;
    b->p_kps = kps;
    b->p_blocks = static_cast<int>(std::min<int64_t>(want, maxb));
    ST_TRY(dmalloc(&b->bar, 4));
    ST_TRY(b->ws_acc.ensure(static_cast<size_t>(sp) * nc * n3 * 8));
  }
  if (!b->persistent) {
    // contraction configurations of this shape (FP64 and the plan precision)
    if (sis_status st = tune_gemm(p, nc, SIS_PREC_FP64, b->h, &b->ws_acc, &b->ws_x, stream)) { delete b; return st; }
    if (p->precision != SIS_PREC_FP64)
      if (sis_status st = tune_gemm(p, nc, p->precision, b->h, &b->ws_acc, &b->ws_x, stream)) { delete b; return st; }
    int splits = std::max(p->gemm_choice[std::make_pair(nc, static_cast<int>(SIS_PREC_FP64))].second,
                          p->gemm_choice[std::make_pair(nc, p->precision)].second);
    if (splits > 1) ST_TRY(b->ws_acc.ensure(static_cast<size_t>(splits) * nc * n3 * 8));
    if (p->precision != SIS_PREC_FP64)
      ST_TRY(b->ws_x.ensure(static_cast<size_t>(nc) * (p->precision == SIS_PREC_FP32 ? n3 : sis::pair_stride(n3)) * 4));
  }
  hipStream_t s = stream;
  if (o->use_graph && !b->persistent) {
    ST_TRY(hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking));
    s = b->cap;
  }
  if (sis_status st = state_init(b, s)) { delete b; return st; }
  if (o->use_graph && !b->persistent) {
    const int kinds = b->refresh > 1 ? 2 : 1;
    for (int k = 0; k < kinds; ++k) {
      ST_TRY(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
      sis_status st = state_iteration(b, b->cap, k);
      hipGraph_t gr = nullptr;
      hipError_t e = hipStreamEndCapture(b->cap, &gr);
      if (st) { if (gr) (void)hipGraphDestroy(gr); delete b; return st; }
      ST_TRY(e);
      b->graph[k] = gr;
      ST_TRY(hipGraphInstantiate(&b->exec[k], b->graph[k], nullptr, nullptr, 0));
    }
  }
#undef ST_TRY
  *out = b;
  g_err.clear();
  return SIS_OK;
}

sis_status sis_state_reset(sis_state_t b, hipStream_t stream) {
  if (!b) return fail(SIS_E_INVALID, "null state");
  return state_init(b, stream);
}

sis_status sis_state_step(sis_state_t b, int32_t n_iters, hipStream_t stream) {
  if (!b) return fail(SIS_E_INVALID, "null state");
  if (n_iters < 0) return fail(SIS_E_INVALID, "n_iters must be >= 0");
  if (b->persistent) {
    if (n_iters == 0) return SIS_OK;
    if (sis_status st = persistent_iterations(b, n_iters, stream)) return st;
    b->total += n_iters;
    return SIS_OK;
  }
  for (int i = 0; i < n_iters; ++i) {
    // FP64 anchors at iteration 0 (h = 0, free) and at R/2, 3R/2, ...: a case that converges
    // within R iterations is still anchored once after the start
    const bool anchor = b->total == 0 || (b->refresh > 1 && b->total % b->refresh == b->refresh / 2);
    const int kind = (b->refresh > 1 && !anchor) ? 1 : 0;
    if (b->total == 0) {
      // the iteration starts from h = 0 (set by state_init): run it eagerly without the contraction
      if (sis_status st = state_iteration(b, stream, kind, true)) return st;
    } else if (b->exec[kind]) {
      HIP_TRY(hipGraphLaunch(b->exec[kind], stream));
    } else if (sis_status st = state_iteration(b, stream, kind)) {
      return st;
    }
    ++b->total;
  }
  return SIS_OK;
}

sis_status sis_state_poll(sis_state_t b, int32_t* n_active, hipStream_t stream) {
  if (!b || !n_active) return fail(SIS_E_INVALID, "null argument");
  std::vector<int32_t> act(b->g->n_cases);
  HIP_TRY(hipMemcpyAsync(act.data(), b->cact, act.size() * 4, hipMemcpyDeviceToHost, stream));
  unsigned words[4] = {0, 0, 0, 0};
  if (b->persistent) HIP_TRY(hipMemcpyAsync(words, b->bar, sizeof(words), hipMemcpyDeviceToHost, stream));
  HIP_TRY(hipStreamSynchronize(stream));
  if (words[2] != 0) return fail(SIS_E_DEVICE, "persistent launch: a grid-barrier wait ran out (results invalid)");
  int n = 0;
  for (int32_t a : act) n += a != 0;
  *n_active = n;
  return SIS_OK;
}

sis_status sis_state_results(sis_state_t b, sis_solve_result* r, hipStream_t stream) {
  if (!b || !r) return fail(SIS_E_INVALID, "null argument");
  const int ncase = b->g->n_cases;
  const int64_t nc = b->g->n_cells;
  const int nsp = b->p->nsp, ss = 2 * nsp + 2;  // state: M[nsp], Q[nsp], residual, iterations
  HIP_TRY(hipStreamSynchronize(stream));
  std::vector<double> st(static_cast<size_t>(ncase) * ss);
  std::vector<int32_t> hit(ncase);
  HIP_TRY(hipMemcpy(st.data(), b->state, ncase * ss * 8, hipMemcpyDeviceToHost));
  HIP_TRY(hipMemcpy(hit.data(), b->iters, ncase * 4, hipMemcpyDeviceToHost));
  if (r->U) HIP_TRY(hipMemcpy(r->U, b->U, nc * nsp * 8, hipMemcpyDeviceToHost));
  if (r->q) HIP_TRY(hipMemcpy(r->q, b->q, nc * nsp * 8, hipMemcpyDeviceToHost));
  bool nan = false, notconv = false;
  for (int c = 0; c < ncase; ++c) {
    for (int s = 0; s < nsp; ++s) {
      const double M = st[c * ss + s], Q = st[c * ss + nsp + s];
      if (r->M) r->M[c * nsp + s] = M;
      if (r->Q) r->Q[c * nsp + s] = Q;
      if (!std::isfinite(M) || !std::isfinite(Q)) nan = true;
    }
    if (r->residual) r->residual[c] = st[c * ss + 2 * nsp];
    if (r->iters) r->iters[c] = hit[c];
    if (!(st[c * ss + 2 * nsp] < b->o.eps)) notconv = true;
  }
  r->seconds = 0.0;
  r->total_iters = b->total;
  if (nan) return fail(SIS_E_NUMERIC, "NaN/Inf in a flow rate");
  if (notconv) return fail(SIS_E_NOT_CONVERGED, "not every case has converged");
  g_err.clear();
  return SIS_OK;
}

sis_status sis_state_destroy(sis_state_t b) {
  if (!b) return fail(SIS_E_INVALID, "null state");
  delete b;
  return SIS_OK;
}

sis_status sis_solve(sis_plan_t p, sis_geom_t g, const sis_solve_opts* o, sis_solve_result* r,
                     hipStream_t user_stream) {
  if (!r) return fail(SIS_E_INVALID, "null result");
  hipStream_t s = user_stream;
  sis_state_t b = nullptr;
  if (sis_status st = sis_state_create(p, g, o, s, &b)) return st;
  const int every = o->check_every > 0 ? o->check_every : 4;
  auto t0 = std::chrono::steady_clock::now();
  int total = 0;
  for (;;) {
    const int k = std::min(every, o->max_it - total);
    if (sis_status st = sis_state_step(b, k, s)) { sis_state_destroy(b); return st; }
    total += k;
    int32_t active = 0;
    if (sis_status st = sis_state_poll(b, &active, s)) { sis_state_destroy(b); return st; }
    if (active == 0 || total >= o->max_it) break;
  }
  auto t1 = std::chrono::steady_clock::now();
  sis_status st = sis_state_results(b, r, s);
  r->seconds = std::chrono::duration<double>(t1 - t0).count();
  std::string keep = g_err;
  sis_state_destroy(b);
  g_err = keep;
  return st;
}

sis_status sis_plan_set_contraction_config(sis_plan_t p, int64_t n_cells, int32_t precision, int32_t tile_rows,
                                           int32_t k_stage, int32_t splits) {
  if (sis_status st = check_plan(p)) return st;
  if (precision < SIS_PREC_FP64 || precision > SIS_PREC_BF16) return fail(SIS_E_INVALID, "unknown precision");
  if (splits < 1 || splits > 32) return fail(SIS_E_INVALID, "splits must be in [1, 32]");
  int tile = -1;
  if (precision == SIS_PREC_BF16X3 && tile_rows == 256 && k_stage == 32) {
    tile = 5;
  } else if (precision == SIS_PREC_BF16X3 || precision == SIS_PREC_BF16) {
    if (k_stage == 64) tile = tile_rows == 128 ? 0 : tile_rows == 64 ? 2 : tile_rows == 32 ? 1 : -1;
  } else if (k_stage == 16) {
    tile = tile_rows == 128 ? 0 : tile_rows == 64 ? 2 : tile_rows == 32 ? 1 : -1;
  } else if (k_stage == 32 && precision == SIS_PREC_FP64) {
    tile = tile_rows == 128 ? 3 : tile_rows == 64 ? 4 : -1;
  }
  if (tile < 0) return fail(SIS_E_INVALID, "no contraction tile of %d rows with k-stage %d for this precision", tile_rows, k_stage);
  if (tile == 5 && !sis::gemm_wide_fits(n_cells, p->ndof, p->ndof))
    return fail(SIS_E_UNSUPPORTED, "the 256 x 256 tile needs both bf16 pair arrays under 4 GiB");
  p->gemm_choice[std::make_pair(n_cells, static_cast<int>(precision))] = std::make_pair(tile, static_cast<int>(splits));
  return SIS_OK;
}

sis_status sis_plan_contraction_config(sis_plan_t p, int64_t n_cells, int32_t precision, int32_t* tile_rows,
                                       int32_t* splits, int32_t* tuned, int32_t* k_stage) {
  if (sis_status st = check_plan(p)) return st;
  if (!tile_rows || !splits || !tuned) return fail(SIS_E_INVALID, "null output");
  int t, s;
  const auto it = p->gemm_choice.find(std::make_pair(n_cells, static_cast<int>(precision)));
  if (it != p->gemm_choice.end()) {
    t = it->second.first;
    s = it->second.second;
    *tuned = 1;
  } else {
    choose_gemm(n_cells, p->ndof, &t, &s);
    *tuned = 0;
  }
  *tile_rows = sis::gemm_tile_rows(t);
  *splits = s;
  if (k_stage) *k_stage = sis::gemm_tile_depth(t, precision);
  return SIS_OK;
}

sis_status sis_plan_timing(sis_plan_t p, int32_t enable) {
  if (sis_status st = check_plan(p)) return st;
  for (auto& e : p->events) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
  p->events.clear();
  for (auto& e : p->fsm_events) { (void)hipEventDestroy(e.first); (void)hipEventDestroy(e.second); }
  p->fsm_events.clear();
  p->timing = enable != 0;
  return SIS_OK;
}

sis_status sis_plan_timing_read(sis_plan_t p, double* ms, int64_t* launches) {
  if (sis_status st = check_plan(p)) return st;
  double tot = 0.0;
  for (auto& e : p->events) {
    HIP_TRY(hipEventSynchronize(e.second));
    float t = 0.f;
    HIP_TRY(hipEventElapsedTime(&t, e.first, e.second));
    tot += t;
  }
  if (ms) *ms = tot;
  if (launches) *launches = static_cast<int64_t>(p->events.size());
  return SIS_OK;
}

}  // extern "C"
