// Device kernels of the SIS hot path for gfx950 (CDNA4, 64-wide wavefronts).
//
//  assemble      plan-time: dense matrix of h -> L+(h) from the fast-spectral
//                real-space kernels (one 32x32 output tile per workgroup,
//                direction tables staged through LDS)
//  gemm          collision contraction acc = X * op^T on MFMA
//                (FP64 v_mfma_f64_16x16x4; FP32 / 3xBF16 variants)
//  finish        per-cell epilogue: correction of eq. guided, delta scaling,
//                source, L, moments A1/A2, invariant projection
//  sweep1d       upwind transport sweep per velocity pair (+v1, -v1),
//                moments of h^{k+1/2} as per-wave partial sums
//  diffusion1d   per-case march of the SIS velocity equation, flow rates,
//                convergence test
#include <hip/hip_runtime.h>

#include "kernels.h"

namespace sis {

namespace {

typedef double v4d __attribute__((ext_vector_type(4)));
typedef float v4f __attribute__((ext_vector_type(4)));
typedef __attribute__((address_space(3))) void lds_void_t;
typedef __attribute__((address_space(1))) void gbl_void_t;

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o >= 1; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Block-wide sum of K values per thread, fixed order.  Result in out[] for all threads.
template <int K>
__device__ inline void block_sum(double (&v)[K], double* sh /* >= 4*K */) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const double s = wave_sum(v[k]);
    if (lane == 0) sh[wave * K + k] = s;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += sh[w * K + k];
    v[k] = s;
  }
  __syncthreads();
}

// ------------------------------------------------------------------ assemble
constexpr int kAsmPB = 8;      // terms staged per LDS round
constexpr int kAsmOuts = 7;    // outputs per thread (n^2 <= 256 * 7)

// One workgroup per (i0 i1, j0 j1) pair of velocity rows: the n x n outputs
// (i2, j2) share the difference row (d0, d1) of every kernel table.
__global__ __launch_bounds__(256) void assemble_kernel(int n, int T, const double* __restrict__ X,
                                                       const double* __restrict__ Y,
                                                       const double* __restrict__ feq, double lossc,
                                                       const double* __restrict__ beta_r,
                                                       double* __restrict__ op, int64_t ldo, int accumulate) {
  const int nd = 2 * n - 1;
  const int n3 = n * n * n;
  const int bi = blockIdx.x, bj = blockIdx.y;
  const int i0 = bi / n, i1 = bi % n, j0 = bj / n, j1 = bj % n;
  const int d0 = i0 - j0 + n - 1, d1 = i1 - j1 + n - 1;
  extern __shared__ double sm[];
  double* sY = sm;
  double* sX = sm + kAsmPB * nd;
  const int nout = n * n;
  double acc[kAsmOuts];
#pragma unroll
  for (int k = 0; k < kAsmOuts; ++k) acc[k] = 0.0;
  const size_t row = (static_cast<size_t>(d0) * nd + d1) * nd;
  const size_t nd3 = static_cast<size_t>(nd) * nd * nd;
  for (int t0 = 0; t0 < T; t0 += kAsmPB) {
    const int tb = min(kAsmPB, T - t0);
    for (int q = threadIdx.x; q < tb * nd; q += blockDim.x) {
      const int tt = q / nd, r = q % nd;
      sY[tt * nd + r] = Y[static_cast<size_t>(t0 + tt) * nd3 + row + r];
    }
    for (int q = threadIdx.x; q < tb * n; q += blockDim.x) {
      const int tt = q / n, r = q % n;
      sX[tt * n + r] = X[static_cast<size_t>(t0 + tt) * n3 + static_cast<size_t>(bi) * n + r];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kAsmOuts; ++k) {
      const int o = threadIdx.x + k * blockDim.x;
      if (o < nout) {
        const int i2 = o / n, j2 = o % n, dd = i2 - j2 + n - 1;
        double a = acc[k];
        for (int tt = 0; tt < tb; ++tt) a += sX[tt * n + i2] * sY[tt * nd + dd];
        acc[k] = a;
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int k = 0; k < kAsmOuts; ++k) {
    const int o = threadIdx.x + k * blockDim.x;
    if (o < nout) {
      const int i2 = o / n, j2 = o % n, dd = i2 - j2 + n - 1;
      const int ii = bi * n + i2, jj = bj * n + j2;
      double v = acc[k];
      if (feq) v -= lossc * feq[ii] * beta_r[row + dd];
      double* dst = op + static_cast<size_t>(ii) * ldo + jj;
      *dst = accumulate ? *dst + v : v;
    }
  }
}

// Restriction of the operator to distributions odd in v3 (and even in v2):
// red[i][j] = sum over the mirror images s(j) of j of sign(s) op[i][s(j)],
// rows and columns over the stored half (quarter) grid of every species.
__global__ void reduce_operator_kernel(const double* __restrict__ op, int64_t ld, double* __restrict__ red,
                                       int nsp, int n, int parity) {
  const int d2 = parity == 2 ? n / 2 : n, d3 = n / 2;
  const int nv = n * d2 * d3, n3 = n * n * n;
  const int64_t ldr = static_cast<int64_t>(nsp) * nv;
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= ldr * ldr) return;
  const int64_t ri = idx / ldr, rj = idx % ldr;
  auto full = [&](int64_t r) {  // full-grid index of a stored (species, velocity) row
    const int s = static_cast<int>(r / nv), v = static_cast<int>(r % nv);
    const int j1 = v / (d2 * d3), j2 = (v / d3) % d2 + (n - d2), j3 = v % d3 + n / 2;
    return static_cast<int64_t>(s) * n3 + (static_cast<int64_t>(j1) * n + j2) * n + j3;
  };
  const int64_t fi = full(ri), fj = full(rj);
  const int j3 = static_cast<int>(fj % n), j2 = static_cast<int>((fj / n) % n);
  const int64_t m3 = fj + (n - 1 - 2 * j3);            // v3 -> -v3
  const double* row = op + fi * ld;
  double s = row[fj] - row[m3];
  if (parity == 2) {
    const int64_t dm2 = static_cast<int64_t>(n - 1 - 2 * j2) * n;  // v2 -> -v2
    s += row[fj + dm2] - row[m3 + dm2];
  }
  red[idx] = s;
}

__global__ void convert_f32_kernel(const double* __restrict__ in, float* __restrict__ out, int64_t count) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < count) out[i] = static_cast<float>(in[i]);
}

__device__ inline uint16_t bf16_rne(float f) {
  const uint32_t b = __float_as_uint(f);
  const uint32_t r = b + 0x7FFFu + ((b >> 16) & 1u);
  return static_cast<uint16_t>(r >> 16);
}
__device__ inline float bf16_to_f32(uint16_t h) { return __uint_as_float(static_cast<uint32_t>(h) << 16); }

// BF16 pair layout of the low-precision contraction operands (rows of K values,
// stored with Kp = K rounded up to 64): row r occupies 2 Kp bf16, and each block of
// 32 k-values holds its 32 hi parts followed by their 32 lo parts, so that one
// 128-byte line carries everything a 32-deep stage needs of the row.  Entries
// k >= K are zero in both halves.  x = X - Xref (Xref null: X); hi = RNE(x),
// lo = RNE(x - hi), or lo = 0 when with_lo is 0.
__global__ void split_pairs_kernel(const double* __restrict__ X, const double* __restrict__ Xref, int64_t rows,
                                   int K, int Kp, uint16_t* __restrict__ P, int with_lo) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= rows * Kp) return;
  const int64_t r = i / Kp;
  const int k = static_cast<int>(i - r * Kp);
  double x = 0.0;
  if (k < K) x = Xref ? X[r * K + k] - Xref[r * K + k] : X[r * K + k];
  const uint16_t h = bf16_rne(static_cast<float>(x));
  const uint16_t l = with_lo ? bf16_rne(static_cast<float>(x - static_cast<double>(bf16_to_f32(h)))) : 0;
  uint16_t* row = P + r * 2 * Kp + (k >> 5) * 64 + (k & 31);
  row[0] = h;
  row[32] = l;
}

// ------------------------------------------------------------------ FP64 MFMA GEMM
// acc[z][m][n] = sum_{k in [z*kps, min(K,(z+1)*kps))} X[m][k] * Op[n][k]
// Both operands are k-contiguous.  LDS tiles are stored k-major so that the
// 16 lanes of an MFMA operand column read 16 consecutive doubles.
constexpr int kBK = 16;
constexpr int kPad = 4;

// BK: k-depth of a stage; NBUF = 2: double-buffered LDS, software-pipelined: the next
// stage's global loads are issued at the start of a stage and written to the other LDS buffer
// two k-steps before its end, and the stage's one barrier sits before its last k-step's MFMAs,
// so that the next stage's first LDS reads overlap them.  NBUF = 1: one buffer (two barriers
// per stage, half the LDS, so deeper stages fit twice per CU).  PAD: row padding of the
// k-major LDS tiles (PAD = 1 with BK = 32 spreads the 64-lane stores of 16 k-rows x 4 rows
// over the banks).
// XCD-aware tile order of the contractions.  Workgroups go to the 8 XCDs
// round-robin in dispatch order, so each XCD's L2 would otherwise see cell and
// operator tiles from all over the grid.  Each XCD instead takes a contiguous
// run of the tile sequence, walked in groups of kGroup cell-tile rows (cell
// tile fastest), so the workgroups resident on one XCD share a few cell and
// operator tiles per k-stage.  A permutation of the (x, y) tiles: results are
// unchanged.  Returns the cell tile in .y and the operator tile in .x.
template <int kGroup = 8>
__device__ inline int2 xcd_tile() {
  const int gx = gridDim.x, gy = gridDim.y, total = gx * gy;
  int b = blockIdx.y * gx + blockIdx.x;
  if (total % 8 == 0) b = (b % 8) * (total / 8) + b / 8;
  const int first_y = (b / (kGroup * gx)) * kGroup;
  const int rows_in_group = min(kGroup, gy - first_y);
  const int in_group = b - first_y * gx;
  return make_int2(in_group / rows_in_group, first_y + in_group % rows_in_group);
}

// One output tile (operator tile bx, cell tile by, split bz) of the FP64 contraction; called by
// gemm_f64_kernel with the block indices and by the persistent 1-D iteration over virtual tiles.
template <int BM, int BN, int WM, int WN, int BK = kBK, int NBUF = 2, int PAD = kPad>
__device__ __forceinline__ void gemm_f64_tile(const double* __restrict__ X, const double* __restrict__ Op,
                                              double* __restrict__ C, int64_t M, int N, int K, int kps, int bx,
                                              int by, int bz) {
  constexpr int WAVES_N = BN / WN;
  constexpr int TM = WM / 16, TN = WN / 16;
  constexpr int A_LD = BM * BK / 2 / 256;
  constexpr int B_LD = BN * BK / 2 / 256;
  static_assert((BM / WM) * (BN / WN) == 4, "4 waves per workgroup");
  static_assert(A_LD >= 1 && B_LD >= 1, "tile too small");
  __shared__ double As[NBUF][BK][BM + PAD];
  __shared__ double Bs[NBUF][BK][BN + PAD];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave / WAVES_N) * WM, wn = (wave % WAVES_N) * WN;
  // plain grid order: the MFMA-bound FP64 tiles measured no faster (planar batch slower) with xcd_tile()
  const int64_t m0 = static_cast<int64_t>(by) * BM;
  const int n0 = bx * BN;
  const int kbeg = bz * kps;
  const int kend = min(K, kbeg + kps);
  double* Cz = C + static_cast<int64_t>(bz) * M * N;

  double2 ra[A_LD], rb[B_LD];
  auto gload = [&](int k0) {
#pragma unroll
    for (int i = 0; i < A_LD; ++i) {
      const int q = tid + 256 * i;
      const int r = q / (BK / 2), kc = (q % (BK / 2)) * 2;
      const int64_t gm = m0 + r;
      const int gk = k0 + kc;
      ra[i] = (gm < M && gk < kend) ? *reinterpret_cast<const double2*>(X + gm * K + gk)
                                    : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int i = 0; i < B_LD; ++i) {
      const int q = tid + 256 * i;
      const int r = q / (BK / 2), kc = (q % (BK / 2)) * 2;
      const int gn = n0 + r;
      const int gk = k0 + kc;
      rb[i] = (gn < N && gk < kend)
                  ? *reinterpret_cast<const double2*>(Op + static_cast<int64_t>(gn) * K + gk)
                  : make_double2(0.0, 0.0);
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int i = 0; i < A_LD; ++i) {
      const int q = tid + 256 * i;
      const int r = q / (BK / 2), kc = (q % (BK / 2)) * 2;
      As[buf][kc][r] = ra[i].x;
      As[buf][kc + 1][r] = ra[i].y;
    }
#pragma unroll
    for (int i = 0; i < B_LD; ++i) {
      const int q = tid + 256 * i;
      const int r = q / (BK / 2), kc = (q % (BK / 2)) * 2;
      Bs[buf][kc][r] = rb[i].x;
      Bs[buf][kc + 1][r] = rb[i].y;
    }
  };

  v4d acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};

  const int nk = kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;
  if (nk > 0) {
    gload(kbeg);
    sstore(0);
  }
  __syncthreads();
  const int kr = lane >> 4, cc = lane & 15;
  if constexpr (NBUF == 2) {
    static_assert((BK / 4) % 2 == 0, "an even number of k-steps per stage");
    constexpr int KS = BK / 4, KW = KS - 2;
    double a[2][TM], b[2][TN];
    auto lread = [&](int buf, int kk, double* ar, double* br) {
#pragma unroll
      for (int i = 0; i < TM; ++i) ar[i] = As[buf][kk * 4 + kr][wm + i * 16 + cc];
#pragma unroll
      for (int j = 0; j < TN; ++j) br[j] = Bs[buf][kk * 4 + kr][wn + j * 16 + cc];
    };
    if (nk > 0) lread(0, 0, a[0], b[0]);
    for (int kt = 0; kt < nk; ++kt) {
      const int cur = kt & 1;
      const bool more = kt + 1 < nk;
      if (more) gload(kbeg + (kt + 1) * BK);
#pragma unroll
      for (int kk = 0; kk < KS; ++kk) {
        const int c = kk & 1;
        if (kk + 1 < KS) lread(cur, kk + 1, a[c ^ 1], b[c ^ 1]);
        if (kk == KW && more) sstore(cur ^ 1);
        if (kk == KS - 1) {
          __syncthreads();       // next buffer written by every wave, this one read by every wave
          if (more) lread(cur ^ 1, 0, a[c ^ 1], b[c ^ 1]);
        }
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[c][i], b[c][j], acc[i][j], 0, 0, 0);
      }
    }
  } else {
    static_assert(NBUF == 1, "one or two LDS buffers");
    for (int kt = 0; kt < nk; ++kt) {
      const int cur = 0;
      if (kt + 1 < nk) gload(kbeg + (kt + 1) * BK);
      // operands of k-step kk + 1 are read from LDS into the other register set
      // while the MFMAs of k-step kk run
      double a[2][TM], b[2][TN];
      auto lread = [&](int kk, double* ar, double* br) {
#pragma unroll
        for (int i = 0; i < TM; ++i) ar[i] = As[cur][kk * 4 + kr][wm + i * 16 + cc];
#pragma unroll
        for (int j = 0; j < TN; ++j) br[j] = Bs[cur][kk * 4 + kr][wn + j * 16 + cc];
      };
      lread(0, a[0], b[0]);
#pragma unroll
      for (int kk = 0; kk < BK / 4; ++kk) {
        const int c = kk & 1;
        if (kk + 1 < BK / 4) lread(kk + 1, a[c ^ 1], b[c ^ 1]);
#pragma unroll
        for (int i = 0; i < TM; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[c][i], b[c][j], acc[i][j], 0, 0, 0);
      }
      // Schedule of the block above (a hint to the compiler's scheduler, which otherwise sinks
      // the reads behind the MFMAs that use the other register set): the first step's reads,
      // then per step one MFMA, the next step's LDS reads (ds_read2: two operands each), the
      // step's other MFMAs.
      constexpr int kReads = (TM + 1) / 2 + (TN + 1) / 2;
      __builtin_amdgcn_sched_group_barrier(0x100, kReads, 0);
#pragma unroll
      for (int kk = 0; kk + 1 < BK / 4; ++kk) {
        __builtin_amdgcn_sched_group_barrier(0x008, 1, 0);
        __builtin_amdgcn_sched_group_barrier(0x100, kReads, 0);
        __builtin_amdgcn_sched_group_barrier(0x008, TM * TN - 1, 0);
      }
      __builtin_amdgcn_sched_group_barrier(0x008, TM * TN, 0);
      __syncthreads();           // every wave is done with the buffer
      if (kt + 1 < nk) sstore(0);
      __syncthreads();
    }
  }
  // D layout of the 16x16x4 FP64 MFMA: lane l, element r -> row (l/16) + 4 r,
  // column l%16 (rows interleaved, unlike the FP32 forms)
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gm = m0 + wm + i * 16 + kr + 4 * r;
        const int gn = n0 + wn + j * 16 + cc;
        if (gm < M && gn < N) Cz[gm * N + gn] = acc[i][j][r];
      }
}

template <int BM, int BN, int WM, int WN, int BK = kBK, int NBUF = 2, int PAD = kPad>
__global__ __launch_bounds__(256) void gemm_f64_kernel(const double* __restrict__ X, const double* __restrict__ Op,
                                                       double* __restrict__ C, int64_t M, int N, int K, int kps) {
  gemm_f64_tile<BM, BN, WM, WN, BK, NBUF, PAD>(X, Op, C, M, N, K, kps, blockIdx.x, blockIdx.y, blockIdx.z);
}

// FP64 contraction on 128 x 128 tiles with LDS-DMA staging: the 128-row tile of the
// autotuner and the default heuristic.  Eight waves (4 along the cells x 2 along the
// operator rows) of 32 x 64 outputs: 2 x 4 blocks of the 16x16x4 FP64 MFMA, 64
// accumulator registers per lane, 127 registers in all, so two workgroups per CU give
// four waves per SIMD to cover each other's barrier and LDS waits.
// A stage is 16 deep and holds k pairs: slot (p, r) of an operand is the 16 bytes
// (k = 2p, 2p + 1) of its row r, 8 pairs x 128 rows per operand, 32 KB per stage with
// both operands.  Lane (kq, c) of an MFMA block reads one pair, (kq + 4 h, c), and feeds
// its first element to one MFMA and its second to the next, so a step of two MFMAs
// covers k = 2 kq + 8 h + {0, 1} over the four lane groups kq and a stage is two such
// ds_read_b128 steps (h = 0, 1) per block.  The stages are written by buffer-load LDS
// DMA (each lane's 16 bytes land at slot (8 j + wave) * 64 + lane of the operand's half
// of the stage for its instruction j, i.e. pair slot / 128, row slot % 128), so no registers or LDS stores
// carry the staging and the rows are copied without the transposing stores of the
// register-staged kernel.  The buffer descriptors start at the tile's first row and end
// after its last valid row; a pair past the split's k range gets an offset beyond the
// end: both read as zeros, which pads ragged cell, operator and k tails.
// Two stage buffers (distinct LDS objects, so that the compiler's LDS-DMA wait tracking
// lets reads of one proceed while the other is filled) and one barrier per stage: before
// it this wave's DMA of the next stage has landed (vmcnt(0)) and its reads of the current
// stage have completed; after it the next stage is visible to every wave and the current
// buffer is free, so the next stage's first reads are issued, then the DMA of the stage
// after it into the freed buffer, then the MFMAs of the current stage's second step.
// Preconditions (checked by the launcher): K even, K <= 2^20 (32-bit offsets within a
// tile's 128 rows).
__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(4))) void gemm_f64_dma_kernel(
    const double* __restrict__ X, const double* __restrict__ Op, double* __restrict__ C, int64_t M, int N, int K,
    int kps) {
  __shared__ double2 buf0[2048];   // [operand][pair 0..7][row 0..127]
  __shared__ double2 buf1[2048];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  // tiles to the XCDs in runs walked in groups of 8 cell-tile rows: the duct's fabric traffic
  // drops from 95 to 40 GB per launch at equal speed (groups of 2, 4, 16, 32: 68, 53, 45, 85 GB)
  const int2 tile = xcd_tile<8>();
  const int64_t m0 = static_cast<int64_t>(tile.y) * 128;
  const int n0 = tile.x * 128;
  const int kbeg = blockIdx.z * kps;
  const int kend = min(K, kbeg + kps);
  const int nk = kend > kbeg ? (kend - kbeg + 15) / 16 : 0;
  double* Cz = C + static_cast<int64_t>(blockIdx.z) * M * N;

  const int rows_a = static_cast<int>(min<int64_t>(128, M - m0));
  const int rows_b = min(128, N - n0);
  const __amdgpu_buffer_rsrc_t rs_a =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(X + m0 * K), 0, rows_a * K * 8, 0x00020000);
  const __amdgpu_buffer_rsrc_t rs_b = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<double*>(Op + static_cast<int64_t>(n0) * K), 0, rows_b * K * 8, 0x00020000);
  // per DMA instruction j of this wave: the lane's pair and its byte offset within the tile
  uint32_t roff[2];
  int pj[2];
#pragma unroll
  for (int j = 0; j < 2; ++j) {
    const int slot = (8 * j + wave) * 64 + lane;
    pj[j] = slot >> 7;
    roff[j] = static_cast<uint32_t>(((slot & 127) * K + 2 * pj[j]) * 8);
  }
  auto issue = [&](double2* buf, int k0) {
    const int krem = kend - k0;
    const uint32_t kb = static_cast<uint32_t>(k0) * 8u;
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const uint32_t vo = 2 * pj[j] < krem ? roff[j] + kb : 0x80000000u;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rs_a, (lds_void_t*)&buf[(8 * j + wave) * 64], 16, vo, 0, 0, 0);
    }
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const uint32_t vo = 2 * pj[j] < krem ? roff[j] + kb : 0x80000000u;
      __builtin_amdgcn_raw_ptr_buffer_load_lds(rs_b, (lds_void_t*)&buf[1024 + (8 * j + wave) * 64], 16, vo, 0, 0,
                                               0);
    }
    __builtin_amdgcn_sched_barrier(0);
  };

  const int kq = lane >> 4, cc = lane & 15;
  const int wm = (wave >> 1) * 32, wn = (wave & 1) * 64;
  v4d acc[2][4];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = v4d{0.0, 0.0, 0.0, 0.0};
  double2 a0[2], b0[4], a1[2], b1[4];
  auto lread = [&](const double2* buf, int h, double2* ar, double2* br) {
#pragma unroll
    for (int i = 0; i < 2; ++i) ar[i] = buf[(kq + 4 * h) * 128 + wm + 16 * i + cc];
#pragma unroll
    for (int j = 0; j < 4; ++j) br[j] = buf[1024 + (kq + 4 * h) * 128 + wn + 16 * j + cc];
  };
  auto mfma = [&](const double2* ar, const double2* br) {
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i].x, br[j].x, acc[i][j], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(ar[i].y, br[j].y, acc[i][j], 0, 0, 0);
  };
  // the stage in `cur` (its first step's operands already in a0, b0), the next one landing
  // in `nxt`; the DMA of stage k_dma goes to `cur` once every wave is past the barrier.  The
  // sched_barriers keep the MFMAs on their side of the barrier (they touch no memory, so the
  // scheduler would otherwise move them across it).
  // The wave's priority is raised from the barrier until the DMA is issued, so that the memory
  // instructions after the barrier are not held behind other waves' MFMAs (planar batch 1.74 ->
  // 1.70 ms, other shapes unchanged).
  auto stage = [&](double2* cur, double2* nxt, int k_dma) {
    lread(cur, 1, a1, b1);
    mfma(a0, b0);
    __builtin_amdgcn_sched_barrier(0);
    __builtin_amdgcn_s_setprio(1);
    __builtin_amdgcn_s_waitcnt(0x0f70);
    __syncthreads();
    lread(nxt, 0, a0, b0);
    __builtin_amdgcn_sched_barrier(0);
    issue(cur, k_dma);
    __builtin_amdgcn_s_setprio(0);
    mfma(a1, b1);
    __builtin_amdgcn_sched_barrier(0);
  };

  if (nk > 0) {
    issue(buf0, kbeg);
    __builtin_amdgcn_s_waitcnt(0x0f70);
    __syncthreads();
    issue(buf1, kbeg + (nk > 1 ? 16 : 0));
    lread(buf0, 0, a0, b0);
  }
  // stage pairs with the buffers named statically, then an odd last stage; past the last
  // stage the DMA target is clamped to the first stage (the freed buffer is not read again)
  int s = 0;
  for (; s + 1 < nk; s += 2) {
    stage(buf0, buf1, kbeg + (s + 2 < nk ? s + 2 : 0) * 16);
    stage(buf1, buf0, kbeg + (s + 3 < nk ? s + 3 : 0) * 16);
  }
  if (s < nk) {
    lread(buf0, 1, a1, b1);
    mfma(a0, b0);
    mfma(a1, b1);
  }
  // drain the clamped DMA before the workgroup can end
  __builtin_amdgcn_s_waitcnt(0x0f70);
  // D layout of the 16x16x4 FP64 MFMA: lane l, element r -> row l/16 + 4 r, column l%16
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gm = m0 + wm + i * 16 + kq + 4 * r;
        const int gn = n0 + wn + j * 16 + cc;
        if (gm < M && gn < N) Cz[gm * N + gn] = acc[i][j][r];
      }
}

// ------------------------------------------------------------------ FP32 MFMA GEMM
// X is converted from double to float when staged; op is stored as float.
template <int BM, int BN, int WM, int WN>
__global__ __launch_bounds__(256) void gemm_f32_kernel(const float* __restrict__ X,
                                                       const float* __restrict__ Op,
                                                       double* __restrict__ C, int64_t M, int N,
                                                       int K, int kps) {
  constexpr int BK = 32;
  constexpr int WAVES_N = BN / WN;
  constexpr int TM = WM / 16, TN = WN / 16;
  constexpr int A_LD = BM * BK / 4 / 256;   // float4 loads of the (pre-rounded) cell operand
  constexpr int B_LD = BN * BK / 4 / 256;   // float4 loads of Op
  static_assert((BM / WM) * (BN / WN) == 4, "4 waves per workgroup");
  static_assert(A_LD >= 1 && B_LD >= 1, "tile too small");
  __shared__ float As[2][BK][BM + 4];
  __shared__ float Bs[2][BK][BN + 4];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave / WAVES_N) * WM, wn = (wave % WAVES_N) * WN;
  const int64_t m0 = static_cast<int64_t>(blockIdx.y) * BM;
  const int n0 = blockIdx.x * BN;
  const int kbeg = blockIdx.z * kps;
  const int kend = min(K, kbeg + kps);
  double* Cz = C + static_cast<int64_t>(blockIdx.z) * M * N;

  float4 ra[A_LD];
  float4 rb[B_LD];
  auto gload = [&](int k0) {
#pragma unroll
    for (int i = 0; i < A_LD; ++i) {
      const int q = tid + 256 * i;
      const int r = q / (BK / 4), kc = (q % (BK / 4)) * 4;
      const int64_t gm = m0 + r;
      const int gk = k0 + kc;
      if (gm < M && gk + 3 < kend) {
        ra[i] = *reinterpret_cast<const float4*>(X + gm * K + gk);
      } else {
        float t[4];
        for (int e = 0; e < 4; ++e) t[e] = (gm < M && gk + e < kend) ? X[gm * K + gk + e] : 0.0f;
        ra[i] = make_float4(t[0], t[1], t[2], t[3]);
      }
    }
#pragma unroll
    for (int i = 0; i < B_LD; ++i) {
      const int q = tid + 256 * i;
      const int r = q / (BK / 4), kc = (q % (BK / 4)) * 4;
      const int gn = n0 + r;
      const int gk = k0 + kc;
      if (gn < N && gk + 3 < kend) {
        rb[i] = *reinterpret_cast<const float4*>(Op + static_cast<int64_t>(gn) * K + gk);
      } else {
        float t[4];
        for (int e = 0; e < 4; ++e)
          t[e] = (gn < N && gk + e < kend) ? Op[static_cast<int64_t>(gn) * K + gk + e] : 0.0f;
        rb[i] = make_float4(t[0], t[1], t[2], t[3]);
      }
    }
  };
  auto sstore = [&](int buf) {
#pragma unroll
    for (int i = 0; i < A_LD; ++i) {
      const int q = tid + 256 * i;
      const int r = q / (BK / 4), kc = (q % (BK / 4)) * 4;
      As[buf][kc][r] = ra[i].x;
      As[buf][kc + 1][r] = ra[i].y;
      As[buf][kc + 2][r] = ra[i].z;
      As[buf][kc + 3][r] = ra[i].w;
    }
#pragma unroll
    for (int i = 0; i < B_LD; ++i) {
      const int q = tid + 256 * i;
      const int r = q / (BK / 4), kc = (q % (BK / 4)) * 4;
      Bs[buf][kc][r] = rb[i].x;
      Bs[buf][kc + 1][r] = rb[i].y;
      Bs[buf][kc + 2][r] = rb[i].z;
      Bs[buf][kc + 3][r] = rb[i].w;
    }
  };

  v4f acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

  const int nk = kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;
  if (nk > 0) {
    gload(kbeg);
    sstore(0);
  }
  __syncthreads();
  const int kr = lane >> 4, cc = lane & 15;
  for (int kt = 0; kt < nk; ++kt) {
    const int cur = kt & 1;
    if (kt + 1 < nk) gload(kbeg + (kt + 1) * BK);
#pragma unroll
    for (int kk = 0; kk < BK / 4; ++kk) {
      float a[TM], b[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) a[i] = As[cur][kk * 4 + kr][wm + i * 16 + cc];
#pragma unroll
      for (int j = 0; j < TN; ++j) b[j] = Bs[cur][kk * 4 + kr][wn + j * 16 + cc];
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j)
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    if (kt + 1 < nk) sstore(cur ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gm = m0 + wm + i * 16 + kr * 4 + r;
        const int gn = n0 + wn + j * 16 + cc;
        if (gm < M && gn < N) Cz[gm * N + gn] = static_cast<double>(acc[i][j][r]);
      }
}

// ------------------------------------------------------------------ 3xBF16 MFMA GEMM
// x ~ xh + xl, op ~ oh + ol (bf16 pairs); acc += xl*oh + xh*ol + xh*oh on
// v_mfma_f32_16x16x32_bf16 with FP32 accumulation.  Both operands arrive in the
// pair layout of split_pairs_kernel (the cell operand is split once per launch
// instead of once per output tile; Kp is a multiple of 64, so every stage is
// full).  k-stage of 64 staged through one LDS buffer per operand half; the next
// stage is prefetched into registers while the current one feeds the MFMAs.
typedef __bf16 v8bf __attribute__((ext_vector_type(8)));
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// NPROD = 1: the hi*hi product alone (lo halves neither loaded nor staged).
// FUSED (32-row tile only): the cell operand is read in FP64 (X, minus Xref when given; K values
// per row) and split into its hi and lo parts while it is staged, exactly as split_pairs_kernel
// does, so that a launch on few cells needs no separate split kernel; results are bit-identical.
template <int BM, int BN, int WM, int WN, int NPROD = 3, bool FUSED = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void gemm_bf16x3_kernel(
    const uint16_t* __restrict__ Xp, const uint16_t* __restrict__ Op, double* __restrict__ C, int64_t M, int N, int Kp,
    int kps, const double* __restrict__ X, const double* __restrict__ Xref, int K) {
  constexpr int BK = 64;                      // two MFMA k-steps per stage
  constexpr int WAVES_N = BN / WN;
  constexpr int TM = WM / 16, TN = WN / 16;
  constexpr int CH = BK / 8;                  // 16-byte chunks per row and stage
  constexpr int A_LD = BM * CH / 256;
  constexpr int B_LD = BN * CH / 256;
  static_assert(BM * CH % 256 == 0 && BN * CH % 256 == 0, "whole staging passes");
  static_assert((BM / WM) * (BN / WN) == 4, "4 waves per workgroup");
  // rows hold the 64 k-values of one m (or n) as eight 16-byte chunks, chunk c
  // of row r stored at slot c ^ ((r / 2) % 8): the 16 rows one MFMA operand read
  // touches and the two rows a 16-lane group of staging writes fills each
  // cover distinct banks.  A lane reads its 8 consecutive k values as one
  // 16-byte vector.
  constexpr int RS = BK;
  static_assert(CH == 8, "eight 16-byte chunks per row");
  __shared__ uint16_t sA[NPROD == 3 ? 2 : 1][BM][RS];
  __shared__ uint16_t sB[NPROD == 3 ? 2 : 1][BN][RS];

  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = (wave / WAVES_N) * WM, wn = (wave % WAVES_N) * WN;
  // Swizzled slots are per-thread constants.  Staging: thread q = tid + 256 i
  // writes chunk tid % 8 of row tid / 8 + 32 i, so (row / 2) % 8 = (tid / 16) % 8.
  // Operand reads: rows wm + 16 i + lane % 16 (wm, 16 i multiples of 16), chunk
  // ks / 8 + lane / 16.
  const int wslot = ((tid & 7) ^ ((tid >> 4) & 7)) << 3;
  const int rsw = (lane & 15) >> 1;
  const int rslot0 = ((lane >> 4) ^ rsw) << 3, rslot1 = ((4 + (lane >> 4)) ^ rsw) << 3;
  const int2 tile = xcd_tile();
  const int64_t m0 = static_cast<int64_t>(tile.y) * BM;
  const int n0 = tile.x * BN;
  const int kbeg = blockIdx.z * kps;
  const int kend = min(Kp, kbeg + kps);
  double* Cz = C + static_cast<int64_t>(blockIdx.z) * M * N;

  // (native vectors: HIP's uint4 struct copies from global memory kept the staging in scratch)
  u32x4 ra[2][A_LD], rb[2][B_LD];
  static_assert(!FUSED || A_LD == 1, "the fused split stages one chunk of eight values per thread");
  double2 xa[4], xr[4];   // FUSED: the eight FP64 values of the thread's chunk (and of the anchor)
  // hi chunk of (row, k), k a multiple of 8 (its lo chunk sits 32 entries further);
  // rows past M or N read the last row: their products land in outputs that are
  // not stored
  auto pair_off = [&](int64_t row, int k) -> int64_t { return row * 2 * Kp + (k >> 5) * 64 + (k & 31); };
  auto gload = [&](int k0) {
    if constexpr (FUSED) {
      const int64_t row = m0 + tid / CH;
      const int k = k0 + (tid % CH) * 8;
      const double2* x2 = reinterpret_cast<const double2*>(X + (row < M ? row : M - 1) * K);
      const double2* r2 = Xref ? reinterpret_cast<const double2*>(Xref + (row < M ? row : M - 1) * K) : nullptr;
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const bool in = k + 2 * j < K;   // K even: a pair is wholly inside or outside
        xa[j] = in ? x2[(k >> 1) + j] : make_double2(0.0, 0.0);
        xr[j] = in && r2 ? r2[(k >> 1) + j] : make_double2(0.0, 0.0);
      }
    } else {
#pragma unroll
      for (int i = 0; i < A_LD; ++i) {
        const int q = tid + 256 * i;
        const int64_t row = m0 + q / CH;
        const int64_t off = pair_off(row < M ? row : M - 1, k0 + (q % CH) * 8);
        ra[0][i] = *reinterpret_cast<const u32x4*>(Xp + off);
        if constexpr (NPROD == 3) ra[1][i] = *reinterpret_cast<const u32x4*>(Xp + off + 32);
      }
    }
#pragma unroll
    for (int i = 0; i < B_LD; ++i) {
      const int q = tid + 256 * i;
      const int64_t row = n0 + q / CH;
      const int64_t off = pair_off(row < N ? row : N - 1, k0 + (q % CH) * 8);
      rb[0][i] = *reinterpret_cast<const u32x4*>(Op + off);
      if constexpr (NPROD == 3) rb[1][i] = *reinterpret_cast<const u32x4*>(Op + off + 32);
    }
  };
  auto sstore = [&]() {
    if constexpr (FUSED) {
      // x - xref rounded to bf16 (hi), the remainder rounded again (lo), as in split_pairs_kernel
      uint32_t hw[4], lw[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const double x0 = xa[j].x - xr[j].x, x1 = xa[j].y - xr[j].y;
        const uint16_t h0 = bf16_rne(static_cast<float>(x0)), h1 = bf16_rne(static_cast<float>(x1));
        hw[j] = static_cast<uint32_t>(h0) | (static_cast<uint32_t>(h1) << 16);
        if constexpr (NPROD == 3) {
          const uint16_t l0 = bf16_rne(static_cast<float>(x0 - static_cast<double>(bf16_to_f32(h0))));
          const uint16_t l1 = bf16_rne(static_cast<float>(x1 - static_cast<double>(bf16_to_f32(h1))));
          lw[j] = static_cast<uint32_t>(l0) | (static_cast<uint32_t>(l1) << 16);
        }
      }
      ra[0][0] = u32x4{hw[0], hw[1], hw[2], hw[3]};
      if constexpr (NPROD == 3) ra[1][0] = u32x4{lw[0], lw[1], lw[2], lw[3]};
    }
#pragma unroll
    for (int i = 0; i < A_LD; ++i) {
      const int r = (tid + 256 * i) / CH, kc = wslot;
      *reinterpret_cast<u32x4*>(&sA[0][r][kc]) = ra[0][i];
      if constexpr (NPROD == 3) *reinterpret_cast<u32x4*>(&sA[NPROD == 3 ? 1 : 0][r][kc]) = ra[1][i];
    }
#pragma unroll
    for (int i = 0; i < B_LD; ++i) {
      const int r = (tid + 256 * i) / CH, kc = wslot;
      *reinterpret_cast<u32x4*>(&sB[0][r][kc]) = rb[0][i];
      if constexpr (NPROD == 3) *reinterpret_cast<u32x4*>(&sB[NPROD == 3 ? 1 : 0][r][kc]) = rb[1][i];
    }
  };

  v4f acc[TM][TN];
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};

  const int nk = kend > kbeg ? (kend - kbeg + BK - 1) / BK : 0;
  if (nk > 0) {
    gload(kbeg);
    sstore();
  }
  __syncthreads();
  // operand layout of the 16x16x32 bf16 MFMA: lane l holds row (l % 16),
  // k = 8 * (l / 16) .. + 7
  const int rr = lane & 15, kq = (lane >> 4) * 8;
  for (int kt = 0; kt < nk; ++kt) {
    if (kt + 1 < nk) gload(kbeg + (kt + 1) * BK);
#pragma unroll
    for (int ks = 0; ks < BK; ks += 32) {
      v8bf ah[TM], al[TM], bh[TN], bl[TN];
#pragma unroll
      for (int i = 0; i < TM; ++i) {
        const int r = wm + i * 16 + rr, c = ks == 0 ? rslot0 : rslot1;
        ah[i] = *reinterpret_cast<const v8bf*>(&sA[0][r][c]);
        if constexpr (NPROD == 3) al[i] = *reinterpret_cast<const v8bf*>(&sA[NPROD == 3 ? 1 : 0][r][c]);
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        const int r = wn + j * 16 + rr, c = ks == 0 ? rslot0 : rslot1;
        bh[j] = *reinterpret_cast<const v8bf*>(&sB[0][r][c]);
        if constexpr (NPROD == 3) bl[j] = *reinterpret_cast<const v8bf*>(&sB[NPROD == 3 ? 1 : 0][r][c]);
      }
#pragma unroll
      for (int i = 0; i < TM; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          if constexpr (NPROD == 3) {
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh[j], acc[i][j], 0, 0, 0);
            acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl[j], acc[i][j], 0, 0, 0);
          }
          acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh[j], acc[i][j], 0, 0, 0);
        }
    }
    if (kt + 1 < nk) {
      __syncthreads();   // every wave is done reading the stage
      sstore();
      __syncthreads();
    }
  }
#pragma unroll
  for (int i = 0; i < TM; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gm = m0 + wm + i * 16 + (lane >> 4) * 4 + r;
        const int gn = n0 + wn + j * 16 + (lane & 15);
        if (gm < M && gn < N) Cz[gm * N + gn] = static_cast<double>(acc[i][j][r]);
      }
}

// 3xBF16 contraction on 256 x 256 output tiles, for large batches.  Eight waves
// (4 along the cells x 2 along the operator rows), each owning 64 x 128 outputs
// (128 FP32 accumulators per lane: two waves per SIMD fit the 256-register
// budget without spills).  Stages are 32 deep: the 256 cell rows and 256
// operator rows of a stage, hi and lo halves, are one 64 KB LDS buffer (rows of
// 128 bytes, chunk c of row r at slot c ^ ((r / 2) % 8), as in the 128-row
// kernel), and two buffers alternate.  The stages are written by LDS-DMA loads
// (global_load_lds_dwordx4: each lane's 16 bytes land at its own slot of a
// 1 KB run of eight rows; the swizzle is applied to the global address each
// lane fetches), issued one stage ahead, so no registers carry the staging.
// One barrier per stage: after it, the stage's data is visible to every wave and
// the other buffer (the previous stage) is free for the next DMA.  The two
// buffers are distinct LDS objects so that the compiler's LDS-DMA wait tracking
// lets reads of one proceed while the other is being filled.  Per stage and
// wave, right after the barrier: the four A fragments (hi and lo) and the first
// half of the operator fragments are read, then the DMA of the next stage is
// issued, then each operator half's 48 MFMAs run, product-major (lo*hi, hi*lo,
// hi*hi) so consecutive MFMAs update different accumulators.  Per output element
// the MFMA sequence is that of the 128-row kernel (same k blocks of 32, same
// product order), so the two agree to the last bit at equal split-K.
// Preconditions (checked by the launcher): rows * 4 Kp < 2^32 bytes for both
// operands (32-bit DMA offsets).

__global__ __launch_bounds__(512) __attribute__((amdgpu_waves_per_eu(2))) void gemm_bf16x3_wide_kernel(
    const uint16_t* __restrict__ Xp, const uint16_t* __restrict__ Op, double* __restrict__ C, int64_t M, int N, int Kp,
    int kps) {
  __shared__ uint4 buf0[512][8];
  __shared__ uint4 buf1[512][8];
  const int tid = threadIdx.x, lane = tid & 63;
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  // groups of 4 cell-tile rows: an XCD's 32 resident workgroups then share 4 cell tiles and
  // 8 operator tiles per stage (2% faster on the duct than 8 x 4, which re-reads more of the
  // cell operand, the array that does not stay in the last-level cache)
  const int2 tile = xcd_tile<4>();
  const int64_t m0 = static_cast<int64_t>(tile.y) * 256;
  const int n0 = tile.x * 256;
  const int kbeg = blockIdx.z * kps;
  const int kend = min(Kp, kbeg + kps);
  const int nk = kend > kbeg ? (kend - kbeg) / 32 : 0;
  double* Cz = C + static_cast<int64_t>(blockIdx.z) * M * N;

  // DMA sources: waves 0-3 fill buffer rows 0-255 (cells), waves 4-7 rows 256-511
  // (operator rows), eight runs of eight rows each; rows past M or N read the last
  // row (their products land in outputs that are not stored)
  const bool isB = wave >= 4;
  const char* gbase = reinterpret_cast<const char*>(isB ? Op : Xp);
  const int64_t rows = isB ? N : M;
  const int64_t row0 = isB ? n0 : m0;
  uint32_t off[8];
#pragma unroll
  for (int i = 0; i < 8; ++i) {
    const int r = (wave & 3) * 64 + i * 8 + (lane >> 3);
    const int c = (lane & 7) ^ ((r >> 1) & 7);
    const int64_t grow = min(row0 + r, rows - 1);
    off[i] = static_cast<uint32_t>(grow * 4 * Kp + (c >> 2) * 64 + (c & 3) * 16);
  }
  auto issue = [&](uint4(*buf)[8], int k0) {
    const uint32_t kb = static_cast<uint32_t>(k0) * 4u;
#pragma unroll
    for (int i = 0; i < 8; ++i)
      __builtin_amdgcn_global_load_lds((gbl_void_t*)(gbase + static_cast<uint64_t>(off[i] + kb)),
                                       (lds_void_t*)&buf[wave * 64 + i * 8][0], 16, 0, 0);
    // keep the loads ahead of the reads and MFMAs that follow
    __builtin_amdgcn_sched_barrier(0);
  };

  const int rr = lane & 15, q = lane >> 4, rsw = rr >> 1;
  const int s_hi = q ^ rsw, s_lo = (4 + q) ^ rsw;
  const int wm = (wave >> 1) * 64, wn = (wave & 1) * 128;
  v4f acc[4][8];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 8; ++j) acc[i][j] = v4f{0.f, 0.f, 0.f, 0.f};
  auto rd = [&](uint4(*buf)[8], int row, int slot) { return *reinterpret_cast<const v8bf*>(&buf[row][slot]); };
  // a stage: the A fragments and the operator's first half are read right after the barrier,
  // before the DMA of the next stage is issued (2.5% faster on the duct than issuing the DMA
  // first); then per operator half 48 MFMAs, product-major, with the second half's eight reads
  // spread over the first half's MFMAs
  v8bf ah[4], al[4], bh0[4], bl0[4];
  auto first_reads = [&](uint4(*buf)[8]) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      ah[i] = rd(buf, wm + 16 * i + rr, s_hi);
      al[i] = rd(buf, wm + 16 * i + rr, s_lo);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      bh0[j] = rd(buf, 256 + wn + 16 * j + rr, s_hi);
      bl0[j] = rd(buf, 256 + wn + 16 * j + rr, s_lo);
    }
    __builtin_amdgcn_sched_barrier(0);
  };
  auto rest = [&](uint4(*buf)[8]) {
    v8bf bh1[4], bl1[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      bh1[j] = rd(buf, 256 + wn + 64 + 16 * j + rr, s_hi);
      bl1[j] = rd(buf, 256 + wn + 64 + 16 * j + rr, s_lo);
    }
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh0[j], acc[i][j], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl0[j], acc[i][j], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh0[j], acc[i][j], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        acc[i][4 + j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(al[i], bh1[j], acc[i][4 + j], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        acc[i][4 + j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bl1[j], acc[i][4 + j], 0, 0, 0);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j)
        acc[i][4 + j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ah[i], bh1[j], acc[i][4 + j], 0, 0, 0);
    for (int g = 0; g < 8; ++g) {
      __builtin_amdgcn_sched_group_barrier(0x008, 6, 0);
      __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);
    }
    __builtin_amdgcn_sched_group_barrier(0x008, 48, 0);
    __builtin_amdgcn_sched_barrier(0);
  };

  // Stage s sits in buffer s % 2.  The loop handles stage pairs with the buffers
  // named statically (no exit between the two halves: a mid-loop exit made the
  // register allocator shuffle the accumulators); an odd last stage follows it.
  // vmcnt(0) before each barrier: this wave's DMA of the stage has landed.  At the
  // end the DMA target is clamped to a valid stage: the buffer is free after the
  // barrier and nothing reads it again.
  if (nk > 0) issue(buf0, kbeg);
  int s = 0;
  for (; s + 1 < nk; s += 2) {
    __builtin_amdgcn_s_waitcnt(0x0f70);
    __syncthreads();
    first_reads(buf0);
    issue(buf1, kbeg + (s + 1) * 32);
    rest(buf0);
    __builtin_amdgcn_s_waitcnt(0x0f70);
    __syncthreads();
    first_reads(buf1);
    issue(buf0, kbeg + (s + 2 < nk ? s + 2 : 0) * 32);
    rest(buf1);
  }
  if (s < nk) {
    __builtin_amdgcn_s_waitcnt(0x0f70);
    __syncthreads();
    first_reads(buf0);
    rest(buf0);
  }
  // drain the clamped DMA of the last loop pass before the workgroup can end
  __builtin_amdgcn_s_waitcnt(0x0f70);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 8; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int64_t gm = m0 + wm + i * 16 + q * 4 + r;
        const int gn = n0 + wn + j * 16 + rr;
        if (gm < M && gn < N) Cz[gm * N + gn] = static_cast<double>(acc[i][j][r]);
      }
}

// Cell operand of the FP32 contraction, formed once per launch: x = X - Xref
// (Xref null: X) rounded to FP32.
__global__ void convert_x_f32_kernel(const double* __restrict__ X, const double* __restrict__ Xref, int64_t count,
                                     float* __restrict__ out) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= count) return;
  out[i] = static_cast<float>(Xref ? X[i] - Xref[i] : X[i]);
}

// ------------------------------------------------------------------ finish
// Row c = (cell, species) of the finish step; called by finish_kernel with the block index and by
// the persistent 1-D iteration.
__device__ __forceinline__ void finish_row(const FinishArgs& a, int64_t c_row, int nsplit, const double* acc_p) {
  __shared__ double sh[4 * 9];
  __shared__ double coef[5];
  const int64_t c = c_row;  // (cell, species) row of n3 values
  const int nsp = a.nsp, sp = static_cast<int>(c % nsp);
  const int64_t cell = c / nsp;
  if (a.active && !a.active[cell]) return;
  const int n3 = a.n3;
  const double del = a.delta[cell];
  const int fl = a.flow ? a.flow[cell] : 0;
  const double dUc = a.dU ? a.dU[c] : 0.0;
  const double dUq0 = a.dU ? a.dU[cell * nsp] : 0.0;
  const double dUq1 = (a.dU && nsp > 1) ? a.dU[cell * nsp + 1] : 0.0;
  const double ms = a.mass_ratio[sp];
  const double* feq = a.feq + static_cast<int64_t>(sp) * n3;
  const double* nu = a.nu + static_cast<int64_t>(sp) * n3;
  // L+ of the correction shapes of species 0 and 1 seen by species sp
  const double* kc0 = a.Kc + static_cast<int64_t>(sp) * n3;
  const double* kc1 = a.Kc + static_cast<int64_t>(nsp + sp) * n3;
  const double* vt1 = a.vtab;
  const double* vt2 = a.vtab + n3;
  const double* vt3 = a.vtab + 2 * static_cast<int64_t>(n3);
  const int64_t base = c * n3;
  const int64_t sstride = a.n_cells * static_cast<int64_t>(n3);
  double m[9];
#pragma unroll
  for (int k = 0; k < 9; ++k) m[k] = 0.0;
  // one unknown: s = L+ h (partial sums and anchor), hv = h; returns the right side and L h
  auto unknown = [&](double s, double hv, double v1, double v2, double v3, double wv, double f, double nuv,
                     double k0, double k1, double& r, double& L) {
    const double vsq = v1 * v1 + v2 * v2 + v3 * v3;
    // L+ of the corrected iterate: the correction of every species of the cell enters
    double lp = s;
    if (a.dU) {
      lp += dUq0 * k0;
      if (nsp > 1) lp += dUq1 * k1;
    }
    const double hk = hv + dUc * 2.0 * ms * v3 * f;
    L = del * (lp - nuv * hk);
    double S = 0.0;
    if (fl == 1) S = v3 * f;
    else if (fl == 2 && nsp == 1) S = v3 * (vsq - 2.5) * f;
    r = del * lp + S;
    const double wL = wv * L;
    m[0] += wL;
    m[1] += wL * v1;
    m[2] += wL * v2;
    m[3] += wL * v3;
    m[4] += wL * vsq;
    m[5] += 2.0 * wv * v1 * v3 * L;
    m[6] += 2.0 * wv * v1 * v3 * hk;
    m[7] += 2.0 * wv * v2 * v3 * L;
    m[8] += 2.0 * wv * v2 * v3 * hk;
  };
  // U pairs (or unknowns) per lane and pass: the loads of all of them (partials, h, anchor) are
  // issued before any store (with one split the partial sum is the output row itself).  Rows
  // of even length are read and written in 16-byte pairs: the kernel is bound by its count of
  // vector-memory instructions.
  constexpr int U = 4;
  const int bs = blockDim.x;
  // pairs need 16-byte alignment of every row touched (caller arrays may be offset views)
  const uintptr_t align = reinterpret_cast<uintptr_t>(a.h + base) | reinterpret_cast<uintptr_t>(a.rhs + base) |
                          (a.lh ? reinterpret_cast<uintptr_t>(a.lh + base) : 0) |
                          (nsplit > 0 ? reinterpret_cast<uintptr_t>(acc_p + base) |
                                              reinterpret_cast<uintptr_t>(acc_p + sstride) : 0) |
                          (a.anchor_mode ? reinterpret_cast<uintptr_t>(a.accref + base) |
                                               reinterpret_cast<uintptr_t>(a.xref + base) : 0);
  if ((n3 & 1) == 0 && (align & 15) == 0) {
    constexpr int UP = U / 2;      // pairs per lane and pass
    const int np = n3 >> 1;
    auto d2p = [](const double* ptr) { return reinterpret_cast<const double2*>(ptr); };
    for (int p0 = threadIdx.x; p0 < np; p0 += UP * bs) {
      double2 sv[UP], hv[UP];
#pragma unroll
      for (int u = 0; u < UP; ++u) {
        sv[u] = make_double2(0.0, 0.0);
        hv[u] = p0 + u * bs < np ? d2p(a.h + base)[p0 + u * bs] : make_double2(0.0, 0.0);
      }
      // split-K partials four at a time, summed in split order
      for (int z0 = 0; z0 < nsplit; z0 += 4) {
        double2 t[4][UP];
#pragma unroll
        for (int dz = 0; dz < 4; ++dz)
#pragma unroll
          for (int u = 0; u < UP; ++u) {
            const int pp = p0 + u * bs;
            t[dz][u] = (z0 + dz < nsplit && pp < np) ? d2p(acc_p + (z0 + dz) * sstride + base)[pp]
                                                       : make_double2(0.0, 0.0);
          }
#pragma unroll
        for (int dz = 0; dz < 4; ++dz)
#pragma unroll
          for (int u = 0; u < UP; ++u)
            if (z0 + dz < nsplit) {
              sv[u].x += t[dz][u].x;
              sv[u].y += t[dz][u].y;
            }
      }
      if (a.anchor_mode == 2)
#pragma unroll
        for (int u = 0; u < UP; ++u)
          if (p0 + u * bs < np) {
            const double2 r = d2p(a.accref + base)[p0 + u * bs];
            sv[u].x += r.x;
            sv[u].y += r.y;
          }
#pragma unroll
      for (int u = 0; u < UP; ++u) {
        const int pp = p0 + u * bs;
        if (pp >= np) break;
        const double2 V1 = d2p(vt1)[pp], V2 = d2p(vt2)[pp], V3 = d2p(vt3)[pp], W = d2p(a.wtab)[pp];
        const double2 F = d2p(feq)[pp], NU = d2p(nu)[pp];
        double2 K0 = make_double2(0.0, 0.0), K1 = make_double2(0.0, 0.0);
        if (a.dU) {
          K0 = d2p(kc0)[pp];
          if (nsp > 1) K1 = d2p(kc1)[pp];
        }
        if (a.anchor_mode == 1) {
          reinterpret_cast<double2*>(a.accref + base)[pp] = sv[u];
          reinterpret_cast<double2*>(a.xref + base)[pp] = hv[u];
        }
        double2 R, L;
        unknown(sv[u].x, hv[u].x, V1.x, V2.x, V3.x, W.x, F.x, NU.x, K0.x, K1.x, R.x, L.x);
        unknown(sv[u].y, hv[u].y, V1.y, V2.y, V3.y, W.y, F.y, NU.y, K0.y, K1.y, R.y, L.y);
        reinterpret_cast<double2*>(a.rhs + base)[pp] = R;
        if (a.lh) reinterpret_cast<double2*>(a.lh + base)[pp] = L;
      }
    }
  } else {
    for (int v0 = threadIdx.x; v0 < n3; v0 += U * bs) {
      double sv[U], hv[U];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        sv[u] = 0.0;
        hv[u] = v0 + u * bs < n3 ? a.h[base + v0 + u * bs] : 0.0;
      }
      for (int z0 = 0; z0 < nsplit; z0 += 4) {
        double t[4][U];
#pragma unroll
        for (int dz = 0; dz < 4; ++dz)
#pragma unroll
          for (int u = 0; u < U; ++u) {
            const int v = v0 + u * bs;
            t[dz][u] = (z0 + dz < nsplit && v < n3) ? acc_p[(z0 + dz) * sstride + base + v] : 0.0;
          }
#pragma unroll
        for (int dz = 0; dz < 4; ++dz)
#pragma unroll
          for (int u = 0; u < U; ++u)
            if (z0 + dz < nsplit) sv[u] += t[dz][u];
      }
      if (a.anchor_mode == 2)
#pragma unroll
        for (int u = 0; u < U; ++u)
          if (v0 + u * bs < n3) sv[u] += a.accref[base + v0 + u * bs];
#pragma unroll
      for (int u = 0; u < U; ++u) {
        const int v = v0 + u * bs;
        if (v >= n3) break;
        if (a.anchor_mode == 1) {
          a.accref[base + v] = sv[u];
          a.xref[base + v] = hv[u];
        }
        double r, L;
        unknown(sv[u], hv[u], vt1[v], vt2[v], vt3[v], a.wtab[v], feq[v], nu[v], a.dU ? kc0[v] : 0.0,
                (a.dU && nsp > 1) ? kc1[v] : 0.0, r, L);
        a.rhs[base + v] = r;
        if (a.lh) a.lh[base + v] = L;
      }
    }
  }
  block_sum<9>(m, sh);
  if (a.project) {
    if (threadIdx.x < 5) {
      double s = 0.0;
      for (int k = 0; k < 5; ++k) s += a.gram_inv[threadIdx.x * 5 + k] * m[k];
      coef[threadIdx.x] = s;
    }
    __syncthreads();
    for (int v = threadIdx.x; v < n3; v += blockDim.x) {
      const double v1 = vt1[v], v2 = vt2[v], v3 = vt3[v];
      const double vsq = v1 * v1 + v2 * v2 + v3 * v3;
      const double corr = feq[v] * (coef[0] + coef[1] * v1 + coef[2] * v2 + coef[3] * v3 + coef[4] * vsq);
      a.rhs[base + v] -= corr;
      if (a.lh) a.lh[base + v] -= corr;
    }
  }
  if (a.amom && threadIdx.x == 0) {
    // with h stored for v2 > 0 only (h even in v2) the v2 v3 moments vanish identically
    a.amom[c * 4 + 0] = m[5];
    a.amom[c * 4 + 1] = m[6];
    a.amom[c * 4 + 2] = a.even_v2 ? 0.0 : m[7];
    a.amom[c * 4 + 3] = a.even_v2 ? 0.0 : m[8];
  }
}

// ------------------------------------------------------------------ sweep
// One thread per velocity pair (v1 > 0 index jp, mirror jm) of one case.
__global__ __launch_bounds__(256) void finish_kernel(FinishArgs a) { finish_row(a, blockIdx.x, a.splits, a.acc); }

// One thread per (case, species, |v1| > 0 velocity pair): the two marches of a velocity are
// serial in x1, so the right sides and stencil coefficients of the next kSweepChunk nodes are
// loaded while the current ones are processed (the dependency chain then holds arithmetic
// only).  Moments are taken afterwards by moments_kernel.
constexpr int kSweepChunk = 8;

__device__ __forceinline__ void sweep1d_block(const SweepArgs& a, int bx, int cs, int sp) {
  const int nsp = a.nsp;
  if (a.case_active && !a.case_active[cs]) return;
  const int half = a.n3 / 2, n3 = a.n3;
  const int t = bx * blockDim.x + threadIdx.x;
  if (t >= half) return;
  const int64_t c0 = a.node_off[cs];
  const int nodes = static_cast<int>(a.node_off[cs + 1] - c0);
  const int d23 = a.d2 * a.d3;
  const int j1h = t / d23, r = t % d23;
  const int jp = a.n / 2 + j1h, jm = a.n / 2 - 1 - j1h;
  const int vp = jp * d23 + r, vm = jm * d23 + r;
  const double v1 = a.v1d[jp];
  const double del = a.delta_case[cs];
  const double* nu = a.nu + static_cast<int64_t>(sp) * n3;
  const double dnp = del * nu[vp], dnm = del * nu[vm];
  const double* __restrict__ rhs = a.rhs;
  double* __restrict__ h = a.h;
  const double* __restrict__ coef = a.coef;
  // row of (cell, species) in the [cell][species][n3] arrays
  auto row = [&](int64_t cell) { return (cell * nsp + sp) * static_cast<int64_t>(n3); };
  double rc[kSweepChunk], ac[kSweepChunk], bc[kSweepChunk], cc[kSweepChunk];
  double rn[kSweepChunk], an[kSweepChunk], bn[kSweepChunk], cn[kSweepChunk];
  // v1 > 0: wall value 0, march towards the symmetry plane (nodes 1 .. nodes-1)
  h[row(c0) + vp] = 0.0;
  double h1 = 0.0, h2 = 0.0;
#pragma unroll
  for (int u = 0; u < kSweepChunk; ++u) {
    const int i = 1 + u;
    const int64_t cell = c0 + (i < nodes ? i : 0);
    rc[u] = rhs[row(cell) + vp];
    ac[u] = coef[cell * 6 + 0];
    bc[u] = coef[cell * 6 + 1];
    cc[u] = coef[cell * 6 + 2];
  }
  for (int base = 1; base < nodes; base += kSweepChunk) {
#pragma unroll
    for (int u = 0; u < kSweepChunk; ++u) {
      const int i = base + kSweepChunk + u;
      const int64_t cell = c0 + (i < nodes ? i : 0);
      rn[u] = rhs[row(cell) + vp];
      an[u] = coef[cell * 6 + 0];
      bn[u] = coef[cell * 6 + 1];
      cn[u] = coef[cell * 6 + 2];
    }
#pragma unroll
    for (int u = 0; u < kSweepChunk; ++u) {
      const int i = base + u;
      if (i < nodes) {
        const double val = (rc[u] - v1 * (bc[u] * h1 + cc[u] * h2)) / (dnp + v1 * ac[u]);
        h[row(c0 + i) + vp] = val;
        h2 = h1;
        h1 = val;
      }
    }
#pragma unroll
    for (int u = 0; u < kSweepChunk; ++u) {
      rc[u] = rn[u];
      ac[u] = an[u];
      bc[u] = bn[u];
      cc[u] = cn[u];
    }
  }
  // v1 < 0: specular reflection at the last node, march to the wall (nodes nodes-2 .. 0)
  const int64_t last = c0 + nodes - 1;
  double g1 = h1, g2 = 0.0;
  h[row(last) + vm] = g1;
#pragma unroll
  for (int u = 0; u < kSweepChunk; ++u) {
    const int i = nodes - 2 - u;
    const int64_t cell = c0 + (i >= 0 ? i : 0);
    rc[u] = rhs[row(cell) + vm];
    ac[u] = coef[cell * 6 + 3];
    bc[u] = coef[cell * 6 + 4];
    cc[u] = coef[cell * 6 + 5];
  }
  for (int base = nodes - 2; base >= 0; base -= kSweepChunk) {
#pragma unroll
    for (int u = 0; u < kSweepChunk; ++u) {
      const int i = base - kSweepChunk - u;
      const int64_t cell = c0 + (i >= 0 ? i : 0);
      rn[u] = rhs[row(cell) + vm];
      an[u] = coef[cell * 6 + 3];
      bn[u] = coef[cell * 6 + 4];
      cn[u] = coef[cell * 6 + 5];
    }
#pragma unroll
    for (int u = 0; u < kSweepChunk; ++u) {
      const int i = base - u;
      if (i >= 0) {
        const double val = (rc[u] - v1 * (bc[u] * g1 + cc[u] * g2)) / (dnm + v1 * ac[u]);
        h[row(c0 + i) + vm] = val;
        g2 = g1;
        g1 = val;
      }
    }
#pragma unroll
    for (int u = 0; u < kSweepChunk; ++u) {
      rc[u] = rn[u];
      ac[u] = an[u];
      bc[u] = bn[u];
      cc[u] = cn[u];
    }
  }
}

__global__ __launch_bounds__(256) void sweep1d_kernel(SweepArgs a) { sweep1d_block(a, blockIdx.x, blockIdx.y, blockIdx.z); }

// Calls f(v1, v2, v3, h) for every unknown of row `row` (n3 values): in 16-byte pairs for
// rows of even length (the moment kernels are bound by their count of memory instructions).
template <typename F>
__device__ inline void for_row(int n3, const double* __restrict__ vtab, const double* __restrict__ h, int64_t row,
                               F&& f) {
  const double* hr = h + row * n3;
  if ((n3 & 1) == 0 && (reinterpret_cast<uintptr_t>(hr) & 15) == 0) {
    const int np = n3 >> 1;
    const double2* h2 = reinterpret_cast<const double2*>(hr);
    const double2* a1 = reinterpret_cast<const double2*>(vtab);
    const double2* a2 = reinterpret_cast<const double2*>(vtab + n3);
    const double2* a3 = reinterpret_cast<const double2*>(vtab + 2 * static_cast<int64_t>(n3));
#pragma unroll 2
    for (int p = threadIdx.x; p < np; p += blockDim.x) {
      const double2 x = h2[p], v1 = a1[p], v2 = a2[p], v3 = a3[p];
      f(v1.x, v2.x, v3.x, x.x);
      f(v1.y, v2.y, v3.y, x.y);
    }
  } else {
    for (int v = threadIdx.x; v < n3; v += blockDim.x)
      f(vtab[v], vtab[n3 + v], vtab[2 * static_cast<int64_t>(n3) + v], hr[v]);
  }
}

__device__ __forceinline__ void moments_row(int n3, int nsp, double ms0, double ms1, const double* __restrict__ vtab,
                                            const double* __restrict__ h, double w, double* __restrict__ mom,
                                            int64_t c) {   // c: (cell, species) row
  __shared__ double sh[4 * 4];
  const double ms = (c % nsp) == 0 ? ms0 : ms1;
  double m[4] = {0.0, 0.0, 0.0, 0.0};
  for_row(n3, vtab, h, c, [&](double v1, double v2, double v3, double hv) {
    const double vsq = v1 * v1 + v2 * v2 + v3 * v3;
    const double x = w * hv;
    m[0] += v3 * x;
    m[1] += (ms * vsq - 2.5) * v3 * x;
    m[2] += v3 * (2.0 * v1 * v1 - 1.0) * x;
    m[3] += 2.0 * ms * v1 * v3 * x;
  });
  block_sum<4>(m, sh);
  if (threadIdx.x == 0)
    for (int k = 0; k < 4; ++k) mom[c * 4 + k] = m[k];
}

__global__ __launch_bounds__(256) void moments_kernel(int n3, int nsp, double ms0, double ms1,
                                                      const double* __restrict__ vtab,
                                                      const double* __restrict__ h, double w,
                                                      double* __restrict__ mom) {
  moments_row(n3, nsp, ms0, ms1, vtab, h, w, mom, blockIdx.x);
}

// ------------------------------------------------------------------ diffusion (1-D)
// One workgroup per case.  The march from the wall is a serial recurrence, so one
// lane carries it; the per-node inputs (moments, source, stencil) are staged into LDS
// by the whole workgroup in coalesced chunks and the outputs written back the same
// way, so the march itself waits on LDS only.
constexpr int kDiffChunk = 256;

__device__ __forceinline__ void diffusion1d_case(const DiffusionArgs& a, int cs) {
  __shared__ double in[8][kDiffChunk];    // Uh, qh, G1, source, ca, cb, cc, x
  __shared__ double out[4][kDiffChunk];   // U, dU, q, U of the new iterate
  if (a.case_active && !a.case_active[cs]) return;   // uniform over the workgroup
  const int64_t c0 = a.node_off[cs];
  const int nodes = static_cast<int>(a.node_off[cs + 1] - c0);
  const double del = a.delta_case[cs];
  const bool pois = a.flow_case[cs] == 1;
  double y1 = 0.0, y2 = 0.0;
  double Mr = 0.0, Qr = 0.0, Up = 0.0, qp = 0.0, xp = 0.0;
  for (int base = 0; base < nodes; base += kDiffChunk) {
    const int cnt = min(kDiffChunk, nodes - base);
    for (int t = threadIdx.x; t < cnt; t += blockDim.x) {
      const int64_t cell = c0 + base + t;
      in[0][t] = a.mom[cell * 4 + 0];
      in[1][t] = a.mom[cell * 4 + 1];
      in[2][t] = a.mom[cell * 4 + 2];
      const double x = a.x[cell];
      in[7][t] = x;
      if (a.sis && base + t > 0) {
        double A1 = 0.0;
        if (a.amom) A1 = a.amom[cell * 4 + 0] + a.N * del * a.amom[cell * 4 + 1];
        in[3][t] = A1 - (pois ? a.N * del * x : 0.0);
        in[4][t] = a.coef[cell * 6 + 0];
        in[5][t] = a.coef[cell * 6 + 1];
        in[6][t] = a.coef[cell * 6 + 2];
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int t = 0; t < cnt; ++t) {
        const int i = base + t;
        const double Uh = in[0][t], qh = in[1][t], G1 = in[2][t];
        double dU = 0.0, Usol = Uh;
        if (a.sis) {
          const double y = i == 0 ? Uh + G1 : (in[3][t] - in[5][t] * y1 - in[6][t] * y2) / in[4][t];
          y2 = y1;
          y1 = y;
          Usol = y - G1;
          dU = Usol - Uh;
        }
        // moments of h^{k+1} = h^{k+1/2} + dU 2 v3 f_eq (eq. guided)
        const double Un = Uh + dU * a.cU, qn = qh + dU * a.cq;
        out[0][t] = Usol;
        out[1][t] = dU;
        out[2][t] = qn;
        out[3][t] = Un;
        const double x = in[7][t];
        if (i > 0) {
          Mr += 0.5 * (Un + Up) * (x - xp);
          Qr += 0.5 * (qn + qp) * (x - xp);
        }
        Up = Un;
        qp = qn;
        xp = x;
      }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < cnt; t += blockDim.x) {
      const int64_t cell = c0 + base + t;
      if (a.U) a.U[cell] = out[0][t];
      if (a.dU) a.dU[cell] = out[1][t];
      if (a.qfield) a.qfield[cell] = out[2][t];
      if (a.ufield) a.ufield[cell] = out[3][t];
    }
    // the next chunk's staging writes only in[]; the march that rewrites out[] starts
    // after the next barrier, which every lane reaches after its stores above
  }
  if (threadIdx.x == 0 && a.state) {
    const double M = 2.0 * Mr, Q = 2.0 * Qr;
    double* st = a.state + cs * 4;
    const double dM = fabs(M - st[0]) / fmax(fabs(M), 1e-300);
    const double dQ = fabs(Q - st[1]) / fmax(fabs(Q), 1e-300);
    const double res = fmax(dM, dQ);
    st[0] = M;
    st[1] = Q;
    st[2] = (M != M || Q != Q) ? __builtin_nan("") : res;
    const int it = a.iters[cs] + 1;
    a.iters[cs] = it;
    if (!(res >= a.eps) || M != M || Q != Q) a.case_active[cs] = 0;
    st[3] = static_cast<double>(it);
  }
}


// The case's flag, as its march left it, copied to the flags of its cells (what the next
// iteration's finish and sweep read), so that no separate expansion launch is needed.
__device__ __forceinline__ void case_flag_to_cells(const DiffusionArgs& a, int cs) {
  __shared__ int32_t flag;
  if (!a.cell_active || !a.case_active) return;
  __syncthreads();
  if (threadIdx.x == 0) flag = __hip_atomic_load(&a.case_active[cs], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  const int64_t c0 = a.node_off[cs], c1 = a.node_off[cs + 1];
  for (int64_t c = c0 + threadIdx.x; c < c1; c += blockDim.x) a.cell_active[c] = flag;
}

__global__ __launch_bounds__(kDiffChunk) void diffusion1d_kernel(DiffusionArgs a) {
  diffusion1d_case(a, blockIdx.x);
  case_flag_to_cells(a, blockIdx.x);
}

// Binary mixture (planar): the velocity equations of species B (own shear
// stress) and A (total stress minus B's), integrated once from the symmetry
// plane and marched from the wall; rows are (cell, species) with species A
// first.  mom[row][4] = {int v3 h, q, G1, P13}; U is per unit molar fraction.
// The two species march independently (lane s carries species s); inputs and outputs
// are staged through LDS as in diffusion1d_kernel.
__device__ __forceinline__ void diffusion1d_mix_case(const DiffusionArgs& a, int cs) {
  __shared__ double in_s[2][4][kDiffChunk];   // per species: Uh, qh, G, source
  __shared__ double in_c[4][kDiffChunk];      // per node: ca, cb, cc, x
  __shared__ double out[2][4][kDiffChunk];    // per species: U, dU, q, U of the new iterate
  __shared__ double red[2][2];                // per species: M, Q integrals
  if (a.case_active && !a.case_active[cs]) return;   // uniform over the workgroup
  const int64_t c0 = a.node_off[cs];
  const int nodes = static_cast<int>(a.node_off[cs + 1] - c0);
  const double del = a.delta_case[cs];
  const double pois = a.flow_case[cs] == 1 ? 1.0 : 0.0;
  const int sp = threadIdx.x;                 // marching lane: species sp (lanes 0, 1)
  double y1 = 0.0, y2 = 0.0;
  double Mr = 0.0, Qr = 0.0, Up = 0.0, qp = 0.0, xp = 0.0;
  for (int base = 0; base < nodes; base += kDiffChunk) {
    const int cnt = min(kDiffChunk, nodes - base);
    for (int t = threadIdx.x; t < cnt; t += blockDim.x) {
      const int64_t cell = c0 + base + t;
      const double x = a.x[cell];
      const double PB = a.mom[(cell * 2 + 1) * 4 + 3];
      in_c[3][t] = x;
      if (a.sis && base + t > 0) {
        in_c[0][t] = a.coef[cell * 6 + 0];
        in_c[1][t] = a.coef[cell * 6 + 1];
        in_c[2][t] = a.coef[cell * 6 + 2];
      }
      for (int s = 0; s < 2; ++s) {
        const int64_t r = cell * 2 + s;
        in_s[s][0][t] = a.mom[r * 4 + 0] / a.chi[s];
        in_s[s][1][t] = a.mom[r * 4 + 1];
        in_s[s][2][t] = a.mom[r * 4 + 2];
        if (a.sis && base + t > 0) {
          const double Nd = a.Ns[s] * del;
          double A = 0.0;
          if (a.amom) A = a.amom[r * 4 + 0] + Nd * a.amom[r * 4 + 1];
          in_s[s][3][t] = s == 1 ? A - Nd * PB / a.mass_ratio[1] : A - Nd * (pois * x - PB);
        }
      }
    }
    __syncthreads();
    if (sp < 2) {
      const double chi = a.chi[sp];
      for (int t = 0; t < cnt; ++t) {
        const int i = base + t;
        const double Uh = in_s[sp][0][t], qh = in_s[sp][1][t], G = in_s[sp][2][t];
        double dU = 0.0, Usol = Uh;
        if (a.sis) {
          const double y = i == 0 ? chi * Uh + G
                                  : (in_s[sp][3][t] - in_c[1][t] * y1 - in_c[2][t] * y2) / in_c[0][t];
          y2 = y1;
          y1 = y;
          Usol = (y - G) / chi;
          dU = Usol - Uh;
        }
        const double Un = Uh + dU * a.cUs[sp], qn = qh + dU * a.cqs[sp];
        out[sp][0][t] = Usol;
        out[sp][1][t] = dU;
        out[sp][2][t] = qn;
        out[sp][3][t] = Un;
        const double x = in_c[3][t];
        if (i > 0) {
          Mr += 0.5 * (Un + Up) * (x - xp);
          Qr += 0.5 * (qn + qp) * (x - xp);
        }
        Up = Un;
        qp = qn;
        xp = x;
      }
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 2 * cnt; e += blockDim.x) {
      const int t = e >> 1, s = e & 1;
      const int64_t r = (c0 + base + t) * 2 + s;
      if (a.U) a.U[r] = out[s][0][t];
      if (a.dU) a.dU[r] = out[s][1][t];
      if (a.qfield) a.qfield[r] = out[s][2][t];
      if (a.ufield) a.ufield[r] = out[s][3][t];
    }
  }
  if (sp < 2) {
    red[sp][0] = Mr;
    red[sp][1] = Qr;
  }
  __syncthreads();
  if (threadIdx.x == 0 && a.state) {
    double* st = a.state + cs * 6;  // M_A, M_B, Q_A, Q_B, residual, iterations
    double res = 0.0;
    bool bad = false;
    for (int s = 0; s < 2; ++s) {
      const double M = 2.0 * a.flow_factor * red[s][0], Q = 2.0 * a.flow_factor * red[s][1];
      res = fmax(res, fmax(fabs(M - st[s]) / fmax(fabs(M), 1e-300), fabs(Q - st[2 + s]) / fmax(fabs(Q), 1e-300)));
      bad = bad || M != M || Q != Q;
      st[s] = M;
      st[2 + s] = Q;
    }
    st[4] = bad ? __builtin_nan("") : res;
    const int it = a.iters[cs] + 1;
    a.iters[cs] = it;
    if (!(res >= a.eps) || bad) a.case_active[cs] = 0;
    st[5] = static_cast<double>(it);
  }
}

__global__ __launch_bounds__(kDiffChunk) void diffusion1d_mix_kernel(DiffusionArgs a) {
  diffusion1d_mix_case(a, blockIdx.x);
  case_flag_to_cells(a, blockIdx.x);
}

// ------------------------------------------------------------------ 2-D sweep
// One workgroup per (case, group of kSweepV velocity quadruples (+-|v1|, +-|v2|, v3)).
// The quadrants are swept in the order (+,+), (-,+), (+,-), (-,-).  Within a
// quadrant every upwind reference of a cell lies on an earlier anti-diagonal of
// the sweep order (ii + jj smaller), mirror ghosts read an earlier quadrant and
// the wrapped periodic references read later anti-diagonals (the previous
// iterate), so the anti-diagonals are processed in order with a workgroup
// barrier between them and the cells of one anti-diagonal in parallel: the
// values read are exactly those of the row-by-row sweep.
constexpr int kSweepV = 4;       // velocity quadruples per workgroup
constexpr int kSweepThreads = 256;

__global__ __launch_bounds__(kSweepThreads) void sweep2d_kernel(Sweep2DArgs a) {
  const int cs = blockIdx.y;
  if (a.case_active && !a.case_active[cs]) return;   // uniform over the workgroup
  const int n = a.n, hn = n / 2, n3 = a.n3, d3 = a.d3;
  const int nsp = a.nsp, sp = blockIdx.z;
  const double* __restrict__ nu = a.nu + static_cast<int64_t>(sp) * n3;
  const int quads = hn * hn * d3;
  // neighbouring velocity groups share cache lines of h and the right sides: with the group
  // count a multiple of 8, consecutive groups go to the same XCD (dispatch is round-robin)
  const int gx = gridDim.x;
  const int grp = (gx % 8 == 0) ? (blockIdx.x % 8) * (gx / 8) + blockIdx.x / 8 : blockIdx.x;
  const int tq = grp * kSweepV + threadIdx.x % kSweepV;
  const bool vvalid = tq < quads;
  const int t = vvalid ? tq : 0;
  const int jq1 = t / (hn * d3), jq2 = (t / d3) % hn, j3 = t % d3;
  const int slot = threadIdx.x / kSweepV, slots = kSweepThreads / kSweepV;
  const int n1 = a.n1[cs], n2 = a.n2[cs];
  const int64_t g0 = a.grid_off[cs];
  const double del = a.delta_case[cs];
  for (int q = 0; q < 4; ++q) {
    const int s1 = (q & 1) ? -1 : 1, s2 = (q & 2) ? -1 : 1;
    const int j1 = s1 > 0 ? hn + jq1 : hn - 1 - jq1;
    const int j2 = s2 > 0 ? hn + jq2 : hn - 1 - jq2;
    const int v = (j1 * n + j2) * d3 + j3;
    const int vm1 = ((n - 1 - j1) * n + j2) * d3 + j3;
    const int vm2 = (j1 * n + (n - 1 - j2)) * d3 + j3;
    const double av1 = fabs(a.v1d[j1]), av2 = fabs(a.v1d[j2]);
    const double dnu = del * nu[v];
    const int sg1 = s1 > 0 ? 0 : 1, sg2 = s2 > 0 ? 0 : 1;
    for (int d = 0; d < n1 + n2 - 1; ++d) {
      const int lo = max(0, d - (n2 - 1)), hi = min(d, n1 - 1);   // ii range of the anti-diagonal
      for (int c0 = lo; c0 <= hi; c0 += slots) {
        const int ii = c0 + slot;
        if (vvalid && ii <= hi) {
          const int jj = d - ii;
          const int i = s1 > 0 ? ii : n1 - 1 - ii;
          const int j = s2 > 0 ? jj : n2 - 1 - jj;
          const int cell = a.gcell[g0 + static_cast<int64_t>(i) * n2 + j];
          if (cell >= 0) {
            const int64_t o1 = (static_cast<int64_t>(cell) * 2 + 0) * 2 + sg1;
            const int64_t o2 = (static_cast<int64_t>(cell) * 2 + 1) * 2 + sg2;
            const int64_t row = static_cast<int64_t>(cell) * nsp + sp;
            double acc = a.rhs[row * n3 + v];
            const double c1[3] = {a.coef[o1 * 3], a.coef[o1 * 3 + 1], a.coef[o1 * 3 + 2]};
            const double c2[3] = {a.coef[o2 * 3], a.coef[o2 * 3 + 1], a.coef[o2 * 3 + 2]};
#pragma unroll
            for (int k = 0; k < 2; ++k) {
              const int8_t k1 = a.kind[o1 * 2 + k];
              if (k1) {
                const int64_t r = static_cast<int64_t>(a.ref[o1 * 2 + k]) * nsp + sp;
                acc -= av1 * c1[k + 1] * a.h[r * n3 + (k1 == 2 ? vm1 : v)];
              }
              const int8_t k2 = a.kind[o2 * 2 + k];
              if (k2) {
                const int64_t r = static_cast<int64_t>(a.ref[o2 * 2 + k]) * nsp + sp;
                acc -= av2 * c2[k + 1] * a.h[r * n3 + (k2 == 2 ? vm2 : v)];
              }
            }
            a.h[row * n3 + v] = acc / (dnu + av1 * c1[0] + av2 * c2[0]);
          }
        }
      }
      __syncthreads();
    }
  }
}

// Pipelined form of the same sweep for cross sections whose anti-diagonals hold at most
// P * 64 cells (min(n1, n2) <= 64 P): each slot owns up to P cells of a diagonal, and the
// read-only data of its cells on the next diagonal (cell index, stencil coefficients,
// upwind references, right side) are loaded while the current diagonal is computed, so
// that after each barrier only the upwind values of h are waited for.  The values and the
// order of the updates are those of sweep2d_kernel.  P is the smallest that covers the
// longest anti-diagonal: the per-cell state of two diagonals sits in registers, so a
// smaller P leaves room for more resident workgroups.
constexpr int kSweepMaxP = 3;

// The four words lane K of each group of four lanes holds, in every lane of the group
// (DPP quad_perm broadcast; every lane of the group must be active).
template <int K>
__device__ inline void quad_broadcast(const uint4& w, uint32_t* out) {
  constexpr int ctrl = K * 0x55;   // quad_perm(K, K, K, K)
  out[0] = static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(w.x), ctrl, 0xF, 0xF, false));
  out[1] = static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(w.y), ctrl, 0xF, 0xF, false));
  out[2] = static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(w.z), ctrl, 0xF, 0xF, false));
  out[3] = static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, static_cast<int>(w.w), ctrl, 0xF, 0xF, false));
}

struct Sweep2DPoint {
  int64_t row;          // (cell * nsp + species), -1: no fluid cell
  double rhs, c1[3], c2[3];
  int32_t r1[2], r2[2];
  int8_t k1[2], k2[2];
};

template <int kSweepP>
__global__ __launch_bounds__(kSweepThreads) void sweep2d_pipelined_kernel(Sweep2DArgs a) {
  const int cs = blockIdx.y;
  if (a.case_active && !a.case_active[cs]) return;   // uniform over the workgroup
  const int n = a.n, hn = n / 2, n3 = a.n3, d3 = a.d3;
  const int nsp = a.nsp, sp = blockIdx.z;
  const double* __restrict__ nu = a.nu + static_cast<int64_t>(sp) * n3;
  const int quads = hn * hn * d3;
  // neighbouring velocity groups share cache lines of h and the right sides: with the group
  // count a multiple of 8, consecutive groups go to the same XCD (dispatch is round-robin)
  const int gx = gridDim.x;
  const int grp = (gx % 8 == 0) ? (blockIdx.x % 8) * (gx / 8) + blockIdx.x / 8 : blockIdx.x;
  const int tq = grp * kSweepV + threadIdx.x % kSweepV;
  const bool vvalid = tq < quads;
  const int t = vvalid ? tq : 0;
  const int jq1 = t / (hn * d3), jq2 = (t / d3) % hn, j3 = t % d3;
  const int slot = threadIdx.x / kSweepV, slots = kSweepThreads / kSweepV;
  const int n1 = a.n1[cs], n2 = a.n2[cs];
  const int64_t g0 = a.grid_off[cs];
  const double del = a.delta_case[cs];
  for (int q = 0; q < 4; ++q) {
    const int s1 = (q & 1) ? -1 : 1, s2 = (q & 2) ? -1 : 1;
    const int j1 = s1 > 0 ? hn + jq1 : hn - 1 - jq1;
    const int j2 = s2 > 0 ? hn + jq2 : hn - 1 - jq2;
    const int v = (j1 * n + j2) * d3 + j3;
    const int vm1 = ((n - 1 - j1) * n + j2) * d3 + j3;
    const int vm2 = (j1 * n + (n - 1 - j2)) * d3 + j3;
    const double av1 = fabs(a.v1d[j1]), av2 = fabs(a.v1d[j2]);
    const double dnu = del * nu[v];
    const int sg1 = s1 > 0 ? 0 : 1, sg2 = s2 > 0 ? 0 : 1;
    static_assert(kSweepV == 4, "the four lanes of a slot (one velocity each) form a DPP quad");
    const int quad = threadIdx.x & 3;
    auto load = [&](int d, int p, Sweep2DPoint& pt) {
      pt.row = -1;
      const int lo = max(0, d - (n2 - 1)), hi = min(d, n1 - 1);
      const int ii = lo + slot + p * slots;
      int cell = -1;                     // the same for the four lanes of the quad
      if (d <= n1 + n2 - 2 && ii <= hi) {
        const int jj = d - ii;
        const int i = s1 > 0 ? ii : n1 - 1 - ii;
        const int j = s2 > 0 ? jj : n2 - 1 - jj;
        cell = a.gcell[g0 + static_cast<int64_t>(i) * n2 + j];
      }
      // the cell's two 32-byte stencil records (axis 1 with the sign of v1, axis 2 with the sign
      // of v2) are loaded 16 bytes per lane and broadcast within the quad: one load instruction
      // instead of fifteen (lanes of cells that do not exist read record 0 and discard it)
      const int64_t o = (static_cast<int64_t>(cell >= 0 ? cell : 0) * 2 + (quad >> 1)) * 2 + ((quad >> 1) ? sg2 : sg1);
      const uint4 w = *reinterpret_cast<const uint4*>(a.rec + o * 8 + (quad & 1) * 4);
      uint32_t r[16];
      quad_broadcast<0>(w, r);
      quad_broadcast<1>(w, r + 4);
      quad_broadcast<2>(w, r + 8);
      quad_broadcast<3>(w, r + 12);
      if (!vvalid || cell < 0) return;
      auto f64 = [&](int k) { return __builtin_bit_cast(double, (static_cast<uint64_t>(r[k + 1]) << 32) | r[k]); };
      pt.c1[0] = f64(0);
      pt.c1[1] = f64(2);
      pt.c1[2] = f64(4);
      pt.c2[0] = f64(8);
      pt.c2[1] = f64(10);
      pt.c2[2] = f64(12);
#pragma unroll
      for (int k = 0; k < 2; ++k) {
        pt.k1[k] = static_cast<int8_t>(r[6 + k] & 3u);
        pt.r1[k] = static_cast<int32_t>(r[6 + k] >> 2);
        pt.k2[k] = static_cast<int8_t>(r[14 + k] & 3u);
        pt.r2[k] = static_cast<int32_t>(r[14 + k] >> 2);
      }
      pt.row = static_cast<int64_t>(cell) * nsp + sp;
      pt.rhs = a.rhs[pt.row * n3 + v];
    };
    Sweep2DPoint cur[kSweepP], nxt[kSweepP];
#pragma unroll
    for (int p = 0; p < kSweepP; ++p) load(0, p, cur[p]);
    for (int d = 0; d < n1 + n2 - 1; ++d) {
      double up[kSweepP][4];
#pragma unroll
      for (int p = 0; p < kSweepP; ++p) {
#pragma unroll
        for (int k = 0; k < 2; ++k) {
          up[p][k] = (cur[p].row >= 0 && cur[p].k1[k])
                         ? a.h[(static_cast<int64_t>(cur[p].r1[k]) * nsp + sp) * n3 + (cur[p].k1[k] == 2 ? vm1 : v)]
                         : 0.0;
          up[p][2 + k] = (cur[p].row >= 0 && cur[p].k2[k])
                             ? a.h[(static_cast<int64_t>(cur[p].r2[k]) * nsp + sp) * n3 + (cur[p].k2[k] == 2 ? vm2 : v)]
                             : 0.0;
        }
      }
#pragma unroll
      for (int p = 0; p < kSweepP; ++p) load(d + 1, p, nxt[p]);
#pragma unroll
      for (int p = 0; p < kSweepP; ++p) {
        const Sweep2DPoint& c = cur[p];
        if (c.row >= 0) {
          double acc = c.rhs;
#pragma unroll
          for (int k = 0; k < 2; ++k) {
            if (c.k1[k]) acc -= av1 * c.c1[k + 1] * up[p][k];
            if (c.k2[k]) acc -= av2 * c.c2[k + 1] * up[p][2 + k];
          }
          a.h[c.row * n3 + v] = acc / (dnu + av1 * c.c1[0] + av2 * c.c2[0]);
        }
      }
      __syncthreads();
#pragma unroll
      for (int p = 0; p < kSweepP; ++p) cur[p] = nxt[p];
    }
  }
}

// Row-blocked form of the same sweep, for cross sections of up to 128 cells along axis 2
// whose distributions fit 2 GiB (32-bit row offsets).  A lane owns one velocity quadruple,
// and every value it reads during the sweep belongs to that quadruple: in-quadrant upwind
// cells (this sweep), mirror ghosts (the quadrant with the mirrored axis's sign flipped: this
// sweep if it came earlier, else the previous iterate) and periodic wraps (cells later in the
// sweep order: the previous iterate).  Any order in which each cell follows its upwind cells
// along both axes therefore reads the values the anti-diagonal order reads; the update of
// each cell is the same expression in the same order (a reference of kind 0 enters with
// coefficient 0 in place of being skipped), so the results agree to the sign of zeros.
//
// A workgroup holds W <= 16 waves of 64 quadruples each, of one case and species, and sweeps
// the four quadrants in the same order (one workgroup per quadrant where no reference is a
// mirror ghost: then the quadrants do not read each other).  Within a quadrant the cells are
// taken in the sweep's orientation (row r, column c counted from the upwind corner); the
// columns are split into W blocks of cw <= CW (4 or 8) columns, and each wave runs over all
// rows of its block, column by column.  The two values left of the block come from wave
// w - 1 through LDS, double-buffered by row parity and handed on by two counters per wave
// (rows published, rows of the left neighbour's values read) instead of a workgroup barrier,
// so the waves run skewed by about a row each.  The two rows above are the lane's registers;
// only references that leave the grid are read from h: those of rows 0 and 1 (axis 1) when
// the quadrant starts, those of columns 0 and 1 (axis 2) with the right sides.  A block
// row's uniform data (grid-ordered stencil records and 32-bit row offsets) is loaded one word
// per lane four rows ahead into a ring of four LDS slots per wave and read back by broadcast
// (coefficients) or into scalar registers (offsets, reference words); the right sides are
// loaded two rows (CW = 4) or one row (CW = 8) ahead into registers that alternate between
// two sets (the row loop is unrolled by two), so that no register copy waits for a load.
// Rows of h and of the right sides are addressed through buffer descriptors, the row offset
// as the scalar offset: a solid or missing cell uses an empty descriptor, whose loads return
// 0 and whose stores are dropped, and gets a finite placeholder update (a = 1).  Lanes past
// the last quadruple repeat it (same values, same stores).  The full barrier at the end of a
// quadrant makes its stores visible to the mirror reads of the next.
constexpr int kRowWaves = 16;
constexpr int kRowSpinMax = 1 << 22; // bound on a wave's wait for its neighbour (never reached)

// Waits until *flag >= target (a counter another wave of the workgroup advances), then
// orders the LDS reads that follow after the writes published before the counter.
__device__ inline void lds_wait_at_least(const int* flag, int target) {
  for (int it = 0; it < kRowSpinMax; ++it) {
    if (__builtin_amdgcn_readfirstlane(__hip_atomic_load(flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP)) >=
        target)
      break;
    __builtin_amdgcn_s_sleep(1);
  }
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// Publishes value in *flag after the wave's earlier LDS accesses.
__device__ inline void lds_publish(int* flag, int value) {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __hip_atomic_store(flag, value, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));

template <int CW>
__global__ __launch_bounds__(64 * kRowWaves) void sweep2d_rows_kernel(
    Sweep2DArgs a, const uint32_t* __restrict__ grec, const uint32_t* __restrict__ growb,
    const double* __restrict__ rhs, double* __restrict__ h) {
  // right sides are loaded two rows ahead for 4 columns per wave, one row ahead for 8 (registers)
  constexpr int kAhead = CW == 4 ? 2 : 1;
  constexpr int kRowWords = 17 * CW;                // 16 record words and a row offset per cell
  constexpr int kRegs = (kRowWords + 63) / 64;
  __shared__ double carry[2][kRowWaves][2][64];     // [row parity][wave][column c - 1, c - 2][lane]
  __shared__ __align__(16) uint32_t stage[kRowWaves][4][kRegs * 64];
  __shared__ double row1[kRowWaves][CW][64];        // second out-of-grid axis-1 reference of row 1
  __shared__ int published[kRowWaves];              // rows whose carry the wave has written
  __shared__ int consumed[kRowWaves];               // rows of its left neighbour's carry it has read
  const int n = a.n, hn = n / 2, n3 = a.n3, d3 = a.d3;
  const int nsp = a.nsp;
  const int quads = hn * hn * d3, groups = (quads + 63) / 64;
  // Workgroups are dispatched round-robin over the 8 XCDs (each with its own L2); numbering
  // them so that consecutive velocity groups of a case share an XCD lets the cache lines they
  // share (their 512-byte segments of a row are not line-aligned) be fetched once.
  const int nwg = gridDim.x, lin = blockIdx.x, per = nwg / 8, rem = nwg % 8, xcd = lin % 8, slot = lin / 8;
  const int logical = xcd < rem ? xcd * (per + 1) + slot : rem * (per + 1) + (xcd - rem) * per + slot;
  const int grp = logical % groups, cs = (logical / groups) % a.n_cases;
  const int sp = (logical / (groups * a.n_cases)) % nsp;
  // without mirror ghosts the quadrants do not read each other: one workgroup per quadrant
  const int qsplit = logical / (groups * a.n_cases * nsp);
  const int q0 = a.quad_split ? qsplit : 0, q1 = a.quad_split ? qsplit + 1 : 4;
  if (a.case_active && !a.case_active[cs]) return;   // uniform over the workgroup
  const int W = blockDim.x >> 6, w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const double* __restrict__ nu = a.nu + static_cast<int64_t>(sp) * n3;
  const uint32_t row_bytes = static_cast<uint32_t>(nsp * n3 * 8);
  // Rows of species sp through buffer descriptors: cell c's row at byte offset growb (a 32-bit
  // scalar offset; the launcher checks that h fits), the lane's velocity in the vector offset.
  // A cell that is not there (solid, outside the grid) uses the empty descriptor: its loads
  // return 0 and its stores are dropped.
  const __amdgpu_buffer_rsrc_t rs_rhs =
      __builtin_amdgcn_make_buffer_rsrc(const_cast<double*>(rhs + static_cast<int64_t>(sp) * n3), 0, 0x7fffffff, 0x00020000);
  const __amdgpu_buffer_rsrc_t rs_h =
      __builtin_amdgcn_make_buffer_rsrc(h + static_cast<int64_t>(sp) * n3, 0, 0x7fffffff, 0x00020000);
  const __amdgpu_buffer_rsrc_t rs_none = __builtin_amdgcn_make_buffer_rsrc(h, 0, 0, 0x00020000);
  // lanes past the last quadruple repeat the last one (same wave, same values, same stores)
  const int tq = grp * 64 + lane;
  const int t = tq < quads ? tq : quads - 1;
  const int jq1 = t / (hn * d3), jq2 = (t / d3) % hn, j3 = t % d3;
  const int n1 = a.n1[cs], n2 = a.n2[cs];
  const int64_t g0 = a.grid_off[cs];
  const double del = a.delta_case[cs];
  const int cw = (n2 + W - 1) / W;                   // <= CW (checked by the launcher)
  const int jb0 = min(w * cw, n2), nb = min(cw, n2 - jb0);
  const int rows = (n1 + 1) & ~1;                    // an even count: row n1 of odd n1 is a placeholder
  auto ld = [&](const __amdgpu_buffer_rsrc_t& rs, uint32_t vo, uint32_t so) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, vo, so, 0));
  };
  for (int q = q0; q < q1; ++q) {
    const int s1 = (q & 1) ? -1 : 1, s2 = (q & 2) ? -1 : 1;
    const int j1 = s1 > 0 ? hn + jq1 : hn - 1 - jq1;
    const int j2 = s2 > 0 ? hn + jq2 : hn - 1 - jq2;
    const int v = (j1 * n + j2) * d3 + j3;
    const int vm1 = ((n - 1 - j1) * n + j2) * d3 + j3;
    const int vm2 = (j1 * n + (n - 1 - j2)) * d3 + j3;
    const uint32_t vb = v * 8u, vm1b = vm1 * 8u, vm2b = vm2 * 8u;
    const double av1 = fabs(a.v1d[j1]), av2 = fabs(a.v1d[j2]);
    const double dnu = del * nu[v];
    const int sg1 = s1 > 0 ? 0 : 1, sg2 = s2 > 0 ? 0 : 1;
    if (lane == 0) {
      published[w] = 0;
      consumed[w] = 0;
    }
    __syncthreads();
    // grid index of the block's column k in oriented row r: rbase(r) + dj k
    const int dj = s2, jstart = s2 > 0 ? jb0 : n2 - 1 - jb0;
    auto rbase = [&](int r) { return g0 + static_cast<int64_t>(s1 > 0 ? r : n1 - 1 - r) * n2 + jstart; };
    // Staging slot of row r: 16 record words per cell (axis 1 with the sign of v1, then axis 2
    // with the sign of v2), then the cells' row offsets (0xffffffff: none), one word per lane.
    // Where there is no cell (outside the block or the grid) the words are read from the
    // tables' extra solid entry (a = 1, no references, no row): every lane loads, and uses
    // the word as loaded, so that all rows issue the same memory instructions and the waits
    // for them stay counted.
    auto load_row = [&](int r, uint32_t (&sv)[kRegs]) {
      const bool rv = r < n1;
      const int64_t gb = rbase(rv ? r : 0);
#pragma unroll
      for (int u = 0; u < kRegs; ++u) {
        const int x = 64 * u + lane;
        const bool isrec = x < 16 * CW;
        const int k = isrec ? x >> 4 : x - 16 * CW, d = x & 15, axis = d >> 3;
        const int64_t gk = rv && k < nb ? gb + dj * k : a.grid_none;
        sv[u] = isrec ? grec[(gk * 4 + axis * 2 + (axis ? sg2 : sg1)) * 8 + (d & 7)] : growb[gk];
      }
    };
    auto put_row = [&](int r, const uint32_t (&sv)[kRegs]) {
#pragma unroll
      for (int u = 0; u < kRegs; ++u) stage[w][r & 3][64 * u + lane] = sv[u];
    };
    auto coef = [&](int r, int k, int wd) {
      return *reinterpret_cast<const double*>(&stage[w][r & 3][16 * k + wd]);
    };
    auto word = [&](int r, int i) { return __builtin_amdgcn_readfirstlane(stage[w][r & 3][i]); };
    auto row_of = [&](int r, int k) { return word(r, 16 * CW + k); };
    auto load_rhs = [&](int r, double (&rr)[CW]) {
#pragma unroll
      for (int k = 0; k < CW; ++k) {
        const uint32_t o = row_of(r, k);
        rr[k] = ld(o != 0xffffffffu ? rs_rhs : rs_none, vb, o);
      }
    };
    // value of a reference word (ref << 2 | kind) at the lane's velocity (mirrored for kind 2)
    auto ref_at = [&](uint32_t x, uint32_t vmir) {
      return ld(x & 3u ? rs_h : rs_none, (x & 3u) == 2 ? vmir : vb, (x >> 2) * row_bytes);
    };
    // out-of-grid axis-2 references: column c, reference st (one and two cells upwind), of the
    // block's first two columns if it holds them
    auto load_edge = [&](int r, double (&ge)[3]) {
#pragma unroll
      for (int e = 0; e < 3; ++e) {
        const int c = e == 2 ? 1 : 0, st = e == 0 ? 0 : 1;
        const bool mine = c >= jb0 && c < jb0 + nb;
        ge[e] = ref_at(mine ? word(r, 16 * (c - jb0) + 14 + st) : 0u, vm2b);
      }
    };
    // out-of-grid axis-1 references take the places of rows r - 1, r - 2: both of row 0 in
    // pr1, pr2, the second one of row 1 in LDS until row 1
    double pr1[CW], pr2[CW];              // rows r - 1, r - 2 of the block
#pragma unroll
    for (int k = 0; k < CW; ++k) {
      const bool have = k < nb;
      const uint32_t* p0 = grec + ((have ? rbase(0) + dj * k : a.grid_none) * 4 + sg1) * 8;
      const uint32_t* p1 = grec + ((have ? rbase(1) + dj * k : a.grid_none) * 4 + sg1) * 8;
      pr1[k] = ref_at(p0[6], vm1b);
      pr2[k] = ref_at(p0[7], vm1b);
      row1[w][k][lane] = ref_at(p1[7], vm1b);
    }
    uint32_t sA[kRegs], sB[kRegs];        // staging words of row r + 3 (A / B alternate)
    double rA[CW], rB[CW], eA[3], eB[3];  // right sides and edge references of even / odd rows
    load_row(0, sA);
    load_row(1, sB);
    put_row(0, sA);
    put_row(1, sB);
    load_row(2, sA);
    put_row(2, sA);
    load_row(3, sB);
    load_rhs(0, rA);
    load_edge(0, eA);
    if (kAhead == 2) {
      load_rhs(1, rB);
      load_edge(1, eB);
    }
    // row r with (rc, ec) of row r, loaded kAhead rows earlier, and the staging words ss of row
    // r + 3 loaded by the previous row; stages them, loads row r + 4's words into sn and, once
    // this row's are consumed, row r + kAhead's right sides and edge references into (rn, en)
    // (the same registers two rows ahead; the other set one row ahead).  Calls alternate the
    // A / B sets.
    auto row = [&](int r, double (&rc)[CW], double (&ec)[3], double (&rn)[CW], double (&en)[3],
                   uint32_t (&ss)[kRegs], uint32_t (&sn)[kRegs]) {
      put_row(r + 3, ss);
      load_row(r + 4, sn);
      if (__builtin_expect(r == 1, 0)) {
#pragma unroll
        for (int k = 0; k < CW; ++k) pr2[k] = row1[w][k][lane];
      }
      double acc0[CW];
#pragma unroll
      for (int k = 0; k < CW; ++k) acc0[k] = rc[k] - av1 * coef(r, k, 2) * pr1[k];
      const double e0 = ec[0], e1 = ec[1], e2 = ec[2];
      load_rhs(r + kAhead, rn);
      load_edge(r + kAhead, en);
      double p1 = 0.0, p2 = 0.0;              // columns c - 1, c - 2 of this row
      if (w > 0) {
        lds_wait_at_least(&published[w - 1], r + 1);
        p1 = carry[r & 1][w - 1][0][lane];
        p2 = carry[r & 1][w - 1][1][lane];
        lds_publish(&consumed[w], r + 1);
      }
      if (__builtin_expect(jb0 == 0, 0)) {
        p1 = e0;
        p2 = e1;
      }
      const double in1 = p1, in2 = p2;
      // column 1's second reference leaves the grid: it replaces the shifted value at k = 1
      // (block from column 0) or k = 0 (block from column 1)
      const double p2k1 = jb0 == 0 ? e2 : in1;
      if (__builtin_expect(jb0 == 1, 0)) p2 = e2;
      double hv[CW];
#pragma unroll
      for (int k = 0; k < CW; ++k) {
        if (k == 1) p2 = p2k1;
        double acc = acc0[k];
        acc -= av2 * coef(r, k, 10) * p1;
        acc -= av1 * coef(r, k, 4) * pr2[k];
        acc -= av2 * coef(r, k, 12) * p2;
        hv[k] = acc / (dnu + av1 * coef(r, k, 0) + av2 * coef(r, k, 8));
        const uint32_t o = row_of(r, k);
        __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, hv[k]), o != 0xffffffffu ? rs_h : rs_none,
                                              vb, o, 0);
        p2 = p1;
        p1 = hv[k];
        pr2[k] = pr1[k];
        pr1[k] = hv[k];
      }
      if (__builtin_expect(nb < CW, 0)) {     // the carry is the block's last two columns
        p1 = in1;
        p2 = in2;
#pragma unroll
        for (int k = 0; k < CW; ++k)
          if (k < nb) {
            p2 = p1;
            p1 = hv[k];
          }
      }
      if (w < W - 1) {
        lds_wait_at_least(&consumed[w + 1], r - 1);  // its read of row r - 2 (same parity) is done
        carry[r & 1][w][0][lane] = p1;
        carry[r & 1][w][1][lane] = p2;
        lds_publish(&published[w], r + 1);
      }
    };
    if (kAhead == 2) {
      for (int r = 0; r < rows; r += 2) {
        row(r, rA, eA, rA, eA, sB, sA);
        row(r + 1, rB, eB, rB, eB, sA, sB);
      }
    } else {
      for (int r = 0; r < rows; r += 2) {
        row(r, rA, eA, rB, eB, sB, sA);
        row(r + 1, rB, eB, rA, eA, sA, sB);
      }
    }
    __syncthreads();
  }
}

// Per (cell, species) row: U3, q3 = int (a v^2 - 5/2) v3 h, G1, G12, G2, P13 = 2a int v1 v3 h,
// P23 = 2a int v2 v3 h (a = m_s / m_A; 1 for one gas).
__global__ __launch_bounds__(256) void moments2d_kernel(int n3, int nsp, double ms0, double ms1,
                                                        const double* __restrict__ vtab,
                                                        const double* __restrict__ h, double w,
                                                        const int32_t* __restrict__ active,
                                                        double* __restrict__ mom) {
  __shared__ double sh[4 * 7];
  const int64_t c = blockIdx.x;
  if (active && !active[c / nsp]) return;
  const double ms = (c % nsp) == 0 ? ms0 : ms1;
  double m[7] = {0, 0, 0, 0, 0, 0, 0};
  for_row(n3, vtab, h, c, [&](double v1, double v2, double v3, double hv) {
    const double vsq = v1 * v1 + v2 * v2 + v3 * v3;
    const double x = w * hv;
    m[0] += v3 * x;
    m[1] += (ms * vsq - 2.5) * v3 * x;
    m[2] += v3 * (2.0 * v1 * v1 - 1.0) * x;
    m[3] += 2.0 * v1 * v2 * v3 * x;
    m[4] += v3 * (2.0 * v2 * v2 - 1.0) * x;
    m[5] += 2.0 * ms * v1 * v3 * x;
    m[6] += 2.0 * ms * v2 * v3 * x;
  });
  block_sum<7>(m, sh);
  if (threadIdx.x == 0) {
    for (int k = 0; k < 7; ++k) mom[c * 8 + k] = m[k];
    mom[c * 8 + 7] = 0.0;
  }
}

// ------------------------------------------------------------------ 2-D diffusion
// Finite-volume form of the SIS velocity equation on one case per workgroup,
// Jacobi-preconditioned conjugate gradients in FP64, then flow rates.
constexpr int kD2Threads = 1024;

__device__ inline double par_sign(int bits, int p1, int p2) {
  return ((bits & 1) ? p1 : 1) * ((bits & 2) ? p2 : 1);
}

template <int K>
__device__ inline void block_sum_big(double (&v)[K], double* sh /* >= 16*K */) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int nw = blockDim.x >> 6;
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const double s = wave_sum(v[k]);
    if (lane == 0) sh[wave * K + k] = s;
  }
  __syncthreads();
#pragma unroll
  for (int k = 0; k < K; ++k) {
    double s = 0.0;
    for (int w = 0; w < nw; ++w) s += sh[w * K + k];
    v[k] = s;
  }
  __syncthreads();
}

// Workspace of species s of case cs: per grid cell Uh G1 G12 G2 A1 A2 (x r p Ap for CG)
// and, for mixtures, P_B13 P_B23 (species B's shear stresses, in every species' slots).
__device__ inline double* d2_work(const Diff2DArgs& a, int cs, int s) {
  return a.work + (static_cast<int64_t>(s) * a.n_grid + a.grid_off[cs]) * kDiffWork;
}

__device__ void d2_fill_work(const Diff2DArgs& a, int cs, int s, double* W, int ng, bool warm) {
  const int64_t g0 = a.grid_off[cs];
  const double del = a.delta_case[cs];
  const int nsp = a.nsp;
  const double chi = a.chi[s], Nd = a.Ns[s] * del;
  for (int g = threadIdx.x; g < ng; g += blockDim.x) {
    const int cell = a.gcell[g0 + g];
    double* w = W + static_cast<int64_t>(g) * kDiffWork;
    if (cell >= 0) {
      const int64_t row = static_cast<int64_t>(cell) * nsp + s;
      const double* m = a.mom + row * 8;
      w[0] = m[0] / chi; w[1] = m[2]; w[2] = m[3]; w[3] = m[4];
      if (a.amom) {
        const double* am = a.amom + row * 4;
        w[4] = am[0] + Nd * am[1];
        w[5] = am[2] + Nd * am[3];
      } else {
        w[4] = 0.0; w[5] = 0.0;
      }
      if (!warm) w[6] = w[0];
      if (nsp == 2) {
        const double* mb = a.mom + (static_cast<int64_t>(cell) * 2 + 1) * 8;
        w[10] = mb[5];
        w[11] = mb[6];
      } else {
        w[10] = 0.0; w[11] = 0.0;
      }
    } else {
      for (int k = 0; k < 6; ++k) w[k] = 0.0;
      w[6] = 0.0;
      w[10] = 0.0; w[11] = 0.0;
    }
    w[7] = 0.0; w[8] = 0.0; w[9] = 0.0;
  }
}

// Right side of the finite-volume velocity equation of species s at an unknown grid
// cell G (Dirichlet neighbours moved to the right) and the diagonal of its row:
// chi_s lap U_s = source_s - (d11 G1 + 2 d12 G12 + d22 G2) + d1 A1 + d2 A2, with
// source = -N delta [Poiseuille] for one gas; for mixtures N_A delta (div P_B - [P])
// (species A) and -N_B delta (m_A/m_B) div P_B (species B).
__device__ double d2_rhs(const Diff2DArgs& a, int s, int64_t g0, int64_t G, const double* W, bool pois, double del,
                         double& diag) {
  const int g = static_cast<int>(G - g0);
  const double* w = W + static_cast<int64_t>(g) * kDiffWork;
  const int32_t* nbr = a.nb + G * 8;
  const int8_t* bits = a.nbm + G * 8;
  const double* np = a.npos + G * 4;
  const double xc = a.cpos[G * 2], yc = a.cpos[G * 2 + 1];
  auto val = [&](int q, int f, int p1, int p2) {
    const int r = nbr[q];
    return r < 0 ? 0.0 : par_sign(bits[q], p1, p2) * W[static_cast<int64_t>(r) * kDiffWork + f];
  };
  const double xE = np[0], xW = np[1], yN = np[2], yS = np[3];
  const double w1 = a.width[G * 2], w2 = a.width[G * 2 + 1];
  auto d11 = [&](int f, int p1, int p2) {
    return ((val(0, f, p1, p2) - w[f]) / (xE - xc) - (w[f] - val(1, f, p1, p2)) / (xc - xW)) / w1;
  };
  auto d22 = [&](int f, int p1, int p2) {
    return ((val(2, f, p1, p2) - w[f]) / (yN - yc) - (w[f] - val(3, f, p1, p2)) / (yc - yS)) / w2;
  };
  const double Nd = a.Ns[s] * del;
  double rhs = 0.0;
  if (a.nsp == 1) {
    rhs = pois ? -Nd : 0.0;
  } else {
    const double coef = s == 1 ? -Nd / a.mass_ratio[1] : Nd;
    if (s == 0 && pois) rhs -= Nd;
    rhs += coef * ((val(0, 10, -1, 1) - val(1, 10, -1, 1)) / (xE - xW) +
                   (val(2, 11, 1, -1) - val(3, 11, 1, -1)) / (yN - yS));
  }
  const double cross = ((val(4, 2, -1, -1) - val(6, 2, -1, -1)) / (yN - yS) -
                        (val(5, 2, -1, -1) - val(7, 2, -1, -1)) / (yN - yS)) / (xE - xW);
  rhs -= d11(1, 1, 1) + 2.0 * cross + d22(3, 1, 1);
  rhs += (val(0, 4, -1, 1) - val(1, 4, -1, 1)) / (xE - xW);
  rhs += (val(2, 5, 1, -1) - val(3, 5, 1, -1)) / (yN - yS);
  double b = -(rhs / a.chi[s]) * a.dA[G];
  diag = 0.0;
  for (int q = 0; q < 4; ++q) {
    const double fw = a.fw[G * 4 + q];
    if (fw == 0.0) continue;
    const int r = nbr[q];
    diag += fw;
    if (a.dflag[g0 + r] != 2) b += fw * W[static_cast<int64_t>(r) * kDiffWork + 0];
  }
  return b;
}

// New velocities, corrections, moments of h^{k+1}, flow rates and the convergence
// test of one case (all species).  usol: the solutions at the unknown cells (null:
// the CG iterate in the workspace; CIS: no solve).
__device__ void d2_outputs(const Diff2DArgs& a, int cs, int ng, const double* usol, int it, double* sh) {
  const int64_t g0 = a.grid_off[cs];
  const int nsp = a.nsp;
  double fr[4] = {0.0, 0.0, 0.0, 0.0};   // (M, Q) per species
  for (int s = 0; s < nsp; ++s) {
    const double* W = d2_work(a, cs, s);
    const int64_t voff = nsp * a.uoff[cs] + static_cast<int64_t>(s) * a.n_unknown[cs];
    for (int g = threadIdx.x; g < ng; g += blockDim.x) {
      const int64_t G = g0 + g;
      const int cell = a.gcell[G];
      if (cell < 0) continue;
      const int64_t row = static_cast<int64_t>(cell) * nsp + s;
      const double* w = W + static_cast<int64_t>(g) * kDiffWork;
      const double Uh = w[0];
      double U = Uh;
      if (a.sis && a.dflag[G] == 2) U = usol ? usol[voff + a.uidx[G]] : w[6];
      const double dU = U - Uh;
      const double Un = Uh + dU * a.cUs[s];
      const double qn = a.mom[row * 8 + 1] + dU * a.cqs[s];
      if (a.U) a.U[row] = U;
      if (a.dU) a.dU[row] = dU;
      if (a.ufield) a.ufield[row] = Un;
      if (a.qfield) a.qfield[row] = qn;
      fr[2 * s] += Un * a.dA[G];
      fr[2 * s + 1] += qn * a.dA[G];
    }
  }
  block_sum_big<4>(fr, sh);
  if (threadIdx.x == 0) {
    // the CG iterate in the workspace is a valid warm start only after a CG solve (the
    // inverse path leaves the workspace's iterate untouched)
    if (a.have_x) a.have_x[cs] = (a.sis && !usol) ? 1 : 0;
    if (a.cg_iters) a.cg_iters[cs] = it;
    if (a.state) {
      double* st = a.state + cs * (2 * nsp + 2);   // M[nsp], Q[nsp], residual, iterations
      double res = 0.0;
      bool bad = false;
      for (int s = 0; s < nsp; ++s) {
        double M = fr[2 * s] / a.area[cs], Q = fr[2 * s + 1] / a.area[cs];
        if (nsp == 2) {
          M *= a.flow_factor;
          Q *= a.flow_factor;
        }
        const double dM = fabs(M - st[s]) / fmax(fabs(M), 1e-300);
        const double dQ = fabs(Q - st[nsp + s]) / fmax(fabs(Q), 1e-300);
        res = fmax(res, fmax(dM, dQ));
        bad = bad || M != M || Q != Q;
        st[s] = M;
        st[nsp + s] = Q;
      }
      st[2 * nsp] = bad ? __builtin_nan("") : res;
      const int k = a.iters[cs] + 1;
      a.iters[cs] = k;
      if (!(res >= a.eps) || bad) a.case_active[cs] = 0;
      st[2 * nsp + 1] = static_cast<double>(k);
    }
  }
}

// Conjugate-gradient form (one gas; cases without a precomputed inverse).
__global__ __launch_bounds__(kD2Threads) void diffusion2d_kernel(Diff2DArgs a) {
  __shared__ double sh[16 * 4];
  const int cs = blockIdx.x;
  if (a.case_active && !a.case_active[cs]) return;
  if (a.direct && a.direct[cs]) return;   // solved by the inverse path
  const int64_t g0 = a.grid_off[cs];
  const int ng = static_cast<int>(a.grid_off[cs + 1] - g0);
  const double del = a.delta_case[cs];
  const bool pois = a.flow_case[cs] == 1;
  double* W = d2_work(a, cs, 0);
  const bool warm = a.have_x && a.have_x[cs];
  d2_fill_work(a, cs, 0, W, ng, warm);
  __syncthreads();
  int it = 0;
  if (a.sis) {
    // right side, initial residual, preconditioned direction
    double red[3] = {0.0, 0.0, 0.0};   // r.z, b.b, r.r
    for (int g = threadIdx.x; g < ng; g += blockDim.x) {
      const int64_t G = g0 + g;
      if (a.dflag[G] != 2) continue;
      double* w = W + static_cast<int64_t>(g) * kDiffWork;
      double diag;
      const double b = d2_rhs(a, 0, g0, G, W, pois, del, diag);
      double Ax = 0.0;
      for (int q = 0; q < 4; ++q) {
        const double fw = a.fw[G * 4 + q];
        if (fw == 0.0) continue;
        const int r = a.nb[G * 8 + q];
        if (a.dflag[g0 + r] == 2) Ax -= fw * W[static_cast<int64_t>(r) * kDiffWork + 6];
      }
      Ax += diag * w[6];
      const double r0 = b - Ax;
      w[7] = r0;
      w[8] = r0 / diag;
      w[9] = b;     // keep b for the norm only during setup
      red[0] += r0 * r0 / diag;
      red[1] += b * b;
      red[2] += r0 * r0;
    }
    block_sum_big<3>(red, sh);
    double rz = red[0];
    const double bnorm = sqrt(red[1]);
    double rnorm = sqrt(red[2]);
    while (rnorm > a.tol * bnorm && it < a.max_iter) {
      // Ap and p.Ap
      double pap[1] = {0.0};
      for (int g = threadIdx.x; g < ng; g += blockDim.x) {
        const int64_t G = g0 + g;
        if (a.dflag[G] != 2) continue;
        double* w = W + static_cast<int64_t>(g) * kDiffWork;
        double diag = 0.0, Ap = 0.0;
        for (int q = 0; q < 4; ++q) {
          const double fw = a.fw[G * 4 + q];
          if (fw == 0.0) continue;
          const int r = a.nb[G * 8 + q];
          diag += fw;
          if (a.dflag[g0 + r] == 2) Ap -= fw * W[static_cast<int64_t>(r) * kDiffWork + 8];
        }
        Ap += diag * w[8];
        w[9] = Ap;
        pap[0] += w[8] * Ap;
      }
      block_sum_big<1>(pap, sh);
      const double alpha = rz / pap[0];
      double nr[2] = {0.0, 0.0};
      for (int g = threadIdx.x; g < ng; g += blockDim.x) {
        const int64_t G = g0 + g;
        if (a.dflag[G] != 2) continue;
        double* w = W + static_cast<int64_t>(g) * kDiffWork;
        double diag = 0.0;
        for (int q = 0; q < 4; ++q) diag += a.fw[G * 4 + q];
        w[6] += alpha * w[8];
        w[7] -= alpha * w[9];
        nr[0] += w[7] * w[7] / diag;
        nr[1] += w[7] * w[7];
      }
      block_sum_big<2>(nr, sh);
      const double beta = nr[0] / rz;
      rz = nr[0];
      rnorm = sqrt(nr[1]);
      for (int g = threadIdx.x; g < ng; g += blockDim.x) {
        const int64_t G = g0 + g;
        if (a.dflag[G] != 2) continue;
        double* w = W + static_cast<int64_t>(g) * kDiffWork;
        double diag = 0.0;
        for (int q = 0; q < 4; ++q) diag += a.fw[G * 4 + q];
        w[8] = w[7] / diag + beta * w[8];
      }
      __syncthreads();
      ++it;
    }
  }
  d2_outputs(a, cs, ng, nullptr, it, sh);
}

// Inverse form, step 1: right sides of the unknown cells of every species (compact per case).
__global__ __launch_bounds__(kD2Threads) void diffusion2d_rhs_kernel(Diff2DArgs a) {
  const int cs = blockIdx.x;
  if (a.case_active && !a.case_active[cs]) return;
  if (!a.direct[cs]) return;
  const int64_t g0 = a.grid_off[cs];
  const int ng = static_cast<int>(a.grid_off[cs + 1] - g0);
  const double del = a.delta_case[cs];
  const bool pois = a.flow_case[cs] == 1;
  for (int s = 0; s < a.nsp; ++s) d2_fill_work(a, cs, s, d2_work(a, cs, s), ng, true);
  __syncthreads();
  if (!a.sis) return;
  for (int s = 0; s < a.nsp; ++s) {
    const double* W = d2_work(a, cs, s);
    const int64_t voff = a.nsp * a.uoff[cs] + static_cast<int64_t>(s) * a.n_unknown[cs];
    for (int g = threadIdx.x; g < ng; g += blockDim.x) {
      const int64_t G = g0 + g;
      if (a.dflag[G] != 2) continue;
      double diag;
      a.bvec[voff + a.uidx[G]] = d2_rhs(a, s, g0, G, W, pois, del, diag);
    }
  }
}

// Inverse form, step 2: y = A^-1 b for the right sides of one group (same cross
// section), one wave per row of the shared inverse, which is read once for all of them.
template <int G>
__device__ void d2_gemv_rows(const Diff2DArgs& a, int grp, int row, int lane) {
  const int nu = a.grp_n[grp];
  const double* Ar = a.ainv + a.grp_aoff[grp] + static_cast<int64_t>(row) * nu;
  const double* b[G];
  double s[G];
#pragma unroll
  for (int m = 0; m < G; ++m) {
    b[m] = a.bvec + a.grp_vec[grp * kInverseGroup + m];
    s[m] = 0.0;
  }
  for (int j = lane; j < nu; j += 64) {
    const double v = Ar[j];
#pragma unroll
    for (int m = 0; m < G; ++m) s[m] += v * b[m][j];
  }
#pragma unroll
  for (int m = 0; m < G; ++m) {
    const double t = wave_sum(s[m]);
    if (lane == 0) a.yvec[a.grp_vec[grp * kInverseGroup + m] + row] = t;
  }
}

__global__ __launch_bounds__(256) void diffusion2d_gemv_kernel(Diff2DArgs a) {
  const int grp = blockIdx.y;
  if (!a.sis) return;
  const int row = blockIdx.x * 4 + (threadIdx.x >> 6), lane = threadIdx.x & 63;
  if (row >= a.grp_n[grp]) return;
  switch (a.grp_size[grp]) {
    case 1: d2_gemv_rows<1>(a, grp, row, lane); break;
    case 2: d2_gemv_rows<2>(a, grp, row, lane); break;
    case 3: d2_gemv_rows<3>(a, grp, row, lane); break;
    case 4: d2_gemv_rows<4>(a, grp, row, lane); break;
    case 5: d2_gemv_rows<5>(a, grp, row, lane); break;
    case 6: d2_gemv_rows<6>(a, grp, row, lane); break;
    case 7: d2_gemv_rows<7>(a, grp, row, lane); break;
    default: d2_gemv_rows<8>(a, grp, row, lane); break;
  }
}

// Inverse form, step 3: outputs, flow rates, convergence.
__global__ __launch_bounds__(kD2Threads) void diffusion2d_out_kernel(Diff2DArgs a) {
  __shared__ double sh[16 * 4];
  const int cs = blockIdx.x;
  if (a.case_active && !a.case_active[cs]) return;
  if (!a.direct[cs]) return;
  const int64_t g0 = a.grid_off[cs];
  const int ng = static_cast<int>(a.grid_off[cs + 1] - g0);
  d2_outputs(a, cs, ng, a.yvec, 0, sh);
}

// Newton-Schulz steps for the inverse of a Jacobi-scaled SPD matrix (plan time).
// Per-block sum of squares of I - P (Frobenius residual, an upper bound of the 2-norm).
__global__ void ns_residual_kernel(const double* __restrict__ P, int n, double* __restrict__ part) {
  __shared__ double sh[4];
  const int64_t count = static_cast<int64_t>(n) * n;
  double m = 0.0;
  for (int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x; i < count;
       i += static_cast<int64_t>(gridDim.x) * blockDim.x) {
    const int64_t r = i / n, c = i % n;
    const double e = (r == c ? 1.0 : 0.0) - P[i];
    m += e * e;
  }
  m = wave_sum(m);
  if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    double v = 0.0;
    for (int w = 0; w < (blockDim.x >> 6); ++w) v += sh[w];
    part[blockIdx.x] = v;
  }
}

__global__ void ns_two_minus_kernel(double* __restrict__ P, int n) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= static_cast<int64_t>(n) * n) return;
  const int64_t r = i / n, c = i % n;
  P[i] = (r == c ? 2.0 : 0.0) - P[i];
}

// out[r][c] = X[r][c] s[r] s[c] for r, c < n (X has leading dimension ldx, out has n)
__global__ void ns_scale_kernel(const double* __restrict__ X, int ldx, int n, const double* __restrict__ s,
                                double* __restrict__ out) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= static_cast<int64_t>(n) * n) return;
  const int64_t r = i / n, c = i % n;
  out[i] = X[r * ldx + c] * s[r] * s[c];
}

// X = alpha I (n x n); S = I, then S[row][col] = val for the listed entries
__global__ void ns_init_kernel(double* __restrict__ X, int n, double alpha) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= static_cast<int64_t>(n) * n) return;
  X[i] = (i / n == i % n) ? alpha : 0.0;
}

__global__ void ns_scatter_kernel(double* __restrict__ S, int n, const int32_t* __restrict__ rc,
                                  const double* __restrict__ val, int64_t count) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i >= count) return;
  S[static_cast<int64_t>(rc[2 * i]) * n + rc[2 * i + 1]] = val[i];
}

// ------------------------------------------------------------------ polar velocity grid (tube)
__global__ void polar_fhat_kernel(int nm, const double* __restrict__ xi, int nv, const double* __restrict__ vnode,
                                  const double* __restrict__ wf, double* __restrict__ fhat) {
  const int m = blockIdx.x * blockDim.x + threadIdx.x;
  if (m >= nm) return;
  const double x0 = xi[m], x1 = xi[nm + m], x2 = xi[2 * nm + m];
  double s = 0.0;
  for (int j = 0; j < nv; ++j)
    s += wf[j] * cos(x0 * vnode[j]) * cos(x1 * vnode[nv + j]) * cos(x2 * vnode[2 * nv + j]);
  fhat[m] = 4.0 * s;
}

__global__ void polar_cos_kernel(int nv, int nm, const double* __restrict__ vnode, const double* __restrict__ xi,
                                 double* __restrict__ X) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= static_cast<int64_t>(nv) * nm) return;
  const int i = static_cast<int>(idx / nm), m = static_cast<int>(idx % nm);
  X[idx] = cos(xi[m] * vnode[i] + xi[nm + m] * vnode[nv + i] + xi[2 * nm + m] * vnode[2 * nv + i]);
}

__global__ void polar_scale_terms_kernel(int Tp, int nm, const double* __restrict__ mt,
                                         const double* __restrict__ fhat, const double* __restrict__ sc,
                                         double* __restrict__ out) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= static_cast<int64_t>(Tp) * nm) return;
  const int m = static_cast<int>(idx % nm);
  out[idx] = mt[idx] * fhat[m] * sc[m];
}

__global__ void polar_coef_kernel(int nv, int Tp, const double* __restrict__ AB, const int32_t* __restrict__ srcT,
                                  const double* __restrict__ c, const double* __restrict__ feq, int inu,
                                  double* __restrict__ aT, double* __restrict__ nu) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= static_cast<int64_t>(nv) * Tp) return;
  const int i = static_cast<int>(idx / Tp), t = static_cast<int>(idx % Tp);
  const int sidx = srcT[t];
  aT[idx] = sidx >= 0 ? c[t] * AB[static_cast<int64_t>(i) * Tp + sidx] : (sidx == -1 ? -feq[i] : 0.0);
  if (t == 0) nu[i] = AB[static_cast<int64_t>(i) * Tp + inu];
}

__global__ void polar_xc_kernel(int nv, int nm, const double* __restrict__ vnode, const double* __restrict__ xi,
                                const double* __restrict__ sc, const double* __restrict__ C, double* __restrict__ Xc) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= static_cast<int64_t>(nv) * nm) return;
  const int i = static_cast<int>(idx / nm), m = static_cast<int>(idx % nm);
  const double ph = xi[m] * vnode[i] + xi[nm + m] * vnode[nv + i] + xi[2 * nm + m] * vnode[2 * nv + i];
  const double cm = C[idx] * sc[m];
  double sn, cs;
  sincos(ph, &sn, &cs);
  Xc[2 * idx] = cm * cs;
  Xc[2 * idx + 1] = cm * sn;
}

__global__ void polar_op2_kernel(int nv, int nm, const double* __restrict__ vnode, const double* __restrict__ xi,
                                 const double* __restrict__ wp, double* __restrict__ Op2) {
  const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (idx >= static_cast<int64_t>(nv) * nm) return;
  const int j = static_cast<int>(idx / nm), m = static_cast<int>(idx % nm);
  double sa, ca, sc_, cc;
  sincos(xi[m] * vnode[j], &sa, &ca);
  const double cb = cos(xi[nm + m] * vnode[nv + j]);
  sincos(xi[2 * nm + m] * vnode[2 * nv + j], &sc_, &cc);
  const double w4 = 4.0 * wp[j] * cb * sc_;
  Op2[2 * idx] = -w4 * sa;
  Op2[2 * idx + 1] = w4 * ca;
}

// ------------------------------------------------------------------ tube
// One workgroup per (case, group of kTubeV (v_r, v_z) pairs).  Inward molecules
// (th > pi/2) are swept from the wall to the centre, then outward ones from the
// centre to the wall; in both passes a node depends on its two r-upwind nodes and
// its two th-upwind (larger th) nodes, so the anti-diagonals of (r, th) are
// processed in order with a workgroup barrier between them.
constexpr int kTubeV = 8;
constexpr int kTubeThreads = 256;

__global__ __launch_bounds__(kTubeThreads) void sweep_tube_kernel(TubeSweepArgs a) {
  const int cs = blockIdx.y;
  if (a.case_active && !a.case_active[cs]) return;
  const int nth = a.n_th, half = nth / 2, nvz = a.n_vz, nv = a.nv;
  const int pairs = a.n_vr * nvz;
  const int tq = blockIdx.x * kTubeV + threadIdx.x % kTubeV;
  const bool valid = tq < pairs;
  const int q = valid ? tq : 0;
  const int ivr = q / nvz, iz = q % nvz;
  const int slot = threadIdx.x / kTubeV, slots = kTubeThreads / kTubeV;
  const int64_t n0 = a.node_off[cs];
  const int n = static_cast<int>(a.node_off[cs + 1] - n0);
  const double del = a.delta_case[cs];
  const double vr = a.vr[ivr];
  const double tc = 1.0 / (2.0 * a.dth);
  auto vix = [&](int k) { return (ivr * nth + k) * nvz + iz; };
  // wall node, inward velocities: molecules leaving a diffuse wall carry h = 0
  for (int kk = slot; kk < half; kk += slots)
    if (valid) a.h[(n0 + n - 1) * nv + vix(half + kk)] = 0.0;
  __syncthreads();
  // inward pass: ii = n - 2 - i, kk = n_th - 1 - k
  for (int d = 0; d <= (n - 2) + (half - 1); ++d) {
    const int lo = max(0, d - (n - 2)), hi = min(d, half - 1);
    for (int c0 = lo; c0 <= hi; c0 += slots) {
      const int kk = c0 + slot;
      if (valid && kk <= hi) {
        const int i = n - 2 - (d - kk), k = nth - 1 - kk;
        const int64_t node = n0 + i;
        const int v = vix(k);
        const double c1 = vr * a.cth[k], ct = vr * a.sth[k] / a.r[node];
        const double* cf = a.cin + node * 3;
        double up = cf[1] * a.h[(node + 1) * nv + v];
        if (i < n - 2) up += cf[2] * a.h[(node + 2) * nv + v];
        double diag = del * a.nu[v] + c1 * cf[0];
        double src = a.rhs[node * nv + v] - c1 * up;
        if (k < nth - 1) {
          const int k2 = min(k + 2, nth - 1);
          diag += ct * 3.0 * tc;
          src += ct * (4.0 * a.h[node * nv + vix(k + 1)] - a.h[node * nv + vix(k2)]) * tc;
        }
        a.h[node * nv + v] = src / diag;
      }
    }
    __syncthreads();
  }
  // outward pass: kk = half - 1 - k; ghosts across the centre hold h(r, pi - th)
  for (int d = 0; d <= (n - 1) + (half - 1); ++d) {
    const int lo = max(0, d - (n - 1)), hi = min(d, half - 1);
    for (int c0 = lo; c0 <= hi; c0 += slots) {
      const int kk = c0 + slot;
      if (valid && kk <= hi) {
        const int i = d - kk, k = half - 1 - kk, km = nth - 1 - k;
        const int64_t node = n0 + i;
        const int v = vix(k);
        const double c1 = vr * a.cth[k], ct = vr * a.sth[k] / a.r[node];
        const double* cf = a.cout + node * 3;
        const double y1 = i >= 1 ? a.h[(node - 1) * nv + v] : a.h[n0 * nv + vix(km)];
        const double y2 = i >= 2 ? a.h[(node - 2) * nv + v] : a.h[(n0 + 1 - i) * nv + vix(km)];
        const double diag = del * a.nu[v] + c1 * cf[0] + ct * 3.0 * tc;
        const double src = a.rhs[node * nv + v] - c1 * (cf[1] * y1 + cf[2] * y2) +
                           ct * (4.0 * a.h[node * nv + vix(k + 1)] - a.h[node * nv + vix(k + 2)]) * tc;
        a.h[node * nv + v] = src / diag;
      }
    }
    __syncthreads();
  }
}

__global__ __launch_bounds__(256) void moments_tube_kernel(int nv, const double* __restrict__ vnode,
                                                           const double* __restrict__ wnode,
                                                           const double* __restrict__ h,
                                                           const int32_t* __restrict__ active,
                                                           double* __restrict__ mom) {
  __shared__ double sh[4 * 5];
  const int64_t c = blockIdx.x;
  if (active && !active[c]) return;
  double m[5] = {0, 0, 0, 0, 0};
  for (int v = threadIdx.x; v < nv; v += blockDim.x) {
    const double v1 = vnode[v], v2 = vnode[nv + v], v3 = vnode[2 * nv + v];
    const double x = wnode[v] * h[c * nv + v];
    m[0] += v3 * x;
    m[1] += (v1 * v1 + v2 * v2 + v3 * v3 - 2.5) * v3 * x;
    m[2] += v3 * (2.0 * v1 * v1 - 1.0) * x;
    m[3] += 2.0 * v3 * (v1 * v1 - v2 * v2) * x;
    m[4] += 2.0 * v1 * v3 * x;
  }
  block_sum<5>(m, sh);
  if (threadIdx.x == 0) {
    for (int k = 0; k < 5; ++k) mom[c * 8 + k] = m[k];
    mom[c * 8 + 5] = 0.0;
    mom[c * 8 + 6] = 0.0;
    mom[c * 8 + 7] = 0.0;
  }
}

// Velocity equation of the tube, one workgroup per case: a march over the radial nodes
// from the wall inwards (one lane; inputs and outputs staged through LDS in coalesced
// chunks as in diffusion1d_kernel), outputs, flow rates 2 int_0^1 f r dr and the
// convergence test.
__global__ __launch_bounds__(kDiffChunk) void diffusion_tube_kernel(TubeDiffArgs a) {
  __shared__ double in[8][kDiffChunk];    // U3, q3, G, source, c0, c1, c2, weight
  __shared__ double out[4][kDiffChunk];   // U, dU, U and q of the new iterate
  const int cs = blockIdx.x;
  if (a.case_active && !a.case_active[cs]) return;   // uniform over the workgroup
  const int64_t n0 = a.node_off[cs];
  const int n = static_cast<int>(a.node_off[cs + 1] - n0);
  const double del = a.delta_case[cs];
  const bool pois = a.flow_case[cs] == 1;
  const double Nd = a.N * del;
  double y1 = 0.0, y2 = 0.0, M = 0.0, Q = 0.0;
  for (int end = n; end > 0; end -= kDiffChunk) {
    const int lo = max(0, end - kDiffChunk), cnt = end - lo;
    for (int t = threadIdx.x; t < cnt; t += blockDim.x) {
      const int i = lo + t;
      const int64_t node = n0 + i;
      const double* m = a.mom + node * 8;
      in[0][t] = m[0];
      in[1][t] = m[1];
      in[2][t] = m[2];
      in[7][t] = a.tw[node];
      if (a.sis && i < n - 1) {
        double A = 0.0;
        if (a.amom) A = a.amom[node * 4 + 0] + Nd * a.amom[node * 4 + 1];
        const double r = a.r[node];
        in[3][t] = A - m[3] / r - (pois ? Nd * r / 2.0 : 0.0);
        in[4][t] = a.cin[node * 3 + 0];
        in[5][t] = a.cin[node * 3 + 1];
        in[6][t] = a.cin[node * 3 + 2];
      }
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      for (int t = cnt - 1; t >= 0; --t) {
        const int i = lo + t;
        const double U3 = in[0][t], q3 = in[1][t], G = in[2][t];
        double dU = 0.0, U = U3;
        if (a.sis) {
          double y;
          if (i == n - 1)
            y = U3 + G;
          else if (i == n - 2)
            y = (in[3][t] - in[5][t] * y1) / in[4][t];
          else
            y = (in[3][t] - in[5][t] * y1 - in[6][t] * y2) / in[4][t];
          y2 = y1;
          y1 = y;
          U = y - G;
          dU = U - U3;
        }
        const double Un = U3 + dU * a.cU, qn = q3 + dU * a.cq;
        out[0][t] = U;
        out[1][t] = dU;
        out[2][t] = Un;
        out[3][t] = qn;
        M += in[7][t] * Un;
        Q += in[7][t] * qn;
      }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < cnt; t += blockDim.x) {
      const int64_t node = n0 + lo + t;
      if (a.U) a.U[node] = out[0][t];
      if (a.dU) a.dU[node] = out[1][t];
      if (a.ufield) a.ufield[node] = out[2][t];
      if (a.qfield) a.qfield[node] = out[3][t];
    }
  }
  if (threadIdx.x == 0 && a.state) {
    double* st = a.state + cs * 4;
    const double dM = fabs(M - st[0]) / fmax(fabs(M), 1e-300);
    const double dQ = fabs(Q - st[1]) / fmax(fabs(Q), 1e-300);
    const double res = fmax(dM, dQ);
    st[0] = M;
    st[1] = Q;
    st[2] = (M != M || Q != Q) ? __builtin_nan("") : res;
    const int k = a.iters[cs] + 1;
    a.iters[cs] = k;
    if (!(res >= a.eps) || M != M || Q != Q) a.case_active[cs] = 0;
    st[3] = static_cast<double>(k);
  }
}

// ------------------------------------------------------------------ persistent 1-D iteration
// Small planar batches (a few dozen cells, the coarse-grid setting) are bound by launch
// latency: one iteration is six dependent launches of a few microseconds of work each.
// This kernel runs n_iters whole iterations in one cooperative launch: the same phases
// as the launched path (contraction over virtual 32 x 128 tiles and split-K slices,
// finish rows, sweep blocks, moment rows, one velocity-equation march per case, which
// also writes its cells' active flags), each a grid-stride loop over the phase's units,
// separated by grid barriers.  Results equal the launched path's to rounding (the
// split-K slicing of the contraction differs).
//
// Grid barrier: one arrival counter that only grows within a launch (barrier number t
// completes when it reaches t * gridDim.x) and a release word; agent-scope fences on
// both sides make each phase's writes visible to every XCD's caches.  The wait is
// bounded: a wait that runs out sets the abort word, every later barrier returns at
// once, and the host reports the launch as failed (no hang).
constexpr int kBarrierSpin = 1 << 22;

__device__ inline void grid_barrier(unsigned* bar, unsigned& gen) {
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    const unsigned target = ++gen;
    if (__hip_atomic_load(&bar[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0) {
      const unsigned arrived = __hip_atomic_fetch_add(&bar[0], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) + 1;
      if (arrived == target * gridDim.x) {
        __hip_atomic_store(&bar[1], target, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        int n = 0;
        while (__hip_atomic_load(&bar[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
          if (++n > kBarrierSpin) {
            __hip_atomic_store(&bar[2], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
          }
          if (__hip_atomic_load(&bar[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) break;
          __builtin_amdgcn_s_sleep(1);
        }
      }
    }
    __threadfence();
  } else {
    ++gen;
  }
  __syncthreads();
}

__global__ __launch_bounds__(256) void sis1d_persistent_kernel(Persist1DArgs a) {
  __shared__ int32_t case_flag;
  unsigned gen = 0;
  const int G = gridDim.x;
  const int n_n = (a.n3 + 127) / 128;
  const int n_m = static_cast<int>((a.n_cells + 31) / 32);
  const int n_tiles = n_n * n_m * a.splits;
  const int nbx = (a.sw.n3 / 2 + 255) / 256;
  const int n_sweep = nbx * a.sw.n_cases;
  for (int it = 0; it < a.n_iters; ++it) {
    const bool zero = a.first_from_zero && it == 0;   // h = 0: L+ h = 0, no contraction
    if (!zero) {
      for (int t = blockIdx.x; t < n_tiles; t += G) {
        const int bz = t / (n_n * n_m), r = t - bz * (n_n * n_m);
        gemm_f64_tile<32, 128, 32, 32>(a.h, a.op, a.acc, a.n_cells, a.n3, a.n3, a.kps, r % n_n, r / n_n, bz);
        __syncthreads();
      }
      grid_barrier(a.bar, gen);
    }
    for (int64_t c = blockIdx.x; c < a.fin.n_cells; c += G) {
      finish_row(a.fin, c, zero ? 0 : a.splits, zero ? nullptr : a.acc);
      __syncthreads();
    }
    grid_barrier(a.bar, gen);
    for (int t = blockIdx.x; t < n_sweep; t += G) sweep1d_block(a.sw, t % nbx, t / nbx, 0);
    grid_barrier(a.bar, gen);
    for (int64_t c = blockIdx.x; c < a.n_cells; c += G) {
      moments_row(a.sw.n3, 1, 1.0, 1.0, a.vtab, a.sw.h, a.w, a.mom, c);
      __syncthreads();
    }
    grid_barrier(a.bar, gen);
    for (int cs = blockIdx.x; cs < a.dif.n_cases; cs += G) {
      diffusion1d_case(a.dif, cs);
      __syncthreads();
      // the case's flag, as its march left it, for the cell-level flags of the next finish
      if (threadIdx.x == 0) case_flag = __hip_atomic_load(&a.dif.case_active[cs], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __syncthreads();
      const int64_t c0 = a.dif.node_off[cs], c1 = a.dif.node_off[cs + 1];
      for (int64_t c = c0 + threadIdx.x; c < c1; c += blockDim.x) a.cell_active[c] = case_flag;
      __syncthreads();
    }
    grid_barrier(a.bar, gen);
  }
}

__global__ void zero_u32_kernel(unsigned* p, int n) {
  if (static_cast<int>(threadIdx.x) < n) p[threadIdx.x] = 0u;
}

__global__ void expand_active_kernel(const int32_t* __restrict__ case_active,
                                     const int32_t* __restrict__ case_of_cell, int64_t n_cells,
                                     int32_t* __restrict__ cell_active) {
  const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
  if (i < n_cells) cell_active[i] = case_active[case_of_cell[i]];
}

}  // namespace

// ------------------------------------------------------------------ launchers
hipError_t launch_assemble(int n, int T, const double* X, const double* Y, const double* feq,
                           double loss_coef, const double* beta_r, double* op, int64_t ldo, int accumulate,
                           hipStream_t s) {
  const int nd = 2 * n - 1;
  const size_t shm = static_cast<size_t>(kAsmPB) * (nd + n) * sizeof(double);
  dim3 grid(n * n, n * n);
  hipLaunchKernelGGL(assemble_kernel, grid, dim3(256), shm, s, n, T, X, Y, feq, loss_coef, beta_r, op, ldo,
                     accumulate);
  return hipGetLastError();
}

hipError_t launch_reduce_operator(const double* op, int64_t ld, double* red, int nsp, int n, int parity,
                                  hipStream_t s) {
  const int d2 = parity == 2 ? n / 2 : n, d3 = n / 2;
  const int64_t ldr = static_cast<int64_t>(nsp) * n * d2 * d3;
  const int64_t count = ldr * ldr;
  hipLaunchKernelGGL(reduce_operator_kernel, dim3(static_cast<unsigned>((count + 255) / 256)), dim3(256), 0, s, op,
                     ld, red, nsp, n, parity);
  return hipGetLastError();
}

int pair_stride(int K) { return (K + 63) / 64 * 64; }

hipError_t launch_split_pairs(const double* X, const double* Xref, int64_t rows, int K, uint16_t* P, int with_lo,
                              hipStream_t s) {
  const int Kp = pair_stride(K);
  const int64_t n = rows * Kp;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(split_pairs_kernel, dim3(static_cast<unsigned>((n + 255) / 256)), dim3(256), 0, s, X, Xref, rows,
                     K, Kp, P, with_lo);
  return hipGetLastError();
}

hipError_t launch_convert_x_f32(const double* X, const double* Xref, int64_t count, float* out, hipStream_t s) {
  hipLaunchKernelGGL(convert_x_f32_kernel, dim3(static_cast<unsigned>((count + 255) / 256)), dim3(256), 0, s, X, Xref,
                     count, out);
  return hipGetLastError();
}

hipError_t launch_convert_f32(const double* op, float* out, int64_t count, hipStream_t s) {
  hipLaunchKernelGGL(convert_f32_kernel, dim3((count + 255) / 256), dim3(256), 0, s, op, out, count);
  return hipGetLastError();
}

int gemm_k_per_split(int K, int splits) {
  const int unit = 64;  // multiple of every BK
  int kps = (K + splits - 1) / splits;
  kps = (kps + unit - 1) / unit * unit;
  return kps;
}

int gemm_tile_rows(int tile) {
  return tile == 5 ? 256 : (tile == 0 || tile == 3) ? 128 : (tile == 2 || tile == 4) ? 64 : 32;
}

int gemm_tile_depth(int tile, int precision) {
  if (tile == 5) return 32;        // 3xBF16, 256 x 256: 32-deep stages in two LDS buffers
  if (precision >= 2) return 64;   // bf16 forms: both operands staged in 64-deep stages
  return tile >= 3 ? 32 : 16;
}

bool gemm_wide_fits(int64_t M, int N, int K) {
  const int64_t row_bytes = 4 * static_cast<int64_t>(pair_stride(K));
  return M * row_bytes < (int64_t(1) << 32) && N * row_bytes < (int64_t(1) << 32);
}

hipError_t launch_gemm(const GemmArgs& g, hipStream_t s) {
  const int BN = 128;
  const int BM = gemm_tile_rows(g.tile);
  dim3 grid((g.N + BN - 1) / BN, static_cast<unsigned>((g.M + BM - 1) / BM), g.splits);
  if (g.tile >= 3 && g.precision == 1) return hipErrorInvalidValue;
  if (g.tile == 5 && g.precision != 2) return hipErrorInvalidValue;
  if ((g.tile == 3 || g.tile == 4) && g.precision != 0) return hipErrorInvalidValue;
  if (g.precision == 0) {
    if (g.K % 2) return hipErrorInvalidValue;   // rows are loaded in 16-byte k pairs
    const int kps = gemm_k_per_split(g.K, g.splits);
    if (g.tile == 0 && g.K <= (1 << 20))
      hipLaunchKernelGGL(gemm_f64_dma_kernel, grid, dim3(512), 0, s, g.X, g.op64, g.acc, g.M, g.N, g.K, kps);
    else if (g.tile == 0)
      hipLaunchKernelGGL((gemm_f64_kernel<128, 128, 64, 64>), grid, dim3(256), 0, s, g.X, g.op64, g.acc, g.M, g.N, g.K, kps);
    else if (g.tile == 2)
      hipLaunchKernelGGL((gemm_f64_kernel<64, 128, 32, 64>), grid, dim3(256), 0, s, g.X, g.op64, g.acc, g.M, g.N, g.K, kps);
    else if (g.tile == 3)
      hipLaunchKernelGGL((gemm_f64_kernel<128, 128, 64, 64, 32, 1, 1>), grid, dim3(256), 0, s, g.X, g.op64, g.acc, g.M, g.N, g.K, kps);
    else if (g.tile == 4)
      hipLaunchKernelGGL((gemm_f64_kernel<64, 128, 32, 64, 32, 1, 1>), grid, dim3(256), 0, s, g.X, g.op64, g.acc, g.M, g.N, g.K, kps);
    else
      hipLaunchKernelGGL((gemm_f64_kernel<32, 128, 32, 32>), grid, dim3(256), 0, s, g.X, g.op64, g.acc, g.M, g.N, g.K, kps);
  } else if (g.precision == 1) {
    const int kps = gemm_k_per_split(g.K, g.splits);
    if (!g.X32) return hipErrorInvalidValue;
    if (g.tile == 0)
      hipLaunchKernelGGL((gemm_f32_kernel<128, 128, 64, 64>), grid, dim3(256), 0, s, g.X32, g.op32, g.acc, g.M, g.N, g.K, kps);
    else if (g.tile == 2)
      hipLaunchKernelGGL((gemm_f32_kernel<64, 128, 32, 64>), grid, dim3(256), 0, s, g.X32, g.op32, g.acc, g.M, g.N, g.K, kps);
    else
      hipLaunchKernelGGL((gemm_f32_kernel<32, 128, 32, 32>), grid, dim3(256), 0, s, g.X32, g.op32, g.acc, g.M, g.N, g.K, kps);
  } else {
    // bf16 forms: operands in the pair layout, k running over the padded Kp (zeros past K); with
    // no cell operand in that layout (Xp null) the 32-row tile splits X (minus Xref) itself
    if (!g.opp) return hipErrorInvalidValue;
    const bool fused = !g.Xp;
    if (fused && (g.tile != 1 || !g.X || g.K % 2)) return hipErrorInvalidValue;
    const int Kp = pair_stride(g.K);
    const int kps = gemm_k_per_split(Kp, g.splits);
    if (g.precision == 3) {
      if (fused)
        hipLaunchKernelGGL((gemm_bf16x3_kernel<32, 128, 32, 32, 1, true>), grid, dim3(256), 0, s, g.Xp, g.opp, g.acc, g.M, g.N, Kp, kps, g.X, g.Xref, g.K);
      else if (g.tile == 0)
        hipLaunchKernelGGL((gemm_bf16x3_kernel<128, 128, 64, 64, 1>), grid, dim3(256), 0, s, g.Xp, g.opp, g.acc, g.M, g.N, Kp, kps, nullptr, nullptr, 0);
      else if (g.tile == 2)
        hipLaunchKernelGGL((gemm_bf16x3_kernel<64, 128, 32, 64, 1>), grid, dim3(256), 0, s, g.Xp, g.opp, g.acc, g.M, g.N, Kp, kps, nullptr, nullptr, 0);
      else
        hipLaunchKernelGGL((gemm_bf16x3_kernel<32, 128, 32, 32, 1>), grid, dim3(256), 0, s, g.Xp, g.opp, g.acc, g.M, g.N, Kp, kps, nullptr, nullptr, 0);
    } else if (g.tile == 5) {
      if (!gemm_wide_fits(g.M, g.N, g.K)) return hipErrorInvalidValue;
      dim3 wgrid((g.N + 255) / 256, static_cast<unsigned>((g.M + 255) / 256), g.splits);
      hipLaunchKernelGGL(gemm_bf16x3_wide_kernel, wgrid, dim3(512), 0, s, g.Xp, g.opp, g.acc, g.M, g.N, Kp, kps);
    } else if (fused) {
      hipLaunchKernelGGL((gemm_bf16x3_kernel<32, 128, 32, 32, 3, true>), grid, dim3(256), 0, s, g.Xp, g.opp, g.acc, g.M, g.N, Kp, kps, g.X, g.Xref, g.K);
    } else if (g.tile == 0) {
      hipLaunchKernelGGL((gemm_bf16x3_kernel<128, 128, 64, 64>), grid, dim3(256), 0, s, g.Xp, g.opp, g.acc, g.M, g.N, Kp, kps, nullptr, nullptr, 0);
    } else if (g.tile == 2) {
      hipLaunchKernelGGL((gemm_bf16x3_kernel<64, 128, 32, 64>), grid, dim3(256), 0, s, g.Xp, g.opp, g.acc, g.M, g.N, Kp, kps, nullptr, nullptr, 0);
    } else {
      hipLaunchKernelGGL((gemm_bf16x3_kernel<32, 128, 32, 32>), grid, dim3(256), 0, s, g.Xp, g.opp, g.acc, g.M, g.N, Kp, kps, nullptr, nullptr, 0);
    }
  }
  return hipGetLastError();
}

hipError_t launch_finish(const FinishArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(finish_kernel, dim3(static_cast<unsigned>(a.n_cells)), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_sweep1d(const SweepArgs& a, hipStream_t s) {
  const int half = a.n3 / 2;
  dim3 grid((half + 255) / 256, a.n_cases, a.nsp);
  hipLaunchKernelGGL(sweep1d_kernel, grid, dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_moments(int n3, int nsp, const double* mass_ratio, int64_t n_rows, const double* vtab,
                          const double* h, double w, double* mom, hipStream_t s) {
  const double m0 = mass_ratio ? mass_ratio[0] : 1.0, m1 = mass_ratio && nsp > 1 ? mass_ratio[1] : 1.0;
  hipLaunchKernelGGL(moments_kernel, dim3(static_cast<unsigned>(n_rows)), dim3(256), 0, s, n3, nsp, m0, m1, vtab, h,
                     w, mom);
  return hipGetLastError();
}

hipError_t launch_diffusion1d(const DiffusionArgs& a, hipStream_t s) {
  if (a.nsp == 2)
    hipLaunchKernelGGL(diffusion1d_mix_kernel, dim3(a.n_cases), dim3(kDiffChunk), 0, s, a);
  else
    hipLaunchKernelGGL(diffusion1d_kernel, dim3(a.n_cases), dim3(kDiffChunk), 0, s, a);
  return hipGetLastError();
}


int sweep2d_form(int max_diag, int max_n2, int64_t row_bytes_total) {
  if (max_n2 <= kRowWaves * 8 && row_bytes_total < (int64_t(1) << 31)) return 1;
  const int slots = kSweepThreads / kSweepV;
  return (max_diag + slots - 1) / slots <= kSweepMaxP ? 2 : 3;
}

hipError_t launch_sweep2d(const Sweep2DArgs& a, hipStream_t s) {
  const int hn = a.n / 2;
  const int count = hn * hn * a.d3;
  const int form = sweep2d_form(a.max_diag, a.max_n2, a.row_bytes_total);
  if (form == 1) {
    const int cwmax = a.max_n2 <= kRowWaves * 4 ? 4 : 8;
    const int W = (a.max_n2 + cwmax - 1) / cwmax;
    dim3 grid(((count + 63) / 64) * a.n_cases * a.nsp * (a.quad_split ? 4 : 1));
    if (cwmax == 4)
      hipLaunchKernelGGL(sweep2d_rows_kernel<4>, grid, dim3(64 * W), 0, s, a, a.grec, a.growb, a.rhs, a.h);
    else
      hipLaunchKernelGGL(sweep2d_rows_kernel<8>, grid, dim3(64 * W), 0, s, a, a.grec, a.growb, a.rhs, a.h);
    return hipGetLastError();
  }
  dim3 grid((count + kSweepV - 1) / kSweepV, a.n_cases, a.nsp);
  const int slots = kSweepThreads / kSweepV;
  const int P = (a.max_diag + slots - 1) / slots;
  if (form == 3)
    hipLaunchKernelGGL(sweep2d_kernel, grid, dim3(kSweepThreads), 0, s, a);
  else if (P <= 1)
    hipLaunchKernelGGL(sweep2d_pipelined_kernel<1>, grid, dim3(kSweepThreads), 0, s, a);
  else if (P == 2)
    hipLaunchKernelGGL(sweep2d_pipelined_kernel<2>, grid, dim3(kSweepThreads), 0, s, a);
  else
    hipLaunchKernelGGL(sweep2d_pipelined_kernel<3>, grid, dim3(kSweepThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_moments2d(int n3, int nsp, const double* mass_ratio, int64_t n_cells, const double* vtab,
                            const double* h, double w, const int32_t* cell_active, double* mom, hipStream_t s) {
  hipLaunchKernelGGL(moments2d_kernel, dim3(static_cast<unsigned>(n_cells * nsp)), dim3(256), 0, s, n3, nsp,
                     mass_ratio[0], nsp > 1 ? mass_ratio[1] : 1.0, vtab, h, w, cell_active, mom);
  return hipGetLastError();
}

hipError_t launch_diffusion2d(const Diff2DArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(diffusion2d_kernel, dim3(a.n_cases), dim3(kD2Threads), 0, s, a);
  if (a.direct) {
    hipLaunchKernelGGL(diffusion2d_rhs_kernel, dim3(a.n_cases), dim3(kD2Threads), 0, s, a);
    if (a.max_unknown > 0 && a.n_groups > 0)
      hipLaunchKernelGGL(diffusion2d_gemv_kernel, dim3((a.max_unknown + 3) / 4, a.n_groups), dim3(256), 0, s, a);
    hipLaunchKernelGGL(diffusion2d_out_kernel, dim3(a.n_cases), dim3(kD2Threads), 0, s, a);
  }
  return hipGetLastError();
}

hipError_t launch_ns_residual(const double* P, int n, double* part, int blocks, hipStream_t s) {
  hipLaunchKernelGGL(ns_residual_kernel, dim3(blocks), dim3(256), 0, s, P, n, part);
  return hipGetLastError();
}

hipError_t launch_ns_two_minus(double* P, int n, hipStream_t s) {
  const int64_t count = static_cast<int64_t>(n) * n;
  hipLaunchKernelGGL(ns_two_minus_kernel, dim3(static_cast<unsigned>((count + 255) / 256)), dim3(256), 0, s, P, n);
  return hipGetLastError();
}

hipError_t launch_ns_scale(const double* X, int ldx, int n, const double* sc, double* out, hipStream_t s) {
  const int64_t count = static_cast<int64_t>(n) * n;
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(ns_scale_kernel, dim3(static_cast<unsigned>((count + 255) / 256)), dim3(256), 0, s, X, ldx, n,
                     sc, out);
  return hipGetLastError();
}

hipError_t launch_ns_scatter(double* S, int n, const int32_t* rc, const double* val, int64_t count, hipStream_t s) {
  if (count == 0) return hipSuccess;
  hipLaunchKernelGGL(ns_scatter_kernel, dim3(static_cast<unsigned>((count + 255) / 256)), dim3(256), 0, s, S, n, rc,
                     val, count);
  return hipGetLastError();
}

hipError_t launch_ns_init(double* X, int n, double alpha, hipStream_t s) {
  const int64_t count = static_cast<int64_t>(n) * n;
  hipLaunchKernelGGL(ns_init_kernel, dim3(static_cast<unsigned>((count + 255) / 256)), dim3(256), 0, s, X, n, alpha);
  return hipGetLastError();
}

int persist1d_max_blocks() {
  int dev = 0, cus = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, sis1d_persistent_kernel, 256, 0) != hipSuccess) return 0;
  return cus * per;
}

hipError_t launch_persist1d(const Persist1DArgs& a, int blocks, hipStream_t s) {
  if (blocks < 1 || blocks > persist1d_max_blocks()) return hipErrorInvalidConfiguration;
  if (a.sw.nsp != 1 || a.fin.nsp != 1 || a.n3 != a.sw.n3) return hipErrorInvalidValue;
  // the barrier words start at zero in every launch (a fill kernel, not a memset node, in
  // case the caller captures the stream)
  hipLaunchKernelGGL(zero_u32_kernel, dim3(1), dim3(64), 0, s, a.bar, 4);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  Persist1DArgs arg = a;
  void* params[] = {&arg};
  return hipLaunchCooperativeKernel(reinterpret_cast<const void*>(sis1d_persistent_kernel), dim3(blocks), dim3(256),
                                    params, 0, s);
}

hipError_t launch_expand_active(const int32_t* case_active, const int32_t* case_of_cell,
                                int64_t n_cells, int32_t* cell_active, hipStream_t s) {
  hipLaunchKernelGGL(expand_active_kernel, dim3(static_cast<unsigned>((n_cells + 255) / 256)), dim3(256), 0, s,
                     case_active, case_of_cell, n_cells, cell_active);
  return hipGetLastError();
}

hipError_t launch_polar_fhat(int nm, const double* xi, int nv, const double* vnode, const double* wf, double* fhat,
                             hipStream_t s) {
  hipLaunchKernelGGL(polar_fhat_kernel, dim3((nm + 255) / 256), dim3(256), 0, s, nm, xi, nv, vnode, wf, fhat);
  return hipGetLastError();
}

static dim3 grid_for(int64_t count) { return dim3(static_cast<unsigned>((count + 255) / 256)); }

hipError_t launch_polar_cos(int nv, int nm, const double* vnode, const double* xi, double* X, hipStream_t s) {
  hipLaunchKernelGGL(polar_cos_kernel, grid_for(static_cast<int64_t>(nv) * nm), dim3(256), 0, s, nv, nm, vnode, xi, X);
  return hipGetLastError();
}

hipError_t launch_polar_scale_terms(int Tp, int nm, const double* mt, const double* fhat, const double* sc,
                                    double* out, hipStream_t s) {
  hipLaunchKernelGGL(polar_scale_terms_kernel, grid_for(static_cast<int64_t>(Tp) * nm), dim3(256), 0, s, Tp, nm, mt,
                     fhat, sc, out);
  return hipGetLastError();
}

hipError_t launch_polar_coef(int nv, int Tp, const double* AB, const int32_t* src, const double* c,
                             const double* feq, int inu, double* aT, double* nu, hipStream_t s) {
  hipLaunchKernelGGL(polar_coef_kernel, grid_for(static_cast<int64_t>(nv) * Tp), dim3(256), 0, s, nv, Tp, AB, src, c,
                     feq, inu, aT, nu);
  return hipGetLastError();
}

hipError_t launch_polar_xc(int nv, int nm, const double* vnode, const double* xi, const double* sc,
                           const double* C, double* Xc, hipStream_t s) {
  hipLaunchKernelGGL(polar_xc_kernel, grid_for(static_cast<int64_t>(nv) * nm), dim3(256), 0, s, nv, nm, vnode, xi,
                     sc, C, Xc);
  return hipGetLastError();
}

hipError_t launch_polar_op2(int nv, int nm, const double* vnode, const double* xi, const double* wp, double* Op2,
                            hipStream_t s) {
  hipLaunchKernelGGL(polar_op2_kernel, grid_for(static_cast<int64_t>(nv) * nm), dim3(256), 0, s, nv, nm, vnode, xi,
                     wp, Op2);
  return hipGetLastError();
}

hipError_t launch_sweep_tube(const TubeSweepArgs& a, hipStream_t s) {
  if (a.max_nodes < 3) return hipErrorInvalidValue;
  const int pairs = a.n_vr * a.n_vz;
  dim3 grid((pairs + kTubeV - 1) / kTubeV, a.n_cases);
  hipLaunchKernelGGL(sweep_tube_kernel, grid, dim3(kTubeThreads), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_moments_tube(int64_t n_nodes, int nv, const double* vnode, const double* wnode, const double* h,
                               const int32_t* active, double* mom, hipStream_t s) {
  if (n_nodes == 0) return hipSuccess;
  hipLaunchKernelGGL(moments_tube_kernel, dim3(static_cast<unsigned>(n_nodes)), dim3(256), 0, s, nv, vnode, wnode,
                     h, active, mom);
  return hipGetLastError();
}

hipError_t launch_diffusion_tube(const TubeDiffArgs& a, hipStream_t s) {
  hipLaunchKernelGGL(diffusion_tube_kernel, dim3(a.n_cases), dim3(kDiffChunk), 0, s, a);
  return hipGetLastError();
}

}  // namespace sis
