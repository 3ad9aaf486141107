// Step a8, eigensolve: the lowest k eigenpairs of the full symmetric-definite
// pencil (H, S) of an open-boundary chain (Sec. 5, the full eigensolver that
// the FFT-based diagonalisation is compared with; Sec. 2.1 eq. (HF-FSpace):
// H C = S C Lambda, C^T S C = I).
//
// Route (all FP64, every step a kernel of this file):
//   1. S = L L^T, blocked right-looking Cholesky; the 64 x 64 diagonal blocks
//      are factored and inverted in LDS, the panel solve and the trailing
//      update are FP64-MFMA GEMMs.
//   2. L^-1 by recursive doubling of the diagonal-block inverses
//      (inv [[A,0],[B,C]] = [[A^-1,0],[-C^-1 B A^-1, C^-1]]), batched GEMMs.
//   3. C = L^-1 H L^-T: two triangle-aware GEMMs, lower tiles mirrored.
//   4. Householder tridiagonalisation C = Q T Q^T, one launch per column:
//      every workgroup forms the column's reflector (a few vectors from L2),
//      then applies the previous step's rank-2 update to its trailing rows
//      and multiplies them by the reflector in the same pass (one read and
//      one write of the trailing matrix per column).
//   5. The k lowest eigenvalues of T by Sturm-count multisection, one launch
//      per round, 4096 points per eigenvalue and round over 8 workgroups.
//   6. Eigenvectors of T by inverse iteration (partial-pivoting tridiagonal
//      LU, three solves), orthonormalised by two Cholesky-QR passes.
//   7. Back-transformation by the reflectors (compact WY blocks of 32) and
//      u = L^-T x.
#include <algorithm>
#include <cfloat>
#include <cmath>

#include <utility>

#include "common.h"
#include "dev_wave.h"

namespace tl {
namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kNB = 64;         // Cholesky / inverse block
constexpr int kWY = 32;         // reflectors per back-transformation block
constexpr int kMaxK = 64;       // eigenpairs per call
constexpr int kMaxN = 7680;     // order (z in LDS during the back-transformation)

// ------------------------------------------------------------------ helpers

__device__ __forceinline__ double wave_sum(double v) { return dev::wave_sum_dpp(v); }

// Reciprocal and reciprocal square root from the hardware estimates refined
// by two Newton steps each (full FP64 accuracy, not necessarily correctly
// rounded); arguments normal and finite.  They shorten the dependent chains
// of the sequential steps against the correctly rounded sequences.
__device__ __forceinline__ double nrcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ double nrsq(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double h = 0.5 * x;
  y = y * fma(-h * y, y, 1.5);
  return y * fma(-h * y, y, 1.5);
}

// Sum over a 256-thread workgroup; every thread gets the result.
__device__ inline double block_sum(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  return red[0] + red[1] + red[2] + red[3];
}

// ------------------------------------------------------------------ GEMM
// C = alpha op(A)... with A row-major M x K and op(B)[k][n] = TB ? B[n][k] :
// B[k][n].  kclip: 0 none; 1 A lower triangular (k <= m); 2 B lower, used as
// is (k >= n); 3 B lower, used transposed (k <= n).  lower: only tiles and
// entries with n <= m; mirror: also store C[n][m].  Batched on blockIdx.z.
struct GemmArgs {
  const double* A;
  const double* B;
  double* C;
  int64_t lda, ldb, ldc;
  int64_t sA, sB, sC;
  int M, N, K;
  double alpha, beta;
  int kclip, lower, mirror;
};

template <bool TB>
__global__ __launch_bounds__(256) void gemm_f64_kernel(GemmArgs g) {
  __shared__ double As[2][64][17];
  __shared__ double Bs[2][64][17];  // [n][k]
  const int m0 = blockIdx.y * 64, n0 = blockIdx.x * 64;
  if (g.lower && n0 > m0) return;  // uniform per workgroup, before any barrier
  const double* A = g.A + (int64_t)blockIdx.z * g.sA;
  const double* B = g.B + (int64_t)blockIdx.z * g.sB;
  double* C = g.C + (int64_t)blockIdx.z * g.sC;
  int kb = 0, ke = g.K;
  if (g.kclip == 1) ke = min(ke, m0 + 64);
  if (g.kclip == 2) kb = n0;
  if (g.kclip == 3) ke = min(ke, n0 + 64);
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  f64x4 acc[2][2];
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) acc[i][j] = f64x4{0.0, 0.0, 0.0, 0.0};
  double ra[4], rb[4];
  auto load = [&](int k0) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      {
        const int r = e >> 4, kk = e & 15, m = m0 + r, k = k0 + kk;
        ra[q] = (m < g.M && k < ke) ? A[(int64_t)m * g.lda + k] : 0.0;
      }
      if (TB) {
        const int c = e >> 4, kk = e & 15, n = n0 + c, k = k0 + kk;
        rb[q] = (n < g.N && k < ke) ? B[(int64_t)n * g.ldb + k] : 0.0;
      } else {
        const int kk = e >> 6, c = e & 63, n = n0 + c, k = k0 + kk;
        rb[q] = (n < g.N && k < ke) ? B[(int64_t)k * g.ldb + n] : 0.0;
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q;
      As[buf][e >> 4][e & 15] = ra[q];
      if (TB)
        Bs[buf][e >> 4][e & 15] = rb[q];
      else
        Bs[buf][e & 63][e >> 6] = rb[q];
    }
  };
  if (kb < ke) {
    load(kb);
    store(0);
    __syncthreads();
    int cur = 0;
    for (int k0 = kb; k0 < ke; k0 += 16) {
      const bool more = k0 + 16 < ke;
      if (more) load(k0 + 16);
#pragma unroll
      for (int kk = 0; kk < 16; kk += 4) {
        double a[2], b[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) a[i] = As[cur][wm * 32 + i * 16 + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
        for (int j = 0; j < 2; ++j) b[j] = Bs[cur][wn * 32 + j * 16 + (lane & 15)][kk + (lane >> 4)];
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
          for (int j = 0; j < 2; ++j)
            acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[i], b[j], acc[i][j], 0, 0, 0);
      }
      if (more) store(cur ^ 1);
      __syncthreads();
      cur ^= 1;
    }
  }
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = m0 + wm * 32 + i * 16 + (lane >> 4) + 4 * r;
        const int n = n0 + wn * 32 + j * 16 + (lane & 15);
        if (m >= g.M || n >= g.N) continue;
        if (g.lower && n > m) continue;
        double v = g.alpha * acc[i][j][r];
        if (g.beta != 0.0) v += g.beta * C[(int64_t)m * g.ldc + n];
        C[(int64_t)m * g.ldc + n] = v;
        if (g.mirror && n != m) C[(int64_t)n * g.ldc + m] = v;
      }
}

tl_status gemm(const GemmArgs& g, bool tb, int batch, hipStream_t stream) {
  if (g.M <= 0 || g.N <= 0 || batch <= 0) return TL_OK;
  dim3 grid((unsigned)ceil_div(g.N, 64), (unsigned)ceil_div(g.M, 64), (unsigned)batch);
  if (tb)
    hipLaunchKernelGGL(gemm_f64_kernel<true>, grid, dim3(256), 0, stream, g);
  else
    hipLaunchKernelGGL(gemm_f64_kernel<false>, grid, dim3(256), 0, stream, g);
  TL_CHECK_LAUNCH();
  return TL_OK;
}

GemmArgs gemm_args(const double* A, int64_t lda, const double* B, int64_t ldb, double* C,
                   int64_t ldc, int M, int N, int K, double alpha, double beta, int kclip) {
  GemmArgs g;
  std::memset(&g, 0, sizeof(g));
  g.A = A;
  g.B = B;
  g.C = C;
  g.lda = lda;
  g.ldb = ldb;
  g.ldc = ldc;
  g.M = M;
  g.N = N;
  g.K = K;
  g.alpha = alpha;
  g.beta = beta;
  g.kclip = kclip;
  return g;
}

// ------------------------------------------------------------------ set-up
// L <- lower triangle of S padded with the identity to Np x Np (upper zero);
// Linv <- 0; info <- 0.
__global__ __launch_bounds__(256) void setup_kernel(const double* __restrict__ S, int N, int Np,
                                                    double* __restrict__ L,
                                                    double* __restrict__ Linv, int* info) {
  const int64_t idx = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (idx == 0) *info = 0;
  if (idx >= (int64_t)Np * Np) return;
  const int r = (int)(idx / Np), c = (int)(idx - (int64_t)r * Np);
  double v = 0.0;
  if (c <= r) v = (r < N) ? S[(int64_t)r * N + c] : (r == c ? 1.0 : 0.0);
  L[idx] = v;
  Linv[idx] = 0.0;
}

constexpr int kLw = kNB + 2;
struct __attribute__((aligned(16))) CholWaveLds {
  double lt[kNB * kLw];  // L by columns: lt[c * kLw + r] = L[r][c], zero above the diagonal
  double rd[kNB];        // 1 / L[i][i]
};

// Column C of the factorisation (a compile-time index, so that a[] stays in
// registers: the whole 64-column nest is too large for the loop unroller).
// No branch inside, so that the updates of a column are not deferred into
// later columns.
template <int C>
__device__ __forceinline__ void chol_wave_col(double (&a)[kNB], int r, double pmin, int& fail,
                                              double& rdr) {
  double piv = dev::readlane_d(a[C], C);
  const bool bad = !(piv > fmax(pmin, 1e-300));  // pivots at or below 1e-300 count as failed
  fail = (bad && fail == 0) ? C + 1 : fail;
  piv = bad ? 1.0 : piv;
  const double rinv = nrsq(piv), lcc = piv * rinv;
  a[C] = r > C ? a[C] * rinv : (r == C ? lcc : 0.0);
  rdr = r == C ? rinv : rdr;
#pragma unroll
  for (int j = C + 1; j < kNB; ++j) a[j] = fma(-a[C], dev::readlane_d(a[C], j), a[j]);
}

template <int... C>
__device__ __forceinline__ void chol_wave_cols(double (&a)[kNB], int r, double pmin, int& fail,
                                               double& rdr, std::integer_sequence<int, C...>) {
  (chol_wave_col<C>(a, r, pmin, fail, rdr), ...);
}

// Step K of X = L^-1 by columns (lane r holds column r of X): X[K][r] is
// final once scaled, then goes into every later row with column K of L.
template <int K>
__device__ __forceinline__ void inv_wave_col(double (&x)[kNB], const CholWaveLds& sh) {
  x[K] *= sh.rd[K];
  const double xk = x[K];
#pragma unroll
  for (int i = (K + 1) & ~1; i < kNB; i += 2) {
    const double2 l = *(const double2*)&sh.lt[K * kLw + i];
    if (i >= K + 1) x[i] = fma(-l.x, xk, x[i]);
    x[i + 1] = fma(-l.y, xk, x[i + 1]);
  }
}

template <int... K>
__device__ __forceinline__ void inv_wave_cols(double (&x)[kNB], const CholWaveLds& sh,
                                              std::integer_sequence<int, K...>) {
  (inv_wave_col<K>(x, sh), ...);
}

// Cholesky factor and inverse of a 64 x 64 symmetric block in one wave,
// with no barrier: lane r keeps row r of the block in a[] (entries c > r
// ignored), every pivot and every column entry L[j][c] reaches the other
// lanes through readlane, and the rank-1 updates are FMAs with a scalar
// operand.  L then goes to LDS by columns and lane r solves column r of
// X = L^-1 in registers, reading the columns of L as LDS broadcasts.  On
// return sh.lt holds L and x[i] = X[i][r] (zero for i < r).  A pivot not
// above pmin is replaced by 1; the return value is the first such column + 1
// (0 if none).
__device__ __forceinline__ int chol_inv_64_wave(double (&a)[kNB], double (&x)[kNB], double pmin,
                                                CholWaveLds& sh) {
  const int r = threadIdx.x & 63;
  int fail = 0;
  double rdr = 1.0;  // 1 / L[r][r] on lane r
  chol_wave_cols(a, r, pmin, fail, rdr, std::make_integer_sequence<int, kNB>{});
  sh.rd[r] = rdr;
#pragma unroll
  for (int c = 0; c < kNB; ++c) sh.lt[c * kLw + r] = c <= r ? a[c] : 0.0;
  // one wave: its LDS accesses complete in program order, no barrier needed
#pragma unroll
  for (int i = 0; i < kNB; ++i) x[i] = i == r ? 1.0 : 0.0;
  inv_wave_cols(x, sh, std::make_integer_sequence<int, kNB>{});
  return fail;
}

// Factor the diagonal block at (p, p) in place (lower) and write its inverse
// into the same block of Linv.  A non-positive pivot records the first
// failing column (1-based) in *info and continues with pivot 1.
__global__ __launch_bounds__(64) void potrf_diag_kernel(double* __restrict__ L,
                                                        double* __restrict__ Linv, int64_t ld,
                                                        int p, int* info) {
  __shared__ CholWaveLds sh;
  const int r = threadIdx.x & 63;
  double a[kNB], x[kNB];
  const double* row = L + (int64_t)(p + r) * ld + p;
#pragma unroll
  for (int c = 0; c < kNB; ++c) a[c] = c <= r ? row[c] : 0.0;
  const int fail = chol_inv_64_wave(a, x, 0.0, sh);
  // column r of L from its LDS copy (a[] is dead after the factorisation)
#pragma unroll
  for (int i = 0; i < kNB; ++i) L[(int64_t)(p + i) * ld + p + r] = sh.lt[r * kLw + i];
  // lane r holds column r of the inverse
#pragma unroll
  for (int i = 0; i < kNB; ++i) Linv[(int64_t)(p + i) * ld + p + r] = x[i];
  if (r == 0 && fail != 0) {
    if (*info == 0) *info = p + fail;
  }
}

// ------------------------------------------------------------------ tridiagonalisation
struct TridArgs {
  double* C;         // N x N symmetric, row stride ld, overwritten
  double* Vt;        // reflector j in row j (length N, zero up to index j, 1 at j+1)
  double* y[2];      // y_j = tau_j A22 v_j, alternating by the parity of j
  double* part[2];   // per-workgroup partial sums of y_j . v_j, alternating
  double* d;         // diagonal of T
  double* e;         // off-diagonal of T
  double* tau;
  int64_t ld;
  int N;
};

constexpr int kTT = 256;  // threads of the tridiagonalisation kernel
constexpr int kTR = 4;    // trailing rows per workgroup

__device__ inline double block_sum_t(double v, double* red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[wave] = v;
  __syncthreads();
  double s = 0.0;
#pragma unroll
  for (int q = 0; q < kTT / 64; ++q) s += red[q];
  return s;
}

typedef double f64x2 __attribute__((ext_vector_type(2)));

// Step j, launched with one workgroup per kTR trailing rows (at least one).
// Every workgroup first forms the reflector of column j itself: row j of
// the matrix still carries step j-1's rank-2 update v w^T + w v^T, with
// w = y_{j-1} - 1/2 tau_{j-1} (y_{j-1} . v) v, which is applied on the fly
// (y . v is the sum of step j-1's nparts partials); v_j (LAPACK dlarfg
// convention, beta = -sign(alpha) ||x||) is kept in LDS and workgroup 0
// stores it with tau_j, d_j and e_j.  Then each workgroup applies step
// j-1's update to its rows (columns > j) and forms y_j[r] = tau_j A[r] v_j in
// the same pass: one read and one write of the trailing matrix per column,
// 16-byte accesses on even column pairs (row stride and vector offsets are
// even), columns <= j masked, and the 256 threads splitting the columns.
constexpr int kPU = 8;   // prologue elements per thread held in registers (n <= 2048)
constexpr int kPP = 2;   // partial sums per thread held in registers (nparts <= 512)

// NP > 0: the trailing rows' column pairs (at most 2 kTT NP columns) are all
// loaded into registers before the reflector is formed, so that the reads of
// the step overlap its reductions; NP = 0 streams the columns one pair ahead.
template <int NP>
__global__ __launch_bounds__(kTT) void tridiag_step_kernel(TridArgs t, int j, int nparts) {
  extern __shared__ double vs[];  // N + 1 entries: x, then v_j
  __shared__ double red[kTT / 64];
  __shared__ double redr[kTT / 64][kTR];
  __shared__ double s_alpha;
  const int N = t.N, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const bool corr = j >= 1;
  const double* __restrict__ yp = t.y[(j + 1) & 1];
  const double* __restrict__ pp = t.part[(j + 1) & 1];
  const double* __restrict__ vp = t.Vt + (int64_t)(corr ? j - 1 : j) * t.ld;
  const double* __restrict__ rowj = t.C + (int64_t)j * t.ld;
  const int r0 = j + 1 + kTR * blockIdx.x;
  // ---- every global load that does not depend on a reduction, issued first
  double pv_[kPP], rx[kPU], vx[kPU], yx[kPU];
#pragma unroll
  for (int u = 0; u < kPP; ++u) {
    const int q = tid + kTT * u;
    pv_[u] = (corr && q < nparts) ? pp[q] : 0.0;
  }
#pragma unroll
  for (int u = 0; u < kPU; ++u) {
    const int i = j + tid + kTT * u;
    const bool ok = i < N;
    rx[u] = ok ? rowj[i] : 0.0;
    vx[u] = (ok && corr) ? vp[i] : 0.0;
    yx[u] = (ok && corr) ? yp[i] : 0.0;
  }
  const double taup = corr ? t.tau[j - 1] : 0.0;
  const double vpj = corr ? vp[j] : 0.0, ypj = corr ? yp[j] : 0.0;
  double vr[kTR], yr_[kTR];
  double* row[kTR];
#pragma unroll
  for (int q = 0; q < kTR; ++q) {
    const int r = r0 + q;
    const bool ok = r < N;
    row[q] = t.C + (int64_t)(ok ? r : j) * t.ld;
    vr[q] = (corr && ok) ? vp[r] : 0.0;
    yr_[q] = (corr && ok) ? yp[r] : 0.0;
  }
  const int cb = (j + 1) & ~1;
  const bool rows = j < N - 1;
  // column pairs of the trailing rows (consumed after the reflector): all of
  // them for NP > 0, else the first
  int c = cb + 2 * tid;
  constexpr int NA = NP > 0 ? NP : 1;
  f64x2 a[NA][kTR], pv2[NA], py2[NA];
#pragma unroll
  for (int u = 0; u < NA; ++u) {
    const int cu = c + 2 * kTT * u;
#pragma unroll
    for (int q = 0; q < kTR; ++q)
      a[u][q] = (rows && cu < N && r0 + q < N) ? *(const f64x2*)(row[q] + cu) : f64x2{0.0, 0.0};
    pv2[u] = (rows && corr && cu < N) ? *(const f64x2*)(vp + cu) : f64x2{0.0, 0.0};
    py2[u] = (rows && corr && cu < N) ? *(const f64x2*)(yp + cu) : f64x2{0.0, 0.0};
  }
  // ---- reflector of column j
  double cw = 0.0;
  if (corr) {
    double sp = 0.0;
#pragma unroll
    for (int u = 0; u < kPP; ++u) sp += pv_[u];
    for (int q = tid + kTT * kPP; q < nparts; q += kTT) sp += pp[q];
    sp = block_sum_t(sp, red);
    cw = 0.5 * taup * sp;
  }
  const double wj = ypj - cw * vpj;
  double sig = 0.0;
  auto xval = [&](int i, double ri, double vi, double yi) {
    double x = ri;
    if (corr) x -= vi * wj + (yi - cw * vi) * vpj;
    vs[i] = x;
    if (i == j + 1) s_alpha = x;
    if (i >= j + 2) sig += x * x;
    if (i == j && blockIdx.x == 0) t.d[j] = x;
  };
#pragma unroll
  for (int u = 0; u < kPU; ++u) {
    const int i = j + tid + kTT * u;
    if (i < N) xval(i, rx[u], vx[u], yx[u]);
  }
  for (int i = j + tid + kTT * kPU; i < N; i += kTT)
    xval(i, rowj[i], corr ? vp[i] : 0.0, corr ? yp[i] : 0.0);
  if (tid == 0) vs[N] = 0.0;
  if (!rows) return;  // last column: only d
  sig = block_sum_t(sig, red);  // its barriers publish s_alpha and vs
  const double alpha = s_alpha;
  double tau = 0.0, beta = alpha, scale = 0.0;
  if (sig > 0.0) {
    // |beta| = sqrt(u) = u rsq(u), 1 / beta = -sign(alpha) rsq(u)
    const double u = fma(alpha, alpha, sig), ru = nrsq(u);
    beta = -copysign(u * ru, alpha);
    tau = (beta - alpha) * -copysign(ru, alpha);
    scale = nrcp(alpha - beta);
  }
  for (int i = j + tid; i < N; i += kTT) vs[i] = i == j ? 0.0 : (i == j + 1 ? 1.0 : vs[i] * scale);
  __syncthreads();  // v_j complete in LDS
  if (blockIdx.x == 0) {
    double* vrow = t.Vt + (int64_t)j * t.ld;
    for (int i = tid; i < N; i += kTT) vrow[i] = i < j ? 0.0 : vs[i];
    if (tid == 0) {
      t.tau[j] = tau;
      t.e[j] = beta;
    }
  }
  // ---- trailing rows r0 .. r0+kTR-1 (> j), one column pair ahead
  double wr[kTR], acc[kTR];
#pragma unroll
  for (int q = 0; q < kTR; ++q) {
    wr[q] = yr_[q] - cw * vr[q];
    acc[q] = 0.0;
  }
  // one column pair (cc, cc+1) of the trailing rows: step j-1's update, the
  // write-back, and the products with v_j.  N <= ld and ld is even, so the
  // pair with cc < N is in the row.
  auto pair = [&](int cc, f64x2 (&ar)[kTR], f64x2 pvc, f64x2 pyc) {
    const bool ok0 = cc >= j + 1, ok1 = cc + 1 < N;
    const double m0 = ok0 ? 1.0 : 0.0, m1 = ok1 ? 1.0 : 0.0;
    const double v0 = vs[cc], v1 = vs[cc + 1];
    const f64x2 pw = pyc - cw * pvc;
#pragma unroll
    for (int q = 0; q < kTR; ++q) {
      if (r0 + q >= N) continue;
      if (corr) {
        ar[q] -= vr[q] * pw + wr[q] * pvc;
        if (ok0 && ok1)
          *(f64x2*)(row[q] + cc) = ar[q];
        else if (ok1)
          row[q][cc + 1] = ar[q].y;
        else if (ok0)
          row[q][cc] = ar[q].x;
      }
      acc[q] += m0 * ar[q].x * v0 + m1 * ar[q].y * v1;
    }
  };
  if constexpr (NP > 0) {
#pragma unroll
    for (int u = 0; u < NP; ++u) {
      const int cu = c + 2 * kTT * u;
      if (cu < N) pair(cu, a[u], pv2[u], py2[u]);
    }
  } else {
    for (; c < N; c += 2 * kTT) {
      const int cn = c + 2 * kTT;
      f64x2 an[kTR], pvn = {0.0, 0.0}, pyn = {0.0, 0.0};
#pragma unroll
      for (int q = 0; q < kTR; ++q)
        an[q] = (cn < N && r0 + q < N) ? *(const f64x2*)(row[q] + cn) : f64x2{0.0, 0.0};
      if (corr && cn < N) {
        pvn = *(const f64x2*)(vp + cn);
        pyn = *(const f64x2*)(yp + cn);
      }
      pair(c, a[0], pv2[0], py2[0]);
#pragma unroll
      for (int q = 0; q < kTR; ++q) a[0][q] = an[q];
      pv2[0] = pvn;
      py2[0] = pyn;
    }
  }
#pragma unroll
  for (int q = 0; q < kTR; ++q) {
    const double sq = wave_sum(acc[q]);
    if (lane == 0) redr[wave][q] = sq;
  }
  __syncthreads();
  if (tid == 0) {
    double pz = 0.0;
    double* __restrict__ yn = t.y[j & 1];
#pragma unroll
    for (int q = 0; q < kTR; ++q) {
      const int r = r0 + q;
      if (r >= N) continue;
      double sq = 0.0;
#pragma unroll
      for (int wv = 0; wv < kTT / 64; ++wv) sq += redr[wv][q];
      const double yr = tau * sq;
      yn[r] = yr;
      pz += yr * vs[r];
    }
    t.part[j & 1][blockIdx.x] = pz;
  }
}

// ------------------------------------------------------------------ bisection
struct TriSpec {
  const double* d;
  const double* e;
  int N;
};

// Gershgorin interval, largest |entry| and the pivot floor of the Sturm
// recurrence (LAPACK dstebz conventions); every thread gets the results.
__device__ inline void tri_bounds(const TriSpec& T, double* red, double& glo, double& ghi,
                                  double& pivmin) {
  double lo = 1e308, hi = -1e308, emax = 0.0;
  for (int i = threadIdx.x; i < T.N; i += blockDim.x) {
    const double el = i > 0 ? fabs(T.e[i - 1]) : 0.0, er = i < T.N - 1 ? fabs(T.e[i]) : 0.0;
    lo = fmin(lo, T.d[i] - el - er);
    hi = fmax(hi, T.d[i] + el + er);
    emax = fmax(emax, er * er);
  }
  lo = dev::wave_min_dpp(lo);
  hi = dev::wave_max_dpp(hi);
  emax = dev::wave_max_dpp(emax);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0) {
    red[wave] = lo;
    red[16 + wave] = hi;
    red[32 + wave] = emax;
  }
  __syncthreads();
  glo = red[0];
  ghi = red[16];
  emax = red[32];
  for (int w = 1; w < nw; ++w) {
    glo = fmin(glo, red[w]);
    ghi = fmax(ghi, red[16 + w]);
    emax = fmax(emax, red[32 + w]);
  }
  pivmin = DBL_MIN * fmax(1.0, emax);
  const double tnorm = fmax(fabs(glo), fabs(ghi));
  const double fudge = 2.1 * DBL_EPSILON * tnorm * T.N + 4.2 * pivmin;
  glo -= fudge;
  ghi += fudge;
}

// Multisection for the k lowest eigenvalues, one launch per round: kBisWG
// workgroups per eigenvalue, each counting at 512 interior points of the
// current bracket (two interleaved Sturm sequences per thread, d and e^2
// staged through LDS, the recurrence's reciprocal from nrcp), so a round
// narrows the bracket 4097-fold.  Workgroup (m, w) reads the candidates that
// the previous round's workgroups of eigenvalue m left in cand_in (their
// largest point with count <= m and smallest above), and writes its own.
constexpr int kBisWG = 8;
constexpr int kBisRounds = 6;   // 6 x 12 bits cover the 53-bit mantissa
constexpr int kBisChunk = 1024;

struct BisArgs {
  TriSpec T;
  const double* bounds;  // glo, ghi, pivmin
  const double* cand_in;   // [k][kBisWG][2]
  double* cand_out;
  int first;             // 1: start from the Gershgorin interval
};

__global__ __launch_bounds__(256) void bisect_bounds_kernel(TriSpec T, double* __restrict__ bounds) {
  __shared__ double red[48];
  double glo, ghi, pivmin;
  tri_bounds(T, red, glo, ghi, pivmin);
  if (threadIdx.x == 0) {
    bounds[0] = glo;
    bounds[1] = ghi;
    bounds[2] = pivmin;
  }
}

__global__ __launch_bounds__(256) void bisect_round_kernel(BisArgs a) {
  __shared__ double rlo[4], rhi[4];
  __shared__ double sd[kBisChunk], se2[kBisChunk];
  const int m = blockIdx.x / kBisWG, w = blockIdx.x % kBisWG, tid = threadIdx.x;
  const int lane = tid & 63, wave = tid >> 6, N = a.T.N;
  const double pivmin = a.bounds[2];
  double lo, hi;
  if (a.first) {
    lo = a.bounds[0];
    hi = a.bounds[1];
  } else {
    const double* c = a.cand_in + (int64_t)m * kBisWG * 2;
    lo = c[0];
    hi = c[1];
    for (int q = 1; q < kBisWG; ++q) {
      lo = fmax(lo, c[2 * q]);
      hi = fmin(hi, c[2 * q + 1]);
    }
    if (hi < lo) hi = lo;
  }
  double* out = a.cand_out + ((int64_t)m * kBisWG + w) * 2;
  const double tol = 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)) + pivmin;
  if (hi - lo <= tol) {  // converged: pass the bracket on (uniform per workgroup)
    if (tid == 0) {
      out[0] = lo;
      out[1] = hi;
    }
    return;
  }
  constexpr double kPts = 2.0 * 256 * kBisWG + 1.0;
  const int p0 = 2 * (w * 256 + tid);
  const double x0 = lo + (hi - lo) * ((double)(p0 + 1) / kPts);
  const double x1 = lo + (hi - lo) * ((double)(p0 + 2) / kPts);
  int c0 = 0, c1 = 0;
  double q0 = a.T.d[0] - x0, q1 = a.T.d[0] - x1;
  if (fabs(q0) < pivmin) q0 = -pivmin;
  if (fabs(q1) < pivmin) q1 = -pivmin;
  c0 += q0 < 0.0;
  c1 += q1 < 0.0;
  for (int base = 1; base < N; base += kBisChunk) {
    const int len = min(kBisChunk, N - base);
    __syncthreads();
    for (int u = tid; u < len; u += 256) {
      sd[u] = a.T.d[base + u];
      const double e = a.T.e[base + u - 1];
      se2[u] = e * e;
    }
    __syncthreads();
    for (int u = 0; u < len; ++u) {
      const double du = sd[u], eu = se2[u];
      q0 = (du - x0) - eu * nrcp(q0);
      q1 = (du - x1) - eu * nrcp(q1);
      if (fabs(q0) < pivmin) q0 = -pivmin;
      if (fabs(q1) < pivmin) q1 = -pivmin;
      c0 += q0 < 0.0;
      c1 += q1 < 0.0;
    }
  }
  double nlo = c1 <= m ? x1 : (c0 <= m ? x0 : lo);
  double nhi = c0 > m ? x0 : (c1 > m ? x1 : hi);
  nlo = dev::wave_max_dpp(nlo);
  nhi = dev::wave_min_dpp(nhi);
  if (lane == 0) {
    rlo[wave] = nlo;
    rhi[wave] = nhi;
  }
  __syncthreads();
  if (tid == 0) {
    double blo = fmax(fmax(rlo[0], rlo[1]), fmax(rlo[2], rlo[3]));
    double bhi = fmin(fmin(rhi[0], rhi[1]), fmin(rhi[2], rhi[3]));
    out[0] = blo;
    out[1] = bhi;
  }
}

__global__ __launch_bounds__(64) void bisect_final_kernel(const double* __restrict__ cand, int k,
                                                          double* __restrict__ evals) {
  const int m = blockIdx.x * 64 + threadIdx.x;
  if (m >= k) return;
  const double* c = cand + (int64_t)m * kBisWG * 2;
  double lo = c[0], hi = c[1];
  for (int q = 1; q < kBisWG; ++q) {
    lo = fmax(lo, c[2 * q]);
    hi = fmin(hi, c[2 * q + 1]);
  }
  if (hi < lo) hi = lo;
  evals[m] = 0.5 * (lo + hi);
}

// ------------------------------------------------------------------ inverse iteration
struct InvArgs {
  TriSpec T;
  const double* evals;
  double* f;     // [5][N][k]: 1/u0, u1, u2, multiplier, swap flag
  double* X;     // [N][k] eigenvectors of T (column m)
  int k;
};

__device__ inline uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

// One thread per eigenvalue: (T - lambda I) = P L U with partial pivoting,
// tiny pivots of U replaced by eps ||T|| (sign kept), three solves from a
// pseudo-random start (SplitMix64 of (m, i), uniform in [-1, 1)), each
// right-hand side scaled by the previous solve's max-norm, then 2-norm
// normalisation.  The sequential passes run over chunks of kIC rows whose
// loads are issued together; arrays are [i][k] so a wave's accesses are
// contiguous.
constexpr int kIC = 8;

__global__ __launch_bounds__(64) void inverse_iter_kernel(InvArgs a) {
  // ||T|| from the Gershgorin interval, by this wave alone
  double lo = 1e308, hi = -1e308;
  const int N = a.T.N, k = a.k;
  for (int i = threadIdx.x; i < N; i += 64) {
    const double el = i > 0 ? fabs(a.T.e[i - 1]) : 0.0, er = i < N - 1 ? fabs(a.T.e[i]) : 0.0;
    lo = fmin(lo, a.T.d[i] - el - er);
    hi = fmax(hi, a.T.d[i] + el + er);
  }
  lo = dev::wave_min_dpp(lo);
  hi = dev::wave_max_dpp(hi);
  const double tnorm = fmax(fabs(lo), fabs(hi));
  const double pert = fmax(DBL_EPSILON * tnorm, DBL_MIN);
  const int m = blockIdx.x * 64 + threadIdx.x;
  if (m >= k) return;
  const double lam = a.evals[m];
  const int64_t P = (int64_t)N * k;
  double* __restrict__ RU0 = a.f;
  double* __restrict__ U1 = a.f + P;
  double* __restrict__ U2 = a.f + 2 * P;
  double* __restrict__ LM = a.f + 3 * P;
  double* __restrict__ SW = a.f + 4 * P;
  double* __restrict__ X = a.X;
  const double* __restrict__ D = a.T.d;
  const double* __restrict__ E = a.T.e;
  // factorisation, rows i = 0 .. N-2 in chunks, then the last row
  double p = D[0] - lam, q = N > 1 ? E[0] : 0.0;
  for (int i0 = 0; i0 < N - 1; i0 += kIC) {
    double dn[kIC], sub[kIC], en[kIC];
#pragma unroll
    for (int u = 0; u < kIC; ++u) {
      const int i = i0 + u;
      sub[u] = i < N - 1 ? E[i] : 0.0;
      dn[u] = i < N - 1 ? D[i + 1] - lam : 0.0;
      en[u] = i + 2 < N ? E[i + 1] : 0.0;
    }
#pragma unroll
    for (int u = 0; u < kIC; ++u) {
      const int i = i0 + u;
      if (i >= N - 1) break;
      double u0, u1, u2, l, sw;
      if (fabs(p) >= fabs(sub[u])) {
        l = p != 0.0 ? sub[u] / p : 0.0;
        u0 = p;
        u1 = q;
        u2 = 0.0;
        p = dn[u] - l * q;
        q = en[u];
        sw = 0.0;
      } else {
        l = p / sub[u];
        u0 = sub[u];
        u1 = dn[u];
        u2 = en[u];
        p = q - l * dn[u];
        q = -l * en[u];
        sw = 1.0;
      }
      if (fabs(u0) < pert) u0 = u0 < 0.0 ? -pert : pert;
      const int64_t o = (int64_t)i * k + m;
      RU0[o] = 1.0 / u0;
      U1[o] = u1;
      U2[o] = u2;
      LM[o] = l;
      SW[o] = sw;
    }
  }
  {
    const int64_t o = (int64_t)(N - 1) * k + m;
    double u0 = p;
    if (fabs(u0) < pert) u0 = u0 < 0.0 ? -pert : pert;
    RU0[o] = 1.0 / u0;
    U1[o] = 0.0;
    U2[o] = 0.0;
    LM[o] = 0.0;
    SW[o] = 0.0;
  }
  double scale = 1.0, ssq = 0.0;
  for (int it = 0; it < 3; ++it) {
    // forward elimination of the right-hand side (it = 0: the start vector)
    auto rhs = [&](int i) -> double {
      if (it == 0) {
        const uint64_t r = splitmix64(((uint64_t)m << 32) ^ (uint64_t)i);
        return (double)(r >> 11) * (2.0 / 9007199254740992.0) - 1.0;
      }
      return X[(int64_t)i * k + m] * scale;
    };
    double bi = rhs(0);
    for (int i0 = 0; i0 < N - 1; i0 += kIC) {
      double bn[kIC], l[kIC], sw[kIC];
#pragma unroll
      for (int u = 0; u < kIC; ++u) {
        const int i = i0 + u;
        const bool ok = i < N - 1;
        const int64_t o = (int64_t)i * k + m;
        bn[u] = ok ? rhs(i + 1) : 0.0;
        l[u] = ok ? LM[o] : 0.0;
        sw[u] = ok ? SW[o] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kIC; ++u) {
        const int i = i0 + u;
        if (i >= N - 1) break;
        double out;
        if (sw[u] != 0.0) {
          out = bn[u];
          bi = bi - l[u] * bn[u];
        } else {
          out = bi;
          bi = bn[u] - l[u] * bi;
        }
        X[(int64_t)i * k + m] = out;
      }
    }
    X[(int64_t)(N - 1) * k + m] = bi;
    // back substitution from the last row, chunks of kIC rows downwards
    double x1 = 0.0, x2 = 0.0, xmax = 0.0;
    ssq = 0.0;
    for (int i1 = N - 1; i1 >= 0; i1 -= kIC) {
      double b[kIC], r0[kIC], c1[kIC], c2[kIC];
#pragma unroll
      for (int u = 0; u < kIC; ++u) {
        const int i = i1 - u;
        const bool ok = i >= 0;
        const int64_t o = (int64_t)i * k + m;
        b[u] = ok ? X[o] : 0.0;
        r0[u] = ok ? RU0[o] : 0.0;
        c1[u] = ok ? U1[o] : 0.0;
        c2[u] = ok ? U2[o] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kIC; ++u) {
        const int i = i1 - u;
        if (i < 0) break;
        const double xi = (b[u] - c1[u] * x1 - c2[u] * x2) * r0[u];
        X[(int64_t)i * k + m] = xi;
        xmax = fmax(xmax, fabs(xi));
        ssq += xi * xi;
        x2 = x1;
        x1 = xi;
      }
    }
    scale = xmax > 0.0 ? 1.0 / xmax : 1.0;
  }
  const double sn = ssq > 0.0 ? 1.0 / sqrt(ssq) : 1.0;
  for (int i = 0; i < N; ++i) X[(int64_t)i * k + m] *= sn;
}

// The same iteration with one workgroup per eigenvalue and everything in
// LDS: d and e staged once, the factors (1/u0, u1, multiplier, swap flag;
// u2 is e[i+1] on swapped rows, else 0) and the iterate.  One lane runs the
// recurrences, reading LDS in chunks of kIC; the wave writes the result.
// LDS: 6 N doubles + N bytes.
__global__ __launch_bounds__(64) void inverse_iter_lds_kernel(InvArgs a) {
  extern __shared__ double lds[];
  __shared__ double s_ssq;
  const int N = a.T.N, k = a.k, m = blockIdx.x, lane = threadIdx.x;
  double* D = lds;
  double* E = lds + N;            // E[i] = e[i] (i < N-1), E[N-1] = 0
  double* RU0 = lds + 2 * N;
  double* U1 = lds + 3 * N;
  double* LM = lds + 4 * N;
  double* X = lds + 5 * N;
  unsigned char* SW = (unsigned char*)(lds + 6 * N);
  double lo = 1e308, hi = -1e308;
  for (int i = lane; i < N; i += 64) {
    const double di = a.T.d[i], ei = i < N - 1 ? a.T.e[i] : 0.0;
    const double el = i > 0 ? fabs(a.T.e[i - 1]) : 0.0;
    D[i] = di;
    E[i] = ei;
    lo = fmin(lo, di - el - fabs(ei));
    hi = fmax(hi, di + el + fabs(ei));
    const uint64_t r = splitmix64(((uint64_t)m << 32) ^ (uint64_t)i);
    X[i] = (double)(r >> 11) * (2.0 / 9007199254740992.0) - 1.0;
  }
  lo = dev::wave_min_dpp(lo);
  hi = dev::wave_max_dpp(hi);
  const double tnorm = fmax(fabs(lo), fabs(hi));
  const double pert = fmax(DBL_EPSILON * tnorm, DBL_MIN);
  __syncthreads();
  double ssq = 0.0;
  if (lane == 0) {
    const double lam = a.evals[m];
    double p = D[0] - lam, q = E[0];
    for (int i0 = 0; i0 < N - 1; i0 += kIC) {
      double dn[kIC], sub[kIC], en[kIC];
#pragma unroll
      for (int u = 0; u < kIC; ++u) {
        const int i = min(i0 + u, N - 2);
        sub[u] = E[i];
        dn[u] = D[i + 1] - lam;
        en[u] = E[i + 1];
      }
#pragma unroll
      for (int u = 0; u < kIC; ++u) {
        const int i = i0 + u;
        if (i >= N - 1) break;
        double u0, rcp, l;
        if (fabs(p) >= fabs(sub[u])) {
          u0 = fabs(p) < pert ? (p < 0.0 ? -pert : pert) : p;
          rcp = 1.0 / u0;
          l = p != 0.0 ? sub[u] * rcp : 0.0;
          U1[i] = q;
          SW[i] = 0;
          p = dn[u] - l * q;
          q = en[u];
        } else {
          const double rs = 1.0 / sub[u];  // |sub| > |p| >= 0
          l = p * rs;
          u0 = fabs(sub[u]) < pert ? (sub[u] < 0.0 ? -pert : pert) : sub[u];
          rcp = u0 == sub[u] ? rs : 1.0 / u0;
          U1[i] = dn[u];
          SW[i] = 1;
          p = q - l * dn[u];
          q = -l * en[u];
        }
        RU0[i] = rcp;
        LM[i] = l;
      }
    }
    {
      const double u0 = fabs(p) < pert ? (p < 0.0 ? -pert : pert) : p;
      RU0[N - 1] = 1.0 / u0;
      U1[N - 1] = 0.0;
      LM[N - 1] = 0.0;
      SW[N - 1] = 0;
    }
    double scale = 1.0;
    for (int it = 0; it < 3; ++it) {
      double bi = X[0] * scale;
      for (int i0 = 0; i0 < N - 1; i0 += kIC) {
        double bn[kIC], l[kIC];
        unsigned char sw[kIC];
#pragma unroll
        for (int u = 0; u < kIC; ++u) {
          const int i = min(i0 + u, N - 2);
          bn[u] = X[i + 1] * scale;
          l[u] = LM[i];
          sw[u] = SW[i];
        }
#pragma unroll
        for (int u = 0; u < kIC; ++u) {
          const int i = i0 + u;
          if (i >= N - 1) break;
          double out;
          if (sw[u]) {
            out = bn[u];
            bi = bi - l[u] * bn[u];
          } else {
            out = bi;
            bi = bn[u] - l[u] * bi;
          }
          X[i] = out;
        }
      }
      X[N - 1] = bi;
      double x1 = 0.0, x2 = 0.0, xmax = 0.0;
      ssq = 0.0;
      for (int i1 = N - 1; i1 >= 0; i1 -= kIC) {
        double b[kIC], r0[kIC], c1[kIC], c2[kIC];
#pragma unroll
        for (int u = 0; u < kIC; ++u) {
          const int i = max(i1 - u, 0);
          b[u] = X[i];
          r0[u] = RU0[i];
          c1[u] = U1[i];
          c2[u] = SW[i] ? E[i + 1 < N ? i + 1 : N - 1] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kIC; ++u) {
          const int i = i1 - u;
          if (i < 0) break;
          const double xi = (b[u] - c1[u] * x1 - c2[u] * x2) * r0[u];
          X[i] = xi;
          xmax = fmax(xmax, fabs(xi));
          ssq += xi * xi;
          x2 = x1;
          x1 = xi;
        }
      }
      scale = xmax > 0.0 ? 1.0 / xmax : 1.0;
    }
    s_ssq = ssq;
  }
  __syncthreads();
  const double ss = s_ssq;
  const double sn = ss > 0.0 ? 1.0 / sqrt(ss) : 1.0;
  for (int i = lane; i < N; i += 64) a.X[(int64_t)i * k + m] = X[i] * sn;
}

// ------------------------------------------------------------------ Cholesky-QR
// Partial Gram matrices of 256-row chunks of X [N][k] (4 LDS stages of 64).
constexpr int kGramRows = 256;

__global__ __launch_bounds__(256) void gram_partial_kernel(const double* __restrict__ X, int N,
                                                           int k, double* __restrict__ part) {
  __shared__ double xs[64][kMaxK + 1];
  const int tid = threadIdx.x;
  double acc[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) acc[q] = 0.0;
  for (int st = 0; st < kGramRows / 64; ++st) {
    const int i0 = blockIdx.x * kGramRows + st * 64;
    __syncthreads();
    for (int e = tid; e < 64 * kMaxK; e += 256) {
      const int r = e >> 6, c = e & 63;
      xs[r][c] = (i0 + r < N && c < k) ? X[(int64_t)(i0 + r) * k + c] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int e = tid + 256 * q, pp = e >> 6, qq = e & 63;
      double s = 0.0;
      for (int r = 0; r < 64; ++r) s += xs[r][pp] * xs[r][qq];
      acc[q] += s;
    }
  }
  double* out = part + (int64_t)blockIdx.x * k * k;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int e = tid + 256 * q, pp = e >> 6, qq = e & 63;
    if (pp < k && qq < k) out[pp * k + qq] = acc[q];
  }
}

// G = sum of the partials (padded to 64 x 64 with the identity) = L L^T;
// writes R^-1 = L^-T (upper, k x k), R = L^T.  A pivot not above 1/4 means
// the vectors were not independent: info = -2.
__global__ __launch_bounds__(256) void chol_small_kernel(const double* __restrict__ part,
                                                         int nparts, int k,
                                                         double* __restrict__ Rinv, int* info) {
  __shared__ CholWaveLds sh;
  // the sum of the partials, by all four waves, goes through LDS (by
  // columns); wave 0 alone then loads its register rows, outside any loop
  const int kk = k * k;
  for (int e = threadIdx.x; e < kk; e += 256) {
    double v0 = 0.0, v1 = 0.0, v2 = 0.0, v3 = 0.0;
    int b = 0;
    for (; b + 3 < nparts; b += 4) {
      v0 += part[(int64_t)b * kk + e];
      v1 += part[(int64_t)(b + 1) * kk + e];
      v2 += part[(int64_t)(b + 2) * kk + e];
      v3 += part[(int64_t)(b + 3) * kk + e];
    }
    for (; b < nparts; ++b) v0 += part[(int64_t)b * kk + e];
    sh.lt[(e % k) * kLw + e / k] = (v0 + v1) + (v2 + v3);
  }
  __syncthreads();
  if (threadIdx.x >= 64) return;
  const int r = threadIdx.x;
  double a[kNB], x[kNB];
  // rows and columns beyond k are the identity's
#pragma unroll
  for (int c = 0; c < kNB; ++c)
    a[c] = (r < k && c < k) ? (c <= r ? sh.lt[c * kLw + r] : 0.0) : (c == r ? 1.0 : 0.0);
  const int fail = chol_inv_64_wave(a, x, 0.25, sh);
  // lane r holds column r of L^-1, i.e. row r of R^-1 = L^-T; it goes out
  // through LDS so that the stores carry no per-element guard (guarded, the
  // compiler sinks the whole solve into the guarded blocks)
#pragma unroll
  for (int i = 0; i < kNB; ++i) sh.lt[i * kLw + r] = x[i];
  for (int e = r; e < kk; e += 64) Rinv[e] = sh.lt[(e % k) * kLw + e / k];
  if (r == 0 && fail != 0) {
    if (*info == 0) *info = -2;
  }
}

// X <- X R^-1, four rows per workgroup.
__global__ __launch_bounds__(256) void apply_rinv_kernel(double* __restrict__ X, int N, int k,
                                                         const double* __restrict__ Rinv) {
  __shared__ double xs[4][kMaxK];
  const int r = blockIdx.x * 4 + (threadIdx.x >> 6), c = threadIdx.x & 63;
  const bool ok = r < N && c < k;
  if (ok) xs[threadIdx.x >> 6][c] = X[(int64_t)r * k + c];
  __syncthreads();
  if (!ok) return;
  double s = 0.0;
  for (int p = 0; p <= c; ++p) s += xs[threadIdx.x >> 6][p] * Rinv[p * k + c];
  X[(int64_t)r * k + c] = s;
}

// ------------------------------------------------------------------ back-transformation
// Compact-WY triangular factor of reflectors j0 .. j0+nb-1 (forward,
// columnwise): T[c][c] = tau_c, T[0:c][c] = -tau_c T[0:c][0:c] (V^T v_c)[0:c].
__global__ __launch_bounds__(256) void larft_kernel(const double* __restrict__ Vt, int64_t ld,
                                                    const double* __restrict__ tau, int N,
                                                    int nrefl, double* __restrict__ Tout) {
  __shared__ double vs[kWY][65];
  __shared__ double gv[kWY][kWY + 1];
  __shared__ double T[kWY][kWY + 1];
  const int b = blockIdx.x, j0 = b * kWY, nb = min(kWY, nrefl - j0), tid = threadIdx.x;
  double acc[4] = {0.0, 0.0, 0.0, 0.0};  // entries tid + 256 q of the 32 x 32 Gram matrix
  for (int c0 = j0 + 1; c0 < N; c0 += 64) {
    __syncthreads();
    for (int e = tid; e < kWY * 64; e += 256) {
      const int r = e / 64, c = e % 64;
      vs[r][c] = (r < nb && c0 + c < N) ? Vt[(int64_t)(j0 + r) * ld + c0 + c] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = tid + 256 * q, p = e / kWY, s = e % kWY;
      double t = 0.0;
      for (int c = 0; c < 64; ++c) t += vs[p][c] * vs[s][c];
      acc[q] += t;
    }
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int e = tid + 256 * q;
    gv[e / kWY][e % kWY] = acc[q];
  }
  for (int e = tid; e < kWY * kWY; e += 256) T[e / kWY][e % kWY] = 0.0;
  __syncthreads();
  // column c needs columns < c: one column per step, its rows in parallel
  for (int c = 0; c < nb; ++c) {
    const double tc = tau[j0 + c];
    if (tid < c) {
      double s = 0.0;
      for (int q = tid; q < c; ++q) s += T[tid][q] * gv[q][c];
      T[tid][c] = -tc * s;
    }
    if (tid == c) T[c][c] = tc;
    __syncthreads();
  }
  for (int e = tid; e < kWY * kWY; e += 256) Tout[(int64_t)b * kWY * kWY + e] = T[e / kWY][e % kWY];
}

// One 1024-thread workgroup per eigenvector: z = Q x with Q = H_0 H_1 ...
// (blocks applied last first), z in LDS; output row m of Z [k][N].  In the
// first pass of a block, wave w forms the dot products of reflectors w and
// w + 16 with z (two wave reductions per wave); the second pass updates z
// elementwise.
constexpr int kBT = 1024;
static_assert(kWY == 2 * (kBT / 64), "two reflectors per wave in the dot-product pass");

__global__ __launch_bounds__(kBT) void backtransform_kernel(const double* __restrict__ X, int k,
                                                            const double* __restrict__ Vt,
                                                            int64_t ld,
                                                            const double* __restrict__ Tf,
                                                            int N, int nrefl, int nblocks,
                                                            double* __restrict__ Z) {
  extern __shared__ double z[];
  __shared__ double vz[kWY];
  __shared__ double pp[kWY];
  const int m = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int i = tid; i < N; i += kBT) z[i] = X[(int64_t)i * k + m];
  __syncthreads();
  for (int b = nblocks - 1; b >= 0; --b) {
    const int j0 = b * kWY, nb = min(kWY, nrefl - j0);
    const double* V = Vt + (int64_t)j0 * ld;
    {
      const int c0 = wave, c1 = wave + kBT / 64;
      const double* v0 = V + (int64_t)c0 * ld;
      const double* v1 = V + (int64_t)c1 * ld;
      double a0 = 0.0, a1 = 0.0;
      // reflector j0 + c is zero up to index j0 + c
      for (int i = j0 + 1 + lane; i < N; i += 64) {
        const double zi = z[i];
        if (c0 < nb) a0 += v0[i] * zi;
        if (c1 < nb) a1 += v1[i] * zi;
      }
      a0 = wave_sum(a0);
      a1 = wave_sum(a1);
      if (lane == 0) {
        vz[c0] = a0;
        vz[c1] = a1;
      }
    }
    __syncthreads();
    if (tid < kWY) {
      const double* T = Tf + (int64_t)b * kWY * kWY + tid * kWY;
      double s = 0.0;
      for (int c = tid; c < kWY; ++c) s += T[c] * vz[c];
      pp[tid] = s;
    }
    __syncthreads();
    for (int i = j0 + 1 + tid; i < N; i += kBT) {
      double s = 0.0;
#pragma unroll
      for (int c = 0; c < kWY; ++c)
        if (c < nb) s += V[(int64_t)c * ld + i] * pp[c];
      z[i] -= s;
    }
    __syncthreads();
  }
  for (int i = tid; i < N; i += kBT) Z[(int64_t)m * N + i] = z[i];
}

// ------------------------------------------------------------------ plan
struct DensePlan {
  int N, Np, k, nrefl, nwy, nchunks;
  size_t off_L, off_Linv, off_C, off_W, off_vec, off_bis, off_f, off_X, off_part, off_R, off_T,
      off_Z, bytes;
};

DensePlan plan_dense(int N, int k) {
  DensePlan p;
  p.N = N;
  p.k = k;
  p.Np = (int)ceil_div(N, kNB) * kNB;
  p.nrefl = std::max(N - 2, 0);
  p.nwy = (int)ceil_div(p.nrefl, kWY);
  p.nchunks = (int)ceil_div(N, kGramRows);
  const size_t np2 = sizeof(double) * (size_t)p.Np * p.Np;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t at = o;
    o = align_up(o + bytes, 256);
    return at;
  };
  p.off_L = take(np2);
  p.off_Linv = take(np2);
  p.off_C = take(np2);
  p.off_W = take(np2);
  p.off_vec = take(sizeof(double) * 7 * (size_t)p.Np);
  p.off_bis = take(sizeof(double) * (4 + 4 * kBisWG * (size_t)k));
  p.off_f = take(sizeof(double) * 5 * (size_t)N * k);
  p.off_X = take(sizeof(double) * (size_t)N * k);
  p.off_part = take(sizeof(double) * (size_t)p.nchunks * k * k);
  p.off_R = take(sizeof(double) * (size_t)k * k);
  p.off_T = take(sizeof(double) * (size_t)std::max(p.nwy, 1) * kWY * kWY);
  p.off_Z = take(sizeof(double) * (size_t)k * N);
  p.bytes = o;
  return p;
}

// Optional HIP events recorded at the stage boundaries of the next calls of
// this thread (profiling hook): 0 before the Cholesky factorisation, 1 after
// L and L^-1, 2 after C = L^-1 H L^-T, 3 after the tridiagonalisation, 4
// after the eigenvalues, 5 after the eigenvectors.
constexpr int kStages = 6;
thread_local hipEvent_t g_stage[kStages] = {};

tl_status stage_mark(int i, hipStream_t stream) {
  if (g_stage[i] != nullptr) TL_HIP(hipEventRecord(g_stage[i], stream));
  return TL_OK;
}

tl_status check_dense(int N, int k) {
  TL_REQUIRE(N >= 1 && N <= kMaxN, "dense eigensolver: N = %d outside [1, %d]", N, kMaxN);
  TL_REQUIRE(k >= 1 && k <= N && k <= kMaxK, "dense eigensolver: k = %d outside [1, min(N, %d)]",
             k, kMaxK);
  return TL_OK;
}

}  // namespace

tl_status dense_gen_eigh_lowest(const double* H, const double* S, int N, int k, double* evals,
                                double* evecs, int* info, void* ws, size_t ws_bytes,
                                hipStream_t stream) {
  TL_TRY(check_dense(N, k));
  TL_REQUIRE(H && S && evals && info, "null argument");
  const DensePlan p = plan_dense(N, k);
  if (ws == nullptr || ws_bytes < p.bytes) {
    set_error("dense eigensolver workspace: need %zu bytes, got %zu", p.bytes, ws_bytes);
    return TL_EWORKSPACE;
  }
  char* base = (char*)ws;
  double* L = (double*)(base + p.off_L);
  double* Linv = (double*)(base + p.off_Linv);
  double* C = (double*)(base + p.off_C);
  double* W = (double*)(base + p.off_W);
  double* vec = (double*)(base + p.off_vec);
  const int Np = p.Np;
  const int64_t ld = Np;

  // 1. Cholesky
  TL_TRY(stage_mark(0, stream));
  hipLaunchKernelGGL(setup_kernel, dim3((unsigned)ceil_div((int64_t)Np * Np, 256)), dim3(256), 0,
                     stream, S, N, Np, L, Linv, info);
  TL_CHECK_LAUNCH();
  for (int q = 0; q < Np; q += kNB) {
    hipLaunchKernelGGL(potrf_diag_kernel, dim3(1), dim3(64), 0, stream, L, Linv, ld, q, info);
    TL_CHECK_LAUNCH();
    const int rest = Np - q - kNB;
    if (rest <= 0) continue;
    double* A21 = L + (int64_t)(q + kNB) * ld + q;
    // L21 = A21 L11^-T (single column tile: in place is safe)
    TL_TRY(gemm(gemm_args(A21, ld, Linv + (int64_t)q * ld + q, ld, A21, ld, rest, kNB, kNB, 1.0,
                          0.0, 3),
                true, 1, stream));
    // A22 -= L21 L21^T, lower triangle only
    GemmArgs g = gemm_args(A21, ld, A21, ld, L + (int64_t)(q + kNB) * (ld + 1), ld, rest, rest,
                           kNB, -1.0, 1.0, 0);
    g.lower = 1;
    TL_TRY(gemm(g, true, 1, stream));
  }
  // 2. L^-1 by doubling: blocks (o, o+s) for o = 0, 2s, ...
  for (int s = kNB; s < Np; s *= 2) {
    // full pairs have a second block of size s; a ragged last pair follows
    int nfull = 0;
    for (int o = 0; o + s < Np; o += 2 * s)
      if (Np - o - s >= s) ++nfull;
    auto level = [&](int o, int s2, int batch) -> tl_status {
      // T1 = L[o+s:o+s+s2, o:o+s] * Linv[o:o+s, o:o+s]
      GemmArgs g1 = gemm_args(L + (int64_t)(o + s) * ld + o, ld, Linv + (int64_t)o * ld + o, ld, W,
                              s, s2, s, s, 1.0, 0.0, 2);
      g1.sA = g1.sB = (int64_t)2 * s * (ld + 1);
      g1.sC = (int64_t)s * s;
      TL_TRY(gemm(g1, false, batch, stream));
      // Linv[o+s:, o:o+s] = -Linv[o+s:, o+s:] * T1
      GemmArgs g2 = gemm_args(Linv + (int64_t)(o + s) * ld + o + s, ld, W, s,
                              Linv + (int64_t)(o + s) * ld + o, ld, s2, s, s2, -1.0, 0.0, 1);
      g2.sA = g2.sC = (int64_t)2 * s * (ld + 1);
      g2.sB = (int64_t)s * s;
      return gemm(g2, false, batch, stream);
    };
    if (nfull > 0) TL_TRY(level(0, s, nfull));
    const int o_last = nfull * 2 * s;
    if (o_last + s < Np) TL_TRY(level(o_last, Np - o_last - s, 1));
  }
  TL_TRY(stage_mark(1, stream));
  // 3. C = Linv H Linv^T (N x N, row stride ld)
  TL_TRY(gemm(gemm_args(Linv, ld, H, N, W, ld, N, N, N, 1.0, 0.0, 1), false, 1, stream));
  {
    GemmArgs g = gemm_args(W, ld, Linv, ld, C, ld, N, N, N, 1.0, 0.0, 3);
    g.lower = 1;
    g.mirror = 1;
    TL_TRY(gemm(g, true, 1, stream));
  }
  TL_TRY(stage_mark(2, stream));
  // 4. tridiagonalisation; reflectors reuse W
  TridArgs t;
  t.C = C;
  t.Vt = W;
  t.y[0] = vec;
  t.y[1] = vec + Np;
  t.part[0] = vec + 2 * Np;
  t.part[1] = vec + 3 * Np;
  t.d = vec + 4 * Np;
  t.e = vec + 5 * Np;
  t.tau = vec + 6 * Np;
  t.ld = ld;
  t.N = N;
  {
    int nparts = 0;
    const size_t lds = sizeof(double) * ((size_t)N + 1);
    for (int j = 0; j < N; ++j) {
      const int grid = std::max(1, (int)ceil_div(N - j - 1, kTR));
      // column pairs per thread for the trailing columns cb .. N-1
      const int np = (int)ceil_div(N - ((j + 1) & ~1), 2 * kTT);
      const dim3 gd((unsigned)grid), bd(kTT);
      switch (np) {
        case 0:
        case 1: hipLaunchKernelGGL(tridiag_step_kernel<1>, gd, bd, lds, stream, t, j, nparts); break;
        case 2: hipLaunchKernelGGL(tridiag_step_kernel<2>, gd, bd, lds, stream, t, j, nparts); break;
        case 3: hipLaunchKernelGGL(tridiag_step_kernel<3>, gd, bd, lds, stream, t, j, nparts); break;
        case 4: hipLaunchKernelGGL(tridiag_step_kernel<4>, gd, bd, lds, stream, t, j, nparts); break;
        default:
          hipLaunchKernelGGL(tridiag_step_kernel<0>, gd, bd, lds, stream, t, j, nparts);
      }
      TL_CHECK_LAUNCH();
      nparts = grid;
    }
  }
  TL_TRY(stage_mark(3, stream));
  // 5. eigenvalues
  TriSpec T{t.d, t.e, N};
  {
    double* bounds = (double*)(base + p.off_bis);
    double* cand[2] = {bounds + 4, bounds + 4 + 2 * kBisWG * (size_t)k};
    hipLaunchKernelGGL(bisect_bounds_kernel, dim3(1), dim3(256), 0, stream, T, bounds);
    TL_CHECK_LAUNCH();
    for (int r = 0; r < kBisRounds; ++r) {
      BisArgs ba{T, bounds, cand[r & 1], cand[(r + 1) & 1], r == 0};
      hipLaunchKernelGGL(bisect_round_kernel, dim3((unsigned)(k * kBisWG)), dim3(256), 0, stream,
                         ba);
      TL_CHECK_LAUNCH();
    }
    hipLaunchKernelGGL(bisect_final_kernel, dim3((unsigned)ceil_div(k, 64)), dim3(64), 0, stream,
                       cand[kBisRounds & 1], k, evals);
    TL_CHECK_LAUNCH();
  }
  TL_TRY(stage_mark(4, stream));
  if (evecs == nullptr) return stage_mark(5, stream);
  // 6. eigenvectors of T
  double* F = (double*)(base + p.off_f);
  double* X = (double*)(base + p.off_X);
  InvArgs ia{T, evals, F, X, k};
  {
    // per-eigenvalue LDS variant when 6 N doubles + N bytes fit in one
    // workgroup's LDS, else the global-memory variant
    const size_t lds = sizeof(double) * 6 * (size_t)N + (size_t)N;
    int dev = 0, max_lds = 0;
    TL_HIP(hipGetDevice(&dev));
    TL_HIP(hipDeviceGetAttribute(&max_lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
    bool use_lds = lds + 64 <= (size_t)max_lds;
    if (use_lds && lds > 65536)
      use_lds = hipFuncSetAttribute((const void*)inverse_iter_lds_kernel,
                                    hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)lds) == hipSuccess;
    (void)hipGetLastError();
    if (use_lds)
      hipLaunchKernelGGL(inverse_iter_lds_kernel, dim3((unsigned)k), dim3(64), lds, stream, ia);
    else
      hipLaunchKernelGGL(inverse_iter_kernel, dim3((unsigned)ceil_div(k, 64)), dim3(64), 0,
                         stream, ia);
    TL_CHECK_LAUNCH();
  }
  double* part = (double*)(base + p.off_part);
  double* R = (double*)(base + p.off_R);
  for (int pass = 0; pass < 2; ++pass) {
    hipLaunchKernelGGL(gram_partial_kernel, dim3((unsigned)p.nchunks), dim3(256), 0, stream, X, N,
                       k, part);
    TL_CHECK_LAUNCH();
    hipLaunchKernelGGL(chol_small_kernel, dim3(1), dim3(256), 0, stream, part, p.nchunks, k, R,
                       info);
    TL_CHECK_LAUNCH();
    hipLaunchKernelGGL(apply_rinv_kernel, dim3((unsigned)ceil_div(N, 4)), dim3(256), 0, stream, X,
                       N, k, R);
    TL_CHECK_LAUNCH();
  }
  // 7. back-transformation
  double* Tf = (double*)(base + p.off_T);
  double* Z = (double*)(base + p.off_Z);
  if (p.nwy > 0) {
    hipLaunchKernelGGL(larft_kernel, dim3((unsigned)p.nwy), dim3(256), 0, stream, W, ld, t.tau,
                       N, p.nrefl, Tf);
    TL_CHECK_LAUNCH();
  }
  hipLaunchKernelGGL(backtransform_kernel, dim3((unsigned)k), dim3(kBT), sizeof(double) * N,
                     stream, X, k, W, ld, Tf, N, p.nrefl, p.nwy, Z);
  TL_CHECK_LAUNCH();
  // u^T = z^T L^-1 (rows of Z times the lower-triangular inverse)
  TL_TRY(gemm(gemm_args(Z, N, Linv, ld, evecs, N, k, N, N, 1.0, 0.0, 2), false, 1, stream));
  return stage_mark(5, stream);
}

size_t dense_eigh_workspace_bytes(int N, int k) { return plan_dense(N, k).bytes; }

}  // namespace tl

extern "C" tl_status tl_set_dense_eigh_events(void* const* events, int count) {
  tl::clear_error();
  TL_REQUIRE(count == 0 || (events != nullptr && count == tl::kStages),
             "give %d events or none", tl::kStages);
  for (int i = 0; i < tl::kStages; ++i)
    tl::g_stage[i] = count ? (hipEvent_t)events[i] : nullptr;
  return TL_OK;
}

extern "C" tl_status tl_dense_gen_eigh_workspace_bytes(int N, int k, size_t* bytes) {
  tl::clear_error();
  TL_REQUIRE(bytes != nullptr, "null output");
  TL_TRY(tl::check_dense(N, k));
  *bytes = tl::dense_eigh_workspace_bytes(N, k);
  return TL_OK;
}

extern "C" tl_status tl_dense_gen_eigh_lowest(const double* H_dev, const double* S_dev, int N,
                                              int k, double* evals_dev, double* evecs_dev,
                                              int* info_dev, void* ws_dev, size_t ws_bytes,
                                              void* stream) {
  tl::clear_error();
  return tl::dense_gen_eigh_lowest(H_dev, S_dev, N, k, evals_dev, evecs_dev, info_dev, ws_dev,
                                   ws_bytes, (hipStream_t)stream);
}
