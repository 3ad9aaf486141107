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
//   4. Householder tridiagonalisation C = Q T Q^T, one column per step: a
//      one-workgroup kernel forms the reflector, a row-parallel kernel applies
//      the previous step's rank-2 update to the trailing matrix and multiplies
//      it by the new reflector in the same pass (one read and one write of the
//      trailing matrix per column).
//   5. The k lowest eigenvalues of T by Sturm-count multisection (256 points
//      per workgroup and round).
//   6. Eigenvectors of T by inverse iteration (partial-pivoting tridiagonal
//      LU, three solves), orthonormalised by two Cholesky-QR passes.
//   7. Back-transformation by the reflectors (compact WY blocks of 32) and
//      u = L^-T x.
#include <algorithm>
#include <cfloat>
#include <cmath>

#include "common.h"

namespace tl {
namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kNB = 64;         // Cholesky / inverse block
constexpr int kWY = 32;         // reflectors per back-transformation block
constexpr int kMaxK = 64;       // eigenpairs per call
constexpr int kMaxN = 7680;     // order (z in LDS during the back-transformation)
constexpr int kMSect = 256;     // multisection points per round

// ------------------------------------------------------------------ helpers

__device__ inline double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
  return v;
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

// Factor the diagonal block at (p, p) in place (lower) and write its inverse
// into the same block of Linv.  A non-positive pivot records the first
// failing column (1-based) in *info and continues with pivot 1.
__global__ __launch_bounds__(256) void potrf_diag_kernel(double* __restrict__ L,
                                                         double* __restrict__ Linv, int64_t ld,
                                                         int p, int* info) {
  __shared__ double a[kNB][kNB + 1];
  __shared__ double x[kNB][kNB + 1];
  __shared__ int fail;
  const int tid = threadIdx.x;
  if (tid == 0) fail = 0;
  for (int e = tid; e < kNB * kNB; e += 256) {
    const int r = e / kNB, c = e % kNB;
    a[r][c] = c <= r ? L[(int64_t)(p + r) * ld + p + c] : 0.0;
  }
  __syncthreads();
  for (int c = 0; c < kNB; ++c) {
    double piv = a[c][c];
    if (!(piv > 0.0)) {
      if (tid == 0 && fail == 0) fail = p + c + 1;
      piv = 1.0;
    }
    const double lcc = sqrt(piv), rinv = 1.0 / lcc;
    __syncthreads();
    if (tid < kNB) {
      if (tid > c) a[tid][c] *= rinv;
      if (tid == c) a[c][c] = lcc;
    }
    __syncthreads();
    const int n2 = kNB - 1 - c;
    for (int e = tid; e < n2 * n2; e += 256) {
      const int r = c + 1 + e / n2, cc = c + 1 + e % n2;
      if (cc <= r) a[r][cc] -= a[r][c] * a[cc][c];
    }
    __syncthreads();
  }
  // inverse of the lower-triangular block, one column per thread
  if (tid < kNB) {
    const int j = tid;
    for (int i = 0; i < j; ++i) x[i][j] = 0.0;
    x[j][j] = 1.0 / a[j][j];
    for (int i = j + 1; i < kNB; ++i) {
      double s = 0.0;
      for (int q = j; q < i; ++q) s += a[i][q] * x[q][j];
      x[i][j] = -s / a[i][i];
    }
  }
  __syncthreads();
  for (int e = tid; e < kNB * kNB; e += 256) {
    const int r = e / kNB, c = e % kNB;
    L[(int64_t)(p + r) * ld + p + c] = c <= r ? a[r][c] : 0.0;
    Linv[(int64_t)(p + r) * ld + p + c] = c <= r ? x[r][c] : 0.0;
  }
  if (tid == 0 && fail != 0) {
    if (*info == 0) *info = fail;
  }
}

// ------------------------------------------------------------------ tridiagonalisation
struct TridArgs {
  double* C;         // N x N symmetric, row stride ld, overwritten
  double* Vt;        // reflector j in row j (length N, zero up to index j, 1 at j+1)
  double* y;         // tau_j * A22 v_j
  double* w;         // w_{j-1}
  double* d;         // diagonal of T
  double* e;         // off-diagonal of T
  double* tau;
  int64_t ld;
  int N;
};

// Reflector of column j.  Finishes w_{j-1} = y - 1/2 tau (y.v) v, takes row j
// of the matrix with the pending rank-2 update of step j-1 applied on the
// fly, and forms v_j, tau_j (LAPACK dlarfg convention, beta = -sign(alpha)
// ||x||), d_j and e_j.
__global__ __launch_bounds__(256) void tridiag_house_kernel(TridArgs t, int j) {
  __shared__ double red[4];
  __shared__ double s_alpha;
  const int N = t.N, tid = threadIdx.x;
  const bool corr = j >= 1;  // the row kernel ran for every j <= N - 2
  const double* vp = corr ? t.Vt + (int64_t)(j - 1) * t.ld : nullptr;
  double* vj = t.Vt + (int64_t)j * t.ld;
  const double* row = t.C + (int64_t)j * t.ld;
  double cw = 0.0, wj = 0.0, vpj = 0.0;
  if (corr) {
    double s = 0.0;
    for (int i = j + tid; i < N; i += 256) s += t.y[i] * vp[i];
    s = block_sum(s, red);
    cw = 0.5 * t.tau[j - 1] * s;
    for (int i = j + tid; i < N; i += 256) t.w[i] = t.y[i] - cw * vp[i];
    vpj = vp[j];
    wj = t.y[j] - cw * vpj;
  }
  // x_i (i >= j) into vj[i]; zeros below
  double sig = 0.0;
  for (int i = tid; i < N; i += 256) {
    if (i < j) {
      vj[i] = 0.0;
      continue;
    }
    double x = row[i];
    if (corr) x -= vp[i] * wj + (t.y[i] - cw * vp[i]) * vpj;
    vj[i] = x;
    if (i == j) t.d[j] = x;
    if (i == j + 1) s_alpha = x;
    if (i >= j + 2) sig += x * x;
  }
  if (j >= N - 1) return;  // last column: only d
  sig = block_sum(sig, red);  // contains the barrier that publishes s_alpha
  const double alpha = s_alpha;
  double tau = 0.0, beta = alpha, scale = 0.0;
  if (sig > 0.0) {
    beta = -copysign(sqrt(alpha * alpha + sig), alpha);
    tau = (beta - alpha) / beta;
    scale = 1.0 / (alpha - beta);
  }
  for (int i = j + 1 + tid; i < N; i += 256) vj[i] = (i == j + 1) ? 1.0 : vj[i] * scale;
  if (tid == 0) {
    vj[j] = 0.0;  // held x_j until the barrier in block_sum
    t.tau[j] = tau;
    t.e[j] = beta;
  }
}

// Rows r > j: apply step j-1's update A -= v w^T + w v^T (columns > j) and
// form y_j[r] = tau_j sum_c A[r][c] v_j[c].  Two rows per wave.
__global__ __launch_bounds__(256) void tridiag_update_kernel(TridArgs t, int j) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int N = t.N;
  const int r0 = j + 1 + (blockIdx.x * 4 + wave) * 2;
  if (r0 >= N) return;
  const bool two = r0 + 1 < N;
  const bool upd = j >= 1;
  const double* vj = t.Vt + (int64_t)j * t.ld;
  const double* vp = upd ? t.Vt + (int64_t)(j - 1) * t.ld : vj;
  double* row0 = t.C + (int64_t)r0 * t.ld;
  double* row1 = two ? row0 + t.ld : row0;
  double vr0 = 0.0, wr0 = 0.0, vr1 = 0.0, wr1 = 0.0;
  if (upd) {
    vr0 = vp[r0];
    wr0 = t.w[r0];
    if (two) {
      vr1 = vp[r0 + 1];
      wr1 = t.w[r0 + 1];
    }
  }
  double acc0 = 0.0, acc1 = 0.0;
  for (int c = j + 1 + lane; c < N; c += 64) {
    const double v = vj[c];
    double a0 = row0[c];
    double a1 = two ? row1[c] : 0.0;
    if (upd) {
      const double pv = vp[c], pw = t.w[c];
      a0 -= vr0 * pw + wr0 * pv;
      row0[c] = a0;
      if (two) {
        a1 -= vr1 * pw + wr1 * pv;
        row1[c] = a1;
      }
    }
    acc0 += a0 * v;
    acc1 += a1 * v;
  }
  acc0 = wave_sum(acc0);
  acc1 = wave_sum(acc1);
  if (lane == 0) {
    const double tj = t.tau[j];
    t.y[r0] = tj * acc0;
    if (two) t.y[r0 + 1] = tj * acc1;
  }
}

// ------------------------------------------------------------------ bisection
struct TriSpec {
  const double* d;
  const double* e;
  int N;
};

__device__ inline int sturm_count(const TriSpec& T, double x, double pivmin) {
  int cnt = 0;
  double q = T.d[0] - x;
  if (fabs(q) < pivmin) q = -pivmin;
  if (q < 0.0) ++cnt;
  for (int i = 1; i < T.N; ++i) {
    const double ei = T.e[i - 1];
    q = (T.d[i] - x) - ei * ei / q;
    if (fabs(q) < pivmin) q = -pivmin;
    if (q < 0.0) ++cnt;
  }
  return cnt;
}

// Gershgorin interval, largest |entry| and the pivot floor of the Sturm
// recurrence (LAPACK dstebz conventions).
__device__ inline void tri_bounds(const TriSpec& T, double* red, double& glo, double& ghi,
                                  double& pivmin) {
  double lo = 1e308, hi = -1e308, emax = 0.0;
  for (int i = threadIdx.x; i < T.N; i += 256) {
    const double el = i > 0 ? fabs(T.e[i - 1]) : 0.0, er = i < T.N - 1 ? fabs(T.e[i]) : 0.0;
    lo = fmin(lo, T.d[i] - el - er);
    hi = fmax(hi, T.d[i] + el + er);
    emax = fmax(emax, er * er);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, o));
    hi = fmax(hi, __shfl_xor(hi, o));
    emax = fmax(emax, __shfl_xor(emax, o));
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) {
    red[wave] = lo;
    red[4 + wave] = hi;
    red[8 + wave] = emax;
  }
  __syncthreads();
  glo = fmin(fmin(red[0], red[1]), fmin(red[2], red[3]));
  ghi = fmax(fmax(red[4], red[5]), fmax(red[6], red[7]));
  emax = fmax(fmax(red[8], red[9]), fmax(red[10], red[11]));
  pivmin = DBL_MIN * fmax(1.0, emax);
  const double tnorm = fmax(fabs(glo), fabs(ghi));
  const double fudge = 2.1 * DBL_EPSILON * tnorm * T.N + 4.2 * pivmin;
  glo -= fudge;
  ghi += fudge;
}

// Eigenvalue m (0-based, ascending) of T per workgroup.
__global__ __launch_bounds__(256) void bisect_kernel(TriSpec T, double* __restrict__ evals) {
  __shared__ double red[12];
  __shared__ double s_lo, s_hi;
  __shared__ double s_x[kMSect];
  __shared__ int s_c[kMSect];
  const int m = blockIdx.x, tid = threadIdx.x;
  double glo, ghi, pivmin;
  tri_bounds(T, red, glo, ghi, pivmin);
  double lo = glo, hi = ghi;
  for (int round = 0; round < 24; ++round) {
    const double tol = 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)) + pivmin;
    if (hi - lo <= tol) break;  // uniform: lo, hi come from shared memory
    const double x = lo + (hi - lo) * ((double)(tid + 1) / (double)(kMSect + 1));
    s_x[tid] = x;
    s_c[tid] = sturm_count(T, x, pivmin);
    __syncthreads();
    if (tid == 0) {
      double nlo = lo, nhi = hi;
      for (int q = 0; q < kMSect; ++q) {
        if (s_c[q] <= m)
          nlo = fmax(nlo, s_x[q]);
        else
          nhi = fmin(nhi, s_x[q]);
      }
      if (nhi < nlo) nhi = nlo;
      s_lo = nlo;
      s_hi = nhi;
    }
    __syncthreads();
    const double olo = lo, ohi = hi;
    lo = s_lo;
    hi = s_hi;
    __syncthreads();
    if (lo == olo && hi == ohi) break;  // no representable progress
  }
  if (tid == 0) evals[m] = 0.5 * (lo + hi);
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
// pseudo-random start, 2-norm normalisation.
__global__ __launch_bounds__(64) void inverse_iter_kernel(InvArgs a) {
  // ||T|| from the Gershgorin interval, by this wave alone
  double lo = 1e308, hi = -1e308;
  const int N = a.T.N, k = a.k;
  for (int i = threadIdx.x; i < N; i += 64) {
    const double el = i > 0 ? fabs(a.T.e[i - 1]) : 0.0, er = i < N - 1 ? fabs(a.T.e[i]) : 0.0;
    lo = fmin(lo, a.T.d[i] - el - er);
    hi = fmax(hi, a.T.d[i] + el + er);
  }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) {
    lo = fmin(lo, __shfl_xor(lo, o));
    hi = fmax(hi, __shfl_xor(hi, o));
  }
  const double tnorm = fmax(fabs(lo), fabs(hi));
  const double pert = fmax(DBL_EPSILON * tnorm, DBL_MIN);
  const int m = blockIdx.x * 64 + threadIdx.x;
  if (m >= k) return;
  const double lam = a.evals[m];
  const int64_t P = (int64_t)N * k;
  double* RU0 = a.f;
  double* U1 = a.f + P;
  double* U2 = a.f + 2 * P;
  double* LM = a.f + 3 * P;
  double* SW = a.f + 4 * P;
  double* X = a.X;
  // factorisation
  double p = a.T.d[0] - lam, q = N > 1 ? a.T.e[0] : 0.0;
  for (int i = 0; i + 1 < N; ++i) {
    const double sub = a.T.e[i];
    const double dn = a.T.d[i + 1] - lam;
    const double en = i + 2 < N ? a.T.e[i + 1] : 0.0;
    const int64_t o = (int64_t)i * k + m;
    double u0, u1, u2, l, sw;
    if (fabs(p) >= fabs(sub)) {
      l = p != 0.0 ? sub / p : 0.0;
      u0 = p;
      u1 = q;
      u2 = 0.0;
      p = dn - l * q;
      q = en;
      sw = 0.0;
    } else {
      l = p / sub;
      u0 = sub;
      u1 = dn;
      u2 = en;
      p = q - l * dn;
      q = -l * en;
      sw = 1.0;
    }
    if (fabs(u0) < pert) u0 = u0 < 0.0 ? -pert : pert;
    RU0[o] = 1.0 / u0;
    U1[o] = u1;
    U2[o] = u2;
    LM[o] = l;
    SW[o] = sw;
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
  // start vector in [-1, 1)
  for (int i = 0; i < N; ++i) {
    const uint64_t r = splitmix64(((uint64_t)m << 32) ^ (uint64_t)i);
    X[(int64_t)i * k + m] = (double)(r >> 11) * (2.0 / 9007199254740992.0) - 1.0;
  }
  for (int it = 0; it < 3; ++it) {
    // forward elimination of the right-hand side
    double bi = X[m];
    for (int i = 0; i + 1 < N; ++i) {
      const int64_t o = (int64_t)i * k + m;
      const double bn = X[o + k];
      const double l = LM[o];
      if (SW[o] != 0.0) {
        X[o] = bn;
        bi = bi - l * bn;
      } else {
        X[o] = bi;
        bi = bn - l * bi;
      }
    }
    X[(int64_t)(N - 1) * k + m] = bi;
    // back substitution
    double x1 = 0.0, x2 = 0.0, xmax = 0.0;
    for (int i = N - 1; i >= 0; --i) {
      const int64_t o = (int64_t)i * k + m;
      const double xi = (X[o] - U1[o] * x1 - U2[o] * x2) * RU0[o];
      X[o] = xi;
      xmax = fmax(xmax, fabs(xi));
      x2 = x1;
      x1 = xi;
    }
    const double s = xmax > 0.0 ? 1.0 / xmax : 1.0;
    double nrm = 0.0;
    for (int i = 0; i < N; ++i) {
      const int64_t o = (int64_t)i * k + m;
      const double v = X[o] * s;
      X[o] = v;
      nrm += v * v;
    }
    if (it == 2) {
      const double sn = nrm > 0.0 ? 1.0 / sqrt(nrm) : 1.0;
      for (int i = 0; i < N; ++i) X[(int64_t)i * k + m] *= sn;
    }
  }
}

// ------------------------------------------------------------------ Cholesky-QR
// Partial Gram matrices of 64-row chunks of X [N][k].
__global__ __launch_bounds__(256) void gram_partial_kernel(const double* __restrict__ X, int N,
                                                           int k, double* __restrict__ part) {
  __shared__ double xs[64][kMaxK + 1];
  const int i0 = blockIdx.x * 64, tid = threadIdx.x;
  for (int e = tid; e < 64 * k; e += 256) {
    const int r = e / k, c = e % k;
    xs[r][c] = i0 + r < N ? X[(int64_t)(i0 + r) * k + c] : 0.0;
  }
  __syncthreads();
  double* out = part + (int64_t)blockIdx.x * k * k;
  for (int e = tid; e < k * k; e += 256) {
    const int p = e / k, q = e % k;
    double s = 0.0;
    for (int r = 0; r < 64; ++r) s += xs[r][p] * xs[r][q];
    out[e] = s;
  }
}

// G = sum of the partials = R^T R; writes R^-1 (upper).  A pivot below
// 1/4 means the vectors were not independent: info = -2.
__global__ __launch_bounds__(256) void chol_small_kernel(const double* __restrict__ part,
                                                         int nparts, int k,
                                                         double* __restrict__ Rinv, int* info) {
  __shared__ double g[kMaxK][kMaxK + 1];
  __shared__ double x[kMaxK][kMaxK + 1];
  __shared__ int bad;
  const int tid = threadIdx.x;
  if (tid == 0) bad = 0;
  for (int e = tid; e < k * k; e += 256) {
    double s = 0.0;
    for (int b = 0; b < nparts; ++b) s += part[(int64_t)b * k * k + e];
    g[e / k][e % k] = s;
  }
  __syncthreads();
  // upper Cholesky G = R^T R, R stored in g's upper triangle
  for (int c = 0; c < k; ++c) {
    double piv = g[c][c];
    if (!(piv > 0.25)) {
      if (tid == 0) bad = 1;
      piv = 1.0;
    }
    const double rcc = sqrt(piv), rinv = 1.0 / rcc;
    __syncthreads();
    if (tid < k) {
      if (tid > c) g[c][tid] *= rinv;
      if (tid == c) g[c][c] = rcc;
    }
    __syncthreads();
    const int n2 = k - 1 - c;
    for (int e = tid; e < n2 * n2; e += 256) {
      const int r = c + 1 + e / n2, cc = c + 1 + e % n2;
      if (cc >= r) g[r][cc] -= g[c][r] * g[c][cc];
    }
    __syncthreads();
  }
  // R^-1 (upper), one column per thread: R x = e_j
  if (tid < k) {
    const int j = tid;
    for (int i = j + 1; i < k; ++i) x[i][j] = 0.0;
    x[j][j] = 1.0 / g[j][j];
    for (int i = j - 1; i >= 0; --i) {
      double s = 0.0;
      for (int q = i + 1; q <= j; ++q) s += g[i][q] * x[q][j];
      x[i][j] = -s / g[i][i];
    }
  }
  __syncthreads();
  for (int e = tid; e < k * k; e += 256) Rinv[e] = x[e / k][e % k];
  if (tid == 0 && bad) {
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
  __syncthreads();
  if (tid == 0) {
    for (int c = 0; c < kWY; ++c)
      for (int r = 0; r < kWY; ++r) T[r][c] = 0.0;
    for (int c = 0; c < nb; ++c) {
      const double tc = tau[j0 + c];
      T[c][c] = tc;
      for (int r = 0; r < c; ++r) {
        double s = 0.0;
        for (int q = r; q < c; ++q) s += T[r][q] * gv[q][c];
        T[r][c] = -tc * s;
      }
    }
  }
  __syncthreads();
  for (int e = tid; e < kWY * kWY; e += 256) Tout[(int64_t)b * kWY * kWY + e] = T[e / kWY][e % kWY];
}

// One workgroup per eigenvector: z = Q x with Q = H_0 H_1 ... (blocks applied
// last first), z in LDS; output row m of Z [k][N].
__global__ __launch_bounds__(256) void backtransform_kernel(const double* __restrict__ X, int k,
                                                            const double* __restrict__ Vt,
                                                            int64_t ld,
                                                            const double* __restrict__ Tf,
                                                            int N, int nrefl, int nblocks,
                                                            double* __restrict__ Z) {
  extern __shared__ double z[];
  __shared__ double red[4][kWY];
  __shared__ double pp[kWY];
  const int m = blockIdx.x, tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  for (int i = tid; i < N; i += 256) z[i] = X[(int64_t)i * k + m];
  __syncthreads();
  for (int b = nblocks - 1; b >= 0; --b) {
    const int j0 = b * kWY, nb = min(kWY, nrefl - j0);
    const double* V = Vt + (int64_t)j0 * ld;
    double acc[kWY];
#pragma unroll
    for (int c = 0; c < kWY; ++c) acc[c] = 0.0;
    for (int i = j0 + 1 + tid; i < N; i += 256) {
      const double zi = z[i];
#pragma unroll
      for (int c = 0; c < kWY; ++c)
        if (c < nb) acc[c] += V[(int64_t)c * ld + i] * zi;
    }
#pragma unroll
    for (int c = 0; c < kWY; ++c) {
      const double s = wave_sum(acc[c]);
      if (lane == 0) red[wave][c] = s;
    }
    __syncthreads();
    if (tid < kWY) {
      const double* T = Tf + (int64_t)b * kWY * kWY + tid * kWY;
      double s = 0.0;
      for (int c = tid; c < kWY; ++c) s += T[c] * (red[0][c] + red[1][c] + red[2][c] + red[3][c]);
      pp[tid] = s;
    }
    __syncthreads();
    for (int i = j0 + 1 + tid; i < N; i += 256) {
      double s = 0.0;
#pragma unroll
      for (int c = 0; c < kWY; ++c)
        if (c < nb) s += V[(int64_t)c * ld + i] * pp[c];
      z[i] -= s;
    }
    __syncthreads();
  }
  for (int i = tid; i < N; i += 256) Z[(int64_t)m * N + i] = z[i];
}

// ------------------------------------------------------------------ plan
struct DensePlan {
  int N, Np, k, nrefl, nwy, nchunks;
  size_t off_L, off_Linv, off_C, off_W, off_vec, off_f, off_X, off_part, off_R, off_T, off_Z,
      bytes;
};

DensePlan plan_dense(int N, int k) {
  DensePlan p;
  p.N = N;
  p.k = k;
  p.Np = (int)ceil_div(N, kNB) * kNB;
  p.nrefl = std::max(N - 2, 0);
  p.nwy = (int)ceil_div(p.nrefl, kWY);
  p.nchunks = (int)ceil_div(N, 64);
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
  p.off_vec = take(sizeof(double) * 5 * (size_t)p.Np);
  p.off_f = take(sizeof(double) * 5 * (size_t)N * k);
  p.off_X = take(sizeof(double) * (size_t)N * k);
  p.off_part = take(sizeof(double) * (size_t)p.nchunks * k * k);
  p.off_R = take(sizeof(double) * (size_t)k * k);
  p.off_T = take(sizeof(double) * (size_t)std::max(p.nwy, 1) * kWY * kWY);
  p.off_Z = take(sizeof(double) * (size_t)k * N);
  p.bytes = o;
  return p;
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
  hipLaunchKernelGGL(setup_kernel, dim3((unsigned)ceil_div((int64_t)Np * Np, 256)), dim3(256), 0,
                     stream, S, N, Np, L, Linv, info);
  TL_CHECK_LAUNCH();
  for (int q = 0; q < Np; q += kNB) {
    hipLaunchKernelGGL(potrf_diag_kernel, dim3(1), dim3(256), 0, stream, L, Linv, ld, q, info);
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
  // 3. C = Linv H Linv^T (N x N, row stride ld)
  TL_TRY(gemm(gemm_args(Linv, ld, H, N, W, ld, N, N, N, 1.0, 0.0, 1), false, 1, stream));
  {
    GemmArgs g = gemm_args(W, ld, Linv, ld, C, ld, N, N, N, 1.0, 0.0, 3);
    g.lower = 1;
    g.mirror = 1;
    TL_TRY(gemm(g, true, 1, stream));
  }
  // 4. tridiagonalisation; reflectors reuse W
  TridArgs t;
  t.C = C;
  t.Vt = W;
  t.y = vec;
  t.w = vec + Np;
  t.d = vec + 2 * Np;
  t.e = vec + 3 * Np;
  t.tau = vec + 4 * Np;
  t.ld = ld;
  t.N = N;
  for (int j = 0; j < N; ++j) {
    hipLaunchKernelGGL(tridiag_house_kernel, dim3(1), dim3(256), 0, stream, t, j);
    TL_CHECK_LAUNCH();
    if (j <= N - 2) {
      const int rows = N - j - 1;
      hipLaunchKernelGGL(tridiag_update_kernel, dim3((unsigned)ceil_div(rows, 8)), dim3(256), 0,
                         stream, t, j);
      TL_CHECK_LAUNCH();
    }
  }
  // 5. eigenvalues
  TriSpec T{t.d, t.e, N};
  hipLaunchKernelGGL(bisect_kernel, dim3((unsigned)k), dim3(256), 0, stream, T, evals);
  TL_CHECK_LAUNCH();
  if (evecs == nullptr) return TL_OK;
  // 6. eigenvectors of T
  double* F = (double*)(base + p.off_f);
  double* X = (double*)(base + p.off_X);
  InvArgs ia{T, evals, F, X, k};
  hipLaunchKernelGGL(inverse_iter_kernel, dim3((unsigned)ceil_div(k, 64)), dim3(64), 0, stream,
                     ia);
  TL_CHECK_LAUNCH();
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
  hipLaunchKernelGGL(backtransform_kernel, dim3((unsigned)k), dim3(256), sizeof(double) * N,
                     stream, X, k, W, ld, Tf, N, p.nrefl, p.nwy, Z);
  TL_CHECK_LAUNCH();
  // u^T = z^T L^-1 (rows of Z times the lower-triangular inverse)
  TL_TRY(gemm(gemm_args(Z, N, Linv, ld, evecs, N, k, N, N, 1.0, 0.0, 2), false, 1, stream));
  return TL_OK;
}

size_t dense_eigh_workspace_bytes(int N, int k) { return plan_dense(N, k).bytes; }

}  // namespace tl

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
