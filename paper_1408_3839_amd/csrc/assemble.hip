// Steps a4/a5: Galerkin entries as products of 1D inner products (proof of
// Lemma 3.1, eq. (nuc_potMatrTot); Sec. 3.4; Lemma 4.1 eqs. (BC-Core),
// (BC-mass), (BC-Laplace)).
//
// a4, per dimension l, one contraction over the grid nodes i:
//   C_l[(t, nu)][(mu, s)] = sum_i X[(t, nu)][i] * Y[(mu, s)][i]
//   X[(t, nu)][i] = p_t(x_i) g_nu(x_i)   (t < T, potential terms)
//                 = (A g_nu)(x_i)         (t = T,   stiffness)
//                 = (S g_nu)(x_i)         (t = T+1, mass)
//   Y[(mu, s)][i] = g_mu(x_i - s a_l)     (cyclic shift by s cells on a torus)
// i.e. G diag(p_t) G_s^T for all terms and shifts at once: an (T+2) m0 x m0 S
// by n GEMM whose operands are formed on the fly from G, P (never stored).
// Since A and S commute with cyclic shifts and are symmetric,
// <A g_(mu,s), g_nu> = sum_i g_mu(x_i - s a) (A g_nu)(x_i).
// Only shifts s = 0..L/2 are contracted: the replicated potential has the
// lattice period, so C_l[mu][nu][-s] = C_l[nu][mu][s].
//
// a5, FP64 in every precision mode, thread per entry of the block column:
//   V_k = sum_t prod_l C_l[t][mu][nu][k_l],
//   T_k = 1/2 (D_1 M_2 M_3 + M_1 D_2 M_3 + M_1 M_2 D_3),  S_k = M_1 M_2 M_3,
//   H_k = T_k - V_k.
#include <algorithm>
#include <cmath>

#include "common.h"

namespace tl {
namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

constexpr int kBM = 32;   // rows of a workgroup tile (2 MFMA row blocks)
constexpr int kBN = 32;   // columns of a workgroup tile (2 MFMA column blocks)
constexpr int kKT = 64;   // nodes per LDS stage
constexpr int kLDP = kKT + 1;
constexpr int kPerThread = kBM * kKT / 256;  // staged values per thread and operand

struct DimArgs {
  const double* G;
  const double* AG;
  const double* SG;
  const double* P;
  double* part;    // [ks][M][N] partial sums over node chunks
  int n, S, cn, M, N, kchunk, ks, tiles_n, block_begin;
};

struct ContractArgs {
  DimArgs d[3];
  int m0, T;
};

// One launch for the three dimensions.  Workgroup = 4 waves = a 32 x 32 tile
// of C_l over one chunk of nodes; each wave owns a 16 x 16 block and issues
// V_MFMA_F64_16X16X4_F64 from LDS.  The next 64-node stage is loaded into
// registers while the current one is multiplied (double buffering).
__global__ __launch_bounds__(256) void contract_f64_kernel(ContractArgs a) {
  __shared__ double Xs[kBM][kLDP];
  __shared__ double Ys[kBN][kLDP];
  const int b = blockIdx.x;
  const int dd = b >= a.d[2].block_begin ? 2 : (b >= a.d[1].block_begin ? 1 : 0);
  const DimArgs& p = a.d[dd];
  const int local = b - p.block_begin;
  const int z = local % p.ks;
  const int rest = local / p.ks;
  const int col0 = (rest % p.tiles_n) * kBN;
  const int row0 = (rest / p.tiles_n) * kBM;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int kbeg = z * p.kchunk;
  const int kend = min(p.n, kbeg + p.kchunk);
  const int wm = wave >> 1, wn = wave & 1;
  double xr[kPerThread], yr[kPerThread];
  // the rows and columns a thread stages are the same in every stage:
  // resolve (term, nu) and (mu, shift) once
  const double* xa[kPerThread];   // P row of the term (or null)
  const double* xb[kPerThread];   // G, AG or SG row of nu
  const double* yb[kPerThread];   // G row of mu
  int ysh[kPerThread];
  bool xok[kPerThread], yok[kPerThread];
#pragma unroll
  for (int j = 0; j < kPerThread; ++j) {
    const int r = (tid + 256 * j) / kKT;
    const int row = row0 + r, col = col0 + r;
    xok[j] = row < p.M;
    yok[j] = col < p.N;
    const int t = xok[j] ? row / a.m0 : 0, nu = xok[j] ? row - t * a.m0 : 0;
    xa[j] = t < a.T ? p.P + (int64_t)t * p.n : nullptr;
    xb[j] = (t < a.T ? p.G : (t == a.T ? p.AG : p.SG)) + (int64_t)nu * p.n;
    const int mu = yok[j] ? col / p.S : 0, sh = yok[j] ? col - mu * p.S : 0;
    yb[j] = p.G + (int64_t)mu * p.n;
    ysh[j] = sh * p.cn;
  }

  auto stage = [&](int k0) {
#pragma unroll
    for (int j = 0; j < kPerThread; ++j) {
      const int kk = (tid + 256 * j) & (kKT - 1);
      const int i = k0 + kk;
      const bool in_k = i < kend;
      double xv = 0.0, yv = 0.0;
      if (xok[j] && in_k) xv = xa[j] ? xa[j][i] * xb[j][i] : xb[j][i];
      if (yok[j] && in_k) {
        int src = i - ysh[j];
        if (src < 0) src += p.n;
        yv = yb[j][src];
      }
      xr[j] = xv;
      yr[j] = yv;
    }
  };
  auto commit = [&]() {
#pragma unroll
    for (int j = 0; j < kPerThread; ++j) {
      const int e = tid + 256 * j;
      Xs[e / kKT][e & (kKT - 1)] = xr[j];
      Ys[e / kKT][e & (kKT - 1)] = yr[j];
    }
  };

  f64x4 acc = {0.0, 0.0, 0.0, 0.0};
  stage(kbeg);
  commit();
  __syncthreads();
  for (int k0 = kbeg; k0 < kend; k0 += kKT) {
    const bool more = k0 + kKT < kend;
    if (more) stage(k0 + kKT);
#pragma unroll
    for (int kk = 0; kk < kKT; kk += 4) {
      double av = Xs[wm * 16 + (lane & 15)][kk + (lane >> 4)];
      double bv = Ys[wn * 16 + (lane & 15)][kk + (lane >> 4)];
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
    }
    __syncthreads();
    if (more) commit();
    __syncthreads();
  }
  // f64 16x16x4 result layout on gfx950: register r of lane l holds
  // D[l / 16 + 4 r][l % 16] (checked with a one-wave probe).
  const int col = col0 + wn * 16 + (lane & 15);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    int row = row0 + wm * 16 + (lane >> 4) + 4 * r;
    if (row < p.M && col < p.N) p.part[((int64_t)z * p.M + row) * p.N + col] = acc[r];
  }
}

// ---------------------------------------------------------------- FP32 mode
// Same tiling; the operands are rounded to FP32 in the staging step and
// multiplied with V_MFMA_F32_16X16X4_F32; each 64-node stage's FP32 sums are
// added into FP64 accumulators.
__global__ __launch_bounds__(256) void contract_f32_kernel(ContractArgs a) {
  __shared__ float Xs[kBM][kLDP];
  __shared__ float Ys[kBN][kLDP];
  const int b = blockIdx.x;
  const int dd = b >= a.d[2].block_begin ? 2 : (b >= a.d[1].block_begin ? 1 : 0);
  const DimArgs& p = a.d[dd];
  const int local = b - p.block_begin;
  const int z = local % p.ks;
  const int rest = local / p.ks;
  const int col0 = (rest % p.tiles_n) * kBN;
  const int row0 = (rest / p.tiles_n) * kBM;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int kbeg = z * p.kchunk;
  const int kend = min(p.n, kbeg + p.kchunk);
  const int wm = wave >> 1, wn = wave & 1;
  float xr[kPerThread], yr[kPerThread];
  const double* xa[kPerThread];
  const double* xb[kPerThread];
  const double* yb[kPerThread];
  int ysh[kPerThread];
  bool xok[kPerThread], yok[kPerThread];
#pragma unroll
  for (int j = 0; j < kPerThread; ++j) {
    const int r = (tid + 256 * j) / kKT;
    const int row = row0 + r, col = col0 + r;
    xok[j] = row < p.M;
    yok[j] = col < p.N;
    const int t = xok[j] ? row / a.m0 : 0, nu = xok[j] ? row - t * a.m0 : 0;
    xa[j] = t < a.T ? p.P + (int64_t)t * p.n : nullptr;
    xb[j] = (t < a.T ? p.G : (t == a.T ? p.AG : p.SG)) + (int64_t)nu * p.n;
    const int mu = yok[j] ? col / p.S : 0, sh = yok[j] ? col - mu * p.S : 0;
    yb[j] = p.G + (int64_t)mu * p.n;
    ysh[j] = sh * p.cn;
  }
  auto stage = [&](int k0) {
#pragma unroll
    for (int j = 0; j < kPerThread; ++j) {
      const int kk = (tid + 256 * j) & (kKT - 1);
      const int i = k0 + kk;
      const bool in_k = i < kend;
      double xv = 0.0, yv = 0.0;
      if (xok[j] && in_k) xv = xa[j] ? xa[j][i] * xb[j][i] : xb[j][i];
      if (yok[j] && in_k) {
        int src = i - ysh[j];
        if (src < 0) src += p.n;
        yv = yb[j][src];
      }
      xr[j] = (float)xv;
      yr[j] = (float)yv;
    }
  };
  auto commit = [&]() {
#pragma unroll
    for (int j = 0; j < kPerThread; ++j) {
      const int e = tid + 256 * j;
      Xs[e / kKT][e & (kKT - 1)] = xr[j];
      Ys[e / kKT][e & (kKT - 1)] = yr[j];
    }
  };
  f64x4 acc = {0.0, 0.0, 0.0, 0.0};
  stage(kbeg);
  commit();
  __syncthreads();
  for (int k0 = kbeg; k0 < kend; k0 += kKT) {
    const bool more = k0 + kKT < kend;
    if (more) stage(k0 + kKT);
    f32x4 acc32 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kk = 0; kk < kKT; kk += 4) {
      float av = Xs[wm * 16 + (lane & 15)][kk + (lane >> 4)];
      float bv = Ys[wn * 16 + (lane & 15)][kk + (lane >> 4)];
      acc32 = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc32, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r] += (double)acc32[r];
    __syncthreads();
    if (more) commit();
    __syncthreads();
  }
  // f32 16x16x4 result layout: register r of lane l holds D[4 (l / 16) + r][l % 16]
  const int col = col0 + wn * 16 + (lane & 15);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    int row = row0 + wm * 16 + 4 * (lane >> 4) + r;
    if (row < p.M && col < p.N) p.part[((int64_t)z * p.M + row) * p.N + col] = acc[r];
  }
}

// ---------------------------------------------------------------- split modes
// Operand splitting in the manner of Ozaki, Ogita, Oishi & Rump (2012): each
// row r of X (and of G) is scaled by a power of two sigma_r >= max|row|, and
// the scaled values are cut into integer slices
//   x/sigma = sum_k n_k 2^(-k beta),  |n_1| <= 2^beta, |n_k| <= 2^(beta-1),
// each exactly representable in bf16 (beta = 8) or fp16 (beta = 9).  A slice
// product summed over one 32-node MFMA (16x16x32) stays below 2^24 and is
// exact in FP32; all products of one level a + b are accumulated in FP32 over
// one MFMA step and then added to a per-level FP64 accumulator.  Only the
// products with a + b <= s + 1 are formed (triangular truncation).

constexpr int kMaxSlices = 8;
constexpr int kSKT = 32;             // nodes per LDS stage = one MFMA K step
constexpr int kSLD = kSKT + 8;       // padded LDS row (elements)

template <typename T>
struct LowTraits;
template <>
struct LowTraits<__bf16> {
  static constexpr int beta = 8;
};
template <>
struct LowTraits<_Float16> {
  static constexpr int beta = 9;
};

struct SliceArgs {
  const double* P[3];
  const double* G[3];
  const double* AG[3];
  const double* SG[3];
  void* xs[3];          // [s][M][n] slices of X rows
  void* ys[3];          // [s][m0][n] slices of G rows
  double* xscale[3];    // [M]
  double* yscale[3];    // [m0]
  int n[3], M[3];
  int rows_begin[7];    // X rows of dims 0..2, then G rows of dims 0..2
  int m0, T, s;
};

// Workgroup per row: max |value| (power-of-two scale), then the slices.
template <typename LowT>
__global__ __launch_bounds__(256) void slice_kernel(SliceArgs a) {
  constexpr int beta = LowTraits<LowT>::beta;
  __shared__ double wmax[4];
  const int b = blockIdx.x;
  int k = 0;
  while (k < 6 && b >= a.rows_begin[k + 1]) ++k;
  const bool isx = k < 3;
  const int d = isx ? k : k - 3;
  const int row = b - a.rows_begin[k];
  const int n = a.n[d];
  const double* base;
  const double* pot = nullptr;
  if (isx) {
    const int t = row / a.m0, nu = row - t * a.m0;
    base = (t < a.T ? a.G[d] : (t == a.T ? a.AG[d] : a.SG[d])) + (int64_t)nu * n;
    if (t < a.T) pot = a.P[d] + (int64_t)t * n;
  } else {
    base = a.G[d] + (int64_t)row * n;
  }
  double mx = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double v = pot ? pot[i] * base[i] : base[i];
    mx = fmax(mx, fabs(v));
  }
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = mx;
  __syncthreads();
  mx = fmax(fmax(wmax[0], wmax[1]), fmax(wmax[2], wmax[3]));
  // sigma = 2^e >= mx, so |x / sigma| <= 1 exactly
  int e = 0;
  if (mx > 0.0) {
    frexp(mx, &e);  // mx = f 2^e, f in [0.5, 1)
  }
  const double sigma = ldexp(1.0, e), inv = ldexp(1.0, -e);
  if (threadIdx.x == 0) (isx ? a.xscale[d] : a.yscale[d])[row] = sigma;
  LowT* out = (LowT*)(isx ? a.xs[d] : a.ys[d]);
  const int64_t rows = isx ? a.M[d] : a.m0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double v = (pot ? pot[i] * base[i] : base[i]) * inv;
    for (int q = 1; q <= a.s; ++q) {
      double sc = ldexp(1.0, q * beta);
      double nk = rint(v * sc);
      v = fma(-nk, ldexp(1.0, -q * beta), v);
      out[((int64_t)(q - 1) * rows + row) * n + i] = (LowT)nk;
    }
  }
}

struct SplitDimArgs {
  const void* xs;       // [s][M][n]
  const void* ys;       // [s][m0][n]
  const double* xscale;
  const double* yscale;
  double* part;
  int n, S, cn, M, N, kchunk, ks, tiles_n, block_begin;
};
struct SplitArgs {
  SplitDimArgs d[3];
  int m0, s;
};

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

template <typename LowT>
struct Vec8;
template <>
struct Vec8<__bf16> {
  typedef bf16x8 type;
  static __device__ inline f32x4 mfma(type a, type b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};
template <>
struct Vec8<_Float16> {
  typedef f16x8 type;
  static __device__ inline f32x4 mfma(type a, type b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};

template <typename LowT, int S>
__global__ __launch_bounds__(256) void contract_split_kernel(SplitArgs a) {
  typedef typename Vec8<LowT>::type v8;
  constexpr int beta = LowTraits<LowT>::beta;
  __shared__ __attribute__((aligned(16))) LowT Xl[S][kBM][kSLD];
  __shared__ __attribute__((aligned(16))) LowT Yl[S][kBN][kSLD];
  const int b = blockIdx.x;
  const int dd = b >= a.d[2].block_begin ? 2 : (b >= a.d[1].block_begin ? 1 : 0);
  const SplitDimArgs& p = a.d[dd];
  const int local = b - p.block_begin;
  const int z = local % p.ks;
  const int rest = local / p.ks;
  const int col0 = (rest % p.tiles_n) * kBN;
  const int row0 = (rest / p.tiles_n) * kBM;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int kbeg = z * p.kchunk;
  const int kend = min(p.n, kbeg + p.kchunk);
  const int wm = wave >> 1, wn = wave & 1;
  const LowT* xs = (const LowT*)p.xs;
  const LowT* ys = (const LowT*)p.ys;
  // staging: thread stages 4 consecutive nodes of one X row and one Y column
  const int sr = tid >> 3;             // row / column within the tile (0..31)
  const int sk = (tid & 7) * 4;        // first node within the stage
  const int xrow = row0 + sr, ycol = col0 + sr;
  const bool xok = xrow < p.M, yok = ycol < p.N;
  const int mu = yok ? ycol / p.S : 0;
  const int ysh = yok ? (ycol - mu * p.S) * p.cn : 0;
  LowT xr[S][4], yr[S][4];
  auto stage = [&](int k0) {
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const int i = k0 + sk + e;
      const bool in_k = i < kend;
      int src = i - ysh;
      if (src < 0) src += p.n;
#pragma unroll
      for (int q = 0; q < S; ++q) {
        xr[q][e] = (xok && in_k) ? xs[((int64_t)q * p.M + xrow) * p.n + i] : (LowT)0.0f;
        yr[q][e] = (yok && in_k) ? ys[((int64_t)q * a.m0 + mu) * p.n + src] : (LowT)0.0f;
      }
    }
  };
  auto commit = [&]() {
#pragma unroll
    for (int q = 0; q < S; ++q)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        Xl[q][sr][sk + e] = xr[q][e];
        Yl[q][sr][sk + e] = yr[q][e];
      }
  };
  double acc[S][4];
#pragma unroll
  for (int l = 0; l < S; ++l)
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[l][r] = 0.0;
  stage(kbeg);
  commit();
  __syncthreads();
  for (int k0 = kbeg; k0 < kend; k0 += kSKT) {
    const bool more = k0 + kSKT < kend;
    if (more) stage(k0 + kSKT);
    v8 av[S], bv[S];
#pragma unroll
    for (int q = 0; q < S; ++q) {
      av[q] = *(const v8*)&Xl[q][wm * 16 + (lane & 15)][8 * (lane >> 4)];
      bv[q] = *(const v8*)&Yl[q][wn * 16 + (lane & 15)][8 * (lane >> 4)];
    }
    // level l = qa + qb (0-based slices), l = 0..S-1
#pragma unroll
    for (int l = 0; l < S; ++l) {
      f32x4 c32 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int qa = 0; qa <= l; ++qa) c32 = Vec8<LowT>::mfma(av[qa], bv[l - qa], c32);
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[l][r] += (double)c32[r];
    }
    __syncthreads();
    if (more) commit();
    __syncthreads();
  }
  const int col = col0 + wn * 16 + (lane & 15);
  const double ysc = col < p.N ? p.yscale[col / p.S] : 0.0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    int row = row0 + wm * 16 + 4 * (lane >> 4) + r;
    if (row < p.M && col < p.N) {
      double v = 0.0;
#pragma unroll
      for (int l = S - 1; l >= 0; --l) v += ldexp(acc[l][r], -(l + 2) * beta);
      p.part[((int64_t)z * p.M + row) * p.N + col] = v * p.xscale[row] * ysc;
    }
  }
}

struct ReduceArgs {
  const double* part[3];
  double* C[3];
  int64_t MN[3];
  int ks[3];
  int64_t begin[3];  // flat start of each dim
};

// Sums the node-chunk partial sums into the compact C_l (all dims at once).
__global__ __launch_bounds__(256) void reduce_partials_kernel(ReduceArgs a, int64_t total) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  int d = idx >= a.begin[2] ? 2 : (idx >= a.begin[1] ? 1 : 0);
  int64_t e = idx - a.begin[d];
  const double* p = a.part[d] + e;
  double v = 0.0;
  for (int s = 0; s < a.ks[d]; ++s) v += p[(int64_t)s * a.MN[d]];
  a.C[d][e] = v;
}

struct CombineArgs {
  const double* C[3];   // compact C_l [M][N]
  int S[3], L[3], periodic[3], N[3];
  int m0, T;
  double* H;
  double* Sm;
};

__device__ inline double lookup(const CombineArgs& a, int d, int t, int mu, int nu, int k) {
  int row, col;
  if (!a.periodic[d] || k < a.S[d]) {
    row = t * a.m0 + nu;
    col = mu * a.S[d] + k;
  } else {  // negative shift: C[mu][nu][-s] = C[nu][mu][s]
    row = t * a.m0 + mu;
    col = nu * a.S[d] + (a.L[d] - k);
  }
  return a.C[d][(int64_t)row * a.N[d] + col];
}

// One wave per entry of the block column: lane t forms the product of term t
// (t < T), lane T the kinetic combination, lane T+1 the mass product; a
// wave-wide sum then gives V (FP64 throughout).
__global__ __launch_bounds__(256) void combine_periodic_kernel(CombineArgs a, int64_t total) {
  const int64_t idx = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (idx >= total) return;
  const int m2 = a.m0 * a.m0;
  const int64_t kflat = idx / m2;
  const int e = (int)(idx - kflat * m2);
  const int mu = e / a.m0, nu = e - mu * a.m0;
  const int k3 = (int)(kflat % a.L[2]);
  const int k2 = (int)((kflat / a.L[2]) % a.L[1]);
  const int k1 = (int)(kflat / ((int64_t)a.L[2] * a.L[1]));
  double V = 0.0, Tk = 0.0, Sk = 0.0;
  for (int t = lane; t < a.T + 2; t += 64) {
    if (t < a.T) {
      V += lookup(a, 0, t, mu, nu, k1) * lookup(a, 1, t, mu, nu, k2) * lookup(a, 2, t, mu, nu, k3);
    } else if (t == a.T) {
      double D1 = lookup(a, 0, a.T, mu, nu, k1), M1 = lookup(a, 0, a.T + 1, mu, nu, k1);
      double D2 = lookup(a, 1, a.T, mu, nu, k2), M2 = lookup(a, 1, a.T + 1, mu, nu, k2);
      double D3 = lookup(a, 2, a.T, mu, nu, k3), M3 = lookup(a, 2, a.T + 1, mu, nu, k3);
      Tk = 0.5 * (D1 * M2 * M3 + M1 * D2 * M3 + M1 * M2 * D3);
    } else {
      Sk = lookup(a, 0, a.T + 1, mu, nu, k1) * lookup(a, 1, a.T + 1, mu, nu, k2) *
           lookup(a, 2, a.T + 1, mu, nu, k3);
    }
  }
  for (int o = 32; o > 0; o >>= 1) V += __shfl_xor(V, o);
  const int tl = a.T % 64, sl = (a.T + 1) % 64;
  Tk = __shfl(Tk, tl);
  Sk = __shfl(Sk, sl);
  if (lane == 0) {
    a.H[idx] = Tk - V;
    a.Sm[idx] = Sk;
  }
}

// Optional HIP events recorded around the contraction launch of the next
// assembly calls of this thread (profiling hook for measured rooflines).
thread_local hipEvent_t g_ev_start = nullptr, g_ev_stop = nullptr;

struct Plan {
  int M[3], N[3], ks[3], kchunk[3], tiles_n[3], blocks[3];
  size_t part_off[3], c_off[3];  // byte offsets in the workspace
  size_t bytes;
  int total_blocks;
};

Plan make_plan(const Geometry& g) {
  Plan p;
  size_t off = 0;
  int nblk = 0;
  for (int d = 0; d < 3; ++d) {
    p.M[d] = (int)((g.pot_terms + 2) * g.m0);
    p.N[d] = g.m0 * g.shifts[d];
    int64_t tiles = ceil_div(p.M[d], kBM) * ceil_div(p.N[d], kBN);
    // enough workgroups to cover the chip, at least two stages per chunk
    int64_t want = std::max<int64_t>(1, ceil_div(512, tiles));
    int64_t maxsplit = std::max<int64_t>(1, g.n[d] / (2 * kKT));
    int ks = (int)std::min(want, maxsplit);
    int kchunk = (int)(ceil_div(ceil_div(g.n[d], ks), kKT) * kKT);
    ks = (int)ceil_div(g.n[d], kchunk);
    p.ks[d] = ks;
    p.kchunk[d] = kchunk;
    p.tiles_n[d] = (int)ceil_div(p.N[d], kBN);
    p.blocks[d] = (int)(tiles * ks);
    nblk += p.blocks[d];
    p.part_off[d] = off;
    off += align_up(sizeof(double) * (size_t)ks * p.M[d] * p.N[d], 256);
    p.c_off[d] = off;
    off += align_up(sizeof(double) * (size_t)p.M[d] * p.N[d], 256);
  }
  p.total_blocks = nblk;
  p.bytes = off;
  return p;
}

// Extra workspace of the split modes: slices of X and G rows and their scales.
struct SplitPlan {
  size_t xs_off[3], ys_off[3], xsc_off[3], ysc_off[3];
  size_t bytes;
};

SplitPlan make_split_plan(const Geometry& g, const Plan& plan, int s, size_t base) {
  SplitPlan sp;
  size_t off = base;
  for (int d = 0; d < 3; ++d) {
    sp.xs_off[d] = off;
    off += align_up(2 * (size_t)s * plan.M[d] * g.n[d], 256);
    sp.ys_off[d] = off;
    off += align_up(2 * (size_t)s * g.m0 * g.n[d], 256);
    sp.xsc_off[d] = off;
    off += align_up(sizeof(double) * (size_t)plan.M[d], 256);
    sp.ysc_off[d] = off;
    off += align_up(sizeof(double) * (size_t)g.m0, 256);
  }
  sp.bytes = off;
  return sp;
}

bool is_split(tl_precision prec) { return prec == TL_SPLIT_BF16 || prec == TL_SPLIT_FP16; }

int default_slices(tl_precision prec) { return prec == TL_SPLIT_FP16 ? 5 : 6; }

template <typename LowT>
tl_status launch_split(const Geometry& g, const Plan& plan, const SplitPlan& sp, char* wsb,
                       const double* G, const double* AG, const double* SG, const double* P,
                       int S, hipStream_t stream) {
  SliceArgs sa;
  std::memset(&sa, 0, sizeof(sa));
  sa.m0 = g.m0;
  sa.T = (int)g.pot_terms;
  sa.s = S;
  int rb = 0;
  for (int d = 0; d < 3; ++d) {
    sa.P[d] = P + g.pot_off[d];
    sa.G[d] = G + g.basis_off[d];
    sa.AG[d] = AG + g.basis_off[d];
    sa.SG[d] = SG + g.basis_off[d];
    sa.xs[d] = wsb + sp.xs_off[d];
    sa.ys[d] = wsb + sp.ys_off[d];
    sa.xscale[d] = (double*)(wsb + sp.xsc_off[d]);
    sa.yscale[d] = (double*)(wsb + sp.ysc_off[d]);
    sa.n[d] = g.n[d];
    sa.M[d] = plan.M[d];
  }
  for (int d = 0; d < 3; ++d) {
    sa.rows_begin[d] = rb;
    rb += plan.M[d];
  }
  for (int d = 0; d < 3; ++d) {
    sa.rows_begin[3 + d] = rb;
    rb += g.m0;
  }
  sa.rows_begin[6] = rb;
  hipLaunchKernelGGL(slice_kernel<LowT>, dim3((unsigned)rb), dim3(256), 0, stream, sa);
  TL_CHECK_LAUNCH();
  SplitArgs a;
  a.m0 = g.m0;
  a.s = S;
  int begin = 0;
  for (int d = 0; d < 3; ++d) {
    SplitDimArgs& q = a.d[d];
    q.xs = wsb + sp.xs_off[d];
    q.ys = wsb + sp.ys_off[d];
    q.xscale = (const double*)(wsb + sp.xsc_off[d]);
    q.yscale = (const double*)(wsb + sp.ysc_off[d]);
    q.part = (double*)(wsb + plan.part_off[d]);
    q.n = g.n[d];
    q.S = g.shifts[d];
    q.cn = g.periodic[d] ? g.cell_nodes[d] : 0;
    q.M = plan.M[d];
    q.N = plan.N[d];
    q.kchunk = plan.kchunk[d];
    q.ks = plan.ks[d];
    q.tiles_n = plan.tiles_n[d];
    q.block_begin = begin;
    begin += plan.blocks[d];
  }
  if (g_ev_start) TL_HIP(hipEventRecord(g_ev_start, stream));
  dim3 grid((unsigned)plan.total_blocks), blk(256);
  switch (S) {
    case 2: hipLaunchKernelGGL((contract_split_kernel<LowT, 2>), grid, blk, 0, stream, a); break;
    case 3: hipLaunchKernelGGL((contract_split_kernel<LowT, 3>), grid, blk, 0, stream, a); break;
    case 4: hipLaunchKernelGGL((contract_split_kernel<LowT, 4>), grid, blk, 0, stream, a); break;
    case 5: hipLaunchKernelGGL((contract_split_kernel<LowT, 5>), grid, blk, 0, stream, a); break;
    case 6: hipLaunchKernelGGL((contract_split_kernel<LowT, 6>), grid, blk, 0, stream, a); break;
    case 7: hipLaunchKernelGGL((contract_split_kernel<LowT, 7>), grid, blk, 0, stream, a); break;
    default: hipLaunchKernelGGL((contract_split_kernel<LowT, 8>), grid, blk, 0, stream, a); break;
  }
  TL_CHECK_LAUNCH();
  if (g_ev_stop) TL_HIP(hipEventRecord(g_ev_stop, stream));
  return TL_OK;
}

}  // namespace

size_t assemble_workspace_bytes(const Geometry& g, tl_precision prec, int n_slices) {
  if (g.mode != TL_MODE_PERIODIC) return 0;
  Plan plan = make_plan(g);
  if (!is_split(prec)) return plan.bytes;
  int S = n_slices > 0 ? n_slices : default_slices(prec);
  return make_split_plan(g, plan, S, plan.bytes).bytes;
}

tl_status assemble_periodic(const Geometry& g, const double* G, const double* AG,
                            const double* SG, const double* P, tl_precision prec, int n_slices,
                            double* H, double* S, void* ws, size_t ws_bytes, hipStream_t stream) {
  Plan plan = make_plan(g);
  const int nsl = is_split(prec) ? (n_slices > 0 ? n_slices : default_slices(prec)) : 0;
  if (is_split(prec) && (nsl < 2 || nsl > kMaxSlices)) {
    set_error("n_slices = %d outside [2, %d]", n_slices, kMaxSlices);
    return TL_EINVAL;
  }
  const size_t need = is_split(prec) ? make_split_plan(g, plan, nsl, plan.bytes).bytes : plan.bytes;
  if (ws == nullptr || ws_bytes < need) {
    set_error("assembly workspace: need %zu bytes, got %zu", need, ws_bytes);
    return TL_EWORKSPACE;
  }
  char* wsb = (char*)ws;
  ContractArgs a;
  a.m0 = g.m0;
  a.T = (int)g.pot_terms;
  int begin = 0;
  for (int d = 0; d < 3; ++d) {
    DimArgs& p = a.d[d];
    p.G = G + g.basis_off[d];
    p.AG = AG + g.basis_off[d];
    p.SG = SG + g.basis_off[d];
    p.P = P + g.pot_off[d];
    p.part = (double*)(wsb + plan.part_off[d]);
    p.n = g.n[d];
    p.S = g.shifts[d];
    p.cn = g.periodic[d] ? g.cell_nodes[d] : 0;
    p.M = plan.M[d];
    p.N = plan.N[d];
    p.kchunk = plan.kchunk[d];
    p.ks = plan.ks[d];
    p.tiles_n = plan.tiles_n[d];
    p.block_begin = begin;
    begin += plan.blocks[d];
  }
  if (prec == TL_SPLIT_BF16) {
    TL_TRY(launch_split<__bf16>(g, plan, make_split_plan(g, plan, nsl, plan.bytes), wsb, G, AG, SG,
                                P, nsl, stream));
  } else if (prec == TL_SPLIT_FP16) {
    TL_TRY(launch_split<_Float16>(g, plan, make_split_plan(g, plan, nsl, plan.bytes), wsb, G, AG,
                                  SG, P, nsl, stream));
  } else {
    if (g_ev_start) TL_HIP(hipEventRecord(g_ev_start, stream));
    if (prec == TL_FP32)
      hipLaunchKernelGGL(contract_f32_kernel, dim3((unsigned)plan.total_blocks), dim3(256), 0,
                         stream, a);
    else
      hipLaunchKernelGGL(contract_f64_kernel, dim3((unsigned)plan.total_blocks), dim3(256), 0,
                         stream, a);
    TL_CHECK_LAUNCH();
    if (g_ev_stop) TL_HIP(hipEventRecord(g_ev_stop, stream));
  }
  ReduceArgs ra;
  int64_t tot = 0;
  for (int d = 0; d < 3; ++d) {
    ra.part[d] = (const double*)(wsb + plan.part_off[d]);
    ra.C[d] = (double*)(wsb + plan.c_off[d]);
    ra.MN[d] = (int64_t)plan.M[d] * plan.N[d];
    ra.ks[d] = plan.ks[d];
    ra.begin[d] = tot;
    tot += ra.MN[d];
  }
  hipLaunchKernelGGL(reduce_partials_kernel, dim3((unsigned)ceil_div(tot, 256)), dim3(256), 0,
                     stream, ra, tot);
  TL_CHECK_LAUNCH();
  CombineArgs c;
  for (int d = 0; d < 3; ++d) {
    c.C[d] = (const double*)(wsb + plan.c_off[d]);
    c.S[d] = g.shifts[d];
    c.L[d] = g.L[d];
    c.periodic[d] = g.periodic[d];
    c.N[d] = plan.N[d];
  }
  c.m0 = g.m0;
  c.T = (int)g.pot_terms;
  c.H = H;
  c.Sm = S;
  int64_t total = g.block_elems;
  hipLaunchKernelGGL(combine_periodic_kernel, dim3((unsigned)ceil_div(total, 4)), dim3(256), 0,
                     stream, c, total);
  TL_CHECK_LAUNCH();
  return TL_OK;
}

}  // namespace tl

extern "C" tl_status tl_set_contraction_events(void* start_event, void* stop_event) {
  tl::clear_error();
  TL_REQUIRE((start_event == nullptr) == (stop_event == nullptr),
             "give both events or neither");
  tl::g_ev_start = (hipEvent_t)start_event;
  tl::g_ev_stop = (hipEvent_t)stop_event;
  return TL_OK;
}

extern "C" tl_status tl_assemble_workspace_bytes(const tl_system* sys, tl_precision prec,
                                                 int n_slices, size_t* bytes) {
  tl::clear_error();
  TL_REQUIRE(bytes != nullptr, "null output");
  tl::Geometry g;
  TL_TRY(tl::digest(sys, &g));
  *bytes = tl::assemble_workspace_bytes(g, prec, n_slices);
  return TL_OK;
}

extern "C" tl_status tl_assemble_core_hamiltonian_block(const tl_system* sys, const double* G_dev,
                                                        const double* AG_dev,
                                                        const double* SG_dev,
                                                        const double* P_dev, tl_precision prec,
                                                        int n_slices, double* H_dev,
                                                        double* S_dev, void* ws_dev,
                                                        size_t ws_bytes, void* stream) {
  tl::clear_error();
  tl::Geometry g;
  TL_TRY(tl::digest(sys, &g));
  TL_REQUIRE(G_dev && AG_dev && SG_dev && P_dev && H_dev && S_dev, "null array argument");
  TL_REQUIRE(prec >= TL_FP64 && prec <= TL_SPLIT_FP16, "unknown precision %d", (int)prec);
  if (g.mode == TL_MODE_PERIODIC)
    return tl::assemble_periodic(g, G_dev, AG_dev, SG_dev, P_dev, prec, n_slices, H_dev, S_dev,
                                 ws_dev, ws_bytes, (hipStream_t)stream);
  tl::set_error("box-mode assembly is not available yet");
  return TL_EUNSUPPORTED;
}
