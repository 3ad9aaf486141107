// Symmetric block-Toeplitz matrices (Sec. 2, Definition of the block Toeplitz
// class; Appendix eq. (block_SToepl)): A = BToepl_s{A_0, ..., A_{L-1}}, block
// (r, c) = A_{r-c} for r >= c and A_{c-r}^T for r < c.  The Remark on block
// Toeplitz matrices: A is the leading L x L block part of the symmetric
// 2L-block circulant C with first block column
//   C_k = A_k (k < L), C_L = 0, C_{2L-k} = A_k^T (0 < k < L),
// so Y = A X is the first L blocks of C [X; 0].  C is diagonalised by the
// block DFT over its 2L cells (Lemma 2.2, the Proposition on block-circulant
// diagonalisation): Xhat_j = sum_c w^(jc) X_c, Yhat_j = Chat_j Xhat_j,
// Y_c = (1 / 2L) sum_j w^(-jc) Yhat_j, w = exp(-2 pi i / 2L).  The inverse
// transform of a real result is taken with the forward transform of real
// data: with Yhat = R + i I, Y_c = (Re DFT(R)_c + Im DFT(I)_c) / 2L.  The
// power method for the largest eigenvalue in magnitude (the senior one) runs
// on this product.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>

#include "common.h"
#include "host_plans.h"

namespace tl {
namespace {

using namespace dev;

struct ToeplitzLayout {
  int L, L2, m0, nvec;
  int64_t Eb, Ev;  // entries per cell: blocks (m0 m0), vectors (m0 nvec)
  size_t off_chat, off_xt, off_xhat, off_r, off_f, off_tab[3], bytes;
  FftArgs fb, fx, fr;  // transforms of the blocks, of X, of [R; I]
};

tl_status layout(int L, int m0, int nvec, ToeplitzLayout* t, char* ws) {
  TL_REQUIRE(L >= 1 && L <= kFftPoints / 2, "L = %d outside [1, %d]", L, kFftPoints / 2);
  TL_REQUIRE(m0 >= 1 && m0 <= TL_MAX_M0, "m0 = %d outside [1, %d]", m0, TL_MAX_M0);
  TL_REQUIRE(nvec >= 1 && nvec <= 1024, "nvec = %d outside [1, 1024]", nvec);
  t->L = L;
  t->L2 = 2 * L;
  t->m0 = m0;
  t->nvec = nvec;
  t->Eb = (int64_t)m0 * m0;
  t->Ev = (int64_t)m0 * nvec;
  size_t o = 0;
  auto take = [&](size_t b) {
    size_t r = o;
    o += align_up(b, 256);
    return r;
  };
  t->off_chat = take(sizeof(double) * 2 * t->L2 * t->Eb);
  t->off_xt = take(sizeof(double) * t->L2 * std::max(t->Ev, t->Eb));  // also the embedded blocks
  t->off_xhat = take(sizeof(double) * 2 * t->L2 * t->Ev);
  t->off_r = take(sizeof(double) * 2 * t->L2 * t->Ev);
  t->off_f = take(sizeof(double) * 4 * t->L2 * t->Ev);
  const int Ls[3] = {t->L2, 1, 1};
  char* b = ws ? ws : nullptr;
  auto ptr = [&](size_t off) { return (double*)(b ? b + off : nullptr); };
  if (!plan_fft_cols(ptr(t->off_xt), ptr(t->off_chat), Ls, t->Eb, 1, &t->fb, 64) ||
      !plan_fft_cols(ptr(t->off_xt), ptr(t->off_xhat), Ls, t->Ev, 1, &t->fx, 64) ||
      !plan_fft_cols(ptr(t->off_r), ptr(t->off_f), Ls, t->Ev, 2, &t->fr, 64)) {
    set_error("no FFT plan for 2L = %d", t->L2);
    return TL_EUNSUPPORTED;
  }
  FftArgs* plans[3] = {&t->fb, &t->fx, &t->fr};
  for (int q = 0; q < 3; ++q) {
    t->off_tab[q] = take(fft_blue_table_bytes(*plans[q]));
    if (b) set_fft_blue_tables(plans[q], b + t->off_tab[q]);
  }
  t->bytes = o;
  return TL_OK;
}

struct EmbedArgs {
  const double* A;  // [L][m0][m0]
  double* Cb;       // [2L][m0][m0]
  int L, m0;
};

__global__ __launch_bounds__(256) void embed_kernel(EmbedArgs a) {
  const int64_t m2 = (int64_t)a.m0 * a.m0;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 2 * a.L * m2) return;
  const int k = (int)(idx / m2);
  const int e = (int)(idx - k * m2), mu = e / a.m0, nu = e - mu * a.m0;
  double v = 0.0;
  if (k < a.L)
    v = a.A[idx];
  else if (k > a.L)
    v = a.A[(int64_t)(2 * a.L - k) * m2 + (int64_t)nu * a.m0 + mu];  // A_{2L-k}^T
  a.Cb[idx] = v;
}

struct PadArgs {
  const double* X;  // [L][E]
  double* Xt;       // [2L][E]
  int L;
  int64_t E;
};

__global__ __launch_bounds__(256) void pad_kernel(PadArgs a) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 2 * a.L * a.E) return;
  a.Xt[idx] = idx < a.L * a.E ? a.X[idx] : 0.0;
}

struct MulArgs {
  const double* Chat;  // [2L][m0][m0] complex
  const double* Xhat;  // [2L][m0][nvec] complex
  double* R;           // [2][2L][m0][nvec] real: Re, Im of Chat_j Xhat_j
  int L2, m0, nvec;
};

__global__ __launch_bounds__(256) void mul_kernel(MulArgs a) {
  const int64_t Ev = (int64_t)a.m0 * a.nvec;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= a.L2 * Ev) return;
  const int j = (int)(idx / Ev);
  const int e = (int)(idx - j * Ev), mu = e / a.nvec, v = e - mu * a.nvec;
  const double* c = a.Chat + 2 * ((int64_t)j * a.m0 + mu) * a.m0;
  const double* x = a.Xhat + 2 * ((int64_t)j * Ev + v);
  double re = 0.0, im = 0.0;
  for (int nu = 0; nu < a.m0; ++nu) {
    const double cr = c[2 * nu], ci = c[2 * nu + 1];
    const double xr = x[2 * (int64_t)nu * a.nvec], xi = x[2 * (int64_t)nu * a.nvec + 1];
    re = fma(cr, xr, fma(-ci, xi, re));
    im = fma(cr, xi, fma(ci, xr, im));
  }
  a.R[idx] = re;
  a.R[a.L2 * Ev + idx] = im;
}

struct CombArgs {
  const double* F;  // [2][2L][E] complex: DFT(R), DFT(I)
  double* Y;        // [L][E]
  int L, L2;
  int64_t E;
};

__global__ __launch_bounds__(256) void comb_kernel(CombArgs a) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= a.L * a.E) return;
  const double fr = a.F[2 * idx];                              // Re DFT(R)_c
  const double fi = a.F[2 * ((int64_t)a.L2 * a.E + idx) + 1];  // Im DFT(I)_c
  a.Y[idx] = (fr + fi) / (double)a.L2;
}

// One power-method update on n = L m0 entries, one workgroup:
// lambda = (x . y) / (x . x), x <- y / |y|.
__global__ __launch_bounds__(1024) void power_update_kernel(double* x, const double* y, int n,
                                                            double* lambda) {
  __shared__ double red[3][16];
  double xy = 0.0, xx = 0.0, yy = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    const double xi = x[i], yi = y[i];
    xy = fma(xi, yi, xy);
    xx = fma(xi, xi, xx);
    yy = fma(yi, yi, yy);
  }
  xy = wave_sum_dpp(xy);
  xx = wave_sum_dpp(xx);
  yy = wave_sum_dpp(yy);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, nw = blockDim.x >> 6;
  if (lane == 0) {
    red[0][wave] = xy;
    red[1][wave] = xx;
    red[2][wave] = yy;
  }
  __syncthreads();
  double s[3] = {0.0, 0.0, 0.0};
  for (int w = 0; w < nw; ++w)
    for (int q = 0; q < 3; ++q) s[q] += red[q][w];
  __syncthreads();  // every thread has read the sums
  const double inv = s[2] > 0.0 ? 1.0 / sqrt(s[2]) : 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) x[i] = y[i] * inv;
  if (threadIdx.x == 0) *lambda = s[1] > 0.0 ? s[0] / s[1] : 0.0;
}

tl_status matvec(const ToeplitzLayout& t, char* ws, const double* X, double* Y,
                 hipStream_t stream) {
  const int64_t nx = 2 * (int64_t)t.L * t.Ev;
  hipLaunchKernelGGL(pad_kernel, dim3((unsigned)ceil_div(nx, 256)), dim3(256), 0, stream,
                     PadArgs{X, (double*)(ws + t.off_xt), t.L, t.Ev});
  TL_CHECK_LAUNCH();
  TL_TRY(launch_fft(t.fx, stream));
  hipLaunchKernelGGL(mul_kernel, dim3((unsigned)ceil_div(nx, 256)), dim3(256), 0, stream,
                     MulArgs{(const double*)(ws + t.off_chat), (const double*)(ws + t.off_xhat),
                             (double*)(ws + t.off_r), t.L2, t.m0, t.nvec});
  TL_CHECK_LAUNCH();
  TL_TRY(launch_fft(t.fr, stream));
  const int64_t ny = (int64_t)t.L * t.Ev;
  hipLaunchKernelGGL(comb_kernel, dim3((unsigned)ceil_div(ny, 256)), dim3(256), 0, stream,
                     CombArgs{(const double*)(ws + t.off_f), Y, t.L, t.L2, t.Ev});
  TL_CHECK_LAUNCH();
  return TL_OK;
}

// ===========================================================================
// Multilevel block-Toeplitz products (the Definition of the d-level class and
// the Remark's embedding at each level): A over L1 x L2 x L3 cells with block
// (r, c) = B(r - c), B given for every shift d in (-L, L)^3.  C over
// 2L1 x 2L2 x 2L3 cells, C_k = B(k') with k'_l = k_l (k_l < L_l), none
// (k_l = L_l), k_l - 2 L_l (k_l > L_l), is block circulant on that lattice and
// A X is its product with X padded by zeros, read on the first L cells (a
// level with L_l = 1 is not doubled); the transforms are 3D (each doubled
// length 7-smooth, at most 4096 embedded cells).

struct Toeplitz3Layout {
  int L[3], L2[3], m0, nvec, P;  // P = 8 L1 L2 L3 embedded cells
  int64_t Eb, Ev;
  size_t off_chat, off_xt, off_xhat, off_r, off_f, off_tab[3], bytes;
  FftArgs fb, fx, fr;
};

tl_status layout3(const int L[3], int m0, int nvec, Toeplitz3Layout* t, char* ws) {
  int P = 1;
  for (int d = 0; d < 3; ++d) {
    TL_REQUIRE(L[d] >= 1, "L[%d] = %d < 1", d, L[d]);
    t->L[d] = L[d];
    t->L2[d] = L[d] > 1 ? 2 * L[d] : 1;
    P *= t->L2[d];
    TL_REQUIRE(P <= kFftPoints, "embedded lattice of more than %d cells", kFftPoints);
  }
  TL_REQUIRE(m0 >= 1 && m0 <= TL_MAX_M0, "m0 = %d outside [1, %d]", m0, TL_MAX_M0);
  TL_REQUIRE(nvec >= 1 && nvec <= 1024, "nvec = %d outside [1, 1024]", nvec);
  t->P = P;
  t->m0 = m0;
  t->nvec = nvec;
  t->Eb = (int64_t)m0 * m0;
  t->Ev = (int64_t)m0 * nvec;
  size_t o = 0;
  auto take = [&](size_t b) {
    size_t r = o;
    o += align_up(b, 256);
    return r;
  };
  t->off_chat = take(sizeof(double) * 2 * P * t->Eb);
  t->off_xt = take(sizeof(double) * P * std::max(t->Ev, t->Eb));
  t->off_xhat = take(sizeof(double) * 2 * P * t->Ev);
  t->off_r = take(sizeof(double) * 2 * P * t->Ev);
  t->off_f = take(sizeof(double) * 4 * P * t->Ev);
  auto ptr = [&](size_t off) { return (double*)(ws ? ws + off : nullptr); };
  if (!plan_fft_cols(ptr(t->off_xt), ptr(t->off_chat), t->L2, t->Eb, 1, &t->fb, 64) ||
      !plan_fft_cols(ptr(t->off_xt), ptr(t->off_xhat), t->L2, t->Ev, 1, &t->fx, 64) ||
      !plan_fft_cols(ptr(t->off_r), ptr(t->off_f), t->L2, t->Ev, 2, &t->fr, 64)) {
    set_error("no FFT plan for the embedded lattice %d x %d x %d", t->L2[0], t->L2[1], t->L2[2]);
    return TL_EUNSUPPORTED;
  }
  FftArgs* plans[3] = {&t->fb, &t->fx, &t->fr};
  for (int q = 0; q < 3; ++q) {
    t->off_tab[q] = take(fft_blue_table_bytes(*plans[q]));
    if (ws) set_fft_blue_tables(plans[q], ws + t->off_tab[q]);
  }
  t->bytes = o;
  return TL_OK;
}

struct Embed3Args {
  const double* B;  // [2L1-1][2L2-1][2L3-1][m0][m0], shift d at d + L - 1
  double* Cb;       // [n1][n2][n3][m0][m0], n_l the embedded extents
  int L[3], n[3], m0;
  int64_t total;
};

__global__ __launch_bounds__(256) void embed3_kernel(Embed3Args a) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= a.total) return;
  const int64_t m2 = (int64_t)a.m0 * a.m0;
  const int64_t cell = idx / m2;
  const int e = (int)(idx - cell * m2);
  const int n3 = a.n[2], n2 = a.n[1];
  const int k3 = (int)(cell % n3), k2 = (int)((cell / n3) % n2), k1 = (int)(cell / (n3 * n2));
  const int k[3] = {k1, k2, k3};
  int src[3];
  bool zero = false;
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int s = k[d] < a.L[d] ? k[d] : k[d] - 2 * a.L[d];  // the shift this cell carries
    zero |= k[d] == a.L[d];
    src[d] = s + a.L[d] - 1;
  }
  double v = 0.0;
  if (!zero) {
    const int64_t b = ((int64_t)src[0] * (2 * a.L[1] - 1) + src[1]) * (2 * a.L[2] - 1) + src[2];
    v = a.B[b * m2 + e];
  }
  a.Cb[idx] = v;
}

struct Pad3Args {
  const double* X;  // [L1][L2][L3][E]
  double* Xt;       // [n1][n2][n3][E]
  int L[3], n[3];
  int64_t E, total;
};

__global__ __launch_bounds__(256) void pad3_kernel(Pad3Args a) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= a.total) return;
  const int64_t cell = idx / a.E;
  const int64_t e = idx - cell * a.E;
  const int n3 = a.n[2], n2 = a.n[1];
  const int k3 = (int)(cell % n3), k2 = (int)((cell / n3) % n2), k1 = (int)(cell / (n3 * n2));
  double v = 0.0;
  if (k1 < a.L[0] && k2 < a.L[1] && k3 < a.L[2])
    v = a.X[(((int64_t)k1 * a.L[1] + k2) * a.L[2] + k3) * a.E + e];
  a.Xt[idx] = v;
}

struct Comb3Args {
  const double* F;  // [2][P][E] complex: DFT(R), DFT(I) over the embedded lattice
  double* Y;        // [L1][L2][L3][E]
  int L[3], n[3], P;
  int64_t E, total;
};

__global__ __launch_bounds__(256) void comb3_kernel(Comb3Args a) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= a.total) return;
  const int64_t cell = idx / a.E;
  const int64_t e = idx - cell * a.E;
  const int r3 = (int)(cell % a.L[2]), r2 = (int)((cell / a.L[2]) % a.L[1]);
  const int r1 = (int)(cell / ((int64_t)a.L[2] * a.L[1]));
  const int64_t src = (((int64_t)r1 * a.n[1] + r2) * a.n[2] + r3) * a.E + e;
  const double fr = a.F[2 * src];
  const double fi = a.F[2 * ((int64_t)a.P * a.E + src) + 1];
  a.Y[idx] = (fr + fi) / (double)a.P;
}

tl_status matvec3(const Toeplitz3Layout& t, char* ws, const double* X, double* Y,
                  hipStream_t stream) {
  const int64_t nx = (int64_t)t.P * t.Ev;
  hipLaunchKernelGGL(pad3_kernel, dim3((unsigned)ceil_div(nx, 256)), dim3(256), 0, stream,
                     Pad3Args{X, (double*)(ws + t.off_xt), {t.L[0], t.L[1], t.L[2]},
                              {t.L2[0], t.L2[1], t.L2[2]}, t.Ev, nx});
  TL_CHECK_LAUNCH();
  TL_TRY(launch_fft(t.fx, stream));
  hipLaunchKernelGGL(mul_kernel, dim3((unsigned)ceil_div(nx, 256)), dim3(256), 0, stream,
                     MulArgs{(const double*)(ws + t.off_chat), (const double*)(ws + t.off_xhat),
                             (double*)(ws + t.off_r), t.P, t.m0, t.nvec});
  TL_CHECK_LAUNCH();
  TL_TRY(launch_fft(t.fr, stream));
  const int64_t ny = (int64_t)t.L[0] * t.L[1] * t.L[2] * t.Ev;
  hipLaunchKernelGGL(comb3_kernel, dim3((unsigned)ceil_div(ny, 256)), dim3(256), 0, stream,
                     Comb3Args{(const double*)(ws + t.off_f), Y, {t.L[0], t.L[1], t.L[2]},
                               {t.L2[0], t.L2[1], t.L2[2]}, t.P, t.Ev, ny});
  TL_CHECK_LAUNCH();
  return TL_OK;
}

// ===========================================================================
// Lowest eigenpairs of the symmetric-definite block-Toeplitz pencil
// (T_H, T_S): the iterative route the paper points to for open boxes whose
// full matrices are too large to diagonalise (Sec. 3.3, closing remark), on
// the fast product above.  The solver is LOBPCG (Knyazev, SIAM J. Sci.
// Comput. 23 (2001)): a block of nb vectors X, the preconditioned residuals
// W and the previous search directions P span the Rayleigh-Ritz basis of
// each step.  Choices of this implementation:
//   * preconditioner: the Strang block circulant of each matrix (first block
//     column A_0, ..., A_{L/2}, A_{L/2}^T..., A_1^T: the periodic matrix with
//     the same blocks, Lemma 2.2), shifted below the circulant pencil's
//     lowest eigenvalue and inverted through the block DFT over L cells:
//     W = F^-1 diag_j (Hhat_j - sigma Shat_j)^-1 F R;
//   * W is made T_S-orthogonal to X before its products are taken, and P
//     (with T_H P, T_S P) after; X itself is T_S-orthonormal, so only [W, P]
//     is orthonormalised in the T_S metric, by SVQB (Stathopoulos
//     and Wu, SIAM J. Sci. Comput. 23 (2002)): columns scaled to unit norm,
//     the Gram matrix diagonalised, directions with eigenvalue below 1e-8 of
//     the largest dropped (T_S-products of nearly dependent directions carry
//     too few digits for a Rayleigh quotient);
//   * the small eigenproblems (order <= 3 nb <= 64) are solved by cyclic
//     Jacobi in one workgroup's LDS;
//   * T_H X and T_S X are recomputed from X every 10 steps (the recurrences
//     that update them drift);
//   * soft locking: a wanted pair whose residual meets the tolerance keeps
//     its place in X but contributes no preconditioned residual.

constexpr int kLobMaxBasis = 64;  // 3 nb, padded
constexpr int kLobMaxNb = 21;
constexpr int kLobLd = kLobMaxBasis + 1;
constexpr double kLobDrop = 1e-8;
constexpr int kLobRefresh = 10;

// Strang circulant blocks of A (first block column), H and S stacked.
struct StrangArgs {
  const double* A[2];  // [L][m0][m0]
  double* out;         // [2][L][m0][m0]
  int L, m0;
};

__global__ __launch_bounds__(256) void strang_kernel(StrangArgs a) {
  const int64_t m2 = (int64_t)a.m0 * a.m0;
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 2 * a.L * m2) return;
  const int w = (int)(idx / (a.L * m2));
  const int64_t rest = idx - w * a.L * m2;
  const int k = (int)(rest / m2);
  const int e = (int)(rest - k * m2), mu = e / a.m0, nu = e - mu * a.m0;
  const double* A = a.A[w];
  double v;
  if (2 * k < a.L)
    v = A[(int64_t)k * m2 + e];
  else if (2 * k == a.L)
    v = 0.5 * (A[(int64_t)k * m2 + e] + A[(int64_t)k * m2 + (int64_t)nu * a.m0 + mu]);
  else
    v = A[(int64_t)(a.L - k) * m2 + (int64_t)nu * a.m0 + mu];  // A_{L-k}^T
  a.out[idx] = v;
}

// scal[0] = lowest eigenvalue over the k-blocks, scal[4] = the second
// smallest of the blocks' lowest eigenvalues, scal[3] = 1 if a block failed
// (not definite or not converged).
__global__ __launch_bounds__(256) void lmin_kernel(const double* evals, const int* info, int L,
                                                   int m0, double* scal) {
  __shared__ double lo1[256], lo2[256];
  __shared__ int bad[256];
  double a1 = INFINITY, a2 = INFINITY;  // smallest and second smallest block minimum
  int b = 0;
  for (int j = threadIdx.x; j < L; j += blockDim.x) {
    if (info[j] != 0) b = 1;
    double v = INFINITY;
    for (int i = 0; i < m0; ++i) {
      const double e = evals[(int64_t)j * m0 + i];
      if (e != e) b = 1;
      else v = fmin(v, e);
    }
    if (v < a1) {
      a2 = a1;
      a1 = v;
    } else {
      a2 = fmin(a2, v);
    }
  }
  lo1[threadIdx.x] = a1;
  lo2[threadIdx.x] = a2;
  bad[threadIdx.x] = b;
  __syncthreads();
  if (threadIdx.x == 0) {
    double m1 = INFINITY, m2 = INFINITY;
    int any = 0;
    for (int t = 0; t < (int)blockDim.x; ++t) {
      any |= bad[t];
      const double c1 = lo1[t], c2 = lo2[t];
      if (c1 < m1) {
        m2 = fmin(m1, c2);
        m1 = c1;
      } else {
        m2 = fmin(m2, c1);
      }
    }
    scal[0] = m1;
    scal[4] = m2;
    scal[3] = any ? 1.0 : 0.0;
  }
}

// scal[1], scal[2]: sum over k of (largest row sum + largest column sum of
// |A_k|) for H and S, a bound on the infinity norm of each Toeplitz matrix.
__global__ __launch_bounds__(256) void tnorm_kernel(const double* H, const double* S, int L,
                                                    int m0, double* scal) {
  __shared__ double red[2][4];
  double acc[2] = {0.0, 0.0};
  const int64_t m2 = (int64_t)m0 * m0;
  for (int k = threadIdx.x; k < L; k += blockDim.x) {
    for (int w = 0; w < 2; ++w) {
      const double* A = (w ? S : H) + k * m2;
      double rmax = 0.0, cmax = 0.0;
      for (int i = 0; i < m0; ++i) {
        double r = 0.0, c = 0.0;
        for (int j = 0; j < m0; ++j) {
          r += fabs(A[i * m0 + j]);
          c += fabs(A[j * m0 + i]);
        }
        rmax = fmax(rmax, r);
        cmax = fmax(cmax, c);
      }
      acc[w] += rmax + cmax;
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int w = 0; w < 2; ++w) {
    const double t = wave_sum_dpp(acc[w]);
    if (lane == 0) red[w][wave] = t;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    const int w = threadIdx.x;
    scal[1 + w] = red[w][0] + red[w][1] + red[w][2] + red[w][3];
  }
}

// Strang block circulant of a multilevel Toeplitz matrix over L1 x L2 x L3
// cells: c_k = B(k') with k'_l = k_l (2 k_l < L_l), k_l - L_l (2 k_l > L_l)
// and the mean of both at 2 k_l = L_l, for H and S.
struct Strang3Args {
  const double* B[2];  // [2L1-1][2L2-1][2L3-1][m0][m0]
  double* out;         // [2][L1 L2 L3][m0][m0]
  int L[3], m0;
  int64_t total;
};

__global__ __launch_bounds__(256) void strang3_kernel(Strang3Args a) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= a.total) return;
  const int64_t m2 = (int64_t)a.m0 * a.m0;
  const int64_t cells = (int64_t)a.L[0] * a.L[1] * a.L[2];
  const int w = (int)(idx / (cells * m2));
  const int64_t rest = idx - w * cells * m2;
  const int64_t cell = rest / m2;
  const int e = (int)(rest - cell * m2);
  const int k3 = (int)(cell % a.L[2]), k2 = (int)((cell / a.L[2]) % a.L[1]);
  const int k1 = (int)(cell / ((int64_t)a.L[2] * a.L[1]));
  const int k[3] = {k1, k2, k3};
  int c0[3], c1[3], nc[3];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    const int twice = 2 * k[d];
    c0[d] = twice < a.L[d] ? k[d] : k[d] - a.L[d];
    c1[d] = k[d];
    nc[d] = twice == a.L[d] ? 2 : 1;
  }
  const double* B = a.B[w];
  double v = 0.0;
  for (int i1 = 0; i1 < nc[0]; ++i1)
    for (int i2 = 0; i2 < nc[1]; ++i2)
      for (int i3 = 0; i3 < nc[2]; ++i3) {
        const int s1 = (i1 ? c1[0] : c0[0]) + a.L[0] - 1;
        const int s2 = (i2 ? c1[1] : c0[1]) + a.L[1] - 1;
        const int s3 = (i3 ? c1[2] : c0[2]) + a.L[2] - 1;
        const int64_t b = ((int64_t)s1 * (2 * a.L[1] - 1) + s2) * (2 * a.L[2] - 1) + s3;
        v += B[b * m2 + e];
      }
  a.out[idx] = v / (double)(nc[0] * nc[1] * nc[2]);
}

// scal[1], scal[2]: sum over all shifts of the largest row sum of |B(d)|,
// the infinity norm bound of the multilevel matrices H and S.
__global__ __launch_bounds__(256) void tnorm3_kernel(const double* H, const double* S, int nblk,
                                                     int m0, double* scal) {
  __shared__ double red[2][4];
  double acc[2] = {0.0, 0.0};
  const int64_t m2 = (int64_t)m0 * m0;
  for (int k = threadIdx.x; k < nblk; k += blockDim.x) {
    for (int w = 0; w < 2; ++w) {
      const double* A = (w ? S : H) + k * m2;
      double rmax = 0.0;
      for (int i = 0; i < m0; ++i) {
        double r = 0.0;
        for (int j = 0; j < m0; ++j) r += fabs(A[i * m0 + j]);
        rmax = fmax(rmax, r);
      }
      acc[w] += rmax;
    }
  }
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  for (int w = 0; w < 2; ++w) {
    const double t = wave_sum_dpp(acc[w]);
    if (lane == 0) red[w][wave] = t;
  }
  __syncthreads();
  if (threadIdx.x < 2) {
    const int w = threadIdx.x;
    scal[1 + w] = red[w][0] + red[w][1] + red[w][2] + red[w][3];
  }
}

// Minv_j = (Hhat_j - sigma Shat_j)^-1 by complex Cholesky, one thread per j
// (Lf: the factor, workspace).  info[j] = 1 + the failing pivot, else 0.
__global__ __launch_bounds__(64) void minv_kernel(const double* hat, int L, int m0, double sigma,
                                                  double* Lf, double* Minv, int* info) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= L) return;
  const int64_t m2 = (int64_t)m0 * m0;
  const double* Hh = hat + 2 * j * m2;
  const double* Sh = hat + 2 * ((int64_t)L + j) * m2;
  double* F = Lf + 2 * j * m2;
  double* X = Minv + 2 * j * m2;
  for (int64_t e = 0; e < m2; ++e) {
    F[2 * e] = Hh[2 * e] - sigma * Sh[2 * e];
    F[2 * e + 1] = Hh[2 * e + 1] - sigma * Sh[2 * e + 1];
  }
  // lower factor in place: F = L L^H
  for (int c = 0; c < m0; ++c) {
    double d = F[2 * (c * m0 + c)];
    for (int k = 0; k < c; ++k) {
      const double re = F[2 * (c * m0 + k)], im = F[2 * (c * m0 + k) + 1];
      d -= re * re + im * im;
    }
    if (!(d > 0.0)) {
      info[j] = 1 + c;
      return;
    }
    d = sqrt(d);
    F[2 * (c * m0 + c)] = d;
    F[2 * (c * m0 + c) + 1] = 0.0;
    for (int r = c + 1; r < m0; ++r) {
      double re = F[2 * (r * m0 + c)], im = F[2 * (r * m0 + c) + 1];
      for (int k = 0; k < c; ++k) {  // -= L[r][k] conj(L[c][k])
        const double ar = F[2 * (r * m0 + k)], ai = F[2 * (r * m0 + k) + 1];
        const double br = F[2 * (c * m0 + k)], bi = F[2 * (c * m0 + k) + 1];
        re -= ar * br + ai * bi;
        im -= ai * br - ar * bi;
      }
      F[2 * (r * m0 + c)] = re / d;
      F[2 * (r * m0 + c) + 1] = im / d;
    }
  }
  // column e of the inverse: L y = e_e, then L^H x = y (x stored in place)
  for (int e = 0; e < m0; ++e) {
    for (int r = 0; r < m0; ++r) {
      double re = r == e ? 1.0 : 0.0, im = 0.0;
      for (int k = 0; k < r; ++k) {
        const double ar = F[2 * (r * m0 + k)], ai = F[2 * (r * m0 + k) + 1];
        const double yr = X[2 * (k * m0 + e)], yi = X[2 * (k * m0 + e) + 1];
        re -= ar * yr - ai * yi;
        im -= ar * yi + ai * yr;
      }
      const double d = F[2 * (r * m0 + r)];
      X[2 * (r * m0 + e)] = re / d;
      X[2 * (r * m0 + e) + 1] = im / d;
    }
    for (int r = m0 - 1; r >= 0; --r) {
      double re = X[2 * (r * m0 + e)], im = X[2 * (r * m0 + e) + 1];
      for (int k = r + 1; k < m0; ++k) {  // -= conj(L[k][r]) x_k
        const double ar = F[2 * (k * m0 + r)], ai = -F[2 * (k * m0 + r) + 1];
        const double xr = X[2 * (k * m0 + e)], xi = X[2 * (k * m0 + e) + 1];
        re -= ar * xr - ai * xi;
        im -= ar * xi + ai * xr;
      }
      const double d = F[2 * (r * m0 + r)];
      X[2 * (r * m0 + e)] = re / d;
      X[2 * (r * m0 + e) + 1] = im / d;
    }
  }
  info[j] = 0;
}

// Start block: entries uniform in (-1, 1) from splitmix64 of (seed, index).
__global__ __launch_bounds__(256) void lob_rand_kernel(double* X, int64_t n, uint64_t seed) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  uint64_t z = seed + 0x9E3779B97F4A7C15ull * (uint64_t)(i + 1);
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  z ^= z >> 31;
  X[i] = (double)(z >> 11) * (2.0 / 9007199254740992.0) - 1.0;
}

// Partial Gram matrices over a chunk of rows: part[chunk][s][a][b] =
// sum_rows V[row][a] U_s[row][b], with V = [V_0 | V_1 | V_2] (nb columns each)
// and U_s likewise, a, b < nblk nb <= 64.
struct GramArgs {
  const double* V[3];
  const double* U[2][3];
  int nblk, nsets, nb;
  int64_t N;
  int chunk_rows;
  double* part;
};

__global__ __launch_bounds__(256) void lob_gram_kernel(GramArgs g) {
  __shared__ double Vs[32][kLobLd];
  __shared__ double Us[2][32][kLobLd];
  const int tid = threadIdx.x, a0 = (tid >> 4) * 4, b0 = (tid & 15) * 4;
  const int n = g.nblk * g.nb;
  const int64_t r0 = (int64_t)blockIdx.x * g.chunk_rows;
  const int64_t r1 = min(g.N, r0 + g.chunk_rows);
  double acc[2][4][4];
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[s][i][j] = 0.0;
  for (int64_t rb = r0; rb < r1; rb += 32) {
    for (int e = tid; e < 32 * kLobMaxBasis; e += 256) {
      const int rr = e >> 6, c = e & 63;
      const int64_t row = rb + rr;
      const bool ok = row < r1 && c < n;
      const int blk = ok ? c / g.nb : 0, cc = c - blk * g.nb;
      const int64_t off = row * g.nb + cc;
      Vs[rr][c] = ok ? g.V[blk][off] : 0.0;
      Us[0][rr][c] = ok ? g.U[0][blk][off] : 0.0;
      Us[1][rr][c] = ok && g.nsets > 1 ? g.U[1][blk][off] : 0.0;
    }
    __syncthreads();
    for (int rr = 0; rr < 32; ++rr) {
      double va[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) va[i] = Vs[rr][a0 + i];
#pragma unroll
      for (int s = 0; s < 2; ++s) {
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          const double ub = Us[s][rr][b0 + j];
#pragma unroll
          for (int i = 0; i < 4; ++i) acc[s][i][j] = fma(va[i], ub, acc[s][i][j]);
        }
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    if (s >= g.nsets) break;
    double* P = g.part + ((int64_t)blockIdx.x * 2 + s) * kLobMaxBasis * kLobMaxBasis;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) P[(a0 + i) * kLobMaxBasis + b0 + j] = acc[s][i][j];
  }
}

// gram[s][a][b] = sum over chunks, in chunk order.
__global__ __launch_bounds__(256) void lob_gram_reduce_kernel(const double* part, int chunks,
                                                              int nsets, double* gram) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  const int per = kLobMaxBasis * kLobMaxBasis;
  if (e >= nsets * per) return;
  const int s = e / per, r = e - s * per;
  double v = 0.0;
  for (int c = 0; c < chunks; ++c) v += part[((int64_t)c * 2 + s) * per + r];
  gram[e] = v;
}

// Cyclic Jacobi on the symmetric n x n matrix A (LDS, row stride kLobLd),
// eigenvectors accumulated into V (columns); parallel round-robin ordering,
// n / 2 disjoint rotations per step.  kLobThreads threads: in the update
// phases thread t applies pair t / 32 to rows (then columns) t % 32 and
// t % 32 + 32.  On return A's diagonal holds the eigenvalues.
constexpr int kLobThreads = 1024;

__device__ void jacobi_lds(double (*A)[kLobLd], double (*V)[kLobLd], int n, double* rot,
                           double* red, int* rotated, int* sweeps) {
  const int tid = threadIdx.x;
  const int ne = n + (n & 1);
  const int npair = ne / 2;
  const int pi = tid >> 5, k0 = tid & 31;
  if (tid == 0) *sweeps = 0;
  for (int e = tid; e < n * n; e += blockDim.x) {
    const int i = e / n, j = e - i * n;
    V[i][j] = i == j ? 1.0 : 0.0;
  }
  __syncthreads();
  for (int sweep = 0; sweep < 30; ++sweep) {
    // off-diagonal and total squared norms
    double off = 0.0, tot = 0.0;
    for (int e = tid; e < n * n; e += blockDim.x) {
      const int i = e / n, j = e - i * n;
      const double v = A[i][j] * A[i][j];
      tot += v;
      if (i != j) off += v;
    }
    off = wave_sum_dpp(off);
    tot = wave_sum_dpp(tot);
    const int lane = tid & 63, wave = tid >> 6, nw = blockDim.x >> 6;
    if (lane == 0) {
      red[wave] = off;
      red[16 + wave] = tot;
    }
    __syncthreads();
    double offs = 0.0, tots = 0.0;
    for (int w = 0; w < nw; ++w) {
      offs += red[w];
      tots += red[16 + w];
    }
    const bool any_rot = sweep == 0 || *rotated != 0;
    __syncthreads();
    // stop once a sweep rotated nothing (every |a_pq| at most 1e-16 of
    // sqrt|a_pp a_qq|: eigenvectors to high relative accuracy), or the
    // off-diagonal part is below 1e-18 of the Frobenius norm
    if (!any_rot || !(offs > 1e-36 * tots) || ne < 2) break;
    if (tid == 0) {
      *sweeps = sweep + 1;
      *rotated = 0;
    }
    __syncthreads();
    for (int step = 0; step < ne - 1; ++step) {
      if (tid < npair) {
        const int i = tid;
        const int p = i == 0 ? 0 : ((i + step - 1) % (ne - 1)) + 1;
        const int q = ((ne - 1 - i + step - 1) % (ne - 1)) + 1;
        double c = 1.0, sn = 0.0;
        if (p < n && q < n) {
          const double apq = A[p][q];
          if (fabs(apq) > 1e-300 && fabs(apq) > 1e-16 * sqrt(fabs(A[p][p] * A[q][q]))) {
            const double tau = (A[q][q] - A[p][p]) / (2.0 * apq);
            const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
            c = 1.0 / sqrt(1.0 + t * t);
            sn = t * c;
            *rotated = 1;
          }
        }
        rot[4 * i] = (double)p;
        rot[4 * i + 1] = (double)q;
        rot[4 * i + 2] = c;
        rot[4 * i + 3] = sn;
      }
      __syncthreads();
      int p = 0, q = 0;
      double c = 1.0, sn = 0.0;
      if (pi < npair) {
        p = (int)rot[4 * pi];
        q = (int)rot[4 * pi + 1];
        c = rot[4 * pi + 2];
        sn = rot[4 * pi + 3];
      }
      const bool act = pi < npair && p < n && q < n && sn != 0.0;
      // rows p, q of J^T A
      if (act) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int k = k0 + 32 * h;
          if (k < n) {
            const double ap = A[p][k], aq = A[q][k];
            A[p][k] = c * ap - sn * aq;
            A[q][k] = sn * ap + c * aq;
          }
        }
      }
      __syncthreads();
      // columns p, q of (J^T A) J and of V J
      if (act) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          const int k = k0 + 32 * h;
          if (k < n) {
            const double ap = A[k][p], aq = A[k][q];
            A[k][p] = c * ap - sn * aq;
            A[k][q] = sn * ap + c * aq;
            const double vp = V[k][p], vq = V[k][q];
            V[k][p] = c * vp - sn * vq;
            V[k][q] = sn * vp + c * vq;
          }
        }
      }
      __syncthreads();
    }
  }
}

// Rayleigh-Ritz on the basis of n columns: gram[0] = V^T T_H V, gram[1] =
// V^T T_S V, the first nfix columns already T_S-orthonormal and T_S-orthogonal
// to the rest.  SVQB of the trailing n - nfix columns, then the lowest nb
// eigenpairs of the projected T_H.  Out: Y (n x nb, row stride nb) with
// X_new = V Y, lam (nb, ascending), info = {kept rank r (r < nb: failure),
// Jacobi sweeps of the two solves}.
__global__ __launch_bounds__(kLobThreads) void lob_small_kernel(const double* gram, int n,
                                                                int nfix, int nb, double* Y,
                                                                double* lam, int* info) {
  extern __shared__ double lds[];
  double(*GA)[kLobLd] = (double(*)[kLobLd])lds;
  double(*GB)[kLobLd] = GA + kLobMaxBasis;
  double(*Q)[kLobLd] = GB + kLobMaxBasis;
  double(*T)[kLobLd] = Q + kLobMaxBasis;
  __shared__ double D[kLobMaxBasis], th[kLobMaxBasis], rot[4 * kLobMaxBasis / 2], red[32];
  __shared__ int inv_idx[kLobMaxBasis], perm[kLobMaxBasis];
  __shared__ int r_sh, rotated, sw1, sw2;
  const int tid = threadIdx.x;
  const int m = n - nfix;  // columns orthonormalised here
  const double* gA = gram;
  const double* gB = gram + kLobMaxBasis * kLobMaxBasis;
  for (int e = tid; e < n * n; e += blockDim.x) {
    const int i = e / n, j = e - i * n;
    GA[i][j] = 0.5 * (gA[i * kLobMaxBasis + j] + gA[j * kLobMaxBasis + i]);
    GB[i][j] = 0.5 * (gB[i * kLobMaxBasis + j] + gB[j * kLobMaxBasis + i]);
  }
  __syncthreads();
  if (tid < m) {
    const double g = GB[nfix + tid][nfix + tid];
    D[tid] = g > 0.0 ? 1.0 / sqrt(g) : 0.0;
  }
  __syncthreads();
  for (int e = tid; e < m * m; e += blockDim.x) {
    const int i = e / m, j = e - i * m;
    T[i][j] = D[i] * GB[nfix + i][nfix + j] * D[j];
  }
  __syncthreads();
  jacobi_lds(T, Q, m, rot, red, &rotated, &sw1);
  if (tid < m) th[tid] = T[tid][tid];
  __syncthreads();
  double tmax = 0.0;
  for (int i = 0; i < m; ++i) tmax = fmax(tmax, th[i]);
  if (tid == 0) {
    int c = 0;
    for (int k = 0; k < m; ++k)
      if (th[k] > kLobDrop * tmax) inv_idx[c++] = k;  // kept column c <- eigenvector k
    r_sh = nfix + c;
  }
  __syncthreads();
  const int r = r_sh;
  // M (n x r) into T: identity on the first nfix columns, D Q_keep theta^-1/2 below
  for (int e = tid; e < n * r; e += blockDim.x) {
    const int i = e / r, c = e - i * r;
    double v;
    if (i < nfix)
      v = c == i ? 1.0 : 0.0;
    else if (c < nfix)
      v = 0.0;
    else {
      const int k = inv_idx[c - nfix];
      v = D[i - nfix] * Q[i - nfix][k] / sqrt(th[k]);
    }
    T[i][c] = v;
  }
  __syncthreads();
  // Q = GA M (n x r)
  for (int e = tid; e < n * r; e += blockDim.x) {
    const int i = e / r, c = e - i * r;
    double v = 0.0;
    for (int k = 0; k < n; ++k) v = fma(GA[i][k], T[k][c], v);
    Q[i][c] = v;
  }
  __syncthreads();
  // GB = M^T GA M (r x r), symmetrised
  for (int e = tid; e < r * r; e += blockDim.x) {
    const int a = e / r, b = e - a * r;
    double v = 0.0, w = 0.0;
    for (int k = 0; k < n; ++k) {
      v = fma(T[k][a], Q[k][b], v);
      w = fma(T[k][b], Q[k][a], w);
    }
    GB[a][b] = 0.5 * (v + w);
  }
  __syncthreads();
  jacobi_lds(GB, GA, r, rot, red, &rotated, &sw2);  // eigenvectors into GA
  if (tid < r) {
    const double v = GB[tid][tid];
    int rank = 0;
    for (int i = 0; i < r; ++i) {
      const double u = GB[i][i];
      rank += (u < v) || (u == v && i < tid);
    }
    perm[rank] = tid;
  }
  __syncthreads();
  if (tid < nb && tid < r) lam[tid] = GB[perm[tid]][perm[tid]];
  // Y = M C[:, perm[:nb]]
  for (int e = tid; e < n * nb; e += blockDim.x) {
    const int i = e / nb, j = e - i * nb;
    double v = 0.0;
    if (j < r) {
      const int c = perm[j];
      for (int k = 0; k < r; ++k) v = fma(T[i][k], GA[k][c], v);
    }
    Y[i * nb + j] = v;
  }
  if (tid == 0) {
    info[0] = r;
    info[1] = sw1;
    info[2] = sw2;
  }
}

// out_f = beta out_f + alpha sum_b in_f[b] Y_b (+ add_f), f = blockIdx.y:
// N x nb tall-skinny blocks times nb x nb pieces of Y (row stride ldy).
struct TsArgs {
  const double* in[3][3];
  const double* Y[3];
  const double* add[3];
  double* out[3];
  int nin, nb, ldy;
  int64_t N;
  double alpha, beta;
};

__global__ __launch_bounds__(256) void lob_ts_kernel(TsArgs a) {
  const int f = blockIdx.y;
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= a.N * a.nb) return;
  const int64_t row = e / a.nb;
  const int j = (int)(e - row * a.nb);
  double v = 0.0;
  for (int b = 0; b < a.nin; ++b) {
    const double* x = a.in[f][b] + row * a.nb;
    const double* y = a.Y[b] + j;
    for (int i = 0; i < a.nb; ++i) v = fma(x[i], y[(int64_t)i * a.ldy], v);
  }
  v *= a.alpha;
  if (a.add[f]) v += a.add[f][e];
  double* o = a.out[f];
  o[e] = a.beta != 0.0 ? fma(a.beta, o[e], v) : v;
}

// R = AX - BX diag(lam)
__global__ __launch_bounds__(256) void lob_resid_kernel(const double* AX, const double* BX,
                                                        const double* lam, double* R, int64_t N,
                                                        int nb) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N * nb) return;
  const int j = (int)(e % nb);
  R[e] = fma(-lam[j], BX[e], AX[e]);
}

// norms[j] = |R_j|^2, norms[nb + j] = |X_j|^2, one workgroup per column.
__global__ __launch_bounds__(256) void lob_colnorm_kernel(const double* R, const double* X,
                                                          int64_t N, int nb, double* norms) {
  __shared__ double red[2][4];
  const int j = blockIdx.x;
  double r = 0.0, x = 0.0;
  for (int64_t i = threadIdx.x; i < N; i += blockDim.x) {
    const double a = R[i * nb + j], b = X[i * nb + j];
    r = fma(a, a, r);
    x = fma(b, b, x);
  }
  r = wave_sum_dpp(r);
  x = wave_sum_dpp(x);
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  if (lane == 0) {
    red[0][wave] = r;
    red[1][wave] = x;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    norms[j] = red[0][0] + red[0][1] + red[0][2] + red[0][3];
    norms[nb + j] = red[1][0] + red[1][1] + red[1][2] + red[1][3];
  }
}

// W[row][j] *= mask[j]: the residuals of locked columns are not expanded
__global__ __launch_bounds__(256) void lob_mask_kernel(double* W, const double* mask, int64_t N,
                                                       int nb) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N * nb) return;
  W[e] *= mask[e % nb];
}

// dst[row][j] = src[row][j] for j < nev (row strides nev and nb)
__global__ __launch_bounds__(256) void lob_cols_kernel(const double* src, double* dst, int64_t N,
                                                       int nb, int nev) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N * nev) return;
  const int64_t row = e / nev;
  dst[e] = src[row * nb + (e - row * nev)];
}

enum LobVec {
  kX, kAX, kBX, kW, kAW, kBW, kP, kAP, kBP, kX2, kAX2, kBX2, kP2, kAP2, kBP2, kBest, kNVec
};

struct LobLayout {
  int Lv[3], cells, m0, nb;
  bool three;  // operators are multilevel products (blocks for every shift)
  int64_t N, Ev;
  ToeplitzLayout tH, tS;
  Toeplitz3Layout tH3, tS3;
  size_t off_tH, off_tS;
  FftArgs fblk, fr, fz;
  size_t off_strang, off_hat, off_evals, off_info, off_lf, off_minv, off_rhat, off_z, off_f;
  size_t off_tab[3];
  size_t off_vec[kNVec];
  size_t off_part, off_gram, off_y, off_lam, off_sinfo, off_norms, off_scal, off_mask;
  size_t off_lambest;
  int chunks, chunk_rows;
  size_t bytes;
};

tl_status lob_layout(const int Lv[3], bool three, int m0, int nb, LobLayout* t, char* ws) {
  TL_REQUIRE(nb >= 1 && nb <= kLobMaxNb, "nb = %d outside [1, %d]", nb, kLobMaxNb);
  TL_REQUIRE(m0 >= 1 && m0 <= TL_MAX_M0, "m0 = %d outside [1, %d]", m0, TL_MAX_M0);
  if (!three) TL_REQUIRE(Lv[0] >= 1 && Lv[0] <= kFftPoints / 2, "L = %d outside [1, %d]", Lv[0],
                         kFftPoints / 2);
  t->three = three;
  t->cells = 1;
  for (int d = 0; d < 3; ++d) {
    t->Lv[d] = Lv[d];
    t->cells *= Lv[d];
  }
  const int cells = t->cells;
  t->m0 = m0;
  t->nb = nb;
  t->N = (int64_t)cells * m0;
  t->Ev = (int64_t)m0 * nb;
  size_t o = 0;
  auto take = [&](size_t b) {
    size_t r = o;
    o += align_up(b, 256);
    return r;
  };
  if (three) {
    TL_TRY(layout3(Lv, m0, nb, &t->tH3, nullptr));
    t->off_tH = take(t->tH3.bytes);
    t->off_tS = take(t->tH3.bytes);
    if (ws) {
      TL_TRY(layout3(Lv, m0, nb, &t->tH3, ws + t->off_tH));
      TL_TRY(layout3(Lv, m0, nb, &t->tS3, ws + t->off_tS));
    } else {
      t->tS3 = t->tH3;
    }
  } else {
    TL_TRY(layout(Lv[0], m0, nb, &t->tH, nullptr));
    t->off_tH = take(t->tH.bytes);
    t->off_tS = take(t->tH.bytes);
    if (ws) {
      TL_TRY(layout(Lv[0], m0, nb, &t->tH, ws + t->off_tH));
      TL_TRY(layout(Lv[0], m0, nb, &t->tS, ws + t->off_tS));
    } else {
      t->tS = t->tH;
    }
  }
  const int64_t m2 = (int64_t)m0 * m0;
  t->off_strang = take(sizeof(double) * 2 * cells * m2);
  t->off_hat = take(sizeof(double) * 4 * cells * m2);
  t->off_evals = take(sizeof(double) * cells * m0);
  t->off_info = take(sizeof(int) * cells);
  t->off_lf = take(sizeof(double) * 2 * cells * m2);
  t->off_minv = take(sizeof(double) * 2 * cells * m2);
  t->off_rhat = take(sizeof(double) * 2 * cells * t->Ev);
  t->off_z = take(sizeof(double) * 2 * cells * t->Ev);
  t->off_f = take(sizeof(double) * 4 * cells * t->Ev);
  for (int v = 0; v < kNVec; ++v) t->off_vec[v] = take(sizeof(double) * t->N * nb);
  t->chunk_rows = (int)std::max<int64_t>(32, align_up((size_t)ceil_div(t->N, 64), 32));
  t->chunks = (int)ceil_div(t->N, t->chunk_rows);
  t->off_part = take(sizeof(double) * t->chunks * 2 * kLobMaxBasis * kLobMaxBasis);
  t->off_gram = take(sizeof(double) * 2 * kLobMaxBasis * kLobMaxBasis);
  t->off_y = take(sizeof(double) * kLobMaxBasis * kLobMaxNb);
  t->off_lam = take(sizeof(double) * kLobMaxNb);
  t->off_sinfo = take(sizeof(int) * 4);
  t->off_norms = take(sizeof(double) * 2 * kLobMaxNb);
  t->off_scal = take(sizeof(double) * 8);
  t->off_mask = take(sizeof(double) * kLobMaxNb);
  t->off_lambest = take(sizeof(double) * kLobMaxNb);
  auto ptr = [&](size_t off) { return (double*)(ws ? ws + off : nullptr); };
  if (!plan_fft_cols(ptr(t->off_strang), ptr(t->off_hat), t->Lv, m2, 2, &t->fblk, 64) ||
      !plan_fft_cols(ptr(t->off_vec[kW]), ptr(t->off_rhat), t->Lv, t->Ev, 1, &t->fr, 64) ||
      !plan_fft_cols(ptr(t->off_z), ptr(t->off_f), t->Lv, t->Ev, 2, &t->fz, 64)) {
    set_error("no FFT plan for the lattice %d x %d x %d", Lv[0], Lv[1], Lv[2]);
    return TL_EUNSUPPORTED;
  }
  FftArgs* plans[3] = {&t->fblk, &t->fr, &t->fz};
  for (int q = 0; q < 3; ++q) {
    t->off_tab[q] = take(fft_blue_table_bytes(*plans[q]));
    if (ws) set_fft_blue_tables(plans[q], ws + t->off_tab[q]);
  }
  t->bytes = o;
  return TL_OK;
}

}  // namespace

tl_status batched_heigh(const double* H, const double* S, int count, int m, double* evals,
                        double* evecs, int* info, hipStream_t stream);

namespace {

tl_status lob_read(const void* dev, void* host, size_t bytes, hipStream_t st) {
  TL_HIP(hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, st));
  TL_HIP(hipStreamSynchronize(st));
  return TL_OK;
}

// Host driver of the solver; every step is a kernel, the host only reads the
// residual norms, the Ritz values and the basis rank to steer the iteration.
class Lobpcg {
 public:
  Lobpcg(const LobLayout& t, char* ws, hipStream_t st) : t_(t), ws_(ws), st_(st) {
    for (int i = 0; i < kNVec; ++i) cur_[i] = i;
  }
  double* v(int logical) const { return (double*)(ws_ + t_.off_vec[cur_[logical]]); }
  double* at(size_t off) const { return (double*)(ws_ + off); }

  tl_status products(int src, int dA, int dB) {
    if (t_.three) {
      TL_TRY(matvec3(t_.tH3, ws_ + t_.off_tH, v(src), v(dA), st_));
      return matvec3(t_.tS3, ws_ + t_.off_tS, v(src), v(dB), st_);
    }
    TL_TRY(matvec(t_.tH, ws_ + t_.off_tH, v(src), v(dA), st_));
    return matvec(t_.tS, ws_ + t_.off_tS, v(src), v(dB), st_);
  }
  // gram[s] = [V_0 | ...]^T [U_s0 | ...]; us1 null: one set
  tl_status gram(const int* vb, const int* us0, const int* us1, int nblk) {
    GramArgs g;
    std::memset(&g, 0, sizeof(g));
    g.nblk = nblk;
    g.nsets = us1 ? 2 : 1;
    g.nb = t_.nb;
    g.N = t_.N;
    g.chunk_rows = t_.chunk_rows;
    g.part = at(t_.off_part);
    for (int b = 0; b < nblk; ++b) {
      g.V[b] = v(vb[b]);
      g.U[0][b] = v(us0[b]);
      if (us1) g.U[1][b] = v(us1[b]);
    }
    hipLaunchKernelGGL(lob_gram_kernel, dim3((unsigned)t_.chunks), dim3(256), 0, st_, g);
    TL_CHECK_LAUNCH();
    const int tot = g.nsets * kLobMaxBasis * kLobMaxBasis;
    hipLaunchKernelGGL(lob_gram_reduce_kernel, dim3((unsigned)ceil_div(tot, 256)), dim3(256), 0,
                       st_, (const double*)at(t_.off_part), t_.chunks, g.nsets, at(t_.off_gram));
    TL_CHECK_LAUNCH();
    return TL_OK;
  }
  // Rayleigh-Ritz on [X | W | P][0..nblk): Y, lam, rank check
  tl_status rayleigh_ritz(int nblk) {
    const int vb[3] = {kX, kW, kP}, ua[3] = {kAX, kAW, kAP}, ub[3] = {kBX, kBW, kBP};
    TL_TRY(gram(vb, ua, ub, nblk));
    const size_t lds = sizeof(double) * 4 * kLobMaxBasis * kLobLd;
    // X is T_S-orthonormal after the first step, and W and P are projected off it
    const int nfix = nblk > 1 ? t_.nb : 0;
    hipLaunchKernelGGL(lob_small_kernel, dim3(1), dim3(kLobThreads), lds, st_,
                       (const double*)at(t_.off_gram), nblk * t_.nb, nfix, t_.nb, at(t_.off_y),
                       at(t_.off_lam), (int*)(ws_ + t_.off_sinfo));
    TL_CHECK_LAUNCH();
    int si[4];
    TL_TRY(lob_read(ws_ + t_.off_sinfo, si, sizeof(si), st_));
    if (si[0] < t_.nb) {
      set_error("Rayleigh-Ritz basis of rank %d below the block size %d", si[0], t_.nb);
      return TL_EINVAL;
    }
    return TL_OK;
  }
  // X <- X Y_x + P_new, P_new = W Y_w + P Y_p (all three families)
  tl_status update(int nblk) {
    const double* Y = at(t_.off_y);
    const int64_t nb = t_.nb;
    const int xs[3] = {kX, kAX, kBX}, ws[3] = {kW, kAW, kBW}, ps[3] = {kP, kAP, kBP};
    const int x2[3] = {kX2, kAX2, kBX2}, p2[3] = {kP2, kAP2, kBP2};
    if (nblk > 1) {
      TsArgs a = base();
      for (int f = 0; f < 3; ++f) {
        a.in[f][0] = v(ws[f]);
        a.in[f][1] = v(ps[f]);
        a.out[f] = v(p2[f]);
      }
      a.Y[0] = Y + nb * nb;
      a.Y[1] = Y + 2 * nb * nb;
      a.nin = nblk - 1;
      TL_TRY(launch_ts(a));
    }
    TsArgs a = base();
    for (int f = 0; f < 3; ++f) {
      a.in[f][0] = v(xs[f]);
      a.out[f] = v(x2[f]);
      a.add[f] = nblk > 1 ? v(p2[f]) : nullptr;
    }
    a.Y[0] = Y;
    a.nin = 1;
    TL_TRY(launch_ts(a));
    for (int f = 0; f < 3; ++f) {
      std::swap(cur_[xs[f]], cur_[x2[f]]);
      if (nblk > 1) std::swap(cur_[ps[f]], cur_[p2[f]]);
    }
    return TL_OK;
  }
  // P <- P - X (BX^T P), with T_H P and T_S P alike
  tl_status project_p() {
    const int vb[1] = {kBX}, ub[1] = {kP};
    TL_TRY(gram(vb, ub, nullptr, 1));
    TsArgs a = base();
    const int xs[3] = {kX, kAX, kBX}, ps[3] = {kP, kAP, kBP};
    for (int f = 0; f < 3; ++f) {
      a.in[f][0] = v(xs[f]);
      a.out[f] = v(ps[f]);
    }
    a.Y[0] = at(t_.off_gram);
    a.ldy = kLobMaxBasis;
    a.nin = 1;
    a.alpha = -1.0;
    a.beta = 1.0;
    return launch_ts(a);
  }
  // W <- W - X (BX^T W)
  tl_status project_w() {
    const int vb[1] = {kBX}, ub[1] = {kW};
    TL_TRY(gram(vb, ub, nullptr, 1));
    TsArgs a = base();
    a.in[0][0] = v(kX);
    a.out[0] = v(kW);
    a.Y[0] = at(t_.off_gram);
    a.ldy = kLobMaxBasis;
    a.nin = 1;
    a.alpha = -1.0;
    a.beta = 1.0;
    hipLaunchKernelGGL(lob_ts_kernel, dim3((unsigned)ceil_div(t_.N * t_.nb, 256), 1), dim3(256),
                       0, st_, a);
    TL_CHECK_LAUNCH();
    return TL_OK;
  }
  // keep (X, lam) as the best iterate so far, or return to it
  tl_status keep_best(bool restore) {
    const size_t bx = sizeof(double) * t_.N * t_.nb, bl = sizeof(double) * t_.nb;
    double* best = (double*)(ws_ + t_.off_vec[kBest]);
    if (restore) {
      TL_HIP(hipMemcpyAsync(v(kX), best, bx, hipMemcpyDeviceToDevice, st_));
      TL_HIP(hipMemcpyAsync(at(t_.off_lam), at(t_.off_lambest), bl, hipMemcpyDeviceToDevice, st_));
    } else {
      TL_HIP(hipMemcpyAsync(best, v(kX), bx, hipMemcpyDeviceToDevice, st_));
      TL_HIP(hipMemcpyAsync(at(t_.off_lambest), at(t_.off_lam), bl, hipMemcpyDeviceToDevice, st_));
    }
    return TL_OK;
  }
  // zero the residual columns whose mask entry is 0 (soft locking)
  tl_status mask(const double* mask_h) {
    TL_HIP(hipMemcpyAsync(at(t_.off_mask), mask_h, sizeof(double) * t_.nb, hipMemcpyHostToDevice,
                          st_));
    hipLaunchKernelGGL(lob_mask_kernel, dim3((unsigned)ceil_div(t_.N * t_.nb, 256)), dim3(256), 0,
                       st_, v(kW), (const double*)at(t_.off_mask), t_.N, t_.nb);
    TL_CHECK_LAUNCH();
    return TL_OK;
  }
  // W <- Strang shift-inverse of W (through the block DFT over L cells)
  tl_status precondition() {
    TL_TRY(launch_fft(t_.fr, st_));
    const int64_t nx = (int64_t)t_.cells * t_.Ev;
    hipLaunchKernelGGL(mul_kernel, dim3((unsigned)ceil_div(nx, 256)), dim3(256), 0, st_,
                       MulArgs{(const double*)at(t_.off_minv), (const double*)at(t_.off_rhat),
                               at(t_.off_z), t_.cells, t_.m0, t_.nb});
    TL_CHECK_LAUNCH();
    TL_TRY(launch_fft(t_.fz, st_));
    hipLaunchKernelGGL(comb_kernel, dim3((unsigned)ceil_div(nx, 256)), dim3(256), 0, st_,
                       CombArgs{(const double*)at(t_.off_f), v(kW), t_.cells, t_.cells, t_.Ev});
    TL_CHECK_LAUNCH();
    return TL_OK;
  }
  // R = AX - BX lam into W; column norms of R and X read back with lam
  tl_status residuals(double* lam_h, double* norms_h) {
    const int64_t n = t_.N * t_.nb;
    hipLaunchKernelGGL(lob_resid_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st_,
                       (const double*)v(kAX), (const double*)v(kBX),
                       (const double*)at(t_.off_lam), v(kW), t_.N, t_.nb);
    TL_CHECK_LAUNCH();
    hipLaunchKernelGGL(lob_colnorm_kernel, dim3((unsigned)t_.nb), dim3(256), 0, st_,
                       (const double*)v(kW), (const double*)v(kX), t_.N, t_.nb,
                       at(t_.off_norms));
    TL_CHECK_LAUNCH();
    TL_HIP(hipMemcpyAsync(lam_h, at(t_.off_lam), sizeof(double) * t_.nb, hipMemcpyDeviceToHost,
                          st_));
    return lob_read(at(t_.off_norms), norms_h, sizeof(double) * 2 * t_.nb, st_);
  }

 private:
  TsArgs base() const {
    TsArgs a;
    std::memset(&a, 0, sizeof(a));
    a.nb = t_.nb;
    a.ldy = t_.nb;
    a.N = t_.N;
    a.alpha = 1.0;
    a.beta = 0.0;
    return a;
  }
  tl_status launch_ts(const TsArgs& a) {
    hipLaunchKernelGGL(lob_ts_kernel, dim3((unsigned)ceil_div(t_.N * t_.nb, 256), 3), dim3(256),
                       0, st_, a);
    TL_CHECK_LAUNCH();
    return TL_OK;
  }
  const LobLayout& t_;
  char* ws_;
  hipStream_t st_;
  int cur_[kNVec];
};

tl_status btoepl_lowest(const double* Hb, const double* Sb, const int Lv[3], bool three, int m0,
                        int nev, int nb, int max_iter, double tol, double shift, const double* x0,
                        double* evals, double* evecs, double* resid, int* iters, int* nconv,
                        char* ws, size_t ws_bytes, hipStream_t st) {
  LobLayout t;
  TL_TRY(lob_layout(Lv, three, m0, nb, &t, ws));
  if (ws_bytes < t.bytes) {
    set_error("workspace: need %zu bytes, got %zu", t.bytes, ws_bytes);
    return TL_EWORKSPACE;
  }
  const size_t lds = sizeof(double) * 4 * kLobMaxBasis * kLobLd;
  TL_HIP(hipFuncSetAttribute((const void*)lob_small_kernel,
                             hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  Lobpcg lob(t, ws, st);
  const int64_t m2 = (int64_t)m0 * m0;
  const int cells = t.cells;
  // the two Toeplitz operators
  for (int w = 0; w < 2; ++w) {
    char* base = ws + (w ? t.off_tS : t.off_tH);
    if (three) {
      const Toeplitz3Layout& tw = w ? t.tS3 : t.tH3;
      Embed3Args a{w ? Sb : Hb, (double*)(base + tw.off_xt), {Lv[0], Lv[1], Lv[2]},
                   {tw.L2[0], tw.L2[1], tw.L2[2]}, m0, (int64_t)tw.P * tw.Eb};
      hipLaunchKernelGGL(embed3_kernel, dim3((unsigned)ceil_div(a.total, 256)), dim3(256), 0, st,
                         a);
      TL_CHECK_LAUNCH();
      TL_TRY(launch_fft(tw.fb, st));
    } else {
      const ToeplitzLayout& tw = w ? t.tS : t.tH;
      const int64_t nbk = 2 * (int64_t)Lv[0] * m2;
      hipLaunchKernelGGL(embed_kernel, dim3((unsigned)ceil_div(nbk, 256)), dim3(256), 0, st,
                         EmbedArgs{w ? Sb : Hb, (double*)(base + tw.off_xt), Lv[0], m0});
      TL_CHECK_LAUNCH();
      TL_TRY(launch_fft(tw.fb, st));
    }
  }
  // preconditioner: Strang k-blocks, their lowest eigenvalue, the shifted inverses
  if (three) {
    Strang3Args sa{{Hb, Sb}, lob.at(t.off_strang), {Lv[0], Lv[1], Lv[2]}, m0,
                   2 * (int64_t)cells * m2};
    hipLaunchKernelGGL(strang3_kernel, dim3((unsigned)ceil_div(sa.total, 256)), dim3(256), 0, st,
                       sa);
  } else {
    StrangArgs sa{{Hb, Sb}, lob.at(t.off_strang), Lv[0], m0};
    hipLaunchKernelGGL(strang_kernel, dim3((unsigned)ceil_div(2 * cells * m2, 256)), dim3(256),
                       0, st, sa);
  }
  TL_CHECK_LAUNCH();
  TL_TRY(launch_fft(t.fblk, st));
  const double* hat = lob.at(t.off_hat);
  int* kinfo = (int*)(ws + t.off_info);
  TL_TRY(batched_heigh(hat, hat + 2 * (int64_t)cells * m2, cells, m0, lob.at(t.off_evals),
                       nullptr, kinfo, st));
  double* scal = lob.at(t.off_scal);
  hipLaunchKernelGGL(lmin_kernel, dim3(1), dim3(256), 0, st, (const double*)lob.at(t.off_evals),
                     (const int*)kinfo, cells, m0, scal);
  TL_CHECK_LAUNCH();
  if (three) {
    const int nblk = (2 * Lv[0] - 1) * (2 * Lv[1] - 1) * (2 * Lv[2] - 1);
    hipLaunchKernelGGL(tnorm3_kernel, dim3(1), dim3(256), 0, st, Hb, Sb, nblk, m0, scal);
  } else {
    hipLaunchKernelGGL(tnorm_kernel, dim3(1), dim3(256), 0, st, Hb, Sb, Lv[0], m0, scal);
  }
  TL_CHECK_LAUNCH();
  double sc[8];
  TL_TRY(lob_read(scal, sc, sizeof(sc), st));
  if (sc[3] != 0.0) {
    set_error("a k-block of the circulant preconditioner is not definite");
    return TL_EINVAL;
  }
  const double lmin = sc[0], nA = sc[1], nB = sc[2];
  // a shift close below the circulant minimum makes the preconditioner an
  // approximate shift-and-invert that separates the clustered bottom states;
  // it stays 10 times above the finite-size offset of the pencil's lowest
  // eigenvalue from the circulant minimum, estimated as a quarter of the gap
  // to the next k-block minimum (a band minimum is quadratic in k)
  const double fin = std::isfinite(sc[4]) ? 0.25 * (sc[4] - lmin) : 0.0;
  const double delta = shift > 0.0 ? shift
                                   : std::max(1e-4 * std::max(1.0, std::fabs(lmin)), 10.0 * fin);
  const double sigma = lmin - delta;
  hipLaunchKernelGGL(minv_kernel, dim3((unsigned)ceil_div(cells, 64)), dim3(64), 0, st, hat,
                     cells, m0, sigma, lob.at(t.off_lf), lob.at(t.off_minv), kinfo);
  TL_CHECK_LAUNCH();
  hipLaunchKernelGGL(lmin_kernel, dim3(1), dim3(256), 0, st, (const double*)lob.at(t.off_evals),
                     (const int*)kinfo, cells, m0, scal);
  TL_CHECK_LAUNCH();
  TL_TRY(lob_read(scal, sc, sizeof(sc), st));
  if (sc[3] != 0.0) {
    set_error("shifted circulant block not positive definite");
    return TL_EINVAL;
  }

  // start block and its Rayleigh-Ritz
  const int64_t nx = t.N * nb;
  if (x0) {
    TL_HIP(hipMemcpyAsync(lob.v(kX), x0, sizeof(double) * nx, hipMemcpyDeviceToDevice, st));
  } else {
    hipLaunchKernelGGL(lob_rand_kernel, dim3((unsigned)ceil_div(nx, 256)), dim3(256), 0, st,
                       lob.v(kX), nx, (uint64_t)0x5EEDull);
    TL_CHECK_LAUNCH();
  }
  TL_TRY(lob.products(kX, kAX, kBX));
  TL_TRY(lob.rayleigh_ritz(1));
  TL_TRY(lob.update(1));

  std::vector<double> lam_h(nb), norms_h(2 * nb), rel(nb), mask_h(nb);
  double worst = 0.0;  // largest relative residual of the wanted pairs
  auto count_converged = [&]() {
    int c = 0;
    worst = 0.0;
    for (int j = 0; j < nb; ++j) {
      rel[j] = std::sqrt(norms_h[j]) /
               ((nA + std::fabs(lam_h[j]) * nB) * std::sqrt(norms_h[nb + j]));
      if (j < nev && rel[j] <= tol) ++c;
      if (j < nev) worst = std::max(worst, rel[j]);
    }
    return c;
  };
  // near the rounding floor the iteration can lose accuracy again; the best
  // iterate (most converged pairs, then smallest worst residual) is kept
  int nblk = 2, it = 0, conv = 0, best_conv = -1;
  double best_worst = INFINITY;
  for (it = 1; it <= max_iter; ++it) {
    if (it % kLobRefresh == 0) TL_TRY(lob.products(kX, kAX, kBX));
    TL_TRY(lob.residuals(lam_h.data(), norms_h.data()));
    conv = count_converged();
    if (conv > best_conv || (conv == best_conv && worst < best_worst)) {
      best_conv = conv;
      best_worst = worst;
      TL_TRY(lob.keep_best(false));
    }
    if (conv == nev) break;
    // soft locking: converged wanted pairs stay in the basis through X but
    // add no new direction (their residuals are rounding noise)
    for (int j = 0; j < nb; ++j) mask_h[j] = (j < nev && rel[j] <= tol) ? 0.0 : 1.0;
    TL_TRY(lob.mask(mask_h.data()));
    TL_TRY(lob.precondition());
    TL_TRY(lob.project_w());
    TL_TRY(lob.products(kW, kAW, kBW));
    if (nblk == 3) TL_TRY(lob.project_p());
    TL_TRY(lob.rayleigh_ritz(nblk));
    TL_TRY(lob.update(nblk));
    nblk = 3;
  }
  // final residuals from fresh products; the best iterate if the last is worse
  TL_TRY(lob.products(kX, kAX, kBX));
  TL_TRY(lob.residuals(lam_h.data(), norms_h.data()));
  conv = count_converged();
  if (conv < best_conv || (conv == best_conv && worst > best_worst)) {
    TL_TRY(lob.keep_best(true));
    TL_TRY(lob.products(kX, kAX, kBX));
    TL_TRY(lob.residuals(lam_h.data(), norms_h.data()));
    conv = count_converged();
  }
  *iters = std::min(it, max_iter);
  *nconv = conv;
  TL_HIP(hipMemcpyAsync(evals, lob.at(t.off_lam), sizeof(double) * nev, hipMemcpyDeviceToDevice,
                        st));
  if (resid)
    TL_HIP(hipMemcpyAsync(resid, rel.data(), sizeof(double) * nev, hipMemcpyHostToDevice, st));
  if (evecs) {
    hipLaunchKernelGGL(lob_cols_kernel, dim3((unsigned)ceil_div(t.N * nev, 256)), dim3(256), 0,
                       st, (const double*)lob.v(kX), evecs, t.N, nb, nev);
    TL_CHECK_LAUNCH();
  }
  TL_HIP(hipStreamSynchronize(st));  // rel is a host buffer of this call
  return TL_OK;
}

}  // namespace
}  // namespace tl

using namespace tl;

extern "C" tl_status tl_btoepl_workspace_bytes(int L, int m0, int nvec, size_t* bytes) {
  clear_error();
  TL_REQUIRE(bytes != nullptr, "null output");
  ToeplitzLayout t;
  TL_TRY(layout(L, m0, nvec, &t, nullptr));
  *bytes = t.bytes;
  return TL_OK;
}

extern "C" tl_status tl_btoepl_setup(const double* A_dev, int L, int m0, int nvec, void* ws_dev,
                                     size_t ws_bytes, void* stream) {
  clear_error();
  ToeplitzLayout t;
  TL_TRY(layout(L, m0, nvec, &t, (char*)ws_dev));
  TL_REQUIRE(A_dev && ws_dev, "null array argument");
  TL_REQUIRE(ws_bytes >= t.bytes, "workspace: need %zu bytes, got %zu", t.bytes, ws_bytes);
  char* ws = (char*)ws_dev;
  const int64_t nb = 2 * (int64_t)L * t.Eb;
  hipLaunchKernelGGL(embed_kernel, dim3((unsigned)ceil_div(nb, 256)), dim3(256), 0,
                     (hipStream_t)stream, EmbedArgs{A_dev, (double*)(ws + t.off_xt), L, m0});
  TL_CHECK_LAUNCH();
  return launch_fft(t.fb, (hipStream_t)stream);
}

extern "C" tl_status tl_btoepl_matvec(const double* X_dev, double* Y_dev, int L, int m0, int nvec,
                                      void* ws_dev, size_t ws_bytes, void* stream) {
  clear_error();
  ToeplitzLayout t;
  TL_TRY(layout(L, m0, nvec, &t, (char*)ws_dev));
  TL_REQUIRE(X_dev && Y_dev && ws_dev, "null array argument");
  TL_REQUIRE(ws_bytes >= t.bytes, "workspace: need %zu bytes, got %zu", t.bytes, ws_bytes);
  return matvec(t, (char*)ws_dev, X_dev, Y_dev, (hipStream_t)stream);
}

extern "C" tl_status tl_btoepl_power(int L, int m0, int iters, double* x_dev, double* y_dev,
                                     double* lambda_dev, void* ws_dev, size_t ws_bytes,
                                     void* stream) {
  clear_error();
  ToeplitzLayout t;
  TL_TRY(layout(L, m0, 1, &t, (char*)ws_dev));
  TL_REQUIRE(x_dev && y_dev && lambda_dev && ws_dev, "null array argument");
  TL_REQUIRE(iters >= 1, "iters = %d < 1", iters);
  TL_REQUIRE(ws_bytes >= t.bytes, "workspace: need %zu bytes, got %zu", t.bytes, ws_bytes);
  const int n = L * m0;
  for (int it = 0; it < iters; ++it) {
    TL_TRY(matvec(t, (char*)ws_dev, x_dev, y_dev, (hipStream_t)stream));
    hipLaunchKernelGGL(power_update_kernel, dim3(1), dim3(1024), 0, (hipStream_t)stream, x_dev,
                       (const double*)y_dev, n, lambda_dev + it);
    TL_CHECK_LAUNCH();
  }
  return TL_OK;
}

extern "C" tl_status tl_btoepl_lowest_workspace_bytes(int L, int m0, int nb, size_t* bytes) {
  clear_error();
  TL_REQUIRE(bytes != nullptr, "null output");
  LobLayout t;
  const int Lv[3] = {L, 1, 1};
  TL_TRY(lob_layout(Lv, false, m0, nb, &t, nullptr));
  *bytes = t.bytes;
  return TL_OK;
}

extern "C" tl_status tl_btoepl_lowest(const double* H_dev, const double* S_dev, int L, int m0,
                                      int nev, int nb, int max_iter, double tol, double shift,
                                      const double* x0_dev, double* evals_dev, double* evecs_dev,
                                      double* resid_dev, int* iters, int* nconv, void* ws_dev,
                                      size_t ws_bytes, void* stream) {
  clear_error();
  TL_REQUIRE(H_dev && S_dev && evals_dev && iters && nconv && ws_dev, "null argument");
  TL_REQUIRE(nb >= 1 && nb <= kLobMaxNb, "nb = %d outside [1, %d]", nb, kLobMaxNb);
  TL_REQUIRE(nev >= 1 && nev <= nb, "nev = %d outside [1, nb = %d]", nev, nb);
  TL_REQUIRE((int64_t)L * m0 >= 3 * (int64_t)nb, "L m0 = %lld below 3 nb = %d",
             (long long)L * m0, 3 * nb);
  TL_REQUIRE(max_iter >= 1, "max_iter = %d < 1", max_iter);
  TL_REQUIRE(tol > 0.0, "tol must be positive");
  const int Lv[3] = {L, 1, 1};
  return btoepl_lowest(H_dev, S_dev, Lv, false, m0, nev, nb, max_iter, tol, shift, x0_dev,
                       evals_dev, evecs_dev, resid_dev, iters, nconv, (char*)ws_dev, ws_bytes,
                       (hipStream_t)stream);
}

extern "C" tl_status tl_btoepl3_workspace_bytes(int L1, int L2, int L3, int m0, int nvec,
                                                size_t* bytes) {
  clear_error();
  TL_REQUIRE(bytes != nullptr, "null output");
  const int L[3] = {L1, L2, L3};
  Toeplitz3Layout t;
  TL_TRY(layout3(L, m0, nvec, &t, nullptr));
  *bytes = t.bytes;
  return TL_OK;
}

extern "C" tl_status tl_btoepl3_setup(const double* B_dev, int L1, int L2, int L3, int m0,
                                      int nvec, void* ws_dev, size_t ws_bytes, void* stream) {
  clear_error();
  const int L[3] = {L1, L2, L3};
  Toeplitz3Layout t;
  TL_TRY(layout3(L, m0, nvec, &t, (char*)ws_dev));
  TL_REQUIRE(B_dev && ws_dev, "null array argument");
  if (ws_bytes < t.bytes) {
    set_error("workspace: need %zu bytes, got %zu", t.bytes, ws_bytes);
    return TL_EWORKSPACE;
  }
  char* ws = (char*)ws_dev;
  Embed3Args a{B_dev, (double*)(ws + t.off_xt), {L1, L2, L3}, {t.L2[0], t.L2[1], t.L2[2]}, m0,
               (int64_t)t.P * t.Eb};
  hipLaunchKernelGGL(embed3_kernel, dim3((unsigned)ceil_div(a.total, 256)), dim3(256), 0,
                     (hipStream_t)stream, a);
  TL_CHECK_LAUNCH();
  return launch_fft(t.fb, (hipStream_t)stream);
}

extern "C" tl_status tl_btoepl3_matvec(const double* X_dev, double* Y_dev, int L1, int L2, int L3,
                                       int m0, int nvec, void* ws_dev, size_t ws_bytes,
                                       void* stream) {
  clear_error();
  const int L[3] = {L1, L2, L3};
  Toeplitz3Layout t;
  TL_TRY(layout3(L, m0, nvec, &t, (char*)ws_dev));
  TL_REQUIRE(X_dev && Y_dev && ws_dev, "null array argument");
  if (ws_bytes < t.bytes) {
    set_error("workspace: need %zu bytes, got %zu", t.bytes, ws_bytes);
    return TL_EWORKSPACE;
  }
  return matvec3(t, (char*)ws_dev, X_dev, Y_dev, (hipStream_t)stream);
}

extern "C" tl_status tl_btoepl3_power(int L1, int L2, int L3, int m0, int iters, double* x_dev,
                                      double* y_dev, double* lambda_dev, void* ws_dev,
                                      size_t ws_bytes, void* stream) {
  clear_error();
  const int L[3] = {L1, L2, L3};
  Toeplitz3Layout t;
  TL_TRY(layout3(L, m0, 1, &t, (char*)ws_dev));
  TL_REQUIRE(x_dev && y_dev && lambda_dev && ws_dev, "null array argument");
  TL_REQUIRE(iters >= 1, "iters = %d < 1", iters);
  if (ws_bytes < t.bytes) {
    set_error("workspace: need %zu bytes, got %zu", t.bytes, ws_bytes);
    return TL_EWORKSPACE;
  }
  const int n = L1 * L2 * L3 * m0;
  for (int it = 0; it < iters; ++it) {
    TL_TRY(matvec3(t, (char*)ws_dev, x_dev, y_dev, (hipStream_t)stream));
    hipLaunchKernelGGL(power_update_kernel, dim3(1), dim3(1024), 0, (hipStream_t)stream, x_dev,
                       (const double*)y_dev, n, lambda_dev + it);
    TL_CHECK_LAUNCH();
  }
  return TL_OK;
}

extern "C" tl_status tl_btoepl3_lowest_workspace_bytes(int L1, int L2, int L3, int m0, int nb,
                                                       size_t* bytes) {
  clear_error();
  TL_REQUIRE(bytes != nullptr, "null output");
  const int Lv[3] = {L1, L2, L3};
  LobLayout t;
  TL_TRY(lob_layout(Lv, true, m0, nb, &t, nullptr));
  *bytes = t.bytes;
  return TL_OK;
}

extern "C" tl_status tl_btoepl3_lowest(const double* H_dev, const double* S_dev, int L1, int L2,
                                       int L3, int m0, int nev, int nb, int max_iter, double tol,
                                       double shift, const double* x0_dev, double* evals_dev,
                                       double* evecs_dev, double* resid_dev, int* iters,
                                       int* nconv, void* ws_dev, size_t ws_bytes, void* stream) {
  clear_error();
  TL_REQUIRE(H_dev && S_dev && evals_dev && iters && nconv && ws_dev, "null argument");
  TL_REQUIRE(L1 >= 1 && L2 >= 1 && L3 >= 1, "lattice extents must be >= 1");
  TL_REQUIRE(nb >= 1 && nb <= kLobMaxNb, "nb = %d outside [1, %d]", nb, kLobMaxNb);
  TL_REQUIRE(nev >= 1 && nev <= nb, "nev = %d outside [1, nb = %d]", nev, nb);
  TL_REQUIRE((int64_t)L1 * L2 * L3 * m0 >= 3 * (int64_t)nb, "L1 L2 L3 m0 below 3 nb = %d",
             3 * nb);
  TL_REQUIRE(max_iter >= 1, "max_iter = %d < 1", max_iter);
  TL_REQUIRE(tol > 0.0, "tol must be positive");
  const int Lv[3] = {L1, L2, L3};
  return btoepl_lowest(H_dev, S_dev, Lv, true, m0, nev, nb, max_iter, tol, shift, x0_dev,
                       evals_dev, evecs_dev, resid_dev, iters, nconv, (char*)ws_dev, ws_bytes,
                       (hipStream_t)stream);
}
