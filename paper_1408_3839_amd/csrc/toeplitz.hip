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
#include <cmath>
#include <cstring>

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
