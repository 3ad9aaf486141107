// Step a6: Fourier block-diagonalisation of a 3-level block-circulant matrix.
//   Abar_j = sum_k w1^(j1 k1) w2^(j2 k2) w3^(j3 k3) A_k,  w_l = exp(-2 pi i / L_l)
// (Lemma 2.2, eq. (DiagMLcirc); Appendix, Proposition on block-circulant
// diagonalisation), at the O(m0^2 L^d log L) cost of Sec. 4.2.
// F_L = F_L1 x F_L2 x F_L3 is applied to every entry of every m0 x m0 block.
// Lattices whose buffer fits a workgroup's LDS (every extent 7-smooth and
// L1 L2 L3 <= 4096, or one axis of any length up to 2048 by Bluestein) take
// the LDS FFT: one launch, each workgroup a set of entry columns over the
// whole lattice (Bluestein lengths: one more small launch that tabulates the
// chirp and the filter's transform, L + M complex values of workspace).  Longer lines fall back to a direct DFT along
// one axis at a time (twiddles from the exact residue j k mod L).
#include <algorithm>
#include <cstring>

#include "common.h"
#include "dev_fft.h"
#include "host_plans.h"

namespace tl {
namespace {

using dev::DftArgs;
constexpr int kMaxTwiddle = dev::kMaxTwiddle;

__global__ __launch_bounds__(dev::kFftThreads) void fft_blue_tables_kernel(dev::FftArgs a) {
  extern __shared__ __align__(16) double smem[];
  dev::fft_blue_tables_body(a, smem);
}

template <bool BLUE>
__global__ __launch_bounds__(dev::kFftThreads) void fft_block_kernel(dev::FftArgs a) {
  extern __shared__ __align__(16) double smem[];
  dev::fft_block_body<BLUE>(a, blockIdx.x, smem);
}

template <bool REAL_IN, bool TABLE>
__global__ __launch_bounds__(256) void dft_axis_kernel(DftArgs a) {
  extern __shared__ double tw[];
  dev::dft_axis_body<REAL_IN, TABLE>(a, blockIdx.x, blockIdx.y, tw);
}

tl_status launch_axis(const DftArgs& a, int64_t outer, hipStream_t stream) {
  dim3 grid((unsigned)(outer * a.len), (unsigned)ceil_div(a.inner, 256));
  const bool table = a.len <= kMaxTwiddle;
  size_t shmem = sizeof(double) * std::max<size_t>(table ? 2 * (size_t)a.len : 0, 2 * 256);
  if (a.real_in && table)
    hipLaunchKernelGGL((dft_axis_kernel<true, true>), grid, dim3(256), shmem, stream, a);
  else if (a.real_in)
    hipLaunchKernelGGL((dft_axis_kernel<true, false>), grid, dim3(256), shmem, stream, a);
  else if (table)
    hipLaunchKernelGGL((dft_axis_kernel<false, true>), grid, dim3(256), shmem, stream, a);
  else
    hipLaunchKernelGGL((dft_axis_kernel<false, false>), grid, dim3(256), shmem, stream, a);
  TL_CHECK_LAUNCH();
  return TL_OK;
}

bool smooth7(int n) {
  for (int p : {2, 3, 5, 7})
    while (n % p == 0) n /= p;
  return n == 1;
}

bool factor_axis(int n, dev::FftAxis* ax) {
  ax->n = n;
  ax->npass = 0;
  int r = n;
  auto push = [&](int R) {
    if (ax->npass >= dev::kFftMaxPasses) return false;
    ax->rad[ax->npass++] = (unsigned char)R;
    r /= R;
    return true;
  };
  while (r % 8 == 0)
    if (!push(8)) return false;
  while (r % 4 == 0)
    if (!push(4)) return false;
  while (r % 2 == 0)
    if (!push(2)) return false;
  for (int R : {3, 5, 7})
    while (r % R == 0)
      if (!push(R)) return false;
  return r == 1;
}

}  // namespace

bool plan_fft(const double* in, double* out, const int L[3], int m0, int64_t batch,
              dev::FftArgs* a, int min_groups) {
  return plan_fft_cols(in, out, L, (int64_t)m0 * m0, batch, a, min_groups);
}

bool plan_fft_cols(const double* in, double* out, const int L[3], int64_t E, int64_t batch,
                   dev::FftArgs* a, int min_groups) {
  std::memset(a, 0, sizeof(*a));
  a->in = in;
  a->out = out;
  a->E = E;
  a->cols = batch * a->E;
  a->P = 1;
  for (int d = 0; d < 3; ++d) {
    a->L[d] = L[d];
    a->P *= L[d];
  }
  if (a->P > dev::kFftPoints) return false;
  int axes[3], na = 0;
  for (int d = 0; d < 3; ++d)
    if (L[d] > 1) axes[na++] = d;
  a->naxes = na;
  if (na == 1 && !smooth7(L[axes[0]])) {
    int M = 2 * L[axes[0]] - 1;
    while (!smooth7(M)) ++M;
    if (M > dev::kFftPoints) return false;
    a->blue = 1;
    a->blue_L = L[axes[0]];
    a->nbuf = M;
    dev::FftAxis& ax = a->ax[0];
    if (!factor_axis(M, &ax)) return false;
    ax.S = 1;
    ax.O = 1;
  } else {
    a->nbuf = a->P;
    for (int i = 0; i < na; ++i) {
      const int d = axes[i];
      dev::FftAxis& ax = a->ax[i];
      if (!factor_axis(L[d], &ax)) return false;
      ax.S = 1;
      for (int e = d + 1; e < 3; ++e) ax.S *= L[e];
      ax.O = 1;
      for (int e = 0; e < d; ++e) ax.O *= L[e];
    }
  }
  int tw = 0;
  for (int i = 0; i < (a->blue ? 1 : na); ++i) {
    a->ax[i].tw_off = tw;
    tw += 64 + (int)ceil_div(a->ax[i].n, 64);
  }
  a->tw_total = tw;
  // columns per workgroup: as many as the LDS buffer holds (at most 64),
  // halved while that would leave fewer than min_groups workgroups
  int W = 2 * (dev::kFftPoints / a->nbuf);
  int w2 = 2;
  while (2 * w2 <= W && 2 * w2 <= 64) w2 *= 2;
  while (w2 > 2 && ceil_div(a->cols, w2) < min_groups) w2 /= 2;
  a->W = w2;
  return true;
}

size_t fft_blue_table_bytes(const dev::FftArgs& a) {
  return a.blue ? align_up(sizeof(double2) * ((size_t)a.blue_L + a.ax[0].n), 256) : 0;
}

void set_fft_blue_tables(dev::FftArgs* a, void* ws) {
  if (!a->blue) return;
  a->chirp = (double2*)ws;
  a->bhat = a->chirp + a->blue_L;
}

tl_status launch_fft(const dev::FftArgs& a, hipStream_t stream) {
  if (a.blue) {
    hipLaunchKernelGGL(fft_blue_tables_kernel, dim3(1), dim3(dev::kFftThreads),
                       dev::fft_tables_lds_bytes(a), stream, a);
    TL_CHECK_LAUNCH();
  }
  const dim3 grid((unsigned)ceil_div(a.cols, a.W)), blk(dev::kFftThreads);
  const size_t shmem = dev::fft_lds_bytes(a);
  hipEvent_t e0, e1;
  stage_events(TL_STAGE_FFT, &e0, &e1);
  if (a.blue)
    launch_with_events(fft_block_kernel<true>, grid, blk, shmem, stream, e0, e1, a);
  else
    launch_with_events(fft_block_kernel<false>, grid, blk, shmem, stream, e0, e1, a);
  TL_CHECK_LAUNCH();
  return TL_OK;
}

size_t block_fft_workspace(int L1, int L2, int L3, int m0, int batch) {
  const int L[3] = {L1, L2, L3};
  dev::FftArgs a;
  if (plan_fft(nullptr, nullptr, L, m0, batch, &a, kFftSingleGroups))
    return fft_blue_table_bytes(a);
  const int na = (L1 > 1) + (L2 > 1) + (L3 > 1);
  const int64_t total = (int64_t)batch * L1 * L2 * L3 * m0 * m0;
  return na >= 2 ? align_up(sizeof(double) * 2 * (size_t)total, 256) : 0;
}

tl_status block_fft(const double* in, int L1, int L2, int L3, int m0, int batch, double* out,
                    void* ws, size_t ws_bytes, hipStream_t stream) {
  const int L[3] = {L1, L2, L3};
  {
    dev::FftArgs fa;
    if (plan_fft(in, out, L, m0, batch, &fa, kFftSingleGroups)) {
      const size_t need = fft_blue_table_bytes(fa);
      if (ws_bytes < need || (need && !ws)) {
        set_error("block_fft workspace: need %zu bytes, got %zu", need, ws_bytes);
        return TL_EWORKSPACE;
      }
      set_fft_blue_tables(&fa, ws);
      return launch_fft(fa, stream);
    }
  }
  // lines longer than the LDS FFT holds: direct DFT, one axis per launch
  const int64_t E = (int64_t)m0 * m0;
  const int64_t total = (int64_t)batch * L1 * L2 * L3 * E;
  int axes[3], na = 0;
  for (int d = 0; d < 3; ++d)
    if (L[d] > 1) axes[na++] = d;
  size_t need = block_fft_workspace(L1, L2, L3, m0, batch);
  if (ws_bytes < need || (need && !ws)) {
    set_error("block_fft workspace: need %zu bytes, got %zu", need, ws_bytes);
    return TL_EWORKSPACE;
  }
  double* tmp = (double*)ws;
  if (na == 0) {  // one cell: the block is its own transform (imaginary part 0)
    DftArgs a{in, out, 1, E, 1};
    return launch_axis(a, batch, stream);
  }
  // pass 0 reads `in`, the last pass writes `out`: in->out (one axis),
  // in->tmp->out (two axes), in->out->tmp->out (three axes).
  const double* src = in;
  for (int p = 0; p < na; ++p) {
    int d = axes[p];
    int64_t inner = E;
    for (int e = d + 1; e < 3; ++e) inner *= L[e];
    int64_t outer = total / (inner * L[d]);
    double* dst = out;
    if (na == 2 && p == 0) dst = tmp;
    if (na == 3 && p == 1) dst = tmp;
    DftArgs a{src, dst, L[d], inner, p == 0};
    TL_TRY(launch_axis(a, outer, stream));
    src = dst;
  }
  return TL_OK;
}

}  // namespace tl

extern "C" tl_status tl_block_fft_workspace_bytes(int L1, int L2, int L3, int m0, int batch,
                                                  size_t* bytes) {
  tl::clear_error();
  TL_REQUIRE(bytes != nullptr, "null output");
  TL_REQUIRE(L1 >= 1 && L2 >= 1 && L3 >= 1 && m0 >= 1 && batch >= 1, "invalid sizes");
  TL_REQUIRE((int64_t)L1 * L2 * L3 <= (1 << 22), "lattice too large");
  *bytes = tl::block_fft_workspace(L1, L2, L3, m0, batch);
  return TL_OK;
}

extern "C" tl_status tl_block_fft(const double* in_dev, int L1, int L2, int L3, int m0, int batch,
                                  double* out_dev, void* ws_dev, size_t ws_bytes, void* stream) {
  tl::clear_error();
  TL_REQUIRE(in_dev && out_dev, "null array argument");
  TL_REQUIRE(L1 >= 1 && L2 >= 1 && L3 >= 1, "lattice extents must be >= 1");
  TL_REQUIRE(m0 >= 1 && m0 <= TL_MAX_M0, "m0 outside [1, %d]", TL_MAX_M0);
  TL_REQUIRE(batch >= 1, "batch must be >= 1");
  TL_REQUIRE((int64_t)L1 * L2 * L3 <= (1 << 22), "lattice too large");
  return tl::block_fft(in_dev, L1, L2, L3, m0, batch, out_dev, ws_dev, ws_bytes,
                       (hipStream_t)stream);
}
