// Step a6: Fourier block-diagonalisation of a 3-level block-circulant matrix.
//   Abar_j = sum_k w1^(j1 k1) w2^(j2 k2) w3^(j3 k3) A_k,  w_l = exp(-2 pi i / L_l)
// (Lemma 2.2, eq. (DiagMLcirc); Appendix, Proposition on block-circulant
// diagonalisation).  F_L = F_L1 x F_L2 x F_L3 is applied one lattice axis at
// a time; each pass is a batched 1D DFT along that axis for every entry of
// every m0 x m0 block.  Twiddles use the exact residue (j k mod L), so the
// phase is never formed from a large angle.
#include <algorithm>

#include "common.h"
#include "dev_fft.h"

namespace tl {
namespace {

using dev::DftArgs;
constexpr int kMaxTwiddle = dev::kMaxTwiddle;

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

}  // namespace

tl_status block_fft(const double* in, int L1, int L2, int L3, int m0, int batch, double* out,
                    void* ws, size_t ws_bytes, hipStream_t stream) {
  const int L[3] = {L1, L2, L3};
  const int64_t E = (int64_t)m0 * m0;
  const int64_t total = (int64_t)batch * L1 * L2 * L3 * E;
  int axes[3], na = 0;
  for (int d = 0; d < 3; ++d)
    if (L[d] > 1) axes[na++] = d;
  size_t need = na >= 2 ? align_up(sizeof(double) * 2 * (size_t)total, 256) : 0;
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
  int na = (L1 > 1) + (L2 > 1) + (L3 > 1);
  int64_t total = (int64_t)batch * L1 * L2 * L3 * m0 * m0;
  *bytes = na >= 2 ? tl::align_up(sizeof(double) * 2 * (size_t)total, 256) : 0;
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
