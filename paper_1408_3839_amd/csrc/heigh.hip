// Step a7: batched eigensolver for the k-block pencils (Hbar_j - lambda Sbar_j)
// of the Fourier-space problem (Sec. 4.2, eq. (HF-FSpace-Block); Proposition
// on block-circulant diagonalisation, eq. (lambdAbc)).
//
// Per block: Cholesky Sbar = L L^H, C = L^-1 Hbar L^-H (Hermitian average),
// then either eigenvalues only (m <= 16: Householder reduction of C to a real
// tridiagonal and Sturm bisection) or complex Jacobi with the parallel
// round-robin ordering and eigenvectors u = L^-H v.  m <= 8 runs in one wave
// with the matrices in registers; larger m uses one workgroup per block and
// LDS (256 threads, one per entry, for the eigenvalues of m <= 16).
// Eigenvalues ascending.
#include <cmath>

#include "common.h"
#include "dev_heigh.h"

namespace tl {
namespace {

template <int MAXM>
__global__ __launch_bounds__(1024) void heigh_kernel(const double* __restrict__ H,
                                                     const double* __restrict__ S, int m,
                                                     double* __restrict__ evals,
                                                     double* __restrict__ evecs,
                                                     int* __restrict__ info) {
  dev::heigh_body<MAXM>(H, S, m, evals, evecs, info, blockIdx.x);
}

// Eigenvalues only, m <= 8: m one-wave workgroups per block, each repeating
// the reduction to tridiagonal form and bisecting one eigenvalue with the
// whole wave, which shortens the dependent chain of the bisection.
__global__ __launch_bounds__(64) void heigh_evals_kernel(const double* __restrict__ H,
                                                         const double* __restrict__ S, int m,
                                                         double* __restrict__ evals,
                                                         int* __restrict__ info) {
  const int64_t blk = blockIdx.x / m;
  const int w = (int)(blockIdx.x - blk * m);
  dev::heigh_wave8_body(H, S, m, evals, nullptr, info, blk, w, m);
}

// Eigenvalues only, 8 < m <= 16: one 256-thread workgroup per block.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 2))) void heigh_evals16_kernel(const double* __restrict__ H,
                                                            const double* __restrict__ S, int m,
                                                            double* __restrict__ evals,
                                                            int* __restrict__ info) {
  dev::heigh_evals16_body(H, S, m, evals, info, blockIdx.x);
}

}  // namespace

tl_status batched_heigh(const double* H, const double* S, int count, int m, double* evals,
                        double* evecs, int* info, hipStream_t stream) {
  int threads = (int)std::max<int64_t>(64, ceil_div((int64_t)m * m, 64) * 64);
  if (m <= 8 && evecs == nullptr && (int64_t)count * m <= INT32_MAX) {
    hipLaunchKernelGGL(heigh_evals_kernel, dim3((unsigned)(count * m)), dim3(64), 0, stream, H, S,
                       m, evals, info);
  } else if (m <= 8) {
    hipLaunchKernelGGL(heigh_kernel<8>, dim3(count), dim3(threads), 0, stream, H, S, m, evals,
                       evecs, info);
  } else if (m <= 16 && evecs == nullptr) {
    hipLaunchKernelGGL(heigh_evals16_kernel, dim3(count), dim3(256), 0, stream, H, S, m, evals,
                       info);
  } else if (m <= 16) {
    hipLaunchKernelGGL(heigh_kernel<16>, dim3(count), dim3(threads), 0, stream, H, S, m, evals,
                       evecs, info);
  } else {
    hipLaunchKernelGGL(heigh_kernel<32>, dim3(count), dim3(threads), 0, stream, H, S, m, evals,
                       evecs, info);
  }
  TL_CHECK_LAUNCH();
  return TL_OK;
}

}  // namespace tl

extern "C" tl_status tl_batched_heigh(const double* H_dev, const double* S_dev, int count, int m0,
                                      double* evals_dev, double* evecs_dev, int* info_dev,
                                      void* stream) {
  tl::clear_error();
  TL_REQUIRE(H_dev && evals_dev && info_dev, "null array argument");
  TL_REQUIRE(m0 >= 1 && m0 <= TL_MAX_M0, "m0 = %d outside [1, %d]", m0, TL_MAX_M0);
  TL_REQUIRE(count >= 1 && count <= (1 << 30), "count = %d out of range", count);
  return tl::batched_heigh(H_dev, S_dev, count, m0, evals_dev, evecs_dev, info_dev,
                           (hipStream_t)stream);
}
