// Eigenvectors of the block-circulant pencil from those of its k-blocks
// (Appendix, Proposition on block-circulant diagonalisation, eq. (eigvecA)):
// with F = F_L1 x F_L2 x F_L3 unitary, U_(j,m) = (F^* x I_m0) (e_j x u_(j,m)),
// i.e. cell c of the state (j, m) holds
//   U_(j,m)[c][mu] = L^(-1/2) exp(2 pi i (j1 c1 / L1 + j2 c2 / L2 + j3 c3 / L3)) u_(j,m)[mu].
// A u_(j,m) normalised to u^H Sbar_j u = 1 gives U^H S U = 1 for the full
// mass matrix, and states of different k-points are S-orthogonal.
#include <cmath>

#include "common.h"

namespace tl {
namespace {

struct BlochArgs {
  const double* evecs;  // [nc][m0][m0] complex, column m = eigenvector m
  const int* states;    // [n] flat state indices j m0 + m
  double* out;          // [n][nc][m0] complex
  int L[3], m0, n;
  int64_t total;        // n nc m0
};

__global__ __launch_bounds__(256) void bloch_kernel(BlochArgs a) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= a.total) return;
  const int nc = a.L[0] * a.L[1] * a.L[2];
  const int64_t per = (int64_t)nc * a.m0;
  const int r = (int)(e / per);
  const int rest = (int)(e - (int64_t)r * per);
  const int c = rest / a.m0, mu = rest - c * a.m0;
  const int st = a.states[r];
  double* o = a.out + 2 * e;
  if (st < 0 || st >= nc * a.m0) {  // not a state of this lattice
    o[0] = NAN;
    o[1] = NAN;
    return;
  }
  const int j = st / a.m0, m = st - j * a.m0;
  const int j12 = j / a.L[2], j3 = j - j12 * a.L[2];
  const int j1 = j12 / a.L[1], j2 = j12 - j1 * a.L[1];
  const int c12 = c / a.L[2], c3 = c - c12 * a.L[2];
  const int c1 = c12 / a.L[1], c2 = c12 - c1 * a.L[1];
  // phase / (2 pi): each term an exact residue over its L before the sum
  const double f = (double)((int64_t)j1 * c1 % a.L[0]) / a.L[0] +
                   (double)((int64_t)j2 * c2 % a.L[1]) / a.L[1] +
                   (double)((int64_t)j3 * c3 % a.L[2]) / a.L[2];
  double sn, cs;
  sincospi(2.0 * f, &sn, &cs);
  const double rs = 1.0 / sqrt((double)nc);
  const double* u = a.evecs + 2 * (((int64_t)j * a.m0 + mu) * a.m0 + m);
  o[0] = rs * (cs * u[0] - sn * u[1]);
  o[1] = rs * (cs * u[1] + sn * u[0]);
}

}  // namespace
}  // namespace tl

extern "C" tl_status tl_bloch_vectors(const double* evecs_dev, int L1, int L2, int L3, int m0,
                                      const int* states_dev, int n_states, double* out_dev,
                                      void* stream) {
  tl::clear_error();
  TL_REQUIRE(L1 >= 1 && L2 >= 1 && L3 >= 1, "lattice sizes must be >= 1");
  TL_REQUIRE(m0 >= 1 && m0 <= TL_MAX_M0, "m0 = %d outside [1, %d]", m0, TL_MAX_M0);
  TL_REQUIRE(n_states >= 0, "n_states = %d < 0", n_states);
  const int64_t nc = (int64_t)L1 * L2 * L3;
  TL_REQUIRE(nc * m0 <= INT32_MAX, "lattice of %lld cells too large", (long long)nc);
  if (n_states == 0) return TL_OK;
  TL_REQUIRE(evecs_dev && states_dev && out_dev, "null array argument");
  tl::BlochArgs a;
  a.evecs = evecs_dev;
  a.states = states_dev;
  a.out = out_dev;
  a.L[0] = L1;
  a.L[1] = L2;
  a.L[2] = L3;
  a.m0 = m0;
  a.n = n_states;
  a.total = (int64_t)n_states * nc * m0;
  TL_REQUIRE(tl::ceil_div(a.total, 256) <= INT32_MAX, "output of %lld values too large",
             (long long)a.total);
  hipLaunchKernelGGL(tl::bloch_kernel, dim3((unsigned)tl::ceil_div(a.total, 256)), dim3(256), 0,
                     (hipStream_t)stream, a);
  TL_CHECK_LAUNCH();
  return TL_OK;
}
