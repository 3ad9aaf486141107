// Device code of step a6 (block DFT over one lattice axis), shared by the
// single-system and the batched launches.
#pragma once
#include "common.h"

namespace tl {
namespace dev {

struct DftArgs {
  const double* in;   // real (first pass) or complex input
  double* out;        // complex output
  int len;            // transform length along the axis
  int64_t inner;      // product of the extents after the axis, times m0*m0
  int real_in;
};

constexpr int kMaxTwiddle = 4096;  // lengths up to this keep their twiddles in LDS

// Workgroup per (outer, j) output line segment: the twiddles w^(j k mod L)
// of its j are tabulated once in LDS, threads run over consecutive block
// entries r (coalesced loads along the m0*m0 entries).
template <bool REAL_IN, bool TABLE>
__device__ inline void dft_axis_body(const DftArgs& a, int64_t oj, int64_t by, double* tw) {
  // oj = outer * len + j; by = chunk of r; tw: [len][2] (cos, sin) in LDS
  const int j = (int)(oj % a.len);
  const int64_t outer = oj / a.len;
  const int64_t r = by * blockDim.x + threadIdx.x;
  const double inv = 2.0 / (double)a.len;
  if (TABLE) {
    for (int k = threadIdx.x; k < a.len; k += blockDim.x) {
      int p = (int)(((int64_t)j * k) % a.len);
      double s, c;
      sincospi((double)p * inv, &s, &c);  // w^p = cos(2 pi p/L) - i sin(2 pi p/L)
      tw[2 * k] = c;
      tw[2 * k + 1] = s;
    }
    __syncthreads();
  }
  if (r >= a.inner) return;
  const int64_t base = outer * a.len * a.inner + r;
  double re = 0.0, im = 0.0;
  int p = 0;
#pragma unroll 8
  for (int k = 0; k < a.len; ++k) {
    double s, c;
    if (TABLE) {
      c = tw[2 * k];
      s = tw[2 * k + 1];
    } else {
      sincospi((double)p * inv, &s, &c);
      p += j;
      if (p >= a.len) p -= a.len;
    }
    int64_t src = base + (int64_t)k * a.inner;
    if (REAL_IN) {
      double x = a.in[src];
      re += c * x;
      im -= s * x;
    } else {
      double xr = a.in[2 * src], xi = a.in[2 * src + 1];
      re += c * xr + s * xi;
      im += c * xi - s * xr;
    }
  }
  const int64_t o = (outer * a.len + j) * a.inner + r;
  a.out[2 * o] = re;
  a.out[2 * o + 1] = im;
}

}  // namespace dev
}  // namespace tl
