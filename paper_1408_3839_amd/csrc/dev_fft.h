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
// entries r (coalesced loads along the m0*m0 entries).  Lines of at most 128
// entries leave threads over: the k sum is then split over 2 or 4 groups of
// threads (k = g, g + groups, ...) whose partial sums meet in LDS in group
// order.  Dynamic LDS: max(2 len (TABLE), 2 * 256) doubles, the twiddles
// first, the partials afterwards in the same space.
template <bool REAL_IN, bool TABLE>
__device__ inline void dft_axis_body(const DftArgs& a, int64_t oj, int64_t by, double* tw) {
  // oj = outer * len + j; by = chunk of 256 entries r
  const int j = (int)(oj % a.len);
  const int64_t outer = oj / a.len;
  const int span = a.inner <= 64 ? 64 : (a.inner <= 128 ? 128 : 256);
  const int ng = 256 / span, kg = (int)threadIdx.x / span, rl = (int)threadIdx.x % span;
  const int64_t r = by * span + rl;
  const bool valid = r < a.inner;
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
  const int64_t base = outer * a.len * a.inner + r;
  double re = 0.0, im = 0.0;
  if (valid) {
    int p = (int)(((int64_t)j * kg) % a.len);
    const int pstep = (int)(((int64_t)j * ng) % a.len);
#pragma unroll 16
    for (int k = kg; k < a.len; k += ng) {
      double s, c;
      if (TABLE) {
        c = tw[2 * k];
        s = tw[2 * k + 1];
      } else {
        sincospi((double)p * inv, &s, &c);
        p += pstep;
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
  }
  if (ng > 1) {  // uniform: every thread reaches the barriers
    if (TABLE) __syncthreads();  // the twiddle reads are done; the partials reuse the space
    double* part = tw;
    part[2 * threadIdx.x] = re;
    part[2 * threadIdx.x + 1] = im;
    __syncthreads();
    if (kg != 0) return;
    for (int g = 1; g < ng; ++g) {
      re += part[2 * (g * span + rl)];
      im += part[2 * (g * span + rl) + 1];
    }
  }
  if (!valid) return;
  const int64_t o = (outer * a.len + j) * a.inner + r;
  a.out[2 * o] = re;
  a.out[2 * o + 1] = im;
}

}  // namespace dev
}  // namespace tl
