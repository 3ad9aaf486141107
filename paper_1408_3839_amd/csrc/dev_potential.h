// Device code of steps a2/a3 (sinc master vectors, lattice-summed potential
// vectors), shared by the single-system and the batched launches.
#pragma once
#include "common.h"

namespace tl {
namespace dev {

// 8-point Gauss-Legendre rule on [-1, 1] (Abramowitz & Stegun, Table 25.4).
static __constant__ double kGLx[4] = {0.18343464249564984, 0.525532409916329, 0.7966664774136267,
                               0.9602898564975363};
static __constant__ double kGLw[4] = {0.36268378337836205, 0.3137066458778876, 0.22238103445337473,
                               0.10122853629037562};

// int_{x-h/2}^{x+h/2} exp(-t^2 (y-A)^2) dy.  For t*h >= 1/2 the erf difference
// is formed where it does not cancel (erfc of two positive or two negative
// arguments); below, every erf difference cancels, and the integrand is so
// smooth on the cell that Gauss-Legendre reaches full precision.
__device__ __forceinline__ double cell_int(double t, double x, double h, double A) {
  if (t * h < 0.5) {
    double acc = 0.0;
    double c = x - A;
    double t2 = t * t;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      double y1 = c + 0.5 * h * kGLx[k];
      double y2 = c - 0.5 * h * kGLx[k];
      acc += kGLw[k] * (exp(-t2 * y1 * y1) + exp(-t2 * y2 * y2));
    }
    return 0.5 * h * acc;
  }
  double u = t * (x - 0.5 * h - A);
  double v = t * (x + 0.5 * h - A);
  double d;
  if (u >= 0.0)
    d = erfc(u) - erfc(v);
  else if (v <= 0.0)
    d = erfc(-v) - erfc(-u);
  else
    d = erf(v) + erf(-u);
  return d * (0.886226925452758014 / t);  // sqrt(pi)/2 / t
}

struct QuadArgs {  // the exponential-sum table, passed by value
  double t[TL_MAX_R];
  double w[TL_MAX_R];
};

// ---- a2 + open transverse dims in one launch.
// Blocks [0, master_blocks): master vectors b~_q[j], j = -J..J.
// Blocks after that: the y / z factors of open dims (one per group and
// term), b_q(x_i; y_g), which need no lattice sum.
struct DirectArgs {
  int R, J, master_blocks;
  double h;
  // open transverse dims (y = 1, z = 2)
  int n_open;                 // number of open transverse dims handled here (0..2)
  int open_dim[2];
  int n[2];
  double x0[2];
  int64_t out_off[2];         // element offset of the dim in P
  int blocks_per_term[2];
  int T;                      // terms = groups * R
  double gpos[2][TL_MAX_SITES];  // group coordinate on each open dim
};

__device__ inline void direct_body(const DirectArgs& a, const QuadArgs& quad,
                                   double* __restrict__ master, double* __restrict__ P, int b) {
  if (b < a.master_blocks) {
    int64_t idx = (int64_t)b * blockDim.x + threadIdx.x;
    int64_t width = 2 * (int64_t)a.J + 1;
    if (idx >= (int64_t)a.R * width) return;
    int q = (int)(idx / width);
    int j = (int)(idx - (int64_t)q * width) - a.J;
    master[idx] = cell_int(quad.t[q], (double)j * a.h, a.h, 0.0);
    return;
  }
  b -= a.master_blocks;
  int od = 0;
  int span0 = a.T * a.blocks_per_term[0];
  if (a.n_open == 2 && b >= span0) {
    od = 1;
    b -= span0;
  }
  int t = b / a.blocks_per_term[od];
  int chunk = b - t * a.blocks_per_term[od];
  int i = chunk * blockDim.x + threadIdx.x;
  if (i >= a.n[od]) return;
  int g = t / a.R, q = t - g * a.R;
  double x = a.x0[od] + a.h * (double)i;
  P[a.out_off[od] + (int64_t)t * a.n[od] + i] = cell_int(quad.t[q], x, a.h, a.gpos[od][g]);
}

struct FoldArgs {
  int n_sites;
  int site_group[TL_MAX_SITES];
  int site_off[3][TL_MAX_SITES];   // site offset per dim, in nodes
  double site_Z[TL_MAX_SITES];
  int group_off[3][TL_MAX_SITES];  // representative offset of each group per dim
  int dims[3];                     // periodic dims handled by this launch
  int c[3], K[3], n[3];
  int64_t out_off[3];
  int R, J;
};

// ---- a3 (torus dims): workgroup per (term, periodic dim).  Threads split the
// image sum of every window node, partial sums meet in LDS, the window is
// then replicated over the torus.
__device__ inline void fold_body(const FoldArgs& p, const QuadArgs& quad,
                                 const double* __restrict__ master, double* __restrict__ P,
                                 int term, int slot, double* sh) {
  // sh: win[c] then part[256] (dynamic LDS of the launch)
  const int dim = p.dims[slot];
  const int c = p.c[slot], K = p.K[slot], n = p.n[slot];
  double* win = sh;
  double* part = sh + c;
  const int t = term;
  const int g = t / p.R;
  const int q = t - g * p.R;
  const double* mq = master + (int64_t)q * (2 * p.J + 1) + p.J;  // mq[j], j in [-J, J]
  const int half = c / 2;
  const int tid = threadIdx.x;
  auto image_sum = [&](int rr, int k_first, int k_step) {
    double acc = 0.0;
    for (int k = -K + k_first; k <= K; k += k_step) {
      if (dim == 0) {
        for (int s = 0; s < p.n_sites; ++s)
          if (p.site_group[s] == g) acc += p.site_Z[s] * mq[rr - p.site_off[0][s] - k * c];
      } else {
        acc += mq[rr - p.group_off[dim][g] - k * c];
      }
    }
    return acc;
  };
  const double wscale = dim == 0 ? quad.w[q] : 1.0;
  if (c <= 256) {
    const int np = 256 / c;
    if (tid < np * c) part[tid] = image_sum(tid % c - half, tid / c, np);
    __syncthreads();
    if (tid < c) {
      double v = 0.0;
      for (int s2 = 0; s2 < np; ++s2) v += part[tid + s2 * c];
      win[tid] = v * wscale;
    }
  } else {
    for (int r = tid; r < c; r += blockDim.x) win[r] = image_sum(r - half, 0, 1) * wscale;
  }
  __syncthreads();
  double* out = P + p.out_off[slot] + (int64_t)t * n;
  for (int i = tid; i < n; i += blockDim.x) out[i] = win[(i + half) % c];
}

constexpr int kNucChunk = 80;
struct BoxArgs {
  double pos[kNucChunk];  // nucleus x coordinate
  double Z[kNucChunk];
  int group[kNucChunk];
  int count, R, n, accumulate;
  double x0, h;
};

// ---- a3 (open dim 0, box mode): thread per (term, node), direct cell
// integrals of every nucleus of the chunk.
__device__ inline void box_potential_body(const BoxArgs& p, const QuadArgs& quad,
                                          double* __restrict__ P, int64_t bx, int t) {
  int64_t idx = bx * blockDim.x + threadIdx.x;
  if (idx >= p.n) return;
  int g = t / p.R;
  int q = t - g * p.R;
  double x = p.x0 + p.h * (double)idx;
  double tt = quad.t[q];
  double acc = 0.0;
  for (int s = 0; s < p.count; ++s) {
    if (p.group[s] != g) continue;
    acc += p.Z[s] * cell_int(tt, x, p.h, p.pos[s]);
  }
  acc *= quad.w[q];
  double* out = P + (int64_t)t * p.n + idx;
  if (p.accumulate)
    *out += acc;
  else
    *out = acc;
}

}  // namespace dev
}  // namespace tl
