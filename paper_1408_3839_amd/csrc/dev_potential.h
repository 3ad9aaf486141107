// Device code of steps a2/a3 (sinc master vectors, lattice-summed potential
// vectors), shared by the single-system and the batched launches.
#pragma once
#include "common.h"
#include "dev_wave.h"

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

// Sum of the Gauss-Legendre cell integrals (the t h < 1/2 rule of cell_int)
// over a run of images whose cells sit at x0 - i D (i = 1 .. n_up) and
// x0 + i D (i = 1 .. n_dn) besides x0 itself, where x0 is the cell of the run
// nearest the Gaussian's centre.  At each rule node y the values
// f_i = exp(-t^2 (y -+ i D)^2) obey f_{i+1} = f_i r_i with
// r_{i+1} = r_i exp(-2 t^2 D^2) (q below): three exponentials per node
// instead of one per image.  Outward from x0 every ratio after the first is
// below one, and the first stays below exp(t^2 h D), so nothing overflows.
__device__ __forceinline__ double gl_run(double t2, double h, double D, double q, double x0,
                                         int n_up, int n_dn) {
  double acc = 0.0;
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const double o = 0.5 * h * kGLx[g];
    double sum = 0.0;
#pragma unroll
    for (int sg = 0; sg < 2; ++sg) {
      const double y0 = sg ? x0 - o : x0 + o;
      const double f0 = exp(-t2 * y0 * y0);
      sum += f0;
      if (n_up > 0) {  // y -> y - D
        double f = f0, r = exp(-t2 * D * (D - 2.0 * y0));
        for (int i = 0; i < n_up; ++i) {
          f *= r;
          r *= q;
          sum += f;
        }
      }
      if (n_dn > 0) {  // y -> y + D
        double f = f0, r = exp(-t2 * D * (D + 2.0 * y0));
        for (int i = 0; i < n_dn; ++i) {
          f *= r;
          r *= q;
          sum += f;
        }
      }
    }
    acc += kGLw[g] * sum;
  }
  return 0.5 * h * acc;
}

struct QuadArgs {  // the exponential-sum table, passed by value
  double t[TL_MAX_R];
  double w[TL_MAX_R];
};

// ---- open transverse dims: the y / z factors (one per group and term),
// b_q(x_i; y_g), which need no lattice sum.
struct DirectArgs {
  int R;
  double h;
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
                                   double* __restrict__ P, int b) {
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
  int chunks[3];                   // workgroups per term: ceil(c / kFoldNodes)
  int64_t out_off[3];
  int n_slots, R;
  double h;
};
constexpr int kFoldNodes = 4;  // window nodes per workgroup, one wave each

// ---- a2 + a3 (torus dims).  Site and lattice offsets are whole numbers of
// nodes, so every image factor is the cell integral b~_q[j] = b_q(j h; 0) of
// the "master" vector at an integer node j.  With one site per group each
// (window node, image) pair meets a different j, so the cell integrals are
// formed right where they are summed instead of being stored and read back.
// One wave per window node of the central cell: lanes take the images
// k = -K + lane, -K + lane + 64, ..., the wave sums them, and the node's value
// is replicated over the torus with the lattice period.
__device__ inline void fold_body(const FoldArgs& p, const QuadArgs& quad, double* __restrict__ P,
                                 int term, int slot, int chunk) {
  const int dim = p.dims[slot];
  const int c = p.c[slot], K = p.K[slot], n = p.n[slot];
  const int lane = threadIdx.x & 63;
  const int r = chunk * kFoldNodes + (int)(threadIdx.x >> 6);  // window node
  if (r >= c) return;  // whole wave
  const int t = term;
  const int g = t / p.R;
  const int q = t - g * p.R;
  const double tq = quad.t[q], h = p.h;
  const int rr = r - c / 2;  // offset of the node from the cell centre
  // A cell whose nearest point lies at t |y| > sqrt(750) from the Gaussian's
  // centre has an integral below 1e-326, zero in FP64: such images are
  // skipped, and a round of 64 images that holds only such cells costs the
  // wave no arithmetic (narrow Gaussians reach a few images only).
  const double tq2 = tq * tq;
  double acc = 0.0;
  const int m = (2 * K + 64) / 64;  // images per lane when each lane takes a run
  const double D = (double)c * h;
  // uniform per wave: Gaussians wide enough to reach every image of a window
  // of at least 193 images take lane runs of m consecutive images summed by
  // the recurrence of gl_run; narrower ones reach a few rounds of images,
  // which the per-image test below keeps cheaper
  if (tq * h < 0.5 && m >= 4 && tq2 * ((K + 1) * D) * ((K + 1) * D) <= 750.0) {
    const double qd = exp(-2.0 * tq2 * D * D);
    const int k_lo = -K + lane * m, k_hi = min(K, k_lo + m - 1);
    if (k_lo <= K) {
      for (int s = 0; s < (dim == 0 ? p.n_sites : 1); ++s) {
        if (dim == 0 && p.site_group[s] != g) continue;
        const int base = rr - (dim == 0 ? p.site_off[0][s] : p.group_off[dim][g]);
        // image nearest the centre within the run: x_k = (base - k c) h
        const int ks = min(k_hi, max(k_lo, (int)rint((double)base / (double)c)));
        const double x0 = (double)(base - ks * c) * h;
        const double e = fmax(fabs(x0) - 0.5 * h, 0.0);
        if (tq2 * e * e > 750.0) continue;  // the whole run is zero
        const double v = gl_run(tq2, h, D, qd, x0, k_hi - ks, ks - k_lo);
        acc += dim == 0 ? p.site_Z[s] * v : v;
      }
    }
  } else {
  for (int k = -K + lane; k <= K; k += 64) {
    if (dim == 0) {
      for (int s = 0; s < p.n_sites; ++s)
        if (p.site_group[s] == g) {
          const double x = (double)(rr - p.site_off[0][s] - k * c) * h;
          const double e = fmax(fabs(x) - 0.5 * h, 0.0);
          if (tq2 * e * e <= 750.0) acc += p.site_Z[s] * cell_int(tq, x, h, 0.0);
        }
    } else {
      const double x = (double)(rr - p.group_off[dim][g] - k * c) * h;
      const double e = fmax(fabs(x) - 0.5 * h, 0.0);
      if (tq2 * e * e <= 750.0) acc += cell_int(tq, x, h, 0.0);
    }
  }
  }
  const double v = wave_sum_dpp(acc) * (dim == 0 ? quad.w[q] : 1.0);
  // node r of the window lands on every i = rr (mod c) of the torus
  double* out = P + p.out_off[slot] + (int64_t)t * n;
  for (int i = (rr % c + c) % c + lane * c; i < n; i += 64 * c) out[i] = v;
}

// The whole of a2/a3 for one system in one launch: blocks [0, fold_blocks)
// run the torus dims (slot by slot, term-major within a slot), the rest the
// open transverse dims.  The branch is uniform per workgroup.
__device__ inline void potential_body(const DirectArgs& a, const FoldArgs& f,
                                      const QuadArgs& quad, int T, int fold_blocks,
                                      double* __restrict__ P, int64_t b) {
  if (b < fold_blocks) {
    int slot = 0;
    int64_t span = (int64_t)T * f.chunks[0];
    while (slot + 1 < f.n_slots && b >= span) {
      b -= span;
      ++slot;
      span = (int64_t)T * f.chunks[slot];
    }
    fold_body(f, quad, P, (int)(b / f.chunks[slot]), slot, (int)(b % f.chunks[slot]));
  } else {
    direct_body(a, quad, P, (int)(b - fold_blocks));
  }
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
  const double tt2 = tt * tt;
  double acc = 0.0;
  for (int s = 0; s < p.count; ++s) {
    if (p.group[s] != g) continue;
    // nuclei whose cell integral lies below FP64's underflow (as in
    // fold_body) are skipped; neighbouring nodes skip the same nuclei
    const double e = fmax(fabs(x - p.pos[s]) - 0.5 * p.h, 0.0);
    if (tt2 * e * e > 750.0) continue;
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
