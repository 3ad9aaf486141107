// Device code of step a1 (basis samples and FEM images), shared by the
// single-system and the batched launches.
#pragma once
#include "common.h"

namespace tl {
namespace dev {

constexpr double kGaussTailExponent = 46.0;  // images within exp(-46) of the peak

// Kernel arguments of the basis step; MaxFn bounds m0 (a launch that shares its
// arguments with other steps carries a shorter table).
template <int MaxFn>
struct BasisArgsN {
  FnParams fn[MaxFn];
  double x0[3], period[3];
  int64_t begin[3];   // flat start of each dimension (rows * n elements each)
  int64_t total;
  int n[3], periodic[3], rows[3];
  double h, box_origin0, box_a;
  int m0;
};
using BasisArgs = BasisArgsN<TL_MAX_M0>;

__device__ inline double factor_value(double x, double A, int l, double alpha, double coef) {
  double r = x - A;
  double e = exp(-alpha * r * r);
  return l ? coef * r * e : coef * e;
}

// g(x_i) for one row; on a torus the images A + j*P that can reach the
// interval within the tail cutoff are summed.
__device__ inline double sample(double x0, double h, double period, int periodic, double A, int l,
                                double alpha, double coef, int i) {
  double x = x0 + h * (double)i;
  if (!periodic) return factor_value(x, A, l, alpha, coef);
  double rcut = sqrt(kGaussTailExponent / alpha);
  int J = (int)ceil(rcut / period) + 1;
  double acc = 0.0;
  for (int j = -J; j <= J; ++j) acc += factor_value(x, A + (double)j * period, l, alpha, coef);
  return acc;
}

// Thread per (row, node) of the three dimensions; bx is the block index.
template <class Args>
__device__ inline void basis_body(const Args& p, double* __restrict__ G,
                                  double* __restrict__ AG, double* __restrict__ SG, int64_t bx) {
  int64_t idx = bx * blockDim.x + threadIdx.x;
  if (idx >= p.total) return;
  const int dim = idx >= p.begin[2] ? 2 : (idx >= p.begin[1] ? 1 : 0);
  const int64_t e = idx - p.begin[dim];
  const int n = p.n[dim];
  const int row = (int)(e / n);
  const int i = (int)(e - (int64_t)row * n);
  const int mu = row % p.m0;
  const int cell = row / p.m0;
  const FnParams& f = p.fn[mu];
  double A = f.center[dim];
  if (p.rows[dim] > p.m0) A += p.box_origin0 + (double)cell * p.box_a;
  const int l = f.l[dim];
  const double alpha = f.alpha, coef = f.coef[dim];
  const double x0 = p.x0[dim], per = p.period[dim];
  const int periodic = p.periodic[dim];
  double gi = sample(x0, p.h, per, periodic, A, l, alpha, coef, i);
  double gl, gr;
  if (periodic) {
    gl = sample(x0, p.h, per, periodic, A, l, alpha, coef, i == 0 ? n - 1 : i - 1);
    gr = sample(x0, p.h, per, periodic, A, l, alpha, coef, i == n - 1 ? 0 : i + 1);
  } else {
    gl = i == 0 ? 0.0 : sample(x0, p.h, per, periodic, A, l, alpha, coef, i - 1);
    gr = i == n - 1 ? 0.0 : sample(x0, p.h, per, periodic, A, l, alpha, coef, i + 1);
  }
  G[idx] = gi;
  AG[idx] = (2.0 * gi - gl - gr) / p.h;
  SG[idx] = (4.0 * gi + gl + gr) * (p.h / 6.0);
}


}  // namespace dev
}  // namespace tl
