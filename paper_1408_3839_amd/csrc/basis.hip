// Step a1: nodal samples of the separable Gaussian basis and their 1D FEM
// images A g, S g (Sec. 3.4: hat-function interpolant of g, 1D stiffness
// (1/h) tridiag(-1,2,-1) and mass (h/6) tridiag(1,4,1)).
#include <cmath>

#include "common.h"

namespace tl {
namespace {

constexpr double kGaussTailExponent = 46.0;  // images within exp(-46) of the peak

struct BasisArgs {
  FnParams fn[TL_MAX_M0];
  double x0, h, period, box_origin0, box_a;
  int n, periodic, rows, m0, box_dim;  // box_dim: rows are cells x functions
};

__device__ inline double factor_value(double x, double A, int l, double alpha, double coef) {
  double r = x - A;
  double e = exp(-alpha * r * r);
  return l ? coef * r * e : coef * e;
}

// g(x_i) for one row; on a torus the images A + j*P that can reach the
// interval within the tail cutoff are summed.
__device__ inline double sample(const BasisArgs& p, double A, int l, double alpha, double coef,
                                int i) {
  double x = p.x0 + p.h * (double)i;
  if (!p.periodic) return factor_value(x, A, l, alpha, coef);
  double rcut = sqrt(kGaussTailExponent / alpha);
  int J = (int)ceil(rcut / p.period) + 1;
  double acc = 0.0;
  for (int j = -J; j <= J; ++j) acc += factor_value(x, A + (double)j * p.period, l, alpha, coef);
  return acc;
}

__global__ __launch_bounds__(256) void basis_kernel(BasisArgs p, double* __restrict__ G,
                                                    double* __restrict__ AG,
                                                    double* __restrict__ SG) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int64_t total = (int64_t)p.rows * p.n;
  if (idx >= total) return;
  int row = (int)(idx / p.n);
  int i = (int)(idx - (int64_t)row * p.n);
  int mu = row % p.m0;
  int cell = row / p.m0;
  const FnParams& f = p.fn[mu];
  int dim = p.box_dim;  // the dimension index of this launch
  double A = f.center[dim];
  if (p.rows > p.m0) A += p.box_origin0 + (double)cell * p.box_a;
  int l = f.l[dim];
  double alpha = f.alpha, coef = f.coef[dim];
  double gi = sample(p, A, l, alpha, coef, i);
  double gl, gr;
  if (p.periodic) {
    gl = sample(p, A, l, alpha, coef, i == 0 ? p.n - 1 : i - 1);
    gr = sample(p, A, l, alpha, coef, i == p.n - 1 ? 0 : i + 1);
  } else {
    gl = i == 0 ? 0.0 : sample(p, A, l, alpha, coef, i - 1);
    gr = i == p.n - 1 ? 0.0 : sample(p, A, l, alpha, coef, i + 1);
  }
  G[idx] = gi;
  AG[idx] = (2.0 * gi - gl - gr) / p.h;
  SG[idx] = (4.0 * gi + gl + gr) * (p.h / 6.0);
}

}  // namespace

tl_status build_basis(const Geometry& g, const tl_system* s, double* G, double* AG, double* SG,
                      hipStream_t stream) {
  BasisArgs p;
  std::memset(&p, 0, sizeof(p));
  for (int mu = 0; mu < g.m0; ++mu) {
    for (int d = 0; d < 3; ++d) {
      p.fn[mu].center[d] = s->fn_center[3 * mu + d];
      p.fn[mu].coef[d] = s->fn_coef[3 * mu + d];
      p.fn[mu].l[d] = s->fn_l[3 * mu + d];
    }
    p.fn[mu].alpha = s->fn_alpha[mu];
  }
  p.m0 = g.m0;
  p.h = g.h;
  p.box_origin0 = g.box_origin0;
  p.box_a = g.a[0];
  for (int d = 0; d < 3; ++d) {
    p.x0 = g.x0[d];
    p.n = g.n[d];
    p.periodic = g.periodic[d];
    p.period = g.periodic[d] ? g.L[d] * g.a[d] : 0.0;
    p.rows = (int)g.basis_rows[d];
    p.box_dim = d;
    int64_t total = (int64_t)p.rows * p.n;
    int blocks = (int)ceil_div(total, 256);
    hipLaunchKernelGGL(basis_kernel, dim3(blocks), dim3(256), 0, stream, p, G + g.basis_off[d],
                       AG + g.basis_off[d], SG + g.basis_off[d]);
    TL_CHECK_LAUNCH();
  }
  return TL_OK;
}

}  // namespace tl

extern "C" tl_status tl_build_basis(const tl_system* sys, double* G_dev, double* AG_dev,
                                    double* SG_dev, void* stream) {
  tl::clear_error();
  tl::Geometry g;
  TL_TRY(tl::digest(sys, &g));
  TL_REQUIRE(G_dev && AG_dev && SG_dev, "null output array");
  return tl::build_basis(g, sys, G_dev, AG_dev, SG_dev, (hipStream_t)stream);
}
