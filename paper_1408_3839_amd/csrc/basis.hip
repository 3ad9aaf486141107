// Step a1: nodal samples of the separable Gaussian basis and their 1D FEM
// images A g, S g (Sec. 3.4: hat-function interpolant of g, 1D stiffness
// (1/h) tridiag(-1,2,-1) and mass (h/6) tridiag(1,4,1)).
#include <cmath>

#include "common.h"
#include "dev_basis.h"
#include "host_plans.h"

namespace tl {
namespace {

__global__ __launch_bounds__(256) void basis_kernel(dev::BasisArgs p, double* __restrict__ G,
                                                    double* __restrict__ AG,
                                                    double* __restrict__ SG) {
  dev::basis_body(p, G, AG, SG, blockIdx.x);
}

}  // namespace

void make_basis_args(const Geometry& g, const tl_system* s, dev::BasisArgs* out) {
  dev::BasisArgs& p = *out;
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
    p.x0[d] = g.x0[d];
    p.n[d] = g.n[d];
    p.periodic[d] = g.periodic[d];
    p.period[d] = g.periodic[d] ? g.L[d] * g.a[d] : 0.0;
    p.rows[d] = (int)g.basis_rows[d];
    p.begin[d] = g.basis_off[d];
  }
  p.total = g.basis_elems;
}

tl_status build_basis(const Geometry& g, const tl_system* s, double* G, double* AG, double* SG,
                      hipStream_t stream) {
  dev::BasisArgs p;
  make_basis_args(g, s, &p);
  hipLaunchKernelGGL(basis_kernel, dim3((unsigned)ceil_div(p.total, 256)), dim3(256), 0, stream, p,
                     G, AG, SG);
  TL_CHECK_LAUNCH();
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
