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

// The orbital of state (j, m) on the grid is a canonical tensor of rank m0
// (the basis is separable and the Bloch phase factorises over the dims):
//   psi(x) = sum_mu w_mu prod_d phi^d_mu(x_d),  w_mu = L^(-1/2) u_(j,m)[mu],
//   phi^d_mu(x_i) = sum_(c=0)^(L_d - 1) exp(2 pi i j_d c / L_d) g^d_mu(x_i - c a_d),
// the shifted periodised sample read c * cell_nodes_d nodes back on the torus
// (an open dim has L_d = 1: phi = g).
struct OrbArgs {
  const double* G;      // basis samples, dim d at off[d]: [m0][n_d]
  const double* evecs;  // [nc][m0][m0] complex, column m = eigenvector m
  const int* states;    // [n] flat state indices j m0 + m
  double* coef;         // [n][m0] complex
  double* fac;          // [n][elems] complex, dims as in G
  int L[3], cn[3], n[3], m0, ns;
  int64_t off[3], elems;
};

__global__ __launch_bounds__(256) void orbital_factors_kernel(OrbArgs a) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)a.ns * a.elems) return;
  const int s = (int)(e / a.elems);
  const int64_t r = e - (int64_t)s * a.elems;
  const int d = r >= a.off[2] ? 2 : (r >= a.off[1] ? 1 : 0);
  const int64_t rr = r - a.off[d];
  const int mu = (int)(rr / a.n[d]);
  const int i = (int)(rr - (int64_t)mu * a.n[d]);
  const int nc = a.L[0] * a.L[1] * a.L[2];
  const int st = a.states[s];
  double* o = a.fac + 2 * e;
  const bool ok = st >= 0 && st < nc * a.m0;
  if (!ok) {
    o[0] = NAN;
    o[1] = NAN;
    if (d == 0 && i == 0) {
      a.coef[2 * ((int64_t)s * a.m0 + mu)] = NAN;
      a.coef[2 * ((int64_t)s * a.m0 + mu) + 1] = NAN;
    }
    return;
  }
  const int j = st / a.m0, m = st - j * a.m0;
  const int j12 = j / a.L[2], j3 = j - j12 * a.L[2];
  const int j1 = j12 / a.L[1], j2 = j12 - j1 * a.L[1];
  const int jd = d == 0 ? j1 : (d == 1 ? j2 : j3);
  const int Ld = a.L[d], nd = a.n[d];
  const double* g = a.G + a.off[d] + (int64_t)mu * nd;
  double re = 0.0, im = 0.0;
  for (int c = 0; c < Ld; ++c) {
    int src = i - (int)(((int64_t)c * a.cn[d]) % nd);
    if (src < 0) src += nd;
    const double v = g[src];
    if (v == 0.0) continue;
    double sn, cs;
    sincospi(2.0 * (double)((int64_t)jd * c % Ld) / Ld, &sn, &cs);
    re = fma(cs, v, re);
    im = fma(sn, v, im);
  }
  o[0] = re;
  o[1] = im;
  if (d == 0 && i == 0) {
    const double rs = 1.0 / sqrt((double)nc);
    const double* u = a.evecs + 2 * (((int64_t)j * a.m0 + mu) * a.m0 + m);
    a.coef[2 * ((int64_t)s * a.m0 + mu)] = rs * u[0];
    a.coef[2 * ((int64_t)s * a.m0 + mu) + 1] = rs * u[1];
  }
}

// The open chain's orbital with coefficients U over the L m0 functions is a
// canonical tensor of rank m0 as well (the transverse factors do not depend
// on the cell): psi = sum_mu phi^x_mu x g^y_mu x g^z_mu with
// phi^x_mu(x_i) = sum_c U[c m0 + mu] g^x_(c,mu)(x_i).
struct ChainOrbArgs {
  const double* G;      // box-mode samples: dim 0 [L m0][n0], dims 1, 2 [m0][n_d]
  const double* U;      // [ns][L m0]
  double* fac;          // [ns][m0 (n0 + n1 + n2)]
  int L, m0, ns, n[3];
  int64_t goff[3], foff[3], elems;
};

__global__ __launch_bounds__(256) void chain_orbital_kernel(ChainOrbArgs a) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (int64_t)a.ns * a.elems) return;
  const int s = (int)(e / a.elems);
  const int64_t r = e - (int64_t)s * a.elems;
  const int d = r >= a.foff[2] ? 2 : (r >= a.foff[1] ? 1 : 0);
  const int64_t rr = r - a.foff[d];
  const int mu = (int)(rr / a.n[d]);
  const int i = (int)(rr - (int64_t)mu * a.n[d]);
  double v;
  if (d == 0) {
    const double* u = a.U + (int64_t)s * a.L * a.m0;
    v = 0.0;
    for (int c = 0; c < a.L; ++c) {
      const int f = c * a.m0 + mu;
      v = fma(u[f], a.G[a.goff[0] + (int64_t)f * a.n[0] + i], v);
    }
  } else {
    v = a.G[a.goff[d] + (int64_t)mu * a.n[d] + i];
  }
  a.fac[e] = v;
}

}  // namespace
}  // namespace tl

extern "C" tl_status tl_chain_orbital_factors(const tl_system* sys, const double* G_dev,
                                              const double* evecs_dev, int n_states,
                                              double* factors_dev, void* stream) {
  tl::clear_error();
  tl::Geometry g;
  TL_TRY(tl::digest(sys, &g));
  if (g.mode != TL_MODE_BOX) {
    tl::set_error("orbital factors of an open chain need a box-mode system");
    return TL_EUNSUPPORTED;
  }
  TL_REQUIRE(n_states >= 0, "n_states = %d < 0", n_states);
  if (n_states == 0) return TL_OK;
  TL_REQUIRE(G_dev && evecs_dev && factors_dev, "null array argument");
  tl::ChainOrbArgs a;
  a.G = G_dev;
  a.U = evecs_dev;
  a.fac = factors_dev;
  a.L = g.L[0];
  a.m0 = g.m0;
  a.ns = n_states;
  int64_t fo = 0;
  for (int d = 0; d < 3; ++d) {
    a.n[d] = g.n[d];
    a.goff[d] = g.basis_off[d];
    a.foff[d] = fo;
    fo += (int64_t)g.m0 * g.n[d];
  }
  a.elems = fo;
  const int64_t total = (int64_t)n_states * a.elems;
  TL_REQUIRE(tl::ceil_div(total, 256) <= INT32_MAX, "output of %lld values too large",
             (long long)total);
  hipLaunchKernelGGL(tl::chain_orbital_kernel, dim3((unsigned)tl::ceil_div(total, 256)),
                     dim3(256), 0, (hipStream_t)stream, a);
  TL_CHECK_LAUNCH();
  return TL_OK;
}

extern "C" tl_status tl_bloch_orbital_factors(const tl_system* sys, const double* G_dev,
                                              const double* evecs_dev, const int* states_dev,
                                              int n_states, double* coef_dev,
                                              double* factors_dev, void* stream) {
  tl::clear_error();
  tl::Geometry g;
  TL_TRY(tl::digest(sys, &g));
  if (g.mode != TL_MODE_PERIODIC) {
    tl::set_error("orbital factors of Bloch states need a periodic system");
    return TL_EUNSUPPORTED;
  }
  TL_REQUIRE(n_states >= 0, "n_states = %d < 0", n_states);
  if (n_states == 0) return TL_OK;
  TL_REQUIRE(G_dev && evecs_dev && states_dev && coef_dev && factors_dev, "null array argument");
  tl::OrbArgs a;
  a.G = G_dev;
  a.evecs = evecs_dev;
  a.states = states_dev;
  a.coef = coef_dev;
  a.fac = factors_dev;
  for (int d = 0; d < 3; ++d) {
    a.L[d] = g.L[d];
    a.n[d] = g.n[d];
    a.cn[d] = g.L[d] > 1 ? g.cell_nodes[d] : 0;
    a.off[d] = g.basis_off[d];
  }
  a.m0 = g.m0;
  a.ns = n_states;
  a.elems = g.basis_elems;
  const int64_t total = (int64_t)n_states * a.elems;
  TL_REQUIRE(tl::ceil_div(total, 256) <= INT32_MAX, "output of %lld values too large",
             (long long)total);
  hipLaunchKernelGGL(tl::orbital_factors_kernel, dim3((unsigned)tl::ceil_div(total, 256)),
                     dim3(256), 0, (hipStream_t)stream, a);
  TL_CHECK_LAUNCH();
  return TL_OK;
}

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
