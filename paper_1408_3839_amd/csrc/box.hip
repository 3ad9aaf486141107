// Step a8, assembly: full core Hamiltonian and mass matrix of an open-boundary
// chain (Sec. 3.3, eq. (nuc_pot) and proof of Lemma 3.1; Lemma 3.1 block
// sparsity; Sec. 3.4).  Every basis function f = (cell c, mu) has its own x
// factor; the y and z factors are those of the unit cell.  So
//   H[f][f'] = sum_t -C^x_t[f][f'] Cy_t[mu][nu] Cz_t[mu][nu]
//              + 1/2 D^x[f][f'] My Mz[mu][nu] + 1/2 M^x[f][f'] (Dy Mz + My Dz)[mu][nu]
//   S[f][f'] = M^x[f][f'] My Mz[mu][nu]
// with C^x_t = G diag(p_t) G^T over the x nodes (the paper's
// G diag(p_q) G^T contraction), D^x, M^x the FEM forms.  The transverse
// factors come from the periodic-path contraction kernels restricted to
// y and z.  The x contraction is symmetric and banded: a 32 x 32 tile of
// functions only sums over the nodes where both tiles' Gaussians are above
// exp(-46) of their peak (Lemma 3.1's overlap constant L0, made exact to
// FP64 resolution), tiles without overlap are zero, and every term's
// contribution is folded into H and S in the tile epilogue, so no
// per-term matrix is stored.
#include <algorithm>
#include <cmath>

#include "common.h"
#include "host_plans.h"

namespace tl {
namespace {

using namespace dev;

constexpr int kBoxKT = 16;          // nodes per LDS stage
constexpr int kBoxMaxT = 64;        // potential terms held in LDS
constexpr int kBoxLD = kBoxKT + 1;
constexpr double kSupportExp = 46.0;

struct CoefArgs {
  const double* Cy;   // compact [(T+2) m0][m0] of dim 1
  const double* Cz;   // compact of dim 2
  double* coef;       // [T+2][m0][m0]
  double* smass;      // [m0][m0]
  int m0, T;
};

// coef[t][mu][nu]: the factor that multiplies C^x_t in H; smass = My Mz.
__global__ __launch_bounds__(256) void box_coef_kernel(CoefArgs a) {
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  int m2 = a.m0 * a.m0;
  if (idx >= (a.T + 2) * m2) return;
  int t = idx / m2, e = idx - t * m2, mu = e / a.m0, nu = e - mu * a.m0;
  // compact layout: row = t' * m0 + nu, column = mu (one shift)
  auto cy = [&](int tt) { return a.Cy[(tt * a.m0 + nu) * a.m0 + mu]; };
  auto cz = [&](int tt) { return a.Cz[(tt * a.m0 + nu) * a.m0 + mu]; };
  double v;
  if (t < a.T)
    v = -cy(t) * cz(t);
  else if (t == a.T)
    v = 0.5 * cy(a.T + 1) * cz(a.T + 1);                 // D^x term: 1/2 My Mz
  else
    v = 0.5 * (cy(a.T) * cz(a.T + 1) + cy(a.T + 1) * cz(a.T));  // M^x: 1/2 (Dy Mz + My Dz)
  a.coef[idx] = v;
  if (t == a.T + 1) a.smass[e] = cy(a.T + 1) * cz(a.T + 1);
}

struct BoxArgs2 {
  const double* G;    // [Nb][n] x factors
  const double* AG;
  const double* SG;
  const double* P;    // [T][n]
  const double* coef;
  const double* smass;
  double* H;
  double* S;
  double center[TL_MAX_M0];  // x offset of function mu in its cell
  double radius[TL_MAX_M0];  // support radius sqrt(46 / alpha_mu)
  double box_origin0, a0, x0, h;
  int n, Nb, m0, T, ntiles;
};

__device__ inline void tile_support(const BoxArgs2& a, int f0, double& lo, double& hi) {
  lo = 1e300;
  hi = -1e300;
  int f1 = min(a.Nb, f0 + 32);
  for (int f = f0; f < f1; ++f) {
    int c = f / a.m0, mu = f - c * a.m0;
    double X = a.box_origin0 + c * a.a0 + a.center[mu];
    lo = fmin(lo, X - a.radius[mu]);
    hi = fmax(hi, X + a.radius[mu]);
  }
}

// Workgroup per upper-triangle tile pair (tr <= tc) of 32 x 32 functions.
__global__ __launch_bounds__(256) void box_contract_kernel(BoxArgs2 a) {
  __shared__ double Gr[kBM][kBoxLD];   // rows: G of the row functions
  __shared__ double Ar[kBM][kBoxLD];   // rows: A g
  __shared__ double Sr[kBM][kBoxLD];   // rows: S g
  __shared__ double Gc[kBN][kBoxLD];   // columns: G of the column functions
  __shared__ double Ps[kBoxMaxT][kBoxKT];
  // upper-triangle pair from the linear block index
  int b = blockIdx.x, tr = 0;
  while (b >= a.ntiles - tr) {
    b -= a.ntiles - tr;
    ++tr;
  }
  const int tc = tr + b;
  const int row0 = tr * kBM, col0 = tc * kBN;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  double rlo, rhi, clo, chi;
  tile_support(a, row0, rlo, rhi);
  tile_support(a, col0, clo, chi);
  int klo = (int)ceil((fmax(rlo, clo) - a.x0) / a.h);
  int khi = (int)floor((fmin(rhi, chi) - a.x0) / a.h) + 1;
  klo = max(klo, 0);
  khi = min(khi, a.n);
  double h_acc[4] = {0.0, 0.0, 0.0, 0.0}, s_acc[4] = {0.0, 0.0, 0.0, 0.0};
  const int orow = row0 + wm * 16 + (lane >> 4);   // + 4 r (f64 result layout)
  const int ocol = col0 + wn * 16 + (lane & 15);
  for (int k0 = klo; k0 < khi; k0 += kBoxKT) {
    for (int e = tid; e < kBM * kBoxKT; e += 256) {
      int r = e / kBoxKT, kk = e - r * kBoxKT, i = k0 + kk;
      bool ok = i < khi;
      int fr = row0 + r, fc = col0 + r;
      bool rok = ok && fr < a.Nb, cok = ok && fc < a.Nb;
      Gr[r][kk] = rok ? a.G[(int64_t)fr * a.n + i] : 0.0;
      Ar[r][kk] = rok ? a.AG[(int64_t)fr * a.n + i] : 0.0;
      Sr[r][kk] = rok ? a.SG[(int64_t)fr * a.n + i] : 0.0;
      Gc[r][kk] = cok ? a.G[(int64_t)fc * a.n + i] : 0.0;
    }
    for (int e = tid; e < a.T * kBoxKT; e += 256) {
      int t = e / kBoxKT, kk = e - t * kBoxKT, i = k0 + kk;
      Ps[t][kk] = i < khi ? a.P[(int64_t)t * a.n + i] : 0.0;
    }
    __syncthreads();
    for (int t = 0; t < a.T + 2; ++t) {
      f64x4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int kk = 0; kk < kBoxKT; kk += 4) {
        const int r = wm * 16 + (lane & 15), k = kk + (lane >> 4);
        double av = t < a.T ? Gr[r][k] * Ps[t][k] : (t == a.T ? Ar[r][k] : Sr[r][k]);
        double bv = Gc[wn * 16 + (lane & 15)][k];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int f = orow + 4 * r, fp = ocol;
        const int mu = f % a.m0, nu = fp % a.m0;
        h_acc[r] += a.coef[(t * a.m0 + mu) * a.m0 + nu] * acc[r];
        if (t == a.T + 1) s_acc[r] += a.smass[mu * a.m0 + nu] * acc[r];
      }
    }
    __syncthreads();
  }
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int f = orow + 4 * r, fp = ocol;
    // a diagonal tile keeps its upper half only, so that H and S are exactly
    // symmetric (the two halves would differ by rounding order)
    if (f < a.Nb && fp < a.Nb && (tr != tc || f <= fp)) {
      a.H[(int64_t)f * a.Nb + fp] = h_acc[r];
      a.S[(int64_t)f * a.Nb + fp] = s_acc[r];
      if (f != fp) {
        a.H[(int64_t)fp * a.Nb + f] = h_acc[r];
        a.S[(int64_t)fp * a.Nb + f] = s_acc[r];
      }
    }
  }
}

__global__ __launch_bounds__(256) void transverse_contract_kernel(ContractArgs a) {
  contract_f64_body(a, blockIdx.x);
}

__global__ __launch_bounds__(256) void transverse_reduce_kernel(ReduceArgs a, int64_t total) {
  reduce_partials_body(a, total, blockIdx.x);
}

}  // namespace

size_t box_workspace_bytes(const Geometry& g) {
  size_t base = assemble_workspace_bytes(g, TL_FP64, 0, kDefaultContractBlocks);
  size_t m2 = (size_t)g.m0 * g.m0;
  return base + align_up(sizeof(double) * ((size_t)g.pot_terms + 3) * m2, 256);
}

tl_status assemble_box(const Geometry& g, const tl_system* s, const double* G, const double* AG,
                       const double* SG, const double* P, tl_precision prec, double* H,
                       double* S, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (prec != TL_FP64) {
    set_error("box-mode assembly runs in FP64");
    return TL_EUNSUPPORTED;
  }
  if (g.pot_terms > kBoxMaxT) {
    set_error("box mode takes at most %d potential terms", kBoxMaxT);
    return TL_EUNSUPPORTED;
  }
  const size_t need = box_workspace_bytes(g);
  if (ws == nullptr || ws_bytes < need) {
    set_error("box assembly workspace: need %zu bytes, got %zu", need, ws_bytes);
    return TL_EWORKSPACE;
  }
  // transverse factors: the periodic-path contraction over y and z only
  AssemblyPlan ap;
  const size_t base = assemble_workspace_bytes(g, TL_FP64, 0, kDefaultContractBlocks);
  TL_TRY(plan_assembly(g, G, AG, SG, P, TL_FP64, 0, H, S, ws, base, kDefaultContractBlocks,
                       &ap));
  ContractArgs c = ap.contract;
  const int skip = c.d[1].block_begin;  // blocks of dim 0, not needed
  c.d[1].block_begin = 0;
  c.d[2].block_begin -= skip;
  c.d[0].block_begin = 0;
  const int blocks = ap.contract_blocks - skip;
  // dim 0 is never selected: every block index is >= d[1].block_begin = 0
  hipLaunchKernelGGL(transverse_contract_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, c);
  TL_CHECK_LAUNCH();
  ReduceArgs ra = ap.reduce;
  const int64_t off1 = ra.begin[1];
  ra.begin[0] = -1;  // never matched (all indices are >= begin[1] = 0)
  ra.begin[1] = 0;
  ra.begin[2] -= off1;
  const int64_t rtot = ap.reduce_total - off1;
  hipLaunchKernelGGL(transverse_reduce_kernel, dim3((unsigned)ceil_div(rtot, 256)), dim3(256), 0,
                     stream, ra, rtot);
  TL_CHECK_LAUNCH();
  const size_t m2 = (size_t)g.m0 * g.m0;
  double* coef = (double*)((char*)ws + base);
  CoefArgs ca{ra.C[1], ra.C[2], coef, coef + ((size_t)g.pot_terms + 2) * m2, g.m0,
              (int)g.pot_terms};
  hipLaunchKernelGGL(box_coef_kernel, dim3((unsigned)ceil_div((g.pot_terms + 2) * m2, 256)),
                     dim3(256), 0, stream, ca);
  TL_CHECK_LAUNCH();
  BoxArgs2 b;
  std::memset(&b, 0, sizeof(b));
  b.G = G + g.basis_off[0];
  b.AG = AG + g.basis_off[0];
  b.SG = SG + g.basis_off[0];
  b.P = P + g.pot_off[0];
  b.coef = ca.coef;
  b.smass = ca.smass;
  b.H = H;
  b.S = S;
  for (int mu = 0; mu < g.m0; ++mu) {
    b.center[mu] = s->fn_center[3 * mu];
    b.radius[mu] = std::sqrt(kSupportExp / s->fn_alpha[mu]) + g.h;
  }
  b.box_origin0 = g.box_origin0;
  b.a0 = g.a[0];
  b.x0 = g.x0[0];
  b.h = g.h;
  b.n = g.n[0];
  b.Nb = (int)g.basis_rows[0];
  b.m0 = g.m0;
  b.T = (int)g.pot_terms;
  b.ntiles = (int)ceil_div(b.Nb, kBM);
  const int pairs = b.ntiles * (b.ntiles + 1) / 2;
  hipLaunchKernelGGL(box_contract_kernel, dim3((unsigned)pairs), dim3(256), 0, stream, b);
  TL_CHECK_LAUNCH();
  return TL_OK;
}

}  // namespace tl
