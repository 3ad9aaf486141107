// Step a8, assembly: full core Hamiltonian and mass matrix of an open-boundary
// chain (Sec. 3.3, eq. (nuc_pot) and proof of Lemma 3.1; Lemma 3.1 block
// sparsity; Sec. 3.4).  Every basis function f = (cell c, mu) has its own x
// factor; the y and z factors are those of the unit cell.  So
//   H[f][f'] = sum_t -C^x_t[f][f'] Cy_t[mu][nu] Cz_t[mu][nu]
//              + 1/2 D^x[f][f'] My Mz[mu][nu] + 1/2 M^x[f][f'] (Dy Mz + My Dz)[mu][nu]
//   S[f][f'] = M^x[f][f'] My Mz[mu][nu]
// with C^x_t = G diag(p_t) G^T over the x nodes (the paper's
// G diag(p_q) G^T contraction), D^x, M^x the FEM forms.  The transverse
// factors come from the periodic-path contraction kernels restricted to y
// and z (FP64).  Their products depend on (mu, nu) only, so the sum over t
// moves inside the x integral: one weighted vector Q_{mu nu} = sum_t
// coef_t[mu][nu] p_t per function pair, and the x contraction of the pair
// (mu, nu) is G_mu diag(Q_{mu nu}) G_nu^T plus the two FEM forms, a single
// contraction per entry instead of one per term.  It is banded: a tile of
// 32 x 32 cells only sums over the nodes where both tiles' Gaussians are
// above exp(-46) of their peak (Lemma 3.1's overlap constant L0, made exact
// to FP64 resolution), and tiles without overlap are zero.
#include <algorithm>
#include <cmath>

#include "common.h"
#include "host_plans.h"

namespace tl {
namespace {

using namespace dev;

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

// Q[mu][nu][i] = sum_t coef[t][mu][nu] p_t(x_i): the potential terms weighted
// by the transverse factors of the pair (mu, nu), summed in FP64 before the
// x contraction (the sum over q of Sec. 3.3 taken inside the x integral).
struct BoxQArgs {
  const double* P;     // [T][n]
  const double* coef;  // [T+2][m0][m0]
  double* Q;           // [m0 m0][n]
  int n, m0, T;
};

__global__ __launch_bounds__(256) void box_q_kernel(BoxQArgs a) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int p = blockIdx.y;  // mu m0 + nu
  if (i >= a.n) return;
  const int m2 = a.m0 * a.m0;
  double v = 0.0;
  for (int t = 0; t < a.T; ++t) v = fma(a.coef[t * m2 + p], a.P[(int64_t)t * a.n + i], v);
  a.Q[(int64_t)p * a.n + i] = v;
}

// One workgroup per (mu <= nu, row-cell tile, column-cell tile):
//   H[(c,mu)][(c',nu)] = sum_i X[c][i] G[(c',nu)][i],
//   X[c][i] = G[(c,mu)][i] Q[mu][nu][i] + coef[T][mu][nu] AG[(c,mu)][i]
//             + coef[T+1][mu][nu] SG[(c,mu)][i],
//   S[(c,mu)][(c',nu)] = My Mz[mu][nu] sum_i SG[(c,mu)][i] G[(c',nu)][i],
// over the nodes where both tiles' Gaussians are above exp(-46) of their
// peak.  Pairs mu < nu take every tile pair, mu = nu the upper triangle; each
// entry is written with its mirror, so H and S are exactly symmetric.
constexpr int kBoxTile = 32;  // cells per tile edge

struct BoxPairArgs {
  const double* G;     // [Nb][n] x factors, row f = c m0 + mu
  const double* AG;
  const double* SG;
  const double* Q;     // [m0 m0][n]
  const double* coef;  // [T+2][m0][m0]
  const double* smass; // [m0][m0]
  double* H;
  double* S;
  double center[TL_MAX_M0];  // x offset of function mu in its cell
  double radius[TL_MAX_M0];  // support radius sqrt(46 / alpha_mu) + h
  double box_origin0, a0, x0, h;
  int n, L0, m0, T, nt;      // nt: cell tiles per side
};

__host__ __device__ inline int box_pair_blocks(int m0, int nt) {
  return m0 * (nt * (nt + 1) / 2) + (m0 * (m0 - 1) / 2) * nt * nt;
}

struct BoxTile {
  int mu, nu, tr, tc, klo, khi;
};

__device__ inline BoxTile box_tile(const BoxPairArgs& a, int b) {
  BoxTile t;
  const int D = a.nt * (a.nt + 1) / 2;
  if (b < a.m0 * D) {  // mu = nu: upper triangle of tile pairs
    t.mu = t.nu = b / D;
    int r = b - t.mu * D;
    t.tr = 0;
    while (r >= a.nt - t.tr) {
      r -= a.nt - t.tr;
      ++t.tr;
    }
    t.tc = t.tr + r;
  } else {  // mu < nu: every tile pair
    const int nt2 = a.nt * a.nt;
    int r = b - a.m0 * D;
    int p = r / nt2;
    r -= p * nt2;
    t.tr = r / a.nt;
    t.tc = r - t.tr * a.nt;
    t.mu = 0;
    while (p >= a.m0 - 1 - t.mu) {
      p -= a.m0 - 1 - t.mu;
      ++t.mu;
    }
    t.nu = t.mu + 1 + p;
  }
  const int r0 = t.tr * kBoxTile, r1 = min(a.L0, r0 + kBoxTile) - 1;
  const int c0 = t.tc * kBoxTile, c1 = min(a.L0, c0 + kBoxTile) - 1;
  const double rlo = a.box_origin0 + r0 * a.a0 + a.center[t.mu] - a.radius[t.mu];
  const double rhi = a.box_origin0 + r1 * a.a0 + a.center[t.mu] + a.radius[t.mu];
  const double clo = a.box_origin0 + c0 * a.a0 + a.center[t.nu] - a.radius[t.nu];
  const double chi = a.box_origin0 + c1 * a.a0 + a.center[t.nu] + a.radius[t.nu];
  const double lo = (fmax(rlo, clo) - a.x0) / a.h, hi = (fmin(rhi, chi) - a.x0) / a.h;
  t.klo = lo <= 0.0 ? 0 : (int)fmin(ceil(lo), (double)a.n);
  t.khi = hi < 0.0 ? 0 : (int)fmin(floor(hi) + 1.0, (double)a.n);
  return t;
}

// The X entry of the H contraction (one expression, so that the split path's
// row maxima bound exactly the values it slices).
__device__ inline double box_x(double g, double ag, double sg, double q, double cD, double cM) {
  return fma(g, q, fma(cD, ag, cM * sg));
}

__device__ inline void box_store(const BoxPairArgs& a, const BoxTile& t, int c, int cp, double hv,
                                 double mv) {
  if (c >= a.L0 || cp >= a.L0) return;
  // a diagonal tile of a pair mu = nu keeps its upper half only
  if (t.mu == t.nu && t.tr == t.tc && c > cp) return;
  const int64_t Nb = (int64_t)a.L0 * a.m0;
  const int64_t f = (int64_t)c * a.m0 + t.mu, fp = (int64_t)cp * a.m0 + t.nu;
  const double sv = a.smass[t.mu * a.m0 + t.nu] * mv;
  a.H[f * Nb + fp] = hv;
  a.S[f * Nb + fp] = sv;
  if (f != fp) {
    a.H[fp * Nb + f] = hv;
    a.S[fp * Nb + f] = sv;
  }
}

// FP64: 4 waves, each a 16 x 16 quarter of the 32 x 32 cell tile, two
// accumulators (H and the mass form); KT nodes per LDS stage, the next
// stage's loads in flight during this stage's MFMAs.
template <int KT>
__global__ __launch_bounds__(256) void box_pair_f64_kernel(BoxPairArgs a) {
  constexpr int LDK = KT + 1;
  constexpr int RSTEP = 256 / KT;          // rows apart of one thread's staged rows
  constexpr int RPT = kBoxTile / RSTEP;    // staged rows per thread
  __shared__ double Xh[kBoxTile][LDK];
  __shared__ double Xm[kBoxTile][LDK];
  __shared__ double Yc[kBoxTile][LDK];
  const BoxTile t = box_tile(a, blockIdx.x);
  const int m2 = a.m0 * a.m0;
  const double cD = a.coef[a.T * m2 + t.mu * a.m0 + t.nu];
  const double cM = a.coef[(a.T + 1) * m2 + t.mu * a.m0 + t.nu];
  const double* Qp = a.Q + (int64_t)(t.mu * a.m0 + t.nu) * a.n;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  // staging: this thread's node kk of rows sr, sr + RSTEP, ..
  const int kk = tid % KT, sr = tid / KT;
  double vx[RPT], vm[RPT], vy[RPT];
  auto load = [&](int k0) {
    const int i = k0 + kk;
    const bool ok = i < t.khi;
    const double q = ok ? Qp[i] : 0.0;
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
      const int c = t.tr * kBoxTile + sr + RSTEP * u, cp = t.tc * kBoxTile + sr + RSTEP * u;
      const int64_t o = ((int64_t)c * a.m0 + t.mu) * a.n + i;
      const bool rok = ok && c < a.L0;
      vx[u] = rok ? box_x(a.G[o], a.AG[o], a.SG[o], q, cD, cM) : 0.0;
      vm[u] = rok ? a.SG[o] : 0.0;
      vy[u] = ok && cp < a.L0 ? a.G[((int64_t)cp * a.m0 + t.nu) * a.n + i] : 0.0;
    }
  };
  f64x4 ah = {0.0, 0.0, 0.0, 0.0}, am = {0.0, 0.0, 0.0, 0.0};
  if (t.klo < t.khi) load(t.klo);
  for (int k0 = t.klo; k0 < t.khi; k0 += KT) {
#pragma unroll
    for (int u = 0; u < RPT; ++u) {
      Xh[sr + RSTEP * u][kk] = vx[u];
      Xm[sr + RSTEP * u][kk] = vm[u];
      Yc[sr + RSTEP * u][kk] = vy[u];
    }
    __syncthreads();
    if (k0 + KT < t.khi) load(k0 + KT);  // in flight during the MFMAs
#pragma unroll
    for (int k = 0; k < KT; k += 4) {
      const int r = lane & 15, kq = k + (lane >> 4);
      const double bv = Yc[wn * 16 + r][kq];
      ah = __builtin_amdgcn_mfma_f64_16x16x4f64(Xh[wm * 16 + r][kq], bv, ah, 0, 0, 0);
      am = __builtin_amdgcn_mfma_f64_16x16x4f64(Xm[wm * 16 + r][kq], bv, am, 0, 0, 0);
    }
    __syncthreads();
  }
  // f64 16x16x4 result layout: register r of lane l holds D[l / 16 + 4 r][l % 16]
  const int cp = t.tc * kBoxTile + wn * 16 + (lane & 15);
#pragma unroll
  for (int r = 0; r < 4; ++r)
    box_store(a, t, t.tr * kBoxTile + wm * 16 + (lane >> 4) + 4 * r, cp, ah[r], am[r]);
}

constexpr int kBoxKT = 32;  // FP64: nodes per LDS stage

// Split modes: the same tiles with the three operands (X, SG rows, G
// columns) sliced in LDS per 32-node stage, relative to the power-of-two
// maxima of their rows over the tile's node range (a first pass), products of
// slice pairs qa + qb < s accumulated per level in FP32 MFMAs and added to
// FP64 every 64 nodes.
template <typename LowT, int S>
__global__ __launch_bounds__(256) void box_pair_split_kernel(BoxPairArgs a) {
  typedef typename Vec8<LowT>::type v8;
  constexpr int beta = LowTraits<LowT>::beta;
  constexpr int TT = kBoxTile, LD = kSplitLd, KS = kSplitK;
  __shared__ __attribute__((aligned(16))) LowT Xs[S][TT][LD];
  __shared__ __attribute__((aligned(16))) LowT Ms[S][TT][LD];
  __shared__ __attribute__((aligned(16))) LowT Ys[S][TT][LD];
  __shared__ int ex[3][TT];  // exponents of the X, SG and G-column rows
  const BoxTile t = box_tile(a, blockIdx.x);
  const int m2 = a.m0 * a.m0;
  const double cD = a.coef[a.T * m2 + t.mu * a.m0 + t.nu];
  const double cM = a.coef[(a.T + 1) * m2 + t.mu * a.m0 + t.nu];
  const double* Qp = a.Q + (int64_t)(t.mu * a.m0 + t.nu) * a.n;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  // row pointers of this thread's row (slicing: row tid / 8, nodes 4 (tid % 8) ..)
  const int xr = tid >> 3, xk = (tid & 7) * 4;
  auto rows = [&](int r, const double*& g, const double*& ag, const double*& sg,
                  const double*& y) {
    const int c = t.tr * TT + r, cp = t.tc * TT + r;
    const int64_t f = (int64_t)min(c, a.L0 - 1) * a.m0 + t.mu;
    const int64_t fp = (int64_t)min(cp, a.L0 - 1) * a.m0 + t.nu;
    g = c < a.L0 ? a.G + f * a.n : nullptr;
    ag = a.AG + f * a.n;
    sg = a.SG + f * a.n;
    y = cp < a.L0 ? a.G + fp * a.n : nullptr;
  };
  // pass 1: row maxima over [klo, khi), 32 lanes per row, 8 rows at a time
  {
    const int j = tid & 31, rq = tid >> 5;
#pragma unroll 1
    for (int rg = 0; rg < TT / 8; ++rg) {
      const int r = rg * 8 + rq;
      const double *g, *ag, *sg, *y;
      rows(r, g, ag, sg, y);
      double mh = 0.0, mm = 0.0, my = 0.0;
      if (g != nullptr)
        for (int i = t.klo + j; i < t.khi; i += 32) {
          const double s = sg[i];
          mh = fmax(mh, fabs(box_x(g[i], ag[i], s, Qp[i], cD, cM)));
          mm = fmax(mm, fabs(s));
        }
      if (y != nullptr)
        for (int i = t.klo + j; i < t.khi; i += 32) my = fmax(my, fabs(y[i]));
#pragma unroll
      for (int o = 16; o >= 1; o >>= 1) {
        mh = fmax(mh, __shfl_xor(mh, o, 32));
        mm = fmax(mm, __shfl_xor(mm, o, 32));
        my = fmax(my, __shfl_xor(my, o, 32));
      }
      if (j == 0) {
        int e = 0;
        if (mh > 0.0) frexp(mh, &e);  // 2^e > max|row|
        ex[0][r] = e;
        e = 0;
        if (mm > 0.0) frexp(mm, &e);
        ex[1][r] = e;
        e = 0;
        if (my > 0.0) frexp(my, &e);
        ex[2][r] = e;
      }
    }
  }
  __syncthreads();
  const double *g, *ag, *sg, *y;
  rows(xr, g, ag, sg, y);
  const int eh = ex[0][xr], em = ex[1][xr], ey = ex[2][xr];
  double vx[4], vm[4], vy[4];
  auto load = [&](int k0) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      const int i = k0 + xk + u;
      const bool ok = i < t.khi;
      const bool rok = ok && g != nullptr;
      vx[u] = rok ? box_x(g[i], ag[i], sg[i], Qp[i], cD, cM) : 0.0;
      vm[u] = rok ? sg[i] : 0.0;
      vy[u] = ok && y != nullptr ? y[i] : 0.0;
    }
  };
  auto slice_step = [&]() {
#pragma unroll
    for (int u = 0; u < 4; u += 2) {
      if constexpr (beta * S <= 52) {
        slice_pair<LowT, S>(vx[u], vx[u + 1], eh, &Xs[0][xr][xk + u], TT * LD);
        slice_pair<LowT, S>(vm[u], vm[u + 1], em, &Ms[0][xr][xk + u], TT * LD);
        slice_pair<LowT, S>(vy[u], vy[u + 1], ey, &Ys[0][xr][xk + u], TT * LD);
      } else {
        const double px[2] = {vx[u], vx[u + 1]}, pm[2] = {vm[u], vm[u + 1]},
                     py[2] = {vy[u], vy[u + 1]};
        slice_values<LowT, S, 2>(px, eh, &Xs[0][xr][xk + u], TT * LD);
        slice_values<LowT, S, 2>(pm, em, &Ms[0][xr][xk + u], TT * LD);
        slice_values<LowT, S, 2>(py, ey, &Ys[0][xr][xk + u], TT * LD);
      }
    }
  };
  f32x4 ch[S], cm[S];
#pragma unroll
  for (int l = 0; l < S; ++l) {
    ch[l] = f32x4{0.f, 0.f, 0.f, 0.f};
    cm[l] = f32x4{0.f, 0.f, 0.f, 0.f};
  }
  f64x4 ah = {0.0, 0.0, 0.0, 0.0}, am = {0.0, 0.0, 0.0, 0.0};
  auto flush = [&]() {
#pragma unroll
    for (int l = S - 1; l >= 0; --l) {
      const double sc = ldexp(1.0, -beta * (l + 2));
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        ah[r] = fma((double)ch[l][r], sc, ah[r]);
        am[r] = fma((double)cm[l][r], sc, am[r]);
      }
      ch[l] = f32x4{0.f, 0.f, 0.f, 0.f};
      cm[l] = f32x4{0.f, 0.f, 0.f, 0.f};
    }
  };
  if (t.klo < t.khi) {
    load(t.klo);
    slice_step();
  }
  __syncthreads();
  int step = 0;
  for (int k0 = t.klo; k0 < t.khi; k0 += KS, ++step) {
    const bool more = k0 + KS < t.khi;
    if (more) load(k0 + KS);  // in flight during the MFMAs
    {
      v8 bv[S], xv[S], mv[S];
      const int r = lane & 15, kq = 8 * (lane >> 4);
#pragma unroll
      for (int q = 0; q < S; ++q) {
        bv[q] = *(const v8*)&Ys[q][wn * 16 + r][kq];
        xv[q] = *(const v8*)&Xs[q][wm * 16 + r][kq];
        mv[q] = *(const v8*)&Ms[q][wm * 16 + r][kq];
      }
#pragma unroll
      for (int qa = 0; qa < S; ++qa)
#pragma unroll
        for (int qb = 0; qa + qb < S; ++qb) {
          ch[qa + qb] = Vec8<LowT>::mfma(xv[qa], bv[qb], ch[qa + qb]);
          cm[qa + qb] = Vec8<LowT>::mfma(mv[qa], bv[qb], cm[qa + qb]);
        }
    }
    if ((step & 1) || !more) flush();
    __syncthreads();  // every wave is done with this stage's slices
    if (more) {
      slice_step();
      __syncthreads();
    }
  }
  // f32 16x16x32 result layout: register r of lane l holds D[4 (l / 16) + r][l % 16]
  const int col = wn * 16 + (lane & 15);
  const int ecol = ex[2][col];
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int row = wm * 16 + 4 * (lane >> 4) + r;
    box_store(a, t, t.tr * TT + row, t.tc * TT + col, ldexp(ah[r], ex[0][row] + ecol),
              ldexp(am[r], ex[1][row] + ecol));
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
  return base + align_up(sizeof(double) * ((size_t)g.pot_terms + 3) * m2, 256) +
         align_up(sizeof(double) * m2 * (size_t)g.n[0], 256);
}

namespace {

template <typename LowT>
tl_status launch_box_split(int n_slices, int blocks, const BoxPairArgs& b, hipStream_t stream,
                           hipEvent_t e0, hipEvent_t e1) {
  switch (n_slices) {
#define TL_BOX_SPLIT(S)                                                                   \
  case S:                                                                                 \
    launch_with_events(box_pair_split_kernel<LowT, S>, dim3((unsigned)blocks), dim3(256), \
                       0, stream, e0, e1, b);                                             \
    break;
    TL_BOX_SPLIT(2)
    TL_BOX_SPLIT(3)
    TL_BOX_SPLIT(4)
    TL_BOX_SPLIT(5)
    TL_BOX_SPLIT(6)
    TL_BOX_SPLIT(7)
#undef TL_BOX_SPLIT
    default:
      set_error("n_slices = %d unsupported", n_slices);
      return TL_EUNSUPPORTED;
  }
  TL_CHECK_LAUNCH();
  return TL_OK;
}

}  // namespace

tl_status assemble_box(const Geometry& g, const tl_system* s, const double* G, const double* AG,
                       const double* SG, const double* P, tl_precision prec, int n_slices,
                       double* H, double* S, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (prec != TL_FP64 && !is_split(prec)) {
    set_error("box-mode assembly runs in FP64 or a split mode");
    return TL_EUNSUPPORTED;
  }
  const int nsl = is_split(prec) ? (n_slices > 0 ? n_slices : default_slices(prec)) : 0;
  if (is_split(prec) && (nsl < 2 || nsl > max_slices(prec))) {
    set_error("n_slices = %d outside [2, %d]", n_slices, max_slices(prec));
    return TL_EINVAL;
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
  double* Q = (double*)((char*)ws + base +
                        align_up(sizeof(double) * ((size_t)g.pot_terms + 3) * m2, 256));
  CoefArgs ca{ra.C[1], ra.C[2], coef, coef + ((size_t)g.pot_terms + 2) * m2, g.m0,
              (int)g.pot_terms};
  hipLaunchKernelGGL(box_coef_kernel, dim3((unsigned)ceil_div((g.pot_terms + 2) * m2, 256)),
                     dim3(256), 0, stream, ca);
  TL_CHECK_LAUNCH();
  BoxQArgs qa{P + g.pot_off[0], coef, Q, g.n[0], g.m0, (int)g.pot_terms};
  hipLaunchKernelGGL(box_q_kernel, dim3((unsigned)ceil_div(g.n[0], 256), (unsigned)m2),
                     dim3(256), 0, stream, qa);
  TL_CHECK_LAUNCH();
  BoxPairArgs b;
  std::memset(&b, 0, sizeof(b));
  b.G = G + g.basis_off[0];
  b.AG = AG + g.basis_off[0];
  b.SG = SG + g.basis_off[0];
  b.Q = Q;
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
  b.L0 = g.L[0];
  b.m0 = g.m0;
  b.T = (int)g.pot_terms;
  b.nt = (int)ceil_div(g.L[0], kBoxTile);
  const int pblocks = box_pair_blocks(b.m0, b.nt);
  hipEvent_t e0, e1;
  stage_events(TL_STAGE_CONTRACTION, &e0, &e1);
  if (prec == TL_FP64) {
    launch_with_events(box_pair_f64_kernel<kBoxKT>, dim3((unsigned)pblocks), dim3(256), 0, stream,
                       e0, e1, b);
    TL_CHECK_LAUNCH();
    return TL_OK;
  }
  if (prec == TL_SPLIT_FP16) return launch_box_split<_Float16>(nsl, pblocks, b, stream, e0, e1);
  return launch_box_split<__bf16>(nsl, pblocks, b, stream, e0, e1);
}

}  // namespace tl
