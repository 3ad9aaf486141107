// Fourier-side separable combination (Theorem on the tensor-structured FFT
// diagonalisation, Sec. 2; Proposition on low-rank Fourier coefficients):
// the block column H_d = T_d - V_d is, term by term, a product over the
// three dimensions of 1D shift arrays, so its lattice DFT
//   Hbar_k = sum_d w^(k.d) H_d
// is the same sum of products of the three 1D DFTs:
//   Chat_l[t][mu][nu](k) = sum_{d=0}^{L_l-1} C_l[t][mu][nu][d] e^(-2 pi i k d / L_l),
//   Vbar_k = sum_t prod_l Chat_l[t](k_l),
//   Tbar_k = 1/2 (Dhat_1 Mhat_2 Mhat_3 + Mhat_1 Dhat_2 Mhat_3 + Mhat_1 Mhat_2 Dhat_3),
//   Sbar_k = Mhat_1 Mhat_2 Mhat_3,   Hbar_k = Tbar_k - Vbar_k.
// Exact (the DFT of a separable product factorises), with the negative
// shifts C_l[mu][nu][-s] = C_l[nu][mu][s] on each torus: the real-space
// combination and the 3-level block FFT are replaced by L_l-point DFTs of
// the compact factors and one complex combination per k-point.
#include <cmath>
#include <cstring>

#include "common.h"
#include "host_plans.h"

namespace tl {
namespace {

using namespace dev;

constexpr int kKdftMaxL = 2048;  // LDS twiddle table per workgroup

struct KdftArgs {
  CombineArgs c;   // compact C_l and their shapes
  double* out[3];  // Chat_l [T+2][m0][m0][L_l] complex, for the transformed dims
  int dim[3];      // transformed dims, in launch order
  int begin[4];    // workgroup prefix over them
};

// Workgroup per (dim, term t, mu): the m0 series (t, mu, nu) of that dim,
// every output k of each; x_d read once per series into LDS.
__global__ __launch_bounds__(256) void kdft_kernel(KdftArgs a) {
  __shared__ double cs[kKdftMaxL], sn[kKdftMaxL], xs[kKdftMaxL];
  const int b = blockIdx.x;
  int slot = 0;
  while (b >= a.begin[slot + 1]) ++slot;
  const int d = a.dim[slot];
  const int local = b - a.begin[slot];
  const int m0 = a.c.m0, L = a.c.L[d];
  const int t = local / m0, mu = local - t * m0;
  for (int m = threadIdx.x; m < L; m += blockDim.x) {
    double s, c;
    sincospi(2.0 * (double)m / (double)L, &s, &c);  // e^(2 pi i m / L)
    cs[m] = c;
    sn[m] = s;
  }
  double* out = a.out[slot];
  for (int nu = 0; nu < m0; ++nu) {
    __syncthreads();  // the previous series is consumed (and the table written)
    for (int j = threadIdx.x; j < L; j += blockDim.x) xs[j] = lookup(a.c, d, t, mu, nu, j);
    __syncthreads();
    for (int k = threadIdx.x; k < L; k += blockDim.x) {
      double re = 0.0, im = 0.0;
      int m = 0;  // k j mod L
      for (int j = 0; j < L; ++j) {
        re = fma(xs[j], cs[m], re);
        im = fma(-xs[j], sn[m], im);
        m += k;
        if (m >= L) m -= L;
      }
      const int64_t o = (((int64_t)t * m0 + mu) * m0 + nu) * L + k;
      out[2 * o] = re;
      out[2 * o + 1] = im;
    }
  }
}

struct KCombineArgs {
  CombineArgs c;
  const double* hat[3];  // Chat_l, or null: the dim is not transformed (L_l = 1)
  double* Hk;            // [L1 L2 L3][m0][m0] complex
  double* Sk;
};

struct Cplx {
  double re, im;
};

__device__ inline Cplx cmul(Cplx a, Cplx b) {
  return Cplx{fma(a.re, b.re, -a.im * b.im), fma(a.re, b.im, a.im * b.re)};
}

__device__ inline Cplx factor(const KCombineArgs& a, int d, int t, int mu, int nu, int k) {
  if (a.hat[d] == nullptr) return Cplx{lookup(a.c, d, t, mu, nu, 0), 0.0};
  const int64_t o = (((int64_t)t * a.c.m0 + mu) * a.c.m0 + nu) * a.c.L[d] + k;
  return Cplx{a.hat[d][2 * o], a.hat[d][2 * o + 1]};
}

// One wave per k-block entry: lane t forms term t's product (t < T), lane T
// the kinetic combination, lane T+1 the mass product; wave sums give Vbar.
__global__ __launch_bounds__(256) void combine_kspace_kernel(KCombineArgs a, int total) {
  const int idx = blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (idx >= total) return;
  const int m0 = a.c.m0, T = a.c.T, m2 = m0 * m0;
  const int kflat = idx / m2;
  const int e = idx - kflat * m2;
  const int mu = e / m0, nu = e - mu * m0;
  const int k12 = kflat / a.c.L[2];
  const int k3 = kflat - k12 * a.c.L[2];
  const int k1 = k12 / a.c.L[1];
  const int k2 = k12 - k1 * a.c.L[1];
  Cplx V{0.0, 0.0}, Tk{0.0, 0.0}, Sk{0.0, 0.0};
  for (int t = lane; t < T + 2; t += 64) {
    if (t < T) {
      const Cplx p = cmul(cmul(factor(a, 0, t, mu, nu, k1), factor(a, 1, t, mu, nu, k2)),
                          factor(a, 2, t, mu, nu, k3));
      V.re += p.re;
      V.im += p.im;
    } else if (t == T) {
      const Cplx D1 = factor(a, 0, T, mu, nu, k1), M1 = factor(a, 0, T + 1, mu, nu, k1);
      const Cplx D2 = factor(a, 1, T, mu, nu, k2), M2 = factor(a, 1, T + 1, mu, nu, k2);
      const Cplx D3 = factor(a, 2, T, mu, nu, k3), M3 = factor(a, 2, T + 1, mu, nu, k3);
      const Cplx x = cmul(cmul(D1, M2), M3), y = cmul(cmul(M1, D2), M3),
                 z = cmul(cmul(M1, M2), D3);
      Tk = Cplx{0.5 * (x.re + y.re + z.re), 0.5 * (x.im + y.im + z.im)};
    } else {
      Sk = cmul(cmul(factor(a, 0, T + 1, mu, nu, k1), factor(a, 1, T + 1, mu, nu, k2)),
                factor(a, 2, T + 1, mu, nu, k3));
    }
  }
  // the wave is whole here (the early return above is per wave)
  V.re = wave_sum_dpp(V.re);
  V.im = wave_sum_dpp(V.im);
  const double tre = readlane_d(Tk.re, T % 64), tim = readlane_d(Tk.im, T % 64);
  const double sre = readlane_d(Sk.re, (T + 1) % 64), sim = readlane_d(Sk.im, (T + 1) % 64);
  if (lane == 0) {
    a.Hk[2 * (int64_t)idx] = tre - V.re;
    a.Hk[2 * (int64_t)idx + 1] = tim - V.im;
    a.Sk[2 * (int64_t)idx] = sre;
    a.Sk[2 * (int64_t)idx + 1] = sim;
  }
}

// Fused form, a workgroup per (mu, nu) pair and chunk of 256 k-points: the
// 1D DFTs of the pair's factors (every term, every dim, from LDS twiddle
// tables) into LDS, then a thread per k-point.  Needs
// (T+2)(L1 + L2 + L3) <= kKPairMax complex values.
constexpr int kKPairMax = 2304;
constexpr int kKPairTw = 256;  // twiddles of the three dims (sum of L_l)

__global__ __launch_bounds__(256) void kspace_pair_kernel(KCombineArgs a) {
  __shared__ double F[2 * kKPairMax];
  __shared__ double X[kKPairMax];  // one dim's real factors [T+2][L_l]
  __shared__ double tw[2 * kKPairTw];
  const CombineArgs& c = a.c;
  const int pair = blockIdx.x, chunk = blockIdx.y;
  const int m0 = c.m0, T = c.T, TT = T + 2;
  const int mu = pair / m0, nu = pair - mu * m0;
  const int L[3] = {c.L[0], c.L[1], c.L[2]};
  const int off[3] = {0, TT * L[0], TT * (L[0] + L[1])};  // complex offsets of the dims
  const int toff[3] = {0, L[0], L[0] + L[1]};
  for (int e = threadIdx.x; e < L[0] + L[1] + L[2]; e += blockDim.x) {
    const int d = e < L[0] ? 0 : (e < L[0] + L[1] ? 1 : 2);
    const int m = e - toff[d];
    double sn, cs;
    sincospi(2.0 * (double)m / (double)L[d], &sn, &cs);  // e^(2 pi i m / L)
    tw[2 * e] = cs;
    tw[2 * e + 1] = sn;
  }
  __syncthreads();
  for (int d = 0; d < 3; ++d) {  // one dim at a time: its factors to LDS, then their DFTs
    const int n = TT * L[d];
    for (int f = threadIdx.x; f < n; f += blockDim.x) {
      const int t = f / L[d], j = f - t * L[d];
      X[f] = lookup(c, d, t, mu, nu, j);
    }
    __syncthreads();
    for (int f = threadIdx.x; f < n; f += blockDim.x) {
      const int t = f / L[d], k = f - t * L[d];
      const double* x = X + t * L[d];
      double re = 0.0, im = 0.0;
      int m = 0;  // k j mod L
      for (int j = 0; j < L[d]; ++j) {
        re = fma(x[j], tw[2 * (toff[d] + m)], re);
        im = fma(-x[j], tw[2 * (toff[d] + m) + 1], im);
        m += k;
        if (m >= L[d]) m -= L[d];
      }
      F[2 * (off[d] + f)] = re;
      F[2 * (off[d] + f) + 1] = im;
    }
    __syncthreads();  // X is reused by the next dim; F is complete after the last
  }
  const int cells = L[0] * L[1] * L[2];
  const int kf = chunk * blockDim.x + threadIdx.x;
  if (kf >= cells) return;
  const int k12 = kf / L[2], k3 = kf - k12 * L[2];
  const int k1 = k12 / L[1], k2 = k12 - k1 * L[1];
  auto fac = [&](int d, int t, int k) {
    const int i = off[d] + t * L[d] + k;
    return Cplx{F[2 * i], F[2 * i + 1]};
  };
  Cplx V{0.0, 0.0};
  for (int t = 0; t < T; ++t) {
    const Cplx p = cmul(cmul(fac(0, t, k1), fac(1, t, k2)), fac(2, t, k3));
    V.re += p.re;
    V.im += p.im;
  }
  const Cplx D1 = fac(0, T, k1), M1 = fac(0, T + 1, k1);
  const Cplx D2 = fac(1, T, k2), M2 = fac(1, T + 1, k2);
  const Cplx D3 = fac(2, T, k3), M3 = fac(2, T + 1, k3);
  const Cplx x = cmul(cmul(D1, M2), M3), y = cmul(cmul(M1, D2), M3), z = cmul(cmul(M1, M2), D3);
  const Cplx Sv = cmul(cmul(M1, M2), M3);
  const int64_t o = (int64_t)kf * m0 * m0 + pair;
  a.Hk[2 * o] = 0.5 * (x.re + y.re + z.re) - V.re;
  a.Hk[2 * o + 1] = 0.5 * (x.im + y.im + z.im) - V.im;
  a.Sk[2 * o] = Sv.re;
  a.Sk[2 * o + 1] = Sv.im;
}

bool kspace_pair_fits(const Geometry& g) {
  const int64_t sumL = (int64_t)g.L[0] + g.L[1] + g.L[2];
  return sumL <= kKPairTw && (g.pot_terms + 2) * sumL <= kKPairMax;
}

size_t hat_bytes(const Geometry& g, int d) {
  return align_up(sizeof(double) * 2 * ((size_t)g.pot_terms + 2) * g.m0 * g.m0 * g.L[d], 256);
}

bool transformed(const Geometry& g, int d) { return g.periodic[d] && g.L[d] > 1; }

}  // namespace

size_t kblocks_workspace_bytes(const Geometry& g, tl_precision prec, int n_slices) {
  size_t b = assemble_workspace_bytes(g, prec, n_slices, kDefaultContractBlocks);
  if (kspace_pair_fits(g)) return b;  // the fused kernel keeps the factors in LDS
  for (int d = 0; d < 3; ++d)
    if (transformed(g, d)) b += hat_bytes(g, d);
  return b;
}

tl_status assemble_kblocks(const Geometry& g, const double* G, const double* AG, const double* SG,
                           const double* P, tl_precision prec, int n_slices, double* Hk,
                           double* Sk, void* ws, size_t ws_bytes, hipStream_t stream) {
  if (g.mode != TL_MODE_PERIODIC) {
    set_error("k-space assembly needs a periodic system");
    return TL_EUNSUPPORTED;
  }
  for (int d = 0; d < 3; ++d)
    if (transformed(g, d) && g.L[d] > kKdftMaxL) {
      set_error("k-space assembly: L[%d] = %d exceeds %d (use the block FFT)", d, g.L[d],
                kKdftMaxL);
      return TL_EUNSUPPORTED;
    }
  if (is_split(prec) && n_slices != 0 && (n_slices < 2 || n_slices > max_slices(prec))) {
    set_error("n_slices = %d outside [2, %d]", n_slices, max_slices(prec));
    return TL_EINVAL;
  }
  const size_t need = kblocks_workspace_bytes(g, prec, n_slices);
  if (ws == nullptr || ws_bytes < need) {
    set_error("k-space assembly workspace: need %zu bytes, got %zu", need, ws_bytes);
    return TL_EWORKSPACE;
  }
  const size_t base = assemble_workspace_bytes(g, prec, n_slices, kDefaultContractBlocks);
  AssemblyPlan ap;
  TL_TRY(plan_assembly(g, G, AG, SG, P, prec, n_slices, nullptr, nullptr, ws, base,
                       kDefaultContractBlocks, &ap));
  TL_TRY(launch_assembly(ap, stream, false));
  if (kspace_pair_fits(g)) {
    KCombineArgs kc;
    std::memset(&kc, 0, sizeof(kc));
    kc.c = ap.combine;
    kc.Hk = Hk;
    kc.Sk = Sk;
    const int cells = g.L[0] * g.L[1] * g.L[2];
    hipLaunchKernelGGL(kspace_pair_kernel,
                       dim3((unsigned)(g.m0 * g.m0), (unsigned)ceil_div(cells, 256)), dim3(256), 0,
                       stream, kc);
    TL_CHECK_LAUNCH();
    return TL_OK;
  }
  KdftArgs ka;
  std::memset(&ka, 0, sizeof(ka));
  ka.c = ap.combine;
  KCombineArgs kc;
  std::memset(&kc, 0, sizeof(kc));
  kc.c = ap.combine;
  char* p = (char*)ws + base;
  int slots = 0, blocks = 0;
  const int per_dim = ((int)g.pot_terms + 2) * g.m0;
  for (int d = 0; d < 3; ++d) {
    if (!transformed(g, d)) continue;
    ka.dim[slots] = d;
    ka.out[slots] = (double*)p;
    kc.hat[d] = (const double*)p;
    ka.begin[slots] = blocks;
    blocks += per_dim;
    p += hat_bytes(g, d);
    ++slots;
  }
  for (int s = slots; s < 4; ++s) ka.begin[s] = blocks;
  if (blocks > 0) {
    hipLaunchKernelGGL(kdft_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, ka);
    TL_CHECK_LAUNCH();
  }
  kc.Hk = Hk;
  kc.Sk = Sk;
  const int total = (int)g.block_elems;  // below 2^31: checked by plan_assembly
  hipLaunchKernelGGL(combine_kspace_kernel, dim3((unsigned)ceil_div(total, 4)), dim3(256), 0,
                     stream, kc, total);
  TL_CHECK_LAUNCH();
  return TL_OK;
}

}  // namespace tl

extern "C" tl_status tl_assemble_kblocks_workspace_bytes(const tl_system* sys, tl_precision prec,
                                                         int n_slices, size_t* bytes) {
  tl::clear_error();
  TL_REQUIRE(bytes != nullptr, "null output");
  tl::Geometry g;
  TL_TRY(tl::digest(sys, &g));
  TL_REQUIRE(g.mode == TL_MODE_PERIODIC, "k-space assembly needs a periodic system");
  TL_REQUIRE(prec >= TL_FP64 && prec <= TL_SPLIT_FP16, "unknown precision %d", (int)prec);
  *bytes = tl::kblocks_workspace_bytes(g, prec, n_slices);
  return TL_OK;
}

extern "C" tl_status tl_assemble_kblocks(const tl_system* sys, const double* G_dev,
                                         const double* AG_dev, const double* SG_dev,
                                         const double* P_dev, tl_precision prec, int n_slices,
                                         double* Hk_dev, double* Sk_dev, void* ws_dev,
                                         size_t ws_bytes, void* stream) {
  tl::clear_error();
  tl::Geometry g;
  TL_TRY(tl::digest(sys, &g));
  TL_REQUIRE(G_dev && AG_dev && SG_dev && P_dev && Hk_dev && Sk_dev, "null array argument");
  TL_REQUIRE(prec >= TL_FP64 && prec <= TL_SPLIT_FP16, "unknown precision %d", (int)prec);
  return tl::assemble_kblocks(g, G_dev, AG_dev, SG_dev, P_dev, prec, n_slices, Hk_dev, Sk_dev,
                              ws_dev, ws_bytes, (hipStream_t)stream);
}
