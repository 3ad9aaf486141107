// Steps a4/a5: Galerkin entries as products of 1D inner products (proof of
// Lemma 3.1, eq. (nuc_potMatrTot); Sec. 3.4; Lemma 4.1 eqs. (BC-Core),
// (BC-mass), (BC-Laplace)).
//
// a4, per dimension l, one contraction over the grid nodes i:
//   C_l[(t, nu)][(mu, s)] = sum_i X[(t, nu)][i] * Y[(mu, s)][i]
//   X[(t, nu)][i] = p_t(x_i) g_nu(x_i)   (t < T, potential terms)
//                 = (A g_nu)(x_i)         (t = T,   stiffness)
//                 = (S g_nu)(x_i)         (t = T+1, mass)
//   Y[(mu, s)][i] = g_mu(x_i - s a_l)     (cyclic shift by s cells on a torus)
// i.e. G diag(p_t) G_s^T for all terms and shifts at once: an (T+2) m0 x m0 S
// by n GEMM whose operands are formed on the fly from G, P (never stored).
// Since A and S commute with cyclic shifts and are symmetric,
// <A g_(mu,s), g_nu> = sum_i g_mu(x_i - s a) (A g_nu)(x_i).
// Only shifts s = 0..L/2 are contracted: the replicated potential has the
// lattice period, so C_l[mu][nu][-s] = C_l[nu][mu][s].
//
// a5, FP64 in every precision mode, thread per entry of the block column:
//   V_k = sum_t prod_l C_l[t][mu][nu][k_l],
//   T_k = 1/2 (D_1 M_2 M_3 + M_1 D_2 M_3 + M_1 M_2 D_3),  S_k = M_1 M_2 M_3,
//   H_k = T_k - V_k.
#include <algorithm>
#include <cmath>

#include "common.h"

namespace tl {
namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kBM = 32;   // rows of a workgroup tile (2 MFMA row blocks)
constexpr int kBN = 32;   // columns of a workgroup tile (2 MFMA column blocks)
constexpr int kKT = 32;   // nodes per LDS stage
constexpr int kLDP = kKT + 1;

struct ContractArgs {
  const double* G;
  const double* AG;
  const double* SG;
  const double* P;
  double* out;     // [ksplit][M][N] partial sums
  int n, m0, T, S, cn, M, N, kchunk;
};

// One workgroup = 4 waves = a 32 x 32 tile of C over one chunk of nodes; each
// wave owns a 16 x 16 block and issues V_MFMA_F64_16X16X4_F64 from LDS.
__global__ __launch_bounds__(256) void contract_f64_kernel(ContractArgs a) {
  __shared__ double Xs[kBM][kLDP];
  __shared__ double Ys[kBN][kLDP];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int col0 = blockIdx.x * kBN;
  const int row0 = blockIdx.y * kBM;
  const int kbeg = blockIdx.z * a.kchunk;
  const int kend = min(a.n, kbeg + a.kchunk);
  const int wm = wave >> 1, wn = wave & 1;
  f64x4 acc = {0.0, 0.0, 0.0, 0.0};
  for (int k0 = kbeg; k0 < kend; k0 += kKT) {
    for (int e = tid; e < kBM * kKT; e += 256) {
      int r = e / kKT, kk = e - r * kKT;
      int row = row0 + r, i = k0 + kk;
      double v = 0.0;
      if (row < a.M && i < kend) {
        int t = row / a.m0, nu = row - t * a.m0;
        int64_t gi = (int64_t)nu * a.n + i;
        if (t < a.T)
          v = a.P[(int64_t)t * a.n + i] * a.G[gi];
        else if (t == a.T)
          v = a.AG[gi];
        else
          v = a.SG[gi];
      }
      Xs[r][kk] = v;
    }
    for (int e = tid; e < kBN * kKT; e += 256) {
      int c = e / kKT, kk = e - c * kKT;
      int col = col0 + c, i = k0 + kk;
      double v = 0.0;
      if (col < a.N && i < kend) {
        int mu = col / a.S, s = col - mu * a.S;
        int src = i - s * a.cn;
        if (src < 0) src += a.n;
        v = a.G[(int64_t)mu * a.n + src];
      }
      Ys[c][kk] = v;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < kKT; kk += 4) {
      double av = Xs[wm * 16 + (lane & 15)][kk + (lane >> 4)];
      double bv = Ys[wn * 16 + (lane & 15)][kk + (lane >> 4)];
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
    }
    __syncthreads();
  }
  // f64 16x16x4 result layout on gfx950: register r of lane l holds
  // D[l / 16 + 4 r][l % 16] (checked with a one-wave probe).
  const int col = col0 + wn * 16 + (lane & 15);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    int row = row0 + wm * 16 + (lane >> 4) + 4 * r;
    if (row < a.M && col < a.N) a.out[((int64_t)blockIdx.z * a.M + row) * a.N + col] = acc[r];
  }
}

struct CombineArgs {
  const double* C[3];
  int ks[3], S[3], L[3], periodic[3];
  int64_t MN[3];
  int N[3];
  int m0, T;
  double* H;
  double* Sm;
};

__device__ inline double lookup(const CombineArgs& a, int d, int t, int mu, int nu, int k) {
  int row, col;
  if (!a.periodic[d] || k < a.S[d]) {
    row = t * a.m0 + nu;
    col = mu * a.S[d] + k;
  } else {  // negative shift: C[mu][nu][-s] = C[nu][mu][s]
    row = t * a.m0 + mu;
    col = nu * a.S[d] + (a.L[d] - k);
  }
  const double* p = a.C[d] + (int64_t)row * a.N[d] + col;
  double v = 0.0;
  for (int s = 0; s < a.ks[d]; ++s) v += p[(int64_t)s * a.MN[d]];
  return v;
}

__global__ __launch_bounds__(256) void combine_periodic_kernel(CombineArgs a, int64_t total) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  int m2 = a.m0 * a.m0;
  int64_t kflat = idx / m2;
  int e = (int)(idx - kflat * m2);
  int mu = e / a.m0, nu = e - mu * a.m0;
  int k3 = (int)(kflat % a.L[2]);
  int k2 = (int)((kflat / a.L[2]) % a.L[1]);
  int k1 = (int)(kflat / ((int64_t)a.L[2] * a.L[1]));
  double V = 0.0;
  for (int t = 0; t < a.T; ++t) {
    double c1 = lookup(a, 0, t, mu, nu, k1);
    double c2 = lookup(a, 1, t, mu, nu, k2);
    double c3 = lookup(a, 2, t, mu, nu, k3);
    V += c1 * c2 * c3;
  }
  double D1 = lookup(a, 0, a.T, mu, nu, k1), M1 = lookup(a, 0, a.T + 1, mu, nu, k1);
  double D2 = lookup(a, 1, a.T, mu, nu, k2), M2 = lookup(a, 1, a.T + 1, mu, nu, k2);
  double D3 = lookup(a, 2, a.T, mu, nu, k3), M3 = lookup(a, 2, a.T + 1, mu, nu, k3);
  double Tk = 0.5 * (D1 * M2 * M3 + M1 * D2 * M3 + M1 * M2 * D3);
  a.H[idx] = Tk - V;
  a.Sm[idx] = M1 * M2 * M3;
}

// Optional HIP events recorded around the contraction launches of the next
// assembly calls of this thread (profiling hook for measured rooflines).
thread_local hipEvent_t g_ev_start = nullptr, g_ev_stop = nullptr;

struct Plan {
  int M[3], N[3], ks[3], kchunk[3];
  size_t part_off[3];  // byte offsets of the partial arrays in the workspace
  size_t bytes;
};

Plan make_plan(const Geometry& g) {
  Plan p;
  size_t off = 0;
  for (int d = 0; d < 3; ++d) {
    p.M[d] = (int)((g.pot_terms + 2) * g.m0);
    p.N[d] = g.m0 * g.shifts[d];
    int64_t tiles = ceil_div(p.M[d], kBM) * ceil_div(p.N[d], kBN);
    int64_t want = std::max<int64_t>(1, ceil_div(2048, tiles));
    int64_t maxsplit = std::max<int64_t>(1, g.n[d] / 128);
    int ks = (int)std::min(want, maxsplit);
    int kchunk = (int)(ceil_div(ceil_div(g.n[d], ks), kKT) * kKT);
    ks = (int)ceil_div(g.n[d], kchunk);
    p.ks[d] = ks;
    p.kchunk[d] = kchunk;
    p.part_off[d] = off;
    off += align_up(sizeof(double) * (size_t)ks * p.M[d] * p.N[d], 256);
  }
  p.bytes = off;
  return p;
}

}  // namespace

size_t assemble_workspace_bytes(const Geometry& g, tl_precision prec, int n_slices) {
  (void)prec;
  (void)n_slices;
  if (g.mode != TL_MODE_PERIODIC) return 0;
  return make_plan(g).bytes;
}

tl_status assemble_periodic(const Geometry& g, const double* G, const double* AG,
                            const double* SG, const double* P, tl_precision prec, int n_slices,
                            double* H, double* S, void* ws, size_t ws_bytes, hipStream_t stream) {
  (void)n_slices;
  if (prec != TL_FP64) {
    set_error("precision mode %d not available for the periodic assembly yet", (int)prec);
    return TL_EUNSUPPORTED;
  }
  Plan plan = make_plan(g);
  if (ws == nullptr || ws_bytes < plan.bytes) {
    set_error("assembly workspace: need %zu bytes, got %zu", plan.bytes, ws_bytes);
    return TL_EWORKSPACE;
  }
  char* wsb = (char*)ws;
  if (g_ev_start) TL_HIP(hipEventRecord(g_ev_start, stream));
  for (int d = 0; d < 3; ++d) {
    ContractArgs a;
    a.G = G + g.basis_off[d];
    a.AG = AG + g.basis_off[d];
    a.SG = SG + g.basis_off[d];
    a.P = P + g.pot_off[d];
    a.out = (double*)(wsb + plan.part_off[d]);
    a.n = g.n[d];
    a.m0 = g.m0;
    a.T = (int)g.pot_terms;
    a.S = g.shifts[d];
    a.cn = g.periodic[d] ? g.cell_nodes[d] : 0;
    a.M = plan.M[d];
    a.N = plan.N[d];
    a.kchunk = plan.kchunk[d];
    dim3 grid((unsigned)ceil_div(a.N, kBN), (unsigned)ceil_div(a.M, kBM), (unsigned)plan.ks[d]);
    hipLaunchKernelGGL(contract_f64_kernel, grid, dim3(256), 0, stream, a);
    TL_CHECK_LAUNCH();
  }
  if (g_ev_stop) TL_HIP(hipEventRecord(g_ev_stop, stream));
  CombineArgs c;
  for (int d = 0; d < 3; ++d) {
    c.C[d] = (const double*)(wsb + plan.part_off[d]);
    c.ks[d] = plan.ks[d];
    c.S[d] = g.shifts[d];
    c.L[d] = g.L[d];
    c.periodic[d] = g.periodic[d];
    c.MN[d] = (int64_t)plan.M[d] * plan.N[d];
    c.N[d] = plan.N[d];
  }
  c.m0 = g.m0;
  c.T = (int)g.pot_terms;
  c.H = H;
  c.Sm = S;
  int64_t total = g.block_elems;
  hipLaunchKernelGGL(combine_periodic_kernel, dim3((unsigned)ceil_div(total, 256)), dim3(256), 0,
                     stream, c, total);
  TL_CHECK_LAUNCH();
  return TL_OK;
}

}  // namespace tl

extern "C" tl_status tl_set_contraction_events(void* start_event, void* stop_event) {
  tl::clear_error();
  TL_REQUIRE((start_event == nullptr) == (stop_event == nullptr),
             "give both events or neither");
  tl::g_ev_start = (hipEvent_t)start_event;
  tl::g_ev_stop = (hipEvent_t)stop_event;
  return TL_OK;
}

extern "C" tl_status tl_assemble_workspace_bytes(const tl_system* sys, tl_precision prec,
                                                 int n_slices, size_t* bytes) {
  tl::clear_error();
  TL_REQUIRE(bytes != nullptr, "null output");
  tl::Geometry g;
  TL_TRY(tl::digest(sys, &g));
  *bytes = tl::assemble_workspace_bytes(g, prec, n_slices);
  return TL_OK;
}

extern "C" tl_status tl_assemble_core_hamiltonian_block(const tl_system* sys, const double* G_dev,
                                                        const double* AG_dev,
                                                        const double* SG_dev,
                                                        const double* P_dev, tl_precision prec,
                                                        int n_slices, double* H_dev,
                                                        double* S_dev, void* ws_dev,
                                                        size_t ws_bytes, void* stream) {
  tl::clear_error();
  tl::Geometry g;
  TL_TRY(tl::digest(sys, &g));
  TL_REQUIRE(G_dev && AG_dev && SG_dev && P_dev && H_dev && S_dev, "null array argument");
  TL_REQUIRE(prec >= TL_FP64 && prec <= TL_SPLIT_FP16, "unknown precision %d", (int)prec);
  if (g.mode == TL_MODE_PERIODIC)
    return tl::assemble_periodic(g, G_dev, AG_dev, SG_dev, P_dev, prec, n_slices, H_dev, S_dev,
                                 ws_dev, ws_bytes, (hipStream_t)stream);
  tl::set_error("box-mode assembly is not available yet");
  return TL_EUNSUPPORTED;
}
