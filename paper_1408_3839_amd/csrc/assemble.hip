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
constexpr int kKT = 64;   // nodes per LDS stage
constexpr int kLDP = kKT + 1;
constexpr int kPerThread = kBM * kKT / 256;  // staged values per thread and operand

struct DimArgs {
  const double* G;
  const double* AG;
  const double* SG;
  const double* P;
  double* part;    // [ks][M][N] partial sums over node chunks
  int n, S, cn, M, N, kchunk, ks, tiles_n, block_begin;
};

struct ContractArgs {
  DimArgs d[3];
  int m0, T;
};

// One launch for the three dimensions.  Workgroup = 4 waves = a 32 x 32 tile
// of C_l over one chunk of nodes; each wave owns a 16 x 16 block and issues
// V_MFMA_F64_16X16X4_F64 from LDS.  The next 64-node stage is loaded into
// registers while the current one is multiplied (double buffering).
__global__ __launch_bounds__(256) void contract_f64_kernel(ContractArgs a) {
  __shared__ double Xs[kBM][kLDP];
  __shared__ double Ys[kBN][kLDP];
  const int b = blockIdx.x;
  const int dd = b >= a.d[2].block_begin ? 2 : (b >= a.d[1].block_begin ? 1 : 0);
  const DimArgs& p = a.d[dd];
  const int local = b - p.block_begin;
  const int z = local % p.ks;
  const int rest = local / p.ks;
  const int col0 = (rest % p.tiles_n) * kBN;
  const int row0 = (rest / p.tiles_n) * kBM;
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int kbeg = z * p.kchunk;
  const int kend = min(p.n, kbeg + p.kchunk);
  const int wm = wave >> 1, wn = wave & 1;
  double xr[kPerThread], yr[kPerThread];
  // the rows and columns a thread stages are the same in every stage:
  // resolve (term, nu) and (mu, shift) once
  const double* xa[kPerThread];   // P row of the term (or null)
  const double* xb[kPerThread];   // G, AG or SG row of nu
  const double* yb[kPerThread];   // G row of mu
  int ysh[kPerThread];
  bool xok[kPerThread], yok[kPerThread];
#pragma unroll
  for (int j = 0; j < kPerThread; ++j) {
    const int r = (tid + 256 * j) / kKT;
    const int row = row0 + r, col = col0 + r;
    xok[j] = row < p.M;
    yok[j] = col < p.N;
    const int t = xok[j] ? row / a.m0 : 0, nu = xok[j] ? row - t * a.m0 : 0;
    xa[j] = t < a.T ? p.P + (int64_t)t * p.n : nullptr;
    xb[j] = (t < a.T ? p.G : (t == a.T ? p.AG : p.SG)) + (int64_t)nu * p.n;
    const int mu = yok[j] ? col / p.S : 0, sh = yok[j] ? col - mu * p.S : 0;
    yb[j] = p.G + (int64_t)mu * p.n;
    ysh[j] = sh * p.cn;
  }

  auto stage = [&](int k0) {
#pragma unroll
    for (int j = 0; j < kPerThread; ++j) {
      const int kk = (tid + 256 * j) & (kKT - 1);
      const int i = k0 + kk;
      const bool in_k = i < kend;
      double xv = 0.0, yv = 0.0;
      if (xok[j] && in_k) xv = xa[j] ? xa[j][i] * xb[j][i] : xb[j][i];
      if (yok[j] && in_k) {
        int src = i - ysh[j];
        if (src < 0) src += p.n;
        yv = yb[j][src];
      }
      xr[j] = xv;
      yr[j] = yv;
    }
  };
  auto commit = [&]() {
#pragma unroll
    for (int j = 0; j < kPerThread; ++j) {
      const int e = tid + 256 * j;
      Xs[e / kKT][e & (kKT - 1)] = xr[j];
      Ys[e / kKT][e & (kKT - 1)] = yr[j];
    }
  };

  f64x4 acc = {0.0, 0.0, 0.0, 0.0};
  stage(kbeg);
  commit();
  __syncthreads();
  for (int k0 = kbeg; k0 < kend; k0 += kKT) {
    const bool more = k0 + kKT < kend;
    if (more) stage(k0 + kKT);
#pragma unroll
    for (int kk = 0; kk < kKT; kk += 4) {
      double av = Xs[wm * 16 + (lane & 15)][kk + (lane >> 4)];
      double bv = Ys[wn * 16 + (lane & 15)][kk + (lane >> 4)];
      acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
    }
    __syncthreads();
    if (more) commit();
    __syncthreads();
  }
  // f64 16x16x4 result layout on gfx950: register r of lane l holds
  // D[l / 16 + 4 r][l % 16] (checked with a one-wave probe).
  const int col = col0 + wn * 16 + (lane & 15);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    int row = row0 + wm * 16 + (lane >> 4) + 4 * r;
    if (row < p.M && col < p.N) p.part[((int64_t)z * p.M + row) * p.N + col] = acc[r];
  }
}

struct ReduceArgs {
  const double* part[3];
  double* C[3];
  int64_t MN[3];
  int ks[3];
  int64_t begin[3];  // flat start of each dim
};

// Sums the node-chunk partial sums into the compact C_l (all dims at once).
__global__ __launch_bounds__(256) void reduce_partials_kernel(ReduceArgs a, int64_t total) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  int d = idx >= a.begin[2] ? 2 : (idx >= a.begin[1] ? 1 : 0);
  int64_t e = idx - a.begin[d];
  const double* p = a.part[d] + e;
  double v = 0.0;
  for (int s = 0; s < a.ks[d]; ++s) v += p[(int64_t)s * a.MN[d]];
  a.C[d][e] = v;
}

struct CombineArgs {
  const double* C[3];   // compact C_l [M][N]
  int S[3], L[3], periodic[3], N[3];
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
  return a.C[d][(int64_t)row * a.N[d] + col];
}

// One wave per entry of the block column: lane t forms the product of term t
// (t < T), lane T the kinetic combination, lane T+1 the mass product; a
// wave-wide sum then gives V (FP64 throughout).
__global__ __launch_bounds__(256) void combine_periodic_kernel(CombineArgs a, int64_t total) {
  const int64_t idx = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
  const int lane = threadIdx.x & 63;
  if (idx >= total) return;
  const int m2 = a.m0 * a.m0;
  const int64_t kflat = idx / m2;
  const int e = (int)(idx - kflat * m2);
  const int mu = e / a.m0, nu = e - mu * a.m0;
  const int k3 = (int)(kflat % a.L[2]);
  const int k2 = (int)((kflat / a.L[2]) % a.L[1]);
  const int k1 = (int)(kflat / ((int64_t)a.L[2] * a.L[1]));
  double V = 0.0, Tk = 0.0, Sk = 0.0;
  for (int t = lane; t < a.T + 2; t += 64) {
    if (t < a.T) {
      V += lookup(a, 0, t, mu, nu, k1) * lookup(a, 1, t, mu, nu, k2) * lookup(a, 2, t, mu, nu, k3);
    } else if (t == a.T) {
      double D1 = lookup(a, 0, a.T, mu, nu, k1), M1 = lookup(a, 0, a.T + 1, mu, nu, k1);
      double D2 = lookup(a, 1, a.T, mu, nu, k2), M2 = lookup(a, 1, a.T + 1, mu, nu, k2);
      double D3 = lookup(a, 2, a.T, mu, nu, k3), M3 = lookup(a, 2, a.T + 1, mu, nu, k3);
      Tk = 0.5 * (D1 * M2 * M3 + M1 * D2 * M3 + M1 * M2 * D3);
    } else {
      Sk = lookup(a, 0, a.T + 1, mu, nu, k1) * lookup(a, 1, a.T + 1, mu, nu, k2) *
           lookup(a, 2, a.T + 1, mu, nu, k3);
    }
  }
  for (int o = 32; o > 0; o >>= 1) V += __shfl_xor(V, o);
  const int tl = a.T % 64, sl = (a.T + 1) % 64;
  Tk = __shfl(Tk, tl);
  Sk = __shfl(Sk, sl);
  if (lane == 0) {
    a.H[idx] = Tk - V;
    a.Sm[idx] = Sk;
  }
}

// Optional HIP events recorded around the contraction launch of the next
// assembly calls of this thread (profiling hook for measured rooflines).
thread_local hipEvent_t g_ev_start = nullptr, g_ev_stop = nullptr;

struct Plan {
  int M[3], N[3], ks[3], kchunk[3], tiles_n[3], blocks[3];
  size_t part_off[3], c_off[3];  // byte offsets in the workspace
  size_t bytes;
  int total_blocks;
};

Plan make_plan(const Geometry& g) {
  Plan p;
  size_t off = 0;
  int nblk = 0;
  for (int d = 0; d < 3; ++d) {
    p.M[d] = (int)((g.pot_terms + 2) * g.m0);
    p.N[d] = g.m0 * g.shifts[d];
    int64_t tiles = ceil_div(p.M[d], kBM) * ceil_div(p.N[d], kBN);
    // enough workgroups to cover the chip, at least two stages per chunk
    int64_t want = std::max<int64_t>(1, ceil_div(512, tiles));
    int64_t maxsplit = std::max<int64_t>(1, g.n[d] / (2 * kKT));
    int ks = (int)std::min(want, maxsplit);
    int kchunk = (int)(ceil_div(ceil_div(g.n[d], ks), kKT) * kKT);
    ks = (int)ceil_div(g.n[d], kchunk);
    p.ks[d] = ks;
    p.kchunk[d] = kchunk;
    p.tiles_n[d] = (int)ceil_div(p.N[d], kBN);
    p.blocks[d] = (int)(tiles * ks);
    nblk += p.blocks[d];
    p.part_off[d] = off;
    off += align_up(sizeof(double) * (size_t)ks * p.M[d] * p.N[d], 256);
    p.c_off[d] = off;
    off += align_up(sizeof(double) * (size_t)p.M[d] * p.N[d], 256);
  }
  p.total_blocks = nblk;
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
  ContractArgs a;
  a.m0 = g.m0;
  a.T = (int)g.pot_terms;
  int begin = 0;
  for (int d = 0; d < 3; ++d) {
    DimArgs& p = a.d[d];
    p.G = G + g.basis_off[d];
    p.AG = AG + g.basis_off[d];
    p.SG = SG + g.basis_off[d];
    p.P = P + g.pot_off[d];
    p.part = (double*)(wsb + plan.part_off[d]);
    p.n = g.n[d];
    p.S = g.shifts[d];
    p.cn = g.periodic[d] ? g.cell_nodes[d] : 0;
    p.M = plan.M[d];
    p.N = plan.N[d];
    p.kchunk = plan.kchunk[d];
    p.ks = plan.ks[d];
    p.tiles_n = plan.tiles_n[d];
    p.block_begin = begin;
    begin += plan.blocks[d];
  }
  if (g_ev_start) TL_HIP(hipEventRecord(g_ev_start, stream));
  hipLaunchKernelGGL(contract_f64_kernel, dim3((unsigned)plan.total_blocks), dim3(256), 0, stream,
                     a);
  TL_CHECK_LAUNCH();
  if (g_ev_stop) TL_HIP(hipEventRecord(g_ev_stop, stream));
  ReduceArgs ra;
  int64_t tot = 0;
  for (int d = 0; d < 3; ++d) {
    ra.part[d] = (const double*)(wsb + plan.part_off[d]);
    ra.C[d] = (double*)(wsb + plan.c_off[d]);
    ra.MN[d] = (int64_t)plan.M[d] * plan.N[d];
    ra.ks[d] = plan.ks[d];
    ra.begin[d] = tot;
    tot += ra.MN[d];
  }
  hipLaunchKernelGGL(reduce_partials_kernel, dim3((unsigned)ceil_div(tot, 256)), dim3(256), 0,
                     stream, ra, tot);
  TL_CHECK_LAUNCH();
  CombineArgs c;
  for (int d = 0; d < 3; ++d) {
    c.C[d] = (const double*)(wsb + plan.c_off[d]);
    c.S[d] = g.shifts[d];
    c.L[d] = g.L[d];
    c.periodic[d] = g.periodic[d];
    c.N[d] = plan.N[d];
  }
  c.m0 = g.m0;
  c.T = (int)g.pot_terms;
  c.H = H;
  c.Sm = S;
  int64_t total = g.block_elems;
  hipLaunchKernelGGL(combine_periodic_kernel, dim3((unsigned)ceil_div(total, 4)), dim3(256), 0,
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
