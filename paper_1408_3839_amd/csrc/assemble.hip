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
#include <mutex>

#include "common.h"
#include "dev_assemble.h"
#include "host_plans.h"

namespace tl {
namespace {

using namespace dev;

__global__ __launch_bounds__(256) void contract_f64_kernel(ContractArgs a) {
  contract_f64_body(a, blockIdx.x);
}
template <int TILE>
__global__ __launch_bounds__(256) void contract_f64_src_kernel(ContractArgs a) {
  contract_f64_src_body<TILE, TILE>(a, blockIdx.x);
}
__global__ __launch_bounds__(256) void contract_f32_kernel(ContractArgs a) {
  contract_f32_body(a, blockIdx.x);
}
template <typename LowT, int S>
__global__ __launch_bounds__(256) void rowmax_kernel(RowMaxArgs a) {
  rowmax_body<LowT, S>(a, blockIdx.x);
}
template <typename LowT, int S, int SPT>
__global__ __launch_bounds__(kSplitThreads) void contract_split_kernel(SplitArgs a) {
  contract_split_src_body<LowT, S, SPT>(a, blockIdx.x);
}
__global__ __launch_bounds__(256) void reduce_partials_kernel(ReduceArgs a, int64_t total) {
  reduce_partials_body(a, total, blockIdx.x);
}
__global__ __launch_bounds__(256) void combine_periodic_kernel(CombineArgs a, int64_t total) {
  combine_periodic_body(a, total, blockIdx.x);
}

__global__ __launch_bounds__(256) void combine_pair_kernel(CombineArgs a) {
  combine_pair_body(a, blockIdx.x, blockIdx.y);
}

}  // namespace

void contraction_events(hipEvent_t* start, hipEvent_t* stop) {
  stage_events(TL_STAGE_CONTRACTION, start, stop);
}

namespace {

struct Plan {
  int M[3], N[3], ks[3], kchunk[3], tiles_n[3], blocks[3];
  size_t part_off[3], c_off[3];  // byte offsets in the workspace
  size_t bytes;
  int total_blocks;
};

// Tiling of the three contractions: tile x tile tiles (32 for FP64/FP32, 64
// for the split modes), node chunks split so that about `want` workgroups
// cover the chip (at least two 64-node stages each).
Plan make_plan(const Geometry& g, int want_blocks, int tile = kBM, int tile_n = 0) {
  if (tile_n <= 0) tile_n = tile;
  Plan p;
  size_t off = 0;
  int nblk = 0;
  for (int d = 0; d < 3; ++d) {
    p.M[d] = (int)((g.pot_terms + 2) * g.m0);
    p.N[d] = g.m0 * g.shifts[d];
    int64_t tiles = ceil_div(p.M[d], tile) * ceil_div(p.N[d], tile_n);
    int64_t want = std::max<int64_t>(1, ceil_div(want_blocks, tiles));
    int64_t maxsplit = std::max<int64_t>(1, g.n[d] / (2 * kKT));
    int ks = (int)std::min(want, maxsplit);
    int kchunk = (int)(ceil_div(ceil_div(g.n[d], ks), kKT) * kKT);
    ks = (int)ceil_div(g.n[d], kchunk);
    p.ks[d] = ks;
    p.kchunk[d] = kchunk;
    p.tiles_n[d] = (int)ceil_div(p.N[d], tile_n);
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

// Extra workspace of the split modes: the exponents of the row maxima of the
// P, G, AG and SG rows of every dimension.
struct SplitPlan {
  size_t ex_off[3][4];
  size_t gs_off[3];
  int ldg[3];
  size_t bytes;
};

SplitPlan make_split_plan(const Geometry& g, int s, size_t base) {
  SplitPlan sp;
  size_t off = base;
  for (int d = 0; d < 3; ++d)
    for (int k = 0; k < 4; ++k) {
      sp.ex_off[d][k] = off;
      off += align_up(sizeof(int) * (size_t)(k == 0 ? g.pot_terms : g.m0), 256);
    }
  for (int d = 0; d < 3; ++d) {  // G-row slices, two copies, 2-byte elements
    sp.ldg[d] = (int)align_up((size_t)g.n[d] + 64, 8);  // even: 4-byte aligned rows
    sp.gs_off[d] = off;
    off += align_up(2 * 2 * (size_t)s * g.m0 * sp.ldg[d], 256);
  }
  sp.bytes = off;
  return sp;
}


// Dynamic LDS budget of the source-row FP64 kernel: three workgroups per CU
// with 32 x 32 tiles, two with 64 x 64 tiles.
constexpr size_t kSrcLdsMax = 53 * 1024;
constexpr size_t kSrcLdsMax64 = 64 * 1024;

// Largest node sub-chunk (256, 128 or 64, at most the chunk unless 64) whose
// worst tile fits the budget, 0 if none does.  The X part of a tile depends
// only on its rows and the Y part only on its columns, so the worst tile is
// the worst row block plus the worst column block.
// Bank multiplicity of one 32-lane B-operand read of the source-row kernel:
// lanes (g, n), g = 0, 1 consecutive nodes, n = 16 consecutive shifts cn
// nodes apart, with ypad pad doubles after every 32 window nodes; 64 banks
// of 4 bytes, lanes at one address share it.
int window_conflicts(int cn, int ypad) {
  int worst = 1;
  for (int h = 15; h < 15 + 32; ++h)
    for (int k = 0; k < 64; k += 2) {
      int addr[32], cnt[64] = {0}, na = 0;
      for (int g = 0; g < 2; ++g)
        for (int n = 0; n < 16; ++n) {
          const int w = (h - n) * cn + k + g;
          const int a2 = 2 * (w + ypad * (w >> 5));
          bool dup = false;
          for (int q = 0; q < na; ++q) dup = dup || addr[q] == a2;
          if (dup) continue;
          addr[na++] = a2;
          ++cnt[a2 & 63];
          ++cnt[(a2 + 1) & 63];
        }
      for (int b = 0; b < 64; ++b) worst = std::max(worst, cnt[b]);
    }
  return worst;
}

int choose_ypad(int cn) {
  if (cn <= 0) return 1;
  return window_conflicts(cn, 2) < window_conflicts(cn, 1) ? 2 : 1;
}

int choose_kc(const Plan& plan, const Geometry& g, int d, int ypad, int tile, size_t* bytes) {
  const int M = plan.M[d], N = plan.N[d], S = g.shifts[d];
  const int cn = g.periodic[d] ? g.cell_nodes[d] : 0;
  const int T = (int)g.pot_terms;
  for (int kc : {256, 128, 64}) {
    if (kc > plan.kchunk[d] && kc > 64) continue;
    int xmax = 0, ymax = 0;
    dev::TileLayout L;
    for (int row0 = 0; row0 < M; row0 += tile) {
      dev::tile_layout(M, N, S, cn, g.m0, T, row0, 0, tile, tile, kc, ypad, &L);
      xmax = std::max(xmax, L.xtotal);
    }
    for (int col0 = 0; col0 < N; col0 += tile) {
      dev::tile_layout(M, N, S, cn, g.m0, T, 0, col0, tile, tile, kc, ypad, &L);
      ymax = std::max(ymax, L.total - L.xtotal);
    }
    const size_t b = sizeof(double) * (size_t)(xmax + ymax);
    if (b <= (tile == 64 ? kSrcLdsMax64 : kSrcLdsMax)) {
      *bytes = b;
      return kc;
    }
  }
  return 0;
}


// Source rows of the worst 64-row split tile: its P rows plus G, AG, SG rows.
int split_src_rows(const Geometry& g) {
  const int M = (int)((g.pot_terms + 2) * g.m0), T = (int)g.pot_terms, m0 = g.m0;
  int worst = 0;
  for (int row0 = 0; row0 < M; row0 += kSplitTile) {
    const int r1 = std::min(M, row0 + kSplitTile) - 1, t0 = row0 / m0, t1 = r1 / m0;
    const int nP = t0 < T ? std::min(t1, T - 1) - t0 + 1 : 0;
    const int n = nP + (t0 < T ? m0 : 0) + (t0 <= T && T <= t1 ? m0 : 0) +
                  (t0 <= T + 1 && T + 1 <= t1 ? m0 : 0);
    worst = std::max(worst, n);
  }
  return worst;
}

}  // namespace

size_t assemble_workspace_bytes(const Geometry& g, tl_precision prec, int n_slices,
                                int want_blocks) {
  if (!is_split(prec)) return make_plan(g, want_blocks).bytes;
  const Plan plan = make_plan(g, want_blocks, kSplitTile, kSplitTileN);
  const int s = n_slices > 0 ? n_slices : default_slices(prec);
  return make_split_plan(g, s, plan.bytes).bytes;
}

tl_status plan_assembly(const Geometry& g, const double* G, const double* AG, const double* SG,
                        const double* P, tl_precision prec, int n_slices, double* H, double* S,
                        void* ws, size_t ws_bytes, int want_blocks, AssemblyPlan* out,
                        int tile_hint) {
  Plan plan = is_split(prec) ? make_plan(g, want_blocks, kSplitTile, kSplitTileN)
                             : make_plan(g, want_blocks);
  const int nsl = is_split(prec) ? (n_slices > 0 ? n_slices : default_slices(prec)) : 0;
  if (is_split(prec) && (nsl < 2 || nsl > max_slices(prec))) {
    set_error("n_slices = %d outside [2, %d]", n_slices, max_slices(prec));
    return TL_EINVAL;
  }
  const SplitPlan sp = make_split_plan(g, std::max(nsl, 2), plan.bytes);
  const size_t need = is_split(prec) ? sp.bytes : plan.bytes;
  if (ws == nullptr || ws_bytes < need) {
    set_error("assembly workspace: need %zu bytes, got %zu", need, ws_bytes);
    return TL_EWORKSPACE;
  }
  char* wsb = (char*)ws;
  AssemblyPlan& ap = *out;
  std::memset(&ap, 0, sizeof(ap));
  ap.prec = prec;
  ap.n_slices = nsl;
  ap.contract_blocks = plan.total_blocks;
  // FP64 / FP32 contraction
  ContractArgs& a = ap.contract;
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
    p.kc = 0;
    p.ypad = 1;
    begin += plan.blocks[d];
  }
  // FP64: the source-row kernel when every dimension's tiles fit its budget,
  // with 64 x 64 tiles when asked for (same node chunks and partial sums;
  // 4x fewer, larger workgroups) and they fit, else 32 x 32
  ap.src_lds = 0;
  ap.src_tile = 0;
  if (prec == TL_FP64) {
    for (int tile : {64, 32}) {
      if (tile > tile_hint) continue;
      size_t need = 0;
      bool ok = true;
      for (int d = 0; d < 3 && ok; ++d) {
        size_t b = 0;
        a.d[d].ypad = choose_ypad(a.d[d].cn);
        const int kc = choose_kc(plan, g, d, a.d[d].ypad, tile, &b);
        ok = kc > 0;
        a.d[d].kc = kc;
        need = std::max(need, b);
      }
      if (!ok) continue;
      ap.src_lds = need;
      ap.src_tile = tile;
      if (tile != kBM) {  // the grid of the larger tiles
        int nb = 0;
        for (int d = 0; d < 3; ++d) {
          DimArgs& p = a.d[d];
          p.tiles_n = (int)ceil_div(p.N, tile);
          p.block_begin = nb;
          nb += (int)(ceil_div(p.M, tile) * p.tiles_n * p.ks);
        }
        ap.contract_blocks = nb;
      }
      break;
    }
    if (ap.src_tile == 0)
      for (int d = 0; d < 3; ++d) a.d[d].kc = 0;
  }
  // split modes: row maxima, then the split contraction from the FP64 rows
  // (64 x 64 tiles: the plan's tiles_n and block counts are for that edge)
  if (is_split(prec)) {
    RowMaxArgs& ra = ap.rowmax;
    int nb = 0;
    for (int d = 0; d < 3; ++d) {
      const double* srcs[4] = {P + g.pot_off[d], G + g.basis_off[d], AG + g.basis_off[d],
                               SG + g.basis_off[d]};
      for (int k = 0; k < 4; ++k) {
        ra.src[d][k] = srcs[k];
        ra.ex[d][k] = (int*)(wsb + sp.ex_off[d][k]);
        ra.rows[d][k] = k == 0 ? (int)g.pot_terms : g.m0;
        ra.begin[4 * d + k] = nb;
        nb += ra.rows[d][k];
      }
      ra.n[d] = g.n[d];
      ra.gs[d] = wsb + sp.gs_off[d];
      ra.ldg[d] = sp.ldg[d];
    }
    ra.m0 = g.m0;
    ra.begin[12] = nb;
    ap.rowmax_blocks = nb;
    SplitArgs& q = ap.split;
    q.m0 = g.m0;
    q.T = (int)g.pot_terms;
    int bb = 0;
    for (int d = 0; d < 3; ++d) {
      SplitDimArgs& r = q.d[d];
      r.G = G + g.basis_off[d];
      r.AG = AG + g.basis_off[d];
      r.SG = SG + g.basis_off[d];
      r.P = P + g.pot_off[d];
      r.eP = ra.ex[d][0];
      r.eG = ra.ex[d][1];
      r.eA = ra.ex[d][2];
      r.eS = ra.ex[d][3];
      r.gs = ra.gs[d];
      r.ldg = ra.ldg[d];
      r.part = a.d[d].part;
      r.n = g.n[d];
      r.S = g.shifts[d];
      r.cn = a.d[d].cn;
      r.M = plan.M[d];
      r.N = plan.N[d];
      r.kchunk = plan.kchunk[d];
      r.ks = plan.ks[d];
      r.tiles_n = plan.tiles_n[d];
      r.block_begin = bb;
      bb += plan.blocks[d];
    }
    ap.contract_blocks = bb;
    const int rows = split_src_rows(g);
    ap.split_spt = rows <= 64 ? 2 : 4;  // staging passes of 32 rows
    ap.split_lds = split_lds_bytes(nsl, 32 * ap.split_spt);
  }
  // partial sums -> compact C_l
  ReduceArgs& ra = ap.reduce;
  int64_t tot = 0;
  for (int d = 0; d < 3; ++d) {
    ra.part[d] = a.d[d].part;
    ra.C[d] = (double*)(wsb + plan.c_off[d]);
    ra.MN[d] = (int64_t)plan.M[d] * plan.N[d];
    ra.ks[d] = plan.ks[d];
    ra.begin[d] = tot;
    tot += ra.MN[d];
  }
  ap.reduce_total = tot;
  // FP64 combination
  CombineArgs& c = ap.combine;
  for (int d = 0; d < 3; ++d) {
    c.C[d] = ra.C[d];
    c.S[d] = g.shifts[d];
    c.L[d] = g.L[d];
    c.periodic[d] = g.periodic[d];
    c.N[d] = plan.N[d];
  }
  c.m0 = g.m0;
  c.T = (int)g.pot_terms;
  c.H = H;
  c.Sm = S;
  if (g.block_elems > INT32_MAX) {
    set_error("block column of %lld entries exceeds 2^31 - 1", (long long)g.block_elems);
    return TL_EUNSUPPORTED;
  }
  ap.combine_total = g.block_elems;
  return TL_OK;
}

namespace {

template <typename LowT, int SPT>
void launch_split_s(const AssemblyPlan& ap, hipStream_t stream, hipEvent_t e0, hipEvent_t e1) {
  const dim3 grid((unsigned)ap.contract_blocks), blk(kSplitThreads);
  const size_t lds = ap.split_lds;
  switch (ap.n_slices) {
    case 2: launch_with_events(contract_split_kernel<LowT, 2, SPT>, grid, blk, lds, stream, e0, e1, ap.split); break;
    case 3: launch_with_events(contract_split_kernel<LowT, 3, SPT>, grid, blk, lds, stream, e0, e1, ap.split); break;
    case 4: launch_with_events(contract_split_kernel<LowT, 4, SPT>, grid, blk, lds, stream, e0, e1, ap.split); break;
    case 5: launch_with_events(contract_split_kernel<LowT, 5, SPT>, grid, blk, lds, stream, e0, e1, ap.split); break;
    case 6: launch_with_events(contract_split_kernel<LowT, 6, SPT>, grid, blk, lds, stream, e0, e1, ap.split); break;
    default: launch_with_events(contract_split_kernel<LowT, 7, SPT>, grid, blk, lds, stream, e0, e1, ap.split); break;
  }
}

template <typename LowT>
void launch_rowmax_t(const AssemblyPlan& ap, hipStream_t stream) {
  const dim3 grid((unsigned)ap.rowmax_blocks), blk(256);
  switch (ap.n_slices) {
    case 2: hipLaunchKernelGGL((rowmax_kernel<LowT, 2>), grid, blk, 0, stream, ap.rowmax); break;
    case 3: hipLaunchKernelGGL((rowmax_kernel<LowT, 3>), grid, blk, 0, stream, ap.rowmax); break;
    case 4: hipLaunchKernelGGL((rowmax_kernel<LowT, 4>), grid, blk, 0, stream, ap.rowmax); break;
    case 5: hipLaunchKernelGGL((rowmax_kernel<LowT, 5>), grid, blk, 0, stream, ap.rowmax); break;
    case 6: hipLaunchKernelGGL((rowmax_kernel<LowT, 6>), grid, blk, 0, stream, ap.rowmax); break;
    default: hipLaunchKernelGGL((rowmax_kernel<LowT, 7>), grid, blk, 0, stream, ap.rowmax); break;
  }
}

void launch_rowmax(const AssemblyPlan& ap, hipStream_t stream) {
  if (ap.prec == TL_SPLIT_BF16)
    launch_rowmax_t<__bf16>(ap, stream);
  else
    launch_rowmax_t<_Float16>(ap, stream);
}

template <typename LowT>
void launch_split_contraction(const AssemblyPlan& ap, hipStream_t stream, hipEvent_t e0,
                              hipEvent_t e1) {
  if (ap.split_spt <= 2)
    launch_split_s<LowT, 2>(ap, stream, e0, e1);
  else
    launch_split_s<LowT, 4>(ap, stream, e0, e1);
}

}  // namespace

tl_status launch_assembly(const AssemblyPlan& ap, hipStream_t stream, bool combine) {
  if (is_split(ap.prec)) {
    launch_rowmax(ap, stream);
    TL_CHECK_LAUNCH();
  }
  // the profiling events (if set) are attached to the contraction launch
  hipEvent_t e0, e1;
  contraction_events(&e0, &e1);
  const dim3 cgrid((unsigned)ap.contract_blocks), cblk(256);
  if (ap.prec == TL_SPLIT_BF16)
    launch_split_contraction<__bf16>(ap, stream, e0, e1);
  else if (ap.prec == TL_SPLIT_FP16)
    launch_split_contraction<_Float16>(ap, stream, e0, e1);
  else if (ap.prec == TL_FP32)
    launch_with_events(contract_f32_kernel, cgrid, cblk, 0, stream, e0, e1, ap.contract);
  else if (ap.src_tile == 64)
    launch_with_events(contract_f64_src_kernel<64>, cgrid, cblk, ap.src_lds, stream, e0, e1,
                       ap.contract);
  else if (ap.src_tile == 32)
    launch_with_events(contract_f64_src_kernel<32>, cgrid, cblk, ap.src_lds, stream, e0, e1,
                       ap.contract);
  else
    launch_with_events(contract_f64_kernel, cgrid, cblk, 0, stream, e0, e1, ap.contract);
  TL_CHECK_LAUNCH();
  hipLaunchKernelGGL(reduce_partials_kernel, dim3((unsigned)ceil_div(ap.reduce_total, 256)),
                     dim3(256), 0, stream, ap.reduce, ap.reduce_total);
  TL_CHECK_LAUNCH();
  if (!combine) return TL_OK;
  const CombineArgs& c = ap.combine;
  if (combine_pair_fits(c.T, c.L)) {
    const int cells = c.L[0] * c.L[1] * c.L[2];
    hipLaunchKernelGGL(combine_pair_kernel,
                       dim3((unsigned)(c.m0 * c.m0), (unsigned)ceil_div(cells, 256)), dim3(256),
                       0, stream, c);
  } else {
    hipLaunchKernelGGL(combine_periodic_kernel, dim3((unsigned)ceil_div(ap.combine_total, 4)),
                       dim3(256), 0, stream, c, ap.combine_total);
  }
  TL_CHECK_LAUNCH();
  return TL_OK;
}

tl_status assemble_periodic(const Geometry& g, const double* G, const double* AG,
                            const double* SG, const double* P, tl_precision prec, int n_slices,
                            double* H, double* S, void* ws, size_t ws_bytes, hipStream_t stream) {
  AssemblyPlan ap;
  TL_TRY(plan_assembly(g, G, AG, SG, P, prec, n_slices, H, S, ws, ws_bytes,
                       kDefaultContractBlocks, &ap));
  return launch_assembly(ap, stream);
}

}  // namespace tl

extern "C" tl_status tl_set_contraction_events(void* start_event, void* stop_event) {
  return tl_set_stage_events(TL_STAGE_CONTRACTION, start_event, stop_event);
}

extern "C" tl_status tl_assemble_workspace_bytes(const tl_system* sys, tl_precision prec,
                                                 int n_slices, size_t* bytes) {
  tl::clear_error();
  TL_REQUIRE(bytes != nullptr, "null output");
  tl::Geometry g;
  TL_TRY(tl::digest(sys, &g));
  *bytes = g.mode == TL_MODE_BOX
               ? tl::box_workspace_bytes(g)
               : tl::assemble_workspace_bytes(g, prec, n_slices, tl::kDefaultContractBlocks);
  return TL_OK;
}

namespace tl {
namespace {

// Scratch memory of the allocation-free assembly entry point: a file-scope
// device array (each device the library runs on holds its own copy until the
// process ends).  Host code never uses the array's name as an address: the
// device address is taken once per device with hipGetSymbolAddress and kept.
constexpr size_t kStaticScratchBytes = size_t(32) << 20;
constexpr int kMaxDevices = 64;
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

tl_status static_scratch(void** out) {
  int dev = -1;
  TL_HIP(hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) {
    set_error("device index %d outside [0, %d)", dev, kMaxDevices);
    return TL_EUNSUPPORTED;
  }
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    TL_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (p == nullptr) {
      set_error("hipGetSymbolAddress returned a null scratch address");
      return TL_EHIP;
    }
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return TL_OK;
}

}  // namespace
}  // namespace tl

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
  return tl::assemble_box(g, sys, G_dev, AG_dev, SG_dev, P_dev, prec, n_slices, H_dev, S_dev, ws_dev,
                         ws_bytes, (hipStream_t)stream);
}

extern "C" tl_status tl_assemble_core_hamiltonian_block_noalloc(
    const tl_system* sys, const double* G_dev, const double* AG_dev, const double* SG_dev,
    const double* P_dev, tl_precision prec, int n_slices, double* H_dev, double* S_dev,
    void* stream) {
  tl::clear_error();
  tl::Geometry g;
  TL_TRY(tl::digest(sys, &g));
  TL_REQUIRE(G_dev && AG_dev && SG_dev && P_dev && H_dev && S_dev, "null array argument");
  TL_REQUIRE(prec >= TL_FP64 && prec <= TL_SPLIT_FP16, "unknown precision %d", (int)prec);
  const size_t need =
      g.mode == TL_MODE_BOX
          ? tl::box_workspace_bytes(g)
          : tl::assemble_workspace_bytes(g, prec, n_slices, tl::kDefaultContractBlocks);
  if (need > tl::kStaticScratchBytes) {
    tl::set_error("allocation-free assembly: this system needs %zu bytes of scratch, the "
                  "static scratch holds %zu; use tl_assemble_core_hamiltonian_block",
                  need, tl::kStaticScratchBytes);
    return TL_EUNSUPPORTED;
  }
  void* ws = nullptr;
  TL_TRY(tl::static_scratch(&ws));
  if (g.mode == TL_MODE_PERIODIC)
    return tl::assemble_periodic(g, G_dev, AG_dev, SG_dev, P_dev, prec, n_slices, H_dev, S_dev,
                                 ws, tl::kStaticScratchBytes, (hipStream_t)stream);
  return tl::assemble_box(g, sys, G_dev, AG_dev, SG_dev, P_dev, prec, n_slices, H_dev, S_dev, ws,
                         tl::kStaticScratchBytes, (hipStream_t)stream);
}
