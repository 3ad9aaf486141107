// Steps a2/a3: canonical 1D vectors of the lattice-summed Newton potential.
//
// The kernel 1/|x| is replaced by its exponential sum sum_q w_q e^{-t_q^2 |x|^2}
// and projected on the piecewise-constant cells of the grid (Sec. 3.2,
// eqs. (galten), (sinc_general)); each Gaussian factor is separable, so the
// projected tensor is a sum of rank-1 terms whose 1D factors are cell
// integrals b_q(x_i; A) = int_{cell i} exp(-t_q^2 (y - A)^2) dy.
//
// Torus dims (Sec. 4.1, eq. (EwaldSumP)): the lattice sum over images
// k = -K..K is evaluated on the central cell only and replicated with the
// lattice period.  Because site offsets and a are multiples of h, every image
// factor is an entry b~_q[j] = b_q(j h; 0) of one "master" vector on the
// accompanying grid (Sec. 3.2, master tensor and eq. (core_tens)).  Each
// entry enters one window node once (per site), so the entries are evaluated
// (ALU-bound, erfc) inside the workgroup that sums them, not stored.
// Open dims: one factor per nucleus, evaluated directly.  Torus and open
// transverse dims share one launch, and for periodic systems that launch can
// also carry the basis samples of Sec. 3.4 (independent work, one kernel
// start instead of two).
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <vector>

#include "common.h"
#include "dev_basis.h"
#include "dev_potential.h"
#include "host_plans.h"

namespace tl {
namespace {

using dev::BoxArgs;
using dev::DirectArgs;
using dev::FoldArgs;
using dev::QuadArgs;
constexpr int kNucChunk = dev::kNucChunk;

__global__ __launch_bounds__(256) void potential_kernel(DirectArgs a, FoldArgs f, QuadArgs quad,
                                                        int T, int fold_blocks,
                                                        double* __restrict__ P) {
  dev::potential_body(a, f, quad, T, fold_blocks, P, blockIdx.x);
}

// Basis functions the combined launch carries by value: the kernel
// arguments stay near 3 KB.
constexpr int kFusedFn = 8;

// Potential vectors and basis samples of one system in one launch: blocks
// [0, pot_blocks) run potential_body, the rest basis_body.  The two read only
// the system and write disjoint arrays; the branch is uniform per workgroup.
__global__ __launch_bounds__(256) void basis_potential_kernel(
    dev::BasisArgsN<kFusedFn> b, double* __restrict__ G, double* __restrict__ AG,
    double* __restrict__ SG, DirectArgs a, FoldArgs f, QuadArgs quad, int T, int fold_blocks,
    int pot_blocks, double* __restrict__ P) {
  const int64_t bx = blockIdx.x;
  if (bx < pot_blocks)
    dev::potential_body(a, f, quad, T, fold_blocks, P, bx);
  else
    dev::basis_body(b, G, AG, SG, bx - pot_blocks);
}

__global__ __launch_bounds__(256) void box_potential_kernel(BoxArgs p, QuadArgs quad,
                                                            double* __restrict__ P) {
  dev::box_potential_body(p, quad, P, blockIdx.x, blockIdx.y);
}

struct GroupInfo {
  std::vector<int> of_nucleus;       // group id per nucleus
  std::vector<double> y, z;          // coordinates of each group
};

GroupInfo make_groups(const tl_system* s) {
  GroupInfo gi;
  std::map<std::pair<double, double>, int> ids;
  for (int nu = 0; nu < s->n_nuc; ++nu) {
    auto key = std::make_pair(s->nuc_pos[3 * nu + 1], s->nuc_pos[3 * nu + 2]);
    auto it = ids.find(key);
    int id;
    if (it == ids.end()) {
      id = (int)gi.y.size();
      ids.emplace(key, id);
      gi.y.push_back(key.first);
      gi.z.push_back(key.second);
    } else {
      id = it->second;
    }
    gi.of_nucleus.push_back(id);
  }
  return gi;
}

}  // namespace

// The lattice sums form their cell integrals in place, so no workspace is
// needed; the query stays part of the interface.
size_t potential_workspace_bytes(const Geometry&, const tl_system*) { return 0; }

tl_status plan_potential(const Geometry& g, const tl_system* s, double* P, void* ws,
                         size_t ws_bytes, PotentialPlan* out) {
  size_t need = potential_workspace_bytes(g, s);
  if (ws_bytes < need || (need > 0 && ws == nullptr)) {
    set_error("potential workspace: need %zu bytes, got %zu", need, ws_bytes);
    return TL_EWORKSPACE;
  }
  PotentialPlan& pp = *out;
  std::memset(&pp, 0, sizeof(pp));
  pp.P = P;
  for (int q = 0; q < g.R; ++q) {
    pp.quad.t[q] = s->t_q[q];
    pp.quad.w[q] = s->w_q[q];
  }
  GroupInfo gi = make_groups(s);
  const int T = (int)g.pot_terms;
  // open transverse dims
  DirectArgs& da = pp.direct;
  da.R = g.R;
  da.h = g.h;
  da.T = T;
  int total_blocks = 0;
  for (int d = 1; d < 3; ++d) {
    if (g.periodic[d]) continue;
    int od = da.n_open++;
    da.open_dim[od] = d;
    da.n[od] = g.n[d];
    da.x0[od] = g.x0[d];
    da.out_off[od] = g.pot_off[d];
    da.blocks_per_term[od] = (int)ceil_div(g.n[d], 256);
    for (int gr = 0; gr < g.n_groups; ++gr) da.gpos[od][gr] = d == 1 ? gi.y[gr] : gi.z[gr];
    total_blocks += T * da.blocks_per_term[od];
  }
  pp.direct_blocks = total_blocks;
  // lattice sums of every torus dim
  FoldArgs& fa = pp.fold;
  fa.n_sites = s->n_nuc;
  fa.R = g.R;
  fa.h = g.h;
  for (int nu = 0; nu < s->n_nuc && nu < TL_MAX_SITES; ++nu) {
    fa.site_group[nu] = gi.of_nucleus[nu];
    fa.site_Z[nu] = s->nuc_Z[nu];
    for (int d = 0; d < 3; ++d)
      fa.site_off[d][nu] = (int)std::lround(s->nuc_pos[3 * nu + d] / g.h);
  }
  for (int gr = 0; gr < g.n_groups && gr < TL_MAX_SITES; ++gr) {
    fa.group_off[1][gr] = (int)std::lround(gi.y[gr] / g.h);
    fa.group_off[2][gr] = (int)std::lround(gi.z[gr] / g.h);
  }
  int slots = 0;
  int fold_blocks = 0;
  for (int d = 0; d < 3; ++d) {
    if (!g.periodic[d]) continue;
    fa.dims[slots] = d;
    fa.c[slots] = g.cell_nodes[d];
    fa.K[slots] = g.K[d];
    fa.n[slots] = g.n[d];
    fa.chunks[slots] = (int)ceil_div(g.cell_nodes[d], dev::kFoldNodes);
    fa.out_off[slots] = g.pot_off[d];
    fold_blocks += T * fa.chunks[slots];
    ++slots;
  }
  fa.n_slots = slots;
  pp.fold_slots = slots;
  pp.fold_blocks = fold_blocks;
  pp.box_dim0 = !g.periodic[0];
  return TL_OK;
}

tl_status lattice_sum_potential(const Geometry& g, const tl_system* s, double* P, void* ws,
                                size_t ws_bytes, hipStream_t stream) {
  PotentialPlan pp;
  TL_TRY(plan_potential(g, s, P, ws, ws_bytes, &pp));
  const int T = (int)g.pot_terms;
  const int blocks = pp.fold_blocks + pp.direct_blocks;
  if (blocks > 0) {
    hipEvent_t e0, e1;
    stage_events(TL_STAGE_LATTICE_SUM, &e0, &e1);
    launch_with_events(potential_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, e0, e1,
                       pp.direct, pp.fold, pp.quad, T, pp.fold_blocks, P);
    TL_CHECK_LAUNCH();
  }
  // open dim 0 (box mode): every nucleus summed directly, in chunks
  if (pp.box_dim0) {
    GroupInfo gi = make_groups(s);
    BoxArgs ba;
    std::memset(&ba, 0, sizeof(ba));
    ba.R = g.R;
    ba.n = g.n[0];
    ba.x0 = g.x0[0];
    ba.h = g.h;
    dim3 grid((unsigned)ceil_div(g.n[0], 256), (unsigned)T);
    for (int start = 0; start < s->n_nuc; start += kNucChunk) {
      int cnt = std::min(kNucChunk, s->n_nuc - start);
      ba.count = cnt;
      ba.accumulate = start > 0;
      for (int k = 0; k < cnt; ++k) {
        ba.pos[k] = s->nuc_pos[3 * (start + k)];
        ba.Z[k] = s->nuc_Z[start + k];
        ba.group[k] = gi.of_nucleus[start + k];
      }
      hipLaunchKernelGGL(box_potential_kernel, grid, dim3(256), 0, stream, ba, pp.quad, P);
      TL_CHECK_LAUNCH();
    }
  }
  return TL_OK;
}

// Both steps, one launch where the system allows it (periodic dim 0 and
// m0 <= kFusedFn); otherwise the two launches of the separate calls.  The
// results are those of build_basis followed by lattice_sum_potential, bit
// for bit: the same device code runs on the same arguments.
tl_status build_basis_and_potential(const Geometry& g, const tl_system* s, double* G, double* AG,
                                    double* SG, double* P, void* ws, size_t ws_bytes,
                                    hipStream_t stream) {
  PotentialPlan pp;
  TL_TRY(plan_potential(g, s, P, ws, ws_bytes, &pp));
  if (pp.box_dim0 || g.m0 > kFusedFn) {
    TL_TRY(build_basis(g, s, G, AG, SG, stream));
    return lattice_sum_potential(g, s, P, ws, ws_bytes, stream);
  }
  dev::BasisArgs full;
  make_basis_args(g, s, &full);
  dev::BasisArgsN<kFusedFn> b;
  std::memset(&b, 0, sizeof(b));
  for (int mu = 0; mu < g.m0; ++mu) b.fn[mu] = full.fn[mu];
  for (int d = 0; d < 3; ++d) {
    b.x0[d] = full.x0[d];
    b.period[d] = full.period[d];
    b.begin[d] = full.begin[d];
    b.n[d] = full.n[d];
    b.periodic[d] = full.periodic[d];
    b.rows[d] = full.rows[d];
  }
  b.total = full.total;
  b.h = full.h;
  b.box_origin0 = full.box_origin0;
  b.box_a = full.box_a;
  b.m0 = full.m0;
  const int T = (int)g.pot_terms;
  const int64_t pot_blocks = (int64_t)pp.fold_blocks + pp.direct_blocks;
  const int64_t blocks = pot_blocks + ceil_div(b.total, 256);
  TL_REQUIRE(blocks <= INT32_MAX, "grid too large");
  hipLaunchKernelGGL(basis_potential_kernel, dim3((unsigned)blocks), dim3(256), 0, stream, b, G,
                     AG, SG, pp.direct, pp.fold, pp.quad, T, pp.fold_blocks, (int)pot_blocks, P);
  TL_CHECK_LAUNCH();
  return TL_OK;
}

}  // namespace tl

extern "C" tl_status tl_potential_workspace_bytes(const tl_system* sys, size_t* bytes) {
  tl::clear_error();
  TL_REQUIRE(bytes != nullptr, "null output");
  tl::Geometry g;
  TL_TRY(tl::digest(sys, &g));
  *bytes = tl::potential_workspace_bytes(g, sys);
  return TL_OK;
}

extern "C" tl_status tl_lattice_sum_potential(const tl_system* sys, double* P_dev, void* ws_dev,
                                              size_t ws_bytes, void* stream) {
  tl::clear_error();
  tl::Geometry g;
  TL_TRY(tl::digest(sys, &g));
  TL_REQUIRE(P_dev != nullptr, "null output array");
  return tl::lattice_sum_potential(g, sys, P_dev, ws_dev, ws_bytes, (hipStream_t)stream);
}

extern "C" tl_status tl_build_basis_and_potential(const tl_system* sys, double* G_dev,
                                                  double* AG_dev, double* SG_dev, double* P_dev,
                                                  void* ws_dev, size_t ws_bytes, void* stream) {
  tl::clear_error();
  tl::Geometry g;
  TL_TRY(tl::digest(sys, &g));
  TL_REQUIRE(G_dev && AG_dev && SG_dev && P_dev, "null output array");
  return tl::build_basis_and_potential(g, sys, G_dev, AG_dev, SG_dev, P_dev, ws_dev, ws_bytes,
                                       (hipStream_t)stream);
}
