// Step a9: a ragged batch of periodic lattice systems through the whole path
// with one launch per stage.  The host writes, once, a descriptor holding
// every instance's launch arguments (the same structs the single-system
// entry points launch with) and the block prefix of every stage; the caller
// uploads it.  Each stage kernel finds its instance by a binary search of
// its block index in that prefix and runs the same device code as the
// single-system kernel on its share.  Nothing is allocated and no host copy
// is made during a run, so a run can be captured in a HIP graph.
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.h"
#include "host_plans.h"

namespace tl {
namespace {

enum Stage {
  kBasis = 0,
  kPotential,
  kRowMax,
  kContract,
  kReduce,
  kCombine,
  kFftTables,
  kDft,      // block FFT of the instances with 7-smooth chain lengths
  kDftBlue,  // block FFT of the others (Bluestein)
  kHeigh,   // k-block eigenvalues of the instances with m0 > 8
  kHeigh8,  // those of the instances with m0 <= 8, one wave per k-block
  kStages
};

struct InstanceJob {
  dev::BasisArgs basis;
  double* G;
  double* AG;
  double* SG;
  PotentialPlan pot;
  int T;  // potential terms
  AssemblyPlan asmb;
  dev::FftArgs fft;
  const double* Hb;
  const double* Sb;
  double* evals;
  int* info;
  int m0;
};

struct BatchDesc {
  int count;
  int64_t prefix[kStages][TL_MAX_BATCH + 1];
  InstanceJob job[TL_MAX_BATCH];
};

__device__ inline int find_job(const int64_t* prefix, int count, int64_t b) {
  int lo = 0, hi = count - 1;
  while (lo < hi) {
    int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= b)
      lo = mid;
    else
      hi = mid - 1;
  }
  return lo;
}

#define TL_BATCH_LOCATE(stage)                                   \
  const int64_t gb_ = blockIdx.x;                                \
  const int ji_ = find_job(d->prefix[stage], d->count, gb_);     \
  const InstanceJob& J = d->job[ji_];                            \
  const int64_t lb = gb_ - d->prefix[stage][ji_];

__global__ __launch_bounds__(256) void batch_basis_kernel(const BatchDesc* __restrict__ d) {
  TL_BATCH_LOCATE(kBasis)
  dev::basis_body(J.basis, J.G, J.AG, J.SG, lb);
}

__global__ __launch_bounds__(256) void batch_potential_kernel(const BatchDesc* __restrict__ d) {
  TL_BATCH_LOCATE(kPotential)
  dev::potential_body(J.pot.direct, J.pot.fold, J.pot.quad, J.T, J.pot.fold_blocks, J.pot.P, lb);
}

template <typename LowT, int S>
__global__ __launch_bounds__(256) void batch_rowmax_kernel(const BatchDesc* __restrict__ d) {
  TL_BATCH_LOCATE(kRowMax)
  dev::rowmax_body<LowT, S>(J.asmb.rowmax, (int)lb);
}

__global__ __launch_bounds__(256) void batch_contract_f64_kernel(const BatchDesc* __restrict__ d) {
  TL_BATCH_LOCATE(kContract)
  dev::contract_f64_body(J.asmb.contract, (int)lb);
}

__global__ __launch_bounds__(256) void batch_contract_f64_src_kernel(
    const BatchDesc* __restrict__ d) {
  TL_BATCH_LOCATE(kContract)
  if (J.asmb.src_tile == 64)  // uniform per workgroup
    dev::contract_f64_src_body<64, 64>(J.asmb.contract, (int)lb);
  else
    dev::contract_f64_src_body<32, 32>(J.asmb.contract, (int)lb);
}

__global__ __launch_bounds__(256) void batch_contract_f32_kernel(const BatchDesc* __restrict__ d) {
  TL_BATCH_LOCATE(kContract)
  dev::contract_f32_body(J.asmb.contract, (int)lb);
}

template <typename LowT, int S, int SPT>
__global__ __launch_bounds__(dev::kSplitThreads) void batch_contract_split_kernel(
    const BatchDesc* __restrict__ d) {
  TL_BATCH_LOCATE(kContract)
  dev::contract_split_src_body<LowT, S, SPT>(J.asmb.split, (int)lb);
}

__global__ __launch_bounds__(256) void batch_reduce_kernel(const BatchDesc* __restrict__ d) {
  TL_BATCH_LOCATE(kReduce)
  dev::reduce_partials_body(J.asmb.reduce, J.asmb.reduce_total, lb);
}

__global__ __launch_bounds__(256) void batch_combine_kernel(const BatchDesc* __restrict__ d) {
  TL_BATCH_LOCATE(kCombine)
  const dev::CombineArgs& c = J.asmb.combine;
  if (dev::combine_pair_fits(c.T, c.L)) {  // the single-system launch's choice
    const int chunks = (c.L[0] * c.L[1] * c.L[2] + 255) / 256;
    dev::combine_pair_body(c, (int)(lb / chunks), (int)(lb % chunks));
  } else {
    dev::combine_periodic_body(c, J.asmb.combine_total, lb);
  }
}

__global__ __launch_bounds__(dev::kFftThreads) void batch_fft_tables_kernel(
    const BatchDesc* __restrict__ d) {
  extern __shared__ __align__(16) double smem[];
  TL_BATCH_LOCATE(kFftTables)
  (void)lb;
  dev::fft_blue_tables_body(J.fft, smem);
}

// The Stockham and the Bluestein transforms run as two launches: one kernel
// holding both bodies takes the union of their registers (over 200 VGPRs,
// one 512-thread workgroup per CU), each alone about 115 (two per CU).
__global__ __launch_bounds__(dev::kFftThreads) void batch_fft_kernel(
    const BatchDesc* __restrict__ d) {
  extern __shared__ __align__(16) double smem[];
  TL_BATCH_LOCATE(kDft)
  dev::fft_block_body<false>(J.fft, lb, smem);
}

__global__ __launch_bounds__(dev::kFftThreads) void batch_fft_blue_kernel(
    const BatchDesc* __restrict__ d) {
  extern __shared__ __align__(16) double smem[];
  TL_BATCH_LOCATE(kDftBlue)
  dev::fft_block_body<true>(J.fft, lb, smem);
}

template <int MAXM>
__global__ __launch_bounds__(MAXM * MAXM < 64 ? 64 : MAXM * MAXM) void batch_heigh_kernel(
    const BatchDesc* __restrict__ d) {
  TL_BATCH_LOCATE(kHeigh)
  dev::heigh_body<MAXM>(J.Hb, J.Sb, J.m0, J.evals, nullptr, J.info, lb);
}

// Eigenvalues of the instances with m0 <= 8: one one-wave workgroup per
// k-block that reduces it once and bisects all its eigenvalues (for a batch
// this beats the single-system launch's wave per eigenvalue, which repeats
// the reduction m0 times), without the idle waves of a wider workgroup.
__global__ __launch_bounds__(64) void batch_heigh8_kernel(const BatchDesc* __restrict__ d) {
  TL_BATCH_LOCATE(kHeigh8)
  dev::heigh_wave8_body(J.Hb, J.Sb, J.m0, J.evals, nullptr, J.info, lb);
}

// Eigenvalues of the instances with 8 < m0 <= 16: the 256-thread
// tridiagonal route of the single-system launches.
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 2))) void
batch_heigh16_kernel(const BatchDesc* __restrict__ d) {
  TL_BATCH_LOCATE(kHeigh)
  dev::heigh_evals16_body(J.Hb, J.Sb, J.m0, J.evals, J.info, lb);
}

struct InstanceSizes {
  Geometry g;
  size_t pot_ws, asm_ws, fft_ws;
};

tl_status instance_sizes(const tl_system* s, tl_precision prec, int n_slices, int want,
                         InstanceSizes* out) {
  TL_TRY(digest(s, &out->g));
  const Geometry& g = out->g;
  if (g.mode != TL_MODE_PERIODIC) {
    set_error("the batched path takes periodic-mode systems");
    return TL_EUNSUPPORTED;
  }
  int axes = (g.L[0] > 1) + (g.L[1] > 1) + (g.L[2] > 1);
  if (axes > 1 || (axes == 1 && g.L[0] == 1)) {
    set_error("the batched path takes (L,1,1) lattices");
    return TL_EUNSUPPORTED;
  }
  if (g.L[0] > 4096) {
    set_error("the batched path takes L <= 4096");
    return TL_EUNSUPPORTED;
  }
  if (!g.periodic[0] && g.L[0] > 1) {
    set_error("batched lattice axis must be periodic");
    return TL_EUNSUPPORTED;
  }
  if (!g.periodic[0]) {
    set_error("the batched path needs a periodic x axis");
    return TL_EUNSUPPORTED;
  }
  {
    const int Ls[3] = {g.L[0], 1, 1};
    dev::FftArgs fa;
    if (!plan_fft(nullptr, nullptr, Ls, g.m0, 2, &fa)) {
      set_error("the batched path takes L <= 2048, or 7-smooth L <= 4096 (L = %d)", g.L[0]);
      return TL_EUNSUPPORTED;
    }
    out->fft_ws = fft_blue_table_bytes(fa);
  }
  out->pot_ws = align_up(potential_workspace_bytes(g, s), 256);
  out->asm_ws = align_up(assemble_workspace_bytes(g, prec, n_slices, want), 256);
  return TL_OK;
}

}  // namespace

}  // namespace tl

using namespace tl;

extern "C" tl_status tl_batch_plan_create(const tl_system* systems, int count, tl_precision prec,
                                          int n_slices, int want_blocks, tl_batch_plan* out) {
  clear_error();
  TL_REQUIRE(systems && out, "null argument");
  TL_REQUIRE(count >= 1 && count <= TL_MAX_BATCH, "count = %d outside [1, %d]", count,
             TL_MAX_BATCH);
  TL_REQUIRE(prec >= TL_FP64 && prec <= TL_SPLIT_FP16, "unknown precision %d", (int)prec);
  if (want_blocks <= 0) want_blocks = kDefaultContractBlocks;
  std::memset(out, 0, sizeof(*out));
  out->count = count;
  out->precision = (int)prec;
  out->n_slices = (prec == TL_SPLIT_BF16 || prec == TL_SPLIT_FP16)
                      ? (n_slices > 0 ? n_slices : (prec == TL_SPLIT_FP16 ? 5 : 6))
                      : 0;
  if (out->n_slices)
    TL_REQUIRE(out->n_slices >= 2 && out->n_slices <= (prec == TL_SPLIT_FP16 ? 6 : 7),
               "n_slices = %d outside [2, %d]", out->n_slices, prec == TL_SPLIT_FP16 ? 6 : 7);
  out->want_blocks = want_blocks;
  out->tile_edge = 64;
  out->desc_bytes = sizeof(BatchDesc);
  for (int i = 0; i < count; ++i) {
    InstanceSizes is;
    tl_status st = instance_sizes(&systems[i], prec, out->n_slices, want_blocks, &is);
    if (st != TL_OK) {
      char msg[1024];
      std::snprintf(msg, sizeof(msg), "instance %d: %s", i, tl_last_error());
      set_error("%s", msg);
      return st;
    }
    const Geometry& g = is.g;
    out->basis_elems += g.basis_elems;
    out->pot_elems += g.pot_elems;
    out->hs_elems += 2 * g.block_elems;
    out->eval_elems += (int64_t)g.L[0] * g.m0;
    out->kblocks += g.L[0];
    out->ws_bytes += is.pot_ws + is.asm_ws + is.fft_ws;
    out->max_m0 = std::max(out->max_m0, g.m0);
    out->max_len = std::max(out->max_len, g.L[0]);
  }
  return TL_OK;
}

extern "C" tl_status tl_batch_write_descriptor(const tl_system* systems, int count,
                                               const tl_batch_plan* plan,
                                               const tl_batch_buffers* buf, void* host_desc,
                                               size_t desc_bytes) {
  clear_error();
  TL_REQUIRE(systems && plan && buf && host_desc, "null argument");
  TL_REQUIRE(count == plan->count, "count differs from the plan");
  TL_REQUIRE(desc_bytes >= sizeof(BatchDesc), "descriptor buffer needs %zu bytes",
             sizeof(BatchDesc));
  TL_REQUIRE(buf->G && buf->AG && buf->SG && buf->P && buf->HS && buf->HSbar && buf->evals &&
                 buf->info && buf->ws,
             "null device buffer");
  TL_REQUIRE(plan->tile_edge == 64 || plan->tile_edge == 32, "tile_edge = %d is not 64 or 32",
             plan->tile_edge);
  const tl_precision prec = (tl_precision)plan->precision;
  std::vector<char> storage(sizeof(BatchDesc));
  BatchDesc* d = (BatchDesc*)storage.data();
  std::memset(d, 0, sizeof(BatchDesc));
  d->count = count;
  int64_t ob = 0, op = 0, ohs = 0, oev = 0, okb = 0;
  size_t ows = 0;
  for (int i = 0; i < count; ++i) {
    const tl_system* s = &systems[i];
    InstanceSizes is;
    TL_TRY(instance_sizes(s, prec, plan->n_slices, plan->want_blocks, &is));
    const Geometry& g = is.g;
    InstanceJob& J = d->job[i];
    make_basis_args(g, s, &J.basis);
    J.G = buf->G + ob;
    J.AG = buf->AG + ob;
    J.SG = buf->SG + ob;
    double* P = buf->P + op;
    char* ws = (char*)buf->ws + ows;
    TL_TRY(plan_potential(g, s, P, ws, is.pot_ws, &J.pot));
    J.T = (int)g.pot_terms;
    double* H = buf->HS + ohs;
    double* S = H + g.block_elems;
    TL_TRY(plan_assembly(g, J.G, J.AG, J.SG, P, prec, plan->n_slices, H, S, ws + is.pot_ws,
                         is.asm_ws, plan->want_blocks, &J.asmb, plan->tile_edge));
    // one lattice axis: transform H and S (outer = 2) along L
    double* Hbar = buf->HSbar + 2 * ohs;
    const int Ls[3] = {g.L[0], 1, 1};
    if (!plan_fft(H, Hbar, Ls, g.m0, 2, &J.fft)) {
      set_error("instance %d: no LDS FFT plan for L = %d", i, g.L[0]);
      return TL_EUNSUPPORTED;
    }
    set_fft_blue_tables(&J.fft, ws + is.pot_ws + is.asm_ws);
    J.Hb = Hbar;
    J.Sb = Hbar + 2 * g.block_elems;
    J.evals = buf->evals + oev;
    J.info = buf->info + okb;
    J.m0 = g.m0;
    // stage block counts of this instance
    int64_t blocks[kStages];
    blocks[kBasis] = ceil_div(g.basis_elems, 256);
    blocks[kPotential] = (int64_t)J.pot.fold_blocks + J.pot.direct_blocks;
    blocks[kRowMax] = J.asmb.rowmax_blocks;
    blocks[kContract] = J.asmb.contract_blocks;
    blocks[kReduce] = ceil_div(J.asmb.reduce_total, 256);
    {
      const dev::CombineArgs& c = J.asmb.combine;
      blocks[kCombine] = dev::combine_pair_fits(c.T, c.L)
                             ? (int64_t)c.m0 * c.m0 * ceil_div(c.L[0] * c.L[1] * c.L[2], 256)
                             : ceil_div(J.asmb.combine_total, 4);
    }
    blocks[kFftTables] = J.fft.blue ? 1 : 0;
    blocks[kDft] = J.fft.blue ? 0 : ceil_div(J.fft.cols, J.fft.W);
    blocks[kDftBlue] = J.fft.blue ? ceil_div(J.fft.cols, J.fft.W) : 0;
    blocks[kHeigh] = g.m0 <= 8 ? 0 : g.L[0];
    blocks[kHeigh8] = g.m0 <= 8 ? g.L[0] : 0;
    for (int st = 0; st < kStages; ++st) d->prefix[st][i + 1] = d->prefix[st][i] + blocks[st];
    ob += g.basis_elems;
    op += g.pot_elems;
    ohs += 2 * g.block_elems;
    oev += (int64_t)g.L[0] * g.m0;
    okb += g.L[0];
    ows += is.pot_ws + is.asm_ws + is.fft_ws;
  }
  std::memcpy(host_desc, d, sizeof(BatchDesc));
  return TL_OK;
}

namespace {

template <typename LowT, int SPT>
void launch_batch_split_s(int S, unsigned grid, size_t lds, const BatchDesc* d,
                          hipStream_t stream, hipEvent_t e0, hipEvent_t e1) {
  const dim3 g(grid), b(dev::kSplitThreads);
  switch (S) {
    case 2: launch_with_events(batch_contract_split_kernel<LowT, 2, SPT>, g, b, lds, stream, e0, e1, d); break;
    case 3: launch_with_events(batch_contract_split_kernel<LowT, 3, SPT>, g, b, lds, stream, e0, e1, d); break;
    case 4: launch_with_events(batch_contract_split_kernel<LowT, 4, SPT>, g, b, lds, stream, e0, e1, d); break;
    case 5: launch_with_events(batch_contract_split_kernel<LowT, 5, SPT>, g, b, lds, stream, e0, e1, d); break;
    case 6: launch_with_events(batch_contract_split_kernel<LowT, 6, SPT>, g, b, lds, stream, e0, e1, d); break;
    default: launch_with_events(batch_contract_split_kernel<LowT, 7, SPT>, g, b, lds, stream, e0, e1, d); break;
  }
}

template <typename LowT>
void launch_batch_rowmax(int S, unsigned grid, const BatchDesc* d, hipStream_t stream) {
  const dim3 g(grid), b(256);
  switch (S) {
    case 2: hipLaunchKernelGGL((batch_rowmax_kernel<LowT, 2>), g, b, 0, stream, d); break;
    case 3: hipLaunchKernelGGL((batch_rowmax_kernel<LowT, 3>), g, b, 0, stream, d); break;
    case 4: hipLaunchKernelGGL((batch_rowmax_kernel<LowT, 4>), g, b, 0, stream, d); break;
    case 5: hipLaunchKernelGGL((batch_rowmax_kernel<LowT, 5>), g, b, 0, stream, d); break;
    case 6: hipLaunchKernelGGL((batch_rowmax_kernel<LowT, 6>), g, b, 0, stream, d); break;
    default: hipLaunchKernelGGL((batch_rowmax_kernel<LowT, 7>), g, b, 0, stream, d); break;
  }
}

template <typename LowT>
void launch_batch_split(int S, int spt, unsigned grid, size_t lds, const BatchDesc* d,
                        hipStream_t stream, hipEvent_t e0, hipEvent_t e1) {
  if (spt <= 2)
    launch_batch_split_s<LowT, 2>(S, grid, lds, d, stream, e0, e1);
  else
    launch_batch_split_s<LowT, 4>(S, grid, lds, d, stream, e0, e1);
}

}  // namespace

extern "C" tl_status tl_batch_run(const tl_batch_plan* plan, const void* host_desc,
                                  const void* desc_dev, void* stream_) {
  clear_error();
  TL_REQUIRE(plan && host_desc && desc_dev, "null argument");
  hipStream_t stream = (hipStream_t)stream_;
  const BatchDesc* hd = (const BatchDesc*)host_desc;
  const BatchDesc* d = (const BatchDesc*)desc_dev;
  TL_REQUIRE(hd->count == plan->count, "descriptor does not match the plan");
  auto blocks = [&](int st) { return (unsigned)hd->prefix[st][hd->count]; };
  const tl_precision prec = (tl_precision)plan->precision;
  hipEvent_t ev0, ev1;
  contraction_events(&ev0, &ev1);

  hipLaunchKernelGGL(batch_basis_kernel, dim3(blocks(kBasis)), dim3(256), 0, stream, d);
  TL_CHECK_LAUNCH();
  if (blocks(kPotential)) {
    hipEvent_t p0, p1;
    stage_events(TL_STAGE_LATTICE_SUM, &p0, &p1);
    launch_with_events(batch_potential_kernel, dim3(blocks(kPotential)), dim3(256), 0, stream,
                       p0, p1, d);
    TL_CHECK_LAUNCH();
  }
  size_t split_lds = 0;
  int split_spt = 2;
  if (prec == TL_SPLIT_BF16 || prec == TL_SPLIT_FP16) {
    if (prec == TL_SPLIT_BF16)
      launch_batch_rowmax<__bf16>(plan->n_slices, blocks(kRowMax), d, stream);
    else
      launch_batch_rowmax<_Float16>(plan->n_slices, blocks(kRowMax), d, stream);
    TL_CHECK_LAUNCH();
    for (int i = 0; i < hd->count; ++i) {
      split_lds = std::max(split_lds, hd->job[i].asmb.split_lds);
      split_spt = std::max(split_spt, hd->job[i].asmb.split_spt);
    }
  }
  // the profiling events (if set) are attached to the contraction launch
  const hipEvent_t e0 = ev0, e1 = ev1;
  const dim3 cgrid(blocks(kContract)), cblk(256);
  if (prec == TL_SPLIT_BF16)
    launch_batch_split<__bf16>(plan->n_slices, split_spt, blocks(kContract), split_lds, d, stream,
                               e0, e1);
  else if (prec == TL_SPLIT_FP16)
    launch_batch_split<_Float16>(plan->n_slices, split_spt, blocks(kContract), split_lds, d,
                                 stream, e0, e1);
  else if (prec == TL_FP32)
    launch_with_events(batch_contract_f32_kernel, cgrid, cblk, 0, stream, e0, e1, d);
  else {
    // the source-row kernel when every instance's tiles fit its LDS budget
    size_t src_lds = 0;
    bool all_src = true;
    for (int i = 0; i < hd->count; ++i) {
      all_src = all_src && hd->job[i].asmb.src_tile > 0;
      src_lds = std::max(src_lds, hd->job[i].asmb.src_lds);
    }
    if (all_src)
      launch_with_events(batch_contract_f64_src_kernel, cgrid, cblk, src_lds, stream, e0, e1, d);
    else
      launch_with_events(batch_contract_f64_kernel, cgrid, cblk, 0, stream, e0, e1, d);
  }
  TL_CHECK_LAUNCH();
  hipLaunchKernelGGL(batch_reduce_kernel, dim3(blocks(kReduce)), dim3(256), 0, stream, d);
  TL_CHECK_LAUNCH();
  hipLaunchKernelGGL(batch_combine_kernel, dim3(blocks(kCombine)), dim3(256), 0, stream, d);
  TL_CHECK_LAUNCH();
  size_t fft_lds = 0, blue_lds = 0, tab_lds = 0;
  for (int i = 0; i < hd->count; ++i) {
    const dev::FftArgs& fa = hd->job[i].fft;
    if (fa.blue) {
      blue_lds = std::max(blue_lds, dev::fft_lds_bytes(fa));
      tab_lds = std::max(tab_lds, dev::fft_tables_lds_bytes(fa));
    } else {
      fft_lds = std::max(fft_lds, dev::fft_lds_bytes(fa));
    }
  }
  if (blocks(kFftTables)) {
    hipLaunchKernelGGL(batch_fft_tables_kernel, dim3(blocks(kFftTables)), dim3(dev::kFftThreads),
                       tab_lds, stream, d);
    TL_CHECK_LAUNCH();
  }
  // the stage's start event goes with the first of the two transform
  // launches, its stop event with the last
  hipEvent_t f0, f1;
  stage_events(TL_STAGE_FFT, &f0, &f1);
  const unsigned nstd = blocks(kDft), nblue = blocks(kDftBlue);
  if (nstd) {
    launch_with_events(batch_fft_kernel, dim3(nstd), dim3(dev::kFftThreads), fft_lds, stream, f0,
                       nblue ? nullptr : f1, d);
    TL_CHECK_LAUNCH();
  }
  if (nblue) {
    launch_with_events(batch_fft_blue_kernel, dim3(nblue), dim3(dev::kFftThreads), blue_lds,
                       stream, nstd ? nullptr : f0, f1, d);
    TL_CHECK_LAUNCH();
  }
  if (blocks(kHeigh8)) {
    hipLaunchKernelGGL(batch_heigh8_kernel, dim3(blocks(kHeigh8)), dim3(64), 0, stream, d);
    TL_CHECK_LAUNCH();
  }
  if (blocks(kHeigh)) {  // instances with m0 > 8
    if (plan->max_m0 <= 16)
      hipLaunchKernelGGL(batch_heigh16_kernel, dim3(blocks(kHeigh)), dim3(256), 0, stream, d);
    else
      hipLaunchKernelGGL(batch_heigh_kernel<32>, dim3(blocks(kHeigh)), dim3(1024), 0, stream, d);
    TL_CHECK_LAUNCH();
  }
  return TL_OK;
}
