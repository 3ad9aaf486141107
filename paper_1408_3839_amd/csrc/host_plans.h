// Host-side launch plans shared by the single-system entry points and the
// batched path: every stage is described by the kernel-argument structs it
// launches with, built once on the host.
#pragma once
#include "common.h"
#include "dev_assemble.h"
#include "dev_basis.h"
#include "dev_fft.h"
#include "dev_heigh.h"
#include "dev_potential.h"

namespace tl {

constexpr int kDefaultContractBlocks = 512;  // workgroups the contraction aims for

inline bool is_split(tl_precision prec) { return prec == TL_SPLIT_BF16 || prec == TL_SPLIT_FP16; }
inline int default_slices(tl_precision prec) { return prec == TL_SPLIT_FP16 ? 5 : 6; }
// beta s + 1 bits of the rounded integer and its bias must fit an int64
inline int max_slices(tl_precision prec) { return prec == TL_SPLIT_FP16 ? 6 : 7; }

struct AssemblyPlan {
  tl_precision prec;
  int n_slices;
  dev::ContractArgs contract;
  dev::RowMaxArgs rowmax;  // split modes: exponents of the source rows' maxima
  dev::SplitArgs split;
  int contract_blocks, rowmax_blocks;
  size_t split_lds;        // split modes: dynamic LDS of the contraction
  int split_spt;           // split modes: staged source rows per thread pass (8 or 16)
  dev::ReduceArgs reduce;
  int64_t reduce_total;
  dev::CombineArgs combine;
  int64_t combine_total;
  size_t src_lds;  // FP64: dynamic LDS of the source-row kernel (0: the staging kernel)
  int src_tile;    // FP64: tile edge of the source-row kernel (32 or 64; 0: staging kernel)
};

size_t assemble_workspace_bytes(const Geometry& g, tl_precision prec, int n_slices,
                                int want_blocks);
// tile_hint: the largest tile edge of the FP64 source-row contraction that
// may be used (32: latency-bound single systems; 64: large batches).
tl_status plan_assembly(const Geometry& g, const double* G, const double* AG, const double* SG,
                        const double* P, tl_precision prec, int n_slices, double* H, double* S,
                        void* ws, size_t ws_bytes, int want_blocks, AssemblyPlan* out,
                        int tile_hint = 32);
// combine = false: contraction and partial-sum reduction only (compact C_l
// left in the workspace for another combination).
tl_status launch_assembly(const AssemblyPlan& ap, hipStream_t stream, bool combine = true);
void contraction_events(hipEvent_t* start, hipEvent_t* stop);

struct PotentialPlan {
  dev::QuadArgs quad;
  dev::DirectArgs direct;
  int direct_blocks;
  dev::FoldArgs fold;
  int fold_slots;
  int fold_blocks;  // torus-dim workgroups, ahead of the direct blocks in the launch
  double* P;
  int box_dim0;   // open dim 0: nuclei summed directly (single-system path only)
};

size_t potential_workspace_bytes(const Geometry& g, const tl_system* s);
tl_status plan_potential(const Geometry& g, const tl_system* s, double* P, void* ws,
                         size_t ws_bytes, PotentialPlan* out);

void make_basis_args(const Geometry& g, const tl_system* s, dev::BasisArgs* p);
tl_status build_basis(const Geometry& g, const tl_system* s, double* G, double* AG, double* SG,
                      hipStream_t stream);

// Block FFT over the lattice index in LDS (one launch, no workspace); false
// when the lattice does not fit a workgroup's buffer.  min_groups: fewer
// columns per workgroup while the launch would have fewer workgroups (a
// single system's transform is latency-bound; a batch has many instances).
constexpr int kFftSingleGroups = 256;
bool plan_fft(const double* in, double* out, const int L[3], int m0, int64_t batch,
              dev::FftArgs* a, int min_groups = 1);
// the same for E real entries per lattice point (any column count, not m0^2)
bool plan_fft_cols(const double* in, double* out, const int L[3], int64_t E, int64_t batch,
                   dev::FftArgs* a, int min_groups = 1);
// workspace of the Bluestein tables (0 for 7-smooth lattices) and their place in it
size_t fft_blue_table_bytes(const dev::FftArgs& a);
void set_fft_blue_tables(dev::FftArgs* a, void* ws);
tl_status launch_fft(const dev::FftArgs& a, hipStream_t stream);

size_t box_workspace_bytes(const Geometry& g);
tl_status assemble_box(const Geometry& g, const tl_system* s, const double* G, const double* AG,
                       const double* SG, const double* P, tl_precision prec, int n_slices,
                       double* H, double* S, void* ws, size_t ws_bytes, hipStream_t stream);

}  // namespace tl
