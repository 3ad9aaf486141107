// Shared host/device helpers of the tl library (gfx950).
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>

#include "../../include/tl.h"

namespace tl {

// ---------------------------------------------------------------- errors
void set_error(const char* fmt, ...);
void clear_error();
// events of the profiling hook for `stage` (TL_STAGE_*); both null when unset
void stage_events(int stage, hipEvent_t* start, hipEvent_t* stop);

#define TL_REQUIRE(cond, ...)            \
  do {                                   \
    if (!(cond)) {                       \
      ::tl::set_error(__VA_ARGS__);      \
      return TL_EINVAL;                  \
    }                                    \
  } while (0)

#define TL_HIP(call)                                                        \
  do {                                                                      \
    hipError_t e_ = (call);                                                 \
    if (e_ != hipSuccess) {                                                 \
      ::tl::set_error("%s failed: %s", #call, hipGetErrorString(e_));       \
      return TL_EHIP;                                                       \
    }                                                                       \
  } while (0)

#define TL_CHECK_LAUNCH()                                                   \
  do {                                                                      \
    hipError_t e_ = hipGetLastError();                                      \
    if (e_ != hipSuccess) {                                                 \
      ::tl::set_error("kernel launch failed: %s", hipGetErrorString(e_));   \
      return TL_EHIP;                                                       \
    }                                                                       \
  } while (0)

#define TL_TRY(expr)               \
  do {                             \
    tl_status s_ = (expr);         \
    if (s_ != TL_OK) return s_;    \
  } while (0)

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

// --------------------------------------------------------- system digest
// Everything the kernels need, validated and flattened on the host.
struct FnParams {          // one unit-cell basis function
  double center[3];
  double alpha;
  double coef[3];
  int l[3];
};

struct Geometry {
  int mode;
  int L[3];
  int periodic[3];
  int n[3];
  int cell_nodes[3];
  int K[3];
  double h;
  double x0[3];
  double a[3];
  double box_origin0;
  int m0;
  int R;
  int n_groups;                 // groups of nuclei with equal (y, z)
  int64_t basis_rows[3];
  int64_t basis_off[3];         // element offset of dim l in G/AG/SG
  int64_t pot_terms;            // R * n_groups
  int64_t pot_off[3];           // element offset of dim l in P
  int64_t basis_elems, pot_elems, block_elems;
  int shifts[3];                // contracted shifts per dim: L/2+1 (torus) or 1
};

tl_status digest(const tl_system* sys, Geometry* g);

// Kernel launch with optional profiling events attached to the kernel itself
// (hipExtLaunchKernel: the start / stop events time exactly this kernel on
// its stream); null events give a plain launch.
template <typename K, typename... A>
inline void launch_with_events(K kernel, dim3 grid, dim3 block, size_t shmem, hipStream_t stream,
                               hipEvent_t start, hipEvent_t stop, A... args) {
  hipExtLaunchKernelGGL(kernel, grid, block, (std::uint32_t)shmem, stream, start, stop, 0u,
                        args...);
}

}  // namespace tl
