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
// factor is a shifted window of one "master" vector b~_q[j] = b_q(j h; 0) on
// the accompanying grid (Sec. 3.2, master tensor and eq. (core_tens)), so the
// master vectors are computed once (ALU-bound, erfc) and the windows are sums
// of shifted reads (a few adds per node).
// Open dims: one factor per nucleus, evaluated directly.
#include <algorithm>
#include <cmath>
#include <map>
#include <vector>

#include "common.h"

namespace tl {
namespace {

// 8-point Gauss-Legendre rule on [-1, 1] (Abramowitz & Stegun, Table 25.4).
__constant__ double kGLx[4] = {0.18343464249564984, 0.525532409916329, 0.7966664774136267,
                               0.9602898564975363};
__constant__ double kGLw[4] = {0.36268378337836205, 0.3137066458778876, 0.22238103445337473,
                               0.10122853629037562};

// int_{x-h/2}^{x+h/2} exp(-t^2 (y-A)^2) dy.  For t*h >= 1/2 the erf difference
// is formed where it does not cancel (erfc of two positive or two negative
// arguments); below, every erf difference cancels, and the integrand is so
// smooth on the cell that Gauss-Legendre reaches full precision.
__device__ double cell_int(double t, double x, double h, double A) {
  if (t * h < 0.5) {
    double acc = 0.0;
    double c = x - A;
    double t2 = t * t;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      double y1 = c + 0.5 * h * kGLx[k];
      double y2 = c - 0.5 * h * kGLx[k];
      acc += kGLw[k] * (exp(-t2 * y1 * y1) + exp(-t2 * y2 * y2));
    }
    return 0.5 * h * acc;
  }
  double u = t * (x - 0.5 * h - A);
  double v = t * (x + 0.5 * h - A);
  double d;
  if (u >= 0.0)
    d = erfc(u) - erfc(v);
  else if (v <= 0.0)
    d = erfc(-v) - erfc(-u);
  else
    d = erf(v) + erf(-u);
  return d * (0.886226925452758014 / t);  // sqrt(pi)/2 / t
}

struct QuadArgs {  // the exponential-sum table, passed by value
  double t[TL_MAX_R];
  double w[TL_MAX_R];
};

// ---- a2 + open transverse dims in one launch.
// Blocks [0, master_blocks): master vectors b~_q[j], j = -J..J.
// Blocks after that: the y / z factors of open dims (one per group and
// term), b_q(x_i; y_g), which need no lattice sum.
struct DirectArgs {
  int R, J, master_blocks;
  double h;
  // open transverse dims (y = 1, z = 2)
  int n_open;                 // number of open transverse dims handled here (0..2)
  int open_dim[2];
  int n[2];
  double x0[2];
  int64_t out_off[2];         // element offset of the dim in P
  int blocks_per_term[2];
  int T;                      // terms = groups * R
  double gpos[2][TL_MAX_SITES];  // group coordinate on each open dim
};

__global__ __launch_bounds__(256) void direct_kernel(DirectArgs a, QuadArgs quad,
                                                     double* __restrict__ master,
                                                     double* __restrict__ P) {
  int b = blockIdx.x;
  if (b < a.master_blocks) {
    int64_t idx = (int64_t)b * blockDim.x + threadIdx.x;
    int64_t width = 2 * (int64_t)a.J + 1;
    if (idx >= (int64_t)a.R * width) return;
    int q = (int)(idx / width);
    int j = (int)(idx - (int64_t)q * width) - a.J;
    master[idx] = cell_int(quad.t[q], (double)j * a.h, a.h, 0.0);
    return;
  }
  b -= a.master_blocks;
  int od = 0;
  int span0 = a.T * a.blocks_per_term[0];
  if (a.n_open == 2 && b >= span0) {
    od = 1;
    b -= span0;
  }
  int t = b / a.blocks_per_term[od];
  int chunk = b - t * a.blocks_per_term[od];
  int i = chunk * blockDim.x + threadIdx.x;
  if (i >= a.n[od]) return;
  int g = t / a.R, q = t - g * a.R;
  double x = a.x0[od] + a.h * (double)i;
  P[a.out_off[od] + (int64_t)t * a.n[od] + i] = cell_int(quad.t[q], x, a.h, a.gpos[od][g]);
}

struct FoldArgs {
  int n_sites;
  int site_group[TL_MAX_SITES];
  int site_off[3][TL_MAX_SITES];   // site offset per dim, in nodes
  double site_Z[TL_MAX_SITES];
  int group_off[3][TL_MAX_SITES];  // representative offset of each group per dim
  int dims[3];                     // periodic dims handled by this launch
  int c[3], K[3], n[3];
  int64_t out_off[3];
  int R, J;
};

// ---- a3 (torus dims): workgroup per (term, periodic dim).  Threads split the
// image sum of every window node, partial sums meet in LDS, the window is
// then replicated over the torus.
__global__ __launch_bounds__(256) void fold_kernel(FoldArgs p, QuadArgs quad,
                                                   const double* __restrict__ master,
                                                   double* __restrict__ P) {
  extern __shared__ double sh[];  // win[c] then part[256]
  const int slot = blockIdx.y;
  const int dim = p.dims[slot];
  const int c = p.c[slot], K = p.K[slot], n = p.n[slot];
  double* win = sh;
  double* part = sh + c;
  const int t = blockIdx.x;
  const int g = t / p.R;
  const int q = t - g * p.R;
  const double* mq = master + (int64_t)q * (2 * p.J + 1) + p.J;  // mq[j], j in [-J, J]
  const int half = c / 2;
  const int tid = threadIdx.x;
  auto image_sum = [&](int rr, int k_first, int k_step) {
    double acc = 0.0;
    for (int k = -K + k_first; k <= K; k += k_step) {
      if (dim == 0) {
        for (int s = 0; s < p.n_sites; ++s)
          if (p.site_group[s] == g) acc += p.site_Z[s] * mq[rr - p.site_off[0][s] - k * c];
      } else {
        acc += mq[rr - p.group_off[dim][g] - k * c];
      }
    }
    return acc;
  };
  const double wscale = dim == 0 ? quad.w[q] : 1.0;
  if (c <= 256) {
    const int np = 256 / c;
    if (tid < np * c) part[tid] = image_sum(tid % c - half, tid / c, np);
    __syncthreads();
    if (tid < c) {
      double v = 0.0;
      for (int s2 = 0; s2 < np; ++s2) v += part[tid + s2 * c];
      win[tid] = v * wscale;
    }
  } else {
    for (int r = tid; r < c; r += blockDim.x) win[r] = image_sum(r - half, 0, 1) * wscale;
  }
  __syncthreads();
  double* out = P + p.out_off[slot] + (int64_t)t * n;
  for (int i = tid; i < n; i += blockDim.x) out[i] = win[(i + half) % c];
}

constexpr int kNucChunk = 80;
struct BoxArgs {
  double pos[kNucChunk];  // nucleus x coordinate
  double Z[kNucChunk];
  int group[kNucChunk];
  int count, R, n, accumulate;
  double x0, h;
};

// ---- a3 (open dim 0, box mode): thread per (term, node), direct cell
// integrals of every nucleus of the chunk.
__global__ __launch_bounds__(256) void box_potential_kernel(BoxArgs p, QuadArgs quad,
                                                            double* __restrict__ P) {
  int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  int t = blockIdx.y;
  if (idx >= p.n) return;
  int g = t / p.R;
  int q = t - g * p.R;
  double x = p.x0 + p.h * (double)idx;
  double tt = quad.t[q];
  double acc = 0.0;
  for (int s = 0; s < p.count; ++s) {
    if (p.group[s] != g) continue;
    acc += p.Z[s] * cell_int(tt, x, p.h, p.pos[s]);
  }
  acc *= quad.w[q];
  double* out = P + (int64_t)t * p.n + idx;
  if (p.accumulate)
    *out += acc;
  else
    *out = acc;
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

int master_half_width(const Geometry& g, const tl_system* s) {
  int J = 0;
  for (int d = 0; d < 3; ++d) {
    if (!g.periodic[d]) continue;
    int maxoff = 0;
    for (int nu = 0; nu < s->n_nuc; ++nu)
      maxoff = std::max(maxoff, (int)std::lround(std::fabs(s->nuc_pos[3 * nu + d]) / g.h));
    J = std::max(J, g.K[d] * g.cell_nodes[d] + g.cell_nodes[d] / 2 + maxoff + 2);
  }
  return J;
}

}  // namespace

size_t potential_workspace_bytes(const Geometry& g, const tl_system* s) {
  int J = master_half_width(g, s);
  if (J == 0) return 0;
  return align_up(sizeof(double) * (size_t)g.R * (2 * (size_t)J + 1), 256);
}

tl_status lattice_sum_potential(const Geometry& g, const tl_system* s, double* P, void* ws,
                                size_t ws_bytes, hipStream_t stream) {
  size_t need = potential_workspace_bytes(g, s);
  if (ws_bytes < need || (need > 0 && ws == nullptr)) {
    set_error("potential workspace: need %zu bytes, got %zu", need, ws_bytes);
    return TL_EWORKSPACE;
  }
  double* master = (double*)ws;
  QuadArgs quad;
  std::memset(&quad, 0, sizeof(quad));
  for (int q = 0; q < g.R; ++q) {
    quad.t[q] = s->t_q[q];
    quad.w[q] = s->w_q[q];
  }
  GroupInfo gi = make_groups(s);
  int J = master_half_width(g, s);
  const int T = (int)g.pot_terms;
  // launch 1: master vectors + open transverse dims
  {
    DirectArgs da;
    std::memset(&da, 0, sizeof(da));
    da.R = g.R;
    da.J = J;
    da.h = g.h;
    da.T = T;
    da.master_blocks = J > 0 ? (int)ceil_div((int64_t)g.R * (2 * J + 1), 256) : 0;
    int total_blocks = da.master_blocks;
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
    if (total_blocks > 0) {
      hipLaunchKernelGGL(direct_kernel, dim3((unsigned)total_blocks), dim3(256), 0, stream, da,
                         quad, master, P);
      TL_CHECK_LAUNCH();
    }
  }
  // launch 2: lattice sums of every torus dim
  {
    FoldArgs fa;
    std::memset(&fa, 0, sizeof(fa));
    fa.n_sites = s->n_nuc;
    fa.R = g.R;
    fa.J = J;
    for (int nu = 0; nu < s->n_nuc; ++nu) {
      fa.site_group[nu] = gi.of_nucleus[nu];
      fa.site_Z[nu] = s->nuc_Z[nu];
      for (int d = 0; d < 3; ++d)
        fa.site_off[d][nu] = (int)std::lround(s->nuc_pos[3 * nu + d] / g.h);
    }
    for (int gr = 0; gr < g.n_groups; ++gr) {
      fa.group_off[1][gr] = (int)std::lround(gi.y[gr] / g.h);
      fa.group_off[2][gr] = (int)std::lround(gi.z[gr] / g.h);
    }
    int slots = 0;
    int cmax = 0;
    for (int d = 0; d < 3; ++d) {
      if (!g.periodic[d]) continue;
      fa.dims[slots] = d;
      fa.c[slots] = g.cell_nodes[d];
      fa.K[slots] = g.K[d];
      fa.n[slots] = g.n[d];
      fa.out_off[slots] = g.pot_off[d];
      cmax = std::max(cmax, g.cell_nodes[d]);
      ++slots;
    }
    if (slots > 0) {
      size_t shmem = sizeof(double) * ((size_t)cmax + 256);
      if (shmem > 64 * 1024) {
        set_error("cell of %d nodes exceeds the LDS window", cmax);
        return TL_EUNSUPPORTED;
      }
      hipLaunchKernelGGL(fold_kernel, dim3((unsigned)T, (unsigned)slots), dim3(256), shmem, stream,
                         fa, quad, master, P);
      TL_CHECK_LAUNCH();
    }
  }
  // box mode: dim 0 sums every nucleus directly, in chunks
  if (!g.periodic[0]) {
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
      hipLaunchKernelGGL(box_potential_kernel, grid, dim3(256), 0, stream, ba, quad, P);
      TL_CHECK_LAUNCH();
    }
  }
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
