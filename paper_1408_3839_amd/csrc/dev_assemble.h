// Device code of steps a4/a5 (1D contractions in every precision mode, the
// partial-sum reduction and the FP64 combination), shared by the
// single-system and the batched launches.
#pragma once
#include "common.h"
#include "dev_wave.h"

namespace tl {
namespace dev {

typedef double f64x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

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
  int kc;          // nodes per LDS sub-chunk of the source-row kernel (64, 128 or 256)
  int ypad;        // source-row kernel: pad doubles after every 32 window nodes (1 or 2)
};

// LDS layout (offsets in doubles) of the source-row FP64 kernel for one
// 32 x 32 tile and a sub-chunk of kc nodes.  A zero row and a ones row come
// first: lanes outside the matrix read zeros, and the kinetic and mass rows
// (no potential factor) multiply by one, so the MFMA loop has no branch or
// select.  X rows (term t, nu) are formed from the P row of t and the G, AG
// or SG row of nu; Y columns (mu, shift) from one window of mu's G row that
// covers all of the tile's shifts of mu.  Rows sit at the stride kc + 2
// (2 mod 32), so the 32 lanes of an operand read (16 rows, 2 nodes) fall in
// distinct banks; window node x sits at x + ypad (x / 32), with ypad chosen
// per dimension so that windows read cn nodes apart do too.  A dimension
// with a single shift (S = 1) needs no windows: each Y column is then the G
// row of its mu over the sub-chunk, which every tile of that dimension
// stages in its G block and reads with no padding (ypd = 0).  Shared by the
// host (sizing) and the kernel.
constexpr int kMaxSrcTile = 64;  // largest tile edge of the source-row kernel

struct TileLayout {
  int t0, nP;               // P rows t0 .. t0+nP-1 (terms below T)
  int offP, offG, offA, offS;  // row blocks; offG/A/S = -1 when the tile has no such row
  int mu0, nmu;             // mu0 .. mu0+nmu-1
  int ypd;                  // pad doubles per 32 window nodes as read (0: Y from the G rows)
  int ysh_hi[kMaxSrcTile];  // per local mu: largest shift of the tile
  int yoff[kMaxSrcTile];    // per local mu: offset of its window
  int ylen[kMaxSrcTile];    // per local mu: window length in nodes (0: not staged)
  int xtotal, total;        // doubles up to the end of the X sources, of everything
};

__host__ __device__ inline int src_zero_len(int kc) { return kc + (kc >> 4) + 4; }
__host__ __device__ inline int src_ones_off(int kc) { return src_zero_len(kc); }

__host__ __device__ inline void tile_layout(int M, int N, int S, int cn, int m0, int T, int row0,
                                            int col0, int bm, int bn, int kc, int ypad,
                                            TileLayout* L) {
  const int ld = kc + 2;
  const int r1 = min(M, row0 + bm) - 1;
  const int t0 = row0 / m0, t1 = r1 / m0;
  L->t0 = t0;
  L->nP = t0 < T ? min(t1, T - 1) - t0 + 1 : 0;
  int off = src_ones_off(kc) + kc;
  L->offP = off;
  off += L->nP * ld;
  L->offG = L->offA = L->offS = -1;
  const bool yrows = S == 1;  // every column is shift 0: the Y columns are G rows
  if (t0 < T || yrows) {
    L->offG = off;
    off += m0 * ld;
  }
  if (t0 <= T && T <= t1) {
    L->offA = off;
    off += m0 * ld;
  }
  if (t0 <= T + 1 && T + 1 <= t1) {
    L->offS = off;
    off += m0 * ld;
  }
  L->xtotal = off;
  const int c1 = min(N, col0 + bn) - 1;
  L->mu0 = col0 / S;
  L->nmu = c1 / S - L->mu0 + 1;
  L->ypd = yrows ? 0 : ypad;
  for (int u = 0; u < L->nmu; ++u) {
    const int mu = L->mu0 + u;
    if (yrows) {
      L->ysh_hi[u] = 0;
      L->yoff[u] = L->offG + mu * ld;
      L->ylen[u] = 0;
      continue;
    }
    const int sh_lo = max(0, col0 - mu * S), sh_hi = min(S - 1, c1 - mu * S);
    const int len = kc + (sh_hi - sh_lo) * cn;
    L->ysh_hi[u] = sh_hi;
    L->yoff[u] = off;
    L->ylen[u] = len;
    off += len + ypad * (len >> 5) + ypad;
  }
  L->total = off;
}

struct ContractArgs {
  DimArgs d[3];
  int m0, T;
};

// One launch for the three dimensions.  Workgroup = 4 waves = a 32 x 32 tile
// of C_l over one chunk of nodes; each wave owns a 16 x 16 block and issues
// V_MFMA_F64_16X16X4_F64 from LDS.  The next 64-node stage is loaded into
// registers while the current one is multiplied (double buffering).
__device__ inline void contract_f64_body(const ContractArgs& a, int b) {
  __shared__ double Xs[kBM][kLDP];
  __shared__ double Ys[kBN][kLDP];
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

// Source-row variant of the FP64 contraction, same chunking, MFMA sequence
// and output as contract_f64_body: per sub-chunk of kc nodes the workgroup
// stages only the distinct source rows of its BM x BN tile (TileLayout) in
// one burst of coalesced loads, then forms X = p_t g_nu and the shifted Y
// from LDS inside the MFMA loop.  Each of the 4 waves owns a BM/2 x BN/2
// quadrant of 16 x 16 MFMA blocks.  Every output block sees the products
// and the order of accumulation of contract_f64_body, so the partial sums
// agree bit for bit whatever the tile size.
template <int BM, int BN>
__device__ inline void contract_f64_src_body(const ContractArgs& a, int b) {
  constexpr int RM = BM / 32, RN = BN / 32;  // 16 x 16 blocks per wave and direction
  extern __shared__ double sm[];
  __shared__ TileLayout L;
  const int dd = b >= a.d[2].block_begin ? 2 : (b >= a.d[1].block_begin ? 1 : 0);
  const DimArgs& p = a.d[dd];
  const int local = b - p.block_begin;
  const int z = local % p.ks;
  const int rest = local / p.ks;
  const int col0 = (rest % p.tiles_n) * BN;
  const int row0 = (rest / p.tiles_n) * BM;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 1, wn = wave & 1;
  const int kbeg = z * p.kchunk, kend = min(p.n, kbeg + p.kchunk);
  const int kc = p.kc, ks2 = __ffs(kc) - 1, ld = kc + 2, ypad = p.ypad, ysh = ypad - 1;
  if (tid == 0) tile_layout(p.M, p.N, p.S, p.cn, a.m0, a.T, row0, col0, BM, BN, kc, ypad, &L);
  {  // the zero and ones rows
    const int zl = src_zero_len(kc);
    for (int e = tid; e < zl + kc; e += 256) sm[e] = e < zl ? 0.0 : 1.0;
  }
  __syncthreads();
  const int ypd = L.ypd;
  // this lane's A rows and B columns as LDS offsets (the node is added);
  // lanes outside the matrix read the zero row
  int xp[RM], xb[RM], yo[RN], yw[RN];
  bool yin[RN];
#pragma unroll
  for (int rb = 0; rb < RM; ++rb) {
    const int row = row0 + wm * (BM / 2) + rb * 16 + (lane & 15);
    xp[rb] = 0;
    xb[rb] = 0;
    if (row < p.M) {
      const int t = row / a.m0, nu = row - t * a.m0;
      xp[rb] = t < a.T ? L.offP + (t - L.t0) * ld : src_ones_off(kc);
      xb[rb] = (t < a.T ? L.offG : (t == a.T ? L.offA : L.offS)) + nu * ld;
    }
  }
#pragma unroll
  for (int cb = 0; cb < RN; ++cb) {
    const int col = col0 + wn * (BN / 2) + cb * 16 + (lane & 15);
    yin[cb] = col < p.N;
    yo[cb] = 0;
    yw[cb] = 0;
    if (yin[cb]) {
      const int mu = col / p.S, sh = col - mu * p.S, u = mu - L.mu0;
      yo[cb] = L.yoff[u];
      yw[cb] = (L.ysh_hi[u] - sh) * p.cn;
    }
  }
  f64x4 acc[RM][RN];
#pragma unroll
  for (int rb = 0; rb < RM; ++rb)
#pragma unroll
    for (int cb = 0; cb < RN; ++cb) acc[rb][cb] = f64x4{0.0, 0.0, 0.0, 0.0};
  for (int k0 = kbeg; k0 < kend; k0 += kc) {
    const int len = min(kc, kend - k0);
    __syncthreads();  // the previous sub-chunk's reads are done
    // every thread keeps one node of the sub-chunk and walks the rows
    const int kn = tid & (kc - 1), r0 = tid >> ks2, rstep = 256 >> ks2;
    const bool kin = kn < len;  // zero past the chunk end (zeroes X there)
    {  // P rows of the tile's terms
      const double* src = p.P + (int64_t)(L.t0 + r0) * p.n + k0 + kn;
#pragma unroll 4
      for (int r = r0; r < L.nP; r += rstep, src += (int64_t)rstep * p.n)
        sm[L.offP + r * ld + kn] = kin ? *src : 0.0;
    }
    for (int q = 0; q < 3; ++q) {  // G / AG / SG rows
      const int off = q == 0 ? L.offG : (q == 1 ? L.offA : L.offS);
      if (off < 0) continue;
      const double* src = (q == 0 ? p.G : (q == 1 ? p.AG : p.SG)) + (int64_t)r0 * p.n + k0 + kn;
#pragma unroll 4
      for (int r = r0; r < a.m0; r += rstep, src += (int64_t)rstep * p.n)
        sm[off + r * ld + kn] = kin ? *src : 0.0;
    }
    for (int u = 0; u < L.nmu; ++u) {  // window x holds node (k0 - sh_hi cn + x) mod n
      const double* g = p.G + (int64_t)(L.mu0 + u) * p.n;
      const int base = k0 - L.ysh_hi[u] * p.cn;
      double* dst = sm + L.yoff[u];
      const int wl = L.ylen[u];
#pragma unroll 4
      for (int x = tid; x < wl; x += 256) {
        int node = base + x;
        while (node < 0) node += p.n;
        while (node >= p.n) node -= p.n;
        dst[x + ((x >> 5) << ysh)] = g[node];
      }
    }
    __syncthreads();
    const int kmax = (len + 3) & ~3;
    constexpr int US = 8 / (RM * RN) > 0 ? 8 / (RM * RN) : 1;  // k steps with operands read first
    int kk = 0;
    for (; kk + 4 * US <= kmax; kk += 4 * US) {
      double av[US][RM], bv[US][RN];
#pragma unroll
      for (int s = 0; s < US; ++s) {
        const int k = kk + 4 * s + (lane >> 4);
#pragma unroll
        for (int rb = 0; rb < RM; ++rb) av[s][rb] = sm[xp[rb] + k] * sm[xb[rb] + k];
#pragma unroll
        for (int cb = 0; cb < RN; ++cb) {
          const int w = yw[cb] + k;
          bv[s][cb] = sm[yo[cb] + w + (w >> 5) * ypd];
        }
      }
#pragma unroll
      for (int s = 0; s < US; ++s)
#pragma unroll
        for (int rb = 0; rb < RM; ++rb)
#pragma unroll
          for (int cb = 0; cb < RN; ++cb)
            acc[rb][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[s][rb], bv[s][cb], acc[rb][cb], 0, 0, 0);
    }
    for (; kk < kmax; kk += 4) {
      const int k = kk + (lane >> 4);
      double av[RM], bv[RN];
#pragma unroll
      for (int rb = 0; rb < RM; ++rb) av[rb] = sm[xp[rb] + k] * sm[xb[rb] + k];
#pragma unroll
      for (int cb = 0; cb < RN; ++cb) {
        const int w = yw[cb] + k;
        bv[cb] = sm[yo[cb] + w + (w >> 5) * ypd];
      }
#pragma unroll
      for (int rb = 0; rb < RM; ++rb)
#pragma unroll
        for (int cb = 0; cb < RN; ++cb)
          acc[rb][cb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[rb], bv[cb], acc[rb][cb], 0, 0, 0);
    }
  }
  // f64 16x16x4 result layout on gfx950: register r of lane l holds
  // D[l / 16 + 4 r][l % 16].
#pragma unroll
  for (int rb = 0; rb < RM; ++rb)
#pragma unroll
    for (int cb = 0; cb < RN; ++cb) {
      const int col = col0 + wn * (BN / 2) + cb * 16 + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int orow = row0 + wm * (BM / 2) + rb * 16 + (lane >> 4) + 4 * r;
        if (orow < p.M && yin[cb]) p.part[((int64_t)z * p.M + orow) * p.N + col] = acc[rb][cb][r];
      }
    }
}

// ---------------------------------------------------------------- FP32 mode
// Same tiling; the operands are rounded to FP32 in the staging step and
// multiplied with V_MFMA_F32_16X16X4_F32; each 64-node stage's FP32 sums are
// added into FP64 accumulators.
__device__ inline void contract_f32_body(const ContractArgs& a, int b) {
  __shared__ float Xs[kBM][kLDP];
  __shared__ float Ys[kBN][kLDP];
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
  float xr[kPerThread], yr[kPerThread];
  const double* xa[kPerThread];
  const double* xb[kPerThread];
  const double* yb[kPerThread];
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
      xr[j] = (float)xv;
      yr[j] = (float)yv;
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
    f32x4 acc32 = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kk = 0; kk < kKT; kk += 4) {
      float av = Xs[wm * 16 + (lane & 15)][kk + (lane >> 4)];
      float bv = Ys[wn * 16 + (lane & 15)][kk + (lane >> 4)];
      acc32 = __builtin_amdgcn_mfma_f32_16x16x4f32(av, bv, acc32, 0, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[r] += (double)acc32[r];
    __syncthreads();
    if (more) commit();
    __syncthreads();
  }
  // f32 16x16x4 result layout: register r of lane l holds D[4 (l / 16) + r][l % 16]
  const int col = col0 + wn * 16 + (lane & 15);
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    int row = row0 + wm * 16 + 4 * (lane >> 4) + r;
    if (row < p.M && col < p.N) p.part[((int64_t)z * p.M + row) * p.N + col] = acc[r];
  }
}

// ---------------------------------------------------------------- split modes
// Operand splitting in the manner of Ozaki, Ogita, Oishi & Rump (2012): each
// row r of X (and of G) is scaled by a power of two sigma_r >= max|row|, and
// the scaled values are cut into integer slices
//   x/sigma = sum_k n_k 2^(-k beta),  |n_1| <= 2^beta, |n_k| <= 2^(beta-1),
// each exactly representable in bf16 (beta = 8) or fp16 (beta = 9).  A slice
// product summed over one 32-node MFMA (16x16x32) stays below 2^24 and is
// exact in FP32; all products of one level a + b are accumulated in FP32 over
// one MFMA step and then added to a per-level FP64 accumulator.  Only the
// products with a + b <= s + 1 are formed (triangular truncation).

constexpr int kMaxSlices = 8;
constexpr int kSliceAlign = 8;       // slice rows padded to a multiple of 8 nodes

template <typename T>
struct LowTraits;
template <>
struct LowTraits<__bf16> {
  static constexpr int beta = 8;
};
template <>
struct LowTraits<_Float16> {
  static constexpr int beta = 9;
};

struct SliceArgs {
  const double* P[3];
  const double* G[3];
  const double* AG[3];
  const double* SG[3];
  void* xs[3];          // [s][M][n] slices of X rows
  void* ys[3];          // [s][m0][n] slices of G rows
  double* xscale[3];    // [M]
  double* yscale[3];    // [m0]
  int n[3], M[3], ld[3];  // ld: padded row stride of the slices
  int rows_begin[7];    // X rows of dims 0..2, then G rows of dims 0..2
  int m0, T, s;
};

// Workgroup per row: max |value| (power-of-two scale), then the slices.
template <typename LowT>
__device__ inline void slice_body(const SliceArgs& a, int b) {
  constexpr int beta = LowTraits<LowT>::beta;
  __shared__ double wmax[4];
  int k = 0;
  while (k < 6 && b >= a.rows_begin[k + 1]) ++k;
  const bool isx = k < 3;
  const int d = isx ? k : k - 3;
  const int row = b - a.rows_begin[k];
  const int n = a.n[d];
  const double* base;
  const double* pot = nullptr;
  if (isx) {
    const int t = row / a.m0, nu = row - t * a.m0;
    base = (t < a.T ? a.G[d] : (t == a.T ? a.AG[d] : a.SG[d])) + (int64_t)nu * n;
    if (t < a.T) pot = a.P[d] + (int64_t)t * n;
  } else {
    base = a.G[d] + (int64_t)row * n;
  }
  double mx = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) {
    double v = pot ? pot[i] * base[i] : base[i];
    mx = fmax(mx, fabs(v));
  }
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o));
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = mx;
  __syncthreads();
  mx = fmax(fmax(wmax[0], wmax[1]), fmax(wmax[2], wmax[3]));
  // sigma = 2^e >= mx, so |x / sigma| <= 1 exactly
  int e = 0;
  if (mx > 0.0) {
    frexp(mx, &e);  // mx = f 2^e, f in [0.5, 1)
  }
  const double sigma = ldexp(1.0, e), inv = ldexp(1.0, -e);
  if (threadIdx.x == 0) (isx ? a.xscale[d] : a.yscale[d])[row] = sigma;
  LowT* out = (LowT*)(isx ? a.xs[d] : a.ys[d]);
  const int64_t rows = isx ? a.M[d] : a.m0;
  const int ld = a.ld[d];
  for (int i = threadIdx.x; i < ld; i += blockDim.x) {
    if (i >= n) {  // zero padding up to the aligned stride
      for (int q = 1; q <= a.s; ++q) out[((int64_t)(q - 1) * rows + row) * ld + i] = (LowT)0.0f;
      continue;
    }
    double v = (pot ? pot[i] * base[i] : base[i]) * inv;
    for (int q = 1; q <= a.s; ++q) {
      double sc = ldexp(1.0, q * beta);
      double nk = rint(v * sc);
      v = fma(-nk, ldexp(1.0, -q * beta), v);
      out[((int64_t)(q - 1) * rows + row) * ld + i] = (LowT)nk;
    }
  }
}

struct SplitDimArgs {
  const void* xs;       // [s][M][ld]
  const void* ys;       // [s][m0][ld]
  const double* xscale;
  const double* yscale;
  double* part;
  int n, ld, S, cn, M, N, kchunk, ks, tiles_n, block_begin;
};
struct SplitArgs {
  SplitDimArgs d[3];
  int m0, s;
};

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));

template <typename LowT>
struct Vec8;
template <>
struct Vec8<__bf16> {
  typedef bf16x8 type;
  static __device__ inline f32x4 mfma(type a, type b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
  }
};
template <>
struct Vec8<_Float16> {
  typedef f16x8 type;
  static __device__ inline f32x4 mfma(type a, type b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
  }
};

template <typename T, int N>
struct VecN {
  typedef T type __attribute__((ext_vector_type(N)));
};

// Stages of 64 nodes (32 for more than six slices, to fit LDS); a thread
// stages NPT consecutive nodes of one X row and of one Y column per slice
// with one vector load and one vector LDS store each.  All products of a
// level are accumulated in FP32 over the stage (exact for the integer
// slices, see above) and added once to the level's FP64 accumulator.
template <typename LowT, int S>
__device__ inline void contract_split_body(const SplitArgs& a, int b) {
  typedef typename Vec8<LowT>::type v8;
  constexpr int beta = LowTraits<LowT>::beta;
  constexpr int STG = S <= 6 ? 64 : 32;
  constexpr int NPT = STG / 8;
  constexpr int LDS_ROW = STG + 8;
  typedef typename VecN<LowT, NPT>::type vrun;
  __shared__ __attribute__((aligned(16))) LowT Xl[S][kBM][LDS_ROW];
  __shared__ __attribute__((aligned(16))) LowT Yl[S][kBN][LDS_ROW];
  const int dd = b >= a.d[2].block_begin ? 2 : (b >= a.d[1].block_begin ? 1 : 0);
  const SplitDimArgs& p = a.d[dd];
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
  const LowT* xs = (const LowT*)p.xs;
  const LowT* ys = (const LowT*)p.ys;
  const int sr = tid >> 3;              // row / column within the tile (0..31)
  const int sk = (tid & 7) * NPT;       // first node of the thread's run
  const int xrow = row0 + sr, ycol = col0 + sr;
  const bool xok = xrow < p.M, yok = ycol < p.N;
  const int mu = yok ? ycol / p.S : 0;
  const int ysh = yok ? (ycol - mu * p.S) * p.cn : 0;
  const int64_t xstride = (int64_t)p.M * p.ld, ystride = (int64_t)a.m0 * p.ld;
  const LowT* xbase = xs + (int64_t)xrow * p.ld;
  const LowT* ybase = ys + (int64_t)mu * p.ld;
  vrun xr[S], yr[S];
  auto stage = [&](int k0) {
    const int i0 = k0 + sk;
    // X: rows are padded to a multiple of 8 nodes, runs are aligned
    if (xok && i0 + NPT <= kend) {
#pragma unroll
      for (int q = 0; q < S; ++q) xr[q] = *(const vrun*)(xbase + q * xstride + i0);
    } else {
#pragma unroll
      for (int q = 0; q < S; ++q)
#pragma unroll
        for (int e = 0; e < NPT; ++e)
          xr[q][e] = (xok && i0 + e < kend) ? xbase[q * xstride + i0 + e] : (LowT)0.0f;
    }
    // Y: the cyclic shift may misalign the run or wrap around the torus
    int src0 = i0 - ysh;
    if (src0 < 0) src0 += p.n;
    if (yok && i0 + NPT <= kend && src0 % NPT == 0 && src0 + NPT <= p.n) {
#pragma unroll
      for (int q = 0; q < S; ++q) yr[q] = *(const vrun*)(ybase + q * ystride + src0);
    } else {
#pragma unroll
      for (int e = 0; e < NPT; ++e) {
        int src = src0 + e;
        if (src >= p.n) src -= p.n;
        const bool ok = yok && i0 + e < kend;
#pragma unroll
        for (int q = 0; q < S; ++q) yr[q][e] = ok ? ybase[q * ystride + src] : (LowT)0.0f;
      }
    }
  };
  auto commit = [&]() {
#pragma unroll
    for (int q = 0; q < S; ++q) {
      *(vrun*)&Xl[q][sr][sk] = xr[q];
      *(vrun*)&Yl[q][sr][sk] = yr[q];
    }
  };
  double acc[S][4];
#pragma unroll
  for (int l = 0; l < S; ++l)
#pragma unroll
    for (int r = 0; r < 4; ++r) acc[l][r] = 0.0;
  stage(kbeg);
  commit();
  __syncthreads();
  for (int k0 = kbeg; k0 < kend; k0 += STG) {
    const bool more = k0 + STG < kend;
    if (more) stage(k0 + STG);
    f32x4 c32[S];
#pragma unroll
    for (int l = 0; l < S; ++l) c32[l] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int kstep = 0; kstep < STG / 32; ++kstep) {
      v8 av[S], bv[S];
#pragma unroll
      for (int q = 0; q < S; ++q) {
        av[q] = *(const v8*)&Xl[q][wm * 16 + (lane & 15)][32 * kstep + 8 * (lane >> 4)];
        bv[q] = *(const v8*)&Yl[q][wn * 16 + (lane & 15)][32 * kstep + 8 * (lane >> 4)];
      }
      // level l = qa + qb (0-based slices), l = 0..S-1; consecutive MFMAs
      // feed different levels so that none waits on the previous result
#pragma unroll
      for (int qa = 0; qa < S; ++qa)
#pragma unroll
        for (int qb = 0; qa + qb < S; ++qb)
          c32[qa + qb] = Vec8<LowT>::mfma(av[qa], bv[qb], c32[qa + qb]);
    }
#pragma unroll
    for (int l = 0; l < S; ++l)
#pragma unroll
      for (int r = 0; r < 4; ++r) acc[l][r] += (double)c32[l][r];
    __syncthreads();
    if (more) commit();
    __syncthreads();
  }
  const int col = col0 + wn * 16 + (lane & 15);
  const double ysc = col < p.N ? p.yscale[col / p.S] : 0.0;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    int row = row0 + wm * 16 + 4 * (lane >> 4) + r;
    if (row < p.M && col < p.N) {
      double v = 0.0;
#pragma unroll
      for (int l = S - 1; l >= 0; --l) v += ldexp(acc[l][r], -(l + 2) * beta);
      p.part[((int64_t)z * p.M + row) * p.N + col] = v * p.xscale[row] * ysc;
    }
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
__device__ inline void reduce_partials_body(const ReduceArgs& a, int64_t total, int64_t bx) {
  int64_t idx = bx * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  int d = idx >= a.begin[2] ? 2 : (idx >= a.begin[1] ? 1 : 0);
  int64_t e = idx - a.begin[d];
  const double* p = a.part[d] + e;
  const int64_t st = a.MN[d];
  const int ks = a.ks[d];
  double v = 0.0;
  int s = 0;
  for (; s + 8 <= ks; s += 8) {  // eight loads in flight, summed in chunk order
    double r[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) r[u] = p[(int64_t)(s + u) * st];
#pragma unroll
    for (int u = 0; u < 8; ++u) v += r[u];
  }
  for (; s < ks; ++s) v += p[(int64_t)s * st];
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
__device__ inline void combine_periodic_body(const CombineArgs& a, int64_t total, int64_t bx) {
  // (32-bit index arithmetic: the host keeps block columns below 2^31 entries)
  const int idx = (int)(bx * 4 + (threadIdx.x >> 6));
  const int lane = threadIdx.x & 63;
  if (idx >= total) return;
  const int m2 = a.m0 * a.m0;
  const int kflat = idx / m2;
  const int e = idx - kflat * m2;
  const int mu = e / a.m0, nu = e - mu * a.m0;
  const int k12 = kflat / a.L[2];
  const int k3 = kflat - k12 * a.L[2];
  const int k1 = k12 / a.L[1];
  const int k2 = k12 - k1 * a.L[1];
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
  // the wave is whole here (the early return above is per wave)
  V = wave_sum_dpp(V);
  Tk = readlane_d(Tk, a.T % 64);
  Sk = readlane_d(Sk, (a.T + 1) % 64);
  if (lane == 0) {
    a.H[idx] = Tk - V;
    a.Sm[idx] = Sk;
  }
}

}  // namespace dev
}  // namespace tl
