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
// row r of X (and each column of Y) is scaled by a power of two
// sigma_r >= max|row|, and the scaled value is cut into integer slices
//   x / sigma = sum_k d_k 2^(-k beta),  |d_1| <= 2^beta, |d_k| <= 2^(beta-1),
// each exactly representable in bf16 (beta = 8) or fp16 (beta = 9).  The
// slices of one value come from the bits of the integer N = rint(x 2^(beta s)
// / sigma): with a bias of 2^(beta-1) in every lower field, the fields minus
// the bias are the balanced digits d_k (k >= 2) and the top field is d_1.
// Slice products are integers below 2^(2 beta); one 32-node MFMA sums 32 of
// them per pair, so each level a + b stays exact in its FP32 accumulator up
// to level 1 over two MFMA steps (higher levels carry their rounding below
// 2^-52 of the entry), and every 64 nodes the level sums are added to one
// FP64 accumulator with their weights 2^(-beta (a + b + 2)).  Only the
// products with a + b < s are formed (triangular truncation).

constexpr int kMaxSlices = 8;
constexpr int kSplitTile = 64;  // rows and columns of a split workgroup tile
constexpr int kSplitK = 32;     // nodes per MFMA step (16x16x32)
constexpr int kSplitLd = 32;    // halves per LDS slice row (conflict-free for 16-byte reads)

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

// Row maxima of the contraction's source rows as power-of-two exponents
// e with 2^e > max|row| (0 for a zero row): P rows (terms), G, AG and SG rows.
// The G rows (the Y operands, shifted copies of m0 rows) are also sliced
// here, once: gs[d] holds [2][s][m0][ldg] slices, copy 0 at node j (mod n),
// copy 1 one node later, so that every run of 4 nodes starts on a 4-byte
// boundary in one of the copies (ldg >= n + 64, a multiple of 8, the tail
// cyclic).
struct RowMaxArgs {
  const double* src[3][4];  // per dim: P, G, AG, SG
  int* ex[3][4];            // per dim: exponents of the P, G, AG, SG rows
  int rows[3][4];           // per dim: T, m0, m0, m0
  int begin[13];            // workgroup prefix over the 12 (dim, kind) row sets
  int n[3];
  void* gs[3];              // per dim: slices of the G rows (LowT)
  int ldg[3];
  int m0;
};

template <typename LowT, int S>
__device__ inline void slice_one(double x, int e, LowT* dst, int64_t qstride);

template <typename LowT, int S>
__device__ inline void rowmax_body(const RowMaxArgs& a, int b) {
  __shared__ double wmax[4];
  __shared__ int eshared;
  int k = 0;
  while (k < 11 && b >= a.begin[k + 1]) ++k;
  const int d = k >> 2, kind = k & 3;
  const int row = b - a.begin[k];
  const int n = a.n[d];
  const double* src = a.src[d][kind] + (int64_t)row * n;
  double mx = 0.0;
  for (int i = threadIdx.x; i < n; i += blockDim.x) mx = fmax(mx, fabs(src[i]));
  mx = wave_max_dpp(mx);
  if ((threadIdx.x & 63) == 0) wmax[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    mx = fmax(fmax(wmax[0], wmax[1]), fmax(wmax[2], wmax[3]));
    int e = 0;
    if (mx > 0.0) frexp(mx, &e);  // mx = f 2^e, f in [0.5, 1): 2^e > mx
    a.ex[d][kind][row] = e;
    eshared = e;
  }
  if (kind != 1) return;  // uniform per workgroup
  __syncthreads();
  const int e = eshared, ldg = a.ldg[d];
  LowT* gs = (LowT*)a.gs[d];
  const int64_t qstride = (int64_t)a.m0 * ldg;
  for (int j = threadIdx.x; j < ldg; j += blockDim.x) {
    const int n0 = j % n, n1 = (j + n - 1) % n;
    slice_one<LowT, S>(src[n0], e, gs + (int64_t)row * ldg + j, qstride);
    slice_one<LowT, S>(src[n1], e, gs + ((int64_t)S * a.m0 + row) * ldg + j, qstride);
  }
}

struct SplitDimArgs {
  const double* G;
  const double* AG;
  const double* SG;
  const double* P;
  const int* eP;     // exponents of the P, G, AG, SG rows (rowmax_body)
  const int* eG;
  const int* eA;
  const int* eS;
  const void* gs;    // slices of the G rows, [2][s][m0][ldg] (rowmax_body)
  double* part;      // [ks][M][N]
  int n, S, cn, M, N, kchunk, ks, tiles_n, block_begin, ldg;
};
struct SplitArgs {
  SplitDimArgs d[3];
  int m0, T;
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

// Slices of NV values scaled by 2^-e, written as NV-element vectors of slice
// q to dst[q * qstride] (LDS).
template <typename LowT, int S, int NV>
__device__ inline void slice_values(const double (&x)[NV], int e, LowT* dst, int qstride) {
  typedef LowT vN __attribute__((ext_vector_type(NV)));
  constexpr int beta = LowTraits<LowT>::beta;
  constexpr uint64_t half = uint64_t(1) << (beta - 1);
  constexpr uint64_t mask = (uint64_t(1) << beta) - 1;
  // bias 2^(beta-1) in each of the s-1 lower fields
  constexpr uint64_t bias = [] {
    uint64_t b = 0;
    for (int k = 0; k < S - 1; ++k) b |= half << (beta * k);
    return b;
  }();
  vN out[S];
#pragma unroll
  for (int j = 0; j < NV; ++j) {
    const double N = rint(ldexp(x[j], beta * S - e));  // |N| <= 2^(beta s), an integer
    const double hi = floor(N * 0x1p-32);
    const double lo = fma(-hi, 0x1p32, N);               // exact, in [0, 2^32)
    const int64_t Ni = (int64_t)(((uint64_t)(int64_t)(int)hi << 32) | (uint64_t)(uint32_t)lo);
    const uint64_t u = (uint64_t)Ni + bias;
#pragma unroll
    for (int k = 1; k < S; ++k) {  // slice S-k: field k-1 from the bottom
      const int dv = (int)((u >> (beta * (k - 1))) & mask) - (int)half;
      out[S - k][j] = (LowT)(float)dv;
    }
    out[0][j] = (LowT)(float)(int)((int64_t)u >> (beta * (S - 1)));
  }
#pragma unroll
  for (int q = 0; q < S; ++q) *(vN*)(dst + q * qstride) = out[q];
}

// Slices of two values (beta s <= 52): N' = N + bias is exact in FP64 and is
// cut at a digit boundary into hi and lo 32-bit parts; every field is a
// bit-field extract.  fp16 digits come from the bit pattern 0x6400 + field
// (the half 1024 + field) minus 1024 + 2^(beta-1), two at a time in a
// packed half add; bf16 digits from the float 2^23 + field minus 2^23 +
// 2^(beta-1).  The pair is written as one 4-byte word per slice.
template <typename LowT, int S>
__device__ inline void slice_pair(double x0, double x1, int e, LowT* dst, int qstride) {
  constexpr int beta = LowTraits<LowT>::beta;
  static_assert(beta * S <= 52, "slice_pair needs beta s <= 52");
  constexpr int m = S - 1 < 3 ? S - 1 : 3;  // low digits held in lo
  constexpr int half = 1 << (beta - 1);
  constexpr unsigned mask = (1u << beta) - 1;
  constexpr double biasd = [] {
    double b = 0.0, w = 1.0;
    for (int k = 0; k < S - 1; ++k, w *= (double)(1 << beta)) b += (double)half * w;
    return b;
  }();
  constexpr double lo_scale = (double)(1ull << (beta * m));
  const double N0 = rint(ldexp(x0, beta * S - e)) + biasd;
  const double N1 = rint(ldexp(x1, beta * S - e)) + biasd;
  const double h0 = floor(N0 * (1.0 / lo_scale)), h1 = floor(N1 * (1.0 / lo_scale));
  const unsigned l0 = (unsigned)fma(-h0, lo_scale, N0), l1 = (unsigned)fma(-h1, lo_scale, N1);
  const int i0 = (int)h0, i1 = (int)h1;
#pragma unroll
  for (int q = 0; q < S; ++q) {
    const int k = S - 1 - q;  // field from the bottom
    unsigned f0, f1;
    int off;                  // field value minus off = digit
    if (q == 0) {             // top: signed, |d| <= 2^beta
      f0 = (unsigned)((i0 >> (beta * (k - m))) + (1 << beta));
      f1 = (unsigned)((i1 >> (beta * (k - m))) + (1 << beta));
      off = 1 << beta;
    } else if (k < m) {
      f0 = (l0 >> (beta * k)) & mask;
      f1 = (l1 >> (beta * k)) & mask;
      off = half;
    } else {
      f0 = ((unsigned)i0 >> (beta * (k - m))) & mask;
      f1 = ((unsigned)i1 >> (beta * (k - m))) & mask;
      off = half;
    }
    if constexpr (sizeof(LowT) == 2 && LowTraits<LowT>::beta == 9) {  // fp16
      typedef _Float16 h2 __attribute__((ext_vector_type(2)));
      const unsigned bits = (f0 | (f1 << 16)) + 0x64006400u;  // halves 1024 + f
      const h2 v = __builtin_bit_cast(h2, bits);
      const _Float16 c = (_Float16)(-(1024 + off));
      *(h2*)(dst + q * qstride) = v + h2{c, c};
    } else {  // bf16
      typedef __bf16 b2 __attribute__((ext_vector_type(2)));
      const float v0 = __builtin_bit_cast(float, 0x4B000000u | f0) - (float)(8388608 + off);
      const float v1 = __builtin_bit_cast(float, 0x4B000000u | f1) - (float)(8388608 + off);
      *(b2*)(dst + q * qstride) = b2{(__bf16)v0, (__bf16)v1};
    }
  }
}

// One value's s slices, slice q at dst[q * qstride].
template <typename LowT, int S>
__device__ inline void slice_one(double x, int e, LowT* dst, int64_t qstride) {
  constexpr int beta = LowTraits<LowT>::beta;
  constexpr uint64_t half = uint64_t(1) << (beta - 1);
  constexpr uint64_t mask = (uint64_t(1) << beta) - 1;
  constexpr uint64_t bias = [] {
    uint64_t b = 0;
    for (int k = 0; k < S - 1; ++k) b |= half << (beta * k);
    return b;
  }();
  const double N = rint(ldexp(x, beta * S - e));
  const double hi = floor(N * 0x1p-32);
  const double lo = fma(-hi, 0x1p32, N);
  const int64_t Ni = (int64_t)(((uint64_t)(int64_t)(int)hi << 32) | (uint64_t)(uint32_t)lo);
  const uint64_t u = (uint64_t)Ni + bias;
#pragma unroll
  for (int k = 1; k < S; ++k)
    dst[(S - k) * qstride] = (LowT)(float)((int)((u >> (beta * (k - 1))) & mask) - (int)half);
  dst[0] = (LowT)(float)(int)((int64_t)u >> (beta * (S - 1)));
}

// Split contraction from FP64 source rows, 64 x 128 tiles (16 waves, each a
// 32 x 16 quadrant of 2 x 1 MFMA blocks).  Per 32-node step the workgroup
// stages the distinct P and G/AG/SG rows of its X rows in LDS, forms X =
// p_t g_nu and slices it into LDS once (shared by the 8 waves of a row
// half); the Y columns g_mu(. - s a) are copied from the G-row slices of the
// pre-pass (two aligned copies, L2-resident); then the triangular slice
// products run on BF16/FP16 MFMA with FP32 level accumulators.  X slices
// never reach HBM.  Dynamic LDS: X slices s 64 kSplitLd halves, Y slices
// s 128 kSplitLd halves, then the FP64 X sources (the tile's P rows and its
// G, AG, SG rows, at most 32 SPT) at 32 nodes.  beta s must stay below 63
// (the integer N and its bias).
constexpr int kSplitTileN = 128;
constexpr int kSplitThreads = 1024;

template <typename LowT, int S, int SPT>
__device__ inline void contract_split_src_body(const SplitArgs& a, int b) {
  typedef typename Vec8<LowT>::type v8;
  constexpr int beta = LowTraits<LowT>::beta;
  constexpr int TM = kSplitTile, TN = kSplitTileN, LD = kSplitLd;
  extern __shared__ __attribute__((aligned(16))) double smem_d[];
  LowT* Xs = (LowT*)smem_d;           // [S][64][LD]
  LowT* Ys = Xs + S * TM * LD;        // [S][128][LD]
  double* src = (double*)(Ys + S * TN * LD);  // FP64 source rows, [rows][32]
  const int dd = b >= a.d[2].block_begin ? 2 : (b >= a.d[1].block_begin ? 1 : 0);
  const SplitDimArgs& p = a.d[dd];
  const int local = b - p.block_begin;
  const int z = local % p.ks;
  const int rest = local / p.ks;
  const int col0 = (rest % p.tiles_n) * TN;
  const int row0 = (rest / p.tiles_n) * TM;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int wm = wave >> 3, wn = wave & 7;
  const int kbeg = z * p.kchunk, kend = min(p.n, kbeg + p.kchunk);
  const int m0 = a.m0, T = a.T;
  // source rows of the tile: P rows t0..t0+nP-1, then G, AG, SG blocks of m0
  const int r1 = min(p.M, row0 + TM) - 1;
  const int t0 = row0 / m0, t1 = r1 / m0;
  const int nP = t0 < T ? min(t1, T - 1) - t0 + 1 : 0;
  const bool hasG = t0 < T, hasA = t0 <= T && T <= t1, hasS = t0 <= T + 1 && T + 1 <= t1;
  const int offG = nP, offA = offG + (hasG ? m0 : 0), offS = offA + (hasA ? m0 : 0);
  const int nsrc = offS + (hasS ? m0 : 0);
  // this thread slices 2 nodes (k = 2 (tid & 15) ..) of X row tid / 16
  const int xr = tid >> 4, xk = (tid & 15) * 2;
  const int xrow = row0 + xr;
  const bool xok = xrow < p.M;
  int ex = 0, xa = -1, xb = 0;
  if (xok) {
    const int xt = xrow / m0, xnu = xrow - xt * m0;
    if (xt < T) {
      xa = xt - t0;
      xb = offG + xnu;
      ex = p.eP[xt] + p.eG[xnu];
    } else if (xt == T) {
      xb = offA + xnu;
      ex = p.eA[xnu];
    } else {
      xb = offS + xnu;
      ex = p.eS[xnu];
    }
  }
  // and copies 4 nodes (k = 4 (tid & 7) ..) of Y column tid / 8: the
  // pre-sliced G row of mu at nodes k - s cn (mod n), from the copy in which
  // that run starts on a 4-byte boundary
  const int yc = tid >> 3, yk = (tid & 7) * 4;
  const int ycol = col0 + yc;
  const bool yok = ycol < p.N;
  const int ymu = yok ? ycol / p.S : 0;
  const int ysh = yok ? (ycol - ymu * p.S) * p.cn : 0;
  const LowT* gsl = (const LowT*)p.gs;
  const int64_t gq = (int64_t)m0 * p.ldg;
  // staging of the FP64 X sources: rows of 32 nodes, 32 rows per pass
  auto src_row = [&](int r) -> const double* {
    if (r < offG) return p.P + (int64_t)(t0 + r) * p.n;
    if (r < offA) return p.G + (int64_t)(r - offG) * p.n;
    if (r < offS) return p.AG + (int64_t)(r - offA) * p.n;
    return p.SG + (int64_t)(r - offS) * p.n;
  };
  const int skn = tid & 31, srr = tid >> 5;
  // the next step's loads are issued before this step's MFMAs (registers);
  // the sources reach LDS after them, the Y slices after the barrier.  Nodes
  // past the chunk end have X = 0 (zero sources): their Y slices need no mask.
  double sv[SPT];
  uint2 yw[S];
  auto load = [&](int k0) {
    const int kn = k0 + skn;
#pragma unroll
    for (int u = 0; u < SPT; ++u) {
      const int r = srr + 32 * u;
      sv[u] = (r < nsrc && kn < kend) ? src_row(r)[kn] : 0.0;
    }
    int node = k0 + yk - ysh;
    if (node < 0) node += p.n;
    if (node >= p.n) node -= p.n;
    const int cp = node & 1;
    const uint32_t* g32 =
        (const uint32_t*)(gsl + (cp * S * m0 + ymu) * (int64_t)p.ldg) + ((node + cp) >> 1);
#pragma unroll
    for (int q = 0; q < S; ++q) {
      const uint32_t* gq32 = g32 + q * (gq >> 1);
      yw[q] = make_uint2(gq32[0], gq32[1]);
    }
  };
  auto store_src = [&]() {  // src is read by slice_step only: may overlap the MFMAs
#pragma unroll
    for (int u = 0; u < SPT; ++u) {
      const int r = srr + 32 * u;
      if (r < nsrc) src[r * kSplitK + skn] = sv[u];
    }
  };
  auto slice_step = [&]() {  // writes Xs and Ys: after the barrier that ends the MFMAs
#pragma unroll
    for (int q = 0; q < S; ++q) *(uint2*)(Ys + (q * TN + yc) * LD + yk) = yw[q];
    double xv[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const double g = src[xb * kSplitK + xk + j];
      xv[j] = xok ? (xa >= 0 ? src[xa * kSplitK + xk + j] * g : g) : 0.0;
    }
    if constexpr (LowTraits<LowT>::beta * S <= 52)
      slice_pair<LowT, S>(xv[0], xv[1], ex, Xs + xr * LD + xk, TM * LD);
    else
      slice_values<LowT, S, 2>(xv, ex, Xs + xr * LD + xk, TM * LD);
  };
  f32x4 c32[2][S];
  f64x4 acc[2];
#pragma unroll
  for (int rb = 0; rb < 2; ++rb) {
    acc[rb] = f64x4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int l = 0; l < S; ++l) c32[rb][l] = f32x4{0.f, 0.f, 0.f, 0.f};
  }
  auto flush = [&]() {
#pragma unroll
    for (int rb = 0; rb < 2; ++rb)
#pragma unroll
      for (int l = S - 1; l >= 0; --l) {
#pragma unroll
        for (int r = 0; r < 4; ++r)
          acc[rb][r] = fma((double)c32[rb][l][r], ldexp(1.0, -beta * (l + 2)), acc[rb][r]);
        c32[rb][l] = f32x4{0.f, 0.f, 0.f, 0.f};
      }
  };
  load(kbeg);
  store_src();
  __syncthreads();
  slice_step();
  __syncthreads();
  int step = 0;
  for (int k0 = kbeg; k0 < kend; k0 += kSplitK, ++step) {
    const bool more = k0 + kSplitK < kend;
    if (more) load(k0 + kSplitK);  // in flight during the MFMAs
    {
      v8 bv[S];
#pragma unroll
      for (int q = 0; q < S; ++q)
        bv[q] = *(const v8*)(Ys + (q * TN + wn * 16 + (lane & 15)) * LD + 8 * (lane >> 4));
#pragma unroll
      for (int rb = 0; rb < 2; ++rb) {
        v8 av[S];
#pragma unroll
        for (int q = 0; q < S; ++q)
          av[q] = *(const v8*)(Xs + (q * TM + wm * 32 + rb * 16 + (lane & 15)) * LD +
                               8 * (lane >> 4));
        // level l = qa + qb; consecutive MFMAs feed different accumulators
#pragma unroll
        for (int qa = 0; qa < S; ++qa)
#pragma unroll
          for (int qb = 0; qa + qb < S; ++qb)
            c32[rb][qa + qb] = Vec8<LowT>::mfma(av[qa], bv[qb], c32[rb][qa + qb]);
      }
    }
    if ((step & 1) || !more) flush();
    if (more) store_src();
    __syncthreads();  // every wave is done with this step's slices
    if (more) {
      slice_step();
      __syncthreads();
    }
  }
  // f32 16x16x32 result layout: register r of lane l holds D[4 (l / 16) + r][l % 16]
  const int col = col0 + wn * 16 + (lane & 15);
  if (col >= p.N) return;
  const int ecol = p.eG[col / p.S];
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int row = row0 + wm * 32 + rb * 16 + 4 * (lane >> 4) + r;
      if (row >= p.M) continue;
      const int t = row / m0, nu = row - t * m0;
      const int erow = t < T ? p.eP[t] + p.eG[nu] : (t == T ? p.eA[nu] : p.eS[nu]);
      p.part[((int64_t)z * p.M + row) * p.N + col] = ldexp(acc[rb][r], erow + ecol);
    }
}

__host__ __device__ inline size_t split_lds_bytes(int s, int nsrc_max) {
  return sizeof(_Float16) * (size_t)s * (kSplitTile + kSplitTileN) * kSplitLd +
         sizeof(double) * (size_t)nsrc_max * kSplitK;
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

// The same combination with a workgroup per (mu, nu) pair and chunk of 256
// block cells: the factors of dims 1 and 2 for every term and shift staged
// once in LDS, a thread per cell d = (d1, d2, d3) summing the products over
// the terms in order (the dim-0 factor is one value per d1, read from the
// compact C_0).  Needs (T+2)(L2 + L3) <= kPairLdsMax.
constexpr int kPairLdsMax = 6144;  // doubles

__host__ __device__ inline bool combine_pair_fits(int T, const int L[3]) {
  return (int64_t)(T + 2) * (L[1] + L[2]) <= kPairLdsMax;
}

__device__ inline void combine_pair_body(const CombineArgs& a, int pair, int chunk) {
  __shared__ double F[kPairLdsMax];
  const int m0 = a.m0, T = a.T, TT = T + 2;
  const int mu = pair / m0, nu = pair - mu * m0;
  const int L1 = a.L[1], L2 = a.L[2];
  double* F1 = F;                  // [T+2][L1]
  double* F2 = F + TT * L1;        // [T+2][L2]
  for (int e = threadIdx.x; e < TT * (L1 + L2); e += blockDim.x) {
    if (e < TT * L1) {
      const int t = e / L1, k = e - t * L1;
      F1[e] = lookup(a, 1, t, mu, nu, k);
    } else {
      const int f = e - TT * L1, t = f / L2, k = f - t * L2;
      F2[f] = lookup(a, 2, t, mu, nu, k);
    }
  }
  __syncthreads();
  const int cells = a.L[0] * L1 * L2;
  const int d = chunk * blockDim.x + threadIdx.x;
  if (d >= cells) return;
  const int d12 = d / L2, d3 = d - d12 * L2;
  const int d1 = d12 / L1, d2 = d12 - d1 * L1;
  double V = 0.0;
  for (int t = 0; t < T; ++t)
    V = fma(lookup(a, 0, t, mu, nu, d1) * F1[t * L1 + d2], F2[t * L2 + d3], V);
  const double D1 = lookup(a, 0, T, mu, nu, d1), M1 = lookup(a, 0, T + 1, mu, nu, d1);
  const double D2 = F1[T * L1 + d2], M2 = F1[(T + 1) * L1 + d2];
  const double D3 = F2[T * L2 + d3], M3 = F2[(T + 1) * L2 + d3];
  const double Tk = 0.5 * (D1 * M2 * M3 + M1 * D2 * M3 + M1 * M2 * D3);
  const int64_t o = (int64_t)d * m0 * m0 + pair;
  a.H[o] = Tk - V;
  a.Sm[o] = M1 * M2 * M3;
}

}  // namespace dev
}  // namespace tl
