// Device code of step a6 (Fourier transform of block columns over the lattice
// index), shared by the single-system and the batched launches: the LDS FFT
// of whole lattices, and a direct DFT along one axis for lines longer than a
// workgroup's LDS holds.
#pragma once
#include "common.h"

namespace tl {
namespace dev {

struct DftArgs {
  const double* in;   // real (first pass) or complex input
  double* out;        // complex output
  int len;            // transform length along the axis
  int64_t inner;      // product of the extents after the axis, times m0*m0
  int real_in;
};

constexpr int kMaxTwiddle = 4096;  // lengths up to this keep their twiddles in LDS

// Workgroup per (outer, j) output line segment: the twiddles w^(j k mod L)
// of its j are tabulated once in LDS, threads run over consecutive block
// entries r (coalesced loads along the m0*m0 entries).  Lines of at most 128
// entries leave threads over: the k sum is then split over 2 or 4 groups of
// threads (k = g, g + groups, ...) whose partial sums meet in LDS in group
// order.  Dynamic LDS: max(2 len (TABLE), 2 * 256) doubles, the twiddles
// first, the partials afterwards in the same space.
template <bool REAL_IN, bool TABLE>
__device__ inline void dft_axis_body(const DftArgs& a, int64_t oj, int64_t by, double* tw) {
  // oj = outer * len + j; by = chunk of 256 entries r
  const int j = (int)(oj % a.len);
  const int64_t outer = oj / a.len;
  const int span = a.inner <= 64 ? 64 : (a.inner <= 128 ? 128 : 256);
  const int ng = 256 / span, kg = (int)threadIdx.x / span, rl = (int)threadIdx.x % span;
  const int64_t r = by * span + rl;
  const bool valid = r < a.inner;
  const double inv = 2.0 / (double)a.len;
  if (TABLE) {
    for (int k = threadIdx.x; k < a.len; k += blockDim.x) {
      int p = (int)(((int64_t)j * k) % a.len);
      double s, c;
      sincospi((double)p * inv, &s, &c);  // w^p = cos(2 pi p/L) - i sin(2 pi p/L)
      tw[2 * k] = c;
      tw[2 * k + 1] = s;
    }
    __syncthreads();
  }
  const int64_t base = outer * a.len * a.inner + r;
  double re = 0.0, im = 0.0;
  if (valid) {
    int p = (int)(((int64_t)j * kg) % a.len);
    const int pstep = (int)(((int64_t)j * ng) % a.len);
#pragma unroll 16
    for (int k = kg; k < a.len; k += ng) {
      double s, c;
      if (TABLE) {
        c = tw[2 * k];
        s = tw[2 * k + 1];
      } else {
        sincospi((double)p * inv, &s, &c);
        p += pstep;
        if (p >= a.len) p -= a.len;
      }
      int64_t src = base + (int64_t)k * a.inner;
      if (REAL_IN) {
        double x = a.in[src];
        re += c * x;
        im -= s * x;
      } else {
        double xr = a.in[2 * src], xi = a.in[2 * src + 1];
        re += c * xr + s * xi;
        im += c * xi - s * xr;
      }
    }
  }
  if (ng > 1) {  // uniform: every thread reaches the barriers
    if (TABLE) __syncthreads();  // the twiddle reads are done; the partials reuse the space
    double* part = tw;
    part[2 * threadIdx.x] = re;
    part[2 * threadIdx.x + 1] = im;
    __syncthreads();
    if (kg != 0) return;
    for (int g = 1; g < ng; ++g) {
      re += part[2 * (g * span + rl)];
      im += part[2 * (g * span + rl) + 1];
    }
  }
  if (!valid) return;
  const int64_t o = (outer * a.len + j) * a.inner + r;
  a.out[2 * o] = re;
  a.out[2 * o + 1] = im;
}

// ------------------------------------------------------------------------
// Block FFT in LDS.  A workgroup takes W real columns (entries (b, e) of the
// batch of block columns, W/2 complex lines) over the whole lattice and
// transforms them with every axis pass in LDS, so each input value is read
// once and each output value written once.
//   * Two real columns form one complex line z = x_a 2^-s_a + i x_b 2^-s_b,
//     each scaled by a power of two to unit maximum (exact), so the rounding
//     of each column stays relative to its own size; after the transform
//     X_a(j) = (Z(j) + conj Z(-j))/2, X_b(j) = (Z(j) - conj Z(-j))/(2i).
//   * Each axis of 7-smooth length is done by self-sorting (Stockham)
//     radix-8/4/2/3/5/7 passes: a pass reads all its butterflies' points into
//     registers, the workgroup synchronises, and writes them to their sorted
//     places (in place, one buffer).
//   * A single axis of another length L uses Bluestein's chirp-z form:
//     w_L^(jk) = c(j) c(k) conj c(j-k), c(k) = exp(-i pi k^2/L), a cyclic
//     convolution of length M >= 2L-1 (M 7-smooth) done by two forward FFTs
//     of length M (the inverse as conj FFT conj); the chirp and the transform
//     of the chirp filter are tabulated once per length by a small kernel.
// Twiddles w_n^m = T2[m >> 6] T1[m & 63] from two small LDS tables per axis.
constexpr int kFftPoints = 4096;  // complex points of a workgroup's buffer (64 KB)
constexpr int kFftThreads = 512;  // threads per workgroup (8 waves)
constexpr int kFftMaxPasses = 16;

struct FftAxis {
  int n;       // transform length (lattice extent, or Bluestein length M)
  int S;       // buffer points after this axis (stride of its index)
  int O;       // lines before this axis (product of the earlier extents)
  int npass;
  int tw_off;  // first complex entry of this axis' tables (T1: 64, T2: ceil(n/64))
  unsigned char rad[kFftMaxPasses];
};

struct FftArgs {
  const double* in;  // [cols/E][P][E] real
  double* out;       // [cols/E][P][E] complex (interleaved)
  int64_t E;         // entries of a block (m0*m0)
  int64_t cols;      // real columns: batch * E
  int L[3];          // lattice extents (1 for absent axes)
  int P;             // L[0] L[1] L[2]
  int W;             // real columns per workgroup (2..64, a power of two)
  int naxes;
  FftAxis ax[3];
  int blue;          // 1: one axis of length blue_L by Bluestein, ax[0].n = M
  int blue_L;
  int nbuf;          // buffer points per line: P, or M
  int tw_total;      // complex table entries of all axes
  double2* chirp;    // Bluestein: c(k), k < blue_L (device, written by the tables kernel)
  double2* bhat;     // Bluestein: transform of the chirp filter / M, M entries
};

__host__ __device__ inline size_t fft_tables_lds_bytes(const FftArgs& a) {
  return sizeof(double) * (2 * (size_t)a.ax[0].n + 2 * (64 + ((size_t)a.ax[0].n + 63) / 64));
}
__host__ __device__ inline size_t fft_lds_bytes(const FftArgs& a) {
  return sizeof(double) *
         ((size_t)a.W * a.nbuf + 2 * (size_t)a.tw_total + (kFftThreads / 64 + 1) * (size_t)a.W);
}

__device__ __forceinline__ double2 c_mul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 c_add(double2 a, double2 b) {
  return make_double2(a.x + b.x, a.y + b.y);
}
__device__ __forceinline__ double2 c_sub(double2 a, double2 b) {
  return make_double2(a.x - b.x, a.y - b.y);
}
__device__ __forceinline__ double2 c_mi(double2 a) { return make_double2(a.y, -a.x); }  // -i a

// cos(2 pi m / R), sin(2 pi m / R) for the odd radices, m in [1, (R-1)/2]
__device__ __forceinline__ constexpr double rcos(int R, int m) {
  return R == 3 ? -0.5
       : R == 5 ? (m == 1 ? 0.30901699437494742410 : -0.80901699437494742410)
                : (m == 1 ? 0.62348980185873353053
                          : (m == 2 ? -0.22252093395631440429 : -0.90096886790241912624));
}
__device__ __forceinline__ constexpr double rsin(int R, int m) {
  return R == 3 ? 0.86602540378443864676
       : R == 5 ? (m == 1 ? 0.95105651629515357212 : 0.58778525229247312917)
                : (m == 1 ? 0.78183148246802980871
                          : (m == 2 ? 0.97492791218182360702 : 0.43388373911755812048));
}

__device__ __forceinline__ void dft4(double2& a0, double2& a1, double2& a2, double2& a3) {
  const double2 t0 = c_add(a0, a2), t1 = c_sub(a0, a2);
  const double2 t2 = c_add(a1, a3), t3 = c_mi(c_sub(a1, a3));
  a0 = c_add(t0, t2);
  a1 = c_add(t1, t3);
  a2 = c_sub(t0, t2);
  a3 = c_sub(t1, t3);
}

// forward DFT of R points in place: y_k = sum_t v_t exp(-2 pi i k t / R)
template <int R>
__device__ __forceinline__ void dft_small(double2 (&v)[R]) {
  if constexpr (R == 2) {
    const double2 t = v[0];
    v[0] = c_add(t, v[1]);
    v[1] = c_sub(t, v[1]);
  } else if constexpr (R == 4) {
    dft4(v[0], v[1], v[2], v[3]);
  } else if constexpr (R == 8) {
    double2 e0 = v[0], e1 = v[2], e2 = v[4], e3 = v[6];
    double2 o0 = v[1], o1 = v[3], o2 = v[5], o3 = v[7];
    dft4(e0, e1, e2, e3);
    dft4(o0, o1, o2, o3);
    constexpr double s = 0.70710678118654752440;
    o1 = make_double2(s * (o1.x + o1.y), s * (o1.y - o1.x));    // * exp(-i pi/4)
    o2 = c_mi(o2);                                              // * -i
    o3 = make_double2(s * (o3.y - o3.x), -s * (o3.x + o3.y));   // * exp(-3 i pi/4)
    v[0] = c_add(e0, o0);
    v[4] = c_sub(e0, o0);
    v[1] = c_add(e1, o1);
    v[5] = c_sub(e1, o1);
    v[2] = c_add(e2, o2);
    v[6] = c_sub(e2, o2);
    v[3] = c_add(e3, o3);
    v[7] = c_sub(e3, o3);
  } else {  // odd R: pair t with R - t
    constexpr int h = (R - 1) / 2;
    double2 sp[h], sm[h];
    double2 y0 = v[0];
#pragma unroll
    for (int t = 1; t <= h; ++t) {
      sp[t - 1] = c_add(v[t], v[R - t]);
      sm[t - 1] = c_sub(v[t], v[R - t]);
      y0 = c_add(y0, sp[t - 1]);
    }
    double2 out[R];
    out[0] = y0;
#pragma unroll
    for (int k = 1; k <= h; ++k) {
      double2 A = v[0], B = make_double2(0.0, 0.0);
#pragma unroll
      for (int t = 1; t <= h; ++t) {
        const int m = (k * t) % R;
        const double c = rcos(R, m <= h ? m : R - m);
        const double sn = m <= h ? rsin(R, m) : -rsin(R, R - m);
        A.x += c * sp[t - 1].x;
        A.y += c * sp[t - 1].y;
        B.x += sn * sm[t - 1].x;
        B.y += sn * sm[t - 1].y;
      }
      out[k] = make_double2(A.x + B.y, A.y - B.x);      // A - i B
      out[R - k] = make_double2(A.x - B.y, A.y + B.x);  // A + i B
    }
#pragma unroll
    for (int k = 0; k < R; ++k) v[k] = out[k];
  }
}

__device__ __forceinline__ double2 fft_twiddle(const double2* tab, int n, int m) {
  const double2* t2 = tab + 64;
  return c_mul(t2[m >> 6], tab[m & 63]);
}

// One self-sorting pass of radix R over every line of axis `ax` (Wc complex
// columns interleaved, layout [outer][i][inner][column]).  Ns = product of
// the radices already applied on this axis.
// Elementwise step folded into the first pass of an axis, applied to each
// point (position m on its line, complex column c) as the pass reads it.
struct PassPre {
  int kind;            // 0: none; 1: scale each column to unit maximum;
                       // 2: scale and multiply by the chirp c(m), zero for m >= L;
                       // 3: multiply by the filter's transform, conjugate
  const double* scl;   // [2 Wc] column exponents (kinds 1, 2)
  const double2* tab;  // chirp (kind 2) or the filter's transform (kind 3), global
  int L;               // chirp length (kind 2)
};

template <int R>
__device__ void fft_pass(double2* buf, int Wc, const FftAxis& ax, int Ns, const double2* tab,
                         const PassPre& pre) {
  constexpr int PT = kFftPoints / kFftThreads;  // points per thread (Wc * n * S * O <= kFftPoints)
  constexpr int NB = (PT + R - 1) / R;           // butterflies per thread
  const int n = ax.n, nq = n / R, S = ax.S;
  const int stride = S * Wc;
  const int count = Wc * S * nq * ax.O;
  const int tstep = n / (Ns * R);
  const int lw = __ffs(Wc) - 1;  // Wc is a power of two
  const bool ns_pow2 = (Ns & (Ns - 1)) == 0;
  double2 v[NB][R];
  int dst[NB], tws[NB];
#pragma unroll
  for (int u = 0; u < NB; ++u) {
    const int b = (int)threadIdx.x + kFftThreads * u;
    if (b < count) {
      const int c = b & (Wc - 1);
      int r = b >> lw, ii = 0, j = r, o = 0;
      if (S > 1) {
        ii = r % S;
        r /= S;
        j = r;
      }
      if (ax.O > 1) {
        j = r % nq;
        o = r / nq;
      }
      const int base = (o * n * S + ii) * Wc + c;
#pragma unroll
      for (int t = 0; t < R; ++t) v[u][t] = buf[base + (j + t * nq) * stride];
      const int k = ns_pow2 ? (j & (Ns - 1)) : j % Ns;
      dst[u] = base + ((j - k) * R + k) * stride;
      tws[u] = k * tstep;
      if (pre.kind == 1 || pre.kind == 2) {
        const int ea = -(int)pre.scl[2 * c], eb = -(int)pre.scl[2 * c + 1];
#pragma unroll
        for (int t = 0; t < R; ++t) v[u][t] = make_double2(ldexp(v[u][t].x, ea), ldexp(v[u][t].y, eb));
      }
      if (pre.kind == 2) {
#pragma unroll
        for (int t = 0; t < R; ++t) {
          const int m = j + t * nq;
          v[u][t] = m < pre.L ? c_mul(v[u][t], pre.tab[m]) : make_double2(0.0, 0.0);
        }
      } else if (pre.kind == 3) {
#pragma unroll
        for (int t = 0; t < R; ++t) {
          const double2 z = c_mul(v[u][t], pre.tab[j + t * nq]);
          v[u][t] = make_double2(z.x, -z.y);
        }
      }
    }
  }
  __syncthreads();
#pragma unroll
  for (int u = 0; u < NB; ++u) {
    const int b = (int)threadIdx.x + kFftThreads * u;
    if (b < count) {
      if (Ns > 1) {  // w^(k t n/(Ns R)) = (w^(k n/(Ns R)))^t: one lookup, then powers
        const double2 w1 = fft_twiddle(tab, n, tws[u]);
        double2 wt = w1;
#pragma unroll
        for (int t = 1; t < R; ++t) {
          v[u][t] = c_mul(v[u][t], wt);
          if (t + 1 < R) wt = c_mul(wt, w1);
        }
      }
      dft_small<R>(v[u]);
#pragma unroll
      for (int t = 0; t < R; ++t) buf[dst[u] + t * Ns * stride] = v[u][t];
    }
  }
  __syncthreads();
}

__device__ inline void fft_axis(double2* buf, int Wc, const FftAxis& ax, const double2* tabs,
                                const PassPre& pre) {
  // the radices come sorted (8s, 4s, 2s, 3s, 5s, 7s): one loop per radix;
  // `pre` goes with the first pass only
  const double2* tab = tabs + ax.tw_off;
  const PassPre none{0, nullptr, nullptr, 0};
  int Ns = 1, p = 0;
  for (; p < ax.npass && ax.rad[p] == 8; ++p, Ns *= 8) fft_pass<8>(buf, Wc, ax, Ns, tab, p ? none : pre);
  for (; p < ax.npass && ax.rad[p] == 4; ++p, Ns *= 4) fft_pass<4>(buf, Wc, ax, Ns, tab, p ? none : pre);
  for (; p < ax.npass && ax.rad[p] == 2; ++p, Ns *= 2) fft_pass<2>(buf, Wc, ax, Ns, tab, p ? none : pre);
  for (; p < ax.npass && ax.rad[p] == 3; ++p, Ns *= 3) fft_pass<3>(buf, Wc, ax, Ns, tab, p ? none : pre);
  for (; p < ax.npass && ax.rad[p] == 5; ++p, Ns *= 5) fft_pass<5>(buf, Wc, ax, Ns, tab, p ? none : pre);
  for (; p < ax.npass && ax.rad[p] == 7; ++p, Ns *= 7) fft_pass<7>(buf, Wc, ax, Ns, tab, p ? none : pre);
}

// chirp c(k) = exp(-i pi k^2 / L) from the exact residue k^2 mod 2L
__device__ __forceinline__ double2 chirp(int k, int L) {
  const int r = (int)(((int64_t)k * k) % (2 * (int64_t)L));
  double s, c;
  sincospi((double)r / (double)L, &s, &c);
  return make_double2(c, -s);
}

// lattice point -k (every axis negated modulo its extent)
__device__ __forceinline__ int neg_point(int k, const int* L) {
  if (L[1] == 1 && L[2] == 1) return k ? L[0] - k : 0;
  const int k3 = k % L[2], r = k / L[2];
  const int k2 = r % L[1], k1 = r / L[1];
  const int n1 = k1 ? L[0] - k1 : 0, n2 = k2 ? L[1] - k2 : 0, n3 = k3 ? L[2] - k3 : 0;
  return (n1 * L[1] + n2) * L[2] + n3;
}

// Bluestein tables of one chain length L (one workgroup): the chirp c(k),
// k < L, and the transform of the filter b(m) = conj c(m), b(M - m) = b(m)
// (zero elsewhere), divided by M.  They depend on L only and are read from
// the L2 cache by every workgroup of the transform.
__device__ void fft_blue_tables_body(const FftArgs& a, double* smem) {
  const int tid = (int)threadIdx.x;
  const int M = a.ax[0].n, L = a.blue_L;
  double2* buf = (double2*)smem;
  double2* tabs = (double2*)(smem + 2 * (size_t)M);
  for (int idx = tid; idx < 64 + (M + 63) / 64; idx += kFftThreads) {
    const int e = idx < 64 ? idx % M : (int)(((int64_t)64 * (idx - 64)) % M);
    double s, c;
    sincospi(-2.0 * (double)e / (double)M, &s, &c);
    tabs[idx] = make_double2(c, s);
  }
  for (int m = tid; m < M; m += kFftThreads) {
    double2 v = make_double2(0.0, 0.0);
    if (m < L) v = chirp(m, L);
    else if (M - m < L) v = chirp(M - m, L);
    buf[m] = make_double2(v.x, -v.y);
    if (m < L) a.chirp[m] = v;
  }
  __syncthreads();
  fft_axis(buf, 1, a.ax[0], tabs, PassPre{0, nullptr, nullptr, 0});  // tables start at 0
  const double invM = 1.0 / (double)M;
  for (int m = tid; m < M; m += kFftThreads)
    a.bhat[m] = make_double2(buf[m].x * invM, buf[m].y * invM);
}

// One workgroup: real columns [group*W, group*W + W) of the batch.
template <bool BLUE>
__device__ void fft_block_body(const FftArgs& a, int64_t group, double* smem) {
  const int tid = (int)threadIdx.x;
  const int W = a.W, Wc = W >> 1, P = a.P, nbuf = a.nbuf;
  double2* buf = (double2*)smem;
  double2* tabs = (double2*)(smem + (size_t)W * nbuf);
  constexpr int NW = kFftThreads / 64;
  double* red = smem + (size_t)W * nbuf + 2 * (size_t)a.tw_total;  // [NW][W] wave maxima
  double* scl = red + NW * W;                                      // [W] column exponents
  // load W real columns: every value of the thread in flight at once (rows
  // of W consecutive entries per wave load, W divides the thread count so
  // each thread keeps its column)
  const int64_t q0 = group * W;
  const int nq = (int)(a.cols - q0 < W ? a.cols - q0 : W);
  const int myq = tid % W;
  const bool has = myq < nq;
  const int64_t qg = q0 + myq;
  const int64_t bq = has ? qg / a.E : 0, eq = has ? qg % a.E : 0;
  const double* src = a.in + bq * P * a.E + eq;
  const int k0 = tid / W, kstep = kFftThreads / W;
  constexpr int LPT = 2 * kFftPoints / kFftThreads;  // W * P <= 2 kFftPoints
  double xv[LPT];
#pragma unroll
  for (int u = 0; u < LPT; ++u) {
    const int k = k0 + u * kstep;
    xv[u] = (has && k < P) ? src[(int64_t)k * a.E] : 0.0;
  }
  // twiddle tables of every axis: T1[i] = w^i (i < 64), T2[i] = w^(64 i)
  for (int idx = tid; idx < a.tw_total; idx += kFftThreads) {
    int d = 0;
    while (d + 1 < a.naxes && idx >= a.ax[d + 1].tw_off) ++d;
    const int n = a.ax[d].n, i = idx - a.ax[d].tw_off;
    const int e = i < 64 ? i % n : (int)(((int64_t)64 * (i - 64)) % n);
    double s, c;
    sincospi(-2.0 * (double)e / (double)n, &s, &c);
    tabs[idx] = make_double2(c, s);
  }
  double mx = 0.0;
#pragma unroll
  for (int u = 0; u < LPT; ++u) {
    const int k = k0 + u * kstep;
    if (k < P) smem[(size_t)k * W + myq] = xv[u];
    mx = fmax(mx, fabs(xv[u]));
  }
  for (int off = W; off < 64; off <<= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
  if ((tid & 63) < W) red[(tid >> 6) * W + myq] = mx;
  __syncthreads();
  if (tid < W) {
    double m = red[tid];
    for (int w = 1; w < NW; ++w) m = fmax(m, red[w * W + tid]);
    int ex = 0;
    if (m > 0.0) frexp(m, &ex);
    scl[tid] = (double)ex;
  }
  __syncthreads();
  // the transforms; the column scaling, the chirps and the filter product
  // are folded into the first pass of each transform
  if (BLUE) {
    fft_axis(buf, Wc, a.ax[0], tabs, PassPre{2, scl, a.chirp, a.blue_L});
    fft_axis(buf, Wc, a.ax[0], tabs, PassPre{3, nullptr, a.bhat, 0});
  } else if (a.naxes > 0) {
    fft_axis(buf, Wc, a.ax[0], tabs, PassPre{1, scl, nullptr, 0});
    for (int d = 1; d < a.naxes; ++d) fft_axis(buf, Wc, a.ax[d], tabs, PassPre{0, nullptr, nullptr, 0});
  }
  // split the packed columns, undo the scaling, store rows of W entries
  double* dst = a.out + 2 * (bq * P * a.E + eq);
  const int sh = has ? (int)scl[myq] : 0;
  const int c = myq >> 1;
  if (!has) return;  // no barrier follows
  for (int k = k0; k < P; k += kstep) {
    const int nk = neg_point(k, a.L);
    double2 z = buf[k * Wc + c];
    double2 y = buf[nk * Wc + c];
    if (BLUE) {  // the convolution's inverse transform (conj) and the chirp
      z = c_mul(make_double2(z.x, -z.y), a.chirp[k]);
      y = c_mul(make_double2(y.x, -y.y), a.chirp[nk]);
    } else if (a.naxes == 0) {  // one cell: the scaling still applies
      z = make_double2(ldexp(z.x, -(int)scl[2 * c]), ldexp(z.y, -(int)scl[2 * c + 1]));
      y = z;
    }
    double xr, xi;
    if (myq & 1) {
      xr = 0.5 * (z.y + y.y);
      xi = 0.5 * (y.x - z.x);
    } else {
      xr = 0.5 * (z.x + y.x);
      xi = 0.5 * (z.y - y.y);
    }
    double2* o = (double2*)(dst + 2 * (int64_t)k * a.E);
    *o = make_double2(ldexp(xr, sh), ldexp(xi, sh));
  }
}

}  // namespace dev
}  // namespace tl
