// Device code of step a7 (batched generalized Hermitian eigensolver of the
// k-block pencils), shared by the single-system and the batched launches.
#pragma once
#include <cfloat>

#include "common.h"
#include "dev_wave.h"

namespace tl {
namespace dev {

struct cx {
  double re, im;
};
__device__ inline cx cmul(cx a, cx b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ inline cx cconj(cx a) { return {a.re, -a.im}; }
__device__ inline cx cadd(cx a, cx b) { return {a.re + b.re, a.im + b.im}; }
__device__ inline cx csub(cx a, cx b) { return {a.re - b.re, a.im - b.im}; }
__device__ inline cx cscale(cx a, double s) { return {a.re * s, a.im * s}; }
__device__ inline double cabs2(cx a) { return a.re * a.re + a.im * a.im; }

constexpr int kMaxSweeps = 60;

// Partner of index x in round r of the round-robin ordering of `me` (even)
// indices: me-1 meets r, every other pair {r+k, r-k} (mod me-1).
__device__ __forceinline__ int rr_partner(int x, int r, int me) {
  const int n1 = me - 1;
  if (x == n1) return r;
  if (x == r) return n1;
  int y = (2 * r - x) % n1;
  return y < 0 ? y + n1 : y;
}

// Jacobi rotation zeroing A[p][q] of the Hermitian 2x2 [[a, b], [conj b, d]]
// (Golub & Van Loan, sym.schur2, after removing the phase of b):
// J = D R, D = diag(1, exp(-i phi)), R = [[c, s], [-s, c]], so
// J[p][p] = c, J[q][p] = -s e^{-i phi}, J[p][q] = s, J[q][q] = c e^{-i phi};
// the diagonal becomes a - t|b|, d + t|b|.  b = 0 (or a padding index q)
// gives the identity.
struct Rot {
  double c, s, tb, ph_re, ph_im;
};

__device__ __forceinline__ Rot make_rot(double a, double d, cx b, bool valid) {
  Rot r = {1.0, 0.0, 0.0, 1.0, 0.0};
  double b2 = cabs2(b);
  if (!valid || !(b2 > 0.0)) return r;
  double inv_ab = rsqrt(b2);
  double tau = 0.5 * (d - a) * inv_ab;
  double at = fabs(tau);
  double t = at > 1e150 ? 0.5 / tau : copysign(1.0 / (at + sqrt(fma(tau, tau, 1.0))), tau);
  r.c = rsqrt(fma(t, t, 1.0));
  r.s = t * r.c;
  r.tb = t * (b2 * inv_ab);
  r.ph_re = b.re * inv_ab;
  r.ph_im = -b.im * inv_ab;
  return r;
}

// Reciprocal and reciprocal square root from the hardware estimates
// (v_rcp_f64, v_rsq_f64) refined by two Newton steps each; the quadratic
// convergence of Newton's iteration takes the estimate to full FP64 accuracy
// (not necessarily correctly rounded).  Arguments must be normal and finite.
__device__ __forceinline__ double nrcp(double x) {
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}
__device__ __forceinline__ double nrsq(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double h = 0.5 * x;
  y = y * fma(-h * y, y, 1.5);
  return y * fma(-h * y, y, 1.5);
}

// The rotation of make_rot with the long-latency operations replaced by the
// refined estimates: sqrt(u) = u rsq(u).  |b|^2 below 1e-290 counts as 0.
__device__ __forceinline__ Rot make_rot_fast(double a, double d, cx b, bool valid) {
  Rot r = {1.0, 0.0, 0.0, 1.0, 0.0};
  const double b2 = cabs2(b);
  if (!valid || !(b2 > 1e-290)) return r;
  const double inv_ab = nrsq(b2);
  const double tau = 0.5 * (d - a) * inv_ab;
  const double at = fabs(tau);
  double t;
  if (at > 1e150) {
    t = 0.5 / tau;
  } else {
    const double u = fma(tau, tau, 1.0);
    t = copysign(nrcp(at + u * nrsq(u)), tau);
  }
  r.c = nrsq(fma(t, t, 1.0));
  r.s = t * r.c;
  r.tb = t * (b2 * inv_ab);
  r.ph_re = b.re * inv_ab;
  r.ph_im = -b.im * inv_ab;
  return r;
}

// Sturm counts at two points x0, x1 of the symmetric tridiagonal with
// diagonal d[0..m-1] and squared off-diagonal e2[0..m-2], entries scaled into
// (-1, 1): the number of eigenvalues below x is the number of sign changes in
// the leading principal minors p_0 = 1, p_k = det(T_k - x I), which obey
// p_k = (d_{k-1} - x) p_{k-1} - e2_{k-2} p_{k-2}.  Rounding in this recurrence
// amounts to relative perturbations of d - x and e2 of a few ulps, as in the
// ratio form q_k = p_k / p_{k-1}, but the dependent chain is one FMA per step.
// An exact zero p_k takes the sign opposite to p_{k-1} (a tiny negative pivot
// in the ratio form).
__device__ __forceinline__ void sturm_count2(const double (&d)[8], const double (&e2)[8], int m,
                                             double x0, double x1, int& c0, int& c1) {
  constexpr double kTiny = 0x1p-500;
  double p0 = d[0] - x0, p1 = d[0] - x1, r0 = 1.0, r1 = 1.0;
  if (p0 == 0.0) p0 = -kTiny;
  if (p1 == 0.0) p1 = -kTiny;
  c0 = p0 < 0.0;
  c1 = p1 < 0.0;
#pragma unroll
  for (int u = 1; u < 8; ++u) {
    if (u >= m) break;
    double n0 = fma(d[u] - x0, p0, -e2[u - 1] * r0);
    double n1 = fma(d[u] - x1, p1, -e2[u - 1] * r1);
    if (n0 == 0.0) n0 = -copysign(kTiny, p0);
    if (n1 == 0.0) n1 = -copysign(kTiny, p1);
    c0 += (n0 < 0.0) != (p0 < 0.0);
    c1 += (n1 < 0.0) != (p1 < 0.0);
    r0 = p0;
    r1 = p1;
    p0 = n0;
    p1 = n1;
  }
}

// The same counts without the zero fix-up on the dependent chain (one FMA per
// step); `zero` reports whether some minor came out exactly zero, in which
// case the counts may be wrong and the caller recounts with sturm_count2.
__device__ __forceinline__ void sturm_count2_fast(const double (&d)[8], const double (&e2)[8], int m,
                                                  double x0, double x1, int& c0, int& c1,
                                                  bool& zero) {
  double p0 = d[0] - x0, p1 = d[0] - x1, r0 = 1.0, r1 = 1.0;
  bool z = p0 == 0.0 || p1 == 0.0;
  c0 = signbit(p0);
  c1 = signbit(p1);
#pragma unroll
  for (int u = 1; u < 8; ++u) {
    if (u >= m) break;
    const double n0 = fma(d[u] - x0, p0, -e2[u - 1] * r0);
    const double n1 = fma(d[u] - x1, p1, -e2[u - 1] * r1);
    z = z || n0 == 0.0 || n1 == 0.0;
    c0 += signbit(n0) != signbit(p0);
    c1 += signbit(n1) != signbit(p1);
    r0 = p0;
    r1 = p1;
    p0 = n0;
    p1 = n1;
  }
  zero = z;
}

// The counts of sturm_count2 / sturm_count2_fast over a fixed 16 steps: the
// caller pads the tridiagonal past m with d = 2 and e2 = 0, which adds no
// sign change for any x below 2 (the scaled spectrum lies in (-1, 1)), so the
// loops need no exit test and unroll completely.
__device__ __forceinline__ void sturm_count16(const double (&d)[16], const double (&e2)[16],
                                              double x0, double x1, int& c0, int& c1) {
  constexpr double kTiny = 0x1p-500;
  double p0 = d[0] - x0, p1 = d[0] - x1, r0 = 1.0, r1 = 1.0;
  if (p0 == 0.0) p0 = -kTiny;
  if (p1 == 0.0) p1 = -kTiny;
  c0 = p0 < 0.0;
  c1 = p1 < 0.0;
#pragma unroll
  for (int u = 1; u < 16; ++u) {
    double n0 = fma(d[u] - x0, p0, -e2[u - 1] * r0);
    double n1 = fma(d[u] - x1, p1, -e2[u - 1] * r1);
    if (n0 == 0.0) n0 = -copysign(kTiny, p0);
    if (n1 == 0.0) n1 = -copysign(kTiny, p1);
    c0 += (n0 < 0.0) != (p0 < 0.0);
    c1 += (n1 < 0.0) != (p1 < 0.0);
    r0 = p0;
    r1 = p1;
    p0 = n0;
    p1 = n1;
  }
}

__device__ __forceinline__ void sturm_count16_fast(const double (&d)[16], const double (&e2)[16],
                                                   double x0, double x1, int& c0, int& c1,
                                                   bool& zero) {
  double p0 = d[0] - x0, p1 = d[0] - x1, r0 = 1.0, r1 = 1.0;
  bool z = p0 == 0.0 || p1 == 0.0;
  c0 = signbit(p0);
  c1 = signbit(p1);
#pragma unroll
  for (int u = 1; u < 16; ++u) {
    const double n0 = fma(d[u] - x0, p0, -e2[u - 1] * r0);
    const double n1 = fma(d[u] - x1, p1, -e2[u - 1] * r1);
    z = z || n0 == 0.0 || n1 == 0.0;
    c0 += signbit(n0) != signbit(p0);
    c1 += signbit(n1) != signbit(p1);
    r0 = p0;
    r1 = p1;
    p0 = n0;
    p1 = n1;
  }
  zero = z;
}

// ---------------------------------------------------------------- m0 <= 8
// One wave per k-block, lane 8 i + j holding entry (i, j) of every 8 x 8
// (padded) matrix in registers: S, its Cholesky factor L, X = L^-1, C, V.
// All exchanges are cross-lane reads, so no step needs a barrier.  Padded
// indices carry S = I, H = 0 and never rotate.  Same stages and the same
// rotation formulas as the LDS version below.
__device__ inline cx shfl_cx(cx v, int src) { return {__shfl(v.re, src), __shfl(v.im, src)}; }

//
// Eigenvalues only (evecs == nullptr): with wave < 0 the wave bisects all m
// eigenvalues together (8 lanes and 16 points per eigenvalue and round); with
// wave >= 0 it bisects eigenvalues wave, wave + nwave, ... one after the other
// with all 64 lanes (128 points per round, about 7 bits), for launches that
// give every block several waves.  The two schedules agree to the bisection
// tolerance, not bit for bit.
__device__ __forceinline__ void heigh_wave8_body(const double* __restrict__ H,
                                        const double* __restrict__ S, int m,
                                        double* __restrict__ evals, double* __restrict__ evecs,
                                        int* __restrict__ info, int64_t blk, int wave = -1,
                                        int nwave = 1) {
  const int lane = threadIdx.x & 63, i = lane >> 3, j = lane & 7;
  const bool in = i < m && j < m;
  const int mm = m * m;
  const cx* Hb = (const cx*)H + blk * mm;
  const cx* Sb = S ? (const cx*)S + blk * mm : nullptr;
  const cx h = in ? Hb[i * m + j] : cx{0.0, 0.0};
  cx s = (in && Sb) ? Sb[i * m + j] : cx{i == j ? 1.0 : 0.0, 0.0};
  // 1. Cholesky S = L L^H, lane (i, j <= i) ends with L[i][j]
  // (1 / L[k][k] and L[i][k] stay in registers for the forward elimination)
  int fail = 0;
  double linv[8];
  cx lcol[8];
  if (Sb) {
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      if (k >= m) break;
      const double d = readlane_d(s.re, 9 * k);
      // pivots at or below 1e-300 (and non-finite ones) count as not positive
      if (!(d > 1e-300) || !isfinite(d)) {
        fail = k + 1;
        break;
      }
      const double inv = nrsq(d), lkk = d * inv;
      if (j == k) s = i == k ? cx{lkk, 0.0} : (i > k ? cscale(s, inv) : s);
      const cx lik = shfl_cx(s, 8 * i + k), ljk = shfl_cx(s, 8 * j + k);
      if (j > k && i >= j) s = csub(s, cmul(lik, cconj(ljk)));
      linv[k] = inv;
      lcol[k] = lik;
    }
    if (j > i) s = {0.0, 0.0};
  }
  if (fail) {
    if (wave > 0) return;
    if (j == 0 && i < m) evals[blk * m + i] = NAN;
    if (evecs && in) ((cx*)evecs)[blk * mm + i * m + j] = {0.0, 0.0};
    if (lane == 0) info[blk] = fail;
    return;
  }
  // 2. X = L^-1 by forward elimination on the identity, C = X H X^H
  cx x = {i == j ? 1.0 : 0.0, 0.0};
  cx c = h;
  if (Sb) {
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      if (r >= m) break;
      if (i == r) x = cscale(x, linv[r]);
      const cx xrj = shfl_cx(x, 8 * r + j);
      if (i > r) x = csub(x, cmul(lcol[r], xrj));
    }
    cx w = {0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 8; ++k) w = cadd(w, cmul(shfl_cx(x, 8 * i + k), shfl_cx(h, 8 * k + j)));
    c = {0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 8; ++k)
      c = cadd(c, cmul(shfl_cx(w, 8 * i + k), cconj(shfl_cx(x, 8 * j + k))));
  }
  {
    const cx ct = shfl_cx(c, 8 * j + i);  // Hermitian average
    c = i == j ? cx{c.re, 0.0} : cscale(cadd(c, cconj(ct)), 0.5);
  }
  if (evecs == nullptr) {
    // eigenvalues only: Householder reduction of C to a real tridiagonal
    // (LAPACK zhetd2 convention: x = C[k+1:, k], beta = -sign(Re alpha)
    // sqrt(|alpha|^2 + |x'|^2), tau = ((beta - Re alpha) - i Im alpha) / beta,
    // v = (1, x' / (alpha - beta)); w = tau C v, w -= 1/2 tau (w^H v) v,
    // C -= v w^H + w v^H), then Sturm bisection on (d, e^2).
    double e2[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      if (k > m - 3) break;  // uniform
      const cx xi = shfl_cx(c, 8 * i + k), xj = shfl_cx(c, 8 * j + k);
      const cx alpha = shfl_cx(c, 8 * (k + 1) + k);
      // |x'|^2 = sum over rows j >= k + 2 of |C[j][k]|^2: every group of 8
      // lanes holds column k in xj, so a group sum gives it to all lanes
      const double sq = group8_sum(j >= k + 2 ? cabs2(xj) : 0.0);
      if (sq == 0.0 && alpha.im == 0.0) {
        e2[k] = alpha.re * alpha.re;  // already reduced: H = I
        continue;
      }
      // |beta| and 1 / |beta| from one refined reciprocal square root
      const double s2 = alpha.re * alpha.re + alpha.im * alpha.im + sq;
      const double rs = nrsq(s2);
      const double beta = -copysign(s2 * rs, alpha.re), rbeta = -copysign(rs, alpha.re);
      const cx tau = {(beta - alpha.re) * rbeta, -alpha.im * rbeta};
      const cx den = {alpha.re - beta, alpha.im};
      const double dd = nrcp(cabs2(den));
      const cx rden = {den.re * dd, -den.im * dd};  // 1 / (alpha - beta)
      const cx vi = i == k + 1 ? cx{1.0, 0.0} : (i > k + 1 ? cmul(xi, rden) : cx{0.0, 0.0});
      const cx vj = j == k + 1 ? cx{1.0, 0.0} : (j > k + 1 ? cmul(xj, rden) : cx{0.0, 0.0});
      // w_i = tau sum_j C[i][j] v_j over the trailing block (row groups of 8 lanes)
      cx t = (i > k && j > k) ? cmul(c, vj) : cx{0.0, 0.0};
      t.re = group8_sum(t.re);
      t.im = group8_sum(t.im);
      cx wi = cmul(tau, t);
      cx wj = shfl_cx(wi, 8 * j);
      // K = -1/2 tau (w^H v), summed over j within every group of 8 lanes
      cx kk = j > k ? cmul(cconj(wj), vj) : cx{0.0, 0.0};
      kk.re = group8_sum(kk.re);
      kk.im = group8_sum(kk.im);
      const cx K = cscale(cmul(tau, kk), -0.5);
      wi = cadd(wi, cmul(K, vi));
      wj = cadd(wj, cmul(K, vj));
      if (i > k && j > k) c = csub(c, cadd(cmul(vi, cconj(wj)), cmul(wi, cconj(vj))));
      e2[k] = beta * beta;
    }
    // the last off-diagonal element needs no reflector
    double d8[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) d8[q] = readlane_d(c.re, 9 * q);
    if (m >= 2) {
      const cx last = shfl_cx(c, 8 * (m - 1) + (m - 2));
#pragma unroll
      for (int q = 0; q < 8; ++q)
        if (q == m - 2) e2[q] = cabs2(last);
    }
    // Gershgorin interval, then an exact power-of-two scaling that puts the
    // spectrum inside (-1, 1) (the leading minors below then stay far from
    // overflow and underflow for m <= 8)
    double lo = 1e308, hi = -1e308;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      if (q >= m) break;
      const double el = q > 0 ? sqrt(e2[q - 1]) : 0.0, er = q < m - 1 ? sqrt(e2[q]) : 0.0;
      lo = fmin(lo, d8[q] - el - er);
      hi = fmax(hi, d8[q] + el + er);
    }
    const double tn = fmax(fabs(lo), fabs(hi));
    int ex = 0;
    if (tn > 0.0 && isfinite(tn)) frexp(tn, &ex);
    ex += 1;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      d8[q] = ldexp(d8[q], -ex);
      e2[q] = ldexp(e2[q], -2 * ex);
    }
    const double fudge = 2.1 * DBL_EPSILON * m * ldexp(tn, -ex);
    lo = ldexp(lo, -ex) - fudge;
    hi = ldexp(hi, -ex) + fudge;
    // stop at an interval of 2 ulp of the scaled norm (absolute) or of the
    // eigenvalue (relative), whichever is larger
    const double atol = 2.0 * DBL_EPSILON * ldexp(tn, -ex);
    if (wave >= 0) {
      // one eigenvalue at a time; lane l counts at the interior points
      // 2l + 1 and 2l + 2 of 129 equal parts, and the new bracket is read
      // from the lanes that hold its ends (the counts rise with x)
      const double f0 = (double)(2 * lane + 1) / 129.0, f1 = (double)(2 * lane + 2) / 129.0;
      for (int idx = wave; idx < m; idx += nwave) {
        double a = lo, b = hi;
        for (int round = 0; round < 24; ++round) {
          if (b - a <= fmax(atol, 2.0 * DBL_EPSILON * fmax(fabs(a), fabs(b)))) break;  // uniform
          const double x0 = a + (b - a) * f0, x1 = a + (b - a) * f1;
          int c0, c1;
          bool zero;
          sturm_count2_fast(d8, e2, m, x0, x1, c0, c1, zero);
          if (__any(zero)) sturm_count2(d8, e2, m, x0, x1, c0, c1);  // rare
          const int K = __popcll(__ballot(c0 <= idx)) + __popcll(__ballot(c1 <= idx));
          const double na = K > 0 ? readlane_d(((K - 1) & 1) ? x1 : x0, (K - 1) >> 1) : a;
          const double nb = K < 128 ? readlane_d((K & 1) ? x1 : x0, K >> 1) : b;
          a = na;
          b = fmax(nb, na);
        }
        if (lane == 0) evals[blk * m + idx] = ldexp(0.5 * (a + b), ex);
      }
      if (wave == 0 && lane == 0) info[blk] = 0;
      return;
    }
    // eigenvalue idx = lane / 8; each lane counts at two points, so a round
    // splits the bracket at sixteen interior points per eigenvalue
    const int idx = lane >> 3, pt = lane & 7;
    const double f0 = (double)(2 * pt + 1) / 17.0, f1 = (double)(2 * pt + 2) / 17.0;
    for (int round = 0; round < 40; ++round) {
      const bool done = hi - lo <= fmax(atol, 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)));
      if (__all(done || idx >= m)) break;
      const double x0 = lo + (hi - lo) * f0, x1 = lo + (hi - lo) * f1;
      int c0, c1;
      bool zero;
      sturm_count2_fast(d8, e2, m, x0, x1, c0, c1, zero);
      if (__any(zero)) sturm_count2(d8, e2, m, x0, x1, c0, c1);  // rare
      // x0 < x1 and counts are monotone: the pair brackets idx locally
      double nlo = c1 <= idx ? x1 : (c0 <= idx ? x0 : lo);
      double nhi = c0 > idx ? x0 : (c1 > idx ? x1 : hi);
      nlo = group8_max(nlo);
      nhi = group8_min(nhi);
      if (!done) {
        lo = nlo;
        hi = fmax(nhi, nlo);
      }
    }
    if (pt == 0 && idx < m) evals[blk * m + idx] = ldexp(0.5 * (lo + hi), ex);
    if (lane == 0) info[blk] = 0;
    return;
  }
  // 3. cyclic Jacobi, round-robin pairs of the even-padded index set; C and
  // V are published once per round through LDS (one wave: the barriers only
  // order the LDS accesses)
  __shared__ cx sc[64], sv[64];
  cx v = {i == j ? 1.0 : 0.0, 0.0};
  const int me = m + (m & 1);
  int converged = (m == 1);
  for (int sweep = 0; sweep < kMaxSweeps && !converged; ++sweep) {
    double off = 0.0, all = 0.0;
    if (in) {
      all = cabs2(c);
      off = i != j ? all : 0.0;
    }
    off = wave_sum_dpp(off);
    all = wave_sum_dpp(all);
    if (off <= 1e-32 * all) {
      converged = 1;
      break;
    }
    for (int r = 0; r < me - 1; ++r) {
      const int ip = i < me ? rr_partner(i, r, me) : i;
      const int jp = j < me ? rr_partner(j, r, me) : j;
      const int pi = min(i, ip), qi = max(i, ip), pj = min(j, jp), qj = max(j, jp);
      __syncthreads();  // the previous round's reads are done
      sc[lane] = c;
      sv[lane] = v;
      __syncthreads();
      const Rot ri = make_rot_fast(sc[9 * pi].re, sc[9 * qi].re, sc[8 * pi + qi],
                                   qi < m && qi != pi);
      const Rot rj = make_rot_fast(sc[9 * pj].re, sc[9 * qj].re, sc[8 * pj + qj],
                                   qj < m && qj != pj);
      const cx c_ijp = sc[8 * i + jp], c_ipj = sc[8 * ip + j];
      const cx c_ipjp = sc[8 * ip + jp], v_ijp = sv[8 * i + jp];
      // column i of J: J[i][i] and J[ip][i]; column j likewise
      const bool fi = i < ip, fj = j < jp;
      const cx Jii = fi ? cx{ri.c, 0.0} : cx{ri.ph_re * ri.c, ri.ph_im * ri.c};
      const cx Jpi = fi ? cx{-ri.ph_re * ri.s, -ri.ph_im * ri.s} : cx{ri.s, 0.0};
      const cx Jjj = fj ? cx{rj.c, 0.0} : cx{rj.ph_re * rj.c, rj.ph_im * rj.c};
      const cx Jpj = fj ? cx{-rj.ph_re * rj.s, -rj.ph_im * rj.s} : cx{rj.s, 0.0};
      cx na;
      if (j == i) {
        na = {c.re + (fi ? -ri.tb : ri.tb), 0.0};
      } else if (j == ip) {
        na = {0.0, 0.0};
      } else {
        const cx t0 = cadd(cmul(c, Jjj), cmul(c_ijp, Jpj));
        const cx t1 = cadd(cmul(c_ipj, Jjj), cmul(c_ipjp, Jpj));
        na = cadd(cmul(cconj(Jii), t0), cmul(cconj(Jpi), t1));
      }
      v = cadd(cmul(v, Jjj), cmul(v_ijp, Jpj));
      c = na;
    }
  }
  // 4. eigenvalues ascending (ties by index), u = L^-H v = X^H v
  const double li = __shfl(c.re, 9 * i), lj = __shfl(c.re, 9 * j);
  const bool before = j < m && (lj < li || (lj == li && j < i));
  const uint64_t mask = __ballot(before);
  const int rank_i = __popcll((mask >> (8 * i)) & 0xFFull);
  if (i == j && i < m) evals[blk * m + rank_i] = c.re;
  if (lane == 0) info[blk] = converged ? 0 : -1;
  if (evecs) {
    cx u = v;
    if (Sb) {
      u = {0.0, 0.0};
#pragma unroll
      for (int k = 0; k < 8; ++k)
        u = cadd(u, cmul(cconj(shfl_cx(x, 8 * k + i)), shfl_cx(v, 8 * k + j)));
    }
    const int rank_j = __shfl(rank_i, 8 * j);
    if (in) ((cx*)evecs)[blk * mm + i * m + rank_j] = u;
  }
}

// ---------------------------------------------------------------- 8 < m0 <= 16
// Eigenvalues only, one 256-thread workgroup per block: thread 16 i + j holds
// entry (i, j) of the 16 x 16 (padded) matrices, so a row is 16 consecutive
// lanes of one wave (row sums are DPP reductions) and columns or single
// entries pass through LDS.  The stages and conventions are those of the
// m0 <= 8 wave (Cholesky, C = X H X^H with X = L^-1, Hermitian average,
// zhetd2 reflectors, Sturm bisection of the power-of-two scaled tridiagonal),
// with 16 lanes and 32 points per eigenvalue and bisection round.
__device__ __forceinline__ double group16_sum(double v) {
  v = group8_sum(v);
  return v + dpp_d<0x140>(v, 0.0);  // row_mirror: the other half of the row of 16
}
__device__ __forceinline__ double group16_max(double v) {
  v = group8_max(v);
  return fmax(v, dpp_d<0x140>(v, v));
}
__device__ __forceinline__ double group16_min(double v) {
  v = group8_min(v);
  return fmin(v, dpp_d<0x140>(v, v));
}

__device__ __forceinline__ void heigh_evals16_body(const double* __restrict__ H,
                                          const double* __restrict__ S, int m,
                                          double* __restrict__ evals, int* __restrict__ info,
                                          int64_t blk) {
  constexpr int LD = 17;
  __shared__ cx colbuf[16];
  __shared__ cx wbuf[16];
  __shared__ cx Ls[16 * LD];  // L, then W = X H
  __shared__ cx Xs[16 * LD];  // X = L^-1
  __shared__ cx Hs[16 * LD];  // H, then C
  __shared__ double dsh[17];
  const int t = threadIdx.x, i = t >> 4, j = t & 15;
  const bool in = i < m && j < m;
  const int mm = m * m;
  const cx* Hb = (const cx*)H + blk * mm;
  const cx* Sb = S ? (const cx*)S + blk * mm : nullptr;
  const cx h = in ? Hb[i * m + j] : cx{0.0, 0.0};
  cx s = (in && Sb) ? Sb[i * m + j] : cx{i == j ? 1.0 : 0.0, 0.0};
  cx c = h;
  if (Sb) {
    // 1. Cholesky S = L L^H: column k of the updated S through LDS, one
    // barrier per pivot (every read of step k precedes the barrier of k + 1)
    int fail = 0;
    for (int k = 0; k < m; ++k) {
      if (j == k) colbuf[i] = s;
      __syncthreads();
      const double d = colbuf[k].re;
      // pivots at or below 1e-300 (and non-finite ones) count as not positive
      if (!(d > 1e-300) || !isfinite(d)) {  // uniform
        fail = k + 1;
        break;
      }
      const double inv = nrsq(d), lkk = d * inv;
      const cx lik = i == k ? cx{lkk, 0.0} : cscale(colbuf[i], inv);
      const cx ljk = j == k ? cx{lkk, 0.0} : cscale(colbuf[j], inv);
      if (j == k && i >= k) s = lik;
      if (j > k && i >= j) s = csub(s, cmul(lik, cconj(ljk)));
      __syncthreads();  // colbuf is rewritten by the next pivot
    }
    if (fail) {
      if (j == 0 && i < m) evals[blk * m + i] = NAN;
      if (t == 0) info[blk] = fail;
      return;
    }
    if (j > i) s = {0.0, 0.0};
    // 2. X = L^-1 (column j by forward substitution in thread j), then
    // W = X H and C = W X^H, each entry a 16-term sum from LDS
    Ls[i * LD + j] = s;
    Hs[i * LD + j] = h;
    __syncthreads();
    if (t < 16) {  // column t of X; each thread reads back only what it wrote
      for (int r = 0; r < 16; ++r) {
        cx acc = {r == t ? 1.0 : 0.0, 0.0};
        for (int k = t; k < r; ++k) acc = csub(acc, cmul(Ls[r * LD + k], Xs[k * LD + t]));
        Xs[r * LD + t] = r < t ? cx{0.0, 0.0} : cscale(acc, 1.0 / Ls[r * LD + r].re);
      }
    }
    __syncthreads();
    cx w = {0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 16; ++k) w = cadd(w, cmul(Xs[i * LD + k], Hs[k * LD + j]));
    Ls[i * LD + j] = w;  // L is no longer read
    __syncthreads();
    c = {0.0, 0.0};
#pragma unroll
    for (int k = 0; k < 16; ++k) c = cadd(c, cmul(Ls[i * LD + k], cconj(Xs[j * LD + k])));
  }
  // Hermitian average
  Hs[i * LD + j] = c;
  __syncthreads();
  {
    const cx ct = Hs[j * LD + i];
    c = i == j ? cx{c.re, 0.0} : cscale(cadd(c, cconj(ct)), 0.5);
  }
  // 3. Householder reduction to a real tridiagonal (zhetd2 convention, as
  // in the m0 <= 8 wave): column k through LDS, w through LDS
  double e2[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) e2[q] = 0.0;
#pragma unroll
  for (int k = 0; k < 14; ++k) {
    if (k > m - 3) break;  // uniform
    if (j == k) colbuf[i] = c;
    __syncthreads();
    const cx alpha = colbuf[k + 1];
    double sq = 0.0;
    for (int q = k + 2; q < m; ++q) sq += cabs2(colbuf[q]);
    if (sq == 0.0 && alpha.im == 0.0) {  // uniform: already reduced, H = I
      e2[k] = alpha.re * alpha.re;
      __syncthreads();  // colbuf is rewritten by the next step
      continue;
    }
    const double s2 = alpha.re * alpha.re + alpha.im * alpha.im + sq;
    const double rs = nrsq(s2);
    const double beta = -copysign(s2 * rs, alpha.re), rbeta = -copysign(rs, alpha.re);
    const cx tau = {(beta - alpha.re) * rbeta, -alpha.im * rbeta};
    const cx den = {alpha.re - beta, alpha.im};
    const double dd = nrcp(cabs2(den));
    const cx rden = {den.re * dd, -den.im * dd};  // 1 / (alpha - beta)
    const cx vi = i == k + 1 ? cx{1.0, 0.0} : (i > k + 1 ? cmul(colbuf[i], rden) : cx{0.0, 0.0});
    const cx vj = j == k + 1 ? cx{1.0, 0.0} : (j > k + 1 ? cmul(colbuf[j], rden) : cx{0.0, 0.0});
    // w_i = tau sum_j C[i][j] v_j over the trailing block (a row is 16 lanes)
    cx tt = (i > k && j > k) ? cmul(c, vj) : cx{0.0, 0.0};
    tt.re = group16_sum(tt.re);
    tt.im = group16_sum(tt.im);
    cx wi = cmul(tau, tt);
    if (j == 0) wbuf[i] = wi;
    __syncthreads();
    cx wj = wbuf[j];
    // K = -1/2 tau (w^H v), the same sum in every row
    cx kk = j > k ? cmul(cconj(wj), vj) : cx{0.0, 0.0};
    kk.re = group16_sum(kk.re);
    kk.im = group16_sum(kk.im);
    const cx K = cscale(cmul(tau, kk), -0.5);
    wi = cadd(wi, cmul(K, vi));
    wj = cadd(wj, cmul(K, vj));
    if (i > k && j > k) c = csub(c, cadd(cmul(vi, cconj(wj)), cmul(wi, cconj(vj))));
    e2[k] = beta * beta;
    __syncthreads();  // colbuf and wbuf are rewritten by the next step
  }
  // diagonal and the last off-diagonal element (no reflector needed)
  if (i == j) dsh[i] = c.re;
  if (i == m - 1 && j == m - 2) dsh[16] = cabs2(c);
  __syncthreads();
  double d16[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) d16[q] = dsh[q];
  if (m >= 2) {
    const double el = dsh[16];
#pragma unroll
    for (int q = 0; q < 16; ++q)
      if (q == m - 2) e2[q] = el;
  }
  // Gershgorin interval and the power-of-two scaling into (-1, 1)
  double lo = 1e308, hi = -1e308;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    if (q >= m) break;
    const double el = q > 0 ? sqrt(e2[q - 1]) : 0.0, er = q < m - 1 ? sqrt(e2[q]) : 0.0;
    lo = fmin(lo, d16[q] - el - er);
    hi = fmax(hi, d16[q] + el + er);
  }
  const double tn = fmax(fabs(lo), fabs(hi));
  int ex = 0;
  if (tn > 0.0 && isfinite(tn)) frexp(tn, &ex);
  ex += 1;
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    d16[q] = ldexp(d16[q], -ex);
    e2[q] = ldexp(e2[q], -2 * ex);
  }
  const double fudge = 2.1 * DBL_EPSILON * m * ldexp(tn, -ex);
  lo = ldexp(lo, -ex) - fudge;
  hi = ldexp(hi, -ex) + fudge;
  const double atol = 2.0 * DBL_EPSILON * ldexp(tn, -ex);
  // padding past m: d = 2, e2 = 0 (no sign change below x = 2)
#pragma unroll
  for (int q = 0; q < 16; ++q)
    if (q >= m) d16[q] = 2.0;
  // 4. eigenvalue idx = row i; each lane counts at two points, so a round
  // splits the bracket at 32 interior points per eigenvalue
  const int idx = i, pt = j;
  const double f0 = (double)(2 * pt + 1) / 33.0, f1 = (double)(2 * pt + 2) / 33.0;
  for (int round = 0; round < 40; ++round) {
    const bool done = hi - lo <= fmax(atol, 2.0 * DBL_EPSILON * fmax(fabs(lo), fabs(hi)));
    if (__all(done || idx >= m)) break;  // per wave: no barrier below
    const double x0 = lo + (hi - lo) * f0, x1 = lo + (hi - lo) * f1;
    int c0, c1;
    bool zero;
    sturm_count16_fast(d16, e2, x0, x1, c0, c1, zero);
    if (__any(zero)) sturm_count16(d16, e2, x0, x1, c0, c1);  // rare
    double nlo = c1 <= idx ? x1 : (c0 <= idx ? x0 : lo);
    double nhi = c0 > idx ? x0 : (c1 > idx ? x1 : hi);
    nlo = group16_max(nlo);
    nhi = group16_min(nhi);
    if (!done) {
      lo = nlo;
      hi = fmax(nhi, nlo);
    }
  }
  if (pt == 0 && idx < m) evals[blk * m + idx] = ldexp(0.5 * (lo + hi), ex);
  if (t == 0) info[blk] = 0;
}

// One k-block per workgroup; blk is the block index (H, S, evals, evecs and
// info are indexed by it).
template <int MAXM>
__device__ inline void heigh_body(const double* __restrict__ H, const double* __restrict__ S,
                                  int m, double* __restrict__ evals, double* __restrict__ evecs,
                                  int* __restrict__ info, int64_t blk_) {
  // m <= 8 takes the one-wave register version whatever the launch width, so
  // a block gets the same bits in the single and the batched launches
  if (MAXM == 8 || m <= 8) {
    if (threadIdx.x < 64) heigh_wave8_body(H, S, m, evals, evecs, info, blk_);
    return;
  }
  constexpr int LD = MAXM + 1;
  // two copies of C and of V so that a Jacobi round needs one barrier
  // (read one copy, write the other); L is the Cholesky factor.
  constexpr bool kDouble = MAXM <= 16;
  constexpr int NB = kDouble ? 2 : 1;
  __shared__ cx Ab[NB][MAXM * LD];
  __shared__ cx Vb[NB][MAXM * LD];
  __shared__ cx B[MAXM * LD];
  // round-robin schedule: partner and pair slot of every index in every round
  __shared__ unsigned char s_partner[MAXM][MAXM];
  __shared__ unsigned char s_slot[MAXM][MAXM];
  __shared__ Rot s_rot[MAXM / 2];
  __shared__ int rank_of[MAXM];
  __shared__ int fail;
  __shared__ double red[2];

  const int tid = threadIdx.x;
  const int nt = blockDim.x;
  const int64_t blk = blk_;
  const int mm = m * m;
  const cx* Hb = (const cx*)H + blk * mm;
  const cx* Sb = S ? (const cx*)S + blk * mm : nullptr;
  cx* A = Ab[0];
  cx* V = Vb[0];

  for (int e = tid; e < mm; e += nt) {
    int i = e / m, j = e - i * m;
    A[i * LD + j] = Hb[e];
    B[i * LD + j] = Sb ? Sb[e] : cx{i == j ? 1.0 : 0.0, 0.0};
  }
  if (tid == 0) fail = 0;
  __syncthreads();

  // 1. Cholesky, right-looking, lower triangle of B.
  if (Sb) {
    for (int k = 0; k < m; ++k) {
      if (tid == 0) {
        double d = B[k * LD + k].re;
        if (!(d > 0.0) || !isfinite(d))
          fail = k + 1;
        else
          B[k * LD + k] = {sqrt(d), 0.0};
      }
      __syncthreads();
      if (fail) break;
      double inv = 1.0 / B[k * LD + k].re;
      for (int i = k + 1 + tid; i < m; i += nt) B[i * LD + k] = cscale(B[i * LD + k], inv);
      __syncthreads();
      int w = m - k - 1;
      for (int e = tid; e < w * w; e += nt) {
        int i = k + 1 + e / w, j = k + 1 + e % w;
        if (j <= i) B[i * LD + j] = csub(B[i * LD + j], cmul(B[i * LD + k], cconj(B[j * LD + k])));
      }
      __syncthreads();
    }
  }
  if (fail) {
    for (int i = tid; i < m; i += nt) evals[blk * m + i] = NAN;
    if (evecs)
      for (int e = tid; e < mm; e += nt) ((cx*)evecs)[blk * mm + e] = {0.0, 0.0};
    if (tid == 0) info[blk] = fail;
    return;
  }

  // 2. C = L^-1 Hbar L^-H.  W = L^-1 Hbar in place in A, then Z = L^-1 W^H in
  // V, C = Z^H back in A.
  if (Sb) {
    for (int i = 0; i < m; ++i) {
      for (int j = tid; j < m; j += nt) {
        cx s = A[i * LD + j];
        for (int k = 0; k < i; ++k) s = csub(s, cmul(B[i * LD + k], A[k * LD + j]));
        A[i * LD + j] = cscale(s, 1.0 / B[i * LD + i].re);
      }
      __syncthreads();
    }
    for (int e = tid; e < mm; e += nt) {
      int i = e / m, j = e - i * m;
      V[i * LD + j] = cconj(A[j * LD + i]);
    }
    __syncthreads();
    for (int i = 0; i < m; ++i) {
      for (int j = tid; j < m; j += nt) {
        cx s = V[i * LD + j];
        for (int k = 0; k < i; ++k) s = csub(s, cmul(B[i * LD + k], V[k * LD + j]));
        V[i * LD + j] = cscale(s, 1.0 / B[i * LD + i].re);
      }
      __syncthreads();
    }
    for (int e = tid; e < mm; e += nt) {
      int i = e / m, j = e - i * m;
      A[i * LD + j] = cconj(V[j * LD + i]);
    }
    __syncthreads();
  }
  // Hermitian average (removes the rounding asymmetry), V = I.  The launch
  // has at least m*m threads: thread e owns entry (e / m, e % m).
  const bool owner = tid < mm;
  const int ei = owner ? tid / m : 0, ej = owner ? tid - (tid / m) * m : 0;
  {
    cx mine = {0.0, 0.0};
    if (owner) {
      cx a = A[ei * LD + ej], b = A[ej * LD + ei];
      mine = ei == ej ? cx{a.re, 0.0} : cscale(cadd(a, cconj(b)), 0.5);
    }
    __syncthreads();
    if (owner) {
      A[ei * LD + ej] = mine;
      V[ei * LD + ej] = {ei == ej ? 1.0 : 0.0, 0.0};
    }
    __syncthreads();
  }

  // 3. Jacobi sweeps with the round-robin ordering of the (even-padded)
  // indices: in every round the me/2 rotations are formed by one thread each
  // and shared through LDS, then every thread updates its own entry of C and
  // of V from the four entries of its 2x2 coupling.
  int converged = (m == 1);
  int cur = 0;
  const int me = m + (m & 1);
  for (int e = tid; e < (me - 1) * me; e += nt) {
    int r = e / me, x = e - r * me;
    int y = rr_partner(x, r, me);
    s_partner[r][x] = (unsigned char)y;
    // slot: 0 for the pair containing me-1, else the distance k in {r+k, r-k}
    int p = min(x, y);
    int slot;
    if (y == me - 1 || x == me - 1) {
      slot = 0;
    } else {
      int k = (p - r) % (me - 1);
      if (k < 0) k += me - 1;
      slot = k <= (me - 1) / 2 ? k : (me - 1) - k;
    }
    s_slot[r][x] = (unsigned char)slot;
  }
  __syncthreads();
  for (int sweep = 0; sweep < kMaxSweeps && !converged; ++sweep) {
    // convergence: off-diagonal Frobenius norm against the whole norm
    if (tid < 2) red[tid] = 0.0;
    __syncthreads();
    double off = 0.0, all = 0.0;
    if (owner) {
      double v = cabs2(A[ei * LD + ej]);
      all = v;
      if (ei != ej) off = v;
    }
    for (int o = 32; o > 0; o >>= 1) {
      off += __shfl_xor(off, o);
      all += __shfl_xor(all, o);
    }
    if ((tid & 63) == 0) {
      atomicAdd(&red[0], off);
      atomicAdd(&red[1], all);
    }
    __syncthreads();
    if (red[0] <= 1e-32 * red[1]) {
      converged = 1;
      break;
    }
    for (int r = 0; r < me - 1; ++r) {
      if (tid < me / 2) {
        // pair of slot tid in round r
        int p, q;
        if (tid == 0) {
          p = r;
          q = me - 1;
        } else {
          p = (r + tid) % (me - 1);
          q = (r - tid + me - 1) % (me - 1);
        }
        if (p > q) {
          int t = p;
          p = q;
          q = t;
        }
        bool valid = q < m;
        cx b = valid ? A[p * LD + q] : cx{0.0, 0.0};
        double a = valid ? A[p * LD + p].re : 0.0;
        double d = valid ? A[q * LD + q].re : 0.0;
        s_rot[tid] = make_rot(a, d, b, valid);
      }
      __syncthreads();
      cx na = {0.0, 0.0}, nv = {0.0, 0.0};
      if (owner) {
        const int i = ei, j = ej;
        const int ip = s_partner[r][i], jp = s_partner[r][j];
        const Rot ri = s_rot[s_slot[r][i]];
        const Rot rj = s_rot[s_slot[r][j]];
        // column i of J: J[i][i] and J[ip][i]
        const bool fi = i < ip, fj = j < jp;
        cx Jii = fi ? cx{ri.c, 0.0} : cx{ri.ph_re * ri.c, ri.ph_im * ri.c};
        cx Jpi = fi ? cx{-ri.ph_re * ri.s, -ri.ph_im * ri.s} : cx{ri.s, 0.0};
        cx Jjj = fj ? cx{rj.c, 0.0} : cx{rj.ph_re * rj.c, rj.ph_im * rj.c};
        cx Jpj = fj ? cx{-rj.ph_re * rj.s, -rj.ph_im * rj.s} : cx{rj.s, 0.0};
        if (j == i || j == ip) {
          // inside one rotated 2x2 block: exact diagonal form
          if (i == j) na = {A[i * LD + i].re + (fi ? -ri.tb : ri.tb), 0.0};
        } else {
          // sum over a in {i, ip}, b in {j, jp} of conj(J[a][i]) A[a][b] J[b][j]
          const bool jin = jp < m, iin = ip < m;
          cx t0 = cmul(A[i * LD + j], Jjj);
          if (jin) t0 = cadd(t0, cmul(A[i * LD + jp], Jpj));
          na = cmul(cconj(Jii), t0);
          if (iin) {
            cx t1 = cmul(A[ip * LD + j], Jjj);
            if (jin) t1 = cadd(t1, cmul(A[ip * LD + jp], Jpj));
            na = cadd(na, cmul(cconj(Jpi), t1));
          }
        }
        nv = cmul(V[i * LD + j], Jjj);
        if (jp < m) nv = cadd(nv, cmul(V[i * LD + jp], Jpj));
      }
      if (kDouble) {
        cur ^= 1;
        A = Ab[cur];
        V = Vb[cur];
        if (owner) {
          A[ei * LD + ej] = na;
          V[ei * LD + ej] = nv;
        }
        __syncthreads();
      } else {
        __syncthreads();
        if (owner) {
          A[ei * LD + ej] = na;
          V[ei * LD + ej] = nv;
        }
        __syncthreads();
      }
    }
  }

  // 4. sort ascending, back-transform u = L^-H v, write out.
  for (int i = tid; i < m; i += nt) {
    double li = A[i * LD + i].re;
    int rk = 0;
    for (int k = 0; k < m; ++k) {
      double lk = A[k * LD + k].re;
      if (lk < li || (lk == li && k < i)) ++rk;
    }
    rank_of[i] = rk;
    evals[blk * m + rk] = li;
  }
  if (tid == 0) info[blk] = converged ? 0 : -1;
  __syncthreads();
  if (evecs) {
    if (Sb) {
      for (int i = m - 1; i >= 0; --i) {
        for (int j = tid; j < m; j += nt) {
          cx s = V[i * LD + j];
          for (int k = i + 1; k < m; ++k) s = csub(s, cmul(cconj(B[k * LD + i]), V[k * LD + j]));
          V[i * LD + j] = cscale(s, 1.0 / B[i * LD + i].re);
        }
        __syncthreads();
      }
    }
    cx* out = (cx*)evecs + blk * mm;
    for (int e = tid; e < mm; e += nt) {
      int i = e / m, j = e - i * m;
      out[i * m + rank_of[j]] = V[i * LD + j];
    }
  }
}

}  // namespace dev
}  // namespace tl
