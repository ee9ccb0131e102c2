// The O(M) banded route to the Fourier coefficients <rho^-1>_l, l = 0..L,
// L = M + M0 (Sec. 3.2.1), on gfx950.
//
// For a pair (target r(t, theta_j), source curve t_s != t) Lemma 3.3 turns the
// coefficients into the solution of a linear difference equation whose
// coefficients are those of rho^2, a trigonometric polynomial in theta_s of
// degree m0 (eqs. (3.11)-(3.15)).  With the first m0 and the last m0
// coefficients known (eq. (3.16)), the other L - 2 m0 + 1 solve the Hermitian
// banded system A x = b of eqs. (3.17)-(3.18),
//   A_{rc} = (2 m0 + r + c) <rho^2>_{r-c},  |r - c| <= m0.
// Three kernels:
//  1. <rho^2>_n, n = 0..8: rho^2 at 16 equispaced source azimuths (exact
//     while its degree is at most 7; 64 otherwise), one per lane, the
//     transform by sums over the lanes of each pair; the largest
//     |<rho^2>_n| / <rho^2>_0 over the call's pairs feeds the m0 rule of
//     eq. (3.13).
//  2. the 2 m0 known coefficients by composite 16-point Gauss-Legendre
//     quadrature (the paper uses adaptive Gauss-Legendre), one pair per
//     wavefront, 4 panels x 16 nodes per pass over the lanes.  The panels are
//     graded geometrically (ratio 4) towards the real part a of the complex
//     root of rho^2, from a first panel of length b (its imaginary part), and
//     are at most 14 / L long elsewhere, so that e^{-i L theta} is integrated
//     to rounding.  Where the coefficients of rho^2 certify that the last m0
//     coefficients are below e^-40 of the first (decays_by), those are set to
//     zero and the panels only need to resolve 1/rho.
//  3. the banded system, one pair per lane: a right-looking L D L^H
//     factorisation with the (m0+1) x (m0+1) active window in registers, the
//     forward substitution fused with it, the factor rows stored to a
//     workspace (coalesced across the lanes) and read back for the backward
//     substitution, four rows of records loaded at a time.  The system is cut
//     (at N/8, N/4 or N/2 rows) where the same certificate puts the dropped
//     coefficients below e^-40 of the first.  A is positive definite when eq. (3.19) holds (Lemma 3.4);
//     a pivot that is not positive is reported per pair.
#include "ffbie_banded.hpp"

namespace ffbie {

int rho2_degree(const Geom& g) {
  int mtop = 0;
  for (int l = 0; l < g.lmax; ++l)
    for (int m = 0; m <= g.mmax; ++m)
      if (g.a[l][m] != 0.0 && m > mtop) mtop = m;
  // R(t_s, .) has degree mtop; rho^2 = R^2 + R_s^2 - 2 R R_s (sin t sin t_s
  // cos(theta_s - theta) + cos t cos t_s) has degree max(2 mtop, mtop + 1).
  // Stretched with unequal x and y axes, R_s^2 (d_x^2 cos^2 + d_y^2 sin^2)
  // keeps a cos(2 theta_s) part: 2 mtop + 2.
  if (g.ax[0] != g.ax[1]) return 2 * mtop + 2;
  return 2 * mtop > mtop + 1 ? 2 * mtop : mtop + 1;
}

namespace {

constexpr double kPi = 3.14159265358979323846;
constexpr double kTwoPi = 6.28318530717958647693;
constexpr double kBandKappa = 7.0;   // panel half-length times the highest order

__device__ __forceinline__ void stage_table(double* tab, const double* __restrict__ tab_g, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) tab[i] = tab_g[i];
  __syncthreads();
}

// A decay certificate from the coefficients of rho^2 alone: if
//   S(y) = sum_{n=1..8} 2 |<rho^2>_n| e^{n y} <= <rho^2>_0 / 2,
// then |rho^2| >= <rho^2>_0 / 2 on the strip |Im theta| <= y (no root there),
// so |<rho^-1>_l| <= (2 / <rho^2>_0)^{1/2} e^{-y |l|} by moving the contour,
// while <rho^-1>_0 >= (3 <rho^2>_0 / 2)^{-1/2}: |<rho^-1>_l| <= 2 e^{-y |l|}
// <rho^-1>_0.  (The root kernel's b need not belong to the root nearest the
// real axis, so it is not used for this.)
__device__ __forceinline__ bool decays_by(const cplx* __restrict__ c2, double y) {
  const double e = exp(y);
  double p = 1.0, s = 0.0;
#pragma unroll
  for (int n = 1; n < kBandC2; ++n) {
    p *= e;
    s = fma(2.0 * sqrt(abs2(c2[n])), p, s);
  }
  return s <= 0.5 * c2[0].re;
}

// exponent with e^{-x} * 2 <= e^{-40}: coefficients past it are below e^-40
// of <rho^-1>_0
constexpr double kDecayExp = 40.7;

// ---------------------------------------------------------------------------
// 1. <rho^2>_n
// ---------------------------------------------------------------------------
// Sum over each segment of NS lanes (16 or 64), returned to every lane of it.
template <int NS>
__device__ __forceinline__ double segment_sum(double v) {
  if constexpr (NS == 64) {
    return wave_sum(v);
  } else {
    v += dpp_zero<0x111>(v);   // row_shr:1
    v += dpp_zero<0x112>(v);   // row_shr:2
    v += dpp_zero<0x114>(v);   // row_shr:4
    v += dpp_zero<0x118>(v);   // row_shr:8
    return __shfl(v, (int)((threadIdx.x & 48) | 15), 64);
  }
}

// NS samples per pair (16 while rho^2 has degree <= 7, else 64), 64 / NS pairs
// per wavefront
template <int MM, int NS>
__global__ __launch_bounds__(256) void band_rho2_kernel(BandArgs a) {
  extern __shared__ double tab[];
  stage_table(tab, a.tab_g, a.P.tab_n);
  constexpr int kPerWave = 64 / NS;
  const int lane = threadIdx.x & 63;
  const int q = lane % NS, seg = lane / NS;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t n_waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const int mask = a.P.tab_n - 1, quarter = 2 * a.P.M;
  const int Kq = q * (8 * a.P.M / NS);        // table index of 2 pi q / NS
  const double nan = __builtin_nan("");
  double worst = 0.0;                          // lane n of a segment: largest ratio at order n
  for (int64_t i0 = wave * kPerWave; i0 < a.n; i0 += n_waves * kPerWave) {
    const int64_t i = i0 + seg;
    if (i >= a.n) continue;                    // a whole segment: no lane of another is touched
    cplx* out = a.c2 + i * kBandC2;
    if (a.status[i] & FFBIE_PAIR_SINGULAR) {
      if (q < kBandC2) out[q] = mk(nan, nan);
      continue;
    }
    const int J = 4 * (a.az_in[i] & (2 * a.P.M - 1));
    PairGeo<MM> p;
    pair_geo<MM>(a.P.g, a.t_in[i], a.ts_in[i], tab, J, mask, quarter, &p);
    double dx, dy, dz;
    dr_grid<MM>(p, tab, Kq, J, mask, quarter, &dx, &dy, &dz);
    const double r2 = fma(dx, dx, fma(dy, dy, dz * dz)) * (1.0 / NS);
    cplx mine = mk(0.0, 0.0);
    double c0 = 0.0;
#pragma unroll
    for (int n = 0; n < kBandC2; ++n) {
      const int idx = n * Kq;
      const double re = segment_sum<NS>(r2 * tab[(idx + quarter) & mask]);
      const double im = -segment_sum<NS>(r2 * tab[idx & mask]);
      if (n == 0) c0 = re;
      if (q == n) mine = mk(re, im);
    }
    if (q < kBandC2) {
      out[q] = mine;
      worst = fmax(worst, sqrt(abs2(mine)) / c0);
    }
  }
  if (!a.ratio_part) return;
  // per-block maxima, no atomics: a reduction kernel combines the blocks
  __shared__ double red[256 / NS][kBandC2];
  const int segs = blockDim.x / NS, sb = threadIdx.x / NS;
  if (q < kBandC2) red[sb][q] = worst;
  __syncthreads();
  if (threadIdx.x < kBandC2) {
    double m = 0.0;
    for (int w = 0; w < segs; ++w) m = fmax(m, red[w][threadIdx.x]);
    a.ratio_part[(int64_t)blockIdx.x * kBandC2 + threadIdx.x] = m;
  }
}

// ratio[n] = max over the blocks of ratio_part[b][n]
__global__ __launch_bounds__(256) void band_ratio_reduce_kernel(const double* __restrict__ part,
                                                                 int blocks, double* __restrict__ out) {
  __shared__ double red[256];
  for (int n = 0; n < kBandC2; ++n) {
    double m = 0.0;
    for (int b = threadIdx.x; b < blocks; b += blockDim.x) m = fmax(m, part[(int64_t)b * kBandC2 + n]);
    red[threadIdx.x] = m;
    __syncthreads();
    for (int w = blockDim.x / 2; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + w]);
      __syncthreads();
    }
    if (threadIdx.x == 0) out[n] = red[0];
    __syncthreads();
  }
}

// ---------------------------------------------------------------------------
// 2. the known coefficients of eq. (3.16) by graded Gauss-Legendre quadrature
// ---------------------------------------------------------------------------
// M0C: a bound on m0 (4 or 8) that sizes the accumulators
template <int MM, int M0C>
__global__ __launch_bounds__(256) void band_moments_kernel(BandArgs a) {
  extern __shared__ double tab[];
  stage_table(tab, a.tab_g, a.P.tab_n);
  const int lane = threadIdx.x & 63;
  const int g = lane & 15, sub = lane >> 4;
  const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
  const int64_t n_waves = ((int64_t)gridDim.x * blockDim.x) >> 6;
  const int mask = a.P.tab_n - 1, quarter = 2 * a.P.M;
  const int L = a.P.L, m0 = a.m0, l0 = L - m0 + 1;
  const double xg1 = 1.0 + a.gl_x[g], wg = a.gl_w[g];
  const double hmax_tail = fmin(2.0 * kBandKappa / L, 0.25 * kPi);
  const double nan = __builtin_nan("");
  for (int64_t i = wave; i < a.n; i += n_waves) {
    cplx* row = a.rhoinv + i * (L + 1);
    if (a.status[i] & FFBIE_PAIR_SINGULAR) {
      if (lane < m0) { row[lane] = mk(nan, nan); row[l0 + lane] = mk(nan, nan); }
      continue;
    }
    const int J = 4 * (a.az_in[i] & (2 * a.P.M - 1));
    PairGeo<MM> p;
    pair_geo<MM>(a.P.g, a.t_in[i], a.ts_in[i], tab, J, mask, quarter, &p);
    const double sj = tab[J & mask], cj = tab[(J + quarter) & mask];
    const RootRec rr = a.roots[i];
    const double a_off = rr.u;
    // Where the certificate shows the last m0 coefficients below e^-40 of
    // <rho^-1>_0 they are taken as zero (they enter only the right-hand sides
    // of the last m0 equations).  Such a pair needs no panels short enough for
    // e^{-i L theta}: its panels resolve the analytic 1/rho, whose
    // singularities lie at least y_tail from the real axis (at most
    // 1.5 y_tail long; measured 1e-15 of <rho^-1>_0 on config-2 pairs).
    const double y_tail = kDecayExp / l0;
    const bool tail_zero = decays_by(a.c2 + i * kBandC2, y_tail);
    const double hmax = tail_zero ? fmin(0.25 * kPi, 1.5 * y_tail) : hmax_tail;
    // panels on each side of a: [0, h0], [h0, 4 h0], ... while shorter than
    // hmax (K panels, last edge eK), then nu equal panels up to pi
    const double h0 = fmin(rr.b, hmax);
    int K = 1;
    double eK = h0;
    while (K < 64) {
      const double nx = 4.0 * eK;
      if (nx - eK >= hmax || nx >= kPi) break;
      eK = nx;
      ++K;
    }
    const int nu = max(1, (int)ceil((kPi - eK) / hmax));
    const double hu = (kPi - eK) / nu;
    const int P = K + nu;
    const int passes = (2 * P + 3) >> 2;
    double Hr[M0C], Hi[M0C], Tr[M0C], Ti[M0C];
#pragma unroll
    for (int l = 0; l < M0C; ++l) { Hr[l] = 0.0; Hi[l] = 0.0; Tr[l] = 0.0; Ti[l] = 0.0; }
    for (int it = 0; it < passes; ++it) {
      const int pp = 4 * it + sub;
      const bool valid = pp < 2 * P;
      const int q = !valid ? 0 : (pp < P ? pp : pp - P);
      const double side = pp < P ? 1.0 : -1.0;
      double lo, hi;
      if (q < K) {
        lo = q == 0 ? 0.0 : ldexp(h0, 2 * (q - 1));
        hi = ldexp(h0, 2 * q);
      } else {
        const int r = q - K;
        lo = fma((double)r, hu, eK);
        hi = r + 1 == nu ? kPi : fma((double)(r + 1), hu, eK);
      }
      const double half = 0.5 * (hi - lo);
      const double s = side * fma(half, xg1, lo);
      const double w = valid ? half * wg : 0.0;
      const double d = a_off + s;                     // source azimuth theta_j + d
      double dh, cD;
      sincos_bounded(0.5 * d, &dh, &cD);
      const double sd = 2.0 * dh * cD, cd = fma(-2.0 * dh, dh, 1.0);
      const double cq = fma(cj, cd, -sj * sd), sq = fma(sj, cd, cj * sd);
      const double sS = fma(sj, cD, cj * dh), cS = fma(cj, cD, -sj * dh);
      double dx, dy, dz;
      dr_values<MM>(p, cq, sq, dh, cD, sS, cS, &dx, &dy, &dz);
      const double f = w * rsqrt_refined(fma(dx, dx, fma(dy, dy, dz * dz)));
      // e^{-i l d}, l = 0..m0-1, and e^{-i (l0 + l) d}
      double er = 1.0, ei = 0.0;
#pragma unroll
      for (int l = 0; l < M0C; ++l) {
        if (l < m0) {
          Hr[l] = fma(f, er, Hr[l]);
          Hi[l] = fma(f, ei, Hi[l]);
          const double nr = fma(er, cd, ei * sd);
          ei = fma(ei, cd, -er * sd);
          er = nr;
        }
      }
      if (!tail_zero) {
        double st, ct;
        sincos_bounded(l0 * d, &st, &ct);
        er = ct;
        ei = -st;
#pragma unroll
        for (int l = 0; l < M0C; ++l) {
          if (l < m0) {
            Tr[l] = fma(f, er, Tr[l]);
            Ti[l] = fma(f, ei, Ti[l]);
            const double nr = fma(er, cd, ei * sd);
            ei = fma(ei, cd, -er * sd);
            er = nr;
          }
        }
      }
    }
    // (1/2pi) e^{-i l theta_j} sum ...; theta_j = pi J / (4M) on the table grid
    cplx mine_h = mk(0.0, 0.0), mine_t = mk(0.0, 0.0);
#pragma unroll
    for (int l = 0; l < M0C; ++l) {
      if (l < m0) {
        const double hr = wave_sum(Hr[l]), hi = wave_sum(Hi[l]);
        const double tr = tail_zero ? 0.0 : wave_sum(Tr[l]);
        const double ti = tail_zero ? 0.0 : wave_sum(Ti[l]);
        if (lane == l) {
          const int ih = l * J, it = (l0 + l) * J;
          const cplx ph = mk(tab[(ih + quarter) & mask], -tab[ih & mask]);
          const cplx pt = mk(tab[(it + quarter) & mask], -tab[it & mask]);
          mine_h = (1.0 / kTwoPi) * (mk(hr, hi) * ph);
          mine_t = (1.0 / kTwoPi) * (mk(tr, ti) * pt);
        }
      }
    }
    if (lane < m0) {
      row[lane] = mine_h;
      row[l0 + lane] = mine_t;
    }
  }
}

// ---------------------------------------------------------------------------
// 3. the banded system of eq. (3.17), one pair per lane
// ---------------------------------------------------------------------------
template <int M0T>
__global__ __launch_bounds__(64) void band_solve_kernel(BandArgs a) {
  const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= a.chunk_n) return;
  const int64_t i = a.chunk0 + k;
  const int L = a.P.L;
  const int N = L - 2 * M0T + 1;                  // unknowns <rho^-1>_{m0} .. <rho^-1>_{L-m0}
  cplx* row = a.rhoinv + i * (L + 1);
  if (a.status[i] & FFBIE_PAIR_SINGULAR) {
    const double nan = __builtin_nan("");
    for (int l = M0T; l <= L - M0T; ++l) row[l] = mk(nan, nan);
    return;
  }
  cplx c2[M0T + 1];
#pragma unroll
  for (int n = 0; n <= M0T; ++n) c2[n] = a.c2[i * kBandC2 + n];
  c2[0].im = 0.0;                                 // rho^2 is real: <rho^2>_0 is real
  // <rho^2>_{r-c} for a static offset
  auto C2 = [&](int o) { return o >= 0 ? c2[o] : conj(c2[-o]); };
  cplx head[M0T], tail[M0T];
#pragma unroll
  for (int l = 0; l < M0T; ++l) {
    head[l] = row[l];
    tail[l] = row[L - M0T + 1 + l];
  }
  // right-hand sides of the first m0 and the last m0 equations (the others
  // have no known term): b_r = - sum over known l = r + j of a_j(r) <rho^-1>_l,
  // a_j(r) = (m0 + 2r + j) <rho^2>_{m0-j} (eq. (3.15))
  cplx bf[M0T], bl[M0T];
#pragma unroll
  for (int r = 0; r < M0T; ++r) {
    cplx s = mk(0.0, 0.0);
#pragma unroll
    for (int j = 0; j + r < M0T; ++j) s = s + ((double)(M0T + 2 * r + j) * C2(M0T - j)) * head[r + j];
    bf[r] = mk(-s.re, -s.im);
    const int rr = N - M0T + r;                   // equation index of the r-th last row
    cplx u = mk(0.0, 0.0);
#pragma unroll
    for (int j = 2 * M0T - r; j <= 2 * M0T; ++j)
      u = u + ((double)(M0T + 2 * rr + j) * C2(M0T - j)) * tail[r + j - 2 * M0T];
    bl[r] = mk(-u.re, -u.im);
  }
  // active window: W[d][e] = current A_{i+d, i+e}, 0 <= e <= d <= m0, and the
  // right-hand sides of rows i..i+m0 (the first m0 rows all start in it)
  cplx W[M0T + 1][M0T + 1], bw[M0T + 1];
#pragma unroll
  for (int d = 0; d <= M0T; ++d) {
#pragma unroll
    for (int e = 0; e <= d; ++e)
      W[d][e] = (double)(2 * M0T + d + e) * C2(d - e);
    bw[d] = d < M0T ? bf[d] : mk(0.0, 0.0);
  }
  const int64_t S = a.stride;
  cplx* fac = a.fac + k;
  // where the decay certificate puts <rho^-1>_l below e^-40 of <rho^-1>_0,
  // the system is cut (Ne rows, zero known values beyond, as in Olver's
  // boundary-value treatment) and the rest of the row is zero
  int Ne = N;
  {
    // the smallest of N/8, N/4, N/2 rows whose first dropped coefficient,
    // l = m0 + Ne, the decay certificate puts below e^-40 of <rho^-1>_0
    const cplx* c2g = a.c2 + i * kBandC2;
#pragma unroll
    for (int f = 8; f >= 2; f >>= 1) {
      const int cand = max(2 * M0T + 1, N / f);
      if (Ne == N && cand < N && decays_by(c2g, kDecayExp / (M0T + cand))) Ne = cand;
    }
  }
  const int tail_from = Ne == N ? N - M0T : N;   // rows with known tail terms
  // the last m0 rows enter the window during the sweep: their right-hand
  // sides wait in the z slot of their own record, written only when the row
  // becomes the pivot
  if (Ne == N) {
#pragma unroll
    for (int q = 0; q < M0T; ++q) fac[(int64_t)(N - M0T + q) * (M0T + 1) * S] = bl[q];
  }
  bool not_pd = false;
  for (int r = 0; r < Ne; ++r) {
    const double D = W[0][0].re;
    not_pd |= !(D > 0.0);
    const double inv = 1.0 / D;
    cplx l[M0T + 1];
#pragma unroll
    for (int d = 1; d <= M0T; ++d) l[d] = W[d][0] * inv;
    const cplx y = bw[0];
    cplx* rec = fac + (int64_t)r * (M0T + 1) * S;
    rec[0] = y * inv;                             // z_r = y_r / D_r
#pragma unroll
    for (int d = 1; d <= M0T; ++d) rec[d * S] = l[d];
#pragma unroll
    for (int d = 1; d <= M0T; ++d) {
      bw[d] = bw[d] - l[d] * y;
#pragma unroll
      for (int e = 1; e <= d; ++e) W[d][e] = W[d][e] - l[d] * conj(W[e][0]);
    }
#pragma unroll
    for (int d = 1; d <= M0T; ++d) {
      bw[d - 1] = bw[d];
#pragma unroll
      for (int e = 1; e <= d; ++e) W[d - 1][e - 1] = W[d][e];
    }
    const int rn = r + 1 + M0T;                   // row entering the window
    const bool in = rn < Ne;
#pragma unroll
    for (int e = 0; e <= M0T; ++e)
      W[M0T][e] = in ? (double)(M0T + 2 * rn + e) * C2(M0T - e) : mk(0.0, 0.0);
    bw[M0T] = mk(0.0, 0.0);
    if (in && rn >= tail_from) bw[M0T] = fac[(int64_t)rn * (M0T + 1) * S];
  }
  // backward substitution L^H x = z: x_r = z_r - sum_d conj(l_d(r)) x_{r+d}
  cplx xw[M0T + 1];
#pragma unroll
  for (int d = 0; d <= M0T; ++d) xw[d] = mk(0.0, 0.0);
  // records are loaded kBlk rows at a time, all loads of a block issued before
  // its arithmetic, so that one memory latency is exposed per block
  constexpr int kBlk = 4;
  for (int r = Ne; r < N; ++r) row[M0T + r] = mk(0.0, 0.0);
  for (int r0 = Ne - 1; r0 >= 0; r0 -= kBlk) {
    cplx blk[kBlk][M0T + 1];
#pragma unroll
    for (int b = 0; b < kBlk; ++b) {
      const int r = r0 - b;
      if (r >= 0) {
        const cplx* rec = fac + (int64_t)r * (M0T + 1) * S;
#pragma unroll
        for (int d = 0; d <= M0T; ++d) blk[b][d] = rec[d * S];
      }
    }
#pragma unroll
    for (int b = 0; b < kBlk; ++b) {
      const int r = r0 - b;
      if (r >= 0) {
        cplx x = blk[b][0];
#pragma unroll
        for (int d = 1; d <= M0T; ++d) x = x - conj(blk[b][d]) * xw[d];
        row[M0T + r] = x;
#pragma unroll
        for (int d = M0T; d >= 2; --d) xw[d] = xw[d - 1];
        xw[1] = x;
      }
    }
  }
  if (not_pd) a.status[i] |= FFBIE_PAIR_NOT_PD;
}

int mm_of(int mmax) { return mmax <= 0 ? 0 : mmax <= 1 ? 1 : mmax <= 2 ? 2 : mmax <= 4 ? 4 : 8; }

int64_t wave_blocks(int64_t n) {
  int64_t b = (n + 3) / 4;                        // 4 pairs (wavefronts) per block
  if (b > 16384) b = 16384;
  return b < 1 ? 1 : b;
}

}  // namespace

#define FFBIE_BAND_MM(X) X(0) X(1) X(2) X(4) X(8)

namespace {
bool rho2_narrow(const BandArgs& a) { return rho2_degree(a.P.g) <= 7 && a.P.M >= 16; }
}  // namespace

int band_rho2_blocks(const BandArgs& a) {
  return (int)wave_blocks(rho2_narrow(a) ? (a.n + 3) / 4 : a.n);
}

hipError_t launch_band_rho2(const BandArgs& a, hipStream_t s) {
  const size_t lds = a.P.tab_n * sizeof(double);
  // 16 samples resolve a trigonometric polynomial of degree <= 7 exactly
  const bool narrow = rho2_narrow(a);
  const int blocks = band_rho2_blocks(a);
  const dim3 grid((unsigned)blocks);
  switch (mm_of(a.P.g.mmax)) {
#define X(MMV)                                                                                   \
  case MMV:                                                                                      \
    if (narrow)                                                                                  \
      hipLaunchKernelGGL((band_rho2_kernel<MMV, 16>), grid, dim3(256), lds, s, a);               \
    else                                                                                         \
      hipLaunchKernelGGL((band_rho2_kernel<MMV, 64>), grid, dim3(256), lds, s, a);               \
    break;
    FFBIE_BAND_MM(X)
#undef X
  }
  if (a.ratio_part)
    hipLaunchKernelGGL(band_ratio_reduce_kernel, dim3(1), dim3(256), 0, s, a.ratio_part, blocks,
                       a.ratio);
  return hipGetLastError();
}

hipError_t launch_band_moments(const BandArgs& a, hipStream_t s) {
  const size_t lds = a.P.tab_n * sizeof(double);
  const dim3 grid((unsigned)wave_blocks(a.n));
  switch (mm_of(a.P.g.mmax)) {
#define X(MMV)                                                                                   \
  case MMV:                                                                                      \
    if (a.m0 <= 4)                                                                               \
      hipLaunchKernelGGL((band_moments_kernel<MMV, 4>), grid, dim3(256), lds, s, a);             \
    else                                                                                         \
      hipLaunchKernelGGL((band_moments_kernel<MMV, 8>), grid, dim3(256), lds, s, a);             \
    break;
    FFBIE_BAND_MM(X)
#undef X
  }
  return hipGetLastError();
}

hipError_t launch_band_solve(const BandArgs& a, hipStream_t s) {
  const unsigned blocks = (unsigned)((a.chunk_n + 63) / 64);
  switch (a.m0) {
#define X(M0V)                                                                                   \
  case M0V:                                                                                      \
    hipLaunchKernelGGL(band_solve_kernel<M0V>, dim3(blocks), dim3(64), 0, s, a);                 \
    break;
    X(1) X(2) X(3) X(4) X(5) X(6) X(7) X(8)
#undef X
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace ffbie
