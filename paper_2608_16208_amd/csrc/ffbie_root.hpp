// Root of rho^2 nearest to the real axis for one (target, source-curve) pair
// (paper Sec. 3.3, Lemma 3.6), plus A_0(b) and A_1(b) - A_0(b).  Host+device so
// the identical code runs in the root kernel and in host-side checks.
#pragma once
#include "ffbie_kernels.hpp"

namespace ffbie {

constexpr double kBFar = 3.0;        // b0 beyond which the quadratic-model root is used

// t, ts: curve parameters; j: target azimuth index in [0, 2M); tab: angle table.
// Returns the record and writes the FFBIE_PAIR_* bits to *status.
template <int MM, bool ST = false>
FFBIE_HD inline RootRec find_root(const Prob& P, const double* tab, double t, int j, double ts,
                                  int* status) {
  const int M = P.M, mask = P.tab_n - 1, quarter = 2 * M;
  const int J = 4 * j;
  PairGeo<MM> pg;
  pair_geo<MM>(P.g, t, ts, tab, J, mask, quarter, &pg);

  // (1) grid minimiser of rho^2 over the 2M azimuths theta_q = pi q / M.  Only
  //     the index of the smallest value is wanted, so rho^2 is expanded
  //     directly: with r_s = R_s(theta) w(theta), |w| = 1, and the target point
  //     r_t, rho^2 = R_s (R_s - 2 w . r_t) + |r_t|^2.  Its rounding error
  //     (~1e-16 absolute) only matters between grid values that agree to that
  //     level, where either is a valid start for the Newton steps below.  The
  //     angle values of theta_q are the same for every pair.
  //     On a surface stretched by D the same expansion reads
  //     rho^2 = R_s^2 |D w|^2 - 2 R_s (D w) . (D r_t) + |D r_t|^2.
  const double sj = tsin(tab, J, mask), cj = tcos(tab, J, mask, quarter);
  const double Rt = pg.R;
  constexpr bool scaled = ST;
  const double s2x = pg.sx * pg.sx, s2y = pg.sy * pg.sy, s2z = pg.sz * pg.sz;
  double wa = pg.sts * (Rt * pg.st * cj), wb = pg.sts * (Rt * pg.st * sj);
  double wc = pg.cts * (Rt * pg.ct);
  double Rt2 = Rt * Rt;
  if (scaled) {
    wa *= s2x;
    wb *= s2y;
    wc *= s2z;
    const double px = Rt * pg.st * cj, py = Rt * pg.st * sj, pz = Rt * pg.ct;
    Rt2 = fma(s2x * px, px, fma(s2y * py, py, s2z * pz * pz));
  }
  const double sts2 = pg.sts * pg.sts, cts2 = pg.cts * pg.cts;
  const double Rs0 = 1.0 + pg.al[0];
  double best = 1e300;
  int qbest = j;
  for (int q = 0; q < 2 * M; ++q) {
    const double cq = tcos(tab, 4 * q, mask, quarter), sq = tsin(tab, 4 * q, mask);
    double Rs = Rs0;
    if (MM >= 1) {
      double c_prev = 1.0, c_cur = cq;
#pragma unroll
      for (int m = 1; m <= MM; ++m) {
        if (m >= 2) {
          const double cn = 2.0 * cq * c_cur - c_prev;
          c_prev = c_cur;
          c_cur = cn;
        }
        Rs = fma(pg.al[m], c_cur, Rs);
      }
    }
    const double d = fma(wa, cq, fma(wb, sq, wc));
    double r2;
    if (!scaled) {
      r2 = fma(Rs, fma(-2.0, d, Rs), Rt2);
    } else {
      const double w2 = fma(sts2 * s2x, cq * cq, fma(sts2 * s2y, sq * sq, s2z * cts2));   // |D w|^2
      r2 = fma(Rs, fma(-2.0, d, Rs * w2), Rt2);
    }
    if (r2 < best) { best = r2; qbest = q; }
  }
  int dq = (qbest - j) & (2 * M - 1);
  if (dq > M) dq -= 2 * M;
  const double h = M_PI / M;
  double x = h * dq;

  double smj[MM + 1], cmj[MM + 1];
#pragma unroll
  for (int m = 0; m <= MM; ++m) {
    smj[m] = tsin(tab, m * J, mask);
    cmj[m] = tcos(tab, m * J, mask, quarter);
  }

  // (2) real minimiser a0 by Newton on d rho^2 / d theta_s, kept within the grid cell
  const double lo = x - h, hi = x + h;
  Rho2 r = rho2_complex<MM, ST>(pg, sj, cj, smj, cmj, mk(x, 0), true);
  for (int it = 0; it < 12; ++it) {
    const double f0 = r.f.re, g1 = r.f1.re, g2 = r.f2.re;
    if (!(g2 > 0)) break;
    const double step = g1 / g2;
    const double bscale = sqrt(fmax(2.0 * f0 / g2, 0.0));
    x = fmin(fmax(x - step, lo), hi);
    r = rho2_complex<MM, ST>(pg, sj, cj, smj, cmj, mk(x, 0), true);
    if (fabs(step) <= 1e-10 * bscale + 1e-300) break;
  }
  int st = 0;
  double b0;
  if (r.f2.re > 0 && r.f.re >= 0) {
    b0 = sqrt(2.0 * r.f.re / r.f2.re);
  } else {
    b0 = 1.0;
    st |= FFBIE_PAIR_ROOT_FALLBACK;
  }
  double u = x, b = b0;

  // (3) complex Newton for theta_+, started off the symmetry line Re = a0.
  //     For b0 >= kBFar the quadratic-model estimate itself parametrises the
  //     swap: s_{a,b} and the nearest zeros of rho^2 are then all far from the
  //     real axis, and the truncation test on the smooth factor decides.
  if (b0 >= kBFar && st == 0) st |= FFBIE_PAIR_FAR;
  if (b0 < kBFar && st == 0) {
    // the offset 0.2 b0 off the line: fewest Newton evaluations and fallbacks
    // among 0 .. 0.8 b0 on samples of config-2 pairs
    cplx z = mk(x + 0.2 * b0, b0);
    Rho2 e = rho2_complex<MM, ST>(pg, sj, cj, smj, cmj, z, false);
    bool conv = false;
    double sn_prev = 1e300;
    for (int it = 0; it < 40 && !conv; ++it) {
      const cplx step = cdiv(e.f, e.f1);
      const double sn = sqrt(abs2(step));
      if (!(sn == sn)) break;
      if (sn <= 1e-2 * z.im) {
        // quadratic regime: full Newton steps; stop once the step reaches the
        // rounding level of rho^2 (it no longer halves)
        z = z - step;
        if (sn <= 1e-14 * z.im || (sn <= 1e-11 * z.im && sn > 0.25 * sn_prev)) {
          conv = true;
          break;
        }
        sn_prev = sn;
        e = rho2_complex<MM, ST>(pg, sj, cj, smj, cmj, z, false);
        continue;
      }
      // far from the root: backtrack until Im z stays positive and |rho^2| decreases
      double lam = 1.0;
      bool ok = false;
      cplx zn = z;
      Rho2 en = e;
      for (int bt = 0; bt < 12; ++bt) {
        zn = z - lam * step;
        if (zn.im > 0.05 * z.im) {
          en = rho2_complex<MM, ST>(pg, sj, cj, smj, cmj, zn, false);
          if (sqrt(abs2(en.f)) <= (1.0 - 0.25 * lam) * sqrt(abs2(e.f))) { ok = true; break; }
        }
        lam *= 0.5;
      }
      if (!ok) break;
      z = zn;
      e = en;
    }
    if (conv && z.im > 0 && z.re == z.re && fabs(z.re) < 1e300) {
      u = z.re;
      b = z.im;
    } else {
      st |= FFBIE_PAIR_ROOT_FALLBACK;
    }
  }
  if (u > M_PI) u -= 2.0 * M_PI;
  if (u <= -M_PI) u += 2.0 * M_PI;

  // (4) A_0 = (2/pi) K(e^{-2b}),  A_1 - A_0 = (2/pi) (expm1(b) K - e^b E)
  double K, E;
  ellip_KE(exp(-2.0 * b), sqrt(-expm1(-2.0 * b)), &K, &E);
  const double A0 = M_2_PI * K;
  const double D1 = M_2_PI * (expm1(b) * K - exp(b) * E);
  // (5) the root-only values of the coefficient passes (see RootRec)
  double eb, omq, sh, ch, ur;
  int qu;
  root_exp_b(b, &eb, &omq);
  root_grid_offset(u, 2 * M, &qu, &ur);
  sincos_bounded(0.5 * ur, &sh, &ch);
  *status = st;
  return RootRec{u, b, A0, D1, eb, omq, sh, ch};
}

}  // namespace ffbie
