// Device-side building blocks for the singularity-swapping coefficient kernels
// (gfx950, wave64, FP64).
//
// Geometry: star family r(t,theta) = R(t,theta) (sin t cos theta, sin t sin theta,
// cos t), R = 1 + sum a_lm sin(l t) cos(m theta)  (paper Sec. 2, eq. (2.1)).
//
// The point difference r(t_s, theta_j + d) - r(t, theta_j) is evaluated with
// product-to-sum identities (sin x - sin y = 2 cos((x+y)/2) sin((x-y)/2), ...),
// which are exact algebraic rewrites with no subtraction of nearly equal
// quantities; this plays the role of the cancellation-free difference of the
// paper's Remark 4.2 at a fraction of the cost of its 16-node line integral.
// On the azimuth grid every angle is a multiple of pi/(4M), so its sine comes
// from an exactly rounded table.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "ffbie.h"

#define FFBIE_HD __host__ __device__

namespace ffbie {

constexpr int kMaxL = 8;       // highest l in the amplitude table
constexpr int kMaxM = 8;       // highest m in the amplitude table
constexpr int kWave = 64;

// Surface description passed by value as a kernel argument.
struct Geom {
  int lmax, mmax;
  double a[kMaxL][kMaxM + 1];
  double ax[3];    // stretch D = diag(ax) of the coordinates (1, 1, 1: the star itself)
  int scaled;      // ax differs from (1, 1, 1)
};

// Problem-wide constants for the coefficient kernels.
struct Prob {
  Geom g;
  double k;        // wavenumber
  double eps0;     // smooth-factor truncation threshold (eq. (3.13) rule)
  int M, M0, L;    // L = M + M0
  int tab_n;       // 8M: period of the angle table (entries sin(pi i / (4M)))
};

// ----------------------------------------------------------------------------
// complex double
// ----------------------------------------------------------------------------
struct cplx {
  double re, im;
};
FFBIE_HD __forceinline__ cplx mk(double r, double i) { return cplx{r, i}; }
FFBIE_HD __forceinline__ cplx operator+(cplx a, cplx b) { return {a.re + b.re, a.im + b.im}; }
FFBIE_HD __forceinline__ cplx operator-(cplx a, cplx b) { return {a.re - b.re, a.im - b.im}; }
FFBIE_HD __forceinline__ cplx operator*(cplx a, cplx b) {
  return {fma(a.re, b.re, -a.im * b.im), fma(a.re, b.im, a.im * b.re)};
}
FFBIE_HD __forceinline__ cplx operator*(double s, cplx a) { return {s * a.re, s * a.im}; }
FFBIE_HD __forceinline__ cplx operator*(cplx a, double s) { return {s * a.re, s * a.im}; }
FFBIE_HD __forceinline__ cplx conj(cplx a) { return {a.re, -a.im}; }
FFBIE_HD __forceinline__ double abs2(cplx a) { return fma(a.re, a.re, a.im * a.im); }
FFBIE_HD __forceinline__ cplx cdiv(cplx a, cplx b) {
  // Smith's algorithm
  if (fabs(b.re) >= fabs(b.im)) {
    double r = b.im / b.re, d = b.re + b.im * r;
    return {(a.re + a.im * r) / d, (a.im - a.re * r) / d};
  }
  double r = b.re / b.im, d = b.re * r + b.im;
  return {(a.re * r + a.im) / d, (a.im * r - a.re) / d};
}

// ----------------------------------------------------------------------------
// complex float: the spectral stage (transforms, truncation, convolutions) of
// the mixed-precision coefficient path
// ----------------------------------------------------------------------------
struct cplxf {
  float re, im;
};
FFBIE_HD __forceinline__ cplxf operator+(cplxf a, cplxf b) { return {a.re + b.re, a.im + b.im}; }
FFBIE_HD __forceinline__ cplxf operator-(cplxf a, cplxf b) { return {a.re - b.re, a.im - b.im}; }
FFBIE_HD __forceinline__ cplxf operator*(cplxf a, cplxf b) {
  return {fmaf(a.re, b.re, -a.im * b.im), fmaf(a.re, b.im, a.im * b.re)};
}
FFBIE_HD __forceinline__ cplxf operator*(float s, cplxf a) { return {s * a.re, s * a.im}; }
FFBIE_HD __forceinline__ cplxf conj(cplxf a) { return {a.re, -a.im}; }
FFBIE_HD __forceinline__ float abs2(cplxf a) { return fmaf(a.re, a.re, a.im * a.im); }

// Number types of the spectral stage: Spec<double> (FP64 path) or Spec<float>.
template <class R>
struct Spec;
template <>
struct Spec<double> {
  using C = cplx;
  FFBIE_HD static __forceinline__ cplx narrow(cplx z) { return z; }
  FFBIE_HD static __forceinline__ cplx wide(cplx z) { return z; }
};
template <>
struct Spec<float> {
  using C = cplxf;
  FFBIE_HD static __forceinline__ cplxf narrow(cplx z) { return {(float)z.re, (float)z.im}; }
  FFBIE_HD static __forceinline__ cplx wide(cplxf z) { return {(double)z.re, (double)z.im}; }
};
// sin and cos of a real argument with |x| <= 2^19 pi (all arguments on this
// path are bounded: k rho, multiples of grid offsets, curve parameters).
// Cody-Waite reduction x = q pi/2 + r, with pi/2 split into three parts of which
// the first two have 33 significant bits (q * part is exact for |q| < 2^20),
// then the Taylor series of sin (to r^17) and cos (to r^16) on |r| <= pi/4,
// whose truncation errors are below 1e-19 and 3e-18.  The split and the
// coefficients 1/n! were evaluated in 50-digit arithmetic.
// fma for polynomial steps c + a b with a constant coefficient c: on the
// device one three-address v_fma_f64 (the same single rounding as fma) that
// takes c from an SGPR pair, where the compiler's two-address v_fmac_f64 form
// would first copy a register-held constant into the destination.  c must be
// the same in every lane (a literal): an SGPR operand holds one value per
// wavefront.
FFBIE_HD __forceinline__ double poly_fma(double a, double b, double c) {
#if defined(__HIP_DEVICE_COMPILE__)
  double d;
  asm("v_fma_f64 %0, %1, %2, %3" : "=v"(d) : "v"(a), "v"(b), "s"(c));
  return d;
#else
  return fma(a, b, c);
#endif
}

// sin and cos of the reduced argument r (|r| <= pi/4) rotated by q quarter turns
FFBIE_HD __forceinline__ void sincos_quadrant(double r, int q, double* s, double* c);

FFBIE_HD __forceinline__ void sincos_bounded(double x, double* s, double* c) {
  const double qf = rint(x * 0.6366197723675814);           // x * 2/pi
  double r = fma(-qf, 1.5707963267341256, x);
  r = fma(-qf, 6.077100506303966e-11, r);
  r = fma(-qf, 2.0222662487959506e-21, r);
  sincos_quadrant(r, static_cast<int>(static_cast<long long>(qf) & 3), s, c);
}

// The same with the quadrant from one 32-bit conversion instead of a 64-bit
// one, for the arguments of the coefficient passes' inner steps (the sampled
// phases k rho and the swap phases n ur), which stay far inside that bound.
FFBIE_HD __forceinline__ void sincos_moderate(double x, double* s, double* c) {
  const double qf = rint(x * 0.6366197723675814);           // x * 2/pi
  double r = fma(-qf, 1.5707963267341256, x);
  r = fma(-qf, 6.077100506303966e-11, r);
  r = fma(-qf, 2.0222662487959506e-21, r);
  sincos_quadrant(r, static_cast<int>(qf) & 3, s, c);
}

FFBIE_HD __forceinline__ void sincos_quadrant(double r, int q, double* s, double* c) {
  const double r2 = r * r;
  double ps = 2.8114572543455206e-15;                         // 1/17!
  ps = poly_fma(ps, r2, -7.647163731819816e-13);                  // -1/15!
  ps = poly_fma(ps, r2, 1.6059043836821613e-10);                  //  1/13!
  ps = poly_fma(ps, r2, -2.505210838544172e-08);                  // -1/11!
  ps = poly_fma(ps, r2, 2.7557319223985893e-06);                  //  1/9!
  ps = poly_fma(ps, r2, -0.0001984126984126984);                  // -1/7!
  ps = poly_fma(ps, r2, 0.008333333333333333);                    //  1/5!
  ps = poly_fma(ps, r2, -0.16666666666666666);                    // -1/3!
  const double sr = fma(ps * r2, r, r);
  double pc = 4.779477332387385e-14;                          // 1/16!
  pc = poly_fma(pc, r2, -1.1470745597729725e-11);                 // -1/14!
  pc = poly_fma(pc, r2, 2.08767569878681e-09);                    //  1/12!
  pc = poly_fma(pc, r2, -2.755731922398589e-07);                  // -1/10!
  pc = poly_fma(pc, r2, 2.48015873015873e-05);                    //  1/8!
  pc = poly_fma(pc, r2, -0.001388888888888889);                   // -1/6!
  pc = poly_fma(pc, r2, 0.041666666666666664);                    //  1/4!
  pc = poly_fma(pc, r2, -0.5);                                    // -1/2!
  const double cr = fma(pc, r2, 1.0);
  const double ss = (q & 1) ? cr : sr;
  const double cc = (q & 1) ? sr : cr;
  *s = (q & 2) ? -ss : ss;
  *c = ((q + 1) & 2) ? -cc : cc;
}

// sin and cos of a complex argument x + iy
FFBIE_HD __forceinline__ void csincos(cplx z, cplx* s, cplx* c) {
  double sx, cx;
  sincos_bounded(z.re, &sx, &cx);
  if (z.im == 0.0) {
    // real argument (sinh 0 = 0, cosh 0 = 1), the same values without expm1
    *s = {sx, cx * 0.0};
    *c = {cx, -sx * 0.0};
    return;
  }
  // sinh via expm1 keeps full relative accuracy for small |Im z|
  const double em = expm1(z.im), emm = expm1(-z.im);
  const double sh = 0.5 * (em - emm);
  const double ch = 1.0 + 0.5 * (em + emm);
  *s = {sx * ch, cx * sh};
  *c = {cx * ch, -sx * sh};
}

// ----------------------------------------------------------------------------
// Angle table: tab[i] = sin(pi i / (4M)), i in [0, 8M).  cos via +2M.
// ----------------------------------------------------------------------------
FFBIE_HD __forceinline__ double tsin(const double* tab, int i, int mask) { return tab[i & mask]; }
FFBIE_HD __forceinline__ double tcos(const double* tab, int i, int mask, int quarter) {
  return tab[(i + quarter) & mask];
}

// ----------------------------------------------------------------------------
// Per-pair geometry.  Written as trigonometric polynomials in the source
// azimuth, with coefficients that depend on (t, t_s) only:
//   R(t_s, th)            = 1 + sum_m al_m cos(m th),   al_m = sum_l a_lm sin(l t_s)
//   R(t_s, th) - R(t, tj) = sum_m be_m cos(m th) + ga_m (cos(m th) - cos(m tj)),
//                           be_m = sum_l a_lm (sin(l t_s) - sin(l t)),  ga_m = sum_l a_lm sin(l t)
// with sin(l t_s) - sin(l t) = 2 cos(l (t_s+t)/2) sin(l (t_s-t)/2) (no cancellation).
// MM is a compile-time bound on the highest azimuthal order m of the surface.
// ----------------------------------------------------------------------------
template <int MM>
struct PairGeo {
  double st, ct, sts, cts;    // sin t, cos t, sin t_s, cos t_s
  double S1, C1;              // sin t_s - sin t, cos t_s - cos t (product forms)
  double R;                   // R(t, theta_j)
  double al[MM + 1], be[MM + 1], ga[MM + 1];
  double sx, sy, sz;          // the stretch D (read only by the stretched instantiations)
};

// A value that is the same in every lane of the wavefront, moved to SGPRs:
// VALU instructions read it from there as their scalar operand, so it holds
// no VGPR while it stays live.
FFBIE_HD __forceinline__ double to_uniform(double v) {
#if defined(__HIP_DEVICE_COMPILE__)
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readfirstlane((int)u);
  const int hi = __builtin_amdgcn_readfirstlane((int)(u >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
#else
  return v;
#endif
}

// The per-pair geometry of one wavefront's pair (the same in every lane) in
// SGPRs.
template <int MM>
FFBIE_HD __forceinline__ void pair_geo_uniform(PairGeo<MM>* p) {
  p->st = to_uniform(p->st); p->ct = to_uniform(p->ct);
  p->sts = to_uniform(p->sts); p->cts = to_uniform(p->cts);
  p->S1 = to_uniform(p->S1); p->C1 = to_uniform(p->C1);
  p->R = to_uniform(p->R);
#pragma unroll
  for (int m = 0; m <= MM; ++m) {
    p->al[m] = to_uniform(p->al[m]);
    p->be[m] = to_uniform(p->be[m]);
    p->ga[m] = to_uniform(p->ga[m]);
  }
  p->sx = to_uniform(p->sx); p->sy = to_uniform(p->sy); p->sz = to_uniform(p->sz);
}

// R(t, theta_j) = 1 + sum_m ga_m cos(m theta_j), theta_j at table index J.
template <int MM>
FFBIE_HD __forceinline__ void pair_geo_R(const double* tab, int J, int mask, int quarter,
                                         PairGeo<MM>* p) {
  double R = 1.0;
#pragma unroll
  for (int m = 0; m <= MM; ++m) R = fma(p->ga[m], tab[(m * J + quarter) & mask], R);
  p->R = R;
}

template <int MM>
FFBIE_HD __forceinline__ void pair_geo(const Geom& g, double t, double ts, const double* tab,
                                         int J, int mask, int quarter, PairGeo<MM>* p) {
  double st, ct, sts, cts, shd, chd, shs, chs;
  sincos_bounded(t, &st, &ct);
  sincos_bounded(ts, &sts, &cts);
  sincos_bounded(0.5 * (ts - t), &shd, &chd);
  sincos_bounded(0.5 * (ts + t), &shs, &chs);
  p->st = st; p->ct = ct; p->sts = sts; p->cts = cts;
  p->sx = g.ax[0]; p->sy = g.ax[1]; p->sz = g.ax[2];
  p->S1 = 2.0 * chs * shd;
  p->C1 = -2.0 * shs * shd;
#pragma unroll
  for (int m = 0; m <= MM; ++m) { p->al[m] = 0.0; p->be[m] = 0.0; p->ga[m] = 0.0; }
  // multiple angles by the Chebyshev recurrences (accurate for small arguments)
  double s_t0 = 0.0, s_t1 = st, s_s0 = 0.0, s_s1 = sts;
  double sd0 = 0.0, sd1 = shd, cs0 = 1.0, cs1 = chs;
  for (int l = 1; l <= g.lmax; ++l) {
    const double Sl = 2.0 * cs1 * sd1;
#pragma unroll
    for (int m = 0; m <= MM; ++m) {
      const double a = (m <= g.mmax) ? g.a[l - 1][m] : 0.0;
      p->al[m] = fma(a, s_s1, p->al[m]);
      p->be[m] = fma(a, Sl, p->be[m]);
      p->ga[m] = fma(a, s_t1, p->ga[m]);
    }
    double nt = 2.0 * ct * s_t1 - s_t0;  s_t0 = s_t1; s_t1 = nt;
    double ns = 2.0 * cts * s_s1 - s_s0; s_s0 = s_s1; s_s1 = ns;
    double nd = 2.0 * chd * sd1 - sd0;   sd0 = sd1;   sd1 = nd;
    double nc = 2.0 * chs * cs1 - cs0;   cs0 = cs1;   cs1 = nc;
  }
  pair_geo_R<MM>(tab, J, mask, quarter, p);
}

// Delta r = r(t_s, theta_q) - r(t, theta_j) from the trigonometric values of
// the grid angles: cq, sq = cos, sin theta_q; dh, cD = sin, cos of
// (theta_q - theta_j)/2; sS, cS = sin, cos of (theta_q + theta_j)/2.
// ST: the surface is stretched by D (the differences are scaled by it); the
// unstretched instantiation carries no trace of D.
template <int MM, bool ST = false>
FFBIE_HD __forceinline__ void dr_values(const PairGeo<MM>& p, double cq, double sq, double dh, double cD,
                                        double sS, double cS, double* dx, double* dy, double* dz) {
  const double dcos = -2.0 * sS * dh;   // cos theta_q - cos theta_j
  const double dsin = 2.0 * cS * dh;    // sin theta_q - sin theta_j
  double dR = p.be[0];
  if (MM >= 1) {
    // cos(m theta_q), sin(m hs), sin(m hd) by the Chebyshev recurrences
    double c_prev = 1.0, c_cur = cq;
    double s_prev = 0.0, s_cur = sS;
    double d_prev = 0.0, d_cur = dh;
#pragma unroll
    for (int m = 1; m <= MM; ++m) {
      if (m >= 2) {
        const double cn = 2.0 * cq * c_cur - c_prev;
        const double sn = 2.0 * cS * s_cur - s_prev;
        const double dn = 2.0 * cD * d_cur - d_prev;
        c_prev = c_cur; c_cur = cn;
        s_prev = s_cur; s_cur = sn;
        d_prev = d_cur; d_cur = dn;
      }
      // cos(m theta_q) - cos(m theta_j) = -2 sin(m hs) sin(m hd)
      const double dc = -2.0 * s_cur * d_cur;
      dR = fma(p.be[m], c_cur, fma(p.ga[m], dc, dR));
    }
  }
  const double wx = p.sts * cq, wy = p.sts * sq, wz = p.cts;
  const double ox = fma(p.S1, cq, p.st * dcos);
  const double oy = fma(p.S1, sq, p.st * dsin);
  const double oz = p.C1;
  *dx = fma(dR, wx, p.R * ox);
  *dy = fma(dR, wy, p.R * oy);
  *dz = fma(dR, wz, p.R * oz);
  if constexpr (ST) {
    *dx *= p.sx;
    *dy *= p.sy;
    *dz *= p.sz;
  }
}

// Delta r for a source azimuth on the table grid: Kq = table index of theta_q,
// J = table index of theta_j (both even).
template <int MM, bool ST = false>
FFBIE_HD __forceinline__ void dr_grid(const PairGeo<MM>& p, const double* tab, int Kq, int J,
                                      int mask, int quarter, double* dx, double* dy, double* dz) {
  const int hd = (Kq - J) >> 1;      // (theta_q - theta_j)/2
  const int hs = (Kq + J) >> 1;      // (theta_q + theta_j)/2
  dr_values<MM, ST>(p, tcos(tab, Kq, mask, quarter), tsin(tab, Kq, mask), tsin(tab, hd, mask),
                MM >= 2 ? tcos(tab, hd, mask, quarter) : 0.0, tsin(tab, hs, mask),
                tcos(tab, hs, mask, quarter), dx, dy, dz);
}

// rho^2 and its first two derivatives in the source azimuth at a complex
// offset d (source azimuth theta_j + d).  sj, cj = sin/cos(theta_j);
// smj[m], cmj[m] = sin/cos(m theta_j).  Used by the root finder.
struct Rho2 {
  cplx f, f1, f2;
};

template <int MM, bool ST = false>
FFBIE_HD __forceinline__ Rho2 rho2_complex(const PairGeo<MM>& p, double sj, double cj,
                                             const double* smj, const double* cmj, cplx d,
                                             bool want2) {
  cplx h = 0.5 * d, sh, ch;
  csincos(h, &sh, &ch);
  // source azimuth theta' = theta_j + 2h
  const cplx cd = ch * ch - sh * sh, sd = 2.0 * (sh * ch);
  const cplx cq = cj * cd - sj * sd, sq = sj * cd + cj * sd;
  // mid angle theta_j + h
  const cplx smid = sj * ch + cj * sh, cmid = cj * ch - sj * sh;
  const cplx dcos = -2.0 * (smid * sh), dsin = 2.0 * (cmid * sh);
  cplx Rs = mk(1, 0), dR = mk(0, 0), Rth = mk(0, 0), Rthth = mk(0, 0);
  // sin(m h), cos(m h) by the Chebyshev recurrences
  cplx s_prev = mk(0, 0), c_prev = mk(1, 0), s_cur = sh, c_cur = ch;
#pragma unroll
  for (int m = 0; m <= MM; ++m) {
    cplx smh, cmh;
    if (m == 0) { smh = mk(0, 0); cmh = mk(1, 0); }
    else if (m == 1) { smh = sh; cmh = ch; }
    else {
      const cplx sn = 2.0 * (ch * s_cur) - s_prev, cn = 2.0 * (ch * c_cur) - c_prev;
      s_prev = s_cur; c_prev = c_cur; s_cur = sn; c_cur = cn;
      smh = sn; cmh = cn;
    }
    // m theta' = m theta_j + 2 m h
    const cplx c2 = cmh * cmh - smh * smh, s2 = 2.0 * (smh * cmh);
    const cplx cmq = cmj[m] * c2 - smj[m] * s2;
    const cplx smq = smj[m] * c2 + cmj[m] * s2;
    const cplx smm = smj[m] * cmh + cmj[m] * smh;   // sin(m (theta_j + h))
    const cplx dcm = -2.0 * (smm * smh);            // cos(m theta') - cos(m theta_j)
    Rs = Rs + p.al[m] * cmq;
    dR = dR + p.be[m] * cmq + p.ga[m] * dcm;
    Rth = Rth + (-p.al[m] * m) * smq;
    Rthth = Rthth + (-p.al[m] * m * m) * cmq;
  }
  const cplx wx = p.sts * cq, wy = p.sts * sq, wz = mk(p.cts, 0);
  const cplx ox = p.S1 * cq + p.st * dcos, oy = p.S1 * sq + p.st * dsin, oz = mk(p.C1, 0);
  // D (1 unless ST) scales the difference and its azimuthal derivatives
  const double gx = ST ? p.sx : 1.0, gy = ST ? p.sy : 1.0, gz = ST ? p.sz : 1.0;
  cplx Dx = dR * wx + p.R * ox, Dy = dR * wy + p.R * oy, Dz = dR * wz + p.R * oz;
  // r_theta(t_s, theta') = D (R_theta w + Rs w_theta),  w_theta = (-sts sin, sts cos, 0)
  cplx tx = Rth * wx - Rs * (p.sts * sq), ty = Rth * wy + Rs * (p.sts * cq), tz = Rth * wz;
  if constexpr (ST) {
    Dx = gx * Dx; Dy = gy * Dy; Dz = gz * Dz;
    tx = gx * tx; ty = gy * ty; tz = gz * tz;
  }
  Rho2 out;
  out.f = Dx * Dx + Dy * Dy + Dz * Dz;
  out.f1 = 2.0 * (Dx * tx + Dy * ty + Dz * tz);
  if (want2) {
    // r_thth = D (R_thth w + 2 R_th w_th + Rs w_thth),  w_thth = (-sts cos, -sts sin, 0)
    const cplx ux = gx * (Rthth * wx - 2.0 * (Rth * (p.sts * sq)) - Rs * (p.sts * cq));
    const cplx uy = gy * (Rthth * wy + 2.0 * (Rth * (p.sts * cq)) - Rs * (p.sts * sq));
    const cplx uz = gz * (Rthth * wz);
    out.f2 = 2.0 * (tx * tx + ty * ty + tz * tz + Dx * ux + Dy * uy + Dz * uz);
  } else {
    out.f2 = mk(0, 0);
  }
  return out;
}

// ----------------------------------------------------------------------------
// Complete elliptic integrals K(m), E(m) (parameter convention, m = e^{-2b})
// by the arithmetic-geometric mean, with sqrt(1 - m) supplied directly so that
// m -> 1 (b -> 0) keeps full relative accuracy.
// ----------------------------------------------------------------------------
FFBIE_HD inline void ellip_KE(double m, double sqrt_1m, double* K, double* E) {
  double a = 1.0, gm = sqrt_1m, c = sqrt(m);
  double sum = 0.5 * c * c, pw = 0.5;
  for (int it = 0; it < 40; ++it) {
    double an = 0.5 * (a + gm);
    c = 0.5 * (a - gm);
    gm = sqrt(a * gm);
    a = an;
    pw *= 2.0;
    sum = fma(pw, c * c, sum);
    if (c <= 1e-17 * a) break;
  }
  *K = M_PI / (2.0 * a);
  *E = *K * (1.0 - sum);
}

// ----------------------------------------------------------------------------
// Refined hardware estimates (device only)
// ----------------------------------------------------------------------------
// 1/sqrt(x) for x > 0: hardware estimate, then two Newton steps
// y <- y + (y/2)(1 - x y^2), each roughly squaring the relative error.
__device__ __forceinline__ double rsqrt_refined(double x) {
  double y = __builtin_amdgcn_rsq(x);
  double e = fma(-x * y, y, 1.0);
  y = fma(0.5 * y, e, y);
  e = fma(-x * y, y, 1.0);
  return fma(0.5 * y, e, y);
}

// sqrt(x) for a normal positive x (no denormal scaling, no zero or infinity
// handling): hardware 1/sqrt estimate y, g = x y and h = y/2 refined by one
// coupled Newton step, then two corrections g += (x - g^2) h.
__device__ __forceinline__ double sqrt_pos(double x) {
  const double y = __builtin_amdgcn_rsq(x);
  double g = x * y, h = 0.5 * y;
  const double r = fma(-g, h, 0.5);
  g = fma(g, r, g);
  h = fma(h, r, h);
  double d = fma(-g, g, x);
  g = fma(d, h, g);
  d = fma(-g, g, x);
  return fma(d, h, g);
}

__device__ __forceinline__ double rcp_refined(double x) {
  // 1/x for a normal positive x: hardware estimate + two Newton steps
  double r = __builtin_amdgcn_rcp(x);
  double e = fma(-x, r, 1.0);
  r = fma(r, e, r);
  e = fma(-x, r, 1.0);
  return fma(r, e, r);
}

// ----------------------------------------------------------------------------
// Wave-level helpers
// ----------------------------------------------------------------------------
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
  __builtin_amdgcn_wave_barrier();
}

// Wave reductions by DPP moves (no LDS traffic): inclusive scans inside each
// row of 16 lanes by shifts of 1, 2, 4, 8, then the last lane of row 2 into
// row 3 and the last lane of row 1 into row 3, so that lane 63 holds the
// reduction of all 64 lanes; it is then read as a uniform value.
// dpp_i32 / dpp_f64_fill: lanes without a source, or in rows that ROW_MASK
// does not write, keep `fill`.
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ int dpp_i32(int fill, int src) {
  return __builtin_amdgcn_update_dpp(fill, src, CTRL, ROW_MASK, 0xf, false);
}
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ double dpp_f64_fill(double fill, double src) {
  const long long f = __double_as_longlong(fill), u = __double_as_longlong(src);
  const int lo = dpp_i32<CTRL, ROW_MASK>((int)f, (int)u);
  const int hi = dpp_i32<CTRL, ROW_MASK>((int)(f >> 32), (int)(u >> 32));
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ float dpp_f32_fill(float fill, float src) {
  return __int_as_float(dpp_i32<CTRL, ROW_MASK>(__float_as_int(fill), __float_as_int(src)));
}
// The value of v in lane `l` (uniform l), as a uniform value.
__device__ __forceinline__ double read_lane(double v, int l) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)u, l), hi = __builtin_amdgcn_readlane((int)(u >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ double lane63(double v) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)u, 63), hi = __builtin_amdgcn_readlane((int)(u >> 32), 63);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
__device__ __forceinline__ float lane63(float v) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), 63));
}

// Moves for the reductions: every row is written and lanes without a source
// read 0 (bound_ctrl), so no old value has to be materialised.  Only lane 63's
// result is used: it is the sum (maximum) over all lanes whatever the row
// broadcasts leave in rows 0-2.
template <int CTRL>
__device__ __forceinline__ double dpp_zero(double v) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)u, CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_mov_dpp((int)(u >> 32), CTRL, 0xf, 0xf, true);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_zero(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xf, 0xf, true));
}
template <class T>
__device__ __forceinline__ T wave_sum_t(T v) {
  v += dpp_zero<0x111>(v);   // row_shr:1
  v += dpp_zero<0x112>(v);   // row_shr:2
  v += dpp_zero<0x114>(v);   // row_shr:4
  v += dpp_zero<0x118>(v);   // row_shr:8
  v += dpp_zero<0x142>(v);   // row_bcast:15
  v += dpp_zero<0x143>(v);   // row_bcast:31
  return lane63(v);
}
// maximum of nonnegative values (lanes without a source contribute 0)
template <class T>
__device__ __forceinline__ T wave_max_t(T v) {
  v = fmax(v, dpp_zero<0x111>(v));
  v = fmax(v, dpp_zero<0x112>(v));
  v = fmax(v, dpp_zero<0x114>(v));
  v = fmax(v, dpp_zero<0x118>(v));
  v = fmax(v, dpp_zero<0x142>(v));
  v = fmax(v, dpp_zero<0x143>(v));
  return lane63(v);
}
__device__ __forceinline__ double wave_sum(double v) { return wave_sum_t(v); }
__device__ __forceinline__ float wave_sum(float v) { return wave_sum_t(v); }
__device__ __forceinline__ double wave_max(double v) { return wave_max_t(v); }
__device__ __forceinline__ float wave_max(float v) { return wave_max_t(v); }

}  // namespace ffbie
