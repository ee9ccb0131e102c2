// Singularity-swapping coefficient kernels for gfx950.
//
// For a target r(t, theta_j) and a source curve t_s the path evaluates the
// azimuthal Fourier coefficients of the single-layer kernel e^{ik rho}/rho
// (paper Sec. 3.2-3.3).  With theta_+ = a + ib the root of rho^2 nearest to
// the real axis (Lemma 3.6), s_{a,b} of eq. (3.22) and the smooth factor
// F = (s_{a,b}/rho^2)^{1/2} of eq. (3.23):
//   <rho^-1>_l = sum_j <F>_j e^{-i(l-j)a} A_{|l-j|}(b)                     eq. (3.25)
// and, since cos(k rho) is analytic in rho^2, the same swap applied to the
// whole singular part cos(k rho)/rho = [F cos(k rho)] s_{a,b}^{-1/2} gives
//   <cos(k rho)/rho>_n = sum_j <F cos(k rho)>_j e^{-i(n-j)a} A_{|n-j|}(b),
// the construction the paper uses for tau_3 in eqs. (4.5)-(4.6).  This is the
// default path for the kernel coefficients; the double convolution of
// eq. (3.10) (<cos(k rho)>_n convolved with <rho^-1>_l) is kept as a variant.
// The smooth part <sin(k rho)/rho>_n comes from the same FFT.
//
// Kernel 1 (ffbie_root_kernel), one lane per pair: grid minimiser of rho^2,
//   Newton on d rho^2 for the real minimiser a0, b0 = sqrt(2 rho^2 / rho^2'')
//   (Sec. 3.3), damped complex Newton for theta_+, then K and E of parameter
//   e^{-2b} for A_0 and A_1.
// Kernel 2 (ffbie_coeff_kernel), one wavefront per pair: samples on the
//   azimuth grid, radix-2 Stockham FFT in LDS, truncation index p of
//   eq. (3.24), A_m(b) by a wave-parallel scan of the 2x2 transfer matrices of
//   Miller's backward recurrence (or of the difference recurrence (3.28) for
//   small b), the convolutions, and a coalesced row write.
#include "ffbie_kernels.hpp"
#include "ffbie_fft128.hpp"
#include "ffbie_root.hpp"

namespace ffbie {

constexpr double kTauFwd = 9.0;      // forward difference recurrence while m_max * b <= this
constexpr double kMillerStart = 1e-280;

__device__ __forceinline__ void load_table(double* tab, const double* __restrict__ tab_g, int n) {
  for (int i = threadIdx.x; i < n; i += blockDim.x) tab[i] = tab_g[i];
  __syncthreads();
}


// ===========================================================================
// Kernel 1: roots (lane per pair)
// ===========================================================================
// Surfaces of azimuthal order <= 2 ask for four wavefronts per SIMD: the
// order-2 kernel then keeps 12 VGPRs in scratch and still runs 5 % faster than
// at the three its 136 VGPRs would allow; higher orders are left to the
// compiler.
template <int MM, bool ST = false>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(MM <= 2 ? 4 : 1, MM <= 2 ? 4 : 8))) void ffbie_root_kernel_t(
    Prob P, const double* __restrict__ tab_g, int64_t n, const double* __restrict__ t_in,
    const int32_t* __restrict__ az_in, const double* __restrict__ ts_in, RootRec* __restrict__ out,
    int32_t* __restrict__ status, double* __restrict__ root_out) {
  extern __shared__ double tab[];
  load_table(tab, tab_g, P.tab_n);
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double t = t_in[i], ts = ts_in[i];
  const int j = az_in[i] & (2 * P.M - 1);
  const double nan = __builtin_nan("");
  if (t == ts || !(t == t) || !(ts == ts)) {
    out[i] = RootRec{nan, nan, nan, nan, nan, nan, nan, nan};
    status[i] = FFBIE_PAIR_SINGULAR;
    if (root_out) { root_out[2 * i] = nan; root_out[2 * i + 1] = nan; }
    return;
  }
  int st;
  const RootRec r = find_root<MM, ST>(P, tab, t, j, ts, &st);
  out[i] = r;
  status[i] = st;
  if (root_out) { root_out[2 * i] = r.u; root_out[2 * i + 1] = r.b; }
}

// ===========================================================================
// A_m(b), m = 0..mtop, into LDS `A`, cooperatively by one wavefront.
//
// For m_max b <= kTauFwd the difference recurrence of eq. (3.28) runs forward
// from A_0 and D_1; otherwise Miller's backward recurrence
//   (2m - 1) y_{m-1} = 4 m cosh(b) y_m - (2m + 1) y_{m+1}
// (the three-term recurrence of the half-integer Legendre functions of
// eq. (3.27)) starts at N >= (m_max + 37/b)/2 and is normalised by A_0.
// Either recurrence is a product of 2x2 transfer matrices: each lane forms the
// product over its own segment of indices, a scan across the 64 lanes (DPP
// row shifts and row broadcasts) composes the segments, and each lane then
// replays its segment from the state entering it.
// ===========================================================================
__device__ __forceinline__ void mat_mul(double a00, double a01, double a10, double a11, double b00,
                                        double b01, double b10, double b11, double* c00,
                                        double* c01, double* c10, double* c11) {
  *c00 = fma(a00, b00, a01 * b10);
  *c01 = fma(a00, b01, a01 * b11);
  *c10 = fma(a10, b00, a11 * b10);
  *c11 = fma(a10, b01, a11 * b11);
}

// One step of the lane scan: every lane multiplies its matrix on the right by
// the one the DPP pattern brings from a lower lane; lanes that the pattern
// gives no source (or whose row it does not write) receive the identity, so
// no per-lane select is needed.
// A diagonal entry moved by a row shift: lanes without a source read 1.0
// (low word 0 by bound_ctrl, high word kept from the fill).
template <int CTRL>
__device__ __forceinline__ double dpp_one(double v) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)u, CTRL, 0xf, 0xf, true);
  const int hi = __builtin_amdgcn_update_dpp(0x3ff00000, (int)(u >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
template <int CTRL, int ROW_MASK>
__device__ __forceinline__ void mat_scan_step(double& e00, double& e01, double& e10, double& e11) {
  double o00, o01, o10, o11;
  if constexpr (ROW_MASK == 0xf) {
    // row shifts: every row written, only missing sources need the identity
    o00 = dpp_one<CTRL>(e00); o01 = dpp_zero<CTRL>(e01);
    o10 = dpp_zero<CTRL>(e10); o11 = dpp_one<CTRL>(e11);
  } else {
    o00 = dpp_f64_fill<CTRL, ROW_MASK>(1.0, e00); o01 = dpp_f64_fill<CTRL, ROW_MASK>(0.0, e01);
    o10 = dpp_f64_fill<CTRL, ROW_MASK>(0.0, e10); o11 = dpp_f64_fill<CTRL, ROW_MASK>(1.0, e11);
  }
  double n00, n01, n10, n11;
  mat_mul(e00, e01, e10, e11, o00, o01, o10, o11, &n00, &n01, &n10, &n11);
  e00 = n00; e01 = n01; e10 = n10; e11 = n11;
}

// Inclusive scan of 2x2 matrices over the 64 lanes in lane order,
// E_l = X_l X_{l-1} ... X_0, with DPP moves instead of LDS permutes: shifts by
// 1, 2, 4, 8 inside each row of 16 lanes, then the last lane of row 0 (2) into
// row 1 (3) and the last lane of row 1 into rows 2 and 3.
__device__ __forceinline__ void mat_scan_lanes(double& e00, double& e01, double& e10, double& e11) {
  mat_scan_step<0x111, 0xf>(e00, e01, e10, e11);   // row_shr:1
  mat_scan_step<0x112, 0xf>(e00, e01, e10, e11);   // row_shr:2
  mat_scan_step<0x114, 0xf>(e00, e01, e10, e11);   // row_shr:4
  mat_scan_step<0x118, 0xf>(e00, e01, e10, e11);   // row_shr:8
  mat_scan_step<0x142, 0xa>(e00, e01, e10, e11);   // row_bcast:15 into rows 1 and 3
  mat_scan_step<0x143, 0xc>(e00, e01, e10, e11);   // row_bcast:31 into rows 2 and 3
}

// A is stored as R (double, or float on the mixed-precision path); the
// recurrences themselves always run in FP64.  eb = e^{-b} and omq = 1 - e^{-b}
// (from expm1) give the recurrence coefficients: 4 cosh b = 2 (1/eb + eb) and
// 8 sinh^2(b/2) = 2 omq^2 / eb, the latter free of cancellation at small b.
//
// Returns the factor by which A still has to be multiplied: 1, except on the
// FP64 Miller path with `defer` set, where the values stay as the recurrence
// left them and the caller applies A_0 / y_0 (to a linear function of A) itself.
template <class R, int CACHE = 1>
__device__ __forceinline__ double singular_factor_wave(double b, double eb, double omq, double A0,
                                                       double D1, int mtop, R* A, bool defer,
                                                       int lane) {
  if (!(b > 0) || !(A0 == A0)) {
    for (int m = lane; m <= mtop; m += 64) A[m] = (R)__builtin_nan("");
    wave_sync();
    return 1.0;
  }
  if (mtop == 0) {
    if (lane == 0) A[0] = (R)A0;
    wave_sync();
    return 1.0;
  }
  // Each lane keeps the coefficients of the first CACHE steps of its segment
  // from the product pass for the replay (with four, segments up to N = 256
  // need no step formed twice, which covers M <= 64); later steps are formed
  // again.  CACHE is what the calling kernel's register budget allows.
  constexpr int kStepCache = CACHE;
  double cal[kStepCache], cbe[kStepCache];
  if ((double)mtop * b <= kTauFwd) {
    // ---- forward: w_{m+1} = F_m w_m, w = (D, A),
    //      F_m = [[alpha, beta], [alpha, 1 + beta]], alpha = (2m-1)/(2m+1),
    //      beta = 8 m sinh^2(b/2)/(2m+1), for m = 1 .. mtop-1
    const double s2 = 2.0 * omq * omq / eb;
    const int cnt = mtop - 1;
    const int S = cnt > 0 ? (cnt + 63) / 64 : 1;
    const int m_first = 1 + lane * S;
    auto coef = [&](int m, double* al, double* be) {
      const double r = rcp_refined(2.0 * m + 1.0);
      *al = (2.0 * m - 1.0) * r;
      *be = s2 * m * r;
    };
    double e00 = 1, e01 = 0, e10 = 0, e11 = 1;
    auto product_step = [&](double al, double be) {
      // F_m E: the second row of F_m is its first plus (0, 1)
      const double n00 = fma(al, e00, be * e10), n01 = fma(al, e01, be * e11);
      e10 = n00 + e10;
      e11 = n01 + e11;
      e00 = n00;
      e01 = n01;
    };
#pragma unroll
    for (int s = 0; s < kStepCache; ++s) {
      const int m = m_first + s;
      if (s < S && m <= mtop - 1) {
        coef(m, &cal[s], &cbe[s]);
        product_step(cal[s], cbe[s]);
      }
    }
    for (int s = kStepCache; s < S; ++s) {
      const int m = m_first + s;
      if (m > mtop - 1) break;
      double al, be;
      coef(m, &al, &be);
      product_step(al, be);
    }
    // inclusive prefix scan: E_l = Phi_l ... Phi_0
    mat_scan_lanes(e00, e01, e10, e11);
    // exclusive: E_{l-1} by a DPP wave shift right by one lane, identity in lane 0
    const double x00 = dpp_f64_fill<0x138, 0xf>(1.0, e00), x01 = dpp_f64_fill<0x138, 0xf>(0.0, e01);
    const double x10 = dpp_f64_fill<0x138, 0xf>(0.0, e10), x11 = dpp_f64_fill<0x138, 0xf>(1.0, e11);
    const double w1D = D1, w1A = A0 + D1;
    double wD = fma(x00, w1D, x01 * w1A), wA = fma(x10, w1D, x11 * w1A);
    auto replay_step = [&](int m, double al, double be) {
      const double nD = fma(al, wD, be * wA);
      wA = wA + nD;
      wD = nD;
      A[m + 1] = (R)wA;
    };
#pragma unroll
    for (int s = 0; s < kStepCache; ++s) {
      const int m = m_first + s;
      if (s < S && m <= mtop - 1) replay_step(m, cal[s], cbe[s]);
    }
    for (int s = kStepCache; s < S; ++s) {
      const int m = m_first + s;
      if (m > mtop - 1) break;
      double al, be;
      coef(m, &al, &be);
      replay_step(m, al, be);
    }
    if (lane == 0) { A[0] = (R)A0; A[1] = (R)(A0 + D1); }
    wave_sync();
    return 1.0;
  }
  // ---- Miller, backward: v_{m-1} = T_m v_m, v_m = (y_m, y_{m+1}),
  //      T_m = [[4 m cosh b/(2m-1), -(2m+1)/(2m-1)], [1, 0]], m = N .. 1
  int meff = mtop;
  int N = max(mtop + 10, (int)ceil(0.5 * (mtop + 37.0 * rcp_refined(b))) + 10);
  if (b * N > 640.0) {
    // the recurrence would leave the double range; A_m < e^{-630} A_0 is set to 0
    N = (int)floor(640.0 / b);
    meff = min(mtop, max(0, N - 10));
    if (N < 1) {   // b > 640: A_m / A_0 < 1e-270 for every m >= 1
      for (int m = lane; m <= mtop; m += 64) A[m] = (R)((m == 0) ? A0 : 0.0);
      wave_sync();
      return 1.0;
    }
  }
  const double ch4 = 2.0 * (rcp_refined(eb) + eb);
  const int S = (N + 63) / 64;
  // segment g = 63 - lane (the highest indices in lane 0), so that the suffix
  // products over segments are prefix products in lane order; step s of the
  // segment is the transition m = top - s
  const int seg = 63 - lane;
  const int top = seg * S + S;      // segment: transitions m = top .. seg*S + 1
  auto coef = [&](int m, double* al, double* be) {
    const double r = rcp_refined(2.0 * m - 1.0);
    *al = ch4 * m * r;
    *be = -(2.0 * m + 1.0) * r;
  };
  double p00 = 1, p01 = 0, p10 = 0, p11 = 1;
  auto product_step = [&](double al, double be) {
    // T_m P with T_m = [[al, be], [1, 0]]: the second row of the product is
    // the first row of P
    const double n00 = fma(al, p00, be * p10), n01 = fma(al, p01, be * p11);
    p10 = p00;
    p11 = p01;
    p00 = n00;
    p01 = n01;
  };
#pragma unroll
  for (int s = 0; s < kStepCache; ++s) {
    const int m = top - s;
    if (s < S && m <= N) {
      coef(m, &cal[s], &cbe[s]);
      product_step(cal[s], cbe[s]);
    }
  }
  for (int s = kStepCache; s < S; ++s) {
    const int m = top - s;
    if (m > N) continue;
    double al, be;
    coef(m, &al, &be);
    product_step(al, be);
  }
  // inclusive suffix scan over segments: Q_g = P_g P_{g+1} ... P_63
  mat_scan_lanes(p00, p01, p10, p11);
  const double q00 = dpp_f64_fill<0x138, 0xf>(1.0, p00), q10 = dpp_f64_fill<0x138, 0xf>(0.0, p10);
  // state entering the segment: Q_{g+1} (y_s, 0)
  double y0 = q00 * kMillerStart, y1 = q10 * kMillerStart;   // (y_top, y_top+1)
  // y_{m-1} = al y_m + be y_{m+1}; store(m - 1, y_{m-1})
  auto replay = [&](auto store) {
#pragma unroll
    for (int s = 0; s < kStepCache; ++s) {
      const int m = top - s;
      if (s < S && m <= N) {
        const double yn = fma(cal[s], y0, cbe[s] * y1);
        y1 = y0;
        y0 = yn;
        store(m - 1, yn);
      }
    }
    for (int s = kStepCache; s < S; ++s) {
      const int m = top - s;
      if (m > N) continue;
      double al, be;
      coef(m, &al, &be);
      const double yn = fma(al, y0, be * y1);
      y1 = y0;
      y0 = yn;
      store(m - 1, yn);
    }
  };
  if constexpr (sizeof(R) == sizeof(double)) {
    // store the unnormalised values, then scale by A_0 / y_0 with y_0 as replayed
    replay([&](int m, double y) { if (m <= mtop) A[m] = y; });
    wave_sync();
    const double scale = A0 * rcp_refined(A[0]);
    if (defer && meff == mtop) return scale;
    wave_sync();
    for (int m = lane; m <= mtop; m += 64) A[m] = (m <= meff) ? A[m] * scale : 0.0;
  } else {
    // the unnormalised values leave the float range: lane 63 holds the whole
    // product Q_0, so y_0 = Q_0[0][0] y_N fixes the normalisation first
    const double scale = A0 / (lane63(p00) * kMillerStart);
    replay([&](int m, double y) { if (m <= mtop) A[m] = (R)((m <= meff) ? y * scale : 0.0); });
    for (int m = N + lane; m <= mtop; m += 64) A[m] = (R)0.0;
  }
  wave_sync();
  return 1.0;
}

// ===========================================================================
// Spectral stage, generic over the complex type C (cplx, or cplxf on the
// mixed-precision path); R is its real type.
//
// Forward DFT X_n = sum_q x_q e^{-2 pi i q n / NF} of one or two sequences,
// radix-2 Stockham autosort in LDS.  On return ia/ib hold the transforms and
// oa/ob are free.
// ===========================================================================
template <class C>
__device__ __forceinline__ void fft_stockham(C*& ia, C*& oa, C*& ib, C*& ob, bool two, int NF, int M,
                                             const double* tab, int mask, int quarter, int lane) {
  using R = decltype(C::re);
  const int half = NF >> 1;
  for (int Ns = 1; Ns < NF; Ns <<= 1) {
    for (int jj = lane; jj < half; jj += 64) {
      const int r = jj & (Ns - 1);
      const int tk = r * ((4 * M) / Ns);            // angle pi r / Ns
      const C wt = C{(R)tcos(tab, tk, mask, quarter), (R)-tsin(tab, tk, mask)};
      const int idxD = ((jj - r) << 1) + r;
      const C v0 = ia[jj], v1 = ia[jj + half] * wt;
      oa[idxD] = v0 + v1;
      oa[idxD + Ns] = v0 - v1;
      if (two) {
        const C u0 = ib[jj], u1 = ib[jj + half] * wt;
        ob[idxD] = u0 + u1;
        ob[idxD + Ns] = u0 - u1;
      }
    }
    wave_sync();
    C* tmp = ia; ia = oa; oa = tmp;
    tmp = ib; ib = ob; ob = tmp;
  }
}

// Twiddle factors of a transform of NF <= 128 points, one entry per (stage,
// lane): at stage Ns = 2^st the butterfly jj = lane uses e^{-i pi r / Ns},
// r = jj mod Ns.  Built once per workgroup into LDS, read with one
// conflict-free load per butterfly.
constexpr int kTwiddleStages = 7;

// Twiddles e^{-2 pi i k / NF} per (stage, lane), entry st * 64 + lane.  The
// Stockham layout holds, for stage Ns = 2^st, k = (lane mod Ns) NF / (2 Ns).
// The layout of fft128_regs (NF = 128) holds the factor by which lane `lane`
// multiplies at stage st (see there).
template <class C>
__device__ __forceinline__ void build_twiddles(C* tw, int NF, int M, const double* tab, int mask,
                                               int quarter, bool reg_layout = false) {
  using R = decltype(C::re);
  for (int idx = threadIdx.x; idx < kTwiddleStages * 64; idx += blockDim.x) {
    const int st = idx >> 6, lane = idx & 63;
    int tk;
    if (!reg_layout) {
      const int Ns = 1 << st;
      const int r = lane & (Ns - 1);
      tk = (Ns < NF) ? r * ((4 * M) / Ns) : 0;
    } else {
      tk = fft128_twiddle_k(st, lane) * ((8 * M) / NF);   // angle 2 pi k / 128 on the table
    }
    tw[idx] = C{(R)tcos(tab, tk, mask, quarter), (R)-tsin(tab, tk, mask)};
  }
}


// Forward DFT as fft_stockham for NF <= 128 with the twiddles of build_twiddles.
template <class C>
__device__ __forceinline__ void fft_stockham_small(C*& ia, C*& oa, C*& ib, C*& ob, bool two, int NF,
                                                   const C* tw, int lane) {
  const int half = NF >> 1;
  for (int st = 0; (1 << st) < NF; ++st) {
    const int Ns = 1 << st;
    if (lane < half) {
      const int jj = lane;
      const int r = jj & (Ns - 1);
      const C wt = tw[(st << 6) + lane];
      const int idxD = ((jj - r) << 1) + r;
      const C v0 = ia[jj], v1 = ia[jj + half] * wt;
      oa[idxD] = v0 + v1;
      oa[idxD + Ns] = v0 - v1;
      if (two) {
        const C u0 = ib[jj], u1 = ib[jj + half] * wt;
        ob[idxD] = u0 + u1;
        ob[idxD + Ns] = u0 - u1;
      }
    }
    wave_sync();
    C* tmp = ia; ia = oa; oa = tmp;
    tmp = ib; ib = ob; ob = tmp;
  }
}

// Forward DFT by radix-4 Stockham stages, with one radix-2 stage at the end
// when log2(NF) is odd.  Stage Ns (Ns = 1, 4, 16, ...): butterfly jj < NF/4
// takes x_{jj + r NF/4} w^r (r = 0..3, w = e^{-2 pi i s / (4 Ns)}, s = jj mod Ns),
// forms their 4-point DFT and writes it to jj' + r Ns, jj' = 4 (jj - s) + s.
// w comes from the radix-2 twiddle table when one is given (entry s of the
// stage 2 Ns), else from the angle table; w^2 and w^3 by multiplication.
template <class C>
__device__ __forceinline__ void fft_stockham_r4(C*& ia, C*& oa, C*& ib, C*& ob, bool two, int NF, int M,
                                                const double* tab, int mask, int quarter, const C* tw,
                                                int lane) {
  using R = decltype(C::re);
  const int q4 = NF >> 2;
  int Ns = 1, st2 = 1;                 // st2 = log2(2 Ns)
  for (; 4 * Ns <= NF; Ns <<= 2, st2 += 2) {
    for (int jj = lane; jj < q4; jj += 64) {
      const int s = jj & (Ns - 1);
      C w1;
      if (tw) {
        w1 = tw[(st2 << 6) + s];
      } else {
        const int tk = s * ((2 * M) / Ns);       // angle pi s / (2 Ns)
        w1 = C{(R)tcos(tab, tk, mask, quarter), (R)-tsin(tab, tk, mask)};
      }
      const C w2 = w1 * w1, w3 = w2 * w1;
      const int idxD = ((jj - s) << 2) + s;
      {
        const C v0 = ia[jj], v1 = ia[jj + q4] * w1, v2 = ia[jj + 2 * q4] * w2, v3 = ia[jj + 3 * q4] * w3;
        const C s02 = v0 + v2, d02 = v0 - v2, s13 = v1 + v3, d13 = v1 - v3;
        const C md13 = C{d13.im, -d13.re};      // -i (v1 - v3)
        oa[idxD] = s02 + s13;
        oa[idxD + Ns] = d02 + md13;
        oa[idxD + 2 * Ns] = s02 - s13;
        oa[idxD + 3 * Ns] = d02 - md13;
      }
      if (two) {
        const C v0 = ib[jj], v1 = ib[jj + q4] * w1, v2 = ib[jj + 2 * q4] * w2, v3 = ib[jj + 3 * q4] * w3;
        const C s02 = v0 + v2, d02 = v0 - v2, s13 = v1 + v3, d13 = v1 - v3;
        const C md13 = C{d13.im, -d13.re};
        ob[idxD] = s02 + s13;
        ob[idxD + Ns] = d02 + md13;
        ob[idxD + 2 * Ns] = s02 - s13;
        ob[idxD + 3 * Ns] = d02 - md13;
      }
    }
    wave_sync();
    C* tmp = ia; ia = oa; oa = tmp;
    tmp = ib; ib = ob; ob = tmp;
  }
  if (Ns < NF) {                       // NF = 2 Ns: a last radix-2 stage
    const int half = NF >> 1;
    for (int jj = lane; jj < half; jj += 64) {
      const int r = jj & (Ns - 1);
      C wt;
      if (tw) {
        wt = tw[((st2 - 1) << 6) + lane];
      } else {
        const int tk = r * ((4 * M) / Ns);      // angle pi r / Ns
        wt = C{(R)tcos(tab, tk, mask, quarter), (R)-tsin(tab, tk, mask)};
      }
      const int idxD = ((jj - r) << 1) + r;
      const C v0 = ia[jj], v1 = ia[jj + half] * wt;
      oa[idxD] = v0 + v1;
      oa[idxD + Ns] = v0 - v1;
      if (two) {
        const C u0 = ib[jj], u1 = ib[jj + half] * wt;
        ob[idxD] = u0 + u1;
        ob[idxD + Ns] = u0 - u1;
      }
    }
    wave_sync();
    C* tmp = ia; ia = oa; oa = tmp;
    tmp = ib; ib = ob; ob = tmp;
  }
}

// Coefficient j of the real sequence packed in the real part of the
// transform X: (X_j + conj(X_{NF-j})) / (2 NF).
template <class C>
__device__ __forceinline__ C real_part_coeff(const C* X, int jj, int NF, decltype(C::re) invNF) {
  return (decltype(C::re))(0.5 * invNF) * (X[jj & (NF - 1)] + conj(X[(NF - jj) & (NF - 1)]));
}
// Coefficient j of the real sequence packed in the imaginary part:
// (X_j - conj(X_{NF-j})) / (2i NF).
template <class C>
__device__ __forceinline__ C imag_part_coeff(const C* X, int jj, int NF, decltype(C::re) invNF) {
  const C d = (decltype(C::re))(0.5 * invNF) * (X[jj & (NF - 1)] - conj(X[(NF - jj) & (NF - 1)]));
  return C{d.im, -d.re};
}

// Truncation index of a real sequence's coefficients (the rule of eq. (3.13)
// applied as for eq. (3.24)): the highest j < NF/2 with |c_j| > eps * scale,
// where scale = max(max_j |c_j|, ref).  `ref` lets the coefficients of
// F cos(k rho) be measured against the size of F itself: |cos(k rho)| <= 1, and
// where cos(k rho) averages out its coefficients are small while the rounding
// floor still follows F.
template <class C>
__device__ __forceinline__ int trunc_index_real(const C* X, int NF, decltype(C::re) invNF, double eps,
                                                double ref, int lane) {
  using R = decltype(C::re);
  R maxv = 0;
  for (int jj = lane; jj < NF / 2; jj += 64) maxv = fmax(maxv, abs2(real_part_coeff(X, jj, NF, invNF)));
  maxv = fmax(wave_max(maxv), (R)(ref * ref));
  const R thr = (R)(eps * eps) * maxv;
  int p = 0;
  for (int jj = lane; jj < NF / 2; jj += 64) {
    const uint64_t bal = __ballot(abs2(real_part_coeff(X, jj, NF, invNF)) > thr);
    if (bal) p = max(p, (jj - lane) + 63 - __clzll(bal));
  }
  return __builtin_amdgcn_readfirstlane(p);
}

// out_n = s e^{-i n a} sum_{|j| <= p} G_j A_{|n-j|} for n = 0..nmax, s the
// factor A still carries.  The phases are FP64: ph holds e^{i n a} for
// n = lane and ph64 = e^{i 64 a}.  Output 0 is one real dot product: G_0 is
// real (the mean of a real sequence, phase 1) and the j and -j terms pair to
// 2 Re G_j A_j.  Outputs n = 1..nmax are spread over the lanes (n = lane + 1
// + 64 i, phase e^{i (lane + 1) a} e^{i 64 a}^i); when their count exceeds a
// multiple of 64 by a few, those last outputs are summed cooperatively (terms
// over lanes, then a wave sum) instead of costing the whole wave another pass,
// with the phase read from the lane that holds it.
// G is Hermitian, G[p - j] = conj(G[p + j]), so the j and -j terms share G_j:
//   sum_j G_j A_{|n-j|} = G_0 A_n + sum_{j >= 1} [Re G_j (A_{|n-j|} + A_{n+j})
//                                               + i Im G_j (A_{|n-j|} - A_{n+j})]
// (the sum of eq. (3.25)).  A must be mirrored: A[-m] = A[m] for m <= p.
template <class C>
__device__ __forceinline__ void swap_convolution(const C* G, int p, const decltype(C::re)* A, int nmax,
                                                 cplx ph, cplx ph64, double scale, C* out, C* mirror,
                                                 C* global_row, int lane) {
  using R = decltype(C::re);
  using SP = Spec<R>;
  const C* Gp = G + p;           // Gp[j], j = -p..p
  {
    R acc0 = 0;
    for (int jj = lane; jj <= p; jj += 64) acc0 = fma(jj == 0 ? Gp[0].re : (R)2 * Gp[jj].re, A[jj], acc0);
    acc0 = wave_sum(acc0);
    if (lane == 0) {
      const C c = SP::narrow(mk(scale * (double)acc0, 0.0));
      out[0] = c;
      if (global_row) global_row[0] = c;
    }
  }
  const int cnt = nmax;          // outputs 1..nmax
  const int rem = cnt & 63;
  const int split = (cnt > 64 && rem <= 4) ? cnt - rem : cnt;
  ph = ph * mk(read_lane(ph.re, 1), read_lane(ph.im, 1)) * scale;   // e^{i (lane + 1) a} s
  for (int i = lane; i < split; i += 64) {
    const int n = i + 1;
    const R An0 = A[n];
    R accr = Gp[0].re * An0, acci = Gp[0].im * An0, accr2 = 0, acci2 = 0;
    int j = 1;
#pragma unroll 2
    for (; j + 1 <= p; j += 2) {
      const C g = Gp[j], g2 = Gp[j + 1];
      const R lo = A[n - j], hi = A[n + j], lo2 = A[n - j - 1], hi2 = A[n + j + 1];
      accr = fma(g.re, lo + hi, accr);
      acci = fma(g.im, lo - hi, acci);
      accr2 = fma(g2.re, lo2 + hi2, accr2);
      acci2 = fma(g2.im, lo2 - hi2, acci2);
    }
    if (j <= p) {
      const C g = Gp[j];
      const R lo = A[n - j], hi = A[n + j];
      accr = fma(g.re, lo + hi, accr);
      acci = fma(g.im, lo - hi, acci);
    }
    accr += accr2;
    acci += acci2;
    const C c = SP::narrow(conj(ph) * mk(accr, acci));
    out[n] = c;
    if (mirror) mirror[-n] = conj(c);
    if (global_row) global_row[n] = c;
    ph = ph * ph64;
  }
  // split < cnt only when split is a multiple of 64: every lane ran split / 64
  // passes, so lane t holds the phase of output split + 1 + t
  for (int i = split; i < cnt; ++i) {
    const int n = i + 1;
    R accr = 0, acci = 0;
    for (int jj = -p + lane; jj <= p; jj += 64) {
      const C g = Gp[jj];
      const R Av = A[n - jj];
      accr = fma(g.re, Av, accr);
      acci = fma(g.im, Av, acci);
    }
    accr = wave_sum(accr);
    acci = wave_sum(acci);
    const cplx phn = mk(read_lane(ph.re, i - split), read_lane(ph.im, i - split));
    if (lane == 0) {
      const C c = SP::narrow(conj(phn) * mk(accr, acci));
      out[n] = c;
      if (mirror) mirror[-n] = conj(c);
      if (global_row) global_row[n] = c;
    }
  }
}

// ===========================================================================
// Kernel 2: coefficients (one wavefront per pair)
//
// LDS per wave: NF-complex buffers z1a, z1b (FFT ping-pong), then either A_m
// and kc (compact layout) or z2a, z2b (and cb, 2L+1 complex, for eq. (3.10)).
// After the FFT, Z1 (and Z2) hold transforms and free1/free2 are free:
//   default path:   Z1 = FFT(F cos(k rho) + i sin(k rho)/rho); GH -> free1;
//                   no <rho^-1>: A -> after z1b, kc -> cb after A;
//                   <rho^-1>: Z2 = FFT(F), GF -> free2, A -> Z2, <rho^-1> -> the
//                   output row, kc -> free2 (after the first convolution)
//   eq. (3.10):     Z1 = FFT(F + i cos(k rho)), Z2 = FFT(sin(k rho)/rho)
//                   C -> free1, GF -> free2, A -> Z1, <rho^-1> -> cb, kc -> free2
// ===========================================================================
// The coefficient path for the pairs w in [beg, end) of one problem, by one
// wavefront (indices into a.list when it is set).  `tab` is the problem's angle
// table in LDS, `tw` its FFT twiddles in LDS (NF <= 128) or null, `wbase` this
// wavefront's LDS workspace, NF the sample count.  R is the real type of the
// spectral stage (transforms, truncation, A_m storage, convolutions, outputs):
// double, or float for the mixed-precision path; geometry, samples, the root
// and the recurrences for A_m run in FP64 either way.
template <int MM, bool REFINE, class R, int RADIX, bool ST = false>
__device__ __forceinline__ void coeff_range(const CoeffArgs& a, const double* tab,
                                            const typename Spec<R>::C* tw, double* wbase, int NF,
                                            int64_t beg, int64_t end) {
  using C = typename Spec<R>::C;
  using SP = Spec<R>;
  const Prob& P = a.P;
  const int M = P.M, M0 = P.M0, L = P.L, mask = P.tab_n - 1, quarter = 2 * M;
  const int lane0 = threadIdx.x & 63;
  const bool paper = a.variant == FFBIE_KAPPA_PAPER_CONV;
  const bool want_c = paper || a.rhoinv != nullptr;
  // the 128-point transforms in registers where the twiddles are laid out for
  // them
  const bool reg_fft = RADIX == 2 && NF == 128 && tw != nullptr;
  C* base = reinterpret_cast<C*>(wbase);
  C* z1a = base;
  C* z1b = z1a + NF;
  // transforms / full layout: z2a, z2b (and cb, full); compact layout: A_m
  // buffer and kc
  C* z2a = z1b + NF;
  C* z2b = z2a + NF;
  C* cb = paper ? z2b + NF : z1b + NF + (M + NF + 2) / 2;
  R* Acompact = reinterpret_cast<R*>(z1b + NF);
  C* kappa = static_cast<C*>(a.kappa);
  C* rhoinv = static_cast<C*>(a.rhoinv);

  const int tstride = (8 * M) / NF;        // table index step of the sample grid
  const int hstep = (4 * M) / NF;          // table index step of half a grid step
  const double nan = __builtin_nan("");
  const double k = P.k;
  const R invNF = (R)1 / (R)NF;
  // sin(k rho)/rho <= k is packed beside F cos(k rho) = O(1) in one transform;
  // it is scaled by an exact power of two near 1/k so that its size does not
  // raise the rounding floor of the other sequence's coefficients
  const int kexp = (k > 1.0) ? (int)ceil(log2(k)) : 0;
  const double s_down = ldexp(1.0, -kexp);
  const R s_up = (R)ldexp(1.0, kexp);

  const double inv_NF = 1.0 / NF;
  double t_prev = nan, ts_prev = nan;
  PairGeo<MM> pg;

  for (int64_t w = beg; w < end; ++w) {
    // The lane index is made opaque once per pair so that lane-derived
    // constants (LDS and global addresses, transform signs and indices) are
    // formed where they are used rather than hoisted out of this loop and held,
    // or spilled, throughout it.
    int lane = lane0;
    asm volatile("" : "+v"(lane));
    const int64_t pi = a.list ? a.list[w] : w;
    const double t = a.t_in[pi], ts = a.ts_in[pi];
    const int j = a.az_in[pi] & (2 * M - 1);
    const RootRec rr = load_root(a.roots, pi);
    int st = a.status[pi] & ((1 << FFBIE_PAIR_P_SHIFT) - 1);
    C* krow = kappa + pi * (int64_t)(2 * M);
    C* crow = rhoinv ? rhoinv + pi * (int64_t)(L + 1) : nullptr;
    if (st & FFBIE_PAIR_SINGULAR) {
      for (int c = lane; c < 2 * M; c += 64) krow[c] = C{(R)nan, (R)nan};
      if (crow)
        for (int c = lane; c <= L; c += 64) crow[c] = C{(R)nan, (R)nan};
      continue;
    }
    const int J = 4 * j;
    if (!(t == t_prev && ts == ts_prev)) {
      pair_geo<MM>(P.g, t, ts, tab, J, mask, quarter, &pg);
      t_prev = t; ts_prev = ts;
    } else {
      pair_geo_R<MM>(tab, J, mask, quarter, &pg);
    }
    const double b = rr.b;
    // a = theta_j + qu * (2 pi / NF) + ur,  |ur| <= pi / NF; e^{-b}, 1 - e^{-b}
    // and, on the 2M-point grid of the main pass, sin and cos of ur/2 come
    // with the root record
    int qu;
    double ur, sur, cur;
    root_grid_offset(rr.u, NF, &qu, &ur);
    if constexpr (!REFINE) {
      sur = rr.sh;
      cur = rr.ch;
    } else {
      sincos_bounded(0.5 * ur, &sur, &cur);
    }
    const double eb = rr.eb, omq = rr.omq;
    const int qj = j * (NF / (2 * M));

    // ---- samples on the NF-point grid: sample(q, z1, z2) gives the inputs of
    //      the transforms (z2 only where a second transform is taken)
    double sumF = 0.0;
    auto sample = [&](int q, C& z1, C& z2) {
      double dx, dy, dz;
      dr_grid<MM, ST>(pg, tab, q * tstride, J, mask, quarter, &dx, &dy, &dz);
      const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
      const double ri = rsqrt_refined(r2);      // 1/rho
      const double rho = r2 * ri;
      double skr, ckr;
      sincos_moderate(k * rho, &skr, &ckr);
      const int hidx = (q - qj - qu) * hstep;   // (theta_q - a)/2 = hidx pi/(4M) - ur/2
      const double sh = fma(tsin(tab, hidx, mask), cur, -tcos(tab, hidx, mask, quarter) * sur);
      const double s = fma(omq, omq, 4.0 * eb * sh * sh);
      const double F = sqrt_pos(s) * ri;       // s >= (1 - e^{-b})^2 > 0
      const double S = (k == 0.0) ? 0.0 : skr * ri;
      sumF += F;
      if (paper) {
        z1 = C{(R)F, (R)ckr};
        z2 = C{(R)S, (R)0};
      } else {
        z1 = C{(R)(F * ckr), (R)(S * s_down)};
        z2 = C{(R)F, (R)0};
      }
    };
    C *Z1 = z1a, *free1 = z1b, *Z2 = z2a, *free2 = z2b;
    // With the transforms in registers the lane's two samples are the
    // bit-reversed positions lane and lane + 64 (samples 2 brev6(lane) + i) and
    // stay in registers (those of a second transform wait in the lane's own
    // slots of z2a); otherwise sample q = lane + 64 i goes to LDS.
    const int fl = lane;
    const int q0 = (int)(__builtin_bitreverse32((unsigned)fl) >> 25);
    C a0, a1;
#pragma unroll 1
    for (int i = 0; i < (reg_fft ? 2 : (NF + 63) / 64); ++i) {
      const int q = reg_fft ? q0 + i : lane + 64 * i;
      if (q < NF) {
        C z1, z2;
        sample(q, z1, z2);
        if (reg_fft) {
          if (i == 0) a0 = z1; else a1 = z1;
          if (want_c) z2a[fl + 64 * i] = z2;
        } else {
          z1a[q] = z1;
          if (want_c) z2a[q] = z2;
        }
      }
    }
    if (reg_fft) {
      fft128_regs(a0, a1, tw, fl);
      const int o = fft128_out_index(fl);
      z1a[o] = a0;
      z1a[o + 64] = a1;
      if (want_c) {
        // every lane has read its own two samples before any lane stores
        // (the transform's cross-lane steps run in lockstep)
        a0 = z2a[fl];
        a1 = z2a[fl + 64];
        fft128_regs(a0, a1, tw, fl);
        z2a[o] = a0;
        z2a[o + 64] = a1;
      }
      wave_sync();
    } else {
      wave_sync();
      // at NF = 128 the radix-2 twiddle table is in the register layout
      if constexpr (RADIX == 4)
        fft_stockham_r4(Z1, free1, Z2, free2, want_c, NF, M, tab, mask, quarter, tw, lane);
      else if (tw && NF != 128)
        fft_stockham_small(Z1, free1, Z2, free2, want_c, NF, tw, lane);
      else
        fft_stockham(Z1, free1, Z2, free2, want_c, NF, M, tab, mask, quarter, lane);
    }

    // truncation indices of the smooth factors.  With one transform and
    // NF <= 128 lane j holds coefficient j < NF/2 of the smooth factor, kept
    // for the coefficient vector below.
    const C* Fsrc = paper ? Z1 : Z2;
    const double F0 = wave_sum(sumF) * inv_NF;  // <F>_0 = max_j |<F>_j| since F > 0
    const bool one_tf = !paper && !want_c && NF <= 128;
    C c_own = C{(R)0, (R)0};
    int pH;
    if (one_tf) {
      if (lane < NF / 2) c_own = real_part_coeff(Z1, lane, NF, invNF);
      const R a2 = abs2(c_own);
      const R maxv = fmax(wave_max(a2), (R)(F0 * F0));
      const uint64_t bal = __ballot(a2 > (R)(P.eps0 * P.eps0) * maxv);
      pH = __builtin_amdgcn_readfirstlane(bal ? 63 - __clzll(bal) : 0);
    } else {
      pH = paper ? 0 : trunc_index_real(Z1, NF, invNF, P.eps0, F0, lane);
    }
    const int pF = want_c ? trunc_index_real(Fsrc, NF, invNF, P.eps0, 0.0, lane) : 0;
    if (max(pF, pH) >= NF / 2 - 2) {
      if (!REFINE && a.flag_list) {
        // not resolved on this grid: queue for the 4M-sample pass
        if (lane == 0) {
          const int32_t slot = atomicAdd(a.flag_count, 1);
          a.flag_list[slot] = pi | a.flag_tag;
          a.status[pi] = st | FFBIE_PAIR_REFINED;
        }
        continue;
      }
      st |= FFBIE_PAIR_UNRESOLVED;
    }
    const int Jq = J + qu * tstride;          // table index of theta_j + qu * gstep

    // ---- weighted coefficient vectors G_j = <f>_j e^{i j a}, |j| <= p
    C* GF = free2;
    C* GH = free1;
    C* Cn = free1 + (M0 - 1);
    const int pmax = max(pF, pH);
    // e^{i n a} for n = lane (table part times e^{i n ur}) and e^{i 64 a} =
    // (e^{i 32 a})^2, shared by the coefficient vectors and the convolutions
    cplx ph_lane, ph64;
    {
      double s1, c1;
      sincos_moderate(lane * ur, &s1, &c1);
      ph_lane = mk(tcos(tab, lane * Jq, mask, quarter), tsin(tab, lane * Jq, mask)) * mk(c1, s1);
      const cplx h = mk(read_lane(ph_lane.re, 32), read_lane(ph_lane.im, 32));
      ph64 = h * h;
    }
    cplx ph = ph_lane;
    for (int jj = lane; jj <= pmax; jj += 64, ph = ph * ph64) {
      if (want_c && jj <= pF) {
        const C G = SP::narrow(SP::wide(real_part_coeff(Fsrc, jj, NF, invNF)) * ph);
        GF[pF + jj] = G;
        GF[pF - jj] = conj(G);
      }
      if (!paper && jj <= pH) {
        const C G = SP::narrow(SP::wide(one_tf ? c_own : real_part_coeff(Z1, jj, NF, invNF)) * ph);
        GH[pH + jj] = G;
        GH[pH - jj] = conj(G);
      }
    }
    if (paper) {
      // <cos(k rho)>_n, |n| <= M0 - 1, from the imaginary part of Z1
      for (int n = lane; n < M0; n += 64) {
        const C Cv = imag_part_coeff(Z1, n, NF, invNF);
        Cn[n] = Cv;
        Cn[-n] = conj(Cv);
      }
    }
    wave_sync();
    // ---- A_m(b)
    R* A = (paper ? reinterpret_cast<R*>(Z1) : (want_c ? reinterpret_cast<R*>(Z2) : Acompact)) +
           NF / 2;
    const int mtop = paper ? L + pF : (want_c ? max(L + pF, M + pH) : M + pH);
    // on the FP64 path A may come back unnormalised: its factor rides on the
    // phases of the convolutions, which are linear in A
    // four cached recurrence steps fit the FP64 kernels of low azimuthal order
    constexpr int kCache = (sizeof(R) == sizeof(double) && MM <= 2) ? 4 : 1;
    const double asc = singular_factor_wave<R, kCache>(b, eb, omq, rr.A0, rr.D1, mtop, A, true, lane);
    for (int m = 1 + lane; m <= max(pF, pH); m += 64) A[-m] = A[m];
    wave_sync();

    // ---- <rho^-1>_l, l = 0..L (eq. (3.25)): for eq. (3.10) into cb[L + l]
    //      (and cb[L - l] = conj), otherwise straight to the output row
    if (paper) {
      swap_convolution<C>(GF, pF, A, L, ph_lane, ph64, asc, cb + L, cb + L, crow, lane);
      wave_sync();
    } else if (want_c) {
      swap_convolution<C>(GF, pF, A, L, ph_lane, ph64, asc, crow, nullptr, nullptr, lane);
      // kc below overwrites GF's buffer (free2), read across lanes above: the
      // wavefront-scope fence keeps the compiler from moving those stores
      // before the other lanes' loads
      wave_sync();
    }
    // ---- kc_n = <cos(k rho)/rho>_n, n = 0..M
    C* kc = want_c ? free2 : cb;
    if (paper) {
      // eq. (3.10): kc_n = sum_{|n'| < M0} C_{n'} c_{n-n'}
      for (int n = lane; n < M; n += 64) {
        R accr = 0, acci = 0;
        for (int np = -(M0 - 1); np <= M0 - 1; ++np) {
          const C Cv = Cn[np];
          const C c = cb[L + n - np];
          accr = fma(Cv.re, c.re, fma(-Cv.im, c.im, accr));
          acci = fma(Cv.re, c.im, fma(Cv.im, c.re, acci));
        }
        kc[n] = C{accr, acci};
      }
      R accr = 0, acci = 0;
      for (int np = -(M0 - 1) + lane; np <= M0 - 1; np += 64) {
        const C Cv = Cn[np];
        const C c = cb[L + M - np];
        accr = fma(Cv.re, c.re, fma(-Cv.im, c.im, accr));
        acci = fma(Cv.re, c.im, fma(Cv.im, c.re, acci));
      }
      accr = wave_sum(accr);
      acci = wave_sum(acci);
      if (lane == 0) kc[M] = C{accr, acci};
    } else {
      // swap applied to cos(k rho)/rho
      swap_convolution<C>(GH, pH, A, M, ph_lane, ph64, asc, kc, nullptr, nullptr, lane);
    }
    wave_sync();
    // ---- kappa_n = kc_n + i <sin(k rho)/rho>_n, n = -M+1..M at column n + M - 1
    for (int c = lane; c < 2 * M; c += 64) {
      const int n = c - M + 1;
      const C kcn = n >= 0 ? kc[n] : conj(kc[-n]);
      const C Sn = paper ? invNF * Z2[n & (NF - 1)] : s_up * imag_part_coeff(Z1, n, NF, invNF);
      krow[c] = C{kcn.re - Sn.im, kcn.im + Sn.re};
    }
    if (lane == 0) a.status[pi] = st | (min(paper ? pF : pH, 0xfff) << FFBIE_PAIR_P_SHIFT);
    wave_sync();
  }
}

// Wavefronts per SIMD asked of the coefficient kernels.  This file is built
// without machine-level loop-invariant hoisting, so the pair loop recomputes
// cheap invariants instead of holding them (or the SGPR pairs of the sincos
// coefficients) in registers: the FP64 kernel for surfaces of azimuthal order
// <= 4 then fits the 128 VGPRs of four wavefronts without spilling, order 8
// the 168 of three, and the FP32 spectral stage for order <= 2 the 96 of five.
template <int MM, class R>
constexpr int coeff_waves_per_simd() {
  return sizeof(R) == 4 && MM <= 2 ? 5 : (MM <= 4 ? 4 : 3);
}
// The persistent batch kernel, whose loop over work items holds more
// registers, asks for fewer.
template <int MM>
constexpr int coeff_persist_waves_per_simd() {
  return MM <= 4 ? 3 : 2;
}

template <int MM, bool REFINE, class R, int RADIX, bool ST = false>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(coeff_waves_per_simd<MM, R>(), coeff_waves_per_simd<MM, R>()))) void ffbie_coeff_kernel_t(
    CoeffArgs a) {
  using C = typename Spec<R>::C;
  constexpr bool single = sizeof(R) == 4;
  extern __shared__ double smem[];
  double* tab = smem;
  load_table(tab, a.tab_g, a.P.tab_n);
  const int twd = coeff_twiddle_doubles(a.NF, single);
  C* tw = twd ? reinterpret_cast<C*>(smem + a.P.tab_n) : nullptr;
  if (tw) {
    build_twiddles(tw, a.NF, a.P.M, tab, a.P.tab_n - 1, 2 * a.P.M, RADIX == 2 && a.NF == 128);
    __syncthreads();
  }
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int waves_per_block = blockDim.x >> 6;
  const bool want_c = a.variant == FFBIE_KAPPA_PAPER_CONV || a.rhoinv != nullptr;
  const int layout = a.variant == FFBIE_KAPPA_PAPER_CONV ? kLdsFull
                     : (a.rhoinv != nullptr ? kLdsTransforms : kLdsCompact);
  const int per_wave = coeff_lds_per_wave(a.NF, a.P.M, a.P.L, layout, single);
  int64_t count = a.n;
  if (a.list) count = *a.list_count;
  const int64_t total_waves = (int64_t)gridDim.x * waves_per_block;
  const int64_t gw = (int64_t)blockIdx.x * waves_per_block + wave;
  const int64_t chunk = (count + total_waves - 1) / total_waves;
  const int64_t beg = gw * chunk, end = min(count, beg + chunk);
  coeff_range<MM, REFINE, R, RADIX, ST>(a, tab, tw, smem + a.P.tab_n + twd + (size_t)wave * per_wave,
                                        a.NF, beg, end);
}

// ===========================================================================
// Batched coefficient path: many problems (surfaces, panel counts, k) of one
// M in one launch.  The angle table and the FFT twiddles depend only on M, so
// each workgroup stages them once.  Work items are runs of b.tile consecutive
// pairs of one problem, numbered problem by problem.  PERSIST: each wavefront
// takes the next item from a global counter on its own (no workgroup barrier
// between items) and leaves once the counter passes the last item; otherwise
// the grid has one wavefront per item and the hardware dispatcher balances
// the load (no loop around the pair loop, so nothing held across items).
// ===========================================================================
__device__ __forceinline__ int batch_find(const int64_t* __restrict__ prefix, int n, int64_t x) {
  int lo = 0, hi = n - 1;                     // last problem with prefix[s] <= x
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (prefix[mid] <= x) lo = mid; else hi = mid - 1;
  }
  return lo;
}

template <int MM, class R, int RADIX, bool PERSIST>
__global__ __launch_bounds__(256)
__attribute__((amdgpu_waves_per_eu(PERSIST ? coeff_persist_waves_per_simd<MM>() : coeff_waves_per_simd<MM, R>(),
                                   PERSIST ? coeff_persist_waves_per_simd<MM>() : coeff_waves_per_simd<MM, R>()))) void
ffbie_coeff_batch_kernel_t(
    BatchArgs b) {
  using C = typename Spec<R>::C;
  constexpr bool single = sizeof(R) == 4;
  extern __shared__ double smem[];
  const CoeffArgs& a0 = b.probs[0];
  const int M = a0.P.M, NF = 2 * M;
  load_table(smem, a0.tab_g, a0.P.tab_n);
  C* tw = coeff_twiddle_doubles(NF, single) ? reinterpret_cast<C*>(smem + b.tab_max) : nullptr;
  if (tw) {
    build_twiddles(tw, NF, M, smem, a0.P.tab_n - 1, 2 * M, RADIX == 2 && NF == 128);
    __syncthreads();
  }
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int per_wave = coeff_lds_per_wave(NF, M, a0.P.L, kLdsCompact, single);
  double* wbase = smem + b.tab_max + b.tw_max + (size_t)wave * per_wave;
  auto run_item = [&](int64_t item) {
    const int s = batch_find(b.item_prefix, b.n_probs, item);
    const CoeffArgs& a = b.probs[s];
    const int64_t t0 = (item - b.item_prefix[s]) * b.tile;
    const int64_t beg = min(a.n, t0), end = min(a.n, t0 + b.tile);
    coeff_range<MM, false, R, RADIX>(a, smem, tw, wbase, NF, beg, end);
  };
  if constexpr (PERSIST) {
    while (true) {
      int64_t item = 0;
      if ((threadIdx.x & 63) == 0) item = atomicAdd(b.item_counter, 1);
      item = __shfl(item, 0);
      if (item >= b.n_items) break;
      run_item(item);
    }
  } else {
    const int64_t item = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave;
    if (item < b.n_items) run_item(item);
  }
}

// Refine pass of the problems [b.prob_lo, b.prob_hi) (one M) of a batch:
// queue entries are (problem << 40 | pair) over the whole batch; each
// wavefront walks the queue with the grid's stride and takes the entries of
// its problems.
template <int MM, class R>
__global__ __launch_bounds__(256) void ffbie_coeff_batch_refine_t(BatchArgs b) {
  extern __shared__ double smem[];
  const CoeffArgs& a0 = b.probs[b.prob_lo];
  load_table(smem, a0.tab_g, a0.P.tab_n);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int waves_per_block = blockDim.x >> 6;
  const int NF = 4 * a0.P.M;
  double* wbase = smem + b.tab_max +
                  (size_t)wave * coeff_lds_per_wave(NF, a0.P.M, a0.P.L, kLdsCompact, sizeof(R) == 4);
  const int count = *b.flag_count;
  const int stride = gridDim.x * waves_per_block;
  for (int w = blockIdx.x * waves_per_block + wave; w < count; w += stride) {
    const int64_t e = b.flag_list[w];
    const int s = (int)(e >> 40);
    if (s < b.prob_lo || s >= b.prob_hi) continue;
    const int64_t pi = e & ((int64_t(1) << 40) - 1);
    coeff_range<MM, true, R, 2>(b.probs[s], smem, nullptr, wbase, NF, pi, pi + 1);
  }
}

// Zeroes n ints (work counters before a launch; a kernel, so that the launch
// sequence can be captured in a graph).
__global__ void ffbie_zero_kernel(int* p, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0;
}

// Root kernel of a batch: one lane per pair, blocks of 256 pairs of one problem.
template <int MM>
__global__ __launch_bounds__(256) void ffbie_root_batch_kernel_t(BatchArgs b) {
  extern __shared__ double tab[];
  const int s = batch_find(b.root_prefix, b.n_probs, blockIdx.x);
  const CoeffArgs& a = b.probs[s];
  load_table(tab, a.tab_g, a.P.tab_n);
  const int64_t i = (blockIdx.x - b.root_prefix[s]) * (int64_t)blockDim.x + threadIdx.x;
  if (i >= a.n) return;
  const double t = a.t_in[i], ts = a.ts_in[i];
  const int j = a.az_in[i] & (2 * a.P.M - 1);
  const double nan = __builtin_nan("");
  RootRec* out = const_cast<RootRec*>(a.roots);
  if (t == ts || !(t == t) || !(ts == ts)) {
    out[i] = RootRec{nan, nan, nan, nan, nan, nan, nan, nan};
    a.status[i] = FFBIE_PAIR_SINGULAR;
    return;
  }
  int st;
  const RootRec r = find_root<MM>(a.P, tab, t, j, ts, &st);
  out[i] = r;
  a.status[i] = st;
}

// ===========================================================================
// Diagnostic kernel: A_m(b) for a batch of b (one wavefront per b)
// ===========================================================================
__global__ __launch_bounds__(256) void ffbie_singular_factor_kernel(int64_t n,
                                                                    const double* __restrict__ b_in,
                                                                    int mtop, double* __restrict__ out) {
  extern __shared__ double smem[];
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  double* A = smem + (size_t)wave * (mtop + 1);
  const int64_t idx = (int64_t)blockIdx.x * (blockDim.x >> 6) + wave;
  if (idx >= n) return;
  const double b = b_in[idx];
  double K = 0, E = 0, A0 = __builtin_nan(""), D1 = __builtin_nan("");
  if (b > 0) {
    ellip_KE(exp(-2.0 * b), sqrt(-expm1(-2.0 * b)), &K, &E);
    A0 = M_2_PI * K;
    D1 = M_2_PI * (expm1(b) * K - exp(b) * E);
  }
  singular_factor_wave<double, 4>(b, exp(-b), -expm1(-b), A0, D1, mtop, A, false, lane);
  for (int m = lane; m <= mtop; m += 64) out[idx * (mtop + 1) + m] = A[m];
}

// ===========================================================================
// Double-layer coefficients (Sec. 4), one wavefront per pair
//
// The kernel of K is 2 dG/d nu_s = tau_0 (ik rho - 1) e^{ik rho} / (2 pi rho^3)
// with tau_0 = nu_s . (r_s - r); K' has tau_0 = nu_t . (r - r_s).  Split as in
// Sec. 4 into a singular and a smooth part,
//   tau_0 (ik rho - 1) e^{ik rho} / rho^3 = -H s_{a,b}^{-3/2} - i P,
//   H = tau_0 (cos k rho + k rho sin k rho) F^3,  F = (s_{a,b}/rho^2)^{1/2},
//   P = tau_0 (sin k rho - k rho cos k rho) / rho^3,
// (H and P are smooth: both factors of k rho are analytic in rho^2), the
// coefficients produced are
//   kK_n = -sum_j <H>_j e^{-i(n-j)a} B_{|n-j|}(b) - i <P>_n,  n = -M+1..M,
// the swap of eq. (4.6) with B_m(0, b) = <s_{0,b}^{-3/2}>_m (eq. (4.7)).
// B_0 comes from the complete elliptic integrals (eq. (4.9)) and B_m from the
// recurrence of Proposition 4.1 (eq. (4.8)), forward for small b and backward
// (where forward would amplify rounding by cosh(b)^m) otherwise.
//
// For small b the sum above loses (B_m ~ 1/b^2 while the result is O(log b))
// and translated swapping is used: with H(a), H'(a) at the real part a of the
// root, g = H - H(a) - H'(a) sin(phi) (phi = theta_s - a) vanishes to second
// order at phi = 0, g = sin^2(phi/2) delta with delta smooth, and
//   <H s^{-3/2}>_n = e^{-ina} [H(a) B_n + H'(a) <sin phi s^{-3/2}>_n]
//                    + sum_j delta_j e^{-i(n-j)a} Bt_{|n-j|},
//   Bt_m = <sin^2(phi/2) s^{-3/2}>_m = (e^b/4) (A_m - (1 - e^{-b})^2 B_m),
//   <sin phi s^{-3/2}>_n = (B_{n-1} - B_{n+1}) / (2i), the difference written
//   through the recurrence without cancellation.
// H(a) needs tau_0 at the root to full relative accuracy; tau_0 = O(rho^2)
// there, so it is evaluated by the line integral of the Remark in Sec. 4:
//   nu(v) . (r(v) - r(v + d)) = int_0^1 (lam - 1) nu(v) . D^2 r(v + lam d)[d, d] dlam
// (16-point Gauss-Legendre in lam, one node per lane).  Everywhere else the
// product-to-sum point difference keeps tau_0's error at O(u rho), which the
// factor F^3 / rho^3 ~ 1/rho^2 leaves O(u) in H.
// ===========================================================================
constexpr double kBackwardB = 0.2;     // B_m by the backward recurrence from this b

// 16-point Gauss-Legendre rule on [0, 1]
__constant__ double kLamX[16] = {
    0.005299532504175031, 0.0277124884633837, 0.06718439880608412, 0.1222977958224985,
    0.19106187779867811, 0.2709916111713863, 0.35919822461037054, 0.4524937450811813,
    0.5475062549188188, 0.6408017753896295, 0.7290083888286136, 0.8089381222013219,
    0.8777022041775016, 0.9328156011939159, 0.9722875115366163, 0.994700467495825};
__constant__ double kLamW[16] = {
    0.013576229705877019, 0.031126761969323853, 0.047579255841246296, 0.062314485627767015,
    0.07479799440828838, 0.08457825969750131, 0.0913017075224618, 0.09472530522753429,
    0.09472530522753429, 0.0913017075224618, 0.08457825969750131, 0.07479799440828838,
    0.062314485627767015, 0.047579255841246296, 0.031126761969323853, 0.013576229705877019};

// R and its first and second partial derivatives at a general parameter point.
struct SurfPt {
  double st, ct, sh, ch;               // sin t, cos t, sin theta, cos theta
  double R, Rt, Rh, Rtt, Rth, Rhh;     // R, R_t, R_theta, R_tt, R_t theta, R_theta theta
};

template <int MM>
__device__ __forceinline__ void surf_point(const Geom& g, double t, double th, SurfPt* p) {
  sincos_bounded(t, &p->st, &p->ct);
  sincos_bounded(th, &p->sh, &p->ch);
  double cm[MM + 1], sm[MM + 1];
  cm[0] = 1.0;
  sm[0] = 0.0;
#pragma unroll
  for (int m = 1; m <= MM; ++m) {
    cm[m] = fma(cm[m - 1], p->ch, -sm[m - 1] * p->sh);
    sm[m] = fma(sm[m - 1], p->ch, cm[m - 1] * p->sh);
  }
  double R = 1.0, Rt = 0.0, Rh = 0.0, Rtt = 0.0, Rth = 0.0, Rhh = 0.0;
  double sl = p->st, cl = p->ct, sp = 0.0, cp = 1.0;    // sin(l t), cos(l t) and l - 1
  for (int l = 1; l <= g.lmax; ++l) {
    // sum_m a cos(m theta), sum_m m a sin(m theta), sum_m m^2 a cos(m theta)
    double ac = 0.0, as = 0.0, am2 = 0.0;
#pragma unroll
    for (int m = 0; m <= MM; ++m) {
      const double a = (m <= g.mmax) ? g.a[l - 1][m] : 0.0;
      ac = fma(a, cm[m], ac);
      as = fma(a * m, sm[m], as);
      am2 = fma(a * (m * m), cm[m], am2);
    }
    const double dl = l;
    R = fma(sl, ac, R);
    Rt = fma(dl * cl, ac, Rt);
    Rh = fma(-sl, as, Rh);
    Rtt = fma(-dl * dl * sl, ac, Rtt);
    Rth = fma(-dl * cl, as, Rth);
    Rhh = fma(-sl, am2, Rhh);
    const double sn = 2.0 * p->ct * sl - sp, cn = 2.0 * p->ct * cl - cp;
    sp = sl; sl = sn;
    cp = cl; cl = cn;
  }
  p->R = R; p->Rt = Rt; p->Rh = Rh; p->Rtt = Rtt; p->Rth = Rth; p->Rhh = Rhh;
}

// Unit normal (r_t x r_theta)/|r_t x r_theta| of r = R omega: with omega, e_t =
// omega_t and e_phi = omega_theta / sin t orthonormal, r_t x r_theta =
// R [R sin t omega - R_t sin t e_t - R_theta e_phi].
__device__ __forceinline__ void unit_normal(double R, double Rt, double Rh, double st, double ct,
                                            double sh, double ch, double* nx, double* ny,
                                            double* nz) {
  const double a = R * st, bt = -Rt * st, c = -Rh;
  const double inv = rsqrt_refined(fma(a, a, fma(bt, bt, c * c)));
  *nx = (a * st * ch + bt * ct * ch - c * sh) * inv;
  *ny = (a * st * sh + bt * ct * sh + c * ch) * inv;
  *nz = (a * ct - bt * st) * inv;
}

// Normal of the stretched surface D r from a normal n of r: D r_t x D r_theta
// = cof(D) (r_t x r_theta), cof(D) = diag(d_y d_z, d_x d_z, d_x d_y);
// renormalised to unit length.
__device__ __forceinline__ void stretch_normal(const Geom& g, double* nx, double* ny, double* nz) {
  const double cx = g.ax[1] * g.ax[2], cy = g.ax[0] * g.ax[2], cz = g.ax[0] * g.ax[1];
  const double mx = cx * *nx, my = cy * *ny, mz = cz * *nz;
  const double inv = rsqrt_refined(fma(mx, mx, fma(my, my, mz * mz)));
  *nx = mx * inv;
  *ny = my * inv;
  *nz = mz * inv;
}

// tau_0 = nu(v) . (r(v) - r(v + d)), v = (tv, hv), d = (dt, dh), by the line
// integral of the Remark in Sec. 4; every lane returns the value.  ST: the
// surface is stretched by D (its second derivatives and normal with it).
template <int MM, bool ST = false>
__device__ __forceinline__ double tau0_line(const Geom& g, double tv, double hv, double dt,
                                            double dh, int lane) {
  SurfPt v;
  surf_point<MM>(g, tv, hv, &v);
  double nx, ny, nz;
  unit_normal(v.R, v.Rt, v.Rh, v.st, v.ct, v.sh, v.ch, &nx, &ny, &nz);
  if constexpr (ST) {
    stretch_normal(g, &nx, &ny, &nz);
    nx *= g.ax[0];   // nu . (D q) = (D nu) . q
    ny *= g.ax[1];
    nz *= g.ax[2];
  }
  double acc = 0.0;
  if (lane < 16) {
    const double lam = kLamX[lane];
    SurfPt p;
    surf_point<MM>(g, fma(lam, dt, tv), fma(lam, dh, hv), &p);
    // omega and its derivatives at the node
    const double wx = p.st * p.ch, wy = p.st * p.sh, wz = p.ct;
    const double tx = p.ct * p.ch, ty = p.ct * p.sh, tz = -p.st;          // omega_t
    const double hx = -p.st * p.sh, hy = p.st * p.ch;                      // omega_theta
    const double thx = -p.ct * p.sh, thy = p.ct * p.ch;                    // omega_t theta
    const double hhx = -wx, hhy = -wy;                                     // omega_theta theta
    // r_tt = R_tt w + 2 R_t w_t - R w; r_th = R_th w + R_t w_h + R_h w_t + R w_th;
    // r_hh = R_hh w + 2 R_h w_h + R w_hh
    const double a2 = dt * dt, ab = 2.0 * dt * dh, b2 = dh * dh;
    const double qx = a2 * (p.Rtt * wx + 2.0 * p.Rt * tx - p.R * wx) +
                      ab * (p.Rth * wx + p.Rt * hx + p.Rh * tx + p.R * thx) +
                      b2 * (p.Rhh * wx + 2.0 * p.Rh * hx + p.R * hhx);
    const double qy = a2 * (p.Rtt * wy + 2.0 * p.Rt * ty - p.R * wy) +
                      ab * (p.Rth * wy + p.Rt * hy + p.Rh * ty + p.R * thy) +
                      b2 * (p.Rhh * wy + 2.0 * p.Rh * hy + p.R * hhy);
    const double qz = a2 * (p.Rtt * wz + 2.0 * p.Rt * tz - p.R * wz) +
                      ab * (p.Rth * wz + p.Rh * tz) + b2 * (p.Rhh * wz);
    acc = (lam - 1.0) * kLamW[lane] * fma(nx, qx, fma(ny, qy, nz * qz));
  }
  return wave_sum(acc);
}

// dc_m = sum_l a_lm l cos(l x): R_t = sum_m dc_m cos(m theta) on the curve t = x.
template <int MM>
__device__ __forceinline__ void pair_dcoef(const Geom& g, double x, double* dc) {
  double sx, cx;
  sincos_bounded(x, &sx, &cx);
#pragma unroll
  for (int m = 0; m <= MM; ++m) dc[m] = 0.0;
  double cl = cx, cp = 1.0;
  for (int l = 1; l <= g.lmax; ++l) {
#pragma unroll
    for (int m = 0; m <= MM; ++m) {
      const double a = (m <= g.mmax) ? g.a[l - 1][m] : 0.0;
      dc[m] = fma(a * l, cl, dc[m]);
    }
    const double cn = 2.0 * cx * cl - cp;
    cp = cl; cl = cn;
  }
}

// (sin x - x cos x) / x^3 for 0 <= x < 1 by its Taylor series,
// sum_{j>=1} (-1)^{j+1} 2j x^{2j-2} / (2j+1)!, to j = 10.
__device__ __forceinline__ double beta_series(double x) {
  const double x2 = x * x;
  double p = -3.9145882126782523e-19;
  p = fma(p, x2, 1.4797143443923793e-16);
  p = fma(p, x2, -4.498331606952833e-14);
  p = fma(p, x2, 1.0706029224547743e-11);
  p = fma(p, x2, -1.9270852604185937e-09);
  p = fma(p, x2, 2.505210838544172e-07);
  p = fma(p, x2, -2.2045855379188714e-05);
  p = fma(p, x2, 0.0011904761904761906);
  p = fma(p, x2, -0.03333333333333333);
  return fma(p, x2, 0.3333333333333333);
}

// y_{s+1} = c_s y_s + e_s for s = 0..T-1 from y_0, by the 64 lanes: each lane
// composes the affine maps of its segment of S consecutive steps, a lane scan
// of the 2x2 matrices [[c, e], [0, 1]] gives the state entering each segment,
// and each lane replays its segment, passing (s, y_{s+1}) to `store`.
template <class Step, class Store>
__device__ __forceinline__ void affine_scan_wave(int T, double y0, Step step, Store store, int lane) {
  if (T <= 0) return;
  const int S = (T + 63) / 64;
  const int s0 = lane * S, s1 = min(T, s0 + S);
  double e00 = 1.0, e01 = 0.0, e10 = 0.0, e11 = 1.0;
  for (int s = s0; s < s1; ++s) {
    double c, e;
    step(s, &c, &e);
    e01 = fma(c, e01, e);
    e00 = c * e00;
  }
  mat_scan_lanes(e00, e01, e10, e11);
  const double x00 = dpp_f64_fill<0x138, 0xf>(1.0, e00), x01 = dpp_f64_fill<0x138, 0xf>(0.0, e01);
  double y = fma(x00, y0, x01);
  for (int s = s0; s < s1; ++s) {
    double c, e;
    step(s, &c, &e);
    y = fma(c, y, e);
    store(s, y);
  }
}

template <int MM, bool REFINE, bool ST = false>
__device__ __forceinline__ void dl_range(const CoeffArgs& a, const double* tab, double* wbase, int NF,
                                         int64_t beg, int64_t end) {
  const Prob& P = a.P;
  const int M = P.M, mask = P.tab_n - 1, quarter = 2 * M;
  const int lane0 = threadIdx.x & 63;
  const bool adj = a.adjoint != 0;
  cplx* z1a = reinterpret_cast<cplx*>(wbase);
  cplx* z1b = z1a + NF;
  double* Abuf = reinterpret_cast<double*>(z1b + NF);
  const int capB = M + NF + 2;
  double* Bbuf = Abuf + dl_cap_a(NF, M);
  double* Btbuf = Bbuf + capB;
  cplx* kc = reinterpret_cast<cplx*>(Btbuf + capB);    // <H s^{-3/2}>_n, n = 0..M
  cplx* Pc = kc + (M + 1);                              // <P>_n, n = 0..M
  cplx* kappa = static_cast<cplx*>(a.kappa);

  const int tstride = (8 * M) / NF;
  const int hstep = (4 * M) / NF;
  const double nan = __builtin_nan("");
  const double k = P.k, k3 = k * k * k;
  const double invNF = 1.0 / NF;
  PairGeo<MM> pg;
  double dc[MM + 1];
  double t_prev = nan, ts_prev = nan;

  for (int64_t w = beg; w < end; ++w) {
    int lane = lane0;
    asm volatile("" : "+v"(lane));
    const int64_t pi = a.list ? a.list[w] : w;
    const double t = a.t_in[pi], ts = a.ts_in[pi];
    const int j = a.az_in[pi] & (2 * M - 1);
    const RootRec rr = load_root(a.roots, pi);
    int st = a.status[pi] & ((1 << FFBIE_PAIR_P_SHIFT) - 1);
    cplx* krow = kappa + pi * (int64_t)(2 * M);
    if (st & FFBIE_PAIR_SINGULAR) {
      for (int c = lane; c < 2 * M; c += 64) krow[c] = cplx{nan, nan};
      continue;
    }
    const int J = 4 * j;
    // consecutive pairs of one (target node, source node) differ only in the
    // target azimuth: the t, t_s parts of the geometry are kept
    if (!(t == t_prev && ts == ts_prev)) {
      pair_geo<MM>(P.g, t, ts, tab, J, mask, quarter, &pg);
      // d/dt coefficients of R on the curve that carries the normal
      pair_dcoef<MM>(P.g, adj ? t : ts, dc);
#pragma unroll
      for (int m = 0; m <= MM; ++m) dc[m] = to_uniform(dc[m]);
      t_prev = t; ts_prev = ts;
    } else {
      pair_geo_R<MM>(tab, J, mask, quarter, &pg);
    }
    pair_geo_uniform<MM>(&pg);
    double nux = 0.0, nuy = 0.0, nuz = 0.0;            // K': unit normal at the target
    if (adj) {
      double Rt = 0.0, Rh = 0.0;
#pragma unroll
      for (int m = 0; m <= MM; ++m) {
        Rt = fma(dc[m], tcos(tab, m * J, mask, quarter), Rt);
        Rh = fma(-(double)m * pg.ga[m], tsin(tab, m * J, mask), Rh);
      }
      unit_normal(pg.R, Rt, Rh, pg.st, pg.ct, tsin(tab, J, mask), tcos(tab, J, mask, quarter), &nux,
                  &nuy, &nuz);
      if constexpr (ST) stretch_normal(P.g, &nux, &nuy, &nuz);
    }
    const double u = rr.u, b = rr.b;
    int qu;
    double ur, sur, cur;
    root_grid_offset(u, NF, &qu, &ur);
    if constexpr (!REFINE) {        // the main pass samples the 2M-point grid
      sur = rr.sh;
      cur = rr.ch;
    } else {
      sincos_bounded(0.5 * ur, &sur, &cur);
    }
    const double eb = rr.eb, omq = rr.omq;
    const int qj = j * (NF / (2 * M));

    // ---- samples of H (real part) and P (imaginary part).  maxN bounds the
    //      rounding of the samples: tau_0 is a dot product with |r_s - r| = rho,
    //      and cos x + x sin x carries rounding ~u x, so H_q is good to about
    //      u rho (1 + x) F^3 -- the level below which its coefficients are noise
    double maxH = 0.0, maxP = 0.0, maxN = 0.0;
    for (int q = lane; q < NF; q += 64) {
      const int Kq = q * tstride;
      double dx, dy, dz;
      dr_grid<MM, ST>(pg, tab, Kq, J, mask, quarter, &dx, &dy, &dz);
      const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
      const double ri = rsqrt_refined(r2);
      const double rho = r2 * ri;
      const double x = k * rho;
      double skr, ckr;
      sincos_moderate(x, &skr, &ckr);
      const int hidx = (q - qj - qu) * hstep;
      const double sh = fma(tsin(tab, hidx, mask), cur, -tcos(tab, hidx, mask, quarter) * sur);
      const double s = fma(omq, omq, 4.0 * eb * sh * sh);
      const double F = sqrt_pos(s) * ri;
      double tau;
      if (adj) {
        tau = -fma(nux, dx, fma(nuy, dy, nuz * dz));
      } else {
        // unit normal at the source (t_s, theta_q)
        const double cq = tcos(tab, Kq, mask, quarter), sq = tsin(tab, Kq, mask);
        double Rs = 1.0, Rts = 0.0, Rhs = 0.0;
#pragma unroll
        for (int m = 0; m <= MM; ++m) {
          const double cm = tcos(tab, m * Kq, mask, quarter), sm = tsin(tab, m * Kq, mask);
          Rs = fma(pg.al[m], cm, Rs);
          Rts = fma(dc[m], cm, Rts);
          Rhs = fma(-(double)m * pg.al[m], sm, Rhs);
        }
        const double A1 = Rs * pg.sts, A2 = -Rts * pg.sts, A3 = -Rhs;
        if constexpr (ST) {
          // the normal A1 omega + A2 e_t + A3 e_phi of r, stretched: cof(D) n
          const double ex = fma(A1, pg.sts, A2 * pg.cts);
          double mx = fma(ex, cq, -A3 * sq), my = fma(ex, sq, A3 * cq);
          double mz = fma(A1, pg.cts, -A2 * pg.sts);
          mx *= P.g.ax[1] * P.g.ax[2];
          my *= P.g.ax[0] * P.g.ax[2];
          mz *= P.g.ax[0] * P.g.ax[1];
          tau = fma(mx, dx, fma(my, dy, mz * dz)) * rsqrt_refined(fma(mx, mx, fma(my, my, mz * mz)));
        } else {
          const double hxy = fma(cq, dx, sq * dy);
          const double wd = fma(pg.sts, hxy, pg.cts * dz);      // omega . d
          const double td = fma(pg.cts, hxy, -pg.sts * dz);     // e_t . d
          const double pd = fma(-sq, dx, cq * dy);              // e_phi . d
          tau = fma(A1, wd, fma(A2, td, A3 * pd)) * rsqrt_refined(fma(A1, A1, fma(A2, A2, A3 * A3)));
        }
      }
      const double F3 = F * F * F;
      const double H = tau * fma(x, skr, ckr) * F3;
      maxN = fmax(maxN, rho * (1.0 + x) * F3);
      const double beta = (x < 1.0) ? k3 * beta_series(x) : (skr - x * ckr) * (ri * ri * ri);
      const double Pv = beta * tau;
      z1a[q] = cplx{H, Pv};
      maxH = fmax(maxH, fabs(H));
      maxP = fmax(maxP, fabs(Pv));
    }
    maxH = wave_max(maxH);
    maxP = wave_max(maxP);
    maxN = wave_max(maxN);
    // P rides in the imaginary part scaled by a power of two to H's size, so
    // that its size does not raise the rounding floor of H's coefficients
    const int sexp = (maxH > 0.0 && maxP > 0.0) ? ilogb(maxH) - ilogb(maxP) : 0;
    if (sexp != 0) {
      const double sP = ldexp(1.0, sexp);
      for (int q = lane; q < NF; q += 64) z1a[q].im *= sP;
    }
    wave_sync();
    cplx *Z = z1a, *Fr = z1b, *Zd = z1a, *Fd = z1b;
    fft_stockham_r4(Z, Fr, Zd, Fd, false, NF, M, tab, mask, quarter, (const cplx*)nullptr, lane);

    // truncation index (the rule of eq. (3.24)) against the larger of H's
    // largest coefficient and its rounding scale: where tau_0 is a small
    // difference of O(rho) terms (targets far from a source curve near a
    // pole) the coefficients reach that floor, not eps0 max |H|
    const int ptr = trunc_index_real(Z, NF, invNF, P.eps0, fmax(maxH, maxN), lane);
    if (ptr >= NF / 2 - 2) {
      if (!REFINE && a.flag_list) {
        if (lane == 0) {
          const int32_t slot = atomicAdd(a.flag_count, 1);
          a.flag_list[slot] = pi;
          a.status[pi] = st | FFBIE_PAIR_REFINED;
        }
        continue;
      }
      st |= FFBIE_PAIR_UNRESOLVED;
    }
    // Coefficients convolved: for b < 0.2 all of them below N_F/2.  B_m grows
    // like 1/b^2, and <H>_j below the truncation threshold still carry more than
    // rounding (dropping them would cost about eps0 max|H| B_0 per coefficient);
    // the translated swap weighs them by j^2 log(1/b).
    const int p = b < kBackwardB ? NF / 2 - 1 : ptr;
    const int Jq = J + qu * tstride;
    cplx ph_lane, ph64;
    {
      double s1, c1;
      sincos_moderate(lane * ur, &s1, &c1);
      ph_lane = mk(tcos(tab, lane * Jq, mask, quarter), tsin(tab, lane * Jq, mask)) * mk(c1, s1);
      const cplx h = mk(read_lane(ph_lane.re, 32), read_lane(ph_lane.im, 32));
      ph64 = h * h;
    }
    // ---- G_j = <H>_j e^{ija} (mirrored, G[p + j]) and <P>_n, n = 0..M
    cplx* G = Fr;
    {
      cplx ph = ph_lane;
      for (int jj = lane; jj <= p; jj += 64, ph = ph * ph64) {
        const cplx gv = real_part_coeff(Z, jj, NF, invNF) * ph;
        G[p + jj] = gv;
        G[p - jj] = conj(gv);
      }
      const double isP = ldexp(1.0, -sexp);
      for (int n = lane; n <= M; n += 64) Pc[n] = isP * imag_part_coeff(Z, n, NF, invNF);
    }
    wave_sync();

    // ---- A_m(b) and B_m(b).  e^b and cosh b are formed only where b < 0.2;
    //      the backward recurrence takes 1/cosh b and e^b/cosh b from e^{-b},
    //      which stay finite for any b
    const double e_b = b < kBackwardB ? rcp_refined(eb) : 0.0;   // e^b
    const double chb = 0.5 * (e_b + eb);                          // cosh b (b < 0.2)
    const int mtopB = M + p;
    const bool backward = b >= kBackwardB;
    const int NB = backward ? max(mtopB, (int)ceil(37.0 / b)) + 8 : mtopB;
    double* A = Abuf;
    singular_factor_wave<double, 4>(b, eb, omq, rr.A0, rr.D1, backward ? NB - 1 : mtopB, A, false, lane);
    double* B = Bbuf + p;
    bool translate = false;
    if (!backward) {
      // B_0 of eq. (4.9): E(e^{-2b}) = (pi/2)(omq A_0 - e^{-b} (A_1 - A_0)), 1 - e^{-2b} = omq (1 + e^{-b})
      const double E = M_PI_2 * fma(omq, rr.A0, -eb * rr.D1);
      const double omq2 = omq * (1.0 + eb);
      const double B0 = 4.0 * E / (M_PI * omq2 * omq2) - rr.A0 / omq2;
      if (lane == 0) B[0] = B0;
      // Plain or translated swap, whichever amplifies the rounding of the
      // samples of H less.  Rounding eps in each <H>_j reaches the plain sum as
      // about eps B_0 sqrt(2p + 1) (B_m ~ B_0 for m b << 1) and the translated
      // one as eps (log(1/b) + 3)/(2 pi) (sum_{j <= p} j^4)^{1/2}: through
      // delta = g / sin^2(phi/2), the coefficients' second moment meets the
      // log(1/b) term of <sin^2(phi/2) s^{-3/2}>.
      {
        const double pp = p;
        const double s4 = pp * (pp + 1.0) * (2.0 * pp + 1.0) * (3.0 * pp * pp + 3.0 * pp - 1.0) / 30.0;
        translate = B0 * sqrt(2.0 * pp + 1.0) > (0.5 * M_1_PI) * (3.0 - log(b)) * sqrt(s4);
      }
      // B_m = cosh(b) B_{m-1} - ((2m - 1)/2) e^b A_{m-1}, m = 1..mtopB
      affine_scan_wave(
          mtopB, B0,
          [&](int s, double* c, double* e) {
            *c = chb;
            *e = -(s + 0.5) * e_b * A[s];
          },
          [&](int s, double y) { B[s + 1] = y; }, lane);
    } else {
      // B_{m-1} = (B_m + ((2m - 1)/2) e^b A_{m-1}) / cosh(b), m = NB..1, from B_NB = 0
      const double den = rcp_refined(fma(eb, eb, 1.0));
      const double ic = 2.0 * eb * den, eic = 2.0 * den;        // 1/cosh b, e^b/cosh b
      affine_scan_wave(
          NB, 0.0,
          [&](int s, double* c, double* e) {
            const int m = NB - s;
            *c = ic;
            *e = (m - 0.5) * eic * A[m - 1];
          },
          [&](int s, double y) {
            const int m = NB - s - 1;
            if (m <= mtopB) B[m] = y;
          },
          lane);
    }
    wave_sync();
    for (int m = 1 + lane; m <= p; m += 64) B[-m] = B[m];
    wave_sync();

    if (!translate || !(b > 0)) {
      swap_convolution<cplx>(G, p, B, M, ph_lane, ph64, 1.0, kc, nullptr, nullptr, lane);
    } else {
      // ---- translated swapping: H(a) with tau_0 by the line integral
      double su, cu, shu, chu;
      sincos_bounded(u, &su, &cu);
      sincos_bounded(0.5 * u, &shu, &chu);
      const double sj = tsin(tab, J, mask), cj = tcos(tab, J, mask, quarter);
      const double th_j = M_PI * j / M;
      double dx, dy, dz;
      dr_values<MM, ST>(pg, fma(cj, cu, -sj * su), fma(sj, cu, cj * su), shu, chu,
                        fma(sj, chu, cj * shu), fma(cj, chu, -sj * shu), &dx, &dy, &dz);
      const double rho_a = sqrt_pos(fma(dx, dx, fma(dy, dy, dz * dz)));
      const double tau_a = adj ? tau0_line<MM, ST>(P.g, t, th_j, ts - t, u, lane)
                               : tau0_line<MM, ST>(P.g, ts, th_j + u, t - ts, -u, lane);
      const double xa = k * rho_a;
      double sa, ca;
      sincos_bounded(xa, &sa, &ca);
      const double Fa = omq / rho_a, Fa3 = Fa * Fa * Fa;
      const double cfa = fma(xa, sa, ca);
      const double Ha = tau_a * cfa * Fa3;
      // H'(a) from the derivatives at the root's real part, not from the
      // interpolant's coefficients, whose rounding the factor n log(1/b) of
      // <sin phi s^{-3/2}>_n would amplify: with (rho^2)' = 2 (r_s - r) . r_s,theta,
      // F^3' = -(3/2) F^3 (rho^2)'/rho^2 (s' = 0 at phi = 0) and
      // d/dphi (cos x + x sin x) = x cos x k (rho^2)'/(2 rho),
      //   H' = F^3 [tau_0' c + tau_0 (x cos x k (rho^2)'/(2 rho) - (3/2) c (rho^2)'/rho^2)],
      // tau_0' = nu_s' . (r_s - r) for K (nu_s . r_s,theta = 0), -nu_t . r_s,theta for K'.
      double hp;
      {
        SurfPt sp;
        surf_point<MM>(P.g, ts, th_j + u, &sp);
        const double wx = sp.st * sp.ch, wy = sp.st * sp.sh, wz = sp.ct;
        const double otx = sp.ct * sp.ch, oty = sp.ct * sp.sh, otz = -sp.st;   // omega_t
        const double ohx = -sp.st * sp.sh, ohy = sp.st * sp.ch;                // omega_theta
        // D (1 unless ST) scales every derivative of r below
        const double gx = ST ? P.g.ax[0] : 1.0, gy = ST ? P.g.ax[1] : 1.0, gz = ST ? P.g.ax[2] : 1.0;
        const double rhx = gx * fma(sp.Rh, wx, sp.R * ohx), rhy = gy * fma(sp.Rh, wy, sp.R * ohy),
                     rhz = gz * (sp.Rh * wz);                                  // r_theta
        const double drho2 = 2.0 * fma(dx, rhx, fma(dy, rhy, dz * rhz));
        double taup;
        if (adj) {
          taup = -fma(nux, rhx, fma(nuy, rhy, nuz * rhz));
        } else {
          const double othx = -sp.ct * sp.sh, othy = sp.ct * sp.ch;            // omega_t theta
          const double rtx = gx * fma(sp.Rt, wx, sp.R * otx), rty = gy * fma(sp.Rt, wy, sp.R * oty),
                       rtz = gz * fma(sp.Rt, wz, sp.R * otz);                  // r_t
          const double rthx = gx * (sp.Rth * wx + sp.Rt * ohx + sp.Rh * otx + sp.R * othx);
          const double rthy = gy * (sp.Rth * wy + sp.Rt * ohy + sp.Rh * oty + sp.R * othy);
          const double rthz = gz * (sp.Rth * wz + sp.Rh * otz);                // r_t theta
          const double rhhx = gx * (sp.Rhh * wx + 2.0 * sp.Rh * ohx - sp.R * wx);
          const double rhhy = gy * (sp.Rhh * wy + 2.0 * sp.Rh * ohy - sp.R * wy);
          const double rhhz = gz * (sp.Rhh * wz);                              // r_theta theta
          // n = r_t x r_theta, n' = r_t theta x r_theta + r_t x r_theta theta
          const double nx = rty * rhz - rtz * rhy, ny = rtz * rhx - rtx * rhz, nz = rtx * rhy - rty * rhx;
          const double npx = (rthy * rhz - rthz * rhy) + (rty * rhhz - rtz * rhhy);
          const double npy = (rthz * rhx - rthx * rhz) + (rtz * rhhx - rtx * rhhz);
          const double npz = (rthx * rhy - rthy * rhx) + (rtx * rhhy - rty * rhhx);
          const double inn = rsqrt_refined(fma(nx, nx, fma(ny, ny, nz * nz)));
          const double vx = nx * inn, vy = ny * inn, vz = nz * inn;
          const double vn = fma(vx, npx, fma(vy, npy, vz * npz));
          const double dvx = (npx - vx * vn) * inn, dvy = (npy - vy * vn) * inn, dvz = (npz - vz * vn) * inn;
          taup = fma(dvx, dx, fma(dvy, dy, dvz * dz));
        }
        const double r2a = rho_a * rho_a;
        hp = Fa3 * fma(taup, cfa,
                       tau_a * (xa * ca * k * drho2 / (2.0 * rho_a) - 1.5 * cfa * drho2 / r2a));
      }
      wave_sync();
      // g = H - H(a) - H'(a) sin(phi): G_0 -= H(a), G_{+-1} +-= i H'(a)/2
      if (lane == 0) {
        G[p].re -= Ha;
        if (p >= 1) {
          G[p + 1].im += 0.5 * hp;
          G[p - 1].im -= 0.5 * hp;
        }
      }
      wave_sync();
      // delta_k = -4 sum_{j > k} (j - k) g_j, k = 0..p-1 (delta_0 real), mirrored
      const int pd = max(p - 1, 0);
      cplx* D = Z + pd;
      for (int kk = lane; kk <= pd; kk += 64) {
        double ar = 0.0, ai = 0.0;
        for (int jj = kk + 1; jj <= p; ++jj) {
          const double wgt = jj - kk;
          ar = fma(wgt, G[p + jj].re, ar);
          ai = fma(wgt, G[p + jj].im, ai);
        }
        const cplx d = cplx{-4.0 * ar, kk == 0 ? 0.0 : -4.0 * ai};
        D[kk] = d;
        D[-kk] = conj(d);
      }
      // Bt_m = (e^b / 4)(A_m - omq^2 B_m), mirrored
      double* Bt = Btbuf + pd;
      const double omq_sq = omq * omq;
      for (int m = lane; m <= mtopB; m += 64) Bt[m] = 0.25 * e_b * fma(-omq_sq, B[m], A[m]);
      wave_sync();
      for (int m = 1 + lane; m <= pd; m += 64) Bt[-m] = Bt[m];
      wave_sync();
      swap_convolution<cplx>(Z, pd, Bt, M, ph_lane, ph64, 1.0, kc, nullptr, nullptr, lane);
      wave_sync();
      // + e^{-ina} [H(a) B_n - i H'(a) Delta_n / 2], Delta_n = B_{n-1} - B_{n+1}
      const double em = expm1(b), emm = expm1(-b);
      const double shb = 0.5 * (em - emm);
      const double ich = rcp_refined(chb);
      cplx ph = ph_lane;
      for (int n = lane; n <= M; n += 64, ph = ph * ph64) {
        double Dn = 0.0;
        if (n >= 1)
          Dn = -B[n] * shb * shb * ich +
               0.5 * e_b * fma((2.0 * n - 1.0) * A[n - 1], ich, (2.0 * n + 1.0) * A[n]);
        kc[n] = kc[n] + conj(ph) * mk(Ha * B[n], -0.5 * hp * Dn);
      }
    }
    wave_sync();
    // ---- kK_n = -<H s^{-3/2}>_n - i <P>_n, n = -M+1..M at column n + M - 1
    for (int c = lane; c < 2 * M; c += 64) {
      const int n = c - M + 1;
      const cplx R = n >= 0 ? kc[n] : conj(kc[-n]);
      const cplx Pn = n >= 0 ? Pc[n] : conj(Pc[-n]);
      krow[c] = cplx{Pn.im - R.re, -R.im - Pn.re};
    }
    if (lane == 0) a.status[pi] = st | (min(ptr, 0xfff) << FFBIE_PAIR_P_SHIFT);
    wave_sync();
  }
}

template <int MM, bool REFINE, bool ST = false>
__global__ __launch_bounds__(256) void ffbie_dl_coeff_kernel_t(CoeffArgs a) {
  extern __shared__ double smem[];
  load_table(smem, a.tab_g, a.P.tab_n);
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int waves_per_block = blockDim.x >> 6;
  const int per_wave = dl_lds_per_wave(a.NF, a.P.M);
  int64_t count = a.n;
  if (a.list) count = *a.list_count;
  const int64_t total_waves = (int64_t)gridDim.x * waves_per_block;
  const int64_t gw = (int64_t)blockIdx.x * waves_per_block + wave;
  const int64_t chunk = (count + total_waves - 1) / total_waves;
  const int64_t beg = gw * chunk, end = min(count, beg + chunk);
  dl_range<MM, REFINE, ST>(a, smem, smem + a.P.tab_n + (size_t)wave * per_wave, a.NF, beg, end);
}

// ---------------------------------------------------------------------------
// Launch helpers (one instantiation per bound on the surface's azimuthal order)
// ---------------------------------------------------------------------------
#define FFBIE_FOR_MM(X) X(0) X(1) X(2) X(4) X(8)

int mm_bucket(int mmax) { return mmax <= 0 ? 0 : mmax <= 1 ? 1 : mmax <= 2 ? 2 : mmax <= 4 ? 4 : 8; }

hipError_t launch_root(const Prob& P, const double* tab, int64_t n, const double* t,
                       const int32_t* az, const double* ts, RootRec* out, int32_t* status,
                       double* root_out, hipStream_t stream) {
  const int threads = 256;
  const int64_t blocks = (n + threads - 1) / threads;
  const size_t lds = P.tab_n * sizeof(double);
  switch (mm_bucket(P.g.mmax)) {
#define X(MMV)                                                                                   \
  case MMV:                                                                                      \
    if (P.g.scaled)                                                                              \
      hipLaunchKernelGGL((ffbie_root_kernel_t<MMV, true>), dim3((unsigned)blocks), dim3(threads), \
                         lds, stream, P, tab, n, t, az, ts, out, status, root_out);              \
    else                                                                                         \
      hipLaunchKernelGGL((ffbie_root_kernel_t<MMV, false>), dim3((unsigned)blocks), dim3(threads), \
                         lds, stream, P, tab, n, t, az, ts, out, status, root_out);              \
    break;
    FFBIE_FOR_MM(X)
#undef X
  }
  return hipGetLastError();
}

hipError_t launch_coeff(const CoeffArgs& a, int64_t blocks, int waves, size_t lds,
                        hipStream_t stream, bool refine, bool single) {
  // refine passes always take radix-2 transforms
  const bool r4 = !refine && (a.radix == 4 || (a.radix == 0 && a.NF >= 256));
  // stretched surfaces (FP64 only; the host rejects the mixed path for them)
  const bool st = a.P.g.scaled != 0;
  if (st && single) return hipErrorInvalidValue;
  switch (mm_bucket(a.P.g.mmax)) {
#define K(MMV, RF, RT, RX, ST)                                                                   \
  hipLaunchKernelGGL((ffbie_coeff_kernel_t<MMV, RF, RT, RX, ST>), dim3((unsigned)blocks),       \
                     dim3(64 * waves), lds, stream, a)
#define KR(MMV, RT, ST)                                                                          \
  if (refine) K(MMV, true, RT, 2, ST); else if (r4) K(MMV, false, RT, 4, ST); else K(MMV, false, RT, 2, ST)
#define X(MMV)                                                                                   \
  case MMV:                                                                                      \
    if (single) { KR(MMV, float, false); }                                                       \
    else if (st) { KR(MMV, double, true); }                                                      \
    else { KR(MMV, double, false); }                                                             \
    break;
    FFBIE_FOR_MM(X)
#undef X
#undef KR
#undef K
  }
  return hipGetLastError();
}

hipError_t launch_batch(const BatchArgs& b, int mm, int64_t blocks, int threads, size_t lds,
                        hipStream_t stream, int phase, bool single) {
  const dim3 grid((unsigned)blocks), block(threads);
  const bool r4 = b.radix == 4;
  switch (mm_bucket(mm)) {
#define P12(MMV, RT)                                                                             \
  if (phase == 2)                                                                                \
    hipLaunchKernelGGL((ffbie_coeff_batch_refine_t<MMV, RT>), grid, block, lds, stream, b);     \
  else if (r4 && b.persistent)                                                                   \
    hipLaunchKernelGGL((ffbie_coeff_batch_kernel_t<MMV, RT, 4, true>), grid, block, lds, stream, b); \
  else if (r4)                                                                                   \
    hipLaunchKernelGGL((ffbie_coeff_batch_kernel_t<MMV, RT, 4, false>), grid, block, lds, stream, b); \
  else if (b.persistent)                                                                         \
    hipLaunchKernelGGL((ffbie_coeff_batch_kernel_t<MMV, RT, 2, true>), grid, block, lds, stream, b); \
  else                                                                                           \
    hipLaunchKernelGGL((ffbie_coeff_batch_kernel_t<MMV, RT, 2, false>), grid, block, lds, stream, b)
#define X(MMV)                                                                                   \
  case MMV:                                                                                      \
    if (phase == 0)                                                                              \
      hipLaunchKernelGGL(ffbie_root_batch_kernel_t<MMV>, grid, block, lds, stream, b);           \
    else if (single)                                                                             \
      P12(MMV, float);                                                                           \
    else                                                                                         \
      P12(MMV, double);                                                                          \
    break;
    FFBIE_FOR_MM(X)
#undef X
#undef P12
  }
  return hipGetLastError();
}

hipError_t launch_zero(int* p, int n, hipStream_t stream) {
  hipLaunchKernelGGL(ffbie_zero_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, stream, p, n);
  return hipGetLastError();
}

hipError_t launch_dl_coeff(const CoeffArgs& a, int64_t blocks, int waves, size_t lds,
                           hipStream_t stream, bool refine) {
  const bool st = a.P.g.scaled != 0;
  switch (mm_bucket(a.P.g.mmax)) {
#define K(MMV, RF, ST)                                                                           \
  hipLaunchKernelGGL((ffbie_dl_coeff_kernel_t<MMV, RF, ST>), dim3((unsigned)blocks),            \
                     dim3(64 * waves), lds, stream, a)
#define X(MMV)                                                                                   \
  case MMV:                                                                                      \
    if (refine) { if (st) K(MMV, true, true); else K(MMV, true, false); }                        \
    else { if (st) K(MMV, false, true); else K(MMV, false, false); }                             \
    break;
    FFBIE_FOR_MM(X)
#undef X
#undef K
  }
  return hipGetLastError();
}

}  // namespace ffbie
