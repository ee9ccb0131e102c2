// 128-point forward DFT held in the registers of one wavefront (gfx950),
// shared by the coefficient kernels and the near-block assembly.
#pragma once
#include "ffbie_device.hpp"

namespace ffbie {

// ---------------------------------------------------------------------------
// 128-point forward DFT held in registers, one wavefront, no LDS passes.
// Radix-2 decimation in time on bit-reversed input: position p = l + 64 R
// (lane l, register R) starts with sample bitrev7(p) = 2 brev6(l) + R, which
// the lane computes itself.  Stage s combines positions p and p + 2^s with the
// factor e^{-2 pi i (p mod 2^s) / 2^{s+1}}:
//   s = 0..3: lanes l and l ^ 2^s, both registers; each lane multiplies its
//             value by its factor (1 in the lower lane), takes the partner's
//             by a DPP move (quad permutes, row shifts, row rotate) and forms
//             sum or difference;
//   s = 4..6: a permlane16 / permlane32 swap exchanges the register bit with
//             lane bit 4 or 5 so that both members of a pair sit in one lane,
//             which then does a full butterfly.
// On return register R of lane l holds X[64 R + 32 L4 + 16 L5 + (l & 15)]
// (L4, L5 = lane bits 4, 5).  The factor lane `lane` applies at stage st is
// e^{-2 pi i k / 128} with k = fft128_twiddle_k(st, lane); tables of these
// (entry st * 64 + lane) are built by the callers.
// ---------------------------------------------------------------------------
FFBIE_HD inline int fft128_twiddle_k(int st, int lane) {
  const int l15 = lane & 15, L4 = (lane >> 4) & 1, L5 = (lane >> 5) & 1;
  if (st <= 3) return ((lane >> st) & 1) ? (lane & ((1 << st) - 1)) << (6 - st) : 0;
  if (st == 4) return l15 << 2;
  if (st == 5) return (16 * L5 + l15) << 1;
  return 32 * L4 + 16 * L5 + l15;
}

// DPP move for patterns that give every lane a source (no old value kept)
template <int CTRL>
__device__ __forceinline__ double dpp_full(double v) {
  const long long u = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)u, CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(u >> 32), CTRL, 0xf, 0xf, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
template <int CTRL>
__device__ __forceinline__ float dpp_full(float v) {
  return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), CTRL, 0xf, 0xf, false));
}

// value of lane l ^ 2^S (S = 0..3)
template <int S, class T>
__device__ __forceinline__ T lane_xor(T v, int lane) {
  if constexpr (S == 0) return dpp_full<0xB1>(v);          // quad_perm [1,0,3,2]
  else if constexpr (S == 1) return dpp_full<0x4E>(v);     // quad_perm [2,3,0,1]
  else if constexpr (S == 2) {
    const T up = dpp_full<0x104>(v), dn = dpp_full<0x114>(v);   // row_shl:4, row_shr:4
    return (lane & 4) ? dn : up;
  } else {
    return dpp_full<0x128>(v);                              // row_ror:8
  }
}

template <int S, class C>
__device__ __forceinline__ void dit_pull_stage(C& x, C w, int lane) {
  using R = decltype(C::re);
  const C t = (S == 0) ? x : x * w;
  const C v = C{lane_xor<S>(t.re, lane), lane_xor<S>(t.im, lane)};
  const R sg = ((lane >> S) & 1) ? (R)-1 : (R)1;
  x = C{fma(sg, t.re, v.re), fma(sg, t.im, v.im)};
}

template <class C>
__device__ __forceinline__ void dit_lane_stage(C& x0, C& x1, C w) {
  const C t = x1 * w;
  x1 = x0 - t;
  x0 = x0 + t;
}

__device__ __forceinline__ void swap_words(bool rows16, unsigned& a, unsigned& b) {
  const auto r = rows16 ? __builtin_amdgcn_permlane16_swap(a, b, false, false)
                        : __builtin_amdgcn_permlane32_swap(a, b, false, false);
  a = r[0];
  b = r[1];
}
__device__ __forceinline__ void swap_lanes(bool rows16, double& a, double& b) {
  const unsigned long long ua = __double_as_longlong(a), ub = __double_as_longlong(b);
  unsigned alo = (unsigned)ua, ahi = (unsigned)(ua >> 32), blo = (unsigned)ub, bhi = (unsigned)(ub >> 32);
  swap_words(rows16, alo, blo);
  swap_words(rows16, ahi, bhi);
  a = __longlong_as_double((long long)(((unsigned long long)ahi << 32) | alo));
  b = __longlong_as_double((long long)(((unsigned long long)bhi << 32) | blo));
}
__device__ __forceinline__ void swap_lanes(bool rows16, float& a, float& b) {
  unsigned ua = __float_as_uint(a), ub = __float_as_uint(b);
  swap_words(rows16, ua, ub);
  a = __uint_as_float(ua);
  b = __uint_as_float(ub);
}
template <class C>
__device__ __forceinline__ void swap_lanes(bool rows16, C& x0, C& x1) {
  swap_lanes(rows16, x0.re, x1.re);
  swap_lanes(rows16, x0.im, x1.im);
}

template <class C>
__device__ __forceinline__ void fft128_regs(C& x0, C& x1, const C* tw, int lane) {
  dit_pull_stage<0>(x0, C{}, lane);
  dit_pull_stage<0>(x1, C{}, lane);
  {
    const C w = tw[64 + lane];
    dit_pull_stage<1>(x0, w, lane);
    dit_pull_stage<1>(x1, w, lane);
  }
  {
    const C w = tw[128 + lane];
    dit_pull_stage<2>(x0, w, lane);
    dit_pull_stage<2>(x1, w, lane);
  }
  {
    const C w = tw[192 + lane];
    dit_pull_stage<3>(x0, w, lane);
    dit_pull_stage<3>(x1, w, lane);
  }
  swap_lanes(true, x0, x1);            // register bit <-> lane bit 4
  dit_lane_stage(x0, x1, tw[256 + lane]);
  swap_lanes(false, x0, x1);           // register bit <-> lane bit 5
  dit_lane_stage(x0, x1, tw[320 + lane]);
  swap_lanes(true, x0, x1);            // register bit <-> lane bit 4
  dit_lane_stage(x0, x1, tw[384 + lane]);
}

// Index of the coefficient that fft128_regs leaves in register 0 of this lane
// (register 1 holds the one 64 above).
__device__ __forceinline__ int fft128_out_index(int lane) {
  return 32 * ((lane >> 4) & 1) + 16 * ((lane >> 5) & 1) + (lane & 15);
}

}  // namespace ffbie
