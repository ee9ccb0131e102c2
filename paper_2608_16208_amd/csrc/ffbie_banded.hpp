// The O(M) banded route to <rho^-1>_l (Sec. 3.2.1): launch records shared by
// the host code and the three kernels of ffbie_banded.hip.
#pragma once
#include "ffbie_kernels.hpp"

namespace ffbie {

constexpr int kBandMaxM0 = 8;               // largest truncation index m0 (eq. (3.13))
constexpr int kBandC2 = kBandMaxM0 + 1;     // <rho^2>_n kept per pair, n = 0..8

struct BandArgs {
  Prob P;
  const double* tab_g;        // angle table of the problem (8M entries)
  int64_t n;                  // pairs
  const double* t_in;
  const int32_t* az_in;
  const double* ts_in;
  const RootRec* roots;       // root kernel output: offset of a from theta_j, and b
  int32_t* status;            // per-pair status (root kernel bits; FFBIE_PAIR_NOT_PD added)
  cplx* c2;                   // [n][kBandC2] <rho^2>_n, n = 0..8
  double* ratio_part;         // [blocks][kBandC2] per-block max of |<rho^2>_n| / <rho^2>_0, or
                              // null when m0 is given (the rule of eq. (3.13) is not needed)
  double* ratio;              // [kBandC2] the maxima over all pairs
  cplx* rhoinv;               // [n][L+1] output
  int m0;
  double gl_x[16], gl_w[16];  // 16-point Gauss-Legendre rule on [-1, 1]
  cplx* fac;                  // factor records of one chunk of pairs
  int64_t chunk0, chunk_n, stride;
};

// degree in theta_s of the trigonometric polynomial rho^2 of the star surface
int rho2_degree(const Geom& g);

// blocks of the <rho^2> launch (the rows of ratio_part)
int band_rho2_blocks(const BandArgs& a);
hipError_t launch_band_rho2(const BandArgs& a, hipStream_t s);
hipError_t launch_band_moments(const BandArgs& a, hipStream_t s);
hipError_t launch_band_solve(const BandArgs& a, hipStream_t s);

}  // namespace ffbie
