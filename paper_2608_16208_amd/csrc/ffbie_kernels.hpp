// Records shared by the host launch code and the coefficient kernels.
#pragma once
#include "ffbie_device.hpp"

namespace ffbie {

// Per-pair output of the root kernel: offset u = a - theta_j of the complex
// root theta_+ = a + ib of rho^2, its imaginary part b, A_0(b) and A_1 - A_0;
// then values the coefficient passes take from the root alone and would
// otherwise form in every lane of their wavefront: eb = e^{-b} and
// omq = 1 - e^{-b} (each to full relative accuracy), and sh, ch = sin, cos of
// ur/2, ur the offset of a from the nearest point of the 2M-point sample grid
// (root_grid_offset with NF = 2M).
struct RootRec {
  double u, b, A0, D1;
  double eb, omq, sh, ch;
};

// The root record of pair `pi`, which must be the same in every lane of the
// wavefront (the coefficient passes take one pair per wavefront).  The address
// is made explicitly uniform and read through the constant address space (the
// passes only read the records, written by the root kernel in an earlier
// launch), so the record is fetched by scalar loads into SGPRs and takes no
// VGPRs.
__device__ __forceinline__ RootRec load_root(const RootRec* roots, int64_t pi) {
#if defined(__HIP_DEVICE_COMPILE__)
  using CRec = const __attribute__((address_space(4))) RootRec;
  const uint64_t p = reinterpret_cast<uint64_t>(roots + pi);
  const uint64_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)p);
  const uint64_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(p >> 32));
  return *(CRec*)((hi << 32) | lo);
#else
  return roots[pi];
#endif
}

// e^{-b} and 1 - e^{-b} from one transcendental, each to full relative
// accuracy: below b = 1/2 from expm1 (e^{-b} > 0.6), above from exp
// (1 - e^{-b} > 0.39).
FFBIE_HD __forceinline__ void root_exp_b(double b, double* eb, double* omq) {
  if (b < 0.5) {
    const double em = expm1(-b);
    *eb = 1.0 + em;
    *omq = -em;
  } else {
    *eb = exp(-b);
    *omq = 1.0 - *eb;
  }
}

// The root's real part a = theta_j + u on an NF-point grid of step
// 2 pi / NF: a = theta_j + qu (2 pi / NF) + ur with |ur| <= pi / NF (any
// rounding of qu is absorbed exactly by ur).
FFBIE_HD __forceinline__ void root_grid_offset(double u, int NF, int* qu, double* ur) {
  const double inv_gstep = NF / (2.0 * M_PI);
  const double gstep = 2.0 * M_PI / NF;
  const double qu_d = rint(u * inv_gstep);
  *qu = (int)qu_d;
  *ur = fma(-qu_d, gstep, u);
}

struct CoeffArgs {
  Prob P;
  const double* tab_g;
  int64_t n;                 // pairs (ignored when `list` is set)
  const double* t_in;
  const int32_t* az_in;
  const double* ts_in;
  const RootRec* roots;
  int32_t* status;
  void* kappa;               // [n][2M] complex128, or complex64 on the mixed-precision path
  void* rhoinv;              // [n][L+1] (same type) or null
  int NF;                    // azimuthal samples: 2M (main pass) or 4M (refine pass)
  const int64_t* list;       // refine pass: pair indices
  const int32_t* list_count; // refine pass: number of indices
  int64_t* flag_list;        // main pass: pairs queued for the refine pass
  int32_t* flag_count;
  int variant;               // FFBIE_KAPPA_SWAP or FFBIE_KAPPA_PAPER_CONV
  int64_t flag_tag;          // or-ed into queued pair indices (problem index << 40 in a batch)
  int radix;                 // main-pass FFT stages: 2 (radix-2 Stockham), 4 (radix-4, one radix-2
                             // stage if needed) or 0 (radix 4 for NF >= 256, else 2); refine
                             // passes use radix 2
  int adjoint;               // double-layer kernel: 0 = K (normal at the source), 1 = K'
                             // (normal at the target)
};

// Default pairs per wavefront and work item of the batched launch.
constexpr int kBatchTile = 16;

// Problems of a batch in one launch; probs[s] holds problem s's arguments
// (its own P, angle table, pair arrays, outputs and workspace slices).  The
// main and refine passes run once per M class: probs then starts at the class
// (main pass) or is the whole batch with [prob_lo, prob_hi) the class (refine).
struct BatchArgs {
  const CoeffArgs* probs;    // device memory
  int n_probs;
  const int64_t* item_prefix;  // [n_probs] first work item of each problem (main pass)
  int64_t n_items;
  const int64_t* root_prefix;  // [n_probs] first 256-pair root block of each problem
  int* item_counter;         // work queue head (zeroed before the launch)
  int64_t* flag_list;        // refine queue: (problem << 40) | pair
  int32_t* flag_count;
  int tab_max;               // doubles reserved for the angle table at the start of LDS
  int tw_max;                // doubles reserved after it for FFT twiddles (0 if none)
  int tile;                  // pairs per work item (one wavefront)
  int prob_lo, prob_hi;      // refine pass: the class's problems
  int radix;                 // main pass: FFT radix of the class (2 or 4)
  int persistent;            // main pass: 1 = wavefronts loop over work items taken
                             // from item_counter; 0 = work item = global wavefront index
};

// Per-wavefront LDS of the coefficient kernel, in doubles, with the spectral
// stage in FP64 or (single) in FP32; the layout in units of its real type:
//   compact (default variant without <rho^-1> output):
//     two NF-complex FFT buffers, A_m (m <= M + NF/2), kc (M + 1 complex)
//   transforms (default variant with <rho^-1> output): four NF-complex buffers;
//     <rho^-1>_l goes straight to the output row
//   full (eq. (3.10) variant): four NF-complex buffers and the <rho^-1> buffer
//     (2L + 1 complex) that the second convolution reads
//     A_m is stored mirrored, A[-m] = A[m] for m <= NF/2, so it needs M + NF + 2 reals
//     (compact) or fits an NF-complex buffer (transforms and full, since L <= NF).
enum { kLdsCompact = 0, kLdsTransforms = 1, kLdsFull = 2 };
// LDS doubles of the per-workgroup FFT twiddle table (transforms of NF <= 128
// points: 7 stages x 64 lanes complex), 0 otherwise.
FFBIE_HD inline int coeff_twiddle_doubles(int NF, bool single) {
  return NF <= 128 ? (single ? 7 * 64 : 7 * 64 * 2) : 0;
}

FFBIE_HD inline int coeff_lds_per_wave(int NF, int M, int L, int layout, bool single) {
  const int reals = layout == kLdsCompact ? 2 * (2 * NF) + 2 * ((M + NF + 2) / 2) + 2 * (M + 1)
                    : layout == kLdsTransforms ? 2 * (4 * NF)
                                               : 2 * (4 * NF + 2 * L + 1);
  return single ? (reals + 1) / 2 : reals;
}

// Per-wavefront LDS of the double-layer coefficient kernel, in doubles: two
// NF-complex FFT buffers, A_m up to the start of the backward recurrence for
// B_m (m <= max(M + NF/2, 200) + 9), B_m and B~_m mirrored (M + NF + 2 each),
// and the two half rows (M + 1 complex each) of the output.
FFBIE_HD inline int dl_cap_a(int NF, int M) { return (M + NF / 2 > 200 ? M + NF / 2 : 200) + 10; }
FFBIE_HD inline int dl_lds_per_wave(int NF, int M) {
  return 2 * (2 * NF) + dl_cap_a(NF, M) + 2 * (M + NF + 2) + 2 * 2 * (M + 1);
}

hipError_t launch_root(const Prob& P, const double* tab, int64_t n, const double* t,
                       const int32_t* az, const double* ts, RootRec* out, int32_t* status,
                       double* root_out, hipStream_t stream);
hipError_t launch_coeff(const CoeffArgs& a, int64_t blocks, int waves, size_t lds,
                        hipStream_t stream, bool refine, bool single);
// phase 0: root pass (threads = 256), 1: main pass, 2: refine pass of one M class.
hipError_t launch_batch(const BatchArgs& b, int mm, int64_t blocks, int threads, size_t lds,
                        hipStream_t stream, int phase, bool single);
hipError_t launch_zero(int* p, int n, hipStream_t stream);
// Double-layer coefficients (a.adjoint selects K or K'): main pass (refine =
// false, NF = 2M, queueing unresolved pairs) or refine pass over the queue.
hipError_t launch_dl_coeff(const CoeffArgs& a, int64_t blocks, int waves, size_t lds,
                           hipStream_t stream, bool refine);
__global__ void ffbie_singular_factor_kernel(int64_t n, const double* __restrict__ b_in, int mtop,
                                             double* __restrict__ out);

}  // namespace ffbie
