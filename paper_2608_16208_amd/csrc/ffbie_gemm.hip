// Complex matrix product C -= A B on the matrix cores of gfx950: the trailing
// update of the blocked LU that solves the dense system of Sec. 3.4
// (eq. (3.29)), in complex128 (v_mfma_f64_16x16x4_f64) and complex64
// (v_mfma_f32_16x16x4_f32, FP32 accumulation).
//
// Layout: column-major complex blocks, element (r, c) of X at X[c * ld + r],
// interleaved (re, im).  A column of A, read as real numbers, is the column of
// the real 2m x k matrix X whose even rows hold Re A and odd rows Im A.  Then
//   C_int = X Br + Xs Bi,
// where C_int is C in the same interleaved real form, Br / Bi are the real and
// imaginary parts of B, and Xs is X with each row pair (2r, 2r+1) replaced by
// (-Im A, Re A) -- lane l of an MFMA operand reads row (l ^ 1) of X and flips
// the sign on even rows.  Both products accumulate into one register tile per
// 16 x 16 real block: 8 complex rows x 16 complex columns, no redundant
// accumulators, 8 m n k real flops in total (the 4-multiplication complex
// product).
//
// A workgroup of four wavefronts (2 x 2) computes a BM x BN complex tile of C;
// wavefront (wm, wn) owns WM x WN of it, i.e. (2 WM / 16) x (WN / 16) MFMA
// blocks.  k advances in steps of BK complex columns, staged through LDS in two
// buffers: while the matrix cores work on one buffer the next step's global
// loads are in flight in registers and land in the other buffer, one barrier
// per step.  Tiles are handed out XCD-aware: consecutive workgroup ids go to
// different XCDs, so the tile order is permuted such that each XCD walks a
// contiguous run of the grouped (GM tile rows at a time) tile order and its L2
// keeps the A and B panels those tiles share.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "ffbie_gemm.hpp"

namespace ffbie {

namespace {

typedef double d4v __attribute__((ext_vector_type(4)));
typedef float f4v __attribute__((ext_vector_type(4)));

// Both instructions take A[i][k] from lane i + 16 k and B[k][j] from lane
// j + 16 k.  Their 16 x 16 results sit differently (checked on gfx950): the
// FP32 one puts row 4 (l / 16) + q of column l % 16 in register q of lane l,
// the FP64 one row l / 16 + 4 q.  row_of_lane(i) is the row of X that lane i
// supplies so that in both cases register q of lane l receives row
// 4 (l / 16) + q of the block, i.e. each lane holds the (re, im) rows of two
// consecutive complex rows of C: the FP64 operand rows are permuted by
// i -> 4 (i % 4) + i / 4.
template <typename R>
struct MfmaAcc;
template <>
struct MfmaAcc<double> {
  using T = d4v;
  static __device__ __forceinline__ T mma(double a, double b, T c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row_of_lane(int i) { return 4 * (i & 3) + (i >> 2); }
};
template <>
struct MfmaAcc<float> {
  using T = f4v;
  static __device__ __forceinline__ T mma(float a, float b, T c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static __device__ __forceinline__ int row_of_lane(int i) { return i; }
};

// one complex value as a single vector load / store (16 B or 8 B)
template <typename R>
struct alignas(2 * sizeof(R)) Cx {
  R re, im;
};

constexpr int kXcds = 8;       // XCDs of the MI355X; workgroup ids are dealt round-robin
constexpr int kGroupM = 8;     // tile rows per group of the grouped tile order

template <typename R, int WM, int WN, int BK, int GM, int GN>
struct GemmShape {
  static constexpr int NT = 64 * GM * GN;           // threads: GM x GN wavefronts
  static constexpr int BM = GM * WM;                // complex rows of the workgroup tile
  static constexpr int BN = GN * WN;                // complex columns
  static constexpr int RT = 2 * WM / 16;            // MFMA blocks per wave, real-row direction
  static constexpr int CT = WN / 16;                // MFMA blocks per wave, column direction
  static constexpr int A_PAD = 64 / sizeof(R);      // 64 B per k row: groups of 16 lanes on
                                                    // alternate bank halves for FP32
  static constexpr int A_LD = 2 * BM + A_PAD;       // reals per k row of the A stage
  static constexpr int B_LD = 2 * BK + 2;           // reals per column of the B stage
  static constexpr int A_ELEMS = BK * A_LD;
  static constexpr int B_ELEMS = BN * B_LD;
  static constexpr int STAGE = A_ELEMS + B_ELEMS;   // reals per LDS buffer
  static constexpr int A_PER_T = BM * BK / NT;      // complex loads per thread per step
  static constexpr int B_PER_T = BN * BK / NT;
  static_assert(BM * BK % NT == 0 && BN * BK % NT == 0, "tile must divide over the threads");
  static_assert(BK % 4 == 0 && WN % 16 == 0 && (2 * WM) % 16 == 0, "MFMA block shape");
};

template <typename R, int WM, int WN, int BK, int GM, int GN>
__global__ __launch_bounds__(64 * GM * GN) void cgemm_sub_kernel(R* __restrict__ C, const R* __restrict__ A,
                                                                 const R* __restrict__ B, int64_t ld, int m,
                                                                 int n, int k, int tiles_m, int tiles_n) {
  using Sh = GemmShape<R, WM, WN, BK, GM, GN>;
  using Acc = typename MfmaAcc<R>::T;
  extern __shared__ __align__(16) unsigned char smem_raw[];
  R* smem = reinterpret_cast<R*>(smem_raw);

  // ---- tile of this workgroup (XCD-aware grouped order) ----
  const int ntiles = tiles_m * tiles_n;
  const int per_xcd = (ntiles + kXcds - 1) / kXcds;
  const int t = (int)(blockIdx.x % kXcds) * per_xcd + (int)(blockIdx.x / kXcds);
  if (t >= ntiles) return;
  const int group = t / (kGroupM * tiles_n);
  const int first_m = group * kGroupM;
  const int gm = min(kGroupM, tiles_m - first_m);
  const int in_group = t - group * kGroupM * tiles_n;
  const int tm = first_m + in_group % gm;
  const int tn = in_group / gm;
  const int m0 = tm * Sh::BM, n0 = tn * Sh::BN;

  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  const int wm = wave % GM, wn = wave / GM;
  const int l16 = lane & 15, g = lane >> 4;

  // ---- global -> register staging ----
  Cx<R> ra[Sh::A_PER_T], rb[Sh::B_PER_T];
  auto load_step = [&](int k0) {
#pragma unroll
    for (int e = 0; e < Sh::A_PER_T; ++e) {
      const int idx = e * Sh::NT + tid;
      const int r = idx % Sh::BM, c = idx / Sh::BM;
      const int gr = m0 + r, gc = k0 + c;
      if (gr < m && gc < k)
        ra[e] = *reinterpret_cast<const Cx<R>*>(A + 2 * ((int64_t)gc * ld + gr));
      else
        ra[e] = Cx<R>{0, 0};
    }
#pragma unroll
    for (int e = 0; e < Sh::B_PER_T; ++e) {
      const int idx = e * Sh::NT + tid;
      const int kk = idx % BK, j = idx / BK;
      const int gk = k0 + kk, gj = n0 + j;
      if (gk < k && gj < n)
        rb[e] = *reinterpret_cast<const Cx<R>*>(B + 2 * ((int64_t)gj * ld + gk));
      else
        rb[e] = Cx<R>{0, 0};
    }
  };
  auto store_step = [&](R* st) {
    R* sa = st;
    R* sb = st + Sh::A_ELEMS;
#pragma unroll
    for (int e = 0; e < Sh::A_PER_T; ++e) {
      const int idx = e * Sh::NT + tid;
      const int r = idx % Sh::BM, c = idx / Sh::BM;
      *reinterpret_cast<Cx<R>*>(sa + c * Sh::A_LD + 2 * r) = ra[e];
    }
#pragma unroll
    for (int e = 0; e < Sh::B_PER_T; ++e) {
      const int idx = e * Sh::NT + tid;
      const int kk = idx % BK, j = idx / BK;
      *reinterpret_cast<Cx<R>*>(sb + j * Sh::B_LD + 2 * kk) = rb[e];
    }
  };

  Acc acc[Sh::RT][Sh::CT];
#pragma unroll
  for (int r = 0; r < Sh::RT; ++r)
#pragma unroll
    for (int c = 0; c < Sh::CT; ++c) acc[r][c] = Acc{0, 0, 0, 0};

  // real row of X this lane supplies for MFMA block r (its partner row is
  // xr ^ 1, negated when xr is even)
  const int prow = MfmaAcc<R>::row_of_lane(l16);
  const int xrow0 = 2 * wm * WM + prow;
  const R sgn = (prow & 1) ? R(1) : R(-1);
  const int bcol0 = wn * WN + l16;

  const int nsteps = (k + BK - 1) / BK;
  load_step(0);
  store_step(smem);
  __syncthreads();
  for (int s = 0; s < nsteps; ++s) {
    const R* st = smem + (s & 1) * Sh::STAGE;
    if (s + 1 < nsteps) load_step((s + 1) * BK);
    const R* sa = st;
    const R* sb = st + Sh::A_ELEMS;
#pragma unroll
    for (int ks = 0; ks < BK / 4; ++ks) {
      const int kk = ks * 4 + g;
      Cx<R> b[Sh::CT];
#pragma unroll
      for (int c = 0; c < Sh::CT; ++c)
        b[c] = *reinterpret_cast<const Cx<R>*>(sb + (bcol0 + c * 16) * Sh::B_LD + 2 * kk);
      const R* arow = sa + kk * Sh::A_LD;
      R x[Sh::RT], xs[Sh::RT];
#pragma unroll
      for (int r = 0; r < Sh::RT; ++r) {
        const int xr = xrow0 + r * 16;
        x[r] = arow[xr];
        xs[r] = sgn * arow[xr ^ 1];
      }
      // all X Br products first, then all Xs Bi: consecutive MFMAs never
      // accumulate into the same registers
#pragma unroll
      for (int r = 0; r < Sh::RT; ++r)
#pragma unroll
        for (int c = 0; c < Sh::CT; ++c) acc[r][c] = MfmaAcc<R>::mma(x[r], b[c].re, acc[r][c]);
#pragma unroll
      for (int r = 0; r < Sh::RT; ++r)
#pragma unroll
        for (int c = 0; c < Sh::CT; ++c) acc[r][c] = MfmaAcc<R>::mma(xs[r], b[c].im, acc[r][c]);
    }
    if (s + 1 < nsteps) store_step(smem + ((s + 1) & 1) * Sh::STAGE);
    __syncthreads();
  }

  // ---- C -= acc: lane holds real rows 4 g .. 4 g + 3 of each block = complex
  // rows 2 g, 2 g + 1, column l16 ----
#pragma unroll
  for (int r = 0; r < Sh::RT; ++r) {
    const int crow = m0 + wm * WM + r * 8 + 2 * g;
#pragma unroll
    for (int c = 0; c < Sh::CT; ++c) {
      const int ccol = n0 + bcol0 + c * 16;
      if (ccol >= n) continue;
      R* col = C + 2 * (int64_t)ccol * ld;
      if (crow < m) {
        Cx<R>* p = reinterpret_cast<Cx<R>*>(col + 2 * (int64_t)crow);
        Cx<R> v = *p;
        v.re -= acc[r][c][0];
        v.im -= acc[r][c][1];
        *p = v;
      }
      if (crow + 1 < m) {
        Cx<R>* p = reinterpret_cast<Cx<R>*>(col + 2 * (int64_t)(crow + 1));
        Cx<R> v = *p;
        v.re -= acc[r][c][2];
        v.im -= acc[r][c][3];
        *p = v;
      }
    }
  }
}

template <typename R, int WM, int WN, int BK, int GM, int GN>
hipError_t launch(hipStream_t stream, R* C, const R* A, const R* B, int64_t ld, int64_t m, int64_t n,
                  int64_t k) {
  using Sh = GemmShape<R, WM, WN, BK, GM, GN>;
  const int64_t tiles_m = (m + Sh::BM - 1) / Sh::BM, tiles_n = (n + Sh::BN - 1) / Sh::BN;
  const int64_t ntiles = tiles_m * tiles_n;
  const int64_t grid = kXcds * ((ntiles + kXcds - 1) / kXcds);
  const size_t lds = 2 * Sh::STAGE * sizeof(R);
  hipLaunchKernelGGL((cgemm_sub_kernel<R, WM, WN, BK, GM, GN>), dim3((unsigned)grid), dim3(Sh::NT), lds, stream,
                     C, A, B, ld, (int)m, (int)n, (int)k, (int)tiles_m, (int)tiles_n);
  return hipGetLastError();
}

// Tile choice (measured on MI355X): on the large updates 128 x 128 complex
// tiles of eight wavefronts (complex128; 67 TFLOP/s at 8192^3) or 128 x 256
// of sixteen (complex64; 134 TFLOP/s), several wavefronts per SIMD, while the
// update still gives every CU at least two tiles; 128 x 64 (complex128) and
// then small four-wavefront tiles for the skinny updates near the leaves of
// the recursion.
constexpr int64_t kTilesPerGrid = 512;

template <typename R>
int64_t tiles(int64_t m, int64_t n, int bm, int bn) {
  return ((m + bm - 1) / bm) * ((n + bn - 1) / bn);
}

}  // namespace

// The large tiles take more than 64 KiB of LDS per workgroup (gfx950 allows
// 160 KiB); they are used only where the device reports room for them.
static bool big_lds_ok(size_t bytes) {
  static int limit = [] {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
      return 0;
    return v;
  }();
  return bytes <= (size_t)limit;
}

hipError_t gemm_sub_c128(hipStream_t stream, double* C, const double* A, const double* B, int64_t ld,
                         int64_t m, int64_t n, int64_t k) {
  if (m <= 0 || n <= 0 || k <= 0) return hipSuccess;
  if (tiles<double>(m, n, 128, 128) >= kTilesPerGrid &&
      big_lds_ok(2 * GemmShape<double, 32, 64, 16, 4, 2>::STAGE * sizeof(double)))
    return launch<double, 32, 64, 16, 4, 2>(stream, C, A, B, ld, m, n, k);
  if (tiles<double>(m, n, 128, 64) >= kTilesPerGrid &&
      big_lds_ok(2 * GemmShape<double, 32, 32, 16, 4, 2>::STAGE * sizeof(double)))
    return launch<double, 32, 32, 16, 4, 2>(stream, C, A, B, ld, m, n, k);
  return launch<double, 32, 16, 16, 2, 2>(stream, C, A, B, ld, m, n, k);
}

hipError_t gemm_sub_c64(hipStream_t stream, float* C, const float* A, const float* B, int64_t ld,
                        int64_t m, int64_t n, int64_t k) {
  if (m <= 0 || n <= 0 || k <= 0) return hipSuccess;
  if (tiles<float>(m, n, 128, 256) >= 2 * kTilesPerGrid &&
      big_lds_ok(2 * GemmShape<float, 32, 64, 16, 4, 4>::STAGE * sizeof(float)))
    return launch<float, 32, 64, 16, 4, 4>(stream, C, A, B, ld, m, n, k);
  return launch<float, 32, 32, 16, 2, 2>(stream, C, A, B, ld, m, n, k);
}

}  // namespace ffbie
