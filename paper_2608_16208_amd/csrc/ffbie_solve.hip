// Dense solvers for the single-layer system S phi~ = g (paper Sec. 3.4; the
// paper does not name a solver).
//
// S is row-major (one row per collocation point).  Read as a column-major
// array the same memory is A = S^T, and A is factored with partial (row)
// pivoting, A = P L U, so the pivot search scans a contiguous column of A;
// then S = U^T L^T P^T and S phi = g is solved by a forward substitution with
// U^T, a backward one with L^T (rows of both are contiguous rows of S) and the
// permutation P.  The factorisation is recursive (split the columns in halves:
// factor the left half, apply its interchanges to the right half, triangular
// solve with the unit-lower block, trailing update, factor the trailing part,
// apply its interchanges back to the left half).  The trailing updates are
// complex GEMMs on the matrix cores (ffbie_gemm.hip); the pivot search,
// interchanges, small triangular solves, substitutions, residuals and
// precision conversion are the kernels below.  The same code runs in complex128 (LU64) and complex64 (the
// LU32 factor of mixed-precision refinement).
//
// Methods:
//   LU64       factor S in place (S is overwritten), solve;
//   LU32+IR64  factor a complex64 copy, then iterative refinement with the
//              residual g - S phi evaluated in complex128 against the untouched S;
//   GMRES      restarted GMRES in complex128 with the row-major matrix-vector
//              product (classical Gram-Schmidt with one re-orthogonalisation).
#include <cmath>
#include <complex>
#include <vector>

#include "ffbie_gemm.hpp"
#include "ffbie_solve.hpp"

namespace ffbie {

namespace {

template <typename R>
struct C2 {
  R re, im;
};

template <typename R>
__device__ __forceinline__ C2<R> cmul(C2<R> a, C2<R> b) {
  return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}
template <typename R>
__device__ __forceinline__ C2<R> csub(C2<R> a, C2<R> b) {
  return {a.re - b.re, a.im - b.im};
}

// ---------------------------------------------------------------------------
// Unblocked LU of a panel of at most kPanel columns of A (the leaves of the
// recursive factorisation).  The panel's rows r0 .. r0+m-1 are split once into
// nb fixed chunks of `chunk` rows, one per workgroup, for all of its columns:
//   panel_search0: each workgroup writes the largest |Re| + |Im| of column c0
//     over its rows (first index on ties), that row index and the row's values
//     on the panel's columns to part[b]; the owner of row r0 also saves that row
//     in part[nb];
//   panel_step(k), one launch per column: every workgroup reduces part[0..nb)
//     to the pivot row p of column k (the same result in each) and updates only
//     its own rows >= r0+k: the interchange of rows r0+k and p on the panel's
//     columns, the scaling of column k below the pivot and the rank-1 update of
//     columns k+1.. .  Rows p and r0+k come from part, so no workgroup reads a
//     row another one writes.  Then, while its rows are at hand, it searches the
//     updated column k+1 over its rows >= r0+k+1 and writes the candidate (and,
//     for the owner, row r0+k+1) to the second part buffer, which the launch
//     for column k+1 reads.  One launch per column instead of a search and an
//     apply launch.
// ---------------------------------------------------------------------------
constexpr int kPanel = 4;

template <typename R>
struct PanelPart {
  R val;
  int64_t idx;
  C2<R> row[kPanel];
};

// Workgroup-wide arg-max of |Re| + |Im| (ties: lowest row) of the candidates
// (b, w) of each thread; returns the winner in best[0], where[0].
template <typename R>
__device__ void block_argmax(R b, int64_t w, R* best, int64_t* where) {
  best[threadIdx.x] = b;
  where[threadIdx.x] = w;
  __syncthreads();
  for (int s = blockDim.x / 2; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      const R o = best[threadIdx.x + s];
      const int64_t ow = where[threadIdx.x + s];
      if (o > best[threadIdx.x] || (o == best[threadIdx.x] && ow < where[threadIdx.x])) {
        best[threadIdx.x] = o;
        where[threadIdx.x] = ow;
      }
    }
    __syncthreads();
  }
}

// Candidate of this workgroup for column c0+k over its rows [beg, end) (an
// empty range keeps val = -1 and reads no row), and row `diag` of the panel
// into part[nb] if this workgroup owns it.  Reads only rows this workgroup
// owns; the caller has made its own writes to them visible (barrier).
template <typename R>
__device__ void panel_candidate(const C2<R>* S, int64_t ld, int64_t c0, int nc, int k, int64_t beg,
                                int64_t end, int64_t own_beg, int64_t own_end, int64_t diag,
                                PanelPart<R>* part, int nb, R* best, int64_t* where) {
  const C2<R>* col = S + (c0 + k) * ld;
  R b = -1;
  int64_t w = beg;
  for (int64_t r = beg + threadIdx.x; r < end; r += blockDim.x) {
    const C2<R> v = col[r];
    const R a = fabs(v.re) + fabs(v.im);
    if (a > b) {
      b = a;
      w = r;
    }
  }
  block_argmax(b, w, best, where);
  if ((int)threadIdx.x < nc) {
    const int j = threadIdx.x;
    if (best[0] >= 0) part[blockIdx.x].row[j] = S[(c0 + j) * ld + where[0]];
    if (diag >= own_beg && diag < own_end) part[nb].row[j] = S[(c0 + j) * ld + diag];
  }
  if (threadIdx.x == 0) {
    part[blockIdx.x].val = best[0];
    part[blockIdx.x].idx = where[0];
  }
}

template <typename R>
__global__ __launch_bounds__(256) void panel_search0_kernel(const C2<R>* S, int64_t ld, int64_t r0,
                                                            int64_t m, int64_t c0, int nc,
                                                            int64_t chunk, PanelPart<R>* part, int nb) {
  __shared__ R best[256];
  __shared__ int64_t where[256];
  const int64_t own_beg = r0 + blockIdx.x * chunk, own_end = min(r0 + m, own_beg + chunk);
  panel_candidate(S, ld, c0, nc, 0, own_beg, own_end, own_beg, own_end, r0, part, nb, best, where);
}

template <typename R>
__global__ __launch_bounds__(256) void panel_step_kernel(C2<R>* S, int64_t ld, int64_t r0, int64_t m,
                                                         int64_t c0, int nc, int k, int64_t chunk,
                                                         const PanelPart<R>* part, PanelPart<R>* next,
                                                         int nb, int64_t* ipiv, int* info) {
  __shared__ R best[256];
  __shared__ int64_t where[256];
  __shared__ C2<R> prow[kPanel], krow[kPanel];
  // pivot of column k: reduce the candidates (chunks in row order: the first
  // chunk wins ties)
  {
    R b = -2;
    int64_t w = 0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) {
      const R o = part[i].val;
      if (o > b) {
        b = o;
        w = i;
      }
    }
    block_argmax(b, w, best, where);
  }
  const int wb = (int)where[0];
  const int64_t p = part[wb].idx;
  const bool zero = !(part[wb].val > 0);
  if ((int)threadIdx.x < nc) {
    prow[threadIdx.x] = part[wb].row[threadIdx.x];
    krow[threadIdx.x] = part[nb].row[threadIdx.x];
  }
  __syncthreads();
  const int64_t rk = r0 + k;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    ipiv[c0 + k] = p;
    if (zero && *info == 0) *info = (int)(c0 + k + 1);
  }
  const int64_t own_beg = r0 + blockIdx.x * chunk, own_end = min(r0 + m, own_beg + chunk);
  const int64_t beg = max(rk, own_beg);
  if (!zero) {                               // an all-zero column: no interchange, no update
    const C2<R> piv = prow[k];
    const R den = piv.re * piv.re + piv.im * piv.im;
    const C2<R> inv = {piv.re / den, -piv.im / den};
    for (int64_t r = beg + threadIdx.x; r < own_end; r += blockDim.x) {
      if (r == rk) {
#pragma unroll
        for (int j = 0; j < kPanel; ++j)
          if (j < nc) S[(c0 + j) * ld + r] = prow[j];
        continue;
      }
      const bool is_p = r == p;
      // the row after the interchange: row p takes old row r0+k (from part)
      C2<R> v[kPanel];
#pragma unroll
      for (int j = 0; j < kPanel; ++j)
        if (j >= k && j < nc) v[j] = is_p ? krow[j] : S[(c0 + j) * ld + r];
      C2<R> l = {0, 0};
#pragma unroll
      for (int j = 0; j < kPanel; ++j)
        if (j == k) l = cmul(v[j], inv);
#pragma unroll
      for (int j = 0; j < kPanel; ++j) {
        if (j >= nc) break;
        if (j < k) {
          if (is_p) S[(c0 + j) * ld + r] = krow[j];
        } else if (j == k) {
          S[(c0 + j) * ld + r] = l;
        } else {
          const C2<R> u = cmul(l, prow[j]);
          S[(c0 + j) * ld + r] = C2<R>{v[j].re - u.re, v[j].im - u.im};
        }
      }
    }
  }
  if (k + 1 >= nc) return;
  __syncthreads();                           // this workgroup's row updates are visible to it
  panel_candidate(S, ld, c0, nc, k + 1, max(rk + 1, own_beg), own_end, own_beg, own_end, rk + 1, next,
                  nb, best, where);
}

// Row interchanges k0..k1-1 (in order) of A on its columns [c0, c1): one
// thread per column (a contiguous row segment of S).
template <typename R>
__global__ __launch_bounds__(256) void laswp_kernel(C2<R>* S, int64_t ld, int64_t k0, int64_t k1,
                                                    const int64_t* __restrict__ ipiv, int64_t c0,
                                                    int64_t c1) {
  const int64_t c = c0 + blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= c1) return;
  for (int64_t k = k0; k < k1; ++k) {
    const int64_t p = ipiv[k];
    if (p != k) {
      C2<R>* colw = S + c * ld;
      const C2<R> t = colw[k];
      colw[k] = colw[p];
      colw[p] = t;
    }
  }
}

// X = L^{-1} X for a unit-lower n x n block L of A (n <= kTrsmBase) at rows
// [r0, r0+n), columns [cl, cl+n), and X at rows [r0, r0+n), columns [cx, cx+nx).
constexpr int kTrsmBase = 16;

template <typename R>
__global__ __launch_bounds__(256) void trsm_base_kernel(C2<R>* S, int64_t ld, int64_t r0, int n,
                                                        int64_t cl, int64_t cx, int64_t nx) {
  __shared__ C2<R> L[kTrsmBase][kTrsmBase];                  // L[i][k] = A(r0 + i, cl + k)
  for (int e = threadIdx.x; e < n * n; e += blockDim.x) L[e % n][e / n] = S[(cl + e / n) * ld + r0 + e % n];
  __syncthreads();
  const int64_t j = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (j >= nx) return;
  C2<R>* xcol = S + (cx + j) * ld + r0;                      // column cx + j of A
  C2<R> x[kTrsmBase];
#pragma unroll
  for (int i = 0; i < kTrsmBase; ++i) {
    if (i < n) {
      C2<R> v = xcol[i];
      for (int k = 0; k < i; ++k) v = csub(v, cmul(L[i][k], x[k]));
      x[i] = v;
      xcol[i] = v;
    }
  }
}

template <typename R>
__global__ void convert_kernel(const C2<double>* __restrict__ src, int64_t lds, C2<R>* dst,
                               int64_t ldd, int64_t N) {
  const int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (c >= N) return;
  for (int64_t r = blockIdx.y; r < N; r += gridDim.y) {
    const C2<double> v = src[r * lds + c];
    dst[r * ldd + c] = C2<R>{(R)v.re, (R)v.im};
  }
}

// ---------------------------------------------------------------------------
// triangular solves with the row-major factors, blocks of kSolveBlock rows
// ---------------------------------------------------------------------------
constexpr int kSolveBlock = 32;

// Solve the diagonal block [k0, k0+nb) of a triangular matrix T with
// T(i, j) = S[i*ld + j] in place: LOWER (forward, T = U^T, non-unit) or upper
// (backward, T = L^T, unit diagonal).  The block is staged in LDS; lane j holds
// y_j and the solved value is broadcast across the wavefront step by step.
template <typename R, bool LOWER>
__global__ __launch_bounds__(64) void tri_diag_kernel(const C2<R>* S, int64_t ld, int64_t k0,
                                                      int nb, C2<R>* y) {
  __shared__ C2<R> T[kSolveBlock][kSolveBlock];
  const int lane = threadIdx.x;
  for (int e = lane; e < nb * nb; e += 64) T[e / nb][e % nb] = S[(k0 + e / nb) * ld + k0 + e % nb];
  __syncthreads();
  C2<R> v = (lane < nb) ? y[k0 + lane] : C2<R>{0, 0};
  if (LOWER) {
    for (int i = 0; i < nb; ++i) {
      if (lane == i) {
        const C2<R> d = T[i][i];
        const R den = d.re * d.re + d.im * d.im;
        v = C2<R>{(v.re * d.re + v.im * d.im) / den, (v.im * d.re - v.re * d.im) / den};
      }
      const C2<R> yi = {__shfl(v.re, i), __shfl(v.im, i)};
      if (lane > i && lane < nb) v = csub(v, cmul(T[lane][i], yi));
    }
  } else {
    for (int i = nb - 1; i >= 0; --i) {
      const C2<R> yi = {__shfl(v.re, i), __shfl(v.im, i)};
      if (lane < i) v = csub(v, cmul(T[lane][i], yi));
    }
  }
  if (lane < nb) y[k0 + lane] = v;
}

// y[r] -= sum_{c in block} S[r][c] y[c] for rows r in [r_begin, r_end): one wave per row.
template <typename R>
__global__ __launch_bounds__(256) void tri_update_kernel(const C2<R>* S, int64_t ld, int64_t k0,
                                                         int nb, int64_t r_begin, int64_t r_end,
                                                         C2<R>* y) {
  const int lane = threadIdx.x & 63;
  const int64_t r = r_begin + blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= r_end) return;
  R sr = 0, si = 0;
  if (lane < nb) {
    const C2<R> a = S[r * ld + k0 + lane];
    const C2<R> b = y[k0 + lane];
    sr = a.re * b.re - a.im * b.im;
    si = a.re * b.im + a.im * b.re;
  }
  for (int o = 32; o > 0; o >>= 1) {
    sr += __shfl_xor(sr, o);
    si += __shfl_xor(si, o);
  }
  if (lane == 0) {
    C2<R> v = y[r];
    y[r] = C2<R>{v.re - sr, v.im - si};
  }
}

// out[r] = b[r] - sum_c S[r][c] x[c] (complex128), one wave per row.
__global__ __launch_bounds__(256) void residual_kernel(const C2<double>* __restrict__ S, int64_t ld,
                                                       int64_t N, const C2<double>* __restrict__ x,
                                                       const C2<double>* __restrict__ b,
                                                       C2<double>* out, double alpha) {
  const int lane = threadIdx.x & 63;
  const int64_t r = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (r >= N) return;
  double sr = 0, si = 0;
  const C2<double>* row = S + r * ld;
  for (int64_t c = lane; c < N; c += 64) {
    const C2<double> a = row[c], v = x[c];
    sr = fma(a.re, v.re, fma(-a.im, v.im, sr));
    si = fma(a.re, v.im, fma(a.im, v.re, si));
  }
  for (int o = 32; o > 0; o >>= 1) {
    sr += __shfl_xor(sr, o);
    si += __shfl_xor(si, o);
  }
  if (lane == 0) {
    const C2<double> bb = b ? b[r] : C2<double>{0, 0};
    out[r] = C2<double>{bb.re - alpha * sr, bb.im - alpha * si};
  }
}

template <typename R>
__global__ void gather_kernel(const C2<R>* src, const int64_t* perm, C2<R>* dst, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) dst[i] = src[perm[i]];
}

template <typename R>
__global__ void to_prec_kernel(const C2<double>* src, C2<R>* dst, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) dst[i] = C2<R>{(R)src[i].re, (R)src[i].im};
}

__global__ void add_kernel(C2<double>* x, const C2<float>* d, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) x[i] = C2<double>{x[i].re + (double)d[i].re, x[i].im + (double)d[i].im};
}

// partial sums of conj(a_k) . w for k < nv (columns of V, stride N), and of |w|^2
__global__ __launch_bounds__(256) void multidot_kernel(const C2<double>* V, int64_t N, int nv,
                                                       const C2<double>* w, C2<double>* partial,
                                                       int nblk) {
  __shared__ double red[2][256];
  const int k = blockIdx.y;
  const C2<double>* a = (k < nv) ? V + (int64_t)k * N : w;
  double sr = 0, si = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < N;
       i += (int64_t)gridDim.x * blockDim.x) {
    const C2<double> p = a[i], q = w[i];
    sr = fma(p.re, q.re, fma(p.im, q.im, sr));
    si = fma(p.re, q.im, fma(-p.im, q.re, si));
  }
  red[0][threadIdx.x] = sr;
  red[1][threadIdx.x] = si;
  __syncthreads();
  for (int s = 128; s > 0; s >>= 1) {
    if ((int)threadIdx.x < s) {
      red[0][threadIdx.x] += red[0][threadIdx.x + s];
      red[1][threadIdx.x] += red[1][threadIdx.x + s];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[k * nblk + blockIdx.x] = C2<double>{red[0][0], red[1][0]};
}

// w -= sum_k h_k V_k ; then optionally scale w into V_out: V_out = w / nrm
__global__ void orth_update_kernel(const C2<double>* V, int64_t N, int nv, const C2<double>* h,
                                   C2<double>* w) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= N) return;
  C2<double> v = w[i];
  for (int k = 0; k < nv; ++k) {
    const C2<double> a = V[(int64_t)k * N + i], c = h[k];
    v.re -= c.re * a.re - c.im * a.im;
    v.im -= c.re * a.im + c.im * a.re;
  }
  w[i] = v;
}

__global__ void scale_copy_kernel(const C2<double>* w, double s, C2<double>* out, int64_t N) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < N) out[i] = C2<double>{w[i].re * s, w[i].im * s};
}

// x += sum_k y_k V_k
__global__ void combine_kernel(const C2<double>* V, int64_t N, int nv, const C2<double>* y,
                               C2<double>* x) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= N) return;
  C2<double> v = x[i];
  for (int k = 0; k < nv; ++k) {
    const C2<double> a = V[(int64_t)k * N + i], c = y[k];
    v.re += c.re * a.re - c.im * a.im;
    v.im += c.re * a.im + c.im * a.re;
  }
  x[i] = v;
}

// ---------------------------------------------------------------------------
// host-side recursion
// ---------------------------------------------------------------------------
inline dim3 grid1(int64_t n, int b = 256) { return dim3((unsigned)((n + b - 1) / b)); }

// Panel steps: up to kPivotBlocks workgroups of >= kPivotRows rows each.
constexpr int kPivotBlocks = 128;
constexpr int64_t kPivotRows = 1024;

// A(rC.., cC..) (m x n) -= A(rA.., cA..) (m x k) * A(rB.., cB..) (k x n), with
// A(r, c) = S[c*ld + r] the column-major view.
hipError_t gemm_sub(hipStream_t st, C2<double>* S, int64_t ld, int64_t r_a, int64_t c_a, int64_t r_b,
                    int64_t c_b, int64_t r_c, int64_t c_c, int64_t m, int64_t n, int64_t k) {
  auto p = [&](int64_t r, int64_t c) { return reinterpret_cast<double*>(S + c * ld + r); };
  return gemm_sub_c128(st, p(r_c, c_c), p(r_a, c_a), p(r_b, c_b), ld, m, n, k);
}
hipError_t gemm_sub(hipStream_t st, C2<float>* S, int64_t ld, int64_t r_a, int64_t c_a, int64_t r_b,
                    int64_t c_b, int64_t r_c, int64_t c_c, int64_t m, int64_t n, int64_t k) {
  auto p = [&](int64_t r, int64_t c) { return reinterpret_cast<float*>(S + c * ld + r); };
  return gemm_sub_c64(st, p(r_c, c_c), p(r_a, c_a), p(r_b, c_b), ld, m, n, k);
}

struct Err {
  hipError_t hip = hipSuccess;
  bool ok() const { return hip == hipSuccess; }
};

// X (rows [r0, r0+n), cols [cx, cx+nx)) = L^{-1} X, L unit lower at cols [cl, cl+n).
template <typename R>
void trsm_rec(SolveCtx& sc, C2<R>* S, int64_t ld, int64_t r0, int64_t n, int64_t cl, int64_t cx,
              int64_t nx, Err& e) {
  if (!e.ok() || n <= 1 || nx <= 0) return;
  if (n <= kTrsmBase) {
    hipLaunchKernelGGL(trsm_base_kernel<R>, grid1(nx), dim3(256), 0, sc.stream, S, ld, r0, (int)n,
                       cl, cx, nx);
    e.hip = hipGetLastError();
    return;
  }
  const int64_t n1 = n / 2, n2 = n - n1;
  trsm_rec(sc, S, ld, r0, n1, cl, cx, nx, e);
  if (!e.ok()) return;
  e.hip = gemm_sub(sc.stream, S, ld, r0 + n1, cl, r0, cx, r0 + n1, cx, n2, nx, n1);
  if (!e.ok()) return;
  trsm_rec(sc, S, ld, r0 + n1, n2, cl + n1, cx, nx, e);
}

// Factor rows [r0, r0+m) x cols [c0, c0+n) (m >= n), row interchanges recorded
// in ipiv[c0 .. c0+n) as absolute row indices, applied inside these columns.
template <typename R>
void getrf_rec(SolveCtx& sc, C2<R>* S, int64_t ld, int64_t r0, int64_t m, int64_t c0, int64_t n,
               int64_t* ipiv, int* info, Err& e) {
  if (!e.ok()) return;
  if (n <= kPanel) {
    auto* part = reinterpret_cast<PanelPart<R>*>(sc.partial);
    const int nb = (int)std::min<int64_t>(kPivotBlocks, (m + kPivotRows - 1) / kPivotRows);
    const int64_t chunk = (m + nb - 1) / nb;
    PanelPart<R>* buf[2] = {part, part + (nb + 1)};
    hipLaunchKernelGGL(panel_search0_kernel<R>, dim3(nb), dim3(256), 0, sc.stream, S, ld, r0, m, c0,
                       (int)n, chunk, buf[0], nb);
    for (int k = 0; k < (int)n && k < m; ++k)
      hipLaunchKernelGGL(panel_step_kernel<R>, dim3(nb), dim3(256), 0, sc.stream, S, ld, r0, m, c0,
                         (int)n, k, chunk, buf[k & 1], buf[(k + 1) & 1], nb, ipiv, info);
    e.hip = hipGetLastError();
    return;
  }
  const int64_t n1 = n / 2, n2 = n - n1;
  getrf_rec(sc, S, ld, r0, m, c0, n1, ipiv, info, e);
  if (!e.ok()) return;
  hipLaunchKernelGGL(laswp_kernel<R>, grid1(n2), dim3(256), 0, sc.stream, S, ld, c0, c0 + n1,
                     ipiv, c0 + n1, c0 + n);
  e.hip = hipGetLastError();
  trsm_rec(sc, S, ld, r0, n1, c0, c0 + n1, n2, e);
  if (!e.ok()) return;
  e.hip = gemm_sub(sc.stream, S, ld, r0 + n1, c0, r0, c0 + n1, r0 + n1, c0 + n1, m - n1, n2, n1);
  if (!e.ok()) return;
  getrf_rec(sc, S, ld, r0 + n1, m - n1, c0 + n1, n2, ipiv, info, e);
  if (!e.ok()) return;
  hipLaunchKernelGGL(laswp_kernel<R>, grid1(n1), dim3(256), 0, sc.stream, S, ld, c0 + n1, c0 + n,
                     ipiv, c0, c0 + n1);
  e.hip = hipGetLastError();
}

// y := L^{-T} U^{-T} y: forward substitution with U^T, backward with L^T.
template <typename R>
hipError_t lu_substitute(SolveCtx& sc, const C2<R>* S, int64_t ld, int64_t N, C2<R>* y) {
  for (int64_t k0 = 0; k0 < N; k0 += kSolveBlock) {
    const int nb = (int)std::min<int64_t>(kSolveBlock, N - k0);
    hipLaunchKernelGGL((tri_diag_kernel<R, true>), dim3(1), dim3(64), 0, sc.stream, S, ld, k0, nb, y);
    if (k0 + nb < N)
      hipLaunchKernelGGL(tri_update_kernel<R>, grid1(N - k0 - nb, 4), dim3(256), 0, sc.stream, S,
                         ld, k0, nb, k0 + nb, N, y);
  }
  for (int64_t k1 = N; k1 > 0; k1 -= kSolveBlock) {
    const int64_t k0 = std::max<int64_t>(0, k1 - kSolveBlock);
    const int nb = (int)(k1 - k0);
    hipLaunchKernelGGL((tri_diag_kernel<R, false>), dim3(1), dim3(64), 0, sc.stream, S, ld, k0, nb,
                       y);
    if (k0 > 0)
      hipLaunchKernelGGL(tri_update_kernel<R>, grid1(k0, 4), dim3(256), 0, sc.stream, S, ld, k0, nb,
                         (int64_t)0, k0, y);
  }
  return hipGetLastError();
}

// x = P z for A = P L U: the interchanges applied in reverse order; q[i] is the
// index of z that lands at position i.
std::vector<int64_t> compose_perm(const std::vector<int64_t>& ipiv) {
  const int64_t N = (int64_t)ipiv.size();
  std::vector<int64_t> q(N);
  for (int64_t i = 0; i < N; ++i) q[i] = i;
  for (int64_t k = N - 1; k >= 0; --k) std::swap(q[k], q[ipiv[k]]);
  return q;
}

double norm2(SolveCtx& sc, const C2<double>* v, int64_t N, hipError_t* err) {
  const int nblk = 256;
  hipLaunchKernelGGL(multidot_kernel, dim3(nblk, 1), dim3(256), 0, sc.stream, v, N, 0, v,
                     reinterpret_cast<C2<double>*>(sc.partial), nblk);
  std::vector<C2<double>> h(nblk);
  *err = hipMemcpyAsync(h.data(), sc.partial, nblk * sizeof(C2<double>), hipMemcpyDeviceToHost,
                        sc.stream);
  if (*err == hipSuccess) *err = hipStreamSynchronize(sc.stream);
  double s = 0;
  for (auto& x : h) s += x.re;
  return std::sqrt(s);
}

}  // namespace

// ---------------------------------------------------------------------------
// entry points used by the C ABI
// ---------------------------------------------------------------------------
template <typename R>
static SolveResult lu_factor_solve_t(SolveCtx& sc, C2<R>* S, int64_t ld, int64_t N, C2<R>* y,
                                     bool factor) {
  SolveResult res;
  if (factor) {
    Err e;
    hipError_t he = hipMemsetAsync(sc.info, 0, sizeof(int), sc.stream);
    if (he != hipSuccess) { res.hip = he; return res; }
    getrf_rec(sc, S, ld, 0, N, 0, N, sc.ipiv, sc.info, e);
    if (!e.ok()) { res.hip = e.hip; return res; }
    int info = 0;
    std::vector<int64_t> ipiv(N);
    res.hip = hipMemcpyAsync(&info, sc.info, sizeof(int), hipMemcpyDeviceToHost, sc.stream);
    if (res.hip == hipSuccess)
      res.hip = hipMemcpyAsync(ipiv.data(), sc.ipiv, N * sizeof(int64_t), hipMemcpyDeviceToHost, sc.stream);
    if (res.hip == hipSuccess) res.hip = hipStreamSynchronize(sc.stream);
    if (res.hip != hipSuccess) return res;
    res.singular_col = info;
    const std::vector<int64_t> perm = compose_perm(ipiv);
    res.hip = hipMemcpyAsync(sc.perm, perm.data(), N * sizeof(int64_t), hipMemcpyHostToDevice, sc.stream);
    if (res.hip != hipSuccess) return res;
    res.hip = hipStreamSynchronize(sc.stream);
    if (res.hip != hipSuccess || info != 0) return res;
  }
  res.hip = lu_substitute(sc, S, ld, N, y);
  if (res.hip != hipSuccess) return res;
  C2<R>* tmp = reinterpret_cast<C2<R>*>(sc.vec_tmp);
  hipLaunchKernelGGL(gather_kernel<R>, grid1(N), dim3(256), 0, sc.stream, y, sc.perm, tmp, N);
  res.hip = hipMemcpyAsync(y, tmp, N * sizeof(C2<R>), hipMemcpyDeviceToDevice, sc.stream);
  return res;
}

SolveResult lu64_factor_solve(SolveCtx& sc, cplx* S, int64_t ld, int64_t N, cplx* y) {
  return lu_factor_solve_t(sc, reinterpret_cast<C2<double>*>(S), ld, N,
                           reinterpret_cast<C2<double>*>(y), true);
}

SolveResult lu64_solve_factored(SolveCtx& sc, const cplx* S, int64_t ld, int64_t N, cplx* y) {
  return lu_factor_solve_t(sc, const_cast<C2<double>*>(reinterpret_cast<const C2<double>*>(S)), ld, N,
                           reinterpret_cast<C2<double>*>(y), false);
}

SolveResult lu32_ir64(SolveCtx& sc, const cplx* S, int64_t ld, int64_t N, const cplx* g, cplx* x,
                      double tol, int max_iter, int* iters, double* rel_res) {
  SolveResult res;
  auto* S64 = reinterpret_cast<const C2<double>*>(S);
  auto* g64 = reinterpret_cast<const C2<double>*>(g);
  auto* x64 = reinterpret_cast<C2<double>*>(x);
  auto* S32 = reinterpret_cast<C2<float>*>(sc.s32);
  auto* r64 = reinterpret_cast<C2<double>*>(sc.vec_r);
  auto* d32 = reinterpret_cast<C2<float>*>(sc.vec_d);
  hipLaunchKernelGGL(convert_kernel<float>, dim3((unsigned)((N + 255) / 256), (unsigned)std::min<int64_t>(N, 8192)), dim3(256),
                     0, sc.stream, S64, ld, S32, N, N);
  res.hip = hipGetLastError();
  if (res.hip != hipSuccess) return res;
  // x = 0, r = g
  res.hip = hipMemsetAsync(x64, 0, N * sizeof(C2<double>), sc.stream);
  if (res.hip != hipSuccess) return res;
  res.hip = hipMemcpyAsync(r64, g64, N * sizeof(C2<double>), hipMemcpyDeviceToDevice, sc.stream);
  if (res.hip != hipSuccess) return res;
  hipError_t he;
  const double gn = norm2(sc, g64, N, &he);
  if (he != hipSuccess) { res.hip = he; return res; }
  double rn = gn;
  int it = 0;
  bool factored = false;
  while (true) {
    if (gn == 0 || rn <= tol * gn || it >= max_iter) break;
    hipLaunchKernelGGL(to_prec_kernel<float>, grid1(N), dim3(256), 0, sc.stream, r64, d32, N);
    SolveResult s = lu_factor_solve_t(sc, S32, N, N, d32, !factored);
    factored = true;
    if (s.hip != hipSuccess || s.singular_col != 0) return s;
    hipLaunchKernelGGL(add_kernel, grid1(N), dim3(256), 0, sc.stream, x64, d32, N);
    hipLaunchKernelGGL(residual_kernel, grid1(N, 4), dim3(256), 0, sc.stream, S64, ld, N, x64, g64,
                       r64, 1.0);
    rn = norm2(sc, r64, N, &he);
    if (he != hipSuccess) { res.hip = he; return res; }
    ++it;
  }
  *iters = it;
  *rel_res = gn > 0 ? rn / gn : 0.0;
  res.converged = gn == 0 || rn <= tol * gn;
  return res;
}

// Restarted GMRES; with a preconditioner, flexible GMRES (right preconditioning
// z_j = P(v_j), x = x0 + Z y, which allows P to change between applications).
// x0 = 0, or x0 = P(g) when `guess` is set.
SolveResult gmres_core(SolveCtx& sc, const cplx* S, int64_t ld, int64_t N, const cplx* g, cplx* x,
                       double tol, int max_iter, int restart, const Precond* P, bool guess,
                       bool keep_x, int* iters, double* rel_res) {
  SolveResult res;
  auto* S64 = reinterpret_cast<const C2<double>*>(S);
  auto* g64 = reinterpret_cast<const C2<double>*>(g);
  auto* x64 = reinterpret_cast<C2<double>*>(x);
  auto* V = reinterpret_cast<C2<double>*>(sc.krylov);        // [restart+1][N]
  auto* Z = reinterpret_cast<C2<double>*>(sc.zbasis);        // [restart][N] (flexible variant)
  auto* w = reinterpret_cast<C2<double>*>(sc.vec_r);
  auto* hdev = reinterpret_cast<C2<double>*>(sc.hvec);
  const int nblk = 256;
  hipError_t he;
  if (P && guess) {
    res.hip = P->apply(P->self, g, x);
  } else if (!keep_x) {
    res.hip = hipMemsetAsync(x64, 0, N * sizeof(C2<double>), sc.stream);
  }
  if (res.hip != hipSuccess) return res;
  const double gn = norm2(sc, g64, N, &he);
  if (he != hipSuccess) { res.hip = he; return res; }
  if (gn == 0) { *iters = 0; *rel_res = 0; res.converged = true; return res; }
  int total = 0;
  double rn = gn;
  using cd = std::complex<double>;
  // every cycle starts from the true residual of the current iterate, so a
  // cycle that ends on the Givens estimate reaching tol is confirmed (or
  // continued) against g - S x
  while (true) {
    // r = g - S x -> V_0
    hipLaunchKernelGGL(residual_kernel, grid1(N, 4), dim3(256), 0, sc.stream, S64, ld, N, x64, g64, w, 1.0);
    const double beta = norm2(sc, w, N, &he);
    if (he != hipSuccess) { res.hip = he; return res; }
    rn = beta;
    if (rn <= tol * gn || total >= max_iter) break;
    hipLaunchKernelGGL(scale_copy_kernel, grid1(N), dim3(256), 0, sc.stream, w, 1.0 / beta, V, N);
    std::vector<cd> Hc((restart + 1) * restart, 0.0), cs(restart), sn(restart), e1(restart + 1, 0.0);
    e1[0] = beta;
    int j = 0;
    for (; j < restart && total < max_iter; ++j, ++total) {
      // w = S V_j, or w = S Z_j with Z_j = P(V_j)
      const C2<double>* src = V + (int64_t)j * N;
      if (P) {
        he = P->apply(P->self, reinterpret_cast<const cplx*>(src), reinterpret_cast<cplx*>(Z + (int64_t)j * N));
        if (he != hipSuccess) { res.hip = he; return res; }
        src = Z + (int64_t)j * N;
      }
      hipLaunchKernelGGL(residual_kernel, grid1(N, 4), dim3(256), 0, sc.stream, S64, ld, N, src,
                         (const C2<double>*)nullptr, w, -1.0);
      std::vector<cd> hcol(j + 2, 0.0);
      for (int pass = 0; pass < 2; ++pass) {
        hipLaunchKernelGGL(multidot_kernel, dim3(nblk, j + 1), dim3(256), 0, sc.stream, V, N, j + 1,
                           w, reinterpret_cast<C2<double>*>(sc.partial), nblk);
        std::vector<C2<double>> part((j + 1) * nblk);
        he = hipMemcpyAsync(part.data(), sc.partial, part.size() * sizeof(C2<double>),
                            hipMemcpyDeviceToHost, sc.stream);
        if (he == hipSuccess) he = hipStreamSynchronize(sc.stream);
        if (he != hipSuccess) { res.hip = he; return res; }
        std::vector<C2<double>> hk(j + 1);
        for (int k = 0; k <= j; ++k) {
          double a = 0, b = 0;
          for (int q = 0; q < nblk; ++q) { a += part[k * nblk + q].re; b += part[k * nblk + q].im; }
          hk[k] = C2<double>{a, b};
          hcol[k] += cd(a, b);
        }
        he = hipMemcpyAsync(hdev, hk.data(), (j + 1) * sizeof(C2<double>), hipMemcpyHostToDevice, sc.stream);
        if (he != hipSuccess) { res.hip = he; return res; }
        hipLaunchKernelGGL(orth_update_kernel, grid1(N), dim3(256), 0, sc.stream, V, N, j + 1, hdev, w);
      }
      const double hn = norm2(sc, w, N, &he);
      if (he != hipSuccess) { res.hip = he; return res; }
      hcol[j + 1] = hn;
      if (hn > 0)
        hipLaunchKernelGGL(scale_copy_kernel, grid1(N), dim3(256), 0, sc.stream, w, 1.0 / hn,
                           V + (int64_t)(j + 1) * N, N);
      // Givens rotations
      for (int k = 0; k < j; ++k) {
        const cd t = cs[k] * hcol[k] + sn[k] * hcol[k + 1];
        hcol[k + 1] = -std::conj(sn[k]) * hcol[k] + cs[k] * hcol[k + 1];
        hcol[k] = t;
      }
      // complex Givens rotation with real cosine zeroing hcol[j+1]
      const double den = std::sqrt(std::norm(hcol[j]) + std::norm(hcol[j + 1]));
      {
        const double a = std::abs(hcol[j]);
        if (a == 0) {
          cs[j] = 0.0;
          sn[j] = 1.0;
        } else {
          const cd ph = hcol[j] / a;
          cs[j] = a / den;
          sn[j] = ph * std::conj(hcol[j + 1]) / den;
        }
      }
      const cd hj = cs[j] * hcol[j] + sn[j] * hcol[j + 1];
      hcol[j] = hj;
      hcol[j + 1] = 0.0;
      e1[j + 1] = -std::conj(sn[j]) * e1[j];
      e1[j] = cs[j] * e1[j];
      for (int k = 0; k <= j; ++k) Hc[k * restart + j] = hcol[k];
      rn = std::abs(e1[j + 1]);
      if (rn <= tol * gn || hn == 0) { ++j; ++total; break; }
    }
    // back substitution y = H^{-1} e1 (j x j upper), x += V y
    std::vector<cd> y(j);
    for (int i = j - 1; i >= 0; --i) {
      cd v = e1[i];
      for (int k = i + 1; k < j; ++k) v -= Hc[i * restart + k] * y[k];
      y[i] = v / Hc[i * restart + i];
    }
    std::vector<C2<double>> yd(j);
    for (int i = 0; i < j; ++i) yd[i] = C2<double>{y[i].real(), y[i].imag()};
    he = hipMemcpyAsync(hdev, yd.data(), j * sizeof(C2<double>), hipMemcpyHostToDevice, sc.stream);
    if (he != hipSuccess) { res.hip = he; return res; }
    hipLaunchKernelGGL(combine_kernel, grid1(N), dim3(256), 0, sc.stream, P ? Z : V, N, j, hdev, x64);
    he = hipStreamSynchronize(sc.stream);
    if (he != hipSuccess) { res.hip = he; return res; }
  }
  // rn is the true residual of x (the loop only ends at its top)
  *iters = total;
  *rel_res = rn / gn;
  res.converged = rn <= tol * gn;
  return res;
}

SolveResult gmres64(SolveCtx& sc, const cplx* S, int64_t ld, int64_t N, const cplx* g, cplx* x,
                    double tol, int max_iter, int restart, int* iters, double* rel_res) {
  return gmres_core(sc, S, ld, N, g, x, tol, max_iter, restart, nullptr, false, false, iters, rel_res);
}

SolveResult fgmres64(SolveCtx& sc, const cplx* S, int64_t ld, int64_t N, const cplx* g, cplx* x,
                     double tol, int max_iter, int restart, const Precond& P, int* iters,
                     double* rel_res, bool* fell_back) {
  *fell_back = false;
  SolveResult r = gmres_core(sc, S, ld, N, g, x, tol, max_iter, restart, &P, true, false, iters, rel_res);
  if (r.hip != hipSuccess || r.converged) return r;
  // the learned preconditioner did not reach tol: the plain solve, from zero
  *fell_back = true;
  int more = 0;
  SolveResult r2 = gmres_core(sc, S, ld, N, g, x, tol, max_iter, restart, nullptr, false, false, &more,
                              rel_res);
  *iters += more;
  return r2;
}

namespace {

__global__ void widen_kernel(const C2<float>* d, C2<double>* z, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) z[i] = C2<double>{(double)d[i].re, (double)d[i].im};
}

// z = (L U)^{-1} v with the complex64 factors: v rounded to complex64, the two
// triangular solves in complex64, the result widened to complex128.
struct Lu32Precond {
  SolveCtx* sc;
  C2<float>* S32;
  int64_t N;
};

hipError_t lu32_apply(void* self, const cplx* v, cplx* z) {
  auto* p = static_cast<Lu32Precond*>(self);
  SolveCtx& sc = *p->sc;
  auto* d32 = reinterpret_cast<C2<float>*>(sc.vec_d);
  hipLaunchKernelGGL(to_prec_kernel<float>, grid1(p->N), dim3(256), 0, sc.stream,
                     reinterpret_cast<const C2<double>*>(v), d32, p->N);
  const SolveResult s = lu_factor_solve_t(sc, p->S32, p->N, p->N, d32, false);
  if (s.hip != hipSuccess) return s.hip;
  hipLaunchKernelGGL(widen_kernel, grid1(p->N), dim3(256), 0, sc.stream, d32,
                     reinterpret_cast<C2<double>*>(z), p->N);
  return hipGetLastError();
}

}  // namespace

SolveResult gmres_lu32(SolveCtx& sc, const cplx* S, int64_t ld, int64_t N, const cplx* g, cplx* x,
                       double tol, int max_iter, int restart, int* iters, double* rel_res) {
  SolveResult res;
  auto* S64 = reinterpret_cast<const C2<double>*>(S);
  auto* S32 = reinterpret_cast<C2<float>*>(sc.s32);
  auto* d32 = reinterpret_cast<C2<float>*>(sc.vec_d);
  hipLaunchKernelGGL(convert_kernel<float>, dim3((unsigned)((N + 255) / 256), (unsigned)std::min<int64_t>(N, 8192)), dim3(256),
                     0, sc.stream, S64, ld, S32, N, N);
  res.hip = hipGetLastError();
  if (res.hip != hipSuccess) return res;
  // factor (with a zero right-hand side, so the solve part is a no-op)
  res.hip = hipMemsetAsync(d32, 0, N * sizeof(C2<float>), sc.stream);
  if (res.hip != hipSuccess) return res;
  res = lu_factor_solve_t(sc, S32, N, N, d32, true);
  if (res.hip != hipSuccess || res.singular_col != 0) return res;
  Lu32Precond pc{&sc, S32, N};
  const Precond P{lu32_apply, &pc};
  return gmres_core(sc, S, ld, N, g, x, tol, max_iter, restart, &P, false, false, iters, rel_res);
}

hipError_t residual64(SolveCtx& sc, const cplx* S, int64_t ld, int64_t N, const cplx* x,
                      const cplx* g, cplx* r) {
  hipLaunchKernelGGL(residual_kernel, grid1(N, 4), dim3(256), 0, sc.stream,
                     reinterpret_cast<const C2<double>*>(S), ld, N,
                     reinterpret_cast<const C2<double>*>(x), reinterpret_cast<const C2<double>*>(g),
                     reinterpret_cast<C2<double>*>(r), 1.0);
  return hipGetLastError();
}

double device_norm2(SolveCtx& sc, const cplx* v, int64_t N, hipError_t* err) {
  return norm2(sc, reinterpret_cast<const C2<double>*>(v), N, err);
}

}  // namespace ffbie
