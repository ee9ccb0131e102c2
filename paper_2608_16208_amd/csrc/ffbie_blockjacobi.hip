// Mode-block-Jacobi preconditioner for the single-layer system.
//
// In the azimuthal Fourier basis phi[(b, j')] = sum_m Phi_m[b] e^{i m theta_j'} the
// matrix S becomes blocks B_{m, m'} over curve nodes; for a surface close to a
// surface of revolution the diagonal blocks dominate.  The preconditioner
// applies the exact inverses of the diagonal blocks:
//   B_m[a][b] = (1/2M) sum_{j, j'} e^{-i m theta_j} S[(a, j), (b, j')] e^{i m theta_j'}
//             = (1/2M) sum_d e^{-i m theta_d} C_ab[d],
//   C_ab[d]   = sum_j S[(a, j), (b, (j - d) mod 2M)]   (wrapped diagonal sums),
// then P(r) = sum_m (B_m^{-1} R_m) e^{i m theta} with R_m the modes of r.
//
// Kernels: one workgroup per node pair (a, b) reads the 2M x 2M sub-block of S
// once (coalesced along rows) and writes the 2M block entries; one workgroup
// per mode factors its block in place (LU with partial pivoting); one
// workgroup per mode solves with its factors.
#include "ffbie_blockjacobi.hpp"

namespace ffbie {

namespace {

__global__ __launch_bounds__(256) void extract_blocks_kernel(const cplx* __restrict__ S, int64_t ld,
                                                             int M, int nodes, cplx* __restrict__ B) {
  extern __shared__ double lds[];
  cplx* C = reinterpret_cast<cplx*>(lds);              // [2M]
  const int NF = 2 * M;
  const int a = blockIdx.x / nodes, b = blockIdx.x % nodes;
  const cplx* base = S + (int64_t)a * NF * ld + (int64_t)b * NF;
  for (int d = threadIdx.x; d < NF; d += blockDim.x) {
    double sr = 0, si = 0;
    for (int j = 0; j < NF; ++j) {
      const cplx v = base[(int64_t)j * ld + ((j - d + NF) & (NF - 1))];
      sr += v.re;
      si += v.im;
    }
    C[d] = mk(sr, si);
  }
  __syncthreads();
  for (int mi = threadIdx.x; mi < NF; mi += blockDim.x) {
    const int m = mi - M + 1;
    double sr = 0, si = 0;
    for (int d = 0; d < NF; ++d) {
      const int q = ((m * d) % NF + NF) % NF;
      double s, c;
      sincos_bounded(M_PI * q / M, &s, &c);          // e^{-i m theta_d} = c - i s
      sr += C[d].re * c + C[d].im * s;
      si += C[d].im * c - C[d].re * s;
    }
    B[((int64_t)mi * nodes + a) * nodes + b] = mk(sr / NF, si / NF);
  }
}

// In-place LU with partial pivoting of one n x n row-major block per workgroup.
__global__ __launch_bounds__(1024) void block_lu_kernel(cplx* B, int n, int32_t* piv, int* info) {
  __shared__ double best[1024];
  __shared__ int where[1024];
  cplx* A = B + (int64_t)blockIdx.x * n * n;
  int32_t* pv = piv + (int64_t)blockIdx.x * n;
  const int tid = threadIdx.x, nt = blockDim.x;
  for (int k = 0; k < n; ++k) {
    double bv = -1;
    int bw = k;
    for (int r = k + tid; r < n; r += nt) {
      const double v = fabs(A[r * n + k].re) + fabs(A[r * n + k].im);
      if (v > bv) { bv = v; bw = r; }
    }
    best[tid] = bv;
    where[tid] = bw;
    __syncthreads();
    for (int s = nt / 2; s > 0; s >>= 1) {
      if (tid < s && (best[tid + s] > best[tid] ||
                      (best[tid + s] == best[tid] && where[tid + s] < where[tid]))) {
        best[tid] = best[tid + s];
        where[tid] = where[tid + s];
      }
      __syncthreads();
    }
    const int p = where[0];
    const bool zero = !(best[0] > 0);
    __syncthreads();
    if (tid == 0) {
      pv[k] = p;
      if (zero && info[blockIdx.x] == 0) info[blockIdx.x] = k + 1;
    }
    if (p != k)
      for (int c = tid; c < n; c += nt) {
        const cplx t = A[k * n + c];
        A[k * n + c] = A[p * n + c];
        A[p * n + c] = t;
      }
    __syncthreads();
    if (zero) continue;
    const cplx d = A[k * n + k];
    const double den = d.re * d.re + d.im * d.im;
    const cplx inv = mk(d.re / den, -d.im / den);
    for (int r = k + 1 + tid; r < n; r += nt) A[r * n + k] = A[r * n + k] * inv;
    __syncthreads();
    const int w = n - k - 1;
    for (int e = tid; e < w * w; e += nt) {
      const int r = k + 1 + e / w, c = k + 1 + e % w;
      A[r * n + c] = A[r * n + c] - A[r * n + k] * A[k * n + c];
    }
    __syncthreads();
  }
}

// E_m = B_m^{-1} R_m for every mode (one workgroup per mode), R, E [mode][node].
__global__ __launch_bounds__(256) void block_solve_kernel(const cplx* B, const int32_t* piv, int n,
                                                          const cplx* R, cplx* E) {
  extern __shared__ double lds[];
  cplx* y = reinterpret_cast<cplx*>(lds);                // [n]
  __shared__ double red[2][256];
  const cplx* A = B + (int64_t)blockIdx.x * n * n;
  const int32_t* pv = piv + (int64_t)blockIdx.x * n;
  const cplx* r = R + (int64_t)blockIdx.x * n;
  if (threadIdx.x == 0) {
    for (int i = 0; i < n; ++i) y[i] = r[i];
    for (int k = 0; k < n; ++k) {
      const int p = pv[k];
      if (p != k) { const cplx t = y[k]; y[k] = y[p]; y[p] = t; }
    }
  }
  __syncthreads();
  // forward (unit lower) then backward (upper), each row a parallel dot product
  for (int pass = 0; pass < 2; ++pass) {
    for (int ii = 0; ii < n; ++ii) {
      const int i = pass == 0 ? ii : n - 1 - ii;
      const int lo = pass == 0 ? 0 : i + 1, hi = pass == 0 ? i : n;
      double sr = 0, si = 0;
      for (int k = lo + threadIdx.x; k < hi; k += blockDim.x) {
        const cplx p = A[i * n + k] * y[k];
        sr += p.re;
        si += p.im;
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
      if (threadIdx.x == 0) {
        cplx v = y[i] - mk(red[0][0], red[1][0]);
        if (pass == 1) v = cdiv(v, A[i * n + i]);
        y[i] = v;
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < n; i += blockDim.x) E[(int64_t)blockIdx.x * n + i] = y[i];
}

// modes R[mi][node] of r [node][2M]
__global__ __launch_bounds__(256) void bj_modes_kernel(const cplx* r, int M, int nodes, cplx* R) {
  const int node = blockIdx.x;
  const int NF = 2 * M;
  const cplx* row = r + (int64_t)node * NF;
  for (int mi = threadIdx.x; mi < NF; mi += blockDim.x) {
    const int m = mi - M + 1;
    double sr = 0, si = 0;
    for (int j = 0; j < NF; ++j) {
      const int q = ((m * j) % NF + NF) % NF;
      double s, c;
      sincos_bounded(M_PI * q / M, &s, &c);
      const cplx v = row[j];
      sr += v.re * c + v.im * s;
      si += v.im * c - v.re * s;
    }
    R[(int64_t)mi * nodes + node] = mk(sr / NF, si / NF);
  }
}

// e[node][j] = sum_m E[mi][node] e^{i m theta_j}
__global__ __launch_bounds__(256) void bj_synth_kernel(const cplx* E, int M, int nodes, cplx* e) {
  const int node = blockIdx.x;
  const int NF = 2 * M;
  for (int j = threadIdx.x; j < NF; j += blockDim.x) {
    double sr = 0, si = 0;
    for (int mi = 0; mi < NF; ++mi) {
      const int m = mi - M + 1;
      const int q = ((m * j) % NF + NF) % NF;
      double s, c;
      sincos_bounded(M_PI * q / M, &s, &c);
      const cplx v = E[(int64_t)mi * nodes + node];
      sr += v.re * c - v.im * s;
      si += v.re * s + v.im * c;
    }
    e[(int64_t)node * NF + j] = mk(sr, si);
  }
}

}  // namespace

hipError_t BlockJacobi::setup(const cplx* S, int64_t ld, int M_, int nodes_, hipStream_t s) {
  M = M_;
  nodes = nodes_;
  const int64_t nb = 2 * (int64_t)M;
  const int64_t need = nb * nodes * nodes;
  hipError_t e;
  if (need > cap) {
    for (void* p : {(void*)B, (void*)piv, (void*)info, (void*)R, (void*)E})
      if (p) (void)hipFree(p);
    B = nullptr; piv = nullptr; info = nullptr; R = nullptr; E = nullptr;
    cap = 0;
    if ((e = hipMalloc(&B, need * sizeof(cplx))) != hipSuccess) return e;
    if ((e = hipMalloc(&piv, nb * nodes * sizeof(int32_t))) != hipSuccess) return e;
    if ((e = hipMalloc(&info, nb * sizeof(int))) != hipSuccess) return e;
    if ((e = hipMalloc(&R, nb * nodes * sizeof(cplx))) != hipSuccess) return e;
    if ((e = hipMalloc(&E, nb * nodes * sizeof(cplx))) != hipSuccess) return e;
    cap = need;
  }
  if ((e = hipMemsetAsync(info, 0, nb * sizeof(int), s)) != hipSuccess) return e;
  hipLaunchKernelGGL(extract_blocks_kernel, dim3(nodes * nodes), dim3(256), nb * sizeof(cplx), s, S, ld,
                     M, nodes, B);
  hipLaunchKernelGGL(block_lu_kernel, dim3((unsigned)nb), dim3(1024), 0, s, B, nodes, piv, info);
  return hipGetLastError();
}

hipError_t BlockJacobi::apply(const cplx* v, cplx* z, hipStream_t s) const {
  const int64_t nb = 2 * (int64_t)M;
  hipLaunchKernelGGL(bj_modes_kernel, dim3(nodes), dim3(256), 0, s, v, M, nodes, R);
  hipLaunchKernelGGL(block_solve_kernel, dim3((unsigned)nb), dim3(256), nodes * sizeof(cplx), s, B, piv,
                     nodes, R, E);
  hipLaunchKernelGGL(bj_synth_kernel, dim3(nodes), dim3(256), 0, s, E, M, nodes, z);
  return hipGetLastError();
}

hipError_t BlockJacobi::solve_modes(const cplx* Rin, cplx* Eout, hipStream_t s) const {
  hipLaunchKernelGGL(block_solve_kernel, dim3((unsigned)(2 * M)), dim3(256), nodes * sizeof(cplx), s, B,
                     piv, nodes, Rin, Eout);
  return hipGetLastError();
}

void BlockJacobi::release() {
  for (void* p : {(void*)B, (void*)piv, (void*)info, (void*)R, (void*)E})
    if (p) (void)hipFree(p);
  *this = BlockJacobi{};
}

}  // namespace ffbie
