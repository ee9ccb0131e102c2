// Learned preconditioner for the dense solve: a small MLP applied per
// azimuthal mode, with BF16 weights and activations on the matrix cores (FP32
// accumulation), trained on the GPU by the kernels below.
//
// Network (shared by all modes m of a residual r):
//   x_m = [Re R_m / s_m, Im R_m / s_m, k / 30, m / M]      (514 inputs)
//   h1 = relu(W1 x + b1), h2 = relu(W2 h1 + b2)             (256, 256)
//   y_m = W3 h2 + b3,  E_m = s_m (y[0:256] + i y[256:512])   (512 outputs)
// where R_m[node] = (1/2M) sum_j r[node, j] e^{-i m theta_j} is the azimuthal
// mode m (m = -M+1..M) of the residual on the 256 curve nodes and s_m = |R_m|_2.
// The preconditioned vector is e[node, j] = sum_m E_m[node] e^{i m theta_j}.
//
// GEMMs: one wavefront per 16 x 16 output tile with v_mfma_f32_16x16x16_bf16;
// operands are read through strides, so the same kernel serves X W^T (forward),
// dZ W (input gradients) and dZ^T A (weight gradients).  The network is small
// (3.3e5 parameters, 128 samples per application), so the kernels are sized for
// latency, not for the matrix-core peak.
#include "ffbie_mlp.hpp"

namespace ffbie {

namespace {

typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// FP32 -> BF16 with round-to-nearest-even (NaN kept quiet).
__device__ __forceinline__ uint16_t to_bf16(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}
__device__ __forceinline__ float from_bf16(uint16_t h) { return __uint_as_float((uint32_t)h << 16); }

struct GemmArgs {
  int M, N, K;
  const uint16_t* A;     // A(m, k) = A[m * sam + k * sak]
  int64_t sam, sak;
  const uint16_t* B;     // B(k, n) = B[k * sbk + n * sbn]
  int64_t sbk, sbn;
  const float* bias;     // [N] or null
  int relu;
  float alpha;
  float* C;              // fp32 out C[m * ldc + n] or null
  int64_t ldc;
  uint16_t* Cb;          // bf16 out or null
  int64_t ldcb;
};

// One wavefront per 16 x 16 tile of C = alpha A B (+ bias, relu).
// Lane layout of the 16x16x16 BF16 MFMA: lane l feeds A[l % 16][4 (l / 16) + i]
// and B[4 (l / 16) + i][l % 16], i < 4, and receives C[4 (l / 16) + i][l % 16].
__global__ __launch_bounds__(256) void gemm_bf16_kernel(GemmArgs g) {
  const int lane = threadIdx.x & 63;
  const int64_t wave = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
  const int tiles_n = (g.N + 15) / 16;
  const int64_t tiles = (int64_t)((g.M + 15) / 16) * tiles_n;
  if (wave >= tiles) return;
  const int m0 = (int)(wave / tiles_n) * 16, n0 = (int)(wave % tiles_n) * 16;
  const int r = lane & 15, kg = lane >> 4;
  f32x4 acc = {0.f, 0.f, 0.f, 0.f};
  for (int k0 = 0; k0 < g.K; k0 += 16) {
    bf16x4 av, bv;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int k = k0 + 4 * kg + i;
      const int am = m0 + r, bn = n0 + r;
      av[i] = (am < g.M && k < g.K) ? (short)g.A[am * g.sam + k * g.sak] : (short)0;
      bv[i] = (bn < g.N && k < g.K) ? (short)g.B[k * g.sbk + bn * g.sbn] : (short)0;
    }
    acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av, bv, acc, 0, 0, 0);
  }
  const int n = n0 + r;
  if (n >= g.N) return;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int m = m0 + 4 * kg + i;
    if (m >= g.M) continue;
    float v = g.alpha * acc[i];
    if (g.bias) v += g.bias[n];
    if (g.relu) v = v > 0.f ? v : 0.f;
    if (g.C) g.C[m * g.ldc + n] = v;
    if (g.Cb) g.Cb[m * g.ldcb + n] = to_bf16(v);
  }
}

hipError_t gemm(const GemmArgs& g, hipStream_t s) {
  const int64_t tiles = (int64_t)((g.M + 15) / 16) * ((g.N + 15) / 16);
  hipLaunchKernelGGL(gemm_bf16_kernel, dim3((unsigned)((tiles + 3) / 4)), dim3(256), 0, s, g);
  return hipGetLastError();
}

__global__ void to_bf16_kernel(const float* x, uint16_t* y, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) y[i] = to_bf16(x[i]);
}

// Minibatch gather: row i of xb (bf16) and of tg (fp32) are rows idx[i] of
// the training inputs x [*][kIn] and targets t [*][kOut].
__global__ void gather_batch_kernel(const float* __restrict__ x, const float* __restrict__ t,
                                    const int32_t* __restrict__ idx, int64_t n, uint16_t* xb,
                                    float* tg) {
  const int64_t row = blockIdx.y;
  if (row >= n) return;
  const int64_t src = idx[row];
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < Mlp::kIn; c += gridDim.x * blockDim.x)
    xb[row * Mlp::kIn + c] = to_bf16(x[src * Mlp::kIn + c]);
  for (int c = blockIdx.x * blockDim.x + threadIdx.x; c < Mlp::kOut; c += gridDim.x * blockDim.x)
    tg[row * Mlp::kOut + c] = t[src * Mlp::kOut + c];
}

// dY = (Y - T) / n  (fp32 and bf16) and the partial sums of |Y - T|^2
__global__ __launch_bounds__(256) void loss_grad_kernel(const float* Y, const float* T, int64_t cnt,
                                                        float inv_n, uint16_t* dYb, double* partial) {
  __shared__ double red[256];
  double s = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < cnt;
       i += (int64_t)gridDim.x * blockDim.x) {
    const float d = Y[i] - T[i];
    s += (double)d * d;
    if (dYb) dYb[i] = to_bf16(d * inv_n);
  }
  red[threadIdx.x] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[blockIdx.x] = red[0];
}

// dZ = dA * (A > 0) in bf16 (A the stored bf16 activation)
__global__ void relu_back_kernel(const float* dA, const uint16_t* A, uint16_t* dZb, int64_t cnt) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < cnt) dZb[i] = to_bf16(from_bf16(A[i]) > 0.f ? dA[i] : 0.f);
}

// db[n] = sum_b dZ[b][n] (bf16 input, fp32 accumulation in a fixed order)
__global__ void bias_grad_kernel(const uint16_t* dZ, int rows, int cols, float* db) {
  const int n = blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= cols) return;
  float s = 0.f;
  for (int b = 0; b < rows; ++b) s += from_bf16(dZ[(int64_t)b * cols + n]);
  db[n] = s;
}

__global__ void adam_kernel(float* p, const float* g, float* m, float* v, int64_t cnt, float lr,
                            float b1, float b2, float eps, float c1, float c2, uint16_t* pb) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= cnt) return;
  const float gi = g[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  const float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  p[i] = pi;
  if (pb) pb[i] = to_bf16(pi);
}

// Azimuthal modes of a vector r [nodes][2M]: R[mi][node] for mi = m + M - 1.
__global__ __launch_bounds__(256) void modes_kernel(const cplx* r, int M, int nodes, cplx* R) {
  const int node = blockIdx.x;
  const int NF = 2 * M;
  const cplx* row = r + (int64_t)node * NF;
  for (int mi = threadIdx.x; mi < NF; mi += blockDim.x) {
    const int m = mi - M + 1;
    double sr = 0, si = 0;
    for (int j = 0; j < NF; ++j) {
      const int q = ((m * j) % NF + NF) % NF;
      double s, c;
      sincos_bounded(M_PI * q / M, &s, &c);          // e^{-i m theta_j} = c - i s
      const cplx v = row[j];
      sr += v.re * c + v.im * s;
      si += v.im * c - v.re * s;
    }
    R[(int64_t)mi * nodes + node] = mk(sr / NF, si / NF);
  }
}

// Features x[mi][0..513] and scales s[mi] from R[mi][node]; one workgroup per mode.
__global__ __launch_bounds__(256) void features_kernel(const cplx* R, int M, int nodes, double k,
                                                       float* x, uint16_t* xb, double* scale,
                                                       const double* given_scale) {
  __shared__ double red[256];
  const int mi = blockIdx.x;
  const cplx* Rm = R + (int64_t)mi * nodes;
  double s;
  if (given_scale) {
    s = given_scale[mi];
  } else {
    double a = 0;
    for (int n = threadIdx.x; n < nodes; n += blockDim.x) a += abs2(Rm[n]);
    red[threadIdx.x] = a;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    s = sqrt(red[0]);
    if (threadIdx.x == 0 && scale) scale[mi] = s;
  }
  const double inv = s > 0 ? 1.0 / s : 0.0;
  const int width = 2 * nodes + (given_scale ? 0 : 2);
  float* xo = x ? x + (int64_t)mi * width : nullptr;
  uint16_t* xbo = xb ? xb + (int64_t)mi * width : nullptr;
  for (int n = threadIdx.x; n < nodes; n += blockDim.x) {
    const float re = (float)(Rm[n].re * inv), im = (float)(Rm[n].im * inv);
    if (xo) { xo[n] = re; xo[nodes + n] = im; }
    if (xbo) { xbo[n] = to_bf16(re); xbo[nodes + n] = to_bf16(im); }
  }
  if (!given_scale && threadIdx.x == 0) {
    const float f0 = (float)(k / 30.0), f1 = (float)((double)(mi - M + 1) / M);
    if (xo) { xo[2 * nodes] = f0; xo[2 * nodes + 1] = f1; }
    if (xbo) { xbo[2 * nodes] = to_bf16(f0); xbo[2 * nodes + 1] = to_bf16(f1); }
  }
}

// e[node][j] = sum_m s_m (y_m[node] + i y_m[nodes + node]) e^{i m theta_j}
__global__ __launch_bounds__(256) void reconstruct_kernel(const float* y, const double* scale, int M,
                                                          int nodes, cplx* e) {
  const int node = blockIdx.x;
  const int NF = 2 * M;
  for (int j = threadIdx.x; j < NF; j += blockDim.x) {
    double sr = 0, si = 0;
    for (int mi = 0; mi < NF; ++mi) {
      const int m = mi - M + 1;
      const int q = ((m * j) % NF + NF) % NF;
      double s, c;
      sincos_bounded(M_PI * q / M, &s, &c);          // e^{+i m theta_j} = c + i s
      const double a = scale[mi] * y[(int64_t)mi * 2 * nodes + node];
      const double b = scale[mi] * y[(int64_t)mi * 2 * nodes + nodes + node];
      sr += a * c - b * s;
      si += a * s + b * c;
    }
    e[(int64_t)node * NF + j] = mk(sr, si);
  }
}

inline dim3 g1(int64_t n) { return dim3((unsigned)((n + 255) / 256)); }

}  // namespace

// ---------------------------------------------------------------------------
size_t Mlp::param_count() { return (size_t)kH * (kIn + 1) + (size_t)kH * (kH + 1) + (size_t)kOut * (kH + 1); }

hipError_t Mlp::ensure_batch(int64_t n) {
  if (n <= cap) return hipSuccess;
  for (void* p : {(void*)xb, (void*)a1, (void*)a2, (void*)y, (void*)dyb, (void*)da, (void*)dzb,
                  (void*)partial})
    if (p) (void)hipFree(p);
  xb = nullptr; a1 = nullptr; a2 = nullptr; y = nullptr; dyb = nullptr; da = nullptr; dzb = nullptr;
  partial = nullptr;
  cap = 0;
  hipError_t e;
  if ((e = hipMalloc(&xb, n * kIn * sizeof(uint16_t))) != hipSuccess) return e;
  if ((e = hipMalloc(&a1, n * kH * sizeof(uint16_t))) != hipSuccess) return e;
  if ((e = hipMalloc(&a2, n * kH * sizeof(uint16_t))) != hipSuccess) return e;
  if ((e = hipMalloc(&y, n * kOut * sizeof(float))) != hipSuccess) return e;
  if ((e = hipMalloc(&dyb, n * kOut * sizeof(uint16_t))) != hipSuccess) return e;
  if ((e = hipMalloc(&da, n * kOut * sizeof(float))) != hipSuccess) return e;
  if ((e = hipMalloc(&dzb, n * kOut * sizeof(uint16_t))) != hipSuccess) return e;
  if ((e = hipMalloc(&partial, 1024 * sizeof(double))) != hipSuccess) return e;
  cap = n;
  return hipSuccess;
}

hipError_t Mlp::alloc() {
  if (params) return hipSuccess;
  const size_t P = param_count();
  hipError_t e;
  if ((e = hipMalloc(&params, P * sizeof(float))) != hipSuccess) return e;
  if ((e = hipMalloc(&grads, P * sizeof(float))) != hipSuccess) return e;
  if ((e = hipMalloc(&m1, P * sizeof(float))) != hipSuccess) return e;
  if ((e = hipMalloc(&m2, P * sizeof(float))) != hipSuccess) return e;
  if ((e = hipMalloc(&wb, P * sizeof(uint16_t))) != hipSuccess) return e;
  return hipSuccess;
}

void Mlp::release() {
  for (void* p : {(void*)params, (void*)grads, (void*)m1, (void*)m2, (void*)wb, (void*)xb,
                  (void*)a1, (void*)a2, (void*)y, (void*)dyb, (void*)da, (void*)dzb, (void*)partial,
                  (void*)R, (void*)feat, (void*)scale, (void*)tg})
    if (p) (void)hipFree(p);
  *this = Mlp{};
}

// parameter block offsets (floats): W1 b1 W2 b2 W3 b3
size_t Mlp::off_W1() { return 0; }
size_t Mlp::off_b1() { return (size_t)kH * kIn; }
size_t Mlp::off_W2() { return off_b1() + kH; }
size_t Mlp::off_b2() { return off_W2() + (size_t)kH * kH; }
size_t Mlp::off_W3() { return off_b2() + kH; }
size_t Mlp::off_b3() { return off_W3() + (size_t)kOut * kH; }

hipError_t Mlp::refresh_bf16(hipStream_t s) {
  const size_t P = param_count();
  hipLaunchKernelGGL(to_bf16_kernel, g1(P), dim3(256), 0, s, params, wb, (int64_t)P);
  return hipGetLastError();
}

// Forward over n samples whose bf16 inputs are in xb; output y (fp32).
hipError_t Mlp::forward(int64_t n, hipStream_t s) {
  hipError_t e;
  GemmArgs g{};
  g.M = (int)n; g.N = kH; g.K = kIn; g.A = xb; g.sam = kIn; g.sak = 1;
  g.B = wb + off_W1(); g.sbk = 1; g.sbn = kIn; g.bias = params + off_b1(); g.relu = 1; g.alpha = 1.f;
  g.Cb = a1; g.ldcb = kH;
  if ((e = gemm(g, s)) != hipSuccess) return e;
  g = GemmArgs{};
  g.M = (int)n; g.N = kH; g.K = kH; g.A = a1; g.sam = kH; g.sak = 1;
  g.B = wb + off_W2(); g.sbk = 1; g.sbn = kH; g.bias = params + off_b2(); g.relu = 1; g.alpha = 1.f;
  g.Cb = a2; g.ldcb = kH;
  if ((e = gemm(g, s)) != hipSuccess) return e;
  g = GemmArgs{};
  g.M = (int)n; g.N = kOut; g.K = kH; g.A = a2; g.sam = kH; g.sak = 1;
  g.B = wb + off_W3(); g.sbk = 1; g.sbn = kH; g.bias = params + off_b3(); g.relu = 0; g.alpha = 1.f;
  g.C = y; g.ldc = kOut;
  return gemm(g, s);
}

// Gradients of L = (1/2n) sum |y - t|^2 into `grads` (after forward); *loss_partial
// receives the per-block sums of |y - t|^2 (count returned in *nblk).
hipError_t Mlp::backward(int64_t n, const float* t, hipStream_t s, int* nblk) {
  hipError_t e;
  const int blocks = (int)std::min<int64_t>(1024, (n * kOut + 255) / 256);
  *nblk = blocks;
  hipLaunchKernelGGL(loss_grad_kernel, dim3(blocks), dim3(256), 0, s, y, t, n * kOut, 1.f / (float)n,
                     dyb, partial);
  // layer 3: dW3 = dY^T A2, db3, dA2 = dY W3
  GemmArgs g{};
  g.M = kOut; g.N = kH; g.K = (int)n; g.A = dyb; g.sam = 1; g.sak = kOut;
  g.B = a2; g.sbk = kH; g.sbn = 1; g.alpha = 1.f; g.C = grads + off_W3(); g.ldc = kH;
  if ((e = gemm(g, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(bias_grad_kernel, g1(kOut), dim3(256), 0, s, dyb, (int)n, kOut, grads + off_b3());
  g = GemmArgs{};                                   // B(n, k) = W3[n][k]
  g.M = (int)n; g.N = kH; g.K = kOut; g.A = dyb; g.sam = kOut; g.sak = 1;
  g.B = wb + off_W3(); g.sbk = kH; g.sbn = 1; g.alpha = 1.f; g.C = da; g.ldc = kH;
  if ((e = gemm(g, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(relu_back_kernel, g1(n * kH), dim3(256), 0, s, da, a2, dzb, n * kH);
  // layer 2: dW2 = dZ2^T A1, db2, dA1 = dZ2 W2
  g = GemmArgs{};
  g.M = kH; g.N = kH; g.K = (int)n; g.A = dzb; g.sam = 1; g.sak = kH;
  g.B = a1; g.sbk = kH; g.sbn = 1; g.alpha = 1.f; g.C = grads + off_W2(); g.ldc = kH;
  if ((e = gemm(g, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(bias_grad_kernel, g1(kH), dim3(256), 0, s, dzb, (int)n, kH, grads + off_b2());
  g = GemmArgs{};                                   // B(n, k) = W2[n][k]
  g.M = (int)n; g.N = kH; g.K = kH; g.A = dzb; g.sam = kH; g.sak = 1;
  g.B = wb + off_W2(); g.sbk = kH; g.sbn = 1; g.alpha = 1.f; g.C = da; g.ldc = kH;
  if ((e = gemm(g, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(relu_back_kernel, g1(n * kH), dim3(256), 0, s, da, a1, dzb, n * kH);
  // layer 1: dW1 = dZ1^T X, db1
  g = GemmArgs{};
  g.M = kH; g.N = kIn; g.K = (int)n; g.A = dzb; g.sam = 1; g.sak = kH;
  g.B = xb; g.sbk = kIn; g.sbn = 1; g.alpha = 1.f; g.C = grads + off_W1(); g.ldc = kIn;
  if ((e = gemm(g, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(bias_grad_kernel, g1(kH), dim3(256), 0, s, dzb, (int)n, kH, grads + off_b1());
  return hipGetLastError();
}

hipError_t Mlp::adam(float lr, hipStream_t s) {
  ++step;
  const float b1 = 0.9f, b2 = 0.999f, eps = 1e-8f;
  const float c1 = 1.f - powf(b1, (float)step), c2 = 1.f - powf(b2, (float)step);
  const size_t P = param_count();
  hipLaunchKernelGGL(adam_kernel, g1(P), dim3(256), 0, s, params, grads, m1, m2, (int64_t)P, lr, b1,
                     b2, eps, c1, c2, (uint16_t*)nullptr);
  return refresh_bf16(s);
}

hipError_t Mlp::gather_batch(const float* x, const float* t, const int32_t* idx, int64_t n, hipStream_t s) {
  hipError_t e;
  if (n > tg_cap) {
    if (tg) (void)hipFree(tg);
    tg = nullptr;
    tg_cap = 0;
    if ((e = hipMalloc(&tg, n * kOut * sizeof(float))) != hipSuccess) return e;
    tg_cap = n;
  }
  hipLaunchKernelGGL(gather_batch_kernel, dim3(1, (unsigned)n), dim3(256), 0, s, x, t, idx, n, xb, tg);
  return hipGetLastError();
}

hipError_t Mlp::inputs_bf16(const float* x, int64_t n, hipStream_t s) {
  hipLaunchKernelGGL(to_bf16_kernel, g1(n * kIn), dim3(256), 0, s, x, xb, n * kIn);
  return hipGetLastError();
}

hipError_t Mlp::ensure_modes(int M, int nodes) {
  const int64_t need = (int64_t)2 * M * nodes;
  if (need <= modes_cap) return hipSuccess;
  for (void* p : {(void*)R, (void*)feat, (void*)scale})
    if (p) (void)hipFree(p);
  R = nullptr; feat = nullptr; scale = nullptr;
  modes_cap = 0;
  hipError_t e;
  if ((e = hipMalloc(&R, need * sizeof(cplx))) != hipSuccess) return e;
  if ((e = hipMalloc(&feat, (int64_t)2 * M * kIn * sizeof(float))) != hipSuccess) return e;
  if ((e = hipMalloc(&scale, (int64_t)2 * M * sizeof(double))) != hipSuccess) return e;
  modes_cap = need;
  return hipSuccess;
}

hipError_t mode_features(Mlp& net, const cplx* r, int M, int nodes, double k, float* x_out,
                         double* scale_out, hipStream_t s) {
  hipError_t e = net.ensure_modes(M, nodes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(modes_kernel, dim3(nodes), dim3(256), 0, s, r, M, nodes, net.R);
  hipLaunchKernelGGL(features_kernel, dim3(2 * M), dim3(256), 0, s, net.R, M, nodes, k, x_out,
                     (uint16_t*)nullptr, scale_out, (const double*)nullptr);
  return hipGetLastError();
}

hipError_t mode_targets(Mlp& net, const cplx* e_vec, const double* scale, int M, int nodes,
                        float* t_out, hipStream_t s) {
  hipError_t e = net.ensure_modes(M, nodes);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(modes_kernel, dim3(nodes), dim3(256), 0, s, e_vec, M, nodes, net.R);
  hipLaunchKernelGGL(features_kernel, dim3(2 * M), dim3(256), 0, s, net.R, M, nodes, 0.0, t_out,
                     (uint16_t*)nullptr, (double*)nullptr, scale);
  return hipGetLastError();
}

hipError_t mode_reconstruct(const float* y, const double* scale, int M, int nodes, cplx* e,
                            hipStream_t s) {
  hipLaunchKernelGGL(reconstruct_kernel, dim3(nodes), dim3(256), 0, s, y, scale, M, nodes, e);
  return hipGetLastError();
}

// z = P(v): modes of v -> features (bf16) -> MLP -> reconstruction
hipError_t mlp_precondition(Mlp& net, const cplx* v, int M, int nodes, double k, cplx* z,
                            hipStream_t s) {
  hipError_t e = net.ensure_modes(M, nodes);
  if (e != hipSuccess) return e;
  if ((e = net.ensure_batch(2 * M)) != hipSuccess) return e;
  hipLaunchKernelGGL(modes_kernel, dim3(nodes), dim3(256), 0, s, v, M, nodes, net.R);
  hipLaunchKernelGGL(features_kernel, dim3(2 * M), dim3(256), 0, s, net.R, M, nodes, k,
                     (float*)nullptr, net.xb, net.scale, (const double*)nullptr);
  if ((e = net.forward(2 * M, s)) != hipSuccess) return e;
  hipLaunchKernelGGL(reconstruct_kernel, dim3(nodes), dim3(256), 0, s, net.y, net.scale, M, nodes, z);
  return hipGetLastError();
}

namespace {
__global__ void add_into_kernel(cplx* z, const cplx* t, int64_t n) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i < n) z[i] = cplx{z[i].re + t[i].re, z[i].im + t[i].im};
}
}  // namespace

hipError_t mlp_precondition_add(Mlp& net, const cplx* v, int M, int nodes, double k, cplx* z, cplx* tmp,
                                hipStream_t s) {
  hipError_t e = mlp_precondition(net, v, M, nodes, k, tmp, s);
  if (e != hipSuccess) return e;
  const int64_t n = (int64_t)2 * M * nodes;
  hipLaunchKernelGGL(add_into_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, z, tmp, n);
  return hipGetLastError();
}

hipError_t gemm_bf16(int M, int N, int K, const uint16_t* A, int64_t sam, int64_t sak,
                     const uint16_t* B, int64_t sbk, int64_t sbn, float* C, int64_t ldc,
                     hipStream_t s) {
  GemmArgs g{};
  g.M = M; g.N = N; g.K = K; g.A = A; g.sam = sam; g.sak = sak; g.B = B; g.sbk = sbk; g.sbn = sbn;
  g.alpha = 1.f; g.C = C; g.ldc = ldc;
  return gemm(g, s);
}

}  // namespace ffbie
