// Learned per-mode preconditioner: network state and kernels (BF16 MFMA).
#pragma once
#include <stdint.h>

#include <algorithm>

#include "ffbie_device.hpp"

namespace ffbie {

struct Mlp {
  static constexpr int kNodes = 256;                 // curve nodes the network is sized for
  static constexpr int kIn = 2 * kNodes + 2;         // mode features + (k/30, m/M)
  static constexpr int kH = 256;                     // hidden width
  static constexpr int kOut = 2 * kNodes;            // correction of one mode
  float* params = nullptr;     // W1 [kH][kIn], b1, W2 [kH][kH], b2, W3 [kOut][kH], b3 (fp32 master)
  float* grads = nullptr;
  float* m1 = nullptr;         // Adam moments
  float* m2 = nullptr;
  uint16_t* wb = nullptr;      // bf16 copy of params
  int step = 0;
  bool ready = false;          // weights set
  // activations of a batch
  int64_t cap = 0;
  uint16_t* xb = nullptr;
  uint16_t* a1 = nullptr;
  uint16_t* a2 = nullptr;
  float* y = nullptr;
  uint16_t* dyb = nullptr;
  float* da = nullptr;
  uint16_t* dzb = nullptr;
  double* partial = nullptr;
  float* tg = nullptr;         // targets of the gathered minibatch
  int64_t tg_cap = 0;
  // mode transforms
  int64_t modes_cap = 0;
  cplx* R = nullptr;
  float* feat = nullptr;
  double* scale = nullptr;

  static size_t param_count();
  static size_t off_W1();
  static size_t off_b1();
  static size_t off_W2();
  static size_t off_b2();
  static size_t off_W3();
  static size_t off_b3();
  hipError_t alloc();
  void release();
  hipError_t ensure_batch(int64_t n);
  hipError_t ensure_modes(int M, int nodes);
  hipError_t refresh_bf16(hipStream_t s);
  hipError_t inputs_bf16(const float* x, int64_t n, hipStream_t s);
  // xb <- bf16 rows idx[0..n) of x [*][kIn], tg <- rows idx[0..n) of t [*][kOut]
  // (after ensure_batch(n))
  hipError_t gather_batch(const float* x, const float* t, const int32_t* idx, int64_t n, hipStream_t s);
  hipError_t forward(int64_t n, hipStream_t s);
  hipError_t backward(int64_t n, const float* t, hipStream_t s, int* nblk);
  hipError_t adam(float lr, hipStream_t s);
};

hipError_t mode_features(Mlp& net, const cplx* r, int M, int nodes, double k, float* x_out,
                         double* scale_out, hipStream_t s);
hipError_t mode_targets(Mlp& net, const cplx* e, const double* scale, int M, int nodes,
                        float* t_out, hipStream_t s);
hipError_t mode_reconstruct(const float* y, const double* scale, int M, int nodes, cplx* e,
                            hipStream_t s);
hipError_t mlp_precondition(Mlp& net, const cplx* v, int M, int nodes, double k, cplx* z,
                            hipStream_t s);
// z += P(v) (the network's correction added to a vector z already holding,
// for instance, the block-Jacobi output); tmp is an N-vector of workspace
hipError_t mlp_precondition_add(Mlp& net, const cplx* v, int M, int nodes, double k, cplx* z, cplx* tmp,
                                hipStream_t s);
hipError_t gemm_bf16(int M, int N, int K, const uint16_t* A, int64_t sam, int64_t sak,
                     const uint16_t* B, int64_t sbk, int64_t sbn, float* C, int64_t ldc,
                     hipStream_t s);

}  // namespace ffbie
