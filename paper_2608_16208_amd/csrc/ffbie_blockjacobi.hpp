// Mode-block-Jacobi preconditioner (inverses of the diagonal azimuthal-mode blocks).
#pragma once
#include "ffbie_device.hpp"

namespace ffbie {

struct BlockJacobi {
  int M = 0, nodes = 0;
  cplx* B = nullptr;         // [2M][nodes][nodes] blocks, LU factors after setup
  int32_t* piv = nullptr;    // [2M][nodes]
  int* info = nullptr;       // [2M] first zero pivot (1-based) per block
  cplx* R = nullptr;         // [2M][nodes] workspace
  cplx* E = nullptr;
  int64_t cap = 0;
  bool ready = false;
  hipError_t setup(const cplx* S, int64_t ld, int M, int nodes, hipStream_t s);
  hipError_t apply(const cplx* v, cplx* z, hipStream_t s) const;
  hipError_t solve_modes(const cplx* R, cplx* E, hipStream_t s) const;
  void release();
};

}  // namespace ffbie
