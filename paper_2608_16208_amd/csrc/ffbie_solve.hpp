// Interface of the dense solvers (row-major complex matrices).
#pragma once
#include "ffbie_device.hpp"

namespace ffbie {

// Device workspaces and handles the solvers use; owned by the context.
struct SolveCtx {
  hipStream_t stream;
  int64_t* ipiv;       // [N] pivot rows
  int64_t* perm;       // [N] permutation of the right-hand side
  int* info;           // first zero pivot (1-based), 0 if none
  void* vec_tmp;       // [N] complex128
  void* vec_r;         // [N] complex128
  void* vec_d;         // [N] complex128 (holds a complex64 vector)
  void* partial;       // reduction partials: 256 x (restart + 1) complex128
  void* hvec;          // [restart + 1] complex128
  void* s32;           // [N][N] complex64 (mixed-precision factor), or null
  void* krylov;        // [restart + 1][N] complex128 (GMRES), or null
  void* zbasis;        // [restart][N] complex128 (flexible GMRES), or null
};

// A preconditioner z = P(v) on the context's stream (for flexible GMRES).
struct Precond {
  hipError_t (*apply)(void* self, const cplx* v, cplx* z);
  void* self;
};

struct SolveResult {
  hipError_t hip = hipSuccess;
  int singular_col = 0;      // 1-based column of an exactly zero pivot
  bool converged = true;
};

SolveResult lu64_factor_solve(SolveCtx& sc, cplx* S, int64_t ld, int64_t N, cplx* y);
// solve with the factors of the last lu64_factor_solve on this context (same S, ld, N)
SolveResult lu64_solve_factored(SolveCtx& sc, const cplx* S, int64_t ld, int64_t N, cplx* y);
SolveResult lu32_ir64(SolveCtx& sc, const cplx* S, int64_t ld, int64_t N, const cplx* g, cplx* x,
                      double tol, int max_iter, int* iters, double* rel_res);
SolveResult gmres64(SolveCtx& sc, const cplx* S, int64_t ld, int64_t N, const cplx* g, cplx* x,
                    double tol, int max_iter, int restart, int* iters, double* rel_res);
// GMRES in complex128 right-preconditioned by the LU factors of a complex64 copy
// of S (GMRES-based iterative refinement)
SolveResult gmres_lu32(SolveCtx& sc, const cplx* S, int64_t ld, int64_t N, const cplx* g, cplx* x,
                       double tol, int max_iter, int restart, int* iters, double* rel_res);
SolveResult fgmres64(SolveCtx& sc, const cplx* S, int64_t ld, int64_t N, const cplx* g, cplx* x,
                     double tol, int max_iter, int restart, const Precond& P, int* iters,
                     double* rel_res, bool* fell_back);
hipError_t residual64(SolveCtx& sc, const cplx* S, int64_t ld, int64_t N, const cplx* x,
                      const cplx* g, cplx* r);
double device_norm2(SolveCtx& sc, const cplx* v, int64_t N, hipError_t* err);

}  // namespace ffbie
