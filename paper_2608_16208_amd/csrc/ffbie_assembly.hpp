// Launch interface of the assembly, right-hand-side and field kernels
// (discrete single-layer system of Sec. 3.4).
#pragma once
#include "ffbie_device.hpp"

namespace ffbie {

constexpr int kNodes = 16;          // Gauss-Legendre nodes per panel and near-rule nodes

// Problem layout shared by the assembly kernels.
struct SysDims {
  int n_panels;
  int M;                             // 2M azimuths
  int64_t N;                         // unknowns: 32 M n_panels
  double h;                          // panel length pi / n_panels
};

// Collocation data in structure-of-arrays form: x, y, z, wq = (h/2) w_l / (2M), jac,
// and the unit normal (r_t x r_theta)/jac.
struct Colloc {
  double* x;
  double* y;
  double* z;
  double* wq;
  double* jac;
  double* nx;
  double* ny;
  double* nz;
};
constexpr int kCollocArrays = 8;

// Near pairs of a range of target panels [p0, p1).
struct NearChunk {
  int p0, p1;
  int64_t pair_base;                 // index of the first pair of panel p0 in the full near set
  int64_t n_pairs;
};

// Relations of panel i: left neighbour (if i > 0), own panel, right neighbour
// (if i < n_panels - 1).
FFBIE_HD inline int near_relations(int i, int n_panels) {
  return 1 + (i > 0 ? 1 : 0) + (i < n_panels - 1 ? 1 : 0);
}
// Relations of all panels before panel i.
FFBIE_HD inline int64_t near_relations_before(int i, int n_panels) {
  if (i <= 0) return 0;
  if (n_panels == 1) return 1;
  // panel 0 and the last panel have 2, panels 1..n_panels-2 have 3
  if (i >= n_panels) return 3 * (int64_t)n_panels - 2;
  return 2 + 3 * (int64_t)(i - 1);
}
// Near pairs of one relation of one target node over all azimuths: 2M x 16.
FFBIE_HD inline int64_t near_pairs_before(int i, const SysDims& d) {
  return near_relations_before(i, d.n_panels) * (int64_t)kNodes * 2 * d.M * kNodes;
}

hipError_t launch_collocation(const Geom& g, const SysDims& d, const double* gl_x,
                              const double* gl_w, Colloc c, double* xyz_out, double* jac_out,
                              double* wq_out, hipStream_t s);
hipError_t launch_near_pairs(const SysDims& d, const NearChunk& ch, const double* gl_x,
                             const double* rule_y /* [16 l][3 rel][16 q] */, double* t,
                             int32_t* az, double* ts, hipStream_t s);
// density = 1: the unknowns are density values (columns carry the Jacobian);
// 0: density x Jacobian (the single-layer system's unknowns).
hipError_t launch_far_assembly(const SysDims& d, double k, Colloc c, cplx* S, int64_t ld,
                               hipStream_t s, int density = 0);
// colscale: per-column factor of the written entries (the Jacobians for
// density unknowns) or null.
hipError_t launch_near_assembly(const SysDims& d, const NearChunk& ch, const cplx* kappa,
                                const double* wl /* [16 l][3 rel][16 q][16 l'] */,
                                const double* tab, cplx* S, int64_t ld, hipStream_t s,
                                const double* colscale = nullptr);
// Far blocks of the double-layer operator K (adjoint = 0) or K' (adjoint = 1):
// (h/2) w_l' (1/2M) tau_0 (ik rho - 1) e^{ik rho} / rho^3.
hipError_t launch_far_assembly_dl(const SysDims& d, double k, Colloc c, int adjoint, cplx* S,
                                  int64_t ld, hipStream_t s, int density);
// S[r, r] += shift (density unknowns) or shift / jac[r] (density x Jacobian):
// shift times the identity.
hipError_t launch_diag_shift(const SysDims& d, double shift, Colloc c, cplx* S, int64_t ld,
                             hipStream_t s, int density);
// Field of the double-layer representation u = 2 int dG/d nu_s psi dsigma.
hipError_t launch_field_dl(const SysDims& d, double k, Colloc c, int64_t n_pts, const double* pts,
                           const cplx* psi, cplx* partial, int n_chunks, cplx* u, hipStream_t s,
                           int density);
hipError_t launch_rhs(const SysDims& d, double k, int kind, const double* p, Colloc c, cplx* g,
                      hipStream_t s);
hipError_t launch_field(const SysDims& d, double k, Colloc c, int64_t n_pts, const double* pts,
                        const cplx* phi, cplx* partial, int n_chunks, cplx* u, hipStream_t s,
                        int density = 0);

// counts[0] += pairs flagged FFBIE_PAIR_UNRESOLVED, counts[1] += pairs flagged
// FFBIE_PAIR_ROOT_FALLBACK among st[0..n); launch_zero_counts clears n counters
// with a kernel (no memset node when a caller captures the stream).
hipError_t launch_count_status(const int32_t* st, int64_t n, unsigned long long* counts,
                               hipStream_t s);
hipError_t launch_zero_counts(unsigned long long* counts, int n, hipStream_t s);

}  // namespace ffbie
