// Host side of the C ABI declared in include/ffbie.h: context, validation,
// exact angle tables, workspaces and kernel launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "ffbie.h"
#include "ffbie_device.hpp"

#include "ffbie_assembly.hpp"
#include "ffbie_blockjacobi.hpp"
#include "ffbie_gemm.hpp"
#include "ffbie_banded.hpp"
#include "ffbie_kernels.hpp"
#include "ffbie_mlp.hpp"
#include "ffbie_solve.hpp"
#include "ffbie_tuning_cache.hpp"

using namespace ffbie;

namespace {
#include "ggq16_table.inc"
}

// ---------------------------------------------------------------------------
// Scratch of ffbie_kernel_coeffs_noalloc: a file-scope device array, one copy
// per GPU the library runs on, held until the process ends.  Layout for up to
// kNoAllocPairs pairs: root records, refine-list slots, status words, then the
// refine-list counter, each part 256-byte aligned.  In host code `scratch` is
// only a handle: its device address on each GPU comes from
// hipGetSymbolAddress (noalloc_scratch below) and is what the kernels receive.
// ---------------------------------------------------------------------------
namespace {
constexpr int64_t kNoAllocPairs = (int64_t)1 << 20;
constexpr size_t kNoAllocRootsOff = 0;
constexpr size_t kNoAllocListOff = kNoAllocRootsOff + kNoAllocPairs * sizeof(ffbie::RootRec);
constexpr size_t kNoAllocStatusOff = kNoAllocListOff + kNoAllocPairs * sizeof(int64_t);
constexpr size_t kNoAllocCountOff = kNoAllocStatusOff + kNoAllocPairs * sizeof(int32_t);
constexpr size_t kNoAllocBytes = kNoAllocCountOff + 256;
static_assert(kNoAllocListOff % 256 == 0 && kNoAllocStatusOff % 256 == 0 && kNoAllocCountOff % 256 == 0,
              "scratch parts must stay 256-byte aligned");
constexpr int kMaxDevices = 64;
constexpr size_t kLdsPerCU = 160 * 1024;   // LDS of one gfx950 compute unit
}  // namespace

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

namespace {
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of `scratch` on `device` (which must be current), looked up
// once per device.
hipError_t noalloc_scratch(int device, void** out) {
  if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch[device]) {
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch[device] = p;
  }
  *out = g_scratch[device];
  return hipSuccess;
}
}  // namespace

struct ffbie_ctx {
  int device = 0;
  int n_cu = 256;            // compute units of the device (grid sizing)
  hipStream_t stream = nullptr;
  std::string err;
  bool has_problem = false;
  Prob prob{};
  int n_panels = 0;
  int variant = FFBIE_KAPPA_SWAP;
  double* d_tab = nullptr;
  // workspaces (grown on demand)
  RootRec* d_roots = nullptr;
  int32_t* d_status = nullptr;
  int64_t* d_list = nullptr;
  int32_t* d_count = nullptr;
  int64_t ws_pairs = 0;
  // optional event timing of the three launches
  bool timing = false;
  bool timed = false;
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  // discrete system (assembly, right-hand sides, field)
  ffbie_near_rule rule{};
  double gl_x[kNodes] = {0}, gl_w[kNodes] = {0};
  bool sys_ready = false;            // rule tables and collocation data of the current problem
  double* d_rule_y = nullptr;        // [16 l][3 rel][16 q]
  double* d_wl = nullptr;            // [16 l][3 rel][16 q][16 l']
  double* d_colloc = nullptr;        // 5 N doubles: x, y, z, wq, jac
  int64_t colloc_n = 0;
  double* d_near_t = nullptr;        // near-pair workspace of one chunk
  int32_t* d_near_az = nullptr;
  double* d_near_ts = nullptr;
  cplx* d_near_kappa = nullptr;
  int64_t near_cap = 0;              // pairs
  int near_cap_M = 0;
  cplx* d_partial = nullptr;         // field partial sums
  int64_t partial_cap = 0;
  // dense solvers
  int64_t solve_n = 0;               // size the vector workspaces were made for
  int64_t* d_ipiv = nullptr;
  int64_t* d_perm = nullptr;
  int* d_info = nullptr;
  cplx* d_vecs = nullptr;            // 3 N complex128
  cplx* d_small = nullptr;           // reduction partials and Hessenberg column
  void* d_s32 = nullptr;
  int64_t s32_n = 0;
  cplx* d_krylov = nullptr;
  int64_t krylov_n = 0;
  // batched coefficients
  double* d_tabs[4] = {nullptr, nullptr, nullptr, nullptr};   // angle tables for M = 16 .. 128
  // FFT radix (0: by N_F), pairs per batch work item, waves per workgroup,
  // persistent batch launches
  ffbie_tuning tune{0, kBatchTile, 4, 0};
  std::string tune_cache;            // autotuner cache file ("" = none)
  ffbie_batch_plan* oneshot = nullptr;    // plan of the last ffbie_kernel_coeffs_batched call
  // learned preconditioner
  Mlp mlp;
  BlockJacobi bj;
  int64_t factored_n = 0;            // size of the LU64 factorisation held (ffbie_lu_factor)
  cplx* d_zbasis = nullptr;
  int64_t zbasis_n = 0;
  // banded route (Sec. 3.2.1): <rho^2>_n per pair, the m0-rule maxima, factor records
  cplx* d_band_c2 = nullptr;
  int64_t band_c2_cap = 0;
  double* d_band_ratio = nullptr;     // [16384 + 1][9]: per-block maxima, then the maxima
  cplx* d_band_fac = nullptr;
  int64_t band_fac_cap = 0;          // complex entries
  // flags of the near pairs of the last assembly
  unsigned long long* d_asm_counts = nullptr;
  int64_t asm_pairs = -1, asm_unresolved = -1, asm_fallback = -1;
  // minibatch order of ffbie_mlp_train
  int32_t* d_train_idx = nullptr;
  int64_t train_idx_cap = 0;
  // device address of this GPU's no-allocation scratch
  unsigned char* d_scratch = nullptr;
};

namespace {

const char* kNoCtx = "ffbie: NULL context";

void plan_free(ffbie_batch_plan* pl);

// Smooth-factor truncation threshold of the mixed-precision path: the FP32
// transforms leave a rounding floor of a few 1e-7 of the largest coefficient,
// so a smaller threshold would make p follow the noise.
constexpr double kEpsMixed = 1e-6;

ffbie_status fail(ffbie_ctx* c, ffbie_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

ffbie_status hip_fail(ffbie_ctx* c, hipError_t e, const char* what) {
  return fail(c, FFBIE_EDEVICE, std::string("ffbie: ") + what + ": " + hipGetErrorString(e));
}

#define FFBIE_HIP(ctx, call)                                  \
  do {                                                        \
    hipError_t e_ = (call);                                   \
    if (e_ != hipSuccess) return hip_fail((ctx), e_, #call);  \
  } while (0)

// sin(pi i / (4M)) correctly rounded from long double, reduced to the first octant
double table_sin(int i, int M) {
  const int n = 8 * M;
  i %= n;
  if (i < 0) i += n;
  int sign = 1;
  if (i >= 4 * M) { i -= 4 * M; sign = -1; }       // sin(x + pi) = -sin x
  if (i > 2 * M) i = 4 * M - i;                      // sin(pi - x) = sin x
  long double v;
  if (i <= M) {
    v = sinl((long double)M_PI * i / (4.0L * M));
  } else {
    v = cosl((long double)M_PI * (2 * M - i) / (4.0L * M));   // sin(pi/2 - y) = cos y
  }
  return sign * (double)v;
}

bool valid_M(int M) { return M == 16 || M == 32 || M == 64 || M == 128; }

// Gauss-Legendre nodes (ascending) and weights on [-1, 1]: Newton on P_16 in
// long double from the asymptotic initial guesses.
void gauss_legendre16(double* x, double* w) {
  const int n = kNodes;
  for (int i = 0; i < n; ++i) {
    long double z = cosl((long double)M_PI * (i + 0.75L) / (n + 0.5L));
    long double dp = 0;
    for (int it = 0; it < 100; ++it) {
      long double p0 = 1, p1 = z;
      for (int k = 2; k <= n; ++k) {
        const long double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = n * (z * p1 - p0) / (z * z - 1);
      const long double dz = p1 / dp;
      z -= dz;
      if (fabsl(dz) < 1e-19L) break;
    }
    long double p0 = 1, p1 = z;
    for (int k = 2; k <= n; ++k) {
      const long double p2 = ((2 * k - 1) * z * p1 - (k - 1) * p0) / k;
      p0 = p1;
      p1 = p2;
    }
    dp = n * (z * p1 - p0) / (z * z - 1);
    x[n - 1 - i] = (double)z;
    w[n - 1 - i] = (double)(2 / ((1 - z * z) * dp * dp));
  }
}

void builtin_rule(ffbie_near_rule* r) {
  std::memcpy(r->self_x, kGgqSelfNode, sizeof(r->self_x));
  std::memcpy(r->self_w, kGgqSelfWeight, sizeof(r->self_w));
  std::memcpy(r->right_x, kGgqRightNode, sizeof(r->right_x));
  std::memcpy(r->right_w, kGgqRightWeight, sizeof(r->right_w));
}

// Rule nodes and weights of target l, relation rel (-1, 0, +1), in the source
// panel's coordinate; the left rule mirrors the right rule of target 15 - l.
void relation_rule(const ffbie_near_rule& R, int l, int rel, double* y, double* w) {
  for (int q = 0; q < kNodes; ++q) {
    if (rel == 0) {
      y[q] = R.self_x[l][q];
      w[q] = R.self_w[l][q];
    } else if (rel == 1) {
      y[q] = R.right_x[l][q];
      w[q] = R.right_w[l][q];
    } else {
      y[q] = -R.right_x[kNodes - 1 - l][kNodes - 1 - q];
      w[q] = R.right_w[kNodes - 1 - l][kNodes - 1 - q];
    }
  }
}

// Lagrange basis of the Gauss-Legendre nodes at y (barycentric form).
void lagrange_row(const double* xg, double y, double* out) {
  long double lam[kNodes], s = 0;
  for (int a = 0; a < kNodes; ++a) {
    long double p = 1;
    for (int b = 0; b < kNodes; ++b)
      if (b != a) p *= (long double)xg[a] - xg[b];
    lam[a] = 1 / p;
  }
  for (int a = 0; a < kNodes; ++a) {
    if (y == xg[a]) {
      for (int b = 0; b < kNodes; ++b) out[b] = (a == b) ? 1.0 : 0.0;
      return;
    }
    s += lam[a] / ((long double)y - xg[a]);
  }
  for (int a = 0; a < kNodes; ++a) out[a] = (double)(lam[a] / ((long double)y - xg[a]) / s);
}

int64_t n_unknowns(const ffbie_ctx* c) { return (int64_t)32 * c->prob.M * c->n_panels; }

SysDims sys_dims(const ffbie_ctx* c) {
  SysDims d;
  d.n_panels = c->n_panels;
  d.M = c->prob.M;
  d.N = n_unknowns(c);
  d.h = M_PI / c->n_panels;
  return d;
}

Colloc colloc_view(const ffbie_ctx* c) {
  const int64_t N = c->colloc_n;
  double* b = c->d_colloc;
  return Colloc{b, b + N, b + 2 * N, b + 3 * N, b + 4 * N, b + 5 * N, b + 6 * N, b + 7 * N};
}

// Validated problem constants from the C-ABI description.
bool make_prob(const ffbie_geometry* g, const ffbie_discretization* d, double k, Prob* out,
               std::string* why) {
  if (!g || !d) { *why = "NULL geometry or discretisation"; return false; }
  if (g->lmax < 0 || g->lmax > kMaxL || g->mmax < 0 || g->mmax > kMaxM || (g->lmax > 0 && !g->a)) {
    *why = "amplitude table must have lmax <= 8, mmax <= 8";
    return false;
  }
  if (!valid_M(d->M)) { *why = "M must be 16, 32, 64 or 128"; return false; }
  if (d->M0 < 1 || d->M0 > d->M) { *why = "need 1 <= M0 <= M"; return false; }
  if (d->n_panels < 1) { *why = "n_panels must be >= 1"; return false; }
  if (!(k >= 0) || !std::isfinite(k)) { *why = "need k >= 0"; return false; }
  if (!(d->eps0 >= 0) || d->eps0 >= 1) { *why = "need 0 <= eps0 < 1"; return false; }
  if (d->kappa_variant != FFBIE_KAPPA_SWAP && d->kappa_variant != FFBIE_KAPPA_PAPER_CONV) {
    *why = "unknown kappa_variant";
    return false;
  }
  Prob P{};
  P.g.lmax = g->lmax;
  P.g.mmax = g->mmax;
  for (int l = 0; l < g->lmax; ++l)
    for (int m = 0; m <= g->mmax; ++m) {
      const double v = g->a[l * (g->mmax + 1) + m];
      if (!std::isfinite(v)) { *why = "non-finite amplitude"; return false; }
      P.g.a[l][m] = v;
    }
  P.g.ax[0] = P.g.ax[1] = P.g.ax[2] = 1.0;
  P.g.scaled = 0;
  if (g->axes) {
    for (int c = 0; c < 3; ++c) {
      const double v = g->axes[c];
      if (!(v > 0) || !std::isfinite(v)) { *why = "axes must be positive and finite"; return false; }
      P.g.ax[c] = v;
      if (v != 1.0) P.g.scaled = 1;
    }
  }
  P.k = k;
  P.eps0 = d->eps0 > 0 ? d->eps0 : 1e-15;
  P.M = d->M;
  P.M0 = d->M0;
  P.L = d->M + d->M0;
  P.tab_n = 8 * d->M;
  *out = P;
  return true;
}

ffbie_status ensure_ws(ffbie_ctx* c, int64_t n) {
  if (n <= c->ws_pairs) return FFBIE_OK;
  if (c->d_roots) hipFree(c->d_roots);
  if (c->d_status) hipFree(c->d_status);
  if (c->d_list) hipFree(c->d_list);
  c->d_roots = nullptr; c->d_status = nullptr; c->d_list = nullptr;
  c->ws_pairs = 0;
  if (hipMalloc(&c->d_roots, n * sizeof(RootRec)) != hipSuccess ||
      hipMalloc(&c->d_status, n * sizeof(int32_t)) != hipSuccess ||
      hipMalloc(&c->d_list, n * sizeof(int64_t)) != hipSuccess)
    return fail(c, FFBIE_ENOMEM, "ffbie: workspace allocation failed");
  c->ws_pairs = n;
  return FFBIE_OK;
}

// waves per workgroup so that the coefficient kernel fits 64 KiB of LDS
int coeff_waves(const Prob& P, int NF, int layout, bool single, size_t* lds_bytes) {
  const size_t per_wave = sizeof(double) * coeff_lds_per_wave(NF, P.M, P.L, layout, single);
  const size_t tab = sizeof(double) * (P.tab_n + coeff_twiddle_doubles(NF, single));
  int w = 4;
  while (w > 1 && tab + w * per_wave > 65536) --w;
  *lds_bytes = tab + w * per_wave;
  return w;
}

}  // namespace

extern "C" {

ffbie_status ffbie_create(ffbie_ctx** out, int device, void* hip_stream) {
  if (!out) return FFBIE_EINVAL;
  *out = nullptr;
  int n = 0;
  if (hipGetDeviceCount(&n) != hipSuccess || device < 0 || device >= n) return FFBIE_EINVAL;
  ffbie_ctx* c = new ffbie_ctx();
  builtin_rule(&c->rule);
  gauss_legendre16(c->gl_x, c->gl_w);
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  if (hipSetDevice(device) != hipSuccess) { delete c; return FFBIE_EDEVICE; }
  int n_cu = 0;
  if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess &&
      n_cu > 0)
    c->n_cu = n_cu;
  if (hipMalloc(&c->d_count, 4 * sizeof(int32_t)) != hipSuccess) { delete c; return FFBIE_ENOMEM; }
  void* sp = nullptr;
  if (noalloc_scratch(device, &sp) != hipSuccess) {
    (void)hipFree(c->d_count);
    delete c;
    return FFBIE_EDEVICE;
  }
  c->d_scratch = static_cast<unsigned char*>(sp);
  *out = c;
  return FFBIE_OK;
}

ffbie_status ffbie_destroy(ffbie_ctx* c) {
  if (!c) return FFBIE_OK;
  hipSetDevice(c->device);
  if (c->oneshot) {
    (void)hipStreamSynchronize(c->stream);
    plan_free(c->oneshot);
  }
  for (auto& e : c->ev)
    if (e) hipEventDestroy(e);
  if (c->d_tab) hipFree(c->d_tab);
  if (c->d_roots) hipFree(c->d_roots);
  if (c->d_status) hipFree(c->d_status);
  if (c->d_list) hipFree(c->d_list);
  if (c->d_count) hipFree(c->d_count);
  for (void* p : {(void*)c->d_rule_y, (void*)c->d_wl, (void*)c->d_colloc, (void*)c->d_near_t,
                  (void*)c->d_near_az, (void*)c->d_near_ts, (void*)c->d_near_kappa,
                  (void*)c->d_partial, (void*)c->d_ipiv, (void*)c->d_perm, (void*)c->d_info,
                  (void*)c->d_vecs, (void*)c->d_small, c->d_s32, (void*)c->d_krylov,
                  (void*)c->d_tabs[0], (void*)c->d_tabs[1], (void*)c->d_tabs[2],
                  (void*)c->d_tabs[3]})
    if (p) hipFree(p);
  if (c->d_zbasis) (void)hipFree(c->d_zbasis);
  if (c->d_band_c2) (void)hipFree(c->d_band_c2);
  if (c->d_band_ratio) (void)hipFree(c->d_band_ratio);
  if (c->d_band_fac) (void)hipFree(c->d_band_fac);
  if (c->d_asm_counts) (void)hipFree(c->d_asm_counts);
  if (c->d_train_idx) (void)hipFree(c->d_train_idx);
  c->mlp.release();
  c->bj.release();
  delete c;
  return FFBIE_OK;
}

const char* ffbie_last_error(const ffbie_ctx* c) { return c ? c->err.c_str() : kNoCtx; }

ffbie_status ffbie_set_problem(ffbie_ctx* c, const ffbie_geometry* g, const ffbie_discretization* d,
                               double k) {
  if (!c) return FFBIE_EINVAL;
  Prob P{};
  std::string why;
  if (!make_prob(g, d, k, &P, &why)) return fail(c, FFBIE_EINVAL, "ffbie_set_problem: " + why);
  FFBIE_HIP(c, hipSetDevice(c->device));
  if (c->d_tab) { hipFree(c->d_tab); c->d_tab = nullptr; }
  std::vector<double> tab(P.tab_n);
  for (int i = 0; i < P.tab_n; ++i) tab[i] = table_sin(i, P.M);
  FFBIE_HIP(c, hipMalloc(&c->d_tab, P.tab_n * sizeof(double)));
  FFBIE_HIP(c, hipMemcpy(c->d_tab, tab.data(), P.tab_n * sizeof(double), hipMemcpyHostToDevice));
  c->prob = P;
  c->variant = d->kappa_variant;
  c->n_panels = d->n_panels;
  c->has_problem = true;
  c->sys_ready = false;
  c->bj.ready = false;
  return FFBIE_OK;
}

}  // extern "C"

namespace {

// The coefficient path on n pairs: root kernel, main pass (2M samples), refine
// pass (4M samples); `single` selects the FP32 spectral stage (complex64
// outputs).  Inputs validated by the caller.
// Scratch the coefficient path works in: a root record and a refine-list
// slot per pair, the status words when the caller passes none, and the
// refine-list counter.
struct CoeffWs {
  RootRec* roots;
  int32_t* status;
  int64_t* list;
  int32_t* count;
};

ffbie_status run_coeffs_ws(ffbie_ctx* c, const CoeffWs& ws, int64_t n, const double* d_t,
                           const int32_t* d_az, const double* d_ts, void* d_kappa, void* d_rhoinv,
                           double* d_root, int32_t* d_pair_status, bool single) {
  const Prob& P = c->prob;
  int32_t* status = d_pair_status ? d_pair_status : ws.status;

  if (c->timing) FFBIE_HIP(c, hipEventRecord(c->ev[0], c->stream));
  // kernel 1: roots, one lane per pair
  FFBIE_HIP(c, launch_root(P, c->d_tab, n, d_t, d_az, d_ts, ws.roots, status, d_root, c->stream));
  FFBIE_HIP(c, launch_zero(ws.count, 1, c->stream));
  // kernel 2: main pass with 2M samples, then the refine pass with 4M samples
  CoeffArgs a{};
  a.P = P;
  if (single) a.P.eps0 = std::max(P.eps0, kEpsMixed);
  a.tab_g = c->d_tab;
  a.n = n;
  a.t_in = d_t;
  a.az_in = d_az;
  a.ts_in = d_ts;
  a.roots = ws.roots;
  a.status = status;
  a.kappa = d_kappa;
  a.rhoinv = d_rhoinv;
  a.variant = c->variant;
  a.radix = c->tune.fft_radix;
  const int layout = c->variant == FFBIE_KAPPA_PAPER_CONV ? kLdsFull
                     : (d_rhoinv != nullptr ? kLdsTransforms : kLdsCompact);
  {
    a.NF = 2 * P.M;
    a.flag_list = ws.list;
    a.flag_count = ws.count;
    size_t lds;
    const int w = coeff_waves(P, a.NF, layout, single, &lds);
    // 32 consecutive pairs per wavefront: fewer wavefronts share out the
    // per-wavefront set-up (tables, spilled constants) without a long tail
    const int64_t pairs_per_wave = 32;
    int64_t blocks = (n + w * pairs_per_wave - 1) / (w * pairs_per_wave);
    if (blocks < 1) blocks = 1;
    if (c->timing) FFBIE_HIP(c, hipEventRecord(c->ev[1], c->stream));
    FFBIE_HIP(c, launch_coeff(a, blocks, w, lds, c->stream, false, single));
    if (c->timing) FFBIE_HIP(c, hipEventRecord(c->ev[2], c->stream));
  }
  {
    a.NF = 4 * P.M;
    a.list = ws.list;
    a.list_count = ws.count;
    a.flag_list = nullptr;
    a.flag_count = nullptr;
    size_t lds;
    const int w = coeff_waves(P, a.NF, layout, single, &lds);
    FFBIE_HIP(c, launch_coeff(a, 512, w, lds, c->stream, true, single));
    if (c->timing) FFBIE_HIP(c, hipEventRecord(c->ev[3], c->stream));
  }
  if (c->timing) c->timed = true;
  return FFBIE_OK;
}

// Double-layer coefficients on n pairs: root kernel (shared with the
// single layer), main pass with 2M samples, refine pass with 4M samples.
ffbie_status run_dl_coeffs(ffbie_ctx* c, int64_t n, const double* d_t, const int32_t* d_az,
                           const double* d_ts, int adjoint, void* d_kappa, double* d_root,
                           int32_t* d_pair_status) {
  ffbie_status s = ensure_ws(c, n);
  if (s != FFBIE_OK) return s;
  const Prob& P = c->prob;
  int32_t* status = d_pair_status ? d_pair_status : c->d_status;
  FFBIE_HIP(c, launch_root(P, c->d_tab, n, d_t, d_az, d_ts, c->d_roots, status, d_root, c->stream));
  FFBIE_HIP(c, launch_zero(c->d_count, 1, c->stream));
  CoeffArgs a{};
  a.P = P;
  a.tab_g = c->d_tab;
  a.n = n;
  a.t_in = d_t;
  a.az_in = d_az;
  a.ts_in = d_ts;
  a.roots = c->d_roots;
  a.status = status;
  a.kappa = d_kappa;
  a.adjoint = adjoint;
  // wavefronts per workgroup (1..4, at most 64 KiB of LDS per workgroup) that
  // put the most wavefronts on a CU's 160 KiB of LDS (the table is per
  // workgroup, so fewer, larger workgroups share it; a leftover that fits no
  // further workgroup is lost); *per_cu receives that count
  auto waves = [&](int NF, size_t* lds, int* per_cu) {
    const size_t per_wave = sizeof(double) * dl_lds_per_wave(NF, P.M);
    const size_t tab = sizeof(double) * P.tab_n;
    int best_w = 1, best = 0;
    for (int w = 1; w <= 4; ++w) {
      const size_t wg = tab + w * per_wave;
      if (wg > 65536) break;
      const int on_cu = (int)(kLdsPerCU / wg) * w;
      if (on_cu >= best) { best = on_cu; best_w = w; }
    }
    *lds = tab + best_w * per_wave;
    *per_cu = best;
    return best_w;
  };
  {
    a.NF = 2 * P.M;
    a.flag_list = c->d_list;
    a.flag_count = c->d_count;
    size_t lds;
    int per_cu;
    const int w = waves(a.NF, &lds, &per_cu);
    const int64_t pairs_per_wave = 8;
    int64_t blocks = (n + w * pairs_per_wave - 1) / (w * pairs_per_wave);
    if (blocks < 1) blocks = 1;
    FFBIE_HIP(c, launch_dl_coeff(a, blocks, w, lds, c->stream, false));
  }
  {
    a.NF = 4 * P.M;
    a.list = c->d_list;
    a.list_count = c->d_count;
    a.flag_list = nullptr;
    a.flag_count = nullptr;
    size_t lds;
    int per_cu;
    const int w = waves(a.NF, &lds, &per_cu);
    // enough workgroups for every CU's share of wavefronts (the queue is
    // split evenly over all wavefronts of the grid)
    const int64_t blocks = std::max<int64_t>(1, (int64_t)c->n_cu * per_cu / w);
    FFBIE_HIP(c, launch_dl_coeff(a, blocks, w, lds, c->stream, true));
  }
  return FFBIE_OK;
}

// The coefficient path with the context's workspace (grown on demand).
ffbie_status run_coeffs(ffbie_ctx* c, int64_t n, const double* d_t, const int32_t* d_az,
                        const double* d_ts, void* d_kappa, void* d_rhoinv, double* d_root,
                        int32_t* d_pair_status, bool single = false) {
  ffbie_status s = ensure_ws(c, n);
  if (s != FFBIE_OK) return s;
  const CoeffWs ws{c->d_roots, c->d_status, c->d_list, c->d_count};
  return run_coeffs_ws(c, ws, n, d_t, d_az, d_ts, d_kappa, d_rhoinv, d_root, d_pair_status, single);
}

// Rule tables (node positions per relation and the weighted Lagrange matrices)
// and collocation data of the current problem.
ffbie_status prepare_system(ffbie_ctx* c) {
  if (c->sys_ready) return FFBIE_OK;
  const SysDims d = sys_dims(c);
  FFBIE_HIP(c, hipSetDevice(c->device));
  std::vector<double> ry(kNodes * 3 * kNodes), wl(kNodes * 3 * kNodes * kNodes);
  for (int l = 0; l < kNodes; ++l)
    for (int rel = -1; rel <= 1; ++rel) {
      double y[kNodes], w[kNodes];
      relation_rule(c->rule, l, rel, y, w);
      for (int q = 0; q < kNodes; ++q) {
        ry[(l * 3 + rel + 1) * kNodes + q] = y[q];
        double L[kNodes];
        lagrange_row(c->gl_x, y[q], L);
        // (h/2) W_q L_{l'}(y_q) and the 1/(2M) of the inverse DFT
        const double f = 0.5 * d.h * w[q] / (2.0 * d.M);
        for (int lp = 0; lp < kNodes; ++lp)
          wl[((l * 3 + rel + 1) * kNodes + q) * kNodes + lp] = f * L[lp];
      }
    }
  if (!c->d_rule_y) FFBIE_HIP(c, hipMalloc(&c->d_rule_y, ry.size() * sizeof(double)));
  if (!c->d_wl) FFBIE_HIP(c, hipMalloc(&c->d_wl, wl.size() * sizeof(double)));
  FFBIE_HIP(c, hipMemcpy(c->d_rule_y, ry.data(), ry.size() * sizeof(double), hipMemcpyHostToDevice));
  FFBIE_HIP(c, hipMemcpy(c->d_wl, wl.data(), wl.size() * sizeof(double), hipMemcpyHostToDevice));
  if (c->colloc_n != d.N) {
    if (c->d_colloc) hipFree(c->d_colloc);
    c->d_colloc = nullptr;
    c->colloc_n = 0;
    if (hipMalloc(&c->d_colloc, kCollocArrays * d.N * sizeof(double)) != hipSuccess)
      return fail(c, FFBIE_ENOMEM, "ffbie: collocation workspace allocation failed");
    c->colloc_n = d.N;
  }
  FFBIE_HIP(c, launch_collocation(c->prob.g, d, c->gl_x, c->gl_w, colloc_view(c), nullptr, nullptr,
                                  nullptr, c->stream));
  c->sys_ready = true;
  return FFBIE_OK;
}

constexpr int64_t kNearKappaBytes = (int64_t)2 << 30;    // near-coefficient workspace bound

ffbie_status ensure_near_ws(ffbie_ctx* c, int64_t pairs) {
  if (pairs <= c->near_cap && c->near_cap_M == c->prob.M) return FFBIE_OK;
  for (void* p : {(void*)c->d_near_t, (void*)c->d_near_az, (void*)c->d_near_ts,
                  (void*)c->d_near_kappa})
    if (p) hipFree(p);
  c->d_near_t = nullptr; c->d_near_az = nullptr; c->d_near_ts = nullptr; c->d_near_kappa = nullptr;
  c->near_cap = 0;
  if (hipMalloc(&c->d_near_t, pairs * sizeof(double)) != hipSuccess ||
      hipMalloc(&c->d_near_az, pairs * sizeof(int32_t)) != hipSuccess ||
      hipMalloc(&c->d_near_ts, pairs * sizeof(double)) != hipSuccess ||
      hipMalloc(&c->d_near_kappa, pairs * 2 * c->prob.M * sizeof(cplx)) != hipSuccess)
    return fail(c, FFBIE_ENOMEM, "ffbie: near-pair workspace allocation failed");
  c->near_cap = pairs;
  c->near_cap_M = c->prob.M;
  return FFBIE_OK;
}

}  // namespace

// Problems of one M inside a batch plan (contiguous in the plan's order).
struct PlanClass {
  int M = 0;
  int lo = 0, hi = 0;                  // problem range
  int64_t pairs = 0;
  ffbie_tuning tune{};
  double tuned_ms = 0.0;
  int64_t n_items = 0;
  int waves = 1, refine_waves = 1;
  size_t lds = 0, refine_lds = 0;
  int tw = 0;                          // doubles of FFT twiddles in LDS
};

struct ffbie_batch_plan {
  ffbie_ctx* ctx = nullptr;
  int flags = 0;
  bool single = false;
  int np = 0;                          // non-empty problems, ordered by decreasing M
  int mm = 0, Mmax = 16;
  int64_t total = 0;                   // pairs
  std::vector<CoeffArgs> args;         // host copy of the descriptors
  std::vector<int64_t> item_prefix;    // per problem, relative to its class
  std::vector<PlanClass> cls;
  int64_t n_root = 0;
  // device memory owned by the plan
  CoeffArgs* d_args = nullptr;
  int64_t* d_item_prefix = nullptr;
  int64_t* d_root_prefix = nullptr;
  RootRec* d_roots = nullptr;
  int32_t* d_status = nullptr;         // status of items without an output array
  int64_t* d_list = nullptr;           // refine queue
  int* d_count = nullptr;              // [0] refine queue length, [1 + c] work counter of class c
  hipStream_t cap_stream = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

// Workgroups x wavefronts of the batched refine pass: the queue length is
// known only on the device, so a fixed grid walks it.
constexpr int kRefineWaves = 2048;
// Upper bound on the workgroups of a persistent main pass.
constexpr int64_t kMainBlocks = 2048;
constexpr int kMaxClasses = 4;         // M = 16, 32, 64, 128

bool valid_tuning(const ffbie_tuning& t, std::string* why) {
  if (t.fft_radix != 0 && t.fft_radix != 2 && t.fft_radix != 4) {
    *why = "fft_radix must be 0, 2 or 4";
    return false;
  }
  if (t.pairs_per_item < 1 || t.pairs_per_item > 256) { *why = "pairs_per_item must be in [1, 256]"; return false; }
  if (t.waves_per_block != 1 && t.waves_per_block != 2 && t.waves_per_block != 4) {
    *why = "waves_per_block must be 1, 2 or 4";
    return false;
  }
  if (t.persistent != 0 && t.persistent != 1) { *why = "persistent must be 0 or 1"; return false; }
  return true;
}

void plan_free(ffbie_batch_plan* pl) {
  if (!pl) return;
  if (pl->exec) (void)hipGraphExecDestroy(pl->exec);
  if (pl->graph) (void)hipGraphDestroy(pl->graph);
  if (pl->cap_stream) (void)hipStreamDestroy(pl->cap_stream);
  for (void* p : {(void*)pl->d_args, (void*)pl->d_item_prefix, (void*)pl->d_root_prefix,
                  (void*)pl->d_roots, (void*)pl->d_status, (void*)pl->d_list, (void*)pl->d_count})
    if (p) (void)hipFree(p);
  delete pl;
}

// Launch shape and work-item numbering of class k for tuning t; uploads the
// class's descriptors (radix) and item prefix and waits for the upload.
ffbie_status plan_shape(ffbie_ctx* c, ffbie_batch_plan* pl, int k, const ffbie_tuning& t) {
  PlanClass& q = pl->cls[k];
  const size_t tab = sizeof(double) * 8 * q.M;
  q.tw = coeff_twiddle_doubles(2 * q.M, pl->single);
  const size_t per_wave = sizeof(double) * coeff_lds_per_wave(2 * q.M, q.M, 2 * q.M, kLdsCompact, pl->single);
  int waves = t.waves_per_block;
  while (waves > 1 && tab + q.tw * sizeof(double) + waves * per_wave > 65536) waves >>= 1;
  q.tune = t;
  q.tune.waves_per_block = waves;
  q.waves = waves;
  q.lds = tab + q.tw * sizeof(double) + waves * per_wave;
  const size_t per_wave_r = sizeof(double) * coeff_lds_per_wave(4 * q.M, q.M, 2 * q.M, kLdsCompact, pl->single);
  q.refine_waves = 4;
  while (q.refine_waves > 1 && tab + q.refine_waves * per_wave_r > 65536) q.refine_waves >>= 1;
  q.refine_lds = tab + q.refine_waves * per_wave_r;
  int64_t n = 0;
  for (int s = q.lo; s < q.hi; ++s) {
    pl->args[s].radix = t.fft_radix;
    pl->item_prefix[s] = n;
    n += (pl->args[s].n + t.pairs_per_item - 1) / t.pairs_per_item;
  }
  q.n_items = n;
  FFBIE_HIP(c, hipMemcpyAsync(pl->d_args + q.lo, pl->args.data() + q.lo, (q.hi - q.lo) * sizeof(CoeffArgs),
                              hipMemcpyHostToDevice, c->stream));
  FFBIE_HIP(c, hipMemcpyAsync(pl->d_item_prefix + q.lo, pl->item_prefix.data() + q.lo,
                              (q.hi - q.lo) * sizeof(int64_t), hipMemcpyHostToDevice, c->stream));
  FFBIE_HIP(c, hipStreamSynchronize(c->stream));      // host data may change next
  return FFBIE_OK;
}

BatchArgs plan_args(const ffbie_batch_plan* pl) {
  BatchArgs b{};
  b.probs = pl->d_args;
  b.n_probs = pl->np;
  b.root_prefix = pl->d_root_prefix;
  b.flag_list = pl->d_list;
  b.flag_count = pl->d_count;
  b.tab_max = 8 * pl->Mmax;
  return b;
}

hipError_t launch_class_main(const ffbie_batch_plan* pl, int k, hipStream_t stream) {
  const PlanClass& q = pl->cls[k];
  BatchArgs b = plan_args(pl);
  b.probs = pl->d_args + q.lo;
  b.n_probs = q.hi - q.lo;
  b.item_prefix = pl->d_item_prefix + q.lo;
  b.n_items = q.n_items;
  b.item_counter = pl->d_count + 1 + k;
  b.tab_max = 8 * q.M;
  b.tw_max = q.tw;
  b.tile = q.tune.pairs_per_item;
  b.radix = (q.tune.fft_radix == 4 || (q.tune.fft_radix == 0 && 2 * q.M >= 256)) ? 4 : 2;
  b.persistent = q.tune.persistent;
  // persistent: at most kMainBlocks workgroups loop over the items; otherwise
  // one wavefront per item
  int64_t blocks = (q.n_items + q.waves - 1) / q.waves;
  if (blocks * 64 * q.waves >= ((int64_t)1 << 32)) b.persistent = 1;   // grid size limit
  if (b.persistent) blocks = std::min<int64_t>(blocks, kMainBlocks);
  return launch_batch(b, pl->mm, blocks, 64 * q.waves, q.lds, stream, 1, pl->single);
}

hipError_t launch_class_refine(const ffbie_batch_plan* pl, int k, hipStream_t stream) {
  const PlanClass& q = pl->cls[k];
  BatchArgs b = plan_args(pl);
  b.tab_max = 8 * q.M;
  b.prob_lo = q.lo;
  b.prob_hi = q.hi;
  return launch_batch(b, pl->mm, kRefineWaves / q.refine_waves, 64 * q.refine_waves, q.refine_lds,
                      stream, 2, pl->single);
}

// Counter reset, root pass, main pass of every M class, refine pass of every
// class, on `stream`; with `timed`, the context's timing events bracket the
// root, main and refine passes.
ffbie_status plan_launch(ffbie_ctx* c, ffbie_batch_plan* pl, hipStream_t stream, bool timed = false) {
  FFBIE_HIP(c, launch_zero(pl->d_count, 1 + kMaxClasses, stream));
  if (timed) FFBIE_HIP(c, hipEventRecord(c->ev[0], stream));
  FFBIE_HIP(c, launch_batch(plan_args(pl), pl->mm, pl->n_root, 256, 8 * pl->Mmax * sizeof(double), stream,
                            0, pl->single));
  if (timed) FFBIE_HIP(c, hipEventRecord(c->ev[1], stream));
  for (int k = 0; k < (int)pl->cls.size(); ++k) FFBIE_HIP(c, launch_class_main(pl, k, stream));
  if (timed) FFBIE_HIP(c, hipEventRecord(c->ev[2], stream));
  for (int k = 0; k < (int)pl->cls.size(); ++k) FFBIE_HIP(c, launch_class_refine(pl, k, stream));
  if (timed) {
    FFBIE_HIP(c, hipEventRecord(c->ev[3], stream));
    c->timed = true;
  }
  return FFBIE_OK;
}

ffbie_status plan_build(ffbie_ctx* c, ffbie_batch_plan* pl, int n_items, const ffbie_batch_item* items,
                        const ffbie_tuning* t) {
  if (n_items < 0 || (n_items > 0 && !items))
    return fail(c, FFBIE_EINVAL, "ffbie batch: invalid item array");
  if (n_items >= (1 << 22)) return fail(c, FFBIE_EINVAL, "ffbie batch: too many items");
  // validate, and order the non-empty problems by decreasing M
  std::vector<Prob> probs(n_items);
  std::vector<int> order;
  for (int i = 0; i < n_items; ++i) {
    const ffbie_batch_item& it = items[i];
    std::string why;
    if (!make_prob(&it.g, &it.d, it.k, &probs[i], &why))
      return fail(c, FFBIE_EINVAL, "ffbie batch: item " + std::to_string(i) + ": " + why);
    if (it.d.kappa_variant != FFBIE_KAPPA_SWAP)
      return fail(c, FFBIE_EINVAL, "ffbie batch: only FFBIE_KAPPA_SWAP is batched");
    if (probs[i].g.scaled)
      return fail(c, FFBIE_EINVAL, "ffbie batch: item " + std::to_string(i) +
                                       ": stretched surfaces (axes != 1) are not batched");
    if (it.n_pairs < 0 || it.n_pairs > ((int64_t)1 << 31))
      return fail(c, FFBIE_EINVAL, "ffbie batch: n_pairs out of range");
    if (it.n_pairs == 0) continue;
    if (!it.d_t || !it.d_az || !it.d_ts || !it.d_kappa)
      return fail(c, FFBIE_EINVAL, "ffbie batch: NULL pair or kappa pointer");
    order.push_back(i);
    pl->total += it.n_pairs;
    pl->mm = std::max(pl->mm, it.g.mmax);
    pl->Mmax = std::max(pl->Mmax, it.d.M);
  }
  pl->np = (int)order.size();
  if (pl->np == 0) return FFBIE_OK;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return items[a].d.M > items[b].d.M; });
  for (int q = 0; q < kMaxClasses; ++q) {
    const int M = 16 << q;
    if (c->d_tabs[q]) continue;
    std::vector<double> tab(8 * M);
    for (int i = 0; i < 8 * M; ++i) tab[i] = table_sin(i, M);
    FFBIE_HIP(c, hipMalloc(&c->d_tabs[q], tab.size() * sizeof(double)));
    FFBIE_HIP(c, hipMemcpy(c->d_tabs[q], tab.data(), tab.size() * sizeof(double), hipMemcpyHostToDevice));
  }
  const int np = pl->np;
  const int64_t total = pl->total;
  if (hipMalloc(&pl->d_args, np * sizeof(CoeffArgs)) != hipSuccess ||
      hipMalloc(&pl->d_item_prefix, np * sizeof(int64_t)) != hipSuccess ||
      hipMalloc(&pl->d_root_prefix, np * sizeof(int64_t)) != hipSuccess ||
      hipMalloc(&pl->d_roots, total * sizeof(RootRec)) != hipSuccess ||
      hipMalloc(&pl->d_status, total * sizeof(int32_t)) != hipSuccess ||
      hipMalloc(&pl->d_list, total * sizeof(int64_t)) != hipSuccess ||
      hipMalloc(&pl->d_count, (1 + kMaxClasses) * sizeof(int)) != hipSuccess)
    return fail(c, FFBIE_ENOMEM, "ffbie batch: workspace allocation failed");
  pl->args.resize(np);
  pl->item_prefix.resize(np);
  std::vector<int64_t> root_prefix(np);
  int64_t off = 0;
  pl->n_root = 0;
  for (int q = 0; q < np; ++q) {
    const ffbie_batch_item& it = items[order[q]];
    CoeffArgs& a = pl->args[q];
    a = CoeffArgs{};
    a.P = probs[order[q]];
    if (pl->single) a.P.eps0 = std::max(a.P.eps0, kEpsMixed);
    int qi = 0;
    while ((16 << qi) != it.d.M) ++qi;
    a.tab_g = c->d_tabs[qi];
    a.n = it.n_pairs;
    a.t_in = it.d_t;
    a.az_in = it.d_az;
    a.ts_in = it.d_ts;
    a.roots = pl->d_roots + off;
    a.status = it.d_pair_status ? it.d_pair_status : pl->d_status + off;
    a.kappa = it.d_kappa;
    a.rhoinv = nullptr;
    a.NF = 2 * it.d.M;
    a.flag_list = pl->d_list;
    a.flag_count = pl->d_count;
    a.variant = FFBIE_KAPPA_SWAP;
    a.flag_tag = (int64_t)q << 40;
    a.radix = t[qi].fft_radix;
    root_prefix[q] = pl->n_root;
    pl->n_root += (it.n_pairs + 255) / 256;
    off += it.n_pairs;
    if (pl->cls.empty() || pl->cls.back().M != it.d.M) {
      PlanClass k;
      k.M = it.d.M;
      k.lo = q;
      pl->cls.push_back(k);
    }
    pl->cls.back().hi = q + 1;
    pl->cls.back().pairs += it.n_pairs;
  }
  FFBIE_HIP(c, hipMemcpyAsync(pl->d_root_prefix, root_prefix.data(), np * sizeof(int64_t),
                              hipMemcpyHostToDevice, c->stream));
  for (int k = 0; k < (int)pl->cls.size(); ++k) {
    int qi = 0;
    while ((16 << qi) != pl->cls[k].M) ++qi;
    const ffbie_status st = plan_shape(c, pl, k, t[qi]);
    if (st != FFBIE_OK) return st;
  }
  return FFBIE_OK;
}

// For every M class, times the class's main pass for each candidate tuning
// (FFT radix x pairs per work item x waves per workgroup) and keeps the
// fastest.  The root pass runs once first; the counters are reset before each
// run, so the refine queue never holds more than one entry per pair.
ffbie_status plan_autotune(ffbie_ctx* c, ffbie_batch_plan* pl) {
  hipEvent_t e0, e1;
  FFBIE_HIP(c, hipEventCreate(&e0));
  FFBIE_HIP(c, hipEventCreate(&e1));
  ffbie_status st = FFBIE_OK;
  hipError_t e = launch_zero(pl->d_count, 1 + kMaxClasses, c->stream);
  if (e == hipSuccess)
    e = launch_batch(plan_args(pl), pl->mm, pl->n_root, 256, 8 * pl->Mmax * sizeof(double), c->stream, 0,
                     pl->single);
  if (e != hipSuccess) st = hip_fail(c, e, "autotune root pass");
  // device key of the tuning cache: architecture and compute-unit count
  std::vector<TuneEntry> cache;
  std::string dev_key;
  bool cache_dirty = false;
  if (!c->tune_cache.empty()) {
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, c->device) == hipSuccess) {
      dev_key = std::string(prop.gcnArchName) + " x" + std::to_string(prop.multiProcessorCount);
      cache = tune_cache_read(c->tune_cache);
    }
  }
  const std::string prec = pl->single ? "f32" : "f64";
  for (int k = 0; k < (int)pl->cls.size() && st == FFBIE_OK; ++k) {
    if (!dev_key.empty()) {
      const TuneEntry* hit = tune_cache_find(cache, dev_key, pl->cls[k].M, prec);
      std::string why;
      if (hit && valid_tuning(hit->t, &why)) {
        st = plan_shape(c, pl, k, hit->t);
        if (st == FFBIE_OK && pl->cls[k].waves == hit->t.waves_per_block) {
          pl->cls[k].tuned_ms = hit->main_ms;
          continue;
        }
        if (st != FFBIE_OK) break;
      }
    }
    ffbie_tuning best = pl->cls[k].tune;
    float best_ms = -1.0f;
    for (int radix : {2, 4})
      for (int ppi : {8, 16, 32})
        for (int waves : {1, 2, 4})
          for (int pers : {0, 1}) {
          if (st != FFBIE_OK) break;
          if ((st = plan_shape(c, pl, k, ffbie_tuning{radix, ppi, waves, pers})) != FFBIE_OK) break;
          if (pl->cls[k].waves != waves) continue;          // does not fit the LDS
          float ms = 0.0f;
          for (int rep = 0; rep < 2 && st == FFBIE_OK; ++rep) {   // the first run warms up
            if ((e = launch_zero(pl->d_count, 1 + kMaxClasses, c->stream)) != hipSuccess ||
                (e = hipEventRecord(e0, c->stream)) != hipSuccess ||
                (e = launch_class_main(pl, k, c->stream)) != hipSuccess ||
                (e = hipEventRecord(e1, c->stream)) != hipSuccess ||
                (e = hipEventSynchronize(e1)) != hipSuccess ||
                (e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess)
              st = hip_fail(c, e, "autotune main pass");
          }
          if (st == FFBIE_OK && (best_ms < 0 || ms < best_ms)) {
            best_ms = ms;
            best = pl->cls[k].tune;
          }
        }
    if (st == FFBIE_OK) {
      st = plan_shape(c, pl, k, best);
      pl->cls[k].tuned_ms = best_ms;
      if (!dev_key.empty()) {
        TuneEntry te;
        te.device = dev_key;
        te.M = pl->cls[k].M;
        te.precision = prec;
        te.t = best;
        te.main_ms = best_ms;
        bool replaced = false;
        for (TuneEntry& e : cache)
          if (e.device == te.device && e.M == te.M && e.precision == te.precision) {
            e = te;
            replaced = true;
          }
        if (!replaced) cache.push_back(te);
        cache_dirty = true;
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (st == FFBIE_OK && cache_dirty && !tune_cache_write(c->tune_cache, cache))
    return fail(c, FFBIE_EDEVICE, "ffbie_batch_plan_create: cannot write the tuning cache " + c->tune_cache);
  return st;
}

// Captures the whole launch sequence into a graph on a private stream;
// execute launches the graph on the context's stream.
ffbie_status plan_capture(ffbie_ctx* c, ffbie_batch_plan* pl) {
  FFBIE_HIP(c, hipStreamCreateWithFlags(&pl->cap_stream, hipStreamNonBlocking));
  FFBIE_HIP(c, hipStreamBeginCapture(pl->cap_stream, hipStreamCaptureModeThreadLocal));
  const ffbie_status st = plan_launch(c, pl, pl->cap_stream);
  hipGraph_t g = nullptr;
  const hipError_t e = hipStreamEndCapture(pl->cap_stream, &g);
  if (st != FFBIE_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  FFBIE_HIP(c, e);
  pl->graph = g;
  FFBIE_HIP(c, hipGraphInstantiate(&pl->exec, pl->graph, nullptr, nullptr, 0));
  return FFBIE_OK;
}

}  // namespace

extern "C" {

ffbie_status ffbie_kernel_coeffs(ffbie_ctx* c, int64_t n, const double* d_t, const int32_t* d_az,
                                 const double* d_ts, void* d_kappa, void* d_rhoinv, double* d_root,
                                 int32_t* d_pair_status) {
  if (!c) return FFBIE_EINVAL;
  if (!c->has_problem) return fail(c, FFBIE_ENOPROBLEM, "ffbie_kernel_coeffs: no problem set");
  if (n < 0) return fail(c, FFBIE_EINVAL, "ffbie_kernel_coeffs: n_pairs < 0");
  if (n == 0) return FFBIE_OK;
  if (!d_t || !d_az || !d_ts || !d_kappa)
    return fail(c, FFBIE_EINVAL, "ffbie_kernel_coeffs: NULL input or kappa pointer");
  if (n > (int64_t)1 << 31) return fail(c, FFBIE_EINVAL, "ffbie_kernel_coeffs: n_pairs > 2^31");
  FFBIE_HIP(c, hipSetDevice(c->device));
  return run_coeffs(c, n, d_t, d_az, d_ts, d_kappa, d_rhoinv, d_root, d_pair_status);
}

ffbie_status ffbie_kernel_coeffs_noalloc(ffbie_ctx* c, int64_t n, const double* d_t,
                                         const int32_t* d_az, const double* d_ts, void* d_kappa,
                                         void* d_rhoinv, double* d_root, int32_t* d_pair_status) {
  if (!c) return FFBIE_EINVAL;
  if (!c->has_problem) return fail(c, FFBIE_ENOPROBLEM, "ffbie_kernel_coeffs_noalloc: no problem set");
  if (n < 0) return fail(c, FFBIE_EINVAL, "ffbie_kernel_coeffs_noalloc: n_pairs < 0");
  if (n > kNoAllocPairs)
    return fail(c, FFBIE_EINVAL, "ffbie_kernel_coeffs_noalloc: n_pairs above the scratch capacity of "
                                 "1048576 pairs");
  if (n == 0) return FFBIE_OK;
  if (!d_t || !d_az || !d_ts || !d_kappa)
    return fail(c, FFBIE_EINVAL, "ffbie_kernel_coeffs_noalloc: NULL input or kappa pointer");
  if (!c->d_scratch) return fail(c, FFBIE_EDEVICE, "ffbie_kernel_coeffs_noalloc: no scratch address");
  FFBIE_HIP(c, hipSetDevice(c->device));
  const CoeffWs ws{reinterpret_cast<RootRec*>(c->d_scratch + kNoAllocRootsOff),
                   reinterpret_cast<int32_t*>(c->d_scratch + kNoAllocStatusOff),
                   reinterpret_cast<int64_t*>(c->d_scratch + kNoAllocListOff),
                   reinterpret_cast<int32_t*>(c->d_scratch + kNoAllocCountOff)};
  return run_coeffs_ws(c, ws, n, d_t, d_az, d_ts, d_kappa, d_rhoinv, d_root, d_pair_status, false);
}

ffbie_status ffbie_kernel_coeffs_mixed(ffbie_ctx* c, int64_t n, const double* d_t,
                                       const int32_t* d_az, const double* d_ts, void* d_kappa,
                                       void* d_rhoinv, double* d_root, int32_t* d_pair_status) {
  if (!c) return FFBIE_EINVAL;
  if (!c->has_problem) return fail(c, FFBIE_ENOPROBLEM, "ffbie_kernel_coeffs_mixed: no problem set");
  if (n < 0) return fail(c, FFBIE_EINVAL, "ffbie_kernel_coeffs_mixed: n_pairs < 0");
  if (c->prob.g.scaled)
    return fail(c, FFBIE_EINVAL, "ffbie_kernel_coeffs_mixed: stretched surfaces (axes != 1) take the FP64 path");
  if (n == 0) return FFBIE_OK;
  if (!d_t || !d_az || !d_ts || !d_kappa)
    return fail(c, FFBIE_EINVAL, "ffbie_kernel_coeffs_mixed: NULL input or kappa pointer");
  if (n > (int64_t)1 << 31) return fail(c, FFBIE_EINVAL, "ffbie_kernel_coeffs_mixed: n_pairs > 2^31");
  FFBIE_HIP(c, hipSetDevice(c->device));
  return run_coeffs(c, n, d_t, d_az, d_ts, d_kappa, d_rhoinv, d_root, d_pair_status, true);
}

ffbie_status ffbie_kernel_coeffs_dl(ffbie_ctx* c, int64_t n, const double* d_t, const int32_t* d_az,
                                    const double* d_ts, int adjoint, void* d_kappa, double* d_root,
                                    int32_t* d_pair_status) {
  if (!c) return FFBIE_EINVAL;
  if (!c->has_problem) return fail(c, FFBIE_ENOPROBLEM, "ffbie_kernel_coeffs_dl: no problem set");
  if (n < 0) return fail(c, FFBIE_EINVAL, "ffbie_kernel_coeffs_dl: n_pairs < 0");
  if (adjoint != 0 && adjoint != 1)
    return fail(c, FFBIE_EINVAL, "ffbie_kernel_coeffs_dl: adjoint must be 0 (K) or 1 (K')");
  if (n == 0) return FFBIE_OK;
  if (!d_t || !d_az || !d_ts || !d_kappa)
    return fail(c, FFBIE_EINVAL, "ffbie_kernel_coeffs_dl: NULL input or kappa pointer");
  if (n > (int64_t)1 << 31) return fail(c, FFBIE_EINVAL, "ffbie_kernel_coeffs_dl: n_pairs > 2^31");
  FFBIE_HIP(c, hipSetDevice(c->device));
  return run_dl_coeffs(c, n, d_t, d_az, d_ts, adjoint, d_kappa, d_root, d_pair_status);
}

ffbie_status ffbie_rhoinv_banded(ffbie_ctx* c, int64_t n, const double* d_t, const int32_t* d_az,
                                 const double* d_ts, int m0, void* d_rhoinv, int32_t* d_pair_status,
                                 int* m0_used) {
  static const char* fn = "ffbie_rhoinv_banded: ";
  if (!c) return FFBIE_EINVAL;
  if (!c->has_problem) return fail(c, FFBIE_ENOPROBLEM, std::string(fn) + "no problem set");
  if (n < 0) return fail(c, FFBIE_EINVAL, std::string(fn) + "n_pairs < 0");
  if (m0 < 0 || m0 > kBandMaxM0) return fail(c, FFBIE_EINVAL, std::string(fn) + "need 0 <= m0 <= 8");
  const Prob& P = c->prob;
  if (P.g.scaled)
    return fail(c, FFBIE_EINVAL, std::string(fn) + "stretched surfaces (axes != 1) are not supported");
  const int deg = rho2_degree(P.g);
  if (m0 == 0 && deg > kBandMaxM0)
    return fail(c, FFBIE_EINVAL, std::string(fn) + "rho^2 has degree " + std::to_string(deg) +
                                     " > 8 in the azimuth: pass m0 explicitly");
  const int m0_cap = m0 ? m0 : deg;
  if (P.L < 4 * m0_cap)
    return fail(c, FFBIE_EINVAL, std::string(fn) + "M + M0 must be at least 4 m0");
  if (m0_used) *m0_used = m0;
  if (n == 0) return FFBIE_OK;
  if (!d_t || !d_az || !d_ts || !d_rhoinv)
    return fail(c, FFBIE_EINVAL, std::string(fn) + "NULL input or output pointer");
  if (n > (int64_t)1 << 31) return fail(c, FFBIE_EINVAL, std::string(fn) + "n_pairs > 2^31");
  FFBIE_HIP(c, hipSetDevice(c->device));
  ffbie_status s = ensure_ws(c, n);
  if (s != FFBIE_OK) return s;
  if (n > c->band_c2_cap) {
    if (c->d_band_c2) hipFree(c->d_band_c2);
    c->d_band_c2 = nullptr;
    c->band_c2_cap = 0;
    if (hipMalloc(&c->d_band_c2, n * kBandC2 * sizeof(cplx)) != hipSuccess)
      return fail(c, FFBIE_ENOMEM, std::string(fn) + "workspace allocation failed");
    c->band_c2_cap = n;
  }
  if (!c->d_band_ratio &&
      hipMalloc(&c->d_band_ratio, (16384 + 1) * kBandC2 * sizeof(double)) != hipSuccess) {
    c->d_band_ratio = nullptr;
    return fail(c, FFBIE_ENOMEM, std::string(fn) + "workspace allocation failed");
  }
  int32_t* status = d_pair_status ? d_pair_status : c->d_status;
  FFBIE_HIP(c, launch_root(P, c->d_tab, n, d_t, d_az, d_ts, c->d_roots, status, nullptr, c->stream));
  BandArgs a{};
  a.P = P;
  a.tab_g = c->d_tab;
  a.n = n;
  a.t_in = d_t;
  a.az_in = d_az;
  a.ts_in = d_ts;
  a.roots = c->d_roots;
  a.status = status;
  a.c2 = c->d_band_c2;
  a.ratio_part = m0 == 0 ? c->d_band_ratio + kBandC2 : nullptr;
  a.ratio = c->d_band_ratio;
  a.rhoinv = static_cast<cplx*>(d_rhoinv);
  for (int q = 0; q < kNodes; ++q) { a.gl_x[q] = c->gl_x[q]; a.gl_w[q] = c->gl_w[q]; }
  FFBIE_HIP(c, launch_band_rho2(a, c->stream));
  if (m0 == 0) {
    // eq. (3.13) over this call's pairs, capped at the degree of rho^2 (the
    // coefficients above it vanish; only the transform's rounding shows there)
    double ratio[kBandC2];
    FFBIE_HIP(c, hipMemcpyAsync(ratio, c->d_band_ratio, sizeof(ratio), hipMemcpyDeviceToHost,
                                c->stream));
    FFBIE_HIP(c, hipStreamSynchronize(c->stream));
    m0 = 1;
    for (int q = 1; q <= deg; ++q)
      if (ratio[q] > P.eps0) m0 = q;
    if (m0_used) *m0_used = m0;
  }
  a.m0 = m0;
  FFBIE_HIP(c, launch_band_moments(a, c->stream));
  // factor records: (M1 + 1) rows of m0 + 1 complex values per pair, pairs in
  // chunks of at most 4 GiB of records
  const int64_t rows = P.L - 2 * m0 + 1;
  const int64_t per_pair = rows * (m0 + 1);
  int64_t chunk = ((int64_t)1 << 32) / (int64_t)(per_pair * sizeof(cplx));
  chunk = std::max<int64_t>(64, chunk / 64 * 64);
  chunk = std::min<int64_t>(chunk, (n + 63) / 64 * 64);
  if (chunk * per_pair > c->band_fac_cap) {
    if (c->d_band_fac) hipFree(c->d_band_fac);
    c->d_band_fac = nullptr;
    c->band_fac_cap = 0;
    if (hipMalloc(&c->d_band_fac, chunk * per_pair * sizeof(cplx)) != hipSuccess)
      return fail(c, FFBIE_ENOMEM, std::string(fn) + "factor workspace allocation failed");
    c->band_fac_cap = chunk * per_pair;
  }
  a.fac = c->d_band_fac;
  a.stride = chunk;
  for (int64_t c0 = 0; c0 < n; c0 += chunk) {
    a.chunk0 = c0;
    a.chunk_n = std::min<int64_t>(chunk, n - c0);
    FFBIE_HIP(c, launch_band_solve(a, c->stream));
  }
  return FFBIE_OK;
}

ffbie_status ffbie_builtin_near_rule(ffbie_near_rule* out) {
  if (!out) return FFBIE_EINVAL;
  builtin_rule(out);
  return FFBIE_OK;
}

ffbie_status ffbie_set_near_rule(ffbie_ctx* c, const ffbie_near_rule* rule) {
  if (!c) return FFBIE_EINVAL;
  ffbie_near_rule r;
  if (rule) {
    r = *rule;
  } else {
    builtin_rule(&r);
  }
  for (int l = 0; l < kNodes; ++l)
    for (int q = 0; q < kNodes; ++q) {
      const double sx = r.self_x[l][q], rx = r.right_x[l][q];
      if (!(std::fabs(sx) < 1.0) || !(std::fabs(rx) < 1.0) || !std::isfinite(r.self_w[l][q]) ||
          !std::isfinite(r.right_w[l][q]))
        return fail(c, FFBIE_EINVAL, "ffbie_set_near_rule: nodes must lie in (-1, 1), weights finite");
      if (std::fabs(sx - c->gl_x[l]) < 1e-13)
        return fail(c, FFBIE_EINVAL, "ffbie_set_near_rule: a self-panel node coincides with its target");
    }
  c->rule = r;
  c->sys_ready = false;
  return FFBIE_OK;
}

ffbie_status ffbie_query(ffbie_ctx* c, int64_t* n_unknowns_out, int64_t* n_near_pairs,
                         int64_t* workspace_bytes) {
  if (!c) return FFBIE_EINVAL;
  if (!c->has_problem) return fail(c, FFBIE_ENOPROBLEM, "ffbie_query: no problem set");
  const SysDims d = sys_dims(c);
  if (n_unknowns_out) *n_unknowns_out = d.N;
  const int64_t near = near_pairs_before(c->n_panels, d);
  if (n_near_pairs) *n_near_pairs = near;
  if (workspace_bytes) {
    const int64_t N = d.N;
    // assembly: near-pair chunk (inputs, kappa rows, coefficient workspace),
    // rule tables, collocation data
    const int64_t cap_pairs = kNearKappaBytes / (int64_t)(2 * d.M * sizeof(cplx));
    const int64_t chunk = std::min<int64_t>(near, cap_pairs + (int64_t)3 * kNodes * 2 * d.M * kNodes);
    const int64_t asm_ws = chunk * (20 + 2 * d.M * (int64_t)sizeof(cplx) + (int64_t)sizeof(RootRec) + 12) +
                           (int64_t)kNodes * 3 * kNodes * (kNodes + 1) * 8 + kCollocArrays * N * 8;
    // the largest solve: vectors and pivots, plus the complex64 copy of S
    // (LU32_IR64, GMRES_LU32) or the Krylov and flexible bases (GMRES forms),
    // or the mode blocks (block-Jacobi)
    const int64_t vecs = 3 * N * (int64_t)sizeof(cplx) + 2 * N * 8 + (256 * 101 + 101) * (int64_t)sizeof(cplx);
    const int64_t lu32 = N * N * 8 + 100 * N * (int64_t)sizeof(cplx) + 101 * N * (int64_t)sizeof(cplx);
    const int64_t nodes = 16 * (int64_t)d.n_panels;
    const int64_t bj = 2 * d.M * nodes * nodes * (int64_t)sizeof(cplx) + 201 * N * (int64_t)sizeof(cplx);
    *workspace_bytes = asm_ws + vecs + std::max(lu32, bj);
  }
  return FFBIE_OK;
}

ffbie_status ffbie_near_pairs(ffbie_ctx* c, double* d_t, int32_t* d_az, double* d_ts) {
  if (!c) return FFBIE_EINVAL;
  if (!c->has_problem) return fail(c, FFBIE_ENOPROBLEM, "ffbie_near_pairs: no problem set");
  if (!d_t || !d_az || !d_ts) return fail(c, FFBIE_EINVAL, "ffbie_near_pairs: NULL output");
  ffbie_status s = prepare_system(c);
  if (s != FFBIE_OK) return s;
  const SysDims d = sys_dims(c);
  NearChunk ch{0, c->n_panels, 0, near_pairs_before(c->n_panels, d)};
  FFBIE_HIP(c, launch_near_pairs(d, ch, c->gl_x, c->d_rule_y, d_t, d_az, d_ts, c->stream));
  return FFBIE_OK;
}

ffbie_status ffbie_collocation(ffbie_ctx* c, double* d_xyz, double* d_jac, double* d_wq) {
  if (!c) return FFBIE_EINVAL;
  if (!c->has_problem) return fail(c, FFBIE_ENOPROBLEM, "ffbie_collocation: no problem set");
  if (!d_xyz) return fail(c, FFBIE_EINVAL, "ffbie_collocation: NULL d_xyz");
  ffbie_status s = prepare_system(c);
  if (s != FFBIE_OK) return s;
  FFBIE_HIP(c, launch_collocation(c->prob.g, sys_dims(c), c->gl_x, c->gl_w, colloc_view(c), d_xyz,
                                  d_jac, d_wq, c->stream));
  return FFBIE_OK;
}

ffbie_status ffbie_rhs(ffbie_ctx* c, int kind, const double* params, void* d_g) {
  if (!c) return FFBIE_EINVAL;
  if (!c->has_problem) return fail(c, FFBIE_ENOPROBLEM, "ffbie_rhs: no problem set");
  if (!params || !d_g) return fail(c, FFBIE_EINVAL, "ffbie_rhs: NULL pointer");
  if (kind != FFBIE_RHS_POINT_SOURCE && kind != FFBIE_RHS_PLANE_WAVE && kind != FFBIE_RHS_PLANE_WAVE_DN &&
      kind != FFBIE_RHS_POINT_SOURCE_DN)
    return fail(c, FFBIE_EINVAL, "ffbie_rhs: unknown kind");
  for (int i = 0; i < 3; ++i)
    if (!std::isfinite(params[i])) return fail(c, FFBIE_EINVAL, "ffbie_rhs: non-finite parameter");
  ffbie_status s = prepare_system(c);
  if (s != FFBIE_OK) return s;
  FFBIE_HIP(c, launch_rhs(sys_dims(c), c->prob.k, kind, params, colloc_view(c),
                          static_cast<cplx*>(d_g), c->stream));
  return FFBIE_OK;
}

ffbie_status ffbie_assemble(ffbie_ctx* c, void* d_S, int64_t ld) {
  return ffbie_assemble_op(c, FFBIE_OP_S, 0.0, FFBIE_UNKNOWN_SCALED, d_S, ld);
}

ffbie_status ffbie_assemble_op(ffbie_ctx* c, int op, double shift, int unknowns, void* d_S,
                               int64_t ld) {
  if (!c) return FFBIE_EINVAL;
  if (!c->has_problem) return fail(c, FFBIE_ENOPROBLEM, "ffbie_assemble: no problem set");
  const SysDims d = sys_dims(c);
  if (!d_S || ld < d.N) return fail(c, FFBIE_EINVAL, "ffbie_assemble: NULL matrix or ld < N");
  if (op != FFBIE_OP_S && op != FFBIE_OP_K && op != FFBIE_OP_KP)
    return fail(c, FFBIE_EINVAL, "ffbie_assemble_op: op must be FFBIE_OP_S, FFBIE_OP_K or FFBIE_OP_KP");
  if (!std::isfinite(shift)) return fail(c, FFBIE_EINVAL, "ffbie_assemble_op: non-finite shift");
  if (unknowns != FFBIE_UNKNOWN_SCALED && unknowns != FFBIE_UNKNOWN_DENSITY)
    return fail(c, FFBIE_EINVAL, "ffbie_assemble_op: unknowns must be FFBIE_UNKNOWN_SCALED or FFBIE_UNKNOWN_DENSITY");
  const int density = unknowns == FFBIE_UNKNOWN_DENSITY ? 1 : 0;
  ffbie_status s = prepare_system(c);
  if (s != FFBIE_OK) return s;
  cplx* S = static_cast<cplx*>(d_S);
  if (op == FFBIE_OP_S)
    FFBIE_HIP(c, launch_far_assembly(d, c->prob.k, colloc_view(c), S, ld, c->stream, density));
  else
    FFBIE_HIP(c, launch_far_assembly_dl(d, c->prob.k, colloc_view(c), op == FFBIE_OP_KP ? 1 : 0, S, ld,
                                        c->stream, density));
  // near blocks, a chunk of target panels at a time
  const int64_t per_rel = (int64_t)kNodes * 2 * d.M * kNodes;      // pairs of one relation
  const int64_t cap_pairs = kNearKappaBytes / (int64_t)(2 * d.M * sizeof(cplx));
  int64_t max_chunk = 0;
  for (int p0 = 0; p0 < c->n_panels;) {
    int p1 = p0 + 1;
    while (p1 < c->n_panels &&
           (near_relations_before(p1 + 1, d.n_panels) - near_relations_before(p0, d.n_panels)) *
                   per_rel <= cap_pairs)
      ++p1;
    const int64_t np = (near_relations_before(p1, d.n_panels) - near_relations_before(p0, d.n_panels)) *
                       per_rel;
    if (np > max_chunk) max_chunk = np;
    p0 = p1;
  }
  s = ensure_near_ws(c, max_chunk);
  if (s != FFBIE_OK) return s;
  if (!c->d_asm_counts) FFBIE_HIP(c, hipMalloc(&c->d_asm_counts, 2 * sizeof(unsigned long long)));
  FFBIE_HIP(c, launch_zero_counts(c->d_asm_counts, 2, c->stream));
  for (int p0 = 0; p0 < c->n_panels;) {
    int p1 = p0 + 1;
    while (p1 < c->n_panels &&
           (near_relations_before(p1 + 1, d.n_panels) - near_relations_before(p0, d.n_panels)) *
                   per_rel <= cap_pairs)
      ++p1;
    NearChunk ch;
    ch.p0 = p0;
    ch.p1 = p1;
    ch.pair_base = near_pairs_before(p0, d);
    ch.n_pairs = near_pairs_before(p1, d) - ch.pair_base;
    FFBIE_HIP(c, launch_near_pairs(d, ch, c->gl_x, c->d_rule_y, c->d_near_t, c->d_near_az,
                                   c->d_near_ts, c->stream));
    if (op == FFBIE_OP_S)
      s = run_coeffs(c, ch.n_pairs, c->d_near_t, c->d_near_az, c->d_near_ts, c->d_near_kappa, nullptr,
                     nullptr, nullptr);
    else
      s = run_dl_coeffs(c, ch.n_pairs, c->d_near_t, c->d_near_az, c->d_near_ts, op == FFBIE_OP_KP ? 1 : 0,
                        c->d_near_kappa, nullptr, nullptr);
    if (s != FFBIE_OK) return s;
    // the pairs' flags are in the context's status workspace
    FFBIE_HIP(c, launch_count_status(c->d_status, ch.n_pairs, c->d_asm_counts, c->stream));
    FFBIE_HIP(c, launch_near_assembly(d, ch, c->d_near_kappa, c->d_wl, c->d_tab, S, ld, c->stream,
                                      density ? colloc_view(c).jac : nullptr));
    p0 = p1;
  }
  if (shift != 0.0) FFBIE_HIP(c, launch_diag_shift(d, shift, colloc_view(c), S, ld, c->stream, density));
  unsigned long long cnt[2] = {0, 0};
  FFBIE_HIP(c, hipMemcpyAsync(cnt, c->d_asm_counts, sizeof(cnt), hipMemcpyDeviceToHost, c->stream));
  FFBIE_HIP(c, hipStreamSynchronize(c->stream));
  c->asm_pairs = near_pairs_before(c->n_panels, d);
  c->asm_unresolved = (int64_t)cnt[0];
  c->asm_fallback = (int64_t)cnt[1];
  if (cnt[0] > 0) {
    char msg[160];
    std::snprintf(msg, sizeof msg,
                  "ffbie_assemble: %llu of %lld near pairs not resolved by 4M azimuthal samples "
                  "(k too large for M)", cnt[0], (long long)c->asm_pairs);
    c->err = msg;
    return FFBIE_WUNRESOLVED;
  }
  return FFBIE_OK;
}

ffbie_status ffbie_assembly_report(ffbie_ctx* c, int64_t* n_near_pairs, int64_t* n_unresolved,
                                   int64_t* n_root_fallback) {
  if (!c) return FFBIE_EINVAL;
  if (c->asm_pairs < 0) return fail(c, FFBIE_EINVAL, "ffbie_assembly_report: no assembly on this context");
  if (n_near_pairs) *n_near_pairs = c->asm_pairs;
  if (n_unresolved) *n_unresolved = c->asm_unresolved;
  if (n_root_fallback) *n_root_fallback = c->asm_fallback;
  return FFBIE_OK;
}

ffbie_status ffbie_eval_field(ffbie_ctx* c, int64_t n_pts, const double* d_pts, const void* d_phi,
                              void* d_u) {
  return ffbie_eval_field_op(c, FFBIE_OP_S, FFBIE_UNKNOWN_SCALED, n_pts, d_pts, d_phi, d_u);
}

ffbie_status ffbie_eval_field_op(ffbie_ctx* c, int op, int unknowns, int64_t n_pts, const double* d_pts,
                                 const void* d_phi, void* d_u) {
  if (!c) return FFBIE_EINVAL;
  if (op != FFBIE_OP_S && op != FFBIE_OP_K)
    return fail(c, FFBIE_EINVAL, "ffbie_eval_field_op: op must be FFBIE_OP_S or FFBIE_OP_K");
  if (unknowns != FFBIE_UNKNOWN_SCALED && unknowns != FFBIE_UNKNOWN_DENSITY)
    return fail(c, FFBIE_EINVAL, "ffbie_eval_field_op: unknowns must be FFBIE_UNKNOWN_SCALED or FFBIE_UNKNOWN_DENSITY");
  const int density = unknowns == FFBIE_UNKNOWN_DENSITY ? 1 : 0;
  if (!c->has_problem) return fail(c, FFBIE_ENOPROBLEM, "ffbie_eval_field: no problem set");
  if (n_pts < 0 || n_pts > 65535) return fail(c, FFBIE_EINVAL, "ffbie_eval_field: need 0 <= n_pts <= 65535");
  if (n_pts == 0) return FFBIE_OK;
  if (!d_pts || !d_phi || !d_u) return fail(c, FFBIE_EINVAL, "ffbie_eval_field: NULL pointer");
  ffbie_status s = prepare_system(c);
  if (s != FFBIE_OK) return s;
  const SysDims d = sys_dims(c);
  int n_chunks = (int)((2048 + n_pts - 1) / n_pts);
  const int max_chunks = (int)((d.N + 255) / 256);
  if (n_chunks > max_chunks) n_chunks = max_chunks;
  if (n_chunks < 1) n_chunks = 1;
  const int64_t need = n_pts * n_chunks;
  if (need > c->partial_cap) {
    if (c->d_partial) hipFree(c->d_partial);
    c->d_partial = nullptr;
    c->partial_cap = 0;
    if (hipMalloc(&c->d_partial, need * sizeof(cplx)) != hipSuccess)
      return fail(c, FFBIE_ENOMEM, "ffbie_eval_field: workspace allocation failed");
    c->partial_cap = need;
  }
  if (op == FFBIE_OP_S)
    FFBIE_HIP(c, launch_field(d, c->prob.k, colloc_view(c), n_pts, d_pts,
                              static_cast<const cplx*>(d_phi), c->d_partial, n_chunks,
                              static_cast<cplx*>(d_u), c->stream, density));
  else
    FFBIE_HIP(c, launch_field_dl(d, c->prob.k, colloc_view(c), n_pts, d_pts,
                                 static_cast<const cplx*>(d_phi), c->d_partial, n_chunks,
                                 static_cast<cplx*>(d_u), c->stream, density));
  return FFBIE_OK;
}

ffbie_status ffbie_enable_timing(ffbie_ctx* c, int on) {
  if (!c) return FFBIE_EINVAL;
  FFBIE_HIP(c, hipSetDevice(c->device));
  if (on && !c->ev[0])
    for (auto& e : c->ev) FFBIE_HIP(c, hipEventCreate(&e));
  c->timing = on != 0;
  c->timed = false;
  return FFBIE_OK;
}

ffbie_status ffbie_get_timing(ffbie_ctx* c, double* ms_root, double* ms_main, double* ms_refine) {
  if (!c) return FFBIE_EINVAL;
  if (!c->timing || !c->timed) return fail(c, FFBIE_EINVAL, "ffbie_get_timing: no timed call");
  FFBIE_HIP(c, hipEventSynchronize(c->ev[3]));
  float t[3];
  for (int i = 0; i < 3; ++i) FFBIE_HIP(c, hipEventElapsedTime(&t[i], c->ev[i], c->ev[i + 1]));
  if (ms_root) *ms_root = t[0];
  if (ms_main) *ms_main = t[1];
  if (ms_refine) *ms_refine = t[2];
  return FFBIE_OK;
}

ffbie_status ffbie_singular_factor(ffbie_ctx* c, int64_t n, const double* d_b, int m_max,
                                   double* d_A) {
  if (!c) return FFBIE_EINVAL;
  if (n < 0 || m_max < 1 || m_max > 1023)
    return fail(c, FFBIE_EINVAL, "ffbie_singular_factor: need n >= 0 and 1 <= m_max <= 1023");
  if (n == 0) return FFBIE_OK;
  if (!d_b || !d_A) return fail(c, FFBIE_EINVAL, "ffbie_singular_factor: NULL pointer");
  FFBIE_HIP(c, hipSetDevice(c->device));
  const int w = 4;
  const size_t lds = sizeof(double) * (size_t)w * (m_max + 1);
  const int64_t blocks = (n + w - 1) / w;
  hipLaunchKernelGGL(ffbie_singular_factor_kernel, dim3((unsigned)blocks), dim3(64 * w), lds,
                     c->stream, n, d_b, m_max, d_A);
  FFBIE_HIP(c, hipGetLastError());
  return FFBIE_OK;
}

ffbie_status ffbie_set_tuning_cache(ffbie_ctx* c, const char* path) {
  if (!c) return FFBIE_EINVAL;
  c->tune_cache = path ? path : "";
  return FFBIE_OK;
}

ffbie_status ffbie_batch_plan_create(ffbie_ctx* c, int n_items, const ffbie_batch_item* items,
                                     int flags, const ffbie_tuning* tuning, ffbie_batch_plan** out) {
  if (!c) return FFBIE_EINVAL;
  if (!out) return fail(c, FFBIE_EINVAL, "ffbie_batch_plan_create: NULL out");
  *out = nullptr;
  if (flags & ~(FFBIE_PLAN_GRAPH | FFBIE_PLAN_AUTOTUNE | FFBIE_PLAN_MIXED))
    return fail(c, FFBIE_EINVAL, "ffbie_batch_plan_create: unknown flag");
  ffbie_tuning t[kMaxClasses];
  for (int q = 0; q < kMaxClasses; ++q) {
    t[q] = tuning ? tuning[q] : c->tune;
    std::string why;
    if (!valid_tuning(t[q], &why)) return fail(c, FFBIE_EINVAL, "ffbie_batch_plan_create: " + why);
  }
  FFBIE_HIP(c, hipSetDevice(c->device));
  ffbie_batch_plan* pl = new ffbie_batch_plan();
  pl->ctx = c;
  pl->flags = flags;
  pl->single = (flags & FFBIE_PLAN_MIXED) != 0;
  ffbie_status st = plan_build(c, pl, n_items, items, t);
  if (st == FFBIE_OK && pl->np > 0 && (flags & FFBIE_PLAN_AUTOTUNE)) st = plan_autotune(c, pl);
  if (st == FFBIE_OK && pl->np > 0 && (flags & FFBIE_PLAN_GRAPH)) st = plan_capture(c, pl);
  if (st != FFBIE_OK) {
    plan_free(pl);
    return st;
  }
  *out = pl;
  return FFBIE_OK;
}

ffbie_status ffbie_batch_plan_execute(ffbie_ctx* c, ffbie_batch_plan* pl) {
  if (!c) return FFBIE_EINVAL;
  if (!pl || pl->ctx != c) return fail(c, FFBIE_EINVAL, "ffbie_batch_plan_execute: plan of another context");
  if (pl->np == 0) return FFBIE_OK;
  FFBIE_HIP(c, hipSetDevice(c->device));
  if (pl->exec) {
    FFBIE_HIP(c, hipGraphLaunch(pl->exec, c->stream));
    return FFBIE_OK;
  }
  return plan_launch(c, pl, c->stream, c->timing);
}

ffbie_status ffbie_batch_plan_get_tuning(const ffbie_batch_plan* pl, int m_class, ffbie_tuning* t,
                                         double* tuned_ms, int* M) {
  if (!pl || m_class < 0 || m_class >= (int)pl->cls.size()) return FFBIE_EINVAL;
  const PlanClass& q = pl->cls[m_class];
  if (t) *t = q.tune;
  if (tuned_ms) *tuned_ms = q.tuned_ms;
  if (M) *M = q.M;
  return FFBIE_OK;
}

int ffbie_batch_plan_classes(const ffbie_batch_plan* pl) { return pl ? (int)pl->cls.size() : 0; }

ffbie_status ffbie_batch_plan_destroy(ffbie_batch_plan* pl) {
  if (!pl) return FFBIE_OK;
  hipSetDevice(pl->ctx->device);
  (void)hipStreamSynchronize(pl->ctx->stream);
  plan_free(pl);
  return FFBIE_OK;
}

ffbie_status ffbie_kernel_coeffs_batched(ffbie_ctx* c, int n_items, const ffbie_batch_item* items) {
  if (!c) return FFBIE_EINVAL;
  FFBIE_HIP(c, hipSetDevice(c->device));
  if (c->oneshot) {                    // the previous call's plan: its kernels may still run
    FFBIE_HIP(c, hipStreamSynchronize(c->stream));
    plan_free(c->oneshot);
    c->oneshot = nullptr;
  }
  ffbie_batch_plan* pl = nullptr;
  ffbie_status st = ffbie_batch_plan_create(c, n_items, items, 0, nullptr, &pl);
  if (st != FFBIE_OK) return st;
  c->oneshot = pl;
  return ffbie_batch_plan_execute(c, pl);
}

ffbie_status ffbie_set_tuning(ffbie_ctx* c, const ffbie_tuning* t) {
  if (!c) return FFBIE_EINVAL;
  if (!t) return fail(c, FFBIE_EINVAL, "ffbie_set_tuning: NULL tuning");
  std::string why;
  if (!valid_tuning(*t, &why)) return fail(c, FFBIE_EINVAL, "ffbie_set_tuning: " + why);
  c->tune = *t;
  return FFBIE_OK;
}

ffbie_status ffbie_get_tuning(const ffbie_ctx* c, ffbie_tuning* t) {
  if (!c || !t) return FFBIE_EINVAL;
  *t = c->tune;
  return FFBIE_OK;
}

}  // extern "C"

namespace {

constexpr int kRestart = 100;

ffbie_status ensure_solve_ws(ffbie_ctx* c, int64_t N, int method) {
  if (c->solve_n != N) {
    for (void* p : {(void*)c->d_ipiv, (void*)c->d_perm, (void*)c->d_info, (void*)c->d_vecs,
                    (void*)c->d_small})
      if (p) hipFree(p);
    c->d_ipiv = nullptr; c->d_perm = nullptr; c->d_info = nullptr; c->d_vecs = nullptr;
    c->d_small = nullptr; c->solve_n = 0;
    if (hipMalloc(&c->d_ipiv, N * sizeof(int64_t)) != hipSuccess ||
        hipMalloc(&c->d_perm, N * sizeof(int64_t)) != hipSuccess ||
        hipMalloc(&c->d_info, sizeof(int)) != hipSuccess ||
        hipMalloc(&c->d_vecs, 3 * N * sizeof(cplx)) != hipSuccess ||
        hipMalloc(&c->d_small, (256 * (kRestart + 1) + kRestart + 1) * sizeof(cplx)) != hipSuccess)
      return fail(c, FFBIE_ENOMEM, "ffbie_solve: workspace allocation failed");
    c->solve_n = N;
  }
  if ((method == FFBIE_SOLVE_LU32_IR64 || method == FFBIE_SOLVE_GMRES_LU32) && c->s32_n != N) {
    if (c->d_s32) hipFree(c->d_s32);
    c->d_s32 = nullptr;
    c->s32_n = 0;
    if (hipMalloc(&c->d_s32, (size_t)N * N * 8) != hipSuccess)
      return fail(c, FFBIE_ENOMEM, "ffbie_solve: complex64 factor allocation failed");
    c->s32_n = N;
  }
  if ((method == FFBIE_SOLVE_FGMRES_MLP || method == FFBIE_SOLVE_GMRES_BLOCKJACOBI ||
       method == FFBIE_SOLVE_GMRES_LU32 || method == FFBIE_SOLVE_FGMRES_BJ_MLP) && c->zbasis_n != N) {
    if (c->d_zbasis) (void)hipFree(c->d_zbasis);
    c->d_zbasis = nullptr;
    c->zbasis_n = 0;
    if (hipMalloc(&c->d_zbasis, (size_t)kRestart * N * sizeof(cplx)) != hipSuccess)
      return fail(c, FFBIE_ENOMEM, "ffbie_solve: flexible basis allocation failed");
    c->zbasis_n = N;
  }
  if ((method == FFBIE_SOLVE_GMRES || method == FFBIE_SOLVE_FGMRES_MLP ||
       method == FFBIE_SOLVE_GMRES_BLOCKJACOBI || method == FFBIE_SOLVE_GMRES_LU32 ||
       method == FFBIE_SOLVE_FGMRES_BJ_MLP) && c->krylov_n != N) {
    if (c->d_krylov) hipFree(c->d_krylov);
    c->d_krylov = nullptr;
    c->krylov_n = 0;
    if (hipMalloc(&c->d_krylov, (size_t)(kRestart + 1) * N * sizeof(cplx)) != hipSuccess)
      return fail(c, FFBIE_ENOMEM, "ffbie_solve: Krylov basis allocation failed");
    c->krylov_n = N;
  }
  return FFBIE_OK;
}

SolveCtx solve_ctx(ffbie_ctx* c) {
  SolveCtx sc;
  sc.stream = c->stream;
  sc.ipiv = c->d_ipiv;
  sc.perm = c->d_perm;
  sc.info = c->d_info;
  sc.vec_tmp = c->d_vecs;
  sc.vec_r = c->d_vecs + c->solve_n;
  sc.vec_d = c->d_vecs + 2 * c->solve_n;
  sc.partial = c->d_small;
  sc.hvec = c->d_small + 256 * (kRestart + 1);
  sc.s32 = c->d_s32;
  sc.krylov = c->d_krylov;
  sc.zbasis = c->d_zbasis;
  return sc;
}

hipError_t bj_apply(void* self, const cplx* v, cplx* z) {
  ffbie_ctx* c = static_cast<ffbie_ctx*>(self);
  return c->bj.apply(v, z, c->stream);
}

hipError_t mlp_apply(void* self, const cplx* v, cplx* z) {
  ffbie_ctx* c = static_cast<ffbie_ctx*>(self);
  return mlp_precondition(c->mlp, v, c->prob.M, 16 * c->n_panels, c->prob.k, z, c->stream);
}

// z = BJ(v) + NN(v): the network corrects the block-Jacobi output (the first
// of the context's solve vectors is its workspace; flexible GMRES uses the
// second)
hipError_t bj_mlp_apply(void* self, const cplx* v, cplx* z) {
  ffbie_ctx* c = static_cast<ffbie_ctx*>(self);
  hipError_t e = c->bj.apply(v, z, c->stream);
  if (e != hipSuccess) return e;
  return mlp_precondition_add(c->mlp, v, c->prob.M, 16 * c->n_panels, c->prob.k, z, c->d_vecs, c->stream);
}

}  // namespace

extern "C" {

ffbie_status ffbie_solve(ffbie_ctx* c, int method, void* d_S, int64_t ld, const void* d_g,
                         void* d_phi, double tol, int max_iter, ffbie_solve_info* info) {
  if (!c) return FFBIE_EINVAL;
  if (!c->has_problem) return fail(c, FFBIE_ENOPROBLEM, "ffbie_solve: no problem set");
  const int64_t N = n_unknowns(c);
  if (!d_S || !d_g || !d_phi || ld < N || d_g == d_phi)
    return fail(c, FFBIE_EINVAL, "ffbie_solve: NULL or aliased buffer, or ld < N");
  if (method != FFBIE_SOLVE_LU64 && method != FFBIE_SOLVE_LU32_IR64 && method != FFBIE_SOLVE_GMRES &&
      method != FFBIE_SOLVE_FGMRES_MLP && method != FFBIE_SOLVE_GMRES_BLOCKJACOBI &&
      method != FFBIE_SOLVE_GMRES_LU32 && method != FFBIE_SOLVE_FGMRES_BJ_MLP)
    return fail(c, FFBIE_EINVAL, "ffbie_solve: unknown method");
  if (method == FFBIE_SOLVE_GMRES_BLOCKJACOBI && 16 * c->n_panels > 512)
    return fail(c, FFBIE_EINVAL, "ffbie_solve: block-Jacobi needs 16 n_panels <= 512");
  if ((method == FFBIE_SOLVE_FGMRES_MLP || method == FFBIE_SOLVE_FGMRES_BJ_MLP) &&
      (!c->mlp.ready || 16 * c->n_panels != Mlp::kNodes))
    return fail(c, FFBIE_EINVAL, "ffbie_solve: the learned preconditioner needs MLP weights and n_panels = 16");
  if (method != FFBIE_SOLVE_LU64 && (!(tol > 0) || max_iter < 1))
    return fail(c, FFBIE_EINVAL, "ffbie_solve: need tol > 0 and max_iter >= 1");
  if (N > 2147483647 / 2) return fail(c, FFBIE_EINVAL, "ffbie_solve: N too large");
  FFBIE_HIP(c, hipSetDevice(c->device));
  ffbie_status s = ensure_solve_ws(c, N, method);
  if (s != FFBIE_OK) return s;
  SolveCtx sc = solve_ctx(c);
  cplx* S = static_cast<cplx*>(d_S);
  const cplx* g = static_cast<const cplx*>(d_g);
  cplx* phi = static_cast<cplx*>(d_phi);
  SolveResult r;
  int iters = 0;
  bool fell_back = false;
  double rel = std::nan("");
  c->factored_n = 0;
  if (method == FFBIE_SOLVE_LU64) {
    FFBIE_HIP(c, hipMemcpyAsync(phi, g, N * sizeof(cplx), hipMemcpyDeviceToDevice, c->stream));
    r = lu64_factor_solve(sc, S, ld, N, phi);
  } else if (method == FFBIE_SOLVE_LU32_IR64) {
    r = lu32_ir64(sc, S, ld, N, g, phi, tol, max_iter, &iters, &rel);
  } else if (method == FFBIE_SOLVE_GMRES) {
    r = gmres64(sc, S, ld, N, g, phi, tol, max_iter, kRestart, &iters, &rel);
  } else if (method == FFBIE_SOLVE_GMRES_LU32) {
    r = gmres_lu32(sc, S, ld, N, g, phi, tol, max_iter, kRestart, &iters, &rel);
  } else if (method == FFBIE_SOLVE_FGMRES_MLP) {
    Precond P{mlp_apply, c};
    r = fgmres64(sc, S, ld, N, g, phi, tol, max_iter, kRestart, P, &iters, &rel, &fell_back);
  } else if (method == FFBIE_SOLVE_FGMRES_BJ_MLP) {
    FFBIE_HIP(c, c->bj.setup(S, ld, c->prob.M, 16 * c->n_panels, c->stream));
    c->bj.ready = true;
    Precond P{bj_mlp_apply, c};
    r = fgmres64(sc, S, ld, N, g, phi, tol, max_iter, kRestart, P, &iters, &rel, &fell_back);
  } else {
    FFBIE_HIP(c, c->bj.setup(S, ld, c->prob.M, 16 * c->n_panels, c->stream));
    c->bj.ready = true;
    Precond P{bj_apply, c};
    r = fgmres64(sc, S, ld, N, g, phi, tol, max_iter, kRestart, P, &iters, &rel, &fell_back);
  }
  if (r.hip != hipSuccess) return hip_fail(c, r.hip, "ffbie_solve");
  FFBIE_HIP(c, hipStreamSynchronize(c->stream));
  if (info) {
    info->iterations = iters;
    info->converged = r.converged ? 1 : 0;
    info->rel_residual = rel;
    info->fell_back = fell_back ? 1 : 0;
  }
  if (r.singular_col != 0) return fail(c, FFBIE_ESINGULAR, "ffbie_solve: exactly zero pivot");
  if (!r.converged) return FFBIE_WNOTCONV;
  return FFBIE_OK;
}

ffbie_status ffbie_lu_factor(ffbie_ctx* c, void* d_S, int64_t ld) {
  if (!c) return FFBIE_EINVAL;
  if (!c->has_problem) return fail(c, FFBIE_ENOPROBLEM, "ffbie_lu_factor: no problem set");
  const int64_t N = n_unknowns(c);
  if (!d_S || ld < N) return fail(c, FFBIE_EINVAL, "ffbie_lu_factor: NULL matrix or ld < N");
  FFBIE_HIP(c, hipSetDevice(c->device));
  ffbie_status s = ensure_solve_ws(c, N, FFBIE_SOLVE_LU64);
  if (s != FFBIE_OK) return s;
  SolveCtx sc = solve_ctx(c);
  // factor with a zero right-hand side (the solve part is then a no-op on it)
  cplx* y = c->d_vecs + 2 * N;
  FFBIE_HIP(c, hipMemsetAsync(y, 0, N * sizeof(cplx), c->stream));
  c->factored_n = 0;
  SolveResult r = lu64_factor_solve(sc, static_cast<cplx*>(d_S), ld, N, y);
  if (r.hip != hipSuccess) return hip_fail(c, r.hip, "ffbie_lu_factor");
  FFBIE_HIP(c, hipStreamSynchronize(c->stream));
  if (r.singular_col != 0) return fail(c, FFBIE_ESINGULAR, "ffbie_lu_factor: exactly zero pivot");
  c->factored_n = N;
  return FFBIE_OK;
}

ffbie_status ffbie_lu_solve(ffbie_ctx* c, const void* d_S, int64_t ld, void* d_x) {
  if (!c) return FFBIE_EINVAL;
  if (!c->has_problem) return fail(c, FFBIE_ENOPROBLEM, "ffbie_lu_solve: no problem set");
  const int64_t N = n_unknowns(c);
  if (!d_S || !d_x || ld < N) return fail(c, FFBIE_EINVAL, "ffbie_lu_solve: NULL buffer or ld < N");
  if (c->factored_n != N || c->solve_n != N)
    return fail(c, FFBIE_EINVAL, "ffbie_lu_solve: no factorisation of this size");
  FFBIE_HIP(c, hipSetDevice(c->device));
  SolveCtx sc = solve_ctx(c);
  SolveResult r = lu64_solve_factored(sc, static_cast<const cplx*>(d_S), ld, N, static_cast<cplx*>(d_x));
  if (r.hip != hipSuccess) return hip_fail(c, r.hip, "ffbie_lu_solve");
  FFBIE_HIP(c, hipStreamSynchronize(c->stream));
  return FFBIE_OK;
}

ffbie_status ffbie_gemm_sub(ffbie_ctx* c, int complex64, int64_t m, int64_t n, int64_t k,
                            const void* d_A, const void* d_B, void* d_C, int64_t ld) {
  if (!c) return FFBIE_EINVAL;
  if (m < 0 || n < 0 || k < 0 || ld < 1 || ld < m || ld < k)
    return fail(c, FFBIE_EINVAL, "ffbie_gemm_sub: negative size or ld < max(m, k)");
  if (m > 2147483647 || n > 2147483647 || k > 2147483647)
    return fail(c, FFBIE_EINVAL, "ffbie_gemm_sub: size above 2^31 - 1");
  if (m == 0 || n == 0 || k == 0) return FFBIE_OK;
  if (!d_A || !d_B || !d_C) return fail(c, FFBIE_EINVAL, "ffbie_gemm_sub: NULL pointer");
  FFBIE_HIP(c, hipSetDevice(c->device));
  if (complex64)
    FFBIE_HIP(c, gemm_sub_c64(c->stream, static_cast<float*>(d_C), static_cast<const float*>(d_A),
                              static_cast<const float*>(d_B), ld, m, n, k));
  else
    FFBIE_HIP(c, gemm_sub_c128(c->stream, static_cast<double*>(d_C), static_cast<const double*>(d_A),
                               static_cast<const double*>(d_B), ld, m, n, k));
  return FFBIE_OK;
}

ffbie_status ffbie_blockjacobi_setup(ffbie_ctx* c, const void* d_S, int64_t ld) {
  if (!c) return FFBIE_EINVAL;
  if (!c->has_problem) return fail(c, FFBIE_ENOPROBLEM, "ffbie_blockjacobi_setup: no problem set");
  const int64_t N = n_unknowns(c);
  if (!d_S || ld < N || 16 * c->n_panels > 512)
    return fail(c, FFBIE_EINVAL, "ffbie_blockjacobi_setup: NULL matrix, ld < N or more than 512 nodes");
  FFBIE_HIP(c, hipSetDevice(c->device));
  FFBIE_HIP(c, c->bj.setup(static_cast<const cplx*>(d_S), ld, c->prob.M, 16 * c->n_panels, c->stream));
  c->bj.ready = true;
  return FFBIE_OK;
}

ffbie_status ffbie_blockjacobi_apply(ffbie_ctx* c, const void* d_v, void* d_z) {
  if (!c) return FFBIE_EINVAL;
  if (!c->has_problem || !c->bj.ready || c->bj.M != c->prob.M || c->bj.nodes != 16 * c->n_panels)
    return fail(c, FFBIE_EINVAL, "ffbie_blockjacobi_apply: no preconditioner for this problem");
  if (!d_v || !d_z) return fail(c, FFBIE_EINVAL, "ffbie_blockjacobi_apply: NULL pointer");
  FFBIE_HIP(c, hipSetDevice(c->device));
  FFBIE_HIP(c, c->bj.apply(static_cast<const cplx*>(d_v), static_cast<cplx*>(d_z), c->stream));
  return FFBIE_OK;
}

ffbie_status ffbie_residual(ffbie_ctx* c, const void* d_S, int64_t ld, const void* d_phi,
                            const void* d_g, void* d_r) {
  if (!c) return FFBIE_EINVAL;
  if (!c->has_problem) return fail(c, FFBIE_ENOPROBLEM, "ffbie_residual: no problem set");
  const int64_t N = n_unknowns(c);
  if (!d_S || !d_g || !d_phi || !d_r || ld < N)
    return fail(c, FFBIE_EINVAL, "ffbie_residual: NULL buffer or ld < N");
  FFBIE_HIP(c, hipSetDevice(c->device));
  SolveCtx sc{};
  sc.stream = c->stream;
  FFBIE_HIP(c, residual64(sc, static_cast<const cplx*>(d_S), ld, N, static_cast<const cplx*>(d_phi),
                          static_cast<const cplx*>(d_g), static_cast<cplx*>(d_r)));
  return FFBIE_OK;
}

int64_t ffbie_mlp_param_count(void) { return (int64_t)Mlp::param_count(); }

ffbie_status ffbie_mlp_init(ffbie_ctx* c, uint64_t seed) {
  if (!c) return FFBIE_EINVAL;
  const size_t P = Mlp::param_count();
  std::vector<float> w(P, 0.f);
  uint64_t st = seed;
  auto uni = [&st]() {                       // SplitMix64 -> [0, 1)
    uint64_t z = (st += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    z ^= z >> 31;
    return (double)(z >> 11) * (1.0 / 9007199254740992.0);
  };
  auto fill = [&](size_t off, int rows, int cols, double a) {
    for (size_t i = 0; i < (size_t)rows * cols; ++i) w[off + i] = (float)(a * (2.0 * uni() - 1.0));
  };
  fill(Mlp::off_W1(), Mlp::kH, Mlp::kIn, std::sqrt(6.0 / Mlp::kIn));
  fill(Mlp::off_W2(), Mlp::kH, Mlp::kH, std::sqrt(6.0 / Mlp::kH));
  fill(Mlp::off_W3(), Mlp::kOut, Mlp::kH, std::sqrt(6.0 / (Mlp::kH + Mlp::kOut)));
  return ffbie_mlp_set_params(c, w.data());
}

ffbie_status ffbie_mlp_set_params(ffbie_ctx* c, const float* params) {
  if (!c) return FFBIE_EINVAL;
  if (!params) return fail(c, FFBIE_EINVAL, "ffbie_mlp_set_params: NULL params");
  const size_t P = Mlp::param_count();
  for (size_t i = 0; i < P; ++i)
    if (!std::isfinite(params[i])) return fail(c, FFBIE_EINVAL, "ffbie_mlp_set_params: non-finite value");
  FFBIE_HIP(c, hipSetDevice(c->device));
  FFBIE_HIP(c, c->mlp.alloc());
  FFBIE_HIP(c, hipMemcpyAsync(c->mlp.params, params, P * sizeof(float), hipMemcpyHostToDevice, c->stream));
  FFBIE_HIP(c, hipMemsetAsync(c->mlp.m1, 0, P * sizeof(float), c->stream));
  FFBIE_HIP(c, hipMemsetAsync(c->mlp.m2, 0, P * sizeof(float), c->stream));
  FFBIE_HIP(c, c->mlp.refresh_bf16(c->stream));
  FFBIE_HIP(c, hipStreamSynchronize(c->stream));
  c->mlp.step = 0;
  c->mlp.ready = true;
  return FFBIE_OK;
}

ffbie_status ffbie_mlp_get_params(ffbie_ctx* c, float* params) {
  if (!c) return FFBIE_EINVAL;
  if (!params || !c->mlp.ready) return fail(c, FFBIE_EINVAL, "ffbie_mlp_get_params: no weights");
  FFBIE_HIP(c, hipSetDevice(c->device));
  FFBIE_HIP(c, hipMemcpyAsync(params, c->mlp.params, Mlp::param_count() * sizeof(float),
                              hipMemcpyDeviceToHost, c->stream));
  FFBIE_HIP(c, hipStreamSynchronize(c->stream));
  return FFBIE_OK;
}

ffbie_status ffbie_mlp_forward(ffbie_ctx* c, int64_t n, const float* d_x, float* d_y) {
  if (!c) return FFBIE_EINVAL;
  if (!c->mlp.ready) return fail(c, FFBIE_EINVAL, "ffbie_mlp_forward: no weights");
  if (n < 0 || n > (1 << 24)) return fail(c, FFBIE_EINVAL, "ffbie_mlp_forward: n out of range");
  if (n == 0) return FFBIE_OK;
  if (!d_x || !d_y) return fail(c, FFBIE_EINVAL, "ffbie_mlp_forward: NULL pointer");
  FFBIE_HIP(c, hipSetDevice(c->device));
  FFBIE_HIP(c, c->mlp.ensure_batch(n));
  FFBIE_HIP(c, c->mlp.inputs_bf16(d_x, n, c->stream));
  FFBIE_HIP(c, c->mlp.forward(n, c->stream));
  FFBIE_HIP(c, hipMemcpyAsync(d_y, c->mlp.y, n * Mlp::kOut * sizeof(float), hipMemcpyDeviceToDevice,
                              c->stream));
  return FFBIE_OK;
}

ffbie_status ffbie_mlp_train_step(ffbie_ctx* c, int64_t n, const float* d_x, const float* d_t,
                                  float lr, int update, float* d_grads, double* loss) {
  if (!c) return FFBIE_EINVAL;
  if (!c->mlp.ready) return fail(c, FFBIE_EINVAL, "ffbie_mlp_train_step: no weights");
  if (n < 1 || n > (1 << 24)) return fail(c, FFBIE_EINVAL, "ffbie_mlp_train_step: n out of range");
  if (!d_x || !d_t) return fail(c, FFBIE_EINVAL, "ffbie_mlp_train_step: NULL pointer");
  if (update && !(lr > 0)) return fail(c, FFBIE_EINVAL, "ffbie_mlp_train_step: need lr > 0");
  FFBIE_HIP(c, hipSetDevice(c->device));
  Mlp& net = c->mlp;
  FFBIE_HIP(c, net.ensure_batch(n));
  FFBIE_HIP(c, net.inputs_bf16(d_x, n, c->stream));
  FFBIE_HIP(c, net.forward(n, c->stream));
  int nblk = 0;
  FFBIE_HIP(c, net.backward(n, d_t, c->stream, &nblk));
  if (d_grads)
    FFBIE_HIP(c, hipMemcpyAsync(d_grads, net.grads, Mlp::param_count() * sizeof(float),
                                hipMemcpyDeviceToDevice, c->stream));
  std::vector<double> part(nblk);
  FFBIE_HIP(c, hipMemcpyAsync(part.data(), net.partial, nblk * sizeof(double), hipMemcpyDeviceToHost,
                              c->stream));
  if (update) FFBIE_HIP(c, net.adam(lr, c->stream));
  FFBIE_HIP(c, hipStreamSynchronize(c->stream));
  if (loss) {
    double sum = 0;
    for (double v : part) sum += v;
    *loss = sum / (2.0 * n);
  }
  return FFBIE_OK;
}

ffbie_status ffbie_mlp_train(ffbie_ctx* c, const ffbie_train_cfg* cfg, ffbie_train_info* info) {
  if (!c) return FFBIE_EINVAL;
  if (!c->mlp.ready) return fail(c, FFBIE_EINVAL, "ffbie_mlp_train: no weights (ffbie_mlp_init first)");
  if (!cfg || !cfg->d_x || !cfg->d_t) return fail(c, FFBIE_EINVAL, "ffbie_mlp_train: NULL config or data");
  if (cfg->n_samples < 1 || cfg->n_samples > 2147483647 || cfg->steps < 1 || cfg->batch < 1 ||
      cfg->batch > 65535 || cfg->batch > cfg->n_samples || !(cfg->lr > 0))
    return fail(c, FFBIE_EINVAL,
                "ffbie_mlp_train: need n_samples >= batch >= 1, batch <= 65535, steps >= 1, lr > 0");
  FFBIE_HIP(c, hipSetDevice(c->device));
  Mlp& net = c->mlp;
  const int64_t n = cfg->n_samples;
  const int B = cfg->batch;
  FFBIE_HIP(c, net.ensure_batch(std::max<int64_t>(B, std::min<int64_t>(n, 16384))));
  if (c->train_idx_cap < n) {
    if (c->d_train_idx) (void)hipFree(c->d_train_idx);
    c->d_train_idx = nullptr;
    c->train_idx_cap = 0;
    if (hipMalloc(&c->d_train_idx, n * sizeof(int32_t)) != hipSuccess)
      return fail(c, FFBIE_ENOMEM, "ffbie_mlp_train: index workspace allocation failed");
    c->train_idx_cap = n;
  }
  // minibatches drawn without replacement: a Fisher-Yates permutation of the
  // samples per epoch (SplitMix64 stream from cfg->seed)
  uint64_t st = cfg->seed;
  auto next = [&st]() {
    uint64_t z = (st += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
  };
  std::vector<int32_t> perm(n);
  auto shuffle = [&]() {
    for (int64_t i = 0; i < n; ++i) perm[i] = (int32_t)i;
    for (int64_t i = n - 1; i > 0; --i) std::swap(perm[i], perm[next() % (uint64_t)(i + 1)]);
  };
  auto read_loss = [&](int nblk, int64_t rows, double* out) -> hipError_t {
    std::vector<double> part(nblk);
    hipError_t e = hipMemcpyAsync(part.data(), net.partial, nblk * sizeof(double), hipMemcpyDeviceToHost,
                                  c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    double sum = 0;
    for (double v : part) sum += v;
    *out = sum / (2.0 * rows);
    return e;
  };
  int64_t pos = n;
  double first = 0, last = 0;
  for (int step = 0; step < cfg->steps; ++step) {
    if (pos + B > n) {
      shuffle();
      FFBIE_HIP(c, hipMemcpyAsync(c->d_train_idx, perm.data(), n * sizeof(int32_t), hipMemcpyHostToDevice,
                                  c->stream));
      FFBIE_HIP(c, hipStreamSynchronize(c->stream));    // perm is rewritten on the host next epoch
      pos = 0;
    }
    FFBIE_HIP(c, net.gather_batch(cfg->d_x, cfg->d_t, c->d_train_idx + pos, B, c->stream));
    pos += B;
    FFBIE_HIP(c, net.forward(B, c->stream));
    int nblk = 0;
    FFBIE_HIP(c, net.backward(B, net.tg, c->stream, &nblk));
    if (step == 0) FFBIE_HIP(c, read_loss(nblk, B, &first));
    if (step == cfg->steps - 1) FFBIE_HIP(c, read_loss(nblk, B, &last));
    const double lr = 0.5 * cfg->lr * (1.0 + std::cos(M_PI * step / cfg->steps));   // cosine decay
    FFBIE_HIP(c, net.adam((float)lr, c->stream));
  }
  // loss over the whole training set with the trained weights (chunks of the
  // batch workspace; the gradients computed on the way are not used)
  double full = 0;
  {
    std::vector<int32_t> ident(n);
    for (int64_t i = 0; i < n; ++i) ident[i] = (int32_t)i;
    FFBIE_HIP(c, hipMemcpyAsync(c->d_train_idx, ident.data(), n * sizeof(int32_t), hipMemcpyHostToDevice,
                                c->stream));
    const int64_t chunk = std::min<int64_t>(net.cap, 16384);
    for (int64_t a = 0; a < n; a += chunk) {
      const int64_t rows = std::min<int64_t>(chunk, n - a);
      FFBIE_HIP(c, net.gather_batch(cfg->d_x, cfg->d_t, c->d_train_idx + a, rows, c->stream));
      FFBIE_HIP(c, net.forward(rows, c->stream));
      int nblk = 0;
      FFBIE_HIP(c, net.backward(rows, net.tg, c->stream, &nblk));
      double l = 0;
      FFBIE_HIP(c, read_loss(nblk, rows, &l));
      full += l * rows;
    }
    full /= (double)n;
  }
  if (info) {
    info->loss_first = first;
    info->loss_last = last;
    info->loss_full = full;
    info->steps = cfg->steps;
  }
  return FFBIE_OK;
}

// Checkpoint: "FFBIEMLP" magic, format version 1, parameter count, Adam step,
// then the float32 parameters, first and second Adam moments (little endian).
namespace {
constexpr char kMlpMagic[8] = {'F', 'F', 'B', 'I', 'E', 'M', 'L', 'P'};
constexpr int32_t kMlpVersion = 1;
}  // namespace

ffbie_status ffbie_mlp_save(ffbie_ctx* c, const char* path) {
  if (!c) return FFBIE_EINVAL;
  if (!path) return fail(c, FFBIE_EINVAL, "ffbie_mlp_save: NULL path");
  if (!c->mlp.ready) return fail(c, FFBIE_EINVAL, "ffbie_mlp_save: no weights");
  FFBIE_HIP(c, hipSetDevice(c->device));
  const size_t P = Mlp::param_count();
  std::vector<float> buf(3 * P);
  FFBIE_HIP(c, hipMemcpyAsync(buf.data(), c->mlp.params, P * sizeof(float), hipMemcpyDeviceToHost, c->stream));
  FFBIE_HIP(c, hipMemcpyAsync(buf.data() + P, c->mlp.m1, P * sizeof(float), hipMemcpyDeviceToHost, c->stream));
  FFBIE_HIP(c, hipMemcpyAsync(buf.data() + 2 * P, c->mlp.m2, P * sizeof(float), hipMemcpyDeviceToHost,
                              c->stream));
  FFBIE_HIP(c, hipStreamSynchronize(c->stream));
  FILE* f = std::fopen(path, "wb");
  if (!f) return fail(c, FFBIE_EINVAL, std::string("ffbie_mlp_save: cannot open ") + path);
  const int64_t count = (int64_t)P, step = c->mlp.step;
  bool ok = std::fwrite(kMlpMagic, 1, 8, f) == 8 && std::fwrite(&kMlpVersion, 4, 1, f) == 1 &&
            std::fwrite(&count, 8, 1, f) == 1 && std::fwrite(&step, 8, 1, f) == 1 &&
            std::fwrite(buf.data(), sizeof(float), buf.size(), f) == buf.size();
  ok = (std::fclose(f) == 0) && ok;
  if (!ok) return fail(c, FFBIE_EINVAL, std::string("ffbie_mlp_save: write failed: ") + path);
  return FFBIE_OK;
}

ffbie_status ffbie_mlp_load(ffbie_ctx* c, const char* path) {
  if (!c) return FFBIE_EINVAL;
  if (!path) return fail(c, FFBIE_EINVAL, "ffbie_mlp_load: NULL path");
  FILE* f = std::fopen(path, "rb");
  if (!f) return fail(c, FFBIE_EINVAL, std::string("ffbie_mlp_load: cannot open ") + path);
  const size_t P = Mlp::param_count();
  char magic[8];
  int32_t ver = 0;
  int64_t count = 0, step = 0;
  std::vector<float> buf(3 * P);
  bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, kMlpMagic, 8) == 0 &&
            std::fread(&ver, 4, 1, f) == 1 && ver == kMlpVersion && std::fread(&count, 8, 1, f) == 1 &&
            count == (int64_t)P && std::fread(&step, 8, 1, f) == 1 && step >= 0 &&
            std::fread(buf.data(), sizeof(float), buf.size(), f) == buf.size();
  std::fclose(f);
  if (!ok) return fail(c, FFBIE_EINVAL, std::string("ffbie_mlp_load: not a network checkpoint of this size: ") + path);
  for (size_t i = 0; i < P; ++i)
    if (!std::isfinite(buf[i])) return fail(c, FFBIE_EINVAL, "ffbie_mlp_load: non-finite parameter");
  FFBIE_HIP(c, hipSetDevice(c->device));
  FFBIE_HIP(c, c->mlp.alloc());
  FFBIE_HIP(c, hipMemcpyAsync(c->mlp.params, buf.data(), P * sizeof(float), hipMemcpyHostToDevice, c->stream));
  FFBIE_HIP(c, hipMemcpyAsync(c->mlp.m1, buf.data() + P, P * sizeof(float), hipMemcpyHostToDevice, c->stream));
  FFBIE_HIP(c, hipMemcpyAsync(c->mlp.m2, buf.data() + 2 * P, P * sizeof(float), hipMemcpyHostToDevice,
                              c->stream));
  FFBIE_HIP(c, c->mlp.refresh_bf16(c->stream));
  FFBIE_HIP(c, hipStreamSynchronize(c->stream));
  c->mlp.step = (int)step;
  c->mlp.ready = true;
  return FFBIE_OK;
}

ffbie_status ffbie_mode_features(ffbie_ctx* c, const void* d_r, float* d_x, double* d_scale) {
  if (!c) return FFBIE_EINVAL;
  if (!c->has_problem || 16 * c->n_panels != Mlp::kNodes)
    return fail(c, FFBIE_EINVAL, "ffbie_mode_features: needs a problem with n_panels = 16");
  if (!d_r || !d_x || !d_scale) return fail(c, FFBIE_EINVAL, "ffbie_mode_features: NULL pointer");
  FFBIE_HIP(c, hipSetDevice(c->device));
  FFBIE_HIP(c, mode_features(c->mlp, static_cast<const cplx*>(d_r), c->prob.M, Mlp::kNodes, c->prob.k,
                             d_x, d_scale, c->stream));
  return FFBIE_OK;
}

ffbie_status ffbie_mode_targets(ffbie_ctx* c, const void* d_e, const double* d_scale, float* d_t) {
  if (!c) return FFBIE_EINVAL;
  if (!c->has_problem || 16 * c->n_panels != Mlp::kNodes)
    return fail(c, FFBIE_EINVAL, "ffbie_mode_targets: needs a problem with n_panels = 16");
  if (!d_e || !d_t || !d_scale) return fail(c, FFBIE_EINVAL, "ffbie_mode_targets: NULL pointer");
  FFBIE_HIP(c, hipSetDevice(c->device));
  FFBIE_HIP(c, mode_targets(c->mlp, static_cast<const cplx*>(d_e), d_scale, c->prob.M, Mlp::kNodes,
                            d_t, c->stream));
  return FFBIE_OK;
}

ffbie_status ffbie_mlp_precondition(ffbie_ctx* c, const void* d_v, void* d_z) {
  if (!c) return FFBIE_EINVAL;
  if (!c->mlp.ready || !c->has_problem || 16 * c->n_panels != Mlp::kNodes)
    return fail(c, FFBIE_EINVAL, "ffbie_mlp_precondition: needs weights and n_panels = 16");
  if (!d_v || !d_z) return fail(c, FFBIE_EINVAL, "ffbie_mlp_precondition: NULL pointer");
  FFBIE_HIP(c, hipSetDevice(c->device));
  FFBIE_HIP(c, mlp_precondition(c->mlp, static_cast<const cplx*>(d_v), c->prob.M, Mlp::kNodes,
                                c->prob.k, static_cast<cplx*>(d_z), c->stream));
  return FFBIE_OK;
}

}  // extern "C"
