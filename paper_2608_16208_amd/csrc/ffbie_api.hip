// Host side of the C ABI declared in include/ffbie.h: context, validation,
// exact angle tables, workspaces and kernel launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "ffbie.h"
#include "ffbie_device.hpp"

#include "ffbie_kernels.hpp"

using namespace ffbie;

struct ffbie_ctx {
  int device = 0;
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
};

namespace {

const char* kNoCtx = "ffbie: NULL context";

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
int coeff_waves(const Prob& P, int NF, bool compact, size_t* lds_bytes) {
  const size_t per_wave = sizeof(double) * coeff_lds_per_wave(NF, P.M, P.L, compact);
  const size_t tab = sizeof(double) * P.tab_n;
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
  c->device = device;
  c->stream = static_cast<hipStream_t>(hip_stream);
  if (hipSetDevice(device) != hipSuccess) { delete c; return FFBIE_EDEVICE; }
  if (hipMalloc(&c->d_count, 4 * sizeof(int32_t)) != hipSuccess) { delete c; return FFBIE_ENOMEM; }
  *out = c;
  return FFBIE_OK;
}

ffbie_status ffbie_destroy(ffbie_ctx* c) {
  if (!c) return FFBIE_OK;
  hipSetDevice(c->device);
  for (auto& e : c->ev)
    if (e) hipEventDestroy(e);
  if (c->d_tab) hipFree(c->d_tab);
  if (c->d_roots) hipFree(c->d_roots);
  if (c->d_status) hipFree(c->d_status);
  if (c->d_list) hipFree(c->d_list);
  if (c->d_count) hipFree(c->d_count);
  delete c;
  return FFBIE_OK;
}

const char* ffbie_last_error(const ffbie_ctx* c) { return c ? c->err.c_str() : kNoCtx; }

ffbie_status ffbie_set_problem(ffbie_ctx* c, const ffbie_geometry* g, const ffbie_discretization* d,
                               double k) {
  if (!c) return FFBIE_EINVAL;
  if (!g || !d) return fail(c, FFBIE_EINVAL, "ffbie_set_problem: NULL geometry or discretisation");
  if (g->lmax < 0 || g->lmax > kMaxL || g->mmax < 0 || g->mmax > kMaxM || (g->lmax > 0 && !g->a))
    return fail(c, FFBIE_EINVAL, "ffbie_set_problem: amplitude table must have lmax <= 8, mmax <= 8");
  if (!valid_M(d->M)) return fail(c, FFBIE_EINVAL, "ffbie_set_problem: M must be 16, 32, 64 or 128");
  if (d->M0 < 1 || d->M0 > d->M) return fail(c, FFBIE_EINVAL, "ffbie_set_problem: need 1 <= M0 <= M");
  if (d->n_panels < 1) return fail(c, FFBIE_EINVAL, "ffbie_set_problem: n_panels must be >= 1");
  if (!(k >= 0) || !std::isfinite(k)) return fail(c, FFBIE_EINVAL, "ffbie_set_problem: need k >= 0");
  if (!(d->eps0 >= 0) || d->eps0 >= 1) return fail(c, FFBIE_EINVAL, "ffbie_set_problem: need 0 <= eps0 < 1");
  if (d->kappa_variant != FFBIE_KAPPA_SWAP && d->kappa_variant != FFBIE_KAPPA_PAPER_CONV)
    return fail(c, FFBIE_EINVAL, "ffbie_set_problem: unknown kappa_variant");
  Prob P{};
  P.g.lmax = g->lmax;
  P.g.mmax = g->mmax;
  for (int l = 0; l < g->lmax; ++l)
    for (int m = 0; m <= g->mmax; ++m) {
      const double v = g->a[l * (g->mmax + 1) + m];
      if (!std::isfinite(v)) return fail(c, FFBIE_EINVAL, "ffbie_set_problem: non-finite amplitude");
      P.g.a[l][m] = v;
    }
  P.k = k;
  P.eps0 = d->eps0 > 0 ? d->eps0 : 1e-15;
  P.M = d->M;
  P.M0 = d->M0;
  P.L = d->M + d->M0;
  P.tab_n = 8 * d->M;
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
  return FFBIE_OK;
}

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
  ffbie_status s = ensure_ws(c, n);
  if (s != FFBIE_OK) return s;
  const Prob& P = c->prob;
  int32_t* status = d_pair_status ? d_pair_status : c->d_status;

  if (c->timing) FFBIE_HIP(c, hipEventRecord(c->ev[0], c->stream));
  // kernel 1: roots, one lane per pair
  FFBIE_HIP(c, launch_root(P, c->d_tab, n, d_t, d_az, d_ts, c->d_roots, status, d_root, c->stream));
  FFBIE_HIP(c, hipMemsetAsync(c->d_count, 0, sizeof(int32_t), c->stream));
  // kernel 2: main pass with 2M samples, then the refine pass with 4M samples
  CoeffArgs a{};
  a.P = P;
  a.tab_g = c->d_tab;
  a.n = n;
  a.t_in = d_t;
  a.az_in = d_az;
  a.ts_in = d_ts;
  a.roots = c->d_roots;
  a.status = status;
  a.kappa = static_cast<cplx*>(d_kappa);
  a.rhoinv = static_cast<cplx*>(d_rhoinv);
  a.variant = c->variant;
  const bool compact = c->variant == FFBIE_KAPPA_SWAP && d_rhoinv == nullptr;
  {
    a.NF = 2 * P.M;
    a.flag_list = c->d_list;
    a.flag_count = c->d_count;
    size_t lds;
    const int w = coeff_waves(P, a.NF, compact, &lds);
    const int64_t pairs_per_wave = 16;
    int64_t blocks = (n + w * pairs_per_wave - 1) / (w * pairs_per_wave);
    if (blocks < 1) blocks = 1;
    if (c->timing) FFBIE_HIP(c, hipEventRecord(c->ev[1], c->stream));
    FFBIE_HIP(c, launch_coeff(a, blocks, w, lds, c->stream, false));
    if (c->timing) FFBIE_HIP(c, hipEventRecord(c->ev[2], c->stream));
  }
  {
    a.NF = 4 * P.M;
    a.list = c->d_list;
    a.list_count = c->d_count;
    a.flag_list = nullptr;
    a.flag_count = nullptr;
    size_t lds;
    const int w = coeff_waves(P, a.NF, compact, &lds);
    FFBIE_HIP(c, launch_coeff(a, 512, w, lds, c->stream, true));
    if (c->timing) FFBIE_HIP(c, hipEventRecord(c->ev[3], c->stream));
  }
  if (c->timing) c->timed = true;
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

}  // extern "C"
