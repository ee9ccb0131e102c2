/*
 * ffbie.h -- C ABI of the MI355X (gfx950) library for the azimuthal Fourier
 * coefficients of the singular 3-D Helmholtz kernels on smooth surfaces.
 *
 * Method: W. Hua, J. Lai, H. Li, W. Lu, "An FFT-accelerated boundary integral
 * equation method for wave scattering by smooth surfaces in three
 * dimensions".  Section and equation numbers below refer to that paper.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every d_* argument is a caller-owned DEVICE pointer (for example the
 *    data_ptr() of a torch tensor on the context's device).  The library never
 *    frees or reallocates it.  Host pointers are copied before the call returns.
 *  - Work is enqueued on the context's HIP stream; calls return before the
 *    device work completes.  The caller synchronises the stream.
 *  - Complex values are interleaved (re, im) float64 pairs, the layout of
 *    torch.complex128.
 *  - Return value: FFBIE_OK (0), an error (< 0) or a warning (> 0).  On an
 *    error nothing is enqueued; ffbie_last_error() describes it.  Per-pair
 *    conditions found on the device are reported through the optional
 *    per-pair status array, never through the return value.
 *  - One context per host thread; a context is not thread safe.
 */
#ifndef FFBIE_H
#define FFBIE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FFBIE_OK = 0,
  FFBIE_EINVAL = -1,         /* invalid argument, shape or unsupported size        */
  FFBIE_ESINGULAR = -2,      /* exactly zero pivot in an LU factorisation            */
  FFBIE_ENOMEM = -4,         /* device allocation of a workspace failed             */
  FFBIE_EDEVICE = -5,        /* a HIP runtime call failed                           */
  FFBIE_ENOPROBLEM = -7,     /* ffbie_set_problem has not been called               */
  FFBIE_WNOTCONV = 2,        /* warning: an iterative solve stopped at max_iter     */
  FFBIE_WUNRESOLVED = 3      /* warning: ffbie_assemble used near pairs whose smooth
                                factor 4M azimuthal samples did not resolve (see
                                ffbie_assembly_report)                              */
} ffbie_status;

/* Per-pair status bits written to d_pair_status by ffbie_kernel_coeffs. */
enum {
  FFBIE_PAIR_OK = 0,
  FFBIE_PAIR_SINGULAR = 1,        /* t == t_s: the coefficients diverge (b = 0); row is NaN */
  FFBIE_PAIR_ROOT_FALLBACK = 2,   /* complex Newton did not converge; the quadratic-model
                                     root estimate was used (accuracy is then governed by
                                     the smooth-factor truncation test)                    */
  FFBIE_PAIR_REFINED = 4,         /* smooth factor not resolved by 2M samples; recomputed
                                     with 4M samples                                        */
  FFBIE_PAIR_UNRESOLVED = 8,      /* smooth factor not resolved even by 4M samples          */
  FFBIE_PAIR_FAR = 16,            /* b0 >= 3: the quadratic-model estimate (a0, b0), not a
                                     Newton-refined root, parametrises the swap             */
  FFBIE_PAIR_NOT_PD = 32          /* ffbie_rhoinv_banded: a pivot of the banded system's
                                     L D L^H factorisation was not positive (the system is
                                     Hermitian but not positive definite for this pair; the
                                     sufficient condition of Lemma 3.4 does not hold)       */
};
/* Bits 8..19 of a pair's status word hold the truncation index p (eq. (3.24))
 * of the smooth factor used for its kernel coefficients: (status >> 8) & 0xfff. */
#define FFBIE_PAIR_P_SHIFT 8

/* How the kernel coefficients <e^{ik rho}/rho>_n are formed from the swap. */
enum {
  FFBIE_KAPPA_SWAP = 0,        /* default: the singularity swap of Sec. 3.3 applied to the
                                  whole singular part, cos(k rho)/rho = [F cos(k rho)] s_{a,b}^{-1/2}
                                  (cos(k rho) is analytic in rho^2), one convolution with A_m(b);
                                  the construction the paper uses for tau_3 in eqs. (4.5)-(4.6) */
  FFBIE_KAPPA_PAPER_CONV = 1   /* eq. (3.10): <cos(k rho)>_n (|n| < M0) convolved with the
                                  swapped <rho^-1>_l of eq. (3.25) */
};

typedef struct ffbie_ctx ffbie_ctx;

/* Surface of the star family, a radial perturbation of the unit sphere in the
 * parametrisation of Sec. 2, eq. (2.1), with t in [0, pi] (polar angle) and
 * theta the azimuth, optionally stretched along the coordinate axes:
 *   r(t, theta) = D R(t, theta) (sin t cos theta, sin t sin theta, cos t),
 *   R(t, theta) = 1 + sum_{l=1..lmax} sum_{m=0..mmax} a[(l-1)(mmax+1) + m] sin(l t) cos(m theta),
 *   D = diag(axes[0], axes[1], axes[2]).
 * lmax = 0 gives the unit sphere; lmax = 0 with axes (1, 2, 3) the ellipsoid
 * x^2 + y^2/4 + z^2/9 = 1 of Sec. 5, Example 1.  `a` and `axes` are HOST
 * pointers copied by ffbie_set_problem; `a` is row-major [lmax][mmax+1];
 * axes NULL means (1, 1, 1), otherwise three positive finite values.  Limits:
 * lmax <= 8, mmax <= 8.  Stretched surfaces run the FP64 single-problem paths
 * (ffbie_kernel_coeffs, _noalloc, ffbie_kernel_coeffs_dl, the S, K and K'
 * operators of the assembly, the solvers and the fields); the mixed-precision
 * path, the batch plans and ffbie_rhoinv_banded take unstretched surfaces only
 * (FFBIE_EINVAL otherwise). */
typedef struct {
  int lmax;
  int mmax;
  const double *a;
  const double *axes;
} ffbie_geometry;

/* Discretisation (Sec. 3.1-3.2): n_panels Gauss-Legendre panels of 16 nodes
 * in t, 2M equispaced azimuths theta_j = pi j / M (eq. (3.8)), M0 modes of
 * cos(k rho) in eq. (3.10) (0 < M0 <= M; the paper uses M0 = M), eps0 the
 * truncation threshold of eq. (3.13) applied to the smooth factor of eq. (3.24)
 * (0 selects 1e-15), kappa_variant one of FFBIE_KAPPA_*.  Supported M: 16, 32,
 * 64, 128. */
typedef struct {
  int n_panels;
  int M;
  int M0;
  double eps0;
  int kappa_variant;   /* FFBIE_KAPPA_SWAP (default) or FFBIE_KAPPA_PAPER_CONV */
} ffbie_discretization;

/* Create a context on HIP device `device`, enqueuing on `hip_stream`
 * (a hipStream_t; NULL selects the default stream).  *out receives the
 * context or NULL on failure. */
ffbie_status ffbie_create(ffbie_ctx **out, int device, void *hip_stream);

/* Release the context and its device workspaces.  Accepts NULL. */
ffbie_status ffbie_destroy(ffbie_ctx *ctx);

/* Text of the last error on this context (valid until the next call); a
 * static string when ctx is NULL. */
const char *ffbie_last_error(const ffbie_ctx *ctx);

/* Set the surface, discretisation and wavenumber k >= 0 (eq. (2.2)).  Uploads
 * the geometry and the angle tables to the device.  Must precede every
 * compute call; may be called again to change the problem. */
ffbie_status ffbie_set_problem(ffbie_ctx *ctx, const ffbie_geometry *g,
                               const ffbie_discretization *d, double k);

/* Azimuthal Fourier coefficients of the single-layer kernel for n_pairs
 * (target, source-curve) pairs by singularity swapping (Sec. 3.2-3.3).
 *
 * A pair is a target point r(t, theta_j) and a source curve t_s (t_s != t):
 *   d_tgt_t[i]   target curve parameter t (float64),
 *   d_tgt_az[i]  target azimuth index j in [0, 2M) (int32), theta_j = pi j / M,
 *   d_src_t[i]   source curve parameter t_s (float64).
 * Outputs (row-major, one row per pair):
 *   d_kappa      [n_pairs][2M] complex128: <e^{ik rho}/rho>_n for n = -M+1..M at
 *                column n + M - 1 -- the coefficients of eq. (3.9), formed as
 *                selected by kappa_variant.  Required.
 *   d_rhoinv     [n_pairs][M+M0+1] complex128: <rho^-1>_l for l = 0..M+M0
 *                (eq. (3.25)).  Optional (NULL).
 *   d_root       [n_pairs][2] float64: (a - theta_j, b) of the complex root
 *                theta_+ = a + i b of rho^2 used for the swap (Lemma 3.6).
 *                Optional (NULL).
 *   d_pair_status[n_pairs] int32: FFBIE_PAIR_* bits.  Optional (NULL).
 * Every row is written.  A pair with t == t_s gets a NaN row and
 * FFBIE_PAIR_SINGULAR.  Returns FFBIE_EINVAL for n_pairs < 0, a NULL d_kappa
 * or inputs, or no problem set.  n_pairs == 0 is a no-op. */
ffbie_status ffbie_kernel_coeffs(ffbie_ctx *ctx, int64_t n_pairs,
                                 const double *d_tgt_t, const int32_t *d_tgt_az,
                                 const double *d_src_t,
                                 void *d_kappa, void *d_rhoinv, double *d_root,
                                 int32_t *d_pair_status);

/* ffbie_kernel_coeffs for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same computation, arguments and outputs, but its scratch
 * (a 64-byte root record, a refine-list slot and a status word per pair, and
 * the refine-list counter) lives in a file-scope device array of the library,
 * one per GPU, allocated with the library's code and held until the process
 * ends: about 76 MiB, room for at most 1048576 pairs.  The call allocates
 * nothing (no hipMalloc, no library allocation) and needs only a problem set by
 * ffbie_set_problem.  n_pairs above 1048576 gives FFBIE_EINVAL.  Every call on
 * one GPU shares that GPU's array and leaves its contents behind (the counter
 * is cleared by a kernel at the start of each call): calls that overlap on one
 * GPU (from other contexts or streams) race and must be ordered by the
 * caller. */
ffbie_status ffbie_kernel_coeffs_noalloc(ffbie_ctx *ctx, int64_t n_pairs,
                                         const double *d_tgt_t, const int32_t *d_tgt_az,
                                         const double *d_src_t,
                                         void *d_kappa, void *d_rhoinv, double *d_root,
                                         int32_t *d_pair_status);

/* Mixed-precision coefficient path: ffbie_kernel_coeffs with the spectral
 * stage in FP32.  The surface samples, the complex root (Lemma 3.6), the
 * recurrences for A_m(b) (eqs. (3.27)-(3.28)) and the swap phases e^{-i n a}
 * stay in FP64; the FFTs of the sampled smooth factors, the truncation test of
 * eq. (3.24), the stored A_m and the convolution sums of eq. (3.25) run in
 * FP32.  Arguments as for ffbie_kernel_coeffs except:
 *   d_kappa      [n_pairs][2M] complex64 (interleaved float32 re, im),
 *   d_rhoinv     [n_pairs][M+M0+1] complex64 or NULL.
 * The truncation threshold is max(eps0, 1e-6): the FP32 transforms carry a
 * rounding floor of a few 1e-7 of the largest coefficient.  Results agree with
 * the FP64 path to about 1e-6 of each row's largest coefficient.  Errors as
 * for ffbie_kernel_coeffs. */
ffbie_status ffbie_kernel_coeffs_mixed(ffbie_ctx *ctx, int64_t n_pairs,
                                       const double *d_tgt_t, const int32_t *d_tgt_az,
                                       const double *d_src_t,
                                       void *d_kappa, void *d_rhoinv, double *d_root,
                                       int32_t *d_pair_status);

/* Azimuthal Fourier coefficients of the double-layer kernel (Sec. 4) for
 * n_pairs pairs, by singularity swapping with the s^{-3/2} coefficients
 * B_m(b) of eqs. (4.7)-(4.9), or translated swapping where that amplifies
 * rounding less (small b, chosen per pair):
 *   kK_n = < tau_0 (ik rho - 1) e^{ik rho} / rho^3 >_n,  n = -M+1..M,
 * with tau_0 = nu(r_s) . (r_s - r) for K (adjoint = 0, normal at the source,
 * eq. (2.13)) or nu(r) . (r - r_s) for K' (adjoint = 1, normal at the target,
 * eq. (2.10)); the kernels of K and K' are these divided by 2 pi.  Pairs,
 * inputs and the optional d_root and d_pair_status are as for
 * ffbie_kernel_coeffs; d_kappa [n_pairs][2M] complex128 receives kK_n at
 * column n + M - 1 (required).  FP64 throughout.  Errors as for
 * ffbie_kernel_coeffs, and FFBIE_EINVAL for adjoint not 0 or 1. */
ffbie_status ffbie_kernel_coeffs_dl(ffbie_ctx *ctx, int64_t n_pairs,
                                    const double *d_tgt_t, const int32_t *d_tgt_az,
                                    const double *d_src_t, int adjoint,
                                    void *d_kappa, double *d_root, int32_t *d_pair_status);

/* <rho^-1>_l, l = 0..L (L = M + M0), by the O(M) banded route of Sec. 3.2.1:
 * an alternative to the singularity swap of ffbie_kernel_coeffs for the same
 * coefficients.  For each pair, with m0 the truncation index of eq. (3.13):
 *   - <rho^2>_n, n = 0..m0, from 64 equispaced samples of rho^2 (exact: rho^2
 *     is a trigonometric polynomial in theta_s);
 *   - the known values of eq. (3.16), <rho^-1>_l for l < m0 and l > L - m0, by
 *     composite 16-point Gauss-Legendre quadrature graded towards the complex
 *     root of rho^2 (Lemma 3.6) and fine enough for e^{-i L theta_s};
 *   - the other L - 2 m0 + 1 coefficients from the Hermitian banded system of
 *     eqs. (3.14)-(3.18), a_j(i) = (m0 + 2i + j) <rho^2>_{m0-j}, by an
 *     unpivoted L D L^H factorisation (A is positive definite where eq. (3.19)
 *     holds, Lemma 3.4).
 * Pairs and inputs as for ffbie_kernel_coeffs.
 *   m0           1..8, or 0 for eq. (3.13) over this call's pairs with the
 *                discretisation's eps0 (the largest n <= deg with
 *                max_pairs |<rho^2>_n| / <rho^2>_0 > eps0, at least 1), where
 *                deg = max(2 m, m + 1) for the highest azimuthal order m of the
 *                surface is the degree of rho^2 (1 for the sphere, Remark 3.5).
 *                The automatic rule waits for the device (one stream
 *                synchronisation).
 *   d_rhoinv     [n_pairs][L+1] complex128, <rho^-1>_l at column l (required).
 *   d_pair_status[n_pairs] int32 or NULL: the root kernel's FFBIE_PAIR_* bits
 *                and FFBIE_PAIR_NOT_PD.
 *   m0_used      host int or NULL: receives the m0 used.
 * The call allocates device workspaces on first use and when n_pairs grows: 144
 * bytes per pair and the factor records of a chunk of pairs (at most 4 GiB).
 * A pair with t == t_s gets a NaN row and FFBIE_PAIR_SINGULAR.  Returns
 * FFBIE_EINVAL for n_pairs < 0, m0 outside 0..8, m0 = 0 on a surface whose
 * rho^2 has degree above 8, M + M0 < 4 m0, or NULL pointers; n_pairs == 0 is a
 * no-op.  FP64 throughout. */
ffbie_status ffbie_rhoinv_banded(ffbie_ctx *ctx, int64_t n_pairs,
                                 const double *d_tgt_t, const int32_t *d_tgt_az,
                                 const double *d_src_t, int m0, void *d_rhoinv,
                                 int32_t *d_pair_status, int *m0_used);

/* Device-side timing of the kernels ffbie_kernel_coeffs launches.  With
 * timing enabled, HIP events are recorded on the context's stream around the
 * root kernel, the main coefficient pass and the refine pass of every call;
 * ffbie_get_timing waits for the last call's events and returns the three
 * durations in milliseconds (any pointer may be NULL).  FFBIE_EINVAL if timing
 * is disabled or no call has been timed. */
ffbie_status ffbie_enable_timing(ffbie_ctx *ctx, int on);
ffbie_status ffbie_get_timing(ffbie_ctx *ctx, double *ms_root, double *ms_main,
                              double *ms_refine);

/* Singular-factor coefficients A_m(b) = <s_{0,b}^{-1/2}>_m of eq. (3.26) for
 * m = 0..m_max and n values of b > 0 (d_b, float64 [n]), written to
 * d_A [n][m_max+1] float64.  Uses the same device routine as
 * ffbie_kernel_coeffs (Miller's backward recurrence normalised by
 * A_0 = (2/pi) K(e^{-2b}), or for small b the difference recurrence of
 * eq. (3.28)).  b <= 0 gives a NaN row.  1 <= m_max <= 1023. */
ffbie_status ffbie_singular_factor(ffbie_ctx *ctx, int64_t n, const double *d_b,
                                   int m_max, double *d_A);

/* Batched coefficients: the coefficient path of ffbie_kernel_coeffs for many
 * independent problems (surfaces, wavenumbers, M) in one persistent launch
 * per phase.  Each item is a problem and its pair list:
 *   g, d, k        as for ffbie_set_problem (d.n_panels is not used;
 *                  d.kappa_variant must be FFBIE_KAPPA_SWAP),
 *   n_pairs, d_t, d_az, d_ts   the pairs, as for ffbie_kernel_coeffs,
 *   d_kappa        [n_pairs][2M] complex128 output (required if n_pairs > 0),
 *   d_pair_status  [n_pairs] int32 output (optional NULL).
 * items is a HOST array of n_items entries.  Results are those of one
 * ffbie_kernel_coeffs call per item.  The problem of ffbie_set_problem is
 * left unchanged.  Work items (waves_per_block x pairs_per_item pairs of one
 * problem, from the context's tuning) are taken from a device-side queue
 * ordered by decreasing M, so problems of different cost share the GPU.
 * The call waits for the previous batched call's kernels and for the small
 * descriptor upload (stream syncs) before enqueuing the kernels. */
typedef struct {
  ffbie_geometry g;
  ffbie_discretization d;
  double k;
  int64_t n_pairs;
  const double *d_t;
  const int32_t *d_az;
  const double *d_ts;
  void *d_kappa;
  int32_t *d_pair_status;
} ffbie_batch_item;
ffbie_status ffbie_kernel_coeffs_batched(ffbie_ctx *ctx, int n_items, const ffbie_batch_item *items);

/* Launch choices of the coefficient kernels:
 *   fft_radix        transforms of the 2M-sample main pass (the 4M-sample
 *                    refine pass uses radix 2): 2: radix-2 Stockham; 4:
 *                    radix-4 stages (with one radix-2 stage when log2(N_F) is
 *                    odd); 0: radix 4 for N_F >= 256 points, else radix 2,
 *   pairs_per_item   pairs a wavefront takes from one batch work item (1..256),
 *   waves_per_block  wavefronts per workgroup of the batched launch (1, 2, 4;
 *                    lowered to what fits 64 KiB of LDS),
 *   persistent       batched main pass: 1 = a bounded grid whose wavefronts
 *                    take work items from a queue until it is empty; 0 = one
 *                    wavefront per work item (taken as 1 when that grid would
 *                    exceed 2^32 work-items).
 * A context starts with {0, 16, 4, 0}; its fft_radix also applies to
 * ffbie_kernel_coeffs(_mixed) and the near blocks of ffbie_assemble.  Results
 * do not depend on the tuning beyond rounding (the transforms differ in
 * operation order). */
typedef struct {
  int fft_radix;
  int pairs_per_item;
  int waves_per_block;
  int persistent;
} ffbie_tuning;
ffbie_status ffbie_set_tuning(ffbie_ctx *ctx, const ffbie_tuning *tuning);
ffbie_status ffbie_get_tuning(const ffbie_ctx *ctx, ffbie_tuning *tuning);

/* Batch plans: the batched coefficient path of ffbie_kernel_coeffs_batched,
 * prepared once and executed any number of times (for instance with new pair
 * data in the same buffers).  The problems are grouped by M; each group (an
 * "M class") runs its main pass as one launch over (problem, run of pairs)
 * work items (persistent or one wavefront per item, see ffbie_tuning) and its
 * refine pass as one persistent launch, after one root launch for all.  ffbie_batch_plan_create validates the items
 * (HOST array; the device buffers they name must stay valid for the plan's
 * life), orders them, uploads the descriptors and allocates the plan's own
 * workspace (root records, refine queue, counters: about 76 B per pair).
 * flags (or-ed):
 *   FFBIE_PLAN_AUTOTUNE  for each M class of the batch, time its main pass for
 *                        every candidate tuning (radix {2, 4} x pairs_per_item
 *                        {8, 16, 32} x waves_per_block {1, 2, 4} x persistent
 *                        {0, 1}) and keep the fastest; the creating call then
 *                        runs the main pass ~72 times,
 *   FFBIE_PLAN_GRAPH     capture the launch sequence (counter reset, root,
 *                        main and refine passes) in a HIP graph that execute
 *                        replays on the context's stream,
 *   FFBIE_PLAN_MIXED     FP32 spectral stage as in ffbie_kernel_coeffs_mixed:
 *                        every item's d_kappa is complex64.
 * tuning: NULL takes the context's tuning for every class; otherwise an
 * array of 4 tunings for the classes M = 16, 32, 64, 128 (the tuning used, or
 * the start point of the autotuner).
 * execute enqueues on the context's stream and returns; outputs are those of
 * ffbie_kernel_coeffs_batched.  Executions of one plan must not overlap (they
 * share its workspace): the stream order guarantees this.  destroy waits for
 * the context's stream, then frees the plan.  ffbie_batch_plan_classes gives
 * the number of M classes (0 for an empty batch); get_tuning reports class
 * m_class's M, the tuning in use and, after autotuning, its main-pass time in
 * ms (FFBIE_EINVAL for a class out of range).
 * With timing enabled (ffbie_enable_timing), executing a plan that has no
 * graph records the root, main and refine passes for ffbie_get_timing.
 * Destroy every plan before its context. */
typedef struct ffbie_batch_plan ffbie_batch_plan;
#define FFBIE_PLAN_GRAPH 1
#define FFBIE_PLAN_AUTOTUNE 2
#define FFBIE_PLAN_MIXED 4
ffbie_status ffbie_batch_plan_create(ffbie_ctx *ctx, int n_items, const ffbie_batch_item *items,
                                     int flags, const ffbie_tuning *tuning,
                                     ffbie_batch_plan **out);
ffbie_status ffbie_batch_plan_execute(ffbie_ctx *ctx, ffbie_batch_plan *plan);
int ffbie_batch_plan_classes(const ffbie_batch_plan *plan);
ffbie_status ffbie_batch_plan_get_tuning(const ffbie_batch_plan *plan, int m_class,
                                         ffbie_tuning *tuning, double *tuned_ms, int *M);
ffbie_status ffbie_batch_plan_destroy(ffbie_batch_plan *plan);

/* On-disk cache of the autotuner's choices.  With a cache file set (path, a
 * HOST string copied by the call; NULL or "" clears it), FFBIE_PLAN_AUTOTUNE
 * first looks each M class up by (device architecture and compute-unit count,
 * M, FP64 or mixed precision): a hit is used without timing (its recorded
 * main-pass time is what ffbie_batch_plan_get_tuning reports), a miss is
 * tuned as usual and added to the file, which is then rewritten (JSON: one
 * flat entry per key, see the entries ffbie writes; written to path.tmp and
 * renamed).  An unreadable or foreign file counts as empty.  Plan creation
 * returns FFBIE_EDEVICE if the file cannot be written.  Entries are checked
 * against the launch limits before use. */
ffbie_status ffbie_set_tuning_cache(ffbie_ctx *ctx, const char *path);

/* ------------------------------------------------------------------------
 * The discrete single-layer system (Sec. 3.1 and 3.4)
 * ------------------------------------------------------------------------
 * Unknowns and collocation points share one ordering: index
 *   r = (i * 16 + l) * 2M + j
 * for panel i in [0, n_panels), Gauss-Legendre node l in [0, 16) and azimuth
 * j in [0, 2M); the point is r(t_i^l, theta_j) with t_i^l the l-th node of the
 * panel [i pi / n_panels, (i + 1) pi / n_panels] and theta_j = pi j / M.
 * N = 32 M n_panels.  The unknown at index r is the density times the surface
 * Jacobian, phi~ = phi J (eq. (3.1)).  Complex vectors are complex128 [N]. */

/* Near-panel quadrature rules (Sec. 3.1): for a target at Gauss-Legendre
 * position x_l of its panel (panel coordinate in (-1, 1)), the t_s integral
 * over its own panel uses nodes self_x[l][q] and weights self_w[l][q]
 * (q < 16) in that panel's coordinate, and over the right-hand neighbour the
 * nodes right_x[l][q], weights right_w[l][q] in the neighbour's coordinate.
 * The left-hand neighbour uses the mirror image of the right-hand rule of
 * target 15 - l (nodes -right_x[15-l][q], same weights).  Weights are for
 * the panel coordinate (they sum to 2 for an exact rule). */
typedef struct {
  double self_x[16][16];
  double self_w[16][16];
  double right_x[16][16];
  double right_w[16][16];
} ffbie_near_rule;

/* Copy the library's built-in rules (16-node generalized Gaussian rules,
 * exact for P_k and P_k log|t_s - t| with k < 16) into *out.  Host only; needs
 * no context or device. */
ffbie_status ffbie_builtin_near_rule(ffbie_near_rule *out);

/* Select the near rules used by ffbie_near_pairs and ffbie_assemble: a HOST
 * pointer, copied; NULL restores the built-in rules.  Nodes must lie in
 * (-1, 1) and differ from the target position for the self panel, else
 * FFBIE_EINVAL.  Persists across ffbie_set_problem. */
ffbie_status ffbie_set_near_rule(ffbie_ctx *ctx, const ffbie_near_rule *rule);

/* Sizes for the current problem: the number of unknowns N = 32 M n_panels,
 * the number of near pairs (target point, near-rule source node):
 * 512 M (3 n_panels - 2) for n_panels >= 2, and an upper bound of the device
 * workspace (bytes) the context allocates for ffbie_assemble plus the most
 * demanding ffbie_solve method on this problem (the complex64 copy of S of
 * LU32_IR64 / GMRES_LU32, or the mode blocks and Krylov bases of the GMRES
 * forms), beyond the caller's own buffers.  Any pointer may be NULL. */
ffbie_status ffbie_query(ffbie_ctx *ctx, int64_t *n_unknowns, int64_t *n_near_pairs,
                         int64_t *workspace_bytes);

/* Write the near pair set as ffbie_kernel_coeffs inputs: d_t, d_az, d_ts
 * [n_near_pairs] (float64, int32, float64).  Order: panel i, node l, azimuth
 * j, relation (left neighbour, own panel, right neighbour; neighbours outside
 * [0, n_panels) are absent), rule node q. */
ffbie_status ffbie_near_pairs(ffbie_ctx *ctx, double *d_t, int32_t *d_az, double *d_ts);

/* Collocation points x_r (d_xyz [N][3] float64), surface Jacobians
 * J = |r_t x r_theta| (d_jac [N], optional NULL) and the quadrature weight of
 * each unknown, w_i^l / (2M) with w_i^l the Gauss-Legendre weight on the panel
 * (d_wq [N], optional NULL), so that a surface integral of phi is
 * sum_r wq_r phi~_r * 2 pi (eq. (3.8) with the 16-point rule of eq. (3.7)). */
ffbie_status ffbie_collocation(ffbie_ctx *ctx, double *d_xyz, double *d_jac, double *d_wq);

/* Right-hand sides on the collocation points (d_g [N] complex128):
 *   FFBIE_RHS_POINT_SOURCE: g = G(x; p) = e^{ik|x - p|} / (4 pi |x - p|) with
 *     p = (params[0], params[1], params[2]), the interior Dirichlet test of
 *     Sec. 5 (exact interior field G(.; p) when p is outside the surface);
 *   FFBIE_RHS_PLANE_WAVE: g = -e^{ik d.x} with d = params[0..2] (unit), the
 *     sound-soft exterior problem for the incident wave e^{ik d.x};
 *   FFBIE_RHS_PLANE_WAVE_DN: g = -d/d nu e^{ik d.x} = -ik (d . nu) e^{ik d.x}
 *     (nu the outward unit normal), the sound-hard exterior problem, whose
 *     second-kind equation (K' - I) phi = g is eq. (2.9) for (ENP);
 *   FFBIE_RHS_POINT_SOURCE_DN: g = d/d nu G(x; p), the interior Neumann test
 *     of Sec. 5 (exact interior field G(.; p) when p is outside the surface).
 * params is a HOST pointer to 3 doubles. */
enum { FFBIE_RHS_POINT_SOURCE = 0, FFBIE_RHS_PLANE_WAVE = 1, FFBIE_RHS_PLANE_WAVE_DN = 2,
       FFBIE_RHS_POINT_SOURCE_DN = 3 };
ffbie_status ffbie_rhs(ffbie_ctx *ctx, int kind, const double *params, void *d_g);

/* Assemble the N x N matrix S of the discretised single-layer equation
 * S phi~ = g (Sec. 3.4, eq. (3.29)) into d_S, ROW-major complex128: entry (r, c) at
 * d_S[r * ld + c], ld >= N.  Row r is the collocation point, column c the
 * unknown.
 *  - far panels (|i - i'| >= 2): S = (h/2) w_{l'} (1/2M) e^{ik rho}/rho with
 *    rho = |x_r - x_c| and h = pi / n_panels (eqs. (3.7)-(3.8));
 *  - near panels (|i - i'| <= 1): S = sum_q (h/2) W_q L_{l'}(y_q) w_{j'} with
 *    the near rule (W_q, y_q), L_{l'} the Lagrange basis of the panel's
 *    Gauss-Legendre nodes (interpolation of phi~ in t_s), and
 *    w_{j'} = (1/2M) sum_{n=-M+1}^{M} kappa_n e^{i n theta_{j'}} the inverse
 *    DFT (discrete Parseval relation) of the kernel coefficients of
 *    ffbie_kernel_coeffs at (x_r, t_s = node y_q) (eqs. (3.9)-(3.10)).
 * Uses a device workspace for the near kernel coefficients (at most about
 * 2 GB, allocated on first use).  FFBIE_EINVAL for a NULL matrix or ld < N;
 * FFBIE_WUNRESOLVED (a warning: S is assembled) if near pairs were flagged
 * unresolved, see ffbie_assembly_report. */
ffbie_status ffbie_assemble(ffbie_ctx *ctx, void *d_S, int64_t ld);

/* Operators of the boundary integral equations of Sec. 2 (eqs. (2.8), (2.10), (2.13)). */
enum {
  FFBIE_OP_S = 0,    /* single layer S = 2 int G phi dsigma (eq. (2.8))          */
  FFBIE_OP_K = 1,    /* double layer K = 2 p.v. int dG/d nu(y) psi dsigma (eq. (2.13)) */
  FFBIE_OP_KP = 2    /* adjoint K' = 2 p.v. int dG/d nu(x) phi dsigma (eq. (2.10)) */
};

/* What the unknowns of an assembled system are. */
enum {
  FFBIE_UNKNOWN_SCALED = 0,   /* density x Jacobian, phi~ = phi J (Sec. 3.4; ffbie_assemble) */
  FFBIE_UNKNOWN_DENSITY = 1   /* the density values themselves: column c carries J_c       */
};

/* Assemble op + shift * I into d_S, with the layout, discretisation, near
 * rule, workspace and return values of ffbie_assemble (op = FFBIE_OP_S,
 * shift = 0, FFBIE_UNKNOWN_SCALED is ffbie_assemble).  For K and K' the far
 * entries are (h/2) w_{l'} (1/2M) tau_0 (ik rho - 1) e^{ik rho} / rho^3 with
 * tau_0 = nu_c . (x_c - x_r) (K) or nu_r . (x_r - x_c) (K'), and the near
 * blocks take the coefficients of ffbie_kernel_coeffs_dl through the same
 * rule.  With FFBIE_UNKNOWN_DENSITY every column c is multiplied by J_c and
 * shift * I is added as it is; with FFBIE_UNKNOWN_SCALED it enters the
 * diagonal as shift / J_r.  shift = +1 with K gives the exterior Dirichlet
 * equation (K + I) psi = g, shift = -1 with K' the exterior Neumann equation
 * (K' - I) phi = g (eqs. (2.12) and (2.9)); for these second-kind systems
 * density unknowns keep the spectrum clustered at the shift, while scaled
 * unknowns spread it by the range of 1/J (large near the poles), which
 * iterative solvers feel.  FFBIE_EINVAL for an unknown op or unknowns value
 * or a non-finite shift. */
ffbie_status ffbie_assemble_op(ffbie_ctx *ctx, int op, double shift, int unknowns, void *d_S,
                               int64_t ld);

/* Near pairs of the last ffbie_assemble on this context: their number, how
 * many the coefficient path flagged FFBIE_PAIR_UNRESOLVED (the smooth factor
 * not resolved even by 4M azimuthal samples: the wavenumber is too large for
 * M, and those near-block entries carry the truncation error of the smooth
 * factor's spectrum) and how many FFBIE_PAIR_ROOT_FALLBACK.  ffbie_assemble
 * returns FFBIE_WUNRESOLVED when the first count is not zero (it reads the
 * counts back, so it returns after the assembly has finished).  Any pointer
 * may be NULL; FFBIE_EINVAL before the first assembly. */
ffbie_status ffbie_assembly_report(ffbie_ctx *ctx, int64_t *n_near_pairs, int64_t *n_unresolved,
                                   int64_t *n_root_fallback);

/* Field of the single-layer representation u(x) = 2 int G(x, y) phi(y) dsigma
 * (eq. (2.6)) at n_pts points off the surface, by the same 16-point-by-2M
 * product rule: u(x) = sum_c wq_c e^{ik|x - x_c|} / |x - x_c| phi~_c.
 * d_pts [n_pts][3] float64, d_phi [N] complex128, d_u [n_pts] complex128. */
ffbie_status ffbie_eval_field(ffbie_ctx *ctx, int64_t n_pts, const double *d_pts,
                              const void *d_phi, void *d_u);

/* Field of a layer representation by the same product rule, for densities
 * given as the unknowns of ffbie_assemble_op (FFBIE_UNKNOWN_*): op =
 * FFBIE_OP_S with scaled unknowns is ffbie_eval_field; op = FFBIE_OP_K the
 * double-layer representation u(x) = 2 int dG(x, y)/d nu(y) psi(y) dsigma
 * (eq. (2.11)), u(x) = sum_c wq_c tau_0 (ik rho - 1) e^{ik rho} / rho^3 psi~_c
 * with tau_0 = nu_c . (x_c - x), rho = |x - x_c| (psi~_c = J_c psi_c for
 * density unknowns).  FFBIE_EINVAL for another op or unknowns value. */
ffbie_status ffbie_eval_field_op(ffbie_ctx *ctx, int op, int unknowns, int64_t n_pts,
                                 const double *d_pts, const void *d_phi, void *d_u);

/* Dense solve of S phi~ = g for the matrix of ffbie_assemble (row-major
 * complex128, leading dimension ld >= N).  The paper leaves the solver open;
 * three are provided:
 *   FFBIE_SOLVE_LU64       LU with partial pivoting in complex128.  S is
 *                          OVERWRITTEN by its factors.  tol, max_iter unused.
 *   FFBIE_SOLVE_LU32_IR64  LU of a complex64 copy of S (workspace N*N*8 bytes),
 *                          then iterative refinement phi += (LU32)^{-1} r with the
 *                          residual r = g - S phi in complex128; S is read only.
 *                          Stops when |r|_2 <= tol |g|_2 or after max_iter steps.
 *   FFBIE_SOLVE_GMRES      restarted GMRES (restart 100) in complex128 with the
 *                          matrix-vector product of S; S is read only (workspace
 *                          101 N complex128).  Stops as above (max_iter counts
 *                          Krylov iterations).
 * d_g [N] and d_phi [N] complex128 (distinct buffers).  The call synchronises
 * the context's stream (iterative methods read norms on the host) and returns
 * after the solve has finished.  info (optional): iterations and the final
 * relative residual |g - S phi| / |g| (NaN for LU64, whose S is destroyed).
 *   FFBIE_SOLVE_FGMRES_MLP flexible GMRES (restart 100) with the learned per-mode
 *                          preconditioner (ffbie_mlp_*) as right preconditioner and
 *                          phi_0 = P(g) as initial guess; if it does not reach tol
 *                          within max_iter, the plain GMRES solve runs from zero for
 *                          up to max_iter more (info->fell_back = 1).  Needs
 *                          set weights and n_panels = 16 (256 curve nodes).
 *   FFBIE_SOLVE_GMRES_BLOCKJACOBI  GMRES (restart 100) right-preconditioned by
 *                          the inverses of the diagonal azimuthal-mode blocks of S
 *                          (see ffbie_blockjacobi_setup), built inside the call;
 *                          phi_0 = P(g).  Needs 16 n_panels <= 512.
 *   FFBIE_SOLVE_FGMRES_BJ_MLP flexible GMRES (restart 100) with P(v) = BJ(v) +
 *                          NN(v): the mode-block-Jacobi correction (as for
 *                          GMRES_BLOCKJACOBI) plus the learned network's
 *                          correction of what block-Jacobi misses (ffbie_mlp_*,
 *                          trained on S^{-1} v - BJ(v)); phi_0 = P(g); falls back to
 *                          plain GMRES as FGMRES_MLP does.  Needs weights and
 *                          n_panels = 16.
 *   FFBIE_SOLVE_GMRES_LU32 GMRES (restart 100) in complex128 right-preconditioned
 *                          by the LU factors of a complex64 copy of S
 *                          (workspace N*N*8 bytes): the GMRES form of mixed-
 *                          precision iterative refinement, which still converges
 *                          when the refinement of FFBIE_SOLVE_LU32_IR64 stalls
 *                          (condition number near 1 / complex64 unit roundoff).
 * Returns FFBIE_ESINGULAR on an exactly zero pivot, FFBIE_WNOTCONV if an
 * iterative method did not reach tol (phi holds the last iterate). */
enum { FFBIE_SOLVE_LU64 = 0, FFBIE_SOLVE_LU32_IR64 = 1, FFBIE_SOLVE_GMRES = 2,
       FFBIE_SOLVE_FGMRES_MLP = 3, FFBIE_SOLVE_GMRES_BLOCKJACOBI = 4, FFBIE_SOLVE_GMRES_LU32 = 5,
       FFBIE_SOLVE_FGMRES_BJ_MLP = 6 };
typedef struct {
  int iterations;
  int converged;
  double rel_residual;
  int fell_back;      /* FGMRES_MLP: 1 if the learned preconditioner did not reach tol
                         and the plain GMRES solve produced phi */
} ffbie_solve_info;
ffbie_status ffbie_solve(ffbie_ctx *ctx, int method, void *d_S, int64_t ld, const void *d_g,
                         void *d_phi, double tol, int max_iter, ffbie_solve_info *info);

/* ------------------------------------------------------------------------
 * Learned preconditioner (the learned part of the solve; the paper's method
 * without it is FFBIE_SOLVE_GMRES / LU64).  A multilayer perceptron
 * 514 -> 256 -> 256 -> 512 (ReLU) is applied to every azimuthal mode m of a
 * residual r on the 256 curve nodes (n_panels = 16):
 *   R_m[node] = (1/2M) sum_j r[node, j] e^{-i m theta_j},  m = -M+1..M,
 *   s_m = |R_m|_2,  x_m = [Re R_m / s_m, Im R_m / s_m, k/30, m/M],
 *   E_m = s_m (y_m[0:256] + i y_m[256:512]),  y_m = MLP(x_m),
 *   P(r)[node, j] = sum_m E_m[node] e^{i m theta_j}.
 * Weights and activations are BF16 on the matrix cores with FP32 accumulation;
 * FP32 master weights, Adam.  Parameters, in this order: W1 [256][514], b1 [256],
 * W2 [256][256], b2 [256], W3 [512][256], b3 [512] (row-major, float32). */
int64_t ffbie_mlp_param_count(void);
/* Deterministic initialisation from `seed` (He-uniform hidden layers, zero biases). */
ffbie_status ffbie_mlp_init(ffbie_ctx *ctx, uint64_t seed);
/* Host float32 arrays of ffbie_mlp_param_count() values (copied). */
ffbie_status ffbie_mlp_set_params(ffbie_ctx *ctx, const float *params);
ffbie_status ffbie_mlp_get_params(ffbie_ctx *ctx, float *params);
/* d_y [n][512] = MLP(d_x [n][514]), float32 device arrays (inputs rounded to BF16). */
ffbie_status ffbie_mlp_forward(ffbie_ctx *ctx, int64_t n, const float *d_x, float *d_y);
/* One step on the loss (1/2n) sum_i |MLP(x_i) - t_i|^2 over n samples (d_x
 * [n][514], d_t [n][512] float32 device): gradients into d_grads (optional,
 * [param_count] float32 device), then an Adam step with learning rate lr if
 * update != 0.  *loss (host, optional) receives the loss before the step.
 * Synchronises the stream. */
ffbie_status ffbie_mlp_train_step(ffbie_ctx *ctx, int64_t n, const float *d_x, const float *d_t,
                                  float lr, int update, float *d_grads, double *loss);
/* Training on a set of samples the method generated (for instance mode
 * features of residuals of assembled systems, ffbie_mode_features, with the
 * corrections they should map to, ffbie_mode_targets): `steps` Adam steps on
 * minibatches of `batch` samples drawn without replacement per epoch (order
 * from `seed`), learning rate lr (1 + cos(pi step / steps)) / 2, all on the
 * device with the kernels of ffbie_mlp_train_step.  Needs weights
 * (ffbie_mlp_init / set_params / load).  info (optional) receives the loss of
 * the first and last minibatch before their step and the loss over the whole
 * set after training.  Synchronises the stream.  FFBIE_EINVAL unless
 * 1 <= batch <= min(n_samples, 65535), steps >= 1 and lr > 0. */
typedef struct {
  int64_t n_samples;     /* rows of d_x and d_t */
  const float *d_x;      /* [n_samples][514] network inputs, float32 device */
  const float *d_t;      /* [n_samples][512] targets, float32 device */
  int steps;
  int batch;
  float lr;
  uint64_t seed;
} ffbie_train_cfg;
typedef struct {
  double loss_first;
  double loss_last;
  double loss_full;
  int steps;
} ffbie_train_info;
ffbie_status ffbie_mlp_train(ffbie_ctx *ctx, const ffbie_train_cfg *cfg, ffbie_train_info *info);
/* Checkpoint of the network and its optimiser state: the float32 parameters
 * (in the order above), both Adam moments and the Adam step count, in a
 * binary file of its own format ("FFBIEMLP", version, count, step, data).
 * load replaces the weights and optimiser state of the context; a file of
 * another format, size or with non-finite parameters gives FFBIE_EINVAL and
 * leaves the context unchanged.  Host paths; synchronise the stream. */
ffbie_status ffbie_mlp_save(ffbie_ctx *ctx, const char *path);
ffbie_status ffbie_mlp_load(ffbie_ctx *ctx, const char *path);

/* Mode features of d_r [N] complex128 for the current problem: d_x [2M][514]
 * float32 and the scales d_scale [2M] float64 (row m + M - 1 is mode m). */
ffbie_status ffbie_mode_features(ffbie_ctx *ctx, const void *d_r, float *d_x, double *d_scale);
/* Training targets for a solution e of S e = r: d_t [2M][512] float32,
 * [Re E_m / s_m, Im E_m / s_m] with the scales of r's features. */
ffbie_status ffbie_mode_targets(ffbie_ctx *ctx, const void *d_e, const double *d_scale, float *d_t);
/* d_z = P(d_v) for the current problem ([N] complex128). */
ffbie_status ffbie_mlp_precondition(ffbie_ctx *ctx, const void *d_v, void *d_z);

/* Factor once, solve many: ffbie_lu_factor overwrites d_S with its LU64
 * factors (as FFBIE_SOLVE_LU64 does) and keeps the interchanges in the context;
 * ffbie_lu_solve then overwrites d_x [N] (the right-hand side on entry) with
 * S^{-1} x, using the factors in d_S (unchanged since the factorisation).  Both
 * synchronise the stream.  FFBIE_EINVAL if no factorisation of this size is held. */
ffbie_status ffbie_lu_factor(ffbie_ctx *ctx, void *d_S, int64_t ld);
ffbie_status ffbie_lu_solve(ffbie_ctx *ctx, const void *d_S, int64_t ld, void *d_x);

/* The trailing-update product of the LU factorisations (FFBIE_SOLVE_LU64,
 * LU32_IR64, GMRES_LU32, ffbie_lu_factor): C -= A B on the matrix cores for
 * complex column-major blocks with the common leading dimension ld (in complex
 * elements): A is m x k, B is k x n, C is m x n, element (r, c) of each at
 * index c * ld + r.  complex64 = 0: complex128 with FP64 MFMA; complex64 != 0:
 * complex64 with FP32 MFMA and FP32 accumulation.  A and B are read only and
 * must not overlap C.  Enqueued on the context's stream; needs no problem set.
 * FFBIE_EINVAL for negative sizes, sizes above 2^31 - 1, ld < max(m, k, 1) or
 * a NULL pointer when m n k > 0. */
ffbie_status ffbie_gemm_sub(ffbie_ctx *ctx, int complex64, int64_t m, int64_t n, int64_t k,
                            const void *d_A, const void *d_B, void *d_C, int64_t ld);

/* Mode-block-Jacobi preconditioner.  In the azimuthal Fourier basis
 * phi[(b, j)] = sum_m Phi_m[b] e^{i m theta_j} (m = -M+1..M) the matrix S splits
 * into blocks over the 16 n_panels curve nodes; setup extracts the 2M diagonal
 * blocks B_m[a][b] = (1/2M) sum_{j,j'} e^{-i m theta_j} S[(a,j),(b,j')] e^{i m theta_j'}
 * from d_S (read only) and factors them (LU, partial pivoting); apply computes
 * z = sum_m (B_m^{-1} V_m) e^{i m theta}.  Workspace 2M (16 n_panels)^2 complex128. */
ffbie_status ffbie_blockjacobi_setup(ffbie_ctx *ctx, const void *d_S, int64_t ld);
ffbie_status ffbie_blockjacobi_apply(ffbie_ctx *ctx, const void *d_v, void *d_z);

/* r = g - S phi in complex128 (row-major S, leading dimension ld); d_r [N]. */
ffbie_status ffbie_residual(ffbie_ctx *ctx, const void *d_S, int64_t ld, const void *d_phi,
                            const void *d_g, void *d_r);

#ifdef __cplusplus
}
#endif

#endif /* FFBIE_H */
