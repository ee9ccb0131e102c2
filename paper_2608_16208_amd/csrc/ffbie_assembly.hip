// Assembly of the discrete single-layer system and of the double-layer
// operators K and K' (Sec. 4), right-hand sides and field evaluation (paper
// Sec. 3.1 and 3.4) for gfx950.
//
// Layout: unknowns and collocation points share the index r = (i*16 + l)*2M + j
// (panel i, Gauss-Legendre node l, azimuth j).  S is row-major: a row is one
// collocation point, so every kernel below writes whole row segments and its
// stores are coalesced.
//
//   collocation   one thread per point: x, y, z, Jacobian and the product
//                 quadrature weight (h/2) w_l / (2M)            (eqs. (3.7)-(3.8))
//   far blocks    |i - i'| >= 2: (h/2) w_l' (1/2M) e^{ik rho}/rho; a block of 256
//                 threads owns 256 columns and walks 8 rows, so each thread keeps
//                 its source point in registers; near columns are skipped
//   near pairs    the (target, near-rule node) pairs fed to the coefficient kernels
//   near blocks   one workgroup per (target point, near panel): contracts the 16
//                 coefficient rows with the Lagrange-times-weight matrix of the
//                 near rule, then inverse-DFTs the 16 contracted rows (discrete
//                 Parseval, eq. (3.9)) with a radix-2 Stockham FFT in LDS and
//                 writes 16 x 2M contiguous entries
//   field, rhs    one workgroup per (point, source chunk) with a fixed-order
//                 reduction; one thread per collocation point
#include "ffbie_assembly.hpp"
#include "ffbie_fft128.hpp"

namespace ffbie {

namespace {

struct GL16 {
  double x[kNodes], w[kNodes];
};

// Point of the star surface and the Jacobian |r_t x r_theta| (eq. (2.1)).
__device__ void surface_point(const Geom& g, double t, double th, double* px, double* py,
                              double* pz, double* jac, double* nrm) {
  double st, ct, sth, cth;
  sincos_bounded(t, &st, &ct);
  sincos_bounded(th, &sth, &cth);
  double R = 1.0, Rt = 0.0, Rth = 0.0;
  for (int l = 1; l <= g.lmax; ++l) {
    double sl, cl;
    sincos_bounded(l * t, &sl, &cl);
    for (int m = 0; m <= g.mmax; ++m) {
      const double a = g.a[l - 1][m];
      if (a == 0.0) continue;
      double sm, cm;
      sincos_bounded(m * th, &sm, &cm);
      R = fma(a * sl, cm, R);
      Rt = fma(a * l * cl, cm, Rt);
      Rth = fma(-a * m * sl, sm, Rth);
    }
  }
  const double ox = st * cth, oy = st * sth, oz = ct;          // omega
  const double tx = ct * cth, ty = ct * sth, tz = -st;         // d omega / dt
  const double hx = -st * sth, hy = st * cth, hz = 0.0;        // d omega / dtheta
  // r = D R omega: D scales r, r_t and r_theta (unit D: the star itself)
  const double gx = g.ax[0], gy = g.ax[1], gz = g.ax[2];
  const double rtx = gx * (Rt * ox + R * tx), rty = gy * (Rt * oy + R * ty), rtz = gz * (Rt * oz + R * tz);
  const double rhx = gx * (Rth * ox + R * hx), rhy = gy * (Rth * oy + R * hy), rhz = gz * (Rth * oz + R * hz);
  const double cx = rty * rhz - rtz * rhy;
  const double cy = rtz * rhx - rtx * rhz;
  const double cz = rtx * rhy - rty * rhx;
  *px = gx * (R * ox);
  *py = gy * (R * oy);
  *pz = gz * (R * oz);
  const double J = sqrt(cx * cx + cy * cy + cz * cz);
  *jac = J;
  nrm[0] = cx / J;
  nrm[1] = cy / J;
  nrm[2] = cz / J;
}

__global__ __launch_bounds__(256) void collocation_kernel(Geom g, SysDims d, GL16 gl, Colloc c,
                                                          double* xyz, double* jac_out,
                                                          double* wq_out) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= d.N) return;
  const int nj = 2 * d.M;
  const int j = (int)(r % nj);
  const int l = (int)((r / nj) % kNodes);
  const int i = (int)(r / (nj * kNodes));
  const double t = i * d.h + 0.5 * d.h * (gl.x[l] + 1.0);
  const double th = M_PI * j / d.M;
  double x, y, z, J, nrm[3];
  surface_point(g, t, th, &x, &y, &z, &J, nrm);
  const double wq = 0.5 * d.h * gl.w[l] / nj;
  c.x[r] = x;
  c.y[r] = y;
  c.z[r] = z;
  c.wq[r] = wq;
  c.jac[r] = J;
  c.nx[r] = nrm[0];
  c.ny[r] = nrm[1];
  c.nz[r] = nrm[2];
  if (xyz) {
    xyz[3 * r] = x;
    xyz[3 * r + 1] = y;
    xyz[3 * r + 2] = z;
  }
  if (jac_out) jac_out[r] = J;
  if (wq_out) wq_out[r] = wq;
}

// One thread per (target point, relation slot, rule node) of the chunk.
__global__ __launch_bounds__(256) void near_pairs_kernel(SysDims d, NearChunk ch, GL16 gl,
                                                         const double* __restrict__ rule_y,
                                                         double* t_out, int32_t* az_out,
                                                         double* ts_out) {
  const int nj = 2 * d.M;
  const int64_t n_tgt = (int64_t)(ch.p1 - ch.p0) * kNodes * nj;
  const int64_t idx = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (idx >= n_tgt * 3 * kNodes) return;
  const int q = (int)(idx % kNodes);
  const int slot = (int)((idx / kNodes) % 3);
  const int64_t tgt = idx / (3 * kNodes);
  const int j = (int)(tgt % nj);
  const int l = (int)((tgt / nj) % kNodes);
  const int i = ch.p0 + (int)(tgt / ((int64_t)nj * kNodes));
  const int nrel = near_relations(i, d.n_panels);
  if (slot >= nrel) return;
  const int rel = (i > 0) ? slot - 1 : slot;               // -1, 0, +1
  const int64_t p = near_pairs_before(i, d) - ch.pair_base +
                    (((int64_t)l * nj + j) * nrel + slot) * kNodes + q;
  const double y = rule_y[(l * 3 + rel + 1) * kNodes + q];
  t_out[p] = i * d.h + 0.5 * d.h * (gl.x[l] + 1.0);
  az_out[p] = j;
  ts_out[p] = (i + rel) * d.h + 0.5 * d.h * (y + 1.0);
}

constexpr int kFarRows = 8;

typedef double dbl2 __attribute__((ext_vector_type(2)));

__global__ __launch_bounds__(256) void far_kernel(SysDims d, double k, Colloc c,
                                                  cplx* __restrict__ S, int64_t ld, int density) {
  const int64_t col = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (col >= d.N) return;
  const int64_t per_panel = (int64_t)kNodes * 2 * d.M;
  const int pc = (int)(col / per_panel);
  const double xc = c.x[col], yc = c.y[col], zc = c.z[col];
  const double wc = density ? c.wq[col] * c.jac[col] : c.wq[col];
  const int64_t r0 = blockIdx.y * (int64_t)kFarRows;
  for (int rr = 0; rr < kFarRows; ++rr) {
    const int64_t r = r0 + rr;
    if (r >= d.N) break;
    const int pr = (int)(r / per_panel);
    if (abs(pr - pc) <= 1) continue;
    const double dx = xc - c.x[r], dy = yc - c.y[r], dz = zc - c.z[r];
    const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
    const double ri = rsqrt_refined(r2);             // far points are distinct: r2 > 0
    const double rho = r2 * ri;
    const double f = wc * ri;
    double s, co;
    sincos_bounded(k * rho, &s, &co);
    // S is written once here and not read back by this pass: streaming stores
    const dbl2 v = {f * co, f * s};
    __builtin_nontemporal_store(v, reinterpret_cast<dbl2*>(S + r * ld + col));
  }
}

// Far blocks of K (ADJ = false: tau_0 = nu_c . (x_c - x_r)) or K' (ADJ = true:
// tau_0 = nu_r . (x_r - x_c)), the integrand of Sec. 4 times the product weight;
// the same row walk and streaming stores as far_kernel.
template <bool ADJ>
__global__ __launch_bounds__(256) void far_kernel_dl(SysDims d, double k, Colloc c,
                                                     cplx* __restrict__ S, int64_t ld, int density) {
  const int64_t col = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (col >= d.N) return;
  const int64_t per_panel = (int64_t)kNodes * 2 * d.M;
  const int pc = (int)(col / per_panel);
  const double xc = c.x[col], yc = c.y[col], zc = c.z[col];
  const double wc = density ? c.wq[col] * c.jac[col] : c.wq[col];
  double ncx = 0.0, ncy = 0.0, ncz = 0.0;
  if (!ADJ) { ncx = c.nx[col]; ncy = c.ny[col]; ncz = c.nz[col]; }
  const int64_t r0 = blockIdx.y * (int64_t)kFarRows;
  for (int rr = 0; rr < kFarRows; ++rr) {
    const int64_t r = r0 + rr;
    if (r >= d.N) break;
    const int pr = (int)(r / per_panel);
    if (abs(pr - pc) <= 1) continue;
    const double dx = xc - c.x[r], dy = yc - c.y[r], dz = zc - c.z[r];
    const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
    const double ri = rsqrt_refined(r2);
    const double rho = r2 * ri;
    const double tau = ADJ ? -fma(c.nx[r], dx, fma(c.ny[r], dy, c.nz[r] * dz))
                           : fma(ncx, dx, fma(ncy, dy, ncz * dz));
    const double f = wc * tau * ri * ri * ri;
    const double x = k * rho;
    double s, co;
    sincos_bounded(x, &s, &co);
    // (ik rho - 1) e^{ik rho} = -(cos x + x sin x) + i (x cos x - sin x)
    const dbl2 v = {-f * fma(x, s, co), f * fma(x, co, -s)};
    __builtin_nontemporal_store(v, reinterpret_cast<dbl2*>(S + r * ld + col));
  }
}

__global__ __launch_bounds__(256) void diag_shift_kernel(SysDims d, double shift, Colloc c,
                                                         cplx* __restrict__ S, int64_t ld, int density) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= d.N) return;
  S[r * ld + r].re += density ? shift : shift / c.jac[r];
}

// Inverse DFT size NF = 2M of G sequences held in LDS (positive exponent,
// radix-2 Stockham); on return `src` holds the transforms.
__device__ void block_ifft(cplx*& src, cplx*& dst, int G, int NF, int M, const double* tab) {
  const int half = NF >> 1;
  const int mask = 8 * M - 1, quarter = 2 * M;
  for (int Ns = 1; Ns < NF; Ns <<= 1) {
    for (int b = threadIdx.x; b < G * half; b += blockDim.x) {
      const int s = b / half;
      const int jj = b - s * half;
      const int r = jj & (Ns - 1);
      const int tk = r * ((4 * M) / Ns);                 // angle pi r / Ns
      const cplx wt = mk(tab[(tk + quarter) & mask], tab[tk & mask]);
      const int idxD = ((jj - r) << 1) + r;
      const cplx* in = src + s * NF;
      cplx* out = dst + s * NF;
      const cplx v0 = in[jj], v1 = in[jj + half] * wt;
      out[idxD] = v0 + v1;
      out[idxD + Ns] = v0 - v1;
    }
    __syncthreads();
    cplx* tmp = src;
    src = dst;
    dst = tmp;
  }
}

__global__ __launch_bounds__(256) void near_kernel(SysDims d, NearChunk ch,
                                                   const cplx* __restrict__ kappa,
                                                   const double* __restrict__ wl,
                                                   const double* __restrict__ tab_g,
                                                   const double* __restrict__ colscale,
                                                   cplx* __restrict__ S, int64_t ld, int G) {
  extern __shared__ double lds[];
  const int M = d.M, NF = 2 * M;
  const int64_t tgt = blockIdx.x / 3;
  const int slot = blockIdx.x % 3;
  const int j = (int)(tgt % NF);
  const int l = (int)((tgt / NF) % kNodes);
  const int i = ch.p0 + (int)(tgt / ((int64_t)NF * kNodes));
  const int nrel = near_relations(i, d.n_panels);
  if (slot >= nrel) return;                          // uniform over the block
  const int rel = (i > 0) ? slot - 1 : slot;
  const int64_t p0 = near_pairs_before(i, d) - ch.pair_base +
                     (((int64_t)l * NF + j) * nrel + slot) * kNodes;
  const cplx* krow = kappa + p0 * NF;                // 16 rows of NF coefficients
  const double* W = wl + (size_t)(l * 3 + rel + 1) * kNodes * kNodes;   // [q][l']

  double* tab = lds;                                 // 8M doubles
  double* w_s = tab + 8 * M;                         // 256 doubles
  cplx* bufA = reinterpret_cast<cplx*>(w_s + kNodes * kNodes);
  cplx* bufB = bufA + G * NF;
  for (int x = threadIdx.x; x < 8 * M; x += blockDim.x) tab[x] = tab_g[x];
  for (int x = threadIdx.x; x < kNodes * kNodes; x += blockDim.x) w_s[x] = W[x];
  __syncthreads();

  const int64_t row = ((int64_t)i * kNodes + l) * NF + j;
  cplx* srow = S + row * ld + (int64_t)(i + rel) * kNodes * NF;
  const double* cs = colscale ? colscale + (int64_t)(i + rel) * kNodes * NF : nullptr;
  for (int g0 = 0; g0 < kNodes; g0 += G) {
    // contract over the rule nodes, store in natural frequency order
    for (int x = threadIdx.x; x < G * NF; x += blockDim.x) {
      const int s = x / NF;
      const int col = x - s * NF;                    // n = col - M + 1
      const int lp = g0 + s;
      cplx acc = mk(0.0, 0.0);
#pragma unroll 4
      for (int q = 0; q < kNodes; ++q) {
        const cplx kv = krow[q * NF + col];
        const double wv = w_s[q * kNodes + lp];
        acc.re = fma(wv, kv.re, acc.re);
        acc.im = fma(wv, kv.im, acc.im);
      }
      bufA[s * NF + ((col - M + 1 + NF) & (NF - 1))] = acc;
    }
    __syncthreads();
    cplx* src = bufA;
    cplx* dst = bufB;
    block_ifft(src, dst, G, NF, M, tab);
    for (int x = threadIdx.x; x < G * NF; x += blockDim.x) {
      const int s = x / NF;
      const int jp = x - s * NF;
      const int64_t cc = (int64_t)(g0 + s) * NF + jp;
      srow[cc] = cs ? cs[cc] * src[s * NF + jp] : src[s * NF + jp];
    }
    __syncthreads();
  }
}

// The same near block for N_F = 128 (M = 64).  The contraction gives each
// thread one column and 8 of the 16 rows, so a coefficient is read from memory
// by two threads instead of by one per row; the inverse DFT of each row,
// w_j' = sum_n c_n e^{+2 pi i n j' / 128} = conj(FFT(conj(c)))_j', is done by one
// wavefront in registers (fft128_regs), whose result goes straight to S.  The
// twiddles come from the angle table in global memory (no LDS copy of it).
__global__ __launch_bounds__(256) void near_kernel128(SysDims d, NearChunk ch,
                                                      const cplx* __restrict__ kappa,
                                                      const double* __restrict__ wl,
                                                      const double* __restrict__ tab_g,
                                                      const double* __restrict__ colscale,
                                                      cplx* __restrict__ S, int64_t ld) {
  constexpr int NF = 128;
  __shared__ double w_s[kNodes * kNodes];
  __shared__ cplx tw[7 * 64];
  __shared__ cplx buf[kNodes * NF];
  const int M = d.M;
  const int64_t tgt = blockIdx.x / 3;
  const int slot = blockIdx.x % 3;
  const int j = (int)(tgt % NF);
  const int l = (int)((tgt / NF) % kNodes);
  const int i = ch.p0 + (int)(tgt / ((int64_t)NF * kNodes));
  const int nrel = near_relations(i, d.n_panels);
  if (slot >= nrel) return;                          // uniform over the block
  const int rel = (i > 0) ? slot - 1 : slot;
  const int64_t p0 = near_pairs_before(i, d) - ch.pair_base +
                     (((int64_t)l * NF + j) * nrel + slot) * kNodes;
  const cplx* krow = kappa + p0 * NF;                // 16 rows of NF coefficients
  const double* W = wl + (size_t)(l * 3 + rel + 1) * kNodes * kNodes;   // [q][l']
  const int mask = 8 * M - 1, quarter = 2 * M;
  for (int x = threadIdx.x; x < kNodes * kNodes; x += blockDim.x) w_s[x] = W[x];
  for (int x = threadIdx.x; x < 7 * 64; x += blockDim.x) {
    const int tk = fft128_twiddle_k(x >> 6, x & 63) * ((8 * M) / NF);
    tw[x] = mk(tab_g[(tk + quarter) & mask], -tab_g[tk & mask]);
  }
  __syncthreads();

  // contraction over the rule nodes, into natural frequency order
  const int col = threadIdx.x & (NF - 1), s0 = (threadIdx.x >> 7) * 8;
  cplx acc[8];
#pragma unroll
  for (int r = 0; r < 8; ++r) acc[r] = mk(0.0, 0.0);
#pragma unroll 4
  for (int q = 0; q < kNodes; ++q) {
    const cplx kv = krow[q * NF + col];
#pragma unroll
    for (int r = 0; r < 8; ++r) {
      const double wv = w_s[q * kNodes + s0 + r];
      acc[r].re = fma(wv, kv.re, acc[r].re);
      acc[r].im = fma(wv, kv.im, acc[r].im);
    }
  }
  const int pos = (col - M + 1 + NF) & (NF - 1);
#pragma unroll
  for (int r = 0; r < 8; ++r) buf[(s0 + r) * NF + pos] = acc[r];
  __syncthreads();

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int q0 = (int)(__builtin_bitreverse32((unsigned)lane) >> 25);
  const int o = fft128_out_index(lane);
  const int64_t row = ((int64_t)i * kNodes + l) * NF + j;
  cplx* srow = S + row * ld + (int64_t)(i + rel) * kNodes * NF;
  const double* cs = colscale ? colscale + (int64_t)(i + rel) * kNodes * NF : nullptr;
  for (int s = wave; s < kNodes; s += 4) {
    cplx x0 = conj(buf[s * NF + q0]), x1 = conj(buf[s * NF + q0 + 1]);
    fft128_regs(x0, x1, tw, lane);
    const int64_t c0 = (int64_t)s * NF + o;
    srow[c0] = cs ? cs[c0] * conj(x0) : conj(x0);
    srow[c0 + 64] = cs ? cs[c0 + 64] * conj(x1) : conj(x1);
  }
}

__global__ __launch_bounds__(256) void rhs_kernel(SysDims d, double k, int kind, double p0,
                                                  double p1, double p2, Colloc c, cplx* g) {
  const int64_t r = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (r >= d.N) return;
  if (kind == FFBIE_RHS_POINT_SOURCE) {
    const double dx = c.x[r] - p0, dy = c.y[r] - p1, dz = c.z[r] - p2;
    const double rho = sqrt(fma(dx, dx, fma(dy, dy, dz * dz)));
    double s, co;
    sincos_bounded(k * rho, &s, &co);
    const double f = 1.0 / (4.0 * M_PI * rho);
    g[r] = mk(f * co, f * s);
  } else if (kind == FFBIE_RHS_PLANE_WAVE) {
    const double ph = k * (p0 * c.x[r] + p1 * c.y[r] + p2 * c.z[r]);
    double s, co;
    sincos_bounded(ph, &s, &co);
    g[r] = mk(-co, -s);
  } else if (kind == FFBIE_RHS_POINT_SOURCE_DN) {
    // d/d nu G(x; p) = e^{ik rho} (ik rho - 1) / (4 pi rho^2) * ((x - p) . nu) / rho
    const double dx = c.x[r] - p0, dy = c.y[r] - p1, dz = c.z[r] - p2;
    const double rho = sqrt(fma(dx, dx, fma(dy, dy, dz * dz)));
    double s, co;
    sincos_bounded(k * rho, &s, &co);
    const double dn = fma(dx, c.nx[r], fma(dy, c.ny[r], dz * c.nz[r])) / rho;
    const double f = dn / (4.0 * M_PI * rho * rho);
    const double kr = k * rho;
    g[r] = mk(f * (-co - kr * s), f * fma(kr, co, -s));
  } else {
    // -d/d nu e^{ik d.x} = -ik (d . nu) e^{ik d.x}
    const double ph = k * (p0 * c.x[r] + p1 * c.y[r] + p2 * c.z[r]);
    const double dn = k * (p0 * c.nx[r] + p1 * c.ny[r] + p2 * c.nz[r]);
    double s, co;
    sincos_bounded(ph, &s, &co);
    g[r] = mk(dn * s, -dn * co);
  }
}

__global__ __launch_bounds__(256) void field_partial_kernel(SysDims d, double k, Colloc c,
                                                            const double* __restrict__ pts,
                                                            const cplx* __restrict__ phi,
                                                            cplx* partial, int n_chunks, int density) {
  __shared__ double red[2][256];
  const int64_t p = blockIdx.y;
  const int chunk = blockIdx.x;
  const int64_t per = (d.N + n_chunks - 1) / n_chunks;
  const int64_t c0 = chunk * per;
  const int64_t c1 = min(d.N, c0 + per);
  const double px = pts[3 * p], py = pts[3 * p + 1], pz = pts[3 * p + 2];
  double ar = 0.0, ai = 0.0;
  for (int64_t s = c0 + threadIdx.x; s < c1; s += blockDim.x) {
    const double dx = c.x[s] - px, dy = c.y[s] - py, dz = c.z[s] - pz;
    const double rho = sqrt(fma(dx, dx, fma(dy, dy, dz * dz)));
    double sn, cs;
    sincos_bounded(k * rho, &sn, &cs);
    const double f = (density ? c.wq[s] * c.jac[s] : c.wq[s]) / rho;
    const cplx v = mk(f * cs, f * sn) * phi[s];
    ar += v.re;
    ai += v.im;
  }
  red[0][threadIdx.x] = ar;
  red[1][threadIdx.x] = ai;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      red[0][threadIdx.x] += red[0][threadIdx.x + w];
      red[1][threadIdx.x] += red[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[p * n_chunks + chunk] = mk(red[0][0], red[1][0]);
}

// Partial sums of the double-layer field, sum_s wq tau_0 (ik rho - 1) e^{ik rho} / rho^3 psi_s,
// tau_0 = nu_s . (x_s - p), with field_partial_kernel's fixed-order reduction.
__global__ __launch_bounds__(256) void field_partial_dl_kernel(SysDims d, double k, Colloc c,
                                                               const double* __restrict__ pts,
                                                               const cplx* __restrict__ psi,
                                                               cplx* partial, int n_chunks, int density) {
  __shared__ double red[2][256];
  const int64_t p = blockIdx.y;
  const int chunk = blockIdx.x;
  const int64_t per = (d.N + n_chunks - 1) / n_chunks;
  const int64_t c0 = chunk * per;
  const int64_t c1 = min(d.N, c0 + per);
  const double px = pts[3 * p], py = pts[3 * p + 1], pz = pts[3 * p + 2];
  double ar = 0.0, ai = 0.0;
  for (int64_t s = c0 + threadIdx.x; s < c1; s += blockDim.x) {
    const double dx = c.x[s] - px, dy = c.y[s] - py, dz = c.z[s] - pz;
    const double r2 = fma(dx, dx, fma(dy, dy, dz * dz));
    const double rho = sqrt(r2);
    const double tau = fma(c.nx[s], dx, fma(c.ny[s], dy, c.nz[s] * dz));
    const double x = k * rho;
    double sn, cs;
    sincos_bounded(x, &sn, &cs);
    const double f = (density ? c.wq[s] * c.jac[s] : c.wq[s]) * tau / (r2 * rho);
    const cplx v = mk(-f * fma(x, sn, cs), f * fma(x, cs, -sn)) * psi[s];
    ar += v.re;
    ai += v.im;
  }
  red[0][threadIdx.x] = ar;
  red[1][threadIdx.x] = ai;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) {
      red[0][threadIdx.x] += red[0][threadIdx.x + w];
      red[1][threadIdx.x] += red[1][threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) partial[p * n_chunks + chunk] = mk(red[0][0], red[1][0]);
}

__global__ void field_sum_kernel(int64_t n_pts, int n_chunks, const cplx* partial, cplx* u) {
  const int64_t p = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (p >= n_pts) return;
  cplx acc = mk(0.0, 0.0);
  for (int c = 0; c < n_chunks; ++c) acc = acc + partial[p * n_chunks + c];
  u[p] = acc;
}

GL16 pack_gl(const double* x, const double* w) {
  GL16 g;
  for (int i = 0; i < kNodes; ++i) {
    g.x[i] = x[i];
    g.w[i] = w[i];
  }
  return g;
}

}  // namespace

// Counts of per-pair status flags over n pairs: counts[0] += pairs with
// FFBIE_PAIR_UNRESOLVED, counts[1] += pairs with FFBIE_PAIR_ROOT_FALLBACK
// (wavefront sums, one atomic per wavefront and counter).
__global__ __launch_bounds__(256) void count_status_kernel(const int32_t* __restrict__ st, int64_t n,
                                                           unsigned long long* counts) {
  unsigned long long u = 0, f = 0;
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t v = st[i];
    u += (v & FFBIE_PAIR_UNRESOLVED) ? 1 : 0;
    f += (v & FFBIE_PAIR_ROOT_FALLBACK) ? 1 : 0;
  }
  for (int o = 32; o > 0; o >>= 1) {
    u += __shfl_xor(u, o);
    f += __shfl_xor(f, o);
  }
  if ((threadIdx.x & 63) == 0) {
    if (u) atomicAdd(counts, u);
    if (f) atomicAdd(counts + 1, f);
  }
}

__global__ void zero_counts_kernel(unsigned long long* counts, int n) {
  if ((int)threadIdx.x < n) counts[threadIdx.x] = 0;
}

hipError_t launch_collocation(const Geom& g, const SysDims& d, const double* gl_x,
                              const double* gl_w, Colloc c, double* xyz, double* jac,
                              double* wq, hipStream_t s) {
  const int64_t blocks = (d.N + 255) / 256;
  hipLaunchKernelGGL(collocation_kernel, dim3((unsigned)blocks), dim3(256), 0, s, g, d,
                     pack_gl(gl_x, gl_w), c, xyz, jac, wq);
  return hipGetLastError();
}

hipError_t launch_near_pairs(const SysDims& d, const NearChunk& ch, const double* gl_x,
                             const double* rule_y, double* t, int32_t* az, double* ts,
                             hipStream_t s) {
  const int64_t n = (int64_t)(ch.p1 - ch.p0) * kNodes * 2 * d.M * 3 * kNodes;
  const int64_t blocks = (n + 255) / 256;
  double zero[kNodes] = {0};
  hipLaunchKernelGGL(near_pairs_kernel, dim3((unsigned)blocks), dim3(256), 0, s, d, ch,
                     pack_gl(gl_x, zero), rule_y, t, az, ts);
  return hipGetLastError();
}

hipError_t launch_far_assembly(const SysDims& d, double k, Colloc c, cplx* S, int64_t ld,
                               hipStream_t s, int density) {
  const dim3 grid((unsigned)((d.N + 255) / 256), (unsigned)((d.N + kFarRows - 1) / kFarRows));
  hipLaunchKernelGGL(far_kernel, grid, dim3(256), 0, s, d, k, c, S, ld, density);
  return hipGetLastError();
}

int near_group(int M) {
  const int NF = 2 * M;
  int G = 1024 / NF;                                 // 2 G NF complex = 32 KiB
  if (G > kNodes) G = kNodes;
  if (G < 1) G = 1;
  return G;
}

hipError_t launch_near_assembly(const SysDims& d, const NearChunk& ch, const cplx* kappa,
                                const double* wl, const double* tab, cplx* S, int64_t ld,
                                hipStream_t s, const double* colscale) {
  const int G = near_group(d.M);
  const int NF = 2 * d.M;
  const size_t lds = sizeof(double) * (8 * d.M + kNodes * kNodes) + sizeof(cplx) * 2 * G * NF;
  const int64_t blocks = (int64_t)(ch.p1 - ch.p0) * kNodes * NF * 3;
  if (NF == 128) {
    hipLaunchKernelGGL(near_kernel128, dim3((unsigned)blocks), dim3(256), 0, s, d, ch, kappa, wl, tab,
                       colscale, S, ld);
    return hipGetLastError();
  }
  hipLaunchKernelGGL(near_kernel, dim3((unsigned)blocks), dim3(256), lds, s, d, ch, kappa, wl, tab,
                     colscale, S, ld, G);
  return hipGetLastError();
}

hipError_t launch_rhs(const SysDims& d, double k, int kind, const double* p, Colloc c, cplx* g,
                      hipStream_t s) {
  const int64_t blocks = (d.N + 255) / 256;
  hipLaunchKernelGGL(rhs_kernel, dim3((unsigned)blocks), dim3(256), 0, s, d, k, kind, p[0], p[1],
                     p[2], c, g);
  return hipGetLastError();
}

hipError_t launch_field(const SysDims& d, double k, Colloc c, int64_t n_pts, const double* pts,
                        const cplx* phi, cplx* partial, int n_chunks, cplx* u, hipStream_t s,
                        int density) {
  hipLaunchKernelGGL(field_partial_kernel, dim3(n_chunks, (unsigned)n_pts), dim3(256), 0, s, d, k,
                     c, pts, phi, partial, n_chunks, density);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(field_sum_kernel, dim3((unsigned)((n_pts + 255) / 256)), dim3(256), 0, s,
                     n_pts, n_chunks, partial, u);
  return hipGetLastError();
}

hipError_t launch_far_assembly_dl(const SysDims& d, double k, Colloc c, int adjoint, cplx* S,
                                  int64_t ld, hipStream_t s, int density) {
  const dim3 grid((unsigned)((d.N + 255) / 256), (unsigned)((d.N + kFarRows - 1) / kFarRows));
  if (adjoint)
    hipLaunchKernelGGL(far_kernel_dl<true>, grid, dim3(256), 0, s, d, k, c, S, ld, density);
  else
    hipLaunchKernelGGL(far_kernel_dl<false>, grid, dim3(256), 0, s, d, k, c, S, ld, density);
  return hipGetLastError();
}

hipError_t launch_diag_shift(const SysDims& d, double shift, Colloc c, cplx* S, int64_t ld,
                             hipStream_t s, int density) {
  hipLaunchKernelGGL(diag_shift_kernel, dim3((unsigned)((d.N + 255) / 256)), dim3(256), 0, s, d,
                     shift, c, S, ld, density);
  return hipGetLastError();
}

hipError_t launch_field_dl(const SysDims& d, double k, Colloc c, int64_t n_pts, const double* pts,
                           const cplx* psi, cplx* partial, int n_chunks, cplx* u, hipStream_t s,
                           int density) {
  hipLaunchKernelGGL(field_partial_dl_kernel, dim3(n_chunks, (unsigned)n_pts), dim3(256), 0, s, d, k,
                     c, pts, psi, partial, n_chunks, density);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(field_sum_kernel, dim3((unsigned)((n_pts + 255) / 256)), dim3(256), 0, s,
                     n_pts, n_chunks, partial, u);
  return hipGetLastError();
}

hipError_t launch_count_status(const int32_t* st, int64_t n, unsigned long long* counts,
                               hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(count_status_kernel, dim3((unsigned)blocks), dim3(256), 0, s, st, n, counts);
  return hipGetLastError();
}

hipError_t launch_zero_counts(unsigned long long* counts, int n, hipStream_t s) {
  hipLaunchKernelGGL(zero_counts_kernel, dim3(1), dim3(64), 0, s, counts, n);
  return hipGetLastError();
}

}  // namespace ffbie
