"""Double-layer operator K and its adjoint K' (Sec. 4), from their definitions.
TEST INFRASTRUCTURE ONLY.

K[psi](r)  = 2 int dG(r; r_s)/d nu(r_s) psi(r_s) d sigma(r_s)   (eq. (2.13)),
K'[phi](r) = 2 int dG(r; r_s)/d nu(r)   phi(r_s) d sigma(r_s)   (eq. (2.10)),
with G(r; r_s) = e^{ik rho} / (4 pi rho), rho = |r - r_s|.  Since
dG/drho = (ik rho - 1) e^{ik rho} / (4 pi rho^2),

    2 dG/d nu(r_s) = tau_0 (ik rho - 1) e^{ik rho} / (2 pi rho^3),
    tau_0 = nu(r_s) . (r_s - r)                                    (K),
    tau_0 = nu(r) . (r - r_s)                                      (K'),

which is the integrand of Sec. 4, (alpha tau_1 - tau_3 - i beta tau_0) / (2 pi),
written back as one function.  The azimuthal coefficients the discretisation
needs (the K analogue of kappa in eq. (3.9)) are therefore

    kK_n(t, theta_j, t_s) = < tau_0 (ik rho - 1) e^{ik rho} / rho^3 >_n,  n = -M+1..M,

evaluated here *as defined*, by the graded composite Gauss-Legendre rule of
``coeffs`` (the integrand is O(1/rho) near the target, like rho^-1).  Nothing
here uses tau_1, tau_3, H_3, B_m, or translated swapping: those are what the
GPU path must reproduce.

tau_0 = O(rho^2) near the target: it is evaluated with the line integral of
the Remark in Sec. 4,
    nu(v) . (r(v) - r(u)) = int_0^1 (lam - 1) nu(v) . D^2 r(v + lam (u - v))[u - v, u - v] d lam,
(32-node Gauss-Legendre in lam) when the parameter points are close, and
directly otherwise.

``b3_coeffs`` gives B_m(0, b) = <s_{0,b}^{-3/2}>_m by quadrature (eq. (4.7)).
"""
import math

import numpy as np

from . import coeffs
from . import geometry as geo
from .special import _rule

_LAM = {}


def _gl01(n):
    if n not in _LAM:
        x, w = np.polynomial.legendre.leggauss(n)
        _LAM[n] = (0.5 * (x + 1.0), 0.5 * w)
    return _LAM[n]


def tau0(amp, t, th, ts, dth, adjoint=False, n_lambda=32, switch=0.5):
    """tau_0 at the source r(ts, th + dth) for the target r(t, th): for K
    nu(r_s) . (r_s - r), for K' (adjoint) nu(r) . (r - r_s).  Broadcasts."""
    t, th, ts, dth = np.broadcast_arrays(*(np.asarray(v, dtype=np.float64) for v in (t, th, ts, dth)))
    shape = t.shape
    t, th, ts, dth = (v.reshape(-1) for v in (t, th, ts, dth))
    w = geo.wrap(dth)
    d = geo.delta_r(amp, t, th, ts, dth)                     # r_s - r
    if adjoint:
        out = -np.einsum("...c,...c->...", geo.normal(amp, t, th), d)
    else:
        out = np.einsum("...c,...c->...", geo.normal(amp, ts, th + dth), d)
    near = (np.abs(t - ts) + np.abs(w)) < switch
    if np.any(near):
        lam, wl = _gl01(n_lambda)
        tn, thn, tsn, wn = t[near], th[near], ts[near], w[near]
        if adjoint:
            # v = target (t, th), u = source (ts, th + w): gamma = v + lam (u - v)
            dt, dh = tsn - tn, wn
            g_t = tn[:, None] + lam[None, :] * dt[:, None]
            g_th = thn[:, None] + lam[None, :] * dh[:, None]
            nu = geo.normal(amp, tn, thn)
        else:
            # v = source, u = target: u - v = (t - ts, -w)
            dt, dh = tn - tsn, -wn
            g_t = tsn[:, None] + lam[None, :] * dt[:, None]
            g_th = (thn + wn)[:, None] + lam[None, :] * dh[:, None]
            nu = geo.normal(amp, tsn, thn + wn)
        rtt, rtth, rthth = geo.second_derivs(amp, g_t, g_th)
        q = (rtt * (dt ** 2)[:, None, None] + 2.0 * rtth * (dt * dh)[:, None, None]
             + rthth * (dh ** 2)[:, None, None])                     # D^2 r [delta, delta]
        val = np.einsum("k,nkc,nc->n", (lam - 1.0) * wl, q, nu)
        out = np.array(out, dtype=np.float64)
        out[near] = val
    return np.asarray(out).reshape(shape)


def kernel_values(amp, k, t, th, ts, dth, adjoint=False):
    """tau_0 (ik rho - 1) e^{ik rho} / rho^3 at the source azimuths th + dth."""
    rho = np.sqrt(geo.rho2(amp, t, th, ts, dth))
    tz = tau0(amp, t, th, ts, dth, adjoint=adjoint)
    return tz * (1j * k * rho - 1.0) * np.exp(1j * k * rho) / rho ** 3


def pair_kcoeffs(amp, k, M, t, j_az, ts, adjoint=False, rtol=1e-13):
    """kK_n for n = -M+1..M of one pair (target r(t, pi j/M), source curve
    ts != t) by graded composite Gauss-Legendre quadrature.  Returns
    (kK, info) with the observed difference of successive rules."""
    if ts == t:
        raise ValueError("t_s == t: the coefficients diverge")
    th = math.pi * j_az / M
    u, r2min, d2 = coeffs.minimiser(amp, t, th, ts)
    beta = math.sqrt(2.0 * r2min / d2) if d2 > 0 else 1.0
    freq = M + 1.5 * k + 1.0
    ns = np.arange(-M + 1, M + 1)
    prev, diff = None, math.inf
    for n, j0, hscale in ((24, -3, 1.0), (32, -5, 0.7), (40, -7, 0.5), (48, -9, 0.35)):
        hmax = min(12.0 / freq, math.pi / 8) * hscale
        x, w = coeffs.graded_rule(u, beta, hmax, n, j0)
        f = kernel_values(amp, k, t, th, ts, x, adjoint=adjoint)
        cur = coeffs._moments(th, x, w, f, ns)
        if prev is not None:
            diff = np.max(np.abs(cur - prev)) / np.max(np.abs(cur))
            if diff <= rtol:
                break
        prev = cur
    return cur, dict(a=u, beta=beta, diff=float(diff), converged=bool(diff <= rtol))


def pairs_kcoeffs(amp, k, M, t, j_az, ts, adjoint=False, processes=None):
    """``pair_kcoeffs`` over arrays of pairs: ([n, 2M] complex, info list)."""
    t = np.asarray(t, dtype=np.float64)
    j_az = np.asarray(j_az)
    ts = np.asarray(ts, dtype=np.float64)
    args = [(amp, k, M, float(t[i]), int(j_az[i]), float(ts[i]), adjoint) for i in range(t.size)]
    if processes and processes > 1 and len(args) > 1:
        import multiprocessing as mp
        with mp.get_context("fork").Pool(processes, initializer=coeffs._one_thread) as pool:
            out = pool.starmap(pair_kcoeffs, args, chunksize=max(1, len(args) // (4 * processes)))
    else:
        out = [pair_kcoeffs(*a) for a in args]
    return np.array([o[0] for o in out]).reshape(t.size, 2 * M), [o[1] for o in out]


def b3_coeffs(b, m_max, rtol=1e-14):
    """B_m(0, b) = (1/2pi) int e^{-i m phi} s_{0,b}^{-3/2} d phi, m = 0..m_max
    (eq. (4.7)), by the graded rule of ``special`` (s^{-3/2} is even in phi)."""
    if not b > 0:
        raise ValueError("B_m(b) needs b > 0")
    q = math.exp(-b)
    omq = -math.expm1(-b)
    ms = np.arange(m_max + 1)
    prev = None
    for n, j0, hs in ((24, -3, 1.0), (32, -5, 0.7), (40, -7, 0.5), (48, -9, 0.35)):
        hmax = min(12.0 / (m_max + 1), math.pi / 8) * hs
        x, w = _rule(b, hmax, n, j0)
        s = omq ** 2 + 4.0 * q * np.sin(0.5 * x) ** 2
        B = (np.cos(np.outer(ms, x)) @ (w * s ** -1.5)) / math.pi
        if prev is not None and np.max(np.abs(B - prev)) <= rtol * B[0]:
            break
        prev = B
    return B
