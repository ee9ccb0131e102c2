"""Azimuthal Fourier coefficients of the singular kernels by direct quadrature.

Definitions (Sec. 3.2): for a 2*pi-periodic f,
    <f>_m = (1/2pi) int_0^{2pi} f(theta_s) e^{-i m theta_s} d theta_s.
For a target r(t, theta) and a source curve t_s != t the path needs
    c_l     = <rho^-1>_l,          l = 0 .. L      (L = M + M0; eq. (3.10))
    kappa_n = <e^{ik rho}/rho>_n,  n = -M+1 .. M   (the indices -m, m in
                                                    [-M, M-1], of eq. (3.9))
This module evaluates those integrals *as defined*, with no singularity
swapping, no FFT and no truncated convolution: a composite Gauss-Legendre
rule on [a* - pi, a* + pi], graded dyadically towards the real minimiser a*
of rho^2 where the integrand is nearly singular, with every sub-interval short
enough to resolve e^{-i l theta_s}.  Two independent rules (24 and 32 nodes,
different grading depth and interval length) are compared; the result of the
finer one is returned together with the observed difference.

Target azimuths lie on the grid theta_j = pi j / M of eq. (3.8).
Test infrastructure only.
"""
import math

import numpy as np

from . import geometry as geo

_GL = {}


def _gl(n):
    if n not in _GL:
        _GL[n] = np.polynomial.legendre.leggauss(n)
    return _GL[n]


def graded_rule(center, beta, hmax, n, j0):
    """Composite n-point GL rule on [center - pi, center + pi].

    Breakpoints at center, center +- beta 2^j for j >= j0 (while < pi), then
    every interval longer than ``hmax`` is split evenly.
    """
    pts = [center - math.pi, center, center + math.pi]
    j = j0
    while beta * 2.0 ** j < math.pi:
        h = beta * 2.0 ** j
        pts += [center - h, center + h]
        j += 1
    pts = np.unique(np.array(pts))
    edges = [pts[0]]
    for a, b in zip(pts[:-1], pts[1:]):
        k = max(1, int(math.ceil((b - a) / hmax)))
        edges.extend(a + (b - a) * np.arange(1, k + 1) / k)
    edges = np.array(edges)
    x, w = _gl(n)
    lo, hi = edges[:-1], edges[1:]
    half = 0.5 * (hi - lo)
    nodes = (0.5 * (hi + lo))[:, None] + half[:, None] * x[None, :]
    weights = half[:, None] * w[None, :]
    return nodes.ravel(), weights.ravel()


def minimiser(amp, t, th, ts, n_scan=4096):
    """Real minimiser of theta_s -> rho^2, as an offset from the target azimuth.

    Grid scan, then Newton on d rho^2/d theta_s.  Returns (u*, rho^2, d^2 rho^2)
    with the minimiser at theta_s = th + u*.
    """
    grid = 2.0 * math.pi * np.arange(n_scan) / n_scan
    grid = np.where(grid > math.pi, grid - 2.0 * math.pi, grid)
    r2 = geo.rho2(amp, t, th, ts, grid)
    i = int(np.argmin(r2))
    u, h = grid[i], 2.0 * math.pi / n_scan
    lo, hi = u - h, u + h
    for _ in range(60):
        _, d1, d2 = geo.rho2_theta_derivs(amp, t, th, ts, u)
        if not d2 > 0:
            break
        u_new = min(max(u - d1 / d2, lo), hi)
        if abs(u_new - u) <= 1e-17 + 1e-16 * abs(u):
            u = u_new
            break
        u = u_new
    r2, _, d2 = geo.rho2_theta_derivs(amp, t, th, ts, u)
    return float(u), float(r2), float(d2)


def _moments(th, x, w, f, orders):
    """(1/2pi) sum_q w_q f_q e^{-i n (th + x_q)} for each n in ``orders``.

    The phase e^{-i n th} is applied as a separate factor so that the small
    offsets x_q are never rounded against th.
    """
    ph = np.exp(-1j * np.outer(orders, x))
    return np.exp(-1j * orders * th) * (ph @ (w * f)) / (2.0 * math.pi)


def pair_coeffs(amp, k, M, L, t, j_az, ts, rtol=1e-14):
    """c_l (l = 0..L) and kappa_n (n = -M+1..M) for one pair by quadrature.

    Parameters: amplitude table ``amp``, wavenumber ``k``, mode count ``M``,
    highest <rho^-1> index ``L``, target curve parameter ``t``, target azimuth
    index ``j_az`` (theta = pi j / M), source curve parameter ``ts``.
    Returns (c, kappa, info) with info = dict(a, beta, diff, converged), where
    a is the minimiser of rho^2 as an offset from theta.
    """
    if ts == t:
        raise ValueError("t_s == t: the coefficients diverge (b = 0)")
    th = math.pi * j_az / M
    u, r2min, d2 = minimiser(amp, t, th, ts)
    beta = math.sqrt(2.0 * r2min / d2) if d2 > 0 else 1.0
    freq = max(L, M) + 1.5 * k + 1.0
    ls = np.arange(L + 1)
    ns = np.arange(-M + 1, M + 1)
    results = []
    diff = math.inf
    for n, j0, hscale in ((24, -3, 1.0), (32, -5, 0.7), (40, -7, 0.5), (48, -9, 0.35)):
        hmax = min(12.0 / freq, math.pi / 8) * hscale
        x, w = graded_rule(u, beta, hmax, n, j0)
        rho = np.sqrt(geo.rho2(amp, t, th, ts, x))
        c = _moments(th, x, w, 1.0 / rho, ls)
        kap = _moments(th, x, w, np.exp(1j * k * rho) / rho, ns)
        results.append((c, kap))
        if len(results) >= 2:
            (c0, k0), (c1, k1) = results[-2], results[-1]
            diff = max(np.max(np.abs(c1 - c0)) / np.max(np.abs(c1)),
                       np.max(np.abs(k1 - k0)) / np.max(np.abs(k1)))
            if diff <= rtol:
                break
    c, kap = results[-1]
    return c, kap, dict(a=u, beta=beta, diff=float(diff), converged=bool(diff <= rtol))


def _one_thread():
    """Worker initializer: one BLAS thread per process (no oversubscription)."""
    try:
        from threadpoolctl import threadpool_limits
        threadpool_limits(1)
    except ImportError:
        pass


def pairs_coeffs(amp, k, M, L, t, j_az, ts, processes=None):
    """``pair_coeffs`` over arrays of pairs; optional multiprocessing pool.

    Returns (c [n, L+1], kappa [n, 2M], info list).
    """
    t = np.asarray(t, dtype=np.float64)
    j_az = np.asarray(j_az)
    ts = np.asarray(ts, dtype=np.float64)
    args = [(amp, k, M, L, float(t[i]), int(j_az[i]), float(ts[i])) for i in range(t.size)]
    if processes and processes > 1 and len(args) > 1:
        import multiprocessing as mp
        ctx = mp.get_context("fork")
        with ctx.Pool(processes, initializer=_one_thread) as pool:
            out = pool.starmap(pair_coeffs, args, chunksize=max(1, len(args) // (4 * processes)))
    else:
        out = [pair_coeffs(*a) for a in args]
    c = np.array([o[0] for o in out]).reshape(t.size, L + 1)
    kap = np.array([o[1] for o in out]).reshape(t.size, 2 * M)
    return c, kap, [o[2] for o in out]


def kappa_tail(amp, k, M, M0, t, j_az, ts, n_max=None):
    """Truncation tail of the cos(k rho) series in eq. (3.10) for one pair:
        sum_{|n| >= M0} |<cos k rho>_n| * max_l |<rho^-1>_l|,
    relative to max_n |kappa_n| (kappa_n, n = -M+1..M, by direct quadrature).
    A kernel-coefficient table built from 2M azimuthal samples cannot be more
    accurate than this for the pair; it tells resolved pairs (tail at rounding
    level) from those a given M cannot resolve (large k against M).

    cos(k rho) is an entire function of rho^2, a smooth periodic function of
    theta_s, so its coefficients come from the trapezoidal rule with many more
    points than the modes read (exponentially convergent), up to |n| <= n_max
    (default 8 max(M, k + 16)).  Returns (tail, info) with info the
    coefficient magnitudes |<cos k rho>_n| for n = -n_max..n_max."""
    c, kap, _ = pair_coeffs(amp, k, M, M + M0, t, j_az, ts)
    n_max = int(n_max or 8 * max(M, int(math.ceil(k)) + 16))
    th = math.pi * j_az / M
    Q = 4 * n_max + 4
    x = 2.0 * math.pi * np.arange(Q) / Q
    f = np.cos(k * np.sqrt(geo.rho2(amp, t, th, ts, x)))
    ns = np.arange(-n_max, n_max + 1)
    coef = (np.exp(-1j * np.outer(ns, x)) @ f) / Q * np.exp(-1j * ns * th)
    tail = np.sum(np.abs(coef[np.abs(ns) >= M0])) * np.max(np.abs(c)) / np.max(np.abs(kap))
    return float(tail), np.abs(coef)

