"""Singular-factor coefficients A_m(b) from their defining integral (oracle).

Eq. (3.26):  A_m(b) = <s_{0,b}^{-1/2}>_m
           = (1/2pi) int_0^{2pi} e^{-i m phi} (1 + e^{-2b} - 2 e^{-b} cos phi)^{-1/2} d phi,
with s_{a,b} the function of eq. (3.22).  The integrand is even in phi, so
A_m = (1/pi) int_0^pi cos(m phi) s^{-1/2} d phi.  s is evaluated as
(1 - e^{-b})^2 + 4 e^{-b} sin^2(phi/2), which is the same function written
without cancellation near phi = 0.  The quadrature is a composite
Gauss-Legendre rule graded dyadically towards phi = 0 on the scale b (where
the integrand is nearly singular for small b), with intervals short enough to
resolve cos(m phi).  Two rules are compared as in ``coeffs``.
Test infrastructure only.
"""
import math

import numpy as np

from .coeffs import _gl


def _rule(b, hmax, n, j0):
    pts = [0.0, math.pi]
    j = j0
    while b * 2.0 ** j < math.pi:
        pts.append(b * 2.0 ** j)
        j += 1
    pts = np.unique(np.array(pts))
    edges = [pts[0]]
    for lo, hi in zip(pts[:-1], pts[1:]):
        k = max(1, int(math.ceil((hi - lo) / hmax)))
        edges.extend(lo + (hi - lo) * np.arange(1, k + 1) / k)
    edges = np.array(edges)
    x, w = _gl(n)
    lo, hi = edges[:-1], edges[1:]
    half = 0.5 * (hi - lo)
    nodes = (0.5 * (hi + lo))[:, None] + half[:, None] * x[None, :]
    return nodes.ravel(), (half[:, None] * w[None, :]).ravel()


def singular_factor(b, m_max, rtol=1e-14):
    """A_m(b) for m = 0..m_max by quadrature of eq. (3.26); b > 0."""
    if not b > 0:
        raise ValueError("A_m(b) needs b > 0")
    q = math.exp(-b)
    one_minus_q = -math.expm1(-b)
    ms = np.arange(m_max + 1)
    prev = None
    for n, j0, hs in ((24, -3, 1.0), (32, -5, 0.7), (40, -7, 0.5)):
        hmax = min(12.0 / (m_max + 1), math.pi / 8) * hs
        x, w = _rule(b, hmax, n, j0)
        s = one_minus_q ** 2 + 4.0 * q * np.sin(0.5 * x) ** 2
        A = (np.cos(np.outer(ms, x)) @ (w / np.sqrt(s))) / math.pi
        if prev is not None and np.max(np.abs(A - prev)) <= rtol * A[0]:
            break
        prev = A
    return A
