"""The O(M) banded route to <rho^-1>_l (Sec. 3.2.1), written from its
definition.  TEST INFRASTRUCTURE ONLY.

For a pair (target r(t, theta), source curve t_s != t) Lemma 3.3 states, for
every integer m,
    sum_n (2m + n) <rho^2>_n <rho^-1>_{-(m+n)} = 0                   (3.11)
and rho^2 is a trigonometric polynomial in theta_s, so the sum is finite.  With
m0 the truncation index of eq. (3.13), m = -(i + m0) and n = m0 - j it becomes
the (2 m0 + 1)-term difference equation of eq. (3.14),
    sum_{j=0}^{2 m0} a_j(i) <rho^-1>_{i+j} = 0,   i = 0 .. M1,
    a_j(i) = (m0 + 2i + j) <rho^2>_{m0-j}                              (3.15)
with M1 = L - 2 m0, L = M + M0.  The first m0 and the last m0 coefficients
(eq. (3.16)) are taken as known -- here from the direct quadrature of their
definition, ``coeffs.pair_coeffs`` -- and the M1 + 1 others,
x = [<rho^-1>_{m0} .. <rho^-1>_{L-m0}] (eq. (3.18)), solve the banded system
A x = b of eq. (3.17), A_{ic} = a_{c-i+m0}(i) for |c - i| <= m0.

Nothing here is blocked, factored by band or recurred: A is built entry by
entry and solved by a dense LU (numpy), b collects the known terms of each
equation.  <rho^2>_n comes from the n_fft-point trapezoidal rule, exact for a
trigonometric polynomial of degree < n_fft / 2 (the star family's rho^2 has
degree <= max(2 mmax, mmax + 1)), with <rho^2>_{-n} = conj <rho^2>_n since
rho^2 is real.
"""
import math

import numpy as np

from . import coeffs
from . import geometry as geo


def rho2_coeffs(amp, t, th, ts, n_max, n_fft=64):
    """<rho^2>_n (Sec. 3.2 convention, source azimuth theta_s absolute) for
    n = 0 .. n_max of the pair (t, th, ts).  Needs n_max < n_fft / 2."""
    if not n_max < n_fft // 2:
        raise ValueError("n_max must be below n_fft / 2")
    x = 2.0 * math.pi * np.arange(n_fft) / n_fft           # theta_s
    r2 = geo.rho2(amp, t, th, ts, x - th)
    n = np.arange(n_max + 1)
    return (np.exp(-1j * np.outer(n, x)) @ r2) / n_fft


def degree_bound(amp):
    """Degree in theta_s of rho^2 for the star family: R(t_s, .) has degree
    mmax, rho^2 = R^2 + R_s^2 - 2 R R_s (sin t sin t_s cos(theta_s - theta)
    + cos t cos t_s).  Stretched by D = diag(d) with d_x != d_y, the term
    R_s^2 (d_x^2 cos^2 theta_s + d_y^2 sin^2 theta_s) sin^2 t_s keeps its
    cos(2 theta_s) part: degree 2 mmax + 2."""
    a = geo.as_amp(amp)
    d = geo.axes_of(amp)
    mmax = max([m for m in range(a.shape[1]) if np.any(a[:, m] != 0.0)], default=0) if a.size else 0
    if d[0] != d[1]:
        return 2 * mmax + 2
    return max(2 * mmax, mmax + 1)


def choose_m0(c2_rows, eps0=1e-14, degree=None):
    """Eq. (3.13) over a set of pairs: the smallest m0 >= 1 such that every
    pair's |<rho^2>_n| / max_n |<rho^2>_n| is at most eps0 for all |n| > m0.
    Read together with Remark 3.5, which gives m0 = 1 for an axisymmetric
    surface, where <rho^2>_{+-1} is not small and every |n| >= 2 vanishes.
    c2_rows: [pairs][n_max + 1], n >= 0, with n_max above the degree of rho^2.
    ``degree``, when given, caps m0: coefficients above the degree of the
    trigonometric polynomial rho^2 vanish identically, and only the rounding
    of the sampled transform (about 1e-16 of the sample values, which near the
    poles exceeds eps0 times a small <rho^2>_0) would be seen there."""
    c2 = np.abs(np.atleast_2d(np.asarray(c2_rows)))
    ratio = c2 / np.max(c2, axis=1, keepdims=True)
    worst = np.max(ratio, axis=0)                            # over pairs, per n
    big = np.nonzero(worst > eps0)[0]
    m0 = int(max(1, big.max())) if big.size else 1
    return min(m0, degree) if degree is not None else m0


def full_c2(c2, m0):
    """<rho^2>_n for n = -m0..m0 as a dict, from n >= 0 and conjugate symmetry;
    zero beyond the given rows."""
    out = {}
    for n in range(-m0, m0 + 1):
        v = c2[abs(n)] if abs(n) < len(c2) else 0.0
        out[n] = v if n >= 0 else np.conj(v)
    return out


def coefficient(c2f, m0, i, j):
    """a_j(i) of eq. (3.15)."""
    return (m0 + 2 * i + j) * c2f[m0 - j]


def system(c2, m0, L, known):
    """A and b of eq. (3.17).  ``known`` maps the indices of eq. (3.16)
    (0..m0-1 and L-m0+1..L) to <rho^-1> values."""
    M1 = L - 2 * m0
    if M1 < 0:
        raise ValueError("L must be at least 2 m0")
    c2f = full_c2(c2, m0)
    A = np.zeros((M1 + 1, M1 + 1), dtype=complex)
    b = np.zeros(M1 + 1, dtype=complex)
    for i in range(M1 + 1):
        for j in range(2 * m0 + 1):
            l = i + j                                        # <rho^-1>_l in equation i
            a = coefficient(c2f, m0, i, j)
            if m0 <= l <= L - m0:
                A[i, l - m0] += a
            else:
                b[i] -= a * known[l]
    return A, b


def rhoinv_banded(amp, M, M0, t, j_az, ts, m0, k=1.0, known=None):
    """<rho^-1>_l, l = 0..M+M0, of one pair by the banded system of Sec. 3.2.1.

    The 2 m0 known coefficients of eq. (3.16) come from ``known`` (a dict
    index -> value) or, by default, from the direct quadrature
    ``coeffs.pair_coeffs``.  Returns (c, info) with info holding A, b, the
    direct-quadrature row used for the known values (or None) and <rho^2>_n."""
    L = M + M0
    th = math.pi * j_az / M
    c2 = rho2_coeffs(amp, t, th, ts, m0)
    direct = None
    if known is None:
        direct, _, _ = coeffs.pair_coeffs(amp, k, M, L, t, j_az, ts)
        known = {l: direct[l] for l in list(range(m0)) + list(range(L - m0 + 1, L + 1))}
    A, b = system(c2, m0, L, known)
    x = np.linalg.solve(A, b)
    c = np.zeros(L + 1, dtype=complex)
    for l, v in known.items():
        c[l] = v
    c[m0:L - m0 + 1] = x
    return c, dict(A=A, b=b, direct=direct, c2=c2)


def positive_definite_condition(c2):
    """The sufficient condition of Lemma 3.4, eq. (3.19):
    2 <rho^2>_0 > sum_l |<rho^2>_l| (both signs of l)."""
    c2 = np.asarray(c2)
    return 2.0 * c2[0].real > abs(c2[0]) + 2.0 * np.sum(np.abs(c2[1:]))
