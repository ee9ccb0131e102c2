"""Pins of the oracle's axis-stretched star surfaces (the ellipsoid of Sec. 5,
Example 1: x^2 + y^2/4 + z^2/9 = 1, the unit sphere stretched by (1, 2, 3)).

Each fact is independent of the oracle's arithmetic:
* the points satisfy the ellipsoid's implicit equation;
* the unit normal is the normalised gradient (x, y/4, z/9) of that equation,
  pointing outwards;
* the divergence theorem with the normals and Jacobians gives the volume
  4 pi abc / 3 = 8 pi;
* the cancellation-free difference matches 40-digit arithmetic;
* the coefficients <rho^-1>_l sum back to 1/rho, and their Lemma 3.3
  identity holds with <rho^2>_n of the stretched surface;
* a stretch with equal x and y axes keeps the surface axisymmetric, and the
  rotation relation of Remark 3.5 then holds for its coefficients.
"""
import math

import mpmath as mp
import numpy as np
import pytest

from oracle import banded as ob
from oracle import coeffs
from oracle import geometry as geo

ELL = geo.Scaled(None, (1.0, 2.0, 3.0))
ELL_STAR = geo.Scaled(np.array([[0.0, 0.2], [0.0, 0.1]]), (1.0, 1.5, 0.8))


def _grid(n=24):
    t = np.linspace(0.05, math.pi - 0.05, n)
    th = np.linspace(0.0, 2 * math.pi, n, endpoint=False) + 0.1
    return np.meshgrid(t, th, indexing="ij")


def test_ellipsoid_points_and_normals():
    T, TH = _grid()
    x = geo.point(ELL, T, TH)
    f = x[..., 0] ** 2 + x[..., 1] ** 2 / 4 + x[..., 2] ** 2 / 9
    assert np.max(np.abs(f - 1.0)) <= 1e-15 * 4
    grad = np.stack([x[..., 0], x[..., 1] / 4, x[..., 2] / 9], axis=-1)
    grad /= np.linalg.norm(grad, axis=-1, keepdims=True)
    nu = geo.normal(ELL, T, TH)
    assert np.max(np.abs(nu - grad)) <= 1e-14


@pytest.mark.parametrize("surface,volume", [(ELL, 8 * math.pi), (ELL_STAR, None)])
def test_divergence_theorem_volume(surface, volume):
    """(1/3) int r . nu J dt dtheta = 4 pi abc / 3 for the ellipsoid; for the
    stretched star, det(D) times the star's volume int R^3 sin t / 3."""
    x, w = np.polynomial.legendre.leggauss(64)
    t = 0.5 * math.pi * (x + 1)
    wt = 0.5 * math.pi * w
    th = 2 * math.pi * np.arange(64) / 64
    T, TH = np.meshgrid(t, th, indexing="ij")
    flux = np.einsum("...c,...c->...", geo.point(surface, T, TH), geo.normal(surface, T, TH))
    v = (wt[:, None] * flux * geo.jacobian(surface, T, TH)).sum() * (2 * math.pi / 64) / 3
    if volume is None:
        D = geo.axes_of(surface)
        volume = np.prod(D) * (wt[:, None] * geo.radius(surface, T, TH) ** 3 * np.sin(T)).sum() \
            * (2 * math.pi / 64) / 3
    assert abs(v - volume) <= 1e-13 * volume


def test_stretched_difference_matches_extended_precision():
    mp.mp.dps = 40
    a = geo.as_amp(ELL_STAR)
    D = [mp.mpf(v) for v in geo.axes_of(ELL_STAR)]

    def r_mp(t, th):
        R = 1 + sum(mp.mpf(a[l - 1, m]) * mp.sin(l * t) * mp.cos(m * th)
                    for l in range(1, a.shape[0] + 1) for m in range(a.shape[1]))
        return [D[0] * R * mp.sin(t) * mp.cos(th), D[1] * R * mp.sin(t) * mp.sin(th),
                D[2] * R * mp.cos(t)]

    t, th = 0.9, 2.3
    for dt, dth in [(1e-9, 2e-9), (-3e-6, 1e-7), (2e-3, -4e-3), (0.4, 2.0)]:
        d = geo.delta_r(ELL_STAR, t, th, t + dt, dth)
        ref = [x - y for x, y in zip(r_mp(mp.mpf(t + dt), mp.mpf(th) + mp.mpf(dth)),
                                     r_mp(mp.mpf(t), mp.mpf(th)))]
        nref = float(mp.sqrt(sum(v * v for v in ref)))
        err = math.sqrt(sum(float(d[c] - ref[c]) ** 2 for c in range(3)))
        assert err <= 8e-16 * nref, (dt, dth, err / nref)


@pytest.mark.parametrize("surface", [ELL, ELL_STAR])
def test_rhoinv_sums_back_and_lemma(surface):
    M, L = 32, 64
    t, ts, j = 0.8, 2.1, 9
    c, _, _ = coeffs.pair_coeffs(surface, 3.0, M, L, t, j, ts)
    th = math.pi * j / M
    xs = np.linspace(-3, 3, 13)
    l = np.arange(1, L + 1)
    series = c[0].real + 2 * np.real(np.exp(1j * np.outer(th + xs, l)) @ c[1:])
    direct = 1 / np.sqrt(geo.rho2(surface, t, th, ts, xs))
    assert np.max(np.abs(series - direct)) < 1e-13 * np.max(direct)
    # Lemma 3.3 with the stretched surface's <rho^2>_n (degree unchanged by D)
    m0 = ob.degree_bound(surface)
    c2 = ob.rho2_coeffs(surface, t, th, ts, m0)
    c2f = ob.full_c2(c2, m0)
    cf = {q: (c[q] if q >= 0 else np.conj(c[-q])) for q in range(-L, L + 1)}
    scale = sum(abs(v) for v in c2f.values()) * np.max(np.abs(c))
    for m in range(-L + m0, L - m0 + 1, 7):
        res = sum((2 * m + n) * c2f[n] * cf[-(m + n)] for n in range(-m0, m0 + 1))
        assert abs(res) <= 1e-14 * (2 * abs(m) + m0) * scale


def test_equal_xy_axes_keep_rotation_invariance():
    surface = geo.Scaled(None, (1.3, 1.3, 0.7))
    assert geo.is_axisymmetric(surface) and not geo.is_axisymmetric(ELL)
    M, L = 16, 32
    t, ts = 1.0, 1.3
    c0, _, _ = coeffs.pair_coeffs(surface, 1.0, M, L, t, 0, ts)
    c5, _, _ = coeffs.pair_coeffs(surface, 1.0, M, L, t, 5, ts)
    l = np.arange(L + 1)
    ref = c0 * np.exp(-1j * l * math.pi * 5 / M)
    assert np.max(np.abs(c5 - ref)) <= 1e-14 * np.max(np.abs(c0))
