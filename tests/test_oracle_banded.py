"""Pins of the oracle's O(M) banded route to <rho^-1>_l (Sec. 3.2.1).

Each fact is independent of the route's own arithmetic:
* <rho^2>_n: the unit sphere's closed form, and the series summed back to
  rho^2 at arbitrary source azimuths for non-axisymmetric stars (normalisation,
  phase and sign of the index); the coefficients vanish above the degree bound;
* the m0 rule of eq. (3.13): 1 for the sphere (Remark 3.5), the degree of
  rho^2 for the stars;
* Lemma 3.4: A is Hermitian, and positive definite where eq. (3.19) holds;
* the banded solution equals the unit sphere's closed form (Legendre functions
  of the second kind) when the 2 m0 known values are taken from that closed
  form: a wrong index, sign or weight in a_j(i), in A or in b breaks this;
* on non-axisymmetric stars, with the known values from the direct quadrature
  of the definition, every coefficient agrees with that quadrature.
"""
import math

import numpy as np
import pytest

import workloads
from oracle import banded as ob
from oracle import coeffs
from oracle import geometry as geo
from test_oracle_pins import _sphere_closed_form

CFG2_AMP = workloads.config(2)["amp"]
CFG3_AMP = workloads.config(3)["amp"]


@pytest.mark.parametrize("t,ts,j,M", [(0.4, 0.45, 3, 16), (1.3, 2.9, 17, 32)])
def test_rho2_coeffs_sphere(t, ts, j, M):
    th = math.pi * j / M
    c2 = ob.rho2_coeffs(None, t, th, ts, 6)
    assert abs(c2[0] - (2 - 2 * math.cos(t) * math.cos(ts))) <= 1e-15
    assert abs(c2[1] + math.sin(t) * math.sin(ts) * np.exp(-1j * th)) <= 1e-15
    assert np.max(np.abs(c2[2:])) <= 4e-15              # DFT rounding of values up to 4


@pytest.mark.parametrize("amp", [CFG2_AMP, CFG3_AMP])
@pytest.mark.parametrize("t,ts,j", [(0.7, 0.70002, 5), (1.6, 1.9, 30), (2.5, 0.4, 61)])
def test_rho2_coeffs_sum_back(amp, t, ts, j):
    M = 32
    th = math.pi * j / M
    D = ob.degree_bound(amp)
    c2 = ob.rho2_coeffs(amp, t, th, ts, D + 3)
    rng = np.random.default_rng(11)
    x = rng.uniform(0, 2 * math.pi, 9)
    n = np.arange(1, D + 1)
    series = c2[0].real + 2 * np.real(np.exp(1j * np.outer(x, n)) @ c2[1:D + 1])
    direct = geo.rho2(amp, t, th, ts, x - th)
    assert np.max(np.abs(series - direct)) <= 1e-14 * np.max(direct) + 1e-15
    scale = np.max(np.abs(c2))
    assert np.max(np.abs(c2[D + 1:])) <= 1e-15 * scale
    assert abs(c2[D]) > 1e-8 * scale


def _pairs(amp, M, n=40, seed=3, tmin=0.05):
    rng = np.random.default_rng(seed)
    t = rng.uniform(tmin, math.pi - tmin, n)
    ts = np.clip(t + rng.choice([-1, 1], n) * 10.0 ** rng.uniform(-6, 0, n), 1e-3, math.pi - 1e-3)
    j = rng.integers(0, 2 * M, n)
    return t, ts, j


@pytest.mark.parametrize("amp,expected", [(None, 1), (CFG2_AMP, 4), (CFG3_AMP, 8),
                                          (np.array([[0.0, 0.15]]), 2)])
def test_choose_m0(amp, expected):
    """Away from the poles the rule alone finds the degree of rho^2; with
    targets near the poles the transform's rounding is above eps0 times the
    small <rho^2>_0 there, and the degree bound caps it."""
    M = 32
    assert ob.degree_bound(amp) == expected
    t, ts, j = _pairs(amp, M, tmin=0.4)
    rows = [ob.rho2_coeffs(amp, t[i], math.pi * j[i] / M, ts[i], 12) for i in range(len(t))]
    assert ob.choose_m0(rows, eps0=1e-14) == expected
    t, ts, j = _pairs(amp, M, tmin=0.01)
    rows = [ob.rho2_coeffs(amp, t[i], math.pi * j[i] / M, ts[i], 12) for i in range(len(t))]
    assert ob.choose_m0(rows, eps0=1e-14, degree=ob.degree_bound(amp)) == expected
    assert ob.choose_m0(rows, eps0=1e-6, degree=ob.degree_bound(amp)) <= expected


@pytest.mark.parametrize("amp", [None, CFG2_AMP, CFG3_AMP])
def test_lemma_hermitian_and_positive_definite(amp):
    M, M0 = 16, 16
    t, ts, j = _pairs(amp, M, n=12, seed=5)
    m0 = ob.degree_bound(amp)
    seen_pd_condition = 0
    for i in range(len(t)):
        c2 = ob.rho2_coeffs(amp, t[i], math.pi * j[i] / M, ts[i], m0)
        known = {l: 1.0 for l in list(range(m0)) + list(range(M + M0 - m0 + 1, M + M0 + 1))}
        A, _ = ob.system(c2, m0, M + M0, known)
        assert np.array_equal(A, A.conj().T)
        if ob.positive_definite_condition(c2):
            seen_pd_condition += 1
            assert np.min(np.linalg.eigvalsh(A)) > 0
    if amp is None:
        assert seen_pd_condition == len(t)       # 1 > cos(t - t_s) for the sphere


@pytest.mark.parametrize("t,ts,j", [(0.3, 0.3 + 1e-6, 7), (1.2, 1.2 + 3e-5, 0), (1.2, 2.9, 3),
                                    (2.0, 2.2, 17)])
def test_banded_equals_sphere_closed_form(t, ts, j):
    M, M0 = 32, 32
    L = M + M0
    ref = _sphere_closed_form(t, math.pi * j / M, ts, L)
    known = {0: ref[0], L: ref[L]}
    c, info = ob.rhoinv_banded(None, M, M0, t, j, ts, 1, known=known)
    err = np.max(np.abs(c - ref)) / np.max(np.abs(ref))
    # measured 1e-17 (far pair) .. 1.3e-13 (near pairs, where the condition
    # number of A reaches 6.4e3 and bounds the rounding at ~7e-13)
    assert err <= 5e-13, err


@pytest.mark.parametrize("amp", [CFG2_AMP, CFG3_AMP])
@pytest.mark.parametrize("t,dts,j", [(0.7, 0.3, 5), (1.2, 0.05, 3), (1.6, 1e-2, 30),
                                     (2.5, -1e-3, 61), (0.9, 1e-4, 7), (1.1, 1e-6, 2)])
def test_banded_matches_direct_quadrature(amp, t, dts, j):
    """Measured 5e-16 .. 1e-13 of the largest coefficient (the known values'
    quadrature error carried through a system of condition number ~3e3)."""
    M, M0 = 32, 32
    m0 = ob.degree_bound(amp)
    c, info = ob.rhoinv_banded(amp, M, M0, t, j, t + dts, m0)
    d = info["direct"]
    err = np.max(np.abs(c - d)) / np.max(np.abs(d))
    assert err <= 1e-12, err
