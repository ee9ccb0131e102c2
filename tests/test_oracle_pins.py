"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these compare the oracle with itself: each checks it against a closed
form, an exact identity, an independent high-precision quadrature or the
inverse of the transform it computes.
"""
import math

import mpmath as mp
import numpy as np
import pytest
import scipy.special as sps

import workloads
from oracle import coeffs, geometry as geo, special

CFG2_AMP = workloads.config(2)["amp"]
CFG3_AMP = workloads.config(3)["amp"]


# ----------------------------------------------------------------------------
# Geometry
# ----------------------------------------------------------------------------

def test_sphere_jacobian_is_sin_t():
    t = np.linspace(0.1, 3.0, 7)[:, None]
    th = np.linspace(0, 6, 5)[None, :]
    assert np.allclose(geo.jacobian(None, t, th), np.sin(t) + 0 * th, rtol=1e-15, atol=0)


@pytest.mark.parametrize("amp", [CFG2_AMP, CFG3_AMP])
def test_star_derivatives_match_mpmath_differentiation(amp):
    mp.mp.dps = 30
    a = np.asarray(amp)

    def r_mp(t, th):
        R = 1 + sum(a[l - 1, m] * mp.sin(l * t) * mp.cos(m * th)
                    for l in range(1, a.shape[0] + 1) for m in range(a.shape[1]))
        return [R * mp.sin(t) * mp.cos(th), R * mp.sin(t) * mp.sin(th), R * mp.cos(t)]

    for t, th in [(0.4, 1.1), (2.2, 4.0)]:
        rt, rth = geo.derivs(amp, t, th)
        rthth = geo.second_theta(amp, t, th)
        for c in range(3):
            assert abs(rt[c] - float(mp.diff(lambda x: r_mp(x, th)[c], t))) < 1e-14
            assert abs(rth[c] - float(mp.diff(lambda y: r_mp(t, y)[c], th))) < 1e-14
            assert abs(rthth[c] - float(mp.diff(lambda y: r_mp(t, y)[c], th, 2))) < 1e-13


@pytest.mark.parametrize("amp", [CFG2_AMP, CFG3_AMP])
def test_star_volume_divergence_theorem(amp):
    """(1/3) int r . (r_t x r_theta) = int_0^pi int_0^2pi R^3 sin t / 3."""
    x, w = np.polynomial.legendre.leggauss(64)
    t = 0.5 * math.pi * (x + 1)
    wt = 0.5 * math.pi * w
    th = 2 * math.pi * np.arange(64) / 64
    T, TH = np.meshgrid(t, th, indexing="ij")
    rt, rth = geo.derivs(amp, T, TH)
    flux = np.einsum("...c,...c->...", geo.point(amp, T, TH), np.cross(rt, rth))
    v1 = (wt[:, None] * flux).sum() * (2 * math.pi / 64) / 3
    v2 = (wt[:, None] * geo.radius(amp, T, TH) ** 3 * np.sin(T)).sum() * (2 * math.pi / 64) / 3
    assert abs(v1 - v2) < 1e-13 * v2
    if np.all(np.asarray(amp) == 0):
        assert abs(v2 - 4 * math.pi / 3) < 1e-13


@pytest.mark.parametrize("amp", [None, CFG2_AMP, CFG3_AMP])
def test_stable_difference_matches_extended_precision(amp):
    mp.mp.dps = 40
    a = geo.as_amp(amp)

    def r_mp(t, th):
        R = 1 + sum(mp.mpf(a[l - 1, m]) * mp.sin(l * t) * mp.cos(m * th)
                    for l in range(1, a.shape[0] + 1) for m in range(a.shape[1]))
        return [R * mp.sin(t) * mp.cos(th), R * mp.sin(t) * mp.sin(th), R * mp.cos(t)]

    t, th = 0.9, 2.3
    for dt, dth in [(1e-9, 2e-9), (-3e-6, 1e-7), (2e-3, -4e-3), (0.1, 0.2), (0.4, 2.0)]:
        d = geo.delta_r(amp, t, th, t + dt, dth)
        ts = t + dt
        ref = [x - y for x, y in zip(r_mp(mp.mpf(ts), mp.mpf(th) + mp.mpf(dth)),
                                     r_mp(mp.mpf(t), mp.mpf(th)))]
        nref = float(mp.sqrt(sum(v * v for v in ref)))
        err = math.sqrt(sum(float(d[c] - ref[c]) ** 2 for c in range(3)))
        assert err <= 4e-16 * nref + 1e-300, (dt, dth, err / nref)


# ----------------------------------------------------------------------------
# Singular factor A_m(b), eq. (3.26)
# ----------------------------------------------------------------------------

@pytest.mark.parametrize("b", [1e-6, 1e-3, 0.05, 0.3, 1.0, 2.5])
def test_singular_factor_legendre_q(b):
    """A_m(b) = e^{b/2} Q_{m-1/2}(cosh b) / pi, eq. (3.27)."""
    mp.mp.dps = 30
    A = special.singular_factor(b, 40)
    ref = np.array([float((mp.exp(mp.mpf(b) / 2) * mp.legenq(m - 0.5, 0, mp.cosh(mp.mpf(b)),
                                                             type=3)).real / mp.pi)
                    for m in range(41)])
    assert np.max(np.abs(A - ref)) <= 2e-15 * ref[0]


@pytest.mark.parametrize("b", [1e-4, 0.2, 1.5])
def test_singular_factor_binomial_series(b):
    """|1 - q e^{i phi}|^{-1} = sum alpha_j q^j e^{ij phi} sum alpha_k q^k e^{-ik phi},
    alpha_j = (1/2)_j / j!, q = e^{-b}: A_m = q^m alpha_m 2F1(1/2, m+1/2; m+1; q^2)."""
    mp.mp.dps = 30
    q = mp.exp(-mp.mpf(b))
    A = special.singular_factor(b, 12)
    for m in range(13):
        alpha_m = mp.rf(0.5, m) / mp.factorial(m)
        ref = q ** m * alpha_m * mp.hyp2f1(0.5, m + 0.5, m + 1, q * q)
        assert abs(A[m] - float(ref)) <= 2e-15 * A[0]


@pytest.mark.parametrize("b", [1e-5, 0.01, 0.7, 3.0])
def test_singular_factor_elliptic(b):
    """A_0 = (2/pi) K(e^{-2b}); A_1 = (2/pi) e^{b} (K - E)(e^{-2b}) (parameter convention)."""
    A = special.singular_factor(b, 2)
    m = math.exp(-2 * b)
    K, E = sps.ellipk(m), sps.ellipe(m)
    if b < 0.1:                               # K near m -> 1 from the complementary parameter
        K = sps.ellipkm1(-math.expm1(-2 * b))
    assert abs(A[0] - 2 / math.pi * K) <= 2e-15 * A[0]
    assert abs(A[1] - 2 / math.pi * math.exp(b) * (K - E)) <= 4e-15 * A[0]


# ----------------------------------------------------------------------------
# <rho^-1>_l
# ----------------------------------------------------------------------------

def _sphere_closed_form(t, th, ts, L):
    """Axisymmetric reduction (Remark 3.5 with eq. (3.27)): for the unit sphere
    rho^2 = B (cosh b - cos(theta_s - theta)), so
    c_l = e^{-i l theta} Q_{l-1/2}(chi) / (pi sqrt(sin t sin ts)),
    chi = (sin^2 t + sin^2 ts + (cos t - cos ts)^2) / (2 sin t sin ts).
    The phase is e^{-i l theta}: eq. (3.20) prints e^{+i m theta}, which does
    not agree with the coefficient convention of Sec. 3.2."""
    mp.mp.dps = 30
    r, rs, z, zs = mp.sin(t), mp.sin(ts), mp.cos(t), mp.cos(ts)
    chi = (r * r + rs * rs + (z - zs) ** 2) / (2 * r * rs)
    return np.array([complex(mp.exp(-1j * l * th) * mp.legenq(l - 0.5, 0, chi, type=3).real
                             / (mp.pi * mp.sqrt(r * rs))) for l in range(L + 1)])


@pytest.mark.parametrize("t,ts,j", [(0.3, 0.3 + 1e-6, 7), (0.3, 0.3 - 1e-9, 63),
                                    (1.2, 1.2 + 3e-5, 0), (1.2, 2.9, 3), (0.05, 3.0, 40),
                                    (2.0, 2.2, 17)])
def test_rhoinv_sphere_closed_form(t, ts, j):
    M, L = 32, 64
    c, _, info = coeffs.pair_coeffs(None, 1.0, M, L, t, j, ts)
    ref = _sphere_closed_form(t, math.pi * j / M, ts, L)
    assert info["converged"]
    assert np.max(np.abs(c - ref)) <= 4e-15 * np.max(np.abs(ref))


def _rho2_fourier(amp, t, th, ts, n=64):
    """<rho^2>_n by an n-point FFT: exact, since rho^2 is a trigonometric
    polynomial in theta_s of degree <= 2 mmax + 2 < n/2 for this family."""
    x = 2 * math.pi * np.arange(n) / n
    r2 = geo.rho2(amp, t, th, ts, x - th)
    return np.fft.fft(r2) / n


@pytest.mark.parametrize("amp,k", [(CFG2_AMP, 5.0), (CFG3_AMP, 20.0)])
@pytest.mark.parametrize("t,ts,j", [(0.7, 0.7 + 2e-5, 5), (1.6, 1.9, 30), (2.5, 0.4, 61)])
def test_rhoinv_lemma_identity(amp, k, t, ts, j):
    """Lemma 3.3, eq. (3.11): sum_n (2m+n) <rho^2>_n <rho^-1>_{-(m+n)} = 0."""
    M, L = 32, 64
    c, _, _ = coeffs.pair_coeffs(amp, k, M, L, t, j, ts)
    th = math.pi * j / M
    r2h = _rho2_fourier(amp, t, th, ts)
    m0 = 10                               # <rho^2>_n = 0 beyond |n| = 2 mmax + 2 <= 10
    cfull = {l: (c[l] if l >= 0 else np.conj(c[-l])) for l in range(-L, L + 1)}
    # residual measured on the absolute scale of the recurrence: |2m + n| times
    # the size of <rho^2> times the largest coefficient
    scale = np.sum(np.abs(r2h)) * np.max(np.abs(c))
    worst = 0.0
    for m in range(-L + m0, L - m0 + 1):
        res = sum((2 * m + n) * r2h[n % 64] * cfull[-(m + n)] for n in range(-m0, m0 + 1))
        worst = max(worst, abs(res) / ((2 * abs(m) + m0) * scale))
    assert worst < 1e-15


@pytest.mark.parametrize("amp", [CFG2_AMP, CFG3_AMP])
def test_rhoinv_fourier_series_sums_back(amp):
    """sum_l c_l e^{i l theta_s} reproduces rho^-1 pointwise (well-separated pair,
    where the series converges fast): pins normalisation and phase convention."""
    M, L = 32, 64
    t, ts, j = 0.8, 2.1, 9
    c, _, _ = coeffs.pair_coeffs(amp, 5.0, M, L, t, j, ts)
    th = math.pi * j / M
    xs = np.linspace(-3, 3, 13)
    l = np.arange(1, L + 1)
    series = c[0].real + 2 * np.real(np.exp(1j * np.outer(th + xs, l)) @ c[1:])
    direct = 1 / np.sqrt(geo.rho2(amp, t, th, ts, xs))
    assert np.max(np.abs(series - direct)) < 1e-13 * np.max(direct)


def test_rhoinv_mpmath_bruteforce_star():
    """Independent tanh-sinh quadrature at 40 digits with the direct
    (extended-precision) difference, on a near pair of the config-2 surface."""
    mp.mp.dps = 40
    a = CFG2_AMP
    M, L = 32, 40
    t, ts, j = 1.1, 1.1 + 4e-4, 11
    c, kap, info = coeffs.pair_coeffs(a, 5.0, M, L, t, j, ts)
    th = mp.pi * j / M

    def r_mp(t, th):
        R = 1 + mp.mpf(a[2, 2]) * mp.sin(3 * t) * mp.cos(2 * th)
        return [R * mp.sin(t) * mp.cos(th), R * mp.sin(t) * mp.sin(th), R * mp.cos(t)]

    p0 = r_mp(mp.mpf(t), th)

    def rho(x):
        p = r_mp(mp.mpf(ts), th + x)
        return mp.sqrt(sum((u - v) ** 2 for u, v in zip(p, p0)))

    u = mp.mpf(info["a"])
    beta = info["beta"]
    brk = sorted({u - mp.pi, u + mp.pi, u} | {u + s * beta * 2 ** e for e in range(-4, 14)
                                              for s in (-1, 1) if beta * 2 ** e < 3})
    for l in (0, 1, 7, 40):
        ref = mp.quad(lambda x: mp.exp(-1j * l * (th + x)) / rho(x), brk) / (2 * mp.pi)
        assert abs(c[l] - complex(ref)) <= 1e-14 * abs(c[0])
    k = mp.mpf(5)
    for n in (-31, 0, 3, 32):
        ref = mp.quad(lambda x: mp.exp(1j * k * rho(x)) * mp.exp(-1j * n * (th + x)) / rho(x),
                      brk) / (2 * mp.pi)
        assert abs(kap[n + M - 1] - complex(ref)) <= 1e-14 * np.max(np.abs(kap))


def test_rhoinv_reciprocity():
    """Double coefficients C_{m,l}(t, ts) = (1/2M) sum_j e^{-i m theta_j} c_l(t, theta_j, ts)
    satisfy C_{m,l}(t, ts) = C_{l,m}(ts, t) (rho is symmetric in its two points)."""
    a = CFG2_AMP
    M, L = 32, 8
    t, ts = 0.9, 1.5
    thj = math.pi * np.arange(2 * M) / M

    def double(t1, t2):
        c = np.array([coeffs.pair_coeffs(a, 5.0, M, L, t1, j, t2)[0] for j in range(2 * M)])
        return np.exp(-1j * np.outer(np.arange(-L, L + 1), thj)) @ np.concatenate(
            [np.conj(c[:, :0:-1]), c], axis=1) / (2 * M)

    C1 = double(t, ts)        # [m + L, l + L]
    C2 = double(ts, t)
    assert np.max(np.abs(C1 - C2.T)) < 1e-12 * np.max(np.abs(C1))


# ----------------------------------------------------------------------------
# <e^{ik rho}/rho>_n
# ----------------------------------------------------------------------------

def test_kappa_reduces_to_rhoinv_at_k0():
    M, L = 32, 64
    c, kap, _ = coeffs.pair_coeffs(CFG2_AMP, 0.0, M, L, 1.3, 4, 1.3 + 1e-4)
    n = np.arange(-M + 1, M + 1)
    expect = np.where(n >= 0, c[np.abs(n)], np.conj(c[np.abs(n)]))
    assert np.max(np.abs(kap - expect)) <= 1e-15 * np.max(np.abs(c))


@pytest.mark.parametrize("amp,k", [(CFG2_AMP, 5.0), (CFG3_AMP, 20.0)])
def test_kappa_fourier_series_sums_back(amp, k):
    M, L = 64, 128
    t, ts, j = 0.8, 2.1, 9
    _, kap, _ = coeffs.pair_coeffs(amp, k, M, L, t, j, ts)
    th = math.pi * j / M
    xs = np.linspace(-3, 3, 13)
    n = np.arange(-M + 1, M + 1)
    series = np.exp(1j * np.outer(th + xs, n)) @ kap
    rho = np.sqrt(geo.rho2(amp, t, th, ts, xs))
    direct = np.exp(1j * k * rho) / rho
    assert np.max(np.abs(series - direct)) < 1e-13 * np.max(np.abs(direct))


# ----------------------------------------------------------------------------
# Truncation tail of eq. (3.10) (kappa_tail)
# ----------------------------------------------------------------------------

def test_kappa_tail_vanishes_at_k0():
    """cos(0 rho) = 1 has the single coefficient <1>_0 = 1: no tail beyond the
    rounding floor of the sum (~2 n_max magnitudes of a few 1e-16 each)."""
    tail, mag = coeffs.kappa_tail(CFG2_AMP, 0.0, 16, 16, 1.1, 3, 1.4)
    assert tail <= 1e-12 and abs(mag[mag.size // 2] - 1.0) <= 1e-15


@pytest.mark.parametrize("n", [12, 20])
def test_kappa_tail_coefficients_match_adaptive_quadrature(n):
    """|<cos k rho>_n| against scipy's adaptive quadrature of the definition."""
    from scipy import integrate
    k, M, t, j, ts = 9.0, 16, 1.0, 5, 1.3
    _, mag = coeffs.kappa_tail(CFG3_AMP, k, M, M, t, j, ts, n_max=32)
    th = math.pi * j / M

    def f(x, part):
        v = math.cos(k * math.sqrt(float(geo.rho2(CFG3_AMP, t, th, ts, np.array([x]))[0])))
        return v * (math.cos(n * x) if part == 0 else -math.sin(n * x))
    re = integrate.quad(f, 0, 2 * math.pi, args=(0,), limit=400, epsabs=1e-15)[0] / (2 * math.pi)
    im = integrate.quad(f, 0, 2 * math.pi, args=(1,), limit=400, epsabs=1e-15)[0] / (2 * math.pi)
    assert abs(mag[32 + n] - math.hypot(re, im)) <= 1e-12


def test_kappa_tail_separates_resolved_from_unresolved():
    """k = 5 is resolved by M = 64 (tail at the rounding floor); k = 25 is not
    by M = 8 (the tail is of the order of the coefficients themselves)."""
    small, _ = coeffs.kappa_tail(CFG2_AMP, 5.0, 64, 64, 0.9, 7, 1.7)
    large, _ = coeffs.kappa_tail(CFG2_AMP, 25.0, 8, 8, 0.9, 7, 1.7)
    # the floor is the sum of 2 n_max + 1 rounding-level magnitudes (n_max = 512
    # here): a few 1e-12
    assert small <= 1e-11 and large >= 1e-3, (small, large)


# ----------------------------------------------------------------------------
# Mode-block-Jacobi reference (oracle/solve.py)
# ----------------------------------------------------------------------------

def _mode_diagonal_matrix(blocks, M, nodes):
    """S[(a, j), (b, j')] = (1/2M) sum_m e^{i m theta_j} B_m[a, b] e^{-i m theta_j'}:
    the matrix whose azimuthal-mode blocks are exactly B_m, written out entry by
    entry (m = -M+1..M)."""
    th = np.pi * np.arange(2 * M) / M
    S = np.zeros((nodes, 2 * M, nodes, 2 * M), dtype=complex)
    for mi, m in enumerate(range(-M + 1, M + 1)):
        for j in range(2 * M):
            for jp in range(2 * M):
                S[:, j, :, jp] += np.exp(1j * m * (th[j] - th[jp])) * blocks[mi] / (2 * M)
    return S.reshape(nodes * 2 * M, nodes * 2 * M)


def test_mode_blocks_recover_the_blocks():
    from oracle import solve as osolve
    M, nodes = 3, 4
    rng = np.random.default_rng(5)
    B = rng.standard_normal((2 * M, nodes, nodes)) + 1j * rng.standard_normal((2 * M, nodes, nodes))
    S = _mode_diagonal_matrix(B, M, nodes)
    assert np.max(np.abs(osolve.mode_blocks(S, M, nodes) - B)) <= 1e-13


def test_blockjacobi_apply_is_exact_inverse_of_mode_diagonal_matrix():
    """For a mode-diagonal S the block-Jacobi preconditioner is S^-1 exactly."""
    from oracle import solve as osolve
    M, nodes = 3, 4
    rng = np.random.default_rng(6)
    B = rng.standard_normal((2 * M, nodes, nodes)) + 1j * rng.standard_normal((2 * M, nodes, nodes))
    B += 3 * np.eye(nodes)
    S = _mode_diagonal_matrix(B, M, nodes)
    v = rng.standard_normal(S.shape[0]) + 1j * rng.standard_normal(S.shape[0])
    z = osolve.blockjacobi_apply(S, v, M, nodes)
    assert np.linalg.norm(z - np.linalg.solve(S, v)) <= 1e-12 * np.linalg.norm(z)


# ----------------------------------------------------------------------------
# Point source G(x; p) = e^{ik|x-p|} / (4 pi |x-p|) (oracle/solve.py)
# ----------------------------------------------------------------------------

def test_point_source_unit_flux_and_helmholtz():
    """G is the outgoing fundamental solution of (Delta + k^2): the flux of
    grad G out of a small sphere around p is -1, (Delta + k^2) G = 0 away from
    p (second differences), and G satisfies the radiation condition."""
    from oracle import solve as osolve
    k, p = 3.0, np.array([0.3, -0.2, 0.5])
    eps = 1e-3
    xg, wg = np.polynomial.legendre.leggauss(24)
    nphi = 48
    phi = 2 * np.pi * np.arange(nphi) / nphi
    ct, ph = np.meshgrid(xg, phi, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    nrm = np.stack([st * np.cos(ph), st * np.sin(ph), ct], axis=-1).reshape(-1, 3)
    w = (wg[:, None] * np.full(nphi, 2 * np.pi / nphi)[None, :]).ravel() * eps ** 2
    h = 1e-6
    dG = (osolve.point_source(k, p + (eps + h) * nrm, p) - osolve.point_source(k, p + (eps - h) * nrm, p)) / (2 * h)
    flux = np.sum(w * dG)
    assert abs(flux - (-1.0)) <= 1e-5, flux
    x0 = np.array([1.0, 0.4, -0.7])
    hh = 1e-3
    lap = sum(osolve.point_source(k, x0 + s * hh * e, p)[0] for e in np.eye(3) for s in (1, -1)) \
        - 6 * osolve.point_source(k, x0, p)[0]
    res = lap / hh ** 2 + k ** 2 * osolve.point_source(k, x0, p)[0]
    assert abs(res) <= 1e-5 * abs(k ** 2 * osolve.point_source(k, x0, p)[0]), res
    # outgoing (Sommerfeld): r (dG/dr - ik G) -> 0, which the incoming wave
    # e^{-ik|x-p|} / (4 pi |x-p|) violates (there it tends to -2ik r G)
    d = np.array([0.6, 0.0, 0.8])
    r = 1e4
    Gr = osolve.point_source(k, p + r * d, p)[0]
    dGr = (osolve.point_source(k, p + (r + 1e-4) * d, p)[0]
           - osolve.point_source(k, p + (r - 1e-4) * d, p)[0]) / 2e-4
    assert abs(r * (dGr - 1j * k * Gr)) <= 1e-3 * abs(k * r * Gr)
