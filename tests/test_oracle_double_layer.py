"""Pins of the oracle's double-layer operator K and its adjoint K' (Sec. 4).

Each fact is independent of the oracle's own arithmetic:
* B_m(0, b) = <s^{-3/2}>_m by quadrature against the closed form of B_0
  through the elliptic integrals E and K (eq. (4.9)) and against the
  recurrence of Proposition 4.1 (eq. (4.8)) driven by A_m from its own
  quadrature;
* tau_0 = nu . (r_s - r) by the line integral of the Remark in Sec. 4
  against the direct difference in 40-digit arithmetic;
* the coefficients sum back to the kernel pointwise;
* Gauss's integral: at k = 0, K[1] = -1 on any closed surface (here a smooth
  non-axisymmetric star);
* on the unit sphere K and K' (whose kernels coincide there) map Y_n^m to
  i k^2 (j_n h_n)'(k) Y_n^m, the mean of the interior and exterior limits of
  the double-layer potential, and the field u = 2 int dG/d nu_s Y_n^m outside
  is 2 i k^2 j_n'(k) h_n(k|x|) Y_n^m;
* the sound-hard Mie series leaves a total field with zero normal derivative
  on the sphere (central differences across r = 1), and the sound-hard
  right-hand side is minus the normal derivative of the incident wave.
"""
import math

import mpmath as mp
import numpy as np
import pytest
import scipy.special as sps

import workloads
from oracle import assembly as oasm
from oracle import double_layer as dl
from oracle import geometry as geo
from oracle import solve as osolve
from oracle import special

CFG3_AMP = workloads.config(3)["amp"]
# R = 1 + 0.2 sin t cos theta + 0.1 sin 2t cos theta: smooth at the poles, not axisymmetric
SMOOTH_AMP = np.array([[0.0, 0.2], [0.0, 0.1]])


@pytest.mark.parametrize("b", [1e-4, 0.01, 0.3, 2.5])
def test_b0_closed_form(b):
    B = dl.b3_coeffs(b, 0)
    m = math.exp(-2 * b)
    omq2 = -math.expm1(-2 * b)
    B0 = 4 * sps.ellipe(m) / (math.pi * omq2 ** 2) - (2 / math.pi) * sps.ellipk(m) / omq2
    assert abs(B[0] - B0) <= 1e-14 * B0


@pytest.mark.parametrize("b", [1e-3, 0.05, 0.7, 3.0])
def test_bm_recurrence(b):
    B = dl.b3_coeffs(b, 16)
    A = special.singular_factor(b, 16)
    rec = np.array([math.cosh(b) * B[m - 1] - 0.5 * (2 * m - 1) * math.exp(b) * A[m - 1] for m in range(1, 17)])
    assert np.max(np.abs(rec - B[1:])) <= 1e-13 * B[0]


@pytest.mark.parametrize("adjoint", [False, True])
def test_tau0_stable_matches_extended_precision(adjoint):
    mp.mp.dps = 40
    a = np.asarray(CFG3_AMP)

    def r_mp(t, th):
        R = 1 + sum(a[l - 1, m] * mp.sin(l * t) * mp.cos(m * th)
                    for l in range(1, a.shape[0] + 1) for m in range(a.shape[1]))
        return mp.matrix([R * mp.sin(t) * mp.cos(th), R * mp.sin(t) * mp.sin(th), R * mp.cos(t)])

    def nu_mp(t, th):
        rt = mp.matrix([mp.diff(lambda x: r_mp(x, th)[i], t) for i in range(3)])
        rth = mp.matrix([mp.diff(lambda x: r_mp(t, x)[i], th) for i in range(3)])
        n = mp.matrix([rt[1] * rth[2] - rt[2] * rth[1], rt[2] * rth[0] - rt[0] * rth[2],
                       rt[0] * rth[1] - rt[1] * rth[0]])
        return n / mp.norm(n)

    worst = 0.0
    for t, ts, dth in ((1.1, 1.1 + 1e-6, 2e-6), (0.7, 0.7 - 3e-4, -1e-4), (2.0, 2.01, 0.02), (0.4, 0.9, 0.3)):
        th = 0.9
        T, TS = mp.mpf(t), mp.mpf(ts)
        TH, THS = mp.mpf(th), mp.mpf(th) + mp.mpf(dth)
        d = r_mp(TS, THS) - r_mp(T, TH)
        nu = nu_mp(T, TH) if adjoint else nu_mp(TS, THS)
        ref = -(nu.T * d)[0] if adjoint else (nu.T * d)[0]
        got = float(dl.tau0(a, t, th, ts, dth, adjoint=adjoint))
        worst = max(worst, abs(got - float(ref)) / abs(float(ref)))
    assert worst <= 1e-12, worst


@pytest.mark.parametrize("adjoint", [False, True])
def test_kcoeffs_sum_back_to_the_kernel(adjoint):
    """sum_n kK_n e^{i n theta_s} reproduces the kernel at source azimuths
    away from the near-singularity (a far pair, M large enough that the
    series is resolved)."""
    M, k, t, j, ts = 64, 3.0, 0.8, 10, 1.9
    kK, info = dl.pair_kcoeffs(CFG3_AMP, k, M, t, j, ts, adjoint=adjoint)
    assert info["converged"]
    th = math.pi * j / M
    ns = np.arange(-M + 1, M + 1)
    for dth in (0.7, -1.9, 2.8):
        f = np.sum(kK * np.exp(1j * ns * (th + dth)))
        ref = dl.kernel_values(CFG3_AMP, k, t, th, ts, np.array([dth]), adjoint=adjoint)[0]
        assert abs(f - ref) <= 1e-11 * np.max(np.abs(kK)) * 2 * M, (dth, f, ref)


def _rule():
    import test_oracle_system as tos
    return tos.load_golden()


def test_gauss_identity_star():
    """K[1] = -1 at k = 0: 2 int d/d nu_s (1 / (4 pi rho)) d sigma_s = -1 for
    targets on a closed surface (the solid angle 2 pi).  Sampled rows of the
    oracle's K at 4 panels, M = 8 applied to psi~ = 1 * J.  Measured 7.0e-6
    (discretisation); a wrong sign or normalisation of tau_0 or of the kernel
    gives an O(1) error."""
    npan, M = 4, 8
    L = oasm.layout(npan, M)
    rows = np.arange(0, 32 * M * npan, 37)
    Kr = oasm.rows(SMOOTH_AMP, 0.0, M, npan, rows, _rule(), processes=8, kind="K")
    jac = geo.jacobian(SMOOTH_AMP, L["t"], L["th"])
    err = np.max(np.abs(Kr @ jac + 1.0))
    assert err <= 3e-5, err


@pytest.fixture(scope="module")
def sphere_k():
    npan, M, k = 4, 8, 1.0
    rule = _rule()
    return npan, M, k, {kind: oasm.matrix(None, k, M, npan, rule, processes=8, kind=kind) for kind in ("K", "Kp")}


@pytest.mark.parametrize("n,m", [(0, 0), (1, 0), (2, 1), (4, 3)])
def test_sphere_double_layer_eigenvalues(sphere_k, n, m):
    npan, M, k, mats = sphere_k
    L = oasm.layout(npan, M)
    Y = osolve.spherical_harmonic(n, m, L["t"], L["th"])
    v = Y * np.sin(L["t"])
    lam = osolve.sphere_double_layer_eigenvalue(n, k)
    for kind, K in mats.items():
        err = np.max(np.abs(K @ v - lam * Y)) / np.max(np.abs(Y))
        # measured 6.7e-6 for n <= 1 and ~1e-8 above at (4 panels, 2M = 16)
        assert err <= 3e-5, (kind, err)


@pytest.mark.parametrize("n,m", [(1, 0), (3, 2)])
def test_double_layer_field_of_spherical_harmonic(n, m):
    """u = 2 int dG/d nu_s Y_n^m dsigma outside the unit sphere is
    2 i k^2 j_n'(k) h_n(k|x|) Y_n^m(x/|x|) (twice the double-layer potential,
    from the addition theorem of G): the oracle's product-rule field at
    |x| = 3 (8 panels, M = 16; smooth integrand, spectrally accurate: measured
    6e-16 and 6e-15, against 4e-9 and 6e-7 at 4 panels, M = 8)."""
    import scipy.special as sps
    npan, M, k = 8, 16, 1.3
    L = oasm.layout(npan, M)
    psi_t = osolve.spherical_harmonic(n, m, L["t"], L["th"]) * np.sin(L["t"])
    rng = np.random.default_rng(4)
    d = rng.standard_normal((6, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    pts = 3.0 * d
    u = oasm.field_double_layer(None, npan, M, k, psi_t, pts)
    tp = np.arccos(np.clip(d[:, 2], -1, 1))
    php = np.arctan2(d[:, 1], d[:, 0])
    ref = 2j * k ** 2 * sps.spherical_jn(n, k, derivative=True) * osolve.hankel1(n, 3 * k) \
        * osolve.spherical_harmonic(n, m, tp, php)
    assert np.max(np.abs(u - ref)) <= 1e-12 * np.max(np.abs(ref))


def test_sound_hard_mie_has_zero_normal_derivative():
    k = 2.2
    dvec = np.array([0.3, -0.4, np.sqrt(1 - 0.25)])
    rng = np.random.default_rng(5)
    xh = rng.standard_normal((8, 3))
    xh /= np.linalg.norm(xh, axis=1)[:, None]
    h = 1e-5

    def total(r):
        x = r * xh
        return np.exp(1j * k * (x @ dvec)) + osolve.mie_scattered_hard(k, x, dvec)

    dudr = (total(1 + h) - total(1 - h)) / (2 * h)
    scale = np.max(np.abs(k * np.exp(1j * k * (xh @ dvec))))
    assert np.max(np.abs(dudr)) <= 1e-8 * scale
    # sound-soft series for contrast: its normal derivative does not vanish
    soft = (np.exp(1j * k * ((1 + h) * xh @ dvec)) + osolve.mie_scattered(k, (1 + h) * xh, dvec)
            - np.exp(1j * k * ((1 - h) * xh @ dvec)) - osolve.mie_scattered(k, (1 - h) * xh, dvec)) / (2 * h)
    assert np.max(np.abs(soft)) > 0.1 * scale


def test_sound_hard_rhs_is_minus_normal_derivative():
    """rhs_plane_wave_dn against a central difference of e^{ik d.x} along the
    normal at the collocation points."""
    amp = SMOOTH_AMP
    npan, M, k = 2, 8, 3.0
    dvec = np.array([0.0, 0.6, 0.8])
    L = oasm.layout(npan, M)
    x = geo.point(amp, L["t"], L["th"])
    nu = geo.normal(amp, L["t"], L["th"])
    h = 1e-6
    fd = (np.exp(1j * k * ((x + h * nu) @ dvec)) - np.exp(1j * k * ((x - h * nu) @ dvec))) / (2 * h)
    g = oasm.rhs_plane_wave_dn(amp, npan, M, k, dvec)
    assert np.max(np.abs(g + fd)) <= 1e-8


def test_point_source_dn_rhs_is_normal_derivative():
    """rhs_point_source_dn against a central difference of G(x; p) along the
    normal at the collocation points (the interior Neumann test of Sec. 5)."""
    amp = SMOOTH_AMP
    npan, M, k = 2, 8, 2.5
    p = np.array([3.0, 4.0, 10.5])
    L = oasm.layout(npan, M)
    x = geo.point(amp, L["t"], L["th"])
    nu = geo.normal(amp, L["t"], L["th"])

    def G(y):
        r = np.linalg.norm(y - p, axis=1)
        return np.exp(1j * k * r) / (4 * np.pi * r)

    h = 1e-5
    fd = (G(x + h * nu) - G(x - h * nu)) / (2 * h)
    g = oasm.rhs_point_source_dn(amp, npan, M, k, p)
    assert np.max(np.abs(g - fd)) <= 1e-9 * np.max(np.abs(g))
