"""Dense solve and analytic references for the single-layer equation.  TEST
INFRASTRUCTURE ONLY.

* ``lu_solve``: LAPACK LU with partial pivoting (scipy), FP64.
* ``mie_scattered``: field scattered by the sound-soft unit sphere for the
  incident plane wave e^{ik d.x} (separation of variables),
      u_s(x) = -sum_n (2n+1) i^n [j_n(k)/h_n(k)] h_n(k|x|) P_n(d.x/|x|);
  ``mie_scattered_hard`` the same for the sound-hard sphere (zero normal
  derivative of the total field), with j_n'(k)/h_n'(k) in place of j_n/h_n.
* ``sphere_single_layer_eigenvalue``: on the unit sphere the operator of
  eq. (2.8), S[phi] = 2 int G phi dsigma, maps the spherical harmonic Y_n^m to
  2ik j_n(k) h_n(k) Y_n^m; ``sphere_double_layer_eigenvalue`` the same for K
  and K' (Sec. 4).
* ``point_source``: G(x; p) = e^{ik|x-p|}/(4 pi |x-p|), the exact interior
  solution of the Dirichlet test of Sec. 5.
"""
import numpy as np
from scipy import linalg, special


def lu_solve(S, g):
    return linalg.lu_solve(linalg.lu_factor(S), g)


def hankel1(n, z):
    return special.spherical_jn(n, z) + 1j * special.spherical_yn(n, z)


def mie_scattered(k, pts, d, nmax=40):
    pts = np.atleast_2d(pts)
    r = np.linalg.norm(pts, axis=1)
    cosg = pts @ np.asarray(d) / r
    u = np.zeros(len(pts), dtype=complex)
    for n in range(nmax + 1):
        a = (2 * n + 1) * (1j ** n) * special.spherical_jn(n, k) / hankel1(n, k)
        u -= a * hankel1(n, k * r) * special.eval_legendre(n, cosg)
    return u


def mie_scattered_hard(k, pts, d, nmax=40):
    pts = np.atleast_2d(pts)
    r = np.linalg.norm(pts, axis=1)
    cosg = pts @ np.asarray(d) / r
    u = np.zeros(len(pts), dtype=complex)
    for n in range(nmax + 1):
        dj = special.spherical_jn(n, k, derivative=True)
        dh = dj + 1j * special.spherical_yn(n, k, derivative=True)
        u -= (2 * n + 1) * (1j ** n) * (dj / dh) * hankel1(n, k * r) * special.eval_legendre(n, cosg)
    return u


def sphere_single_layer_eigenvalue(n, k):
    return 2j * k * special.spherical_jn(n, k) * hankel1(n, k)


def sphere_double_layer_eigenvalue(n, k):
    """On the unit sphere K[Y_n^m] = K'[Y_n^m] = i k^2 (j_n h_n)'(k) Y_n^m: the
    double-layer potential of Y_n^m is i k^2 h_n'(k) j_n(k|x|) Y_n^m inside and
    i k^2 j_n'(k) h_n(k|x|) Y_n^m outside; K (factor 2, principal value) is the
    sum of the two limits on the surface."""
    jn, dj = special.spherical_jn(n, k), special.spherical_jn(n, k, derivative=True)
    hn = hankel1(n, k)
    dh = dj + 1j * special.spherical_yn(n, k, derivative=True)
    return 1j * k ** 2 * (dj * hn + jn * dh)


def spherical_harmonic(n, m, t, th):
    """Y_n^m(t, th) with t the polar angle (scipy's sph_harm convention)."""
    try:
        return special.sph_harm_y(n, m, t, th)
    except AttributeError:                       # older scipy
        return special.sph_harm(m, n, th, t)


def point_source(k, x, p):
    rho = np.linalg.norm(np.atleast_2d(x) - np.asarray(p), axis=1)
    return np.exp(1j * k * rho) / (4 * np.pi * rho)


def mode_blocks(S, M, nodes):
    """Diagonal azimuthal-mode blocks B_m = F_m S F_m^+ of a matrix on the
    (node, azimuth) grid, from the definition
    B_m[a][b] = (1/2M) sum_{j,j'} e^{-i m theta_j} S[(a,j),(b,j')] e^{i m theta_j'},
    m = -M+1..M; returns [2M, nodes, nodes]."""
    th = np.pi * np.arange(2 * M) / M
    S4 = np.asarray(S).reshape(nodes, 2 * M, nodes, 2 * M)
    out = np.empty((2 * M, nodes, nodes), dtype=complex)
    for mi, m in enumerate(range(-M + 1, M + 1)):
        e = np.exp(1j * m * th)
        out[mi] = np.einsum("j,ajbk,k->ab", e.conj(), S4, e) / (2 * M)
    return out


def blockjacobi_apply(S, v, M, nodes):
    """z = sum_m (B_m^{-1} V_m) e^{i m theta} with V_m the modes of v."""
    th = np.pi * np.arange(2 * M) / M
    ms = np.arange(-M + 1, M + 1)
    V = np.asarray(v).reshape(nodes, 2 * M) @ np.exp(-1j * np.outer(th, ms)) / (2 * M)   # [node, m]
    B = mode_blocks(S, M, nodes)
    E = np.stack([np.linalg.solve(B[i], V[:, i]) for i in range(2 * M)], axis=1)        # [node, m]
    return (E @ np.exp(1j * np.outer(ms, th))).reshape(-1)
