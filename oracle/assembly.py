"""The discrete single-layer system, written from its definition.  TEST
INFRASTRUCTURE ONLY.

Sec. 3.1 and 3.4: unknowns phi~ = phi J at the collocation points
r(t_i^l, theta_j) (panel i, Gauss-Legendre node l, azimuth j = 0..2M-1), in the
order r = (i*16 + l)*2M + j.  With h = pi / n_panels and W = (h/2) w_l the
Gauss-Legendre weight on a panel:

* far panels (|i - i'| >= 2), eqs. (3.7)-(3.8):
      S[r, c] = W_{l'} (1/2M) e^{ik rho}/rho,  rho = |x_r - x_c|;
* near panels (|i - i'| <= 1): the t_s integral over panel i' uses the 16
  nodes y_q and weights w_q of the near rule (Sec. 3.1); at each node the
  azimuthal integral is the discrete Parseval form of eq. (3.9),
      w_{j'}(t_s) = (1/2M) sum_{n=-M+1}^{M} kappa_n(t, theta_j, t_s) e^{i n theta_{j'}},
  and phi~ at the node is the Lagrange interpolant of the panel's 16
  Gauss-Legendre values (Sec. 3.4), so
      S[r, (i', l', j')] = sum_q (h/2) w_q ell_{l'}(y_q) w_{j'}(t_s(y_q)).
  The coefficients kappa_n come from ``coeffs.pairs_coeffs`` (direct
  quadrature of their definition).

Field (eq. (2.6) discretised the same way): u(x) = sum_c W_c (1/2M)
e^{ik|x - x_c|}/|x - x_c| phi~_c.
"""
import math

import numpy as np

from . import coeffs
from . import geometry as geo
from . import ggq

N16 = 16


def gauss_legendre():
    return np.polynomial.legendre.leggauss(N16)


def lagrange(xg, y):
    """ell_a(y) = prod_{b != a} (y - x_b) / (x_a - x_b), a = 0..15."""
    out = np.ones(N16)
    for a in range(N16):
        for b in range(N16):
            if b != a:
                out[a] *= (y - xg[b]) / (xg[a] - xg[b])
    return out


def layout(n_panels, M):
    """Per-unknown panel, node, azimuth, t, theta, and quadrature weight W/(2M)."""
    xg, wg = gauss_legendre()
    h = math.pi / n_panels
    r = np.arange(32 * M * n_panels)
    j = r % (2 * M)
    l = (r // (2 * M)) % N16
    i = r // (32 * M)
    t = i * h + 0.5 * h * (xg[l] + 1.0)
    th = math.pi * j / M
    wq = 0.5 * h * wg[l] / (2 * M)
    return dict(i=i, l=l, j=j, t=t, th=th, wq=wq, h=h)


def collocation(amp, n_panels, M):
    L = layout(n_panels, M)
    x = geo.point(amp, L["t"], L["th"])
    jac = geo.jacobian(amp, L["t"], L["th"])
    return x, jac, L["wq"]


def near_rule_nodes(tab, l, rel):
    return ggq.relation_rule(tab, l, rel)


def near_relations(i, n_panels):
    return [rel for rel in (-1, 0, 1) if 0 <= i + rel < n_panels]


def near_pairs(n_panels, M, tab):
    """All near pairs (t, j, t_s) in the library's order: panel, node, azimuth,
    relation, rule node."""
    xg, _ = gauss_legendre()
    h = math.pi / n_panels
    T, J, TS = [], [], []
    for i in range(n_panels):
        for l in range(N16):
            t = i * h + 0.5 * h * (xg[l] + 1.0)
            for j in range(2 * M):
                for rel in near_relations(i, n_panels):
                    y, _ = near_rule_nodes(tab, l, rel)
                    T.append(np.full(N16, t))
                    J.append(np.full(N16, j))
                    TS.append((i + rel) * h + 0.5 * h * (y + 1.0))
    return np.concatenate(T), np.concatenate(J).astype(np.int32), np.concatenate(TS)


def parseval_weights(kappa, M):
    """w_{j'} = (1/2M) sum_{n=-M+1}^{M} kappa_n e^{i n pi j'/M}, row-wise."""
    n = np.arange(-M + 1, M + 1)
    jp = np.arange(2 * M)
    E = np.exp(1j * np.pi * np.outer(n, jp) / M) / (2 * M)
    return kappa @ E


def near_block(kappa16, tab, l, rel, M, h):
    """Entries [16 l'][2M j'] of one (target, near panel) block from the 16
    coefficient rows of the target and the rule nodes of relation rel."""
    xg, _ = gauss_legendre()
    y, w = near_rule_nodes(tab, l, rel)
    wts = parseval_weights(kappa16, M)                        # [q][j']
    out = np.zeros((N16, 2 * M), dtype=complex)
    for q in range(N16):
        out += np.outer(0.5 * h * w[q] * lagrange(xg, y[q]), wts[q])
    return out


def near_kappa(amp, k, M, n_panels, rows, tab, processes=None, kind="S"):
    """Kernel coefficients of the near pairs of the given target rows:
    dict (row, rel) -> [16][2M].  For the sphere (amp all zero) the
    coefficients at azimuth j are those at azimuth 0 times e^{-i n theta_j}
    (rotation invariance, the axisymmetric relation of Remark 3.5)."""
    L = layout(n_panels, M)
    axisym = geo.is_axisymmetric(amp)
    keys, T, J, TS = [], [], [], []
    for r in rows:
        i, l, j = int(L["i"][r]), int(L["l"][r]), int(L["j"][r])
        for rel in near_relations(i, n_panels):
            y, _ = near_rule_nodes(tab, l, rel)
            keys.append((r, rel))
            T.append(np.full(N16, L["t"][r]))
            J.append(np.full(N16, 0 if axisym else j))
            TS.append((i + rel) * L["h"] + 0.5 * L["h"] * (y + 1.0))
    T, J, TS = np.concatenate(T), np.concatenate(J), np.concatenate(TS)
    def coefficient_rows(t_, j_, ts_):
        if kind == "S":
            return coeffs.pairs_coeffs(amp, k, M, 2 * M, t_, j_, ts_, processes=processes)[1]
        from . import double_layer
        return double_layer.pairs_kcoeffs(amp, k, M, t_, j_, ts_, adjoint=(kind == "Kp"),
                                          processes=processes)[0]

    if axisym:
        # one computation per distinct (t, t_s)
        uniq, inv = np.unique(np.stack([T, TS], 1), axis=0, return_inverse=True)
        kap_u = coefficient_rows(uniq[:, 0], np.zeros(len(uniq), int), uniq[:, 1])
        kap = kap_u[inv.ravel()]
        n = np.arange(-M + 1, M + 1)
        jrow = np.repeat([int(L["j"][r]) for r, _ in keys], N16)
        kap = kap * np.exp(-1j * np.outer(np.pi * jrow / M, n))
    else:
        kap = coefficient_rows(T, J, TS)
    return {key: kap[N16 * a:N16 * (a + 1)] for a, key in enumerate(keys)}


def rows(amp, k, M, n_panels, row_ids, tab, processes=None, kind="S"):
    """Full rows of S (kind "S"), of the double-layer operator K ("K") or of
    its adjoint K' ("Kp") for the given row indices, [len(row_ids)][N].  The
    far entries of K and K' are W_{l'} (1/2M) tau_0 (ik rho - 1) e^{ik rho} /
    rho^3 with tau_0 = nu_c . (x_c - x_r) (K) or nu_r . (x_r - x_c) (K'), the
    integrand of Sec. 4; the near blocks take the coefficients of
    double_layer.pairs_kcoeffs through the same rule as S."""
    L = layout(n_panels, M)
    N = 32 * M * n_panels
    x = geo.point(amp, L["t"], L["th"])
    nu = geo.normal(amp, L["t"], L["th"]) if kind != "S" else None
    kap = near_kappa(amp, k, M, n_panels, row_ids, tab, processes=processes, kind=kind)
    out = np.zeros((len(row_ids), N), dtype=complex)
    for a, r in enumerate(row_ids):
        i, l = int(L["i"][r]), int(L["l"][r])
        far = np.abs(L["i"] - i) >= 2
        d = x[far] - x[r]
        rho = np.linalg.norm(d, axis=1)
        if kind == "S":
            out[a, far] = L["wq"][far] * np.exp(1j * k * rho) / rho
        else:
            tz = np.einsum("nc,nc->n", nu[far], d) if kind == "K" else -(d @ nu[r])
            out[a, far] = L["wq"][far] * tz * (1j * k * rho - 1.0) * np.exp(1j * k * rho) / rho ** 3
        for rel in near_relations(i, n_panels):
            blk = near_block(kap[(r, rel)], tab, l, rel, M, L["h"])
            c0 = (i + rel) * 32 * M
            out[a, c0:c0 + 32 * M] = blk.ravel()
    return out


def matrix(amp, k, M, n_panels, tab, processes=None, kind="S"):
    return rows(amp, k, M, n_panels, np.arange(32 * M * n_panels), tab, processes=processes, kind=kind)


def field_double_layer(amp, n_panels, M, k, psi, pts):
    """Field of the double-layer representation of eq. (2.11),
    u(x) = 2 int dG(x, y)/d nu(y) psi(y) d sigma, by the product rule:
    u(x) = sum_c W_c tau_0 (ik rho - 1) e^{ik rho} / rho^3 psi~_c with
    tau_0 = nu_c . (x_c - x)."""
    x, _, wq = collocation(amp, n_panels, M)
    L = layout(n_panels, M)
    nu = geo.normal(amp, L["t"], L["th"])
    pts = np.atleast_2d(pts)
    out = np.zeros(len(pts), dtype=complex)
    for a, p in enumerate(pts):
        d = x - p
        rho = np.linalg.norm(d, axis=1)
        tz = np.einsum("nc,nc->n", nu, d)
        out[a] = np.sum(wq * tz * (1j * k * rho - 1.0) * np.exp(1j * k * rho) / rho ** 3 * psi)
    return out


def rhs_point_source(amp, n_panels, M, k, p):
    x, _, _ = collocation(amp, n_panels, M)
    rho = np.linalg.norm(x - np.asarray(p), axis=1)
    return np.exp(1j * k * rho) / (4 * np.pi * rho)


def rhs_plane_wave(amp, n_panels, M, k, d):
    x, _, _ = collocation(amp, n_panels, M)
    return -np.exp(1j * k * (x @ np.asarray(d)))


def rhs_plane_wave_dn(amp, n_panels, M, k, d):
    """-d/d nu e^{ik d.x} = -ik (d . nu) e^{ik d.x} on the collocation points
    (the sound-hard exterior problem)."""
    x, _, _ = collocation(amp, n_panels, M)
    L = layout(n_panels, M)
    nu = geo.normal(amp, L["t"], L["th"])
    return -1j * k * (nu @ np.asarray(d)) * np.exp(1j * k * (x @ np.asarray(d)))


def rhs_point_source_dn(amp, n_panels, M, k, p):
    """d/d nu G(x; p) on the collocation points, G = e^{ik rho} / (4 pi rho):
    dG/drho (x - p) . nu / rho with dG/drho = e^{ik rho} (ik rho - 1) / (4 pi rho^2)
    (the interior Neumann test of Sec. 5)."""
    x, _, _ = collocation(amp, n_panels, M)
    L = layout(n_panels, M)
    nu = geo.normal(amp, L["t"], L["th"])
    d = x - np.asarray(p)
    rho = np.linalg.norm(d, axis=1)
    dGdr = np.exp(1j * k * rho) * (1j * k * rho - 1.0) / (4 * np.pi * rho ** 2)
    return dGdr * np.einsum("nc,nc->n", d, nu) / rho


def field(amp, n_panels, M, k, phi, pts):
    x, _, wq = collocation(amp, n_panels, M)
    pts = np.atleast_2d(pts)
    out = np.zeros(len(pts), dtype=complex)
    for a, p in enumerate(pts):
        rho = np.linalg.norm(x - p, axis=1)
        out[a] = np.sum(wq * np.exp(1j * k * rho) / rho * phi)
    return out
