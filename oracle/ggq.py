"""Near-panel quadrature rules for the oracle (Sec. 3.1).  TEST INFRASTRUCTURE.

The t_s integral over the target's own panel and its two neighbours carries
the logarithmic singularity of Theorem 3.1; the paper integrates it with
16-node generalized Gaussian rules, one per target position, whose nodes and
weights it takes from an external generator.  This module builds its own
such rules, written independently of the GPU package:

* exactness set, in the panel coordinate y in [-1, 1] with target x0:
    self panel       T_k(y), T_k(y) log|y - x0|        (k < 16, Chebyshev T_k)
    right neighbour  T_k(y), T_k(y) log(y + 2 - x0)
  (any basis of polynomials of degree < 16 spans the same space);
* exact moments by QUADPACK's algebraic-logarithmic weights (QAWS), split at
  x0 for the self panel;
* rule by node elimination (Bremer, Gimbutas, Rokhlin 2010): rank-revealing
  selection of a Chebyshev rule from a graded oversampled rule, then removal of
  one node at a time with a Gauss-Newton re-fit of the moments, down to 16
  (where elimination stalls, continuation in x0 from a neighbouring target);
* symmetry: the self rule for -x0 is the mirror image of the one for x0, and
  the left-neighbour rule for x0 is the mirror of the right-neighbour rule for
  -x0.

Rules of this kind are not unique, so a rule is judged by its exactness
(``moment_residual``, checked in the tests with 30-digit moments from mpmath),
and parity of the GPU near blocks is taken with the same rule loaded on both
sides.
"""
import numpy as np
from numpy.polynomial import chebyshev as C
from numpy.polynomial.legendre import leggauss
from scipy import integrate
from scipy.linalg import qr

N = 16


def functions(y, x0, rel):
    """Values and y-derivatives of the 32 exactness functions, (32, len(y))."""
    y = np.asarray(y, dtype=float)
    T = np.stack([C.chebval(y, np.eye(N)[k]) for k in range(N)])
    dT = np.stack([C.chebval(y, C.chebder(np.eye(N)[k])) for k in range(N)])
    d = (y - x0) if rel == 0 else (y + 2.0 - x0)
    g = np.log(np.abs(d))
    return np.vstack([T, T * g]), np.vstack([dT, dT * g + T / d])


def exact_moments(x0, rel):
    """int_{-1}^{1} of the 32 functions, by QUADPACK with log weights."""
    m = np.zeros(2 * N)
    for k in range(N):
        tk = lambda y, k=k: C.chebval(y, np.eye(N)[k])
        m[k] = integrate.quad(tk, -1.0, 1.0, epsabs=1e-16, epsrel=1e-15, limit=200)[0]
        if rel == 0:
            a = integrate.quad(tk, x0, 1.0, weight="alg-loga", wvar=(0.0, 0.0),
                               epsabs=1e-16, epsrel=1e-15, limit=200)[0]
            b = integrate.quad(tk, -1.0, x0, weight="alg-logb", wvar=(0.0, 0.0),
                               epsabs=1e-16, epsrel=1e-15, limit=200)[0]
            m[N + k] = a + b
        else:
            # log(y + 2 - x0) is smooth on [-1, 1]; split near its end y = -1
            f = lambda y, k=k: C.chebval(y, np.eye(N)[k]) * np.log(y + 2.0 - x0)
            pts = [-1.0 + (1.0 - x0) * 2.0 ** j for j in range(0, 6) if -1.0 + (1.0 - x0) * 2.0 ** j < 1.0]
            m[N + k] = integrate.quad(f, -1.0, 1.0, points=pts, epsabs=1e-16, epsrel=1e-15, limit=400)[0]
    return m


def _oversampled(x0, rel, per=24, depth=44):
    g, w = leggauss(per)
    if rel == 0:
        cuts = {-1.0, 1.0}
        for s in (-1.0, 1.0):
            span = 1.0 - s * x0
            cuts |= {x0 + s * span * 0.5 ** j for j in range(depth)}
        cuts = sorted(c for c in cuts if -1.0 <= c <= 1.0 and c != x0)
        cells = [(a, b) for a, b in zip(cuts[:-1], cuts[1:]) if not (a < x0 < b)]
    else:
        cuts = sorted({-1.0, 1.0} | {-1.0 + 2.0 * 0.5 ** j for j in range(depth)})
        cells = list(zip(cuts[:-1], cuts[1:]))
    X = np.concatenate([0.5 * (b - a) * g + 0.5 * (a + b) for a, b in cells])
    W = np.concatenate([0.5 * (b - a) * w for a, b in cells])
    return X, W


def _refit(x, w, x0, rel, m, tol, iters=80):
    """Gauss-Newton (minimum-norm steps, backtracking) on sum_q w_q f(x_q) = m."""
    n = x.size
    F, D = functions(x, x0, rel)
    r = F @ w - m
    for _ in range(iters):
        if np.linalg.norm(r) <= tol:
            return x, w, True
        J = np.hstack([D * w, F])
        dz = np.linalg.lstsq(J, -r, rcond=1e-13)[0]
        t = 1.0
        while t > 1e-9:
            xn, wn = x + t * dz[:n], w + t * dz[n:]
            if np.all(np.abs(xn) < 1.0) and (rel != 0 or np.min(np.abs(xn - x0)) > 1e-13):
                Fn, Dn = functions(xn, x0, rel)
                rn = Fn @ wn - m
                if np.linalg.norm(rn) < np.linalg.norm(r):
                    break
            t *= 0.5
        else:
            return x, w, False
        x, w, F, D, r = xn, wn, Fn, Dn, rn
    return x, w, np.linalg.norm(r) <= tol


def _continuation(x, w, xa, xb, rel, steps=24, tol_rel=1e-12):
    """Carry a 16-node rule for target xa along x0 from xa to xb."""
    for s in np.linspace(0.0, 1.0, steps + 1)[1:]:
        x0 = xa + s * (xb - xa)
        m = exact_moments(x0, rel)
        x, w, ok = _refit(x, w, x0, rel, m, tol_rel * np.linalg.norm(m))
        if not ok:
            return None
    x, w, _ = _refit(x, w, xb, rel, m, 1e-16 * np.linalg.norm(m))
    o = np.argsort(x)
    return x[o], w[o]


def rule(x0, rel):
    """A 16-node rule for target x0 (panel coordinate) and relation rel
    (0 = self, 1 = right neighbour): (nodes ascending, weights)."""
    m = exact_moments(x0, rel)
    X, W = _oversampled(x0, rel)
    F, _ = functions(X, x0, rel)
    # Chebyshev rule on the numerical range of the function space
    U, s, Vt = np.linalg.svd(F * np.sqrt(W), full_matrices=False)
    rank = int(np.sum(s > 1e-14 * s[0]))
    keep = np.sort(qr(Vt[:rank], pivoting=True, mode="economic")[2][:rank])
    for tol_rel in (3e-14, 1e-13, 3e-13, 1e-12):
        tol = tol_rel * np.linalg.norm(m)
        x = X[keep].copy()
        w = np.linalg.lstsq(F[:, keep], m, rcond=None)[0]
        x, w, _ = _refit(x, w, x0, rel, m, tol)
        proj = U[:, :rank].T / s[:rank, None]
        while x.size > N:
            Fx, _ = functions(x, x0, rel)
            weight = np.abs(w) * np.sum((proj @ Fx) ** 2, axis=0)
            for i in np.argsort(weight):
                xn, wn, ok = _refit(np.delete(x, i), np.delete(w, i), x0, rel, m, tol)
                if ok:
                    x, w = xn, wn
                    break
            else:
                break
        if x.size == N and np.all(w > 0):
            x, w, _ = _refit(x, w, x0, rel, m, 1e-16 * np.linalg.norm(m))
            o = np.argsort(x)
            return x[o], w[o]
    raise RuntimeError(f"node elimination stalled at {x.size} nodes (x0={x0}, rel={rel})")


def table():
    """Rules for all 16 Gauss-Legendre targets: dict with arrays
    self_x, self_w, right_x, right_w of shape (16, 16)."""
    xg = leggauss(N)[0]
    out = {k: np.zeros((N, N)) for k in ("self_x", "self_w", "right_x", "right_w")}
    for l in range(N // 2, N):
        x, w = rule(xg[l], 0)
        out["self_x"][l], out["self_w"][l] = x, w
        out["self_x"][N - 1 - l], out["self_w"][N - 1 - l] = -x[::-1], w[::-1]
    stalled = []
    for l in range(N):
        try:
            out["right_x"][l], out["right_w"][l] = rule(xg[l], 1)
        except RuntimeError:
            stalled.append(l)
    for l in stalled:                      # continuation from the nearest solved target
        for m in sorted((m for m in range(N) if m not in stalled), key=lambda m: abs(m - l)):
            got = _continuation(out["right_x"][m], out["right_w"][m], xg[m], xg[l], 1)
            if got is not None and np.all(got[1] > 0):
                out["right_x"][l], out["right_w"][l] = got
                break
        else:
            raise RuntimeError(f"no 16-node right-neighbour rule for target {l}")
    return out


def relation_rule(tab, l, rel):
    """Nodes and weights in the source panel's coordinate for target index l;
    rel = -1 (left neighbour), 0 (self), +1 (right neighbour)."""
    if rel == 0:
        return tab["self_x"][l], tab["self_w"][l]
    if rel == 1:
        return tab["right_x"][l], tab["right_w"][l]
    return -tab["right_x"][N - 1 - l][::-1], tab["right_w"][N - 1 - l][::-1]


def moment_residual(x, w, x0, rel, dps=30):
    """Max over the 32 exactness functions of |rule - integral| / int |f|,
    with the integrals in `dps`-digit arithmetic (mpmath, Legendre basis so
    that the check does not reuse this module's basis or moments)."""
    import mpmath as mp
    mp.mp.dps = dps
    x0m = mp.mpf(float(x0))
    worst = 0.0
    for k in range(N):
        for lg in (False, True):
            if rel == 0:
                f = lambda y: mp.legendre(k, y) * (mp.log(abs(y - x0m)) if lg else 1)
                exact = mp.quad(f, [-1, x0m, 1])
                absint = mp.quad(lambda y: abs(f(y)), [-1, x0m, 1])
            else:
                f = lambda y: mp.legendre(k, y) * (mp.log(y + 2 - x0m) if lg else 1)
                exact = mp.quad(f, [-1, 1])
                absint = mp.quad(lambda y: abs(f(y)), mp.linspace(-1, 1, 9))
            approx = mp.fsum(mp.mpf(float(wq)) * f(mp.mpf(float(xq))) for xq, wq in zip(x, w))
            worst = max(worst, float(abs(approx - exact) / absint))
    return worst
