"""Generator of the built-in near-panel quadrature table (Sec. 3.1).

The log-singular t_s integral over the self panel and the two adjacent panels
uses, for each of the 16 Gauss-Legendre target positions x0 of a panel,
16-node generalized Gaussian rules (Bremer, Gimbutas and Rokhlin 2010).  In
the panel coordinate y in [-1, 1] they integrate exactly (to about 1e-14
relative) the 32 functions
    self panel:   P_k(y),  P_k(y) log|y - x0|,        k = 0..15,
    right panel:  P_k(y),  P_k(y) log(y + 2 - x0),    k = 0..15,
(the right-hand neighbour is the panel [1, 3] seen from the target's panel).
The left-hand rule for target x0 is the mirror image of the right-hand rule
for target -x0; the self rule for x0 < 0 is the mirror of the one for -x0.

Construction (node elimination):
  1. a graded composite Gauss-Legendre rule resolving the log singularity
     gives the moments and an oversampled starting rule;
  2. the function space is compressed to its numerical rank r by an SVD, and
     a pivoted QR of the orthonormal samples picks r nodes (Chebyshev rule);
  3. nodes are removed one at a time, least significant first, each removal
     followed by Gauss-Newton on the remaining nodes and weights, until 16
     nodes remain (acceptance threshold on the moment residual 3e-14 of the
     moment norm, relaxed to 1e-13 and 3e-13 where elimination stalls), then
     a last Gauss-Newton polish; a target on which elimination still stalls
     is reached by continuation in x0 from a neighbouring target's rule.

Run ``python -m paper_2608_16208_amd.ggq_gen`` to rewrite
``csrc/ggq16_table.inc``; the generated file is committed with the sources.
"""
import os
import sys

import numpy as np
from numpy.polynomial.legendre import leggauss
from scipy.linalg import qr

NK = 16                     # polynomial degree bound and node count
_HERE = os.path.dirname(os.path.abspath(__file__))
OUT = os.path.join(_HERE, "csrc", "ggq16_table.inc")


def _legendre(y):
    """Normalized Legendre values and derivatives, shape (NK, len(y))."""
    P = np.zeros((NK,) + y.shape)
    D = np.zeros_like(P)
    P[0] = 1.0
    P[1] = y
    D[1] = 1.0
    for k in range(1, NK - 1):
        P[k + 1] = ((2 * k + 1) * y * P[k] - k * P[k - 1]) / (k + 1)
        D[k + 1] = D[k - 1] + (2 * k + 1) * P[k]
    s = np.sqrt((2 * np.arange(NK) + 1) / 2.0).reshape((NK,) + (1,) * y.ndim)
    return P * s, D * s


def _system(y, x0, rel):
    """The 32 functions of the exactness set and their y-derivatives."""
    P, D = _legendre(y)
    if rel == 0:
        g, dg = np.log(np.abs(y - x0)), 1.0 / (y - x0)
    else:
        g, dg = np.log(y + 2.0 - x0), 1.0 / (y + 2.0 - x0)
    return np.concatenate([P, P * g]), np.concatenate([D, D * g + P * dg])


def _graded_rule(x0, rel, levels=40, ng=30):
    """Composite Gauss-Legendre rule graded geometrically toward the singular
    point; for the self panel x0 is a cut and the two innermost cells
    [x0, x0 +- d 2^-(levels-1)] are left out and integrated analytically in
    _moments."""
    g, w = leggauss(ng)
    cuts = [-1.0, 1.0]
    if rel == 0:
        cuts.append(x0)
        for side in (-1.0, 1.0):
            d = 1.0 - side * x0
            cuts += [x0 + side * d * 2.0 ** (-j) for j in range(levels)]
    else:
        cuts += [-1.0 + 2.0 * 2.0 ** (-j) for j in range(levels)]
    cuts = np.unique(np.clip(cuts, -1.0, 1.0))
    X, W = [], []
    for a, b in zip(cuts[:-1], cuts[1:]):
        if rel == 0 and (a == x0 or b == x0):
            continue
        X.append(0.5 * (b - a) * g + 0.5 * (a + b))
        W.append(0.5 * (b - a) * w)
    return np.concatenate(X), np.concatenate(W), levels


def _moments(x0, rel):
    X, W, levels = _graded_rule(x0, rel)
    F, _ = _system(X, x0, rel)
    mom = F @ W
    if rel == 0:
        # innermost cells, to first order in u = |y - x0| <= e = d 2^-(levels-1):
        # int_0^e (P(x0) + s P'(x0) u) (1, log u) du
        P, D = _legendre(np.array([x0]))
        for side in (-1.0, 1.0):
            e = (1.0 - side * x0) * 2.0 ** (-(levels - 1))
            mom[:NK] += P[:, 0] * e + side * D[:, 0] * (0.5 * e * e)
            mom[NK:] += P[:, 0] * (e * np.log(e) - e) + side * D[:, 0] * (0.5 * e * e * np.log(e) - 0.25 * e * e)
    return X, W, mom


def _gauss_newton(x, w, x0, rel, mom, tol, iters=60):
    n = len(x)
    F, G = _system(x, x0, rel)
    res = F @ w - mom
    nr = np.linalg.norm(res)
    for _ in range(iters):
        if nr < tol:
            return x, w, True
        J = np.concatenate([G * w[None, :], F], axis=1)
        step = np.linalg.lstsq(J, -res, rcond=1e-13)[0]
        lam, ok = 1.0, False
        for _ in range(30):
            xn, wn = x + lam * step[:n], w + lam * step[n:]
            if np.all(np.abs(xn) < 1.0) and (rel != 0 or np.all(np.abs(xn - x0) > 1e-13)):
                Fn, Gn = _system(xn, x0, rel)
                rn = Fn @ wn - mom
                if np.linalg.norm(rn) < nr:
                    ok = True
                    break
            lam *= 0.5
        if not ok:
            break
        x, w, F, G, res, nr = xn, wn, Fn, Gn, rn, np.linalg.norm(rn)
    return x, w, nr < tol


def _eliminate(x0, rel, tol_rel, eps=1e-14):
    X, W, mom = _moments(x0, rel)
    F, _ = _system(X, x0, rel)
    U, S, Vt = np.linalg.svd(F * np.sqrt(W)[None, :], full_matrices=False)
    r = int((S > eps * S[0]).sum())
    piv = qr(Vt[:r], pivoting=True, mode="economic")[2]
    sel = np.sort(piv[:r])
    x = X[sel]
    w = np.linalg.lstsq(F[:, sel], mom, rcond=None)[0]
    tol = tol_rel * np.linalg.norm(mom)
    x, w, _ = _gauss_newton(x, w, x0, rel, mom, tol)
    C = U[:, :r] / S[:r]
    while len(x) > NK:
        Fx, _ = _system(x, x0, rel)
        sig = np.abs(w) * ((C.T @ Fx) ** 2).sum(0)
        for i in np.argsort(sig):
            xn, wn, ok = _gauss_newton(np.delete(x, i), np.delete(w, i), x0, rel, mom, tol)
            if ok:
                x, w = xn, wn
                break
        else:
            break
    if len(x) == NK:                      # final polish toward the moment floor
        x, w, _ = _gauss_newton(x, w, x0, rel, mom, 1e-16 * np.linalg.norm(mom))
    o = np.argsort(x)
    return x[o], w[o]


def _continue(x, w, xa, xb, rel, tol_rel=1e-13, steps=40):
    for s in np.linspace(0.0, 1.0, steps + 1)[1:]:
        x0 = xa + s * (xb - xa)
        mom = _moments(x0, rel)[2]
        x, w, ok = _gauss_newton(x, w, x0, rel, mom, tol_rel * np.linalg.norm(mom))
        if not ok:
            return None
    o = np.argsort(x)
    return x[o], w[o]


def _rules_for(rel, targets, xg, log):
    rules = {}
    for l in targets:
        for tol_rel in (3e-14, 1e-13, 3e-13):
            x, w = _eliminate(xg[l], rel, tol_rel)
            if len(x) == NK and np.all(w > 0):
                rules[l] = (x, w)
                break
        log(f"rel {rel} target {l}: {len(x)} nodes by elimination")
    for l in targets:
        if l in rules:
            continue
        for m in sorted(rules, key=lambda m: abs(m - l)):
            out = _continue(*rules[m], xg[m], xg[l], rel)
            if out is not None and np.all(out[1] > 0):
                rules[l] = out
                log(f"rel {rel} target {l}: by continuation from target {m}")
                break
        else:
            raise RuntimeError(f"no 16-node rule for relation {rel}, target {l}")
    return rules


def generate(log=print):
    """Returns (self_nodes, self_weights, right_nodes, right_weights), each
    [16 targets][16 nodes] in panel coordinates on [-1, 1]."""
    xg = leggauss(NK)[0]
    sr = _rules_for(0, range(NK // 2, NK), xg, log)
    rr = _rules_for(1, range(NK), xg, log)
    sx = np.zeros((NK, NK)); sw = np.zeros((NK, NK))
    rx = np.zeros((NK, NK)); rw = np.zeros((NK, NK))
    for l in range(NK // 2, NK):
        sx[l], sw[l] = sr[l]
        sx[NK - 1 - l], sw[NK - 1 - l] = -sr[l][0][::-1], sr[l][1][::-1]
    for l in range(NK):
        rx[l], rw[l] = rr[l]
    return sx, sw, rx, rw


def write_table(path=OUT, log=print):
    sx, sw, rx, rw = generate(log)

    def block(name, a):
        rows = ",\n".join("  {" + ", ".join(float(v).hex() for v in row) + "}" for row in a)
        return f"static const double {name}[16][16] = {{\n{rows}}};\n"

    txt = ("// Generated by paper_2608_16208_amd/ggq_gen.py: 16-node generalized Gaussian\n"
           "// rules in panel coordinates, [target Gauss-Legendre index][node].\n"
           "// Self panel: exact for P_k(y), P_k(y) log|y - x0|; right neighbour: exact\n"
           "// for P_k(y), P_k(y) log(y + 2 - x0); k < 16.  Left = mirror of right.\n"
           + block("kGgqSelfNode", sx) + block("kGgqSelfWeight", sw)
           + block("kGgqRightNode", rx) + block("kGgqRightWeight", rw))
    tmp = path + ".tmp"
    with open(tmp, "w") as f:
        f.write(txt)
    os.replace(tmp, path)
    return sx, sw, rx, rw


if __name__ == "__main__":
    write_table(log=lambda s: print(s, file=sys.stderr, flush=True))
