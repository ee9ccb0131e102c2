"""Seeded synthetic workloads shared by the tests, the benchmark and the oracle.

This module holds shapes, seeds and sampling only -- none of the method's
arithmetic.  Every surface is a radial perturbation of the unit sphere,
    R(t, theta) = 1 + sum_{l,m} a[l-1, m] sin(l t) cos(m theta),
with t in [0, pi] split into ``n_panels`` equal panels of 16 Gauss-Legendre
nodes (Sec. 3.1) and 2M equispaced target azimuths theta_j = pi j / M
(eq. (3.8)).  The paper measures on analytic surfaces only; these seeded
stand-ins have the same structure (panel/node layout, azimuth grid, near and
far pair mix).
"""
import math

import numpy as np

GL_ORDER = 16


def gl_nodes(n=GL_ORDER):
    """Gauss-Legendre nodes and weights on [-1, 1] (numpy's rule)."""
    return np.polynomial.legendre.leggauss(n)


def panel_edges(n_panels, length=math.pi):
    return length * np.arange(n_panels + 1) / n_panels


def curve_nodes(n_panels, length=math.pi):
    """t_i^l for all panels, shape (n_panels, 16), and the GL weights w_i^l."""
    x, w = gl_nodes()
    e = panel_edges(n_panels, length)
    half = 0.5 * (e[1:] - e[:-1])
    mid = 0.5 * (e[1:] + e[:-1])
    return mid[:, None] + half[:, None] * x[None, :], half[:, None] * w[None, :]


def star_amplitudes(lmax, mmax, scale, rng):
    """Amplitude table a[l-1, m] ~ U(-scale, scale), drawn l-major."""
    return rng.uniform(-scale, scale, size=(lmax, mmax + 1))


def random_direction(rng):
    d = rng.standard_normal(3)
    return d / np.linalg.norm(d)


def config(i):
    """The five benchmark configurations (shapes, seeds, amplitudes)."""
    if i == 1:
        return dict(name="sphere-k1-Np8-M32", amp=np.zeros((0, 1)), k=1.0, n_panels=8, M=32,
                    d=np.array([0.0, 0.0, 1.0]), seed=1)
    if i == 2:
        amp = np.zeros((3, 3))
        amp[2, 2] = 0.2                      # 0.2 sin(3t) cos(2 theta)
        rng = np.random.default_rng(2)
        return dict(name="star-k5-Np16-M64", amp=amp, k=5.0, n_panels=16, M=64,
                    d=random_direction(rng), seed=2)
    if i == 3:
        rng = np.random.default_rng(3)
        amp = star_amplitudes(4, 4, 0.1, rng)
        return dict(name="star20-k20-Np32-M128", amp=amp, k=20.0, n_panels=32, M=128,
                    d=random_direction(rng), seed=3)
    raise ValueError(i)


def _min_radius(amp, n=256):
    t = np.linspace(0, math.pi, n)
    th = np.linspace(0, 2 * math.pi, n, endpoint=False)
    R = np.ones((n, n))
    for l in range(amp.shape[0]):
        for m in range(amp.shape[1]):
            R += amp[l, m] * np.outer(np.sin((l + 1) * t), np.cos(m * th))
    return R.min()


BATCH_M = (16, 24, 32, 48, 64, 96, 128)     # M in [16, 128] with 2M = 2^a 3^b


def batch_surface(s):
    """Member s of the 64-surface batch: 20 amplitudes a_lm ~ U(-0.15, 0.15)
    (l = 1..4, m = 0..4, l-major; redrawn while min R < 0.5 on a 256^2 grid),
    then n_panels ~ U{4..32}, M uniform on BATCH_M (16 .. 128, the sizes whose
    2M-point transforms factor into radix 2 and 3) and k ~ U[2, 25], all from
    rng(100 + s)."""
    rng = np.random.default_rng(100 + s)
    amp = star_amplitudes(4, 4, 0.15, rng)
    while _min_radius(amp) < 0.5:
        amp = star_amplitudes(4, 4, 0.15, rng)
    n_panels = int(rng.integers(4, 33))
    M = int(rng.choice(BATCH_M))
    k = float(rng.uniform(2.0, 25.0))
    return dict(name=f"batch-star-{s}", amp=amp, k=k, n_panels=n_panels, M=M, seed=100 + s)


def learned_surface(i, held_out=False):
    """Surfaces of the learned-preconditioner study: 20 amplitudes
    a_lm ~ U(-0.1, 0.1) (l = 1..4, m = 0..4, l-major; redrawn while min R < 0.5),
    then k ~ U[5, 30]; rng(1000 + i) for training, rng(2000 + i) held out.
    16 panels (256 curve nodes), M = 64."""
    rng = np.random.default_rng((2000 if held_out else 1000) + i)
    amp = star_amplitudes(4, 4, 0.1, rng)
    while _min_radius(amp) < 0.5:
        amp = star_amplitudes(4, 4, 0.1, rng)
    k = float(rng.uniform(5.0, 30.0))
    return dict(name=f"learned-{'test' if held_out else 'train'}-{i}", amp=amp, k=k, n_panels=16, M=64,
                seed=(2000 if held_out else 1000) + i)


# The interior point-source protocol of Sec. 5 on an analytic star surface
# (azimuthal order 1 keeps the poles smooth): R = 1 + 0.2 sin t cos(theta) +
# 0.1 sin(2t) cos(theta).  Source r* = (3, 4, 10.5) outside; the test region
# is the ball |r - (0, -0.2, 0.1)| < 0.2 of the paper's Example 1, sampled at
# seeded points; (k, n_panels, M) follow the paper's (k, N_p, 2M) rows with the
# nearest supported M.
INTERIOR_AMP = np.array([[0.0, 0.2], [0.0, 0.1]])
INTERIOR_SOURCE = np.array([3.0, 4.0, 10.5])
INTERIOR_ROWS = ((1.0, 4, 16), (2.0, 4, 16), (4.0, 4, 16), (8.0, 8, 32), (16.0, 16, 64))


# Sec. 5, Example 1: the ellipsoid x^2 + y^2/4 + z^2/9 = 1 (the unit sphere
# stretched by these axes), and the rows of the paper's Table 1: k, then for
# S, K and K' the (N_p, 2M) used and the error E_j it reports.  The rows run
# here take the same N_p and the next supported 2M (a power of two).
ELLIPSOID_AXES = (1.0, 2.0, 3.0)
PAPER_TABLE1 = (
    (1.0, (4, 30), 6.4e-11, (4, 40), 7.6e-12, (4, 40), 1.3e-11),
    (2.0, (4, 30), 1.2e-10, (4, 40), 1.6e-11, (4, 40), 9.3e-12),
    (4.0, (4, 30), 8.4e-10, (4, 40), 1.2e-10, (4, 40), 2.6e-10),
    (8.0, (8, 60), 9.7e-11, (8, 60), 2.3e-11, (8, 60), 2.2e-10),
    (16.0, (16, 100), 9.6e-10, (16, 100), 7.2e-11, (16, 100), 8.0e-12),
)


def supported_M(two_m):
    """The smallest supported M (16, 32, 64, 128) with 2M >= two_m."""
    for M in (16, 32, 64, 128):
        if 2 * M >= two_m:
            return M
    raise ValueError(two_m)


def interior_test_points(n=200, seed=5, center=(0.0, -0.2, 0.1), radius=0.2):
    """Seeded points uniform in the test ball Omega_T."""
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1)[:, None]
    return np.asarray(center) + radius * d * rng.uniform(0.0, 1.0, n)[:, None] ** (1.0 / 3.0)


def all_pairs(n_panels, M, length=math.pi):
    """Every (target node, target azimuth, source curve node) with t_s != t.

    Order: target node i (outer), source node s, target azimuth j (inner).
    Returns float64 t, int32 j, float64 ts.
    """
    t_nodes = curve_nodes(n_panels, length)[0].ravel()
    n = t_nodes.size
    ii, ss = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    keep = ii != ss
    ii, ss = ii[keep], ss[keep]
    nj = 2 * M
    t = np.repeat(t_nodes[ii], nj)
    ts = np.repeat(t_nodes[ss], nj)
    j = np.tile(np.arange(nj, dtype=np.int32), ii.size)
    return t, j, ts


def sample_pairs(n_panels, M, n, seed, near_fraction=0.3, length=math.pi):
    """Seeded sample of pairs: curve-node pairs plus near pairs.

    A fraction ``near_fraction`` of the pairs put the source a log-uniform
    distance 10^-7 .. 10^-1 (times the panel length) from the target node, as
    the near-panel quadrature nodes do; the rest pair two distinct curve nodes.
    """
    rng = np.random.default_rng(seed)
    t_nodes = curve_nodes(n_panels, length)[0].ravel()
    nt = t_nodes.size
    n_near = int(round(near_fraction * n))
    n_far = n - n_near
    i = rng.integers(0, nt, size=n_far)
    s = (i + rng.integers(1, nt, size=n_far)) % nt
    t_far, ts_far = t_nodes[i], t_nodes[s]
    i2 = rng.integers(0, nt, size=n_near)
    h = length / n_panels
    off = h * 10.0 ** rng.uniform(-7, -1, size=n_near) * rng.choice([-1.0, 1.0], size=n_near)
    t_near = t_nodes[i2]
    ts_near = np.clip(t_near + off, 1e-3, length - 1e-3)
    t = np.concatenate([t_far, t_near])
    ts = np.concatenate([ts_far, ts_near])
    j = rng.integers(0, 2 * M, size=n).astype(np.int32)
    return t, j, ts
