"""Pins of the oracle's learned-preconditioner network and mode transforms."""
import numpy as np

from oracle import mlp as omlp


def _params(seed, scale=0.05):
    rng = np.random.default_rng(seed)
    return rng.uniform(-scale, scale, omlp.param_count())


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    p = _params(1)
    x = rng.standard_normal((5, omlp.N_IN))
    t = rng.standard_normal((5, omlp.N_OUT))
    _, g = omlp.gradients(p, x, t)
    h = 1e-6
    offs = np.cumsum([0] + [int(np.prod(s)) for s in omlp.SHAPES])
    # entries from every parameter block
    idx = np.concatenate([rng.integers(offs[b], offs[b + 1], 5) for b in range(len(omlp.SHAPES))])
    for i in idx:
        e = np.zeros_like(p)
        e[i] = h
        lp, _ = omlp.gradients(p + e, x, t)
        lm, _ = omlp.gradients(p - e, x, t)
        fd = (lp - lm) / (2 * h)
        # rounding of the O(100) loss over 2h gives ~1e-8; a wrong term is O(|g|)
        assert abs(fd - g[i]) <= 1e-5 * abs(g[i]) + 5e-8, (i, fd, g[i])


def test_loss_is_half_mean_square():
    rng = np.random.default_rng(2)
    p = np.zeros(omlp.param_count())
    x = rng.standard_normal((3, omlp.N_IN))
    t = rng.standard_normal((3, omlp.N_OUT))
    loss, _ = omlp.gradients(p, x, t)        # zero network: y = 0
    assert abs(loss - 0.5 * np.sum(t * t) / 3) < 1e-12


def test_bf16_rounding_ties_to_even_and_nearest():
    assert omlp.bf16_round(1.0) == 1.0
    assert omlp.bf16_round(1 + 2.0 ** -8) == 1.0                   # tie -> even
    assert omlp.bf16_round(1 + 3 * 2.0 ** -8) == 1 + 2.0 ** -6     # tie -> even
    assert omlp.bf16_round(-(1 + 3 * 2.0 ** -8)) == -(1 + 2.0 ** -6)
    rng = np.random.default_rng(3)
    v = rng.uniform(-4, 4, 200).astype(np.float32).astype(np.float64)
    r = omlp.bf16_round(v)
    for a, b in zip(v, r):
        e = np.floor(np.log2(abs(a)))
        grid = np.arange(-2 ** 9, 2 ** 9) * 2.0 ** (e - 7)              # bf16 spacing at a
        assert abs(b - a) <= np.min(np.abs(grid - a)) + 1e-300


def test_modes_roundtrip_and_single_mode():
    M, nodes = 8, 6
    rng = np.random.default_rng(4)
    e = rng.standard_normal(nodes * 2 * M) + 1j * rng.standard_normal(nodes * 2 * M)
    s = np.linalg.norm(omlp.modes(e, M, nodes), axis=1)
    y = omlp.targets(e, s, M, nodes)
    assert np.max(np.abs(omlp.reconstruct(y, s, M, nodes) - e)) < 1e-13
    th = np.pi * np.arange(2 * M) / M
    r = np.outer(np.arange(1, nodes + 1), np.exp(3j * th)).ravel()     # pure mode m = 3
    R = omlp.modes(r, M, nodes)
    assert np.allclose(R[3 + M - 1], np.arange(1, nodes + 1)) and np.abs(np.delete(R, 3 + M - 1, 0)).max() < 1e-13
    x, sc = omlp.features(r, M, nodes, k=6.0)
    assert abs(np.linalg.norm(x[3 + M - 1, :2 * nodes]) - 1.0) < 1e-14
    assert x[0, -2] == 6.0 / 30 and x[3 + M - 1, -1] == 3 / M
