"""GPU parity of the O(M) banded route to <rho^-1>_l (Sec. 3.2.1).

The library's route (ffbie_rhoinv_banded) is checked against
* the oracle's banded route (known values of eq. (3.16) by direct quadrature
  of their definition, a dense solve of eq. (3.17)) and against that direct
  quadrature itself, on seeded pairs of configs 1-3;
* the unit sphere's closed form (Legendre functions of the second kind);
* the singularity-swapping path's <rho^-1> (ffbie_kernel_coeffs), on sampled
  rows of the full config-2 all-pairs launch that bench.py times.
Tolerance, relative to each row's largest coefficient: the banded route's
rounding is that of a linear solve, about u cond(A) (u = 2^-53), and cond(A)
grows like L^2: on seeded pairs 6.4e3 (L = 64), 2.1e4 (L = 128) and 9.3e4
(L = 256), at most 1.6 L^2, with the oracle's error at most 2.2 u cond(A).
Rows checked against the oracle take 8 u cond(A) of that row's A (from the
oracle) plus 1e-14; rows checked against the swap path, whose own error is
~1e-14, take 8 u (2 L^2).
"""
import math
import multiprocessing as mp

import numpy as np
import pytest

import workloads
from oracle import banded as ob
from oracle import coeffs as ocoeffs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

U = 2.0 ** -53


def swap_tol(L):
    return 8 * U * 2 * L * L


@pytest.fixture(scope="module")
def ctx():
    import paper_2608_16208_amd as ffbie
    c = ffbie.Context(0)
    yield c
    c.close()


def _banded(ctx, cfg, t, j, ts, m0=0, M0=None):
    ctx.set_problem(cfg["amp"], cfg["n_panels"], cfg["M"], cfg["k"], M0=M0)
    dev = ctx.device
    out = ctx.rhoinv_banded(torch.tensor(t, device=dev), torch.tensor(j, device=dev),
                            torch.tensor(ts, device=dev), m0=m0)
    torch.cuda.synchronize()
    return out["rhoinv"].cpu().numpy(), out["status"].cpu().numpy(), out["m0"]


def _oracle_row(args):
    amp, M, t, j, ts, m0 = args
    c, info = ob.rhoinv_banded(amp, M, M, t, j, ts, m0)
    ev = np.linalg.eigvalsh(info["A"])
    return c, info["direct"], ev.max() / ev.min()


def _oracle(cfg, t, j, ts, m0, processes=8):
    """The oracle's banded rows, its direct-quadrature rows and cond(A) per row."""
    args = [(cfg["amp"], cfg["M"], float(t[i]), int(j[i]), float(ts[i]), m0) for i in range(len(t))]
    with mp.get_context("fork").Pool(processes, initializer=ocoeffs._one_thread) as pool:
        res = pool.map(_oracle_row, args, chunksize=2)
    return tuple(np.array([r[q] for r in res]) for q in range(3))


def _row_tol(cond):
    return 8 * U * cond + 1e-14


def _row_err(a, b):
    return np.max(np.abs(a - b), axis=1) / np.max(np.abs(b), axis=1)


@pytest.mark.parametrize("cfgi", [1, 2, 3])
def test_banded_matches_oracle_sampled_pairs(ctx, cfgi):
    cfg = workloads.config(cfgi)
    t, j, ts = workloads.sample_pairs(cfg["n_panels"], cfg["M"], 48, seed=300 + cfgi)
    got, st, m0 = _banded(ctx, cfg, t, j, ts)
    assert m0 == ob.degree_bound(cfg["amp"]), m0
    assert not (st & 1).any()
    ref, direct, cond = _oracle(cfg, t, j, ts, m0)
    e_banded = _row_err(got, ref)
    e_direct = _row_err(got, direct)
    print("config %d m0 %d: vs oracle banded %.2e, vs direct quadrature %.2e (max cond %.1e, worst "
          "error / (u cond) %.2f), not-PD pairs %d"
          % (cfgi, m0, e_banded.max(), e_direct.max(), cond.max(), (e_direct / (U * cond)).max(),
             int(((st & 32) > 0).sum())), flush=True)
    assert np.all(e_direct <= _row_tol(cond)), (e_direct / _row_tol(cond)).max()
    assert np.all(e_banded <= 2 * _row_tol(cond)), (e_banded / _row_tol(cond)).max()


def test_banded_sphere_closed_form(ctx):
    from test_oracle_pins import _sphere_closed_form
    cfg = workloads.config(1)
    M = cfg["M"]
    t = np.array([0.3, 1.2, 1.2, 2.0, 0.05])
    ts = np.array([0.3 + 1e-6, 1.2 + 3e-5, 2.9, 2.2, 3.0])
    j = np.array([7, 0, 3, 17, 40], dtype=np.int32)
    got, st, m0 = _banded(ctx, cfg, t, j, ts)
    assert m0 == 1                              # Remark 3.5
    ref = np.array([_sphere_closed_form(t[i], math.pi * j[i] / M, ts[i], 2 * M) for i in range(len(t))])
    err = _row_err(got, ref)
    _, _, cond = _oracle(cfg, t, j, ts, 1)
    assert np.all(err <= _row_tol(cond)), (err, cond)


def test_banded_m0_above_degree_agrees(ctx):
    """An explicit m0 above the degree of rho^2 adds bands of (rounding-level)
    zero coefficients and more known values: the same coefficients."""
    cfg = workloads.config(2)
    t, j, ts = workloads.sample_pairs(cfg["n_panels"], cfg["M"], 256, seed=41)
    a, _, m0a = _banded(ctx, cfg, t, j, ts, m0=0)
    b, _, m0b = _banded(ctx, cfg, t, j, ts, m0=6)
    assert (m0a, m0b) == (4, 6)
    assert _row_err(b, a).max() <= swap_tol(2 * cfg["M"])


@pytest.mark.parametrize("M", [16, 32, 128])
def test_banded_matches_swap_other_sizes(ctx, M):
    """Against the swap path on the pairs its 2M or 4M samples resolve (status
    without FFBIE_PAIR_UNRESOLVED: at M = 16 some config-2 pairs are not), and
    the rows that differ most against the oracle's direct quadrature."""
    import paper_2608_16208_amd as ffbie
    cfg = dict(workloads.config(2))
    cfg["M"] = M
    t, j, ts = workloads.sample_pairs(cfg["n_panels"], M, 4096, seed=7 + M)
    got, st, m0 = _banded(ctx, cfg, t, j, ts)
    ctx.set_problem(cfg["amp"], cfg["n_panels"], M, cfg["k"])
    dev = ctx.device
    sw = ctx.kernel_coeffs(torch.tensor(t, device=dev), torch.tensor(j, device=dev),
                           torch.tensor(ts, device=dev), rhoinv=True)
    ref = sw["rhoinv"].cpu().numpy()
    resolved = (sw["status"].cpu().numpy() & ffbie.PAIR_UNRESOLVED) == 0
    err = _row_err(got, ref)
    print("M %d: banded vs swap worst %.2e, median %.2e over %d resolved pairs (%d unresolved)"
          % (M, err[resolved].max(), np.median(err[resolved]), resolved.sum(), (~resolved).sum()),
          flush=True)
    assert err[resolved].max() <= swap_tol(2 * M), err[resolved].max()
    worst = np.argsort(-err)[:8]
    _, direct, cond = _oracle(cfg, t[worst], j[worst], ts[worst], m0)
    e = _row_err(got[worst], direct)
    assert np.all(e <= _row_tol(cond)), (e, cond)


def test_banded_config2_all_pairs_full_size_sampled(ctx):
    """The launch bench.py times: all 8,355,840 pairs of config 2 (M = 64).
    Every row against the swap path's, a sample against the oracle."""
    cfg = workloads.config(2)
    t, j, ts = workloads.all_pairs(cfg["n_panels"], cfg["M"])
    ctx.set_problem(cfg["amp"], cfg["n_panels"], cfg["M"], cfg["k"])
    dev = ctx.device
    tt, jj, tss = (torch.tensor(v, device=dev) for v in (t, j, ts))
    band = ctx.rhoinv_banded(tt, jj, tss)
    assert band["m0"] == 4
    sw = ctx.kernel_coeffs(tt, jj, tss, rhoinv=True)
    torch.cuda.synchronize()
    a, b = band["rhoinv"], sw["rhoinv"]
    err = torch.amax(torch.abs(a - b), dim=1) / torch.amax(torch.abs(b), dim=1)
    worst = float(err.max())
    st = band["status"].cpu().numpy()
    print("all pairs: banded vs swap worst %.2e, not-PD pairs %d" % (worst, int(((st & 32) > 0).sum())),
          flush=True)
    assert not (st & 1).any()
    assert worst <= swap_tol(2 * cfg["M"]), worst
    rng = np.random.default_rng(9)
    idx = np.sort(rng.choice(t.size, 24, replace=False))
    _, direct, cond = _oracle(cfg, t[idx], j[idx], ts[idx], 4)
    e = _row_err(a[idx].cpu().numpy(), direct)
    assert np.all(e <= _row_tol(cond)), (e / _row_tol(cond)).max()
    del band, sw, a, b


def test_banded_singular_pair_empty_and_errors(ctx):
    import paper_2608_16208_amd as ffbie
    cfg = workloads.config(2)
    got, st, m0 = _banded(ctx, cfg, np.array([0.7, 0.7]), np.array([3, 5], dtype=np.int32),
                          np.array([0.7, 0.9]))
    assert st[0] & ffbie.PAIR_SINGULAR and np.isnan(got[0]).all()
    assert not (st[1] & ffbie.PAIR_SINGULAR) and np.isfinite(got[1]).all()
    dev = ctx.device
    empty = torch.zeros(0, dtype=torch.float64, device=dev)
    out = ctx.rhoinv_banded(empty, torch.zeros(0, dtype=torch.int32, device=dev), empty)
    assert out["rhoinv"].shape == (0, cfg["M"] * 2 + 1)
    one = torch.tensor([0.7], dtype=torch.float64, device=dev)
    az = torch.tensor([3], dtype=torch.int32, device=dev)
    for bad in (-1, 9):
        with pytest.raises(ffbie.FfbieError):
            ctx.rhoinv_banded(one, az, one + 0.1, m0=bad)
    ctx.set_problem(cfg["amp"], cfg["n_panels"], 16, cfg["k"], M0=4)   # L = 20 < 4 m0
    with pytest.raises(ffbie.FfbieError):
        ctx.rhoinv_banded(one, az, one + 0.1, m0=8)
