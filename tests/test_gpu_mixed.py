"""GPU parity of the mixed-precision coefficient path (FP32 spectral stage,
FP64 samples, root and A_m recurrences; complex64 outputs).

Tolerance: per-pair relative 2-norm error <= 1e-5 against the FP64 oracle.
The path truncates the smooth factor at 1e-6 of its largest coefficient (the
FP32 transforms leave a rounding floor of a few 1e-7 there); the dropped tail
decays geometrically, and the FP32 sums over 2p + 1 <= NF terms add
O(sqrt(NF) u_32) ~ 1e-6, so the bound leaves a factor of a few over the
expected ~2e-6.  The values observed are reported in the assertion messages.
"""
import numpy as np
import pytest

import workloads
from oracle import coeffs as ocoeffs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL_MIXED = 1e-5


@pytest.fixture(scope="module")
def ctx():
    import paper_2608_16208_amd as ffbie
    c = ffbie.Context(0)
    yield c
    c.close()


def _run(ctx, cfg, t, j, ts, variant=0, mixed=True, rhoinv=True):
    ctx.set_problem(cfg["amp"], cfg["n_panels"], cfg["M"], cfg["k"], variant=variant)
    dev = ctx.device
    out = ctx.kernel_coeffs(torch.tensor(t, device=dev), torch.tensor(j, device=dev),
                            torch.tensor(ts, device=dev), rhoinv=rhoinv, mixed=mixed)
    torch.cuda.synchronize()
    return {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}


def _oracle(cfg, t, j, ts, processes=8):
    M = cfg["M"]
    c_o, k_o, info = ocoeffs.pairs_coeffs(cfg["amp"], cfg["k"], M, 2 * M, t, j, ts,
                                          processes=processes)
    assert all(i["converged"] for i in info)
    return c_o, k_o


def _relerr(x, ref):
    return np.linalg.norm(x.astype(np.complex128) - ref, axis=1) / np.linalg.norm(ref, axis=1)


@pytest.mark.parametrize("variant", [0, 1])
@pytest.mark.parametrize("cfgi", [1, 2, 3])
def test_mixed_matches_oracle_sampled_pairs(ctx, cfgi, variant):
    cfg = workloads.config(cfgi)
    t, j, ts = workloads.sample_pairs(cfg["n_panels"], cfg["M"], 160, seed=100 + cfgi)
    out = _run(ctx, cfg, t, j, ts, variant=variant)
    assert out["kappa"].dtype == np.complex64 and out["rhoinv"].dtype == np.complex64
    assert not (out["status"] & 8).any(), "unresolved smooth factor"
    c_o, k_o = _oracle(cfg, t, j, ts)
    ek, ec = _relerr(out["kappa"], k_o), _relerr(out["rhoinv"], c_o)
    print("config %d variant %d: max rel err kappa %.2e rhoinv %.2e" % (cfgi, variant, ek.max(), ec.max()))
    assert ek.max() <= TOL_MIXED and ec.max() <= TOL_MIXED, (ek.max(), ec.max())


def test_mixed_config2_all_pairs_full_size(ctx):
    """The benchmarked launch in mixed precision: all 8,355,840 pairs of
    config 2.  Every row is compared with the FP64 path of the same launch, and
    rows sampled uniformly (plus refined and root-fallback pairs) with the
    oracle."""
    cfg = workloads.config(2)
    t, j, ts = workloads.all_pairs(cfg["n_panels"], cfg["M"])
    ctx.set_problem(cfg["amp"], cfg["n_panels"], cfg["M"], cfg["k"])
    dev = ctx.device
    tt, jj, tss = (torch.tensor(v, device=dev) for v in (t, j, ts))
    o32 = ctx.kernel_coeffs(tt, jj, tss, mixed=True)
    o64 = ctx.kernel_coeffs(tt, jj, tss)
    torch.cuda.synchronize()
    st = o32["status"].cpu().numpy()
    assert not (st & 1).any() and not (st & 8).any(), ((st & 8) > 0).sum()
    worst = 0.0
    n = t.size
    for a in range(0, n, 1 << 20):
        k32 = o32["kappa"][a:a + (1 << 20)].to(torch.complex128)
        k64 = o64["kappa"][a:a + (1 << 20)]
        e = torch.linalg.vector_norm(k32 - k64, dim=1) / torch.linalg.vector_norm(k64, dim=1)
        worst = max(worst, e.max().item())
    print("all pairs: worst row vs FP64 path %.2e" % worst)
    assert worst <= TOL_MIXED, worst
    rng = np.random.default_rng(7)
    idx = np.sort(rng.choice(n, 40, replace=False))
    special = np.where(st & 6)[0]
    idx = np.unique(np.concatenate([idx, special[:: max(1, len(special) // 24)]]))
    kap = o32["kappa"][torch.tensor(idx, device=dev)].cpu().numpy()
    _, k_o = _oracle(cfg, t[idx], j[idx], ts[idx])
    ek = _relerr(kap, k_o)
    print("all pairs: sampled rows vs oracle %.2e" % ek.max())
    assert ek.max() <= TOL_MIXED, ek.max()


def test_mixed_refine_and_singular(ctx):
    """Near the pole of the config-2 surface, with M = 16, the FP32 smooth
    factor is not resolved by 2M = 32 samples: those pairs take the 4M-sample
    pass in FP32 too and still match.  A pair with t == t_s gets a NaN row."""
    cfg = dict(workloads.config(2), M=16)
    t = np.array([0.1723, 3.0527, 0.9, 0.7])
    ts = np.array([0.2204, 3.0341, 0.9 + 1e-5, 0.7])
    j = np.array([31, 0, 3, 5], dtype=np.int32)
    out = _run(ctx, cfg, t, j, ts)
    assert (out["status"][:2] & 4).all() and not (out["status"][:3] & 8).any(), out["status"]
    assert out["status"][3] & 1 and np.isnan(out["kappa"][3]).all()
    c_o, k_o = _oracle(cfg, t[:3], j[:3], ts[:3], processes=1)
    ek, ec = _relerr(out["kappa"][:3], k_o), _relerr(out["rhoinv"][:3], c_o)
    print("refine/near-pole pairs: kappa", ek, "rhoinv", ec)
    assert ek.max() <= TOL_MIXED and ec.max() <= TOL_MIXED, (ek, ec)


def test_mixed_rejects_complex128_output(ctx):
    import paper_2608_16208_amd as ffbie
    cfg = workloads.config(1)
    ctx.set_problem(cfg["amp"], cfg["n_panels"], cfg["M"], cfg["k"])
    dev = ctx.device
    x = torch.zeros(4, dtype=torch.float64, device=dev)
    with pytest.raises(ffbie.FfbieError):
        ctx.kernel_coeffs(x + 0.5, torch.zeros(4, dtype=torch.int32, device=dev), x + 0.6,
                          mixed=True,
                          kappa=torch.empty((4, 2 * cfg["M"]), dtype=torch.complex128, device=dev))
