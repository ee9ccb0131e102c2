"""Batched coefficient path: many problems (surfaces of the star family,
different M, k and pair counts) in one persistent launch per phase.

Each problem's rows must equal those of a single-problem call (same device
arithmetic; compared to 1e-14 and reported when bitwise equal), and sampled rows
must match the oracle to the 1e-10 bar of the coefficient path.
"""
import numpy as np
import pytest

import workloads
from oracle import coeffs as ocoeffs

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2608_16208_amd as ffbie
    c = ffbie.Context(0)
    yield c
    c.close()


def _problems():
    out = []
    for cfgi, n, seed in ((1, 300, 11), (2, 700, 12), (3, 500, 13)):
        cfg = workloads.config(cfgi)
        t, j, ts = workloads.sample_pairs(cfg["n_panels"], cfg["M"], n, seed=seed)
        out.append(dict(amp=cfg["amp"], M=cfg["M"], k=cfg["k"], t=t, az=j, ts=ts, n_panels=cfg["n_panels"],
                        oracle=True))
    # a batch member of the large-batch family: M = 16 and M = 128, and an empty problem
    for i, (M, npan) in enumerate(((16, 5), (128, 9))):
        cfg = workloads.batch_surface(i)
        t, j, ts = workloads.sample_pairs(npan, M, 400, seed=20 + i)
        # (at M = 16 and k up to 25 the 2M-point samples of sin(k rho)/rho can alias, so
        # only the equality with single-problem calls is checked for these)
        out.append(dict(amp=cfg["amp"], M=M, k=cfg["k"], t=t, az=j, ts=ts, n_panels=npan, oracle=False))
    out.append(dict(amp=None, M=32, k=1.0, t=np.zeros(0), az=np.zeros(0, np.int32), ts=np.zeros(0), n_panels=1))
    return out


def test_batch_matches_single_calls_and_oracle(ctx):
    probs = _problems()
    dev = ctx.device
    batch = ctx.kernel_coeffs_batched([dict(amp=p["amp"], M=p["M"], k=p["k"], t=torch.tensor(p["t"]),
                                            az=torch.tensor(p["az"]), ts=torch.tensor(p["ts"]))
                                       for p in probs])
    torch.cuda.synchronize()
    bitwise = True
    for p, b in zip(probs, batch):
        if len(p["t"]) == 0:
            assert b["kappa"].shape == (0, 2 * p["M"])
            continue
        ctx.set_problem(p["amp"], p["n_panels"], p["M"], p["k"])
        one = ctx.kernel_coeffs(torch.tensor(p["t"], device=dev), torch.tensor(p["az"], device=dev),
                                torch.tensor(p["ts"], device=dev))
        kb, k1 = b["kappa"].cpu().numpy(), one["kappa"].cpu().numpy()
        sb, s1 = b["status"].cpu().numpy(), one["status"].cpu().numpy()
        assert np.array_equal(sb, s1)
        bitwise &= np.array_equal(kb, k1)
        err = np.max(np.abs(kb - k1)) / np.max(np.abs(k1))
        assert err <= 1e-14, err
        if not p.get("oracle"):
            continue
        idx = np.linspace(0, len(p["t"]) - 1, 12).astype(int)
        _, ko, _ = ocoeffs.pairs_coeffs(p["amp"], p["k"], p["M"], 2 * p["M"], p["t"][idx], p["az"][idx],
                                        p["ts"][idx], processes=8)
        e = np.linalg.norm(kb[idx] - ko, axis=1) / np.linalg.norm(ko, axis=1)
        assert e.max() <= 1e-10, e.max()
    print("batched rows bitwise equal to single calls:", bitwise)


def test_batch_repeated_calls_are_deterministic(ctx):
    probs = _problems()[:3]
    items = [dict(amp=p["amp"], M=p["M"], k=p["k"], t=torch.tensor(p["t"]), az=torch.tensor(p["az"]),
                  ts=torch.tensor(p["ts"])) for p in probs]
    a = [o["kappa"].cpu().numpy() for o in ctx.kernel_coeffs_batched(items)]
    b = [o["kappa"].cpu().numpy() for o in ctx.kernel_coeffs_batched(items)]
    for x, y in zip(a, b):
        assert np.array_equal(x, y)


def _items(probs):
    return [dict(amp=p["amp"], M=p["M"], k=p["k"], t=torch.tensor(p["t"]), az=torch.tensor(p["az"]),
                 ts=torch.tensor(p["ts"])) for p in probs]


def _single(ctx, p, mixed=False):
    dev = ctx.device
    ctx.set_problem(p["amp"], p["n_panels"], p["M"], p["k"])
    one = ctx.kernel_coeffs(torch.tensor(p["t"], device=dev), torch.tensor(p["az"], device=dev),
                            torch.tensor(p["ts"], device=dev), mixed=mixed)
    return one["kappa"].cpu().numpy(), one["status"].cpu().numpy()


def test_plan_graph_replays_match_eager(ctx):
    """A plan captured in a HIP graph, replayed three times with other work of
    the program (a single-problem call, torch kernels, host syncs) between the
    replays: every replay must reproduce the eager batched result bit for bit."""
    probs = _problems()
    eager = [o["kappa"].cpu().numpy() for o in ctx.kernel_coeffs_batched(_items(probs))]
    plan = ctx.batch_plan(_items(probs), graph=True)
    dev = ctx.device
    for rep in range(3):
        for o in plan.outs:
            o["kappa"].zero_()
        torch.cuda.synchronize()
        plan.execute()
        # unrelated eager work between replays
        p = probs[1]
        ctx.set_problem(p["amp"], p["n_panels"], p["M"], p["k"])
        ctx.kernel_coeffs(torch.tensor(p["t"][:50], device=dev), torch.tensor(p["az"][:50], device=dev),
                          torch.tensor(p["ts"][:50], device=dev))
        (torch.ones(1 << 20, device=dev) * rep).sum().item()
        torch.cuda.synchronize()
        for e, o in zip(eager, plan.outs):
            assert np.array_equal(e, o["kappa"].cpu().numpy()), rep
    plan.close()


def test_plan_autotune_picks_a_candidate_and_keeps_results(ctx):
    """The autotuner times radix x pairs-per-item x waves candidates on each M
    class of the plan's own batch; with its choices the rows agree with
    single-problem calls (radix 2) to rounding."""
    probs = _problems()
    plan = ctx.batch_plan(_items(probs), autotune=True)
    tun = plan.tuning()
    assert sorted(t["M"] for t in tun) == [16, 32, 64, 128]
    for t in tun:
        assert t["fft_radix"] in (2, 4) and t["pairs_per_item"] in (8, 16, 32)
        assert t["waves_per_block"] in (1, 2, 4) and t["tuned_ms"] > 0
        assert t["persistent"] in (0, 1)
    plan.execute()
    torch.cuda.synchronize()
    for p, o in zip(probs, plan.outs):
        if len(p["t"]) == 0:
            continue
        k1, s1 = _single(ctx, p)
        kb = o["kappa"].cpu().numpy()
        assert np.array_equal(o["status"].cpu().numpy() & 0xff, s1 & 0xff)
        err = np.max(np.abs(kb - k1)) / np.max(np.abs(k1))
        assert err <= 1e-12, err
    print("autotuned:", tun)
    plan.close()


def test_plan_explicit_tuning_per_M(ctx):
    """A tuning table by M is applied class by class."""
    probs = _problems()
    want = {64: dict(fft_radix=4, pairs_per_item=8, waves_per_block=1, persistent=1),
            128: dict(fft_radix=2, pairs_per_item=32, waves_per_block=2, persistent=0)}
    plan = ctx.batch_plan(_items(probs), tuning=want)
    got = {t["M"]: t for t in plan.tuning()}
    for M, w in want.items():
        for key, v in w.items():
            assert got[M][key] == v, (M, key, got[M])
    base = ctx.get_tuning()
    assert got[16]["fft_radix"] == base["fft_radix"]
    plan.execute()
    torch.cuda.synchronize()
    ref = [o["kappa"].cpu().numpy() for o in ctx.kernel_coeffs_batched(_items(probs))]
    for r, o in zip(ref, plan.outs):
        if r.size:
            assert np.max(np.abs(r - o["kappa"].cpu().numpy())) <= 1e-12 * np.max(np.abs(r))
    plan.close()


@pytest.mark.parametrize("cfgi", [1, 2, 3])
def test_radix4_transforms_match_oracle(ctx, cfgi):
    """Radix-4 Stockham stages (with a final radix-2 stage for odd log2 N_F)
    give the same coefficients as the oracle at the FP64 bar."""
    cfg = workloads.config(cfgi)
    t, j, ts = workloads.sample_pairs(cfg["n_panels"], cfg["M"], 120, seed=300 + cfgi)
    p = dict(amp=cfg["amp"], M=cfg["M"], k=cfg["k"], t=t, az=j, ts=ts, n_panels=cfg["n_panels"])
    saved = ctx.get_tuning()
    try:
        ctx.set_tuning(fft_radix=4)
        k4, s4 = _single(ctx, p)
    finally:
        ctx.set_tuning(**saved)
    assert not (s4 & 8).any()
    _, ko, _ = ocoeffs.pairs_coeffs(cfg["amp"], cfg["k"], cfg["M"], 2 * cfg["M"], t, j, ts, processes=8)
    e = np.linalg.norm(k4 - ko, axis=1) / np.linalg.norm(ko, axis=1)
    print("radix 4, config %d: max rel err %.2e" % (cfgi, e.max()))
    assert e.max() <= 1e-10, e.max()


def test_plan_mixed_matches_single_mixed_calls(ctx):
    """A mixed-precision plan (complex64 outputs, captured in a graph) gives the
    rows of single-problem mixed calls.  The batched and single-problem kernels
    are separate instantiations of the same per-pair routine, and the compiler
    may fuse and order their FP32 operations differently, so rows are compared
    to the mixed-precision bound (1e-5 of the row's largest value) and the pair
    flags exactly."""
    probs = _problems()
    plan = ctx.batch_plan(_items(probs), mixed=True, graph=True)
    plan.execute()
    torch.cuda.synchronize()
    worst = 0.0
    for p, o in zip(probs, plan.outs):
        assert o["kappa"].dtype == torch.complex64
        if len(p["t"]) == 0:
            continue
        k1, s1 = _single(ctx, p, mixed=True)
        kb = o["kappa"].cpu().numpy()
        assert np.array_equal(o["status"].cpu().numpy() & 0xff, s1 & 0xff)
        err = np.max(np.abs(kb - k1), axis=1) / np.max(np.abs(k1), axis=1)
        worst = max(worst, float(err.max()))
    print("mixed plan vs single mixed calls: %.2e" % worst)
    assert worst <= 1e-5, worst
    plan.close()


@pytest.mark.parametrize("mixed", [False, True])
def test_persistent_and_per_item_launches_agree(ctx, mixed):
    """The batched main pass as a persistent launch (wavefronts loop over a
    work queue) and as one wavefront per work item run the same per-pair
    routine: the rows agree to rounding and the pair flags exactly."""
    probs = _problems()
    outs = []
    for pers in (0, 1):
        tun = dict(fft_radix=2, pairs_per_item=16, waves_per_block=4, persistent=pers)
        plan = ctx.batch_plan(_items(probs), mixed=mixed, tuning=tun)
        assert all(t["persistent"] == pers for t in plan.tuning())
        plan.execute()
        torch.cuda.synchronize()
        outs.append([(o["kappa"].cpu().numpy(), o["status"].cpu().numpy()) for o in plan.outs])
        plan.close()
    tol = 1e-5 if mixed else 1e-12
    for (ka, sa), (kb, sb) in zip(*outs):
        assert np.array_equal(sa & 0xff, sb & 0xff)
        if ka.size:
            assert np.max(np.abs(ka - kb)) <= tol * np.max(np.abs(ka))


def test_tuning_validation(ctx):
    import paper_2608_16208_amd as ffbie
    for bad in (dict(fft_radix=3), dict(pairs_per_item=0), dict(waves_per_block=3),
                dict(persistent=2)):
        with pytest.raises(ffbie.FfbieError):
            ctx.set_tuning(**bad)
    assert ctx.get_tuning()["fft_radix"] in (0, 2, 4)


def test_batch_surfaces_full_near_sets_as_benchmarked(ctx):
    """The benchmarked batch configuration: the full near sets of eight of the
    64 batch surfaces (every M class, k up to 25) through an autotuned batch
    plan captured in a graph.  Every row is compared with single-problem calls
    (1e-12 of the row's largest value; different FFT radix or work shape only
    change rounding), and sampled rows whose smooth factor is resolved (no
    FFBIE_PAIR_UNRESOLVED flag: small M with large k is not) with the oracle
    (1e-10)."""
    surfs, items = [], []
    for s in (0, 2, 3, 7, 8, 13, 19, 21):     # members whose M the library supports
        c = workloads.batch_surface(s)
        assert c["M"] in (16, 32, 64, 128)
        ctx.set_problem(c["amp"], c["n_panels"], c["M"], c["k"])
        t, az, ts = ctx.near_pairs()
        surfs.append(dict(c, t=t, az=az, ts=ts))
        items.append(dict(amp=c["amp"], M=c["M"], k=c["k"], t=t, az=az, ts=ts))
    assert len({c["M"] for c in surfs}) >= 3
    plan = ctx.batch_plan(items, autotune=True, graph=True)
    plan.execute()
    torch.cuda.synchronize()
    rng = np.random.default_rng(17)
    worst, n_oracle = 0.0, 0
    for c, o in zip(surfs, plan.outs):
        ctx.set_problem(c["amp"], c["n_panels"], c["M"], c["k"])
        one = ctx.kernel_coeffs(c["t"], c["az"], c["ts"])
        k1, kb = one["kappa"], o["kappa"]
        e = (kb - k1).abs().amax(dim=1) / k1.abs().amax(dim=1)
        worst = max(worst, float(e.max().item()))
        assert torch.equal(o["status"] & 0xff, one["status"] & 0xff)
        resolved = np.where((o["status"].cpu().numpy() & 8) == 0)[0]
        if resolved.size:
            idx = np.sort(rng.choice(resolved, min(6, resolved.size), replace=False))
            t, j, ts = (x.cpu().numpy()[idx] for x in (c["t"], c["az"], c["ts"]))
            _, ko, _ = ocoeffs.pairs_coeffs(c["amp"], c["k"], c["M"], 2 * c["M"], t, j, ts, processes=8)
            eo = np.linalg.norm(kb.cpu().numpy()[idx] - ko, axis=1) / np.linalg.norm(ko, axis=1)
            assert eo.max() <= 1e-10, (c["name"], eo.max())
            n_oracle += 1
        del one
    print("batch surfaces: worst row vs single calls %.2e; %d surfaces also vs the oracle" % (worst, n_oracle))
    assert worst <= 1e-12, worst
    assert n_oracle >= 4
    plan.close()


def test_batch_members_with_unsupported_M_are_rejected(ctx):
    """Members with M in {24, 48, 96} (2M = 2^a 3^b with b > 0) need radix-3
    transforms, which the library does not have: set_problem and batch plans
    reject them with FFBIE_EINVAL (the benchmark reports them as skipped)."""
    import paper_2608_16208_amd as ffbie
    odd = [s for s in range(64) if workloads.batch_surface(s)["M"] not in (16, 32, 64, 128)]
    assert odd
    c = workloads.batch_surface(odd[0])
    with pytest.raises(ffbie.FfbieError, match="M"):
        ctx.set_problem(c["amp"], c["n_panels"], c["M"], c["k"])
    t = torch.zeros(1, dtype=torch.float64)
    with pytest.raises(ffbie.FfbieError):
        ctx.batch_plan([dict(amp=c["amp"], M=c["M"], k=c["k"], t=t + 1.0, az=torch.zeros(1, dtype=torch.int32),
                             ts=t + 1.5)])

