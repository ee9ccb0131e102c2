"""The coefficient entry point that allocates nothing
(ffbie_kernel_coeffs_noalloc) against ffbie_kernel_coeffs: two calls in a
row on the same GPU, the second with fewer pairs, each compared row by row
with the allocating entry point (same kernels: equal to the last bit), with
pairs that take the 4M-sample refine pass so that the scratch's refine list
and counter are used; sizes beyond the scratch are rejected."""
import ctypes

import numpy as np
import pytest

import workloads

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2608_16208_amd as ffbie
    c = ffbie.Context(0)
    yield c
    c.close()


def _compare(ctx, amp, n_panels, M, k, n, seed):
    import paper_2608_16208_amd as ffbie
    ctx.set_problem(amp, n_panels, M, k)
    t, j, ts = workloads.sample_pairs(n_panels, M, n, seed=seed, near_fraction=0.5)
    dev = ctx.device
    T, J, TS = torch.tensor(t, device=dev), torch.tensor(j, device=dev), torch.tensor(ts, device=dev)
    ref = ctx.kernel_coeffs(T, J, TS, root=True)
    out = ctx.kernel_coeffs(T, J, TS, root=True, noalloc=True)
    torch.cuda.synchronize()
    st = out["status"].cpu().numpy()
    assert torch.equal(out["status"], ref["status"])
    assert torch.equal(out["root"], ref["root"])
    a, b = out["kappa"], ref["kappa"]
    same_nan = torch.isnan(a) == torch.isnan(b)
    assert bool(same_nan.all())
    assert torch.equal(torch.nan_to_num(a), torch.nan_to_num(b))
    return int(((st & ffbie.PAIR_REFINED) > 0).sum())


def test_noalloc_matches_allocating_entry_point_twice(ctx):
    cfg2, cfg3 = workloads.config(2), workloads.config(3)
    # first call: config-2 shape at M = 16 (many pairs need the 4M-sample pass)
    refined1 = _compare(ctx, cfg2["amp"], 8, 16, cfg2["k"], 20000, seed=31)
    # second call, fewer pairs: config 3 (M = 128)
    refined2 = _compare(ctx, cfg3["amp"], cfg3["n_panels"], cfg3["M"], cfg3["k"], 3000, seed=32)
    print("no-alloc entry point: %d and %d pairs took the refine pass" % (refined1, refined2))
    assert refined1 > 0


def test_noalloc_rejects_sizes_beyond_scratch(ctx):
    import paper_2608_16208_amd as ffbie
    cfg = workloads.config(2)
    ctx.set_problem(cfg["amp"], cfg["n_panels"], cfg["M"], cfg["k"])
    x = torch.zeros(4, dtype=torch.float64, device=ctx.device)
    j = torch.zeros(4, dtype=torch.int32, device=ctx.device)
    kap = torch.zeros((4, 2 * cfg["M"]), dtype=torch.complex128, device=ctx.device)
    p = lambda v: ctypes.c_void_p(v.data_ptr())
    rc = ctx.lib.ffbie_kernel_coeffs_noalloc(ctx.h, (1 << 20) + 1, p(x), p(j), p(x), p(kap), None, None, None)
    assert rc == -1 and b"capacity" in ctx.lib.ffbie_last_error(ctx.h)
    assert ctx.lib.ffbie_kernel_coeffs_noalloc(ctx.h, 0, None, None, None, None, None, None, None) == 0
