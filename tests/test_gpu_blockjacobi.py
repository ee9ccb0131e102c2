"""Mode-block-Jacobi preconditioner: GPU against the oracle's definition on a
random matrix, exactness on a surface of revolution (where S is block diagonal
in the azimuthal modes), and the preconditioned GMRES against plain GMRES."""
import numpy as np
import pytest

import workloads
from oracle import solve as osolve

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_2608_16208_amd as ffbie
    c = ffbie.Context(0)
    yield c
    c.close()


def test_blockjacobi_apply_matches_oracle_on_random_matrix(ctx):
    ctx.set_problem(None, 1, 16, 1.0)            # 16 nodes x 32 azimuths: N = 512
    N, _ = ctx.query()
    rng = np.random.default_rng(0)
    A = rng.standard_normal((N, N)) + 1j * rng.standard_normal((N, N)) + 4 * np.sqrt(N) * np.eye(N)
    v = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    ctx.blockjacobi_setup(torch.tensor(A, device=ctx.device))
    z = ctx.blockjacobi_apply(torch.tensor(v, device=ctx.device)).cpu().numpy()
    ref = osolve.blockjacobi_apply(A, v, 16, 16)
    assert np.linalg.norm(z - ref) / np.linalg.norm(ref) <= 1e-12


def test_blockjacobi_is_exact_on_the_sphere(ctx):
    """On a surface of revolution the modes decouple: P = S^{-1}, so the
    preconditioned solve converges at once and matches LU64."""
    import paper_2608_16208_amd as ffbie
    cfg = workloads.config(1)
    ctx.set_problem(cfg["amp"], cfg["n_panels"], cfg["M"], cfg["k"])
    S = ctx.assemble()
    g = ctx.rhs(ffbie.RHS_PLANE_WAVE, cfg["d"])
    phi, info = ctx.solve(S, g, method=ffbie.SOLVE_GMRES_BLOCKJACOBI, tol=1e-12, max_iter=50)
    assert info["converged"] and info["iterations"] <= 2, info
    W = S.clone()
    ref, _ = ctx.solve(W, g, method=ffbie.SOLVE_LU64)
    assert (phi - ref).abs().norm().item() / ref.abs().norm().item() <= 1e-10


def test_blockjacobi_cuts_gmres_iterations_on_a_star(ctx):
    import paper_2608_16208_amd as ffbie
    cfg = workloads.config(2)
    ctx.set_problem(cfg["amp"], cfg["n_panels"], cfg["M"], cfg["k"])
    S = ctx.assemble()
    g = ctx.rhs(ffbie.RHS_PLANE_WAVE, cfg["d"])
    _, plain = ctx.solve(S, g, method=ffbie.SOLVE_GMRES, tol=1e-8, max_iter=500)
    _, bj = ctx.solve(S, g, method=ffbie.SOLVE_GMRES_BLOCKJACOBI, tol=1e-8, max_iter=500)
    print("config 2 GMRES iterations: plain", plain["iterations"], "block-Jacobi", bj["iterations"])
    assert bj["converged"] and bj["iterations"] < plain["iterations"] / 2
