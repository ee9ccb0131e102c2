"""GPU double-layer systems (Sec. 2, Sec. 4): the assembled K and K' against
the oracle, the second-kind equations for the exterior Dirichlet and Neumann
problems, and first- against second-kind solves.

* sampled rows of K and K' (configs 1 and 2) entry by entry against the
  oracle's rows (direct-quadrature coefficients through the same near rule):
  1e-10 of the row's largest entry, the single-layer rows' bar;
* the identity shift lands on the diagonal as shift / J;
* the sound-hard right-hand side and the double-layer field against the
  oracle (1e-13 and 1e-12: plain sums);
* sound-soft sphere (config 1) by (K + I) psi = g and the double-layer field,
  sound-hard sphere by (K' - I) phi = -du_inc/dnu and the single-layer field,
  each against its Mie series;
* config-2 star: the first-kind S and the second-kind K + I solutions give
  the exact field of an interior point source and the same scattered field
  of a plane wave, and GMRES needs fewer iterations on K + I.
"""
import numpy as np
import pytest

import workloads
from oracle import assembly as oasm
from oracle import solve as osolve

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _rule():
    from test_oracle_system import load_golden
    return load_golden()


@pytest.fixture(scope="module")
def ctx():
    import paper_2608_16208_amd as ffbie
    c = ffbie.Context(0)
    yield c
    c.close()


def _far_points(n, seed):
    rng = np.random.default_rng(seed)
    d = rng.standard_normal((n, 3))
    return d / np.linalg.norm(d, axis=1)[:, None] * rng.uniform(3, 5, n)[:, None]


@pytest.mark.parametrize("op", [1, 2])
@pytest.mark.parametrize("cfgi", [1, 2])
def test_dl_rows_match_oracle(ctx, cfgi, op):
    cfg = workloads.config(cfgi)
    ctx.set_near_rule(_rule())
    ctx.set_problem(cfg["amp"], cfg["n_panels"], cfg["M"], cfg["k"])
    N, _ = ctx.query()
    A = ctx.assemble(op=op)
    rep = ctx.last_assembly
    assert rep["status"] == 0 and rep["unresolved"] == 0, rep
    print("config %d op %d: %d of %d near pairs unresolved" % (cfgi, op, rep["unresolved"], rep["pairs"]))
    rng = np.random.default_rng(40 + cfgi + op)
    per_panel = 32 * cfg["M"]
    rows = sorted({int(rng.integers(0, per_panel)), int(N - 1 - rng.integers(0, per_panel)),
                   *[int(v) for v in rng.choice(N, 2, replace=False)]})
    got = A[torch.tensor(rows, device=ctx.device)].cpu().numpy()
    del A
    torch.cuda.empty_cache()
    ref = oasm.rows(cfg["amp"], cfg["k"], cfg["M"], cfg["n_panels"], rows, _rule(), processes=8,
                    kind="K" if op == 1 else "Kp")
    for a, r in enumerate(rows):
        err = np.max(np.abs(got[a] - ref[a])) / np.max(np.abs(ref[a]))
        print("config %d op %d row %d: %.2e" % (cfgi, op, r, err))
        assert np.isfinite(got[a]).all() and err <= 1e-10, (r, err)


def test_identity_shift_and_density_unknowns(ctx):
    """Scaled unknowns: shift * I lands on the diagonal as shift / J.  Density
    unknowns: every column carries J_c and shift * I is added as it is."""
    import paper_2608_16208_amd as ffbie
    cfg = workloads.config(2)
    ctx.set_near_rule(None)
    ctx.set_problem(cfg["amp"], 4, 16, cfg["k"])
    K0 = ctx.assemble(op=1)
    K1 = ctx.assemble(op=1, shift=1.0)
    _, jac, _ = ctx.collocation()
    D = (K1 - K0).cpu().numpy()
    J = jac.cpu().numpy()
    assert np.max(np.abs(np.diag(D) - 1.0 / J)) <= 1e-15 * np.max(1.0 / J)
    np.fill_diagonal(D, 0.0)
    assert not D.any()
    Kd = ctx.assemble(op=1, shift=-1.0, unknowns=ffbie.UNKNOWN_DENSITY).cpu().numpy()
    ref = K0.cpu().numpy() * J[None, :] - np.eye(J.size)
    assert np.max(np.abs(Kd - ref)) <= 1e-15 * np.max(np.abs(ref))


def test_sound_hard_rhs_and_dl_field_match_oracle(ctx):
    import paper_2608_16208_amd as ffbie
    cfg = workloads.config(2)
    ctx.set_problem(cfg["amp"], cfg["n_panels"], cfg["M"], cfg["k"])
    N, _ = ctx.query()
    g = ctx.rhs(ffbie.RHS_PLANE_WAVE_DN, cfg["d"]).cpu().numpy()
    ref = oasm.rhs_plane_wave_dn(cfg["amp"], cfg["n_panels"], cfg["M"], cfg["k"], cfg["d"])
    assert np.max(np.abs(g - ref)) / np.max(np.abs(ref)) <= 1e-12     # normals: 1e-13 level
    p_out = [3.0, 4.0, 10.5]
    g = ctx.rhs(ffbie.RHS_POINT_SOURCE_DN, p_out).cpu().numpy()
    ref = oasm.rhs_point_source_dn(cfg["amp"], cfg["n_panels"], cfg["M"], cfg["k"], p_out)
    assert np.max(np.abs(g - ref)) / np.max(np.abs(ref)) <= 1e-12
    rng = np.random.default_rng(8)
    psi = rng.standard_normal(N) + 1j * rng.standard_normal(N)
    pts = _far_points(32, 9)
    u = ctx.eval_field(torch.tensor(pts), torch.tensor(psi), op=ffbie.OP_K).cpu().numpy()
    uref = oasm.field_double_layer(cfg["amp"], cfg["n_panels"], cfg["M"], cfg["k"], psi, pts)
    assert np.max(np.abs(u - uref)) / np.max(np.abs(uref)) <= 1e-12


def test_sphere_second_kind_dirichlet_and_neumann_match_mie(ctx):
    """Config 1 (k = 1, 8 panels, M = 32): the exterior Dirichlet problem by
    (K + I) psi = -u_inc and the double-layer field, the exterior Neumann
    problem by (K' - I) phi = -du_inc/dnu and the single-layer field."""
    import paper_2608_16208_amd as ffbie
    cfg = workloads.config(1)
    ctx.set_near_rule(None)
    ctx.set_problem(cfg["amp"], cfg["n_panels"], cfg["M"], cfg["k"])
    pts = torch.tensor(_far_points(64, 1))
    A = ctx.assemble(op=ffbie.OP_K, shift=1.0)
    g = ctx.rhs(ffbie.RHS_PLANE_WAVE, cfg["d"])
    psi, _ = ctx.solve(A, g, method=ffbie.SOLVE_LU64)
    u = ctx.eval_field(pts, psi, op=ffbie.OP_K).cpu().numpy()
    ref = osolve.mie_scattered(cfg["k"], pts.numpy(), cfg["d"])
    e_soft = np.linalg.norm(u - ref) / np.linalg.norm(ref)
    del A
    A = ctx.assemble(op=ffbie.OP_KP, shift=-1.0)
    g = ctx.rhs(ffbie.RHS_PLANE_WAVE_DN, cfg["d"])
    phi, _ = ctx.solve(A, g, method=ffbie.SOLVE_LU64)
    u = ctx.eval_field(pts, phi).cpu().numpy()
    ref = osolve.mie_scattered_hard(cfg["k"], pts.numpy(), cfg["d"])
    e_hard = np.linalg.norm(u - ref) / np.linalg.norm(ref)
    del A
    torch.cuda.empty_cache()
    print("sphere: sound-soft by K + I %.2e, sound-hard by K' - I %.2e" % (e_soft, e_hard))
    assert e_soft <= 1e-8 and e_hard <= 1e-8, (e_soft, e_hard)


def test_star_first_and_second_kind_agree(ctx):
    """Config 2 (N = 32768), exterior Dirichlet problem two ways: the first-kind
    S phi = g and the second-kind (K + I) psi = g with density unknowns.
    * exact check: data g = G(.; p) of a source p inside the surface, whose
      exterior solution is G(.; p) itself: both fields (LU64) against it;
    * plane wave: the two fields agree, and restarted GMRES reaches a 1e-10
      residual in fewer iterations on K + I.
    (With unknowns scaled by J the identity becomes diag(1/J), up to ~1e3
    next to the poles, and GMRES stalls: reported, not asserted.)"""
    import paper_2608_16208_amd as ffbie
    cfg = workloads.config(2)
    ctx.set_near_rule(None)
    ctx.set_problem(cfg["amp"], cfg["n_panels"], cfg["M"], cfg["k"])
    P = _far_points(64, 2)
    pts = torch.tensor(P)
    p_in = np.array([0.1, -0.2, 0.15])
    exact = osolve.point_source(cfg["k"], P, p_in)
    g = ctx.rhs(ffbie.RHS_PLANE_WAVE, cfg["d"])
    g_ps = ctx.rhs(ffbie.RHS_POINT_SOURCE, list(p_in))
    out = {}
    for name, op, shift, unk, its in (("S", ffbie.OP_S, 0.0, ffbie.UNKNOWN_SCALED, 3000),
                                      ("K+I", ffbie.OP_K, 1.0, ffbie.UNKNOWN_DENSITY, 3000),
                                      ("K+I scaled", ffbie.OP_K, 1.0, ffbie.UNKNOWN_SCALED, 300)):
        A = ctx.assemble(op=op, shift=shift, unknowns=unk)
        x_it, info = ctx.solve(A, g, method=ffbie.SOLVE_GMRES, tol=1e-10, max_iter=its)
        ctx.lu_factor(A)
        x = ctx.lu_solve(A, g)
        x_ps = ctx.lu_solve(A, g_ps)
        del A
        torch.cuda.empty_cache()
        fop = ffbie.OP_S if op == ffbie.OP_S else ffbie.OP_K
        u = ctx.eval_field(pts, x, op=fop, unknowns=unk).cpu().numpy()
        u_it = ctx.eval_field(pts, x_it, op=fop, unknowns=unk).cpu().numpy()
        u_ps = ctx.eval_field(pts, x_ps, op=fop, unknowns=unk).cpu().numpy()
        out[name] = dict(u=u, info=info, e_it=np.linalg.norm(u_it - u) / np.linalg.norm(u),
                         e_ps=np.linalg.norm(u_ps - exact) / np.linalg.norm(exact))
    s_, k_, ks = out["S"], out["K+I"], out["K+I scaled"]
    diff = np.linalg.norm(s_["u"] - k_["u"]) / np.linalg.norm(s_["u"])
    diff2 = np.linalg.norm(ks["u"] - k_["u"]) / np.linalg.norm(k_["u"])
    print("config 2: point source inside, field error S %.2e, K + I %.2e; plane wave: fields of S and "
          "K + I differ by %.2e (K + I scaled vs density %.2e); GMRES iterations to 1e-10: S %d (%s, "
          "field %.1e from LU), K + I %d (%s, field %.1e from LU), K + I with scaled unknowns %d (%s, "
          "residual %.1e)"
          % (s_["e_ps"], k_["e_ps"], diff, diff2, s_["info"]["iterations"], s_["info"]["converged"],
             s_["e_it"], k_["info"]["iterations"], k_["info"]["converged"], k_["e_it"],
             ks["info"]["iterations"], ks["info"]["converged"], ks["info"]["rel_residual"]))
    assert s_["e_ps"] <= 1e-7 and k_["e_ps"] <= 1e-7, (s_["e_ps"], k_["e_ps"])
    assert diff <= 1e-7 and diff2 <= 1e-10, (diff, diff2)
    assert k_["info"]["converged"] and k_["e_it"] <= 1e-8, k_
    assert k_["info"]["iterations"] < s_["info"]["iterations"], (s_["info"], k_["info"])
