"""Training and evaluation of the learned per-mode preconditioner.

Everything runs through the C ABI: the systems are assembled by the library
(`assemble`), the training pairs are the mode features of Krylov-type vectors r
and of their mode-block-Jacobi corrections e (`blockjacobi_setup/apply`,
`mode_features`, `mode_targets`), and the network is trained by the library's
BF16 matrix-core kernels (`mlp_train_step`, Adam).  A trained network replaces
the per-surface block extraction and factorisation by one network evaluation.  The trained
network serves as the right preconditioner and initial guess of flexible
GMRES (`solve(..., SOLVE_FGMRES_MLP)`), which falls back to plain GMRES when it
does not reach the tolerance.

Command lines:
    python -m paper_2608_16208_amd.learned train --out weights.ffbiemlp [--systems 200]
    python -m paper_2608_16208_amd.learned study [--train 200 --test 50] [--save/--load ckpt]
                                                 [--system first|second]
"""
import argparse
import time

import numpy as np

import workloads

from . import (Context, OP_K, OP_S, RHS_PLANE_WAVE, RHS_POINT_SOURCE, SOLVE_FGMRES_MLP, SOLVE_GMRES,
               SOLVE_LU64, UNKNOWN_DENSITY, UNKNOWN_SCALED)

# The exterior Dirichlet problem as a system: the first-kind single-layer
# equation S phi = g (eq. (2.7)) on density x Jacobian, or the second-kind
# double-layer equation (K + I) psi = g (eq. (2.12)) on density values.
SYSTEMS = {"first": dict(op=OP_S, shift=0.0, unknowns=UNKNOWN_SCALED),
           "second": dict(op=OP_K, shift=1.0, unknowns=UNKNOWN_DENSITY)}


def _assemble(ctx, system):
    return ctx.assemble(**SYSTEMS[system])


def _field(ctx, pts, x, system):
    sy = SYSTEMS[system]
    return ctx.eval_field(pts, x, op=sy["op"], unknowns=sy["unknowns"])


def _inputs(ctx, S, rng, n_rhs):
    """Vectors the preconditioner is trained on: for a plane wave g from a random
    direction and an exterior point source, the normalised Krylov directions
    g, S g, S^2 g, ... that GMRES feeds to its preconditioner.  (White-noise
    vectors are not used: they load the near-null directions of the
    first-kind system, high azimuthal modes next to the poles.)"""
    import torch
    out = []
    seeds = []
    d = rng.standard_normal(3)
    seeds.append(ctx.rhs(RHS_PLANE_WAVE, d / np.linalg.norm(d)))
    p = rng.standard_normal(3)
    seeds.append(ctx.rhs(RHS_POINT_SOURCE, rng.uniform(2.0, 4.0) * p / np.linalg.norm(p)))
    per = max(1, n_rhs // len(seeds))
    for v in seeds:
        v = v / v.abs().norm()
        for _ in range(per):
            out.append(v)
            w = -ctx.residual(S, v, torch.zeros_like(v))        # S v
            v = w / w.abs().norm()
    return out[:n_rhs]


def make_dataset(ctx, surfaces, M=64, n_rhs=8, seed=0, min_scale=1e-6, log=None):
    """(X [n, 514], T [n, 512]) float32 device tensors.  Targets are the
    mode-block-Jacobi corrections B_m^{-1} R_m of each input (the inverse of
    the diagonal azimuthal-mode blocks of the system), scaled like the
    features; modes whose size s_m is below min_scale times the largest are
    dropped (they carry no information)."""
    import torch
    rng = np.random.default_rng(seed)
    X, T = [], []
    for i, sf in enumerate(surfaces):
        ctx.set_problem(sf["amp"], 16, M, sf["k"])
        S = ctx.assemble()
        ctx.blockjacobi_setup(S)
        for r in _inputs(ctx, S, rng, n_rhs):
            e = ctx.blockjacobi_apply(r)
            x, sc = ctx.mode_features(r)
            t = ctx.mode_targets(e, sc)
            keep = sc >= min_scale * sc.max()
            X.append(x[keep])
            T.append(t[keep])
        del S
        torch.cuda.empty_cache()
        if log:
            log(f"system {i + 1}/{len(surfaces)} (k = {sf['k']:.2f})")
    return torch.cat(X), torch.cat(T)


def make_dataset_correction(ctx, surfaces, M=64, n_rhs=4, seed=0, min_scale=1e-6, log=None,
                            system="first"):
    """Training pairs for the preconditioner P(v) = BJ(v) + NN(v): inputs are
    the mode features of Krylov-type vectors v of each system, targets the
    modes of the part of S^{-1} v that mode-block-Jacobi misses,
    S^{-1} v - BJ(v), scaled like the features.  S^{-1} v comes from an LU64
    factorisation of each system (a copy of S).  `system` selects the first-
    or second-kind equation (SYSTEMS).  Returns (X, T) float32 device
    tensors."""
    import torch
    rng = np.random.default_rng(seed)
    X, T = [], []
    for i, sf in enumerate(surfaces):
        ctx.set_problem(sf["amp"], 16, M, sf["k"])
        S = _assemble(ctx, system)
        ctx.blockjacobi_setup(S)
        vs = _inputs(ctx, S, rng, n_rhs)
        W = S.clone()
        del S
        torch.cuda.empty_cache()
        ctx.lu_factor(W)
        for v in vs:
            d = ctx.lu_solve(W, v) - ctx.blockjacobi_apply(v)
            x, sc = ctx.mode_features(v)
            t = ctx.mode_targets(d, sc)
            keep = sc >= min_scale * sc.max()
            X.append(x[keep])
            T.append(t[keep])
        del W
        torch.cuda.empty_cache()
        if log and (i % 10 == 0 or i == len(surfaces) - 1):
            log(f"system {i + 1}/{len(surfaces)} (k = {sf['k']:.2f})")
    return torch.cat(X), torch.cat(T)


def study(ctx, n_train=200, n_test=50, M=64, n_rhs=4, steps=3000, batch=2048, lr=1e-3, tol=1e-9,
          max_iter=400, load=None, save_path=None, log=None, system="first"):
    """The learned-preconditioner study at its stated scale: a network trained
    on n_train method-generated systems (star surfaces with 20 amplitudes
    U(-0.1, 0.1), k ~ U[5, 30], 16 panels, M) to correct the mode-block-Jacobi
    output, then used as P = BJ + NN by flexible GMRES (and its initial guess)
    on n_test held-out surfaces, next to plain GMRES, block-Jacobi GMRES and
    LU64.  For each held-out system (plane wave from a fixed direction): the
    LU64 field at 64 far points is the reference; each iterative solve runs to
    the residual tolerance `tol` (at most max_iter iterations) and reports its
    iterations, time and field error, and whether it is within 1e-8 of the
    reference (time-to-1e-8 = assembly + solve + field when it is).  With
    `load` the network is read from a checkpoint instead of trained.
    `system`: "first" (S phi = g) or "second" ((K + I) psi = g), SYSTEMS."""
    import torch
    from . import SOLVE_GMRES_BLOCKJACOBI, SOLVE_FGMRES_BJ_MLP
    out = {"n_train": n_train, "n_test": n_test, "M": M, "tol": tol, "max_iter": max_iter,
           "system": system}
    if load:
        ctx.mlp_load(load)
        out["network"] = "loaded from checkpoint"
    else:
        ctx.mlp_init(1234)
        t0 = time.perf_counter()
        X, T = make_dataset_correction(ctx, [workloads.learned_surface(i) for i in range(n_train)], M=M,
                                       n_rhs=n_rhs, log=log, system=system)
        out["dataset"] = {"samples": int(X.shape[0]), "s": time.perf_counter() - t0}
        t0 = time.perf_counter()
        out["training"] = dict(train(ctx, X, T, steps=steps, batch=batch, lr=lr, log=log),
                               s=time.perf_counter() - t0)
        del X, T
        torch.cuda.empty_cache()
        if save_path:
            ctx.mlp_save(save_path)
    rng = np.random.default_rng(1)
    dpts = rng.standard_normal((64, 3))
    pts = torch.tensor(dpts / np.linalg.norm(dpts, axis=1)[:, None] * rng.uniform(3, 5, 64)[:, None])
    rows = []
    for j in range(n_test):
        sf = workloads.learned_surface(j, held_out=True)
        ctx.set_problem(sf["amp"], 16, M, sf["k"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        S = _assemble(ctx, system)
        torch.cuda.synchronize()
        t_asm = time.perf_counter() - t0
        d = np.array([0.3, -0.5, 0.81])
        g = ctx.rhs(RHS_PLANE_WAVE, d / np.linalg.norm(d))
        W = S.clone()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        phi_ref, _ = ctx.solve(W, g, method=SOLVE_LU64)
        u_ref = _field(ctx, pts, phi_ref, system)
        torch.cuda.synchronize()
        t_lu = time.perf_counter() - t0
        del W
        torch.cuda.empty_cache()
        row = {"k": sf["k"], "assembly_s": t_asm, "lu64": {"s": t_asm + t_lu},
               "unresolved_near_pairs": ctx.last_assembly["unresolved"]}
        for name, method in (("gmres", SOLVE_GMRES), ("gmres_blockjacobi", SOLVE_GMRES_BLOCKJACOBI),
                             ("fgmres_bj_nn", SOLVE_FGMRES_BJ_MLP)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            phi, info = ctx.solve(S, g, method=method, tol=tol, max_iter=max_iter)
            u = _field(ctx, pts, phi, system)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            e = float(((u - u_ref).abs().norm() / u_ref.abs().norm()).item())
            row[name] = {"iterations": info["iterations"], "converged": info["converged"],
                         "fell_back": info["fell_back"], "rel_residual": info["rel_residual"],
                         "field_error": e, "s": t_asm + dt, "reaches_1e-8": e <= 1e-8}
        rows.append(row)
        del S
        torch.cuda.empty_cache()
        if log:
            log("held-out %d (k = %.1f): GMRES %d, BJ %d, BJ+NN %d iterations%s; LU64 %.2f s"
                % (j, sf["k"], row["gmres"]["iterations"], row["gmres_blockjacobi"]["iterations"],
                   row["fgmres_bj_nn"]["iterations"], " (fell back)" if row["fgmres_bj_nn"]["fell_back"] else "",
                   row["lu64"]["s"]))
    out["held_out"] = rows

    def agg(name):
        it = [r[name]["iterations"] for r in rows]
        ok = [r[name]["reaches_1e-8"] for r in rows]
        t = [r[name]["s"] for r in rows if r[name]["reaches_1e-8"]]
        return {"median_iterations": float(np.median(it)), "mean_iterations": float(np.mean(it)),
                "reach_1e-8": int(sum(ok)), "of": len(rows),
                "median_time_to_1e-8_s": float(np.median(t)) if t else None,
                "fell_back": int(sum(r[name]["fell_back"] for r in rows))}
    out["summary"] = {n: agg(n) for n in ("gmres", "gmres_blockjacobi", "fgmres_bj_nn")}
    out["summary"]["lu64"] = {"median_time_to_1e-8_s": float(np.median([r["lu64"]["s"] for r in rows]))}
    both = [r for r in rows if r["gmres_blockjacobi"]["converged"] and r["fgmres_bj_nn"]["converged"]
            and not r["fgmres_bj_nn"]["fell_back"]]
    out["summary"]["bj_nn_fewer_iterations_than_bj"] = sum(
        r["fgmres_bj_nn"]["iterations"] < r["gmres_blockjacobi"]["iterations"] for r in both)
    out["summary"]["compared"] = len(both)
    return out


def train(ctx, X, T, steps=2000, batch=2048, lr=1e-3, seed=0, log=None):
    """Adam with cosine decay on minibatches drawn without replacement per
    epoch, by the library's own training loop (ffbie_mlp_train).  Returns the
    loss record {loss_first, loss_last, loss_full, steps}."""
    info = ctx.mlp_train(X, T, steps=steps, batch=min(batch, X.shape[0]), lr=lr, seed=seed)
    if log:
        log(f"{steps} steps: minibatch loss {info['loss_first']:.4e} -> {info['loss_last']:.4e}, "
            f"training set {info['loss_full']:.4e}")
    return info


def evaluate(ctx, surfaces, M=64, tol=1e-8, max_iter=600):
    """Per surface (plane-wave right-hand side): iterations and solve times of
    plain GMRES, GMRES with the mode-block-Jacobi preconditioner, and flexible
    GMRES with the network."""
    import torch
    from . import SOLVE_GMRES_BLOCKJACOBI
    rows = []
    for sf in surfaces:
        ctx.set_problem(sf["amp"], 16, M, sf["k"])
        S = ctx.assemble()
        d = np.array([0.3, -0.5, 0.81])
        g = ctx.rhs(RHS_PLANE_WAVE, d / np.linalg.norm(d))
        row = {"k": sf["k"]}
        for name, method in (("gmres", SOLVE_GMRES), ("gmres_blockjacobi", SOLVE_GMRES_BLOCKJACOBI),
                             ("fgmres_mlp", SOLVE_FGMRES_MLP)):
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            phi, info = ctx.solve(S, g, method=method, tol=tol, max_iter=max_iter)
            torch.cuda.synchronize()
            row[name] = {"iterations": info["iterations"], "s": time.perf_counter() - t0,
                         "rel_residual": info["rel_residual"], "fell_back": info["fell_back"]}
        rows.append(row)
        del S
        torch.cuda.empty_cache()
    return rows


def save(ctx, path):
    """The network and its Adam state (ffbie_mlp_save)."""
    ctx.mlp_save(path)


def load(ctx, path):
    ctx.mlp_load(path)


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd")
    a1 = sub.add_parser("train", help="train the per-mode network on block-Jacobi corrections")
    a1.add_argument("--out", required=True)
    a1.add_argument("--systems", type=int, default=200)
    a1.add_argument("--rhs", type=int, default=8)
    a1.add_argument("--steps", type=int, default=3000)
    a1.add_argument("--batch", type=int, default=2048)
    a1.add_argument("--lr", type=float, default=1e-3)
    a1.add_argument("--M", type=int, default=64)
    a2 = sub.add_parser("study", help="train P = BJ + NN and evaluate it on held-out surfaces")
    a2.add_argument("--train", type=int, default=200)
    a2.add_argument("--test", type=int, default=50)
    a2.add_argument("--rhs", type=int, default=4)
    a2.add_argument("--steps", type=int, default=3000)
    a2.add_argument("--batch", type=int, default=2048)
    a2.add_argument("--lr", type=float, default=1e-3)
    a2.add_argument("--M", type=int, default=64)
    a2.add_argument("--save", default=None, help="write the trained network here")
    a2.add_argument("--load", default=None, help="evaluate a saved network instead of training")
    a2.add_argument("--json", default=None, help="write the study's record here")
    a2.add_argument("--system", default="first", choices=sorted(SYSTEMS),
                    help="first-kind S phi = g or second-kind (K + I) psi = g")
    args = ap.parse_args()
    log = lambda s: print(s, flush=True)
    ctx = Context(0)
    if args.cmd == "study":
        import json
        res = study(ctx, n_train=args.train, n_test=args.test, M=args.M, n_rhs=args.rhs, steps=args.steps,
                    batch=args.batch, lr=args.lr, load=args.load, save_path=args.save, log=log,
                    system=args.system)
        log(json.dumps(res["summary"]))
        if args.json:
            with open(args.json, "w") as fh:
                json.dump(res, fh)
        return
    ctx.mlp_init(1234)
    surfs = [workloads.learned_surface(i) for i in range(args.systems)]
    t0 = time.time()
    X, T = make_dataset(ctx, surfs, M=args.M, n_rhs=args.rhs, log=log)
    log(f"dataset {X.shape[0]} samples in {time.time() - t0:.1f} s")
    t0 = time.time()
    rec = train(ctx, X, T, steps=args.steps, batch=args.batch, lr=args.lr, log=log)
    log(f"trained in {time.time() - t0:.1f} s; loss {rec['loss_first']:.3e} -> {rec['loss_full']:.3e}")
    save(ctx, args.out)


if __name__ == "__main__":
    main()
