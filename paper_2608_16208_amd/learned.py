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

Command line (writes the library's network checkpoint):
    python -m paper_2608_16208_amd.learned --out weights.ffbiemlp [--systems 200]
"""
import argparse
import time

import numpy as np

import workloads

from . import (Context, RHS_PLANE_WAVE, RHS_POINT_SOURCE, SOLVE_FGMRES_MLP, SOLVE_GMRES,
               SOLVE_LU64)


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
    ap.add_argument("--out", required=True)
    ap.add_argument("--systems", type=int, default=200)
    ap.add_argument("--rhs", type=int, default=8)
    ap.add_argument("--steps", type=int, default=3000)
    ap.add_argument("--batch", type=int, default=2048)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--M", type=int, default=64)
    args = ap.parse_args()
    log = lambda s: print(s, flush=True)
    ctx = Context(0)
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
