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

Command line (writes the weights with numpy, no pickle):
    python -m paper_2608_16208_amd.learned --out weights.npz [--systems 200]
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
    """Adam on minibatches drawn without replacement per epoch; returns the losses."""
    import torch
    g = torch.Generator(device="cpu").manual_seed(seed)
    n = X.shape[0]
    losses, perm, pos = [], torch.randperm(n, generator=g), 0
    for step in range(steps):
        if pos + batch > n:
            perm, pos = torch.randperm(n, generator=g), 0
        idx = perm[pos:pos + batch].to(X.device)
        pos += batch
        xb, tb = X[idx].contiguous(), T[idx].contiguous()
        lr_s = lr * 0.5 * (1 + np.cos(np.pi * step / steps))        # cosine decay
        loss, _ = ctx.mlp_train_step(xb, tb, lr=lr_s)
        losses.append(loss)
        if log and (step % 200 == 0 or step == steps - 1):
            log(f"step {step}: loss {loss:.4e}")
    return losses


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


def save(path, params):
    np.savez(path, params=np.asarray(params, dtype=np.float32))


def load(path):
    with np.load(path, allow_pickle=False) as f:
        return f["params"]


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
    losses = train(ctx, X, T, steps=args.steps, batch=args.batch, lr=args.lr, log=log)
    log(f"trained in {time.time() - t0:.1f} s; loss {losses[0]:.3e} -> {losses[-1]:.3e}")
    save(args.out, ctx.mlp_get_params())


if __name__ == "__main__":
    main()
