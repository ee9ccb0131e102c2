#!/usr/bin/env python3
"""Benchmark of the azimuthal kernel-coefficient path on one MI355X.

One step = one ffbie_kernel_coeffs call over the whole workload: the root
kernel, the main coefficient pass and the 4M-sample refine pass (geometry,
pair sampling, root, smooth factor, singular factor A_m(b), convolutions and
the coefficient-table write).  Workload: the star surface
R = 1 + 0.2 sin(3t) cos(2 theta), k = 5, 16 panels x 16 Gauss-Legendre nodes
(256 curve nodes), M = 64 (128 azimuths), every (target node, target
azimuth, source node) pair with t_s != t: 8,355,840 pairs, 2M = 128
coefficients each.  Inputs are resident in HBM before the timed region.

Prints one JSON line (rank 0) with the roofline of the main coefficient pass.
"""
import argparse
import hashlib
import json
import math
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "kernel coeff pair-modes/s + time-to-1e-8 field error, mixed vs plain FP64 GPU"
PEAK_FP64_VALU = 78.6e12     # 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz
# FP32 VALU issue rate without packed (two-per-lane) instructions, which the
# library's kernels are compiled without: the same 256 x 4 x 16 x 2 x 2.4 GHz
PEAK_FP32_VALU_UNPACKED = 78.6e12
COEFF_KERNEL = "ffbie_coeff_kernel"
TRAFFIC_SUMMARY = os.path.join(ROOT, "profiles", "coeff_kernel_config2_allpairs_hbm_traffic.md")


def algorithmic_flops_per_pair(NF, M, M0, p, m0, newton_iters=6.0, miller_extra=100.0):
    """Flops one pair needs by the method of Sec. 3.3 with eq. (3.10): sampling,
    three real FFTs, Newton, Miller, both convolutions at the cheaper of direct
    and zero-padded-FFT cost (FMA = 2 flops, complex multiply = 6, a complex
    FFT of size N = 5 N log2 N, real = half)."""
    L = M + M0
    lg = math.log2(NF)
    w = 8 * NF + 12 * NF + 3 * 2.5 * NF * lg
    w += 16 * newton_iters * (2 * m0 + 1)
    w += 6 * (L + p + miller_extra)
    n1 = 2 ** math.ceil(math.log2(L + 1 + 2 * p))
    w += min(4 * (2 * p + 1) * (L + 1), 15 * n1 * math.log2(n1) + 6 * n1) + 6 * (L + 1)
    n2 = 2 ** math.ceil(math.log2(2 * M0 + 2 * L + 1))
    w += min(8 * (2 * M0) * (2 * M), 15 * n2 * math.log2(n2) + 6 * n2)
    w += 5 * NF
    return w


def kernel_source_digest():
    h = hashlib.sha256()
    # the kernel sources and the build script (its flags shape the code too)
    for f in ("csrc/ffbie_kernels.hip", "csrc/ffbie_device.hpp", "csrc/ffbie_kernels.hpp",
              "csrc/ffbie_root.hpp", "build.py"):
        with open(os.path.join(ROOT, "paper_2608_16208_amd", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(key):
    """HBM bytes per launch of the main coefficient pass (key "variant0",
    "variant1" or "mixed") from the committed rocprofv3 counter summary, if it
    was taken from the current kernel source."""
    if not os.path.exists(TRAFFIC_SUMMARY):
        return None
    txt = open(TRAFFIC_SUMMARY).read()
    m = re.search(r"source_digest:\s*(\w+)", txt)
    if not m or m.group(1) != kernel_source_digest():
        return None
    m = re.search(rf"{key}_hbm_bytes_per_launch:\s*([0-9.eE+]+)", txt)
    return float(m.group(1)) if m else None


def cpu_baseline(cfg, n_sample, processes):
    """The oracle (direct quadrature of the coefficients) on a seeded sample of
    the same workload, timed on the host cores; pair-modes/s."""
    import numpy as np
    import workloads
    from oracle import coeffs as ocoeffs
    t, j, ts = workloads.all_pairs(cfg["n_panels"], cfg["M"])
    rng = np.random.default_rng(12345)
    sel = np.sort(rng.choice(t.size, n_sample, replace=False))
    t0 = time.perf_counter()
    ocoeffs.pairs_coeffs(cfg["amp"], cfg["k"], cfg["M"], 2 * cfg["M"], t[sel], j[sel], ts[sel],
                         processes=processes)
    dt = time.perf_counter() - t0
    return dict(value=n_sample * 2 * cfg["M"] / dt, unit="pair-modes/s", cores=processes,
                kind="oracle",
                sample=f"{n_sample} seeded pairs of the same all-pairs workload, "
                       f"{dt:.1f} s wall on {processes} processes")


def _timed(torch, fn):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = fn()
    torch.cuda.synchronize()
    return out, time.perf_counter() - t0


def time_to_field_error(ctx, cfg, torch, np, ffbie, target=1e-8, learned_systems=4):
    """Time to a field within `target` (relative l2 over 64 far points) of the
    plain FP64 LU field of the same discretised system: assembly + solve +
    field evaluation, for LU64 (the reference itself), LU32 + FP64 iterative
    refinement and GMRES.  Sound-soft exterior problem, incident plane wave
    along the workload's direction d, points at radius 3..5."""
    ctx.set_near_rule(None)
    ctx.set_problem(cfg["amp"], cfg["n_panels"], cfg["M"], cfg["k"])
    S = ctx.assemble()                                  # warm-up (allocations, code objects)
    S, t_asm = _timed(torch, lambda: ctx.assemble(S))
    g = ctx.rhs(ffbie.RHS_PLANE_WAVE, cfg["d"])
    rng = np.random.default_rng(1)
    d = rng.standard_normal((64, 3))
    pts = torch.tensor(d / np.linalg.norm(d, axis=1)[:, None] * rng.uniform(3, 5, 64)[:, None])
    W = S.clone()
    (phi, _), t_lu = _timed(torch, lambda: ctx.solve(W, g, method=ffbie.SOLVE_LU64))
    del W
    torch.cuda.empty_cache()
    u_ref, t_f = _timed(torch, lambda: ctx.eval_field(pts, phi))
    out = {"reference": "plain FP64 LU field of the same system, 64 points at |x| in [3, 5]",
           "assembly_s": t_asm, "field_eval_s": t_f, "n_unknowns": int(S.shape[0]),
           "lu64": {"s": t_asm + t_lu + t_f, "solve_s": t_lu}}

    def err(phi_):
        u = ctx.eval_field(pts, phi_)
        return float(((u - u_ref).abs().norm() / u_ref.abs().norm()).item())

    for it in range(1, 9):
        (phi, info), t = _timed(torch, lambda: ctx.solve(S, g, method=ffbie.SOLVE_LU32_IR64,
                                                        tol=1e-15, max_iter=it))
        e = err(phi)
        if e <= target or it == 8:
            out["lu32_ir64"] = {"s": t_asm + t + t_f, "solve_s": t, "refinement_steps": it,
                                "field_error": e, "rel_residual": info["rel_residual"]}
            break
    for name, method in (("gmres", ffbie.SOLVE_GMRES), ("gmres_blockjacobi", ffbie.SOLVE_GMRES_BLOCKJACOBI),
                         ("gmres_lu32", ffbie.SOLVE_GMRES_LU32)):
        for tol in (1e-7, 3e-8, 1e-8, 3e-9, 1e-9, 1e-10):
            (phi, info), t = _timed(torch, lambda: ctx.solve(S, g, method=method, tol=tol, max_iter=3000))
            e = err(phi)
            if e <= target or tol == 1e-10:
                out[name] = {"s": t_asm + t + t_f, "solve_s": t, "iterations": info["iterations"],
                             "residual_tol": tol, "field_error": e}
                break
    if learned_systems > 0:
        # the learned form: a network trained (untimed) by the library's own kernels on the
        # mode-block-Jacobi corrections of star surfaces, then flexible GMRES with it,
        # falling back to plain GMRES (timed together)
        import workloads
        from paper_2608_16208_amd import learned
        ctx.mlp_init(7)

        def mild(i):
            r = np.random.default_rng(6000 + i)
            return dict(amp=workloads.star_amplitudes(4, 4, 0.04, r), k=float(r.uniform(2.0, 6.0)))
        X, T = learned.make_dataset(ctx, [mild(i) for i in range(learned_systems)], M=cfg["M"], n_rhs=8, seed=1)
        learned.train(ctx, X, T, steps=400, batch=1024, lr=1e-3)
        del X, T
        ctx.set_problem(cfg["amp"], cfg["n_panels"], cfg["M"], cfg["k"])
        for tol in (1e-8, 1e-9, 1e-10):
            (phi, info), t = _timed(torch, lambda: ctx.solve(S, g, method=ffbie.SOLVE_FGMRES_MLP, tol=tol,
                                                            max_iter=300))
            e = err(phi)
            if e <= target or tol == 1e-10:
                out["fgmres_mlp"] = {"s": t_asm + t + t_f, "solve_s": t, "iterations": info["iterations"],
                                     "fell_back": info["fell_back"], "residual_tol": tol, "field_error": e,
                                     "trained_on": "%d star surfaces, amplitudes U(-0.04, 0.04), k in [2, 6]"
                                                   % learned_systems}
                break
    del S
    torch.cuda.empty_cache()
    return out


def config3_solve(ctx, torch, np, ffbie):
    """Dense solves at the config-3 geometry (20 amplitudes, k = 20, 32 panels)
    with M = 64 (N = 65536; the FP64 matrix is 69 GB): LU64 against LU32 + FP64
    refinement, each to a field within 1e-8 of the LU64 field."""
    import workloads
    cfg = workloads.config(3)
    ctx.set_near_rule(None)
    ctx.set_problem(cfg["amp"], cfg["n_panels"], 64, cfg["k"])
    S, t_asm = _timed(torch, lambda: ctx.assemble())
    g = ctx.rhs(ffbie.RHS_PLANE_WAVE, cfg["d"])
    rng = np.random.default_rng(1)
    d = rng.standard_normal((64, 3))
    pts = torch.tensor(d / np.linalg.norm(d, axis=1)[:, None] * rng.uniform(3, 5, 64)[:, None])
    W = S.clone()
    (phi, _), t_lu = _timed(torch, lambda: ctx.solve(W, g, method=ffbie.SOLVE_LU64))
    del W
    torch.cuda.empty_cache()
    u_ref = ctx.eval_field(pts, phi)
    out = {"n_unknowns": int(S.shape[0]), "assembly_s": t_asm, "lu64_s": t_asm + t_lu, "lu64_solve_s": t_lu}
    for it in range(1, 6):
        (phi, info), t = _timed(torch, lambda: ctx.solve(S, g, method=ffbie.SOLVE_LU32_IR64, tol=1e-15,
                                                        max_iter=it))
        u = ctx.eval_field(pts, phi)
        e = float(((u - u_ref).abs().norm() / u_ref.abs().norm()).item())
        if e <= 1e-8 or it == 5:
            out["lu32_ir64"] = {"s": t_asm + t, "solve_s": t, "refinement_steps": it, "field_error": e,
                                "rel_residual": info["rel_residual"]}
            break
    for tol in (1e-8, 1e-9, 1e-10, 1e-11):
        (phi, info), t = _timed(torch, lambda: ctx.solve(S, g, method=ffbie.SOLVE_GMRES_LU32, tol=tol,
                                                        max_iter=200))
        u = ctx.eval_field(pts, phi)
        e = float(((u - u_ref).abs().norm() / u_ref.abs().norm()).item())
        if e <= 1e-8 or tol == 1e-11:
            out["gmres_lu32"] = {"s": t_asm + t, "solve_s": t, "iterations": info["iterations"],
                                 "residual_tol": tol, "field_error": e}
            break
    del S
    torch.cuda.empty_cache()
    return out


def near_set_rate(ctx, cfg, torch):
    """Kernel coefficients of the near set (target x near-rule node pairs, the
    method's own workload inside the assembly): pair-modes/s."""
    ctx.set_problem(cfg["amp"], cfg["n_panels"], cfg["M"], cfg["k"])
    t, az, ts = ctx.near_pairs()
    n = t.numel()
    kap = torch.empty((n, 2 * cfg["M"]), dtype=torch.complex128, device=ctx.device)
    ctx.kernel_coeffs(t, az, ts, kappa=kap, status=False)
    reps = 3
    _, dt = _timed(torch, lambda: [ctx.kernel_coeffs(t, az, ts, kappa=kap, status=False)
                                   for _ in range(reps)])
    del kap
    torch.cuda.empty_cache()
    return {"pairs": n, "ms": 1e3 * dt / reps, "value": n * 2 * cfg["M"] * reps / dt,
            "unit": "pair-modes/s"}


def batch_rate(ctx, torch, n_surfaces=64, arena_bytes=32 << 30):
    """Batched coefficient path on the near sets of 64 star surfaces with their
    own M, k and panel counts, against a per-surface launch loop.  The outputs
    (~374 GB complex128, ~187 GB complex64) go through one reusable arena of
    `arena_bytes`, a chunk of whole surfaces per batch plan.  The plans (one per
    chunk) are built before the clock starts: the first chunk's plan autotunes
    the launch (FFT radix, pairs per work item, waves per workgroup) and the
    others take its tuning; each plan's launches are captured in a HIP graph.
    Timed: executing every chunk's plan (FP64, then the mixed-precision path),
    and the loop of single-problem calls (set_problem + kernel_coeffs per
    surface) over the same surfaces."""
    import workloads
    surfs = []
    for s in range(n_surfaces):
        c = workloads.batch_surface(s)
        ctx.set_problem(c["amp"], c["n_panels"], c["M"], c["k"])
        t, az, ts = ctx.near_pairs()
        surfs.append(dict(amp=c["amp"], M=c["M"], k=c["k"], n_panels=c["n_panels"], t=t, az=az, ts=ts))
    modes = sum(sf["t"].numel() * 2 * sf["M"] for sf in surfs)
    arena = torch.empty(arena_bytes // 16, dtype=torch.complex128, device=ctx.device)
    out = {"surfaces": n_surfaces, "pair_modes": int(modes), "pairs": int(sum(sf["t"].numel() for sf in surfs)),
           "arena_GB": arena_bytes / 2 ** 30, "unit": "pair-modes/s"}

    def chunked(elem_bytes):
        chunks, cur, used = [], [], 0
        for sf in surfs:
            b = sf["t"].numel() * 2 * sf["M"] * elem_bytes
            if cur and used + b > arena_bytes:
                chunks.append(cur)
                cur, used = [], 0
            cur.append(sf)
            used += b
        chunks.append(cur)
        return chunks

    def views(ch, dtype):
        flat = arena.view(dtype)
        items, off = [], 0
        for sf in ch:
            n = sf["t"].numel()
            items.append(dict(sf, kappa=flat[off:off + n * 2 * sf["M"]].view(n, 2 * sf["M"])))
            off += n * 2 * sf["M"]
        return items

    # per-surface launch loop (FP64)
    def loop():
        for ch in chunked(16):
            for it in views(ch, torch.complex128):
                ctx.set_problem(it["amp"], it["n_panels"], it["M"], it["k"])
                ctx.kernel_coeffs(it["t"], it["az"], it["ts"], kappa=it["kappa"], status=False)
    loop()
    _, dt = _timed(torch, loop)
    out["per_surface_loop"] = {"s": dt, "value": modes / dt}

    for name, mixed, dtype, eb in (("batched", False, torch.complex128, 16),
                                   ("batched_mixed", True, torch.complex64, 8)):
        chunks = chunked(eb)
        t0 = time.perf_counter()
        first = ctx.batch_plan(views(chunks[0], dtype), autotune=True, graph=True, mixed=mixed)
        tuning = first.tuning()
        by_m = {t["M"]: t for t in tuning}
        plans = [first] + [ctx.batch_plan(views(ch, dtype), graph=True, mixed=mixed, tuning=by_m)
                           for ch in chunks[1:]]
        torch.cuda.synchronize()
        setup = time.perf_counter() - t0
        for pl in plans:
            pl.execute()
        _, dt = _timed(torch, lambda: [pl.execute() for pl in plans])
        out[name] = {"s": dt, "value": modes / dt, "chunks": len(chunks), "tuning_by_M": tuning,
                     "plan_setup_s": setup}
        for pl in plans:
            pl.close()
    del arena
    torch.cuda.empty_cache()
    out["value"] = out["batched"]["value"]
    out["s"] = out["batched"]["s"]
    out["chunks"] = out["batched"]["chunks"]
    return out


def hbm_ceilings(torch, gib=14):
    """What plain device kernels (torch fill, copy, reduction) reach on this
    GPU: the practical ceilings the HBM-bound kernels of the path are measured
    against beside the nominal 8 TB/s (TB/s, best of 5 HIP-event-timed runs)."""
    dev = torch.device("cuda", 0)
    n = gib * 2**30 // 16
    x = torch.empty(n, dtype=torch.complex128, device=dev)
    y = torch.empty(n // 2, dtype=torch.complex128, device=dev)

    def best(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ms = []
        for _ in range(5):
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        return min(ms)
    out = {"bytes": n * 16,
           "write_TBps": n * 16 / best(lambda: x.fill_(1.0 + 2.0j)) / 1e9,
           "copy_TBps": n * 16 / best(lambda: y.copy_(x[: n // 2])) / 1e9,
           "read_TBps": n * 16 / best(lambda: torch.sum(x.real)) / 1e9}
    del x, y
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--variant", type=int, default=0, help="0: swap of cos(k rho)/rho, 1: eq. (3.10)")
    ap.add_argument("--cpu-sample", type=int, default=6144)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-second-variant", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision coefficient run")
    ap.add_argument("--config3-solve", action="store_true",
                    help="also time LU64 against LU32 + IR64 at the config-3 geometry, N = 65536")
    ap.add_argument("--no-ceilings", action="store_true", help="skip the plain-kernel HBM ceilings")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched many-surface measurement")
    ap.add_argument("--no-solve", action="store_true",
                    help="skip the assembly + solve + field measurement")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 2 GiB device copy (reference dispatch for HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the benchmark runs on one GPU only; --gpus must be 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import workloads
    import paper_2608_16208_amd as ffbie

    if args.copy_calibration:
        a = torch.ones(256 * 1024 * 1024, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b
        torch.cuda.empty_cache()

    cfg = workloads.config(2)
    M, M0 = cfg["M"], cfg["M"]
    t, j, ts = workloads.all_pairs(cfg["n_panels"], M)
    n = t.size
    dev = torch.device("cuda", 0)
    tt = torch.tensor(t, device=dev)
    jj = torch.tensor(j, device=dev)
    tss = torch.tensor(ts, device=dev)
    kappa = torch.empty((n, 2 * M), dtype=torch.complex128, device=dev)
    kappa_mixed = None
    status = torch.empty((n,), dtype=torch.int32, device=dev)
    ctx = ffbie.Context(0)

    def run_variant(variant, steps, warmup, mixed=False):
        ctx.set_problem(cfg["amp"], cfg["n_panels"], M, cfg["k"], M0=M0, variant=variant)
        ctx.enable_timing(True)
        kap = kappa_mixed if mixed else kappa
        for _ in range(warmup):
            ctx.kernel_coeffs(tt, jj, tss, kappa=kap, status=True, mixed=mixed)
        torch.cuda.synchronize()
        per = []
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        wall0 = time.perf_counter()
        e0.record()
        for _ in range(steps):
            out = ctx.kernel_coeffs(tt, jj, tss, kappa=kap, status=True, mixed=mixed)
            per.append(ctx.timing())
        e1.record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - wall0
        ms = e0.elapsed_time(e1)
        st = out["status"].cpu().numpy()
        return ms, wall, np.array(per), st

    ms, wall, per, st = run_variant(args.variant, args.steps, args.warmup)
    ms_step = ms / args.steps
    value = n * 2 * M * args.steps / (ms * 1e-3)
    p = (st >> ffbie.P_SHIFT) & 0xFFF
    ok = (st & (ffbie.PAIR_SINGULAR | ffbie.PAIR_UNRESOLVED)) == 0
    p_mean = float(p[ok].mean())
    NF = 2 * M
    m0 = 2 * max(1, cfg["amp"].shape[1] - 1)      # highest Fourier mode of rho^2
    w_pair = algorithmic_flops_per_pair(NF, M, M0, p_mean, m0)
    main_ms = float(per[:, 1].mean())
    achieved = w_pair * n / (main_ms * 1e-3)
    traffic = measured_traffic("variant%d" % args.variant)

    result = {
        "metric": METRIC,
        "value": value,
        "unit": "pair-modes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {
            "workload": "star surface R=1+0.2 sin(3t) cos(2 theta), k=5, 16 panels x 16 GL nodes, "
                        "M=64 (128 azimuths), all 8,355,840 (target node, azimuth, source node) "
                        "pairs; kernel coefficients <e^{ik rho}/rho>_n, n=-63..64",
            "pairs": int(n),
            "pair_modes_per_step": int(n * 2 * M),
            "kappa_variant": "swap of cos(k rho)/rho" if args.variant == 0 else "eq. (3.10)",
        },
        "roofline": {
            "bound": "alu",
            "achieved": achieved / 1e12,
            "peak": PEAK_FP64_VALU / 1e12,
            "unit": "TFLOP/s",
            "frac": achieved / PEAK_FP64_VALU,
            "traffic": traffic,
            "kernel": COEFF_KERNEL + " (main pass)",
            "flops_per_pair": w_pair,
            "p_mean": p_mean,
        },
        "kernels_ms": {"root": float(per[:, 0].mean()), "coeff_main": main_ms,
                       "coeff_refine": float(per[:, 2].mean())},
        "pair_status": {"root_fallback": int(((st & ffbie.PAIR_ROOT_FALLBACK) > 0).sum()),
                        "far_model": int(((st & ffbie.PAIR_FAR) > 0).sum()),
                        "refined": int(((st & ffbie.PAIR_REFINED) > 0).sum()),
                        "unresolved": int(((st & ffbie.PAIR_UNRESOLVED) > 0).sum())},
        "time_to_1e-8_field_error": None,
        "wall_s_timed": wall,
    }
    # <rho^-1>_l, l = 0..L, emitted beside the kappa table (the full-layout launch)
    rho = torch.empty((n, M + M0 + 1), dtype=torch.complex128, device=dev)
    ctx.set_problem(cfg["amp"], cfg["n_panels"], M, cfg["k"], M0=M0, variant=0)
    ctx.enable_timing(True)
    ctx.kernel_coeffs(tt, jj, tss, kappa=kappa, rhoinv_out=rho, status=True)
    (_, dt_r) = _timed(torch, lambda: ctx.kernel_coeffs(tt, jj, tss, kappa=kappa, rhoinv_out=rho, status=True))
    result["with_rhoinv"] = {"ms_per_call": 1e3 * dt_r, "rhoinv_coeffs_per_s": n * (M + M0 + 1) / dt_r,
                             "pair_modes_per_s": n * 2 * M / dt_r,
                             "coeff_main_ms": float(ctx.timing()[1])}
    del rho
    if not args.no_second_variant:
        other = 1 - args.variant
        ms2, _, per2, _ = run_variant(other, max(1, args.steps // 2), 1)
        result["value_other_variant"] = {
            "kappa_variant": "eq. (3.10)" if other == 1 else "swap of cos(k rho)/rho",
            "value": n * 2 * M * max(1, args.steps // 2) / (ms2 * 1e-3),
            "coeff_main_ms": float(per2[:, 1].mean())}
    if not args.no_mixed:
        # the same launch with the FP32 spectral stage (complex64 table)
        kappa_mixed = torch.empty((n, 2 * M), dtype=torch.complex64, device=dev)
        msx, _, perx, stx = run_variant(0, args.steps, args.warmup, mixed=True)
        okx = (stx & (ffbie.PAIR_SINGULAR | ffbie.PAIR_UNRESOLVED)) == 0
        p_mean_x = float(((stx >> ffbie.P_SHIFT) & 0xFFF)[okx].mean())
        main_x = float(perx[:, 1].mean())
        ach_x = algorithmic_flops_per_pair(NF, M, M0, p_mean_x, m0) * n / (main_x * 1e-3)
        worst = 0.0
        for a in range(0, n, 1 << 20):
            k64 = kappa[a:a + (1 << 20)]
            e = (torch.linalg.vector_norm(kappa_mixed[a:a + (1 << 20)].to(torch.complex128) - k64, dim=1)
                 / torch.linalg.vector_norm(k64, dim=1))
            worst = max(worst, float(e.max().item()))
        result["mixed"] = {
            "value": n * 2 * M * args.steps / (msx * 1e-3), "unit": "pair-modes/s",
            "ms_per_step": msx / args.steps, "dtype": "f32 spectral stage, f64 samples/root/A_m",
            "kernels_ms": {"root": float(perx[:, 0].mean()), "coeff_main": main_x,
                           "coeff_refine": float(perx[:, 2].mean())},
            "p_mean": p_mean_x, "refined": int(((stx & ffbie.PAIR_REFINED) > 0).sum()),
            "max_row_rel_err_vs_fp64": worst, "stated_bound": 1e-5,
            "roofline": {"bound": "alu", "achieved": ach_x / 1e12, "peak": PEAK_FP32_VALU_UNPACKED / 1e12,
                         "unit": "TFLOP/s", "frac": ach_x / PEAK_FP32_VALU_UNPACKED,
                         "traffic": measured_traffic("mixed"),
                         "kernel": COEFF_KERNEL + " (main pass, FP32 spectral stage)"}}
        del kappa_mixed
    del kappa
    torch.cuda.empty_cache()
    if not args.no_solve:
        result["time_to_1e-8_field_error"] = time_to_field_error(ctx, cfg, torch, np, ffbie)
        result["near_set"] = near_set_rate(ctx, cfg, torch)
    if args.config3_solve:
        result["config3_geometry_solve"] = config3_solve(ctx, torch, np, ffbie)
    if not args.no_batch:
        result["batch_64_surfaces"] = batch_rate(ctx, torch)
    if not args.no_ceilings:
        result["hbm_ceilings"] = hbm_ceilings(torch)
    if not args.no_cpu_baseline:
        procs = min(16, os.cpu_count() or 1)
        result["cpu_baseline"] = cpu_baseline(cfg, args.cpu_sample, procs)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
