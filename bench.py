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
COUNTER_SUMMARY = os.path.join(ROOT, "profiles", "coeff_kernel_config2_allpairs_kernel_stats.md")


def own_flops_per_pair(kind, NF, M, M0, p, miller_extra=100.0):
    """Flops the main coefficient pass itself performs for one pair (FMA = 2,
    complex multiply = 6, complex FFT of N points = 5 N log2 N; square roots,
    reciprocals and sincos are counted apart by special_ops_per_pair; the
    root search is the root kernel's and is counted by root_flops_per_pair).
    ``p`` is the truncation index of eq. (3.24) the pair used.
      kind "swap":   one complex N_F-point transform of F cos(k rho) +
                     i sin(k rho)/rho, A_m for m <= M + p, one (M+1) x (2p+1)
                     swap convolution for <cos(k rho)/rho> and its phases;
      kind "swap+rhoinv": two transforms, A_m to L + p, the convolution of
                     eq. (3.25) over l = 0..L and the swap convolution;
      kind "paper":  eq. (3.10): two transforms, A_m to L + p, the
                     convolution of eq. (3.25) over l = 0..L, and the direct
                     (M+1) x (2 M0 - 1) complex convolution with <cos k rho>.
    Samples (20 N_F) are common to all three."""
    L = M + M0
    lg = math.log2(NF)
    w = 20 * NF
    conv_swap = 4 * (2 * p + 1) * (M + 1) + 6 * (M + 1) + 6 * (p + 1)
    conv_rho = 4 * (2 * p + 1) * (L + 1) + 6 * (L + 1) + 6 * (p + 1)
    if kind == "swap":
        w += 5 * NF * lg + 6 * (M + p + miller_extra) + conv_swap
    elif kind == "swap+rhoinv":
        w += 2 * 5 * NF * lg + 6 * (L + p + miller_extra) + conv_rho + conv_swap
    elif kind == "paper":
        w += 2 * 5 * NF * lg + 6 * (L + p + miller_extra) + conv_rho + 8 * (2 * M0 - 1) * (M + 1)
    else:
        raise ValueError(kind)
    return w


def special_ops_per_pair(NF):
    """Transcendental operations per pair (sqrt, 1/sqrt, sincos of each sample
    and the smooth factor's square root), reported apart from the flops."""
    return 5 * NF


def root_flops_per_pair(M, m0, newton_iters=6.0):
    """The root kernel's work per pair: the grid minimiser over the 2M
    azimuths (~10 flops per grid point) and the complex Newton iterations on a
    trigonometric polynomial of degree m0 (16 flops per term)."""
    return 10 * 2 * M + 16 * newton_iters * (2 * m0 + 1)


def kernel_source_digest():
    """Digest of what shapes the coefficient kernels' code: their sources and
    their compile line (the build flags and their per-file additions)."""
    from paper_2608_16208_amd import build as b
    h = hashlib.sha256()
    for f in ("csrc/ffbie_kernels.hip", "csrc/ffbie_device.hpp", "csrc/ffbie_kernels.hpp",
              "csrc/ffbie_root.hpp"):
        with open(os.path.join(ROOT, "paper_2608_16208_amd", f), "rb") as fh:
            h.update(fh.read())
    flags = [f for f in b.FLAGS if not f.startswith("-I")] + b.EXTRA.get("csrc/ffbie_kernels.hip", [])
    h.update(" ".join(flags).encode())
    return h.hexdigest()[:16]


def measured_counts(key):
    """A per-launch figure (HBM bytes "variant0_hbm_bytes_per_launch", or the
    FP64 instruction counts per pair "fp64_fma_per_pair" ...) from the committed
    rocprofv3 summaries, if they were taken from the current kernel source."""
    for path in (TRAFFIC_SUMMARY, COUNTER_SUMMARY):
        if not os.path.exists(path):
            continue
        txt = open(path).read()
        m = re.search(r"source_digest:\s*(\w+)", txt)
        if not m or m.group(1) != kernel_source_digest():
            continue
        m = re.search(rf"{key}:\s*([0-9.eE+]+)", txt)
        if m:
            return float(m.group(1))
    return None


def measured_traffic(key):
    """HBM bytes per launch of the main coefficient pass (key "variant0",
    "variant1" or "mixed") from the committed counter summary, or None."""
    return measured_counts(f"{key}_hbm_bytes_per_launch")


def host_cpu():
    """Core counts and model of the host the oracle is timed on."""
    info = {"nproc": os.cpu_count(), "affinity": len(os.sched_getaffinity(0))}
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                info["model"] = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return info


def cpu_baseline(cfg, n_sample, n_single, max_procs=16):
    """The oracle (direct quadrature of the coefficients, oracle/coeffs.py) on
    a seeded, stratified sample of the benchmarked workload, timed on the host:
    80 % of the pairs drawn uniformly from the all-pairs workload, 20 % small-b
    near pairs (sources 1e-7 .. 1e-1 panel lengths from the target, the spread
    of the near-panel quadrature nodes), once in a single process and once on
    all host cores (capped at the one-GPU share of 16).  Pair-modes/s; the
    all-cores figure is `value`."""
    import numpy as np
    import workloads
    from oracle import coeffs as ocoeffs
    M = cfg["M"]

    def sample(n, seed):
        rng = np.random.default_rng(seed)
        t, j, ts = workloads.all_pairs(cfg["n_panels"], M)
        n_near = n // 5
        sel = np.sort(rng.choice(t.size, n - n_near, replace=False))
        tn, jn, tsn = workloads.sample_pairs(cfg["n_panels"], M, n_near, seed=seed + 1, near_fraction=1.0)
        return (np.concatenate([t[sel], tn]), np.concatenate([j[sel], jn]), np.concatenate([ts[sel], tsn]))

    hc = host_cpu()
    procs = max(1, min(max_procs, hc["affinity"]))
    out = {"unit": "pair-modes/s", "kind": "oracle", "host": hc}
    for name, n, p_, seed in (("single_core", n_single, 1, 54321), ("all_cores", n_sample, procs, 12345)):
        t, j, ts = sample(n, seed)
        t0 = time.perf_counter()
        ocoeffs.pairs_coeffs(cfg["amp"], cfg["k"], M, 2 * M, t, j, ts, processes=p_)
        dt = time.perf_counter() - t0
        out[name] = {"value": n * 2 * M / dt, "pairs": n, "processes": p_, "wall_s": dt}
    out["value"] = out["all_cores"]["value"]
    out["cores"] = procs
    out["sample"] = (f"{n_sample} seeded pairs (80 % uniform over the all-pairs workload, 20 % small-b near "
                     f"pairs) on {procs} processes x 1 thread; single process: {n_single} pairs of the same mix")
    return out


def log(msg):
    """Progress line on stderr (the JSON result is the only line on stdout)."""
    print("[bench] " + msg, file=sys.stderr, flush=True)


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


def double_layer_block(ctx, cfg, torch, np, ffbie, tt, jj, tss, kappa, steps=3, solve=True):
    """The double-layer operators of Sec. 4 on config 2.
    * coefficients <tau_0 (ik rho - 1) e^{ik rho} / rho^3>_n of K and K' for
      the same 8,355,840 pairs as the headline workload, pair-modes/s (root +
      main + refine launches, HIP-synchronised wall time per call);
    * the exterior Dirichlet problem as the second-kind system (K + I) psi = g
      (density unknowns) next to the first-kind S phi = g: assembly time,
      GMRES iterations and time to a field within 1e-8 of each system's own
      LU64 field, and both LU64 fields against the exact field of a point
      source inside the surface."""
    n = tt.numel()
    M = cfg["M"]
    ctx.set_near_rule(None)
    ctx.set_problem(cfg["amp"], cfg["n_panels"], M, cfg["k"])
    out = {"workload": "config 2, all pairs, M = 64"}
    for name, adj in (("K", False), ("K'", True)):
        ctx.kernel_coeffs_dl(tt, jj, tss, adjoint=adj, kappa=kappa)
        _, dt = _timed(torch, lambda: [ctx.kernel_coeffs_dl(tt, jj, tss, adjoint=adj, kappa=kappa)
                                       for _ in range(steps)])
        st = ctx.kernel_coeffs_dl(tt, jj, tss, adjoint=adj, kappa=kappa)["status"].cpu().numpy()
        out[name] = {"pair_modes_per_s": n * 2 * M * steps / dt, "ms_per_call": 1e3 * dt / steps,
                     "refined": int(((st & ffbie.PAIR_REFINED) > 0).sum()),
                     "unresolved": int(((st & ffbie.PAIR_UNRESOLVED) > 0).sum())}
    if not solve:
        return out
    rng = np.random.default_rng(1)
    d = rng.standard_normal((64, 3))
    P = d / np.linalg.norm(d, axis=1)[:, None] * rng.uniform(3, 5, 64)[:, None]
    pts = torch.tensor(P)
    p_in = np.array([0.1, -0.2, 0.15])
    rho = np.linalg.norm(P - p_in, axis=1)
    exact = np.exp(1j * cfg["k"] * rho) / (4 * np.pi * rho)
    g = ctx.rhs(ffbie.RHS_PLANE_WAVE, cfg["d"])
    g_ps = ctx.rhs(ffbie.RHS_POINT_SOURCE, list(p_in))
    for name, op, shift, unk in (("first_kind_S", ffbie.OP_S, 0.0, ffbie.UNKNOWN_SCALED),
                                 ("second_kind_K_plus_I", ffbie.OP_K, 1.0, ffbie.UNKNOWN_DENSITY)):
        fop = ffbie.OP_S if op == ffbie.OP_S else ffbie.OP_K
        A = ctx.assemble(op=op, shift=shift, unknowns=unk)
        A, t_asm = _timed(torch, lambda: ctx.assemble(A, op=op, shift=shift, unknowns=unk))
        W = A.clone()
        ctx.lu_factor(W)
        u_ref = ctx.eval_field(pts, ctx.lu_solve(W, g), op=fop, unknowns=unk)
        u_ps = ctx.eval_field(pts, ctx.lu_solve(W, g_ps), op=fop, unknowns=unk).cpu().numpy()
        del W
        torch.cuda.empty_cache()
        rec = {"assembly_s": t_asm,
               "point_source_field_error": float(np.linalg.norm(u_ps - exact) / np.linalg.norm(exact))}
        for tol in (1e-7, 3e-8, 1e-8, 3e-9, 1e-9, 1e-10):
            (x, info), t = _timed(torch, lambda: ctx.solve(A, g, method=ffbie.SOLVE_GMRES, tol=tol, max_iter=3000))
            u = ctx.eval_field(pts, x, op=fop, unknowns=unk)
            e = float(((u - u_ref).abs().norm() / u_ref.abs().norm()).item())
            if e <= 1e-8 or tol == 1e-10:
                rec["gmres"] = {"residual_tol": tol, "iterations": info["iterations"], "solve_s": t,
                                "field_error_vs_own_lu": e, "time_to_1e-8_s": t_asm + t}
                break
        out[name] = rec
        del A
        torch.cuda.empty_cache()
    return out


def banded_block(ctx, cfg, torch, np, ffbie, tt, jj, tss, kappa, steps=3, sample=1 << 18):
    """The O(M) banded route to <rho^-1>_l of Sec. 3.2.1 (ffbie_rhoinv_banded)
    next to the swap path emitting the same table (ffbie_kernel_coeffs with
    <rho^-1>): the config-2 all-pairs launch (M = M0 = 64, m0 by the rule of
    eq. (3.13)), its largest row difference from the swap path, and the
    crossover study the paper leaves out: ms per call of both routes on a
    seeded sample of config-2 pairs (30 % near pairs) at M = 16 .. 128."""
    import workloads
    n = tt.numel()
    M = cfg["M"]
    dev = tt.device
    ctx.set_problem(cfg["amp"], cfg["n_panels"], M, cfg["k"])
    band = torch.empty((n, 2 * M + 1), dtype=torch.complex128, device=dev)
    out = ctx.rhoinv_banded(tt, jj, tss, rhoinv=band)
    m0 = out["m0"]
    _, dt = _timed(torch, lambda: [ctx.rhoinv_banded(tt, jj, tss, rhoinv=band) for _ in range(steps)])
    st = out["status"].cpu().numpy()
    ref = torch.empty_like(band)
    ctx.kernel_coeffs(tt, jj, tss, kappa=kappa, rhoinv_out=ref, status=False)
    _, dt_s = _timed(torch, lambda: [ctx.kernel_coeffs(tt, jj, tss, kappa=kappa, rhoinv_out=ref, status=False)
                                     for _ in range(steps)])
    worst = 0.0
    for a in range(0, n, 1 << 20):
        d = (torch.amax(torch.abs(band[a:a + (1 << 20)] - ref[a:a + (1 << 20)]), dim=1)
             / torch.amax(torch.abs(ref[a:a + (1 << 20)]), dim=1))
        worst = max(worst, float(d.max().item()))
    del band, ref
    torch.cuda.empty_cache()
    res = {"workload": "config 2, all %d pairs, M = M0 = %d, L = %d" % (n, M, 2 * M), "m0": m0,
           "ms_per_call": 1e3 * dt / steps, "rhoinv_coeffs_per_s": n * (2 * M + 1) * steps / dt,
           "swap_with_rhoinv_ms_per_call": 1e3 * dt_s / steps, "ratio_banded_to_swap": dt / dt_s,
           "max_row_rel_diff_vs_swap": worst,
           "not_positive_definite_pairs": int(((st & ffbie.PAIR_NOT_PD) > 0).sum())}
    cross = []
    for Mx in (16, 32, 64, 128):
        t, j, ts = workloads.sample_pairs(cfg["n_panels"], Mx, sample, seed=1)
        a_t, a_j, a_ts = (torch.tensor(v, device=dev) for v in (t, j, ts))
        ctx.set_problem(cfg["amp"], cfg["n_panels"], Mx, cfg["k"])
        rb = torch.empty((sample, 2 * Mx + 1), dtype=torch.complex128, device=dev)
        rs = torch.empty_like(rb)
        kx = torch.empty((sample, 2 * Mx), dtype=torch.complex128, device=dev)
        ctx.rhoinv_banded(a_t, a_j, a_ts, rhoinv=rb)
        _, tb = _timed(torch, lambda: [ctx.rhoinv_banded(a_t, a_j, a_ts, rhoinv=rb) for _ in range(5)])
        so = ctx.kernel_coeffs(a_t, a_j, a_ts, kappa=kx, rhoinv_out=rs)
        _, tsw = _timed(torch, lambda: [ctx.kernel_coeffs(a_t, a_j, a_ts, kappa=kx, rhoinv_out=rs,
                                                          status=False) for _ in range(5)])
        sst = so["status"].cpu().numpy()
        cross.append({"M": Mx, "pairs": sample, "banded_ms": 1e3 * tb / 5, "swap_with_rhoinv_ms": 1e3 * tsw / 5,
                      "ratio_banded_to_swap": tb / tsw,
                      "swap_refined": int(((sst & ffbie.PAIR_REFINED) > 0).sum()),
                      "swap_unresolved": int(((sst & ffbie.PAIR_UNRESOLVED) > 0).sum())})
        del rb, rs, kx
    res["crossover"] = cross
    ctx.set_problem(cfg["amp"], cfg["n_panels"], M, cfg["k"])
    return res


def _interior_errors(ctx, torch, np, ffbie):
    """E_j of the interior point-source protocol of Sec. 5 for one discretisation:
    (IDP) by S and by K - I, (INP) by K' + I, LU64, E_j = ||u_num - u_exa||_2 /
    #(points) over 200 seeded points of the test ball, source r* = (3, 4, 10.5).
    Returns error(amp, axes, k, n_panels, M, name) for name in S, K, K'."""
    import workloads
    P = workloads.interior_test_points()
    src = workloads.INTERIOR_SOURCE
    pts = torch.tensor(P)
    ctx.set_near_rule(None)
    ops = {"S": (ffbie.OP_S, 0.0, ffbie.UNKNOWN_SCALED, ffbie.RHS_POINT_SOURCE, ffbie.OP_S),
           "K": (ffbie.OP_K, -1.0, ffbie.UNKNOWN_DENSITY, ffbie.RHS_POINT_SOURCE, ffbie.OP_K),
           "K'": (ffbie.OP_KP, 1.0, ffbie.UNKNOWN_DENSITY, ffbie.RHS_POINT_SOURCE_DN, ffbie.OP_S)}

    def error(amp, axes, k, npan, M, name):
        ctx.set_problem(amp, npan, M, k, axes=axes)
        r = np.linalg.norm(P - src, axis=1)
        exact = np.exp(1j * k * r) / (4 * np.pi * r)
        op, shift, unk, rhs, fop = ops[name]
        g = ctx.rhs(rhs, list(src))
        A = ctx.assemble(op=op, shift=shift, unknowns=unk)
        x, _ = ctx.solve(A, g, method=ffbie.SOLVE_LU64)
        u = ctx.eval_field(pts, x, op=fop, unknowns=unk).cpu().numpy()
        del A
        torch.cuda.empty_cache()
        return float(np.linalg.norm(u - exact) / len(exact))
    return error


def interior_protocol(ctx, torch, np, ffbie):
    """The interior point-source protocol of Sec. 5 (see _interior_errors):
    * the ellipsoid of Example 1 at the rows of the paper's Table 1 (same N_p,
      the next supported 2M), the paper's E_j beside each;
    * an analytic star surface (workloads.INTERIOR_AMP) at INTERIOR_ROWS."""
    import workloads
    error = _interior_errors(ctx, torch, np, ffbie)
    t0 = time.perf_counter()
    ell = []
    for k, dS, eS, dK, eK, dKp, eKp in workloads.PAPER_TABLE1:
        rec = {"k": k}
        for name, (npan, two_m), paper in (("S", dS, eS), ("K", dK, eK), ("K'", dKp, eKp)):
            M = workloads.supported_M(two_m)
            rec[name] = {"N_p": npan, "2M": 2 * M, "E": error(None, workloads.ELLIPSOID_AXES, k, npan, M, name),
                         "paper_2M": two_m, "paper_E": paper}
        ell.append(rec)
    star = []
    for k, npan, M in workloads.INTERIOR_ROWS:
        rec = {"k": k, "N_p": npan, "2M": 2 * M, "N": 32 * M * npan}
        for name in ("S", "K", "K'"):
            rec["E_" + name] = error(workloads.INTERIOR_AMP, None, k, npan, M, name)
        star.append(rec)
    return {"points": "200 seeded points of the ball |r - (0, -0.2, 0.1)| < 0.2, r* = (3, 4, 10.5)",
            "ellipsoid_table1": ell,
            "star": {"surface": "R = 1 + 0.2 sin t cos(theta) + 0.1 sin 2t cos(theta)", "rows": star},
            "wall_s": time.perf_counter() - t0}


def ellipsoid_convergence(ctx, torch, np, ffbie):
    """The convergence study of Sec. 5, Example 1 at k = 16: E_S, E_K and E_K'
    of the interior protocol on the ellipsoid with N_p = 16 panels and 2M =
    32 .. 256, and with 2M = 128 and N_p = 4 .. 32 (the paper's study sweeps
    2M at N_p = 16 and N_p at 2M = 100)."""
    import workloads
    error = _interior_errors(ctx, torch, np, ffbie)
    t0 = time.perf_counter()
    k = 16.0
    runs = {"vs_2M (N_p = 16)": [(16, M) for M in (16, 32, 64, 128)],
            "vs_N_p (2M = 128)": [(npan, 64) for npan in (4, 8, 16, 32)]}
    out = {"k": k, "surface": "ellipsoid x^2 + y^2/4 + z^2/9 = 1"}
    for label, rows in runs.items():
        recs = []
        for npan, M in rows:
            rec = {"N_p": npan, "2M": 2 * M, "N": 32 * M * npan}
            for name in ("S", "K", "K'"):
                rec["E_" + name] = error(None, workloads.ELLIPSOID_AXES, k, npan, M, name)
            recs.append(rec)
            log("convergence %s: %s" % (label, json.dumps(rec)))
        out[label] = recs
    out["wall_s"] = time.perf_counter() - t0
    return out


def config3_block(ctx, torch, np, ffbie, solve=True):
    """Config 3: the star surface with 20 seeded amplitudes U(-0.1, 0.1), k = 20,
    32 panels, M = 128.
    * near-set kernel coefficients (6,160,384 target x near-rule-node pairs,
      256 coefficients each) on the FP64 path and the mixed path (FP32 spectral
      stage, complex64 table), pair-modes/s, and the mixed table's largest row
      error against the FP64 one;
    * dense solves at this geometry and k with M = 64 (N = 65536; the FP64
      matrix at M = 128 would be 275 GB): LU64 against LU32 + FP64 refinement
      and GMRES preconditioned by the complex64 LU, each judged by its field
      at 64 far points against the LU64 field (time-to-1e-8)."""
    import workloads
    cfg = workloads.config(3)
    M = cfg["M"]
    out = {"surface": "R = 1 + sum_{l<=4, m<=4} a_lm sin(l t) cos(m theta), a_lm ~ U(-0.1, 0.1) from rng(3)",
           "k": cfg["k"], "n_panels": cfg["n_panels"], "M": M}
    ctx.set_near_rule(None)
    ctx.set_problem(cfg["amp"], cfg["n_panels"], M, cfg["k"])
    ctx.enable_timing(True)
    t, az, ts = ctx.near_pairs()
    n = t.numel()
    near = {"pairs": int(n), "pair_modes": int(n * 2 * M)}
    kap = torch.empty((n, 2 * M), dtype=torch.complex128, device=ctx.device)
    kapx = torch.empty((n, 2 * M), dtype=torch.complex64, device=ctx.device)
    for name, k_out, mixed in (("fp64", kap, False), ("mixed", kapx, True)):
        ctx.kernel_coeffs(t, az, ts, kappa=k_out, status=False, mixed=mixed)
        reps = 3
        per = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            o = ctx.kernel_coeffs(t, az, ts, kappa=k_out, status=True, mixed=mixed)
            per.append(ctx.timing())
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / reps
        st = o["status"].cpu().numpy()
        ok = (st & (ffbie.PAIR_SINGULAR | ffbie.PAIR_UNRESOLVED)) == 0
        p_mean = float(((st >> ffbie.P_SHIFT) & 0xFFF)[ok].mean())
        main_ms = float(np.mean([q[1] for q in per]))
        w = own_flops_per_pair("swap", 2 * M, M, M, p_mean)
        near[name] = {"ms": 1e3 * dt, "value": n * 2 * M / dt, "unit": "pair-modes/s",
                      "coeff_main_ms": main_ms, "p_mean": p_mean,
                      "refined": int(((st & ffbie.PAIR_REFINED) > 0).sum()),
                      "unresolved": int(((st & ffbie.PAIR_UNRESOLVED) > 0).sum()),
                      "frac_of_78.6TFLOPs": w * n / (main_ms * 1e-3) / PEAK_FP64_VALU}
    worst = 0.0
    for a in range(0, n, 1 << 19):
        k64 = kap[a:a + (1 << 19)]
        e = (torch.linalg.vector_norm(kapx[a:a + (1 << 19)].to(torch.complex128) - k64, dim=1)
             / torch.linalg.vector_norm(k64, dim=1))
        worst = max(worst, float(e.max().item()))
    near["mixed"]["max_row_rel_err_vs_fp64"] = worst
    out["near_set"] = near
    log("config-3 near set done")
    del kap, kapx, t, az, ts
    torch.cuda.empty_cache()
    if not solve:
        return out

    Ms = 64
    ctx.set_problem(cfg["amp"], cfg["n_panels"], Ms, cfg["k"])
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
    N = int(S.shape[0])
    log("config-3 LU64 (N = %d) %.2f s" % (N, t_lu))
    sol = {"M": Ms, "n_unknowns": N, "assembly_s": t_asm,
           "reference": "LU64 field of the same system, 64 points at |x| in [3, 5]",
           "lu64": {"s": t_asm + t_lu, "solve_s": t_lu, "TFLOPs": 8 / 3 * N ** 3 / t_lu / 1e12}}

    def ferr(phi_):
        u = ctx.eval_field(pts, phi_)
        return float(((u - u_ref).abs().norm() / u_ref.abs().norm()).item())

    (phi, info), t = _timed(torch, lambda: ctx.solve(S, g, method=ffbie.SOLVE_LU32_IR64, tol=1e-12, max_iter=5))
    sol["lu32_ir64"] = {"s": t_asm + t, "solve_s": t, "refinement_steps": info["iterations"],
                        "field_error": ferr(phi), "rel_residual": info["rel_residual"],
                        "reaches_1e-8": ferr(phi) <= 1e-8}
    (phi, info), t = _timed(torch, lambda: ctx.solve(S, g, method=ffbie.SOLVE_GMRES_LU32, tol=1e-10,
                                                    max_iter=200))
    sol["gmres_lu32"] = {"s": t_asm + t, "solve_s": t, "iterations": info["iterations"],
                         "residual_tol": 1e-10, "field_error": ferr(phi), "reaches_1e-8": ferr(phi) <= 1e-8}
    out["solve_M64"] = sol
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
    own M, k and panel counts, against a per-surface launch loop.  Members the
    library rejects are listed under "skipped" with the reason.  The outputs
    (~374 GB complex128, ~187 GB complex64) go through one reusable arena of
    `arena_bytes`, a chunk of whole surfaces per batch plan.  The plans (one per
    chunk) are built before the clock starts: the first chunk's plan autotunes
    the launch (FFT radix, pairs per work item, waves per workgroup) and the
    others take its tuning; each plan's launches are captured in a HIP graph.
    Plan set-up is reported cold (the autotuner times its candidates and
    writes the on-disk tuning cache) and warm (the cache supplies them).
    Timed: executing every chunk's plan (FP64, then the mixed-precision path),
    and the loop of single-problem calls (set_problem + kernel_coeffs per
    surface) over the same surfaces."""
    import workloads
    import paper_2608_16208_amd as ffbie
    surfs, skipped = [], []
    for s in range(n_surfaces):
        c = workloads.batch_surface(s)
        try:
            ctx.set_problem(c["amp"], c["n_panels"], c["M"], c["k"])
        except ffbie.FfbieError as e:
            # the library rejects the member (M whose 2M-point transforms need
            # radix 3); it is reported, not redrawn
            skipped.append({"surface": s, "M": c["M"], "n_panels": c["n_panels"], "reason": str(e)})
            continue
        t, az, ts = ctx.near_pairs()
        surfs.append(dict(amp=c["amp"], M=c["M"], k=c["k"], n_panels=c["n_panels"], t=t, az=az, ts=ts))
    modes = sum(sf["t"].numel() * 2 * sf["M"] for sf in surfs)
    arena = torch.empty(arena_bytes // 16, dtype=torch.complex128, device=ctx.device)
    out = {"surfaces": n_surfaces, "surfaces_run": len(surfs), "skipped": skipped,
           "pair_modes": int(modes), "pairs": int(sum(sf["t"].numel() for sf in surfs)),
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

    # the autotuner's choices go to an on-disk cache: the first set of plans
    # tunes and writes it (cold), a second set reads it (warm)
    import tempfile
    cache_dir = tempfile.mkdtemp(prefix="ffbie_tune_")
    ctx.set_tuning_cache(os.path.join(cache_dir, "tuning.json"))

    def make_plans(chunks, dtype, mixed):
        t0 = time.perf_counter()
        first = ctx.batch_plan(views(chunks[0], dtype), autotune=True, graph=True, mixed=mixed)
        tuning = first.tuning()
        by_m = {t["M"]: t for t in tuning}
        plans = [first] + [ctx.batch_plan(views(ch, dtype), graph=True, mixed=mixed, tuning=by_m)
                           for ch in chunks[1:]]
        torch.cuda.synchronize()
        return plans, tuning, time.perf_counter() - t0

    for name, mixed, dtype, eb in (("batched", False, torch.complex128, 16),
                                   ("batched_mixed", True, torch.complex64, 8)):
        chunks = chunked(eb)
        plans, _, setup_cold = make_plans(chunks, dtype, mixed)
        for pl in plans:
            pl.close()
        plans, tuning, setup = make_plans(chunks, dtype, mixed)
        for pl in plans:
            pl.execute()
        _, dt = _timed(torch, lambda: [pl.execute() for pl in plans])
        out[name] = {"s": dt, "value": modes / dt, "chunks": len(chunks), "tuning_by_M": tuning,
                     "plan_setup_s": setup, "plan_setup_cold_s": setup_cold}
        for pl in plans:
            pl.close()
    ctx.set_tuning_cache(None)
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
    ap.add_argument("--cpu-sample", type=int, default=4096,
                    help="pairs of the all-cores oracle sample")
    ap.add_argument("--cpu-sample-single", type=int, default=256,
                    help="pairs of the single-process oracle sample")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-second-variant", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision coefficient run")
    ap.add_argument("--no-config3", action="store_true",
                    help="skip the config-3 block (near-set coefficients at M = 128, FP64 and mixed, "
                         "and the N = 65536 solves)")
    ap.add_argument("--no-ceilings", action="store_true", help="skip the plain-kernel HBM ceilings")
    ap.add_argument("--no-banded", action="store_true",
                    help="skip the O(M) banded <rho^-1> route and its crossover study")
    ap.add_argument("--no-double-layer", action="store_true",
                    help="skip the double-layer block (K and K' coefficients, second-kind solve)")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batched many-surface measurement")
    ap.add_argument("--no-solve", action="store_true",
                    help="skip the assembly + solve + field measurement")
    ap.add_argument("--convergence", action="store_true",
                    help="add the k = 16 ellipsoid convergence study (about two minutes of solves)")
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
    log("main workload timed: %.3f ms per step" % (ms / args.steps))
    ms_step = ms / args.steps
    value = n * 2 * M * args.steps / (ms * 1e-3)
    ok = (st & (ffbie.PAIR_SINGULAR | ffbie.PAIR_UNRESOLVED)) == 0
    p_mean = float(((st >> ffbie.P_SHIFT) & 0xFFF)[ok].mean())
    NF = 2 * M
    m0 = 2 * max(1, cfg["amp"].shape[1] - 1)      # highest Fourier mode of rho^2
    kind = "swap" if args.variant == 0 else "paper"
    w_pair = own_flops_per_pair(kind, NF, M, M0, p_mean)
    main_ms = float(per[:, 1].mean())
    root_ms = float(per[:, 0].mean())
    achieved = w_pair * n / (main_ms * 1e-3)
    traffic = measured_traffic("variant%d" % args.variant)
    roofline = {
        "bound": "alu",
        "achieved": achieved / 1e12,
        "peak": PEAK_FP64_VALU / 1e12,
        "unit": "TFLOP/s",
        "frac": achieved / PEAK_FP64_VALU,
        "traffic": traffic,
        "kernel": COEFF_KERNEL + " (main pass)",
        "flops_per_pair": w_pair,
        "flops_counted": "own work of this launch: %s" % kind,
        "special_ops_per_pair": special_ops_per_pair(NF),
        "p_mean": p_mean,
    }
    # what the FP64 units executed, from the committed SQ counters of this build
    fma, add, mul = (measured_counts("fp64_%s_per_pair" % x) for x in ("fma", "add", "mul"))
    if args.variant == 0 and None not in (fma, add, mul):
        ex = 64 * (2 * fma + add + mul) * n / (main_ms * 1e-3)
        roofline["executed_fp64_TFLOPs"] = ex / 1e12
        roofline["executed_fp64_frac"] = ex / PEAK_FP64_VALU

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
        "roofline": roofline,
        "kernels_ms": {"root": root_ms, "coeff_main": main_ms,
                       "coeff_refine": float(per[:, 2].mean())},
        "root_kernel": {"ms": root_ms, "flops_per_pair": root_flops_per_pair(M, m0),
                        "TFLOPs": root_flops_per_pair(M, m0) * n / (root_ms * 1e-3) / 1e12},
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
    main_r = float(ctx.timing()[1])
    w_r = own_flops_per_pair("swap+rhoinv", NF, M, M0, p_mean)
    result["with_rhoinv"] = {"ms_per_call": 1e3 * dt_r, "rhoinv_coeffs_per_s": n * (M + M0 + 1) / dt_r,
                             "pair_modes_per_s": n * 2 * M / dt_r, "coeff_main_ms": main_r,
                             "flops_per_pair": w_r, "frac": w_r * n / (main_r * 1e-3) / PEAK_FP64_VALU}
    del rho
    if not args.no_second_variant:
        other = 1 - args.variant
        ms2, _, per2, st2 = run_variant(other, max(1, args.steps // 2), 1)
        ok2 = (st2 & (ffbie.PAIR_SINGULAR | ffbie.PAIR_UNRESOLVED)) == 0
        p2 = float(((st2 >> ffbie.P_SHIFT) & 0xFFF)[ok2].mean())
        main2 = float(per2[:, 1].mean())
        w2 = own_flops_per_pair("paper" if other == 1 else "swap", NF, M, M0, p2)
        result["value_other_variant"] = {
            "kappa_variant": "eq. (3.10)" if other == 1 else "swap of cos(k rho)/rho",
            "value": n * 2 * M * max(1, args.steps // 2) / (ms2 * 1e-3),
            "coeff_main_ms": main2, "p_mean": p2, "flops_per_pair": w2,
            "frac": w2 * n / (main2 * 1e-3) / PEAK_FP64_VALU}
    if not args.no_mixed:
        # the same launch with the FP32 spectral stage (complex64 table)
        kappa_mixed = torch.empty((n, 2 * M), dtype=torch.complex64, device=dev)
        msx, _, perx, stx = run_variant(0, args.steps, args.warmup, mixed=True)
        okx = (stx & (ffbie.PAIR_SINGULAR | ffbie.PAIR_UNRESOLVED)) == 0
        p_mean_x = float(((stx >> ffbie.P_SHIFT) & 0xFFF)[okx].mean())
        main_x = float(perx[:, 1].mean())
        w_x = own_flops_per_pair("swap", NF, M, M0, p_mean_x)
        ach_x = w_x * n / (main_x * 1e-3)
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
                         "flops_per_pair": w_x, "flops_counted": "own work of this launch: swap",
                         "traffic": measured_traffic("mixed"),
                         "kernel": COEFF_KERNEL + " (main pass, FP32 spectral stage)"}}
        del kappa_mixed
    log("variants and mixed path done")
    if not args.no_double_layer:
        result["double_layer"] = double_layer_block(ctx, cfg, torch, np, ffbie, tt, jj, tss, kappa,
                                                    solve=not args.no_solve)
        log("double-layer block done")
    if not args.no_banded:
        result["banded_rhoinv"] = banded_block(ctx, cfg, torch, np, ffbie, tt, jj, tss, kappa)
        log("banded block done")
    del kappa, tt, jj, tss, status
    torch.cuda.empty_cache()
    if not args.no_solve:
        result["time_to_1e-8_field_error"] = time_to_field_error(ctx, cfg, torch, np, ffbie)
        result["near_set"] = near_set_rate(ctx, cfg, torch)
        log("config-2 solves done")
        result["interior_protocol"] = interior_protocol(ctx, torch, np, ffbie)
        log("interior protocol done")
        if args.convergence:
            result["ellipsoid_convergence"] = ellipsoid_convergence(ctx, torch, np, ffbie)
            log("convergence study done")
    if not args.no_config3:
        result["config3"] = config3_block(ctx, torch, np, ffbie, solve=not args.no_solve)
        log("config-3 block done")
    if not args.no_batch:
        result["batch_64_surfaces"] = batch_rate(ctx, torch)
        log("batch done")
    if not args.no_ceilings:
        result["hbm_ceilings"] = hbm_ceilings(torch)
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(cfg, args.cpu_sample, args.cpu_sample_single)
        log("cpu baseline done")
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
