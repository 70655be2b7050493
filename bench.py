#!/usr/bin/env python3
"""Throughput benchmark of GAP-TV video SCI reconstruction on one MI355X.

One step = one whole reconstruction of a synthetic CACTI-style measurement
(1024 x 1024 pixels, B = 24 frames, shifted Bernoulli(0.5) masks, moving
shapes on a gradient background plus N(0, 0.02) texture): GAP with isotropic
(ITV2D) TV, 200 outer x 10 FGP inner iterations, lambda = 0.1, float32, plus
the FP64 PSNR and residual reductions on the result. Inputs are resident in
HBM before the timed region starts.

Prints ONE JSON line: the throughput in voxel-iterations per second
(voxels x inner iterations / s, timed without per-kernel events), the roofline
position of the dominant kernel (its launches timed with HIP events inside the
library over an identical repeat of the timed steps), the HBM traffic
measured by rocprofv3 counters when the committed counter summary still
matches the kernel source and tile choice, the FP64 oracle timed on the host
cores on a bounded sample of the same workload, and the side measurements:
time-to-PSNR of the batched solve against per-measurement solves, and the
16-bit dual storage variants with their error.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GAP-TV voxel-iter/s, % HBM roofline; time-to-PSNR learned/batched vs plain"
HBM_PEAK_GBS = 8000.0
# FP32 VALU lane-operations per second with packed FP32 disabled:
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz.
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
PROFILE_DIR = os.path.join(ROOT, "profiles")

# FP32 VALU operations per voxel of one FGP inner iteration, counted from the
# algorithm (Algorithm 1, FGP box): theta = x - lambda D^T w (2 sub, 1 add,
# 1 fma), z = D theta (2 sub), q = w + z/(8 lambda) (2 fma), projection
# (ATV: 2 clamps; ITV2D: squared norm 2, 1/sqrt and min 2, 2 mul), momentum
# w = p + beta (p - p_prev) (2 sub, 2 fma).
OPS_PER_VOXEL_ITER = {"atv": 14, "itv2d": 18}
OPS_THETA_EPILOGUE = 4  # theta = x - lambda D^T p once per voxel at the end of the pass


def fgp_stream_bytes_per_voxel(n_inner: int, elem: int) -> float:
    """Algorithmic HBM bytes per voxel summed over the n_inner streaming FGP
    passes of one denoiser call: every pass reads x (4 B) and writes p^(s+1)
    (2 elem); pass s >= 1 also reads p^(s) (2 elem); pass s >= 2 also reads
    p^(s-1) (2 elem) for the momentum term (the first momentum coefficient is
    zero)."""
    total = 0.0
    for s in range(n_inner):
        b = 4 + 2 * elem
        if s >= 1:
            b += 2 * elem
        if s >= 2:
            b += 2 * elem
        total += b
    return total


def source_hash(files) -> str:
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, "paper_2005_08028_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


KERNEL_SOURCES = {
    "fgp_stream": ("k_fgp.hip", "sci_math.h"),
    "fgp_fused": ("k_fgp_tile.h", "k_fgp_rows.h", "k_fgp_tile_shapes.h", "sci_math.h"),
}


def read_traffic(family: str, tag: str):
    """HBM bytes per launch of the chosen tiling from the committed rocprofv3
    counter summary (FETCH_SIZE and WRITE_SIZE scaled by a plain copy of known
    size; one entry per tiling), or None when it is missing, has no entry for
    this tiling, or was taken on another kernel source."""
    path = os.path.join(PROFILE_DIR, f"hbm_traffic_{family}_cacti_1024x24.txt")
    if not os.path.exists(path):
        return None
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha256") != source_hash(KERNEL_SOURCES[family]):
        return None
    try:
        return float(kv[f"hbm_bytes_per_launch[{tag}]"])
    except (KeyError, ValueError):
        return None


def passes_of(tag: str) -> int:
    # tag = "shape<k>/passes<p>"
    try:
        return int(tag.split("passes")[1])
    except (IndexError, ValueError):
        return 1


def roofline_for(family, n_launch, ms_total, V, N, tv, elem, tag):
    avg_s = ms_total / n_launch / 1e3
    out = {"kernel": family, "avg_launch_us": round(avg_s * 1e6, 2), "launches": n_launch}
    if family == "fgp_stream":
        b = V * fgp_stream_bytes_per_voxel(N, elem) / N
        out.update({"bound": "hbm", "achieved": round(b / avg_s / 1e9, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                    "frac": round(b / avg_s / 1e9 / HBM_PEAK_GBS, 4), "bytes_per_launch": b})
    elif family == "fgp_fused":
        m = N / passes_of(tag)  # inner iterations per launch
        ops = V * (m * OPS_PER_VOXEL_ITER[tv] + OPS_THETA_EPILOGUE / passes_of(tag))
        a = ops / avg_s / 1e12
        out.update({"bound": "alu", "achieved": round(a, 2), "peak": round(VALU_PEAK_TOPS, 2),
                    "unit": "TOP/s (fp32 VALU lane-ops)", "frac": round(a / VALU_PEAK_TOPS, 4),
                    "ops_per_launch": ops})
        if passes_of(tag) == 1:  # one pass: reads x, writes theta
            out["hbm_GBs_algorithmic"] = round(V * 8.0 / avg_s / 1e9, 1)
    out["traffic"] = read_traffic(family, tag) if family in KERNEL_SOURCES else None
    return out


def measure_batched_vtv(scitv, synth, h, dev, reps=3):
    """Batched GAP-VTV (one row-pipelined VTV pass per problem and outer
    iteration inside one graph launch) over 16 measurements of 256^2 and
    512^2 with 8 or 10 frames, against the same measurements solved one by
    one (no graph); both give the same bits."""
    import torch
    lam, T, N = 0.1, 20, 5
    items = []
    for k in range(16):
        n, B = (256, 8) if k % 2 == 0 else (512, 10)
        pr = synth.make_problem(n, n, B, seed=4100 + k, sigma=0.01)
        C = torch.from_numpy(pr.masks).to(dev)
        Y = scitv.sci_forward(h, C, torch.from_numpy(pr.truth).to(dev)) + torch.from_numpy(pr.noise).to(dev)
        items.append(dict(Y=Y, C=C, X_out=torch.empty_like(C), Theta_out=torch.empty_like(C), outer_iters=T))
    voxels = sum(it["C"].numel() for it in items)
    prm = scitv.solver_params(outer_iters=T, tv="vtv", lam=lam, n_inner=N, use_graph=True)
    one = scitv.solver_params(outer_iters=T, tv="vtv", lam=lam, n_inner=N)

    def batched():
        scitv.sci_gap_tv_batched(h, items, prm)

    def plain():
        for it in items:
            scitv.sci_gap_tv(h, it["Y"], it["C"], one, X_out=it["X_out"], Theta_out=it["Theta_out"])

    out = {}
    for name, fn in (("plain_ms", plain), ("batched_ms", batched)):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        out[name] = round((time.perf_counter() - t0) / reps * 1e3, 3)
    return {"workload": "16 measurements, 256x256x8 and 512x512x10 alternating, GAP-VTV lambda=0.1, 20 outer x 5 inner",
            "voxels": voxels, **out, "speedup_batched_vs_plain": round(out["plain_ms"] / out["batched_ms"], 3)}


def measure_batched(scitv, synth, h, dev, steps):
    """Batched solve of 64 measurements of mixed sizes against the same
    measurements solved one by one (default tiles, no graph), both run to
    each measurement's time-to-PSNR iteration count."""
    import torch
    specs = synth.batched_specs(64, seed=4000)
    lam, T, N = 0.1, 50, 5
    items = []
    truths = []
    t0 = time.perf_counter()
    for sp in specs:
        pr = synth.make_problem(sp["nx"], sp["ny"], sp["B"], sp["seed"], mask=sp["mask"], mask_p=sp["mask_p"],
                                sigma=sp["sigma"])
        C = torch.from_numpy(pr.masks).to(dev)
        Xt = torch.from_numpy(pr.truth).to(dev)
        Y = scitv.sci_forward(h, C, Xt) + torch.from_numpy(pr.noise).to(dev)
        items.append(dict(Y=Y, C=C, X_out=torch.empty_like(C), Theta_out=torch.empty_like(C), outer_iters=T))
        truths.append(Xt)
    gen_s = time.perf_counter() - t0
    voxels = sum(it["C"].numel() for it in items)
    # reference PSNR at the full iteration count (batched == per-problem bit for bit)
    prm = scitv.solver_params(outer_iters=T, tv="atv", lam=lam, n_inner=N, use_graph=False)
    scitv.sci_gap_tv_batched(h, items, prm)
    full = [scitv.sci_psnr(h, it["X_out"], xt) for it, xt in zip(items, truths)]
    # time-to-PSNR: first outer iteration reaching (full PSNR - 0.1 dB)
    one = scitv.solver_params(outer_iters=1, tv="atv", lam=lam, n_inner=N)
    tstar = []
    for it, xt, pf in zip(items, truths, full):
        th = scitv.sci_adjoint(h, it["C"], it["Y"])
        x = torch.empty_like(th)
        th2 = torch.empty_like(th)
        ts = T
        for t in range(1, T + 1):
            scitv.sci_gap_tv(h, it["Y"], it["C"], one, X_out=x, Theta_out=th2, X_init=th)
            th, th2 = th2, th
            if scitv.sci_psnr(h, x, xt) >= pf - 0.1:
                ts = t
                break
        tstar.append(ts)
    for it, ts in zip(items, tstar):
        it["outer_iters"] = ts
    # plain: one sci_gap_tv per measurement, default tiles, no graph
    plain = [scitv.solver_params(outer_iters=ts, tv="atv", lam=lam, n_inner=N, tile_shape=1) for ts in tstar]

    def run_plain():
        for it, pp in zip(items, plain):
            scitv.sci_gap_tv(h, it["Y"], it["C"], pp, X_out=it["X_out"], Theta_out=it["Theta_out"])

    bprm = scitv.solver_params(outer_iters=T, tv="atv", lam=lam, n_inner=N, use_graph=True)
    best, times = scitv.sci_autotune_batched(h, items, bprm)

    def run_batched():
        scitv.sci_gap_tv_batched(h, items, bprm)

    res = {}
    for name, fn in (("plain", run_plain), ("batched", run_batched)):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        res[name] = (time.perf_counter() - t0) / steps * 1e3
    got = [scitv.sci_psnr(h, it["X_out"], xt) for it, xt in zip(items, truths)]
    ok = all(g >= f - 0.1 - 1e-9 for g, f in zip(got, full))
    return {
        "workload": "64 measurements, nx=ny in {256,512,1024}, B in {8,10,16}, Bernoulli(p in [0.3,0.7]) masks, "
                    "sigma in [0,0.02]; GAP-ATV lambda=0.1, 5 FGP inner, each run to its time-to-PSNR iteration "
                    "(full-50-iteration PSNR - 0.1 dB)",
        "voxels": voxels, "t_star_mean": sum(tstar) / len(tstar), "t_star_min": min(tstar), "t_star_max": max(tstar),
        "plain_ms": round(res["plain"], 3), "batched_ms": round(res["batched"], 3),
        "speedup_batched_vs_plain": round(res["plain"] / res["batched"], 3),
        "target_speedup": 2.0, "target_met": res["plain"] / res["batched"] >= 2.0,
        "batched_tile_shape": best, "batched_shape_ms": [round(t, 4) for t in times],
        "all_reach_target_psnr": ok, "input_generation_s": round(gen_s, 1),
    }


def say(msg):
    """Progress line on stderr (the JSON line alone goes to stdout)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def measure_learned(scitv, synth, h, dev, Y, C, X_true, lam, n_crops=20000, n_held=800, epochs=2, T_eval=200,
                    every_counts=1, every_timed=5, cap=500):
    """Learned warm start, trained and evaluated as the workload specifies:
    training pairs are 128x128x16 crops (all 16 frames) of full-frame FGP
    solves at relative duality gap <= 1e-6 on 512x512x16 GAP-ITV2D runs
    (shifted Bernoulli(0.5) masks, textured scenes, seeds 5000 + i; each
    outer iteration of a run gives 16 crops), plus held-out crops from
    scenes the training never sees (seeds 5900 + i). Two networks: the
    specified one (input x^(t), output the dual) and the correcting one
    (input x^(t) and the previous outer iteration's final dual, output added
    to that dual). Evaluation on the 1024x1024x24 measurement: GAP-ITV2D
    whose inner FGP runs until relative gap <= 1e-4 (cap `cap`), T_eval
    outer iterations, inner iterations counted with a gap check every
    `every_counts` iterations; time-to-PSNR (first outer iteration whose
    PSNR reaches the cold start's final PSNR - 0.1 dB, and the time of a run
    of that many outer iterations, gap checks every `every_timed`) for cold,
    warm-dual and learned starts, next to plain GAP-TV with 10 fixed inner
    iterations."""
    import numpy as np
    import torch
    from paper_2005_08028_amd import warmstart
    tv, crop, outer_train = "itv2d", 128, 25
    t0 = time.perf_counter()
    train = warmstart.CropSet(n_crops, 16, crop, dev)
    held = warmstart.CropSet(n_held, 16, crop, dev)
    seed = 5000
    for cs, first in ((train, 5000), (held, 5900)):
        seed = first
        while cs.n < cs.X.shape[0]:
            pr = synth.make_problem(512, 512, 16, seed, mask="shifted", texture_sigma=0.02)
            Ct = torch.from_numpy(pr.masks).to(dev)
            Yt = scitv.sci_forward(h, Ct, torch.from_numpy(pr.truth).to(dev))
            warmstart.fill_crop_set(h, cs, Yt, Ct, tv, lam, outer_train, tol=1e-4, target_tol=1e-6)
            seed += 1
        say(f"learned: {cs.n} crops from seeds {first}..{seed - 1}")
    torch.cuda.synchronize()
    gen_s = time.perf_counter() - t0
    nets, curves, train_ms = {}, {}, {}
    for name, c_in, last, lr in (("x_only", 1, 0.1, 1e-4), ("correcting", 3, 0.0, 3e-5)):
        net = scitv.sci_wsnet_create(h, c_in=c_in, c_out=2)
        scitv.sci_wsnet_set_params(h, net, warmstart.init_params(0, c_in=c_in, last_scale=last))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        hist = warmstart.train_epochs(h, net, train, c_in == 3, epochs, lr, held=held, n_held=256,
                                      log_every=max(1, train.n // 4), progress=lambda m: say(f"learned {name}: {m}"))
        torch.cuda.synchronize()
        train_ms[name] = round((time.perf_counter() - t1) / (epochs * train.n) * 1e3, 3)
        nets[name] = net
        curves[name] = [(st, None if tl is None else round(tl, 6), None if hl is None else round(hl, 6))
                        for st, tl, hl in hist]
    del train, held
    torch.cuda.empty_cache()
    # network throughput at the evaluation size
    x0 = scitv.sci_adjoint(h, C, Y)
    base = torch.zeros((2,) + tuple(x0.shape), device=dev)
    net = nets["correcting"]
    scitv.sci_wsnet_forward(h, net, x0, tv=tv, base=base)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(5):
        scitv.sci_wsnet_forward(h, net, x0, tv=tv, base=base)
    torch.cuda.synchronize()
    fwd_ms = (time.perf_counter() - t1) / 5 * 1e3
    V = x0.numel()
    macs = 27 * (3 * 16 + 16 * 16 + 16 * 16 + 16 * 2)  # per voxel, the four layers
    variants = {"cold": (None, 0), "warm_dual": (None, 1), "learned_x_only": ("x_only", 0),
                "learned_correcting": ("correcting", 0), "learned_correcting_gap_checked": ("correcting", 1)}

    def run(name, T, every):
        netname, warm = variants[name]
        prm = scitv.solver_params(outer_iters=T, tv=tv, lam=lam, gap_tol=1e-4, n_inner_max=cap,
                                  gap_check_every=every, warm_dual=bool(warm))
        kw = {"net": nets[netname]} if netname else {}
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        x, its, fb, ns = scitv.sci_gap_tv_adaptive(h, Y, C, prm, **kw)
        torch.cuda.synchronize()
        return x, its, fb, ns, (time.perf_counter() - t1) * 1e3

    res = {}
    for name in variants:
        x, its, fb, ns, ms = run(name, T_eval, every_counts)
        res[name] = {"inner_iters": its, "fallbacks": fb, "net_starts": ns, "ms_counting_run": round(ms, 1),
                     "psnr_db": round(scitv.sci_psnr(h, x, X_true), 4)}
        say(f"learned: {name}: {its} inner iterations over {T_eval} outer, PSNR {res[name]['psnr_db']}")
    fixed = lambda T: scitv.solver_params(outer_iters=T, tv=tv, lam=lam, n_inner=10)
    x, _ = scitv.sci_gap_tv(h, Y, C, fixed(T_eval))
    p_plain = scitv.sci_psnr(h, x, X_true)
    # two targets: the cold start's final PSNR and plain GAP-TV's, each - 0.1 dB
    targets = {"cold_final": res["cold"]["psnr_db"] - 0.1, "plain_final": p_plain - 0.1}
    target = targets["cold_final"]

    def first_reaching(psnr_at, label="", hint=8):
        """First outer iteration t <= T_eval whose PSNR reaches the target
        (None if none does): bracket around `hint` by doubling steps, then
        bisect (the PSNR rises with t on these runs)."""
        cache = {}

        def ok(tt):
            if tt not in cache:
                cache[tt] = psnr_at(tt)
                say(f"learned: {label} PSNR after {tt} outer iterations {cache[tt]:.4f} (target {target:.4f})")
            return cache[tt] >= target

        hint = max(1, min(T_eval, hint))
        step = 1
        if ok(hint):
            hi, lo = hint, hint - 1
            while lo >= 1 and ok(lo):
                hi, step = lo, step * 2
                lo = max(0, hi - step)
        else:
            lo, hi = hint, min(T_eval, hint + 1)
            while not ok(hi):
                if hi == T_eval:
                    return None
                lo, step = hi, step * 2
                hi = min(T_eval, lo + step)
        while hi - lo > 1:  # ok(hi) holds; lo == 0 or not ok(lo)
            mid = (lo + hi) // 2
            if ok(mid):
                hi = mid
            else:
                lo = mid
        return hi

    def plain_ms(T):
        scitv.sci_gap_tv(h, Y, C, fixed(T))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        scitv.sci_gap_tv(h, Y, C, fixed(T))
        torch.cuda.synchronize()
        return (time.perf_counter() - t1) * 1e3

    res["plain_fixed_10"] = {"inner_iters": 10 * T_eval, "psnr_db": round(p_plain, 4)}
    for tname, tval in targets.items():
        target = tval
        hint = 8
        # the warm-dual start first (the cheapest); its t* is the others' starting guess
        for name in ["warm_dual"] + [v for v in variants if v != "warm_dual"]:
            ts = first_reaching(lambda t: scitv.sci_psnr(h, run(name, t, every_timed)[0], X_true), name, hint)
            res[name][f"t_star_{tname}"] = ts
            if ts:
                hint = ts if name == "warm_dual" else hint
                run(name, ts, every_timed)
                res[name][f"ms_to_{tname}"] = round(run(name, ts, every_timed)[4], 1)
        ts = first_reaching(lambda t: scitv.sci_psnr(h, scitv.sci_gap_tv(h, Y, C, fixed(t))[0], X_true), "plain",
                            hint)
        res["plain_fixed_10"][f"t_star_{tname}"] = ts
        if ts:
            res["plain_fixed_10"][f"ms_to_{tname}"] = round(plain_ms(ts), 1)
        say(f"learned: time to {tname} target {tval:.4f} dB: " +
            ", ".join(f"{k} {v.get('ms_to_' + tname)} ms" for k, v in res.items()))
    for n in nets.values():
        scitv.sci_wsnet_destroy(n)

    def ratio(a, b, tname="cold_final"):
        ka = f"ms_to_{tname}"
        return None if not res[a].get(ka) or not res[b].get(ka) else round(res[a][ka] / res[b][ka], 3)
    return {
        "workload": f"train: {n_crops} crops 128x128x16 of full-frame 512x512x16 GAP-ITV2D FGP solves at relative gap "
                    f"<= 1e-6 ({outer_train} outer iterations per scene), {epochs} epochs, {n_held} held-out crops; "
                    f"eval: the 1024x1024x24 measurement, {T_eval} outer GAP-ITV2D, inner FGP to relative gap <= 1e-4 "
                    f"(cap {cap}; checked every {every_counts} for the counts, every {every_timed} for the timed "
                    f"runs); time-to-PSNR targets: the cold start's final PSNR - 0.1 dB = "
                    f"{targets['cold_final']:.4f} dB, plain GAP-TV's (10 fixed inner) final PSNR - 0.1 dB = "
                    f"{targets['plain_final']:.4f} dB",
        "data_generation_s": round(gen_s, 1), "train_ms_per_step_128x128x16": train_ms,
        "loss_curves_step_train_heldout": curves,
        "forward_ms_1024x1024x24": round(fwd_ms, 3),
        "forward_tflops_algorithmic": round(2 * macs * V / (fwd_ms / 1e3) / 1e12, 2),
        "time_to_target_cold_over_learned_correcting": ratio("cold", "learned_correcting_gap_checked"),
        "time_to_target_warm_over_learned_correcting": ratio("warm_dual", "learned_correcting_gap_checked"),
        "time_to_plain_target_plain_over_learned_correcting": ratio("plain_fixed_10",
                                                                    "learned_correcting_gap_checked",
                                                                    "plain_final"),
        "target_speedup_vs_plain": 2.0,
        **res,
    }


def measure_net(scitv, h, dev, C, Y, reps):
    """Throughput of the warm-start network's MFMA kernels: the forward pass of
    the correcting network (3 input channels) at 1024x1024x24 and training
    steps (forward, loss, data and weight gradients, Adam) at 512x512x16,
    against the algorithmic FLOPs of the four 3x3x3 layers
    (2 * 27 * (3*16 + 16*16 + 16*16 + 16*2) per voxel forward; about 3x that
    per training step)."""
    import numpy as np
    import torch
    from paper_2005_08028_amd import warmstart
    net = scitv.sci_wsnet_create(h, c_in=3, c_out=2)
    scitv.sci_wsnet_set_params(h, net, warmstart.init_params(0, c_in=3, last_scale=0.1))
    x0 = scitv.sci_adjoint(h, C, Y)
    base = torch.zeros((2,) + tuple(x0.shape), device=dev)
    flop_fwd = 2 * 27 * (3 * 16 + 16 * 16 + 16 * 16 + 16 * 2)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps * 1e3

    fwd_ms = timed(lambda: scitv.sci_wsnet_forward(h, net, x0, tv="itv2d", base=base))
    r = np.random.default_rng(0)
    xs = torch.from_numpy(r.uniform(size=(16, 512, 512)).astype(np.float32)).to(dev)
    bs = torch.from_numpy(r.uniform(-1, 1, size=(2, 16, 512, 512)).astype(np.float32)).to(dev)
    ts = torch.from_numpy(r.uniform(-1, 1, size=(2, 16, 512, 512)).astype(np.float32)).to(dev)
    step_ms = timed(lambda: scitv.sci_wsnet_train_step(h, net, xs, ts, 1e-5, base=bs, want_loss=False))
    scitv.sci_wsnet_destroy(net)
    V, Vt = x0.numel(), xs.numel()
    return {"forward_ms_1024x1024x24": round(fwd_ms, 3),
            "forward_tflops_algorithmic": round(flop_fwd * V / (fwd_ms / 1e3) / 1e12, 2),
            "train_step_ms_512x512x16": round(step_ms, 3),
            "train_step_tflops_algorithmic": round(3 * flop_fwd * Vt / (step_ms / 1e3) / 1e12, 2),
            "bf16_mfma_peak_tflops": 2500.0}


def measure_paper_shaped(scitv, synth, h, dev, T=150, N=5, lam=0.1, every=10, curves_on=True):
    """The paper's real-data shape (512x512, B=10, ITV3D-FGP, 150 iterations)
    on a synthetic scene: time of one GAP-VTV solve, and PSNR against the
    iteration count for GAP, ADMM, FISTA and TwIST (each run afresh to every
    checkpoint, so momentum and ADMM multipliers are never reset)."""
    import torch
    pr = synth.make_problem(512, 512, 10, 4001, mask="bernoulli", sigma=0.0, texture_sigma=0.02)
    C = torch.from_numpy(pr.masks).to(dev)
    Xt = torch.from_numpy(pr.truth).to(dev)
    Y = scitv.sci_forward(h, C, Xt)
    V = C.numel()
    X = torch.empty_like(C)

    def solve_ms(schedule, reps=3):
        prm = scitv.solver_params(outer_iters=T, tv="vtv", lam=lam, n_inner=N, schedule=schedule)
        scitv.sci_gap_tv(h, Y, C, prm, X_out=X)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            scitv.sci_gap_tv(h, Y, C, prm, X_out=X)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps * 1e3

    ms_stream = solve_ms("stream")
    ms = solve_ms("auto")  # the fused (row-pipelined) VTV denoiser
    fns = {"gap": scitv.sci_gap_tv, "admm": scitv.sci_admm_tv, "fista": scitv.sci_fista_tv,
           "twist": scitv.sci_twist_tv}
    per_framework = {}
    for name, fn in fns.items():  # one full T x N solve per outer framework, default schedule
        q = scitv.solver_params(outer_iters=T, tv="vtv", lam=lam, n_inner=N, rho=0.01)
        fn(h, Y, C, q, X_out=X)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(2):
            fn(h, Y, C, q, X_out=X)
        torch.cuda.synchronize()
        per_framework[name] = round((time.perf_counter() - t0) / 2 * 1e3, 2)
    curves = {}
    for name, fn in (fns.items() if curves_on else ()):
        pts = []
        for t in range(every, T + 1, every):
            # one lambda for all four (FISTA / TwIST scale it by 1/L inside their denoiser)
            q = scitv.solver_params(outer_iters=t, tv="vtv", lam=lam, n_inner=N, rho=0.01)
            x, _ = fn(h, Y, C, q)
            pts.append((t, round(scitv.sci_psnr(h, x, Xt), 3)))
        curves[name] = pts
    return {
        "workload": f"512x512x10 synthetic scene (Bernoulli(0.5) masks, texture 0.02), ITV3D (VTV) FGP, "
                    f"{T} outer x {N} inner, lambda={lam}",
        "gap_vtv_ms_per_solve": round(ms, 2), "voxel_iter_per_s": V * T * N / (ms / 1e3),
        "gap_vtv_ms_per_solve_streaming_schedule": round(ms_stream, 2),
        "ms_per_solve_by_framework": per_framework,
        "paper_context": "the paper reports about 3 minutes for 150 iterations at this shape on a laptop CPU",
        "psnr_vs_outer_iterations": curves,
    }


def measure_kernels(scitv, h, dev, C, Y, X_true):
    """Every step of the path timed on the 1024x1024x24 volume, against its
    algorithmic HBM bytes (HBM-bound kernels; the fused denoiser is reported
    in `roofline`). Single-kernel entry points are timed with events around
    the call; denoiser passes through the library's per-kernel profiler."""
    import torch
    V, npix = C.numel(), Y.numel()
    out = []

    def row(step, us, nbytes, note=""):
        gbs = nbytes / (us * 1e-6) / 1e9
        out.append({"step": step, "us_per_call": round(us, 2), "algorithmic_MB": round(nbytes / 1e6, 1),
                    "GBs": round(gbs, 1), "frac_of_8TBs": round(gbs / 8000.0, 3), **({"note": note} if note else {})})

    def timed(fn, reps=10):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e3

    Yo, Xo = torch.empty_like(Y), torch.empty_like(C)
    row("a2 forward (sci_forward)", timed(lambda: scitv.sci_forward(h, C, X_true, Y=Yo)), 8 * V + 4 * npix)
    row("a3 adjoint (sci_adjoint)", timed(lambda: scitv.sci_adjoint(h, C, Y, X=Xo)), 8 * V + 4 * npix)
    row("a8 PSNR reduction (sci_psnr)", timed(lambda: scitv.sci_psnr(h, Xo, X_true)), 8 * V, "includes the read-back")
    row("a8 residual reduction (sci_residual_sq)", timed(lambda: scitv.sci_residual_sq(h, C, Xo, Y)),
        8 * V + 4 * npix, "includes the read-back")
    p0 = torch.zeros((2,) + tuple(C.shape), device=dev)
    row("a8 duality-gap reduction (sci_dual_gap)", timed(lambda: scitv.sci_dual_gap(h, Xo, p0, "itv2d", 0.1)),
        12 * V, "includes the read-back")

    def profiled(fn, fams):
        fn()
        torch.cuda.synchronize()
        scitv.sci_profile_enable(h, True)
        fn()
        torch.cuda.synchronize()
        scitv.sci_profile_enable(h, False)
        res = {}
        for f in fams:
            n, ms = scitv.sci_profile_read(h, f)
            res[f] = (n, ms)
        return res

    N = 10
    per_pass_fgp = (12 + 20 + (N - 2) * 28) / N  # B/voxel: pass 1 reads x, pass 2 adds p, then p and p_prev
    per_pass_pg = (12 + (N - 1) * 20) / N        # no momentum: x and p
    # fused VTV at B = 24: two row-pipelined passes of 5 per call; the first reads x and
    # writes p and p_prev (20 B/voxel), the second reads x, p, p_prev and writes theta (24 B)
    per_pass_vtv_fused = (20 + 24) / 2
    cases = [
        ("a6 FGP pass, ITV2D, streaming schedule (tile kernel, 1 iteration)",
         dict(tv="itv2d", schedule="stream"), per_pass_fgp, "fgp_stream", ""),
        ("a6 FGP pass, VTV, streaming schedule (row-streaming kernel, all frames of a pixel)",
         dict(tv="vtv", schedule="stream"), per_pass_fgp, "fgp_stream", ""),
        ("a6 FGP pass, VTV, fused schedule (row-pipelined kernel, 5 iterations per pass)", dict(tv="vtv"),
         per_pass_vtv_fused, "fgp_fused", "bound by arithmetic and the per-iteration norm exchange, not HBM"),
        ("f1 Chambolle-2004 pass, ITV2D, projected gradient, streaming schedule",
         dict(tv="itv2d", chambolle04=True, accel=False, schedule="stream"), per_pass_pg, "fgp_stream", ""),
        ("f1 Chambolle-2004, ITV2D, fused schedule (row-pipelined kernel, 10 iterations per pass)",
         dict(tv="itv2d", chambolle04=True, accel=False), 8.0, "fgp_fused", "bound by arithmetic, not HBM"),
        ("f3 ATV-Clip pass, streaming schedule", dict(tv="atv", clip=True, schedule="stream"), per_pass_pg,
         "fgp_stream", ""),
        ("f3 ATV-Clip, fused schedule (row-pipelined kernel, 10 iterations per pass)", dict(tv="atv", clip=True),
         8.0, "fgp_fused", "bound by arithmetic, not HBM"),
    ]
    for name, kw, bpv, fam, note in cases:
        prm = scitv.solver_params(outer_iters=2, lam=0.1, n_inner=N, **kw)
        r = profiled(lambda: scitv.sci_gap_tv(h, Y, C, prm), (fam, "tv_theta", "project"))
        n, ms = r[fam]
        if n == 0:
            raise RuntimeError(f"kernel table: no {fam} launches recorded for {name}")
        row(name, ms * 1e3 / n, bpv * V, note)
        if r["tv_theta"][0]:
            n, ms = r["tv_theta"]
            row("a7 theta = x - lambda D^T p (" + kw["tv"] + ")", ms * 1e3 / n, 16 * V)
        n, ms = r["project"]
        # binary masks travel as one 32-bit word of frame bits per pixel
        row("a4 GAP projection (packed binary masks)", ms * 1e3 / n, 8 * V + 12 * npix)
    T = 4
    prm = scitv.solver_params(outer_iters=T, lam=0.1, rho=0.01, n_inner=N, tv="itv2d")
    r = profiled(lambda: scitv.sci_admm_tv(h, Y, C, prm), ("project",))
    n, ms = r["project"]
    # reads theta, u and writes s = u + x each pass; x itself only on the last
    row("a5 ADMM x-update (+ denoiser input, packed binary masks)", ms * 1e3 / n, (12 + 4 / T) * V + 12 * npix)
    return out


def cpu_model() -> str:
    try:
        import subprocess
        for line in subprocess.run(["lscpu"], capture_output=True, text=True, timeout=10).stdout.splitlines():
            if line.lower().startswith("model name"):
                return line.split(":", 1)[1].strip()
    except Exception:
        pass
    return "unknown"


def cpu_baseline(scitv, h, dev, pr, C, nx, ny, B, N, T, lam, tv, args):
    """The FP64 oracle on the host cores, on a bounded sample of the workload
    (the first outer iterations of the same solve): at all cores and at one
    thread (a shorter sample). The sample's measurement is formed by the
    oracle in FP64 (rounded once to float32) and both sides consume it; the
    GPU's error against the oracle on that sample is reported for float32,
    bfloat16 and float16 dual storage."""
    import numpy as np
    import torch
    from oracle import oracle as orc
    V = nx * ny * B
    lam32 = float(np.float32(lam))
    Yo = orc.measurement(pr.masks, pr.truth, pr.noise)
    Yd = torch.from_numpy(Yo).to(dev)
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count()
    cores = min(cores, int(os.environ.get("OMP_NUM_THREADS", cores)))
    runs = {}
    for threads, Ts in ((cores, args.cpu_outer), (1, 1)):
        used = orc.set_threads(threads)
        t0 = time.perf_counter()
        xr, _ = orc.gap_tv(Yo, pr.masks, lam32, Ts, N, tv=tv)
        tc = time.perf_counter() - t0
        runs[threads] = {"value": V * Ts * N / tc, "outer": Ts, "seconds": round(tc, 1), "x": xr, "used": used}
    orc.set_threads(cores)
    xr = runs[cores]["x"]
    err = {}
    for dt, sched in (("f32", args.schedule), ("bf16", "stream"), ("f16", "stream")):
        prs = scitv.solver_params(outer_iters=args.cpu_outer, tv=tv, lam=lam, n_inner=N, schedule=sched,
                                  dual_dtype=dt)
        xs, _ = scitv.sci_gap_tv(h, Yd, C, prs)
        xg = xs.cpu().numpy().astype(np.float64)
        err[dt] = {"rel_l2": float(np.linalg.norm(xg - xr) / np.linalg.norm(xr)),
                   "max_abs": float(np.abs(xg - xr).max()),
                   "dpsnr_db": round(orc.psnr(xg, pr.truth) - orc.psnr(xr, pr.truth), 6)}
    one = runs[1]
    return {
        "value": runs[cores]["value"], "unit": "voxel-iter/s", "cores": runs[cores]["used"], "kind": "oracle",
        "sample": f"same {nx}x{ny}x{B} inputs, GAP-{tv.upper()} {args.cpu_outer} outer x {N} inner (of {T}), "
                  f"FP64, {runs[cores]['seconds']} s on {cores} threads",
        "cpu_model": cpu_model(),
        "one_thread": {"value": one["value"], "unit": "voxel-iter/s", "cores": one["used"],
                       "sample": f"GAP-{tv.upper()} {one['outer']} outer x {N} inner, {one['seconds']} s"},
        "gpu_error_vs_oracle_on_sample": err,
    }


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--outer", type=int, default=200, help="outer iterations per step (default: the full 200)")
    ap.add_argument("--schedule", default="auto", choices=["auto", "stream", "fused"])
    ap.add_argument("--dual-dtype", default="f32", choices=["f32", "bf16", "f16"])
    ap.add_argument("--no-autotune", action="store_true", help="skip the tile autotuner (default shape and passes)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-outer", type=int, default=3, help="outer iterations of the oracle sample")
    ap.add_argument("--no-extras", action="store_true", help="skip the batched and 16-bit side measurements")
    ap.add_argument("--kernel-table-only", action="store_true",
                    help="only time every step of the path on the 1024x1024x24 measurement and print that table "
                         "(a short run to profile all kernels; not the benchmark line)")
    ap.add_argument("--paper-shaped-only", action="store_true",
                    help="only time the 512x512x10 GAP-VTV solve on both schedules (a short run to profile the "
                         "VTV kernels; not the benchmark line)")
    ap.add_argument("--denoise-only", default=None,
                    choices=["atv", "itv2d", "vtv", "atv-ch", "itv2d-ch", "vtv-ch", "atv-clip"],
                    help="only run cold 10-iteration denoiser calls (default schedule) on the 1024x1024x24 "
                         "back-projection, --steps times, and print their mean time (a short run to profile one "
                         "denoiser kernel; not the benchmark line)")
    ap.add_argument("--batched-only", action="store_true",
                    help="only run the batched-solve measurement (64 measurements) and print its JSON (a short run "
                         "to profile the batched graph; not the benchmark line)")
    ap.add_argument("--net-only", action="store_true",
                    help="only time the warm-start network's kernels (forward at 1024x1024x24, training steps at "
                         "512x512x16) and print their JSON (a short run to profile the MFMA kernels; not the "
                         "benchmark line)")
    ap.add_argument("--learned-only", action="store_true",
                    help="only run the learned warm start's full protocol (20000 training crops, 200 outer "
                         "iterations) and print its JSON (minutes; not the benchmark line)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run plain 1 GiB device copies (reference for HBM counter scaling)")
    args = ap.parse_args()

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this implementation runs on a single GPU; --gpus must be 1 "
              "(multi-GPU sharding is a design note, not built).", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        return 1
    from paper_2005_08028_amd import build as hipbuild
    if not os.path.exists(hipbuild.LIB):
        hipbuild.build()
    from paper_2005_08028_amd import scitv, synth

    wl = "cacti_1024x24"
    cfg = synth.CONFIGS[wl]
    nx, ny, B = cfg["nx"], cfg["ny"], cfg["B"]
    T, N, lam = args.outer, cfg["N"], cfg["lam"]
    V = nx * ny * B
    dev = torch.device("cuda:0")
    pr = synth.problem_from_config(wl)
    ctx = scitv.Context(0)
    h = ctx.handle
    C = torch.from_numpy(pr.masks).to(dev)
    X_true = torch.from_numpy(pr.truth).to(dev)
    Y = scitv.sci_forward(h, C, X_true) + torch.from_numpy(pr.noise).to(dev)
    X_out = torch.empty_like(C)
    Th_out = torch.empty_like(C)
    prm = scitv.solver_params(outer_iters=T, tv=cfg["tv"], lam=lam, n_inner=N, schedule=args.schedule,
                              dual_dtype=args.dual_dtype)

    if args.paper_shaped_only:
        res = measure_paper_shaped(scitv, synth, h, dev, curves_on=False)
        ctx.close()
        print(json.dumps({"paper_shaped_vtv_512x512x10": res}), flush=True)
        return 0
    if args.batched_only:
        res = measure_batched(scitv, synth, h, dev, max(1, min(args.steps, 3)))
        res_vtv = measure_batched_vtv(scitv, synth, h, dev)
        ctx.close()
        print(json.dumps({"batched": res, "batched_vtv": res_vtv}), flush=True)
        return 0
    if args.net_only:
        res = measure_net(scitv, h, dev, C, Y, max(3, args.steps))
        ctx.close()
        print(json.dumps({"network": res}), flush=True)
        return 0
    if args.learned_only:
        res = measure_learned(scitv, synth, h, dev, Y, C, X_true, lam)
        ctx.close()
        print(json.dumps({"learned_warm_start": res}), flush=True)
        return 0
    if args.denoise_only:
        kind = args.denoise_only.split("-")
        tp = scitv.tv_params(tv=kind[0], lam=lam, n_inner=N, accel=len(kind) == 1,
                             chambolle04=kind[-1] == "ch", clip=kind[-1] == "clip", dual_dtype=args.dual_dtype)
        x0 = scitv.sci_adjoint(h, C, Y)
        th = torch.empty_like(x0)
        scitv.sci_tv_denoise(h, x0, tp, Theta_out=th)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            scitv.sci_tv_denoise(h, x0, tp, Theta_out=th)
        torch.cuda.synchronize()
        us = (time.perf_counter() - t0) / args.steps * 1e6
        ctx.close()
        print(json.dumps({"denoise_only": args.denoise_only, "dual_dtype": args.dual_dtype, "shape": [B, nx, ny],
                          "n_inner": N, "calls": args.steps,
                          "us_per_call": round(us, 2)}), flush=True)
        return 0
    if args.kernel_table_only:
        table = measure_kernels(scitv, h, dev, C, Y, X_true)
        ctx.close()
        print(json.dumps({"kernel_table_1024x1024x24": table}), flush=True)
        return 0

    tuned = None
    tag = "shape1/passes%d" % ((N + 4) // 5)
    if not args.no_autotune and cfg["tv"] in ("atv", "itv2d"):
        # tile shape and pass count of the fused denoiser, timed on this measurement's back-projection
        x0 = scitv.sci_adjoint(h, C, Y)
        best, passes, times = scitv.sci_autotune(h, x0, prm.tv)
        tuned = {"best_shape": best, "rows_waves_cols": scitv.sci_tile_shape_info(best), "passes": passes,
                 "ms_per_denoise_by_shape_and_passes": [[round(t, 4) for t in row] for row in times]}
        tag = "shape%d/passes%d" % (best, passes if args.schedule != "stream" else N)
        del x0

    def step():
        scitv.sci_gap_tv(h, Y, C, prm, X_out=X_out, Theta_out=Th_out)
        psnr = scitv.sci_psnr(h, X_out, X_true)
        resid = scitv.sci_residual_sq(h, C, X_out, Y)
        return psnr, resid

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        psnr, resid = step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    # kernel durations: the same steps again with the library's HIP event pair
    # around every launch on its stream (the events add about 2 us per launch,
    # so the throughput above is timed without them)
    scitv.sci_profile_enable(h, True)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed_prof = time.perf_counter() - t1
    scitv.sci_profile_enable(h, False)

    fams = {}
    for fam in ("fgp_stream", "fgp_fused", "tv_theta", "project", "setup"):
        n, ms = scitv.sci_profile_read(h, fam)
        if n:
            fams[fam] = (n, ms)
    dom = max(fams, key=lambda f: fams[f][1])
    elem = 4 if args.dual_dtype == "f32" else 2
    roofline = roofline_for(dom, fams[dom][0], fams[dom][1], V, N, cfg["tv"], elem,
                            tag if dom == "fgp_fused" else "stream")

    steps = args.steps
    value = V * T * N * steps / elapsed
    out = {
        "metric": METRIC, "value": value, "unit": "voxel-iter/s", "n_gpus": 1, "steps": steps,
        "warmup": args.warmup, "ms_per_step": elapsed / steps * 1e3, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": f"{wl}: GAP-ITV2D {nx}x{ny}x{B}, {T} outer x {N} inner FGP, lambda={lam}, "
                               f"shifted Bernoulli(0.5) masks, textured moving-shape scene",
                   "nx": nx, "ny": ny, "B": B, "outer_iters": T, "inner_iters": N, "tv": cfg["tv"],
                   "schedule": args.schedule, "dual_dtype": args.dual_dtype, "graph": False, "tiling": tag},
        "roofline": roofline,
        # the one-pass byte model of an inner iteration (read x, p, p_prev; write p: 28 B per voxel with
        # float32 duals): the rate a schedule with one HBM pass per iteration could reach at 8 TB/s, and
        # this run's whole-solve rate against it (above 1 means the temporal blocking beats the model)
        "one_pass_hbm_model": {"bytes_per_voxel_iter": 28 if args.dual_dtype == "f32" else 16,
                               "voxel_iter_per_s_at_8TBs": 8e12 / (28 if args.dual_dtype == "f32" else 16),
                               "value_over_model": V * T * N * steps / elapsed /
                               (8e12 / (28 if args.dual_dtype == "f32" else 16))},
        "kernel_ms_per_step": {f: round(ms / steps, 3) for f, (n, ms) in fams.items()},
        "ms_per_step_profiled_repeat": elapsed_prof / steps * 1e3,
        "psnr_db": round(psnr, 4), "residual_sq": resid, "autotune": tuned,
    }

    if args.calibrate_copy:
        a = torch.empty(1 << 28, dtype=torch.float32, device=dev)  # 1 GiB
        b = torch.empty_like(a)
        a.fill_(1.0)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = a.numel() * 4

    if not args.no_extras:
        # 16-bit dual storage on the streaming schedule (the fused single pass keeps duals on chip)
        ref = X_out.clone()
        mp = {}
        for dt in ("f32", "bf16", "f16"):
            p16 = scitv.solver_params(outer_iters=T, tv=cfg["tv"], lam=lam, n_inner=N, schedule="stream",
                                      dual_dtype=dt)
            scitv.sci_autotune(h, X_out, p16.tv)
            x16 = torch.empty_like(C)
            scitv.sci_gap_tv(h, Y, C, p16, X_out=x16)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            scitv.sci_gap_tv(h, Y, C, p16, X_out=x16)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) * 1e3
            rel = float(torch.linalg.vector_norm((x16 - ref).double()) / torch.linalg.vector_norm(ref.double()))
            mp[dt] = {"ms_per_solve": round(ms, 2), "voxel_iter_per_s": V * T * N / (ms / 1e3),
                      "rel_l2_vs_fused_fp32": rel,
                      "dpsnr_db_vs_fused_fp32": round(scitv.sci_psnr(h, x16, X_true) - psnr, 5)}
        out["dual_storage_stream_schedule"] = mp
        # VTV on the fused schedule: a 10-iteration call at B = 24 is two on-chip passes, and the dual
        # crosses between them once, as one record per voxel in the storage type
        x0 = scitv.sci_adjoint(h, C, Y)
        thv = torch.empty_like(x0)
        vt = {}
        for dt in ("f32", "bf16", "f16"):
            tp = scitv.tv_params(tv="vtv", lam=lam, n_inner=N, dual_dtype=dt)
            scitv.sci_tv_denoise(h, x0, tp, Theta_out=thv)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(20):
                scitv.sci_tv_denoise(h, x0, tp, Theta_out=thv)
            torch.cuda.synchronize()
            vt[dt] = round((time.perf_counter() - t0) / 20 * 1e6, 2)
        out["vtv_fused_denoise_us_by_dual_storage"] = {"shape": [B, nx, ny], "n_inner": N, "calls": 20, **vt}
        del x0, thv
        out["batched"] = measure_batched(scitv, synth, h, dev, max(1, min(steps, 3)))
        out["batched_vtv"] = measure_batched_vtv(scitv, synth, h, dev)
        # the workload's learned warm start at reduced scale (the full protocol: --learned-only)
        out["learned_warm_start"] = measure_learned(scitv, synth, h, dev, Y, C, X_true, lam, n_crops=2000,
                                                    n_held=400, epochs=1, T_eval=30, every_counts=5)
        out["learned_warm_start"]["scale"] = "reduced: 2000 training crops, 1 epoch, 30 outer iterations, gap " \
                                             "checked every 5; bench.py --learned-only runs the full protocol"
        out["paper_shaped_vtv_512x512x10"] = measure_paper_shaped(scitv, synth, h, dev)
        out["kernel_table_1024x1024x24"] = measure_kernels(scitv, h, dev, C, Y, X_true)

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(scitv, h, dev, pr, C, nx, ny, B, N, T, lam, cfg["tv"], args)
    ctx.close()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
