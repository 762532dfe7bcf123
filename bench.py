#!/usr/bin/env python
"""Benchmark of the many-body active-sphere solve on one MI355X.

One step = one full solve of the trap workload to a binary64 relative residual of 1e-10:
right-hand side pass, initial guess, GMRES (or mixed-precision refinement), output pass.
Default workload: N = 100000 spheres, cube of side 430, seed 1000 (number density 1.26e-3),
mean and strain slip along random orientations, trap force -0.5 R.

Prints ONE JSON line. `value` is the pair-block evaluation rate of the headline solve
(all passes, inputs resident in device memory); `ms_per_step` is its time to solution.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "pair-blocks/s; time to 1e-10 residual at N=1e5, plain FP64 vs mixed+warm start"
FP64_PEAK_TF = 78.6     # MI355X vector FP64
FP32_PEAK_TF = 157.3    # MI355X vector FP32 (published figure, counts packed FP32)
# algorithmic FLOP per pair block of the system operator (FMA = 2, rsqrt = 1), the count the roofline's
# `achieved` uses: differences 3, r^2 5, rsqrt 1, powers 5, w = Sigma x 15, q 5, c1 c2 c3 9, trace term 4,
# c1 x and c2 x 6, five accumulated components 43
P2_FLOP_PER_PAIR_ALG = 95
# the same block as implemented (accumulating raw moments, projecting once per receiver): differences
# 3, r^2 5, 1/r 1, powers 4, Szz 1, w 15, q 5, c1 3, c2 4, v 9, moments 18, r^-5 Sigma 10
P2_FLOP_PER_PAIR = 78
FLOW_FLOP_PER_PAIR = 68  # field-point flow from force and flow stresslet (no torque, no rank-3 mode)
# the pass of the septlet, vortlet and spinlet slip modes (all three present), per pair, counted from
# the implemented formulas (FMA = 2, rsqrt = 1): geometry 14; strain target gamma 115, psi 97,
# lambda 126; motion target 85, 53, 82; flow target 69, 33, 61
HIGH_FLOP_PER_PAIR = {"strain": 352, "motion": 234, "flow": 177}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=100_000)
    ap.add_argument("--side", type=float, default=430.0)
    ap.add_argument("--seed", type=int, default=1000)
    ap.add_argument("--skip-cpu", action="store_true", help="do not time the CPU oracle")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--headline", default="mixed_pc",
                    choices=["plain_fp64", "fp64_diag", "mixed_diag", "fp64_learned", "mixed_learned",
                             "fp64_pc", "mixed_pc", "mixed_diag_pc", "mixed_learned_pc"])
    ap.add_argument("--near-order", type=int, default=4,
                    help="Neumann order of the near-field preconditioner in the *_pc variants")
    ap.add_argument("--aux-near-cutoff", type=float, default=8.0,
                    help="near-field cutoff of the batched and time-stepping runs (order 2)")
    ap.add_argument("--near-cutoff", type=float, default=12.0,
                    help="near-field preconditioner cutoff (centre distance) of the *_pc variants")
    ap.add_argument("--skip-warmstart", action="store_true", help="no learned warm start (no training)")
    ap.add_argument("--warmstart-configs", type=int, default=200)
    ap.add_argument("--warmstart-epochs", type=int, default=20)
    ap.add_argument("--skip-batched", action="store_true")
    ap.add_argument("--skip-stepper", action="store_true")
    ap.add_argument("--skip-kernels", action="store_true", help="skip the per-size pair-pass timings")
    ap.add_argument("--stepper-steps", type=int, default=1000)
    ap.add_argument("--scale-n", type=int, default=0,
                    help="also time the preconditioned binary64 and mixed solves at this N (benchmark "
                         "density), with and without spatial ordering; 0 (default) skips it")
    ap.add_argument("--profile-passes", action="store_true",
                    help="short run for hardware counters: one launch of every binary64 pass kernel at N")
    ap.add_argument("--skip-rank3", action="store_true", help="skip the traction rank <= 3 timings")
    ap.add_argument("--skip-plane", action="store_true", help="skip the plane (stress-free, no-slip) timings")
    ap.add_argument("--skip-periodic", action="store_true", help="skip the periodic box timings")
    ap.add_argument("--profile-rank3", action="store_true",
                    help="profiling mode: a 256 MiB device copy (counter calibration), then --steps "
                         "rank <= 3 operator applications at N = 10^4")
    ap.add_argument("--profile-geometries", action="store_true",
                    help="profiling mode: the plane, wall and periodic-box sections of the bench line alone "
                         "(their passes at 10^4 and --n spheres and the solves at 10^4), printed as JSON")
    ap.add_argument("--profile-mesh", action="store_true",
                    help="profiling mode: the particle-mesh Ewald operator in the periodic box, 10^5 spheres "
                         "on a 256^3 mesh and 10^6 on a 512^3 mesh, 6 untimed and 5 timed passes each")
    ap.add_argument("--profile-matvec", action="store_true",
                    help="profiling mode: a 256 MiB device copy (counter calibration), then --steps "
                         "binary64 and --steps binary32 operator applications at the autotuned shapes")
    return ap.parse_args()


def profile_matvec(a, w):
    """Short run for hardware-counter passes: calibration copy, then the two operator kernels."""
    import torch

    from paper_1411_0278_amd import mbstokes
    src = torch.empty(32 * 1024 * 1024, dtype=torch.float64, device="cuda:0").fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)  # 256 MiB read + 256 MiB written
    torch.cuda.synchronize()
    R = torch.as_tensor(w.R, dtype=torch.float64).to("cuda:0")
    x = torch.as_tensor(w.v2s, dtype=torch.float64).contiguous().to("cuda:0")
    ctx = mbstokes.Context(0)
    t64, t32 = ctx.mbs_autotune(R, None)
    times = {}
    for prec, t in ((mbstokes.MBS_FP64, t64), (mbstokes.MBS_FP32, t32)):
        ctx.set_params(tile=t + 1)
        y = ctx.mbs_matvec(R, x, precision=prec)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(a.steps):
            ctx.mbs_matvec(R, x, y, precision=prec)
        e1.record()
        torch.cuda.synchronize()
        times["f64" if prec == mbstokes.MBS_FP64 else "f32"] = e0.elapsed_time(e1) / a.steps
    ctx.close()
    print(json.dumps({"mode": "profile-matvec", "n": w.n, "tiles": [t64, t32], "ms_per_launch": times,
                      "copy_bytes": 2 * src.numel() * 8}), flush=True)


def profile_passes(a, w):
    """Short run for hardware-counter passes over the binary64 pass kernels at N: right-hand side,
    outputs, flow at N field points, the higher slip modes' three passes, and one mixed-precision
    preconditioned solve (its fused final residual + outputs pass). Default launch shapes."""
    import torch

    from paper_1411_0278_amd import inputs, mbstokes
    d = mbstokes.to_device(w, "cuda:0")
    g, ps, l = inputs.higher_slip_modes(w.p, 1.0, 1.0, 1.0)
    f = lambda v: torch.as_tensor(v, dtype=torch.float64).contiguous().to("cuda:0")
    hm = dict(gam=f(g), psi=f(ps), lam=f(l))
    ctx = mbstokes.Context(0)
    sig = torch.randn((w.n, 5), dtype=torch.float64, device="cuda:0")
    gen = torch.Generator(device="cuda:0").manual_seed(5)
    X = (torch.rand((w.n, 3), dtype=torch.float64, device="cuda:0", generator=gen) - 0.5) * a.side
    ctx.mbs_rhs_ex(d["R"], d["v2s"], None, Fe=d["Fe"], **hm)
    ctx.mbs_outputs_ex(d["R"], sig, d["v1s"], d["v2s"], None, Fe=d["Fe"], **hm)
    ctx.mbs_flow_ex(X, d["R"], sig, Fe=d["Fe"], **hm)
    ctx.set_params(precision=mbstokes.MBS_MIXED, tol=1e-10, near_cutoff=a.near_cutoff, near_order=a.near_order)
    V, W, S, st = ctx.mbs_solve(d["R"], d["p"], d["v1s"], d["v2s"], None, d["Fe"], None)
    torch.cuda.synchronize()
    ctx.close()
    print(json.dumps({"mode": "profile-passes", "n": w.n, "solve_iters": st["iters"], "out_fused": st["out_fused"]}),
          flush=True)


P2_SOURCES = ("mbs_p2.hip", "mbs_pair.h", "mbs_device.h")
RANK3_SOURCES = ("mbs_rank3.hip", "mbs_device.h")


def profile_rank3(a):
    """Short run for hardware-counter passes: calibration copy, then the rank <= 3 operator at 10^4."""
    import torch

    from paper_1411_0278_amd import inputs, mbstokes
    src = torch.empty(32 * 1024 * 1024, dtype=torch.float64, device="cuda:0").fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)  # 256 MiB read + 256 MiB written
    w = inputs.config1()
    R = torch.as_tensor(w.R, dtype=torch.float64).to("cuda:0")
    gen = torch.Generator(device="cuda:0").manual_seed(3)
    x = torch.randn((w.n, 20), dtype=torch.float64, device="cuda:0", generator=gen)
    ctx = mbstokes.Context(0)
    y = ctx.mbs_matvec_r3(R, x)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(a.steps):
        ctx.mbs_matvec_r3(R, x, y)
    e1.record()
    torch.cuda.synchronize()
    ctx.close()
    print(json.dumps({"mode": "profile-rank3", "n": w.n, "ms_per_launch": e0.elapsed_time(e1) / a.steps,
                      "copy_bytes": 2 * src.numel() * 8}), flush=True)


def bench_rank3(ctx, a):
    """Traction ranks <= 3 (septlet, vortlet and potential-dipole traction modes solved for beside the
    stresslet; 20 unknowns per sphere, binary64). The operator pass at 10^4 spheres (the trap box of
    side 200) and at the benchmark N; at 10^4 also the right-hand-side and output passes and the
    solve to 1e-10 with every slip mode present (uniaxial modes from the orientations: s = 3(pp - I/3),
    d = p, gamma, psi, lambda of the orientations, F = -0.5 R). Median of 5 launches after 2 warm-ups
    (3 solves after 1), HIP events on the launch stream; the roofline is the executed FLOP per pair
    from the committed counters against the binary64 vector peak."""
    import statistics

    import numpy as np
    import torch

    from paper_1411_0278_amd import inputs, mbstokes

    def median_ms(fn, warm=2, reps=5):
        for _ in range(warm):
            fn()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return statistics.median(ts)

    out = {"unknowns_per_sphere": 20, "dtype": "f64", "peak_tflops_f64_vector": 78.6}
    for label, w in (("n10000", inputs.trap_workload(10_000, 200.0, 1, v3t=1.0)),
                     ("n%d" % a.n, inputs.trap_workload(a.n, a.side, a.seed, v3t=1.0))):
        n = w.n
        f = lambda v: torch.as_tensor(np.ascontiguousarray(v), dtype=torch.float64).to("cuda:0")
        R = f(w.R)
        gen = torch.Generator(device="cuda:0").manual_seed(3)
        x = torch.randn((n, 20), dtype=torch.float64, device="cuda:0", generator=gen)
        y = torch.empty_like(x)
        ms = median_ms(lambda: ctx.mbs_matvec_r3(R, x, y), reps=5 if n <= 20_000 else 3)
        pairs = n * (n - 1)
        row = {"n": n, "matvec": {"ms": round(ms, 4), "pair_blocks_per_s": pairs / (ms * 1e-3)}}
        # executed FLOP per pair is a property of the pair arithmetic: the counters taken at 10^4
        # apply at every size
        rec = measured_counters("k_rank3_op", 10_000, RANK3_SOURCES)
        ex = rec.get("executed_flop_per_pair") if rec else None
        row["matvec"]["executed_flop_per_pair"] = ex
        row["matvec"]["counters_taken_at_n"] = 10_000 if ex else None
        row["matvec"]["executed_tflops"] = round(ex * pairs / (ms * 1e-3) / 1e12, 3) if ex else None
        row["matvec"]["frac_executed"] = round(ex * pairs / (ms * 1e-3) / 1e12 / 78.6, 4) if ex else None
        if n <= 20_000:
            g, ps, l = inputs.higher_slip_modes(w.p, 1.0, 1.0, 1.0)
            hm = dict(gam=f(g), psi=f(ps), lam=f(l))
            d = mbstokes.to_device(w, "cuda:0")
            ms = median_ms(lambda: ctx.mbs_rhs_r3(d["R"], d["v2s"], d["v3t"], Fe=d["Fe"], **hm))
            row["rhs"] = {"ms": round(ms, 4)}
            ms = median_ms(lambda: ctx.mbs_outputs_r3(d["R"], x, d["v1s"], d["v2s"], hm["lam"], Fe=d["Fe"]))
            row["outputs"] = {"ms": round(ms, 4)}
            ctx.set_params(tol=1e-10, max_iter=300, precision=mbstokes.MBS_FP64, guess=mbstokes.MBS_GUESS_ZERO,
                           near_cutoff=0.0, superposition=0)
            sts = []
            for k in range(4):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                V, W, S, xs, st = ctx.mbs_solve_r3(d["R"], d["v1s"], d["v2s"], d["v3t"], Fe=d["Fe"], **hm)
                torch.cuda.synchronize()
                if k:
                    st["wall_ms"] = 1e3 * (time.perf_counter() - t0)
                    sts.append(st)
            med = sorted(sts, key=lambda t: t["wall_ms"])[len(sts) // 2]
            row["solve"] = {"ms": round(med["wall_ms"], 3), "device_ms": round(med["t_total_ms"], 3),
                            "iters": med["iters"], "fp64_matvecs": med["fp64_matvecs"],
                            "rel_resid": med["rel_resid"], "t_op64_ms": round(med["t_op64_ms"], 3)}
            # right-preconditioned by the near-field series over the pairs within the cutoff
            row["solve_pc"] = {}
            for cut, order in ((8.0, 2), (12.0, 4)):
                ctx.set_params(near_cutoff=cut, near_order=order)
                sts = []
                for k in range(4):
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    _, _, _, _, st = ctx.mbs_solve_r3(d["R"], d["v1s"], d["v2s"], d["v3t"], Fe=d["Fe"], **hm)
                    torch.cuda.synchronize()
                    if k:
                        st["wall_ms"] = 1e3 * (time.perf_counter() - t0)
                        sts.append(st)
                med = sorted(sts, key=lambda t: t["wall_ms"])[len(sts) // 2]
                row["solve_pc"][f"{cut:g}a_order{order}"] = {
                    "ms": round(med["wall_ms"], 3), "device_ms": round(med["t_total_ms"], 3), "iters": med["iters"],
                    "fp64_matvecs": med["fp64_matvecs"], "rel_resid": med["rel_resid"]}
            ctx.set_params(near_cutoff=0.0, near_order=0)
            # how far the rank <= 2 truncation is from it on the same spheres (the modes' one-body
            # closure against solving for them): relative change of V and Omega
            V2, W2, S2, _ = ctx.mbs_solve_ex(d["R"], d["p"], d["v1s"], d["v2s"], d["v3t"], Fe=d["Fe"], **hm)
            row["vs_rank2"] = {"rel_change_V": float((V - V2).norm() / V.norm()),
                               "rel_change_Omega": float((W - W2).norm() / W.norm())}
        out[label] = row
        print(f"bench: rank-3 {label} matvec {row['matvec']['ms']} ms", file=sys.stderr, flush=True)
    return out


def kernel_source_hash(files=P2_SOURCES):
    h = hashlib.sha256()
    for f in files:
        h.update(open(os.path.join(ROOT, "paper_1411_0278_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def measured_counters(kernel, n, files=P2_SOURCES):
    """The committed PMC record of a kernel at size n (HBM bytes per launch, executed FLOP per pair),
    if the counters were taken on the current source of the files it is built from; else None."""
    path = os.path.join(ROOT, "profiles", "pmc_traffic.json")
    if not os.path.exists(path):
        return None
    try:
        rec = json.load(open(path)).get(f"{kernel}@n{n}")
    except Exception:
        return None
    if not rec or rec.get("source_sha") != kernel_source_hash(files):
        return None
    return rec


def time_variant(ctx, d, mb, name, precision, guess, steps, warmup, near_cutoff=0.0, near_order=2):
    import torch
    ctx.set_params(precision=precision, guess=guess, tol=1e-10, near_cutoff=near_cutoff,
                   near_order=near_order if near_cutoff > 0 else 2)
    args = (d["R"], d["p"], d["v1s"], d["v2s"], d.get("v3t"), d["Fe"], d.get("Te"))
    for k in range(warmup):
        ctx.mbs_solve(*args)
        print(f"bench: {name} warmup {k + 1}/{warmup} done", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    stats = []
    for k in range(steps):
        _, _, _, st = ctx.mbs_solve(*args)
        stats.append(st)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    print(f"bench: {name} {steps} solves in {dt:.3f} s", file=sys.stderr, flush=True)
    pairs = sum(s["pair_blocks"] for s in stats)
    return dict(name=name, seconds=dt, ms_per_step=1e3 * dt / steps, pair_blocks_per_s=pairs / dt,
                iters=stats[-1]["iters"], refinements=stats[-1]["refinements"],
                fp64_matvecs=stats[-1]["fp64_matvecs"], fp32_matvecs=stats[-1]["fp32_matvecs"],
                rel_resid=max(s["rel_resid"] for s in stats),
                t_op64_ms=sum(s["t_op64_ms"] for s in stats), t_op32_ms=sum(s["t_op32_ms"] for s in stats),
                n_op64=sum(s["fp64_matvecs"] for s in stats), n_op32=sum(s["fp32_matvecs"] for s in stats),
                t_rhs_ms=stats[-1]["t_rhs_ms"], t_out_ms=stats[-1]["t_out_ms"],
                t_iter_ms=stats[-1]["t_iter_ms"])


def roofline(v, n):
    """Dominant kernel of the step: the operator application with the larger summed time."""
    use32 = v["t_op32_ms"] > v["t_op64_ms"]
    t_ms, cnt = (v["t_op32_ms"], v["n_op32"]) if use32 else (v["t_op64_ms"], v["n_op64"])
    if cnt == 0 or t_ms <= 0:
        return None
    per_launch_s = t_ms / cnt / 1e3
    pairs = n * (n - 1)
    achieved = P2_FLOP_PER_PAIR_ALG * pairs / per_launch_s / 1e12
    peak = FP32_PEAK_TF if use32 else FP64_PEAK_TF
    kernel = "k_p2_f32" if use32 else "k_p2_f64"
    rec = measured_counters(kernel, n) or {}
    out = {"bound": "alu", "kernel": kernel, "achieved": round(achieved, 3), "peak": peak,
           "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
           "traffic": rec.get("bytes_per_launch"), "avg_launch_ms": round(per_launch_s * 1e3, 4),
           "frac_basis": f"algorithmic: {P2_FLOP_PER_PAIR_ALG} FLOP per pair block (the closed-form block's count) x N(N-1)",
           "flop_per_pair": P2_FLOP_PER_PAIR_ALG,
           "implemented_flop_per_pair": P2_FLOP_PER_PAIR,
           "frac_implemented": round(P2_FLOP_PER_PAIR * pairs / per_launch_s / 1e12 / peak, 4)}
    ex = rec.get("executed_flop_per_pair")
    out["executed_flop_per_pair"] = ex
    out["frac_executed"] = round(ex * pairs / per_launch_s / 1e12 / peak, 4) if ex else None
    return out


def bench_kernels(ctx, a):
    """Pair-pass throughput on their own: the operator (binary64 and binary32) at N = 256, 10^4 and
    10^5 (each with its own autotuned shape), and the right-hand-side and output passes at 10^5.
    Median of 5 launches after 2 warm-ups, HIP events on the launch stream."""
    import statistics

    import torch

    from paper_1411_0278_amd import inputs, mbstokes

    def median_ms(fn):
        for _ in range(2):
            fn()
        ts = []
        for _ in range(5):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return statistics.median(ts)

    out = {}
    for label, w in (("n256", inputs.config0()), ("n10000", inputs.config1()),
                     ("n100000", inputs.trap_workload(a.n, a.side, a.seed))):
        d = mbstokes.to_device(w, "cuda:0")
        n = w.n
        tiles = ctx.mbs_autotune(d["R"], None)
        x = d["v2s"].contiguous()
        y = torch.empty_like(x)
        row = {"tiles": list(tiles)}
        for name, prec in (("p2_f64", mbstokes.MBS_FP64), ("p2_f32", mbstokes.MBS_FP32)):
            ms = median_ms(lambda: ctx.mbs_matvec(d["R"], x, y, precision=prec))
            row[name] = {"ms": round(ms, 4), "pair_blocks_per_s": n * (n - 1) / (ms * 1e-3),
                         "tflops_algorithmic": round(P2_FLOP_PER_PAIR_ALG * n * (n - 1) / (ms * 1e-3) / 1e12, 3),
                         "tflops_implemented": round(P2_FLOP_PER_PAIR * n * (n - 1) / (ms * 1e-3) / 1e12, 3)}
        if n == a.n:
            # as in the benchmark solve: no torque, no rank-3 slip
            ms = median_ms(lambda: ctx.mbs_rhs(d["R"], d["v2s"], None, d["Fe"], None))
            row["p1"] = {"ms": round(ms, 4), "pair_blocks_per_s": n * (n - 1) / (ms * 1e-3)}
            sig = torch.randn((n, 5), dtype=torch.float64, device="cuda:0")
            ms = median_ms(lambda: ctx.mbs_outputs(d["R"], sig, d["v1s"], d["v2s"], None, d["Fe"], None))
            row["p3"] = {"ms": round(ms, 4), "pair_blocks_per_s": n * (n - 1) / (ms * 1e-3)}
            # flow at as many field points as spheres (uniform in the cube; timing only)
            gen = torch.Generator(device="cuda:0").manual_seed(5)
            X = (torch.rand((n, 3), dtype=torch.float64, device="cuda:0", generator=gen) - 0.5) * a.side
            ms = median_ms(lambda: ctx.mbs_flow(X, d["R"], sig, Fe=d["Fe"]))
            row["flow"] = {"ms": round(ms, 4), "field_points": n, "pair_blocks_per_s": n * n / (ms * 1e-3),
                           "tflops_algorithmic": round(FLOW_FLOP_PER_PAIR * n * n / (ms * 1e-3) / 1e12, 3)}
            row["higher_modes"] = bench_higher_modes(ctx, d, w, sig, X, median_ms,
                                                     0.0 if a.skip_cpu else min(10.0, a.cpu_seconds))
        out[label] = row
        print(f"bench: pair passes at {label} timed", file=sys.stderr, flush=True)
    return out


def bench_higher_modes(ctx, d, w, sig, X, median_ms, cpu_seconds=0.0):
    """The septlet, vortlet and spinlet slip modes (uniaxial along p) at N = 10^5: the pass each
    extended entry point adds (its time minus that of the plain entry point), and a solve with them.
    With cpu_seconds > 0 the oracle's blocks of the same strain pass are timed beside it on a bounded
    row sample (one host core)."""
    import time as _time

    import torch

    from paper_1411_0278_amd import inputs, mbstokes
    n = w.n
    g, ps, l = inputs.higher_slip_modes(w.p, 1.0, 1.0, 1.0)
    f = lambda a_: torch.as_tensor(a_, dtype=torch.float64).contiguous().to("cuda:0")
    hm = dict(gam=f(g), psi=f(ps), lam=f(l))
    row = {}
    base = median_ms(lambda: ctx.mbs_rhs(d["R"], d["v2s"], None, d["Fe"], None))
    ext = median_ms(lambda: ctx.mbs_rhs_ex(d["R"], d["v2s"], None, Fe=d["Fe"], **hm))
    row["strain_pass"] = {"ms": round(ext - base, 4), "flop_per_pair": HIGH_FLOP_PER_PAIR["strain"],
                          "tflops_algorithmic": round(HIGH_FLOP_PER_PAIR["strain"] * n * (n - 1) / ((ext - base) * 1e-3) / 1e12, 3)}
    base = median_ms(lambda: ctx.mbs_outputs(d["R"], sig, d["v1s"], d["v2s"], None, d["Fe"], None))
    ext = median_ms(lambda: ctx.mbs_outputs_ex(d["R"], sig, d["v1s"], d["v2s"], None, Fe=d["Fe"], **hm))
    row["motion_pass"] = {"ms": round(ext - base, 4), "flop_per_pair": HIGH_FLOP_PER_PAIR["motion"],
                          "tflops_algorithmic": round(HIGH_FLOP_PER_PAIR["motion"] * n * (n - 1) / ((ext - base) * 1e-3) / 1e12, 3)}
    base = median_ms(lambda: ctx.mbs_flow(X, d["R"], sig, Fe=d["Fe"]))
    ext = median_ms(lambda: ctx.mbs_flow_ex(X, d["R"], sig, Fe=d["Fe"], **hm))
    row["flow_pass"] = {"ms": round(ext - base, 4), "flop_per_pair": HIGH_FLOP_PER_PAIR["flow"],
                        "tflops_algorithmic": round(HIGH_FLOP_PER_PAIR["flow"] * n * n / ((ext - base) * 1e-3) / 1e12, 3)}
    ctx.set_params(precision=mbstokes.MBS_MIXED, guess=mbstokes.MBS_GUESS_ZERO, tol=1e-10, near_cutoff=12.0,
                   near_order=4)
    ctx.mbs_solve_ex(d["R"], d["p"], d["v1s"], d["v2s"], None, Fe=d["Fe"], **hm)
    torch.cuda.synchronize()
    t0 = _time.perf_counter()
    V, W, S, st = ctx.mbs_solve_ex(d["R"], d["p"], d["v1s"], d["v2s"], None, Fe=d["Fe"], **hm)
    torch.cuda.synchronize()
    row["solve_mixed_pc"] = {"ms": round(1e3 * (_time.perf_counter() - t0), 3), "iters": st["iters"],
                             "rel_resid": st["rel_resid"]}
    ctx.set_params(precision=mbstokes.MBS_FP64, near_cutoff=0.0, near_order=2)
    if cpu_seconds > 0:
        import numpy as np

        from oracle import galerkin
        prm = galerkin.Params(eta=w.eta, a=w.a)
        kinds = (("SEPT", g), ("VORT", ps), ("SPIN", l))
        for kind, _ in kinds:  # build the symbolic blocks (untimed)
            galerkin.pair_matrix(w.R, "E", kind, prm, np.array([0]))
        done, rng, t0 = 0, np.random.default_rng(2), _time.perf_counter()
        while _time.perf_counter() - t0 < cpu_seconds:
            rows = rng.choice(n, 2, replace=False)
            for kind, vals in kinds:
                galerkin.pair_matrix(w.R, "E", kind, prm, rows) @ vals.ravel()
            done += len(rows)
        dt = _time.perf_counter() - t0
        row["oracle_strain_pass"] = {"pair_blocks_per_s": done * (n - 1) / dt, "cores": 1,
                                     "sample": f"{done} receiver rows of the three modes' strain blocks against "
                                               f"all {n} sources ({dt:.1f} s, numpy single thread)"}
    return row


def bench_batched(ctx, a):
    """512 independent configurations, N log-uniform in [64, 4096], density 0.004, one batched call."""
    import numpy as np
    import torch

    from paper_1411_0278_amd import inputs, mbstokes
    t0 = time.perf_counter()
    ws = inputs.config3()
    off = np.cumsum([0] + [w.n for w in ws])
    cat = lambda f: torch.as_tensor(np.concatenate([getattr(w, f) for w in ws])).to("cuda:0")
    R, v1s, v2s, Fe = cat("R"), cat("v1s"), cat("v2s"), cat("Fe")
    print(f"bench: batched workload of {len(ws)} configurations ({int(off[-1])} spheres) built in "
          f"{time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    def run(rc):
        ctx.set_params(precision=mbstokes.MBS_FP64, guess=mbstokes.MBS_GUESS_ZERO, tol=1e-10, near_cutoff=rc,
                       near_order=2)
        ctx.mbs_solve_batched(off, R, v1s, v2s, None, Fe, None)      # capture + warm-up
        torch.cuda.synchronize()
        reps = 3
        t1 = time.perf_counter()
        for _ in range(reps):
            V, W, S, stats, lat = ctx.mbs_solve_batched(off, R, v1s, v2s, None, Fe, None)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t1) / reps
        lat = np.array(lat)
        pairs = sum(st["pair_blocks"] for st in stats)
        return {"configs": len(ws), "spheres": int(off[-1]), "near_cutoff": rc, "ms_per_batch": 1e3 * dt,
                "configs_per_s": len(ws) / dt, "pair_blocks_per_s": pairs / dt,
                "latency_ms_min": float(lat.min()), "latency_ms_p50": float(np.percentile(lat, 50)),
                "latency_ms_p99": float(np.percentile(lat, 99)), "latency_ms_max": float(lat.max()),
                "launch": "one graph launch per batch from the second call of a batch shape on",
                "max_iters": int(max(st["iters"] for st in stats)),
                "max_rel_resid": float(max(st["rel_resid"] for st in stats))}

    t_tune = time.perf_counter()
    item, item_ms = ctx.mbs_autotune_batched(off, R)
    print(f"bench: batched work items of {item} receivers (autotuned in {time.perf_counter() - t_tune:.2f} s)",
          file=sys.stderr, flush=True)
    out = run(a.aux_near_cutoff)
    out["item_receivers"] = item
    out["item_pass_ms"] = {str(k): round(v, 4) for k, v in item_ms.items()}
    out["without_preconditioner"] = run(0.0)
    ctx.set_params(near_cutoff=0.0)
    return out


def bench_stepper(ctx, a):
    """N = 1e4 trap, slip (V1s, V2s, V3t) = (p, 3(pp - I/3), p), Adams-Bashforth dt = 0.01, as specified.

    The specified trap is stiff for this box (k = 0.5 pulls the cloud in at speeds of order 100 and
    nothing keeps spheres apart), so spheres overlap within a few steps; the run continues (each
    step still solves the Galerkin system of the current positions) and reports the first overlap
    step and how many steps met the tolerance. Per-step solve time comes from the library's events.
    """
    import torch

    from paper_1411_0278_amd import inputs, mbstokes
    w = inputs.config1()
    out = {"n": w.n, "steps": a.stepper_steps, "dt": 0.01, "near_cutoff": a.aux_near_cutoff,
           "guess": "previous step's stresslet (first step: one-body)", "max_iter_per_step": 60}
    ctx.mbs_autotune(torch.as_tensor(w.R).to("cuda:0"), None)  # pair-kernel shapes for this N
    for name, prec in (("fp64", mbstokes.MBS_FP64), ("mixed", mbstokes.MBS_MIXED)):
        R = torch.as_tensor(w.R).to("cuda:0")
        p = torch.as_tensor(w.p).to("cuda:0")
        ctx.set_params(precision=prec, guess=mbstokes.MBS_GUESS_USER, tol=1e-10, near_cutoff=a.aux_near_cutoff, near_order=2,
                       max_iter=60)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        stats, md = ctx.mbs_step(R, p, 0.5, (1.0, 1.0, 1.0), 0.01, a.stepper_steps, order=2,
                                 want_min_dist=True, allow_noconv=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        done = [s for s in stats if s["t_total_ms"] > 0]
        nd = len(done)
        first_overlap = next((k for k, v in enumerate(md[:nd]) if v < 2.0), None)
        phys = done[:first_overlap] if first_overlap is not None else done
        # the physical part of the run first: the steps before any two spheres overlap
        out[name] = {
            "before_overlap": {
                "steps": len(phys),
                "solve_ms_per_step": (sum(s["t_total_ms"] for s in phys) / len(phys)) if phys else None,
                "iters_per_step": (sum(s["iters"] for s in phys) / len(phys)) if phys else None,
                "steps_converged": sum(1 for s in phys if s["rel_resid"] <= 1e-10)},
            "first_overlap_step": first_overlap,
            "whole_run": {
                "note": "after the first overlap the system is no longer positive definite; most steps stop "
                        "at the iteration cap",
                "steps_completed": nd, "seconds": dt, "ms_per_step": 1e3 * dt / max(1, nd),
                "steps_converged": sum(1 for s in done if s["rel_resid"] <= 1e-10),
                "mean_iters": sum(s["iters"] for s in done) / max(1, nd),
                "fp64_matvecs": sum(s["fp64_matvecs"] for s in done),
                "fp32_matvecs": sum(s["fp32_matvecs"] for s in done),
                "min_distance_last": md[nd - 1] if nd else None}}
        print(f"bench: stepper {name} {nd} steps in {dt:.2f} s", file=sys.stderr, flush=True)
    ctx.set_params(guess=mbstokes.MBS_GUESS_ZERO, precision=mbstokes.MBS_FP64, max_iter=300)
    return out


def bench_paper_trap(ctx, a):
    """The trap of section V: 10^4 active spheres spread over the sphere R* = 1256.6a, pointing out
    (the stable state without interactions); AB2 with dt = 2 (tau_r = 8 pi eta a / k = 1675.5).
    Superposition approximation (the paper's own equations of motion) up to 8 tau_r, and the full
    many-body solve up to tau_r. Reports per-step time and, at t = tau_r, 2 tau_r, 8 tau_r, the mean
    p.R/|R| (1 at the start), the mean |R|/R* and the share of spheres pointing inward."""
    import numpy as np
    import torch

    from paper_1411_0278_amd import inputs, mbstokes
    w = inputs.paper_trap_workload()
    rstar = 1256.6
    k = -w.Fe[0, 0] / w.R[0, 0]
    tau_r = (8.0 * np.pi * w.eta * w.a) / k
    dt = 2.0
    per = int(round(tau_r / dt))
    coef = (-1.0, 0.0, 0.0)

    def snapshot(R, p, t):
        Rn, pn = R.cpu().numpy(), p.cpu().numpy()
        r = np.linalg.norm(Rn, axis=1)
        pr = (pn * Rn).sum(1) / r
        return {"t_over_tau_r": round(t / tau_r, 3), "mean_p_dot_rhat": float(pr.mean()),
                "mean_radius_over_Rstar": float(r.mean() / rstar), "inward_share": float((pr < 0).mean())}

    out = {"n": w.n, "Rstar_over_a": rstar, "k": k, "tau_r": tau_r, "dt": dt, "slip": "V^a = p (mean slip only)"}
    for mode, sup, horizon in (("superposition", 1, (1, 2, 8)), ("many_body", 0, (1,))):
        R = torch.as_tensor(w.R).to("cuda:0")
        p = torch.as_tensor(w.p).to("cuda:0")
        ctx.set_params(superposition=sup, precision=mbstokes.MBS_MIXED, guess=mbstokes.MBS_GUESS_USER,
                       tol=1e-10, near_cutoff=0.0, max_iter=60)
        snaps, done, secs, steps = [snapshot(R, p, 0.0)], 0, 0.0, 0
        hist = torch.zeros(11 * w.n, dtype=torch.float64, device="cuda:0")  # integrator history
        for mult in horizon:
            todo = mult * per - done
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, md = ctx.mbs_step(R, p, k, coef, dt, todo, order=2, want_min_dist=True, allow_noconv=True,
                                 hist=hist, hist_valid=done > 0)
            torch.cuda.synchronize()
            secs += time.perf_counter() - t0
            steps += todo
            done = mult * per
            s = snapshot(R, p, done * dt)
            s["min_distance"] = float(min(md))
            snaps.append(s)
        out[mode] = {"steps": steps, "seconds": secs, "ms_per_step": 1e3 * secs / steps, "snapshots": snaps}
        print(f"bench: paper trap {mode} {steps} steps in {secs:.1f} s", file=sys.stderr, flush=True)
    ctx.set_params(superposition=0, precision=mbstokes.MBS_FP64, guess=mbstokes.MBS_GUESS_ZERO, max_iter=300)
    return out


def bench_two_particle_orbits(ctx, horizon_tau=100, snap_tau=10):
    """Two active spheres in the trap of section V at R* = 12.56a (the two-particle figure): sphere 1
    at the pole, sphere 2 at the angle theta0 from it in the x-z plane, both pointing outward, mean
    slip only (V^a = p, as the 10^4-sphere run; the figure's stresslet and potential-dipole strengths
    are not given). AB2 with dt = 0.1 (tau_r / 167) for up to horizon_tau rotation times, stopped at
    the first step whose centre distance falls below 2a (the model has no contact force, so the motion
    past contact means nothing). A snapshot every snap_tau: polar angles of both centres in the x-z
    plane (from +z towards -x, degrees), |R|/R*, the centre distance and p.R/|R|. Superposition for
    every theta0, the many-body solve for three of them."""
    import numpy as np
    import torch

    from paper_1411_0278_amd import mbstokes
    rstar, eta, a = 12.56, ctx.params.eta, ctx.params.a
    k = 6.0 * np.pi * eta * a / (rstar * a)
    tau_r = 8.0 * np.pi * eta * a / k
    dt = 0.1
    per = int(round(tau_r / dt))
    out = {"Rstar_over_a": rstar, "k": k, "tau_r": tau_r, "dt": dt, "steps_per_tau_r": per,
           "slip": "V^a = p (mean slip only)", "plane": "x-z", "stop": "first centre distance < 2a",
           "orbits": []}

    def snap(R, p, t):
        Rn, pn = R.cpu().numpy(), p.cpu().numpy()
        r = np.linalg.norm(Rn, axis=1)
        ang = np.degrees(np.arctan2(-Rn[:, 0], Rn[:, 2])) % 360.0
        return {"t_over_tau_r": round(t / tau_r, 2), "polar_deg": [round(float(v), 2) for v in ang],
                "radius_over_Rstar": [round(float(v), 5) for v in r / rstar],
                "distance_over_a": round(float(np.linalg.norm(Rn[0] - Rn[1]) / a), 4),
                "p_dot_rhat": [round(float(v), 6) for v in (pn * Rn).sum(1) / r],
                "out_of_plane": float(np.abs(Rn[:, 1]).max() + np.abs(pn[:, 1]).max())}

    for theta0, modes in ((180, (1, 0)), (115, (1, 0)), (190, (1, 0)), (260, (1, 0))):
        th = np.radians(theta0)
        R0 = rstar * a * np.array([[0.0, 0.0, 1.0], [-np.sin(th), 0.0, np.cos(th)]])
        p0 = R0 / np.linalg.norm(R0, axis=1, keepdims=True)
        for sup in modes:
            R = torch.as_tensor(R0).to("cuda:0")
            p = torch.as_tensor(p0).to("cuda:0")
            hist = torch.zeros(22, dtype=torch.float64, device="cuda:0")
            ctx.set_params(superposition=sup, precision=mbstokes.MBS_FP64, guess=mbstokes.MBS_GUESS_ZERO,
                           tol=1e-12, near_cutoff=0.0, max_iter=60)
            snaps, mind, done, contact = [snap(R, p, 0.0)], float("inf"), 0, None
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for blk in range(horizon_tau):
                _, md = ctx.mbs_step(R, p, k, (-1.0, 0.0, 0.0), dt, per, order=2, want_min_dist=True,
                                     hist=hist, hist_valid=done > 0)
                hit = [i for i, v in enumerate(md) if v < 2.0 * a]
                if hit:  # the configuration after step done + hit[0] + 1 overlaps
                    contact = (done + hit[0] + 1) * dt / tau_r
                    mind = min(mind, min(md[:hit[0]]) if hit[0] else mind)
                    done += per
                    break
                mind = min(mind, min(md))
                done += per
                if (blk + 1) % snap_tau == 0:
                    snaps.append(snap(R, p, done * dt))
            torch.cuda.synchronize()
            secs = time.perf_counter() - t0
            rad = [v for s_ in snaps for v in s_["radius_over_Rstar"]]
            out["orbits"].append({
                "theta0": theta0, "mode": "superposition" if sup else "many_body", "steps": done,
                "ms_per_step": 1e3 * secs / done, "contact_at_t_over_tau_r": round(contact, 3) if contact else None,
                "min_distance_before_contact_over_a": round(mind / a, 4),
                "radius_over_Rstar_range": [min(rad), max(rad)],
                "min_p_dot_rhat": min(v for s_ in snaps for v in s_["p_dot_rhat"]), "snapshots": snaps})
            print(f"bench: two-particle orbit theta0={theta0} {'superposition' if sup else 'many-body'} "
                  f"{done} steps in {secs:.1f} s, contact at {contact}", file=sys.stderr, flush=True)
    ctx.set_params(superposition=0, precision=mbstokes.MBS_FP64, guess=mbstokes.MBS_GUESS_ZERO, tol=1e-10,
                   max_iter=300)
    return out


def bench_plane(ctx, a):
    """Spheres above a plane (params.plane: 1 stress-free, every sphere also acting through its
    mirror image; 2 no-slip wall, Blake's image system): the trap spheres of the box of side 200
    (10^4) and of the benchmark (10^5) with the plane 1.5a below the lowest one. The operator with
    and without the plane (binary64; binary32, whose image part is binary32 for the stress-free plane
    and binary64 for the wall), and at 10^4 the solve to 1e-10 (binary64; binary64 and mixed with the
    near-field preconditioner at 12a, order 4). Median of 5 launches after 2 warm-ups, HIP events."""
    import statistics

    import torch

    from paper_1411_0278_amd import inputs, mbstokes

    def median_ms(fn, warm=2, reps=5):
        for _ in range(warm):
            fn()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return statistics.median(ts)

    out = {"plane": "1.5a below the lowest sphere"}
    for kind, kname in ((1, "free_slip"), (2, "no_slip")):
        rows = {}
        for label, w in (("n10000", inputs.trap_workload(10_000, 200.0, 1)),
                         ("n%d" % a.n, inputs.trap_workload(a.n, a.side, a.seed))):
            n = w.n
            z_w = float(w.R[:, 2].min() - 1.5 * w.a)
            d = mbstokes.to_device(w, "cuda:0")
            x = d["v2s"].contiguous()
            y = torch.empty_like(x)
            row = {"n": n, "plane_z": z_w}
            for name, prec in (("f64", mbstokes.MBS_FP64), ("f32", mbstokes.MBS_FP32)):
                ctx.set_params(plane=0)
                free = median_ms(lambda: ctx.mbs_matvec(d["R"], x, y, precision=prec))
                ctx.set_params(plane=kind, plane_z=z_w)
                withp = median_ms(lambda: ctx.mbs_matvec(d["R"], x, y, precision=prec))
                row["matvec_" + name] = {"free_ms": round(free, 4), "plane_ms": round(withp, 4),
                                        "image_pass_ms": round(withp - free, 4)}
            if n <= 20_000:
                row["solve"] = {}
                for vname, prec, cut, order in (("fp64", mbstokes.MBS_FP64, 0.0, 2),
                                                ("fp64_pc", mbstokes.MBS_FP64, 12.0, 4),
                                                ("mixed_pc", mbstokes.MBS_MIXED, 12.0, 4)):
                    ctx.set_params(plane=kind, plane_z=z_w, precision=prec, near_cutoff=cut, near_order=order,
                                   tol=1e-10, guess=mbstokes.MBS_GUESS_ZERO)
                    sts = []
                    for k in range(3):
                        V, W, S, st = ctx.mbs_solve(d["R"], d["p"], d["v1s"], d["v2s"], None, d["Fe"], None)
                        if k:
                            sts.append(st)
                    med = sorted(sts, key=lambda t: t["t_total_ms"])[len(sts) // 2]
                    row["solve"][vname] = {"ms": round(med["t_total_ms"], 3), "iters": med["iters"],
                                           "fp64_matvecs": med["fp64_matvecs"],
                                           "fp32_matvecs": med["fp32_matvecs"], "rel_resid": med["rel_resid"]}
            ctx.set_params(plane=0, plane_z=0.0, precision=mbstokes.MBS_FP64, near_cutoff=0.0, near_order=2)
            rows[label] = row
            print(f"bench: plane {kname} {label} {row['matvec_f64']}", file=sys.stderr, flush=True)
        out[kname] = rows
    return out


def _lattice_positions(n, L, seed):
    """n sites of a cubic lattice filling the box, chosen at random and jittered so that every
    minimum-image distance stays >= 2.2a (the lattice is periodic, so across faces too)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    m = int(np.ceil(n ** (1.0 / 3.0) - 1e-9))
    h = L / m
    g = (np.arange(m) + 0.5) * h
    sites = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    sites = sites[rng.choice(len(sites), n, replace=False)]
    return sites + rng.uniform(-1.0, 1.0, (n, 3)) * max(0.0, (h - 2.2) / 2)


def profile_mesh():
    """Profiling mode: the particle-mesh Ewald operator in the periodic box at density 0.004, 10^5
    spheres on a 256^3 mesh and 10^6 on a 512^3 mesh, 6 untimed and 5 timed passes each."""
    import time

    import torch

    from paper_1411_0278_amd import inputs, mbstokes
    ctx = mbstokes.Context(0)
    out = {"mode": "profile-mesh"}
    for n, M in ((100_000, 256), (1_000_000, 512)):
        L = (n / 0.004) ** (1.0 / 3.0)
        w = inputs.trap_workload(n, L, 3)
        w.R = _lattice_positions(n, L, 3)
        d = mbstokes.to_device(w, "cuda:0")
        x = d["v2s"].contiguous()
        y = torch.empty_like(x)
        ctx.set_params(box=L, ewald_mesh=M)
        for _ in range(6):
            ctx.mbs_matvec(d["R"], x, y)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            ctx.mbs_matvec(d["R"], x, y)
        torch.cuda.synchronize()
        out["n%d_M%d_ms" % (n, M)] = round((time.perf_counter() - t0) / 5 * 1e3, 3)
        print(f"profile-mesh: n={n} M={M} {out['n%d_M%d_ms' % (n, M)]} ms per pass", file=sys.stderr, flush=True)
        ctx.set_params(box=0.0, ewald_mesh=0)
    ctx.close()
    print(json.dumps(out), flush=True)


def bench_periodic(ctx, a):
    """Spheres in a periodic cubic box (params.box, Ewald summation) at the benchmark density
    (0.004 spheres per a^3 on jittered lattice sites): the operator
    at 10^4 and 10^5 spheres against the unbounded operator of the same spheres, and at 10^4 the
    right-hand side, outputs and the solve to 1e-10 (binary64, and with the near-field preconditioner
    at 8a). Default splitting. The same with smooth particle-mesh Ewald (params.ewald_mesh, mesh spacing
    at most 1.25a, default splitting for the mesh): operator (with the largest relative difference of
    its result from the direct sums), right-hand side, outputs and the binary64 solve to 1e-10 (also with
    the near-field preconditioner at 12a, order 4) at 10^4 and 10^5 spheres, and at 10^6 the mesh
    operator and solves beside one direct pass. Median of 5
    launches after 2 warm-ups, HIP events (solves: the device time in their stats)."""
    import statistics

    import numpy as np
    import torch

    from paper_1411_0278_amd import inputs, mbstokes

    def median_ms(fn, warm=2, reps=5):
        for _ in range(warm):
            fn()
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1))
        return statistics.median(ts)

    lattice_positions = _lattice_positions

    def mesh_for(L):
        M = 16
        while L / M > 1.25:
            M *= 2
        return M

    out = {"density": 0.004, "splitting": "default: xi L = max(13, 13 (n/1e4)^0.15), rc = 6.5/xi, kmax = 13 xi",
           "mesh_splitting": "default: xi = min(pi M / (14 L), 0.5/a), rc = 5/xi, B-splines of order 8",
           "positions": "jittered cubic lattice sites, minimum-image distance >= 2.2a; orientations, slip and "
                        "forces of the trap workload"}
    for n, seed in ((10_000, 1), (a.n, a.seed)):
        L = (n / 0.004) ** (1.0 / 3.0)
        w = inputs.trap_workload(n, L, seed)
        w.R = lattice_positions(n, L, seed)
        d = mbstokes.to_device(w, "cuda:0")
        x = d["v2s"].contiguous()
        y = torch.empty_like(x)
        row = {"n": n, "box": L}
        ctx.set_params(box=0.0)
        row["matvec_unbounded_ms"] = round(median_ms(lambda: ctx.mbs_matvec(d["R"], x, y)), 4)
        ctx.set_params(box=L)
        row["matvec_ms"] = round(median_ms(lambda: ctx.mbs_matvec(d["R"], x, y)), 4)
        if n <= 20_000:
            row["rhs_ms"] = round(median_ms(lambda: ctx.mbs_rhs(d["R"], d["v2s"], None, d["Fe"], None, b=y)), 4)
            V, W, S = (torch.empty((n, k), dtype=torch.float64, device="cuda:0") for k in (3, 3, 5))
            row["outputs_ms"] = round(median_ms(lambda: ctx.mbs_outputs(d["R"], x, d["v1s"], d["v2s"], None, d["Fe"], None,
                                                                          V=V, W=W, S=S)), 4)
            row["solve"] = {}
            for vname, cut in (("fp64", 0.0), ("fp64_pc", 8.0)):
                ctx.set_params(box=L, precision=mbstokes.MBS_FP64, near_cutoff=cut, near_order=2, tol=1e-10,
                               guess=mbstokes.MBS_GUESS_ZERO)
                sts = []
                for k in range(3):
                    _, _, _, st = ctx.mbs_solve(d["R"], d["p"], d["v1s"], d["v2s"], None, d["Fe"], None)
                    if k:
                        sts.append(st)
                med = sorted(sts, key=lambda t: t["t_total_ms"])[len(sts) // 2]
                row["solve"][vname] = {"ms": round(med["t_total_ms"], 3), "iters": med["iters"],
                                       "rel_resid": med["rel_resid"]}
        ctx.set_params(box=L, near_cutoff=0.0, precision=mbstokes.MBS_FP64)
        ctx.mbs_matvec(d["R"], x, y)  # the direct sums' operator, kept for the comparison
        M = mesh_for(L)
        ctx.set_params(box=L, ewald_mesh=M)
        ym = torch.empty_like(x)
        mesh = {"M": M, "matvec_ms": round(median_ms(lambda: ctx.mbs_matvec(d["R"], x, ym)), 4)}
        mesh["vs_direct_maxrel"] = float((ym - y).abs().max() / y.abs().max())
        V, W, S = (torch.empty((n, k), dtype=torch.float64, device="cuda:0") for k in (3, 3, 5))
        mesh["rhs_ms"] = round(median_ms(lambda: ctx.mbs_rhs(d["R"], d["v2s"], None, d["Fe"], None, b=y)), 4)
        mesh["outputs_ms"] = round(median_ms(lambda: ctx.mbs_outputs(d["R"], x, d["v1s"], d["v2s"], None, d["Fe"],
                                                                       None, V=V, W=W, S=S)), 4)
        for vname, cut, order in (("solve_fp64", 0.0, 2), ("solve_fp64_pc", 12.0, 4)):
            ctx.set_params(box=L, ewald_mesh=M, tol=1e-10, guess=mbstokes.MBS_GUESS_ZERO, near_cutoff=cut,
                           near_order=order)
            sts = []
            for k in range(3):
                _, _, _, st = ctx.mbs_solve(d["R"], d["p"], d["v1s"], d["v2s"], None, d["Fe"], None)
                if k:
                    sts.append(st)
            med = sorted(sts, key=lambda t: t["t_total_ms"])[len(sts) // 2]
            mesh[vname] = {"ms": round(med["t_total_ms"], 3), "iters": med["iters"], "rel_resid": med["rel_resid"]}
        row["mesh"] = mesh
        ctx.set_params(box=0.0, ewald_mesh=0, near_cutoff=0.0, near_order=2, precision=mbstokes.MBS_FP64)
        out["n%d" % n] = row
        print(f"bench: periodic n={n} {row.get('matvec_ms')} ms, mesh {mesh['matvec_ms']} ms", file=sys.stderr,
              flush=True)
    n = 1_000_000
    L = (n / 0.004) ** (1.0 / 3.0)
    w = inputs.trap_workload(n, L, 3)
    w.R = lattice_positions(n, L, 3)
    d = mbstokes.to_device(w, "cuda:0")
    x = d["v2s"].contiguous()
    y, ym = torch.empty_like(x), torch.empty_like(x)
    M = mesh_for(L)
    ctx.set_params(box=L, ewald_mesh=M)
    row = {"n": n, "box": L, "M": M, "mesh_matvec_ms": round(median_ms(lambda: ctx.mbs_matvec(d["R"], x, ym)), 4)}
    print(f"bench: periodic n={n} mesh {row['mesh_matvec_ms']} ms", file=sys.stderr, flush=True)
    for vname, cut, order in (("mesh_solve_fp64", 0.0, 2), ("mesh_solve_fp64_pc", 12.0, 4)):
        ctx.set_params(box=L, ewald_mesh=M, tol=1e-10, guess=mbstokes.MBS_GUESS_ZERO, near_cutoff=cut, near_order=order)
        sts = []
        for k in range(2):
            _, _, _, st = ctx.mbs_solve(d["R"], d["p"], d["v1s"], d["v2s"], None, d["Fe"], None)
            if k:
                sts.append(st)
        row[vname] = {"ms": round(sts[0]["t_total_ms"], 3), "iters": sts[0]["iters"], "rel_resid": sts[0]["rel_resid"]}
        print(f"bench: periodic n={n} {vname} {row[vname]}", file=sys.stderr, flush=True)
    ctx.set_params(near_cutoff=0.0, near_order=2)
    ctx.set_params(box=L, ewald_mesh=0)
    row["direct_matvec_ms_one_pass"] = round(median_ms(lambda: ctx.mbs_matvec(d["R"], x, y), warm=0, reps=1), 1)
    row["mesh_vs_direct_maxrel"] = float((ym - y).abs().max() / y.abs().max())
    ctx.set_params(box=0.0, ewald_mesh=0)
    out["n%d" % n] = row
    print(f"bench: periodic n={n} direct {row['direct_matvec_ms_one_pass']} ms", file=sys.stderr, flush=True)
    return out


def _host_info():
    """Host cores available to this process and the CPU model (from /proc/cpuinfo)."""
    import platform
    avail = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    # one GPU's share of the host: at most 16 worker processes
    cores = max(1, min(avail, 16, int(os.environ.get("OMP_NUM_THREADS", avail) or avail)))
    return {"cores_available": avail, "cores_used": cores, "cpu_model": model, "nproc": os.cpu_count()}


_CPU = {}


def _cpu_init(R, x, eta, a):
    _CPU.update(R=R, x=x, eta=eta, a=a)


def _cpu_rows_for(seconds):
    """Oracle operator rows (all sources) until the time is up; returns (rows, seconds)."""
    import numpy as np

    from oracle import galerkin
    R, x = _CPU["R"], _CPU["x"]
    prm = galerkin.Params(eta=_CPU["eta"], a=_CPU["a"])
    galerkin.matvec_rows(R, x, np.array([0]), prm)  # builds the symbolic blocks (untimed)
    rng = np.random.default_rng(os.getpid())
    rows = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds:
        galerkin.matvec_rows(R, x, rng.choice(len(R), 2, replace=False), prm)
        rows += 2
    return rows, time.perf_counter() - t0


def _cpu_subset_rows(job):
    """Rows of the oracle's dense system, right-hand side and outputs for a standalone workload."""
    from oracle import galerkin
    kind, w, rows, extra = job
    prm = galerkin.Params(eta=w.eta, a=w.a)
    if kind == "A":
        return galerkin.pair_matrix(w.R, "E", "S", prm, rows), galerkin.rhs(w.R, w.v2s, w.v3t, w.Fe, w.Te, prm, rows)
    return galerkin.outputs(w.R, w.v1s, w.v2s, w.v3t, w.Fe, w.Te, extra, prm, rows)


def _cpu_matvec_rows(job):
    """Rows of the oracle's operator y = A x for one block of receivers (all sources)."""
    from oracle import galerkin
    R, x, rows, eta, a = job
    return galerkin.matvec_rows(R, x, rows, galerkin.Params(eta=eta, a=a))


def _cpu_pool(cores, initargs=None):
    """Spawned worker processes with one BLAS thread each (they run only the oracle, never the GPU)."""
    import multiprocessing as mp
    keys = ("OMP_NUM_THREADS", "OPENBLAS_NUM_THREADS", "MKL_NUM_THREADS")
    saved = {k: os.environ.get(k) for k in keys}
    for k in keys:
        os.environ[k] = "1"
    try:
        if initargs is None:
            return mp.get_context("spawn").Pool(cores)
        return mp.get_context("spawn").Pool(cores, initializer=_cpu_init, initargs=initargs)
    finally:
        for k, v in saved.items():
            if v is None:
                os.environ.pop(k, None)
            else:
                os.environ[k] = v


def cpu_baseline(w, seconds, gpu_beside):
    """The oracle timed on the host's cores (one GPU's share, at most 16):
    * operator rows of the benchmark workload against all its sources, in parallel worker
      processes for about `seconds`: pair-blocks/s (the bench line's unit);
    * the N = 256 workload end to end (dense assembly, LAPACK solve, outputs) as the oracle runs it:
      serial assembly, LAPACK on all used cores;
    * the 2000 spheres nearest the trap centre of the benchmark workload solved as their own system:
      rows assembled in the worker processes, LAPACK solve on all used cores, outputs in the workers.
    * the oracle's whole operator y = A x at 2000 and 10^4 spheres, rows split over the workers.
    gpu_beside: the GPU's times for the same two solves, reported next to them."""
    import numpy as np

    from oracle import galerkin
    from paper_1411_0278_amd import inputs
    host = _host_info()
    cores = host["cores_used"]
    x = np.random.default_rng(0).standard_normal((w.n, 5))
    with _cpu_pool(cores, (w.R, x, w.eta, w.a)) as pool:
        t0 = time.perf_counter()
        res = pool.map(_cpu_rows_for, [seconds] * cores, chunksize=1)
        wall = time.perf_counter() - t0
    rows = sum(r for r, _ in res)
    span = max(s for _, s in res)
    out = {"value": rows * (w.n - 1) / span, "unit": "pair-blocks/s", "cores": cores, "kind": "oracle",
           "sample": f"{rows} rows of the system operator against all {w.n} sources ({rows * (w.n - 1):.3g} "
                     f"pair blocks) in {cores} worker processes, {span:.1f} s each ({wall:.1f} s with start-up), "
                     f"numpy one thread per process",
           "host": host}
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:  # pragma: no cover
        threadpool_limits = None
    limit = threadpool_limits(limits=cores) if threadpool_limits else None
    try:
        w0 = inputs.config0()
        galerkin.solve(inputs.trap_workload(8, 10.0, 0), galerkin.Params(eta=w0.eta, a=w0.a))  # symbolic set-up
        t0 = time.perf_counter()
        galerkin.solve(w0, galerkin.Params(eta=w0.eta, a=w0.a))
        out["config0_end_to_end_s"] = round(time.perf_counter() - t0, 3)
        ws = inputs.nearest_to_origin(w, 2000)
        prm = galerkin.Params(eta=ws.eta, a=ws.a)
        g = galerkin.constants(prm)["gamma"]
        blocks = np.array_split(np.arange(ws.n), 4 * cores)
        with _cpu_pool(cores) as pool:
            t0 = time.perf_counter()
            parts = pool.map(_cpu_subset_rows, [("A", ws, r, None) for r in blocks])
            K = np.concatenate([p[0] for p in parts])
            b = np.concatenate([p[1] for p in parts])
            t_asm = time.perf_counter() - t0
            t1 = time.perf_counter()
            sig = np.linalg.solve(np.eye(5 * ws.n) / g - K, b).reshape(-1, 5)
            t_lu = time.perf_counter() - t1
            t1 = time.perf_counter()
            pool.map(_cpu_subset_rows, [("O", ws, r, sig) for r in blocks])
            t_out = time.perf_counter() - t1
            out["subset2000_standalone_s"] = round(time.perf_counter() - t0, 3)
        out["subset2000_phases_s"] = {"assembly": round(t_asm, 3), "lapack_solve": round(t_lu, 3),
                                      "outputs": round(t_out, 3)}
        # the oracle's whole operator y = A x (every row against every source) at 2000 spheres (the
        # standalone subset) and at 10^4 (the trap box of side 200), rows split over the workers
        out["p2_matvec"] = {}
        for label, wm in (("n2000", ws), ("n10000", inputs.config1())):
            xm = np.random.default_rng(1).standard_normal((wm.n, 5))
            blocks = np.array_split(np.arange(wm.n), 8 * cores)
            with _cpu_pool(cores) as pool:
                # every worker builds its symbolic blocks first (each warm-up task takes seconds, so
                # the pool hands one to every idle worker)
                pool.map(_cpu_matvec_rows, [(wm.R[:8], xm[:8], np.arange(2), wm.eta, wm.a)] * cores, chunksize=1)
                t0 = time.perf_counter()
                ym = np.concatenate(pool.map(_cpu_matvec_rows, [(wm.R, xm, r, wm.eta, wm.a) for r in blocks]))
                t_mv = time.perf_counter() - t0
            assert ym.shape == (wm.n, 5)
            out["p2_matvec"][label] = {"s": round(t_mv, 3), "pair_blocks_per_s": wm.n * (wm.n - 1) / t_mv}
    finally:
        if limit is not None:
            limit.restore_original_limits()
    out["gpu_beside"] = gpu_beside
    return out


def bench_small_solves(a, w):
    """GPU time to solution of the two workloads the CPU oracle also solves end to end: N = 256
    (density 0.004) and the 2000 spheres nearest the trap centre of the benchmark workload, binary64
    GMRES from zero to 1e-10, plain and with the near-field preconditioner (8a, order 2). Fresh
    context, shapes autotuned per size; median of 5 solves after 2 warm-ups (the Arnoldi steps replay
    from graphs from the second solve on)."""
    import statistics

    import torch

    from paper_1411_0278_amd import inputs, mbstokes
    out = {}
    for name, wl in (("config0_n256", inputs.config0()), ("subset2000", inputs.nearest_to_origin(w, 2000))):
        ctx = mbstokes.Context(0)
        d = mbstokes.to_device(wl, "cuda:0")
        ctx.mbs_autotune(d["R"], None)
        args = (d["R"], d["p"], d["v1s"], d["v2s"], d["v3t"], d["Fe"], d["Te"])
        row = {"n": wl.n}
        for label, cut in (("fp64", 0.0), ("fp64_pc", 8.0)):
            ctx.set_params(precision=mbstokes.MBS_FP64, tol=1e-10, near_cutoff=cut, near_order=2)
            times = []
            for k in range(7):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                _, _, _, st = ctx.mbs_solve(*args)
                torch.cuda.synchronize()
                if k >= 2:
                    times.append(1e3 * (time.perf_counter() - t0))
            row[label] = {"ms": round(statistics.median(times), 4), "iters": st["iters"], "rel_resid": st["rel_resid"]}
        ctx.close()
        out[name] = row
        print(f"bench: small solve {name} {row}", file=sys.stderr, flush=True)
    return out


def bench_scale(a):
    """Preconditioned binary64 and mixed solves of one larger trap workload (same density as the
    benchmark), each with the solver's spatial ordering on and off: one timed solve each after the
    context has been set up by an untimed one."""
    import torch

    from paper_1411_0278_amd import inputs, mbstokes
    n = a.scale_n
    side = a.side * (n / a.n) ** (1 / 3)
    t0 = time.perf_counter()
    w = inputs.trap_workload(n, side, a.seed)
    print(f"bench: scale workload n={n} side={side:.1f} built in {time.perf_counter() - t0:.1f} s",
          file=sys.stderr, flush=True)
    d = mbstokes.to_device(w, "cuda:0")
    ctx = mbstokes.Context(0)
    ctx.mbs_autotune(d["R"], None)
    args = (d["R"], d["p"], d["v1s"], d["v2s"], None, d["Fe"], None)
    out = {"n": n, "side": round(side, 2), "near_cutoff": a.near_cutoff, "near_order": a.near_order}
    # binary32 operator error against binary64 with the spheres in the given order and in Morton
    # order (mbs_matvec takes the order it is given; the solver reorders by itself)
    import numpy as np
    lo, hi = w.R.min(0), w.R.max(0)
    q = ((w.R - lo) / (hi - lo + 1e-9) * 1023).astype(np.uint64)
    code = np.zeros(n, dtype=np.uint64)
    for b in range(10):
        for c in range(3):
            code |= ((q[:, c] >> np.uint64(b)) & np.uint64(1)) << np.uint64(3 * b + c)
    err = {}
    x_np = np.random.default_rng(3).standard_normal((n, 5))
    for order_name, perm in (("caller_order", np.arange(n)), ("morton_order", np.argsort(code, kind="stable"))):
        R = torch.as_tensor(np.ascontiguousarray(w.R[perm])).to("cuda:0")
        x = torch.as_tensor(np.ascontiguousarray(x_np[perm])).to("cuda:0")
        y64 = ctx.mbs_matvec(R, x)
        y32 = ctx.mbs_matvec(R, x, precision=mbstokes.MBS_FP32)
        err[order_name] = float(torch.linalg.norm(y32 - y64) / torch.linalg.norm(y64))
    out["f32_operator_rel_err"] = err
    ctx.set_params(precision=mbstokes.MBS_MIXED, near_cutoff=a.near_cutoff, near_order=a.near_order, tol=1e-10)
    ctx.mbs_solve(*args)  # workspace and neighbour lists set up
    for name, prec in (("fp64_pc", mbstokes.MBS_FP64), ("mixed_pc", mbstokes.MBS_MIXED)):
        for order_name, order in (("spatial_order", 1), ("caller_order", -1)):
            ctx.set_params(precision=prec, near_cutoff=a.near_cutoff, near_order=a.near_order, tol=1e-10,
                           spatial_order=order)
            torch.cuda.synchronize()
            t = time.perf_counter()
            _, _, _, st = ctx.mbs_solve(*args)
            torch.cuda.synchronize()
            out[f"{name}_{order_name}"] = {"s": round(time.perf_counter() - t, 3), "iters": st["iters"],
                                           "fp64_matvecs": st["fp64_matvecs"], "fp32_matvecs": st["fp32_matvecs"],
                                           "rel_resid": st["rel_resid"]}
            print(f"bench: scale {name} {order_name} {out[f'{name}_{order_name}']}", file=sys.stderr, flush=True)
    ctx.close()
    return out


def main():
    a = parse()
    if a.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU; runs on several GPUs are not "
                                   "supported (the operator would shard by receiver rows)"}))
        sys.exit(2)
    import torch

    from paper_1411_0278_amd import inputs, mbstokes
    print(f"bench: generating workload n={a.n} side={a.side} seed={a.seed}", file=sys.stderr, flush=True)
    w = inputs.trap_workload(a.n, a.side, a.seed)
    if a.profile_passes:
        profile_passes(a, w)
        return
    if a.profile_matvec:
        profile_matvec(a, w)
        return
    if a.profile_rank3:
        profile_rank3(a)
        return
    if a.profile_mesh:
        profile_mesh()
        return
    if a.profile_geometries:
        ctx = mbstokes.Context(0)
        print(json.dumps({"mode": "profile-geometries", "plane": bench_plane(ctx, a),
                          "periodic": bench_periodic(ctx, a)}), flush=True)
        ctx.close()
        return
    d = mbstokes.to_device(w, "cuda:0")
    # the workload has no external torque and no rank-3 trace slip: pass NULL (= zero)
    d.pop("Te")
    d.pop("v3t")
    ctx = mbstokes.Context(0)
    t_tune = time.perf_counter()
    tiles = ctx.mbs_autotune(d["R"], None)
    print(f"bench: autotuned pair-kernel shapes {tiles} in {time.perf_counter() - t_tune:.1f} s",
          file=sys.stderr, flush=True)
    variants = {}
    extra = {}
    rc = a.near_cutoff
    plan = [("plain_fp64", mbstokes.MBS_FP64, mbstokes.MBS_GUESS_ZERO, 0.0, None),
            ("fp64_diag", mbstokes.MBS_FP64, mbstokes.MBS_GUESS_DIAG, 0.0, None),
            ("mixed_zero", mbstokes.MBS_MIXED, mbstokes.MBS_GUESS_ZERO, 0.0, None),
            ("mixed_diag", mbstokes.MBS_MIXED, mbstokes.MBS_GUESS_DIAG, 0.0, None),
            ("fp64_pc", mbstokes.MBS_FP64, mbstokes.MBS_GUESS_ZERO, rc, None),
            ("mixed_pc", mbstokes.MBS_MIXED, mbstokes.MBS_GUESS_ZERO, rc, None),
            ("mixed_diag_pc", mbstokes.MBS_MIXED, mbstokes.MBS_GUESS_DIAG, rc, None)]
    nets = {}
    if not a.skip_warmstart:
        import tempfile

        from paper_1411_0278_amd import warmstart
        print("bench: training the warm-start networks", file=sys.stderr, flush=True)
        wdir = tempfile.mkdtemp(prefix="mbs_bench_")
        nets = {0: os.path.join(wdir, "geometry.bin"), 1: os.path.join(wdir, "geometry_rhs.bin")}
        reps = warmstart.train_pipeline(ctx, a.warmstart_configs, max(1, a.warmstart_configs // 20),
                                        a.warmstart_epochs,
                                        log=lambda m: print("bench: " + m, file=sys.stderr, flush=True),
                                        feature_sets=(0, 1), weights=nets)
        L = mbstokes.MBS_GUESS_LEARNED
        plan += [("fp64_learned", mbstokes.MBS_FP64, L, 0.0, 0), ("mixed_learned", mbstokes.MBS_MIXED, L, 0.0, 0),
                 ("mixed_learned_pc", mbstokes.MBS_MIXED, L, rc, 0),
                 ("fp64_learned_rhs", mbstokes.MBS_FP64, L, 0.0, 1),
                 ("mixed_learned_rhs", mbstokes.MBS_MIXED, L, 0.0, 1),
                 ("mixed_learned_rhs_pc", mbstokes.MBS_MIXED, L, rc, 1)]
        # surrogate error of the guesses against the converged solution of this workload
        ctx.set_params(precision=mbstokes.MBS_FP64, guess=mbstokes.MBS_GUESS_ZERO, tol=1e-12, near_cutoff=rc,
                       near_order=a.near_order)
        sig = torch.empty((a.n, 5), dtype=torch.float64, device="cuda:0")
        ctx.mbs_solve(d["R"], d["p"], d["v1s"], d["v2s"], None, d["Fe"], None, Sigma=sig)
        err = {"zero": 1.0, "diag": warmstart.surrogate_error(ctx, d, sig, mbstokes.MBS_GUESS_DIAG)}
        for fs, key in ((0, "learned"), (1, "learned_rhs")):
            ctx.mbs_warmstart_load(nets[fs])
            err[key] = warmstart.surrogate_error(ctx, d, sig, L)
        extra["warmstart"] = {"geometry_80": reps[0], "geometry_rhs_160": reps[1], "surrogate_rel_err": err}
    elif "learned" in a.headline:
        a.headline = "mixed_pc"
    for name, prec, guess, cut, net in plan:
        if net is not None:
            ctx.mbs_warmstart_load(nets[net])
        steps = a.steps if name in (a.headline, "plain_fp64") else max(1, min(a.steps, 2))
        variants[name] = time_variant(ctx, d, mbstokes, name, prec, guess, steps, a.warmup, cut, a.near_order)
        variants[name]["near_cutoff"] = cut
        variants[name]["near_order"] = a.near_order if cut > 0 else 0
    if not a.skip_batched:
        extra["batched"] = bench_batched(ctx, a)
    if not a.skip_kernels:
        extra["pair_passes"] = bench_kernels(ctx, a)
    if not a.skip_stepper:
        extra["stepper"] = bench_stepper(ctx, a)
        extra["paper_trap"] = bench_paper_trap(ctx, a)
        extra["paper_trap"]["two_particle"] = bench_two_particle_orbits(ctx)
    if not a.skip_rank3:
        extra["rank3"] = bench_rank3(ctx, a)
    if not a.skip_plane:
        extra["plane"] = bench_plane(ctx, a)
    if not a.skip_periodic:
        extra["periodic"] = bench_periodic(ctx, a)
    if a.scale_n > 0:
        extra["scale"] = bench_scale(a)
    head = variants[a.headline]
    out = {
        "metric": METRIC,
        "value": head["pair_blocks_per_s"],
        "unit": "pair-blocks/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if head["n_op32"] else "f64",
        "data": "synthetic",
        "config": {"workload": f"trap spheres N={a.n} cube side {a.side:g} seed {a.seed}, "
                               f"slip V1s=p V2s=3(pp-I/3), F=-0.5R, solve to 1e-10",
                   "n": a.n, "headline": a.headline, "tol": 1e-10, "tiles": list(tiles),
                   "near_cutoff": rc, "near_order": a.near_order},
        "roofline": roofline(head, a.n),
        "time_to_1e-10_ms": {k: round(v["ms_per_step"], 3) for k, v in variants.items()},
        "iterations": {k: v["iters"] for k, v in variants.items()},
        "speedup_vs_plain_fp64": round(variants["plain_fp64"]["ms_per_step"] / head["ms_per_step"], 4),
        "variants": variants,
        **extra,
    }
    ctx.close()
    if not a.skip_cpu:
        beside = bench_small_solves(a, w)
        print("bench: timing the CPU oracle", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w, a.cpu_seconds, beside)
    else:
        out["cpu_baseline"] = None
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
