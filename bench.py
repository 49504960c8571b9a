#!/usr/bin/env python3
"""Benchmark of the phase-screen + Fresnel propagation hot path on one MI355X.

One step is the whole batched path on synthetic input: 8 phase screens of
8192^2 pixels (Kolmogorov, R_diff = 30 px at 650 nm), each propagated at 32
wavelengths spanning 400-900 nm (R_F = 90 px at 650 nm, R_F ~ sqrt(lambda),
phase ~ 1/lambda), co-added, and smeared by uniform stellar disks of radius
{0.5, 1, 2, 4} R_F.  The metric is grid points x wavelengths per second.

Prints one JSON line on stdout; progress goes to stderr.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline] [--no-secondary]
                  [--secondary NAME,...]
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
FP32_VECTOR_PEAK_TFLOPS = 157.3  # MI355X FP32 vector, published (packed FMA)
# Algorithmic bytes of the whole batched step per grid point x wavelength:
# per realisation the screen 20 B/pt, per wavelength 16 B/pt (the first
# pass's write and the second pass's read of the one exchange per 2-D
# transform), the screen read once 4 B/pt, the co-added pattern 4 B/pt and
# the four smears about 96 B/pt: 636 B/pt over 32 wavelengths.
STEP_BYTES_PER_PT_LAMBDA = 636.0 / 32.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


# device sources of the row-pass kernels (the FFT passes) and of the
# transposes, the two kernel families that dominate the step
ROW_KERNEL_SOURCES = ("device_common.hpp", "fft_plan.hpp", "lds_layout.hpp", "row_program.h", "row_kernel.hpp",
                      "row_launch.h", "transpose_tile.hpp",
                      "row_inst.hip", "twiddles.cpp")
AUX_KERNEL_SOURCES = ("device_common.hpp", "aux_kernels.h", "aux_kernels.hip", "transpose_tile.hpp")


def kernel_sources(kernel: str):
    return AUX_KERNEL_SOURCES if kernel.startswith("transpose_") else ROW_KERNEL_SOURCES


def source_hash(kernel: str = "row_") -> str:
    """Hash of the device sources of `kernel` (row passes or transposes);
    ties a stored counter profile to the kernel it was taken on."""
    h = hashlib.sha256()
    for name in kernel_sources(kernel):
        with open(os.path.join(ROOT, "paper_1301_0514_amd", "csrc", name), "rb") as fh:
            h.update(name.encode())
            h.update(fh.read())
    return h.hexdigest()[:16]


def stored_profile(kernel: str, plan_variant: int | None = None) -> dict:
    """The key = value lines of the committed rocprofv3 --pmc summary of
    `kernel` (profiles/traffic_*.txt), if it was taken on the current kernel
    sources and, for row passes, FFT plan variant; else {}."""
    want = source_hash(kernel)
    if not kernel.startswith("row_"):
        plan_variant = None
    for p in glob.glob(os.path.join(ROOT, "profiles", "traffic_*.txt")):
        vals = {}
        with open(p) as fh:
            for line in fh:
                if "=" in line and not line.lstrip().startswith("#"):
                    k, v = (t.strip() for t in line.split("=", 1))
                    vals[k] = v
        if plan_variant is not None and vals.get("plan_variant") not in (None, str(plan_variant)):
            continue
        if vals.get("kernel") == kernel and vals.get("source_sha256") == want:
            return vals
    return {}


def stored_traffic(kernel: str, plan_variant: int | None = None):
    """HBM bytes per launch of `kernel` (FETCH_SIZE + WRITE_SIZE, calibrated)
    from its stored profile, or None."""
    vals = stored_profile(kernel, plan_variant)
    try:
        return float(vals["fetch_bytes_per_launch"]) + float(vals["write_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def stored_float(kernel: str, key: str, plan_variant: int | None = None):
    try:
        return float(stored_profile(kernel, plan_variant)[key])
    except (KeyError, ValueError):
        return None


def cpu_baseline_configs(O, presets, log) -> list:
    """The FP64 oracle timed on the host's cores, per named configuration,
    all cores and one thread: the median of three runs where one run takes
    under 10 s, one run otherwise; a single-thread run estimated above 60 s
    (all-core time x threads) is skipped and the estimate is reported."""
    import numpy as np

    all_cores = O.num_threads()

    def med(fn, budget_s):
        t = []
        for _ in range(3):
            t0 = time.perf_counter()
            fn()
            t.append(time.perf_counter() - t0)
            if t[0] >= budget_s:
                break
        return float(np.median(t)), len(t)

    p1 = presets.PLAIN_FP64
    c2 = presets.SINGLE_4096[0]
    c3 = [c for c in presets.PAPER_SCALE if c.N == 10000 and abs(c.beta - 11 / 3) < 1e-9][0]
    g = presets.GRAD_2048

    def plain():
        O.propagate(O.screen(p1.N, p1.R, p1.beta, 1, 0), p1.rho)

    def single4096():
        O.propagate(O.screen(c2.N, c2.R, c2.beta, 1, 0), c2.rho)

    def paper10000():
        O.propagate(O.screen(c3.N, c3.R, c3.beta, 1, 0), c3.rho)

    def grad2048():
        phi = O.screen(g.N, g.R, g.beta, 1, 0)
        I = O.propagate(phi, g.rho)
        O.propagate_vjp(phi, g.rho, 1.0, 2.0 * (I - 1.0))

    plan = [("plain FP64 256^2: screen + propagation", p1.N ** 2, plain),
            ("single wavelength 4096^2 (R_diff 8 px): one screen + propagation", c2.N ** 2, single4096),
            ("paper scale 10000^2 (beta 11/3): one screen + propagation", c3.N ** 2, paper10000),
            ("differentiation 2048^2: one screen, propagation and adjoint", g.N ** 2, grad2048)]
    rows = []
    for name, pts, fn in plan:
        row = {"config": name, "unit": "grid points/s"}
        O.set_num_threads(all_cores)
        t, k = med(fn, 10.0)
        row["all_cores"] = {"threads": all_cores, "runs": k, "median_s": t, "value": pts / t}
        est = t * all_cores
        if est <= 60.0:
            O.set_num_threads(1)
            t1, k1 = med(fn, 10.0)
            row["single_thread"] = {"threads": 1, "runs": k1, "median_s": t1, "value": pts / t1}
        else:
            row["single_thread"] = {"threads": 1, "skipped": "estimated %.0f s per run" % est}
        log("cpu baseline %s: %.2f s on %d threads%s" % (
            name, t, all_cores, "" if "median_s" not in row["single_thread"] else
            ", %.2f s on one" % row["single_thread"]["median_s"]))
        rows.append(row)
    O.set_num_threads(all_cores)
    return rows


# the secondary configurations timed after the step, in order
SECONDARY = ["batched_vs_plain", "single4096", "paper_scale", "aperture8192", "m_theory", "structure16000",
             "ks20000", "grad2048"]


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--secondary", default="all",
                    help="comma-separated secondary configurations to run (default all): " + ",".join(SECONDARY))
    ap.add_argument("--no-graph", dest="graph", action="store_false",
                    help="time eager calls instead of replays of the captured step")
    ap.add_argument("--calib-copy-gb", type=float, default=0.0,
                    help="first copy this many GB device-to-device with one plain copy kernel, as the "
                         "reference of known size for the FETCH_SIZE/WRITE_SIZE counters")
    args = ap.parse_args(argv)
    if args.secondary != "all":
        bad = [n for n in args.secondary.split(",") if n not in SECONDARY]
        if bad:
            print("unknown secondary configuration(s) %s; choose from %s" % (bad, ",".join(SECONDARY)),
                  file=sys.stderr)
            return 2
    if args.gpus != 1:
        print("bench.py measures the single-GPU path only (one MI355X); --gpus %d is not supported" % args.gpus,
              file=sys.stderr)
        return 2

    import numpy as np
    import torch

    sys.path.insert(0, ROOT)
    from paper_1301_0514_amd import presets, scint

    scint.load_library()  # raises if the HIP library is not built
    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        return 1
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)

    if args.calib_copy_gb > 0:
        n = int(args.calib_copy_gb * 1e9) // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: %d bytes read, %d bytes written" % (4 * n, 4 * n))
        del src, dst

    # the library's default workspace is a quarter of the free HBM, at most
    # 32 GiB; this run owns the GPU and gives it 80 GiB, so that the
    # propagation runs as 8 pipelined jobs of 32 wavelengths (64 GiB; 3 %
    # faster than the default's 8-wavelength jobs) and the 20000^2 K_s run
    # below as 4 jobs of 6 wavelengths (73 GiB)
    workspace_gib = 80
    scint.set_workspace_budget(workspace_gib << 30)

    cfg = presets.POLY_8192
    N, n_real, lams, radii = cfg.N, cfg.n_real, cfg.lambdas, cfg.smear_radii
    n_lam = len(lams)
    phi = torch.empty((n_real, N, N), dtype=torch.float32, device=dev)
    I_sum = torch.empty_like(phi)
    I_ext = torch.empty((n_real, len(radii), N, N), dtype=torch.float32, device=dev)

    def step():
        scint.ps_generate(N, 1.0, cfg.R_ref, cfg.beta, cfg.seed, 0, n_real, out=phi)
        scint.illumination_polychromatic(phi, 1.0, cfg.z, cfg.lam_ref, lams, out=I_sum)
        scint.source_smear(I_sum, 1.0, radii, out=I_ext)

    log("warmup %d steps (N=%d, %d screens, %d wavelengths, %d radii)" % (args.warmup, N, n_real, n_lam, len(radii)))
    # the whole step (screens, all wavelengths, smears) is captured into one
    # HIP graph after the warm-up; the timed region replays it
    stream = torch.cuda.Stream()
    graph = None
    if args.graph:
        graph, stream = scint.capture_graph(step, warmup=args.warmup, stream=stream)
    else:
        with torch.cuda.stream(stream):
            for _ in range(args.warmup):
                step()
    torch.cuda.synchronize()

    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    with torch.cuda.stream(stream):
        ev0.record()
        for _ in range(args.steps):
            if graph is not None:
                graph.replay()
            else:
                step()
        ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_total = ev0.elapsed_time(ev1)
    ms_step = ms_total / args.steps
    units = float(N) * N * n_lam * n_real
    value = units / (ms_step / 1e3)
    log("timed %d steps (%s): %.2f ms/step (wall %.2f s)" % (args.steps, "graph replay" if graph else "eager",
                                                          ms_step, wall))
    # the same step timed replay by replay (events around each), reported
    # as the median beside the bracketed mean above
    n_rep = max(20, args.steps)
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(n_rep + 1)]
    torch.cuda.synchronize()
    with torch.cuda.stream(stream):
        evs[0].record()
        for i in range(n_rep):
            if graph is not None:
                graph.replay()
            else:
                step()
            evs[i + 1].record()
    torch.cuda.synchronize()
    per_rep = sorted(evs[i].elapsed_time(evs[i + 1]) for i in range(n_rep))
    replays = {"n": n_rep, "median_ms": float(np.median(per_rep)), "min_ms": per_rep[0], "max_ms": per_rep[-1]}
    log("%d single replays: median %.2f ms (%.2f-%.2f)" % (n_rep, replays["median_ms"], per_rep[0], per_rep[-1]))
    # per-kernel durations: the same step run eagerly with the library's
    # event timing on (events cannot be recorded per kernel inside a replay)
    scint.timing_enable(True)
    with torch.cuda.stream(stream):
        for _ in range(args.steps):
            step()
    torch.cuda.synchronize()
    rep = scint.timing_report()
    scint.timing_enable(False)
    ms_eager = sum(v["ms"] for v in rep.values()) / args.steps
    log("instrumented eager steps: %.2f ms of kernels per step" % ms_eager)

    # dominant kernel and its roofline.  `bytes` are the algorithmic bytes
    # of each launch: every array the method reads or writes in that pass,
    # once (for the first propagation pass 8 B per point x wavelength
    # written plus the 4-B screen read once; for the second 8 B per point x
    # wavelength read plus the 4-B pattern written once; transposes zero).
    # `schedule_bytes` are the operands as the launches move them (loop
    # re-reads, transposes), reported beside them.
    dom = max(rep.items(), key=lambda kv: kv[1]["ms"])
    dname, d = dom
    avg_ms = d["ms"] / d["launches"]
    bytes_per_launch = d["bytes"] / d["launches"]
    sched_per_launch = d["schedule_bytes"] / d["launches"]
    flops_per_launch = d["flops"] / d["launches"]
    gbps = bytes_per_launch / (avg_ms / 1e3) / 1e9
    tflops = flops_per_launch / (avg_ms / 1e3) / 1e12
    # plan variant the dominant kernel ran with (row passes are named row_<program>_<dtype>_N<size>)
    try:
        dom_variant = scint.plan_variant(int(dname.rsplit("_N", 1)[1]), torch.float32)[0]
    except (IndexError, ValueError, scint.ScintError):
        dom_variant = None
    traffic = stored_traffic(dname, dom_variant)
    # the other two ceilings from the stored SQ counters of the same kernel:
    # VALU issue (wave64 instructions x 4 cycles over 1024 SIMDs x active
    # cycles) and LDS bank conflicts per LDS-active cycle
    valu_issue = stored_float(dname, "valu_issue_frac", dom_variant)
    lds_conflict = stored_float(dname, "lds_bank_conflict_frac", dom_variant)

    def per_launch(v, key):
        return v[key] / v["launches"]

    kernels = {k: {"ms_per_step": v["ms"] / args.steps, "launches_per_step": v["launches"] / args.steps,
                   "avg_launch_ms": v["ms"] / v["launches"],
                   "algorithmic_GBps": per_launch(v, "bytes") / (v["ms"] / v["launches"] / 1e3) / 1e9,
                   "schedule_GBps": per_launch(v, "schedule_bytes") / (v["ms"] / v["launches"] / 1e3) / 1e9,
                   "algorithmic_TFLOPs": per_launch(v, "flops") / (v["ms"] / v["launches"] / 1e3) / 1e12}
               for k, v in sorted(rep.items(), key=lambda kv: -kv[1]["ms"])}
    for k, v in kernels.items():
        log("  %-40s %8.3f ms/step  %6.1f launches  %7.1f GB/s alg  %7.1f GB/s sched  %6.2f TFLOP/s" % (
            k, v["ms_per_step"], v["launches_per_step"], v["algorithmic_GBps"], v["schedule_GBps"],
            v["algorithmic_TFLOPs"]))
    # the path is priced against HBM by its algorithmic bytes; the VALU issue
    # fraction (from the kernel's SQ counters) is the ceiling that binds the
    # FFT passes, and the schedule's own bytes show the traffic it moves
    roofline = {"bound": "hbm", "kernel": dname, "achieved": gbps, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": gbps / HBM_PEAK_GBS, "traffic": traffic,
                "algorithmic_bytes_per_launch": bytes_per_launch, "avg_launch_ms": avg_ms,
                "bytes_per_unit": "8 B per grid point x wavelength + 4 B per grid point (first propagation "
                                  "pass: field written per wavelength, screen read once)",
                "schedule_bytes_per_launch": sched_per_launch,
                "schedule_GBps": sched_per_launch / (avg_ms / 1e3) / 1e9,
                "algorithmic_flops_per_launch": flops_per_launch, "alu_achieved_TFLOPs": tflops,
                "alu_frac": tflops / FP32_VECTOR_PEAK_TFLOPS,
                "valu_issue_frac": valu_issue, "lds_bank_conflict_frac": lds_conflict}
    step_sched = sum(v["schedule_bytes"] for v in rep.values()) / args.steps
    step_alg = STEP_BYTES_PER_PT_LAMBDA * float(N) * N * n_lam * n_real

    out = {
        "metric": "screen+Fresnel grid points/sec (x lambda) at 1 MI355X; % HBM roofline; RMS err vs FP64",
        "value": value,
        "unit": "grid points*lambda/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded Philox screens; no dataset exists for this method)",
        "config": {"workload": "poly8192: 8 screens of 8192^2, 32 wavelengths 400-900 nm co-added, "
                               "4 disk smears {0.5,1,2,4} R_F; R_F(650 nm)=90 px, R_diff(650 nm)=30 px, beta=11/3",
                   "N": N, "n_real": n_real, "n_lambda": n_lam, "smear_radii_px": radii,
                   "workspace_budget_GiB": workspace_gib, "parallelism": "single GPU"},
        "roofline": roofline,
        "timing": "graph replay of the whole step" if graph is not None else "eager calls",
        "replays": replays,
        "kernel_ms_per_step_eager": ms_eager,
        "step_algorithmic_GB": step_alg / 1e9,
        "step_algorithmic_bytes_per_pt_lambda": STEP_BYTES_PER_PT_LAMBDA,
        "step_frac_of_hbm_roofline": (step_alg / (ms_step / 1e3)) / (HBM_PEAK_GBS * 1e9),
        "step_ms_at_hbm_roofline": step_alg / (HBM_PEAK_GBS * 1e9) * 1e3,
        "step_schedule_GB": step_sched / 1e9,
        "step_schedule_GBps": step_sched / (ms_step / 1e3) / 1e9,
        "kernels": kernels,
    }

    # FFT plans the tuner chose (times: one propagation row pass per plan)
    plans = {}
    for n_ in (N, 2048, 4096, 10000, 16384):
        v_, ms_ = scint.plan_variant(n_)
        plans[str(n_)] = {"variant": v_, "tuner_ms": ms_}
    out["fft_plans"] = plans

    # ---------------------------------------------------------------- CPU baseline + accuracy
    if not args.no_cpu_baseline:
        import oracle as O

        O.build()
        # a bounded sample (about 10 s on 16 host threads): the screen and 8
        # of the wavelengths, spread over the band
        sel = sorted({round(i * (n_lam - 1) / 7) for i in range(8)})
        log("cpu baseline: oracle screen + %d of %d wavelengths at %d^2 (FP64)" % (len(sel), n_lam, N))
        t0 = time.perf_counter()
        phi_ref = O.screen(N, cfg.R_ref, cfg.beta, cfg.seed, 0)
        I_refs = []
        for j in sel:
            rho = O.fresnel_radius_px(1.0, lams[j], cfg.z)
            I_refs.append(O.propagate(phi_ref, rho, cfg.lam_ref / lams[j]))
        cpu_s = time.perf_counter() - t0
        cpu_units = float(N) * N * len(sel)
        out["cpu_baseline"] = {"value": cpu_units / cpu_s, "unit": "grid points*lambda/s",
                               "cores": O.num_threads(), "kind": "oracle",
                               "sample": "FP64 oracle: one %d^2 screen + its propagation at %d of the %d "
                                         "wavelengths (%s nm), %.1f s"
                                         % (N, len(sel), n_lam, ", ".join("%.0f" % (lams[j] * 1e9) for j in sel),
                                            cpu_s)}
        # accuracy of the FP32 path against the FP64 oracle on the same sample
        g_phi = phi[0:1].double().cpu().numpy()[0]
        d = g_phi - phi_ref
        acc = {"phi_rms_rel": float(np.sqrt(np.mean(d * d)) / np.sqrt(np.mean(phi_ref * phi_ref)))}
        erms, emax = [], []
        for j, I_ref in zip(sel, I_refs):
            Ig = scint.illumination_polychromatic(phi[0:1], 1.0, cfg.z, cfg.lam_ref, [lams[j]])
            Ig = Ig.double().cpu().numpy()[0]
            m = I_ref.mean()
            diff = Ig - I_ref
            erms.append(float(np.sqrt(np.mean(diff * diff)) / m))
            emax.append(float(np.abs(diff).max() / m))
        acc["I_rms_rel_max_over_lambda"] = max(erms)
        acc["I_max_rel_max_over_lambda"] = max(emax)
        acc["bar"] = {"rms": 2e-5, "max": 1e-3}
        out["accuracy_vs_fp64_oracle"] = acc
        log("accuracy: phi rms %.2e, I rms %.2e, I max %.2e" % (acc["phi_rms_rel"], max(erms), max(emax)))
        del phi_ref, I_refs
        out["cpu_baseline"]["configs"] = cpu_baseline_configs(O, presets, log)
        O.set_num_threads(out["cpu_baseline"]["cores"])


    # ---------------------------------------------------------------- secondary configurations
    if not args.no_secondary:
        sec = {}
        chosen = SECONDARY if args.secondary == "all" else args.secondary.split(",")

        def want(name):
            return name in chosen

        def timed(fn, reps):
            fn()
            torch.cuda.synchronize()
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(reps):
                fn()
            b.record()
            torch.cuda.synchronize()
            return a.elapsed_time(b) / reps

        if want("batched_vs_plain"):
            # plain single-wavelength path, 32 calls, against the batched call (one screen)
            one = phi[0:1]
            acc_plain = torch.empty_like(one)
            tmp = torch.empty_like(one)

            def plain():
                acc_plain.zero_()
                for lam in lams:
                    scint.fresnel_propagate(one, 1.0, lam, cfg.z, cfg.lam_ref / lam, out=tmp)
                    acc_plain.add_(tmp, alpha=1.0 / n_lam)

            batched_out = torch.empty_like(one)

            def batched():
                scint.illumination_polychromatic(one, 1.0, cfg.z, cfg.lam_ref, lams, out=batched_out)

            t_plain = timed(plain, 2)
            t_batched = timed(batched, 3)
            diff = (acc_plain - batched_out).abs().max().item()
            sec["batched_vs_plain_single_lambda"] = {"ms_plain_32_calls": t_plain, "ms_batched": t_batched,
                                                      "speedup": t_plain / t_batched, "max_abs_diff": diff}
            log("batched vs plain: %.2f ms vs %.2f ms (x%.2f)" % (t_batched, t_plain, t_plain / t_batched))
            del acc_plain, tmp, batched_out

        if want("single4096"):
            # single wavelength 4096^2, one screen+propagation per call, 12 calls
            p4 = presets.SINGLE_4096
            Iout = torch.empty((1, 4096, 4096), dtype=torch.float32, device=dev)

            def single4096():
                for c in p4:
                    for s in c.seeds:
                        r = scint.load_library().ps_screen_fresnel(
                            c.N, 1.0, c.R, c.beta, s, 0, 1, c.lam, c.z, 0, None,
                            scint._ptr(Iout), None, scint._stream(dev))
                        if r != 0:
                            raise RuntimeError("ps_screen_fresnel failed %d" % r)

            t4 = timed(single4096, 3)
            sec["single_4096_screen_fresnel"] = {"ms_per_12_calls": t4, "pt_per_s": 12 * 4096.0 ** 2 / (t4 / 1e3)}
            log("4096^2 single lambda: %.3f ms per call" % (t4 / 12))
            del Iout

        if want("paper_scale"):
            for c in presets.PAPER_SCALE:
                if abs(c.beta - 11 / 3) > 1e-9:
                    continue
                out_t = torch.empty((1, c.N, c.N), dtype=torch.float32, device=dev)

                def paper():
                    r = scint.load_library().ps_screen_fresnel(c.N, 1.0, c.R, c.beta, 1, 0, 1, c.lam, c.z, 0, None,
                                                                scint._ptr(out_t), None, scint._stream(dev))
                    if r != 0:
                        raise RuntimeError("ps_screen_fresnel failed %d" % r)

                tp = timed(paper, 3)
                sec["paper_%d_screen_fresnel" % c.N] = {"ms_per_call": tp, "pt_per_s": c.N ** 2 / (tp / 1e3)}
                log("%d^2 single lambda: %.3f ms" % (c.N, tp))
                del out_t

        if want("aperture8192"):
            # aperture mode (one-FFT numerics with the window), 8192^2 at the
            # conjugate relation N delta^2 = lambda z, on the bench's first screen
            Na = 8192
            phia = phi[:1] if phi.shape[-1] == Na else torch.zeros((1, Na, Na), dtype=torch.float32, device=dev)
            lam_a = 2.162e-6
            Ia = torch.empty_like(phia)

            def aperture():
                scint.fresnel_aperture(phia, 1.0, lam_a, Na / lam_a, margin_rf=10.0, out=Ia)

            ta = timed(aperture, 3)
            sec["aperture_8192_fresnel"] = {"ms_per_call": ta, "pt_per_s": Na ** 2 / (ta / 1e3)}
            log("aperture mode 8192^2: %.3f ms" % ta)
            del Ia

        if want("m_theory"):
            # m against Eq. xparam (Sect. 4.1, Fig. mx), periodic mode on the
            # paper's geometry, 16 realisations per configuration
            from statistics import mean as _mean
            from paper_1301_0514_amd import sweep
            t0 = time.perf_counter()
            pts = sweep.m_versus_theory(8192, 25.0, 2.162e-6, 160 * sweep.PC, 1000 * sweep.PC, [200, 300, 400, 500],
                                        [0.25, 0.5], n_real=16, mode="periodic")
            t_sweep = time.perf_counter() - t0
            rows = []
            for rd in (200, 300, 400, 500):
                for rs in (0.25, 0.5):
                    g = [p for p in pts if p.r_diff_km == rd and p.r_s_rsun == rs]
                    rows.append({"r_diff_km": rd, "r_s_rsun": rs, "m_theory": g[0].m_theory,
                                 "m_mean": _mean(p.m for p in g), "ratio_mean": _mean(p.m / p.m_theory for p in g),
                                 "n_ref": g[0].n_ref})
            sec["m_versus_theory_8192"] = {"seconds": t_sweep, "patterns": len(pts), "rows": rows}
            log("m sweep: %d patterns in %.2f s" % (len(pts), t_sweep))

        if want("structure16000"):
            # structure-function check of a 16000^2 screen (Sect. 3.1.1): the
            # paper's 540-km configuration (28.85 km pixels, R_diff = 500 km)
            Ns = 16000
            phis = scint.ps_generate(Ns, 28.85, 500.0, 11 / 3, 1, 0, 1, torch.float32, device=dev)
            t0 = time.perf_counter()
            _, rrec = scint.structure_function(phis, 28.85)
            t_sf = time.perf_counter() - t0
            sec["structure_function_16000"] = {"seconds_incl_first_use": t_sf, "rdiff_rec_km": rrec[0],
                                               "rdiff_input_km": 500.0}
            t0 = time.perf_counter()
            scint.structure_function(phis, 28.85)
            sec["structure_function_16000"]["seconds"] = time.perf_counter() - t0
            log("structure function 16000^2: R_diff^rec %.1f km (input 500 km), %.3f s" % (
                rrec[0], sec["structure_function_16000"]["seconds"]))
            del phis

        if want("ks20000"):
            # the paper's scale: one 20000^2 screen through the 21-wavelength K_s
            # band (Sect. 3.2.4)
            kc = presets.PAPER_KS_20000
            phik = scint.ps_generate(kc.N, kc.delta, kc.r_diff, 11 / 3, kc.seed, 0, 1, torch.float32, device=dev)
            Ik = torch.empty_like(phik)

            def ks_band():
                scint.illumination_polychromatic(phik, kc.delta, kc.z, kc.lam_ref, kc.lambdas(), out=Ik)

            tk = timed(ks_band, 2)
            sec["paper_ks_20000_21_lambda"] = {"ms_per_call": tk,
                                               "pt_per_s": kc.N ** 2 * kc.n_lambda / (tk / 1e3),
                                               "m": scint.ps_modulation_index(Ik)[0]}
            log("K_s band 20000^2 x 21 lambda: %.1f ms, m = %.3f" % (tk, sec["paper_ks_20000_21_lambda"]["m"]))
            del phik, Ik

        if want("grad2048"):
            # forward + adjoint, 16 x 2048^2: the forward keeps the field as the
            # adjoint's checkpoint; the recomputing adjoint is timed beside it
            g = presets.GRAD_2048
            nr = presets.GRAD_N_REAL
            It = torch.empty((nr, g.N, g.N), dtype=torch.float32, device=dev)
            for i in range(nr):
                It[i:i + 1] = scint.ps_screen_fresnel(g.N, 1.0, g.R, g.beta, presets.GRAD_TARGET_SEED0 + i, g.lam, g.z)
            gphi = torch.empty_like(It)
            Igr = torch.empty_like(It)
            phig = torch.empty_like(It)
            fieldg = torch.empty((nr, g.N, g.N, 2), dtype=torch.float32, device=dev)

            def fwd_adj(checkpoint):
                lib = scint.load_library()
                st = scint._stream(dev)
                r = lib.ps_screen_fresnel(g.N, 1.0, g.R, g.beta, 1, 0, nr, g.lam, g.z, 0, scint._ptr(phig),
                                          scint._ptr(Igr), scint._ptr(fieldg) if checkpoint else None, st)
                if r != 0:
                    raise RuntimeError("ps_screen_fresnel failed %d" % r)
                _, gI = scint.ps_l2_loss(Igr, It)
                scint.fresnel_propagate_vjp(phig, 1.0, g.lam, g.z, gI, 1.0, out=gphi,
                                            field=fieldg if checkpoint else None)

            tg = timed(lambda: fwd_adj(True), 3)
            tr = timed(lambda: fwd_adj(False), 3)
            # algorithmic bytes: forward 44 B/pt (screen, field and pattern
            # kept) + adjoint 36 B/pt
            sec["grad_2048x16_forward_adjoint"] = {"ms_per_step": tg, "pt_per_s": nr * g.N ** 2 / (tg / 1e3),
                                                   "ms_per_step_recomputing_adjoint": tr,
                                                   "frac_of_hbm_roofline_80B_per_pt":
                                                       80.0 * nr * g.N ** 2 / (tg / 1e3) / (HBM_PEAK_GBS * 1e9)}
            log("16 x 2048^2 forward+adjoint: %.3f ms with the checkpoint, %.3f ms recomputing" % (tg, tr))
        out["secondary"] = sec

    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
