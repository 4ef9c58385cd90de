#!/usr/bin/env python3
"""DS-GRFT throughput benchmark on one MI355X.

Workload: the M = 1024 search (N = 4096 range bins, P = 2, v in +-600 m/s,
a in +-50 m/s^2; 2460 coarse cells x 10^4 fine cells x 4096 rows = 1.008e11
cells, 1.03e14 cells*pulses) on a seeded synthetic echo with 8 targets at
-20 dB per-pulse SNR.  One step = the whole DS-GRFT hot path over the echo
(coarse tables, gather + de-ramp, fine search with fused |.|^2/argmax,
LRT detection with peak parameters), echo already resident in HBM.

Prints one JSON line (rank 0, N = 1 only).
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

METRIC = "DS-GRFT cells·pulses/s (M=1024); MFMA vs FP32 speedup at rel err≤1e-3"
PEAK_TFLOPS = {"f16": 2500.0, "f16_3m": 2500.0, "f16_sym": 2500.0, "bf16": 2500.0,
               "bf16_glo": 2500.0, "bf16_sym": 2500.0, "fp8": 5000.0, "fp8_sym": 5000.0,
               "f32": 157.3, "f32fft": 157.3}
DTYPE = {"f16_3m": "f16", "f16_sym": "f16", "f32fft": "f32", "bf16_glo": "bf16",
         "bf16_sym": "bf16", "fp8_sym": "fp8"}
KERNEL = {"f16_3m": "k_fine_mfma3 (f16, three real products per complex product)",
          "f16_sym": "k_fine_mfma_sym<f16> (f16, fine cells in conjugate pairs, four real "
                     "products per pair)",
          "bf16_sym": "k_fine_mfma_sym<bf16> (bf16 split parts over conjugate pairs of fine "
                      "cells, four real products per pair and part)",
          "fp8_sym": "k_fine_mfma_sym8 (e4m3 split parts over conjugate pairs of fine cells, "
                     "four real products per pair and part)"}
FORM_TEXT = {"f16_3m": "f16 MFMA, three real products per complex product (Gauss), split 1, "
                       "FP32 accumulation",
             "f16_sym": "f16 MFMA, fine cells in conjugate pairs (four real products for the "
                        "cells at +d and -d), split 1, FP32 accumulation",
             "bf16_sym": "bf16 MFMA over conjugate pairs of fine cells, split parts Fh Gh + Fh Gl "
                         "(+ Fl Gh for split 3), FP32 accumulation",
             "fp8_sym": "e4m3 MFMA with block scales over conjugate pairs of fine cells, split "
                        "parts Fh Gh + Fl Gh + Fh Gl (+ Fl Gl for split 4), FP32 accumulation",
             "f32fft": "FP32, fine velocities by slow-time FFT"}
SWEEP = (("f16_sym", 1), ("f16_3m", 1), ("f16", 1), ("f16", 2), ("f16", 3), ("f16", 4),
         ("bf16_sym", 2), ("bf16_sym", 3), ("bf16", 1), ("bf16", 2), ("bf16_glo", 2),
         ("bf16", 3), ("bf16", 4), ("fp8_sym", 3), ("fp8_sym", 4), ("fp8", 1), ("fp8", 2),
         ("fp8", 3), ("fp8", 4),
         ("f32fft", 1))
SWEEP_STEPS = 3
HBM_GBPS = 8000.0
FINE_SRC = os.path.join(ROOT, "paper_2403_06788_amd", "csrc", "fine_mfma.hip")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_hash() -> str:
    return hashlib.sha256(open(FINE_SRC, "rb").read()).hexdigest()[:16]


def _recorded(form, split, kind):
    """A committed rocprofv3 counter summary of the fine kernel
    (profiles/fine_mfma_<form>x<split>_m1024_<kind>.json, or the older name
    without the split), if it was taken on the current kernel source."""
    for name in (f"fine_mfma_{form}x{split}_m1024_{kind}.json", f"fine_mfma_{form}_m1024_{kind}.json"):
        try:
            d = json.load(open(os.path.join(ROOT, "profiles", name)))
        except (OSError, ValueError):
            continue
        if d.get("kernel_sha") == kernel_hash() and d.get("form") == f"{form}x{split}":
            return d
    return None


def recorded_traffic(form, split):
    """Per-launch HBM traffic of the fine kernel from the committed rocprofv3
    counter summary, or None if absent or taken on another kernel version."""
    d = _recorded(form, split, "traffic")
    return None if d is None else d.get("bytes_per_launch")


def recorded_mfma_util(form, split):
    """Executed-MFMA utilisation of the fine kernel (MFMA-busy cycles over
    active cycles x SIMDs) from the committed rocprofv3 counter summary, or
    None if absent or taken on another kernel version."""
    d = _recorded(form, split, "mfma_util")
    return None if d is None else round(d.get("mfma_util"), 4)


def oracle_rows(echo, grid, cells, rows, mgift="td"):
    """Oracle power rows for sampled (cell, rows): {cell: P [rows, n_fine]}."""
    import numpy as np
    from oracle import fd as OF
    from oracle import transforms as OT
    out = {}
    if mgift == "fd":
        Np = OF.pad_length(grid)
        S = OF.range_spectrum(echo, Np)
        F = OT.fine_matrix(grid)
        r = np.asarray(rows) - grid.n_begin
        for k in cells:
            out[int(k)] = np.abs(OF.mgift_fd(echo, grid, int(k), Np, S)[:, r].T @ F) ** 2
        return out
    for k in cells:
        y = OT.dsgrft_cell(echo, grid, int(k), rows=rows)
        out[int(k)] = np.abs(y) ** 2
    return out


def fine_roofline(plan, prof, form, split):
    """Roofline of the fine-search kernel from a dsgrft_profile: the
    algorithmic rate (8 flops per cell-pulse; for the FFT form the radix-2
    FFT flops of its transforms) and, for the MFMA forms, the executed MFMA
    rate (launched matrix products, padding included)."""
    launches = max(prof["fine_launches"], 1)
    avg_s = prof["fine_ms"] / launches * 1e-3
    fft = form == "f32fft"
    if fft:
        # FFT form: R de-chirped M-point FFTs per (unit, row), not 8 flops
        # per cell-pulse
        flops = prof["fine_cell_pulses"] / launches / (plan.M * plan.R * plan.R) \
            * plan.R * fft_flops(plan.M)
    else:
        flops = prof["fine_flops"] / launches
    peak = PEAK_TFLOPS[form]
    achieved = flops / avg_s / 1e12
    out = {"bound": "alu" if fft else "mfma", "achieved": round(achieved, 2),
           "peak": peak, "unit": "TFLOP/s", "frac": round(achieved / peak, 4),
           "traffic": None if fft else recorded_traffic(form, split),
           "mfma_util": None if fft else recorded_mfma_util(form, split),
           "kernel": f"k_fine_fft_w<{plan.M // 64}>" if fft
                     else KERNEL.get(form, f"k_fine_mfma<{form}, split {split}>"),
           "avg_launch_ms": round(avg_s * 1e3, 4),
           "flops_per_launch": flops,
           "launches": prof["fine_launches"]}
    if form not in ("f32", "f32fft"):
        ex = prof["fine_mfma_flops"] / launches
        out["executed"] = {"tflops": round(ex / avg_s / 1e12, 2),
                           "frac": round(ex / avg_s / 1e12 / peak, 4),
                           "flops_per_launch": ex,
                           "note": "launched MFMA products (padding included) over the "
                                   "same launch time; achieved/frac above count 8 flops per "
                                   "cell-pulse"}
    return out


def sampled_error(pm, af, ref, rows, tol):
    """max |dP|/P_ref_max over sampled rows, and argmax agreement (near-tie
    rule: exact where the oracle's top-2 gap exceeds 2 tol * scale)."""
    import numpy as np
    scale = max(float(v.max()) for v in ref.values())
    err, bad, clear = 0.0, 0, 0
    for k, P in ref.items():
        pm_o, af_o = P.max(-1), P.argmax(-1)
        srt = np.sort(P, -1)
        gap = srt[:, -1] - srt[:, -2]
        for i, r in enumerate(rows):
            e = abs(float(pm[k, r]) - pm_o[i]) / scale
            err = max(err, e)
            if gap[i] > 2 * tol * scale:
                clear += 1
                bad += int(af[k, r] != af_o[i])
            elif P[i, af[k, r]] < pm_o[i] - 2 * tol * scale:
                bad += 1
    return err, bad, clear, scale


GOLDEN3 = os.path.join(ROOT, "tests", "golden", "detect_config3.json")


def load_golden():
    """The FP64 oracle's largest reduced entries of the M=1024 search
    (tests/golden/detect_config3.json, written by an oracle-only script):
    (cells, rows, powers, fine indices, near-tie lists, peak power)."""
    import numpy as np
    try:
        g = json.load(open(GOLDEN3))
    except (OSError, ValueError):
        return None
    e = g["entries"]
    return dict(k=np.array([x[0] for x in e]), r=np.array([x[1] for x in e]),
                p=np.array([x[3] for x in e]), f=np.array([x[2] for x in e]),
                near=[x[4] for x in e], pmax=g["pmax"], n=len(e))


def golden_error(pm, af, gold, tol=1e-3):
    """Largest |dP| / P_max of a device reduced map over the golden's entries
    (the map's highest powers), and the entries whose fine index is outside
    the oracle's near-tie set (2 tol P_max)."""
    if gold is None:
        return None, None
    d = pm[gold["k"], gold["r"]].astype("float64")
    err = float(abs(d - gold["p"]).max() / gold["pmax"])
    band = 2 * tol * gold["pmax"]
    fd = af[gold["k"], gold["r"]]
    bad = 0
    for i in range(gold["n"]):
        if fd[i] != gold["f"][i]:
            ties = {int(q) for q, pq in gold["near"][i] if pq >= gold["p"][i] - band}
            bad += int(int(fd[i]) not in ties)
    return err, bad


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--form", default="f16_sym")
    ap.add_argument("--mgift", default="td", choices=("td", "fd"),
                    help="coarse compensation: time-domain gather or frequency domain")
    ap.add_argument("--split", type=int, default=1)
    ap.add_argument("--f32-cells", type=int, default=96)
    ap.add_argument("--f32-repeats", type=int, default=3)
    ap.add_argument("--no-sweep", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--profile-pass", action="store_true",
                    help="short run for rocprofv3 counter passes")
    ap.add_argument("--workload", type=int, default=3, choices=(2, 3, 4, 5, 6, 7),
                    help="2: single-scale TD-GRFT against DS-GRFT at M=512; "
                         "3: the M=1024 search (default, headline metric); "
                         "4: adjoint at M=512; 5: third-order search at M=2048 "
                         "on a 64-coarse-cell subset; 6: Monte-Carlo detection "
                         "probability vs SNR (M=256); 7: DS-KT-MFP search on the "
                         "M=1024 workload")
    ap.add_argument("--trials", type=int, default=100,
                    help="Monte-Carlo trials per SNR point (workload 6)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "bench.py measures one GPU; the search would shard "
                          "over coarse cells across GPUs, but runs on several GPUs "
                          "are not implemented", "n_gpus": args.gpus}))
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    from paper_2403_06788_amd.plan import Plan

    if args.workload == 2:
        return bench_grft(args)
    if args.workload == 4:
        return bench_adjoint(args)
    if args.workload == 5:
        return bench_jerk(args)
    if args.workload == 6:
        return bench_pd(args)
    if args.workload == 7:
        return bench_kt(args)
    case = synth.config_case(3)
    c = synth.CONFIGS[3]
    r = c["radar"]
    echo_np = case["echo"]
    plan = Plan(r.fc, r.fs, r.prf, c["M"], c["N"], c["order"], c["axes"], mgift=args.mgift)
    echo = torch.from_numpy(echo_np).cuda()
    cells = plan.n_coarse
    cp_total = float(cells) * plan.rows * plan.n_fine * plan.M
    pfa = 1e-9                           # LRT at sigma^2 = 1 (synthetic noise power)
    pm = torch.empty((cells, plan.rows), dtype=torch.float32, device="cuda")
    af = torch.empty((cells, plan.rows), dtype=torch.int32, device="cuda")

    def step(form, split, n=cells):
        plan.search(echo, form, split, n=n, out=(pm[:n], af[:n]))
        return plan.detect(pm[:n], af[:n], pfa, 1.0, cap=4096) if n == cells else None

    if args.profile_pass:
        # calibration copy of known size, then one search of 16 cells
        x = torch.empty(1 << 28, dtype=torch.float32, device="cuda")  # 1 GiB
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        plan.search(echo, args.form, args.split, n=16, out=(pm[:16], af[:16]))
        torch.cuda.synchronize()
        log(f"profile pass done: copy 1 GiB + {args.form}x{args.split} on 16 cells")
        return

    log(f"plan: {cells} coarse cells x {plan.n_fine} fine x {plan.rows} rows, "
        f"M={plan.M}; workspace {plan.workspace_bytes / 2**20:.0f} MiB")
    for _ in range(args.warmup):
        step(args.form, args.split)
    torch.cuda.synchronize()
    log(f"warmup done ({args.warmup} steps)")
    plan.profile_begin(4096)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        step(args.form, args.split)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    prof = plan.profile_end()
    ms = (t1 - t0) * 1e3 / args.steps
    value = cp_total / (ms * 1e-3)
    log(f"timed {args.steps} steps: {ms:.1f} ms/step, {value:.3e} cells*pulses/s")
    pm_main, af_main = pm.cpu().numpy(), af.cpu().numpy()
    peaks, count, best = plan.detect(pm, af, pfa, 1.0, cap=4096)
    # cell-averaging CFAR along range on the same reduced map (beside the LRT)
    plan.detect_cfar(pm, af, 2, 16, 1.5, cap=4096)
    torch.cuda.synchronize()
    t = time.perf_counter()
    _, cfar_count, _ = plan.detect_cfar(pm, af, 2, 16, 1.5, cap=4096)
    cfar_ms = (time.perf_counter() - t) * 1e3

    roofline = fine_roofline(plan, prof, args.form, args.split)
    # attainable matrix-core rate on random operands (power-limited clock)
    ceiling = {}
    for fm in ("f16", "bf16", "fp8"):
        tf, ghz = Plan.mfma_probe(fm, 50.0)
        ceiling[fm] = {"tflops": round(tf, 1), "clock_ghz": round(ghz, 3),
                       "frac_of_published": round(tf / PEAK_TFLOPS[fm], 4)}
    log(f"MFMA probe (register-only, random operands): f16 {ceiling['f16']['tflops']} TFLOP/s "
        f"at {ceiling['f16']['clock_ghz']} GHz, bf16 {ceiling['bf16']['tflops']} TFLOP/s, "
        f"e4m3 {ceiling['fp8']['tflops']} TFLOP/s at {ceiling['fp8']['clock_ghz']} GHz")
    op = DTYPE.get(args.form, args.form)
    if "executed" in roofline and op in ceiling:
        roofline["attainable"] = dict(ceiling[op], note=(
            "register-only loop of the same MFMA on random operands, no memory traffic "
            "(dsgrft_mfma_probe); the published peak assumes a clock the chip does not "
            "hold under random-data matrix load"))
        roofline["executed"]["frac_of_attainable"] = round(
            roofline["executed"]["tflops"] / ceiling[op]["tflops"], 4)
    fine_avg_s = roofline["avg_launch_ms"] * 1e-3
    achieved, peak = roofline["achieved"], roofline["peak"]
    gather_avg_s = prof["gather_ms"] / max(prof["gather_launches"], 1) * 1e-3
    gather_bytes = prof["gather_bytes"] / max(prof["gather_launches"], 1)
    gather = {"bound": "hbm", "achieved": round(gather_bytes / gather_avg_s / 1e9, 1),
              "peak": HBM_GBPS, "unit": "GB/s",
              "frac": round(gather_bytes / gather_avg_s / 1e9 / HBM_GBPS, 4),
              "avg_launch_ms": round(gather_avg_s * 1e3, 4),
              "bytes_per_launch": gather_bytes,
              "note": "elapsed time on the producer stream while the fine search of the "
                      "previous batch runs beside it (two-stream pipeline)"}
    # the gather alone: one-batch searches, whose gather runs before any fine
    # search is enqueued (nothing else on the GPU while it runs)
    plan.search(echo, args.form, args.split, n=16, out=(pm[:16], af[:16]))
    plan.profile_begin(64)
    for _ in range(8):
        torch.cuda.synchronize()
        plan.search(echo, args.form, args.split, n=16, out=(pm[:16], af[:16]))
    torch.cuda.synchronize()
    p1 = plan.profile_end()
    g1_s = p1["gather_ms"] / max(p1["gather_launches"], 1) * 1e-3
    g1_b = p1["gather_bytes"] / max(p1["gather_launches"], 1)
    gather_alone = {"bound": "hbm", "achieved": round(g1_b / g1_s / 1e9, 1), "peak": HBM_GBPS,
                    "unit": "GB/s", "frac": round(g1_b / g1_s / 1e9 / HBM_GBPS, 4),
                    "avg_launch_ms": round(g1_s * 1e3, 4), "bytes_per_launch": g1_b,
                    "launches": p1["gather_launches"],
                    "traffic": (_recorded(args.form, args.split, "traffic") or {}).get(
                        "gather_bytes_per_launch"),
                    "note": "one 16-cell batch at a time, nothing running beside it; algorithmic "
                            "bytes (8 B read per sample): the 32 MiB echo stays in the 256 MiB "
                            "Infinity Cache, so re-reads of it are not all DRAM traffic and frac "
                            "can exceed 1"}
    if gather_alone["traffic"]:
        # DRAM-side bytes of the same launch shape (rocprofv3 FETCH_SIZE + WRITE_SIZE)
        gather_alone["traffic_gbps"] = round(gather_alone["traffic"] / g1_s / 1e9, 1)
        gather_alone["traffic_frac"] = round(gather_alone["traffic"] / g1_s / 1e9 / HBM_GBPS, 4)
    log(f"fine kernel: {achieved:.1f} TFLOP/s ({achieved / peak:.1%} of {peak}); "
        f"gather {gather['achieved']:.0f} GB/s beside the fine search, "
        f"{gather_alone['achieved']:.0f} GB/s alone")

    # ---- accuracy on sampled rows vs the FP64 oracle ----------------------
    from oracle.grid import Axis, Radar, make_grid
    grid = make_grid(Radar(r.fc, r.fs, r.prf), c["M"], c["N"], c["order"],
                     [Axis(*a) for a in c["axes"]])
    rng = np.random.default_rng(2024)
    bk, brow = int(best["coarse"]), int(best["row"])
    s_cells = sorted(set([bk, 0, 1] + [int(x) for x in rng.choice(cells, 5, replace=False)]))
    s_rows = sorted(set([brow] + [int(x) for x in rng.choice(plan.rows, 40, replace=False)]))
    t = time.perf_counter()
    ref = oracle_rows(echo_np, grid, s_cells, s_rows, args.mgift)
    log(f"oracle rows: {len(s_cells)} cells x {len(s_rows)} rows in {time.perf_counter() - t:.1f} s")
    forms = {}
    err, bad, clear, scale = sampled_error(pm_main, af_main, ref, s_rows, 1e-3)
    # the golden holds the oracle's time-domain (nearest-bin) map; the
    # frequency-domain compensation computes a different map
    gold = load_golden() if args.mgift == "td" else None
    gerr, gbad = golden_error(pm_main, af_main, gold)
    forms[f"{args.form}x{args.split}"] = {"cells_pulses_per_s": value, "ms": round(ms, 2),
                                         "steps": args.steps, "rel_err": err,
                                         "argmax_bad": bad, "argmax_checked": clear,
                                         "golden_rel_err": gerr, "golden_argmax_bad": gbad,
                                         "roofline_frac": roofline["frac"],
                                         "executed_frac": roofline.get("executed", {}).get("frac"),
                                         "executed_frac_of_attainable":
                                             roofline.get("executed", {}).get("frac_of_attainable"),
                                         "mfma_util": roofline["mfma_util"],
                                         "fine_avg_launch_ms": roofline["avg_launch_ms"]}
    # ---- other forms: a 16-cell warm-up, then SWEEP_STEPS timed steps -------
    if not args.no_sweep:
        for form, split in SWEEP:
            if (form, split) == (args.form, args.split):
                continue
            step(form, split, n=16)
            torch.cuda.synchronize()
            plan.profile_begin(4096)
            t = time.perf_counter()
            for _ in range(SWEEP_STEPS):
                step(form, split)
            torch.cuda.synchronize()
            dt = (time.perf_counter() - t) / SWEEP_STEPS
            rf = fine_roofline(plan, plan.profile_end(), form, split)
            pm_np, af_np = pm.cpu().numpy(), af.cpu().numpy()
            e, b, cl, _ = sampled_error(pm_np, af_np, ref, s_rows, 1e-3)
            ge, gb = golden_error(pm_np, af_np, gold)
            forms[f"{form}x{split}"] = {"cells_pulses_per_s": cp_total / dt,
                                        "ms": round(dt * 1e3, 2), "steps": SWEEP_STEPS,
                                        "rel_err": e, "argmax_bad": b, "argmax_checked": cl,
                                        "golden_rel_err": ge, "golden_argmax_bad": gb,
                                        "roofline_frac": rf["frac"],
                                        "executed_frac": rf.get("executed", {}).get("frac"),
                                        "executed_frac_of_attainable": None
                                        if "executed" not in rf or DTYPE.get(form, form) not in ceiling
                                        else round(rf["executed"]["tflops"]
                                                   / ceiling[DTYPE.get(form, form)]["tflops"], 4),
                                        "mfma_util": rf["mfma_util"],
                                        "fine_avg_launch_ms": rf["avg_launch_ms"]}
            log(f"{form}x{split}: {dt * 1e3:.1f} ms, rel err {e:.2e} (golden entries "
                f"{ge if ge is None else f'{ge:.2e}'}), "
                f"{rf['frac']:.3f} of peak (algorithmic)")
    # ---- plain FP32 form on a sample of coarse cells ------------------------
    n32 = min(args.f32_cells, cells)
    step("f32", 1, n=16)
    torch.cuda.synchronize()
    t = time.perf_counter()
    for _ in range(args.f32_repeats):
        step("f32", 1, n=n32)
    torch.cuda.synchronize()
    dt32 = (time.perf_counter() - t) / args.f32_repeats
    cp32 = float(n32) * plan.rows * plan.n_fine * plan.M
    f32_rate = cp32 / dt32
    pm32, af32 = pm[:n32].cpu().numpy(), af[:n32].cpu().numpy()
    ref32 = {k: v for k, v in ref.items() if k < n32}
    e32 = sampled_error(pm32, af32, ref32, s_rows, 1e-5)[0] if ref32 else None
    forms["f32x1"] = {"cells_pulses_per_s": f32_rate, "sample_cells": n32,
                      "repeats": args.f32_repeats, "ms_sample": round(dt32 * 1e3, 2),
                      "rel_err": e32}
    log(f"f32 plain: {f32_rate:.3e} cells*pulses/s on {n32} cells x {args.f32_repeats}")
    # within 1e-3: on the sampled rows and, where the golden is present, on
    # the oracle's largest entries of the whole map
    ok_forms = {k: v for k, v in forms.items()
                if k != "f32x1" and v["rel_err"] <= 1e-3 and v["argmax_bad"] == 0
                and (v.get("golden_rel_err") is None or v["golden_rel_err"] <= 1e-3)
                and not v.get("golden_argmax_bad")}
    fastest = max(ok_forms, key=lambda k: ok_forms[k]["cells_pulses_per_s"]) if ok_forms else None
    bf16_ok = [k for k in ok_forms if k.startswith("bf16")]
    bf16_best = max(bf16_ok, key=lambda k: ok_forms[k]["cells_pulses_per_s"]) if bf16_ok else None

    # ---- CPU baseline: the oracle on a bounded sample ------------------------
    cpu = None
    if not args.no_cpu:
        from oracle import detect as OD
        try:
            from threadpoolctl import threadpool_info
            threads = max([d.get("num_threads", 1) for d in threadpool_info()] or [1])
        except Exception:
            threads = os.cpu_count()
        t = time.perf_counter()
        done = 0
        while done < 64 and (done == 0 or time.perf_counter() - t < 15.0):
            OD.dsgrft_reduced(echo_np, grid, cells=[done])
            done += 1
        dtc = time.perf_counter() - t
        cpu = {"value": done * plan.rows * plan.n_fine * plan.M / dtc,
               "unit": "cells·pulses/s", "cores": int(threads), "kind": "oracle",
               "sample": f"{done} coarse cells x {plan.rows} rows x {plan.n_fine} fine "
                         f"x {plan.M} pulses in {dtc:.1f} s (FP64 numpy, BLAS threads "
                         f"{threads}, host cpu_count {os.cpu_count()})"}
        log(f"cpu oracle: {cpu['value']:.3e} cells*pulses/s")

    out = {
        "metric": METRIC, "value": value, "unit": "cells·pulses/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms, 3), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": DTYPE.get(args.form, args.form), "data": "synthetic",
        "config": {"workload": "DS-GRFT search, M=1024 pulses, N=4096 range bins, "
                               "P=2 (v +-600 m/s, a +-50 m/s^2), 2460 coarse x 10^4 fine "
                               "cells, 8 targets at -20 dB, fc=1 GHz, fs=10 MHz, PRF=500 Hz",
                   "form": FORM_TEXT.get(args.form,
                                         f"{args.form} MFMA, split {args.split}, FP32 accumulation"),
                   "mgift": "time-domain nearest-bin gather" if args.mgift == "td"
                            else "frequency-domain coarse compensation (Alg. 1)",
                   "cells": cells * plan.rows * plan.n_fine, "pulses": plan.M},
        "roofline": roofline,
        "mfma_ceiling": ceiling,
        "gather_roofline": gather,
        "gather_roofline_alone": gather_alone,
        "cpu_baseline": cpu,
        "paper_times": PAPER_TIMES,
        "speedup_vs_f32": round(value / f32_rate, 2),
        "rel_err": err,
        "detections": int(count),
        "cfar": {"guard": 2, "train": 16, "alpha": 1.5, "detections": int(cfar_count),
                 "ms": round(cfar_ms, 3)},
        "forms": forms,
        "forms_within_1e-3": sorted(ok_forms),
        "fastest_within_1e-3": None if fastest is None else {
            "form": fastest, "cells_pulses_per_s": ok_forms[fastest]["cells_pulses_per_s"],
            "speedup_vs_f32": round(ok_forms[fastest]["cells_pulses_per_s"] / f32_rate, 2)},
        "bf16_fastest_within_1e-3": None if bf16_best is None else {
            "form": bf16_best, "cells_pulses_per_s": ok_forms[bf16_best]["cells_pulses_per_s"],
            "ms": ok_forms[bf16_best]["ms"], "rel_err": ok_forms[bf16_best]["rel_err"],
            "speedup_vs_f32": round(ok_forms[bf16_best]["cells_pulses_per_s"] / f32_rate, 2),
            "roofline_frac": ok_forms[bf16_best]["roofline_frac"],
            "executed_frac": ok_forms[bf16_best]["executed_frac"],
            "executed_frac_of_attainable": ok_forms[bf16_best].get("executed_frac_of_attainable")},
    }
    print(json.dumps(out), flush=True)


def _sync():
    import torch
    torch.cuda.synchronize()


ADJ_FLOPS_PER_TAP = 20

# The paper's own run times (Table IV): MATLAB on a CPU, for its Experiment 2
# scenario, whose range-bin counts and grids it does not state, so they do not
# convert to cells*pulses/s.  Reported beside the measurements as context.
PAPER_TIMES = {"dsgrft_s": 141.7, "ds_kt_mfp_s": 41.1,
               "hardware": "Intel Core i7-11700 (8 cores, 2.5 GHz), 32 GB, MATLAB 2019b",
               "scenario": "fc 28 GHz, fs 491.52 MHz, PRF 1905 Hz, M=512, P=2 (Experiment 2)",
               "comparable": False}


def bench_adjoint(args):
    """M=512 adjoint: forward + backward over 4096 candidates, gradient checks
    and off-grid refinement of the target candidates."""
    import numpy as np
    import torch

    import synth
    from paper_2403_06788_amd.plan import Plan
    case = synth.config_case(4)
    c = synth.CONFIGS[4]
    r = c["radar"]
    plan = Plan(r.fc, r.fs, r.prf, c["M"], c["N"], c["order"], c["axes"])
    echo = torch.from_numpy(case["echo"]).cuda()
    rng = np.random.Generator(np.random.PCG64(1004))
    th = synth.adjoint_candidates(rng, r, c["M"], c["N"], case["targets"], c["v"], c["a"])
    theta = torch.from_numpy(th).cuda()
    gJ = torch.ones(len(th), dtype=torch.float64, device="cuda")

    def step():
        J, saved = plan.adjoint_forward(echo, theta)
        return plan.adjoint_backward(echo, theta, saved, gJ)
    for _ in range(args.warmup):
        step()
    _sync()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        gt, ge = step()
    _sync()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    # dominant kernel: the forward (k_adj_fwd), timed alone with events on the
    # stream it is launched on (torch's current stream)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    nrep = 5
    ev0.record()
    for _ in range(nrep):
        plan.adjoint_forward(echo, theta)
    ev1.record()
    _sync()
    fwd_s = ev0.elapsed_time(ev1) * 1e-3 / nrep
    # FP64 work per (candidate, pulse, range tap): distance (1), reciprocal
    # (two Newton steps on a single-precision seed, 8), weight and derivative
    # (3), four accumulations (8)
    fwd_flops = float(len(th)) * plan.M * c["N"] * ADJ_FLOPS_PER_TAP
    roofline = {"bound": "alu", "achieved": round(fwd_flops / fwd_s / 1e12, 2),
                "peak": 78.6, "unit": "TFLOP/s",
                "frac": round(fwd_flops / fwd_s / 1e12 / 78.6, 4), "traffic": None,
                "kernel": "k_adj_fwd (FP64)", "avg_launch_ms": round(fwd_s * 1e3, 4),
                "flops_per_launch": fwd_flops}
    # device central differences, candidates away from coarse-cell edges
    J, _ = plan.adjoint_forward(echo, theta)
    gt = gt.cpu().numpy()
    hs = np.array([1e-4 * plan.dr, 1e-4 * plan.step[0], 1e-4 * plan.step[1]])
    inside = np.ones(len(th), dtype=bool)
    for p in (0, 1):
        u = th[:, p + 1] / plan.step[p] - plan.i_lo[p] + 0.5
        fr = (u / plan.R) % 1.0
        inside &= (fr > 0.01) & (fr < 0.99)
    idx = np.nonzero(inside)[0]
    fd_err = []
    for q in range(3):
        e = np.zeros(3)
        e[q] = hs[q]
        Jp, _ = plan.adjoint_forward(echo, torch.from_numpy(th[idx] + e))
        Jm, _ = plan.adjoint_forward(echo, torch.from_numpy(th[idx] - e))
        fd = (Jp.cpu().numpy() - Jm.cpu().numpy()) / (2 * hs[q])
        fd_err.append(float(np.abs(fd - gt[idx, q]).max() / np.abs(gt[idx, q]).max()))
    # oracle gradient on a sample
    from oracle import adjoint as OA
    from oracle.grid import Axis, Radar, make_grid
    grid = make_grid(Radar(r.fc, r.fs, r.prf), c["M"], c["N"], c["order"],
                     [Axis(*a) for a in c["axes"]])
    o_err = 0.0
    for b in np.random.default_rng(3).choice(len(th), 8, replace=False):
        _, _, go, _ = OA.gradients(case["echo"], grid, th[b])
        o_err = max(o_err, float(np.abs(gt[b] - go).max() / max(np.abs(go).max(), 1e-30)))
    # refinement of the 16 jittered candidates of each target
    t0 = time.perf_counter()
    thr, Jr = plan.refine(echo, theta[:16 * len(case["targets"])], iters=40)
    _sync()
    t_ref = time.perf_counter() - t0
    thr, Jr = thr.cpu().numpy(), Jr.cpu().numpy()
    J0 = J.cpu().numpy()[:16 * len(case["targets"])]
    errs = []
    for ti, tg in enumerate(case["targets"]):
        sl = slice(16 * ti, 16 * ti + 16)
        b = int(np.argmax(Jr[sl]))
        best = thr[sl][b]
        errs.append((abs(best[0] - tg.r0), abs(best[1] - tg.v), abs(best[2] - tg.a)))
    errs = np.array(errs)
    out = {"metric": "DS-GRFT adjoint candidates/s (M=512): J, dJ/dtheta and dJ/decho",
           "value": len(th) / (ms * 1e-3), "unit": "candidates/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms, 3),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64", "data": "synthetic",
           "config": {"workload": "adjoint, M=512 pulses, N=2048 bins, P=2, 16 targets at "
                                  "-10 dB, 4096 candidates (16 jittered per target + 3840 uniform)"},
           "roofline": roofline,
           "grad_vs_central_diff_max_rel": fd_err, "grad_vs_oracle_max_rel": o_err,
           "fd_candidates": int(len(idx)),
           "refine": {"candidates": 16 * len(case["targets"]), "iters": 40,
                      "seconds": round(t_ref, 3),
                      "J_increase_median": float(np.median(Jr / np.maximum(J0, 1e-30))),
                      "target_error_median": {"r0_m": float(np.median(errs[:, 0])),
                                              "v_mps": float(np.median(errs[:, 1])),
                                              "a_mps2": float(np.median(errs[:, 2]))},
                      "target_error_max": {"r0_m": float(errs[:, 0].max()),
                                           "v_mps": float(errs[:, 1].max()),
                                           "a_mps2": float(errs[:, 2].max())},
                      "fine_steps": {"dr_m": plan.dr, "dv_mps": plan.step[0],
                                     "da_mps2": plan.step[1]}}}
    print(json.dumps(out), flush=True)


def bench_grft(args):
    """M=512, N=2048, P=2 (v +-600 m/s, a +-50 m/s^2): the single-scale
    TD-GRFT (eq. (13), every lattice point on its own walk) against DS-GRFT
    on the same echo and lattice, whose cells it matches one to one."""
    import numpy as np
    import torch

    import synth
    from paper_2403_06788_amd.plan import Plan
    case = synth.config_case(2)
    c = synth.CONFIGS[2]
    r = c["radar"]
    plan = Plan(r.fc, r.fs, r.prf, c["M"], c["N"], c["order"], c["axes"])
    echo = torch.from_numpy(case["echo"]).cuda()
    n = plan.n_coarse
    cp_cell = float(plan.rows) * plan.n_fine * plan.M
    res = {}

    def timed(fn, ncells, key):
        fn(min(ncells, 2))
        _sync()
        t0 = time.perf_counter()
        out = fn(ncells)
        _sync()
        dt = time.perf_counter() - t0
        res[key] = {"cells_pulses_per_s": ncells * cp_cell / dt, "s": round(dt, 4),
                    "coarse_cells": ncells}
        log(f"{key}: {ncells} coarse cells in {dt:.3f} s, {ncells * cp_cell / dt:.3e} cells*pulses/s")
        return out
    pm_ds, _ = timed(lambda k: plan.search(echo, "f16_sym", 1, n=k), n, "dsgrft_f16_symx1")
    timed(lambda k: plan.search(echo, "f16_3m", 1, n=k), n, "dsgrft_f16_3mx1")
    pm_32, _ = timed(lambda k: plan.search(echo, "f32", 1, n=k), min(n, 32), "dsgrft_f32x1")
    ng = min(n, 32)
    pm_g, _ = timed(lambda k: plan.grft(echo, 0, k), ng, "grft_f32")
    # the two transforms differ where the fine walk leaves the coarse walk's
    # bin; compare their per-(cell, row) maxima on the GRFT sample
    a, b = pm_g.cpu().numpy().astype(np.float64), pm_32[:ng].cpu().numpy().astype(np.float64)
    # the TD-GRFT call is one k_grft launch (plus a fill and an unpack of
    # ~0.1 ms): its rate at 8 flops per cell-pulse against the FP32 peak
    g_tflops = res["grft_f32"]["cells_pulses_per_s"] * 8 / 1e12
    out = {"metric": "TD-GRFT and DS-GRFT cells·pulses/s (M=512, P=2)",
           "value": res["dsgrft_f16_symx1"]["cells_pulses_per_s"], "unit": "cells·pulses/s",
           "n_gpus": 1, "steps": 1, "warmup": 1, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f16", "data": "synthetic",
           "config": {"workload": "M=512 pulses, N=2048 bins, P=2 (v +-600 m/s, a +-50 m/s^2), "
                                  f"{n} coarse x {plan.n_fine} fine cells x {plan.rows} rows, "
                                  "3 targets at -15 dB",
                      "cells": n * plan.rows * plan.n_fine, "pulses": plan.M},
           "forms": res,
           "speedup_dsgrft_vs_grft": {
               "f16_symx1": res["dsgrft_f16_symx1"]["cells_pulses_per_s"] / res["grft_f32"]["cells_pulses_per_s"],
               "f16_3mx1": res["dsgrft_f16_3mx1"]["cells_pulses_per_s"] / res["grft_f32"]["cells_pulses_per_s"],
               "f32x1": res["dsgrft_f32x1"]["cells_pulses_per_s"] / res["grft_f32"]["cells_pulses_per_s"]},
           "reduced_map_ds_over_grft": {"max_ratio": float(b.max() / a.max()),
                                        "median_ratio": float(np.median(b / np.maximum(a, 1e-30)))},
           "grft_roofline": {"bound": "alu", "achieved": round(g_tflops, 2), "peak": 157.3,
                             "unit": "TFLOP/s", "frac": round(g_tflops / 157.3, 4),
                             "kernel": "k_grft (FP32)",
                             "note": "wall clock of the 32-cell call, 8 flops per cell-pulse"}}
    print(json.dumps(out), flush=True)


def bench_jerk(args):
    """M=2048, P=3 search on 64 coarse cells (the 4 targets' cells + 60
    seeded random ones): MFMA forms vs the plain FP32 form."""
    import numpy as np
    import torch

    import synth
    from paper_2403_06788_amd.plan import Plan
    case = synth.config_case(5)
    c = synth.CONFIGS[5]
    r = c["radar"]
    plan = Plan(r.fc, r.fs, r.prf, c["M"], c["N"], c["order"], c["axes"])
    echo = torch.from_numpy(case["echo"]).cuda()

    def cell_of(tg):
        ks = []
        for p, val in enumerate((tg.v, tg.a, tg.j)):
            k = int(np.floor((val / plan.step[p] - plan.i_lo[p] + 0.5) / plan.R))
            ks.append(min(max(k, 0), plan.K[p] - 1))
        return (ks[2] * plan.K[1] + ks[1]) * plan.K[0] + ks[0]
    tcells = [cell_of(t) for t in case["targets"]]
    rng = np.random.Generator(np.random.PCG64(1005))
    others = [int(x) for x in rng.choice(plan.n_coarse, 60, replace=False)]
    cells = torch.tensor(tcells + others, dtype=torch.int64, device="cuda")
    n = cells.numel()
    cp = float(n) * plan.rows * plan.n_fine * plan.M
    res = {}
    for form, split in (("f16_sym", 1), ("bf16_sym", 3), ("bf16_sym", 2), ("f16_3m", 1),
                        ("f16", 1), ("bf16", 1), ("bf16", 3)):
        plan.search(echo, form, split, cells=cells[:1])
        _sync()
        t0 = time.perf_counter()
        pm, af = plan.search(echo, form, split, cells=cells)
        _sync()
        dt = time.perf_counter() - t0
        res[f"{form}x{split}"] = {"cells_pulses_per_s": cp / dt, "s": round(dt, 3),
                                  "target_cell_max": [float(pm[i].max()) for i in range(4)]}
        log(f"{form}x{split}: {dt:.2f} s, {cp / dt:.3e} cells*pulses/s")
    plan.search(echo, "f32", 1, cells=cells[:1])
    _sync()
    t0 = time.perf_counter()
    pm32, _ = plan.search(echo, "f32", 1, cells=cells[:2])
    _sync()
    dt = time.perf_counter() - t0
    res["f32x1"] = {"cells_pulses_per_s": 2 * plan.rows * plan.n_fine * plan.M / dt,
                    "sample_cells": 2, "s": round(dt, 3)}
    out = {"metric": "DS-GRFT cells·pulses/s (M=2048, P=3, 64-coarse-cell subset)",
           "value": res["f16_symx1"]["cells_pulses_per_s"], "unit": "cells·pulses/s",
           "n_gpus": 1, "steps": 1, "warmup": 1, "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f16", "data": "synthetic",
           "config": {"workload": "third-order search, M=2048 pulses, N=8192 bins, v +-900, "
                                  "a +-100, j +-20; 64 of 1708224 coarse cells (4 target cells + "
                                  "60 seeded) x 10^6 fine cells x 8192 rows",
                      "cells": n * plan.rows * plan.n_fine, "pulses": plan.M},
           "forms": res,
           "speedup_vs_f32": {k: v["cells_pulses_per_s"] / res["f32x1"]["cells_pulses_per_s"]
                              for k, v in res.items() if k != "f32x1"}}
    print(json.dumps(out), flush=True)




def fft_flops(M):
    """Algorithmic FP32 flops of one fine-acceleration pass of the FFT form
    per range row: de-chirp (6 M), radix-2 FFT count (5 M log2 M) and
    |.|^2 (3 M)."""
    return 9 * M + 5 * M * (M.bit_length() - 1)


def bench_kt(args):
    """DS-KT-MFP (Alg. 4) on the M=1024, N=4096 workload: range FFT,
    keystone, per-cell folding/acceleration compensation + IFFT, gather and
    the FFT fine search over the M x R fine cells of every coarse cell."""
    import torch

    import synth
    from paper_2403_06788_amd.plan import Plan
    case = synth.config_case(3)
    c = synth.CONFIGS[3]
    r = c["radar"]
    plan = Plan(r.fc, r.fs, r.prf, c["M"], c["N"], c["order"], c["axes"], mgift="kt")
    echo = torch.from_numpy(case["echo"]).cuda()
    cells = plan.n_coarse
    cp_total = float(cells) * plan.rows * plan.n_fine * plan.M
    pfa = 1e-9
    pm = torch.empty((cells, plan.rows), dtype=torch.float32, device="cuda")
    af = torch.empty((cells, plan.rows), dtype=torch.int32, device="cuda")

    def step():
        plan.search(echo, "f32fft", 1, out=(pm, af))
        return plan.detect(pm, af, pfa, 1.0, cap=4096)
    log(f"DS-KT-MFP plan: {plan.kt_folds} folds x {plan.K[1]} coarse accelerations = "
        f"{cells} cells x {plan.n_fine} fine x {plan.rows} rows, N'={plan.fd_pad}; "
        f"workspace {plan.workspace_bytes / 2**20:.0f} MiB")
    for _ in range(args.warmup):
        step()
    _sync()
    log(f"warmup done ({args.warmup} steps)")
    plan.profile_begin(4096)
    _sync()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    _sync()
    t1 = time.perf_counter()
    prof = plan.profile_end()
    ms = (t1 - t0) * 1e3 / args.steps
    value = cp_total / (ms * 1e-3)
    log(f"timed {args.steps} steps: {ms:.1f} ms/step, {value:.3e} cells*pulses/s")
    _, count, best = plan.detect(pm, af, pfa, 1.0, cap=4096)
    nl = max(prof["fine_launches"], 1)
    fine_avg_s = prof["fine_ms"] / nl * 1e-3
    flops_launch = prof["fine_cell_pulses"] / nl / (plan.M * plan.n_fine) * plan.R \
        * fft_flops(plan.M)
    achieved = flops_launch / fine_avg_s / 1e12
    peak = PEAK_TFLOPS["f32fft"]
    out = {"metric": "DS-KT-MFP cells·pulses/s (M=1024)", "value": value,
           "unit": "cells·pulses/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "DS-KT-MFP search, M=1024 pulses, N=4096 range bins, P=2 "
                                  "(v +-600 m/s, a +-50 m/s^2), N'=8192, "
                                  f"{plan.kt_folds} folding factors x {plan.K[1]} coarse "
                                  f"accelerations, {plan.n_fine} fine cells each, 8 targets "
                                  "at -20 dB, fc=1 GHz, fs=10 MHz, PRF=500 Hz",
                      "cells": cells * plan.rows * plan.n_fine, "pulses": plan.M},
           "roofline": {"bound": "alu", "achieved": round(achieved, 2), "peak": peak,
                        "unit": "TFLOP/s", "frac": round(achieved / peak, 4), "traffic": None,
                        "kernel": f"k_fine_fft_w<{plan.M // 64}, full bins>",
                        "avg_launch_ms": round(fine_avg_s * 1e3, 4),
                        "flops_per_launch": flops_launch, "launches": prof["fine_launches"]},
           "gather_ms_per_step": round(prof["gather_ms"] / args.steps, 3),
           "fine_ms_per_step": round(prof["fine_ms"] / args.steps, 3),
           "cpu_baseline": None,
           "paper_times": PAPER_TIMES,
           "cpu_baseline_note": "not measured: at this size the oracle's keystone alone takes "
                                "minutes and each coarse cell's fine map ~1e11 complex MACs, "
                                "so no bounded sample of the workload fits (the DS-GRFT line "
                                "carries the oracle baseline)",
           "detections": int(count),
           "best": {"coarse": int(best["coarse"]), "row": int(best["row"]),
                    "fine": int(best["fine"]), "power": float(best["power"])}}
    print(json.dumps(out), flush=True)


PD_PFA = 1e-8          # per-cell false-alarm probability of the LRT threshold
PD_DETECTORS = ("ds_td", "ds_fd", "ds_kt", "grft")


def kt_cell(plan, v, a):
    """DS-KT-MFP coarse cell (folding factor, coarse acceleration) holding
    the nearest lattice point of (v, a)."""
    import numpy as np
    i1 = int(np.floor(v / plan.step[0] + 0.5))
    q = (i1 + plan.M // 2) // plan.M - plan.kt_q_lo
    q = min(max(q, 0), plan.kt_folds - 1)
    k2 = int(np.floor((a / plan.step[1] - plan.i_lo[1] + 0.5) / plan.R))
    k2 = min(max(k2, 0), plan.K[1] - 1)
    return k2 * plan.kt_folds + q


def pd_trial(plans, echo, target, gamma2):
    """Detection statistics of one trial: for each detector, the largest
    reduced power over the target's coarse cell and its two neighbours along
    v (DS-KT-MFP: the target's folding-factor cell, M R fine cells), in range
    rows round(r0 / dr) +- 2, and whether it exceeds gamma2.  DS-GRFT uses
    the f16 MFMA form, DS-KT-MFP the FFT form; the single-scale TD-GRFT runs
    in FP32."""
    import numpy as np
    import torch
    p = plans["ds_td"]
    ks = []
    for q, val in enumerate((target.v, target.a)):
        k = int(np.floor((val / p.step[q] - p.i_lo[q] + 0.5) / p.R))
        ks.append(min(max(k, 0), p.K[q] - 1))
    kt = ks[1] * p.K[0] + ks[0]
    lo, hi = max(0, ks[0] - 1), min(p.K[0] - 1, ks[0] + 1)
    cells = list(range(ks[1] * p.K[0] + lo, ks[1] * p.K[0] + hi + 1))
    rb = int(round(target.r0 / p.dr))
    r0, r1 = max(0, rb - 2), min(p.rows, rb + 3)
    out = {}
    ktc = kt_cell(plans["ds_kt"], target.v, target.a)
    for name in PD_DETECTORS:
        if name == "grft":
            pm, _ = p.grft(echo, cells[0], len(cells))
        elif name == "ds_kt":
            pm, _ = plans[name].search(echo, "f32fft", 1,
                                       cells=torch.tensor([ktc], dtype=torch.int64))
        else:
            pm, _ = plans[name].search(echo, "f16", 1, cc_begin=cells[0], n=len(cells))
        stat = float(pm[:, r0:r1].max())
        out[name] = (stat, stat > gamma2)
    return out, cells, (r0, r1), kt, ktc


def bench_pd(args):
    """Monte-Carlo detection probability vs per-pulse SNR (the shape of the
    paper's Exp. 2): one random target per trial (uniform r0, v, a), sigma^2 = 1
    noise, LRT threshold at P_FA = 1e-8 per cell, for DS-GRFT with the
    time-domain gather, DS-GRFT with the frequency-domain mGIFT, DS-KT-MFP and
    single-scale TD-GRFT; noise-only trials give the false-alarm rate of the
    neighbourhood test."""
    import numpy as np
    import torch

    import synth
    from paper_2403_06788_amd.plan import Plan
    sc = synth.PD_SCENARIO
    r = sc["radar"]
    plans = {"ds_td": Plan(r.fc, r.fs, r.prf, sc["M"], sc["N"], sc["order"], sc["axes"]),
             "ds_fd": Plan(r.fc, r.fs, r.prf, sc["M"], sc["N"], sc["order"], sc["axes"],
                           mgift="fd"),
             "ds_kt": Plan(r.fc, r.fs, r.prf, sc["M"], sc["N"], sc["order"], sc["axes"],
                           mgift="kt")}
    gamma2 = plans["ds_td"].threshold(1.0, PD_PFA)
    rng = np.random.Generator(np.random.PCG64(2406))
    snrs = [None] + [float(x) for x in np.arange(-16.0, -3.9, 1.0)]
    curves = {d: [] for d in PD_DETECTORS}
    t0 = time.perf_counter()
    n_trials = 0
    for snr in snrs:
        hits = {d: 0 for d in PD_DETECTORS}
        for _ in range(args.trials):
            tg = synth.draw_targets(rng, r, sc["M"], sc["N"], 1,
                                    -200.0 if snr is None else snr, 1.0,
                                    sc["v"], sc["a"], sc["j"])[0]
            echo_np = synth.make_echo(r, sc["M"], sc["N"], [] if snr is None else [tg], 1.0, rng)
            echo = torch.from_numpy(echo_np).cuda()
            res = pd_trial(plans, echo, tg, gamma2)[0]
            for d in PD_DETECTORS:
                hits[d] += int(res[d][1])
            n_trials += 1
        for d in PD_DETECTORS:
            curves[d].append(hits[d] / args.trials)
        log(f"snr {snr}: " + ", ".join(f"{d} {hits[d] / args.trials:.2f}" for d in PD_DETECTORS))
    dt = time.perf_counter() - t0

    def snr_at(pd_curve, level):
        xs, ys = snrs[1:], pd_curve[1:]
        for i in range(1, len(xs)):
            if ys[i - 1] < level <= ys[i]:
                return xs[i - 1] + (level - ys[i - 1]) / (ys[i] - ys[i - 1]) * (xs[i] - xs[i - 1])
        return None
    at = {d: {"pd_0.5": snr_at(curves[d], 0.5), "pd_0.9": snr_at(curves[d], 0.9)}
          for d in PD_DETECTORS}
    loss = None
    if at["ds_td"]["pd_0.9"] is not None and at["ds_fd"]["pd_0.9"] is not None:
        loss = at["ds_td"]["pd_0.9"] - at["ds_fd"]["pd_0.9"]
    out = {"metric": "Monte-Carlo trials/s (4 detectors, M=256)", "value": n_trials / dt,
           "unit": "trials/s", "n_gpus": 1, "higher_is_better": True, "data": "synthetic",
           "vs_baseline": None,
           "config": {"workload": "Pd vs per-pulse SNR, M=256 pulses, N=512 bins, P=2, "
                                  "v +-300 m/s, a +-50 m/s^2, one target per trial, "
                                  f"{args.trials} trials per point, P_FA {PD_PFA} per cell"},
           "snr_db": snrs[1:], "false_alarm_rate": {d: curves[d][0] for d in PD_DETECTORS},
           "pd": {d: curves[d][1:] for d in PD_DETECTORS}, "snr_at": at,
           "td_minus_fd_db_at_pd_0.9": loss}
    print(json.dumps(out), flush=True)

if __name__ == "__main__":
    main()
