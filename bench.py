"""Benchmark: cell-updates/s of the batched FP32 step on one MI355X.

Workload (the batched FP32 configuration the metric is quoted on): 2D
periodic stochastic heat equation, 512 x 512 cells x 256 independent
realisations, forward Euler, r = 0.1, eps = 1e-2, T0 = 1 plus an equilibrium
perturbation; the equal-time spatial statistics are sampled every 10 steps.
A "step" is one time step of all 256 realisations (Philox + Box-Muller face
noise, face fluxes, divergence update, and the sampling on sample steps).
Inputs are resident in HBM when the timed region starts.

Printed: one JSON line with the throughput, the roofline of the step kernel
(HIP-event timing of its back-to-back launches on its stream inside the timed
region, algorithmic bytes 8 B per FP32 cell-update), the plain
single-realisation rate (one launch per step),
the state error against the FP64 oracle on a sampled realisation, and the
oracle's own rate on the host CPU.
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

METRIC = "cell-updates/s (incl. RNG) + % HBM roofline, batched FP32 vs plain, at stated error"
HBM_PEAK_GBS = 8000.0
KERNEL_SRC = os.path.join(ROOT, "paper_2406_12157_amd", "csrc", "she_knd.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_step2d_c3.json")
VALU_FILE = os.path.join(ROOT, "profiles", "valu_step2d_c3.json")
PEAK_CLOCK_GHZ = 2.4


def _section(text: str, start: str, end: str) -> str:
    i = text.index(start)
    return text[i:text.index(end, i) + len(end)]


def kernel_hash() -> str:
    """Hash of what decides the 2D step kernel's HBM traffic: its source, the
    noise header, the host functions that pick its launch shapes (plan_nd,
    and build_plan for the two-step march) and the parameter structs it
    takes; edits elsewhere leave it unchanged."""
    csrc = os.path.join(ROOT, "paper_2406_12157_amd", "csrc")
    h = hashlib.sha256()
    for name in ("she_knd.hip", "she_rng.hpp"):
        with open(os.path.join(csrc, name), "rb") as f:
            h.update(f.read())
    with open(os.path.join(csrc, "she_capi.hip")) as f:
        t = f.read()
    for start in ("static she_status plan_nd(", "static she_status build_plan("):
        h.update(_section(t, start, "\n}\n").encode())
    with open(os.path.join(csrc, "she_internal.hpp")) as f:
        t = f.read()
    for start in ("struct ParamsND {", "struct StepArg {"):
        h.update(_section(t, start, "\n};\n").encode())
    return h.hexdigest()[:16]


def make_handle(she, cfg, stats, tuning_flags=0, burn_in=0, batch_samples=0):
    """The handle the benchmark times (burn-in and batch length change what
    is sampled, not the launch shapes)."""
    insts = [she.Instance(n=i["n"], eq=i["eq"], bc=i["bc"], scheme=i["scheme"], noise=i["noise"], r=i["r"],
                          eps=i["eps"], u0=i["u0"], u_left=i["u_left"], u_right=i["u_right"],
                          init_sd=i["init_sd"], seed=i["seed"], realisation=i["realisation"])
             for i in cfg["instances"]]
    return she.Handle(insts, precision=cfg["precision"], burn_in=burn_in, sample_every=cfg["sample_every"],
                      stats=stats, tuning_flags=tuning_flags, batch_samples=batch_samples), insts


def timed_region(torch, h, steps, every):
    """Wall time of `steps` sampled steps (burn-in 0) and the HIP-event time of
    the step kernel inside them: each sampling period's run of back-to-back
    non-sample steps, an even number of them (2D FE takes two steps per
    launch), is one call bracketed by events on the library's stream (torch's
    current stream); the remaining one or two steps, ending with the sample
    step, follow unbracketed.  Returns (wall seconds, kernel ms per step,
    steps timed)."""
    ev = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    done = 0
    while done < steps:
        r = (every - h.steps % every) % every      # steps until the next sample step completes
        plain = min(steps - done, (r if r > 0 else every) - 1)
        plain -= plain % 2
        if plain > 0:
            a = torch.cuda.Event(enable_timing=True)
            b = torch.cuda.Event(enable_timing=True)
            a.record()
            h.run(plain)
            b.record()
            ev.append((a, b, plain))
            done += plain
        if done < steps:
            rest = min(steps - done, (r if r > 0 else every) - plain)
            h.run(rest)
            done += rest
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    n = sum(k for _, _, k in ev)
    kms = sum(a.elapsed_time(b) for a, b, _ in ev) / max(1, n)
    return wall, kms, n


def state_error(she, torch, cfg, realisation, steps):
    """Max relative state error of one realisation after `steps` steps vs the
    FP64 oracle started from the same field (bounded: one realisation)."""
    import numpy as np
    import oracle
    c1 = dict(cfg)
    c1["instances"] = [cfg["instances"][realisation]]
    h, insts = make_handle(she, c1, 0)
    u = h.read_field(0)
    h.step(steps)
    got = h.read_field(0)
    h.close()
    i = c1["instances"][0]
    d = oracle.Desc(dim=2, n=tuple(i["n"]) + (1,), eq=i["eq"], scheme=i["scheme"], noise=i["noise"],
                    r=float(np.float32(i["r"])), sigma=float(np.float32(np.sqrt(2 * i["r"] * i["eps"]))),
                    u0=i["u0"], u_left=i["u_left"], u_right=i["u_right"], seed=i["seed"],
                    realisation=i["realisation"])
    oracle.advance(d, u, 0, steps)
    return float(np.max(np.abs(got - u) / np.abs(u)))


def cpu_baseline(cfg, seconds: float):
    """The oracle (single thread, FP64) on one realisation of the workload for
    about `seconds` of CPU time; rate in cell-updates/s."""
    import oracle
    import numpy as np
    i = cfg["instances"][0]
    d = oracle.Desc(dim=2, n=tuple(i["n"]) + (1,), eq=i["eq"], scheme=i["scheme"], noise=i["noise"], r=i["r"],
                    sigma=float(np.sqrt(2 * i["r"] * i["eps"])), u0=i["u0"], u_left=i["u_left"],
                    u_right=i["u_right"], init_sd=i["init_sd"], seed=i["seed"], realisation=i["realisation"])
    u = oracle.init(d)
    st = oracle.Stats(d, burn_in=0, every=cfg["sample_every"], per_cell=False)
    cells = d.ncells
    steps, t_used = 0, 0.0
    t0 = time.perf_counter()
    while t_used < seconds:
        oracle.advance(d, u, steps, 5, st)
        steps += 5
        t_used = time.perf_counter() - t0
    return dict(value=cells * steps / t_used, unit="cell-updates/s", cores=1, kind="oracle",
                sample="1 of 256 realisations, 512x512, %d steps (FE, sampling every %d), %.1f s"
                       % (steps, cfg["sample_every"], t_used))


def read_traffic(cells_per_launch):
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except Exception:
        return None
    if t.get("kernel_hash") != kernel_hash():
        return None
    return t.get("hbm_bytes_per_launch")


def read_valu(kernel_ms, per_period):
    """VALU issue of the 2D step kernel: the VALU instructions one launch
    executes (SQ_INSTS_VALU from a committed counter pass, weighted by one
    sample launch in the `per_period` launches of a sampling period), at four
    cycles per wave64 instruction, as cycles per SIMD over the live launch
    time at the 2.4 GHz peak clock.  A lower bound on the VALU's busy share:
    transcendental and 64-bit integer instructions hold it longer.  None once
    the kernel differs from the one counted."""
    try:
        with open(VALU_FILE) as f:
            v = json.load(f)
    except Exception:
        return None
    if v.get("kernel_hash") != kernel_hash():
        return None
    q = v["valu_insts_per_launch"]
    qs = v.get("sample_valu_insts_per_launch") or q
    insts = ((per_period - 1) * q + qs) / per_period
    cycles = insts * 4 / v["simds"]
    return dict(insts_per_launch=insts, issue_cycles_per_simd=cycles, peak_clock_ghz=PEAK_CLOCK_GHZ,
                frac=cycles / (PEAK_CLOCK_GHZ * 1e9 * kernel_ms * 1e-3), source="profiles/valu_step2d_c3.json")


def other_workload(args, torch, she, W):
    """Throughput of c1, c2, c4 or c5 with the statistics its configuration
    names, timed over `--steps` steps after `--warmup` (she_run, burn-in 0).
    The 1D workloads keep their state in registers, so they are bound by the
    per-step latency of the resident kernel, not by HBM; c5 gets the HBM
    roofline of its step kernel as c3 does."""
    cfg = {"c1": W.c1, "c2": W.c2, "c4": W.c4, "c5": W.c5}[args.workload]()
    stats = {"c1": she.STAT_MOMENTS | she.STAT_CORR, "c2": she.STAT_MOMENTS | she.STAT_CORR, "c4": 0,
             "c5": she.STAT_SPATIAL}[args.workload]
    h, insts = make_handle(she, cfg, stats)
    cells = sum(i.ncells for i in insts)
    h.run(args.warmup)
    torch.cuda.synchronize()
    roofline = None
    if args.workload == "c5":
        wall, kms, nev = timed_region(torch, h, args.steps, cfg["sample_every"])
        bpl = 8.0 * cells
        ach = bpl / (kms * 1e-3) / 1e9
        roofline = dict(bound="hbm", achieved=ach, peak=HBM_PEAK_GBS, unit="GB/s", frac=ach / HBM_PEAK_GBS,
                        traffic=None, kernel="k_step3d<float,4,dk>", kernel_ms=kms, kernel_launches_timed=nev,
                        algorithmic_bytes_per_launch=bpl)
    else:
        t0 = time.perf_counter()
        h.run(args.steps)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
    h.close()
    out = {"metric": METRIC, "value": cells * args.steps / wall, "unit": "cell-updates/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": wall / args.steps * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64" if cfg["precision"] == 1 else "f32", "data": "synthetic",
           "config": {"workload": cfg["name"], "instances": len(insts), "cells": cells,
                      "sample_every": cfg["sample_every"], "stats_mask": int(stats), "parallelism": "single GPU"},
           "roofline": roofline}
    print(json.dumps(out), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--realisations", type=int, default=256)
    ap.add_argument("--scheme", choices=["fe", "pc"], default="fe")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-error", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one 1 GiB device-to-device copy (reference for HBM counters)")
    ap.add_argument("--workload", choices=["c3", "c1", "c2", "c4", "c5"], default="c3",
                    help="c3 (default): the benchmark line; the others: a throughput line of that "
                         "workload with its statistics, for profiling")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: this build runs on one GPU only (--gpus 1); the path would shard by realisation "
              "with no per-step communication, but no multi-GPU run is provided.", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2406_12157_amd import she, workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    she.load()
    if args.workload != "c3":
        other_workload(args, torch, she, W)
        return
    scheme = W.EM if args.scheme == "fe" else W.HEUN
    cfg = W.c3(realisations=args.realisations, scheme=scheme)
    every = cfg["sample_every"]

    h, insts = make_handle(she, cfg, she.STAT_SPATIAL | she.STAT_SK)
    cells = sum(i.ncells for i in insts)
    h.run(args.warmup)
    torch.cuda.synchronize()
    wall, kms, nev = timed_region(torch, h, args.steps, every)
    st0 = h.stats(0)
    h.close()
    value = cells * args.steps / wall
    ms_per_step = wall / args.steps * 1e3

    # FE runs two steps per launch (every sampling period here is even), PC one;
    # the algorithmic bytes are 8 B per cell-update either way
    per_launch = 2 if args.scheme == "fe" else 1
    launch_ms = kms * per_launch
    bytes_per_launch = 8.0 * cells * per_launch
    achieved = bytes_per_launch / (launch_ms * 1e-3) / 1e9
    traffic = read_traffic(cells) if args.scheme == "fe" else None  # counted on the FE kernel
    roofline = dict(bound="hbm", achieved=achieved, peak=HBM_PEAK_GBS, unit="GB/s", frac=achieved / HBM_PEAK_GBS,
                    traffic=traffic, kernel="k_step2d<float,8,heat,%s>" % ("fe x2" if per_launch == 2 else args.scheme),
                    kernel_ms=launch_ms, kernel_launches_timed=nev // per_launch,
                    cell_updates_per_launch=cells * per_launch, algorithmic_bytes_per_launch=bytes_per_launch,
                    valu=read_valu(launch_ms, every // per_launch) if args.scheme == "fe" else None)

    out = {"metric": METRIC, "value": value, "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": cfg["name"], "grid": [512, 512], "realisations": args.realisations,
                      "scheme": args.scheme, "r": 0.1, "eps": 1e-2, "sample_every": every,
                      "stats": "spatial mean/variance + radially binned S(k) per sample (FP64 sums)", "parallelism": "single GPU"},
           "roofline": roofline}

    if not args.no_plain:
        pcfg = W.c3(realisations=1, scheme=scheme)
        ph, pinsts = make_handle(she, pcfg, she.STAT_SPATIAL | she.STAT_SK, tuning_flags=she.TUNE_SINGLE_STEP)
        ph.run(args.warmup)
        psteps = max(200, args.steps // 2)
        pwall, pkms, _ = timed_region(torch, ph, psteps, every)
        ph.close()
        out["plain"] = {"value": pinsts[0].ncells * psteps / pwall, "ms_per_step": pwall / psteps * 1e3,
                        "kernel_ms": pkms, "form": "1 realisation, one kernel launch per step, no graph"}
        out["batched_over_plain"] = value / out["plain"]["value"]
    if not args.no_error:
        err_steps = 20
        out["error"] = {"state_max_rel_vs_fp64_oracle": state_error(she, torch, cfg, args.realisations - 1,
                                                                     err_steps),
                        "steps": err_steps, "realisation": args.realisations - 1,
                        "stats_samples": st0["n_samples"]}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(cfg, args.cpu_seconds)
    if args.copy_calibration:
        src = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_calibration_bytes"] = {"read": src.numel() * 4, "write": dst.numel() * 4}
        del src, dst
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
