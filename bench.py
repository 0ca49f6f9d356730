"""Benchmark: cell-updates/s of the batched FP32 step on one MI355X.

Workload (the batched FP32 configuration the metric is quoted on): 2D
periodic stochastic heat equation, 512 x 512 cells x 256 independent
realisations, forward Euler, r = 0.1, eps = 1e-2, T0 = 1 plus an equilibrium
perturbation; the equal-time statistics (spatial mean and variance, radially
binned S(k)) are sampled every 10 steps.  A "step" is one time step of all
256 realisations (Philox + Box-Muller face noise, face fluxes, divergence
update, and the sampling and S(k) transforms on sample steps).  Inputs are
resident in HBM when the timed region starts.

Printed: one JSON line with
  * the throughput of the whole step;
  * the roofline of the step kernel: its duration from HIP events around its
    back-to-back launches on the library's stream inside the timed region,
    against the VALU issue peak (the kernel is bound by instruction issue:
    committed SQ_INSTS_VALU counters) and against the HBM peak (algorithmic 8
    B per FP32 cell-update, and the bus bytes of committed FETCH_SIZE /
    WRITE_SIZE counters);
  * the plain single-realisation rate (one launch per step, no graph);
  * the error of the run at the workload's stated configuration (1e4 steps,
    burn-in 1e3, batches of 45 samples): state of the last realisation
    against the FP64 oracle, spatial variance and S(k) shells against the
    scheme's closed forms with batch-means error bars.  Its GPU run goes
    first, straight ahead of the warm-up, so that the timed steps find the
    GPU past the slower first ~50 ms of load after idle; its oracle check
    comes after the timed region;
  * the oracle's own rate on the host CPU, single-thread and all-core.

--workload c1|c2|c4|c5 prints the same kind of line for the other
configurations (throughput with their statistics, an error leg each, and for
c5 the roofline of the 3D step kernel).
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
PEAK_CLOCK_GHZ = 2.4
# non-packed VALU issue: 256 CUs x 4 SIMDs x 16 lanes per clock (a wave64
# instruction takes 4 cycles on a SIMD) at the 2.4 GHz peak clock
VALU_PEAK_TLANE = 256 * 4 * 16 * PEAK_CLOCK_GHZ * 1e9 / 1e12
SIMDS = 1024
CSRC = os.path.join(ROOT, "paper_2406_12157_amd", "csrc")
PROFILES = os.path.join(ROOT, "profiles")


def _section(text: str, start: str, end: str) -> str:
    i = text.index(start)
    return text[i:text.index(end, i) + len(end)]


def kernel_hash(variant: str) -> str:
    """Hash of what decides a step kernel's instruction stream and HBM
    traffic: the kernel header, the transform header (the row transforms of
    sample launches), the noise header, the translation unit that
    instantiates the kernel (variant: she_k2d_f32x8.hip for c3, she_k3d_f32.hip
    for c5), the host functions that pick its launch shapes and the parameter
    structs it takes.  Counter records carry it; a record whose hash differs
    is stale and not used."""
    h = hashlib.sha256()
    for name in ("she_step_nd.hpp", "she_fft.hpp", "she_rng.hpp", variant):
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(f.read())
    with open(os.path.join(CSRC, "she_capi.hip")) as f:
        t = f.read()
    for start in ("static she_status plan_nd(", "static she_status build_plan("):
        h.update(_section(t, start, "\n}\n").encode())
    with open(os.path.join(CSRC, "she_internal.hpp")) as f:
        t = f.read()
    for start in ("struct InstND {", "struct ParamsND {", "struct StepArg {"):
        h.update(_section(t, start, "\n};\n").encode())
    return h.hexdigest()[:16]


def read_record(name: str, variant: str):
    """A committed counter record (profiles/<name>), or None if absent or
    stale."""
    try:
        with open(os.path.join(PROFILES, name)) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    return rec if rec.get("kernel_hash") == kernel_hash(variant) else None


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
    the step kernel inside them.  Each sampling period's back-to-back
    non-sample steps, an even number of them (2D FE takes two steps per
    launch), are one call bracketed by events on the library's stream (torch's
    current stream).  The pair of steps that holds the sample step follows
    unbracketed as one call: the pair that ends on it when the distance to it
    is even, else the pair that starts with it (a two-step launch may sample
    either of its steps).  Steps past the last sample step of the region go
    bracketed in pairs, and a last odd one alone.  The calls are planned and
    their events created and recorded once before the region starts, so the
    region holds no first-use cost of the event machinery.  Returns (wall
    seconds, kernel ms per step, steps timed)."""
    plan = []                # (steps, bracketed)
    t, done = h.steps, 0
    while done < steps:
        d = (every - t % every) % every or every    # steps until the next sample step completes
        left = steps - done
        if left < d:
            # no sample step in what is left
            plain = left - left % 2
            calls = [(plain, True), (left - plain, False)]
        else:
            plain = d - 2 if d % 2 == 0 else d - 1
            calls = [(plain, True), (min(2, left - plain), False)]
        for k, br in calls:
            if k > 0:
                plan.append((k, br))
                t += k
                done += k
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) if br else None
          for _, br in plan]
    for e in ev:
        if e:
            e[0].record()
            e[1].record()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for (k, br), e in zip(plan, ev):
        if br:
            e[0].record()
            h.run(k)
            e[1].record()
        else:
            h.run(k)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    timed = [(e, k) for (k, br), e in zip(plan, ev) if br]
    n = sum(k for _, k in timed)
    kms = sum(e[0].elapsed_time(e[1]) for e, _ in timed) / max(1, n)
    return wall, kms, n


# ---------------------------------------------------------------- closed forms

def gamma_beta(r: float, ns):
    """gamma = (1/n) sum_{k != 0} h_k and beta = (1/n) sum_{k != 0} h_k
    cos^2(pi k_x / n_x), h_k = 1 / (1 - x_k / 2), x_k = 4 r sum_d
    sin^2(pi k_d / n_d): the FE stationary spectrum of a periodic grid."""
    import numpy as np
    s2 = [np.sin(np.pi * np.arange(n) / n) ** 2 for n in ns]
    x = 4.0 * r * sum(np.meshgrid(*s2, indexing="ij"))
    h = 1.0 / (1.0 - 0.5 * x)
    cos2 = np.meshgrid(*([1.0 - s2[0]] + [np.ones(n) for n in ns[1:]]), indexing="ij")[0]
    h.flat[0] = 0.0
    n = float(np.prod(ns))
    return float(h.sum() / n), float((h * cos2).sum() / n), h


def shell_mean(values, ns):
    """Average of a mode array over the shells round(|k|), signed k."""
    import numpy as np
    ks = [np.where(2 * np.arange(n) < n, np.arange(n), np.arange(n) - n) for n in ns]
    k2 = sum(g.astype(float) ** 2 for g in np.meshgrid(*ks, indexing="ij"))
    b = np.floor(np.sqrt(k2) + 0.5).astype(int)
    nb = int(np.floor(np.sqrt(sum(0.25 * n * n for n in ns)) + 0.5)) + 1
    s = np.bincount(b.ravel(), weights=values.ravel(), minlength=nb)
    c = np.bincount(b.ravel(), minlength=nb)
    return np.where(c > 0, s / np.maximum(c, 1), 0.0), c


def oracle_desc(oracle, i, precision):
    import numpy as np
    r, s = i["r"], float(np.sqrt(2 * i["r"] * i["eps"]))
    if precision == 0:
        r, s = float(np.float32(r)), float(np.float32(s))
    return oracle.Desc(dim=len(i["n"]), n=tuple(i["n"]) + (1,) * (3 - len(i["n"])), eq=i["eq"], bc=i["bc"],
                       scheme=i["scheme"], noise=i["noise"], r=r, sigma=s, u0=i["u0"], u_left=i["u_left"],
                       u_right=i["u_right"], init_sd=i["init_sd"], seed=i["seed"], realisation=i["realisation"])


def max_rel(a, b):
    import numpy as np
    return float(np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300)))


def c3_error_start(she, cfg, batch=45):
    """Creates the error leg's handle (the workload at its stated
    configuration, in the benchmark's launch shapes), reads the last
    realisation's initial field and enqueues the stated steps; c3_error
    finishes the leg.  Returns the leg's state."""
    h, _ = make_handle(she, cfg, she.STAT_SPATIAL | she.STAT_SK, burn_in=cfg["burn_in"], batch_samples=batch)
    q_last = len(cfg["instances"]) - 1
    u = h.read_field(q_last)
    h.run(cfg["steps"])
    return h, q_last, u


def c3_error(cfg, leg):
    """The error leg: state of the last realisation against the FP64 oracle
    after the stated steps, and the statistics of all realisations against
    the closed forms (spatial variance eps m^2 gamma / (1 - eps beta_x) per
    realisation, m its conserved mean; S(k) shells k != 0 against N_tot eps
    m^2 h_k / (1 - eps beta_x) averaged over the shell), each with its error
    bar: batch-means SE for the spatial variance, the spread over
    realisations for the shells (their slow modes outlast the batches)."""
    import numpy as np
    import oracle
    oracle.set_threads(0)
    h, q_last, u = leg
    i0 = cfg["instances"][0]
    n, eps, r = tuple(i0["n"]), i0["eps"], i0["r"]
    got = h.read_field(q_last)
    stats = [h.stats(q, sk=True, se=True) for q in range(len(cfg["instances"]))]
    h.close()
    gamma, beta, hk = gamma_beta(r, n)
    ncell = float(np.prod(n))
    m = np.array([g["sum_u"] / ncell for g in stats])
    var_th = eps * m * m * gamma / (1.0 - eps * beta)
    rel = np.array([g["var"][0] for g in stats]) / var_th - 1.0
    se_rel = np.array([g["var_se"][0] for g in stats]) / var_th
    sh, modes = shell_mean(hk, n)
    ok = modes > 0
    ok[0] = False
    qbar = eps * m * m / (1.0 - eps * beta)
    relk = np.array([g["sk"][ok] for g in stats]) / (ncell * qbar[:, None] * sh[None, ok]) - 1.0
    rk, sek = relk.mean(axis=0), relk.std(axis=0, ddof=1) / np.sqrt(len(stats))
    t0 = time.perf_counter()
    oracle.advance(oracle_desc(oracle, cfg["instances"][q_last], 0), u, 0, cfg["steps"])
    return {"state_max_rel_vs_fp64_oracle": max_rel(got, u), "state_steps": cfg["steps"], "realisation": q_last,
            "oracle_seconds": time.perf_counter() - t0,
            "samples": stats[0]["n_samples"], "batches": stats[0]["n_batches"],
            "spatial_variance": {"closed_form_m1": eps * gamma / (1.0 - eps * beta),
                                 "rel_mean_over_realisations": float(rel.mean()),
                                 "se_rel_of_mean": float(np.sqrt(np.sum(se_rel ** 2)) / len(rel)),
                                 "max_abs_rel_over_realisations": float(np.max(np.abs(rel))),
                                 "within_1e-3_plus_4.5se": bool(np.all(np.abs(rel) <= 1e-3 + 4.5 * se_rel))},
            "sk_shells": {"shells": int(ok.sum()), "max_abs_rel_mean": float(np.max(np.abs(rk))),
                          "within_1e-3_plus_4.5se": bool(np.all(np.abs(rk) <= 1e-3 + 4.5 * sek))}}


# ---------------------------------------------------------------- CPU baseline

def cpu_info():
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        avail = len(os.sched_getaffinity(0))
    except AttributeError:
        avail = os.cpu_count()
    return model, os.cpu_count(), avail


def cpu_baseline(cfg, seconds: float):
    """The oracle (FP64) on one realisation of the workload: about seconds/2
    on one thread, then seconds/2 on every core it may use (its OpenMP
    loops over independent faces and cells); rates in cell-updates/s.  The
    all-core rate is `value`, with the threads it used."""
    import numpy as np
    import oracle
    i = cfg["instances"][0]
    d = oracle_desc(oracle, i, 1)
    model, logical, avail = cpu_info()
    rates = {}
    steps_done = {}
    for threads in (1, avail):
        oracle.set_threads(threads)
        u = oracle.init(d)
        st = oracle.Stats(d, burn_in=0, every=cfg["sample_every"], per_cell=False)
        steps, t_used = 0, 0.0
        t0 = time.perf_counter()
        while t_used < seconds / 2:
            oracle.advance(d, u, steps, 5, st)
            steps += 5
            t_used = time.perf_counter() - t0
        rates[threads] = d.ncells * steps / t_used
        steps_done[threads] = (steps, t_used)
    used = oracle.get_threads()
    oracle.set_threads(0)
    n = "x".join(str(v) for v in i["n"])
    return dict(value=rates[avail], unit="cell-updates/s", cores=used, kind="oracle",
                sample="1 of %d realisations, %s, FE with sampling every %d: %d steps in %.1f s on %d threads; "
                       "%d steps in %.1f s on 1 thread" % (len(cfg["instances"]), n, cfg["sample_every"],
                                                           steps_done[avail][0], steps_done[avail][1], used,
                                                           steps_done[1][0], steps_done[1][1]),
                single_thread=rates[1], cpu_model=model, logical_cpus=logical, cpus_available=avail)


# ---------------------------------------------------------------- roofline

def roofline(kms_per_step, cells, per_launch, every, kernel, variant, valu_file, traffic_file):
    """Roofline of a step kernel from its HIP-event time per step, which
    brackets the launches outside sample steps only.  Bound: the VALU issue
    when a counter record for this kernel exists (achieved = lane-instructions
    of such a launch, SQ_INSTS_VALU x 64, over the launch time; peak =
    non-packed issue of 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz), else HBM.
    The sample launches' count (which includes the row transforms of S(k)
    in 2D) is reported beside it.  The HBM
    side is reported either way: algorithmic bytes (8 B per FP32
    cell-update) and, from a FETCH_SIZE / WRITE_SIZE record, the bus bytes."""
    launch_ms = kms_per_step * per_launch
    cu = cells * per_launch
    alg_bytes = 8.0 * cu
    alg_gbs = alg_bytes / (launch_ms * 1e-3) / 1e9
    hbm = dict(achieved=alg_gbs, peak=HBM_PEAK_GBS, unit="GB/s", frac=alg_gbs / HBM_PEAK_GBS,
               algorithmic_bytes_per_launch=alg_bytes)
    traffic = None
    t = read_record(traffic_file, variant) if traffic_file else None
    if t:
        traffic = t["hbm_bytes_per_launch"]
        bus = traffic / (launch_ms * 1e-3) / 1e9
        hbm.update(bus_bytes_per_launch=traffic, bus_achieved=bus, bus_frac=bus / HBM_PEAK_GBS,
                   source="profiles/" + traffic_file)
    out = dict(kernel=kernel, kernel_ms=launch_ms, cell_updates_per_launch=cu, traffic=traffic, hbm=hbm)
    v = read_record(valu_file, variant) if valu_file else None
    if v:
        q = v["valu_insts_per_launch"]
        qs = v.get("sample_valu_insts_per_launch") or q
        lane = q * 64
        ach = lane / (launch_ms * 1e-3) / 1e12
        out.update(bound="alu", achieved=ach, peak=VALU_PEAK_TLANE, unit="Tlane-instr/s", frac=ach / VALU_PEAK_TLANE,
                   lane_instr_per_launch=lane, lane_instr_per_cell_update=lane / cu,
                   sample_lane_instr_per_launch=qs * 64, valu_source="profiles/" + valu_file)
    else:
        out.update(bound="hbm", achieved=alg_gbs, peak=HBM_PEAK_GBS, unit="GB/s", frac=alg_gbs / HBM_PEAK_GBS)
    return out


def copy_bandwidth(torch, nbytes, reps=10):
    """Device-to-device copy rate (GB/s, bytes read + written) at a footprint
    of nbytes each way: the streaming rate this part reaches there, the
    second reference of the HBM roofline (the first is the 8 TB/s peak)."""
    n = nbytes // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        dst.copy_(src)
    b.record()
    torch.cuda.synchronize()
    gbs = 2.0 * n * 4 * reps / (a.elapsed_time(b) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return gbs


def add_copy_reference(roof, gbs):
    """HBM fractions of a roofline against the measured copy rate."""
    hbm = roof["hbm"]
    hbm["copy_achieved"] = gbs
    hbm["frac_of_copy"] = hbm["achieved"] / gbs
    if "bus_achieved" in hbm:
        hbm["bus_frac_of_copy"] = hbm["bus_achieved"] / gbs


# ---------------------------------------------------------------- other workloads

def checked_leg(fn, *args):
    """Runs a leg that follows the timed region (error check, CPU baseline); a
    leg that raises is reported in the line, with its message, instead of
    ending the run before the line is printed."""
    try:
        return fn(*args)
    except Exception as e:  # noqa: BLE001 - reported, not swallowed
        return {"failed": "%s: %s" % (type(e).__name__, e)}


def other_error_start(she, name, cfg, stats):
    """Creates the error leg's handles of c1, c2, c4 or c5, reads the initial
    fields it checks and enqueues their runs; other_error finishes the leg.
    Returns the leg's state."""
    import numpy as np
    leg = {}
    if name == "c4":
        insts = cfg["instances"]
        h, _ = make_handle(she, cfg, 0)
        ns = np.array([i["n"][0] for i in insts])
        picks = sorted({int(np.argmax(ns)), int(np.argmin(ns)), 17, 503})
        init = {q: h.read_field(q) for q in picks}
        h.step(cfg["steps"])
        leg["state"] = (h, picks, init, cfg["steps"])
        return leg
    steps = 3 if name == "c5" else (cfg["steps"] if name == "c1" else 100000)
    h, _ = make_handle(she, cfg, 0)
    u = h.read_field(0)
    h.step(steps)
    leg["state"] = (h, [0], {0: u}, steps)
    if name in ("c1", "c5"):
        L = 450 if name == "c1" else 4
        hv, _ = make_handle(she, cfg, stats, burn_in=cfg["burn_in"], batch_samples=L)
        hv.run(cfg["steps"])
        leg["var"] = hv
    return leg


def other_error(name, cfg, leg):
    """Error leg of c1, c2, c4, c5: the state against the FP64 oracle on the
    same noise (c1 and c2 over their stated runs, c4 on sampled instances
    over its 1e4 steps, c5 over 3 full-size steps), and where the scheme fixes
    it the spatial variance against its closed form with its batch-means
    error bar (c1: eps m^2 gamma / (1 - eps beta); c5: (m / dV) gamma)."""
    import numpy as np
    import oracle
    oracle.set_threads(0)
    prec = cfg["precision"]
    insts = cfg["instances"]
    h, picks, init, steps = leg["state"]
    errs = []
    for q in picks:
        u = init[q].copy()
        oracle.advance(oracle_desc(oracle, insts[q], prec), u, 0, steps)
        errs.append(max_rel(h.read_field(q), u))
    h.close()
    out = {"state_max_rel_vs_fp64_oracle": max(errs), "state_steps": steps}
    if name == "c4":
        out["instances_checked"] = picks
        return out
    inst = insts[0]
    n = tuple(inst["n"])
    if "var" in leg:
        hv = leg["var"]
        g = hv.stats(0, se=True)
        hv.close()
        gamma, beta, _ = gamma_beta(inst["r"], n)
        m = g["sum_u"] / float(np.prod(n))
        want = inst["eps"] * m * m * gamma / (1.0 - inst["eps"] * beta) if name == "c1" else m * inst["eps"] * gamma
        rel = g["spatial_var"] / want - 1.0
        out["spatial_variance"] = {"value": g["spatial_var"], "closed_form": want, "rel": rel,
                                   "se_rel": g["spatial_var_se"] / want, "batches": g["n_batches"],
                                   "within_1e-3_plus_4.5se": bool(abs(rel) <= 1e-3 + 4.5 * g["spatial_var_se"] / want)}
    return out


def other_workload(args, torch, she, W):
    """Throughput of c1, c2, c4 or c5 with the statistics its configuration
    names, timed over `--steps` steps after `--warmup` (she_run, burn-in 0).
    The 1D workloads keep their state in registers, so they are bound by the
    per-step latency of the resident kernel, not by HBM; c5 gets the roofline
    of its step kernel as c3 does."""
    name = args.workload
    cfg = {"c1": W.c1, "c2": W.c2, "c4": W.c4, "c5": W.c5}[name]()
    stats = {"c1": she.STAT_MOMENTS | she.STAT_CORR, "c2": she.STAT_MOMENTS | she.STAT_CORR, "c4": 0,
             "c5": she.STAT_SPATIAL}[name]
    h, insts = make_handle(she, cfg, stats)
    cells = sum(i.ncells for i in insts)
    # the error leg's GPU runs go first, straight ahead of the warm-up (as
    # for c3); its oracle checks follow the timed region
    leg = None if args.no_error else other_error_start(she, name, cfg, stats)
    h.run(args.warmup)
    torch.cuda.synchronize()
    roof = None
    if name == "c5":
        wall, kms, _ = timed_region(torch, h, args.steps, cfg["sample_every"])
        roof = roofline(kms, cells, 1, cfg["sample_every"], "k_step3d<float,4,dk,fe>", "she_k3d_f32.hip",
                        "valu_step3d_c5.json", "traffic_step3d_c5.json")
        h.close()
        add_copy_reference(roof, copy_bandwidth(torch, 4 * cells))
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
           "roofline": roof}
    if not args.no_error:
        out["error"] = checked_leg(other_error, name, cfg, leg)
    print(json.dumps(out), flush=True)


# ---------------------------------------------------------------- main

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--realisations", type=int, default=256)
    ap.add_argument("--scheme", choices=["fe", "pc"], default="fe")
    ap.add_argument("--cpu-seconds", type=float, default=20.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-error", action="store_true")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one 1 GiB device-to-device copy (reference for HBM counters)")
    ap.add_argument("--workload", choices=["c3", "c1", "c2", "c4", "c5"], default="c3",
                    help="c3 (default): the benchmark line; the others: a line of that workload with its "
                         "statistics and error leg")
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
    # The error leg's GPU run (its stated 1e4 steps, about a second) goes
    # first, straight ahead of the warm-up: the first ~50 ms of load after the
    # GPU has been idle, even briefly, run 10-20% slower than the steady state
    # (the part's power management), and a short timed region would measure
    # that transient.  Its oracle check follows the timed region.
    err_cfg = W.c3(realisations=args.realisations, scheme=scheme)
    leg = None if args.no_error else c3_error_start(she, err_cfg)
    h.run(args.warmup)
    torch.cuda.synchronize()
    wall, kms, _ = timed_region(torch, h, args.steps, every)
    h.close()
    value = cells * args.steps / wall
    ms_per_step = wall / args.steps * 1e3

    # FE runs two steps per launch (every sampling period here is even), PC
    # one; the counter records were taken on the FE kernel
    fe = args.scheme == "fe"
    roof = roofline(kms, cells, 2 if fe else 1, every,
                    "k_step2d<float,8,heat,%s>" % ("fe x2" if fe else "pc"), "she_k2d_f32x8.hip",
                    "valu_step2d_c3.json" if fe else None, "traffic_step2d_c3.json" if fe else None)
    add_copy_reference(roof, copy_bandwidth(torch, 4 * cells))
    out = {"metric": METRIC, "value": value, "unit": "cell-updates/s", "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": cfg["name"], "grid": [512, 512], "realisations": args.realisations,
                      "scheme": args.scheme, "r": 0.1, "eps": 1e-2, "sample_every": every,
                      "stats": "spatial mean/variance + radially binned S(k) per sample (FP64 sums)",
                      "parallelism": "single GPU"},
           "roofline": roof}

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
        out["error"] = checked_leg(c3_error, err_cfg, leg)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = checked_leg(cpu_baseline, cfg, args.cpu_seconds)
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
