#!/usr/bin/env python
"""Benchmark: pair-exchange evaluations per second on one MI355X.

Workload (default ``water96``): cubic box L = 23.5 bohr, 96^3 grid, 256
localised Gaussian orbitals band-limited to 20 Ha, erfc-screened kernel
w = 0.106 bohr^-1 -- a synthetic stand-in for the paper's 64-water-like
condensed-phase boxes.  One step is one SCF step's exchange work on the GPU:
Loewdin orthonormalisation (float64), K psi for all 32,896 orbital pairs with
E_x (float32 FFT path), and the exchange matrix M = dV Psi^T (K Psi).

Prints one JSON line.  ``value`` = pairs / second of the whole step.  The
``roofline`` object is measured live with HIP events around every launch of
the dominant pass during the timed steps; ``cpu_baseline`` times the float64
CPU oracle on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "pair-exchange evals/s and K-psi time per SCF step, FP32 vs FP64 at fixed dE_x"
HBM_PEAK_GBS = 8000.0
MFMA_FP32_PEAK_TFLOPS = 157.3


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


# sources of the pair-pipeline kernels: a recorded traffic figure applies only
# to the kernels built from exactly these files
TRAFFIC_SOURCES = ("fft.hpp", "exchange_kernels.hpp", "exchange_f32.hip", "exchange_f64.hip")


def kernel_sources_sha1():
    import hashlib
    h = hashlib.sha1()
    for name in TRAFFIC_SOURCES:
        with open(os.path.join(ROOT, "paper_2309_00651_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def traffic_from_profiles(kernel_pass, workload):
    """HBM bytes per launch measured by rocprofv3 counters (profiles/), or None
    when none are recorded or the kernels' sources changed since."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel_pass}_{workload}.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            rec = json.load(f)
        if rec.get("sources_sha1") != kernel_sources_sha1():
            return None
        return rec.get("bytes_per_launch")
    except Exception:
        return None


def cpu_baseline(system, psi, seconds_target=10.0):
    """Time the float64 oracle on a subset of orbitals of the same workload."""
    import numpy as np

    import oracle
    cores = max(1, min(os.cpu_count() or 1, 16))
    vg = oracle.coulomb_kernel(system.shape, system.box, system.kernel, system.param)
    # probe: one pair to size the sample
    t0 = time.perf_counter()
    oracle.pair_energy(psi[0], psi[1], vg, 1.0)
    t_pair = max(time.perf_counter() - t0, 1e-4)
    pairs_target = seconds_target * cores / t_pair
    k = int(max(4, min(system.n_orb, (math.sqrt(8 * pairs_target + 1) - 1) / 2)))
    sub = np.ascontiguousarray(psi[:k])
    t0 = time.perf_counter()
    oracle.exchange(sub, system.box, vg, workers=cores)
    dt = time.perf_counter() - t0
    pairs = k * (k + 1) // 2
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            model = next((ln.split(":", 1)[1].strip() for ln in f
                          if ln.startswith("model name")), None)
    except OSError:
        pass
    return {"value": pairs / dt, "unit": "pair-exchange evals/s", "cores": cores,
            "kind": "oracle", "host_cpus": os.cpu_count(), "cpu_model": model,
            "sample": f"{k} of {system.n_orb} orbitals ({pairs} pairs) of the {system.name} "
                      f"workload, float64, scipy FFT, {cores} worker processes, {dt:.1f} s"}


TUNE_CACHE = os.path.join(ROOT, "paper_2309_00651_amd", "tune", "mi355x.txt")


def _passes(prof, steps):
    """Per-pass time per step and rate of the method's bytes (the library's
    algorithmic tally: each operand read or written once, pair grids on the
    kept kz planes only)."""
    return {k: {"ms_per_step": v["ms"] / steps,
                "GBps": (v["bytes"] / (v["ms"] * 1e-3) / 1e9) if v["ms"] > 0 else None,
                "frac_of_hbm_peak": (v["bytes"] / (v["ms"] * 1e-3) / 1e9 / HBM_PEAK_GBS)
                if v["ms"] > 0 else None}
            for k, v in prof.items()}


PAIR_PASSES = ("pair_fwd", "plane", "inv_acc", "rows_fwd", "cols_conv", "rows_inv")


def _pipeline_frac(prof):
    ms = sum(prof[k]["ms"] for k in PAIR_PASSES if k in prof)
    by = sum(prof[k]["bytes"] for k in PAIR_PASSES if k in prof)
    return (by / (ms * 1e-3) / 1e9 / HBM_PEAK_GBS) if ms > 0 else None


def _event_times(fn, steps, warmup):
    """Per-call times (ms) from HIP events on the current stream, after
    warm-up calls."""
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
    ev[0].record()
    for k in range(steps):
        fn()
        ev[k + 1].record()
    torch.cuda.synchronize()
    return [ev[k].elapsed_time(ev[k + 1]) for k in range(steps)]


def _median(xs):
    xs = sorted(xs)
    n = len(xs)
    return xs[n // 2] if n % 2 else 0.5 * (xs[n // 2 - 1] + xs[n // 2])


def _golden_ex(name):
    path = os.path.join(ROOT, "tests", "golden", f"{name}_full_oracle.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)["ex"]


def measure_batched6(steps, warmup, options, tune_cache, singles=True):
    """Six systems of different grids in one plan: K psi + E_x for all of
    them, (a) replayed from a captured hipGraph, (b) launched eagerly from the
    same plan (systems on forked streams), (c) six single-system plans in
    turn.  Per-system kernel configurations come from the tune cache (plan
    option tune_cache=); the per-pass rates are those of one profiled eager
    call."""
    import torch

    from paper_2309_00651_amd import hfx
    from workloads import configs

    systems = configs.BATCHED6
    dev = torch.device("cuda:0")
    specs = [hfx.SystemSpec(s.n, s.box, s.n_orb, s.kernel, s.param) for s in systems]
    n_pairs = sum(s.n_pairs for s in systems)
    log(f"batched6: generating {len(systems)} systems, {n_pairs} pairs")
    psi = torch.cat([torch.from_numpy(s.orbitals().reshape(-1)) for s in systems]).to(dev)
    opts = options
    if tune_cache and os.path.exists(tune_cache):
        opts = f"{options};tune_cache={tune_cache}" if options else f"tune_cache={tune_cache}"
    plan = hfx.Plan(specs, hfx.FP32, options=opts, device=dev)
    kpsi = torch.empty(psi.shape, dtype=torch.float32, device=dev)
    ex = torch.empty(len(systems), dtype=torch.float64, device=dev)
    log("batched6: graph replay")
    g = plan.graph(hfx.GRAPH_APPLY, psi, kpsi, ex)
    t_graph = _event_times(g.launch, steps, warmup)
    ex_graph = [float(x) for x in ex.cpu()]
    log("batched6: eager multi-system plan")
    t_eager = _event_times(lambda: plan.apply_exchange(psi, kpsi=kpsi, ex=ex), steps, 1)
    assert [float(x) for x in ex.cpu()] == ex_graph, "graph replay and eager launch disagree"
    g.close()
    # the batch's algorithmic bytes (the library's tally: pair grids on the
    # kept kz planes only) over the graph replay's time
    plan.profile(True)
    plan.apply_exchange(psi, kpsi=kpsi, ex=ex)
    prof_all = plan.profile_read()
    plan.profile(False)
    describe = [plan.describe(i) for i in range(len(systems))]
    del plan
    ms_graph = _median(t_graph)
    bytes_all = sum(v["bytes"] for v in prof_all.values())
    bytes_pipe = sum(prof_all[k]["bytes"] for k in PAIR_PASSES if k in prof_all)
    out = {"pairs": n_pairs, "ms_graph_replay_median": ms_graph,
           "ms_graph_replay_mean": sum(t_graph) / len(t_graph),
           "ms_eager_one_plan_median": _median(t_eager),
           "pairs_per_s": n_pairs / (ms_graph * 1e-3), "steps": steps,
           "algorithmic_GB_per_call": bytes_all / 1e9,
           "hbm_frac_of_graph_replay": bytes_all / (ms_graph * 1e-3) / 1e9 / HBM_PEAK_GBS,
           "pair_pipeline_bytes_frac_of_graph_replay":
               bytes_pipe / (ms_graph * 1e-3) / 1e9 / HBM_PEAK_GBS,
           "kernel_configs": describe, "plan_options": opts, "ex": ex_graph}
    gold = [_golden_ex(s.name) for s in systems]
    if all(x is not None for x in gold):
        out["rel_dEx_vs_oracle_max"] = max(abs(a - b) / abs(b) for a, b in zip(ex_graph, gold))
    if singles:
        log("batched6: six single-system plans in turn")
        plans = [hfx.Plan(sp, hfx.FP32, options=opts, device=dev) for sp in specs]
        views, off = [], 0
        for s in systems:
            k = s.n_orb * s.n ** 3
            views.append((psi[off:off + k], kpsi[off:off + k]))
            off += k

        def seq():
            for pl, (pv, kv) in zip(plans, views):
                pl.apply_exchange(pv, kpsi=kv)
        t_seq = _event_times(seq, max(2, steps // 2), 1)
        out["ms_six_single_plans_median"] = _median(t_seq)
        out["batch_gain_vs_single_plans"] = _median(t_seq) / ms_graph
        # per-pass rates of the kernels, each system's plan profiled alone (in
        # the batched plan the systems' launches overlap, which stretches every
        # event-timed launch)
        per = {}
        for sname, pl, (pv, kv) in zip([s.name for s in systems], plans, views):
            pl.profile(True)
            pl.apply_exchange(pv, kpsi=kv)
            pr = pl.profile_read()
            pl.profile(False)
            per[sname] = {k: v for k, v in _passes(pr, 1).items() if k in PAIR_PASSES}
            per[sname]["pair_pipeline_hbm_frac"] = _pipeline_frac(pr)
        out["passes_per_system"] = per
        del plans
    del psi, kpsi
    torch.cuda.empty_cache()
    return out


def measure_size_classes(steps, warmup):
    """Sixteen small systems on one grid with uneven orbital counts (24^3,
    L = 10 bohr, 8..23 random plane-wave orbitals, 5 Ha, truncated Coulomb):
    K psi + E_x of all of them per call, replayed from a graph, (a) with size
    classes (the default here: two classes of eight systems, each batch step
    one launch per pass), (b) with group=0 (sixteen forked launch sequences),
    (c) sixteen single plans in turn.  All three give the same results bit
    for bit."""
    import numpy as np
    import torch

    from paper_2309_00651_amd import hfx
    from workloads import generate

    dev = torch.device("cuda:0")
    n, L = 24, 10.0
    counts = list(range(8, 24))
    psis = [generate.random_pw((n,) * 3, (L,) * 3, no, 5.0, 20231300 + no) for no in counts]
    specs = [hfx.SystemSpec(n, (L,) * 3, no) for no in counts]
    flat = torch.from_numpy(np.concatenate([p.reshape(-1) for p in psis])).to(dev)
    n_pairs = sum(no * (no + 1) // 2 for no in counts)
    out = {"systems": len(counts), "grid": n, "orbitals": counts, "pairs": n_pairs}
    ex_ref = None
    for tag, opt in (("classes", "ecut=5"), ("group0", "ecut=5;group=0")):
        plan = hfx.Plan(specs, hfx.FP32, options=opt, device=dev)
        kpsi = torch.empty(flat.shape, dtype=torch.float32, device=dev)
        ex = torch.empty(len(counts), dtype=torch.float64, device=dev)
        g = plan.graph(hfx.GRAPH_APPLY, flat, kpsi, ex)
        t = _event_times(g.launch, steps, warmup)
        e = [float(x) for x in ex.cpu()]
        if ex_ref is None:
            ex_ref = e
        assert e == ex_ref, "grouped and per-system launches disagree"
        out[f"ms_graph_{tag}"] = _median(t)
        out[f"classes_{tag}"] = sorted({plan.describe(i).split("class=")[1]
                                        for i in range(len(counts))})
        g.close()
        del plan, kpsi
    plans = [hfx.Plan(sp, hfx.FP32, options="ecut=5", device=dev) for sp in specs]
    views, off = [], 0
    kp = torch.empty(flat.shape, dtype=torch.float32, device=dev)
    for no in counts:
        k = no * n ** 3
        views.append((flat[off:off + k], kp[off:off + k]))
        off += k

    def seq():
        for pl, (pv, kv) in zip(plans, views):
            pl.apply_exchange(pv, kpsi=kv)
    out["ms_single_plans"] = _median(_event_times(seq, steps, warmup))
    out["pairs_per_s_classes"] = n_pairs / (out["ms_graph_classes"] * 1e-3)
    out["gain_vs_group0"] = out["ms_graph_group0"] / out["ms_graph_classes"]
    out["gain_vs_single_plans"] = out["ms_single_plans"] / out["ms_graph_classes"]
    del plans, flat, kp
    torch.cuda.empty_cache()
    return out


def measure_large128(steps, warmup, options, fp64_steps):
    """The 128^3 / 512-orbital box: K psi + E_x of all 131,328 pairs on the
    raw generated orbitals (the input of the stored full-loop reference), in
    float32 and float64, with per-pass rates from a profiled call."""
    import torch

    from paper_2309_00651_amd import hfx
    from workloads import configs

    s = configs.LARGE128
    dev = torch.device("cuda:0")
    log(f"large128: generating {s.n_orb} orbitals on {s.n}^3")
    psi = torch.from_numpy(s.orbitals()).to(dev)
    spec = hfx.SystemSpec(s.n, s.box, s.n_orb, s.kernel, s.param)
    out = {"pairs": s.n_pairs}
    gold = _golden_ex(s.name)
    for prec, tag, n_steps in ((hfx.FP32, "fp32", steps), (hfx.FP64, "fp64", fp64_steps)):
        if n_steps <= 0:
            continue
        plan = hfx.Plan(spec, prec, options=options, device=dev)
        kpsi = torch.empty(psi.shape, dtype=plan.kpsi_dtype, device=dev)
        ex = torch.empty(1, dtype=torch.float64, device=dev)
        log(f"large128 {tag}: {warmup} warm-up + {n_steps} timed calls")
        t = _event_times(lambda: plan.apply_exchange(psi, kpsi=kpsi, ex=ex), n_steps, warmup)
        plan.profile(True)
        plan.apply_exchange(psi, kpsi=kpsi, ex=ex)
        prof = plan.profile_read()
        plan.profile(False)
        e = float(ex[0])
        out[tag] = {"ms_median": _median(t), "ms_mean": sum(t) / len(t), "calls": n_steps,
                    "pairs_per_s": s.n_pairs / (_median(t) * 1e-3), "passes": _passes(prof, 1),
                    "pair_pipeline_hbm_frac": _pipeline_frac(prof), "ex": e,
                    "kernel_config": plan.describe()}
        if gold is not None:
            out[tag]["rel_dEx_vs_oracle"] = abs(e - gold) / abs(gold)
        del plan, kpsi
        torch.cuda.empty_cache()
    if "fp32" in out and "fp64" in out:
        out["fp32_speedup_vs_fp64"] = out["fp64"]["ms_median"] / out["fp32"]["ms_median"]
    del psi
    torch.cuda.empty_cache()
    return out


def bench_batched6(args):
    """--workload batched6: the six-system batch as its own JSON line."""
    r = measure_batched6(args.steps, args.warmup, args.options, args.tune_cache)
    line = {
        "metric": "pair-exchange evals/s, six systems of different grids in one batch",
        "value": r["pairs_per_s"], "unit": "pair-exchange evals/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": r["ms_graph_replay_mean"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batched6: grids 64^3..120^3 at spacing 23.5/96 bohr, 64..384 "
                               "random plane-wave orbitals (5 Ha), truncated Coulomb; step = "
                               "K psi + E_x for all six systems",
                   "pairs": r["pairs"], "plan_options": r["plan_options"]},
        "extra": r,
    }
    print(json.dumps(line), flush=True)


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="water96")
    ap.add_argument("--fp64-steps", type=int, default=3)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-smtace", action="store_true",
                    help="skip the s-MTACE screening timings (profiled runs of the step)")
    ap.add_argument("--options", default=None, help="float32 plan options, e.g. 'tiles=2'")
    ap.add_argument("--fp64-options", default=None, help="float64 plan options")
    ap.add_argument("--no-band-limit", action="store_true",
                    help="do not tell the plans the workload's orbital cutoff (ecut=); the "
                         "passes then also transform the kz planes beyond the pair band")
    ap.add_argument("--tune-cache", default=TUNE_CACHE,
                    help="tune cache of the batched plan's per-system configurations")
    ap.add_argument("--no-extra-workloads", action="store_true",
                    help="skip the six-system batch and the 128^3 box after the main workload")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run only a plain 1 GiB device-to-device copy (5 times): the "
                         "reference dispatch for scaling rocprofv3 FETCH_SIZE/WRITE_SIZE")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path "
              f"(asked for --gpus {args.gpus}, WORLD_SIZE={world}).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.copy_calibration:
        n = 1 << 28  # 2^28 float32 = 1 GiB read + 1 GiB written per copy
        src = torch.ones(n, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": 4 * n, "copies": 5}), flush=True)
        return

    # The synthetic orbitals are band-limited by construction ((1/2)|G|^2 <=
    # ecut of the workload), so the plans are told the cutoff (plan option
    # ecut=) unless --no-band-limit: kz planes beyond the pair densities' band
    # are then skipped (exact up to rounding; parity tests cover both forms).
    from workloads import configs as _cfg
    cuts = {s.ecut for s in (_cfg.BATCHED6 if args.workload == "batched6"
                             else [_cfg.ALL[args.workload]])}
    args.default_options = args.options is None and args.fp64_options is None
    if not args.no_band_limit and len(cuts) == 1:
        band = f"ecut={cuts.pop():g}"
        args.options = band if args.options is None else f"{band};{args.options}"
        args.fp64_options = band if args.fp64_options is None else f"{band};{args.fp64_options}"
    else:
        args.default_options = False

    if args.workload == "batched6":
        bench_batched6(args)
        return

    from paper_2309_00651_amd import hfx
    from workloads import configs

    system = configs.ALL[args.workload]
    log(f"generating {system.name}: n={system.n} n_orb={system.n_orb}")
    psi = system.orbitals()
    dev = torch.device("cuda:0")
    spec = hfx.SystemSpec(system.n, system.box, system.n_orb, system.kernel, system.param)
    psi0 = torch.from_numpy(psi).to(dev)
    n_pairs = system.n_pairs

    def run(prec, steps, warmup, profile):
        opts = args.fp64_options if prec == hfx.FP64 else args.options
        plan = hfx.Plan(spec, prec, options=opts, device=dev)
        p = psi0.clone()
        kpsi = torch.empty(p.shape, dtype=plan.kpsi_dtype, device=dev)
        ex = torch.empty(1, dtype=torch.float64, device=dev)
        m = torch.empty(system.n_orb ** 2, dtype=torch.float64, device=dev)
        plan.workspace()

        def step():
            plan.orthonormalize(p)
            plan.apply_exchange(p, kpsi=kpsi, ex=ex)
            plan.exchange_matrix(p, kpsi, m=m)
        for _ in range(warmup):
            step()
        torch.cuda.synchronize()
        if profile:
            plan.profile(True)
        # one event between consecutive steps: the mean over the timed
        # region and the median of the steps come from the same record
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
        t0 = time.perf_counter()
        ev[0].record()
        for k in range(steps):
            step()
            ev[k + 1].record()
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        per_step = [ev[k].elapsed_time(ev[k + 1]) for k in range(steps)]
        ev_ms = ev[0].elapsed_time(ev[steps])
        prof = plan.profile_read() if profile else None
        plan.profile(False)
        out = dict(ms=ev_ms / steps, ms_median=_median(per_step), wall_ms=1e3 * wall / steps,
                   prof=prof, ex=float(ex[0]), m=m, kpsi=kpsi, psi=p, describe=plan.describe())
        return out, plan

    def time_ace(plan, r, reps=3):
        """ACE (Eq. (vx_ace)) from the step's K psi and M: projector build and
        one application to all orbitals, each timed with HIP events; E_x from
        1/2 sum <psi|V^ACE psi> as a check."""
        p = plan.ace_build(r["kpsi"], r["m"])
        o = plan.ace_apply(p, r["psi"])
        torch.cuda.synchronize()

        def ev(fn):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(reps):
                fn()
            b.record()
            b.synchronize()
            return a.elapsed_time(b) / reps
        t_build = ev(lambda: plan.ace_build(r["kpsi"], r["m"], p=p))
        t_apply = ev(lambda: plan.ace_apply(p, r["psi"], out=o))
        dv = system.L ** 3 / system.n ** 3
        ex_ace = 0.5 * dv * float(torch.sum(r["psi"] * o))
        del p, o
        return t_build, t_apply, ex_ace

    def time_screen(psi_o, rho_cut, reps=3):
        """s-MTACE screening (pairs with int |psi_a psi_b| >= rho_cut) of the
        step's orthonormal orbitals: the screening call (host wall time) and
        K psi + E_x over the kept pairs, against the unscreened call, each
        timed with HIP events on a fresh float32 plan."""
        plan = hfx.Plan(spec, hfx.FP32, options=args.options, device=dev)
        kpsi = torch.empty(psi_o.shape, dtype=plan.kpsi_dtype, device=dev)
        ex = torch.empty(1, dtype=torch.float64, device=dev)

        def ev():
            plan.apply_exchange(psi_o, kpsi=kpsi, ex=ex)
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(reps):
                plan.apply_exchange(psi_o, kpsi=kpsi, ex=ex)
            b.record()
            b.synchronize()
            return a.elapsed_time(b) / reps, float(ex[0])
        t_full, e_full = ev()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        kept = plan.screen(psi_o, rho_cut)[0]
        t_scr = 1e3 * (time.perf_counter() - t0)
        info = plan.schedule_info()
        t_kept, e_kept = ev()
        plan.profile(True)
        plan.apply_exchange(psi_o, kpsi=kpsi, ex=ex)
        prof = plan.profile_read()
        plan.profile(False)
        passes = {k: {"ms": v["ms"], "GBps": v["bytes"] / (v["ms"] * 1e-3) / 1e9 if v["ms"] > 0
                      else None}
                  for k, v in prof.items() if k in ("pair_fwd", "plane", "inv_acc")}
        out = {"rho_cut": rho_cut, "pairs_kept": kept, "pairs": n_pairs, "passes": passes,
               "pair_grids": info[2], "tile_pairs": info[1], "batches": info[0],
               "screen_call_ms": t_scr, "kpsi_ms_screened": t_kept, "kpsi_ms_all_pairs": t_full,
               "speedup": t_full / t_kept, "rel_dEx_screening": abs(e_kept - e_full) / abs(e_full)}
        del plan, kpsi
        return out

    def time_scdm(psi_o, reps=2):
        """SCDM localisation of the step's orthonormal orbitals (pivoted QR
        pivots, density-matrix columns, Loewdin), timed with HIP events, and
        the pairs an s-MTACE cut of 2.5e-2 keeps on its output."""
        plan = hfx.Plan(spec, hfx.FP32, options=args.options, device=dev)
        phi, piv = plan.scdm(psi_o)
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            plan.scdm(psi_o, phi=phi, pivots=piv)
        b.record()
        b.synchronize()
        kept = plan.screen(phi, 2.5e-2)[0]
        del plan, phi
        return {"scdm_ms": a.elapsed_time(b) / reps, "pairs_kept_rho_2.5e-2_after_scdm": kept}

    # achievable HBM rate on this device: device-to-device copy of 1 GiB
    # (1 GiB read + 1 GiB written), median of 5, timed with HIP events
    def copy_rate():
        src = torch.ones(1 << 28, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        times = []
        for _ in range(5):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            dst.copy_(src)
            b.record()
            b.synchronize()
            times.append(a.elapsed_time(b))
        del src, dst
        return 2.0 * (1 << 30) / (sorted(times)[2] * 1e-3) / 1e9
    copy_gbps = copy_rate()
    log(f"device copy: {copy_gbps:.0f} GB/s")

    log(f"fp32: {args.warmup} warm-up + {args.steps} timed steps")
    r32, plan32 = run(hfx.FP32, args.steps, args.warmup, True)
    ms = r32["ms"]
    prof = r32["prof"]
    # dominant pass by summed time
    dom = max(prof.items(), key=lambda kv: kv[1]["ms"])
    dname, d = dom
    if dname == "contract":
        achieved = d["flops"] / (d["ms"] * 1e-3) / 1e12
        roof = {"bound": "mfma", "achieved": achieved, "peak": MFMA_FP32_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / MFMA_FP32_PEAK_TFLOPS, "traffic": None}
    else:
        achieved = d["bytes"] / (d["ms"] * 1e-3) / 1e9
        # counters were taken with the default plan options (the workload's cutoff)
        tr = traffic_from_profiles(dname, system.name) if args.default_options else None
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBS, "traffic": tr}
    roof["kernel"] = dname
    roof["launches"] = d["launches"]
    roof["avg_launch_ms"] = d["ms"] / max(d["launches"], 1)
    passes = {k: {"ms_per_step": v["ms"] / args.steps,
                  "GBps": (v["bytes"] / (v["ms"] * 1e-3) / 1e9) if v["ms"] > 0 else None,
                  "TFLOPs": (v["flops"] / (v["ms"] * 1e-3) / 1e12) if v["ms"] > 0 else None}
              for k, v in prof.items()}
    pair_ms = sum(prof[k]["ms"] for k in ("pair_fwd", "plane", "inv_acc", "rows_fwd",
                                          "cols_conv", "rows_inv") if k in prof) / args.steps
    hbm_pair_bytes = sum(prof[k]["bytes"] for k in ("pair_fwd", "plane", "inv_acc", "rows_fwd",
                                                    "cols_conv", "rows_inv") if k in prof)
    exch_frac = hbm_pair_bytes / args.steps / (pair_ms * 1e-3) / 1e9 / HBM_PEAK_GBS
    log(f"fp32 {ms:.2f} ms/step, dominant pass {dname} {achieved:.1f}")

    ace_build_ms, ace_apply_ms, ex_ace = time_ace(plan32, r32)
    log(f"ace: build {ace_build_ms:.2f} ms, apply {ace_apply_ms:.2f} ms")
    smtace = [] if args.no_smtace else [time_screen(r32["psi"], rc) for rc in (2.5e-2, 2.0e-3)]
    scdm = None if args.no_smtace else time_scdm(r32["psi"])
    if scdm:
        log(f"scdm: {scdm['scdm_ms']:.1f} ms")
    for sc in smtace:
        log(f"s-MTACE rho_cut {sc['rho_cut']:g}: {sc['pairs_kept']} of {n_pairs} pairs, "
            f"K psi {sc['kpsi_ms_screened']:.2f} ms (all pairs {sc['kpsi_ms_all_pairs']:.2f} ms)")
    del r32["kpsi"], r32["m"], r32["psi"]

    extra = {"kpsi_ms_per_step_fp32": pair_ms, "pair_pipeline_hbm_frac": exch_frac,
             "ace_build_ms": ace_build_ms, "ace_apply_ms": ace_apply_ms,
             "ace_apply_fp64_tflops": 4.0 * system.n_orb ** 2 * system.n ** 3 / (ace_apply_ms * 1e-3) / 1e12,
             "rel_dEx_ace_vs_exact": abs(ex_ace - r32["ex"]) / abs(r32["ex"]),
             "device_copy_GBps": copy_gbps,
             "pair_pipeline_frac_of_device_copy": exch_frac * HBM_PEAK_GBS / copy_gbps,
             "dominant_frac_of_device_copy": (achieved / copy_gbps) if roof["bound"] == "hbm" else None,
             "passes": passes, "ex_fp32": r32["ex"], "s_mtace": smtace, "scdm": scdm,
             "kernel_config_fp32": r32["describe"]}
    if not args.no_fp64:
        log(f"fp64: 1 warm-up + {args.fp64_steps} timed steps")
        r64, _ = run(hfx.FP64, args.fp64_steps, 1, True)
        p64 = {k: {"ms_per_step": v["ms"] / args.fp64_steps,
                   "GBps": (v["bytes"] / (v["ms"] * 1e-3) / 1e9) if v["ms"] > 0 else None}
               for k, v in r64["prof"].items()}
        extra.update({"ms_per_step_fp64": r64["ms"], "ex_fp64": r64["ex"], "passes_fp64": p64,
                      "kernel_config_fp64": r64["describe"],
                      "fp32_speedup_vs_fp64": r64["ms"] / ms,
                      "rel_dEx_fp32_vs_fp64": abs(r32["ex"] - r64["ex"]) / abs(r64["ex"])})
        del r64
    extra["ms_per_step_median_fp32"] = r32["ms_median"]
    extra["timing"] = ("HIP events between consecutive steps on the launching stream; "
                       "ms_per_step is the mean over the timed steps, the median is reported "
                       "beside it; per-pass times come from event brackets around every launch")
    del plan32
    torch.cuda.empty_cache()
    if not args.no_extra_workloads:
        band5 = None if args.no_band_limit else "ecut=5"
        band20 = None if args.no_band_limit else "ecut=20"
        extra["batched6"] = measure_batched6(5, 1, band5, args.tune_cache)
        b6 = extra["batched6"]
        log(f"batched6: graph replay {b6['ms_graph_replay_median']:.1f} ms "
            f"({b6['pairs_per_s']:.0f} pairs/s), six single plans "
            f"{b6.get('ms_six_single_plans_median', float('nan')):.1f} ms")
        extra["size_classes"] = measure_size_classes(5, 2)
        sc = extra["size_classes"]
        log(f"size classes: {sc['ms_graph_classes']:.2f} ms (group=0 {sc['ms_graph_group0']:.2f}"
            f", single plans {sc['ms_single_plans']:.2f})")
        extra["large128"] = measure_large128(3, 1, band20, 0 if args.no_fp64 else 2)
        l1 = extra["large128"]
        log(f"large128: fp32 {l1['fp32']['ms_median']:.1f} ms "
            f"({l1['fp32']['pairs_per_s']:.0f} pairs/s)")
    golden = os.path.join(ROOT, "tests", "golden", f"{system.name}_oracle.json")
    if os.path.exists(golden):
        with open(golden) as f:
            g = json.load(f)
        extra["rel_dEx_fp32_vs_oracle"] = abs(r32["ex"] - g["ex"]) / abs(g["ex"])

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cpu = cpu_baseline(system, psi)

    line = {
        "metric": METRIC,
        "value": n_pairs / (ms * 1e-3),
        "unit": "pair-exchange evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{system.name}: L={system.L} bohr, {system.n}^3 grid, "
                               f"{system.n_orb} "
                               + ("localised Gaussian" if system.family == "gaussians"
                                  else "random plane-wave")
                               + f" orbitals ({system.ecut:g} Ha), "
                               + (f"erfc w={system.param}" if system.kernel == 1
                                  else "truncated Coulomb")
                               + f"; step = orthonormalise + K psi (all {n_pairs} pairs) + "
                               "E_x + exchange matrix",
                   "n": system.n, "n_orb": system.n_orb, "pairs": n_pairs,
                   "precision": "fp32 FFT/kernel, fp64 orthonormalisation and sums",
                   "plan_options": args.options, "fp64_plan_options": args.fp64_options},
        "roofline": roof,
        "cpu_baseline": cpu,
        "extra": extra,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
