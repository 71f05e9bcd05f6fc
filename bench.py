"""Benchmark of the crack LBM hot path on one MI355X.

A step is one time step of the method: the fused collide-stream sweep over the
whole plate followed by the crack step (K_III, criterion, tip advance, newly
severed links).  Default workload: the 16384 x 8192 plate (134M sites) with a
4096-site edge crack driven at 0.5 c_s, run with the state stored as FP64,
FP32, FP16 and BF16 (the last three shifted by the static equilibrium, FP32
arithmetic), in the five-population layout and in the equilibrium layout
(rest population and w only; the moving populations are rebuilt from the
equilibrium of their emitting site, exact at omega = 1), with one to eight
time steps per sweep ("-tb", "-tb3" .. "-tb8": two to eight steps per sweep,
each step's crack step still run).

Per storage: a warm-up on the timed plate itself (start-up steps, code
loading, clocks), one timed interval of --steps steps (HIP events on the
solver's stream), the field error at its end against the first storage (FP64,
five populations), and a short leg of whole T-step sweeps with per-launch
events for the sweep kernel's duration.  Then an untimed leg runs the whole
10000-step workload in a few storages for the K_III(t) errors (the load
waves reach the crack only after ~8200 steps).

The JSON line reports the headline storage's GLUPS (FP16, equilibrium layout,
eight steps per sweep, stochastic rounding) as `value`; `roofline` is that of
the one-step five-population FP16 sweep (28 B per site update), and
`roofline_headline_kernel` the headline kernel's fraction in its own bytes.

    python bench.py [--steps K] [--warmup W] [--storage f16s-eq-tb8-sr] [--workload precision]
"""
from __future__ import annotations

import argparse
import dataclasses
import hashlib
import json
import math
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
METRIC = "GLUPS and % of HBM roofline, fp16-storage vs fp32 at stated K_III error"


def parse_storage(name: str):
    """Storage name -> (storage, rounding, layout): a "-sr" suffix selects
    stochastic rounding of the 16-bit stores, an "-eq" part the equilibrium
    layout (rest population and w only), an "-eq-tb" part that layout with
    two time steps per sweep ("-eq-tb3" .. "-eq-tb8": three to eight), e.g.
    "f16s-eq-tb3-sr"."""
    rounding = "nearest"
    if name.endswith("-sr"):
        name, rounding = name[:-3], "stochastic"
    name = re.sub(r"-tb[2-8]?$", "", name)
    layout = "full"
    if name.endswith("-eq"):
        name, layout = name[:-3], "eq"
    return name, rounding, layout


def time_block(name: str) -> int:
    """Time steps per sweep of a storage name ("-tb": 2, "-tb3" .. "-tb8": 3 .. 8)."""
    m = re.search(r"-tb([2-8]?)(-|$)", name)
    return (int(m.group(1)) if m.group(1) else 2) if m else 1


def block_kernel(name: str) -> str:
    """The sweep kernel a storage name runs."""
    return "sweep_block" if time_block(name) >= 2 else "sweep_step"


def sweep_bytes_per_site(name: str) -> float:
    """Algorithmic bytes of one sweep per site: read and write of the stored
    populations (five, or one in the equilibrium layout) and of w."""
    st, _, layout = parse_storage(name)
    e = {"f64": 8, "f32": 4, "f32plain": 4, "f16s": 2, "bf16s": 2}[st]
    we = 8 if st == "f64" else 4
    return 2.0 * ((1 if layout == "eq" else 5) * e + we) / time_block(name)


def plate_config(p, storage, trace_cap):
    """Solver config of plate p in the named storage (see parse_storage)."""
    from paper_2206_12412_amd import Config
    storage, rounding, layout = parse_storage(storage)
    return Config(nx=p.nx, ny=p.ny, storage=storage, rounding=rounding, layout=layout,
                  kappa=p.kappa, mu=p.mu, rho=p.rho,
                  has_crack=True, crack_x0=p.crack_x0, crack_tip=p.crack_tip, growth=p.growth,
                  v_rel=p.v_rel, K_C=p.K_C, r0=p.r0, v_max=p.v_max,
                  tau_hist=p.traction_history(), wdot0=p.wdot0(), trace_cap=trace_cap)


# the files (under csrc/) that shape the sweep kernels: their sources and the
# build flags
KERNEL_SOURCES = ("sweep.hip", "sweep2.hip", "sweep_block.hpp", "sweep_block_f64.hip",
                  "sweep_block_f32.hip", "sweep_block_f16.hip", "sweep_block_f16_t8.hip",
                  "sweep_block_bf16.hip", "sweep_core.hpp", "lbm_internal.hpp", "../build.py")


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2206_12412_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_for(storage: str, workload: str, sites: int):
    """HBM bytes per sweep launch from the committed rocprofv3 counter summary
    (FETCH_SIZE + WRITE_SIZE scaled by a copy kernel of known size), or None when
    no summary exists for this kernel source."""
    path = os.path.join(ROOT, "profiles", f"sweep_{storage}_{workload}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        t = json.load(fh)
    if t.get("kernel_source_sha") != kernel_source_hash():
        return None
    return t.get("bytes_per_launch")


def run_storage(p, storage, steps, warmup, torch, ref=None, tune=False):
    """Time `steps` steps of plate p in this storage, as one interval.

    The plate is warmed up by `warmup` steps of its own (at least the two
    five-plane start-up steps that a fresh equilibrium-layout plate runs, so
    those, code loading and clock ramp fall outside the timed interval); the
    interval is timed with HIP events on the solver's stream between two
    synchronisations.  After it, w is exported (compared with the reference
    run's w at the same step when one is given) and a short kernel-timing leg
    runs whole T-step sweeps with per-launch HIP events, so that the sweep
    kernel's launch duration is sampled on full sweeps only and the events do
    not perturb the timed interval.  The leg starts with two untimed sweeps
    (the export leaves the GPU idle, and the first sweeps after it run at a
    lower clock: with two samples of six steps the mean was 17 % above the
    kernel trace's) and samples at least four sweeps and 24 steps."""
    from paper_2206_12412_amd import Solver, plan_tail
    T = time_block(storage)
    warm = max(int(warmup), 2)
    k_steps = T * max(4, -(-24 // T))  # whole sweeps, at least four and 24 steps
    s = Solver(plate_config(p, storage, warm + steps + 2 * T + k_steps))
    tuned = s.autotune(trial_steps=5) if tune else None  # on a scratch copy of the plate
    if T >= 2:
        if tune:  # the T-step sweep's own shapes, also on a scratch copy
            tuned = {"one_step": tuned, "time_block": s.autotune_time_block(T)}
        else:
            s.set_time_block(T)
    s.step(warm)
    # the sweeps of the timed call: whole sweeps of T steps, then the planned
    # end of a call whose step count is not a multiple of T (the speculative
    # sweeps of the K criterion choose their own lengths)
    sweeps = None
    if T == 1:
        sweeps = [1] * steps
    elif p.growth != 2:
        tail = plan_tail(parse_storage(storage)[0], T, steps)
        sweeps = [T] * ((steps - sum(tail)) // T) + tail
    torch.cuda.synchronize()
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    start.record(s.stream)
    s.step(steps)
    stop.record(s.stream)
    torch.cuda.synchronize()
    ms = start.elapsed_time(stop)
    w = s.fields()[0]
    out = {
        "ms": ms,
        "glups": p.sites * steps / (ms * 1e-3) / 1e9,
        "bytes_per_site": s.bytes_per_site(),
        "sites": s.sites(),
        "launch": s.launch(),
        "autotune": tuned,
        "first_step": warm,
        "sweeps": sweeps,
    }
    if ref is None:
        out["w_end"] = w
    else:
        out["field_error"] = field_error(w, ref["w_end"])
        out["tip_path_identical"] = bool(np.array_equal(s.traces(warm, steps)["tip"],
                                                        ref["tip"]))
    if ref is None:
        out["tip"] = s.traces(warm, steps)["tip"]
    del w
    s.step(2 * T)
    s.timing(True, stride=1)
    s.step(k_steps)
    tm = s.timing(False)
    launches = tm["steps"] // T
    if launches:
        out["kernel_ms_per_launch"] = tm["sweep_ms"] / launches
        out["crack_ms_per_launch"] = tm["crack_ms"] / launches
        out["steps_per_launch"] = T
        out["timed_launches"] = launches
    s.close()
    del s
    torch.cuda.empty_cache()
    return out


def sweep_costs(p, storages, torch, out_md):
    """Time of one sweep of T = 1 .. 8 steps with the default shapes on plate
    p, per storage (per-sweep mean of twenty sweeps in one call, best of
    three), beside the table the library plans call ends from; writes a
    markdown summary."""
    from paper_2206_12412_amd import Solver, sweep_cost
    rows = []
    for storage in storages:
        st = parse_storage(storage)[0]
        s = Solver(plate_config(p, storage, 4000))
        s.step(4)
        got = {}
        for T in range(1, 9):
            s.set_time_block(T)
            s.step(2 * T)
            best = float("inf")
            for _ in range(3):
                a = torch.cuda.Event(enable_timing=True)
                b = torch.cuda.Event(enable_timing=True)
                a.record(s.stream)
                s.step(20 * T)
                b.record(s.stream)
                torch.cuda.synchronize()
                best = min(best, a.elapsed_time(b) * 1e3 / 20)
            got[T] = best
        s.close()
        del s
        torch.cuda.empty_cache()
        rows.append((storage, got, {T: sweep_cost(st, T) for T in range(1, 9)}))
        print(f"bench: sweep costs {storage}: " + ", ".join(f"{T}: {v:.1f}" for T, v in got.items()),
              file=sys.stderr, flush=True)
    cmd = "python3 bench.py " + " ".join(sys.argv[1:])
    out = [f"# Sweep time per step count: {os.path.basename(out_md)}", "",
           "Command:", "", "    " + cmd, "",
           f"Plate {p.nx} x {p.ny} ({p.name}), equilibrium layout, default launch shapes; "
           "us per sweep of T steps (20 sweeps in one call, best of three), and in brackets the "
           "table lbm_plan_tail works from (lbm_sweep_cost).", "",
           "| storage | " + " | ".join(f"T = {T}" for T in range(1, 9)) + " |",
           "|---|" + "---|" * 8]
    for storage, got, lib in rows:
        out.append(f"| {storage} | " + " | ".join(f"{got[T]:.1f} ({lib[T]:.1f})" for T in range(1, 9))
                   + " |")
    out += ["", "Per step (us), measured: "]
    for storage, got, _ in rows:
        out.append(f"* {storage}: " + ", ".join(f"T = {T} {got[T] / T:.1f}" for T in range(1, 9)))
    with open(out_md, "w") as fh:
        fh.write("\n".join(out) + "\n")
    print(f"wrote {out_md}", file=sys.stderr, flush=True)


def field_error(w, r):
    """RMS and max of w - r relative to the reference field (None where the
    reference is still zero)."""
    d = w - r
    rms_r = float(np.sqrt(np.mean(r * r)))
    if rms_r == 0:
        return {"rms_rel": None, "max_rel": None}
    return {"rms_rel": float(np.sqrt(np.mean(d * d))) / rms_r,
            "max_rel": float(np.abs(d).max() / np.abs(r).max())}


def run_k_leg(p, storage, steps, torch):
    """Untimed run of the whole workload (all `steps` steps, so that the load
    waves reach the crack and K is defined) for the K_III and field errors:
    returns the K trace and the final w."""
    from paper_2206_12412_amd import Solver
    T = time_block(storage)
    s = Solver(plate_config(p, storage, steps))
    if T >= 2:
        s.set_time_block(T)
    s.step(steps)
    K = s.sif(0, steps)
    tip = s.traces(0, steps)["tip"]
    w = s.fields()[0]
    s.close()
    del s
    torch.cuda.empty_cache()
    return {"K": K, "tip": tip, "w": w}


def copy_bandwidth(torch, mib: int = 4096, reps: int = 10) -> float:
    """GB/s of a plain streaming kernel that reads and writes every byte once
    (read + write counted): the practical ceiling of the sweeps.  An
    elementwise kernel (torch.neg on FP32) rather than a device copy, whose
    blit kernel reaches 4.6 TB/s on 4 GiB against 6.2 TB/s."""
    n = mib << 20
    a = torch.ones(n // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    torch.neg(a, out=b)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        torch.neg(a, out=b)
    e1.record()
    torch.cuda.synchronize()
    gbs = 2.0 * n * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return gbs


def k_errors(K, K_ref):
    """K_III error statistics against the reference trace (steps where the
    reference K is defined and non-zero)."""
    ok = ~np.isnan(K_ref) & (K_ref != 0)
    if not ok.any():
        return {"K_err_rel_max": None}
    Kmax = np.abs(K_ref[ok]).max()
    d = np.abs(K - K_ref)
    # the closing tenth of the run, where K is fully developed
    late = ok & (np.arange(len(K_ref)) >= int(0.9 * len(K_ref)))
    strong = ok & (np.abs(K_ref) >= 0.5 * Kmax)
    return {
        # max_n |K_n - K_n^ref| / max_n |K^ref|
        "K_err_rel_max": float(d[ok].max() / Kmax),
        # |K - K^ref| / |K^ref| at the last step
        "K_err_rel_final": float(d[-1] / abs(K_ref[-1])) if ok[-1] else None,
        # max_n |K_n - K_n^ref| / |K_n^ref| over the closing tenth of the run
        "K_err_rel_late_max": float((d[late] / np.abs(K_ref[late])).max()) if late.any() else None,
        # the same over every step with |K^ref| >= max |K^ref| / 2
        "K_err_rel_strong_max": float((d[strong] / np.abs(K_ref[strong])).max()),
    }


def cpu_baseline(p, budget_s: float):
    """The oracle as it stands on this host's cores, on the same plate (and a
    shorter single-core sample for reference)."""
    import oracle as O

    def rate(threads, budget):
        s = O.Oracle(O.OracleConfig(
            nx=p.nx, ny=p.ny, kappa=p.kappa, mu=p.mu, rho=p.rho, has_crack=True,
            crack_x0=p.crack_x0, crack_tip=p.crack_tip, growth=p.growth, v_rel=p.v_rel, K_C=p.K_C,
            r0=p.r0, v_max=p.v_max, tau_hist=p.traction_history(), trace_cap=0, threads=threads))
        s.step(1)  # first touch of the pages
        n, t0 = 0, time.perf_counter()
        while True:
            s.step(1)
            n += 1
            el = time.perf_counter() - t0
            if el >= budget:
                break
        s.close()
        return p.sites * n / el / 1e9, n, el

    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
    v, n, el = rate(threads, budget_s)
    v1, n1, el1 = rate(1, budget_s / 3)
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": v, "unit": "GLUPS", "cores": threads, "kind": "oracle",
            "sample": f"{n} steps of the full {p.nx}x{p.ny} plate, FP64, {el:.1f} s",
            "single_core": {"value": v1, "sample": f"{n1} steps, {el1:.1f} s"}, "cpu_model": model}


def run_batched(args, torch):
    """64 uneven plates: one batch (per-step launches and one persistent
    launch) against the same plates stepped one after another, each as its own
    single-plate solver.  Every plate's final field must agree bitwise."""
    import synth
    from paper_2206_12412_amd import Batch, Solver

    plates = synth.config_batched()
    steps = args.steps if args.steps is not None else plates[0].steps
    storage = args.batch_storage
    cfgs = [plate_config(p, storage, steps) for p in plates]
    sites = sum(p.sites for p in plates)
    say = lambda m: print(f"bench: {m}", file=sys.stderr, flush=True)  # noqa: E731

    def timed(fn):
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record()
        fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1)

    b = Batch(cfgs)
    tuned = None
    if not args.no_tune:
        say(f"batched: autotuning the launch shape ({len(plates)} plates, {sites} sites)")
        tuned = b.autotune(trial_steps=4)
        say(f"batched: tuned {tuned}")
    if args.warmup > 0:
        w = Batch([dataclasses.replace(c, trace_cap=0) for c in cfgs])
        w.set_launch(b.launch()["rows"], b.launch()["waves"], b.launch()["occupancy"])
        w.step(args.warmup)
        w.run_persistent(args.warmup)
        torch.cuda.synchronize()
        w.close()
        del w
    say(f"batched: per-step launches, {steps} steps")
    ms_step = timed(lambda: b.step(steps))
    bp = Batch(cfgs)
    shape = b.launch()
    bp.set_launch(shape["rows"], shape["waves"], shape["occupancy"])
    say(f"batched: one persistent launch, {steps} steps")
    ms_pers = timed(lambda: bp.run_persistent(steps))
    pers_blocks = bp.launch()["persistent_blocks"]
    say("batched: the same plates one after another")
    ms_seq = 0.0
    equal_seq = equal_pers = 0
    for k, c in enumerate(cfgs):
        s1 = Solver(c)
        ms_seq += timed(lambda: s1.step(steps))
        w1 = s1.fields()[0]
        equal_seq += int(np.array_equal(w1, b.plates[k].fields()[0]))
        equal_pers += int(np.array_equal(w1, bp.plates[k].fields()[0]))
        s1.close()
        del s1
    bps = sweep_bytes_per_site(storage)
    g = lambda ms: sites * steps / (ms * 1e-3) / 1e9  # noqa: E731
    best_ms = min(ms_step, ms_pers)
    achieved = sites * bps / (best_ms / steps * 1e-3) / 1e9
    line = {
        "metric": METRIC, "value": round(g(best_ms), 2), "unit": "GLUPS", "n_gpus": 1,
        "steps": steps, "warmup": args.warmup, "ms_per_step": round(best_ms / steps, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if parse_storage(storage)[0] == "f64" else "f32", "data": "synthetic",
        "config": {"workload": f"batched-{len(plates)}-plates", "plates": len(plates),
                   "sites": sites, "storage": storage, "parallelism": "single-gpu",
                   "mode": "per-step" if ms_step <= ms_pers else "persistent"},
        "batched_per_step_glups": round(g(ms_step), 2),
        "batched_persistent_glups": round(g(ms_pers), 2),
        "sequential_glups": round(g(ms_seq), 2),
        "speedup_vs_sequential": round(ms_seq / best_ms, 3),
        "launch": shape, "autotune": tuned, "persistent_blocks": pers_blocks,
        "bitwise_equal_plates": {"per_step": equal_seq, "persistent": equal_pers,
                                 "of": len(plates)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "whole batched step (all kernels)"},
    }
    b.close()
    bp.close()
    if not args.no_cpu:
        say("batched: oracle CPU baseline")
        line["cpu_baseline"] = cpu_baseline(plates[0], args.cpu_seconds)
    print(json.dumps(line), flush=True)


def run_strip(args, torch):
    """The steady-growth strip of Sec. 5.1 at v = 0.2 .. 0.8: K sampled 300
    times over the last 15 L / c_s against eq. (sif-mandal) and the paper's
    own statistics, with both boundary schemes (per-link bounce-back, and the
    paper's macroscopic scheme of Sec. 3.1), in FP64 and FP16 storage."""
    import synth
    from paper_2206_12412_amd import Solver
    with open(os.path.join(ROOT, "tests", "golden", "steady_strip_table.json")) as fh:
        table = json.load(fh)
    paper = {r[0]: dict(zip(table["columns"], r)) for r in table["rows"]}
    rows = {}
    for scheme in ("link", "macro"):
        for name in ("f64", "f16s-eq-sr"):
            st, rd, layout = parse_storage(name)
            for v in (0.2, 0.4, 0.6, 0.8):
                m = synth.mandal_strip(v)
                s = Solver(strip_config(st, rd, layout, dict(m["config"], bc_scheme=scheme)))
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                s.step(m["steps"])
                torch.cuda.synchronize()
                el = time.perf_counter() - t0
                K = s.traces()["K"][m["sample_steps"]] / math.sqrt(16.0)  # in units with L = 1
                s.close()
                q = np.percentile(K, [25, 50, 75])
                kt = m["K_theo"] / 4.0
                pr = paper[v]
                rows.setdefault(scheme, {}).setdefault(name, {})[str(v)] = {
                    "K_theo": round(kt, 5), "mean": round(float(K.mean()), 5),
                    "sigma": round(float(K.std()), 5), "median": round(float(q[1]), 5),
                    "minus_25": round(float(q[1] - q[0]), 5), "plus_75": round(float(q[2] - q[1]), 5),
                    "median_rel_to_theo": round(float(q[1] / kt - 1.0), 4),
                    "paper_median_rel_to_theo": round(pr["median"] / pr["K_theo"] - 1.0, 4),
                    "median_in_paper_band": bool(pr["median"] - pr["minus_25"] <= q[1]
                                                 <= pr["median"] + pr["plus_75"]),
                    "theo_in_band": bool(q[0] <= kt <= q[2]),
                    "sites": m["config"]["nx"] * m["config"]["ny"], "steps": m["steps"],
                    "ms_per_step": round(el * 1e3 / m["steps"], 4)}
    worst = max(abs(r["median_rel_to_theo"]) for r in rows["macro"]["f64"].values())
    line = {"metric": "K_III of steady crack growth in a strip against eq. (sif-mandal)",
            "value": worst, "unit": "max |median / K_theo - 1| over v (macroscopic scheme, FP64)",
            "n_gpus": 1, "higher_is_better": False, "data": "synthetic",
            "config": {"workload": "steady-strip (Sec. 5.1), 2L x (0.5 + v t_f + 2.5) L, dh = L/16"},
            "schemes": rows}
    print(json.dumps(line), flush=True)


def strip_config(storage, rounding, layout, kw):
    from paper_2206_12412_amd import Config
    return Config(storage=storage, rounding=rounding, layout=layout, **kw)


def run_adjoint(args, torch):
    """2048 x 1024 plate with a stationary 512-site crack, 5000 steps: the
    sensor-trace loss against a run with a 10 % sinusoidal traction
    perturbation, its gradient with respect to the traction history and the
    initial velocity from the discrete adjoint, the adjoint's cost against the
    forward run, and central differences (FP64 runs) along 16 unit directions."""
    import synth
    from paper_2206_12412_amd import Config, Solver

    p = synth.config_adjoint()
    T = args.steps if args.steps is not None else p.steps
    sens = synth.adjoint_sensors(p.nx, p.ny)
    storage = args.adjoint_storage
    say = lambda m: print(f"bench: {m}", file=sys.stderr, flush=True)  # noqa: E731
    base = dict(nx=p.nx, ny=p.ny, has_crack=True, crack_x0=p.crack_x0, crack_tip=p.crack_tip,
                sensors=sens, trace_cap=T)
    tau0 = np.full(T, p.tau)

    def run(name, tau, wd0=None):
        """(solver after T steps, its sensor traces, ms of the T steps)"""
        st, rd, layout = parse_storage(name)
        s = Solver(Config(storage=st, rounding=rd, layout=layout, tau_hist=tau, wdot0=wd0, **base))
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(s.stream)
        s.step(T)
        e1.record(s.stream)
        torch.cuda.synchronize()
        return s, s.sensor_traces(), e0.elapsed_time(e1)

    def traces(st, tau, wd0=None):
        s, tr, _ = run(st, tau, wd0)
        s.close()
        return tr

    say(f"adjoint: target run, {T} steps")
    target = traces("f64", synth.adjoint_target_history(T, tau0=p.tau))
    if args.warmup > 0:
        st, rd, layout = parse_storage(storage)
        w = Solver(Config(storage=st, rounding=rd, layout=layout, tau_hist=tau0,
                          **dict(base, trace_cap=args.warmup)))
        w.step(args.warmup)
        torch.cuda.synchronize()
        w.close()
    say(f"adjoint: forward run ({storage})")
    s, tr, fwd_ms = run(storage, tau0)
    loss = float(((tr - target) ** 2).sum())
    g = torch.from_numpy(2.0 * (tr - target)).cuda()
    say("adjoint: backward run")
    s.adjoint(g)  # first call: code objects
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dtau, dwd0, _, adj_ms = s.adjoint(g, timing=True)
    adj_wall_ms = (time.perf_counter() - t0) * 1e3
    s.close()
    dwd0 = dwd0.cpu().numpy()
    say("adjoint: central differences on FP64 runs")
    h = 1e-4
    fd, ad = [], []
    for d_tau, d_wd in synth.adjoint_directions(T, (p.ny, p.nx), count=args.directions):
        lp = float(((traces("f64", tau0 + h * d_tau, h * d_wd) - target) ** 2).sum())
        lm = float(((traces("f64", tau0 - h * d_tau, -h * d_wd) - target) ** 2).sum())
        fd.append((lp - lm) / (2 * h))
        ad.append(float(dtau @ d_tau + (dwd0 * d_wd).sum()))
    fd, ad = np.array(fd), np.array(ad)
    sites = p.nx * p.ny
    # the adjoint state is FP64 or FP32 whatever the forward storage; five
    # planes + W, or plane 0 + W in the equilibrium layout
    ae = 8 if parse_storage(storage)[0] == "f64" else 4
    bps = 2.0 * ((1 if parse_storage(storage)[2] == "eq" else 5) * ae + ae)
    sweep_ms = adj_ms / (T + 1)
    achieved = sites * bps / (sweep_ms * 1e-3) / 1e9
    line = {
        "metric": METRIC, "value": round(sites * (T + 1) / (adj_ms * 1e-3) / 1e9, 2),
        "unit": "GLUPS", "n_gpus": 1, "steps": T, "warmup": args.warmup,
        "ms_per_step": round(sweep_ms, 4), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64" if ae == 8 else "f32", "data": "synthetic",
        "config": {"workload": f"adjoint-{p.nx}x{p.ny}", "nx": p.nx, "ny": p.ny,
                   "crack_sites": p.ell, "sensors": int(len(sens)), "storage": storage,
                   "parallelism": "single-gpu"},
        "loss": loss,
        "forward_ms_per_step": round(fwd_ms / T, 4),
        "adjoint_ms_per_step": round(sweep_ms, 4),
        "adjoint_over_forward": round((adj_ms / (T + 1)) / (fwd_ms / T), 3),
        "adjoint_wall_ms": round(adj_wall_ms, 1),
        "recomputed_forward_steps": 0,
        "gradient_check": {
            "directions": int(len(fd)), "h": h, "reference": "central differences of FP64 runs",
            "rel_err_norm": float(np.linalg.norm(ad - fd) / np.linalg.norm(fd)),
            "rel_err_max": float(np.max(np.abs(ad - fd) / np.abs(fd))),
        },
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "kernel": "adj_step (whole adjoint sweep, one launch per step)"},
    }
    print(json.dumps(line), flush=True)


def _read_csv(path):
    import csv
    with open(path) as fh:
        return list(csv.DictReader(fh))


def _short(name: str) -> str:
    for key in ("sweep_step", "sweep_block_edges", "sweep_block_tall", "sweep_block",
                "crack_seq", "crack_kernel", "batch_step", "batch_crack",
                "batch_persistent", "adj_step", "adj_inject", "adj_export", "copyBuffer", "init_rows",
                "export_rows", "zero_kernel", "init_mask"):
        if key in name:
            return key
    return name[:40]


def _instance(name: str) -> str:
    """Storage and template flags of a sweep kernel name, mangled or not
    (the demangler of this ROCm prints __bf16 as `bool _Accum`): e.g.
    "f16 sr eq fused" for sweep_step, "f16 T=6 rows=32" for the T-step ones."""
    if "DF16b" in name or "__bf16" in name or "bool _Accum" in name:
        st = "bf16"
    elif "DF16_" in name or "_Float16" in name:
        st = "f16"
    elif "Ifff" in name or "<float" in name:
        st = "f32"
    elif "Iddd" in name or "<double" in name:
        st = "f64"
    else:
        return ""
    if "sweep_step" in name:
        m = re.search(r"Li[24]E((?:Lb[01]E){4})", name)
        flags = [c == "1" for c in re.findall(r"Lb([01])E", m.group(1))] if m else None
        if flags is None:
            m = re.search(r", [24], (true|false), (true|false), (true|false), (true|false)>", name)
            flags = [x == "true" for x in m.groups()] if m else None
        if not flags:
            return st
        shift, sr, eq, fused = flags
        return " ".join([st] + (["sr"] if sr else []) + (["eq"] if eq else ["five planes"]) +
                        (["+crack step"] if fused else []))
    if "sweep_block" in name:
        head = name.split("(")[0]  # the template arguments, not the parameter types
        ints = re.findall(r"Li(\d+)E", head) or re.findall(r", (\d+)(?=[,>])", head)
        ints = [int(x) for x in ints]
        sr = "ELb1ELi" in head or re.search(r", true, \d+, \d+", head) is not None
        if "tall" in name and len(ints) >= 3:
            return f"{st}{' sr' if sr else ''} T={ints[-1]} rows={ints[-2]}"
        if len(ints) >= 2:
            return f"{st}{' sr' if sr else ''} T={ints[-1]} rows={ints[-2]}"
    return st


def summarize_trace(dirpath: str, out_md: str, command: str):
    """Markdown summary of a `rocprofv3 --kernel-trace --stats` run."""
    rows = _read_csv(os.path.join(dirpath, "run_kernel_stats.csv"))
    lines = [f"# Kernel trace: {os.path.basename(out_md)}", "", "Command:", "",
             f"    {command}", "", "| kernel | instance | calls | avg us | min us | max us | % time | full name |",
             "|---|---|---|---|---|---|---|---|"]
    for r in rows:
        lines.append(f"| {_short(r['Name'])} | {_instance(r['Name'])} | {r['Calls']} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | "
                     f"{float(r['Percentage']):.2f} | `{r['Name'][:110]}` |")
    with open(out_md, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def summarize_pmc(fetch_dir: str, write_dir: str, storage: str, workload: str, copy_bytes: int,
                  command: str, out_dir: str):
    """HBM bytes per sweep launch from FETCH_SIZE and WRITE_SIZE runs,
    each scaled by the same counter's reading for a device copy of copy_bytes.
    The sweep is the sweep_step instantiation with the most launches (in the
    equilibrium layout the first two steps of a fresh plate run the
    five-plane instantiation, which is left out); for a time-blocked storage
    ("-tb", "-tb3" .. "-tb8") the T-step sweep, whose two launches
    (sweep_block or sweep_block_tall over the fast chunks of the strips without
    a plate edge, sweep_block_edges over the rest) are summed, each the
    instantiation with the most launches."""
    import synth
    p = {"precision": synth.config_precision, "sif": synth.config_sif_fp32,
         "plain": synth.config_plain_fp64}[workload]()
    out = {"storage": storage, "workload": workload, "kernel_source_sha": kernel_source_hash(),
           "command": command, "copy_bytes": copy_bytes}
    total = 0.0
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = [r for r in _read_csv(os.path.join(d, "run_counter_collection.csv"))
                if r["Counter_Name"] == counter]
        copy = max(float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"])
        factor = copy_bytes / (copy * 1024.0)
        tb = time_block(storage)
        parts = ["sweep_block_edges", "sweep_block"] if tb >= 2 else ["sweep_step"]
        # the instantiations of this storage: its type, rounding, layout and T
        # (the run also times the record storage, and a run's last sweep may be
        # shorter)
        st_name, st_round, st_layout = parse_storage(storage)
        want_type = {"f64": "f64", "f32": "f32", "f32plain": "f32", "f16s": "f16",
                     "bf16s": "bf16"}[st_name]

        def of_t(k):
            words = _instance(k).split()
            if not words or words[0] != want_type or (("sr" in words) != (st_round == "stochastic")):
                return False
            if tb >= 2:
                return f"T={tb}" in words
            return ("eq" in words) == (st_layout == "eq")
        kib, picked, other = 0.0, [], {}
        for want in parts:
            names = {}
            for r in rows:
                k = r["Kernel_Name"]
                if want in k and of_t(k) and not any(q in k for q in parts if q != want and want in q):
                    names.setdefault(k, []).append(float(r["Counter_Value"]))
            if not names:  # a plate whose sweep has no launch of this kind
                continue
            name = max(names, key=lambda k: len(names[k]))
            vals = names[name]
            kib += sum(vals) / len(vals)
            picked.append((name[:160], len(vals)))
            other.update({k[:160]: len(v) for k, v in names.items() if k != name})
        out[counter] = {"KiB_per_launch": kib, "copy_KiB": copy, "factor": factor,
                        "bytes_per_launch": kib * 1024.0 * factor,
                        "launches": picked[-1][1], "kernels": picked,
                        "other_sweep_launches": other}
        total += kib * 1024.0 * factor
    bps = sweep_bytes_per_site(storage)
    sites = p.nx * p.ny
    out["bytes_per_launch"] = total
    out["algorithmic_bytes_per_launch"] = sites * bps * time_block(storage)
    out["traffic_over_algorithmic"] = total / out["algorithmic_bytes_per_launch"]
    base = os.path.join(out_dir, f"sweep_{storage}_{workload}_traffic")
    with open(base + ".json", "w") as fh:
        json.dump(out, fh, indent=1)
    f, w = out["FETCH_SIZE"], out["WRITE_SIZE"]
    with open(base + ".md", "w") as fh:
        fh.write(f"# HBM traffic of {block_kernel(storage)} ({storage}, {workload} workload)\n\n"
                 f"Commands (one run per counter, C = FETCH_SIZE then WRITE_SIZE):\n\n    {command}\n\n"
                 f"| counter | KiB / launch | copy of {copy_bytes} B reads | scale | bytes / launch |\n"
                 f"|---|---|---|---|---|\n"
                 f"| FETCH_SIZE | {f['KiB_per_launch']:.1f} | {f['copy_KiB']:.1f} KiB | {f['factor']:.4f} | {f['bytes_per_launch']:.4e} |\n"
                 f"| WRITE_SIZE | {w['KiB_per_launch']:.1f} | {w['copy_KiB']:.1f} KiB | {w['factor']:.4f} | {w['bytes_per_launch']:.4e} |\n\n"
                 f"Total {total:.4e} B per launch against {out['algorithmic_bytes_per_launch']:.4e} algorithmic "
                 f"({sites} sites x {bps * time_block(storage):g} B): ratio {out['traffic_over_algorithmic']:.4f}.\n"
                 f"Kernel source sha256[:16] = {out['kernel_source_sha']}.\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="precision",
                    choices=["precision", "sif", "plain", "batched", "adjoint", "strip"])
    ap.add_argument("--adjoint-storage", default="f32-eq",
                    help="storage (and layout) of the adjoint workload's run")
    ap.add_argument("--directions", type=int, default=16,
                    help="adjoint workload: random directions of the gradient check")
    ap.add_argument("--batch-storage", default="f32-eq",
                    help="storage (and layout) of the batched workload")
    ap.add_argument("--no-tune", action="store_true", help="batched: keep the default launch shape")
    ap.add_argument("--tune", action="store_true",
                    help="single plate: autotune each storage before timing (the library's "
                         "defaults are this search's result for the precision plate)")
    ap.add_argument("--storage", default="f16s-eq-tb8-sr",
                    help='headline storage; "-eq" selects the equilibrium layout, "-eq-tb" that '
                         'layout with two time steps per sweep ("-eq-tb3" .. "-eq-tb8": three to '
                         'eight), a "-sr" suffix stochastic rounding (e.g. f16s-eq-tb6-sr)')
    ap.add_argument("--compare",
                    default="f64,f32,f16s,f16s-sr,bf16s-sr,f64-eq,f32-eq,f16s-eq-sr,bf16s-eq-sr,"
                            "f16s-eq-tb-sr,f16s-eq-tb4-sr,"
                            "f64-eq-tb8,f32-eq-tb6,f32-eq-tb7,f32-eq-tb8,f16s-eq-tb6-sr,"
                            "f16s-eq-tb7-sr,f16s-eq-tb8-sr,bf16s-eq-tb7-sr,bf16s-eq-tb8-sr",
                    help="storages run; the first is the error reference")
    ap.add_argument("--record", default="f16s-sr",
                    help="storage whose one-step five-population sweep is the roofline of record")
    ap.add_argument("--k-steps", type=int, default=None,
                    help="steps of the untimed K_III / field error leg (default: the workload's; "
                         "0 skips it)")
    ap.add_argument("--k-compare", default="f64,f32,f16s-sr,bf16s-sr,f32-eq-tb7,f16s-eq-tb6-sr,"
                                           "f16s-eq-tb7-sr,bf16s-eq-tb7-sr,bf16s-eq-tb8-sr",
                    help="storages of the K_III / field error leg; the first is the reference")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--calibrate-copy", type=int, default=0,
                    help="also run a plain device copy of this many MiB (counter calibration)")
    ap.add_argument("--summarize-trace", nargs=3, metavar=("DIR", "OUT_MD", "COMMAND"),
                    help="write a markdown summary of a rocprofv3 kernel-trace directory and exit")
    ap.add_argument("--out-dir", default=os.path.join(ROOT, "profiles"),
                    help="where --summarize-pmc writes its summary")
    ap.add_argument("--sweep-costs", metavar="OUT_MD",
                    help="time one sweep of 1 .. 8 steps for the --compare storages on the "
                         "workload's plate, write a markdown summary and exit")
    ap.add_argument("--summarize-pmc", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "COPY_MIB", "COMMAND"),
                    help="write profiles/sweep_<storage>_<workload>_traffic.{json,md} and exit")
    args = ap.parse_args()

    if args.summarize_trace:
        summarize_trace(*args.summarize_trace)
        return
    if args.summarize_pmc:
        fd, wd, mib, cmd = args.summarize_pmc
        summarize_pmc(fd, wd, args.storage, args.workload, int(mib) << 20, cmd, args.out_dir)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(the sharding design is described, not built); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    import synth
    from paper_2206_12412_amd import load_library

    load_library()  # fails loudly when the HIP library is not built
    assert torch.cuda.is_available(), "bench.py needs a GPU"

    if args.workload == "batched":
        run_batched(args, torch)
        return
    if args.workload == "adjoint":
        run_adjoint(args, torch)
        return
    if args.workload == "strip":
        run_strip(args, torch)
        return
    p = {"precision": synth.config_precision, "sif": synth.config_sif_fp32,
         "plain": synth.config_plain_fp64}[args.workload]()
    # timed steps: the driver passes --steps; by default 1200 (whole sweeps for
    # T = 2 .. 6 and 8), while the untimed error leg runs the whole workload
    if args.sweep_costs:
        sweep_costs(p, [s for s in args.compare.split(",") if s], torch, args.sweep_costs)
        return
    steps = args.steps if args.steps is not None else (1200 if args.workload == "precision" else p.steps)
    storages = [s for s in args.compare.split(",") if s]
    for extra in (args.record, args.storage):
        if extra not in storages:
            storages.append(extra)
    ref_name = storages[0]

    if args.calibrate_copy > 0:
        n = args.calibrate_copy << 20
        a = torch.ones(n, dtype=torch.uint8, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        print(f"calibration copy of {n} bytes done", file=sys.stderr, flush=True)
        del a, b

    results = {}
    ref = None
    for st in storages:
        print(f"bench: {p.name} storage={st} steps={steps} warmup={args.warmup}", file=sys.stderr,
              flush=True)
        results[st] = run_storage(p, st, steps, args.warmup, torch, ref, tune=args.tune)
        if ref is None:
            ref = results[st]
        print(f"bench: {st}: {results[st]['glups']:.1f} GLUPS", file=sys.stderr, flush=True)
    ref.pop("w_end", None)

    # K_III and field errors over the whole workload (untimed)
    k_steps = args.k_steps if args.k_steps is not None else (p.steps if args.workload == "precision" else 0)
    k_storages = [s for s in args.k_compare.split(",") if s] if k_steps > 0 else []
    if k_storages and args.storage not in k_storages:
        k_storages.append(args.storage)
    k_res = {}
    for st in k_storages:
        print(f"bench: K leg, storage={st}, {k_steps} steps", file=sys.stderr, flush=True)
        r = run_k_leg(p, st, k_steps, torch)
        if not k_res:
            k_res[st] = r
            continue
        r0 = k_res[k_storages[0]]
        k_res[st] = dict(k_errors(r["K"], r0["K"]), field_error=field_error(r["w"], r0["w"]),
                         tip_path_identical=bool(np.array_equal(r["tip"], r0["tip"])))
    k_ref = k_storages[0] if k_storages else None
    if k_ref:
        k_res[k_ref] = {"reference": True}

    # (not in a counter run: its copies would be taken for the calibration copy)
    copy_gbs = copy_bandwidth(torch) if args.calibrate_copy == 0 else None

    per = {}
    for st, r in results.items():
        e = {"glups": round(r["glups"], 2), "ms_per_step": round(r["ms"] / steps, 4),
             "bytes_per_site": r["bytes_per_site"], "launch": r["launch"]}
        if "kernel_ms_per_launch" in r:
            T = r["steps_per_launch"]
            own = r["sites"] * r["bytes_per_site"] * T  # algorithmic bytes of one launch
            gbs = own / (r["kernel_ms_per_launch"] * 1e-3) / 1e9
            e["kernel"] = block_kernel(st)
            e["steps_per_launch"] = T
            e["kernel_ms_per_launch"] = round(r["kernel_ms_per_launch"], 4)
            e["crack_ms_per_launch"] = round(r["crack_ms_per_launch"], 4)
            e["kernel_GBps"] = round(gbs, 1)
            e["hbm_frac"] = round(gbs / HBM_PEAK_GBS, 4)
            e["copy_frac"] = round(gbs / copy_gbs, 4) if copy_gbs else None
            tr = traffic_for(st, args.workload, p.sites)
            if tr:
                e["traffic_over_algorithmic"] = round(tr / own, 4)
        if r.get("autotune"):
            e["autotune"] = r["autotune"]
        if st != ref_name:
            e["field_err_vs_" + ref_name] = r["field_error"]
            e["tip_path_identical"] = r["tip_path_identical"]
        if st in k_res and st != k_ref:
            e["whole_run_errors_vs_" + k_ref] = k_res[st]
        per[st] = e

    head = results[args.storage]
    line = {
        "metric": METRIC,
        "value": round(head["glups"], 2),
        "unit": "GLUPS",
        "n_gpus": 1,
        "steps": steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms"] / steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if parse_storage(args.storage)[0] != "f64" else "f64",
        "data": "synthetic",
        "config": {"workload": p.name, "nx": p.nx, "ny": p.ny, "crack_sites": p.ell,
                   "growth": "prescribed" if p.growth == 1 else "sif", "v_rel": p.v_rel,
                   "tau": p.tau, "storage": parse_storage(args.storage)[0],
                   "rounding": parse_storage(args.storage)[1],
                   "layout": parse_storage(args.storage)[2],
                   "steps_per_sweep": time_block(args.storage),
                   "timed_steps": [head["first_step"], head["first_step"] + steps],
                   "parallelism": "single-gpu"},
        "storages": per,
        # K leg storages that are not timed (e.g. BF16 with eight steps per sweep)
        "k_leg_only": {st: v for st, v in k_res.items() if st not in per and st != k_ref},
        "error_reference": ref_name,
        "copy_GBps": round(copy_gbs, 1) if copy_gbs else None,
    }
    # FP16 storage against FP32 storage: in the headline's layout, and in the
    # five-population layout (the layout the 48 / 28 B/site ratio is stated for)
    same32 = "f32" + args.storage[len(parse_storage(args.storage)[0]):].replace("-sr", "")
    if same32 in results and args.storage != same32:
        line["vs_f32_glups"] = round(head["glups"] / results[same32]["glups"], 3)
        line["vs_f32_reference"] = same32
    if args.record in results and "f32" in results:
        line["fp16_vs_fp32_five_planes"] = {
            "fp16": args.record, "fp32": "f32",
            "glups_ratio": round(results[args.record]["glups"] / results["f32"]["glups"], 3),
            "kernel_ratio_sampled": round(results["f32"]["kernel_ms_per_launch"]
                                          / results[args.record]["kernel_ms_per_launch"], 3)}
    if args.storage in k_res and args.storage != k_ref:
        line["K_III_error"] = dict(
            {k: v for k, v in k_res[args.storage].items() if k.startswith("K_err")},
            storage=args.storage, reference=k_ref + " (five planes, FP64: bit for bit the FP64 oracle)",
            steps=k_steps, workload=p.name)
    # roofline of record: the one-step five-plane sweep of the FP16 storage,
    # whose algorithmic bytes are read + write of the five populations (2 B)
    # and of w (4 B) per site update.  Its launch duration is the timed
    # region's time per step: one sweep launch per step (each crack step runs
    # inside the next sweep, and the call's last one is one launch in 1200
    # steps).  The per-launch event samples of the kernel leg count each
    # kernel's dispatch as well (~3 % more), and are reported beside it.
    if args.record in results and "kernel_ms_per_launch" in results[args.record]:
        r = results[args.record]
        alg = r["sites"] * sweep_bytes_per_site(args.record)
        launch_ms = r["ms"] / steps
        achieved = alg / (launch_ms * 1e-3) / 1e9
        tr = traffic_for(args.record, args.workload, p.sites)
        line["roofline"] = {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": tr,
            "kernel": f"sweep_step ({args.record}: five populations, one step per launch)",
            "bytes_per_site": sweep_bytes_per_site(args.record),
            "algorithmic_bytes_per_launch": alg,
            "kernel_ms": round(launch_ms, 4),
            "kernel_ms_source": "timed region, one sweep launch per step",
            "kernel_ms_sampled": round(r["kernel_ms_per_launch"], 4),
            "copy_frac": round(achieved / copy_gbs, 4) if copy_gbs else None}
    # the headline's own kernel: T steps per launch in the equilibrium layout,
    # counted in the bytes it must move (rest population and w, read and
    # written once per launch, whatever its step count), not in the
    # five-population bytes of the steps it replaces
    # (launch duration: the timed region's time per sweep -- its fast launch,
    # with the boundary launch beside it, the crack steps beside the next
    # sweep; a call of a step count that is not a multiple of T ends with the
    # planned sweeps of up to eight steps, counted as they run)
    if "kernel_ms_per_launch" in head and args.storage != args.record:
        T = head["steps_per_launch"]
        alg = head["sites"] * head["bytes_per_site"] * T
        n_sweeps = len(head["sweeps"]) if head.get("sweeps") else steps / T
        launch_ms = head["ms"] / n_sweeps
        achieved = alg / (launch_ms * 1e-3) / 1e9
        tr = traffic_for(args.storage, args.workload, p.sites)
        line["roofline_headline_kernel"] = {
            "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": tr,
            "kernel": f"{block_kernel(args.storage)} ({args.storage})", "steps_per_launch": T,
            "bytes_per_site_per_launch": head["bytes_per_site"] * T,
            "algorithmic_bytes_per_launch": alg,
            "kernel_ms": round(launch_ms, 4),
            "kernel_ms_per_step": round(head["ms"] / steps, 4),
            "timed_sweeps": (head["sweeps"] if head.get("sweeps") and len(head["sweeps"]) <= 16
                             else len(head["sweeps"]) if head.get("sweeps") else None),
            "kernel_ms_source": "timed region, per sweep",
            "kernel_ms_sampled": round(head["kernel_ms_per_launch"], 4),
            "note": "equilibrium layout (only the rest population and w are state at omega = 1); "
                    "its bytes are not the five-population bytes the roofline of record counts"}
    if not args.no_cpu:
        print("bench: oracle CPU baseline", file=sys.stderr, flush=True)
        line["cpu_baseline"] = cpu_baseline(p, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
