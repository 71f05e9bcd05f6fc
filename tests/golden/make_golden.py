"""Writes the stored expected values under tests/golden/ by running the oracle.

Calls only ``oracle`` (and the seeded workloads of ``synth``); nothing here
comes from the HIP library.  Run from the repository root:

    python tests/golden/make_golden.py [plain] [sif] [sif-perturbed]
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle as O  # noqa: E402
import synth  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))


def oracle_for(p: synth.Plate, trace_cap: int, wdot_scale: float = 1.0) -> O.Oracle:
    return O.Oracle(O.OracleConfig(
        nx=p.nx, ny=p.ny, kappa=p.kappa, mu=p.mu, rho=p.rho, has_crack=True,
        crack_x0=p.crack_x0, crack_tip=p.crack_tip, growth=p.growth, v_rel=p.v_rel, K_C=p.K_C,
        r0=p.r0, v_max=p.v_max, tau_hist=p.traction_history(), wdot0=p.wdot0() * wdot_scale,
        trace_cap=trace_cap))


def run_perturbed(p: synth.Plate, eps: float, fname: str):
    """The same run with the initial velocity scaled by 1 + eps: how far the
    oracle's own K-criterion path moves under a perturbation at the level of
    rounding (the cut events, the tip and K traces)."""
    s = oracle_for(p, p.steps, 1.0 + eps)
    t0 = time.time()
    s.step(p.steps)
    tr = s.traces()
    out = {"workload": p.name, "wdot0_scale": 1.0 + eps, "eps": eps, "steps": p.steps,
           "K": [float(x) for x in tr["K"]], "tip": [float(x) for x in tr["tip"]],
           "events": s.events()[:, :2].tolist()}
    print(f"{p.name} perturbed by {eps:g}: {time.time() - t0:.1f} s", flush=True)
    with open(os.path.join(HERE, fname), "w") as fh:
        json.dump(out, fh, separators=(",", ":"))


def sample_sites(nx, ny, count, seed):
    rng = np.random.default_rng(seed)
    return np.stack([rng.integers(0, nx, count), rng.integers(0, ny, count)], axis=1)


def run(p: synth.Plate, snaps, fname, nsamp=256):
    s = oracle_for(p, p.steps)
    sites = sample_sites(p.nx, p.ny, nsamp, 1234)
    out = {"workload": p.name, "nx": p.nx, "ny": p.ny, "steps": p.steps,
           "sites": sites.tolist(), "snapshots": {}}
    t0 = time.time()
    done = 0
    for n in snaps:
        s.step(n - done)
        done = n
        w, wd = s.fields()
        out["snapshots"][str(n)] = {
            "w": [float(w[j, i]) for i, j in sites],
            "wdot": [float(wd[j, i]) for i, j in sites],
            "w_absmax": float(np.abs(w).max()), "w_l2": float(np.linalg.norm(w)),
            "wdot_absmax": float(np.abs(wd).max()), "wdot_sum": float(wd.sum()),
        }
        print(f"{p.name}: step {n} ({time.time() - t0:.1f} s)", flush=True)
    tr = s.traces()
    out["K"] = [float(x) for x in tr["K"]]
    out["tip"] = [float(x) for x in tr["tip"]]
    out["flags"] = [int(x) for x in tr["flags"]]
    out["events"] = s.events()[:, :2].tolist()
    with open(os.path.join(HERE, fname), "w") as fh:
        json.dump(out, fh, separators=(",", ":"))


if __name__ == "__main__":
    which = sys.argv[1:] or ["plain"]
    if "plain" in which:
        run(synth.config_plain_fp64(), [500, 1000, 1500, 2000], "plain_fp64_256x128.json")
    if "sif" in which:
        run(synth.config_sif_fp32(), [2000, 3200, 5000, 10000, 20000], "sif_4096x2048.json")
    if "sif-perturbed" in which:
        run_perturbed(synth.config_sif_fp32(), 1e-14, "sif_4096x2048_perturbed.json")
