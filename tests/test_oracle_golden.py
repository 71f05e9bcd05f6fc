"""The oracle reproduces the stored run of the 256 x 128 plain FP64 workload
(written by tests/golden/make_golden.py from the oracle itself): a regression
guard on top of the pins in test_oracle_pins.py."""
import json
import os

import numpy as np

import oracle as O
import synth

HERE = os.path.dirname(os.path.abspath(__file__))


def test_plain_fp64_run_matches_stored_values():
    with open(os.path.join(HERE, "golden", "plain_fp64_256x128.json")) as fh:
        g = json.load(fh)
    p = synth.config_plain_fp64()
    s = O.Oracle(O.OracleConfig(nx=p.nx, ny=p.ny, has_crack=True, crack_x0=p.crack_x0,
                                crack_tip=p.crack_tip, growth=p.growth, v_rel=p.v_rel,
                                tau_hist=p.traction_history(), trace_cap=p.steps))
    sites = np.array(g["sites"])
    done = 0
    for n in sorted(int(k) for k in g["snapshots"]):
        s.step(n - done)
        done = n
        w, wd = s.fields()
        snap = g["snapshots"][str(n)]
        np.testing.assert_array_equal(w[sites[:, 1], sites[:, 0]], snap["w"])
        np.testing.assert_array_equal(wd[sites[:, 1], sites[:, 0]], snap["wdot"])
    tr = s.traces()
    np.testing.assert_array_equal(tr["tip"], g["tip"])
    np.testing.assert_array_equal(tr["K"], g["K"])
    assert s.events()[:, :2].tolist() == g["events"]
