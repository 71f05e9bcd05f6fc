"""Batched plates: a plate stepped inside a batch evolves bit for bit as the
same plate stepped alone (same per-site arithmetic), in both run modes (one
launch set per step, and one persistent cooperative launch for many steps)."""
import sys

import numpy as np
import pytest

import oracle as O
import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2206_12412_amd import Batch, Config, LBMError, Solver  # noqa: E402


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def plate_configs(storage, steps, small=True):
    """Uneven plates: sizes, loads, prescribed speeds and the K criterion.  A
    storage ending in "-eq" selects the equilibrium layout, then "-sr"
    stochastic rounding (one seed per plate)."""
    layout = "eq" if storage.endswith("-eq") else "full"
    storage = storage[:-3] if storage.endswith("-eq") else storage
    rounding = "stochastic" if storage.endswith("-sr") else "nearest"
    storage = storage[:-3] if storage.endswith("-sr") else storage
    rng = np.random.default_rng(5)
    sizes = [(96, 48), (300, 64), (64, 130), (257, 34), (130, 200), (33, 8)] if small else \
        [(512, 512), (1024, 512), (1024, 1024), (2048, 1024)]
    cfgs = []
    for k, (nx, ny) in enumerate(sizes):
        ell = max(nx // 4, 1)
        tau = float(rng.uniform(5e-4, 2e-3))
        c = Config(nx=nx, ny=ny, storage=storage, rounding=rounding, layout=layout, seed=100 + k,
                   has_crack=True, crack_tip=ell - 0.5,
                   tau_hist=np.array([tau]), trace_cap=steps,
                   wdot0=rng.normal(0, 1e-4, (ny, nx)))
        if k % 2 == 0:
            c.growth, c.v_rel = 1, float(rng.uniform(0.1, 0.7))
        else:
            c.growth, c.K_C = 2, 1.05 * synth.k_static_edge(tau, ell)
        cfgs.append(c)
    # a plate with two tips, an off-centre crack row and Dirichlet edges
    n = np.arange(steps)
    wD = np.zeros((max(steps, 1), 4))
    wD[:, 1] = 0.01 * np.sin(np.pi * np.arange(wD.shape[0]) / 60.0)
    cfgs.append(Config(nx=150, ny=40, storage=storage, rounding=rounding, layout=layout, seed=99,
                       has_crack=True,
                       crack_row=12, crack_x0=60.5, crack_tip=80.5, both_tips=True, growth=1,
                       v_rel=0.45, dirichlet=1 | 2, wD_hist=wD, trace_cap=steps,
                       wdot0=rng.normal(0, 1e-4, (40, 150))))
    # one plate without a crack and one periodic plate
    cfgs.append(Config(nx=70, ny=20, storage=storage, rounding=rounding, layout=layout,
                       tau_hist=np.array([1e-3])))
    cfgs.append(Config(nx=80, ny=24, storage=storage, rounding=rounding, layout=layout, periodic=True,
                       wdot0=rng.normal(0, 1e-3, (24, 80))))
    return cfgs


def same_state(a, b, label):
    np.testing.assert_array_equal(a.populations(), b.populations(), err_msg=label)
    wa, wda = a.fields()
    wb, wdb = b.fields()
    np.testing.assert_array_equal(wa, wb, err_msg=label)
    if a.cfg.has_crack:
        ta, tb = a.traces(), b.traces()
        for key in ("K", "tip", "v", "flags"):
            np.testing.assert_array_equal(ta[key], tb[key], err_msg=f"{label} {key}")
        assert a.cut_events().tolist() == b.cut_events().tolist(), label
        if a.cfg.both_tips:
            ta, tb = a.traces(tip="left"), b.traces(tip="left")
            for key in ("K", "tip", "v", "flags"):
                np.testing.assert_array_equal(ta[key], tb[key], err_msg=f"{label} left {key}")


@pytest.mark.parametrize("storage", ["f32", "f64", "f16s", "f16s-sr", "bf16s-sr"])
def test_batched_steps_equal_single_plates(storage):
    steps = 150
    cfgs = plate_configs(storage, steps)
    say(f"batch of {len(cfgs)} plates, {storage}, {steps} steps")
    b = Batch(cfgs)
    b.step(steps)
    for k, c in enumerate(cfgs):
        s = Solver(c)
        s.step(steps)
        same_state(b.plates[k], s, f"plate {k}")
        s.close()
    b.close()


def test_batch_launch_shapes_do_not_change_results():
    steps = 60
    cfgs = plate_configs("f32", steps)
    a = Batch(cfgs)
    a.step(steps)
    b = Batch(cfgs)
    b.set_launch(3, 2, 2)
    b.step(steps)
    for k in range(len(cfgs)):
        same_state(a.plates[k], b.plates[k], f"plate {k}")


@pytest.mark.parametrize("storage", ["f32", "f64", "bf16s-sr", "f32-eq", "f64-eq", "f16s-sr-eq"])
def test_persistent_run_equals_per_step_launches(storage):
    """In the equilibrium layout the persistent kernel takes interior tasks of
    its own height (loads of the next rows in flight); the plates include
    ragged widths and heights below and above that height."""
    cfgs = plate_configs(storage, 200)
    say(f"persistent batch, {storage}: 2 steps first")
    a = Batch(cfgs)
    a.run_persistent(2)
    b = Batch(cfgs)
    b.step(2)
    for k in range(len(cfgs)):
        np.testing.assert_array_equal(a.plates[k].fields()[0], b.plates[k].fields()[0])
    say("  then 198 more steps")
    a.run_persistent(198)
    b.step(198)
    assert a.launch()["persistent_blocks"] > 0
    for k in range(len(cfgs)):
        same_state(a.plates[k], b.plates[k], f"plate {k}")


def test_batched_plate_matches_the_oracle():
    steps = 120
    cfgs = plate_configs("f64", steps)
    b = Batch(cfgs)
    b.step(steps)
    for k in (0, 1, 3):
        c = cfgs[k]
        ref = O.Oracle(O.OracleConfig(nx=c.nx, ny=c.ny, has_crack=True, crack_tip=c.crack_tip,
                                      growth=c.growth, v_rel=c.v_rel, K_C=c.K_C,
                                      tau_hist=c.tau_hist, wdot0=c.wdot0, trace_cap=steps))
        ref.step(steps)
        w_ref = ref.fields()[0]
        np.testing.assert_allclose(b.plates[k].fields()[0], w_ref, rtol=0,
                                   atol=1e-12 * np.abs(w_ref).max())
        # the K-criterion speed goes through tanh, whose last bit may differ
        np.testing.assert_allclose(b.plates[k].traces()["tip"], ref.traces()["tip"], rtol=0,
                                   atol=1e-9)
    # the plate with two tips, its crack on row 12 and Dirichlet edges
    c = cfgs[6]
    assert c.both_tips
    ref = O.Oracle(O.OracleConfig(nx=c.nx, ny=c.ny, has_crack=True, crack_row=c.crack_row,
                                  crack_x0=c.crack_x0, crack_tip=c.crack_tip, both_tips=True,
                                  growth=c.growth, v_rel=c.v_rel, dirichlet=c.dirichlet,
                                  wD_hist=c.wD_hist, wdot0=c.wdot0, trace_cap=steps))
    ref.step(steps)
    w_ref = ref.fields()[0]
    np.testing.assert_allclose(b.plates[6].fields()[0], w_ref, rtol=0,
                               atol=1e-12 * np.abs(w_ref).max())
    for tip in ("right", "left"):
        np.testing.assert_array_equal(b.plates[6].traces(tip=tip)["tip"], ref.traces(tip)["tip"])
    assert b.plates[6].cut_events().tolist() == ref.events()[:, :2].tolist()


def test_plates_of_a_batch_are_not_stepped_alone():
    b = Batch(plate_configs("f32", 10)[:2])
    with pytest.raises(RuntimeError):
        b.plates[0].step(1)
    from paper_2206_12412_amd.lbm import _check
    with pytest.raises(LBMError):  # the C entry point refuses as well
        _check(b._lib.lbm_step(b.plates[0]._h, 1))
    with pytest.raises(LBMError):
        Batch([Config(nx=16, ny=8, storage="f32"), Config(nx=16, ny=8, storage="f64")])


def test_autotune_picks_a_grid_shape_and_leaves_the_plate_alone():
    cfg = plate_configs("f32", 40)[1]
    s = Solver(cfg)
    s.step(20)
    w_before = s.fields()[0]
    t = s.autotune(trial_steps=2)
    say(f"tuned single plate: {t}")
    assert t["rows"] in (1, 2, 4, 8) and t["waves"] in (1, 2, 4, 8)
    assert t["occupancy"] in (0, 2, 3, 4, 5, 6) and t["ms_per_step"] > 0
    got = s.launch()
    assert (got["rows"], got["waves"], got["occupancy"]) == (t["rows"], t["waves"], t["occupancy"])
    np.testing.assert_array_equal(s.fields()[0], w_before)
    s.step(20)
    ref = Solver(cfg)
    ref.step(40)
    same_state(s, ref, "tuned plate")


def test_batch_autotune_keeps_results():
    cfgs = plate_configs("f32", 30)
    b = Batch(cfgs)
    t = b.autotune(trial_steps=1)
    say(f"tuned batch: {t}")
    b.step(30)
    ref = Batch(cfgs)
    ref.step(30)
    for k in range(len(cfgs)):
        same_state(b.plates[k], ref.plates[k], f"plate {k}")
    with pytest.raises(RuntimeError):
        b.plates[0].autotune()


@pytest.mark.parametrize("storage", ["f64", "f16s-sr"])
def test_checkpoint_restart_reproduces_the_run(storage):
    """A run restarted from a checkpoint (in the same or in a fresh handle)
    repeats the original steps bit for bit, traces and cut events included."""
    cfg = plate_configs(storage, 300)[0]   # prescribed growth
    cfg.sensors = np.array([[10, 5], [50, 30], [80, 23]])
    a = Solver(cfg)
    a.step(120)
    ck = a.checkpoint()
    a.step(180)
    b = Solver(cfg)
    b.restore(ck)
    assert b.steps_done == 120
    b.step(180)
    same_state(a, b, "fresh handle")
    np.testing.assert_array_equal(a.sensor_traces(), b.sensor_traces())
    a.restore(ck)
    a.step(180)
    same_state(a, b, "same handle")
    other = Solver(plate_configs(storage, 300)[1])
    from paper_2206_12412_amd import LBMError
    with pytest.raises(LBMError):
        other.restore(ck)
