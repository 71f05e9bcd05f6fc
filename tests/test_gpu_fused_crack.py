"""The crack step of Alg. 1 runs after each step's sweep.  On the one-step
path the sweep of step n + 1 runs the crack step of step n in the same launch
(one more wave beside the boundary rows; the crack-row waves forecast the
links it severs from the same state and field), and lbm_step ends with that
call's last crack step in a launch of its own.  A plate stepped N steps in one
call therefore takes the fused path N - 1 times, the same plate stepped one
step per call never: the two must agree bit for bit, fields, traces, cut
events and sensor traces included.  Batched plates fold their crack steps the
same way when every plate's crack runs along +x (or it has none)."""
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2206_12412_amd import Batch, Config, Solver  # noqa: E402


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def make(storage, **kw):
    layout = "full"
    if storage.endswith("-eq"):
        storage, layout = storage[:-3], "eq"
    rounding = "nearest"
    if storage.endswith("-sr"):
        storage, rounding = storage[:-3], "stochastic"
    return Config(storage=storage, layout=layout, rounding=rounding, seed=7, **kw)


def cases(steps):
    rng = np.random.default_rng(3)
    tau = 1.5e-3
    out = {
        # prescribed speed, ragged width (the last strip is partly empty)
        "prescribed": dict(nx=300, ny=64, has_crack=True, crack_x0=-0.5, crack_tip=40.5,
                           growth=1, v_rel=0.45, tau_hist=np.array([tau]), trace_cap=steps),
        # a crack of length zero: the first cut comes from a fused crack step
        "from-nothing": dict(nx=200, ny=40, has_crack=True, crack_x0=-0.5, crack_tip=-0.5,
                             growth=1, v_rel=0.6, tau_hist=np.array([tau]), trace_cap=steps),
        # the K criterion (eq. sifCriterion, eq. v-tanh), K from a band of columns
        "sif": dict(nx=260, ny=96, has_crack=True, crack_x0=-0.5, crack_tip=49.5, growth=2,
                    K_C=0.95 * synth.k_static_edge(tau, 50.0), k_band=3,
                    tau_hist=np.array([tau]), trace_cap=steps),
        # two tips, an off-centre crack row, Dirichlet edges and sensors
        "two-tips": dict(nx=150, ny=40, has_crack=True, crack_row=12, crack_x0=60.5,
                         crack_tip=80.5, both_tips=True, growth=1, v_rel=0.45, dirichlet=1 | 2,
                         wD_hist=np.column_stack([np.zeros(steps),
                                                  0.01 * np.sin(np.arange(steps) / 9.0),
                                                  np.zeros(steps), np.zeros(steps)]),
                         sensors=np.array([[10, 5], [70, 12], [140, 30]]), trace_cap=steps,
                         wdot0=rng.normal(0, 1e-4, (40, 150))),
        # no crack, sensors only (the crack wave records them)
        "sensors-only": dict(nx=90, ny=33, tau_hist=np.array([tau]),
                             sensors=np.array([[0, 0], [45, 16], [89, 32]]), trace_cap=steps,
                             wdot0=rng.normal(0, 1e-4, (33, 90))),
    }
    return out


def same(a, b, label, cfg):
    np.testing.assert_array_equal(a.populations(), b.populations(), err_msg=label)
    wa, wda = a.fields()
    wb, wdb = b.fields()
    np.testing.assert_array_equal(wa, wb, err_msg=label)
    np.testing.assert_array_equal(wda, wdb, err_msg=label)
    if cfg.sensors is not None:
        np.testing.assert_array_equal(a.sensor_traces(), b.sensor_traces(), err_msg=label)
    if cfg.has_crack:
        for tip in (("right", "left") if cfg.both_tips else ("right",)):
            ta, tb = a.traces(tip=tip), b.traces(tip=tip)
            for key in ("K", "tip", "v", "flags"):
                np.testing.assert_array_equal(ta[key], tb[key], err_msg=f"{label} {tip} {key}")
        assert a.cut_events().tolist() == b.cut_events().tolist(), label
        # repr: an undefined K is NaN on both sides
        ca, cb = a.crack_state(), b.crack_state()
        assert {k: repr(v) for k, v in ca.items()} == {k: repr(v) for k, v in cb.items()}, label


@pytest.mark.parametrize("case", ["prescribed", "from-nothing", "sif", "two-tips", "sensors-only"])
@pytest.mark.parametrize("storage", ["f64", "f32", "f32-eq", "f16s-sr", "bf16s-sr-eq"])
def test_fused_crack_steps_equal_separate_crack_launches(case, storage):
    steps = 160
    kw = cases(steps)[case]
    say(f"fused crack step: {case}, {storage}, {steps} steps")
    a = Solver(make(storage, **kw))
    b = Solver(make(storage, **kw))
    a.step(steps)            # 159 crack steps inside the next sweep, the last alone
    for _ in range(steps):   # every crack step in a launch of its own
        b.step(1)
    same(a, b, f"{case} {storage}", a.cfg)
    if kw.get("has_crack") and kw.get("growth") == 1:
        assert len(a.cut_events()) > 0


@pytest.mark.parametrize("waves", [1, 2, 8])
def test_fused_crack_step_with_other_launch_shapes(waves):
    """The crack wave is the last task of the boundary part: alone in its
    workgroup (one wave per group) or beside boundary rows (more)."""
    steps = 120
    kw = cases(steps)["two-tips"]
    a = Solver(make("f32", **kw))
    a.set_launch(2, waves, 0)
    a.step(steps)
    b = Solver(make("f32", **kw))
    for _ in range(steps):
        b.step(1)
    same(a, b, f"waves={waves}", a.cfg)


def test_calls_of_mixed_lengths_and_a_checkpoint_in_between():
    """Calls of several lengths in a row (each ends with its own crack step)
    and a checkpoint taken between two calls restore the same run."""
    steps = 150
    kw = cases(steps)["sif"]
    a = Solver(make("f16s-sr", **kw))
    b = Solver(make("f16s-sr", **kw))
    for n in (1, 7, 2, 40):
        a.step(n)
    ck = a.checkpoint()
    a.step(100)
    b.step(50)
    b.restore(ck)
    b.step(100)
    same(a, b, "mixed", a.cfg)


@pytest.mark.parametrize("storage", ["f64", "f32", "f32-eq", "f16s-sr", "bf16s-sr-eq"])
def test_batched_fused_crack_steps_equal_separate_crack_launches(storage):
    """A batch of the plates above (and one plate with no crack step at all)
    stepped N steps in one call folds N - 1 crack steps of every plate into
    the next batched sweep; stepped one step per call it folds none."""
    steps = 120
    kw = cases(steps)
    cfgs = [make(storage, **kw[c]) for c in ("prescribed", "from-nothing", "sif", "two-tips",
                                              "sensors-only")]
    cfgs.append(make(storage, nx=70, ny=20, tau_hist=np.array([1e-3])))
    say(f"batched fused crack step: {storage}, {len(cfgs)} plates, {steps} steps")
    a = Batch(cfgs)
    b = Batch(cfgs)
    for n in (1, steps - 41, 40):  # the first call steps one step alone
        a.step(n)
    for _ in range(steps):
        b.step(1)
    for k, c in enumerate(cfgs):
        same(a.plates[k], b.plates[k], f"{storage} plate {k}", c)
        if c.has_crack and c.growth == 1:
            assert len(a.plates[k].cut_events()) > 0
