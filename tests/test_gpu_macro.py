"""The macroscopic boundary scheme of Sec. 3.1 on the GPU (bc_scheme "macro")
against the oracle's: the sweep as for the per-link scheme, then every
boundary point takes w from the quadratic through its boundary condition and
the next two interior points, and its populations from eq. (f-macro-bc).

Bars: FP64 fields within 1e-12 of the oracle (the oracle solves S w_B = R by
iteration and collides through the general BGK expression, the GPU
substitutes and writes f_eq(w_B, wdot_B) directly, so the last bits
differ); FP32 within 1e-5; FP16 storage within about three times the error
measured on MI355X; tips and cut events bit-exact under a prescribed speed;
K within the same bars."""
import math
import sys

import numpy as np
import pytest

import oracle as O
import synth
from _errlog import record

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2206_12412_amd import Config, LBMError, Solver  # noqa: E402

# FP16: three times the largest error measured (w 1.4e-3 on the plate with
# every edge held, relative to its largest |w|); K keeps the 1e-3 bar
# (measured 2.6e-4)
TOL = {"f64": 1e-12, "f32": 1e-5, "f16s-sr": 4e-3}
KTOL = {"f64": 1e-12, "f32": 1e-5, "f16s-sr": 1e-3}


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def cases(steps):
    rng = np.random.default_rng(5)
    n = np.arange(steps)
    wD = np.zeros((steps, 4))
    wD[:, 1] = 0.02 * np.sin(np.pi * n / 90.0) * (n < 90)
    wD[:, 2] = 2e-3
    return {
        # a growing edge crack with loaded faces, a top-edge pulse (prescribed
        # w) and a bottom-edge traction
        "edge-crack": dict(nx=40, ny=22, has_crack=True, crack_row=10, crack_x0=-0.5,
                           crack_tip=9.5, growth=O.GROW_PRESCRIBED, v_rel=0.45,
                           tau_hist=np.array([1e-3]), dirichlet=O.EDGE_TOP, wD_hist=wD,
                           face_traction=4e-4, wdot0=rng.normal(0, 1e-4, (22, 40)),
                           trace_cap=steps),
        # a growing centre crack with two tips, a held left edge
        "two-tips": dict(nx=36, ny=20, has_crack=True, crack_row=12, crack_x0=13.5,
                         crack_tip=20.5, both_tips=True, growth=O.GROW_PRESCRIBED, v_rel=0.4,
                         tau_hist=np.array([1e-3]), dirichlet=O.EDGE_LEFT | O.EDGE_TOP,
                         wD_hist=wD, wdot0=rng.normal(0, 1e-4, (20, 36)), trace_cap=steps),
        # a larger plate over several strips, the crack reaching the far edge
        "wide": dict(nx=700, ny=60, has_crack=True, crack_tip=520.5, growth=O.GROW_PRESCRIBED,
                     v_rel=0.6, tau_hist=np.array([1.5e-3]), wdot0=rng.normal(0, 1e-4, (60, 700)),
                     trace_cap=steps),
        # no crack, every edge held
        "no-crack": dict(nx=130, ny=17, dirichlet=15, wD_hist=wD, wdot0=rng.normal(0, 1e-3, (17, 130))),
        # the K criterion
        "sif": dict(nx=300, ny=40, has_crack=True, crack_tip=80.5, growth=O.GROW_SIF, K_C=0.006,
                    tau_hist=np.array([1.5e-3]), trace_cap=steps),
    }


def gpu_solver(storage, layout, kw):
    if storage.endswith("-sr"):
        return Solver(Config(storage=storage[:-3], rounding="stochastic", seed=4, layout=layout,
                             bc_scheme="macro", **kw), device="cuda:0")
    return Solver(Config(storage=storage, layout=layout, bc_scheme="macro", **kw), device="cuda:0")


@pytest.mark.parametrize("case", ["edge-crack", "two-tips", "wide", "no-crack", "sif"])
@pytest.mark.parametrize("storage,layout", [("f64", "full"), ("f64", "eq"), ("f32", "full"),
                                            ("f32", "eq"), ("f16s-sr", "eq")])
def test_macro_scheme_against_the_oracle(case, storage, layout):
    steps = 240
    kw = cases(steps)[case]
    say(f"macroscopic scheme {case} {storage} {layout}")
    ref = O.Oracle(O.OracleConfig(bc_scheme=O.BC_MACRO, **kw))
    gpu = gpu_solver(storage, layout, kw)
    worst = 0.0
    for n in (1, 37, steps):
        ref.step(n - gpu.steps_done)
        gpu.step(n - gpu.steps_done)
        w_r, wd_r = ref.fields()
        w_g, wd_g = gpu.fields()
        e = np.abs(w_g - w_r).max() / np.abs(w_r).max()
        worst = max(worst, e)
        if storage == "f64":
            ed = np.abs(wd_g - wd_r).max() / np.abs(wd_r).max()
            assert ed <= 1e-11, (n, ed)
    record("w", worst, storage=storage, layout=layout)
    say(f"  w error {worst:.2e}")
    assert worst <= TOL[storage], worst
    if kw.get("has_crack"):
        tr, tg = ref.traces(), gpu.traces()
        ok = ~np.isnan(tr["K"])
        assert np.array_equal(ok, ~np.isnan(tg["K"]))
        kerr = np.abs(tg["K"][ok] - tr["K"][ok]).max() / np.abs(tr["K"][ok]).max()
        record("K", kerr, storage=storage, layout=layout)
        if case == "sif":
            # the K criterion: K before the first cut; the same columns severed
            ev_r, ev_g = ref.events(), gpu.cut_events()
            first = int(ev_r[0, 0])
            pre = ok & (np.arange(len(ok)) < first)
            kerr = np.abs(tg["K"][pre] - tr["K"][pre]).max() / np.abs(tr["K"][pre]).max()
            assert kerr <= KTOL[storage], kerr
            assert len(ev_r) > 5 and ev_g[:, 1].tolist() == ev_r[:, 1].tolist()
            if storage == "f64":
                assert ev_g[:, 0].tolist() == ev_r[:, 0].tolist()
        else:
            assert kerr <= KTOL[storage], kerr
            np.testing.assert_array_equal(tg["tip"], tr["tip"])
            assert gpu.cut_events()[:, :2].tolist() == ref.events()[:, :2].tolist()
            if kw.get("both_tips"):
                np.testing.assert_array_equal(gpu.traces(tip="left")["tip"], ref.traces("left")["tip"])
    gpu.close()


def test_macro_scheme_differs_from_bounce_back():
    """The two boundary schemes give different fields (the option is live)."""
    kw = cases(120)["edge-crack"]
    a = Solver(Config(storage="f64", bc_scheme="macro", **kw), device="cuda:0")
    b = Solver(Config(storage="f64", **kw), device="cuda:0")
    a.step(120)
    b.step(120)
    wa, wb = a.fields()[0], b.fields()[0]
    assert np.abs(wa - wb).max() > 1e-3 * np.abs(wb).max()


@pytest.mark.parametrize("v", [0.2, 0.4, 0.6, 0.8])
@pytest.mark.parametrize("storage,layout", [("f64", "full"), ("f16s-sr", "eq")])
def test_macro_scheme_steady_strip(v, storage, layout):
    """The strip of Sec. 5.1 with the macroscopic scheme: tips bit-exact, the
    sampled K as the oracle's, and the median within 3.5 % of eq.
    (sif-mandal) (the paper: +0.8 % .. 0.0 %; bounce-back: -10.4 % at 0.2)."""
    m = synth.mandal_strip(v)
    ref = O.Oracle(O.OracleConfig(bc_scheme=O.BC_MACRO, **m["config"]))
    gpu = gpu_solver(storage, layout, m["config"])
    ref.step(m["steps"])
    gpu.step(m["steps"])
    tr, tg = ref.traces(), gpu.traces()
    np.testing.assert_array_equal(tg["tip"], tr["tip"])
    K_r, K_g = tr["K"][m["sample_steps"]], tg["K"][m["sample_steps"]]
    kerr = np.abs(K_g - K_r).max() / np.abs(K_r).max()
    record("K", kerr, storage=storage, layout=layout)
    rel = np.median(K_g) / m["K_theo"] - 1.0
    say(f"strip v={v} {storage}: median K / K_theo - 1 = {rel:+.4f}; K error {kerr:.2e}")
    assert kerr <= KTOL[storage]
    assert abs(rel) <= 0.035


def test_macro_scheme_refusals():
    kw = cases(10)["edge-crack"]
    s = Solver(Config(storage="f32", layout="eq", bc_scheme="macro", **kw), device="cuda:0")
    with pytest.raises(LBMError):
        s.set_time_block(4)
    s.close()
    with pytest.raises(LBMError):
        # the crack line two rows from the bottom edge
        Solver(Config(storage="f32", bc_scheme="macro", nx=40, ny=6, has_crack=True,
                      crack_tip=5.5), device="cuda:0")
