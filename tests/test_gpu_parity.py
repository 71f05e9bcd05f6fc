"""Parity of the HIP path (through the C-ABI) with the FP64 oracle.

Bars: FP64 fields within 1e-12 relative (normwise, max norm), FP32 fields
within 1e-5; crack-tip positions, cut events and the cut mask bit-exact under
a prescribed speed; K_III within 1e-12 (FP64).  Under the K criterion the tip
path is the list of (step, column) cut events, compared together with the
guard margins that make that comparison meaningful.
"""
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

from paper_2206_12412_amd import Config, Solver  # noqa: E402

# FP64 and FP32: the bars of the method's statement.  The reduced
# precisions (unshifted FP32, FP16 and BF16 storage) are held to about three
# times the largest error measured on MI355X over this file's cases (the
# 2000-step plain workload: w 2.3e-5 / 1.2e-4 / 1.2e-3, K 1.1e-5 / 8e-5 /
# 5.9e-4), so that a regression of a few times shows; K of FP16 storage keeps
# the 1e-3 bar of the precision extension (largest measured 5.3e-4).
TOL = {"f64": 1e-12, "f32": 1e-5, "f32plain": 7e-5, "f16s": 4e-4, "bf16s": 4e-3}
KTOL = {"f64": 1e-12, "f32": 1e-5, "f32plain": 5e-5, "f16s": 1e-3, "bf16s": 2e-3}
# "-sr": the same storage with stochastic rounding of the 16-bit stores
for _d in (TOL, KTOL):
    _d.update({"f16s-sr": _d["f16s"], "bf16s-sr": _d["bf16s"]})


def gpu_config(storage, **kw):
    if storage.endswith("-sr"):
        return Config(storage=storage[:-3], rounding="stochastic", seed=11, **kw)
    return Config(storage=storage, **kw)


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def pair(storage="f64", **kw):
    say(f"case storage={storage} {kw.get('nx')}x{kw.get('ny')} growth={kw.get('growth', 0)}")
    ref = O.Oracle(O.OracleConfig(**kw))
    gkw = dict(kw)
    gkw.pop("threads", None)
    per = gkw.pop("periodic", False)
    gpu = Solver(gpu_config(storage, periodic=per, **gkw), device="cuda:0")
    return ref, gpu


def relerr(a, b):
    scale = np.abs(b).max()
    return np.abs(a - b).max() / (scale if scale > 0 else 1.0)


def plain_kw(nx, ny, ell, v=0.3, tau=1e-3, steps=0, **extra):
    kw = dict(nx=nx, ny=ny, has_crack=True, crack_x0=-0.5, crack_tip=ell - 0.5,
              growth=O.GROW_PRESCRIBED, v_rel=v, tau_hist=np.array([tau]), trace_cap=steps)
    kw.update(extra)
    return kw


def compare_run(storage, kw, steps, checkpoints=None, exact_crack=True, tol=None):
    tol = TOL[storage] if tol is None else tol
    ref, gpu = pair(storage, **kw)
    checkpoints = checkpoints or [steps]
    done = 0
    worst = 0.0
    for n in checkpoints:
        ref.step(n - done)
        gpu.step(n - done)
        done = n
        w_r, wd_r = ref.fields()
        w_g, wd_g = gpu.fields()
        e = relerr(w_g, w_r)
        worst = max(worst, e)
        record("w", e, storage=storage, step=n)
        assert e <= tol, (storage, n, e)
        if storage == "f64":
            assert relerr(wd_g, wd_r) <= 1e-12, (n, relerr(wd_g, wd_r))
    if kw.get("has_crack"):
        tr_r, tr_g = ref.traces(), gpu.traces()
        if exact_crack:
            np.testing.assert_array_equal(tr_g["tip"], tr_r["tip"])
            np.testing.assert_array_equal(tr_g["flags"], tr_r["flags"])
            assert gpu.cut_events()[:, 0].tolist() == ref.events()[:, 0].tolist()
            assert gpu.cut_events()[:, 1].tolist() == ref.events()[:, 1].tolist()
            mv_r, mh_r = ref.mask()
            mv_g, mh_g = gpu.mask()
            np.testing.assert_array_equal(mv_g, mv_r)
            np.testing.assert_array_equal(mh_g, mh_r)
        Kr, Kg = tr_r["K"], tr_g["K"]
        assert np.array_equal(np.isnan(Kr), np.isnan(Kg))
        ok = ~np.isnan(Kr)
        if ok.any():
            kerr = np.abs(Kg[ok] - Kr[ok]).max() / max(np.abs(Kr[ok]).max(), 1e-300)
            record("K", kerr, storage=storage)
            ktol = KTOL[storage]
            assert kerr <= ktol, (storage, kerr)
    gpu.close()
    return worst


# ---------------------------------------------------------------- plain run --

def test_plain_fp64_full_workload_bit_exact_tip_and_fields():
    """256 x 128, 64-site crack at 0.3 c_s for 2000 steps, FP64."""
    p = synth.config_plain_fp64()
    kw = plain_kw(p.nx, p.ny, p.ell, p.v_rel, p.tau, p.steps)
    worst = compare_run("f64", kw, p.steps, [500, 1000, 1279, 1280, 2000])
    say(f"plain f64 worst rel err {worst:.3e}")


@pytest.mark.parametrize("storage", ["f32", "f16s", "bf16s", "f32plain", "f16s-sr", "bf16s-sr"])
def test_plain_workload_reduced_precision(storage):
    p = synth.config_plain_fp64()
    kw = plain_kw(p.nx, p.ny, p.ell, p.v_rel, p.tau, p.steps)
    worst = compare_run(storage, kw, p.steps, [500, 1000, 2000])
    say(f"plain {storage} worst rel err {worst:.3e}")


def test_fp64_is_bit_identical_to_the_oracle():
    """Same operations in the same order without contraction: the FP64 state
    equals the oracle's bit for bit."""
    kw = plain_kw(100, 40, 20, v=0.45, steps=300)
    ref, gpu = pair("f64", **kw)
    ref.step(300)
    gpu.step(300)
    np.testing.assert_array_equal(gpu.populations(), ref.pops())
    np.testing.assert_array_equal(gpu.fields()[0], ref.fields()[0])
    np.testing.assert_array_equal(gpu.traces()["K"], ref.traces()["K"])


# ------------------------------------------------- sizes, tiles, ragged ends --

@pytest.mark.parametrize("nx,ny,ell", [(77, 34, 9), (130, 10, 40), (1000, 66, 300), (257, 2, 64),
                                       (1, 2, 0), (65, 130, 64), (513, 36, 1), (33, 8, 33)])
@pytest.mark.parametrize("storage", ["f64", "f32", "f16s", "f16s-sr"])
def test_ragged_sizes(nx, ny, ell, storage):
    steps = 150
    kw = plain_kw(nx, ny, max(ell, 0), v=0.6, steps=steps)
    rng = np.random.default_rng(nx * 1000 + ny)
    kw["wdot0"] = rng.normal(0, 1e-4, (ny, nx))
    # noise-only fields, relative to the largest |w| of small plates: about
    # three times the largest error measured (4.8e-3 nearest, 9.5e-4
    # stochastic rounding, over all sizes)
    tol = {"f16s": 1.5e-2, "f16s-sr": 3e-3}.get(storage)
    compare_run(storage, kw, steps, [1, 7, steps], tol=tol)


@pytest.mark.parametrize("rows,waves,occ", [(1, 1, 0), (3, 2, 2), (16, 4, 0), (64, 8, 3),
                                            (1000, 1, 8), (2, 4, 4)])
@pytest.mark.parametrize("storage", ["f64", "f32", "bf16s", "f16s-sr"])
def test_launch_shapes_give_identical_results(rows, waves, occ, storage):
    kw = plain_kw(300, 90, 70, v=0.5, steps=120)
    base = Solver(gpu_config(storage, **kw), device="cuda:0")
    other = Solver(gpu_config(storage, **kw), device="cuda:0")
    other.set_launch(rows, waves, occ)
    assert other.launch()["occupancy"] == occ
    base.step(120)
    other.step(120)
    np.testing.assert_array_equal(base.populations(), other.populations())
    np.testing.assert_array_equal(base.fields()[0], other.fields()[0])


# ----------------------------------------------------------- special modes --

@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_periodic_lattice(storage):
    nx, ny = 200, 60
    I, J = np.meshgrid(np.arange(nx), np.arange(ny))
    w0 = 0.3 * np.cos(2 * np.pi * (3 * I / nx + 2 * J / ny))
    rng = np.random.default_rng(4)
    kw = dict(nx=nx, ny=ny, periodic=True, w0=w0, wdot0=rng.normal(0, 1e-2, (ny, nx)),
              has_crack=True, crack_x0=40.0, crack_tip=120.7)
    compare_run(storage, kw, 400, [1, 50, 400])


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_face_loaded_stationary_crack(storage):
    kw = dict(nx=256, ny=128, has_crack=True, crack_tip=127.5, face_traction=1e-3, trace_cap=300)
    compare_run(storage, kw, 300, [100, 300])


@pytest.mark.parametrize("storage", ["f64", "f32"])
def test_centre_crack_k_band_and_traction_history(storage):
    rng = np.random.default_rng(9)
    kw = dict(nx=180, ny=64, has_crack=True, crack_x0=30.2, crack_tip=80.0, growth=O.GROW_PRESCRIBED,
              v_rel=0.7, k_band=5, r0=3.0, tau_hist=rng.uniform(-2e-3, 2e-3, 97), trace_cap=400,
              mu=2.0, rho=0.5, kappa=2.5)
    compare_run(storage, kw, 400, [37, 400])


def test_no_crack_plate():
    """Uniformly step-loaded plate without a crack.  Its early-time field is a
    1-D step response whose FP32 error plateaus near 3e-5 of max|w| for any
    FP32 rounding (of the stored values or of the arithmetic alike; a float32
    emulation of the same scheme gives the identical number), so FP32 is held
    to 5e-5 here; FP64 keeps its 1e-12 bar."""
    kw = dict(nx=120, ny=50, tau_hist=np.array([1e-3]))
    compare_run("f64", kw, 200)
    compare_run("f32", kw, 200, tol=5e-5)


# ----------------------------------------------------------- K criterion --

def test_sif_criterion_reduced_workload():
    """The K-criterion workload scaled to 512 x 256 (crack 128, K_C = 1.5
    K_static): FP64 cut events, K and tips identical to the oracle's."""
    p = synth.config_sif_fp32().scaled(512, 256, 128, 6000)
    p.K_C = 1.5 * synth.k_static_edge(p.tau, p.ell)
    kw = dict(nx=p.nx, ny=p.ny, has_crack=True, crack_tip=p.crack_tip, growth=O.GROW_SIF,
              K_C=p.K_C, r0=p.r0, v_max=p.v_max, tau_hist=p.traction_history(),
              wdot0=p.wdot0(), trace_cap=p.steps)
    ref, g64 = pair("f64", **kw)
    ref.step(p.steps)
    g64.step(p.steps)
    ev_r = ref.events()[:, :2].tolist()
    assert len(ev_r) > 10
    assert g64.cut_events().tolist() == ev_r
    tr_r, tr_g = ref.traces(), g64.traces()
    ok = ~np.isnan(tr_r["K"])
    assert np.abs(tr_g["K"][ok] - tr_r["K"][ok]).max() <= 1e-12 * np.abs(tr_r["K"][ok]).max()
    np.testing.assert_allclose(tr_g["tip"], tr_r["tip"], rtol=0, atol=1e-9)


def sif_path_margins(tr, a0, K_C, r0):
    """Per step, how far the oracle's run stays from each threshold that
    decides the crack path: the criterion |K/K_C - 1| (eq. sifCriterion), the
    distance of the tip to the next lattice column (a cut happens when the
    tip reaches it, Alg. 1) and the distance of a - r_min to an integer (it
    selects the K column floor(a - r_min), with r_min = r0 / (1 - v) of the
    previous step, eq. r(v))."""
    K, a, v = tr["K"], tr["tip"], tr["v"]
    km = np.abs(K / K_C - 1)
    am = np.abs(a - np.round(a))
    a_prev = np.concatenate([[a0], a[:-1]])
    v_prev = np.concatenate([[0.0], v[:-1]])
    x = a_prev - r0 / (1.0 - v_prev)
    cm = np.abs(x - np.round(x))
    return km, am, cm


@pytest.mark.parametrize("storage", ["f32", "f32-eq"])
def test_sif_criterion_exact_events_where_the_margins_hold(storage):
    """Bit-exact cut events under the K criterion in FP32.  An edge crack
    (400 x 160, 100 sites) whose faces are loaded suddenly (tau* = 2e-3), with
    K_C = 0.005: K passes K_C within one step and stays 5 % or more above it
    while the tip grows, so in the oracle's own run every criterion decision,
    every column the tip reaches and every K column lies at least 1e-3 from
    its threshold, 100x the FP32 K error.  The FP32 run must sever the same
    links at the same steps: all of the oracle's events (166)."""
    steps = 400
    rng = np.random.default_rng(0)
    kw = dict(nx=400, ny=160, has_crack=True, crack_tip=99.5, growth=O.GROW_SIF, K_C=0.005,
              r0=2.0, v_max=0.85, face_traction=2e-3, tau_hist=np.array([1e-3]),
              wdot0=rng.normal(0, 1e-6, (160, 400)), trace_cap=steps)
    st, layout = storage.replace("-eq", ""), ("eq" if "-eq" in storage else "full")
    ref = O.Oracle(O.OracleConfig(**kw))
    ref.step(steps)
    tr_r = ref.traces()
    ev_r = ref.events()[:, :2].tolist()
    km, am, cm = sif_path_margins(tr_r, kw["crack_tip"], kw["K_C"], kw["r0"])
    ok = ~np.isnan(tr_r["K"])
    margin = min(km[ok].min(), am.min(), cm[ok].min())
    gpu = Solver(Config(storage=st, layout=layout, **kw), device="cuda:0")
    gpu.step(steps)
    tr_g = gpu.traces()
    ev_g = gpu.cut_events().tolist()
    kerr = np.abs(tr_g["K"][ok] - tr_r["K"][ok]).max() / np.abs(tr_r["K"][ok]).max()
    record("K", kerr, storage=storage)
    say(f"sif exact events {storage}: {len(ev_r)} cuts; margins K {km[ok].min():.2e}, tip "
        f"{am.min():.2e}, K column {cm[ok].min():.2e}; K err {kerr:.2e}; tip deviation "
        f"{np.abs(tr_g['tip'] - tr_r['tip']).max():.2e}")
    assert margin >= 1e-3
    assert kerr <= 1e-5
    assert len(ev_r) >= 150
    assert ev_g == ev_r
    np.testing.assert_array_equal((tr_g["flags"] & 1) != 0, (tr_r["flags"] & 1) != 0)
    assert np.abs(tr_g["tip"] - tr_r["tip"]).max() <= 1e-4


def test_stochastic_rounding_is_deterministic_per_seed():
    """Same seed: identical states (the draws depend on site, step and seed
    only); another seed: a different state within the same bound."""
    kw = plain_kw(300, 90, 70, v=0.5, steps=200)
    a = Solver(Config(storage="f16s", rounding="stochastic", seed=3, **kw), device="cuda:0")
    b = Solver(Config(storage="f16s", rounding="stochastic", seed=3, **kw), device="cuda:0")
    c = Solver(Config(storage="f16s", rounding="stochastic", seed=4, **kw), device="cuda:0")
    b.set_launch(5, 1, 2)
    for s in (a, b, c):
        s.step(200)
    np.testing.assert_array_equal(a.populations(), b.populations())
    assert not np.array_equal(a.fields()[0], c.fields()[0])
    ref = O.Oracle(O.OracleConfig(**kw))
    ref.step(200)
    w_r = ref.fields()[0]
    for s in (a, c):
        record("w", relerr(s.fields()[0], w_r), storage="f16s-sr")
        assert relerr(s.fields()[0], w_r) <= 7e-4  # 3x the largest measured (2.3e-4)



# ------------------------------ Dirichlet edges, crack row, two tips (Sec. 5.2) --

def dirichlet_two_tip_kw(nx, ny, steps, row, x0, a0, v=0.4):
    n = np.arange(steps)
    wD = np.zeros((steps, 4))
    wD[:, 1] = 0.02 * np.sin(np.pi * n / 120.0) * (n < 120)   # top: half sine pulse
    wD[:, 2] = 3e-3                                         # left: constant
    rng = np.random.default_rng(nx + ny)
    return dict(nx=nx, ny=ny, has_crack=True, crack_row=row, crack_x0=x0, crack_tip=a0,
                both_tips=True, growth=O.GROW_PRESCRIBED, v_rel=v, tau_hist=np.array([1e-3]),
                dirichlet=1 | 2 | 4, wD_hist=wD, wdot0=rng.normal(0, 1e-4, (ny, nx)),
                trace_cap=steps)


@pytest.mark.parametrize("nx,ny,row,x0,a0", [(36, 20, 12, 13.5, 20.5), (300, 90, 60, 120.5, 170.5),
                                             (513, 34, 5, 200.5, 260.5)])
@pytest.mark.parametrize("storage", ["f64", "f32", "f16s-sr"])
def test_dirichlet_edges_off_centre_crack_two_tips(nx, ny, row, x0, a0, storage):
    steps = 240
    kw = dirichlet_two_tip_kw(nx, ny, steps, row, x0, a0)
    tol = 2e-3 if storage.startswith("f16s") else None  # 3x the largest measured (7.1e-4)
    compare_run(storage, kw, steps, [1, 60, steps], tol=tol)
    ref, gpu = pair(storage, **kw)
    ref.step(steps)
    gpu.step(steps)
    tl_r, tl_g = ref.traces("left"), gpu.traces(tip="left")
    np.testing.assert_array_equal(tl_g["tip"], tl_r["tip"])
    np.testing.assert_array_equal(tl_g["flags"], tl_r["flags"])
    ok = ~np.isnan(tl_r["K"])
    if ok.any():
        kerr = np.abs(tl_g["K"][ok] - tl_r["K"][ok]).max() / np.abs(tl_r["K"][ok]).max()
        record("K_left", kerr, storage=storage)
        assert kerr <= KTOL[storage], kerr
    info = gpu.crack_state()
    assert info["tip_left"] == tl_r["tip"][-1] and info["tip"] == ref.traces()["tip"][-1]


def test_two_tip_k_criterion_demo_fp64():
    """The K-criterion example of Sec. 5.2 at its own size (512 x 192, two
    tips, Dirichlet upper and lower edges, half-sine pulse): FP64 fields,
    traces of both tips and the cut events equal the oracle's."""
    import synth
    d = synth.two_tip_demo(4000)
    say("two-tip K-criterion demo, FP64, 4000 steps")
    ref = O.Oracle(O.OracleConfig(**d))
    gpu = Solver(Config(storage="f64", **d))
    ref.step(4000)
    gpu.step(4000)
    w_r, w_g = ref.fields()[0], gpu.fields()[0]
    assert relerr(w_g, w_r) <= 1e-12
    for tip in ("right", "left"):
        tr, tg = ref.traces(tip), gpu.traces(tip=tip)
        np.testing.assert_array_equal(tg["flags"], tr["flags"])
        np.testing.assert_allclose(tg["tip"], tr["tip"], rtol=0, atol=1e-9)
        ok = ~np.isnan(tr["K"])
        assert np.abs(tg["K"][ok] - tr["K"][ok]).max() <= 1e-12 * np.abs(tr["K"][ok]).max()
    ev_r = ref.events()
    assert gpu.cut_events().tolist() == [[int(e[0]), int(e[1])] for e in ev_r]
    assert len(ev_r) > 10  # both tips grew


# ------------------------------------ steady growth in a strip (Sec. 5.1) --

@pytest.mark.parametrize("v", [0.2, 0.8])
@pytest.mark.parametrize("storage,layout,rounding", [("f64", "full", "nearest"),
                                                     ("f64", "eq", "nearest"),
                                                     ("f32", "eq", "nearest"),
                                                     ("f16s", "eq", "stochastic")])
def test_steady_strip_against_the_oracle(v, storage, layout, rounding):
    """The Sec. 5.1 strip (Dirichlet +-w0/2 edges with the sin^2 ramp, edge
    crack at a prescribed speed): tips bit-exact, fields and the sampled K
    statistics as the oracle's within the storage's bounds."""
    m = synth.mandal_strip(v)
    say(f"steady strip v={v} {storage} {layout} {rounding}")
    ref = O.Oracle(O.OracleConfig(**m["config"]))
    gpu = Solver(Config(storage=storage, layout=layout, rounding=rounding, seed=3, **m["config"]))
    ref.step(m["steps"])
    gpu.step(m["steps"])
    w_r, w_g = ref.fields()[0], gpu.fields()[0]
    # FP16: 3x the largest error measured over the four speeds (4.2e-4)
    tol = {"f64": 1e-12, "f32": 1e-5, "f16s": 1.3e-3}[storage]
    record("w", relerr(w_g, w_r), storage=storage, layout=layout)
    assert relerr(w_g, w_r) <= tol
    tr, tg = ref.traces(), gpu.traces()
    np.testing.assert_array_equal(tg["tip"], tr["tip"])
    assert gpu.cut_events()[:, 1].tolist() == ref.events()[:, 1].tolist()
    K_r, K_g = tr["K"][m["sample_steps"]], tg["K"][m["sample_steps"]]
    ktol = {"f64": 1e-12, "f32": 1e-5, "f16s": 1e-3}[storage]
    record("K", np.abs(K_g - K_r).max() / np.abs(K_r).max(), storage=storage, layout=layout)
    assert np.abs(K_g - K_r).max() <= ktol * np.abs(K_r).max()
    assert abs(np.median(K_g) / np.median(K_r) - 1.0) <= ktol
    say(f"  median K / K_theo - 1 = {np.median(K_g) / m['K_theo'] - 1:+.4f}")


# -------------------------------- a crack along another direction (Alg. 1) --

def inclined_kw(nx, ny, dx, dy, steps, v=0.45, both=True):
    rng = np.random.default_rng(nx * 7 + ny)
    n = np.arange(steps)
    wD = np.zeros((steps, 4))
    wD[:, 2] = 4e-3 * np.minimum(n / 50.0, 1.0)   # left edge held, ramped
    return dict(nx=nx, ny=ny, has_crack=True, crack_row=ny // 2 - 3, crack_x0=nx / 2 - 2.3,
                crack_tip=nx / 2 + 4.1, both_tips=both, growth=O.GROW_PRESCRIBED, v_rel=v,
                crack_dx=dx, crack_dy=dy, tau_hist=np.array([1e-3]), dirichlet=4, wD_hist=wD,
                wdot0=rng.normal(0, 1e-4, (ny, nx)), trace_cap=steps)


def same_links(gpu, ref):
    """Cut links per step as sets (the kernel tests the candidate links in
    another order than the breadth-first search)."""
    g = sorted(map(tuple, gpu.cut_links().tolist()))
    r = sorted(map(tuple, ref.events().tolist()))
    assert g == r and len(r) > 4


@pytest.mark.parametrize("dx,dy", [(0.92, 0.39), (-0.3, 1.0), (0.6, -0.8), (0.0, 1.0), (1.0, 1.0)])
@pytest.mark.parametrize("nx,ny", [(96, 70), (131, 53)])
def test_inclined_crack_fp64_against_the_oracle(dx, dy, nx, ny):
    steps = 220
    kw = inclined_kw(nx, ny, dx, dy, steps)
    for layout in ("full", "eq"):
        say(f"inclined crack ({dx}, {dy}) {nx}x{ny} f64 {layout}")
        ref = O.Oracle(O.OracleConfig(**kw))
        gpu = Solver(Config(storage="f64", layout=layout, **kw))
        mv_r, mh_r = ref.mask()
        mv_g, mh_g = gpu.mask()
        np.testing.assert_array_equal(mv_g, mv_r)
        np.testing.assert_array_equal(mh_g, mh_r)
        for n in (60, steps):
            ref.step(n - gpu.steps_done)
            gpu.step(n - gpu.steps_done)
            w_r, w_g = ref.fields()[0], gpu.fields()[0]
            assert relerr(w_g, w_r) <= 1e-12, (n, relerr(w_g, w_r))
        for tip in ("right", "left"):
            tr, tg = ref.traces(tip), gpu.traces(tip=tip)
            np.testing.assert_array_equal(tg["tip"], tr["tip"])
            np.testing.assert_array_equal(tg["flags"], tr["flags"])
            ok = ~np.isnan(tr["K"])
            assert np.array_equal(ok, ~np.isnan(tg["K"]))
            if ok.any():
                assert np.abs(tg["K"][ok] - tr["K"][ok]).max() <= 1e-12 * np.abs(tr["K"][ok]).max()
        same_links(gpu, ref)
        mv_r, mh_r = ref.mask()
        mv_g, mh_g = gpu.mask()
        np.testing.assert_array_equal(mv_g, mv_r)
        np.testing.assert_array_equal(mh_g, mh_r)
        gpu.close()


@pytest.mark.parametrize("deg,L0", [(10, 18.0), (30, 23.7), (30, 27.2), (45, 21.1), (60, 19.4),
                                    (80, 25.3), (-35, 22.6), (135, 17.9)])
def test_inclined_crack_K_from_the_near_tip_field_on_the_gpu(deg, L0):
    """The GPU's K for a crack along another direction, checked against the
    closed form rather than the oracle: the asymptotic mode III field
    w = (2K/mu) sqrt(r / 2 pi) sin(phi / 2), written in the crack's own polar
    coordinates around the tip (Sec. 2.2), is the initial displacement; with
    kappa = 40 one step changes w by the discrete Laplacian / kappa^2 (the
    field is harmonic, so by ~1e-4 of K), and the crack step's K must equal
    the K of the field within 3 %: the pair of sites across the first link
    that crosses the crack line at or beyond r_min sits off phi = +-pi, and r
    is measured to the projection of the pair's midpoint."""
    nx, ny, mu, K = 70, 60, 1.5, 0.05
    th = math.radians(deg)
    ux, uy = math.cos(th), math.sin(th)
    x0, row = (10.3, 12) if ux > 0 else (55.2, 12)
    if uy < 0:
        row = 45
    yc = row + 0.5
    tx, ty = x0 + L0 * ux, yc + L0 * uy
    jj, ii = np.mgrid[0:ny, 0:nx]
    px, py = ii - tx, jj - ty
    xl = px * ux + py * uy        # along the crack (ahead of the tip > 0)
    yl = -px * uy + py * ux       # across it
    r = np.hypot(xl, yl)
    phi = np.arctan2(yl, xl)
    w0 = 2 * K / mu * np.sqrt(r / (2 * math.pi)) * np.sin(phi / 2)
    s = Solver(Config(nx=nx, ny=ny, storage="f64", has_crack=True, crack_row=row, crack_x0=x0,
                      crack_tip=x0 + L0, mu=mu, kappa=40.0, r0=2.0, crack_dx=ux, crack_dy=uy,
                      w0=w0, trace_cap=1), device="cuda:0")
    s.step(1)
    Kg = float(s.traces()["K"][0])
    say(f"inclined crack at {deg} deg: GPU K {Kg:.5f} against the field's {K} "
        f"({Kg / K - 1:+.4f})")
    assert Kg == pytest.approx(K, rel=0.03)
    s.close()


@pytest.mark.parametrize("storage", ["f32-eq", "f16s-eq-sr", "f32"])
def test_inclined_crack_reduced_precision(storage):
    steps = 300
    kw = inclined_kw(160, 90, 0.8, 0.45, steps)
    st = storage.replace("-eq", "")
    layout = "eq" if "-eq" in storage else "full"
    ref = O.Oracle(O.OracleConfig(**kw))
    gpu = gpu_config(st, layout=layout, **kw)
    gpu = Solver(gpu)
    ref.step(steps)
    gpu.step(steps)
    tol = TOL[st] if st in TOL else 5e-4  # FP16: 3x the measured 1.4e-4
    record("w", relerr(gpu.fields()[0], ref.fields()[0]), storage=storage)
    assert relerr(gpu.fields()[0], ref.fields()[0]) <= tol
    np.testing.assert_array_equal(gpu.traces()["tip"], ref.traces()["tip"])
    same_links(gpu, ref)


def test_inclined_crack_in_a_batch_equals_the_plate_alone():
    from paper_2206_12412_amd import Batch
    steps = 120
    cfgs = [Config(storage="f32", layout="eq", **inclined_kw(100, 64, -0.5, 0.7, steps)),
            Config(storage="f32", layout="eq", **inclined_kw(90, 80, 1.0, 0.0, steps)),
            Config(storage="f32", layout="eq", **inclined_kw(70, 90, 0.2, -1.0, steps, both=False))]
    b = Batch(cfgs)
    b.step(steps)
    for k, c in enumerate(cfgs):
        s = Solver(c)
        s.step(steps)
        np.testing.assert_array_equal(b.plates[k].fields()[0], s.fields()[0])
        assert b.plates[k].cut_links().tolist() == s.cut_links().tolist()


def test_adjoint_refuses_an_inclined_crack():
    s = Solver(Config(storage="f32", sensors=np.array([[3, 4]]), **inclined_kw(60, 40, 0.6, 0.8, 10)))
    s.step(10)
    with pytest.raises(Exception):
        s.adjoint(torch.zeros((10, 1), dtype=torch.float64, device="cuda"))
