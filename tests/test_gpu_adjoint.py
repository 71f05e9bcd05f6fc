"""Discrete adjoint on the GPU (lbm_adjoint_run) and its autograd bridge.

* FP64: the gradients with respect to the traction history and the initial
  fields equal the oracle's discrete adjoint (1e-12 normwise), stationary
  cracks, ragged sizes, sensors on the crack faces and at the edges.
* A crack growing at a prescribed speed: the map is affine in the inputs
  (the cut sequence does not depend on them), so the FP64 central
  difference is exact up to rounding; the adjoint must match it.
* FP32 (the adjoint of the shifted FP32 run) against FP64 central
  differences within 1e-4; FP16 storage uses the same FP32 adjoint.
* torch.autograd through sensor_run gives the same gradients.
"""
import sys

import numpy as np
import pytest

import oracle as O

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2206_12412_amd import Config, Solver  # noqa: E402
from paper_2206_12412_amd.autograd import sensor_run  # noqa: E402


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def rel(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def case(nx, ny, T, ell, seed, sensors=None, periodic=False, growth=0, v=0.0):
    rng = np.random.default_rng(seed)
    if sensors is None:
        sensors = np.stack([rng.integers(0, nx, 12), rng.integers(0, ny, 12)], axis=1)
        sensors = np.unique(sensors, axis=0)
    kw = dict(nx=nx, ny=ny, tau_hist=1e-3 * (1 + 0.2 * rng.normal(size=T)),
              wdot0=1e-4 * rng.normal(size=(ny, nx)), trace_cap=T)
    if ell is not None:
        kw.update(has_crack=True, crack_tip=ell - 0.5, growth=growth, v_rel=v)
    if periodic:
        kw.update(tau_hist=np.zeros(T))
    target = 1e-3 * rng.normal(size=(T, len(sensors)))
    return kw, np.asarray(sensors), target


def gpu_grads(storage, kw, sensors, target, periodic=False):
    T = kw["trace_cap"]
    s = Solver(Config(storage=storage, periodic=periodic, sensors=sensors, **kw))
    s.step(T)
    tr = s.sensor_traces()
    g = torch.from_numpy(2.0 * (tr - target)).cuda()
    dtau, dwd0, dw0 = s.adjoint(g)
    s.close()
    return tr, dtau, dwd0.cpu().numpy(), dw0.cpu().numpy()


@pytest.mark.parametrize("nx,ny,T,ell", [(40, 24, 80, 10), (77, 34, 120, 20), (300, 66, 90, 120),
                                         (33, 8, 50, 4), (130, 10, 40, None)])
def test_fp64_adjoint_equals_the_oracle(nx, ny, T, ell):
    kw, sens, target = case(nx, ny, T, ell, seed=nx)
    say(f"adjoint FP64 {nx}x{ny}, {T} steps, crack {ell}, {len(sens)} sensors")
    tr, dtau, dwd0, dw0 = gpu_grads("f64", kw, sens, target)
    ocfg = O.OracleConfig(**kw)
    tr_o = O.sensor_traces(ocfg, sens, T)
    assert rel(tr, tr_o) <= 1e-12
    r_tau, r_wd0, r_w0 = O.sensor_adjoint(ocfg, sens, 2.0 * (tr_o - target))
    e = (rel(dtau, r_tau), rel(dwd0, r_wd0), rel(dw0, r_w0))
    say(f"  rel errors tau {e[0]:.2e} wdot0 {e[1]:.2e} w0 {e[2]:.2e}")
    assert max(e) <= 1e-12, e


def test_fp64_adjoint_sensors_on_crack_faces_edges_and_periodic():
    nx, ny, T = 50, 20, 70
    j0 = ny // 2 - 1
    sens = np.array([[3, j0], [3, j0 + 1], [0, 0], [nx - 1, ny - 1], [25, 0], [nx - 1, 7], [12, j0 + 1]])
    kw, _, target = case(nx, ny, T, 15, seed=3, sensors=sens)
    tr, dtau, dwd0, dw0 = gpu_grads("f64", kw, sens, target)
    ocfg = O.OracleConfig(**kw)
    r = O.sensor_adjoint(ocfg, sens, 2.0 * (O.sensor_traces(ocfg, sens, T) - target))
    assert max(rel(dtau, r[0]), rel(dwd0, r[1]), rel(dw0, r[2])) <= 1e-12
    # periodic lattice (no edge loads: only the initial fields matter)
    kw, _, target = case(nx, ny, T, None, seed=4, sensors=sens, periodic=True)
    tr, dtau, dwd0, dw0 = gpu_grads("f64", kw, sens, target, periodic=True)
    ocfg = O.OracleConfig(periodic=True, **kw)
    r = O.sensor_adjoint(ocfg, sens, 2.0 * (O.sensor_traces(ocfg, sens, T) - target))
    assert max(rel(dwd0, r[1]), rel(dw0, r[2])) <= 1e-12
    assert np.all(dtau == 0.0)


def loss_gpu(storage, kw, sens, target, tau, wd0):
    T = kw["trace_cap"]
    c = dict(kw, tau_hist=tau, wdot0=wd0)
    s = Solver(Config(storage=storage, sensors=sens, **c))
    s.step(T)
    tr = s.sensor_traces()
    s.close()
    return float(((tr - target) ** 2).sum())


def test_growing_crack_adjoint_matches_exact_central_differences():
    """Prescribed speed: the cut sequence is fixed, the loss is quadratic in
    the inputs, and the central difference is exact up to rounding."""
    nx, ny, T = 120, 40, 200
    kw, sens, target = case(nx, ny, T, 30, seed=8, growth=1, v=0.45)
    s = Solver(Config(storage="f64", sensors=sens, **kw))
    s.step(T)
    assert len(s.cut_events()) > 20
    tr = s.sensor_traces()
    dtau, dwd0, _ = s.adjoint(torch.from_numpy(2.0 * (tr - target)).cuda())
    dwd0 = dwd0.cpu().numpy()
    rng = np.random.default_rng(1)
    for _ in range(3):
        d_tau, d_wd = rng.normal(size=T), rng.normal(size=(ny, nx))
        h = 1e-3
        fd = (loss_gpu("f64", kw, sens, target, kw["tau_hist"] + h * d_tau, kw["wdot0"] + h * d_wd)
              - loss_gpu("f64", kw, sens, target, kw["tau_hist"] - h * d_tau, kw["wdot0"] - h * d_wd)) / (2 * h)
        ad = dtau @ d_tau + (dwd0 * d_wd).sum()
        say(f"  growing crack: adjoint {ad:.12e} central difference {fd:.12e}")
        assert ad == pytest.approx(fd, rel=1e-9)


@pytest.mark.parametrize("storage", ["f32", "f16s"])
def test_reduced_precision_adjoint_against_fp64_central_differences(storage):
    """Directional derivatives along 8 random unit directions in the joint
    (tau history, wdot0) space, normwise over the directions.  Two errors:
    the whole reduced-precision pipeline (traces of the FP32 / FP16-storage
    run feeding the FP32 adjoint), and the FP32 adjoint alone (fed with the
    loss gradient of the FP64 traces).  The loss compares with a target run
    whose traction differs by 10 %, so the trace mismatch is a small
    difference of large numbers and the forward's rounding dominates."""
    nx, ny, T = 256, 128, 400
    kw, sens, target = case(nx, ny, T, 64, seed=5)
    kw["wdot0"] = np.zeros((ny, nx))
    n = np.arange(T)
    tgt_kw = dict(kw, tau_hist=1e-3 * (1 + 0.1 * np.sin(2 * np.pi * n / 80)))
    s = Solver(Config(storage="f64", sensors=sens, **tgt_kw))
    s.step(T)
    target = s.sensor_traces()
    s.close()
    kw["tau_hist"] = np.full(T, 1e-3)
    s = Solver(Config(storage="f64", sensors=sens, **kw))
    s.step(T)
    tr64 = s.sensor_traces()
    s.close()
    s = Solver(Config(storage=storage, sensors=sens, **kw))
    s.step(T)
    tr = s.sensor_traces()
    dtau, dwd0, _ = s.adjoint(torch.from_numpy(2.0 * (tr - target)).cuda())
    dtau_a, dwd0_a, _ = s.adjoint(torch.from_numpy(2.0 * (tr64 - target)).cuda())
    dwd0, dwd0_a = dwd0.cpu().numpy(), dwd0_a.cpu().numpy()
    rng = np.random.default_rng(1)
    fd, ad, ad_a = [], [], []
    for _ in range(8):
        d_tau, d_wd = rng.normal(size=T), rng.normal(size=(ny, nx))
        nrm = np.sqrt((d_tau ** 2).sum() + (d_wd ** 2).sum())
        d_tau, d_wd = d_tau / nrm, d_wd / nrm
        h = 1e-4
        fd.append((loss_gpu("f64", kw, sens, target, kw["tau_hist"] + h * d_tau, h * d_wd)
                   - loss_gpu("f64", kw, sens, target, kw["tau_hist"] - h * d_tau, -h * d_wd)) / (2 * h))
        ad.append(dtau @ d_tau + (dwd0 * d_wd).sum())
        ad_a.append(dtau_a @ d_tau + (dwd0_a * d_wd).sum())
    fd, ad, ad_a = map(np.array, (fd, ad, ad_a))
    e_all = np.linalg.norm(ad - fd) / np.linalg.norm(fd)
    e_adj = np.linalg.norm(ad_a - fd) / np.linalg.norm(fd)
    say(f"  {storage}: pipeline {e_all:.2e}, adjoint alone {e_adj:.2e}")
    assert e_adj <= 1e-5
    assert e_all <= (1e-4 if storage == "f32" else 2e-2)


def test_autograd_function_gives_the_adjoint_gradients():
    nx, ny, T = 64, 32, 100
    kw, sens, target = case(nx, ny, T, 16, seed=9)
    cfg = Config(nx=nx, ny=ny, storage="f64", has_crack=True, crack_tip=15.5, sensors=sens)
    tau = torch.tensor(kw["tau_hist"], requires_grad=True)
    wd0 = torch.tensor(kw["wdot0"], requires_grad=True)
    tr = sensor_run(tau, wd0, cfg)
    loss = ((tr - torch.from_numpy(target).cuda()) ** 2).sum()
    loss.backward()
    ocfg = O.OracleConfig(**kw)
    tr_o = O.sensor_traces(ocfg, sens, T)
    r_tau, r_wd0, _ = O.sensor_adjoint(ocfg, sens, 2.0 * (tr_o - target))
    assert rel(tau.grad.numpy(), r_tau) <= 1e-12
    assert rel(wd0.grad.numpy(), r_wd0) <= 1e-12


def test_fp64_adjoint_with_dirichlet_edges_and_off_centre_crack():
    nx, ny, T = 64, 30, 90
    rng = np.random.default_rng(12)
    sens = np.unique(np.stack([rng.integers(0, nx, 10), rng.integers(0, ny, 10)], axis=1), axis=0)
    n = np.arange(T)
    wD = np.zeros((T, 4))
    wD[:, 1] = 0.01 * np.sin(np.pi * n / 50.0)
    wD[:, 3] = -2e-3
    kw = dict(nx=nx, ny=ny, has_crack=True, crack_row=19, crack_x0=20.5, crack_tip=35.5,
              tau_hist=1e-3 * (1 + 0.2 * rng.normal(size=T)), dirichlet=1 | 2 | 8, wD_hist=wD,
              wdot0=1e-4 * rng.normal(size=(ny, nx)), trace_cap=T)
    target = 1e-3 * rng.normal(size=(T, len(sens)))
    tr, dtau, dwd0, dw0 = gpu_grads("f64", kw, sens, target)
    ocfg = O.OracleConfig(**kw)
    r = O.sensor_adjoint(ocfg, sens, 2.0 * (O.sensor_traces(ocfg, sens, T) - target))
    assert max(rel(dwd0, r[1]), rel(dw0, r[2])) <= 1e-12
    assert rel(dtau, r[0]) <= 1e-12  # the traction acts on the (free) left edge only: none


@pytest.mark.parametrize("storage", ["f32", "f64"])
@pytest.mark.parametrize("growth", [0, 1])
def test_equilibrium_layout_adjoint_equals_five_planes(storage, growth):
    """At omega = 1 all five adjoint populations a sweep writes are equal; the
    equilibrium-layout adjoint keeps one plane and gives the same gradients
    bit for bit (same loss gradient fed to both)."""
    kw, sens, target = case(150, 44, 120, 40, seed=31, growth=growth, v=0.4)
    n = np.arange(120)
    wD = np.zeros((120, 4))
    wD[:, 0] = 5e-3 * np.sin(np.pi * n / 70.0)
    kw.update(dirichlet=1, wD_hist=wD)
    say(f"adjoint eq vs full {storage} growth={growth}")
    out = {}
    for layout in ("full", "eq"):
        s = Solver(Config(storage=storage, layout=layout, sensors=sens, **kw))
        s.step(120)
        if layout == "full":
            g = torch.from_numpy(2.0 * (s.sensor_traces() - target)).cuda()
        dtau, dwd0, dw0 = s.adjoint(g)
        out[layout] = (np.asarray(dtau), dwd0.cpu().numpy(), dw0.cpu().numpy())
        s.close()
    for a, b in zip(out["full"], out["eq"]):
        np.testing.assert_array_equal(a, b)
