"""The entry point that allocates nothing: lbm_batch_run_persistent_static,
the persistent batched run with its synchronisation words in the library's
fixed device array, against lbm_batch_run_persistent (words in the batch's
own device block), through the C-ABI.  Two calls in a row on one GPU (the
array keeps the first call's contents), the second with a smaller batch;
every plate bit for bit equal to the existing entry point's."""
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2206_12412_amd import Batch, Config, LBMError  # noqa: E402


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def configs(sizes, steps, storage, layout, seed):
    rng = np.random.default_rng(seed)
    out = []
    for k, (nx, ny) in enumerate(sizes):
        ell = max(nx // 4, 1)
        tau = float(rng.uniform(5e-4, 2e-3))
        c = Config(nx=nx, ny=ny, storage=storage, layout=layout, has_crack=True,
                   crack_tip=ell - 0.5, tau_hist=np.array([tau]), trace_cap=steps,
                   wdot0=rng.normal(0, 1e-4, (ny, nx)))
        if k % 2 == 0:
            c.growth, c.v_rel = 1, float(rng.uniform(0.1, 0.7))
        else:
            c.growth, c.K_C = 2, 1.05 * synth.k_static_edge(tau, ell)
        out.append(c)
    return out


def same(a, b, label):
    np.testing.assert_array_equal(a.populations(), b.populations(), err_msg=label)
    np.testing.assert_array_equal(a.fields()[0], b.fields()[0], err_msg=label)
    ta, tb = a.traces(), b.traces()
    for key in ("K", "tip", "v", "flags"):
        np.testing.assert_array_equal(ta[key], tb[key], err_msg=f"{label} {key}")
    assert a.cut_events().tolist() == b.cut_events().tolist(), label


@pytest.mark.parametrize("storage,layout", [("f32", "eq"), ("f64", "full")])
def test_static_persistent_run_equals_the_persistent_run(storage, layout):
    calls = [([(96, 48), (300, 64), (64, 130), (257, 34), (130, 200), (33, 8), (512, 96)], 120),
             ([(70, 40), (160, 30)], 90)]  # the second call: fewer, smaller plates
    for n, (sizes, steps) in enumerate(calls):
        say(f"no-alloc persistent run, call {n + 1}: {len(sizes)} plates, {storage} {layout}, "
            f"{steps} steps")
        cfgs = configs(sizes, steps, storage, layout, seed=20 + n)
        ref = Batch(cfgs)
        new = Batch(cfgs)
        ref.run_persistent(3)
        new.run_persistent_static(3)
        ref.run_persistent(steps - 3)
        new.run_persistent_static(steps - 3)
        assert new.launch()["persistent_blocks"] > 0
        for k in range(len(cfgs)):
            same(new.plates[k], ref.plates[k], f"call {n + 1} plate {k}")
        ref.close()
        new.close()


def test_static_persistent_run_rejects_invalid_calls():
    from paper_2206_12412_amd.lbm import load_library
    lib = load_library()
    cfgs = configs([(16, 8)] * 3, 4, "f32", "full", seed=3)
    b = Batch(cfgs)
    b.run_persistent_static(4)  # small batches fit
    b.close()
    assert lib.lbm_batch_run_persistent_static(None, 1) != 0
    with pytest.raises(LBMError):
        Batch(cfgs).run_persistent_static(-1)
