"""The C-ABI library loads, exports every symbol include/lbm.h declares, and
rejects unusable configurations before touching a GPU (runs without a GPU)."""
import ctypes as C
import os
import re
import subprocess

import pytest

import paper_2206_12412_amd as P
from paper_2206_12412_amd import lbm as L

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    src = open(os.path.join(ROOT, "include", "lbm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z0-9_]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert declared_functions() == sorted(P.EXPORTS)


def test_library_exports_every_declared_symbol():
    lib = P.load_library()
    for name in declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", P.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(re.findall(r" T (lbm_\w+)", out))
    assert set(declared_functions()) <= exported


def init_rc(**kw):
    keep = []
    cfg = P.Config(**kw).to_c(keep)
    lib = P.load_library()
    h = C.c_void_p()
    return lib.lbm_init(C.byref(cfg), C.byref(h)), lib.lbm_last_error().decode()


@pytest.mark.parametrize("kw,code", [
    (dict(nx=16, ny=8, omega=0.9), -4),
    (dict(nx=16, ny=8, kappa=1.4), -4),
    (dict(nx=0, ny=8), -1),
    (dict(nx=16, ny=7, has_crack=True, crack_tip=3.5), -1),
    (dict(nx=16, ny=8, has_crack=True, crack_tip=16.0), -5),
    (dict(nx=16, ny=8, has_crack=True, crack_x0=-1.0, crack_tip=3.5), -5),
    (dict(nx=16, ny=8, growth=1, v_rel=0.2), -1),
    (dict(nx=16, ny=8, has_crack=True, crack_tip=3.5, growth=1, v_rel=1.0), -1),
    (dict(nx=16, ny=8, has_crack=True, crack_tip=3.5, growth=2, K_C=0.0), -1),
    (dict(nx=16, ny=8, has_crack=True, crack_tip=3.5, k_band=0), -1),
    (dict(nx=16, ny=8, storage=9), -1),
    (dict(nx=16, ny=8, periodic=True, has_crack=True, crack_tip=3.5, growth=1, v_rel=0.2), -1),
    (dict(nx=16, ny=8, storage="f32", rounding="stochastic"), -1),
    (dict(nx=16, ny=8, storage="f64", rounding="stochastic"), -1),
    (dict(nx=16, ny=8, storage="f16s", rounding=7), -1),
])
def test_invalid_configurations_fail_before_any_gpu_call(kw, code):
    rc, msg = init_rc(**kw)
    assert rc == code and msg


def test_device_block_checks():
    lib = P.load_library()
    keep = []
    cfg = P.Config(nx=16, ny=8).to_c(keep)
    need = lib.lbm_state_bytes(C.byref(cfg))
    assert need > 0
    h = C.c_void_p()
    assert lib.lbm_init(C.byref(cfg), C.byref(h)) == -1  # null dev_buf
    cfg.dev_buf = 256 * 1000 + 8
    cfg.dev_bytes = need
    assert lib.lbm_init(C.byref(cfg), C.byref(h)) == -1  # misaligned
    cfg.dev_buf = 256 * 1000
    cfg.dev_bytes = need - 1
    assert lib.lbm_init(C.byref(cfg), C.byref(h)) == -2  # too small
    bad = P.Config(nx=16, ny=8, omega=0.5).to_c(keep)
    assert lib.lbm_state_bytes(C.byref(bad)) == 0


def test_state_bytes_scale_with_storage():
    sizes = {s: P.state_bytes(P.Config(nx=4096, ny=2048, storage=s)) for s in P.STORAGE}
    assert sizes["f64"] > sizes["f32"] > sizes["f16s"]
    assert sizes["f16s"] == sizes["bf16s"]
    # two buffers of five planes plus w (twice for shifted storage)
    assert sizes["f32"] >= (2 * 5 * 4 + 2 * 4) * 4096 * 2048


def test_solver_refuses_cpu_device():
    with pytest.raises(RuntimeError):
        P.Solver(P.Config(nx=16, ny=8), device="cpu")


def test_layout_validation():
    rc, msg = init_rc(nx=16, ny=8, layout=2)
    assert rc == -1 and "layout" in msg
    rc, msg = init_rc(nx=16, ny=8, storage="f32plain", layout="eq")
    assert rc == -1 and "layout" in msg
    for st in ("f64", "f32", "f16s", "bf16s"):
        rc, msg = init_rc(nx=16, ny=8, storage=st, layout="eq")
        assert rc == -1 and "dev_buf" in msg  # valid up to the missing device block
    # the moving planes stay allocated: same state size in both layouts
    a = P.state_bytes(P.Config(nx=300, ny=70, storage="f16s"))
    b = P.state_bytes(P.Config(nx=300, ny=70, storage="f16s", layout="eq"))
    assert a == b


@pytest.mark.parametrize("kw", [
    dict(nx=16, ny=8, periodic=True, bc_scheme="macro"),
    dict(nx=16, ny=6, has_crack=True, crack_tip=3.5, bc_scheme="macro"),
    dict(nx=16, ny=16, has_crack=True, crack_row=7, crack_tip=3.5, crack_dx=0.6, crack_dy=0.8,
         bc_scheme="macro"),
    dict(nx=16, ny=8, bc_scheme=5),
])
def test_macroscopic_scheme_refuses_what_it_cannot_take(kw):
    rc, msg = init_rc(**kw)
    assert rc == -1 and msg


def test_batch_refuses_the_macroscopic_scheme():
    keep = []
    arr = (L._Config * 2)(P.Config(nx=16, ny=8).to_c(keep),
                          P.Config(nx=16, ny=8, bc_scheme="macro").to_c(keep))
    assert P.load_library().lbm_batch_state_bytes(arr, 2) == 0


def splits(m, largest=8):
    """Every split of m steps into sweeps of 1 .. largest steps, longest first."""
    if m == 0:
        yield ()
        return
    for t in range(min(m, largest), 0, -1):
        for rest in splits(m - t, t):
            yield (t,) + rest


@pytest.mark.parametrize("storage", ["f16s", "bf16s", "f32", "f64"])
def test_tail_plan_is_the_cheapest_end_of_a_call(storage):
    """lbm_plan_tail (host only): the call runs whole sweeps of T steps, then
    the tail; checked against every split of the rest and of up to three
    T-step sweeps before it, enumerated here."""
    cost = {t: P.sweep_cost(storage, t) for t in range(1, 9)}
    best_of = {}
    for m in range(0, 32):
        best_of[m] = min(sum(cost[t] for t in s) for s in splits(m))
    for T in range(1, 9):
        for n in list(range(0, 70)) + [1199, 1200, 1201, 10 ** 6 + 5]:
            tail = P.plan_tail(storage, T, n)
            assert all(1 <= t <= 8 for t in tail) and len(tail) <= 32
            assert list(tail) == sorted(tail, reverse=True)
            bulk = n - sum(tail)
            assert bulk >= 0 and bulk % T == 0, (T, n, tail)
            if T == 1 or n % T == 0:
                assert tail == [], (T, n, tail)
                continue
            q, r = divmod(n, T)
            jmax = min(q, 3)
            want = min((jmax - j) * cost[T] + best_of[j * T + r] for j in range(jmax + 1))
            got = (jmax * T + r - sum(tail)) // T * cost[T] + sum(cost[t] for t in tail)
            assert got == pytest.approx(want, rel=1e-12), (T, n, tail)
            # never slower than ending with one shorter sweep
            assert got <= jmax * cost[T] + cost[r] + 1e-9


def test_tail_plan_examples_and_refusals():
    assert P.plan_tail("f16s", 6, 20) == [7, 7]      # 6 + 7 + 7 instead of 6 + 6 + 6 + 2
    assert P.plan_tail("f16s", 6, 1200) == []
    assert P.plan_tail("f16s", 1, 7) == []
    assert P.plan_tail("f64", 8, 20) == [4]
    lib = P.load_library()
    tail = (C.c_int32 * 32)()
    n = C.c_int32()
    assert lib.lbm_plan_tail(0, 0, 10, tail, C.byref(n)) == -1
    assert lib.lbm_plan_tail(0, 9, 10, tail, C.byref(n)) == -1
    assert lib.lbm_plan_tail(7, 6, 10, tail, C.byref(n)) == -1
    assert lib.lbm_plan_tail(0, 6, -1, tail, C.byref(n)) == -1
    assert lib.lbm_plan_tail(0, 6, 10, None, C.byref(n)) == -1
    us = C.c_double()
    assert lib.lbm_sweep_cost(2, 0, C.byref(us)) == -1
    assert lib.lbm_sweep_cost(2, 6, None) == -1
    assert lib.lbm_set_tail_plan(None, 1) == -1
