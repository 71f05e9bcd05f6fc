"""ctypes binding of liblbmcrack (include/lbm.h): argument marshalling only.

PyTorch provides the device memory block (one uint8 tensor of
``lbm_state_bytes`` bytes) and the HIP stream (torch's current stream on the
device); every step of the method runs in the library's HIP kernels.  There is
no fallback: without the built library on a GPU device the calls raise.
"""
from __future__ import annotations

import ctypes as C
import os
import dataclasses
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbmcrack.so")

LBM_F64, LBM_F32, LBM_F16S, LBM_BF16S, LBM_F32_PLAIN = 0, 1, 2, 3, 4
STORAGE = {"f64": LBM_F64, "f32": LBM_F32, "f16s": LBM_F16S, "bf16s": LBM_BF16S,
           "f32plain": LBM_F32_PLAIN}
GROW_NONE, GROW_PRESCRIBED, GROW_SIF = 0, 1, 2
BC_WALLS, BC_PERIODIC = 0, 1
ROUNDING = {"nearest": 0, "stochastic": 1}
# "full": five populations and w per site; "eq": the rest population and w
# (the moving populations rebuilt from the equilibrium of the emitting site,
# exact at omega = 1; shifted storages only)
LAYOUT = {"full": 0, "eq": 1}
# boundary points: "link" bounce-back per link, "macro" the scheme of Sec. 3.1
BC_SCHEME = {"link": 0, "macro": 1}
EDGE_BOTTOM, EDGE_TOP, EDGE_LEFT, EDGE_RIGHT = 1, 2, 4, 8
FLAG_GREW, FLAG_WALL, FLAG_K_UNDEF = 1, 2, 4

ERRORS = {-1: "LBM_EINVAL", -2: "LBM_ENOMEM", -3: "LBM_EHIP", -4: "LBM_EUNSTABLE",
          -5: "LBM_ECRACK", -6: "LBM_ESTATE"}

# every symbol include/lbm.h declares
EXPORTS = ("lbm_state_bytes", "lbm_init", "lbm_step", "lbm_crack_state", "lbm_sif", "lbm_traces",
           "lbm_cut_events", "lbm_cut_links", "lbm_get_fields", "lbm_get_populations", "lbm_get_mask",
           "lbm_timing", "lbm_get_launch", "lbm_set_launch", "lbm_set_time_block", "lbm_time_block_stats",
           "lbm_autotune_time_block",
           "lbm_bytes_per_site", "lbm_free", "lbm_last_error", "lbm_batch_state_bytes",
           "lbm_batch_init", "lbm_batch_step", "lbm_batch_run_persistent",
           "lbm_batch_run_persistent_static", "lbm_batch_plate",
           "lbm_batch_set_launch", "lbm_batch_get_launch", "lbm_batch_timing", "lbm_batch_sites",
           "lbm_batch_free", "lbm_autotune", "lbm_batch_autotune", "lbm_round16",
           "lbm_sensor_traces", "lbm_adjoint_bytes", "lbm_adjoint_init", "lbm_adjoint_run",
           "lbm_adjoint_timing", "lbm_adjoint_free", "lbm_checkpoint_bytes", "lbm_checkpoint",
           "lbm_restore", "lbm_traces_left", "lbm_set_tail_plan", "lbm_plan_tail", "lbm_sweep_cost")


class LBMError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code


class _Config(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("storage", C.c_int32), ("bc_mode", C.c_int32),
        ("kappa", C.c_double), ("omega", C.c_double), ("mu", C.c_double), ("rho", C.c_double),
        ("has_crack", C.c_int32), ("crack_x0", C.c_double), ("crack_tip", C.c_double),
        ("growth", C.c_int32), ("v_rel", C.c_double), ("K_C", C.c_double), ("r0", C.c_double),
        ("v_max", C.c_double), ("k_band", C.c_int32), ("face_traction", C.c_double),
        ("tau_hist", C.POINTER(C.c_double)), ("n_hist", C.c_int64),
        ("w0", C.POINTER(C.c_double)), ("wdot0", C.POINTER(C.c_double)),
        ("trace_cap", C.c_int64), ("rounding", C.c_int32), ("seed", C.c_uint32),
        ("n_sensors", C.c_int32), ("sensors", C.POINTER(C.c_int32)),
        ("crack_row", C.c_int32), ("both_tips", C.c_int32), ("dirichlet", C.c_int32),
        ("wD_hist", C.POINTER(C.c_double)), ("n_wD", C.c_int64),
        ("layout", C.c_int32),
        ("crack_dx", C.c_double), ("crack_dy", C.c_double), ("bc_scheme", C.c_int32),
        ("dev_buf", C.c_void_p), ("dev_bytes", C.c_size_t),
        ("stream", C.c_void_p),
    ]


class CrackInfo(C.Structure):
    _fields_ = [("tip", C.c_double), ("v", C.c_double), ("K", C.c_double), ("r", C.c_double),
                ("step", C.c_int64), ("flags", C.c_int32), ("n_events", C.c_int32),
                ("col_K", C.c_int32), ("n_cut", C.c_int32),
                ("tip_left", C.c_double), ("v_left", C.c_double), ("K_left", C.c_double),
                ("r_left", C.c_double), ("flags_left", C.c_int32), ("col_K_left", C.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_lib = None


def load_library(path: str = LIB_PATH):
    """Load liblbmcrack.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: run paper_2206_12412_amd/build.py (or "
                           "__graft_entry__.build()) first; there is no CPU fallback")
    # torch first: its HIP runtime is then the one the library binds to, so
    # that both see the same devices, streams and memory (loading the library
    # first would bind it to another copy of the runtime, without a context)
    import torch  # noqa: F401
    lib = C.CDLL(path)
    P, d, i32, i64, vp = C.POINTER, C.c_double, C.c_int32, C.c_int64, C.c_void_p
    lib.lbm_state_bytes.argtypes = [P(_Config)]
    lib.lbm_state_bytes.restype = C.c_size_t
    lib.lbm_init.argtypes = [P(_Config), P(vp)]
    lib.lbm_step.argtypes = [vp, i64]
    lib.lbm_crack_state.argtypes = [vp, P(CrackInfo)]
    lib.lbm_sif.argtypes = [vp, P(d), i64, i64]
    lib.lbm_traces.argtypes = [vp, P(d), P(d), P(i32), i64, i64]
    lib.lbm_traces_left.argtypes = [vp, P(d), P(d), P(d), P(i32), i64, i64]
    lib.lbm_cut_events.argtypes = [vp, P(i64), P(i32), i64, P(i64)]
    lib.lbm_cut_links.argtypes = [vp, P(i64), P(i32), P(i32), P(i32), i64, P(i64)]
    lib.lbm_set_time_block.argtypes = [vp, i32, i32, i32]
    lib.lbm_set_time_block.restype = i32
    lib.lbm_time_block_stats.argtypes = [vp, P(i64), P(i64)]
    lib.lbm_time_block_stats.restype = i32
    lib.lbm_autotune_time_block.argtypes = [vp, i32, i32, P(i32), P(i32), P(d)]
    lib.lbm_set_tail_plan.argtypes = [vp, i32]
    lib.lbm_set_tail_plan.restype = i32
    lib.lbm_plan_tail.argtypes = [i32, i32, i64, P(i32), P(i32)]
    lib.lbm_plan_tail.restype = i32
    lib.lbm_sweep_cost.argtypes = [i32, i32, P(d)]
    lib.lbm_sweep_cost.restype = i32
    lib.lbm_autotune_time_block.restype = i32
    lib.lbm_get_fields.argtypes = [vp, P(d), P(d)]
    lib.lbm_get_populations.argtypes = [vp, P(d)]
    lib.lbm_get_mask.argtypes = [vp, P(C.c_uint8), P(C.c_uint8)]
    lib.lbm_timing.argtypes = [vp, i32, P(d), P(d), P(i64)]
    lib.lbm_get_launch.argtypes = [vp, P(i32), P(i32), P(i32), P(i32)]
    lib.lbm_set_launch.argtypes = [vp, i32, i32, i32]
    lib.lbm_bytes_per_site.argtypes = [vp]
    lib.lbm_bytes_per_site.restype = d
    lib.lbm_free.argtypes = [vp]
    lib.lbm_free.restype = None
    lib.lbm_last_error.restype = C.c_char_p
    lib.lbm_batch_state_bytes.argtypes = [P(_Config), i32]
    lib.lbm_batch_state_bytes.restype = C.c_size_t
    lib.lbm_batch_init.argtypes = [P(_Config), i32, vp, C.c_size_t, vp, P(vp)]
    lib.lbm_batch_step.argtypes = [vp, i64]
    lib.lbm_batch_run_persistent.argtypes = [vp, i64]
    lib.lbm_batch_run_persistent_static.argtypes = [vp, i64]
    lib.lbm_batch_plate.argtypes = [vp, i32]
    lib.lbm_batch_plate.restype = vp
    lib.lbm_batch_set_launch.argtypes = [vp, i32, i32, i32]
    lib.lbm_batch_get_launch.argtypes = [vp, P(i32), P(i32), P(i32), P(i32)]
    lib.lbm_batch_timing.argtypes = [vp, i32, P(d), P(i64)]
    lib.lbm_batch_sites.argtypes = [vp]
    lib.lbm_batch_sites.restype = i64
    lib.lbm_batch_free.argtypes = [vp]
    lib.lbm_batch_free.restype = None
    lib.lbm_autotune.argtypes = [vp, i32, P(i32), P(i32), P(i32), P(d)]
    lib.lbm_round16.argtypes = [vp, vp, i64, i32, i32, i32, C.c_uint32, i64, vp]
    lib.lbm_sensor_traces.argtypes = [vp, vp, i64, i64, i32]
    lib.lbm_checkpoint_bytes.argtypes = [vp]
    lib.lbm_checkpoint_bytes.restype = C.c_size_t
    lib.lbm_checkpoint.argtypes = [vp, vp]
    lib.lbm_restore.argtypes = [vp, vp]
    lib.lbm_adjoint_bytes.argtypes = [vp]
    lib.lbm_adjoint_bytes.restype = C.c_size_t
    lib.lbm_adjoint_init.argtypes = [vp, vp, C.c_size_t, P(vp)]
    lib.lbm_adjoint_run.argtypes = [vp, vp, vp, vp, vp]
    lib.lbm_adjoint_timing.argtypes = [vp, P(d), P(i64)]
    lib.lbm_adjoint_free.argtypes = [vp]
    lib.lbm_adjoint_free.restype = None
    lib.lbm_batch_autotune.argtypes = [vp, i32, P(i32), P(i32), P(i32), P(d)]
    for name in ("lbm_traces_left", "lbm_checkpoint", "lbm_restore", "lbm_sensor_traces", "lbm_adjoint_init", "lbm_adjoint_run", "lbm_adjoint_timing",
                 "lbm_round16", "lbm_autotune", "lbm_batch_autotune", "lbm_batch_init", "lbm_batch_step", "lbm_batch_run_persistent",
                 "lbm_batch_run_persistent_static", "lbm_batch_set_launch", "lbm_batch_get_launch", "lbm_batch_timing"):
        getattr(lib, name).restype = i32
    for name in ("lbm_init", "lbm_step", "lbm_crack_state", "lbm_sif", "lbm_traces",
                 "lbm_cut_events", "lbm_cut_links", "lbm_get_fields", "lbm_get_populations",
                 "lbm_get_mask", "lbm_timing", "lbm_get_launch", "lbm_set_launch"):
        getattr(lib, name).restype = i32
    _lib = lib
    return lib


def _check(rc: int):
    if rc != 0:
        raise LBMError(rc, load_library().lbm_last_error().decode())


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


@dataclass
class Config:
    """Mirror of lbm_config without the device block and stream."""
    nx: int
    ny: int
    storage: str = "f32"
    periodic: bool = False
    kappa: float = 2.0
    omega: float = 1.0
    mu: float = 1.0
    rho: float = 1.0
    has_crack: bool = False
    crack_x0: float = -0.5
    crack_tip: float = -0.5
    growth: int = GROW_NONE
    v_rel: float = 0.0
    K_C: float = 0.0
    r0: float = 2.0
    v_max: float = 0.85
    k_band: int = 1
    face_traction: float = 0.0
    tau_hist: Optional[np.ndarray] = None
    w0: Optional[np.ndarray] = None
    wdot0: Optional[np.ndarray] = None
    trace_cap: int = 0
    rounding: str = "nearest"      # 16-bit storages: "nearest" or "stochastic"
    seed: int = 0
    sensors: Optional[np.ndarray] = None   # (n, 2) sites (i, j) whose w is recorded per step
    crack_row: int = -1                   # crack line y = crack_row + 1/2; -1 = mid-line
    both_tips: bool = False               # the left end grows in -x as well
    dirichlet: int = 0                    # EDGE_* bits of the edges holding a prescribed w
    wD_hist: Optional[np.ndarray] = None  # (n, 4) wall w* of (bottom, top, left, right) per step
    layout: str = "full"                  # "full" (five populations) or "eq" (see LAYOUT)
    crack_dx: float = 1.0                 # growth direction of the right tip (Alg. 1, d);
    crack_dy: float = 0.0                 # (1, 0) = +x along crack_row
    bc_scheme: str = "link"               # "link" (bounce-back per link) or "macro" (Sec. 3.1)

    def to_c(self, keep: list) -> _Config:
        c = _Config()
        for name in ("nx", "ny", "kappa", "omega", "mu", "rho", "crack_x0", "crack_tip", "growth",
                     "v_rel", "K_C", "r0", "v_max", "k_band", "face_traction", "trace_cap"):
            setattr(c, name, getattr(self, name))
        c.storage = STORAGE[self.storage] if isinstance(self.storage, str) else int(self.storage)
        c.bc_mode = BC_PERIODIC if self.periodic else BC_WALLS
        c.has_crack = int(self.has_crack)
        c.rounding = ROUNDING[self.rounding] if isinstance(self.rounding, str) else int(self.rounding)
        c.layout = LAYOUT[self.layout] if isinstance(self.layout, str) else int(self.layout)
        c.crack_dx, c.crack_dy = float(self.crack_dx), float(self.crack_dy)
        c.bc_scheme = BC_SCHEME[self.bc_scheme] if isinstance(self.bc_scheme, str) else int(self.bc_scheme)
        c.crack_row = int(self.crack_row)
        c.both_tips = int(self.both_tips)
        c.dirichlet = int(self.dirichlet)
        if self.wD_hist is not None:
            wd = np.ascontiguousarray(self.wD_hist, dtype=np.float64).reshape(-1, 4)
            keep.append(wd)
            c.wD_hist = _dp(wd)
            c.n_wD = wd.shape[0]
        c.seed = int(self.seed) & 0xFFFFFFFF
        if self.sensors is not None:
            sens = np.ascontiguousarray(self.sensors, dtype=np.int32).reshape(-1, 2)
            keep.append(sens)
            c.n_sensors = sens.shape[0]
            c.sensors = sens.ctypes.data_as(C.POINTER(C.c_int32))
        if self.tau_hist is not None:
            t = np.ascontiguousarray(self.tau_hist, dtype=np.float64).ravel()
            keep.append(t)
            c.tau_hist = _dp(t)
            c.n_hist = t.size
        for name in ("w0", "wdot0"):
            a = getattr(self, name)
            if a is not None:
                a = np.ascontiguousarray(a, dtype=np.float64)
                if a.shape != (self.ny, self.nx):
                    raise ValueError(f"{name} must have shape (ny, nx)")
                keep.append(a)
                setattr(c, name, _dp(a))
        return c


def state_bytes(cfg: Config) -> int:
    keep = []
    return int(load_library().lbm_state_bytes(C.byref(cfg.to_c(keep))))


def round16(x, storage: str = "f16s", rounding: str = "nearest", plane: int = 0, seed: int = 0,
            step: int = 0):
    """lbm_round16 on a CUDA float32 tensor; returns the 16-bit tensor."""
    import torch

    lib = load_library()
    x = x.contiguous()
    if x.dtype != torch.float32 or x.device.type != "cuda":
        raise ValueError("x must be a float32 tensor on a GPU")
    out = torch.empty(x.shape, dtype=torch.float16 if storage == "f16s" else torch.bfloat16,
                      device=x.device)
    st = torch.cuda.current_stream(x.device)
    _check(lib.lbm_round16(x.data_ptr(), out.data_ptr(), x.numel(), STORAGE[storage],
                           ROUNDING[rounding], int(plane), int(seed) & 0xFFFFFFFF, int(step),
                           st.cuda_stream))
    return out


def plan_tail(storage: str, steps_per_sweep: int, nsteps: int) -> list:
    """lbm_plan_tail: the sweep lengths that end a call of nsteps steps at
    steps_per_sweep steps per sweep (host only)."""
    tail = (C.c_int32 * 32)()
    n = C.c_int32()
    _check(load_library().lbm_plan_tail(STORAGE[storage], int(steps_per_sweep), int(nsteps), tail,
                                        C.byref(n)))
    return [int(tail[k]) for k in range(n.value)]


def sweep_cost(storage: str, steps: int) -> float:
    """lbm_sweep_cost: the time (us) of one sweep of `steps` steps the plan
    works from (host only)."""
    us = C.c_double()
    _check(load_library().lbm_sweep_cost(STORAGE[storage], int(steps), C.byref(us)))
    return us.value


def _tune(fn, handle, trial_steps: int) -> dict:
    r, w, o, ms = C.c_int32(), C.c_int32(), C.c_int32(), C.c_double()
    _check(fn(handle, int(trial_steps), C.byref(r), C.byref(w), C.byref(o), C.byref(ms)))
    return {"rows": r.value, "waves": w.value, "occupancy": o.value, "ms_per_step": ms.value}


class Solver:
    """One plate on one GPU, driven through the C-ABI."""

    def __init__(self, cfg: Config, device: str = "cuda", stream=None):
        import torch

        lib = load_library()
        self.cfg = cfg
        keep: list = []
        c = cfg.to_c(keep)
        nbytes = lib.lbm_state_bytes(C.byref(c))
        if nbytes == 0:
            _check(-1)
        dev = torch.device(device)
        if dev.type != "cuda":
            raise RuntimeError("the solver runs on a GPU device only")
        self._buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        ptr = self._buf.data_ptr()
        ptr += (-ptr) % 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        c.dev_buf = ptr
        c.dev_bytes = nbytes
        c.stream = self.stream.cuda_stream
        h = C.c_void_p()
        _check(lib.lbm_init(C.byref(c), C.byref(h)))
        self._h = h
        self._lib = lib
        self.steps_done = 0

    def close(self):
        if getattr(self, "_h", None):
            self._lib.lbm_free(self._h)
            self._h = None

    def __del__(self):
        self.close()

    @property
    def shape(self):
        return (self.cfg.ny, self.cfg.nx)

    def step(self, n: int = 1):
        _check(self._lib.lbm_step(self._h, int(n)))
        self.steps_done += int(n)

    def crack_state(self) -> dict:
        info = CrackInfo()
        _check(self._lib.lbm_crack_state(self._h, C.byref(info)))
        return info.as_dict()

    def sif(self, first: int = 0, count: Optional[int] = None) -> np.ndarray:
        if count is None:
            count = min(self.steps_done, self.cfg.trace_cap) - first
        out = np.empty(count)
        _check(self._lib.lbm_sif(self._h, _dp(out), int(first), int(count)))
        return out

    def traces(self, first: int = 0, count: Optional[int] = None, tip: str = "right") -> dict:
        """Per-step K, tip position, speed and flags of the right (or, with
        two tips, the left) tip."""
        if count is None:
            count = min(self.steps_done, self.cfg.trace_cap) - first
        K, a, v = np.empty(count), np.empty(count), np.empty(count)
        fl = np.empty(count, np.int32)
        fp = fl.ctypes.data_as(C.POINTER(C.c_int32))
        if tip == "left":
            _check(self._lib.lbm_traces_left(self._h, _dp(K), _dp(a), _dp(v), fp, int(first),
                                             int(count)))
        elif count:
            _check(self._lib.lbm_sif(self._h, _dp(K), int(first), int(count)))
            _check(self._lib.lbm_traces(self._h, _dp(a), _dp(v), fp, int(first), int(count)))
        return {"K": K, "tip": a, "v": v, "flags": fl}

    def sensor_traces(self, first: int = 0, count: Optional[int] = None, device: bool = False):
        """w at the sensor sites after each step, [count][n_sensors] (numpy,
        or a float64 tensor on the solver's device)."""
        n = 0 if self.cfg.sensors is None else len(np.asarray(self.cfg.sensors).reshape(-1, 2))
        if count is None:
            count = min(self.steps_done, self.cfg.trace_cap) - first
        if device:
            import torch

            out = torch.empty((count, n), dtype=torch.float64, device=self._buf.device)
            if count and n:
                _check(self._lib.lbm_sensor_traces(self._h, out.data_ptr(), int(first), int(count), 1))
            return out
        out = np.empty((count, n))
        if count and n:
            _check(self._lib.lbm_sensor_traces(self._h, _dp(out), int(first), int(count), 0))
        return out

    def adjoint(self, g, timing: bool = False):
        """Discrete adjoint through every step taken, for a loss whose
        gradient with respect to the sensor traces is g ([steps][n_sensors],
        float64 tensor on the solver's device).  Returns (dL/dtau per step as
        numpy, dL/dwdot0 and dL/dw0 as float64 tensors [ny][nx]) and, with
        timing, the adjoint kernel time in ms."""
        import torch

        lib = self._lib
        nbytes = lib.lbm_adjoint_bytes(self._h)
        if nbytes == 0:
            _check(-1)
        dev = self._buf.device
        buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        ptr = buf.data_ptr() + (-buf.data_ptr()) % 256
        a = C.c_void_p()
        _check(lib.lbm_adjoint_init(self._h, ptr, nbytes, C.byref(a)))
        try:
            g = g.to(device=dev, dtype=torch.float64).contiguous()
            T = self.steps_done
            dtau = np.empty(T)
            dwd0 = torch.empty(self.shape, dtype=torch.float64, device=dev)
            dw0 = torch.empty(self.shape, dtype=torch.float64, device=dev)
            _check(lib.lbm_adjoint_run(a, g.data_ptr(), _dp(dtau), dwd0.data_ptr(), dw0.data_ptr()))
            ms = C.c_double()
            _check(lib.lbm_adjoint_timing(a, C.byref(ms), None))
        finally:
            lib.lbm_adjoint_free(a)
        return (dtau, dwd0, dw0, ms.value) if timing else (dtau, dwd0, dw0)

    def checkpoint(self):
        """The state after the steps taken so far, as a device uint8 tensor."""
        import torch

        n = self._lib.lbm_checkpoint_bytes(self._h)
        buf = torch.empty(n + 256, dtype=torch.uint8, device=self._buf.device)
        off = (-buf.data_ptr()) % 256
        _check(self._lib.lbm_checkpoint(self._h, buf.data_ptr() + off))
        return buf[off:off + n]

    def restore(self, ckpt):
        """Continue from a checkpoint of a plate with the same configuration."""
        import torch

        ptr = ckpt.data_ptr()
        if ptr % 256:  # the library wants a 256-byte aligned block
            tmp = torch.empty(ckpt.numel() + 256, dtype=torch.uint8, device=ckpt.device)
            off = (-tmp.data_ptr()) % 256
            tmp[off:off + ckpt.numel()].copy_(ckpt)
            ckpt, ptr = tmp, tmp.data_ptr() + off
        _check(self._lib.lbm_restore(self._h, ptr))
        self.steps_done = int(self.crack_state()["step"])

    def cut_events(self) -> np.ndarray:
        n = C.c_int64()
        _check(self._lib.lbm_cut_events(self._h, None, None, 0, C.byref(n)))
        steps = np.empty(n.value, np.int64)
        cols = np.empty(n.value, np.int32)
        if n.value:
            _check(self._lib.lbm_cut_events(self._h, steps.ctypes.data_as(C.POINTER(C.c_int64)),
                                            cols.ctypes.data_as(C.POINTER(C.c_int32)), n.value,
                                            C.byref(n)))
        return np.stack([steps, cols.astype(np.int64)], axis=1)

    def cut_links(self) -> np.ndarray:
        """(step, i, j, orientation) of every link severed by growth, in order
        (orientation 0: vertical link (i,j)-(i,j+1), 1: horizontal (i,j)-(i+1,j))."""
        n = C.c_int64()
        _check(self._lib.lbm_cut_links(self._h, None, None, None, None, 0, C.byref(n)))
        steps = np.empty(n.value, np.int64)
        ijo = [np.empty(n.value, np.int32) for _ in range(3)]
        if n.value:
            P32 = C.POINTER(C.c_int32)
            _check(self._lib.lbm_cut_links(self._h, steps.ctypes.data_as(C.POINTER(C.c_int64)),
                                           *(a.ctypes.data_as(P32) for a in ijo), n.value,
                                           C.byref(n)))
        return np.stack([steps] + [a.astype(np.int64) for a in ijo], axis=1)

    def fields(self):
        w = np.empty(self.shape)
        wd = np.empty(self.shape)
        _check(self._lib.lbm_get_fields(self._h, _dp(w), _dp(wd)))
        return w, wd

    def populations(self) -> np.ndarray:
        f = np.empty((5,) + self.shape)
        _check(self._lib.lbm_get_populations(self._h, _dp(f)))
        return f

    def mask(self):
        v = np.empty(self.shape, np.uint8)
        h = np.empty(self.shape, np.uint8)
        P = C.POINTER(C.c_uint8)
        _check(self._lib.lbm_get_mask(self._h, v.ctypes.data_as(P), h.ctypes.data_as(P)))
        return v, h

    def timing(self, enable, stride: int = 1):
        """Start (True; every `stride`-th step) or stop (False) per-kernel
        HIP-event timing; returns the summed sweep and crack kernel times and
        the number of timed steps."""
        sw, k = C.c_double(), C.c_double()
        n = C.c_int64()
        _check(self._lib.lbm_timing(self._h, int(stride) if enable else 0, C.byref(sw), C.byref(k),
                                    C.byref(n)))
        return {"sweep_ms": sw.value, "crack_ms": k.value, "steps": n.value}

    def sites(self) -> int:
        return self.cfg.nx * self.cfg.ny

    def launch(self):
        v, r, w, o = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        _check(self._lib.lbm_get_launch(self._h, C.byref(v), C.byref(r), C.byref(w), C.byref(o)))
        return {"vec": v.value, "rows": r.value, "waves": w.value, "occupancy": o.value}

    def set_launch(self, rows: int, waves: int, occupancy: int = 0):
        _check(self._lib.lbm_set_launch(self._h, int(rows), int(waves), int(occupancy)))

    def set_time_block(self, steps: int = 2, rows: int = 0, waves: int = 0):
        """Advance `steps` (1 to 8) time steps per sweep; see lbm_set_time_block."""
        _check(self._lib.lbm_set_time_block(self._h, int(steps), int(rows), int(waves)))

    def set_tail_plan(self, on: bool = True):
        """Whether a call whose step count is not a multiple of T ends with
        the planned sweeps (plan_tail) or with one shorter sweep; see
        lbm_set_tail_plan."""
        _check(self._lib.lbm_set_tail_plan(self._h, 1 if on else 0))

    def autotune_time_block(self, steps: int, trial_sweeps: int = 4) -> dict:
        """Searches the T-step sweep's shapes (steps = T) on a scratch plate
        built from this plate's config (this plate's state is untouched) and
        sets steps = T with the fastest shape here."""
        scratch = Solver(dataclasses.replace(self.cfg, trace_cap=0), device=str(self._buf.device),
                         stream=self.stream)
        r, w, ms = C.c_int32(), C.c_int32(), C.c_double()
        try:
            _check(self._lib.lbm_autotune_time_block(scratch._h, int(steps), int(trial_sweeps),
                                                     C.byref(r), C.byref(w), C.byref(ms)))
        finally:
            scratch.close()
            del scratch
        self.set_time_block(steps, r.value, w.value)
        return {"steps": int(steps), "rows": r.value, "waves": w.value, "ms_per_step": ms.value}

    def time_block_stats(self) -> dict:
        """T-step sweeps run under the K criterion and how many were run again
        with fewer steps (a link severed before their last step)."""
        n, r = C.c_int64(), C.c_int64()
        _check(self._lib.lbm_time_block_stats(self._h, C.byref(n), C.byref(r)))
        return {"sweeps": n.value, "reruns": r.value}

    def autotune(self, trial_steps: int = 8) -> dict:
        """Searches the launch-shape grid on a scratch plate built from this
        plate's config (this plate's state is untouched) and applies the
        fastest shape here."""
        scratch = Solver(dataclasses.replace(self.cfg, trace_cap=0), device=str(self._buf.device),
                         stream=self.stream)
        try:
            out = _tune(self._lib.lbm_autotune, scratch._h, trial_steps)
        finally:
            scratch.close()
            del scratch
        self.set_launch(out["rows"], out["waves"], out["occupancy"])
        return out

    def bytes_per_site(self) -> float:
        return float(self._lib.lbm_bytes_per_site(self._h))


class _PlateView(Solver):
    """Query handle of one plate of a batch (owned by the batch)."""

    def __init__(self, batch, k: int, cfg: Config, h):  # noqa: super().__init__ not called
        self.cfg = cfg
        self._h = h
        self._lib = batch._lib
        self._batch = batch
        self.stream = batch.stream

    @property
    def steps_done(self):
        return self._batch.steps_done

    @steps_done.setter
    def steps_done(self, v):
        pass

    def close(self):
        self._h = None

    def step(self, n: int = 1):
        raise RuntimeError("plates of a batch are stepped through the batch")

    def set_launch(self, rows: int, waves: int, occupancy: int = 0):
        raise RuntimeError("the launch shape of a batch is set on the batch")

    def set_time_block(self, steps: int = 2, rows: int = 0, waves: int = 0):
        raise RuntimeError("plates of a batch step one time step per sweep")

    def autotune(self, trial_steps: int = 8) -> dict:
        raise RuntimeError("a batch is tuned as a whole (Batch.autotune)")


class Batch:
    """Many plates (same storage) advanced together on one GPU."""

    def __init__(self, cfgs, device: str = "cuda", stream=None):
        import torch

        lib = load_library()
        self.cfgs = list(cfgs)
        keep: list = []
        arr = (_Config * len(self.cfgs))(*[c.to_c(keep) for c in self.cfgs])
        nbytes = lib.lbm_batch_state_bytes(arr, len(self.cfgs))
        if nbytes == 0:
            _check(-1)
        dev = torch.device(device)
        if dev.type != "cuda":
            raise RuntimeError("the batch runs on a GPU device only")
        self._buf = torch.empty(nbytes + 256, dtype=torch.uint8, device=dev)
        ptr = self._buf.data_ptr()
        ptr += (-ptr) % 256
        self.stream = stream if stream is not None else torch.cuda.current_stream(dev)
        b = C.c_void_p()
        _check(lib.lbm_batch_init(arr, len(self.cfgs), ptr, nbytes, self.stream.cuda_stream,
                                  C.byref(b)))
        self._b = b
        self._lib = lib
        self.steps_done = 0
        self.plates = []
        for k, c in enumerate(self.cfgs):
            h = lib.lbm_batch_plate(b, k)
            self.plates.append(_PlateView(self, k, c, C.c_void_p(h)))

    def close(self):
        if getattr(self, "_b", None):
            for p in self.plates:
                p.close()
            self._lib.lbm_batch_free(self._b)
            self._b = None

    def __del__(self):
        self.close()

    def step(self, n: int = 1):
        _check(self._lib.lbm_batch_step(self._b, int(n)))
        self.steps_done += int(n)

    def run_persistent(self, n: int):
        _check(self._lib.lbm_batch_run_persistent(self._b, int(n)))
        self.steps_done += int(n)

    def run_persistent_static(self, n: int):
        """run_persistent with the synchronisation words in the library's
        fixed device array (lbm_batch_run_persistent_static: allocates nothing)."""
        _check(self._lib.lbm_batch_run_persistent_static(self._b, int(n)))
        self.steps_done += int(n)

    def set_launch(self, rows: int, waves: int, occupancy: int = 0):
        _check(self._lib.lbm_batch_set_launch(self._b, int(rows), int(waves), int(occupancy)))

    def autotune(self, trial_steps: int = 4) -> dict:
        """lbm_batch_autotune on a scratch batch of the same plates; applies
        the fastest shape to this batch."""
        scratch = Batch([dataclasses.replace(c, trace_cap=0) for c in self.cfgs],
                        device=str(self._buf.device), stream=self.stream)
        try:
            out = _tune(self._lib.lbm_batch_autotune, scratch._b, trial_steps)
        finally:
            scratch.close()
            del scratch
        self.set_launch(out["rows"], out["waves"], out["occupancy"])
        return out

    def launch(self):
        r, w, o, pb = C.c_int32(), C.c_int32(), C.c_int32(), C.c_int32()
        _check(self._lib.lbm_batch_get_launch(self._b, C.byref(r), C.byref(w), C.byref(o),
                                              C.byref(pb)))
        return {"rows": r.value, "waves": w.value, "occupancy": o.value,
                "persistent_blocks": pb.value}

    def timing(self, enable: bool):
        ms = C.c_double()
        n = C.c_int64()
        _check(self._lib.lbm_batch_timing(self._b, int(enable), C.byref(ms), C.byref(n)))
        return {"ms": ms.value, "intervals": n.value}

    def sites(self) -> int:
        return int(self._lib.lbm_batch_sites(self._b))
