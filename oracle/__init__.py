"""FP64 CPU oracle of the D2Q5 lattice Boltzmann method for antiplane shear with
dynamic mode III cracks (arXiv:2206.12412, Sec. 3 and Sec. 4, Alg. 1).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares no code
with the HIP library ``paper_2206_12412_amd`` and never imports it.

The arithmetic lives in ``lbm_oracle.c`` (plain C, FP64, loops over j, i, alpha);
this module only builds it with gcc and marshals arguments through ctypes.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB = os.path.join(_HERE, "liblbm_oracle.so")

GROW_NONE, GROW_PRESCRIBED, GROW_SIF = 0, 1, 2
EDGE_BOTTOM, EDGE_TOP, EDGE_LEFT, EDGE_RIGHT = 1, 2, 4, 8
FLAG_GREW, FLAG_WALL, FLAG_K_UNDEF = 1, 2, 4
BC_LINK, BC_MACRO = 0, 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (no fast-math, no FMA contraction)."""
    if force or not os.path.exists(_LIB):
        cmd = ["gcc", "-O2", "-std=c11", "-D_GNU_SOURCE", "-ffp-contract=off", "-fopenmp",
               "-fPIC", "-shared", "-Wall", "-o", _LIB + ".tmp", _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(_LIB + ".tmp", _LIB)
    return _LIB


class _Cfg(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("periodic", C.c_int32),
        ("kappa", C.c_double), ("omega", C.c_double), ("mu", C.c_double), ("rho", C.c_double),
        ("has_crack", C.c_int32), ("crack_x0", C.c_double), ("crack_tip", C.c_double),
        ("growth", C.c_int32), ("v_rel", C.c_double), ("K_C", C.c_double), ("r0", C.c_double),
        ("v_max", C.c_double), ("k_band", C.c_int32), ("face_traction", C.c_double),
        ("tau_hist", C.POINTER(C.c_double)), ("n_hist", C.c_int64),
        ("w0", C.POINTER(C.c_double)), ("wdot0", C.POINTER(C.c_double)),
        ("trace_cap", C.c_int64), ("threads", C.c_int32),
        ("crack_row", C.c_int32), ("both_tips", C.c_int32), ("dirichlet", C.c_int32),
        ("wD_hist", C.POINTER(C.c_double)), ("n_wD", C.c_int64),
        ("crack_dx", C.c_double), ("crack_dy", C.c_double), ("bc_scheme", C.c_int32),
    ]


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = C.CDLL(_LIB)
        P = C.POINTER
        d, i32, i64, u8 = C.c_double, C.c_int32, C.c_int64, C.c_uint8
        lib.orc_create.restype = C.c_void_p
        lib.orc_create.argtypes = [P(_Cfg), P(i32)]
        lib.orc_free.argtypes = [C.c_void_p]
        lib.orc_step.argtypes = [C.c_void_p, i64]
        lib.orc_step.restype = i32
        lib.orc_get_fields.argtypes = [C.c_void_p, P(d), P(d)]
        lib.orc_get_pops.argtypes = [C.c_void_p, P(d)]
        lib.orc_set_state.argtypes = [C.c_void_p, P(d), P(d)]
        lib.orc_get_mask.argtypes = [C.c_void_p, P(u8), P(u8)]
        lib.orc_crack.argtypes = [C.c_void_p, P(d), P(d), P(i64), P(i32)]
        lib.orc_traces.argtypes = [C.c_void_p, P(d), P(d), P(d), P(i32), i64]
        lib.orc_traces.restype = i64
        lib.orc_traces_left.argtypes = [C.c_void_p, P(d), P(d), P(d), P(i32), i64]
        lib.orc_traces_left.restype = i64
        lib.orc_events.argtypes = [C.c_void_p, P(i64), P(i32), P(i32), P(i32), i64]
        lib.orc_events.restype = i64
        lib.orc_constants.argtypes = [C.c_void_p, P(d)]
        lib.orc_check_links.argtypes = [C.c_void_p, d, d, i32, P(i32), P(i32), P(i32), P(i32), i32]
        lib.orc_sif.argtypes = [d, d, d]
        lib.orc_sif.restype = d
        lib.orc_eval_K.argtypes = [C.c_void_p, d]
        lib.orc_eval_K.restype = d
        lib.orc_adjoint_step.argtypes = [C.c_void_p, P(d), P(d)]
        lib.orc_adjoint_step.restype = d
        _lib = lib
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


@dataclass
class OracleConfig:
    """Plate, lattice and crack parameters in lattice units (dh = 1)."""
    nx: int
    ny: int
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
    threads: int = 0
    crack_row: int = -1           # crack line y = crack_row + 1/2; -1 = ny/2 - 1
    both_tips: bool = False       # the left end grows in -x as well
    dirichlet: int = 0            # EDGE_* bits of the edges with a prescribed w
    wD_hist: Optional[np.ndarray] = None   # [n][4] w* of (bottom, top, left, right) per step
    crack_dx: float = 1.0         # growth direction of the right tip (Alg. 1, d); (1, 0) = +x
    crack_dy: float = 0.0
    bc_scheme: int = 0            # BC_LINK (per-link bounce-back) or BC_MACRO (Sec. 3.1)
    _keep: list = field(default_factory=list, repr=False)


class Oracle:
    """Handle on one oracle simulation."""

    def __init__(self, cfg: OracleConfig):
        lib = _load()
        self.cfg = cfg
        c = _Cfg()
        for name in ("nx", "ny", "kappa", "omega", "mu", "rho", "crack_x0", "crack_tip", "growth",
                     "v_rel", "K_C", "r0", "v_max", "k_band", "face_traction", "trace_cap",
                     "threads", "crack_row", "dirichlet", "crack_dx", "crack_dy", "bc_scheme"):
            setattr(c, name, getattr(cfg, name))
        c.periodic = int(cfg.periodic)
        c.has_crack = int(cfg.has_crack)
        c.both_tips = int(cfg.both_tips)
        keep = []
        if cfg.wD_hist is not None:
            wd = np.ascontiguousarray(cfg.wD_hist, dtype=np.float64).reshape(-1, 4)
            keep.append(wd)
            c.wD_hist = _dp(wd)
            c.n_wD = wd.shape[0]
        if cfg.tau_hist is not None:
            t = np.ascontiguousarray(cfg.tau_hist, dtype=np.float64)
            keep.append(t)
            c.tau_hist = _dp(t)
            c.n_hist = t.size
        else:
            c.n_hist = 0
        for name in ("w0", "wdot0"):
            a = getattr(cfg, name)
            if a is not None:
                a = np.ascontiguousarray(a, dtype=np.float64)
                assert a.shape == (cfg.ny, cfg.nx)
                keep.append(a)
                setattr(c, name, _dp(a))
        err = C.c_int32(0)
        h = lib.orc_create(C.byref(c), C.byref(err))
        if not h:
            raise ValueError(f"oracle rejected the configuration (code {err.value})")
        self._h = h
        self._lib = lib

    def close(self):
        if getattr(self, "_h", None):
            self._lib.orc_free(self._h)
            self._h = None

    __del__ = close

    def step(self, n: int = 1):
        rc = self._lib.orc_step(self._h, int(n))
        if rc != 0:
            raise RuntimeError(f"oracle step failed (code {rc})")

    @property
    def shape(self):
        return (self.cfg.ny, self.cfg.nx)

    def fields(self):
        w = np.empty(self.shape)
        wd = np.empty(self.shape)
        self._lib.orc_get_fields(self._h, _dp(w), _dp(wd))
        return w, wd

    def pops(self):
        f = np.empty((5,) + self.shape)
        self._lib.orc_get_pops(self._h, _dp(f))
        return f

    def set_state(self, f: np.ndarray, w: np.ndarray):
        f = np.ascontiguousarray(f, dtype=np.float64)
        w = np.ascontiguousarray(w, dtype=np.float64)
        assert f.shape == (5,) + self.shape and w.shape == self.shape
        self._lib.orc_set_state(self._h, _dp(f), _dp(w))

    def mask(self):
        v = np.empty(self.shape, np.uint8)
        h = np.empty(self.shape, np.uint8)
        P = C.POINTER(C.c_uint8)
        self._lib.orc_get_mask(self._h, v.ctypes.data_as(P), h.ctypes.data_as(P))
        return v, h

    def crack(self):
        tip, v = C.c_double(), C.c_double()
        step, flags = C.c_int64(), C.c_int32()
        self._lib.orc_crack(self._h, C.byref(tip), C.byref(v), C.byref(step), C.byref(flags))
        return {"tip": tip.value, "v": v.value, "step": step.value, "flags": flags.value}

    def traces(self, tip: str = "right"):
        """Per-step K, tip position, speed and flags of the right (or left) tip."""
        n = max(self.cfg.trace_cap, 0)
        K, a, v = np.empty(n), np.empty(n), np.empty(n)
        fl = np.empty(n, np.int32)
        fn = self._lib.orc_traces if tip == "right" else self._lib.orc_traces_left
        m = fn(self._h, _dp(K), _dp(a), _dp(v), fl.ctypes.data_as(C.POINTER(C.c_int32)), n)
        return {"K": K[:m], "tip": a[:m], "v": v[:m], "flags": fl[:m]}

    def events(self):
        n = self._lib.orc_events(self._h, None, None, None, None, 0)
        st = np.empty(n, np.int64)
        i, j, o = (np.empty(n, np.int32) for _ in range(3))
        P = C.POINTER(C.c_int32)
        self._lib.orc_events(self._h, st.ctypes.data_as(C.POINTER(C.c_int64)),
                             i.ctypes.data_as(P), j.ctypes.data_as(P), o.ctypes.data_as(P), n)
        return np.stack([st, i, j, o], axis=1) if n else np.zeros((0, 4), np.int64)

    def constants(self):
        out = np.empty(7)
        self._lib.orc_constants(self._h, _dp(out))
        return dict(zip(("cs", "c", "dt", "lam", "A0", "Ak", "coef"), out))

    def check_links(self, a_prev: float, a_new: float, b_col: int, cap: int = 64):
        P = C.POINTER(C.c_int32)
        bfs = np.zeros((cap, 3), np.int32)
        allv = np.zeros((cap, 3), np.int32)
        nb, na = C.c_int32(), C.c_int32()
        self._lib.orc_check_links(self._h, a_prev, a_new, b_col, bfs.ctypes.data_as(P),
                                  C.byref(nb), allv.ctypes.data_as(P), C.byref(na), cap)
        return bfs[:nb.value], allv[:na.value]

    def eval_K(self, vK: float) -> float:
        """K at the current tip from the current w (r_min for crack speed vK)."""
        return self._lib.orc_eval_K(self._h, vK)

    def adjoint_step(self, lam_f: np.ndarray, lam_w: np.ndarray) -> float:
        """In place: (lam_f, lam_w) <- A^T (lam_f, lam_w); returns d<lam, s'>/d tau."""
        assert lam_f.dtype == np.float64 and lam_f.flags.c_contiguous
        assert lam_w.dtype == np.float64 and lam_w.flags.c_contiguous
        return self._lib.orc_adjoint_step(self._h, _dp(lam_f), _dp(lam_w))


def sensor_traces(cfg: OracleConfig, sensors: np.ndarray, steps: int) -> np.ndarray:
    """w at the sensor sites (i, j) after each of `steps` steps, [steps][n]."""
    s = Oracle(cfg)
    sens = np.asarray(sensors).reshape(-1, 2)
    out = np.empty((steps, len(sens)))
    for n in range(steps):
        s.step(1)
        out[n] = s.fields()[0][sens[:, 1], sens[:, 0]]
    return out


def sensor_adjoint(cfg: OracleConfig, sensors: np.ndarray, g: np.ndarray):
    """Discrete adjoint of a run of T = len(g) steps for a loss L of the
    sensor traces with dL/dw_s(after step n) = g[n, s] (the crack must stay
    where cfg puts it: the adjoint applies the initial mask to every step).

    lambda_T = (0, dL/dw_T); lambda_{n} = A^T lambda_{n+1} + (0, dL/dw_n);
    dL/dtau_n = b^T lambda_{n+1} (returned by each adjoint step).  The
    initial state f_0 = f_eq(w_0, wdot_0), i.e. f^0 = wdot_0 - A0 w_0 and
    f^k = Ak w_0, then gives dL/dwdot_0 = lambda_f^0 and
    dL/dw_0 = lambda_w - A0 lambda_f^0 + Ak (lambda_f^1 + ... + lambda_f^4).
    Returns (dL/dtau [T], dL/dwdot_0 [ny][nx], dL/dw_0 [ny][nx])."""
    s = Oracle(cfg)
    k = s.constants()
    sens = np.asarray(sensors).reshape(-1, 2)
    g = np.asarray(g, dtype=np.float64)
    T = g.shape[0]
    lam_f = np.zeros((5, cfg.ny, cfg.nx))
    lam_w = np.zeros((cfg.ny, cfg.nx))
    dtau = np.empty(T)
    for n in range(T, 0, -1):
        lam_w[sens[:, 1], sens[:, 0]] += g[n - 1]
        dtau[n - 1] = s.adjoint_step(lam_f, lam_w)
    dwd0 = lam_f[0].copy()
    dw0 = lam_w + (-k["A0"] * lam_f[0] + k["Ak"] * (((lam_f[1] + lam_f[2]) + lam_f[3]) + lam_f[4]))
    return dtau, dwd0, dw0


def sif(delta: float, r: float, mu: float = 1.0) -> float:
    """eq. (sif): K = delta (mu/4) sqrt(2 pi / r)."""
    return _load().orc_sif(delta, r, mu)
