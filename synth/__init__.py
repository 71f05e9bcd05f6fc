"""Seeded synthetic workloads shared by the tests, the benchmark and the smoke check.

This module only states plate sizes, loads, crack parameters and seeds, and draws
the random numbers the workloads need (initial-velocity noise, batched plate
parameters, sensor positions, probe directions).  It holds none of the lattice
Boltzmann arithmetic and imports neither the oracle nor the HIP library; both
sides receive the same arrays from here.

Units are lattice units: dh = 1, mu = rho = 1 (so c_s = 1), kappa = c / c_s = 2.
An edge crack of ``ell`` sites runs from the left edge x = -1/2 along the
mid-line y = ny/2 - 1/2 to the tip a0 = ell - 1/2.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field, replace
from typing import Optional

import numpy as np

GROW_NONE, GROW_PRESCRIBED, GROW_SIF = 0, 1, 2


@dataclass
class Plate:
    """One plate: geometry, load, crack rule and run length."""
    name: str
    nx: int
    ny: int
    ell: int                      # initial edge-crack length in sites
    tau: float                    # sigma_yz applied on the top (+) and bottom (-) edges
    steps: int
    growth: int = GROW_NONE
    v_rel: float = 0.0            # prescribed crack speed / c_s
    K_C: float = 0.0              # critical SIF (K criterion)
    r0: float = 2.0               # r_min at v = 0 (eq. r(v)), in sites
    v_max: float = 0.85           # maximum crack speed of the tanh law
    kappa: float = 2.0
    mu: float = 1.0
    rho: float = 1.0
    noise_sigma: float = 0.0      # std of the initial-velocity noise
    seed: Optional[int] = None
    tau_hist: Optional[np.ndarray] = field(default=None, repr=False)

    @property
    def crack_x0(self) -> float:
        return -0.5

    @property
    def crack_tip(self) -> float:
        return self.ell - 0.5

    @property
    def sites(self) -> int:
        return self.nx * self.ny

    def traction_history(self) -> np.ndarray:
        """sigma_yz per step; a step load is a one-entry history."""
        if self.tau_hist is not None:
            return np.asarray(self.tau_hist, dtype=np.float64)
        return np.array([self.tau], dtype=np.float64)

    def wdot0(self) -> Optional[np.ndarray]:
        """Initial velocity field [ny][nx] (FP64), or None for a plate at rest."""
        if self.noise_sigma == 0.0:
            return None
        rng = np.random.default_rng(self.seed)
        return rng.normal(0.0, self.noise_sigma, size=(self.ny, self.nx))

    def scaled(self, nx: int, ny: int, ell: int, steps: int, **kw) -> "Plate":
        return replace(self, nx=nx, ny=ny, ell=ell, steps=steps, **kw)


def k_static_edge(tau: float, ell: float) -> float:
    """Static K_III of an edge crack of length ell under remote antiplane shear tau.

    By mirror symmetry about the traction-free edge this is the Griffith crack of
    length 2 ell, K = tau sqrt(pi ell); used to set K_C = 1.5 K_static.
    """
    return tau * math.sqrt(math.pi * ell)


# --- the five workloads ----------------------------------------------------------

def config_plain_fp64() -> Plate:
    """256 x 128 plate, 64-site edge crack, step traction 1e-3, crack driven at
    0.3 c_s for 2000 steps, FP64 (the tip reaches the far edge at step 1279)."""
    return Plate("plain-fp64-256x128", 256, 128, 64, 1e-3, 2000,
                 growth=GROW_PRESCRIBED, v_rel=0.3)


def config_sif_fp32() -> Plate:
    """4096 x 2048 plate, 1024-site edge crack, step traction 1e-3, growth by the
    K criterion with K_C = 1.5 K_static, 20000 steps, initial-velocity noise
    N(0, 1e-6^2) drawn from seed 0."""
    tau, ell = 1e-3, 1024
    return Plate("sif-fp32-4096x2048", 4096, 2048, ell, tau, 20000, growth=GROW_SIF,
                 K_C=1.5 * k_static_edge(tau, ell), noise_sigma=1e-6, seed=0)


def config_precision() -> Plate:
    """16384 x 8192 plate (134M sites), 4096-site edge crack, crack driven at
    0.5 c_s, 10000 steps; run with each storage type."""
    return Plate("precision-16384x8192", 16384, 8192, 4096, 1e-3, 10000,
                 growth=GROW_PRESCRIBED, v_rel=0.5)


BATCH_SIZES = ((512, 512), (1024, 512), (1024, 1024), (2048, 1024))


def config_batched(n_plates: int = 64, seed: int = 1, steps: int = 5000) -> list:
    """64 independent plates: sizes uniform over BATCH_SIZES (nx x ny), crack
    length nx/4, tau ~ U[5e-4, 2e-3], speed ~ U[0.1, 0.7] c_s; odd-indexed
    plates grow by the K criterion with K_C = 1.5 K_static instead."""
    rng = np.random.default_rng(seed)
    idx = rng.integers(0, len(BATCH_SIZES), size=n_plates)
    taus = rng.uniform(5e-4, 2e-3, size=n_plates)
    vs = rng.uniform(0.1, 0.7, size=n_plates)
    plates = []
    for k in range(n_plates):
        nx, ny = BATCH_SIZES[idx[k]]
        ell = nx // 4
        if k % 2 == 1:
            p = Plate(f"batch{k}", nx, ny, ell, float(taus[k]), steps, growth=GROW_SIF,
                      K_C=1.5 * k_static_edge(float(taus[k]), ell))
        else:
            p = Plate(f"batch{k}", nx, ny, ell, float(taus[k]), steps, growth=GROW_PRESCRIBED,
                      v_rel=float(vs[k]))
        plates.append(p)
    return plates


def config_adjoint() -> Plate:
    """2048 x 1024 plate, stationary 512-site edge crack, 5000 steps, base
    traction 1e-3 (the gradient is taken at this point)."""
    return Plate("adjoint-2048x1024", 2048, 1024, 512, 1e-3, 5000)


def adjoint_target_history(steps: int, tau0: float = 1e-3, amp: float = 0.1,
                           period: float = 800.0) -> np.ndarray:
    """Traction history of the target run: tau0 (1 + amp sin(2 pi n / period))."""
    n = np.arange(steps, dtype=np.float64)
    return tau0 * (1.0 + amp * np.sin(2.0 * np.pi * n / period))


def adjoint_sensors(nx: int, ny: int, count: int = 32, seed: int = 0) -> np.ndarray:
    """Distinct interior sensor sites (i, j), away from the walls and the crack rows."""
    rng = np.random.default_rng(seed)
    j0 = ny // 2 - 1
    out = set()
    while len(out) < count:
        i = int(rng.integers(2, nx - 2))
        j = int(rng.integers(2, ny - 2))
        if abs(j - j0) <= 2 or abs(j - (j0 + 1)) <= 2:
            continue
        out.add((i, j))
    return np.array(sorted(out), dtype=np.int32)


def adjoint_directions(n_tau: int, shape: tuple, count: int = 16, seed: int = 1):
    """Random unit directions in the joint (traction history, initial velocity) space."""
    rng = np.random.default_rng(seed)
    dirs = []
    for _ in range(count):
        dt_ = rng.normal(size=n_tau)
        dw = rng.normal(size=shape)
        nrm = math.sqrt(float(np.dot(dt_, dt_)) + float(np.sum(dw * dw)))
        dirs.append((dt_ / nrm, dw / nrm))
    return dirs


def two_tip_demo(steps: int = 4000, L: int = 64) -> dict:
    """The K-criterion example of Sec. 5.2: a plate 8L wide and 3L high
    (dh = L/64: 512 x 192 sites), a centre crack of length L on the line 2L
    above the lower edge (y = 2L - 1/2 in site coordinates, between rows 127
    and 128) that can grow at both tips, K_C = 0.0055 mu sqrt(L), r0 = 0.03 L,
    v_max = 0.85; the lower edge held at w = 0, the upper edge displaced by
    a half sine w = 0.01 L sin(pi t / 8) for t < 8 L / c_s (t in L / c_s), the
    lateral edges and the crack faces traction-free.  With c_s = 1 and
    dt = 1/2 a step is 1/128 of L / c_s; step n uses t = n dt."""
    nx, ny = 8 * L, 3 * L
    n = np.arange(steps, dtype=np.float64)
    t = n * 0.5 / L                       # in units of L / c_s
    wD = np.zeros((steps, 4))
    wD[:, 1] = np.where(t < 8.0, 0.01 * L * np.sin(np.pi * t / 8.0), 0.0)
    centre = nx / 2 - 0.5
    return dict(nx=nx, ny=ny, has_crack=True, crack_row=2 * L - 1, crack_x0=centre - L / 2,
                crack_tip=centre + L / 2, both_tips=True, growth=GROW_SIF,
                K_C=0.0055 * np.sqrt(L), r0=0.03 * L, v_max=0.85, dirichlet=1 | 2,
                wD_hist=wD, trace_cap=steps)


# r_min / dh chosen per speed for the steady-growth strip (the second column
# of the table of Sec. 5.1)
STRIP_R_MIN = {0.2: 1.5, 0.4: 2.25, 0.6: 4.0, 0.8: 8.0}


def mandal_strip(v: float, L: int = 16, w0: float = 0.2, t0: float = 10.0,
                 t_quasi: float = 20.0) -> dict:
    """The steady-growth strip of Sec. 5.1 (lengths in units of L, times in
    L / c_s): a strip of height 2L (dh = L / 16: 32 rows, walls half-way past
    the edge rows), its upper and lower edges held at +-w0/2 times the ramp
    sin^2(pi t / (2 t0)) up to t0 and 1 after it, lateral edges and crack
    faces traction-free; an edge crack of length L/2 on the mid-line, driven
    at the prescribed speed v from the first step; r_min taken from the
    table (r0 = r_min (1 - v)).  The run ends at t_f = t0 + t_quasi; the
    right edge b = 0.5 + v t_f + 2.5 (beyond v c_s t_f + 2L).  Returns the
    Config keyword arguments, the 300 sampled steps of [t_f - 15, t_f] and
    the steady K of eq. (sif-mandal) in lattice units.

    Lattice units: mu = 1, dh = 1, c_s = 1, dt = 1/2, so one L / c_s is 2 L
    steps; w0 is in units of L (w0 L in lattice units), and K (stress times
    sqrt(length)) is sqrt(L) times its value in units where L = 1."""
    t_f = t0 + t_quasi
    steps = int(round(t_f * 2 * L))
    nx = int(math.ceil((0.5 + v * t_f + 2.5) * L))
    n = np.arange(steps, dtype=np.float64)
    t = n * 0.5 / L
    ramp = np.where(t < t0, np.sin(0.5 * np.pi * t / t0) ** 2, 1.0)
    wD = np.zeros((steps, 4))
    wD[:, 0] = -0.5 * w0 * L * ramp   # bottom edge y = -L
    wD[:, 1] = 0.5 * w0 * L * ramp    # top edge y = +L
    r_min = STRIP_R_MIN[v]
    beta = math.sqrt(1.0 - v * v)
    K_theo = w0 * math.sqrt(2.0 * beta / (2.0 * beta + 1.0)) * math.sqrt(L)
    sample = np.unique(np.round(np.linspace(steps - 1 - 15 * 2 * L, steps - 1, 300)).astype(int))
    kw = dict(nx=nx, ny=2 * L, has_crack=True, crack_x0=-0.5, crack_tip=0.5 * L - 0.5,
              growth=GROW_PRESCRIBED, v_rel=v, r0=r_min * (1.0 - v), dirichlet=1 | 2,
              wD_hist=wD, trace_cap=steps)
    return {"config": kw, "steps": steps, "sample_steps": sample, "K_theo": K_theo,
            "t_f": t_f, "r_min": r_min}
