"""torch.autograd bridge: the sensor traces of a plate run as a differentiable
function of the traction history and of the initial velocity field.

Forward: one solver run of T = len(tau_hist) steps (tau_hist[n] loads step n)
recording w at the sensor sites after every step.  Backward: the library's
discrete adjoint (lbm_adjoint_run) through the same T steps, fed with the
incoming gradient of the traces.  The solver of the forward run is kept until
backward: its recorded cut events give the severed links of every step, and
the adjoint sweep reads no other forward state, so no step is recomputed.
"""
from __future__ import annotations

import dataclasses

import torch

from .lbm import Config, Solver


class SensorRun(torch.autograd.Function):
    """traces[n, s] = w at sensor s after step n."""

    @staticmethod
    def forward(ctx, tau_hist: torch.Tensor, wdot0: torch.Tensor, cfg: Config, device: str):
        T = int(tau_hist.numel())
        if T < 1:
            raise ValueError("tau_hist needs at least one step")
        c = dataclasses.replace(cfg, tau_hist=tau_hist.detach().double().cpu().numpy(),
                                wdot0=wdot0.detach().double().cpu().numpy(), trace_cap=T)
        s = Solver(c, device=device)
        s.step(T)
        traces = s.sensor_traces(device=True)
        ctx.solver = s
        ctx.meta = (tau_hist.device, tau_hist.dtype, wdot0.device, wdot0.dtype)
        return traces

    @staticmethod
    def backward(ctx, g: torch.Tensor):
        s = ctx.solver
        dtau, dwd0, _ = s.adjoint(g)
        ctx.solver = None
        s.close()
        tdev, tdt, wdev, wdt = ctx.meta
        return (torch.from_numpy(dtau).to(device=tdev, dtype=tdt), dwd0.to(device=wdev, dtype=wdt),
                None, None)


def sensor_run(tau_hist: torch.Tensor, wdot0: torch.Tensor, cfg: Config,
               device: str = "cuda") -> torch.Tensor:
    """Differentiable sensor traces [T][n_sensors] (float64 on `device`) of the
    plate cfg (cfg.sensors set; cfg.tau_hist, cfg.wdot0 and cfg.trace_cap are
    replaced by the arguments)."""
    return SensorRun.apply(tau_hist, wdot0, cfg, device)
