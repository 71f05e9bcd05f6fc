"""MI355X (gfx950) lattice Boltzmann solver for antiplane shear with dynamic
mode III cracks (arXiv:2206.12412), behind the C-ABI of include/lbm.h."""
from .lbm import (BC_PERIODIC, Batch, BC_WALLS, EXPORTS, FLAG_GREW, FLAG_K_UNDEF, FLAG_WALL, GROW_NONE,
                  GROW_PRESCRIBED, GROW_SIF, LIB_PATH, STORAGE, Config, CrackInfo, LBMError, Solver,
                  load_library, plan_tail, state_bytes, sweep_cost)

__all__ = ["BC_PERIODIC", "Batch", "BC_WALLS", "EXPORTS", "FLAG_GREW", "FLAG_K_UNDEF", "FLAG_WALL",
           "GROW_NONE", "GROW_PRESCRIBED", "GROW_SIF", "LIB_PATH", "STORAGE", "Config", "CrackInfo",
           "LBMError", "Solver", "load_library", "plan_tail", "state_bytes", "sweep_cost"]
