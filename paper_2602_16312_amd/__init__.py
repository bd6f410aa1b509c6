"""MI355X-native agglomerated-multigrid PCG for the SIPDG monodomain system
(arXiv 2602.16312): a C-ABI library of gfx950 HIP kernels (libdgmg.so) and
its thin Python binding."""
from .api import (build_hierarchy, setup_levels, pcg_solve, ionic_step, time_step,
                  apply, vcycle, mass_apply, State, Solver, Hierarchy)

__all__ = ["build_hierarchy", "setup_levels", "pcg_solve", "ionic_step", "time_step",
           "apply", "vcycle", "mass_apply", "State", "Solver", "Hierarchy"]
