"""Convenience set-up of a solver from a problem description (a mapping with
the mesh arrays and physical/solver parameters, as produced by the seeded
workload generators).  Marshalling only: all work happens in libdgmg.so."""
import numpy as np

from . import api


def grid_bins(n, dim, factors):
    """Bins per axis of each grid-grouped level for an n^dim structured mesh."""
    bins = [[1, 1, 1]]
    m = n
    for f in factors:
        m //= f
        bins.append([m] * dim + [1] * (3 - dim))
    return bins


def build(prob, precision="fp64", lam_override=None, cell_scale=None,
          device_setup=True, bdf=2, **mg):
    """(hierarchy, solver) for a problem mapping."""
    agglo = prob.get("agglo", ("grid",))
    if agglo[0] == "rtree_str":
        h = api.build_hierarchy(prob["xyz"], prob["cell_vtx"], agglo[2], method="rtree_str",
                                fanout=agglo[1])
    else:
        levels = 1 + len(prob["group"])
        h = api.build_hierarchy(prob["xyz"], prob["cell_vtx"], levels, method="grid",
                                grid_bins=grid_bins(prob["n"], prob["dim"], prob["group"]))
    s = api.setup_levels(h, prob["p"], prob["D_cell"], prob["chi"], prob["Cm"],
                         prob["dt"], prob["model"], np.asarray(prob["params"], float),
                         penalty=prob["penalty"], bdf=bdf, cell_scale=cell_scale,
                         precision=precision, lam_override=lam_override,
                         device_setup=device_setup, **mg)
    return h, s
