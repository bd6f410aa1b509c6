"""The C-ABI library loads, exports every symbol its header declares, and
rejects bad input on the host (no GPU needed)."""
import os
import re

import numpy as np
import pytest

from paper_2602_16312_amd import _ffi as F
from paper_2602_16312_amd import api, problem
from workloads import make_problem

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    txt = open(os.path.join(ROOT, "include", "dgmg.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dgmg_[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = F.lib()
    syms = declared_symbols()
    assert len(syms) >= 14
    for s in syms:
        assert hasattr(lib, s), s
    assert sorted(F.EXPORTS) == syms


def test_bad_inputs_are_rejected_on_host():
    pr = make_problem("c1", n=8)
    with pytest.raises(F.DGMGError) as e:
        api.build_hierarchy(pr["xyz"], pr["cell_vtx"], 0)
    assert e.value.code == -1
    bad = pr["cell_vtx"].copy()
    bad[0, 0] = 10 ** 6
    with pytest.raises(F.DGMGError):
        api.build_hierarchy(pr["xyz"], bad, 1)
    # bins that do not nest
    with pytest.raises(F.DGMGError):
        api.build_hierarchy(pr["xyz"], pr["cell_vtx"], 3, grid_bins=[[1, 1, 1], [3, 3, 1], [2, 2, 1]])
    h = api.build_hierarchy(pr["xyz"], pr["cell_vtx"], 2, grid_bins=[[1, 1, 1], [2, 2, 1]])
    with pytest.raises(F.DGMGError):
        api.setup_levels(h, 1, pr["D_cell"], 1.0, 1.0, 0.01, "fhn", [1.0, 2.0], device_setup=False)
    with pytest.raises(F.DGMGError) as e:
        api.setup_levels(h, 5, pr["D_cell"], 1.0, 1.0, 0.01, "fhn", pr["params"], device_setup=False)
    assert e.value.code == -6
    # inverted cell -> non-positive Jacobian
    inv = pr["cell_vtx"].copy()
    inv[3] = inv[3][[1, 0, 3, 2]]
    with pytest.raises(F.DGMGError):
        h2 = api.build_hierarchy(pr["xyz"], inv, 1)
        api.setup_levels(h2, 1, pr["D_cell"], 1.0, 1.0, 0.01, "fhn", pr["params"],
                         device_setup=False)
    # solve calls on a host-only solver fail cleanly
    s = api.setup_levels(h, 1, pr["D_cell"], 1.0, 1.0, 0.01, "fhn", pr["params"],
                         device_setup=False)
    rc = F.lib().dgmg_vcycle(s.handle, None, None, None)
    assert rc == -1


def test_indefinite_coarse_operator_is_reported():
    """A negative penalty makes the one-level operator indefinite; the
    coarse Cholesky reports ENOTSPD."""
    pr = make_problem("c1", n=4)
    h = api.build_hierarchy(pr["xyz"], pr["cell_vtx"], 1)
    with pytest.raises(F.DGMGError) as e:
        api.setup_levels(h, 1, pr["D_cell"] * 1e5, 1.0, 1.0, 1e3, "fhn", pr["params"],
                         penalty=("fixed", -50.0), device_setup=False)
    assert e.value.code == -2


PAIRS = [("dgmg_mesh", "Mesh"), ("dgmg_agglo_opts", "AggloOpts"), ("dgmg_disc", "Disc"),
         ("dgmg_physics", "Physics"), ("dgmg_allocator", "Allocator"), ("dgmg_mg_opts", "MGOpts"),
         ("dgmg_solver_info", "SolverInfo"), ("dgmg_pcg_opts", "PCGOpts"),
         ("dgmg_pcg_stats", "PCGStats"), ("dgmg_state", "State")]


def test_binding_structs_match_the_header(tmp_path):
    """Size and every field offset of the binding's structures against the C
    compiler's layout of the header's structures."""
    import subprocess
    import ctypes as C
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "dgmg.h"', "int main(void) {"]
    for cname, pyname in PAIRS:
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in getattr(F, pyname)._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for ln in out:
        if ln:
            cname, key, val = ln.split()
            got[(cname, key)] = int(val)
    for cname, pyname in PAIRS:
        cls = getattr(F, pyname)
        assert got[(cname, "size")] == C.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)
