"""Writes tests/golden/c5_adjoint.json with the FP64 oracle only:
sensor targets of the 256x256 Q2 Aliev-Panfilov adjoint problem (forward run at
the seeded lognormal scalings s_true, 50 steps), and at s = 1 the loss, the
gradient projected on 16 seeded unit directions (seed 2607) and the gradient at
64 seeded cells (seed 2608).  Run: python tests/golden/make_c5_golden.py"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from workloads import make_problem  # noqa: E402
from oracle.adjoint import AdjointProblem, make_targets  # noqa: E402

STEPS, TOL, CK = 50, 1e-13, 10


def main():
    t0 = time.time()
    pr = make_problem("c5")
    targets = make_targets(pr, STEPS, pr["s_true"], tol=TOL)
    print("targets", time.time() - t0, flush=True)
    ap = AdjointProblem(pr, targets, STEPS, tol=TOL, checkpoint=CK)
    s = np.ones(pr["n_cells"])
    loss, grad = ap.gradient(s)
    print("gradient", time.time() - t0, flush=True)
    rng = np.random.default_rng(2607)
    dirs = []
    for _ in range(16):
        d = rng.standard_normal(pr["n_cells"])
        dirs.append(float(grad @ (d / np.linalg.norm(d))))
    cells = np.random.default_rng(2608).choice(pr["n_cells"], 64, replace=False)
    out = dict(source="FP64 oracle (oracle/adjoint.py), tol 1e-13, checkpoints every 10 steps",
               steps=STEPS, tol=TOL, targets=targets.tolist(), loss=loss,
               grad_dot_dirs=dirs, dir_seed=2607, sample_cells=cells.tolist(),
               grad_at_cells=grad[cells].tolist(), grad_norm=float(np.linalg.norm(grad)))
    json.dump(out, open(os.path.join(os.path.dirname(os.path.abspath(__file__)),
                                     "c5_adjoint.json"), "w"))
    print("done", time.time() - t0)


if __name__ == "__main__":
    main()
