"""Writes c4_penalty_pair.json: on the 1.0M-hex jittered shell with the
paper's penalty coefficient (factor 1), the pair of face-neighbour cells whose
16 x 16 principal submatrix of A_0 = c_M M + A has the most negative
eigenvalue (a principal submatrix of a positive definite matrix is positive
definite, so one negative eigenvalue proves A_0 indefinite).  Calls only the
oracle and the seeded input generators; takes a few minutes.

Usage: python tests/golden/make_c4_penalty_pair.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from workloads import make_problem  # noqa: E402
from oracle.assemble import cell_matrices, face_matrices, interior_faces, unpack_sym  # noqa: E402


def main():
    pr = make_problem("c4", penalty=("paper", 1.0))
    xyz, cells, p = pr["xyz"], pr["cell_vtx"], pr["p"]
    d, b = 3, pr["b"]
    X = xyz[cells]
    Dm = unpack_sym(pr["D_cell"], d)
    Mk, Sk, vol = cell_matrices(X, Dm, p)
    cM = 1.5 * pr["chi"] * pr["Cm"] / pr["dt"]
    diag = Sk + cM * Mk                         # becomes the diagonal blocks of A_0
    plus, minus, axis = interior_faces(cells, d)
    off = np.zeros((len(plus), b, b))           # A_0[plus rows, minus columns]
    for k in range(d):
        sel = np.flatnonzero(axis == k)
        for s0 in range(0, len(sel), 200000):
            s = sel[s0:s0 + 200000]
            Af = face_matrices(X[plus[s]], X[minus[s]], Dm[plus[s]], Dm[minus[s]], k,
                               vol[plus[s]], vol[minus[s]], p, pr["penalty"])
            np.add.at(diag, plus[s], Af[:, :b, :b])
            np.add.at(diag, minus[s], Af[:, b:, b:])
            off[s] = Af[:, :b, b:]
    best, bf = np.inf, -1
    for s0 in range(0, len(plus), 200000):
        sl = slice(s0, s0 + 200000)
        P = np.zeros((len(plus[sl]), 2 * b, 2 * b))
        P[:, :b, :b] = diag[plus[sl]]
        P[:, b:, b:] = diag[minus[sl]]
        P[:, :b, b:] = off[sl]
        P[:, b:, :b] = off[sl].transpose(0, 2, 1)
        ev = np.linalg.eigvalsh(P)[:, 0] / np.abs(P).max(axis=(1, 2))
        j = int(np.argmin(ev))
        if ev[j] < best:
            best, bf = float(ev[j]), s0 + j
    out = {"mesh": "c4 shell, h 0.0147, jitter 0.15 h, seed 2603", "penalty_factor": 1.0,
           "cells": [int(plus[bf]), int(minus[bf])], "axis": int(axis[bf]),
           "min_eigenvalue_over_max_entry": best}
    with open(os.path.join(HERE, "c4_penalty_pair.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(out)


if __name__ == "__main__":
    main()
