"""Writes the stored oracle values of tests/golden/ (calls only the oracle and
the seeded input generators).

The paper prints no numerical values for a worked example (its results are
figures), so these files are drift guards of the oracle, not pins of it: the
pins are the closed forms, invariants, brute-force cases and the Mie series of
the oracle tests.  A change of the oracle's arithmetic that moves one of these
values must be justified by the passage of the paper it follows, and the file
rewritten by this script in the same commit.

Usage:  python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

# 120-edge sphere (icosphere level 1, radius 1 m), c dt = 0.15 m, one
# modulated-Gaussian plane wave (f0 = bandwidth = 0.1 per metre), 200 steps
CASE = {"mesh": "icosphere(1)", "c_dt_m": 0.15, "f0_per_m": 0.1, "n_steps": 200,
        "sample_edges": [0, 17, 59, 119], "sample_steps": [10, 25, 50, 100, 199]}


def compute():
    from oracle import operators as O, excitation as E, mot
    from workloads import meshes, waves
    xyz, tri = meshes.icosphere(1)
    asm = O.Assembly(xyz, tri, CASE["c_dt_m"])
    asm.build()
    f0 = CASE["f0_per_m"]
    w = waves.Wave((0.0, 0.0, -1.0), (1.0, 0.0, 0.0), 1.0, waves.mod_gauss_t0(f0, asm.D), 0, 0.0, f0, f0)
    r = E.rhs(asm, w, CASE["n_steps"])
    y = mot.march(asm.T, r)
    j = mot.currents(asm.proj.PLH, asm.proj.PS, asm.dtn, y)
    T = np.asarray(asm.T)
    return {
        "ne": int(T.shape[1]),
        "K": int(T.shape[0] - 1),
        "block_frobenius": [float(np.linalg.norm(T[k])) for k in range(T.shape[0])],
        "cond1_T0": float(mot.condition_1(T[0])),
        "current": [[float(j[i, e]) for e in CASE["sample_edges"]] for i in CASE["sample_steps"]],
        "current_peak": float(np.abs(j).max()),
    }


def main():
    out = {"case": CASE, "values": compute()}
    with open(os.path.join(HERE, "oracle_sphere120.json"), "w") as f:
        json.dump(out, f, indent=1)
        f.write("\n")


if __name__ == "__main__":
    main()
