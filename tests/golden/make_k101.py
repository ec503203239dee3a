"""Writes tests/golden/oracle_sphere1920_k101.json: the oracle's march of the
1920-edge sphere at the lag count of the 7680-edge workload (K = 101), sampled
(calls only the oracle and the seeded input generators; about three minutes
of CPU).

The oracle's own values, stored because its assembly at this size takes
minutes: the GPU parity test at K = 101 (tests/test_gpu_k101.py) compares
every form of the library against them.  Like oracle_sphere120.json they pin
nothing about the oracle; a change of the oracle's arithmetic that moves them
must be justified by the passage of the paper it follows, and the file
rewritten by this script in the same commit.

Stored: the current j_i (eq. post_processing) at 24 edges every 4th step, and
the 2-norm of the whole current vector at every step.

Usage:  python tests/golden/make_k101.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

# icosphere level 3 (1920 edges), radius 1 m, c dt = 0.02 m (K = 101), one
# x-polarised wave along -z, modulated Gaussian at 150 MHz (centre and
# bandwidth, t0 = 6 sigma + 1 m), 600 steps: the pulse peaks near step 150
CASE = {"mesh": "icosphere(3)", "c_dt_m": 0.02, "f0_hz": 150e6, "t0_diameter_m": 2.0, "n_steps": 600,
        "sample_edges": list(range(0, 1920, 80)), "sample_every": 4}


def wave():
    from workloads import waves
    f0 = waves.hz_to_per_m(CASE["f0_hz"])
    return waves.Wave((0.0, 0.0, -1.0), (1.0, 0.0, 0.0), 1.0, waves.mod_gauss_t0(f0, CASE["t0_diameter_m"]), 0, 0.0,
                      f0, f0)


def compute():
    from oracle import operators as O, excitation as E, mot
    from workloads import meshes
    xyz, tri = meshes.icosphere(3)
    asm = O.Assembly(xyz, tri, CASE["c_dt_m"])
    asm.build()
    r = E.rhs(asm, wave(), CASE["n_steps"])
    j = mot.currents(asm.proj.PLH, asm.proj.PS, asm.dtn, mot.march(asm.T, r))
    steps = list(range(0, CASE["n_steps"], CASE["sample_every"]))
    return {
        "ne": int(j.shape[1]),
        "K": int(asm.K),
        "sample_steps": steps,
        "current": [[float(j[i, e]) for e in CASE["sample_edges"]] for i in steps],
        "current_norm": [float(v) for v in np.linalg.norm(j, axis=1)],
    }


def main():
    out = {"case": CASE, "values": compute()}
    with open(os.path.join(HERE, "oracle_sphere1920_k101.json"), "w") as f:
        json.dump(out, f)
        f.write("\n")


if __name__ == "__main__":
    main()
