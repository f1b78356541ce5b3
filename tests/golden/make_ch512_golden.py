"""Writes tests/golden/ch3d_512_p{2,4,6}_100.txt: the FP64 oracle's state of
the precision-study workload after 100 steps, at sampled sites.

Workload: 3D Cahn-Hilliard (Eq. model-b) on a 512^3 periodic grid, dx = 1,
dt = 0.005, c1 = c2 = 1, c0 = U[-0.05, 0.05] from the counter-based
generator with seed 404, stencil orders 2, 4 and 6.  Only oracle/ and synth/
are called.  Each file holds the exact (correctly rounded) sums of the
initial and final states and the final value at 2048 sites drawn with a
fixed numpy seed plus the eight grid corners.

Run from the repository root: python tests/golden/make_ch512_golden.py
(about half an hour on eight cores).
"""
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402
import synth  # noqa: E402

N, SEED, DT, STEPS = 512, 404, 0.005, 100
PARAMS = [1.0, 1.0]


def sample_sites(n=N, count=2048, seed=4040):
    rng = np.random.default_rng(seed)
    idx = rng.integers(0, n, size=(count, 3))
    corners = np.array([[z, y, x] for z in (0, n - 1) for y in (0, n - 1) for x in (0, n - 1)])
    return np.concatenate([corners, idx])


def main(orders=(2, 4, 6)):
    oracle.build()
    shape = (N, N, N)
    f0 = synth.initial_fields(2, shape, SEED, synth.IC_UNIFORM, (-0.05, 0.05))
    m0 = oracle.exact_sum(f0[0])
    sites = sample_sites()
    for order in orders:
        t = time.time()
        out = oracle.run(2, f0, 3, 1.0, DT, order, PARAMS, STEPS)[0]
        m1 = oracle.exact_sum(out)
        path = os.path.join(HERE, "ch3d_512_p%d_100.txt" % order)
        with open(path, "w") as fh:
            fh.write("# 3D Cahn-Hilliard (Eq. model-b), 512^3 periodic, dx 1, dt %.3f, c1 = c2 = 1,\n" % DT)
            fh.write("# c0 = U[-0.05, 0.05] seed %d, order %d, FP64 oracle after %d steps.\n" % (SEED, order, STEPS))
            fh.write("# Written by tests/golden/make_ch512_golden.py (oracle/ and synth/ only).\n")
            fh.write("mass0: %.17g\n" % m0)
            fh.write("mass: %.17g\n" % m1)
            fh.write("# z y x value\n")
            for (z, y, x) in sites:
                fh.write("%d %d %d %.17g\n" % (z, y, x, out[z, y, x]))
        print("order %d: %.0f s" % (order, time.time() - t), flush=True)


if __name__ == "__main__":
    main(tuple(int(a) for a in sys.argv[1:]) or (2, 4, 6))
