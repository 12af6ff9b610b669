"""Writes oracle_c1_100steps.npz: the FP64 oracle's state after the 100 steps
of the tiny plane-wave workload (4^3 cubes x 6 = 384 tets, periodic, N = 2,
planar P wave of strain amplitude 1e-6, no damage; CFL 0.5).

Only the oracle and the seeded input generator run here; the GPU parity test
of the same workload compares the library with this state.

    python tests/golden/make_oracle_c1.py
"""
import os
import sys

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle.step import from_workload  # noqa: E402
from workloads import make_workload  # noqa: E402

OUT = os.path.join(HERE, "oracle_c1_100steps.npz")


def main():
    torch.set_num_threads(os.cpu_count() or 1)
    w = make_workload("c1")
    S = from_workload(w)
    U0 = S.project(w.ic)
    U = S.run(U0, w.nsteps)
    np.savez_compressed(OUT, U0=U0.numpy(), U=U.numpy(), nsteps=w.nsteps, dt=w.dt,
                        n=w.mesh["n"], N=w.N)
    print(OUT)


if __name__ == "__main__":
    main()
