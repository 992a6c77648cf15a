"""Write the oracle regression fixtures (oracle_*.npz) in this folder.

Calls only the FP64 oracle and the seeded input generators; no value here
comes from the GPU path.  Run from the repository root:
    python tests/golden/make_golden.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2204_08834_amd import inputs  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))

CASES = [
    ("oracle_walls_8x6x5.npz", dict(nx=8, ny=6, nz=5, L=(1.0, 0.75, 0.5), bc=1, seed=21)),
    ("oracle_periodic_6x8x12.npz", dict(nx=6, ny=8, nz=12, L=(2.0, 2.0, 3.0), bc=0, seed=22)),
    ("oracle_walls_16x16x8.npz", dict(nx=16, ny=16, nz=8, L=(2.0, 2.0, 1.0), bc=1, seed=23)),
]


def main():
    for fname, c in CASES:
        nx, ny, nz = c["nx"], c["ny"], c["nz"]
        Lx, Ly, Lz = c["L"]
        f = inputs.uniform_velocity_rhs(nx, ny, nz, Lx, Ly, Lz, c["bc"], c["seed"])
        dx, dy, dz = Lx / nx, Ly / ny, Lz / nz
        p = oracle.solve(f, dx, dy, dz, c["bc"])
        np.savez(os.path.join(HERE, fname), shape=np.array([nx, ny, nz]),
                 spacing=np.array([dx, dy, dz]), bc_z=np.array(c["bc"]), f=f, p=p)
        print("wrote", fname)


if __name__ == "__main__":
    main()
