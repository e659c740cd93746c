"""Writes the golden regression records under tests/golden/ by calling only the
CPU oracle.  Run from the repository root:  python tests/golden/make_golden.py

The inputs are small, seeded and synthetic (paper_2411_00761_amd.datagen); the
records pin the oracle's byte output so that any later change to its arithmetic
or to the record layout shows up as a diff that must be justified.
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

import oracle as O  # noqa: E402
from paper_2411_00761_amd import datagen  # noqa: E402


def cases():
    x = datagen.uniform_frame(300, seed=1)
    g = O.grids_for(x, O.EB_ABS, 1e-2)
    yield "s_uniform_300_k5", O.compress_s(x, g, 5)[0]
    traj = datagen.MDTrajectory(512, seed=2)
    f0, f1 = traj.next_frame(), traj.next_frame()
    g = O.grids_for(f0, O.EB_REL_GLOBAL, 1e-3)
    rec, perm, q = O.compress_s(f0, g, 3)
    yield "s_md_512_k3", rec
    yield "t_md_512", O.compress_t(f1, g, perm, q, ref_seq=0, seq=1)[0]
    c = datagen.cosmology_snapshot(400, box=16.0, n_halos=5, seed=3)
    g = O.grids_for(c, O.EB_REL_PER_FIELD, 1e-3)
    yield "s_cosmo6_400_k2", O.compress_s(c, g, 2)[0]


if __name__ == "__main__":
    for name, rec in cases():
        with open(os.path.join(HERE, name + ".hex"), "w") as fh:
            fh.write(rec.hex() + "\n")
        print(name, len(rec))
