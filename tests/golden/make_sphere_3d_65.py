"""Write the 100-step oracle reference of the 3D spherical shock tube.

Workload: 3D Q1 grid 65^3 on [0,1]^3, interior nodes jittered by up to
0.2 h (seed 0), seeded random node order (seed 1); rho, p = (1, 1) inside
the sphere r < 0.3 around the centre, (0.125, 0.1) outside, at rest;
gamma 1.4, boundary held, SSP-RK3 at CFL 0.5, 100 steps.

Calls only the CPU oracle.  Stores the dt of every step, SHA-256 digests of
the state (float64, C order, little endian) after steps 1, 10, 50 and 100,
and the final state of 64 seeded sample nodes.

    python tests/golden/make_sphere_3d_65.py
"""
import hashlib
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2007_00094_amd import inputs  # noqa: E402

OUT = os.path.join(HERE, "sphere_3d_65_100steps.txt")
STEPS = 100
CHECKPOINTS = (1, 10, 50, 100)


def digest(U):
    return hashlib.sha256(np.ascontiguousarray(U, dtype="<f8").tobytes()).hexdigest()


def sample_nodes(n):
    return np.sort(np.random.default_rng(7).choice(n, 64, replace=False))


def main():
    mesh, U = inputs.workload("sphere_3d")
    o = oracle.Oracle(mesh)
    dts, hashes = [], {}
    for k in range(1, STEPS + 1):
        U, dt, st = o.step(U)
        assert st in (0, 1), st
        dts.append(dt)
        if k in CHECKPOINTS:
            hashes[k] = digest(U)
            print(f"step {k} dt {dt:.6e} sha256 {hashes[k][:16]}", flush=True)
    lines = ["# oracle SSP-RK3 reference, written by tests/golden/make_sphere_3d_65.py",
             "# sphere_3d 65^3 random order (jitter seed 0, order seed 1), CFL 0.5",
             f"steps {STEPS}"]
    lines += [f"sha256 {k} {h}" for k, h in hashes.items()]
    lines += ["dt " + " ".join(f"{d:.17g}" for d in dts)]
    for i in sample_nodes(mesh.n_nodes):
        lines.append(f"sample {i} " + " ".join(f"{v:.17g}" for v in U[i]))
    open(OUT, "w").write("\n".join(lines) + "\n")
    print("wrote", OUT)


if __name__ == "__main__":
    main()
