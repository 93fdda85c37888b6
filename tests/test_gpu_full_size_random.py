"""GPU parity at the benchmark's size in the other node ordering: the 3D
Mach 3 blob flow on the 257^3 jittered mesh numbered by a seeded random
permutation (every neighbour gather misses; no row block's neighbourhood
fits the LDS staging).

* plain context: two CFL steps on the whole mesh; the second step's output
  on sampled patches against the oracle stepping the GPU's state with the
  GPU's dt;
* the same mesh with the library's own Morton renumbering
  (IDP_FLAG_RENUMBER): the same two steps bit for bit, dt included.
"""
import numpy as np
import pytest

from paper_2007_00094_amd import inputs
from test_gpu_full_size import N_BIG, announce, check_step_patches

pytestmark = pytest.mark.gpu


def test_mach3_257_random_order_plain_and_renumbered(oracle_mod):
    import torch
    from paper_2007_00094_amd.solver import Solver
    announce(f"mach3_3d {N_BIG}^3 random order: mesh, plain solver")
    mesh, U0 = inputs.workload("mach3_3d", n=N_BIG, order="random")
    s = Solver(mesh, staging=True, sell_sigma=64)
    U = torch.tensor(U0, device="cuda")
    dts = []
    dt, st = s.step(U)
    assert st == 0
    dts.append(dt)
    U1 = U.cpu().numpy()
    dt, st = s.step(U)
    assert st == 0
    dts.append(dt)
    U2 = U.cpu().numpy()
    s.close()
    del U
    torch.cuda.empty_cache()
    pe = inputs.PatchExtractor(mesh)
    rng = np.random.default_rng(13)
    samples = np.concatenate([rng.choice(mesh.n_nodes, 8, replace=False),
                              [int(np.argmax(U0[:, 0]))]])
    announce(f"  step 2 on {len(samples)} sampled patches vs the oracle")
    check_step_patches(oracle_mod, pe, samples, U1, U2, dts[1])
    announce(f"mach3_3d {N_BIG}^3 random order: renumbered solver, 2 steps")
    r = Solver(mesh, staging=True, sell_sigma=64, renumber=True)
    V = torch.tensor(U0, device="cuda")
    for k in range(2):
        dt, st = r.step(V)
        assert st == 0 and dt == dts[k]
    assert np.array_equal(V.cpu().numpy(), U2)
    r.close()
