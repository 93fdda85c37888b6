"""GPU: batches of independent meshes in one context (per-instance tau),
under both schedules (one launch per sweep; one persistent launch over a
work-item queue), against the oracle run on each instance alone, bit for
bit.  Each test prints its case before touching the GPU."""
import numpy as np
import pytest

from paper_2007_00094_amd import capi, inputs

pytestmark = pytest.mark.gpu

SCHEDULES = [("launches", 0), ("persistent", 1), ("persistent", 3), ("persistent", 16),
             ("persistent", -2), ("persistent", -8)]


def announce(msg):
    print(f"[gpu case] {msg}", flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


def small_batch(dim=2, sides=(9, 17, 5, 23, 12, 33), seed0=200):
    """Uneven sizes (ragged slice tails, a 5-node side), random quadrant states."""
    out = []
    for k, side in enumerate(sides):
        m = inputs.q1_grid(side, dim, 0.2, seed=seed0 + k, order="morton" if k % 2 else "lex")
        if dim == 2:
            u = inputs.ic_four_quadrant(m.coords, inputs.random_quadrant_states(seed0 + k))
        else:
            u = inputs.ic_sphere(m.coords)
        out.append((m, u))
    return out


def oracle_run(oracle_mod, mesh, u, steps, dt=0.0):
    o = oracle_mod.Oracle(mesh, dirichlet=mesh.boundary)
    taus = []
    for _ in range(steps):
        u, used, st = o.step(u, dt)
        assert st == 0
        taus.append(used)
    return u, taus


def make(batch, **kw):
    from paper_2007_00094_amd.solver import BatchSolver
    return BatchSolver([m for m, _ in batch], **kw)


@pytest.mark.parametrize("kind,tile", SCHEDULES)
def test_batch_2d_matches_oracle_per_instance(torch, oracle_mod, kind, tile):
    announce(f"2D batch of 6 instances, 4 CFL steps, schedule {kind} tile {tile}")
    batch = small_batch()
    bs = make(batch)
    U = torch.tensor(np.concatenate([u for _, u in batch]), device="cuda")
    taus, rc = bs.steps(U, 4, schedule=bs.schedule(kind, tile))
    assert rc == 0
    got = U.cpu().numpy()
    for k, (m, u) in enumerate(batch):
        ref, rtau = oracle_run(oracle_mod, m, u, 4)
        assert np.array_equal(taus[:, k], rtau), k
        assert np.array_equal(got[bs.offsets[k]:bs.offsets[k + 1]], ref), k


@pytest.mark.parametrize("kind,tile", [("launches", 0), ("persistent", 2)])
def test_batch_3d_matches_oracle_per_instance(torch, oracle_mod, kind, tile):
    announce(f"3D batch (5^3, 7^3, 4^3), 2 CFL steps, schedule {kind} tile {tile}")
    batch = small_batch(dim=3, sides=(5, 7, 4), seed0=300)
    bs = make(batch)
    U = torch.tensor(np.concatenate([u for _, u in batch]), device="cuda")
    taus, rc = bs.steps(U, 2, schedule=bs.schedule(kind, tile))
    assert rc == 0
    got = U.cpu().numpy()
    for k, (m, u) in enumerate(batch):
        ref, rtau = oracle_run(oracle_mod, m, u, 2)
        assert np.array_equal(taus[:, k], rtau), k
        assert np.array_equal(got[bs.offsets[k]:bs.offsets[k + 1]], ref), k


def test_batch_fixed_dt_and_max_dt(torch, oracle_mod):
    announce("2D batch: per-instance max_dt, then 3 steps with fixed per-instance dt")
    batch = small_batch()
    bs = make(batch)
    U = torch.tensor(np.concatenate([u for _, u in batch]), device="cuda")
    dts = bs.max_dt(U)
    for k, (m, u) in enumerate(batch):
        o = oracle_mod.Oracle(m, dirichlet=m.boundary)
        assert dts[k] == o.max_dt(u), k
    fixed = 0.5 * dts
    for kind, tile in (("launches", 0), ("persistent", 4)):
        V = U.clone()
        taus, rc = bs.steps(V, 3, dt=fixed, schedule=bs.schedule(kind, tile))
        assert rc == 0
        assert np.array_equal(taus, np.tile(fixed, (3, 1)))
        got = V.cpu().numpy()
        for k, (m, u) in enumerate(batch):
            ref, _ = oracle_run(oracle_mod, m, u, 3, dt=fixed[k])
            assert np.array_equal(got[bs.offsets[k]:bs.offsets[k + 1]], ref), (kind, k)


def test_batch_dt_too_large_is_an_error(torch):
    announce("2D batch: one instance's dt above its bound -> IDP_EDT, both schedules")
    batch = small_batch()
    bs = make(batch)
    U = torch.tensor(np.concatenate([u for _, u in batch]), device="cuda")
    dts = bs.max_dt(U) / bs.params.cfl
    bad = 0.5 * dts
    bad[3] = 1.5 * dts[3]
    for kind, tile in (("launches", 0), ("persistent", 1)):
        with pytest.raises(capi.IdpError) as ei:
            bs.steps(U.clone(), 2, dt=bad, schedule=bs.schedule(kind, tile))
        assert ei.value.code == capi.IDP_EDT


def test_batch_matches_single_contexts(torch):
    announce("first 8 instances of the 64-mesh workload: batch (persistent 4, launches) "
             "vs one Solver each, 3 steps")
    from paper_2007_00094_amd.solver import Solver
    batch = inputs.batch_workload()[:8]
    bs = make(batch)
    U0 = np.concatenate([u for _, u in batch])
    ref = []
    for m, u in batch:
        s = Solver(m)
        V = torch.tensor(u, device="cuda")
        for _ in range(3):
            s.step(V)
        ref.append(V.cpu().numpy())
        s.close()
    ref = np.concatenate(ref)
    for kind, tile in (("persistent", 4), ("launches", 0)):
        U = torch.tensor(U0, device="cuda")
        _, rc = bs.steps(U, 3, schedule=bs.schedule(kind, tile))
        assert rc == 0
        assert np.array_equal(U.cpu().numpy(), ref), kind


def test_tuner_keeps_state_and_results(torch):
    announce("2D batch: autotuner over the candidate schedules, then the tuned default")
    batch = small_batch()
    bs = make(batch)
    U0 = torch.tensor(np.concatenate([u for _, u in batch]), device="cuda")
    keep = U0.clone()
    best, ms = bs.tune(U0, 2)
    assert torch.equal(U0, keep)
    assert len(ms) == 10 and all(v > 0 for v in ms.values()), ms
    assert best.kind in (capi.IDP_SCHED_LAUNCHES, capi.IDP_SCHED_PERSISTENT)
    A, B = U0.clone(), U0.clone()
    bs.steps(A, 2)                                        # tuned default
    bs.steps(B, 2, schedule=bs.schedule("launches"))
    assert torch.equal(A, B)


def test_single_instance_calls_refuse_a_batch(torch):
    announce("2D batch: idp_step / idp_max_dt on a batch context -> IDP_ENOTSUP")
    import ctypes as C
    batch = small_batch()[:2]
    bs = make(batch)
    U = torch.tensor(np.concatenate([u for _, u in batch]), device="cuda")
    L = capi.lib()
    out = C.c_double()
    assert L.idp_step(bs._h, C.c_void_p(U.data_ptr()), 0.0, None) == capi.IDP_ENOTSUP
    assert L.idp_max_dt(bs._h, C.c_void_p(U.data_ptr()), C.byref(out)) == capi.IDP_ENOTSUP


def test_batch_calls_refuse_a_renumbered_context(torch):
    """A context built with IDP_FLAG_RENUMBER keeps its state in its own
    numbering; the batch calls (which take the concatenated state as is)
    answer IDP_ENOTSUP instead of stepping the caller's order wrongly."""
    announce("2D renumbered single mesh: batch steps / max_dt / tune -> IDP_ENOTSUP")
    import ctypes as C
    from paper_2007_00094_amd.solver import Solver
    m = inputs.q1_grid(9, 2, 0.2, seed=5, order="random")
    u = inputs.ic_four_quadrant(m.coords, inputs.random_quadrant_states(5))
    s = Solver(m, renumber=True)
    U = torch.tensor(u, device="cuda")
    L = capi.lib()
    dt = (C.c_double * 1)()
    p = C.c_void_p(U.data_ptr())
    assert L.idp_batch_steps(s._h, p, 1, None, None, None) == capi.IDP_ENOTSUP
    assert L.idp_batch_max_dt(s._h, p, dt) == capi.IDP_ENOTSUP
    assert L.idp_batch_tune(s._h, p, 1, None, None, None) == capi.IDP_ENOTSUP
    assert np.array_equal(U.cpu().numpy(), u)
    s.close()


_FULL_BATCH = {}


@pytest.mark.parametrize("kind,tile", [("launches", 0), ("persistent", 64),
                                       ("persistent", -32)])
def test_full_batch_workload_sampled_instances(torch, oracle_mod, kind, tile):
    """The benchmark's batch (64 2D meshes, sides 33-513, per-instance CFL
    dt) for 3 steps under the launch schedule and the persistent one (fixed
    tiles; tiles per instance size): the smallest, the largest and two more
    instances bit for bit against the oracle run alone, and the whole batch
    bit for bit the same under every schedule."""
    announce(f"full 64-mesh batch workload, 3 steps, schedule {kind} tile {tile}, "
             "sampled instances vs oracle")
    batch = inputs.batch_workload()
    bs = make(batch)
    U = torch.tensor(np.concatenate([u for _, u in batch]), device="cuda")
    from paper_2007_00094_amd.solver import BatchSolver
    used, _ = bs.steps(U, 3, schedule=BatchSolver.schedule(kind, tile))
    Ug = U.cpu().numpy()
    if kind == "launches":
        _FULL_BATCH["launches"] = Ug
    elif "launches" in _FULL_BATCH:
        assert np.array_equal(Ug, _FULL_BATCH["launches"])
    off = np.cumsum([0] + [m.n_nodes for m, _ in batch])
    sizes = [m.n_nodes for m, _ in batch]
    picks = sorted({int(np.argmin(sizes)), int(np.argmax(sizes)), 7, 40})
    for k in picks:
        m, u = batch[k]
        uo, taus = oracle_run(oracle_mod, m, u, 3)
        assert np.array_equal(used[:, k], taus), k
        assert np.array_equal(Ug[off[k]:off[k + 1]], uo), k

