"""GPU: idp_batch_steps_noalloc (the batch step whose scratch lives in a
static device array) against idp_batch_steps with the launch schedule, bit
for bit, on two calls in a row (the second with a smaller batch and fewer
steps, so the shared array holds the first call's contents), plus its size
limit and its refusal of a renumbered context.  Every call goes through the
C-ABI; each case is printed before it touches the GPU."""
import ctypes as C

import numpy as np
import pytest

from paper_2007_00094_amd import capi, inputs

pytestmark = pytest.mark.gpu


def announce(msg):
    print(f"[gpu case] {msg}", flush=True)


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


def batch_of(sides, dim, seed0):
    out = []
    for k, side in enumerate(sides):
        m = inputs.q1_grid(side, dim, 0.2, seed=seed0 + k, order="morton" if k % 2 else "lex")
        if dim == 2:
            u = inputs.ic_four_quadrant(m.coords, inputs.random_quadrant_states(seed0 + k))
        else:
            u = inputs.ic_sphere(m.coords)
        out.append((m, u))
    return out


def device_bytes(h):
    nb = C.c_size_t()
    capi.check("idp_info", capi.lib().idp_info(h, None, None, C.byref(nb)))
    return int(nb.value)


def run_both(torch, bs, U0, n_steps, dt=None):
    """(reference state, reference taus, no-alloc state, no-alloc taus)."""
    L = capi.lib()
    K = bs.count
    dta = None
    if dt is not None:
        dt = np.ascontiguousarray(dt, dtype=np.float64)
        dta = dt.ctypes.data_as(capi._dp)
    A = torch.tensor(U0, device="cuda")
    ta = np.zeros((n_steps, K))
    sched = capi.idp_schedule(capi.IDP_SCHED_LAUNCHES, 0)
    rc = L.idp_batch_steps(bs._h, C.c_void_p(A.data_ptr()), n_steps, dta,
                           ta.ctypes.data_as(capi._dp), C.byref(sched))
    assert rc == 0, capi.strerror(rc)
    B = torch.tensor(U0, device="cuda")
    tb = np.full((n_steps, K), -1.0)
    before = device_bytes(bs._h)
    rc = L.idp_batch_steps_noalloc(bs._h, C.c_void_p(B.data_ptr()), n_steps, dta,
                                   tb.ctypes.data_as(capi._dp))
    assert rc == 0, capi.strerror(rc)
    assert device_bytes(bs._h) == before        # the context allocated nothing
    torch.cuda.synchronize()
    return A.cpu().numpy(), ta, B.cpu().numpy(), tb


def test_noalloc_matches_batch_steps_on_two_calls(torch):
    from paper_2007_00094_amd.solver import BatchSolver
    announce("no-alloc call 1: 2D batch of 6 uneven meshes, 5 CFL steps")
    big = batch_of((9, 17, 5, 23, 12, 33), 2, 400)
    bs1 = BatchSolver([m for m, _ in big])
    U1 = np.concatenate([u for _, u in big])
    ra, ta, rb, tb = run_both(torch, bs1, U1, 5)
    assert np.array_equal(ta, tb)
    assert np.array_equal(ra, rb)
    announce("no-alloc call 2: 2D batch of 2 smaller meshes, 2 steps with fixed dt")
    small = batch_of((7, 11), 2, 500)
    bs2 = BatchSolver([m for m, _ in small])
    U2 = np.concatenate([u for _, u in small])
    dts = 0.5 * bs2.max_dt(torch.tensor(U2, device="cuda"))
    ra, ta, rb, tb = run_both(torch, bs2, U2, 2, dt=dts)
    assert np.array_equal(ta, np.tile(dts, (2, 1))) and np.array_equal(ta, tb)
    assert np.array_equal(ra, rb)
    bs1.close()
    bs2.close()


def test_noalloc_single_mesh_3d_matches_idp_step(torch):
    from paper_2007_00094_amd.solver import BatchSolver, Solver
    announce("no-alloc on a one-instance 3D context (9^3 sphere), 3 steps vs idp_step")
    m = inputs.q1_grid(9, 3, 0.2, seed=7, order="morton")
    u = inputs.ic_sphere(m.coords)
    s = Solver(m)
    A = torch.tensor(u, device="cuda")
    taus = [s.step(A)[0] for _ in range(3)]
    s.close()
    bs = BatchSolver([m])
    B = torch.tensor(u, device="cuda")
    tb = np.zeros((3, 1))
    rc = capi.lib().idp_batch_steps_noalloc(bs._h, C.c_void_p(B.data_ptr()), 3, None,
                                           tb.ctypes.data_as(capi._dp))
    assert rc == 0, capi.strerror(rc)
    assert np.array_equal(tb[:, 0], taus)
    assert torch.equal(A, B)
    bs.close()


def test_noalloc_limits_and_refusals(torch):
    from paper_2007_00094_amd.solver import BatchSolver, Solver
    announce("no-alloc: more steps than the static array holds -> IDP_ESCRATCH, "
             "renumbered context -> IDP_ENOTSUP, bad dt -> IDP_EINVAL")
    L = capi.lib()
    batch = batch_of((9, 5), 2, 600)
    bs = BatchSolver([m for m, _ in batch])
    U0 = np.concatenate([u for _, u in batch])
    U = torch.tensor(U0, device="cuda")
    p = C.c_void_p(U.data_ptr())
    # 16 + 32 K + 8 n_steps K bytes must fit in 1 MiB (K = 2)
    too_many = (1 << 20) // 16 + 1
    assert L.idp_batch_steps_noalloc(bs._h, p, too_many, None, None) == capi.IDP_ESCRATCH
    bad = np.array([1e-3, -1.0])
    assert L.idp_batch_steps_noalloc(bs._h, p, 1, bad.ctypes.data_as(capi._dp), None) == \
        capi.IDP_EINVAL
    assert L.idp_batch_steps_noalloc(bs._h, p, 0, None, None) == 0
    assert np.array_equal(U.cpu().numpy(), U0)
    bs.close()
    m = inputs.q1_grid(9, 2, 0.2, seed=5, order="random")
    s = Solver(m, renumber=True)
    V = torch.tensor(inputs.ic_four_quadrant(m.coords), device="cuda")
    assert L.idp_batch_steps_noalloc(s._h, C.c_void_p(V.data_ptr()), 1, None, None) == \
        capi.IDP_ENOTSUP
    s.close()
