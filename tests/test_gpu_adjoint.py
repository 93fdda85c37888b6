"""GPU: the hand-written adjoint through the C-ABI against the reference
adjoint (oracle/adjoint_ref.py: autograd of a plain restatement of the
scheme) and against central differences of the GPU forward.

The two adjoints differentiate the same branches of the same arithmetic in
different operation orders, so they agree to rounding (1e-9 of the
cotangent's size is asked) wherever no branch decision sits within
rounding of its threshold.  In a uniform region the entropy bound is tight
by construction (psi(U^L) = 0 and P_ij = 0), so whether the limiter returns
0 or 1 there is decided by rounding; the forward result is the same, the
derivative with respect to P_ij is not.  The element-wise comparisons
therefore use generic smooth states without uniform regions (their
adjoints agree to about 1e-15).  Each test prints its case before touching
the GPU.
"""
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


@pytest.fixture(scope="module")
def ref_mod():
    from oracle import adjoint_ref
    return adjoint_ref


def flow_blobs(n, u0=(0.31, 0.17, 0.07)):
    m, _ = inputs.workload("adjoint_3d", n=n)
    rho = 1.0 + 0.1 * inputs.gaussian_blobs(m.coords, 2, lo=0.2, hi=0.8)
    U0 = inputs.conserved(rho, np.tile(np.asarray(u0), (m.n_nodes, 1)), rho.copy())
    return m, U0


def generic(n, dim):
    m = inputs.q1_grid(n, dim, 0.2, seed=3, order="morton")
    return m, inputs.ic_generic_smooth(m.coords)


CASES = {
    "generic_2d_17": lambda: generic(17, 2),
    "generic_3d_9": lambda: generic(9, 3),
}


def close(a, b, tol=1e-9):
    scale = np.abs(b).max()
    return np.abs(a - b).max() <= tol * scale, np.abs(a - b).max() / scale


@pytest.mark.parametrize("case", list(CASES))
def test_stage_vjp_matches_reference(torch, oracle_mod, ref_mod, case):
    announce(f"stage VJP vs reference adjoint: {case}")
    from paper_2007_00094_amd.solver import Solver
    m, U0 = CASES[case]()
    s = Solver(m)
    o = oracle_mod.Oracle(m, dirichlet=m.boundary)
    ref = ref_mod.Reference(o, dirichlet=m.boundary)
    tau = o.max_dt(U0)
    W = np.random.default_rng(4).normal(size=U0.shape)
    U = torch.tensor(U0, device="cuda")
    got = s.euler_stage_vjp(U, tau, torch.tensor(W, device="cuda")).cpu().numpy()
    Ut = torch.tensor(U0, requires_grad=True)
    (torch.tensor(W) * ref.stage(Ut, tau)).sum().backward()
    ok, err = close(got, Ut.grad.numpy())
    assert ok, err


@pytest.mark.parametrize("newton_max", [1, 4])
def test_stage_vjp_with_other_newton_bounds(torch, oracle_mod, ref_mod, newton_max):
    # newton_max <= 2 and above run different instantiations of the limiter
    # VJPs (brackets kept in registers, or in an indexed array)
    announce(f"stage VJP vs reference adjoint: generic_3d_9, newton_max={newton_max}")
    from paper_2007_00094_amd.solver import Solver
    m, U0 = generic(9, 3)
    s = Solver(m, newton_max=newton_max)
    o = oracle_mod.Oracle(m, dirichlet=m.boundary, newton_max=newton_max)
    ref = ref_mod.Reference(o, dirichlet=m.boundary, newton_max=newton_max)
    tau = o.max_dt(U0)
    W = np.random.default_rng(5).normal(size=U0.shape)
    got = s.euler_stage_vjp(torch.tensor(U0, device="cuda"), tau,
                            torch.tensor(W, device="cuda")).cpu().numpy()
    Ut = torch.tensor(U0, requires_grad=True)
    (torch.tensor(W) * ref.stage(Ut, tau)).sum().backward()
    ok, err = close(got, Ut.grad.numpy())
    assert ok, err


def test_step_vjp_matches_reference(torch, oracle_mod, ref_mod):
    announce("step VJP vs reference adjoint: generic_3d_9 after 2 steps")
    from paper_2007_00094_amd.solver import Solver
    m, U0 = generic(9, 3)
    s = Solver(m)
    o = oracle_mod.Oracle(m, dirichlet=m.boundary)
    ref = ref_mod.Reference(o, dirichlet=m.boundary)
    U = U0.copy()
    for _ in range(2):
        U, dt, _ = o.step(U)
    W = np.random.default_rng(6).normal(size=U0.shape)
    got = s.step_vjp(torch.tensor(U, device="cuda"), dt, torch.tensor(W, device="cuda")).cpu().numpy()
    Ut = torch.tensor(U, requires_grad=True)
    (torch.tensor(W) * ref.step(Ut, dt)).sum().backward()
    ok, err = close(got, Ut.grad.numpy())
    assert ok, err


def test_checkpointed_adjoint_matches_reference_and_step_chain(torch, oracle_mod, ref_mod):
    announce("generic_3d_9, 7 steps, checkpoints every 3: adjoint vs step-VJP chain and reference")
    from paper_2007_00094_amd.solver import Solver
    m, U0 = generic(9, 3)
    s = Solver(m)
    o = oracle_mod.Oracle(m, dirichlet=m.boundary)
    ref = ref_mod.Reference(o, dirichlet=m.boundary)
    U, dts, states = U0.copy(), [], [U0.copy()]
    for _ in range(7):
        U, dt, _ = o.step(U)
        dts.append(dt)
        states.append(U.copy())
    Ud = torch.tensor(U0, device="cuda")
    s.forward_checkpoints(Ud, dts, 3)
    assert np.array_equal(Ud.cpu().numpy(), U)            # the forward is the oracle's, bitwise
    W = np.random.default_rng(8).normal(size=U0.shape)
    g = s.adjoint_checkpoints(dts, 3, torch.tensor(W, device="cuda")).cpu().numpy()
    # again: now the last segment is recomputed too (the forward's tape is used up)
    g2 = s.adjoint_checkpoints(dts, 3, torch.tensor(W, device="cuda")).cpu().numpy()
    assert np.array_equal(g, g2)
    chain = torch.tensor(W, device="cuda")
    for k in range(6, -1, -1):
        chain = s.step_vjp(torch.tensor(states[k], device="cuda"), dts[k], chain)
    assert np.array_equal(g, chain.cpu().numpy())
    Ut = torch.tensor(U0, requires_grad=True)
    V = Ut
    for dt in dts:
        V = ref.step(V, dt)
    (torch.tensor(W) * V).sum().backward()
    ok, err = close(g, Ut.grad.numpy(), 1e-8)
    assert ok, err


def test_checkpointed_adjoint_matches_reference_over_50_steps(torch, oracle_mod, ref_mod):
    """A long horizon: 17^3 generic smooth state, 50 steps, checkpoints every
    10.  The GPU adjoint against the chain of the reference adjoint's step
    VJPs taken at the oracle's states (the GPU forward is the oracle's, bit
    for bit), to 1e-9 of the cotangent's size."""
    announce("generic_3d_17, 50 steps, checkpoints every 10: adjoint vs reference step-VJP chain")
    from paper_2007_00094_amd.solver import Solver
    m, U0 = generic(17, 3)
    s = Solver(m)
    o = oracle_mod.Oracle(m, dirichlet=m.boundary)
    ref = ref_mod.Reference(o, dirichlet=m.boundary)
    U, dts, states = U0.copy(), [], [U0.copy()]
    for _ in range(50):
        U, dt, st = o.step(U)
        assert st == 0
        dts.append(dt)
        states.append(U.copy())
    Ud = torch.tensor(U0, device="cuda")
    s.forward_checkpoints(Ud, dts, 10)
    assert np.array_equal(Ud.cpu().numpy(), U)
    W = np.random.default_rng(21).normal(size=U0.shape)
    g = s.adjoint_checkpoints(dts, 10, torch.tensor(W, device="cuda")).cpu().numpy()
    chain = torch.tensor(W)
    for k in range(49, -1, -1):
        Ut = torch.tensor(states[k], requires_grad=True)
        (chain * ref.step(Ut, dts[k])).sum().backward()
        chain = Ut.grad
    ok, err = close(g, chain.numpy(), 1e-9)
    print(f"  max difference / max |cotangent| = {err:.2e}", flush=True)
    assert ok, err
    s.close()


# ------------------------------------------------- central differences
# The scheme is piecewise smooth: every max, min, clamp, branch and
# argmin/argmax is a kink.  A central difference is a derivative of one
# branch only if no decision differs between the +eps and -eps runs, so the
# checks below run those two forwards with the library's decision trace
# (idp_trace_decisions) and count the decisions that differ, by kind:
#   visc  the branches of the wave-speed bound and of d_ij's max;
#   side  which candidate set min(l_ij, l_ji) (either pass);
#   alpha the signs inside the indicator's absolute values;
#   argk  the entries that set a node's density and entropy bounds;
#   cut   the limiter's density cuts (either pass);
#   search the limiter's stopping test and enclosure safeguards: near the
#         root Psi(hi) is zero up to rounding, so whether the search stops
#         at hi or one step later at lo is decided by rounding; both end
#         within rounding of the same root (soft kinks, counted apart).
_CUT_BITS = 0x7           # kLimRhoMax | kLimRhoMin | kLimClamp of one candidate


def _flips(A, B, npairs, n):
    """Decisions that differ between two traces, by kind."""
    import torch
    pb = (npairs * 8 + 255) // 256 * 256
    rb = (n * 4 + 255) // 256 * 256
    x = A[:, :pb].view(torch.int64)[:, :npairs] ^ B[:, :pb].view(torch.int64)[:, :npairs]
    cut = 0
    for shift in (16, 24, 32, 40):
        cut += int(((x >> shift) & _CUT_BITS).ne(0).sum())
    lim = 0
    for shift in (16, 24, 32, 40):
        lim += int(((x >> shift) & 0xFF).ne(0).sum())
    ra = A[:, pb:pb + 4 * n].view(torch.int32)
    rbb = B[:, pb:pb + 4 * n].view(torch.int32)
    aa = A[:, pb + rb:pb + rb + 4 * n].view(torch.int32)
    ab = B[:, pb + rb:pb + rb + 4 * n].view(torch.int32)
    return {"visc": int((x & 0x3FFF).ne(0).sum()),
            "side": int((x & (3 << 48)).ne(0).sum()),
            "alpha": int(ra.ne(rbb).sum()),
            "argk": int(aa.ne(ab).sum()),
            "cut": cut,
            "search": lim - cut}


def _fd_study(s, m, U0, dts, every, box_lo, box_hi, ndir, seed, eps, trace=None, ends=False):
    """Adjoint of J = sum_{x_i in box} m_i |m_i|^2/(2 rho_i) at the final
    state w.r.t. the initial density, and the central difference with step
    eps along ndir seeded smooth unit directions v.  trace(d): whether the
    two runs of direction d are traced (flips counted, else None); ends:
    also the adjoint at both ends U0 +- eps v of the segment.  Yields
    (direction, adjoint, quotient, flips, adjoints at the ends)."""
    import torch
    from paper_2007_00094_amd.autograd import ssprk3
    box = torch.tensor(np.all((m.coords >= box_lo) & (m.coords <= box_hi), axis=1),
                       device="cuda")
    mi = torch.tensor(s.matrices()["m_i"], device="cuda")

    def J(Ux):
        mom = Ux[:, 1:4]
        return (mi * box * (mom * mom).sum(1) / (2 * Ux[:, 0])).sum()

    def grad(U):
        Ut = torch.tensor(U, device="cuda", requires_grad=True)
        Jv = J(ssprk3(s, Ut, dts, every=every))
        Jv.backward()
        return Ut.grad[:, 0].cpu().numpy(), Jv.item()

    g = grad(U0)[0]
    npairs = (s.nnz - m.n_nodes) // 2
    bufs = [None, None]

    def run(U, k):
        V = torch.tensor(U, device="cuda")
        if k is None:
            s.forward_checkpoints(V, dts, every)
        else:
            bufs[k], _ = s.trace_decisions(V, dts, bufs[k])
        return J(V).item()

    rng = np.random.default_rng(seed)
    for d in range(ndir):
        v = np.zeros(m.n_nodes)
        for _ in range(2):
            c = rng.uniform(0.3, 0.7, size=3)
            v += rng.normal() * np.exp(-np.sum((m.coords - c) ** 2, 1) / (2 * 0.1 ** 2))
        v *= 1 - m.boundary
        v /= np.linalg.norm(v)
        Up, Um = U0.copy(), U0.copy()
        Up[:, 0] += eps * v
        Um[:, 0] -= eps * v
        tr = trace is not None and trace(d)
        at_ends = None
        if ends and not tr:
            gp, Jp = grad(Up)
            gm, Jm = grad(Um)
            at_ends = (float(gm @ v), float(gp @ v))
        else:
            Jp, Jm = run(Up, 0 if tr else None), run(Um, 1 if tr else None)
            if ends:
                at_ends = (float(grad(Um)[0] @ v), float(grad(Up)[0] @ v))
        fl = _flips(bufs[0], bufs[1], npairs, m.n_nodes) if tr else None
        yield d, float(g @ v), (Jp - Jm) / (2 * eps), fl, at_ends


def _smooth_case(n, steps):
    import torch
    from paper_2007_00094_amd.solver import Solver
    m = inputs.q1_grid(n, 3, 0.2, seed=0, order="morton")
    U0 = inputs.ic_generic_smooth(m.coords)
    s = Solver(m)
    U = torch.tensor(U0, device="cuda")
    dts = []
    for _ in range(steps):
        dt, st = s.step(U)
        assert st == 0
        dts.append(dt)
    return s, m, U0, dts


def _limiter_flips(fl):
    return fl["side"] + fl["cut"]


def test_adjoint_matches_central_differences_where_no_decision_flips():
    """Smooth data without flat regions (generic smooth state), 9^3, 5 steps,
    checkpoints every 2, J the kinetic energy in [0.3, 0.7]^3, 12 seeded
    directions: along every direction on which no decision other than the
    soft search kinks differs between the +-eps runs (measured: all of
    them), the adjoint matches the central difference with eps 1e-6 to
    1e-6 relative."""
    announce("generic smooth 9^3, 5 steps: adjoint vs central differences on flip-free directions")
    s, m, U0, dts = _smooth_case(9, 5)
    checked = 0
    for d, gv, f6, fl, _ in _fd_study(s, m, U0, dts, 2, 0.3, 0.7, 12, 11, 1e-6,
                                      trace=lambda d: True):
        rel = abs(gv - f6) / abs(f6)
        hard = fl["visc"] + fl["side"] + fl["alpha"] + fl["argk"] + fl["cut"]
        print(f"  direction {d}: adjoint {gv:.10e} fd(1e-6) {f6:.10e} rel {rel:.2e} "
              f"flips {fl}", flush=True)
        if hard == 0:
            checked += 1
            assert rel <= 1e-6, (d, gv, f6)
    assert checked >= 8
    s.close()


def _mean_value_check(gv, f6, ends, tol):
    """Lebourg's mean value theorem for a piecewise smooth J: the secant
    slope along the segment [U0 - eps v, U0 + eps v] is a derivative of J
    at some point of it.  With the adjoint sampled at the centre and both
    ends, the quotient must lie within their range, widened by tol."""
    lo, hi = min(gv, *ends), max(gv, *ends)
    return lo - tol <= f6 <= hi + tol


def test_adjoint_matches_central_differences_on_smooth_data():
    """Smooth data without flat regions on the adjoint configuration's mesh
    and horizon: 65^3 Morton, 200 steps with checkpoints every 20, the
    configuration's J, 16 seeded directions, central differences with eps
    1e-6, both runs traced.  Over 600 stages a handful of ties in the
    viscosity's branches, the indicator's signs and the bounds'
    argmin/argmax differ between the +-eps runs, besides the soft search
    kinks (printed).  Along every direction where no limiter decision
    (which side sets min(l_ij, l_ji), a density cut) differs, the adjoint
    matches the quotient to 1e-6 relative; where one does, the quotient
    straddles a kink of a limiter coefficient and must lie within the
    range of the adjoints at the centre and both ends of the segment
    (mean value theorem), widened by 1e-6 of the directional derivatives'
    RMS (absolute rounding noise of J: about 1e-13 here)."""
    announce("generic smooth 65^3, 200 steps, every 20: adjoint vs central differences, "
             "decision flips counted")
    s, m, U0, dts = _smooth_case(65, 200)
    rows = list(_fd_study(s, m, U0, dts, 20, 0.4, 0.6, 16, 2007, 1e-6,
                          trace=lambda d: True, ends=True))
    rms = float(np.sqrt(np.mean([f6 * f6 for _, _, f6, _, _ in rows])))
    strict = 0
    for d, gv, f6, fl, ends in rows:
        rel = abs(gv - f6) / abs(f6)
        print(f"  direction {d}: adjoint {gv:.10e} (ends {ends[0]:.10e}, {ends[1]:.10e}) "
              f"fd(1e-6) {f6:.10e} rel {rel:.2e} flips {fl}", flush=True)
        if _limiter_flips(fl) == 0:
            strict += 1
            assert rel <= 1e-6, (d, gv, f6)
        else:
            assert _mean_value_check(gv, f6, ends, 1e-6 * rms), (d, gv, f6, ends)
    print(f"  {strict} of {len(rows)} directions without a limiter flip", flush=True)
    s.close()


def test_autograd_two_trajectories_on_one_solver(torch):
    """Two ssprk3 runs on one solver before one backward: each run's
    gradient is its own (the first one's backward redoes its forward, whose
    checkpoints the second run replaced), bit for bit the gradient of the
    same run on a solver of its own."""
    announce("autograd: two interleaved ssprk3 runs on one solver, generic_3d_9, 4 steps")
    from paper_2007_00094_amd.autograd import ssprk3
    from paper_2007_00094_amd.solver import Solver
    m, U0 = generic(9, 3)
    U1 = U0.copy()
    U1[:, 0] *= 1.0 + 0.01 * np.sin(7.0 * m.coords[:, 0])
    rng = np.random.default_rng(12)
    Wa, Wb = rng.normal(size=U0.shape), rng.normal(size=U0.shape)
    s = Solver(m)
    V = torch.tensor(U0, device="cuda")
    dts = [s.step(V)[0] for _ in range(4)]
    a = torch.tensor(U0, device="cuda", requires_grad=True)
    b = torch.tensor(U1, device="cuda", requires_grad=True)
    ya, yb = ssprk3(s, a, dts, every=2), ssprk3(s, b, dts, every=2)
    ((torch.tensor(Wa, device="cuda") * ya).sum() +
     (torch.tensor(Wb, device="cuda") * yb).sum()).backward()
    for U, W, got in ((U0, Wa, a.grad), (U1, Wb, b.grad)):
        alone = Solver(m)
        x = torch.tensor(U, device="cuda", requires_grad=True)
        (torch.tensor(W, device="cuda") * ssprk3(alone, x, dts, every=2)).sum().backward()
        assert torch.equal(got, x.grad)
        alone.close()
    assert not torch.equal(a.grad, b.grad)
    s.close()


def test_adjoint_refuses_batches_and_bad_arguments(torch):
    announce("adjoint error paths")
    import ctypes as C
    from paper_2007_00094_amd.solver import BatchSolver, Solver
    m, U0 = flow_blobs(5)
    bs = BatchSolver([m, m])
    U = torch.tensor(np.concatenate([U0, U0]), device="cuda")
    L = capi.lib()
    p = C.c_void_p(U.data_ptr())
    assert L.idp_step_vjp(bs._h, p, 1e-3, p, C.c_void_p(U.clone().data_ptr())) == capi.IDP_ENOTSUP
    s = Solver(m, newton_max=9)
    V = torch.tensor(U0, device="cuda")
    W = V.clone()
    assert L.idp_step_vjp(s._h, C.c_void_p(V.data_ptr()), 1e-3, C.c_void_p(V.data_ptr()),
                          C.c_void_p(W.data_ptr())) == capi.IDP_ENOTSUP
    s2 = Solver(m)
    d = (C.c_double * 2)(1e-3, 1e-3)
    assert L.idp_adjoint_checkpoints(s2._h, 2, d, 1, C.c_void_p(V.data_ptr()),
                                     C.c_void_p(W.data_ptr())) == capi.IDP_EINVAL


def test_adjoint_at_full_size_against_central_differences():
    """The adjoint configuration as specified: 65^3, isothermal Gaussian
    blobs at rest, 200 steps with checkpoints every 20, gradient of the
    kinetic energy in [0.4, 0.6]^3 w.r.t. the initial density, central
    differences with eps 1e-6 along 32 seeded directions.  Far from the
    blobs the state is uniform to rounding, so many decisions there are
    ties that rounding breaks: between the +-eps runs about a million of
    them differ (counted on the first four directions), and the adjoint
    itself moves by about 1e-6 to 1e-5 of its size between the two ends of
    the segment (printed): J is not differentiable to that precision there,
    and three samples of its derivative do not bound the secant slope.  So
    the quotient must differ from the adjoint by no more than the adjoint
    varies over the centre and both ends of the segment, plus 1e-6 of the
    directional derivatives' RMS (measured: the median difference is 4e-6
    of the quotient, the median variation 1.6e-5)."""
    announce("adjoint_3d_65, 200 steps, every 20: adjoint vs central differences "
             "(mean value check), decision flips counted")
    import torch
    from paper_2007_00094_amd.solver import Solver
    m, U0 = inputs.workload("adjoint_3d", n=65)
    s = Solver(m)
    U = torch.tensor(U0, device="cuda")
    dts = []
    for _ in range(200):
        dt, st = s.step(U)
        assert st == 0
        dts.append(dt)
    rows = list(_fd_study(s, m, U0, dts, 20, 0.4, 0.6, 32, 2007, 1e-6,
                          trace=lambda d: d < 4, ends=True))
    rms = float(np.sqrt(np.mean([f6 * f6 for _, _, f6, _, _ in rows])))
    rel, spread = [], []
    for d, gv, f6, fl, ends in rows:
        rel.append(abs(gv - f6) / abs(f6))
        spread.append((max(gv, *ends) - min(gv, *ends)) / abs(gv))
        print(f"  direction {d}: adjoint {gv:.10e} (ends {ends[0]:.10e}, {ends[1]:.10e}) "
              f"fd(1e-6) {f6:.10e} rel {rel[-1]:.2e} adjoint spread {spread[-1]:.2e} "
              f"flips {fl}", flush=True)
        assert abs(gv - f6) <= (max(gv, *ends) - min(gv, *ends)) + 1e-6 * rms, \
            (d, gv, f6, ends)
    print(f"  relative difference to fd(1e-6): median {np.median(rel):.2e}; adjoint spread "
          f"over the segment: median {np.median(spread):.2e}", flush=True)
    s.close()
