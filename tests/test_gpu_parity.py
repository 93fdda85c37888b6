"""GPU parity: the HIP path through the C-ABI against the CPU oracle.

The library evaluates every formula in the oracle's operation order with
IEEE add/sub/mul/div/sqrt and the same fixed-method x^y, so results are
compared bit for bit (the stated tolerance, 1e-12 relative per step and
1e-9 after 100 steps, is then met with margin).  Each test prints the case
it runs before touching the GPU.
"""
import numpy as np
import pytest

from paper_2007_00094_amd import capi, inputs

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


def solver(mesh, **kw):
    from paper_2007_00094_amd.solver import Solver
    return Solver(mesh, **kw)


def rel_diff(a, b):
    a, b = np.asarray(a), np.asarray(b)
    scale = np.max(np.abs(b), axis=0)
    scale = np.where(scale > 0, scale, 1.0)
    return np.max(np.abs(a - b), axis=0) / scale


def announce(msg):
    print(f"[gpu case] {msg}", flush=True)


def test_device_math_bitwise(torch, oracle_mod):
    announce("device x^y, sqrt, div vs host")
    mesh = inputs.q1_grid(3, 2)
    s = solver(mesh)
    rng = np.random.default_rng(1)
    xs, ys = [], []
    for y in (2.4, -1.4, 1 / 2.4, -1.4 / 2.4, -(0.4) / 2.8, 2.8 / 0.4, 0.5 / 1.4):
        x = np.concatenate([10 ** rng.uniform(-6, 6, 3000), rng.uniform(0.5, 2.0, 3000)])
        xs.append(x)
        ys.append(np.full_like(x, y))
    x = np.concatenate(xs + [np.array([0.0, 1.0, 2.0])])
    y = np.concatenate(ys + [np.array([2.4, 2.4, 3.0])])
    got = s.device_math(0, torch.tensor(x, device="cuda"), torch.tensor(y, device="cuda")).cpu().numpy()
    ref = np.array([oracle_mod.pow_(a, b) for a, b in zip(x, y)])
    assert np.array_equal(got, ref), np.count_nonzero(got != ref)
    q = 10 ** rng.uniform(-300, 300, 20000)
    gs = s.device_math(1, torch.tensor(q, device="cuda")).cpu().numpy()
    assert np.array_equal(gs, np.sqrt(q))
    a, b = rng.normal(size=20000) * 10 ** rng.uniform(-100, 100, 20000), rng.normal(size=20000)
    gd = s.device_math(2, torch.tensor(a, device="cuda"), torch.tensor(b, device="cuda")).cpu().numpy()
    assert np.array_equal(gd, a / b)
    s.close()


MATRIX_CASES = [(2, 17, "lex"), (2, 17, "random"), (3, 9, "random"), (3, 6, "morton")]


@pytest.mark.parametrize("dim,n,order", MATRIX_CASES)
def test_matrices_bitwise(torch, oracle_mod, dim, n, order):
    announce(f"matrices dim={dim} n={n} order={order}")
    mesh = inputs.q1_grid(n, dim, 0.2, seed=5, order=order)
    s = solver(mesh)
    M = s.matrices()
    o = oracle_mod.Oracle(mesh)
    assert np.array_equal(M["row_ptr"], o.row_ptr())
    assert np.array_equal(M["col"].astype(np.int64), o.col())
    assert np.array_equal(M["m_ij"], o.m_ij())
    assert np.array_equal(M["c_ij"], o.c_ij())
    assert np.array_equal(M["m_i"], o.m_i())
    s.close()


STAGE_CASES = [("four_quadrant", 2, 33, "random"), ("sphere", 3, 11, "random"),
               ("mach3", 3, 9, "morton")]


def _case(name, dim, n, order):
    mesh = inputs.q1_grid(n, dim, 0.2, seed=0, order=order)
    if name == "four_quadrant":
        U = inputs.ic_four_quadrant(mesh.coords)
    elif name == "sphere":
        U = inputs.ic_sphere(mesh.coords)
    else:
        U = inputs.ic_mach3_blobs(mesh.coords)
    return mesh, U


@pytest.mark.parametrize("name,dim,n,order", STAGE_CASES)
def test_stage_intermediates_bitwise(torch, oracle_mod, name, dim, n, order):
    """Every intermediate of one forward-Euler stage (Alg. 1 steps 1-6)."""
    announce(f"stage intermediates {name} dim={dim} n={n} {order}")
    mesh, U0 = _case(name, dim, n, order)
    o = oracle_mod.Oracle(mesh)
    tau = o.max_dt(U0)
    E_ref, w_ref = o.euler_stage(U0, tau)
    s = solver(mesh)
    U = torch.tensor(U0, device="cuda")
    E, w = s.euler_stage(U, tau)
    g = lambda k: s.debug(k)
    tp = o.tpos()
    sym = lambda l: np.minimum(l, l[tp])
    pairs = [("d", g(capi.IDP_DBG_D), o.d_ij()), ("alpha", g(capi.IDP_DBG_ALPHA), o.alpha()),
             ("tau_i", g(capi.IDP_DBG_TAUI), o.tau_i()), ("R", g(capi.IDP_DBG_R), o.R()),
             ("U^L", g(capi.IDP_DBG_UL), o.U_low()), ("bounds", g(capi.IDP_DBG_BOUNDS), o.bounds()),
             ("min l1", g(capi.IDP_DBG_L1), sym(o.l1())), ("min l2", g(capi.IDP_DBG_L2), sym(o.l2())),
             ("U pass 1", g(capi.IDP_DBG_UPASS), o.U_pass1()), ("E(U)", E.cpu().numpy(), E_ref),
             ("P", g(capi.IDP_DBG_P), o.P()), ("l1 raw", g(capi.IDP_DBG_L1RAW), o.l1()),
             ("l2 raw", g(capi.IDP_DBG_L2RAW), o.l2())]
    for nm, a, b in pairs:
        assert np.array_equal(a, b), (nm, np.max(rel_diff(a, b)))
    # the recomputed candidates are the ones the pair sweeps took the minima of
    assert np.array_equal(sym(g(capi.IDP_DBG_L1RAW)), g(capi.IDP_DBG_L1))
    assert np.array_equal(sym(g(capi.IDP_DBG_L2RAW)), g(capi.IDP_DBG_L2))
    assert w == w_ref
    s.close()


def _run_steps(torch, oracle_mod, mesh, U0, steps, every_step=True, relax=False, **kw):
    o = oracle_mod.Oracle(mesh, relax=relax)
    s = solver(mesh, relax=relax, **kw)
    U = torch.tensor(U0, device="cuda")
    Uo = U0.copy()
    worst = 0.0
    for k in range(steps):
        dt, st = s.step(U)
        Uo, dto, sto = o.step(Uo)
        assert st == sto and dt == dto, (k, st, sto, dt, dto)
        if every_step or k == steps - 1:
            Ug = U.cpu().numpy()
            worst = max(worst, float(np.max(rel_diff(Ug, Uo))))
            assert np.array_equal(Ug, Uo), (k, worst)
    s.close()
    return worst


def test_step_parity_four_quadrant_50_steps(torch, oracle_mod):
    """2D 33^2 jittered four-quadrant Riemann problem, held boundary,
    CFL 0.5, 50 SSP-RK3 steps: every step bit-identical, dt identical."""
    announce("four-quadrant 2D 33^2, 50 steps")
    mesh, U0 = inputs.workload("four_quadrant_2d")
    assert _run_steps(torch, oracle_mod, mesh, U0, 50) == 0.0


@pytest.mark.parametrize("relax,renumber", [(False, False), (True, False), (True, True)])
def test_step_parity_vortex_relaxed_bounds(torch, oracle_mod, relax, renumber):
    """Translated isentropic vortex on a smoothly warped 2D 33^2 mesh in
    random node order, 30 steps, with the paper's bounds and with the
    bounds widened by (m_i/|Omega|)^(1.5/d) (remark of Section 3.9; |Omega|
    summed in the caller's node order, also when the library renumbers)."""
    announce(f"vortex 2D 33^2 warped random order, relax={relax} renumber={renumber}, 30 steps")
    mesh = inputs.q1_grid(33, 2, jitter=0.0, warp=0.05, order="random")
    U0 = inputs.isentropic_vortex(mesh.coords, radius=0.1, u_inf=(0.5, 0.25))
    assert _run_steps(torch, oracle_mod, mesh, U0, 30, relax=relax, renumber=renumber) == 0.0


def test_step_parity_relaxed_bounds_3d(torch, oracle_mod):
    """3D 13^3 Mach 3 blobs, Morton order, relaxed bounds: 5 steps bitwise;
    the adjoint refuses a relaxed context."""
    announce("relaxed bounds 3D 13^3 Morton, 5 steps")
    mesh = inputs.q1_grid(13, 3, 0.2, seed=0, order="morton")
    U0 = inputs.ic_mach3_blobs(mesh.coords)
    assert _run_steps(torch, oracle_mod, mesh, U0, 5, relax=True) == 0.0
    s = solver(mesh, relax=True)
    U = torch.tensor(U0, device="cuda")
    with pytest.raises(RuntimeError, match="not supported"):
        s.forward_checkpoints(U, [1e-4], every=1)
    s.close()


@pytest.mark.parametrize("dim,n,steps", [(2, 33, 20), (3, 13, 4)])
def test_split_p_variant_is_bitwise(torch, oracle_mod, dim, n, steps):
    """The paper's variant 3 (the low-order sweep stores the viscous part of
    P_ij, the limiter sweeps and passes read it): the oracle's steps, bit
    for bit, staged (Morton) and gathered (random order)."""
    for order in ("morton", "random"):
        announce(f"variant 3 (split P_ij): dim={dim} n={n} {order}, {steps} steps")
        mesh = inputs.q1_grid(n, dim, 0.2, seed=0, order=order)
        U0 = inputs.ic_four_quadrant(mesh.coords) if dim == 2 else inputs.ic_sphere(mesh.coords)
        assert _run_steps(torch, oracle_mod, mesh, U0, steps, split_p=True) == 0.0


def test_step_parity_sphere_3d(torch, oracle_mod):
    announce("sphere 3D 17^3 random order, 10 steps")
    mesh = inputs.q1_grid(17, 3, 0.2, seed=0, order="random", perm_seed=1)
    U0 = inputs.ic_sphere(mesh.coords)
    assert _run_steps(torch, oracle_mod, mesh, U0, 10) == 0.0


def test_step_parity_ragged_tail(torch, oracle_mod):
    """Sizes that leave a partial last slice and mixed row lengths."""
    announce("ragged 2D 13x13 (169 nodes) and 3D 7^3")
    for dim, n in ((2, 13), (3, 7)):
        mesh = inputs.q1_grid(n, dim, 0.2, seed=3, order="random")
        U0 = inputs.ic_sphere(mesh.coords)
        assert _run_steps(torch, oracle_mod, mesh, U0, 3) == 0.0


def test_max_dt_and_free_stream(torch, oracle_mod):
    announce("max_dt parity and free stream")
    mesh = inputs.q1_grid(9, 3, 0.2, seed=2, order="random")
    U0 = inputs.ic_uniform(mesh.n_nodes, 3, rho=1.4, vel=[3.0, 0.2, -0.1], p=1.0)
    o = oracle_mod.Oracle(mesh)
    s = solver(mesh)
    U = torch.tensor(U0, device="cuda")
    assert s.max_dt(U) == o.max_dt(U0)
    for _ in range(3):
        s.step(U)
    assert np.array_equal(U.cpu().numpy(), U0)
    s.close()


STAGING_CASES = [
    ("mach3 3D 33^3 Morton (staged blocks)", 3, 33, "morton", "mach3"),
    ("four-quadrant 2D 65^2 lex (staged blocks)", 2, 65, "lex", "quad"),
    ("sphere 3D 17^3 random (every halo too large: gathers)", 3, 17, "random", "sphere"),
]


@pytest.mark.parametrize("name,dim,n,order,ic", STAGING_CASES)
def test_lds_staging_is_bitwise_the_gather_path(torch, oracle_mod, name, dim, n, order, ic):
    """Row sweeps and the viscosity sweep that stage their block's
    neighbourhood in LDS give the same bits as the cooperative gathers, and
    both the oracle's."""
    announce(f"LDS staging vs gathers: {name}")
    from paper_2007_00094_amd.solver import Solver
    mesh = inputs.q1_grid(n, dim, 0.2, seed=0, order=order, perm_seed=1)
    U0 = {"mach3": lambda: inputs.ic_mach3_blobs(mesh.coords),
          "quad": lambda: inputs.ic_four_quadrant(mesh.coords),
          "sphere": lambda: inputs.ic_sphere(mesh.coords)}[ic]()
    outs = []
    for staging in (True, False):
        s = Solver(mesh, staging=staging)
        U = torch.tensor(U0, device="cuda")
        for _ in range(3):
            s.step(U)
        outs.append(U.cpu().numpy())
        s.close()
    assert np.array_equal(outs[0], outs[1])
    o = oracle_mod.Oracle(mesh, dirichlet=mesh.boundary)
    V = U0.copy()
    for _ in range(3):
        V, _, st = o.step(V)
        assert st == 0
    assert np.array_equal(outs[0], V)


@pytest.mark.parametrize("dim,n,sigma", [(3, 33, 64), (3, 17, 256), (2, 65, 64)])
def test_sell_window_is_bitwise(torch, oracle_mod, dim, n, sigma):
    """Rows sorted by length within windows of sigma rows (SELL-C-sigma of
    Section 4.3) instead of across the mesh: same bits as the oracle."""
    announce(f"SELL window sigma={sigma}: dim={dim} n={n} Morton")
    from paper_2007_00094_amd.solver import Solver
    mesh = inputs.q1_grid(n, dim, 0.2, seed=0, order="morton")
    U0 = inputs.ic_four_quadrant(mesh.coords) if dim == 2 else inputs.ic_mach3_blobs(mesh.coords)
    s = Solver(mesh, sell_sigma=sigma)
    U = torch.tensor(U0, device="cuda")
    o = oracle_mod.Oracle(mesh, dirichlet=mesh.boundary)
    V = U0.copy()
    for _ in range(3):
        s.step(U)
        V, _, st = o.step(V)
        assert st == 0
    assert np.array_equal(U.cpu().numpy(), V)
    s.close()


@pytest.mark.parametrize("dim", [2, 3])
def test_single_cell_mesh(torch, oracle_mod, dim):
    """The smallest mesh: one cell, every row the full stencil of 2^dim
    nodes; three steps without boundary hold bitwise the oracle's, and with
    the default hold (every node on the boundary) the state unchanged."""
    announce(f"single-cell mesh dim={dim}")
    from paper_2007_00094_amd.solver import Solver
    mesh = inputs.q1_grid(2, dim, 0.2, seed=0, order="random")
    U0 = inputs.ic_generic_smooth(mesh.coords)
    free = np.zeros(mesh.n_nodes, np.uint8)
    s = Solver(mesh, dirichlet=free)
    o = oracle_mod.Oracle(mesh, dirichlet=free)
    U = torch.tensor(U0, device="cuda")
    Uo = U0.copy()
    for _ in range(3):
        dt, st = s.step(U)
        Uo, dto, sto = o.step(Uo)
        assert dt == dto and st == sto
        assert np.array_equal(U.cpu().numpy(), Uo)
    s.close()
    s = Solver(mesh)
    U = torch.tensor(U0, device="cuda")
    s.step(U)
    assert np.array_equal(U.cpu().numpy(), U0)
    s.close()


@pytest.mark.parametrize("dim,n", [(2, 33), (3, 17)])
def test_renumbered_context_is_bitwise_the_plain_one(torch, oracle_mod, dim, n):
    """IDP_FLAG_RENUMBER on a randomly numbered mesh: steps, max_dt, a stage,
    every debug export, the matrices and the adjoint entry points bit for
    bit those of the plain context (and the oracle's), all in the caller's
    numbering."""
    announce(f"renumbered context dim={dim} n={n} random order")
    from paper_2007_00094_amd.solver import Solver
    mesh = inputs.q1_grid(n, dim, 0.2, seed=5, order="random")
    U0 = inputs.ic_four_quadrant(mesh.coords) if dim == 2 else inputs.ic_sphere(mesh.coords)
    a, b = Solver(mesh), Solver(mesh, renumber=True)
    assert a.nnz == b.nnz
    assert a.max_dt(torch.tensor(U0, device="cuda")) == b.max_dt(torch.tensor(U0, device="cuda"))
    Ma, Mb = a.matrices(), b.matrices()
    for k in Ma:
        assert np.array_equal(Ma[k], Mb[k]), k
    tau = a.max_dt(torch.tensor(U0, device="cuda"))
    Ea, _ = a.euler_stage(torch.tensor(U0, device="cuda"), tau)
    Eb, _ = b.euler_stage(torch.tensor(U0, device="cuda"), tau)
    assert np.array_equal(Ea.cpu().numpy(), Eb.cpu().numpy())
    for what in (capi.IDP_DBG_D, capi.IDP_DBG_ALPHA, capi.IDP_DBG_R, capi.IDP_DBG_UL,
                 capi.IDP_DBG_BOUNDS, capi.IDP_DBG_L1, capi.IDP_DBG_L2, capi.IDP_DBG_UPASS,
                 capi.IDP_DBG_TAUI):
        assert np.array_equal(a.debug(what), b.debug(what)), what
    o = oracle_mod.Oracle(mesh, dirichlet=mesh.boundary)
    Ua, Ub, Uo = torch.tensor(U0, device="cuda"), torch.tensor(U0, device="cuda"), U0.copy()
    for _ in range(3):
        dta, sta = a.step(Ua)
        dtb, stb = b.step(Ub)
        Uo, dto, sto = o.step(Uo)
        assert dta == dtb == dto and sta == stb == sto
        assert np.array_equal(Ub.cpu().numpy(), Uo)
    assert np.array_equal(Ua.cpu().numpy(), Ub.cpu().numpy())
    # the adjoint entry points in the caller's numbering, bit for bit
    W = torch.tensor(np.random.default_rng(9).normal(size=U0.shape), device="cuda")
    U = torch.tensor(U0, device="cuda")
    assert np.array_equal(a.euler_stage_vjp(U, tau, W).cpu().numpy(),
                          b.euler_stage_vjp(U, tau, W).cpu().numpy())
    assert np.array_equal(a.step_vjp(U, tau, W).cpu().numpy(), b.step_vjp(U, tau, W).cpu().numpy())
    dts = [0.5 * tau] * 5
    Va, Vb = torch.tensor(U0, device="cuda"), torch.tensor(U0, device="cuda")
    a.forward_checkpoints(Va, dts, 2)
    b.forward_checkpoints(Vb, dts, 2)
    assert np.array_equal(Va.cpu().numpy(), Vb.cpu().numpy())
    assert np.array_equal(a.adjoint_checkpoints(dts, 2, W).cpu().numpy(),
                          b.adjoint_checkpoints(dts, 2, W).cpu().numpy())
    a.close()
    b.close()


def test_determinism(torch):
    announce("determinism: two runs, sphere 3D 13^3")
    mesh = inputs.q1_grid(13, 3, 0.2, seed=0, order="random")
    U0 = inputs.ic_sphere(mesh.coords)
    outs = []
    for _ in range(2):
        s = solver(mesh)
        U = torch.tensor(U0, device="cuda")
        for _ in range(4):
            s.step(U)
        outs.append(U.cpu().numpy())
        s.close()
    assert np.array_equal(outs[0], outs[1])


def test_error_paths(torch):
    announce("error codes: state, dt, mesh, arguments")
    mesh, U0 = inputs.workload("four_quadrant_2d", n=9)
    s = solver(mesh)
    U = torch.tensor(U0, device="cuda")
    dt = s.max_dt(U)
    bad = U0.copy()
    bad[5, 0] = -1.0
    Ub = torch.tensor(bad, device="cuda")
    with pytest.raises(capi.IdpError) as ei:
        s.step(Ub)
    assert ei.value.code == capi.IDP_ESTATE
    assert np.array_equal(Ub.cpu().numpy(), bad)           # untouched
    with pytest.raises(capi.IdpError) as ei:
        s.step(U, dt=2.01 * dt)                              # dt > m_i/(-2 d_ii)
    assert ei.value.code == capi.IDP_EDT
    assert np.array_equal(U.cpu().numpy(), U0)
    used, st = s.step(U, dt=0.5 * dt)                        # still usable
    assert used == 0.5 * dt and st == 0
    with pytest.raises(ValueError):
        s.step(U[:, :2].contiguous())
    with pytest.raises(capi.IdpError) as ei:
        s.max_dt(Ub)
    assert ei.value.code == capi.IDP_ESTATE
    s.close()
    cells = mesh.cells.copy()
    cells[2] = cells[2][[1, 0, 3, 2]]
    with pytest.raises(capi.IdpError) as ei:
        solver(None, dim=2, coords=mesh.coords, cells=cells)
    assert ei.value.code == capi.IDP_EMESH
    cells[2, 0] = mesh.n_nodes + 5
    with pytest.raises(capi.IdpError) as ei:
        solver(None, dim=2, coords=mesh.coords, cells=cells)
    assert ei.value.code == capi.IDP_EINVAL


def test_async_steps_and_status(torch, oracle_mod):
    announce("asynchronous steps on the torch stream")
    mesh, U0 = inputs.workload("four_quadrant_2d", n=17)
    s = solver(mesh, asynchronous=True)
    U = torch.tensor(U0, device="cuda")
    for _ in range(5):
        s.step(U)
    assert s.status() == 0
    o = oracle_mod.Oracle(mesh)
    Uo = U0
    for _ in range(5):
        Uo, _, _ = o.step(Uo)
    assert np.array_equal(U.cpu().numpy(), Uo)
    s.close()


def test_layout_tuner_returns_a_candidate_and_candidates_agree(torch):
    announce("layout autotuner: 3D 17^3 Morton, sigma x staging")
    from paper_2007_00094_amd.solver import tune_layout
    mesh = inputs.q1_grid(17, 3, 0.2, seed=0, order="morton")
    U0 = inputs.ic_mach3_blobs(mesh.coords)
    best, times = tune_layout(mesh, U0, steps=1)
    assert len(times) == 4 and (best["sell_sigma"], best["staging"]) in times
    assert all(t > 0 for t in times.values())
