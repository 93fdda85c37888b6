"""The reference adjoint (oracle/adjoint_ref.py, torch autograd of a plain
restatement of the scheme) pinned to the C oracle and to finite differences.

Finite differences of this scheme are only meaningful where no discrete
decision flips between the +eps and -eps runs: the bounds of Section 3.9
are as tight as the local spread of the solution, so in nearly uniform
regions (a far field that differs from its neighbours by 1e-9) a
white-noise perturbation of 1e-7 moves every limiter and max/min decision.
The checks therefore perturb with smooth, localised directions (sums of
Gaussian bumps).
"""
import numpy as np
import pytest
import torch

from paper_2007_00094_amd import inputs


@pytest.fixture(scope="module")
def ref_mod():
    from oracle import adjoint_ref
    return adjoint_ref


def flow_blobs(n, u0=(0.31, 0.17, 0.07)):
    m, _ = inputs.workload("adjoint_3d", n=n)
    rho = 1.0 + 0.1 * inputs.gaussian_blobs(m.coords, 2, lo=0.2, hi=0.8)
    U0 = inputs.conserved(rho, np.tile(np.asarray(u0), (m.n_nodes, 1)), rho.copy())
    return m, U0


def bump_directions(mesh, count, seed, comps=(0,)):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        v = np.zeros((mesh.n_nodes, mesh.dim + 2))
        for _ in range(2):
            c = rng.uniform(0.3, 0.7, size=mesh.dim)
            bump = np.exp(-np.sum((mesh.coords - c) ** 2, 1) / (2 * 0.1 ** 2))
            for k in comps:
                v[:, k] += rng.normal() * bump
        out.append(v)
    return out


@pytest.mark.parametrize("case", ["four_quadrant_2d", "adjoint_3d_flow"])
def test_reference_stage_and_steps_match_the_oracle(oracle_mod, ref_mod, case):
    if case == "four_quadrant_2d":
        m, U0 = inputs.workload("four_quadrant_2d", n=17, order="random")
    else:
        m, U0 = flow_blobs(9)
    o = oracle_mod.Oracle(m, dirichlet=m.boundary)
    ref = ref_mod.Reference(o, dirichlet=m.boundary)
    tau = o.max_dt(U0)
    E_c, _ = o.euler_stage(U0, tau)
    assert (o.l1() < 1.0).any()                 # the limiter acts
    E_t = ref.stage(torch.tensor(U0), tau).numpy()
    assert np.abs(E_t - E_c).max() <= 1e-12 * np.abs(E_c).max()
    U, Ut = U0.copy(), torch.tensor(U0)
    for _ in range(3):
        U, dt, st = o.step(U)
        assert st == 0
        Ut = ref.step(Ut, dt)
    assert np.abs(Ut.numpy() - U).max() <= 1e-11 * np.abs(U).max()


def test_reference_gradient_matches_central_differences_of_the_oracle(oracle_mod, ref_mod):
    """J = kinetic energy in [0.3, 0.7]^3 after 2 steps with frozen dt;
    gradient w.r.t. the initial density (E fixed) against central
    differences of the C oracle along smooth directions."""
    m, U0 = flow_blobs(13)
    o = oracle_mod.Oracle(m, dirichlet=m.boundary)
    ref = ref_mod.Reference(o, dirichlet=m.boundary)
    U, dts = U0.copy(), []
    for _ in range(2):
        U, dt, _ = o.step(U)
        dts.append(dt)
    mi = torch.tensor(o.m_i())

    def J_oracle(U0x):
        U = U0x.copy()
        for dt in dts:
            U, _, st = o.step(U, dt)
            assert st == 0
        return ref_mod.kinetic_energy_in_box(torch.tensor(U), m.coords, mi, 0.3, 0.7).item()

    rho0 = torch.tensor(U0[:, 0].copy(), requires_grad=True)
    Ut = torch.cat([rho0[:, None], torch.tensor(U0[:, 1:])], 1)
    for dt in dts:
        Ut = ref.step(Ut, dt)
    ref_mod.kinetic_energy_in_box(Ut, m.coords, mi, 0.3, 0.7).backward()
    g = rho0.grad.numpy()

    def fd(v, eps):
        Up, Um = U0.copy(), U0.copy()
        Up[:, 0] += eps * v
        Um[:, 0] -= eps * v
        return (J_oracle(Up) - J_oracle(Um)) / (2 * eps)

    smooth = 0
    for v in bump_directions(m, 4, seed=11):
        v = v[:, 0] * (1 - m.boundary)
        f7, f8 = fd(v, 1e-7), fd(v, 1e-8)
        if abs(f7 - f8) > 1e-5 * abs(f7):
            continue            # a decision flips inside +-eps: no derivative to compare
        smooth += 1
        assert abs(f7 - g @ v) <= 2e-5 * abs(f7), (f7, g @ v)
    assert smooth >= 3


def test_low_order_part_derivative_matches_finite_differences(oracle_mod, ref_mod):
    """With the limiter switched off (l = 0: the low-order update), the
    stage is smooth; its autograd VJP against central differences."""
    m, U0 = flow_blobs(9)
    o = oracle_mod.Oracle(m, dirichlet=m.boundary)

    class LowOrder(ref_mod.Reference):
        def limiter(self, U, P, rmin, rmax, phimin):
            return torch.zeros_like(U[:, 0])

    ref = LowOrder(o, dirichlet=m.boundary)
    tau = o.max_dt(U0)
    rng = np.random.default_rng(3)
    W = torch.tensor(rng.normal(size=U0.shape))
    U = torch.tensor(U0, requires_grad=True)
    (W * ref.stage(U, tau)).sum().backward()
    g = U.grad.numpy()
    for k in range(3):
        v = rng.normal(size=U0.shape) * (1 - m.boundary)[:, None]
        f = [(W * ref.stage(torch.tensor(U0 + s * 1e-6 * v), tau)).sum().item() for s in (1, -1)]
        fd = (f[0] - f[1]) / 2e-6
        assert abs(fd - (g * v).sum()) <= 1e-7 * abs((g * v).sum()), k


def test_limiter_derivative_matches_the_oracle_limiter(oracle_mod, ref_mod):
    """Unrolled Alg. 2/3 derivative (the Newton branch, entropy bound
    active) against central differences of the C oracle's scalar limiter."""
    m, _ = flow_blobs(5)
    o = oracle_mod.Oracle(m)
    ref = ref_mod.Reference(o)
    rng = np.random.default_rng(7)
    g = 1.4
    found = 0
    for _ in range(4000):
        rho = rng.uniform(0.5, 2.0)
        vel = rng.normal(size=3) * 0.5
        p = rng.uniform(0.5, 2.0)
        U = inputs.conserved(np.array([rho]), vel[None, :], np.array([p]))[0]
        P = rng.normal(size=5) * 0.3
        phi_u = p / (g - 1) * rho ** (-g)
        bnd = np.array([rho * 0.5, rho * 1.5, phi_u * rng.uniform(0.9, 0.999)])
        t = oracle_mod.limiter(U, P, bnd)
        if not (0.05 < t < 0.95):
            continue
        # smooth locally: two step sizes agree
        x = np.concatenate([U, P, bnd])

        def fo(xx):
            return oracle_mod.limiter(xx[:5], xx[5:10], xx[10:])

        direc = rng.normal(size=13)
        fd1 = (fo(x + 1e-7 * direc) - fo(x - 1e-7 * direc)) / 2e-7
        fd2 = (fo(x + 1e-8 * direc) - fo(x - 1e-8 * direc)) / 2e-8
        if abs(fd1 - fd2) > 1e-5 * max(abs(fd1), 1e-3):
            continue
        xt = torch.tensor(x, requires_grad=True)
        tt = ref.limiter(xt[None, :5], xt[None, 5:10], xt[10:11], xt[11:12], xt[12:13])
        assert abs(tt.item() - t) <= 1e-14
        tt.sum().backward()
        ad = (xt.grad.numpy() * direc).sum()
        assert abs(ad - fd1) <= 1e-5 * max(abs(fd1), 1e-3), (ad, fd1)
        found += 1
        if found == 20:
            break
    assert found >= 10
