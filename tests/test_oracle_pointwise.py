"""Pins of the oracle's pointwise building blocks (CPU only).

Each check uses something other than the oracle's own formula: closed forms
of the ideal-gas EOS, finite differences, an exact Riemann solver written
from the textbook construction, and brute-force bisection of the limiter's
admissible interval.
"""
import math

import numpy as np
import pytest

import exact_riemann as er
from paper_2007_00094_amd.inputs import conserved

G = 1.4


def prim_to_U(rho, u, p):
    u = np.atleast_1d(np.asarray(u, dtype=np.float64))
    return conserved(np.array([rho]), u[None, :], np.array([p]))[0]


# ------------------------------------------------------------------ pow

def _ulp_err(a, exact):
    return abs(a - exact) / math.ulp(exact)


def test_pow_against_decimal_reference(oracle_mod):
    """The fixed-method x^y is within a few ulp of the exact power
    (60-digit decimal), over the argument ranges the scheme uses."""
    from decimal import Decimal, getcontext
    getcontext().prec = 60
    rng = np.random.default_rng(41)
    worst = 0.0
    for y in (2.4, -1.4, 1 / 2.4, -1.4 / 2.4, -(0.4) / 2.8, 2.8 / 0.4, 0.5, 1.5 / 3):
        for x in np.concatenate([10 ** rng.uniform(-4, 4, 300), rng.uniform(0.5, 2, 300)]):
            z = y * math.log(x)
            exact = float((Decimal(float(x)).ln() * Decimal(y)).exp())
            err = _ulp_err(oracle_mod.pow_(x, y), exact)
            worst = max(worst, err)
            assert err <= 4.0, (x, y, z, err)
    assert worst <= 4
    # glibc agrees to a few ulp as well; exact cases are exact
    assert oracle_mod.pow_(1.0, 2.4) == 1.0
    assert oracle_mod.pow_(2.0, 3.0) == 8.0
    assert oracle_mod.pow_(4.0, 0.5) == 2.0
    assert math.isnan(oracle_mod.pow_(-1.0, 2.0))


# ------------------------------------------------------------------ EOS

def test_exact_riemann_solver_rankine_hugoniot():
    """Sanity of the test utility itself: Sod data, jump conditions hold
    across the right shock and the star values match Toro's table 4.2."""
    rl, ul, pl, rr, ur, pr = 1.0, 0.0, 1.0, 0.125, 0.0, 0.1
    ps = er.star_pressure(rl, ul, pl, rr, ur, pr)
    assert abs(ps - 0.30313) < 1e-5
    _, us, _ = er.sample(rl, ul, pl, rr, ur, pr, 0.5)
    assert abs(us - 0.92745) < 1e-5
    cr = math.sqrt(G * pr / rr)
    S = ur + cr * math.sqrt((G + 1) / (2 * G) * ps / pr + (G - 1) / (2 * G))
    rs = er.sample(rl, ul, pl, rr, ur, pr, S - 1e-9)[0]
    assert abs(rr * (ur - S) - rs * (us - S)) < 1e-9
    assert abs(rr * ur * (ur - S) + pr - (rs * us * (us - S) + ps)) < 1e-9


@pytest.mark.parametrize("dim", [2, 3])
def test_eos_closed_forms(oracle_mod, dim):
    rng = np.random.default_rng(7)
    for _ in range(200):
        rho = 10 ** rng.uniform(-3, 3)
        p = 10 ** rng.uniform(-3, 3)
        u = rng.uniform(-5, 5, size=dim)
        U = prim_to_U(rho, u, p)
        assert abs(oracle_mod.pressure(U) - p) <= 1e-11 * (p + 0.5 * rho * u @ u)
        c = oracle_mod.speed_of_sound(U)
        assert abs(c * c - G * oracle_mod.pressure(U) / rho) <= 1e-13 * c * c
        eps = p / (G - 1)
        # phi rho^gamma = eps ; eta^(gamma+1) = rho eps
        phi = oracle_mod.specific_entropy(U)
        assert abs(phi * rho ** G - oracle_mod.pressure(U) / (G - 1)) <= 1e-12 * eps
        eta = oracle_mod.harten_entropy(U)
        re = rho * oracle_mod.pressure(U) / (G - 1)
        assert abs(eta ** (G + 1) - re) <= 1e-12 * re


@pytest.mark.parametrize("dim", [2, 3])
def test_entropy_derivative_central_fd(oracle_mod, dim):
    rng = np.random.default_rng(11)
    for _ in range(50):
        U = prim_to_U(rng.uniform(0.2, 3), rng.uniform(-2, 2, size=dim),
                      rng.uniform(0.2, 3))
        d = oracle_mod.harten_entropy_derivative(U)
        for k in range(dim + 2):
            h = 1e-6 * max(1.0, abs(U[k]))
            e = np.zeros(dim + 2)
            e[k] = h
            fd = (oracle_mod.harten_entropy(U + e) - oracle_mod.harten_entropy(U - e)) / (2 * h)
            assert abs(fd - d[k]) <= 1e-7 * max(1.0, abs(d[k]))


# ------------------------------------------------------ wave-speed bound

def _rand_unit(rng, dim):
    n = rng.normal(size=dim)
    return n / np.linalg.norm(n)


@pytest.mark.parametrize("dim", [2, 3])
def test_lambda_equal_states(oracle_mod, dim):
    """Equal states: the bound is |u.n| + c exactly."""
    rng = np.random.default_rng(3)
    for _ in range(200):
        n = _rand_unit(rng, dim)
        rho, p = 10 ** rng.uniform(-2, 2), 10 ** rng.uniform(-2, 2)
        u = rng.uniform(-5, 5, size=dim)
        U = prim_to_U(rho, u, p)
        lam, _ = oracle_mod.lambda_max(n, U, U)
        ref = abs(u @ n) + math.sqrt(G * p / rho)
        # p is recovered from E: cancellation grows with kinetic/internal
        amp = 1.0 + 0.5 * rho * (u @ u) / (p / (G - 1))
        assert abs(lam - ref) <= 1e-14 * amp * ref


def _pair(rng, dim):
    rl, rr = 10 ** rng.uniform(-3, 3, size=2)
    pl, pr = 10 ** rng.uniform(-3, 3, size=2)
    ul, ur = rng.uniform(-10, 10, size=(2, dim)) / math.sqrt(dim)
    return rl, ul, pl, rr, ur, pr


@pytest.mark.parametrize("dim", [2, 3])
def test_lambda_is_guaranteed_upper_bound(oracle_mod, dim):
    """Section 3.7: lambda~_max bounds the exact maximal wave speed of the
    projected 1D Riemann problem from above, for any pair of states."""
    rng = np.random.default_rng(5 + dim)
    tight = 0
    for _ in range(3000):
        rl, ul, pl, rr, ur, pr = _pair(rng, dim)
        n = _rand_unit(rng, dim)
        lam, pstar = oracle_mod.lambda_max(n, prim_to_U(rl, ul, pl),
                                           prim_to_U(rr, ur, pr))
        ex, ps_ex = er.max_wave_speed(rl, ul @ n, pl, rr, ur @ n, pr)
        assert lam >= ex * (1 - 1e-12), (lam, ex)
        assert pstar >= ps_ex * (1 - 1e-8)  # p* near vacuum is ill-conditioned
        tight += lam <= ex * (1 + 1e-9)
    assert tight > 100  # the bound is sharp on a good share of pairs


@pytest.mark.parametrize("dim", [2, 3])
def test_lambda_two_rarefaction_is_exact(oracle_mod, dim):
    """If both waves are rarefactions (exact p* <= min(p_L, p_R)) the
    two-rarefaction pressure is the exact star pressure."""
    rng = np.random.default_rng(17)
    hits = 0
    while hits < 300:
        rl, ul, pl, rr, ur, pr = _pair(rng, dim)
        n = _rand_unit(rng, dim)
        ex, ps_ex = er.max_wave_speed(rl, ul @ n, pl, rr, ur @ n, pr)
        # skip near-vacuum fans: p* ~ N^7 with N a cancelling difference
        if not (1e-4 * min(pl, pr) < ps_ex <= min(pl, pr)):
            continue
        hits += 1
        lam, pstar = oracle_mod.lambda_max(n, prim_to_U(rl, ul, pl),
                                           prim_to_U(rr, ur, pr))
        assert abs(pstar - ps_ex) <= 1e-10 * ps_ex
        assert abs(lam - ex) <= 1e-11 * max(ex, 1e-300)


def _lambda_literal_projection(n, Ui, Uj, dim):
    """Section 3.7 evaluated with the projected energy E~ written out
    (numpy, glibc pow), to pin the p~ = p(U) identity used by the oracle."""
    def proj(U):
        rho, m, E = U[0], U[1:dim + 1], U[dim + 1]
        mt = n @ m
        Et = E - (m - mt * n) @ (m - mt * n) / (2 * rho)
        u = mt / rho
        p = (G - 1) * (Et - 0.5 * mt * mt / rho)
        return rho, u, p, math.sqrt(G * p / rho)
    ri, ui, pi, ci = proj(Ui)
    rj, uj, pj, cj = proj(Uj)
    num = ci + cj - 0.5 * (G - 1) * (uj - ui)
    ptil = pj * (max(num, 0.0) / (ci * (pi / pj) ** (-(G - 1) / (2 * G)) + cj)) ** (2 * G / (G - 1))
    pmax = max(pi, pj)

    def f(r, p, c, q):
        if q >= p:
            return math.sqrt(2) * (q - p) / math.sqrt(r * ((G + 1) * q + (G - 1) * p))
        return ((q / p) ** ((G - 1) / (2 * G)) - 1) * 2 * c / (G - 1)
    psi = f(ri, pi, ci, pmax) + f(rj, pj, cj, pmax) + uj - ui
    ps = ptil if psi < 0 else min(pmax, ptil)
    l1 = ui - ci * math.sqrt(1 + (G + 1) / (2 * G) * max((ps - pi) / pi, 0.0))
    l3 = uj + cj * math.sqrt(1 + (G + 1) / (2 * G) * max((ps - pj) / pj, 0.0))
    return max(max(-l1, 0.0), max(l3, 0.0))


@pytest.mark.parametrize("dim", [2, 3])
def test_lambda_matches_literal_projection(oracle_mod, dim):
    rng = np.random.default_rng(43)
    for _ in range(1000):
        rl, ul, pl, rr, ur, pr = _pair(rng, dim)
        if rng.uniform() < 0.5:  # keep part of the sample at moderate Mach
            ul, ur = ul / 10, ur / 10
        n = _rand_unit(rng, dim)
        Ui, Uj = prim_to_U(rl, ul, pl), prim_to_U(rr, ur, pr)
        a, _ = oracle_mod.lambda_max(n, Ui, Uj)
        b = _lambda_literal_projection(n, Ui, Uj, dim)
        amp = 1.0 + max(0.5 * rl * (ul @ ul) / (pl / (G - 1)),
                        0.5 * rr * (ur @ ur) / (pr / (G - 1)))
        assert abs(a - b) <= 1e-12 * amp * a, (a, b)


@pytest.mark.parametrize("dim", [2, 3])
def test_lambda_orientation_and_rotation(oracle_mod, dim):
    """lambda(n, Ui, Uj) = lambda(-n, Uj, Ui), and only u.n matters."""
    rng = np.random.default_rng(23)
    for _ in range(300):
        rl, ul, pl, rr, ur, pr = _pair(rng, dim)
        n = _rand_unit(rng, dim)
        Ui, Uj = prim_to_U(rl, ul, pl), prim_to_U(rr, ur, pr)
        a, _ = oracle_mod.lambda_max(n, Ui, Uj)
        b, _ = oracle_mod.lambda_max(-n, Uj, Ui)
        assert abs(a - b) <= 1e-13 * a
        # rotate everything by a random orthogonal matrix
        Q, _ = np.linalg.qr(rng.normal(size=(dim, dim)))
        c, _ = oracle_mod.lambda_max(Q @ n, prim_to_U(rl, Q @ ul, pl),
                                     prim_to_U(rr, Q @ ur, pr))
        # p is recovered from E: cancellation grows with kinetic/internal
        amp = 1.0 + max(0.5 * rl * (ul @ ul) / (pl / (G - 1)),
                        0.5 * rr * (ur @ ur) / (pr / (G - 1)))
        assert abs(a - c) <= 1e-13 * amp * a


# --------------------------------------------------------------- limiter

def _psi(U, dim, phi_min):
    rho = U[0]
    re = rho * U[dim + 1] - 0.5 * U[1:dim + 1] @ U[1:dim + 1]
    return re - phi_min * rho ** (G + 1)


def _admissible(U, P, t, b, dim):
    V = U + t * P
    return b[0] <= V[0] <= b[1] and _psi(V, dim, b[2]) >= 0.0


def _bisect(U, P, b, dim):
    if _admissible(U, P, 1.0, b, dim):
        return 1.0
    lo, hi = 0.0, 1.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if _admissible(U, P, mid, b, dim):
            lo = mid
        else:
            hi = mid
    return lo


def _limiter_case(rng, dim):
    rho = rng.uniform(0.2, 2.0)
    p = rng.uniform(0.1, 2.0)
    u = rng.uniform(-1.5, 1.5, size=dim)
    U = prim_to_U(rho, u, p)
    phi = (p / (G - 1)) * rho ** (-G)
    b = np.array([rho * (1 - rng.uniform(0, 0.2)), rho * (1 + rng.uniform(0, 0.2)),
                  phi * (1 - rng.uniform(0, 0.1))])
    P = rng.normal(size=dim + 2) * np.abs(U) * rng.uniform(0.01, 1.0)
    return U, P, b


@pytest.mark.parametrize("dim", [2, 3])
def test_limiter_inside_bounds_returns_one(oracle_mod, dim):
    rng = np.random.default_rng(29)
    n = 0
    while n < 200:
        U, P, b = _limiter_case(rng, dim)
        P *= 1e-3
        if not _admissible(U, P, 1.0, b, dim):
            continue
        n += 1
        assert oracle_mod.limiter(U, P, b) == 1.0


@pytest.mark.parametrize("dim", [2, 3])
def test_limiter_against_bisection(oracle_mod, dim):
    """Alg. 2 returns an admissible t (density in bounds, Psi >= 0 up to
    rounding) that does not exceed the true largest admissible t, and with
    Newton iterations it gets close to it."""
    rng = np.random.default_rng(31 + dim)
    gaps = []
    for _ in range(2000):
        U, P, b = _limiter_case(rng, dim)
        t = oracle_mod.limiter(U, P, b, newton_max=2, tol=1e-10)
        ttrue = _bisect(U, P, b, dim)
        assert 0.0 <= t <= 1.0
        assert t <= ttrue + 1e-12
        V = U + t * P
        assert V[0] >= b[0] * (1 - 1e-12) and V[0] <= b[1] * (1 + 1e-12)
        assert _psi(V, dim, b[2]) >= -1e-12 * abs(V[0] * V[dim + 1])
        gaps.append(ttrue - t)
        # with many Newton steps the gap closes (tol-limited)
        t8 = oracle_mod.limiter(U, P, b, newton_max=8, tol=0.0)
        assert t8 <= ttrue + 1e-12
        assert ttrue - t8 <= 1e-6
    gaps = np.array(gaps)
    assert np.median(gaps) <= 1e-6


def test_limiter_swapped_roots_keep_admissibility(oracle_mod):
    """For rho(P) < 0 the third derivative of Psi along the line is
    positive; the swapped-root reading of Alg. 3 stays admissible where the
    unswapped form can step past the root."""
    rng = np.random.default_rng(37)
    dim = 3
    viol_literal = 0
    for _ in range(3000):
        U, P, b = _limiter_case(rng, dim)
        if P[0] >= 0:
            P[0] = -P[0]
        t = oracle_mod.limiter(U, P, b, newton_max=3, tol=0.0)
        V = U + t * P
        assert _psi(V, dim, b[2]) >= -1e-12 * abs(V[0] * V[dim + 1])
        tl = oracle_mod.limiter(U, P, b, newton_max=3, tol=0.0, literal=True)
        Vl = U + tl * P
        viol_literal += _psi(Vl, dim, b[2]) < -1e-12 * abs(Vl[0] * Vl[dim + 1])
    # report, do not require: the literal form is the unsafe variant
    print("literal Alg. 3 violations:", viol_literal)
