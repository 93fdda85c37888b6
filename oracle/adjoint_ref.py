"""Reference adjoint of the IDP Q1 Euler scheme -- test infrastructure only.

Only tests (and the benchmark's CPU baseline) may use this module; the
library never does.

A plain PyTorch restatement (CPU, float64) of one limited forward-Euler
stage (Alg. 1 with the readings the C oracle implements) and of the SSP-RK3
step with a given time step, vectorised over the stencil entries instead of
looping row by row.  torch.autograd differentiates it: that is the reference
gradient the hand-written HIP adjoint is checked against.  Where the
forward takes a max, a min, a clamp or a branch, the derivative follows the
branch the forward took; at an exact tie it follows the branch the
forward's comparison picks (the later operand of max(a, b) = a > b ? a : b).
The limiter's Newton iterations (Alg. 2/3) are unrolled with masks, so
their derivative is the derivative of the iterates, not of the exact root.

The graph and the matrices m_ij, c_ij, m_i, lambda_i are taken from the C
oracle (Section 3.1-3.2); everything else is recomputed here.  Pinned by
tests/test_oracle_adjoint.py: its stages agree with the C oracle's to
rounding, and its gradients agree with central differences of the C
oracle's steps.
"""
from __future__ import annotations

import numpy as np
import torch

_T = torch.float64


def _pos(x):
    return 0.5 * (torch.abs(x) + x)


def _neg(x):
    return 0.5 * (torch.abs(x) - x)


def _safe(den, ok):
    """den where ok, else 1 (keeps unused branches finite under autograd)."""
    return torch.where(ok, den, torch.ones_like(den))


class Reference:
    """Forward stage / step of one mesh in torch, for autograd.

    oracle_obj: an ``oracle.Oracle`` of the mesh (graph and matrices).
    """

    def __init__(self, oracle_obj, *, dirichlet=None, gamma=1.4, passes=2,
                 newton_max=2, newton_tol=1e-10):
        o = oracle_obj
        self.dim, self.nc, self.n = o.dim, o.nc, o.n
        self.g = float(gamma)
        self.passes, self.newton_max, self.tol = int(passes), int(newton_max), float(newton_tol)
        rp = o.row_ptr()
        col = o.col()
        tpos = o.tpos()
        rows = np.repeat(np.arange(o.n), np.diff(rp))
        I = torch.tensor(rows)
        J = torch.tensor(col)
        self.I, self.J = I, J
        self.cij = torch.tensor(o.c_ij(), dtype=_T)
        mij = torch.tensor(o.m_ij(), dtype=_T)
        self.mi = torch.tensor(o.m_i(), dtype=_T)
        self.lam = torch.tensor(o.lam(), dtype=_T)
        off = I != J
        eo = torch.nonzero(off).flatten()
        where_off = torch.full((len(rows),), -1, dtype=torch.long)
        where_off[eo] = torch.arange(len(eo))
        self.Io, self.Jo = I[eo], J[eo]
        self.To = where_off[torch.tensor(tpos)[eo]]      # transposed off-diagonal entry
        self.co = self.cij[eo]
        self.cto = self.cij[torch.tensor(tpos)[eo]]     # c_ji
        # c_ij + c_ji is the boundary integral of phi_i phi_j n: zero up to
        # rounding unless both nodes lie on the boundary
        self.mirror = (torch.abs(self.co + self.cto).sum(1)
                       <= 2.0 ** -36 * (torch.abs(self.co) + torch.abs(self.cto)).sum(1))
        self.mo = mij[eo]
        if dirichlet is None:
            dirichlet = np.zeros(o.n, dtype=bool)
        self.hold = torch.tensor(np.asarray(dirichlet, dtype=bool))

    # ------------------------------------------------------------ nodes
    def node(self, U):
        """Section 2 per node: rho, m, E, eps, p, c, eta/rho, phi, eta', v, f."""
        D, g = self.dim, self.g
        rho, m, E = U[:, 0], U[:, 1:1 + D], U[:, D + 1]
        eps = E - 0.5 * (m * m).sum(1) / rho
        p = (g - 1.0) * eps
        c = torch.sqrt(g * p / rho)
        re = rho * eps
        er = re ** (1.0 / (g + 1.0)) / rho
        phi = eps * rho ** (-g)
        fac = re ** (-g / (g + 1.0)) / (g + 1.0)
        etap = torch.cat([(fac * E)[:, None], -fac[:, None] * m, (fac * rho)[:, None]], 1)
        v = m / rho[:, None]
        rows = [m]
        for a in range(D):
            rows.append(v * m[:, a:a + 1] + p[:, None] * torch.eye(D, dtype=_T)[a])
        rows.append(v * (E + p)[:, None])
        F = torch.stack(rows, 1)                       # [n, nc, D]
        return dict(rho=rho, m=m, E=E, p=p, c=c, er=er, phi=phi, etap=etap, F=F)

    # --------------------------------------------------- wave-speed bound
    def lambda_max(self, nv, Ai, Aj, ia, ja):
        """Section 3.7 two-rarefaction bound for the projected states."""
        g = self.g
        rho_i, rho_j = Ai["rho"][ia], Aj["rho"][ja]
        p_i, p_j = Ai["p"][ia], Aj["p"][ja]
        c_i, c_j = Ai["c"][ia], Aj["c"][ja]
        ui = (nv * Ai["m"][ia]).sum(1) / rho_i
        uj = (nv * Aj["m"][ja]).sum(1) / rho_j
        num = c_i + c_j - 0.5 * (g - 1.0) * (uj - ui)
        den = c_i * (p_i / p_j) ** (-(g - 1.0) / (2.0 * g)) + c_j
        ptil = p_j * (_pos(num) / den) ** (2.0 * g / (g - 1.0))
        pmax = torch.where(p_i > p_j, p_i, p_j)

        def branch(rho, ps, cs, pp):
            shock = 1.4142135623730951 * (pp - ps) / torch.sqrt(
                rho * ((g + 1.0) * pp + (g - 1.0) * ps))
            raref = ((pp / ps) ** ((g - 1.0) / (2.0 * g)) - 1.0) * 2.0 * cs / (g - 1.0)
            return torch.where(pp >= ps, shock, raref)

        psi = branch(rho_i, p_i, c_i, pmax) + branch(rho_j, p_j, c_j, pmax) + uj - ui
        pstar = torch.where(psi < 0.0, ptil, torch.where(pmax < ptil, pmax, ptil))
        f = (g + 1.0) / (2.0 * g)
        lam1 = ui - c_i * torch.sqrt(1.0 + f * _pos((pstar - p_i) / p_i))
        lam3 = uj + c_j * torch.sqrt(1.0 + f * _pos((pstar - p_j) / p_j))
        a, b = _neg(lam1), _pos(lam3)
        return torch.where(a > b, a, b)

    # ----------------------------------------------------------- limiter
    def _psi(self, U, P, t, phimin):
        g, D = self.g, self.dim
        V = U + t[:, None] * P
        rho, E = V[:, 0], V[:, D + 1]
        m2 = (V[:, 1:1 + D] * V[:, 1:1 + D]).sum(1)
        mP = (V[:, 1:1 + D] * P[:, 1:1 + D]).sum(1)
        rg1 = rho ** (g + 1.0)
        psi = rho * E - 0.5 * m2 - phimin * rg1
        dpsi = P[:, 0] * E + rho * P[:, D + 1] - mP - phimin * (g + 1.0) * (rg1 / rho) * P[:, 0]
        return psi, dpsi

    @staticmethod
    def _newton(tL, tR, psiL, psiR, dpsiL, dpsiR, rhoP):
        """Alg. 3 (sign -1) with the oracle's readings."""
        eps = 2.220446049250313e-16
        scaling = 1.0 / (tR - tL + eps)
        d12 = (psiR - psiL) * scaling
        d112 = (d12 - dpsiL) * scaling
        d122 = (dpsiR - d12) * scaling
        LL = dpsiL * dpsiL - 4.0 * psiL * d112
        LR = dpsiR * dpsiR - 4.0 * psiR * d122
        LL = torch.where(LL < 0.0, torch.zeros_like(LL), LL)
        LR = torch.where(LR < 0.0, torch.zeros_like(LR), LR)
        sL = torch.where(LL > 0.0, torch.sqrt(_safe(LL, LL > 0.0)), torch.zeros_like(LL))
        sR = torch.where(LR > 0.0, torch.sqrt(_safe(LR, LR > 0.0)), torch.zeros_like(LR))
        denL, denR = dpsiL - sL, dpsiR - sR
        rootL = torch.where(denL != 0.0, tL - 2.0 * psiL / _safe(denL, denL != 0.0), tL)
        rootR = torch.where(denR != 0.0, tR - 2.0 * psiR / _safe(denR, denR != 0.0), tR)
        up = rhoP >= 0.0
        nl = torch.where(up, rootL, rootR)
        nr = torch.where(up, rootR, rootL)
        nl = torch.where(~(nl >= tL), tL, nl)
        nl = torch.where(~(nl <= tR), tR, nl)
        nr = torch.where(~(nr <= tR), tR, nr)
        nr = torch.where(~(nr >= tL), tL, nr)
        nr = torch.where(nr < nl, nl, nr)
        return nl, nr

    def limiter(self, U, P, rmin, rmax, phimin):
        """Alg. 2 for many (U, P, bounds) at once; returns t_L."""
        rhoU, rhoP = U[:, 0], P[:, 0]
        zero, one = torch.zeros_like(rhoU), torch.ones_like(rhoU)
        tL, tR = zero, one
        nz = rhoP != 0.0
        absP = _safe(torch.abs(rhoP), nz)
        up = rhoU + tR * rhoP > rmax
        tR = torch.where(up, torch.where(nz, torch.abs(rmax - rhoU) / absP, zero), tR)
        lo = rhoU + tR * rhoP < rmin
        tR = torch.where(lo, torch.where(nz, torch.abs(rmin - rhoU) / absP, zero), tR)
        tR = torch.where(tR > 1.0, one, tR)
        tR = torch.where(tR < 0.0, zero, tR)
        active = torch.ones_like(rhoU, dtype=torch.bool)
        for _ in range(self.newton_max):
            psiR, dpsiR = self._psi(U, P, tR, phimin)
            done = active & (psiR >= 0.0)
            tL = torch.where(done, tR, tL)
            active = active & ~done
            psiL, dpsiL = self._psi(U, P, tL, phimin)
            active = active & ~(psiL <= self.tol)
            nl, nr = self._newton(tL, tR, psiL, psiR, dpsiL, dpsiR, rhoP)
            tL = torch.where(active, nl, tL)
            tR = torch.where(active, nr, tR)
        # a direction below 2^-40 of its state is rounding noise: the
        # coefficient is taken as locally constant there (its branches are
        # decided by rounding; the hand-written adjoint does the same)
        noise = torch.amax(torch.abs(P), 1) <= 2.0 ** -40 * torch.amax(torch.abs(U), 1)
        return torch.where(noise, tL.detach(), tL)

    # ------------------------------------------------------------- stage
    def stage(self, U, tau, keep=None):
        """E(U): one limited forward-Euler update with step tau (Alg. 1).
        keep (a dict, optional) receives the intermediates (U^L, R, the
        bounds, alpha, d per off-diagonal entry), gradients retained."""
        D, n, g = self.dim, self.n, self.g
        I, J, Io, Jo, To = self.I, self.J, self.Io, self.Jo, self.To
        A = self.node(U)
        # step 1: graph viscosity, both orientations (Section 3.3, 3.7)
        aij = torch.sqrt((self.co * self.co).sum(1))
        aji = torch.sqrt((self.cto * self.cto).sum(1))
        nij = self.co / _safe(aij, aij > 0)[:, None]
        nji = self.cto / _safe(aji, aji > 0)[:, None]
        t1 = torch.where(aij > 0, self.lambda_max(nij, A, A, Io, Jo) * aij, torch.zeros_like(aij))
        t2 = torch.where(aji > 0, self.lambda_max(nji, A, A, Jo, Io) * aji, torch.zeros_like(aji))
        # where c_ji = -c_ij the two problems mirror each other: the pair's
        # lower node id gives the one orientation evaluated
        d = torch.where(self.mirror, torch.where(Io < Jo, t1, t2), torch.where(t1 > t2, t1, t2))
        # step 2: indicator over all j in I(i) (Section 3.8)
        mc = (A["m"][J] * self.cij).sum(1)
        a = torch.zeros(n, dtype=_T).index_add(0, I, (A["er"][J] - A["er"][I]) * mc)
        fdall = ((A["F"][J] - A["F"][I]) * self.cij[:, None, :]).sum(2)
        b = torch.zeros(n, self.nc, dtype=_T).index_add(0, I, fdall)
        er = A["er"]
        N = torch.abs(a - (A["etap"] * b).sum(1) + er * b[:, 0])
        shift = torch.zeros_like(A["etap"])
        shift[:, 0] = 1.0
        Dn = torch.abs(a) + (torch.abs(A["etap"] - shift * er[:, None]) * torch.abs(b)).sum(1)
        alpha = torch.where(Dn > 0, N / _safe(Dn, Dn > 0), torch.zeros_like(Dn))
        # step 3: low-order update, bar states, bounds
        fd = fdall[I != J]
        dU = U[Jo] - U[Io]
        dH = d * (alpha[Io] + alpha[Jo]) / 2.0
        R = torch.zeros(n, self.nc, dtype=_T).index_add(0, Io, -fd + dH[:, None] * dU)
        Lw = torch.zeros(n, self.nc, dtype=_T).index_add(0, Io, -fd + d[:, None] * dU)
        UL = U + (tau / self.mi)[:, None] * Lw
        rho = A["rho"]
        rbar = 0.5 * (rho[Io] + rho[Jo]) - torch.where(
            d > 0, fd[:, 0] / (2.0 * _safe(d, d > 0)), torch.zeros_like(d))
        rmin = rho.scatter_reduce(0, Io, rbar, "amin", include_self=True)
        rmax = rho.scatter_reduce(0, Io, rbar, "amax", include_self=True)
        phimin = A["phi"].scatter_reduce(0, Io, A["phi"][Jo], "amin", include_self=True)
        if keep is not None:
            for k, v in (("UL", UL), ("R", R), ("rmin", rmin), ("rmax", rmax),
                         ("phimin", phimin), ("alpha", alpha), ("d", d)):
                v.retain_grad()
                keep[k] = v
        # step 4: directions (eq. def-p) and the first pass
        coef = tau / (self.lam[Io] * self.mi[Io])
        bij = -self.mo / self.mi[Jo]
        bji = -self.mo / self.mi[Io]
        P = coef[:, None] * (bij[:, None] * R[Jo] - bji[:, None] * R[Io] + (dH - d)[:, None] * dU)
        lamo = self.lam[Io][:, None]
        if keep is not None:
            P.retain_grad()
            keep["P"] = P
        l1 = self.limiter(UL[Io], P, rmin[Io], rmax[Io], phimin[Io])
        s1 = torch.where(l1 < l1[To], l1, l1[To])
        Up = UL + torch.zeros(n, self.nc, dtype=_T).index_add(0, Io, lamo * s1[:, None] * P)
        if self.passes < 2:
            return Up
        # steps 5-6: second pass on the rescaled directions
        P2 = (1.0 - s1)[:, None] * P
        l2 = self.limiter(Up[Io], P2, rmin[Io], rmax[Io], phimin[Io])
        s2 = torch.where(l2 < l2[To], l2, l2[To])
        return Up + torch.zeros(n, self.nc, dtype=_T).index_add(0, Io, lamo * s2[:, None] * P2)

    def step(self, U, dt):
        """SSP-RK3 in increment form with a given dt; held nodes keep U^n."""
        h = self.hold[:, None]
        U1 = torch.where(h, U, self.stage(U, dt))
        U2 = torch.where(h, U, U + 0.25 * (self.stage(U1, dt) - U))
        return torch.where(h, U, U + (2.0 / 3.0) * (self.stage(U2, dt) - U))


def kinetic_energy_in_box(U, coords, mi, lo=0.4, hi=0.6, dim=3):
    """J = sum over nodes x_i in [lo, hi]^dim of m_i |m|^2 / (2 rho)."""
    inside = np.all((coords >= lo) & (coords <= hi), axis=1)
    sel = torch.tensor(inside)
    m = U[:, 1:1 + dim]
    ke = (m * m).sum(1) / (2.0 * U[:, 0])
    return (mi * ke * sel).sum()
