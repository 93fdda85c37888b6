"""Pins of the oracle's stencil graph and matrices m_ij, c_ij, m_i (CPU).

Closed forms on uniform grids (tensor products of the 1D P1 mass and
derivative matrices), and identities that hold on any Q1 mesh: partition of
unity (sum_j c_ij = 0), exact reproduction of linear functions
(sum_j c_ij x_j^T = m_i I), total volume, antisymmetry away from the
boundary and the boundary-face mass matrix for boundary pairs.
"""
import itertools

import numpy as np
import pytest

from paper_2007_00094_amd import inputs


def _m1(k, l, n, h):
    if abs(k - l) > 1:
        return 0.0
    if k == l:
        return h / 3.0 if k in (0, n - 1) else 2.0 * h / 3.0
    return h / 6.0


def _c1(k, l, n):
    if abs(k - l) > 1:
        return 0.0
    if k == l:
        if n == 1:
            return 0.0
        return -0.5 if k == 0 else (0.5 if k == n - 1 else 0.0)
    return 0.5 if l == k + 1 else -0.5


@pytest.mark.parametrize("dim,n", [(2, 6), (3, 4)])
@pytest.mark.parametrize("order", ["lex", "random"])
def test_uniform_grid_closed_forms(oracle_mod, dim, n, order):
    mesh = inputs.q1_grid(n, dim, jitter=0.0, order=order, perm_seed=5)
    o = oracle_mod.Oracle(mesh)
    h = 1.0 / (n - 1)
    rp, col, mij, cij = o.row_ptr(), o.col(), o.m_ij(), o.c_ij()
    ijk = mesh.grid_ijk()
    for i in range(o.n):
        row = col[rp[i]:rp[i + 1]]
        assert np.all(np.diff(row) > 0)  # ascending, unique
        # stencil = all nodes within Chebyshev distance 1
        nb = np.nonzero(np.max(np.abs(ijk - ijk[i]), axis=1) <= 1)[0]
        assert set(row.tolist()) == set(nb.tolist())
        for q in range(rp[i], rp[i + 1]):
            j = col[q]
            a, b = ijk[i], ijk[j]
            m = np.prod([_m1(a[k], b[k], n, h) for k in range(dim)])
            assert abs(mij[q] - m) <= 1e-15 * h ** dim
            for k in range(dim):
                c = _c1(a[k], b[k], n) * np.prod(
                    [_m1(a[l], b[l], n, h) for l in range(dim) if l != k])
                assert abs(cij[q, k] - c) <= 1e-15 * h ** (dim - 1)
    assert np.allclose(o.lam()[(ijk.min(1) > 0) & (ijk.max(1) < n - 1)],
                       1.0 / (3 ** dim - 1), rtol=0, atol=0)


@pytest.mark.parametrize("dim,n", [(2, 17), (3, 9)])
def test_jittered_identities(oracle_mod, dim, n):
    mesh = inputs.q1_grid(n, dim, jitter=0.2, seed=4, order="random")
    o = oracle_mod.Oracle(mesh)
    h = 1.0 / (n - 1)
    rp, col, mij, cij, mi = o.row_ptr(), o.col(), o.m_ij(), o.c_ij(), o.m_i()
    tp = o.tpos()
    x = mesh.coords
    assert abs(mi.sum() - 1.0) <= 1e-14
    assert abs(o.volume - 1.0) <= 1e-14
    bnd = mesh.boundary.astype(bool)
    for i in range(o.n):
        sl = slice(rp[i], rp[i + 1])
        js = col[sl]
        # partition of unity
        assert np.max(np.abs(cij[sl].sum(0))) <= 1e-15 * h ** (dim - 1) * 27
        assert abs(mij[sl].sum() - mi[i]) <= 1e-15 * mi[i] * 27
        # linear reproduction: sum_j c_ij x_j^T = m_i I
        G = cij[sl].T @ x[js]
        assert np.max(np.abs(G - mi[i] * np.eye(dim))) <= 1e-13 * mi[i]
        for q in range(rp[i], rp[i + 1]):
            j = col[q]
            assert col[tp[q]] == i
            assert mij[q] == mij[tp[q]]          # symmetric (bitwise)
            if not (bnd[i] and bnd[j]):
                assert np.max(np.abs(cij[q] + cij[tp[q]])) <= 1e-15 * 8 * h ** (dim - 1)


@pytest.mark.parametrize("dim,n", [(2, 9), (3, 6)])
def test_boundary_pairs_face_mass(oracle_mod, dim, n):
    """c_ij + c_ji = integral over the boundary of phi_i phi_j n; boundary
    nodes are not jittered, so on each flat face this is minus/plus the
    uniform (d-1)-dimensional face mass matrix."""
    mesh = inputs.q1_grid(n, dim, jitter=0.2, seed=9, order="lex")
    o = oracle_mod.Oracle(mesh)
    h = 1.0 / (n - 1)
    rp, col, cij, tp = o.row_ptr(), o.col(), o.c_ij(), o.tpos()
    ijk = mesh.grid_ijk()
    for i in range(o.n):
        for q in range(rp[i], rp[i + 1]):
            j = col[q]
            s = cij[q] + cij[tp[q]]
            ref = np.zeros(dim)
            for k in range(dim):
                for side, sgn in ((0, -1.0), (n - 1, 1.0)):
                    if ijk[i, k] == side and ijk[j, k] == side:
                        ref[k] += sgn * np.prod([
                            _m1(ijk[i, l], ijk[j, l], n, h)
                            for l in range(dim) if l != k])
            assert np.max(np.abs(s - ref)) <= 1e-15 * 8 * h ** (dim - 1)


def test_invalid_cell_rejected(oracle_mod):
    mesh = inputs.q1_grid(4, 2, jitter=0.0)
    cells = mesh.cells.copy()
    cells[3] = cells[3][[1, 0, 3, 2]]  # mirrored cell: det J < 0
    with pytest.raises(ValueError, match="-2"):
        oracle_mod.Oracle(dim=2, coords=mesh.coords, cells=cells)
