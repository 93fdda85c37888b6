"""Seeded synthetic inputs: jittered Q1 meshes, node orderings, initial states.

This module is shared by the HIP path's tests/bench and by the CPU oracle's
tests.  It holds no arithmetic of the numerical scheme: it only builds the
mesh (node coordinates, cell connectivity, Dirichlet flags) and the initial
conserved state U = (rho, m, E) of each workload.

Conventions (the paper fixes none of them; they define the workloads):
  * domain [0,1]^d, ``n`` nodes per side, h = 1/(n-1);
  * lexicographic grid id  g = ix + n*iy (+ n*n*iz);
  * interior nodes are jittered by independent U(-jitter*h, jitter*h) per
    coordinate (boundary nodes stay on the boundary);
  * a cell lists its 2^d vertices in lexicographic reference order
    b = bx + 2*by (+ 4*bz), vertex b sitting at reference corner (bx,by,bz);
  * node ordering: 'lex', 'random' (seeded permutation) or 'morton'
    (Z-order of the integer grid coordinates);
  * conserved state per node in the order (rho, m_1..m_d, E),
    E = p/(gamma-1) + rho|u|^2/2 (ideal gas, gamma = 7/5 by default).
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

GAMMA = 1.4


@dataclass
class Mesh:
    dim: int
    n_side: int
    coords: np.ndarray      # [N, dim] float64
    cells: np.ndarray       # [Nc, 2^dim] int64
    boundary: np.ndarray    # [N] uint8, 1 = node on the domain boundary
    grid_id: np.ndarray     # [N] int64, lexicographic grid id of each node

    @property
    def n_nodes(self) -> int:
        return int(self.coords.shape[0])

    @property
    def n_cells(self) -> int:
        return int(self.cells.shape[0])

    def grid_ijk(self) -> np.ndarray:
        """Integer grid coordinates [N, dim] of every node."""
        g = self.grid_id
        n = self.n_side
        out = np.empty((g.shape[0], self.dim), dtype=np.int64)
        for k in range(self.dim):
            out[:, k] = g % n
            g = g // n
        return out


def _spread_bits(v: np.ndarray, dim: int) -> np.ndarray:
    """Insert (dim-1) zero bits between the low 21 bits of v (uint64)."""
    v = v.astype(np.uint64)
    out = np.zeros_like(v)
    for b in range(21):
        out |= ((v >> np.uint64(b)) & np.uint64(1)) << np.uint64(b * dim)
    return out


def morton_order(ijk: np.ndarray) -> np.ndarray:
    """Old ids sorted by Z-order (Morton) code of integer coordinates."""
    dim = ijk.shape[1]
    code = np.zeros(ijk.shape[0], dtype=np.uint64)
    for k in range(dim):
        code |= _spread_bits(ijk[:, k], dim) << np.uint64(k)
    return np.argsort(code, kind="stable")


def q1_grid(n: int, dim: int, jitter: float = 0.2, seed: int = 0,
            order: str = "lex", perm_seed: int = 1, warp: float = 0.0) -> Mesh:
    """Structured Q1 grid of n^dim nodes on [0,1]^dim with seeded jitter.

    ``order`` picks the node numbering handed to the solver; the cells are
    emitted in lexicographic cell order with vertices renumbered.  ``warp``
    adds a smooth displacement that vanishes on the boundary: coordinate k
    moves by warp * prod_l sin(pi x_l) * sin(2 pi x_(k+1 mod d)), so the
    cells stay images of a smooth map (convergence studies need this; a
    random jitter is a rough map).
    """
    if dim not in (2, 3):
        raise ValueError("dim must be 2 or 3")
    if n < 2:
        raise ValueError("n must be >= 2")
    h = 1.0 / (n - 1)
    N = n ** dim
    axes = [np.arange(n, dtype=np.int64)] * dim
    grids = np.meshgrid(*axes, indexing="ij")            # grids[k][ix,iy,..]
    # lexicographic id g = ix + n*iy + n^2*iz -> flatten in Fortran order
    ijk = np.stack([gk.reshape(-1, order="F") for gk in grids], axis=1)
    coords = ijk.astype(np.float64) * h
    on_bnd = np.zeros(N, dtype=bool)
    for k in range(dim):
        on_bnd |= (ijk[:, k] == 0) | (ijk[:, k] == n - 1)
    rng = np.random.default_rng(seed)
    if jitter > 0.0:
        off = rng.uniform(-jitter * h, jitter * h, size=(N, dim))
        off[on_bnd] = 0.0
        coords = coords + off
    if warp != 0.0:
        bump = np.prod(np.sin(np.pi * coords), axis=1)
        disp = np.stack([warp * bump * np.sin(2.0 * np.pi * coords[:, (k + 1) % dim])
                         for k in range(dim)], axis=1)
        coords = coords + disp
    # cells, lexicographic cell order, vertex b = bx + 2 by + 4 bz
    cax = [np.arange(n - 1, dtype=np.int64)] * dim
    cg = np.meshgrid(*cax, indexing="ij")
    cijk = np.stack([c.reshape(-1, order="F") for c in cg], axis=1)
    nv = 1 << dim
    cells = np.empty((cijk.shape[0], nv), dtype=np.int64)
    stride = np.array([n ** k for k in range(dim)], dtype=np.int64)
    for b in range(nv):
        bits = np.array([(b >> k) & 1 for k in range(dim)], dtype=np.int64)
        cells[:, b] = (cijk + bits) @ stride
    grid_id = np.arange(N, dtype=np.int64)
    if order == "lex":
        old_of_new = grid_id
    elif order == "random":
        old_of_new = np.random.default_rng(perm_seed).permutation(N)
    elif order == "morton":
        old_of_new = morton_order(ijk)
    else:
        raise ValueError(f"unknown order {order!r}")
    new_of_old = np.empty(N, dtype=np.int64)
    new_of_old[old_of_new] = np.arange(N, dtype=np.int64)
    return Mesh(dim=dim, n_side=n,
                coords=np.ascontiguousarray(coords[old_of_new]),
                cells=np.ascontiguousarray(new_of_old[cells]),
                boundary=on_bnd[old_of_new].astype(np.uint8),
                grid_id=grid_id[old_of_new].copy())


# ---------------------------------------------------------------- states

def conserved(rho, vel, p, gamma: float = GAMMA) -> np.ndarray:
    """Pack primitive (rho, u, p) into conserved (rho, rho*u, E) rows."""
    rho = np.asarray(rho, dtype=np.float64)
    vel = np.asarray(vel, dtype=np.float64)
    p = np.asarray(p, dtype=np.float64)
    dim = vel.shape[1]
    U = np.empty((rho.shape[0], dim + 2), dtype=np.float64)
    U[:, 0] = rho
    U[:, 1:dim + 1] = rho[:, None] * vel
    U[:, dim + 1] = p / (gamma - 1.0) + 0.5 * rho * np.sum(vel * vel, axis=1)
    return U


# Four-quadrant Riemann data, (rho, u, v, p); Q1 = upper right, then
# counter-clockwise (x >= 1/2 is "right", y >= 1/2 is "up").
FOUR_QUADRANT = (
    (1.0, 0.0, 0.0, 1.0),
    (0.5197, -0.7259, 0.0, 0.4),
    (0.1072, -0.7259, -1.4045, 0.0439),
    (0.2579, 0.0, -1.4045, 0.15),
)


def quadrant_index(coords: np.ndarray) -> np.ndarray:
    right = coords[:, 0] >= 0.5
    up = coords[:, 1] >= 0.5
    q = np.where(up, np.where(right, 0, 1), np.where(right, 3, 2))
    return q


def ic_four_quadrant(coords: np.ndarray, states=FOUR_QUADRANT,
                     gamma: float = GAMMA) -> np.ndarray:
    """2D four-quadrant Riemann problem (states given as rho, u, v, p)."""
    st = np.asarray(states, dtype=np.float64)
    q = quadrant_index(coords)
    return conserved(st[q, 0], st[q, 1:3], st[q, 3], gamma)


def random_quadrant_states(seed: int):
    """Seeded four-quadrant states: rho~U[0.1,2], p~U[0.05,2], |u|<=1.5."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(4):
        rho = rng.uniform(0.1, 2.0)
        p = rng.uniform(0.05, 2.0)
        r = 1.5 * math.sqrt(rng.uniform(0.0, 1.0))
        th = rng.uniform(0.0, 2.0 * math.pi)
        out.append((rho, r * math.cos(th), r * math.sin(th), p))
    return tuple(out)


def ic_sphere(coords: np.ndarray, radius: float = 0.3,
              inside=(1.0, 1.0), outside=(0.125, 0.1),
              gamma: float = GAMMA) -> np.ndarray:
    """Spherical (circular in 2D) shock tube at rest, centre (1/2,...)."""
    dim = coords.shape[1]
    r2 = np.sum((coords - 0.5) ** 2, axis=1)
    ins = r2 < radius * radius
    rho = np.where(ins, inside[0], outside[0])
    p = np.where(ins, inside[1], outside[1])
    return conserved(rho, np.zeros((coords.shape[0], dim)), p, gamma)


def gaussian_blobs(coords: np.ndarray, seed: int, count: int = 8,
                   lo: float = 0.1, hi: float = 0.9, sigma: float = 0.08
                   ) -> np.ndarray:
    """Sum of ``count`` unit Gaussians with seeded centres in [lo,hi]^d."""
    dim = coords.shape[1]
    rng = np.random.default_rng(seed)
    centres = rng.uniform(lo, hi, size=(count, dim))
    acc = np.zeros(coords.shape[0], dtype=np.float64)
    for c in centres:
        r2 = np.sum((coords - c) ** 2, axis=1)
        acc += np.exp(-r2 / (2.0 * sigma * sigma))
    return acc


def ic_mach3_blobs(coords: np.ndarray, seed: int = 2,
                   gamma: float = GAMMA) -> np.ndarray:
    """Uniform Mach 3 flow (rho=1.4, p=1, u=3 e_x) with a density blob field
    of amplitude 0.2 (eight seeded Gaussians, sigma 0.08)."""
    dim = coords.shape[1]
    rho = 1.4 + 0.2 * gaussian_blobs(coords, seed, lo=0.1, hi=0.9)
    vel = np.zeros((coords.shape[0], dim))
    vel[:, 0] = 3.0
    return conserved(rho, vel, np.ones_like(rho), gamma)


def ic_smooth_blobs(coords: np.ndarray, seed: int = 2,
                    gamma: float = GAMMA) -> np.ndarray:
    """rho = 1 + 0.1 * (eight seeded Gaussians in [0.2,0.8]^d), p=1, u=0."""
    dim = coords.shape[1]
    rho = 1.0 + 0.1 * gaussian_blobs(coords, seed, lo=0.2, hi=0.8)
    return conserved(rho, np.zeros((coords.shape[0], dim)),
                     np.ones_like(rho), gamma)


def ic_isothermal_blobs(coords: np.ndarray, seed: int = 2,
                        gamma: float = GAMMA) -> np.ndarray:
    """rho = 1 + 0.1 * (eight seeded Gaussians in [0.2,0.8]^d), p = rho
    (background pressure 1, uniform temperature), u = 0.  The blobs release
    acoustic waves; with a uniform pressure the state would be steady, and
    with p = rho^gamma the specific entropy would be uniform, which puts
    every limiter decision on the entropy bound itself."""
    dim = coords.shape[1]
    rho = 1.0 + 0.1 * gaussian_blobs(coords, seed, lo=0.2, hi=0.8)
    return conserved(rho, np.zeros((coords.shape[0], dim)), rho.copy(), gamma)


def smooth_field(coords: np.ndarray, seed: int, terms: int = 3) -> np.ndarray:
    """A smooth seeded field of unit size: sum of `terms` products of sines
    with random wave numbers 1-2 and phases (no flat region)."""
    rng = np.random.default_rng(seed)
    out = np.zeros(coords.shape[0])
    for _ in range(terms):
        w = rng.uniform(1.0, 2.0, size=coords.shape[1]) * 2.0 * np.pi
        ph = rng.uniform(0.0, 2.0 * np.pi, size=coords.shape[1])
        out += np.prod(np.sin(coords * w + ph), axis=1) / terms
    return out


def ic_generic_smooth(coords: np.ndarray, seed: int = 5, gamma: float = GAMMA) -> np.ndarray:
    """rho = 1 + 0.3 f1, p = 1 + 0.3 f2, u = 0.3 (f3, f4, f5) with smooth
    seeded fields f_k: a smooth state with no uniform region, so that no
    bound of Section 3.9 is tight by construction."""
    dim = coords.shape[1]
    rho = 1.0 + 0.3 * smooth_field(coords, seed)
    p = 1.0 + 0.3 * smooth_field(coords, seed + 1)
    vel = np.stack([0.3 * smooth_field(coords, seed + 2 + k) for k in range(dim)], axis=1)
    return conserved(rho, vel, p, gamma)


def isentropic_vortex(coords: np.ndarray, t: float = 0.0, centre=(0.5, 0.5),
                      radius: float = 0.1, beta: float = 5.0, u_inf=(0.0, 0.0),
                      gamma: float = GAMMA) -> np.ndarray:
    """The standard isentropic vortex (a closed-form smooth solution of the 2D
    Euler equations) carried by the uniform flow ``u_inf``, at time ``t``.

    With r the distance to the moving centre in units of ``radius``: the
    velocity perturbation is beta/(2 pi) exp((1 - r^2)/2) times the rotated
    offset, the temperature T = 1 - (gamma-1) beta^2/(8 gamma pi^2)
    exp(1 - r^2), rho = T^(1/(gamma-1)), p = rho^gamma.  The radial pressure
    gradient balances the centripetal acceleration at every radius, so the
    vortex is a steady state for u_inf = 0 and is translated otherwise.
    """
    x = np.asarray(coords, dtype=np.float64)
    c = np.array(centre, dtype=np.float64) + t * np.array(u_inf, dtype=np.float64)
    dx = (x[:, 0] - c[0]) / radius
    dy = (x[:, 1] - c[1]) / radius
    r2 = dx * dx + dy * dy
    amp = beta / (2.0 * math.pi) * np.exp(0.5 * (1.0 - r2))
    vel = np.empty((x.shape[0], 2))
    vel[:, 0] = u_inf[0] - amp * dy
    vel[:, 1] = u_inf[1] + amp * dx
    temp = 1.0 - (gamma - 1.0) * beta * beta / (8.0 * gamma * math.pi ** 2) * np.exp(1.0 - r2)
    rho = temp ** (1.0 / (gamma - 1.0))
    return conserved(rho, vel, rho ** gamma, gamma)


def ic_uniform(n_nodes: int, dim: int, rho=1.0, vel=None, p=1.0,
               gamma: float = GAMMA) -> np.ndarray:
    v = np.zeros((n_nodes, dim)) if vel is None else np.tile(
        np.asarray(vel, dtype=np.float64), (n_nodes, 1))
    return conserved(np.full(n_nodes, rho), v, np.full(n_nodes, p), gamma)


# ------------------------------------------------------------- workloads

def workload(name: str, n: int | None = None, order: str | None = None):
    """(mesh, U0) of a named synthetic workload.

    four_quadrant_2d : 2D 33^2 jittered grid, four-quadrant Riemann IC
    sphere_3d        : 3D 65^3 jittered, random order, spherical shock tube
    mach3_3d         : 3D 257^3 jittered, Morton order, Mach 3 + blobs
    smooth_3d        : 3D 65^3 jittered, smooth Gaussian density, at rest
    adjoint_3d       : 3D 65^3 jittered, isothermal Gaussian blobs, at rest
    """
    if name == "four_quadrant_2d":
        m = q1_grid(n or 33, 2, 0.2, seed=0, order=order or "lex")
        return m, ic_four_quadrant(m.coords)
    if name == "sphere_3d":
        m = q1_grid(n or 65, 3, 0.2, seed=0, order=order or "random",
                    perm_seed=1)
        return m, ic_sphere(m.coords)
    if name == "mach3_3d":
        m = q1_grid(n or 257, 3, 0.2, seed=0, order=order or "morton",
                    perm_seed=1)
        return m, ic_mach3_blobs(m.coords, seed=2)
    if name == "smooth_3d":
        m = q1_grid(n or 65, 3, 0.2, seed=0, order=order or "lex")
        return m, ic_smooth_blobs(m.coords, seed=2)
    if name == "adjoint_3d":
        m = q1_grid(n or 65, 3, 0.2, seed=0, order=order or "morton")
        return m, ic_isothermal_blobs(m.coords, seed=2)
    raise ValueError(f"unknown workload {name!r}")


def batch_workload(count: int = 64, smin: int = 33, smax: int = 513, seed0: int = 100,
                   order: str = "morton"):
    """Independent 2D four-quadrant problems of uneven sizes: instance k
    draws its side s_k log-uniformly in [smin, smax] from seed seed0 + k,
    and uses the same seed for its jitter and its four states.  Returns a
    list of (mesh, U0)."""
    out = []
    for k in range(count):
        seed = seed0 + k
        rng = np.random.default_rng(seed)
        side = int(round(math.exp(rng.uniform(math.log(smin), math.log(smax)))))
        m = q1_grid(side, 2, 0.2, seed=seed, order=order)
        out.append((m, ic_four_quadrant(m.coords, random_quadrant_states(seed))))
    return out


# --------------------------------------------------------------- patches

class PatchExtractor:
    """Sub-meshes around chosen nodes (node -> cell adjacency built once).

    ``extract(centres, radius)`` returns the cells that touch a node within
    graph distance ``radius`` of the centres (neighbours = nodes sharing a
    cell).  Node and cell relative orders are preserved, so the row of any
    node whose support lies inside the patch has the same columns, in the
    same order, as in the full mesh.  Returns (sub_mesh, node_map, dist):
    node_map[k] is the full-mesh id of patch node k and dist its graph
    distance to the centres (radius + 1 for the outer layer).
    """

    def __init__(self, mesh: Mesh):
        self.mesh = mesh
        cells = mesh.cells
        nv = cells.shape[1]
        flat = cells.reshape(-1)
        srt = np.argsort(flat, kind="stable")
        self.cell_of = (srt // nv).astype(np.int64)
        cnt = np.bincount(flat, minlength=mesh.n_nodes)
        self.ptr = np.zeros(mesh.n_nodes + 1, dtype=np.int64)
        np.cumsum(cnt, out=self.ptr[1:])

    def _cells_around(self, nodes):
        return np.unique(np.concatenate(
            [self.cell_of[self.ptr[v]:self.ptr[v + 1]] for v in nodes]))

    def extract(self, centre_nodes, radius: int):
        mesh = self.mesh
        cells = mesh.cells
        dist = {}
        front = np.unique(np.asarray(centre_nodes, dtype=np.int64))
        for v in front:
            dist[int(v)] = 0
        for r in range(1, radius + 2):
            nb = np.unique(cells[self._cells_around(front)].reshape(-1))
            nb = np.array([v for v in nb if int(v) not in dist], dtype=np.int64)
            for v in nb:
                dist[int(v)] = r
            front = nb
        inner = np.array([v for v, d in dist.items() if d <= radius], dtype=np.int64)
        cs = self._cells_around(inner)
        nodes = np.unique(cells[cs].reshape(-1))          # ascending full ids
        remap = {int(v): k for k, v in enumerate(nodes)}
        sub_cells = np.vectorize(remap.__getitem__, otypes=[np.int64])(cells[cs])
        sub = Mesh(dim=mesh.dim, n_side=mesh.n_side,
                   coords=np.ascontiguousarray(mesh.coords[nodes]),
                   cells=np.ascontiguousarray(sub_cells),
                   boundary=mesh.boundary[nodes].copy(),
                   grid_id=mesh.grid_id[nodes].copy())
        d = np.array([dist.get(int(v), radius + 1) for v in nodes], dtype=np.int64)
        return sub, nodes, d


def extract_patch(mesh: Mesh, centre_nodes, radius: int):
    """One-off PatchExtractor(mesh).extract(centre_nodes, radius)."""
    return PatchExtractor(mesh).extract(centre_nodes, radius)
