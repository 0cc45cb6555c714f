"""Seeded synthetic inputs for the particle-in-cell workloads.

This module is shared by the GPU path, the benchmark and the CPU oracle, and
therefore holds none of the method's arithmetic: it only

* describes meshes (uniform boxes, displaced structured grids, octree leaves),
* samples a prescribed velocity field at caller-given points,
* draws the random numbers that particle generation consumes (per-cell
  counts, reference coordinates in the unit cell, ids).

Mapping reference coordinates to physical ones, evaluating the finite element
field, advecting, locating, sorting, interpolating: all of that lives on each
side separately.

Conventions shared by both sides (they define the inputs, not the method):

* Uniform mesh on ``[lo, hi]`` with ``n[i]`` cells per axis; cell index
  ``i + n0*(j + n1*k)`` (x fastest).
* Q2 nodes of a uniform (or displaced structured) mesh form the grid of
  ``(2 n0 + 1) x (2 n1 + 1) [x (2 n2 + 1)]`` points; node ``(a, b, c)`` has index
  ``a + (2 n0 + 1)*(b + (2 n1 + 1)*c)`` and, on the undisplaced mesh, sits at
  ``lo + (a, b, c) * h / 2``.
* Field arrays are component-major, ``U[comp][node]``.
* Particle inputs are listed cell by cell in cell-index order; ``xr`` holds
  reference coordinates in ``[0, 1)^dim`` as ``xr[axis][particle]``.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

__all__ = [
    "UniformMesh", "FourierField", "rotation_velocity",
    "uniform_q2_nodes", "sample_nodes", "normalise_nodal",
    "draw_reference_particles", "octree_shell_leaves",
    "config1", "config2", "config3", "config4", "config5",
]


# --------------------------------------------------------------------------
# meshes
# --------------------------------------------------------------------------
@dataclass
class UniformMesh:
    dim: int
    n: tuple
    lo: tuple = (0.0, 0.0, 0.0)
    hi: tuple = (1.0, 1.0, 1.0)

    def __post_init__(self):
        n = list(self.n) + [1] * (3 - len(self.n))
        self.n = tuple(int(v) for v in n[:3])
        lo = list(self.lo) + [0.0] * (3 - len(self.lo))
        hi = list(self.hi) + [1.0] * (3 - len(self.hi))
        self.lo = tuple(float(v) for v in lo[:3])
        self.hi = tuple(float(v) for v in hi[:3])
        if self.dim == 2:
            self.n = (self.n[0], self.n[1], 1)

    @property
    def n_cells(self) -> int:
        return int(np.prod(self.n[: self.dim]))

    @property
    def node_shape(self) -> tuple:
        return tuple(2 * self.n[i] + 1 for i in range(self.dim))

    @property
    def n_nodes(self) -> int:
        return int(np.prod(self.node_shape))

    @property
    def h(self) -> tuple:
        return tuple((self.hi[i] - self.lo[i]) / self.n[i] for i in range(3))

    @property
    def n_vertices(self) -> int:
        return int(np.prod([self.n[i] + 1 for i in range(self.dim)]))


def uniform_q2_nodes(mesh: UniformMesh) -> np.ndarray:
    """Coordinates of the Q2 node grid of an undisplaced uniform mesh, [dim][n_nodes]."""
    axes = [mesh.lo[i] + 0.5 * np.arange(2 * mesh.n[i] + 1) * mesh.h[i] for i in range(mesh.dim)]
    grids = np.meshgrid(*axes, indexing="ij")          # grids[i][a, b, c]
    # node index a + (2n0+1)(b + (2n1+1)c): x fastest => Fortran order of (a, b, c)
    return np.stack([g.ravel(order="F") for g in grids]).astype(np.float64)


def uniform_vertices(mesh: UniformMesh) -> np.ndarray:
    """Coordinates of the (n0+1)x(n1+1)[x(n2+1)] vertex grid, [dim][n_vertices], x fastest."""
    axes = [mesh.lo[i] + np.arange(mesh.n[i] + 1) * mesh.h[i] for i in range(mesh.dim)]
    grids = np.meshgrid(*axes, indexing="ij")
    return np.stack([g.ravel(order="F") for g in grids]).astype(np.float64)


def displaced_vertices(mesh: UniformMesh, amplitude: float, seed: int) -> np.ndarray:
    """Vertex grid with interior vertices moved by up to ``amplitude*h`` per axis.

    Boundary vertices only move tangentially so that the domain stays the box.
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    v = uniform_vertices(mesh)
    shape = tuple(mesh.n[i] + 1 for i in range(mesh.dim))
    idx = np.stack(np.meshgrid(*[np.arange(s) for s in shape], indexing="ij"))
    idx = np.stack([g.ravel(order="F") for g in idx])
    for ax in range(mesh.dim):
        d = rng.uniform(-amplitude, amplitude, size=v.shape[1]) * mesh.h[ax]
        on_bnd = (idx[ax] == 0) | (idx[ax] == mesh.n[ax])
        d[on_bnd] = 0.0
        v[ax] += d
    return v


# --------------------------------------------------------------------------
# velocity fields
# --------------------------------------------------------------------------
def rotation_velocity(points: np.ndarray, centre=(0.5, 0.5)) -> np.ndarray:
    """Rigid rotation u = (-(y - cy), x - cx) at points [2][N]."""
    x, y = points[0], points[1]
    return np.stack([-(y - centre[1]), x - centre[0]])


@dataclass
class FourierField:
    """Divergence-free field from a random sum of Fourier modes.

    3D: u = curl A with A(x) = sum_m a_m sin(2 pi k_m.x + phi_m);
    2D: u = (d psi/dy, -d psi/dx) with psi(x) = sum_m a_m sin(2 pi k_m.x + phi_m).
    Amplitudes a_m ~ N(0, 1) (vectors in 3D), wave-vector components drawn
    uniformly from {1..kmax} with a random sign, phases ~ U[0, 2 pi).
    With ``tangential`` the potential is multiplied by prod_i sin(pi x_i) on the
    unit box, which makes the normal velocity vanish on every face.
    """
    dim: int
    seed: int
    n_modes: int = 8
    kmax: int = 4
    tangential: bool = False
    a: np.ndarray = field(init=False)
    k: np.ndarray = field(init=False)
    phi: np.ndarray = field(init=False)

    def __post_init__(self):
        rng = np.random.Generator(np.random.PCG64(self.seed))
        d = self.dim
        ncomp = 3 if d == 3 else 1
        self.a = rng.standard_normal((self.n_modes, ncomp))
        mag = rng.integers(1, self.kmax + 1, size=(self.n_modes, d))
        sign = np.where(rng.random((self.n_modes, d)) < 0.5, -1.0, 1.0)
        self.k = (mag * sign).astype(np.float64)
        self.phi = rng.random(self.n_modes) * 2.0 * math.pi

    def _potential_and_grad(self, p):
        """A (or psi) and its gradient at points p [d][N]; shapes [ncomp][N], [ncomp][d][N]."""
        d = self.dim
        arg = 2.0 * math.pi * (self.k @ p) + self.phi[:, None]        # [M][N]
        s, c = np.sin(arg), np.cos(arg)
        A = np.einsum("mc,mn->cn", self.a, s)
        gA = 2.0 * math.pi * np.einsum("mc,mj,mn->cjn", self.a, self.k, c)
        if self.tangential:
            sp = np.sin(math.pi * p)                                   # [d][N]
            S = np.prod(sp, axis=0)
            gS = np.empty_like(p)
            for j in range(d):
                others = np.prod(np.delete(sp, j, axis=0), axis=0)
                gS[j] = math.pi * np.cos(math.pi * p[j]) * others
            gA = gA * S[None, None, :] + A[:, None, :] * gS[None, :, :]
            A = A * S[None, :]
        return A, gA

    def velocity(self, points: np.ndarray) -> np.ndarray:
        p = np.asarray(points, dtype=np.float64)
        _, g = self._potential_and_grad(p)
        if self.dim == 2:
            return np.stack([g[0, 1], -g[0, 0]])
        # curl: (dAz/dy - dAy/dz, dAx/dz - dAz/dx, dAy/dx - dAx/dy)
        return np.stack([g[2, 1] - g[1, 2], g[0, 2] - g[2, 0], g[1, 0] - g[0, 1]])


def sample_nodes(fn, nodes: np.ndarray) -> np.ndarray:
    return np.ascontiguousarray(fn(nodes), dtype=np.float64)


def normalise_nodal(U: np.ndarray) -> np.ndarray:
    """Scale a nodal field so that the largest nodal Euclidean norm is 1."""
    m = float(np.sqrt((U * U).sum(axis=0)).max())
    return U / m if m > 0 else U


# --------------------------------------------------------------------------
# particle draws
# --------------------------------------------------------------------------
def draw_reference_particles(counts: np.ndarray, dim: int, seed: int):
    """Reference coordinates ~ U[0,1)^dim for ``counts[c]`` particles per cell.

    Returns (counts int32, xr [dim][N] float64, ids uint32) with particles listed
    cell by cell and ids = running index (so the initial order is (cell, id)).
    """
    counts = np.asarray(counts, dtype=np.int64)
    n = int(counts.sum())
    rng = np.random.Generator(np.random.PCG64(seed))
    xr = rng.random((dim, n))
    ids = np.arange(n, dtype=np.uint32)
    return counts.astype(np.int32), np.ascontiguousarray(xr), ids


# --------------------------------------------------------------------------
# octree leaves for the shell-refined mesh
# --------------------------------------------------------------------------
def octree_shell_leaves(base_level=3, max_level=7, r_in=0.35, r_out=0.45, width=3.0,
                        centre=(0.5, 0.5, 0.5)):
    """Leaves of an octree on the unit cube refined toward a spherical shell.

    Start from the uniform level ``base_level`` grid; for l = base..max-1 refine
    every leaf of level l if l < base+1 or the distance from its box to the shell
    {r_in <= |x - centre| <= r_out} is below width * 2^-l.  Returns
    (level uint8 [N], anchor int32 [3][N]) with anchors in units of the finest
    cell (2^-max_level), listed in Morton order of the anchors.  The caller may
    check 2:1 balance; the default parameters produce a vertex-balanced tree.
    """
    c = np.asarray(centre, dtype=np.float64)

    def box_shell_distance(lo, size):
        # distance from axis-aligned boxes to the shell, vectorised
        hi = lo + size[None, :]
        q = np.maximum(np.maximum(lo - c[:, None], 0.0), c[:, None] - hi)
        dmin = np.sqrt((q * q).sum(axis=0))                  # nearest point of box to centre
        far = np.maximum(np.abs(lo - c[:, None]), np.abs(hi - c[:, None]))
        dmax = np.sqrt((far * far).sum(axis=0))              # farthest point
        below = np.maximum(r_in - dmax, 0.0)                  # box entirely inside r_in
        above = np.maximum(dmin - r_out, 0.0)                 # box entirely outside r_out
        return np.maximum(below, above)

    fine = 1 << max_level
    n0 = 1 << base_level
    s0 = fine // n0
    g = np.stack(np.meshgrid(np.arange(n0), np.arange(n0), np.arange(n0), indexing="ij")).reshape(3, -1)
    anchors = g * s0
    levels = np.full(anchors.shape[1], base_level, dtype=np.int64)
    done_a, done_l = [], []
    for lev in range(base_level, max_level):
        sel = levels == lev
        a = anchors[:, sel]
        size = np.full(a.shape[1], 2.0 ** -lev)
        lo = a / fine
        refine = (lev < base_level + 1) | (box_shell_distance(lo, size) < width * 2.0 ** -lev)
        done_a.append(a[:, ~refine])
        done_l.append(np.full((~refine).sum(), lev))
        a = a[:, refine]
        half = (fine >> (lev + 1))
        kids = [a + np.array([[dx], [dy], [dz]]) * half
                for dz in (0, 1) for dy in (0, 1) for dx in (0, 1)]
        anchors = np.concatenate(kids, axis=1) if kids else np.zeros((3, 0), np.int64)
        levels = np.full(anchors.shape[1], lev + 1)
    done_a.append(anchors)
    done_l.append(levels)
    A = np.concatenate(done_a, axis=1)
    L = np.concatenate(done_l)

    def morton(a):
        key = np.zeros(a.shape[1], dtype=np.uint64)
        for bit in range(max_level):
            for ax in range(3):
                key |= ((a[ax].astype(np.uint64) >> np.uint64(bit)) & np.uint64(1)) << np.uint64(3 * bit + ax)
        return key

    order = np.argsort(morton(A), kind="stable")
    return L[order].astype(np.uint8), np.ascontiguousarray(A[:, order].astype(np.int32))


def balance_octree(level, anchor, max_level):
    """Refine leaves until every pair of leaves sharing at least a point differs by
    at most one level (vertex 2:1 balance).  Returns leaves in Morton order.
    Plain loops: meant for small meshes."""
    fine = 1 << max_level
    lv = [int(v) for v in level]
    an = [tuple(int(anchor[a][k]) for a in range(3)) for k in range(len(lv))]
    while True:
        table = np.empty((fine, fine, fine), np.int64)
        for k, (l, a) in enumerate(zip(lv, an)):
            s = 1 << (max_level - l)
            table[a[2]:a[2] + s, a[1]:a[1] + s, a[0]:a[0] + s] = k
        levels = np.array(lv)
        refine = []
        for k, (l, a) in enumerate(zip(lv, an)):
            s = 1 << (max_level - l)
            lo = [max(v - 1, 0) for v in a]
            hi = [min(v + s + 1, fine) for v in a]
            nb = np.unique(table[lo[2]:hi[2], lo[1]:hi[1], lo[0]:hi[0]])
            if levels[nb].max() > l + 1:
                refine.append(k)
        if not refine:
            break
        rset = set(refine)
        nl, na = [], []
        for k, (l, a) in enumerate(zip(lv, an)):
            if k not in rset:
                nl.append(l)
                na.append(a)
                continue
            h = 1 << (max_level - l - 1)
            for dz in (0, 1):
                for dy in (0, 1):
                    for dx in (0, 1):
                        nl.append(l + 1)
                        na.append((a[0] + dx * h, a[1] + dy * h, a[2] + dz * h))
        lv, an = nl, na
    A = np.array(an, np.int64).T
    key = np.zeros(A.shape[1], dtype=np.uint64)
    for bit in range(max_level):
        for ax in range(3):
            key |= ((A[ax].astype(np.uint64) >> np.uint64(bit)) & np.uint64(1)) << np.uint64(3 * bit + ax)
    order = np.argsort(key, kind="stable")
    return np.array(lv, np.uint8)[order], np.ascontiguousarray(A[:, order].astype(np.int32))


def morton_sort(level, anchor, max_level):
    """Leaves listed in Morton order of their anchors (finest-cell units)."""
    A = np.asarray(anchor, np.int64)
    key = np.zeros(A.shape[1], dtype=np.uint64)
    for bit in range(max_level):
        for ax in range(3):
            key |= ((A[ax].astype(np.uint64) >> np.uint64(bit)) & np.uint64(1)) << np.uint64(3 * bit + ax)
    order = np.argsort(key, kind="stable")
    return np.asarray(level, np.uint8)[order], np.ascontiguousarray(A[:, order].astype(np.int32))


def refine_leaves(level, anchor, max_level, mask):
    """Replace every leaf with mask set (and level < max_level) by its eight children."""
    level = np.asarray(level)
    anchor = np.asarray(anchor, np.int64)
    mask = np.asarray(mask, bool) & (level < max_level)
    keep_l, keep_a = level[~mask], anchor[:, ~mask]
    pl, pa = level[mask].astype(np.int64), anchor[:, mask]
    kids_l, kids_a = [], []
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                h = (1 << (max_level - pl - 1))
                kids_a.append(pa + np.stack([dx * h, dy * h, dz * h]))
                kids_l.append(pl + 1)
    L = np.concatenate([keep_l.astype(np.int64)] + kids_l)
    A = np.concatenate([keep_a] + kids_a, axis=1)
    return morton_sort(L, A, max_level)


def coarsen_leaves(level, anchor, max_level, mask):
    """Merge every complete group of eight sibling leaves that all have mask set into their parent."""
    level = np.asarray(level).astype(np.int64)
    anchor = np.asarray(anchor, np.int64)
    mask = np.asarray(mask, bool) & (level > 0)
    groups = {}
    for k in np.nonzero(mask)[0]:
        ps = 1 << (max_level - level[k] + 1)                 # parent size in finest units
        pa = tuple(int(v) for v in (anchor[:, k] // ps) * ps)
        groups.setdefault((int(level[k]), pa), []).append(k)
    merged = set()
    new_l, new_a = [], []
    for (lv, pa), ks in groups.items():
        if len(ks) == 8:
            merged.update(ks)
            new_l.append(lv - 1)
            new_a.append(pa)
    keep = np.array([k for k in range(level.size) if k not in merged], np.int64)
    L = np.concatenate([level[keep], np.array(new_l, np.int64)])
    A = np.concatenate([anchor[:, keep], np.array(new_a, np.int64).T.reshape(3, -1)], axis=1)
    return morton_sort(L, A, max_level)


def coarsen_finest(level, anchor, max_level):
    """Merge every group of eight sibling leaves at the finest level into its parent (vectorised; in a
    tree built by refinement the finest leaves always come in complete sibling groups)."""
    level = np.asarray(level).astype(np.int64)
    anchor = np.asarray(anchor, np.int64)
    fine = level == max_level
    parents = np.unique(((anchor[:, fine] >> 1) << 1).T, axis=0).T
    L = np.concatenate([level[~fine], np.full(parents.shape[1], max_level - 1)])
    A = np.concatenate([anchor[:, ~fine], parents], axis=1)
    return morton_sort(L, A, max_level)


# --------------------------------------------------------------------------
# workload configurations
# --------------------------------------------------------------------------
def config1():
    """2D unit square, 32x32, rigid rotation, 16 per cell, RK2, CFL 0.5, 100 steps."""
    mesh = UniformMesh(2, (32, 32))
    U = sample_nodes(rotation_velocity, uniform_q2_nodes(mesh))
    counts = np.full(mesh.n_cells, 16, dtype=np.int32)
    counts, xr, ids = draw_reference_particles(counts, 2, seed=1)
    dt = 0.5 * (1.0 / 32) / math.sqrt(0.5)
    return dict(name="uniform2d-32x32-rotation-rk2", mesh=mesh, U=U, counts=counts, xr=xr, ids=ids,
                dt=dt, scheme=2, steps=100, n_prop=1, prop_dtype=np.float64, eval_f32=False)


def config2(eval_f32=True, tangential=False, n=64, ppc=20, steps=50):
    """3D unit cube, 64^3, random divergence-free field, 20 per cell, RK4, CFL 0.5, 50 steps."""
    mesh = UniformMesh(3, (n, n, n))
    f = FourierField(3, seed=2, tangential=tangential)
    U = normalise_nodal(sample_nodes(f.velocity, uniform_q2_nodes(mesh)))
    counts = np.full(mesh.n_cells, ppc, dtype=np.int32)
    counts, xr, ids = draw_reference_particles(counts, 3, seed=3)
    dt = 0.5 / n
    return dict(name=f"uniform3d-{n}^3-fourier-rk4", mesh=mesh, U=U, counts=counts, xr=xr, ids=ids,
                dt=dt, scheme=4, steps=steps, n_prop=3, prop_dtype=np.float32, eval_f32=eval_f32)


def config3_counts(n_leaves: int, seed: int = 4):
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.integers(5, 81, size=n_leaves).astype(np.int32)


def config3():
    """Shell-refined octree, random field, 5..80 per cell, clamp to [8, 64], RK2, 50 steps."""
    level, anchor = octree_shell_leaves()
    f = FourierField(3, seed=2, tangential=False)
    counts = config3_counts(level.shape[0])
    counts, xr, ids = draw_reference_particles(counts, 3, seed=4 + 1000)
    # the finest leaves (edge 2^-7) bind the step: dt = CFL * h_min / max|u| with max|u| = 1 at the nodes
    return dict(name="octree-shell-l3..7-rk2", level=level, anchor=anchor, max_level=7, field=f,
                counts=counts, xr=xr, ids=ids, scheme=2, steps=50, n_prop=1, prop_dtype=np.float64,
                pop_min=8, pop_max=64, pop_seed=40, cfl=0.5, dt=0.5 * 2.0 ** -7)


def config4_problem(p: int):
    rng = np.random.Generator(np.random.PCG64(100 + p))
    dim = int(rng.integers(2, 4))
    n = int(rng.integers(16, 129)) if dim == 2 else int(rng.integers(16, 49))
    ppc = int(rng.integers(4, 41))
    scheme = 2 if rng.random() < 0.5 else 4
    mesh = UniformMesh(dim, (n,) * dim)
    f = FourierField(dim, seed=100 + p)
    U = normalise_nodal(sample_nodes(f.velocity, uniform_q2_nodes(mesh)))
    counts = np.full(mesh.n_cells, ppc, dtype=np.int32)
    counts, xr, ids = draw_reference_particles(counts, dim, seed=10_000 + p)
    return dict(name=f"batch-{p}", mesh=mesh, U=U, counts=counts, xr=xr, ids=ids, dt=0.5 / n,
                scheme=scheme, steps=20, n_prop=1, prop_dtype=np.float64, eval_f32=False)


def config4(n_problems=64):
    return [config4_problem(p) for p in range(n_problems)]


def config5(n=32, ppc=32):
    """3D 32^3, tangential random field (trainable), 32 per cell, RK4, 50 steps, dt 2^-6."""
    mesh = UniformMesh(3, (n, n, n))
    nodes = uniform_q2_nodes(mesh)
    U = normalise_nodal(sample_nodes(FourierField(3, seed=5, tangential=True).velocity, nodes))
    Up = normalise_nodal(sample_nodes(FourierField(3, seed=6, tangential=True).velocity, nodes))
    counts = np.full(mesh.n_cells, ppc, dtype=np.int32)
    counts, xr, ids = draw_reference_particles(counts, 3, seed=9)
    return dict(name=f"adjoint-{n}^3-rk4", mesh=mesh, U=U, U_pert=Up, counts=counts, xr=xr, ids=ids,
                dt=2.0 ** -6, scheme=4, steps=50, ckpt_every=10, noise_seed=7, noise_sigma=1e-3,
                fd_seed=8, n_prop=0, prop_dtype=np.float64, eval_f32=False)


def target_noise(n: int, dim: int, seed: int = 7, sigma: float = 1e-3) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return sigma * rng.standard_normal((dim, n))


def fd_directions(count: int, size: int, seed: int = 8) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    v = rng.standard_normal((count, size))
    return v / np.abs(v).max(axis=1, keepdims=True)
