"""Python front end of the FP64 CPU oracle (test infrastructure only).

Only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
may import this module.  It loads ``liboracle.so`` (built from
``pic_oracle.c`` with gcc, see ``build_oracle``) and adds the parts of the
oracle that are clearest in NumPy:

* the octree's Q2 node numbering and hanging-node constraints,
* the per-cell linear least-squares fit (batched SVD),
* convenience drivers that run whole workloads.

Method references (Gassmoeller et al., arXiv:1612.03369) are given per function.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
import threading

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "pic_oracle.c")
LIB = os.path.join(HERE, "liboracle.so")
LOST = 0xFFFFFFFF

_lock = threading.Lock()
_lib = None


def build_oracle(force: bool = False) -> str:
    """Compile the C oracle with gcc (OpenMP, -O2, no fast-math)."""
    if force or not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        tmp = LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
                               "-ffp-contract=off", "-o", tmp, SRC, "-lm"])
        os.replace(tmp, LIB)
    return LIB


class Mesh(C.Structure):
    _fields_ = [("dim", C.c_int), ("kind", C.c_int), ("n", C.c_int * 3),
                ("lo", C.c_double * 3), ("hi", C.c_double * 3), ("vert", C.c_void_p),
                ("n_cells", C.c_int64), ("max_level", C.c_int), ("level", C.c_void_p),
                ("anchor", C.c_void_p), ("fine_to_leaf", C.c_void_p), ("cell_nodes", C.c_void_p)]


class Store(C.Structure):
    _fields_ = [("n", C.c_int64), ("cap", C.c_int64), ("dim", C.c_int), ("n_prop", C.c_int),
                ("x", C.c_void_p), ("xr", C.c_void_p), ("cell", C.c_void_p), ("id", C.c_void_p),
                ("prop", C.c_void_p)]


class Stats(C.Structure):
    _fields_ = [("live", C.c_int64), ("lost", C.c_int64), ("moved", C.c_int64), ("near_face", C.c_int64)]


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build_oracle()
            L = C.CDLL(LIB)
            P = C.c_void_p
            L.orc_n_cells.restype = C.c_int64
            L.orc_n_cells.argtypes = [P]
            L.orc_locate.restype = C.c_int
            L.orc_locate.argtypes = [P, P, P, P]
            L.orc_map_to_real.argtypes = [P, C.c_int64, P, P]
            L.orc_eval.argtypes = [P, P, C.c_int64, C.c_int64, P, P]
            L.orc_seed.restype = C.c_int
            L.orc_seed.argtypes = [P, P, P, C.c_int64, P, C.c_int, P]
            L.orc_advect.argtypes = [P, P, C.c_int64, C.c_double, C.c_int, P, P, P]
            L.orc_advect_odes.argtypes = [P, P, C.c_int64, C.c_double, C.c_int, C.c_double, C.c_double,
                                          C.c_int, C.c_int, P, P, P]
            L.orc_sort_perm.restype = C.c_int64
            L.orc_advect_t.argtypes = [P, P, P, C.c_int64, C.c_double, C.c_double, C.c_double, C.c_int, P, P, P]
            L.orc_advect_t.restype = None
            L.orc_advect_odes_t.argtypes = [P, P, P, C.c_int64, C.c_double, C.c_double, C.c_double, C.c_int,
                                            C.c_double, C.c_double, C.c_int, C.c_int, P, P, P]
            L.orc_advect_odes_t.restype = None
            L.orc_cell_mean.argtypes = [C.c_int64, P, P, C.c_int, P, P]
            L.orc_cell_mean.restype = None
            L.orc_interp_points.argtypes = [P, P, P, C.c_int, C.c_int, P, P]
            L.orc_interp_points.restype = None
            L.orc_seed_mh.argtypes = [P, P, P, C.c_int, C.c_uint64, C.c_uint32, P, P]
            L.orc_seed_mh.restype = C.c_int
            L.orc_transfer.argtypes = [P, P, P, P]
            L.orc_transfer.restype = C.c_int
            L.orc_sort_perm.argtypes = [C.c_int64, C.c_int64, P, P, P, P]
            L.orc_step.restype = C.c_int
            L.orc_step.argtypes = [P, P, C.c_int64, C.c_double, C.c_int, P, P, P]
            L.orc_splitmix64.restype = C.c_uint64
            L.orc_splitmix64.argtypes = [C.c_uint64]
            L.orc_uniform01.restype = C.c_double
            L.orc_uniform01.argtypes = [C.c_uint64] * 5
            L.orc_population.restype = C.c_int
            L.orc_population.argtypes = [P, P, P, C.c_int, C.c_int, C.c_uint64, C.c_uint64, P, P, P]
            L.orc_cell_average.argtypes = [C.c_int64, P, P, P, P]
            L.orc_adjoint.restype = C.c_double
            L.orc_adjoint.argtypes = [P, P, C.c_int64, C.c_double, C.c_int, C.c_int, C.c_int64,
                                      P, P, P, P, P, P, P]
            L.orc_set_threads.restype = C.c_int
            L.orc_set_threads.argtypes = [C.c_int]
            L.orc_seed_per_cell.restype = C.c_int
            L.orc_seed_per_cell.argtypes = [P, P, C.c_uint64, C.c_uint32, C.c_int, P]
            L.orc_octree_fine_table.restype = C.c_int
            L.orc_octree_fine_table.argtypes = [C.c_int64, C.c_int, P, P, P]
            _lib = L
    return _lib


def _p(a):
    return a.ctypes.data_as(C.c_void_p) if a is not None else None


# ----------------------------------------------------------------------
# meshes
# ----------------------------------------------------------------------
class OracleMesh:
    """A mesh as the oracle sees it; keeps the numpy arrays alive."""

    def __init__(self, dim, kind, n=(1, 1, 1), lo=(0, 0, 0), hi=(1, 1, 1), vert=None,
                 level=None, anchor=None, max_level=0):
        self.dim, self.kind = dim, kind
        self.n = tuple(list(n) + [1] * (3 - len(n)))[:3]
        self.lo = tuple(list(lo) + [0.0] * (3 - len(lo)))[:3]
        self.hi = tuple(list(hi) + [1.0] * (3 - len(hi)))[:3]
        self.vert = None if vert is None else np.ascontiguousarray(vert, np.float64)
        self.level = None if level is None else np.ascontiguousarray(level, np.uint8)
        self.anchor = None if anchor is None else np.ascontiguousarray(anchor, np.int32)
        self.max_level = max_level
        self.fine = None
        self.cell_nodes = None
        self.node_lattice = None
        self.hanging = None
        if kind == 2:
            nc = self.level.shape[0]
            f = 1 << max_level
            self.fine = np.empty(f ** 3, np.int32)
            rc = lib().orc_octree_fine_table(nc, max_level, _p(self.level), _p(self.anchor), _p(self.fine))
            if rc != 0:
                raise ValueError("octree leaves do not tile the cube")
            self._octree_nodes()
        self.c = Mesh()
        self.c.dim, self.c.kind = dim, kind
        for a in range(3):
            self.c.n[a] = int(self.n[a])
            self.c.lo[a] = float(self.lo[a])
            self.c.hi[a] = float(self.hi[a])
        self.c.vert = _p(self.vert)
        self.c.n_cells = 0 if level is None else int(self.level.shape[0])
        self.c.max_level = max_level
        self.c.level = _p(self.level)
        self.c.anchor = _p(self.anchor)
        self.c.fine_to_leaf = _p(self.fine)
        self.c.cell_nodes = _p(self.cell_nodes)

    @classmethod
    def uniform(cls, m):
        return cls(m.dim, 0, m.n, m.lo, m.hi)

    @classmethod
    def displaced(cls, m, vert):
        return cls(m.dim, 1, m.n, m.lo, m.hi, vert=vert)

    @classmethod
    def octree(cls, level, anchor, max_level):
        return cls(3, 2, level=level, anchor=anchor, max_level=max_level)

    @property
    def n_cells(self):
        return int(lib().orc_n_cells(C.byref(self.c)))

    @property
    def n_nodes(self):
        if self.kind == 2:
            return int(self.node_lattice.shape[1])
        return int(np.prod([2 * self.n[a] + 1 for a in range(self.dim)]))

    # -- octree Q2 nodes -------------------------------------------------
    def _octree_nodes(self):
        """Q2 nodes of the octree leaves and their hanging-node constraints.

        Lattice units are half of the finest cell.  Unique lattice points are
        numbered in ascending x + M*(y + M*z) order (M = 2^(L+1) + 1).  A node is
        hanging if it lies in the closed box of a leaf without being one of that
        leaf's 27 nodes; it is then the Q2 interpolant of the coarsest such leaf.
        """
        L = self.max_level
        lv = self.level.astype(np.int64)
        a = self.anchor.astype(np.int64) * 2                      # lattice units
        s = (np.int64(1) << (L - lv))                              # half-size in lattice units
        loc = np.array([[i, j, k] for k in range(3) for j in range(3) for i in range(3)], np.int64)  # [27][3]
        pts = a.T[:, None, :] + loc[None, :, :] * s[:, None, None]  # [nc][27][3]
        M = (1 << (L + 1)) + 1
        key = pts[..., 0] + M * (pts[..., 1] + M * pts[..., 2])
        uniq, inv = np.unique(key.ravel(), return_inverse=True)
        self.cell_nodes = np.ascontiguousarray(inv.reshape(-1, 27).astype(np.int32))
        self.node_lattice = np.stack([uniq % M, (uniq // M) % M, uniq // (M * M)]).astype(np.int64)
        self.node_key = uniq

    def q2_node_coords(self):
        if self.kind == 2:
            M = 1 << (self.max_level + 1)
            return np.stack([self.lo[a] + (self.hi[a] - self.lo[a]) * self.node_lattice[a] / M
                             for a in range(3)])
        if self.kind == 0:
            axes = [self.lo[a] + 0.5 * np.arange(2 * self.n[a] + 1) * (self.hi[a] - self.lo[a]) / self.n[a]
                    for a in range(self.dim)]
            g = np.meshgrid(*axes, indexing="ij")
            return np.stack([x.ravel(order="F") for x in g])
        # displaced: Phi_K of the node's reference point, taken from any cell owning it
        nn = self.n_nodes
        out = np.full((self.dim, nn), np.nan)
        nx = 2 * self.n[0] + 1
        ny = 2 * self.n[1] + 1
        for K in range(self.n_cells):
            i = K % self.n[0]
            j = (K // self.n[0]) % self.n[1]
            k = K // (self.n[0] * self.n[1]) if self.dim == 3 else 0
            for l in range(9 if self.dim == 2 else 27):
                aa, bb, cc = l % 3, (l // 3) % 3, l // 9
                g = (2 * i + aa) + nx * ((2 * j + bb) + ny * (2 * k + cc))
                t = np.array([aa / 2, bb / 2, cc / 2][: self.dim], np.float64)
                out[:, g] = self.map_to_real(K, t)
        return out

    def hanging_constraints(self):
        """List of (node, leaf) pairs: hanging node and the coarsest leaf constraining it.

        Sorted by the constraining leaf's level (coarse first)."""
        if self.kind != 2:
            return []
        L = self.max_level
        M = (1 << (L + 1)) + 1
        key_to_node = {int(k): i for i, k in enumerate(self.node_key)}
        lv = self.level.astype(np.int64)
        a = self.anchor.astype(np.int64) * 2
        out = {}
        for K in np.argsort(lv, kind="stable"):
            s = 1 << (L - int(lv[K]))                  # node spacing of leaf K in lattice units
            x0, y0, z0 = (int(a[0, K]), int(a[1, K]), int(a[2, K]))
            own = set()
            for k in range(3):
                for j in range(3):
                    for i in range(3):
                        own.add((x0 + i * s) + M * ((y0 + j * s) + M * (z0 + k * s)))
            if s == 1:
                continue
            # every lattice point on the closed box of K at finer spacing that is a node
            for k in range(0, 2 * s + 1):
                for j in range(0, 2 * s + 1):
                    for i in range(0, 2 * s + 1):
                        if 0 < i < 2 * s and 0 < j < 2 * s and 0 < k < 2 * s:
                            continue                   # interior of K: no other leaf's node there
                        kk = (x0 + i) + M * ((y0 + j) + M * (z0 + k))
                        if kk in own or kk not in key_to_node:
                            continue
                        node = key_to_node[kk]
                        if node not in out or lv[out[node]] > lv[K]:
                            out[node] = int(K)
        pairs = sorted(out.items(), key=lambda p: (int(lv[p[1]]), p[0]))
        return pairs

    def resolve_hanging(self, U):
        """Overwrite hanging nodes with the constraining leaf's Q2 interpolant."""
        U = np.array(U, dtype=np.float64, copy=True)
        L = self.max_level
        M = 1 << (L + 1)
        for node, K in self.hanging_constraints():
            s = 1 << (L - int(self.level[K]))
            p = self.node_lattice[:, node]
            t = (p - 2 * self.anchor[:, K].astype(np.int64)) / (2.0 * s)
            U[:, node] = self.eval(U, K, t)
        return U

    # -- thin wrappers ---------------------------------------------------
    def locate(self, x):
        x = np.ascontiguousarray(x, np.float64)
        cell = np.zeros(1, np.int32)
        xr = np.zeros(3, np.float64)
        ok = lib().orc_locate(C.byref(self.c), _p(x), _p(cell), _p(xr))
        return (int(cell[0]), xr[: self.dim].copy()) if ok else (None, None)

    def map_to_real(self, K, xr):
        xr = np.ascontiguousarray(xr, np.float64)
        x = np.zeros(3, np.float64)
        lib().orc_map_to_real(C.byref(self.c), int(K), _p(xr), _p(x))
        return x[: self.dim].copy()

    def eval(self, U, K, xr):
        U = np.ascontiguousarray(U, np.float64)
        xr = np.ascontiguousarray(xr, np.float64)
        u = np.zeros(3, np.float64)
        lib().orc_eval(C.byref(self.c), _p(U), U.shape[1], int(K), _p(xr), _p(u))
        return u[: self.dim].copy()


# ----------------------------------------------------------------------
# particle store
# ----------------------------------------------------------------------
class OracleStore:
    def __init__(self, dim, cap, n_prop):
        self.dim, self.cap, self.n_prop = dim, int(cap), int(n_prop)
        self.x = np.zeros((dim, self.cap))
        self.xr = np.zeros((dim, self.cap))
        self.cell = np.zeros(self.cap, np.int32)
        self.id = np.zeros(self.cap, np.uint32)
        self.prop = np.zeros((max(n_prop, 1), self.cap))
        self.c = Store()
        self.c.cap, self.c.dim, self.c.n_prop = self.cap, dim, n_prop
        self.c.x, self.c.xr = _p(self.x), _p(self.xr)
        self.c.cell, self.c.id, self.c.prop = _p(self.cell), _p(self.id), _p(self.prop)
        self.c.n = 0
        self.cell_start = None

    @property
    def n(self):
        return int(self.c.n)

    def view(self):
        n = self.n
        return dict(x=self.x[:, :n].copy(), xr=self.xr[:, :n].copy(), cell=self.cell[:n].copy(),
                    id=self.id[:n].copy(), prop=self.prop[: self.n_prop, :n].copy(),
                    cell_start=None if self.cell_start is None else self.cell_start.copy())


def seed(mesh: OracleMesh, counts, xr, ids, n_prop, cap=None, init_position=True):
    """Reference-local generation (Sec. 2.2, remark on local generation)."""
    counts = np.ascontiguousarray(counts, np.int32)
    xr = np.ascontiguousarray(xr, np.float64)
    ids = np.ascontiguousarray(ids, np.uint32)
    n = xr.shape[1]
    st = OracleStore(mesh.dim, cap or n, n_prop)
    rc = lib().orc_seed(C.byref(mesh.c), _p(counts), _p(xr), n, _p(ids), int(init_position), C.byref(st.c))
    if rc != 0:
        raise ValueError("capacity too small")
    cs = np.zeros(mesh.n_cells + 1, np.int64)
    cs[1:] = np.cumsum(counts)
    st.cell_start = cs
    return st


def step(mesh: OracleMesh, U, dt, scheme, st: OracleStore, stats: Stats | None = None):
    """One time step: advect + locate (Sec. 2.3, 2.4), drop lost, stable re-sort."""
    U = np.ascontiguousarray(U, np.float64)
    cs = np.zeros(mesh.n_cells + 1, np.int64)
    s = stats if stats is not None else Stats()
    lib().orc_step(C.byref(mesh.c), _p(U), U.shape[1], float(dt), int(scheme), C.byref(st.c), _p(cs),
                   C.byref(s))
    st.cell_start = cs
    st._U_keepalive = U
    return s


def advect(mesh: OracleMesh, U, dt, scheme, st: OracleStore, U1=None, dt_u=None, since=0.0):
    """Advection + location without reordering; returns (key, near).

    With U1 the field changes in time (Sec. 2.3): U at t^n, U1 at t^n + dt_u, interpolated linearly in
    time; the step covers [t^n + since, t^n + since + dt]."""
    U = np.ascontiguousarray(U, np.float64)
    key = np.zeros(max(st.n, 1), np.uint32)
    near = np.zeros(max(st.n, 1), np.uint8)
    if U1 is None:
        lib().orc_advect(C.byref(mesh.c), _p(U), U.shape[1], float(dt), int(scheme), C.byref(st.c),
                         _p(key), _p(near))
    else:
        U1 = np.ascontiguousarray(U1, np.float64)
        assert U1.shape == U.shape and dt_u is not None and dt_u > 0
        lib().orc_advect_t(C.byref(mesh.c), _p(U), _p(U1), U.shape[1], float(dt_u), float(since), float(dt),
                           int(scheme), C.byref(st.c), _p(key), _p(near))
    return key[: st.n], near[: st.n]


def advect_odes(mesh: OracleMesh, U, dt, scheme, st: OracleStore, alpha, beta, damage_prop, deform_prop,
                U1=None, dt_u=None, since=0.0):
    """Advection + location with the damage and deformation-gradient equations of Sec. 2.6 integrated
    by the same RK scheme (no reordering); returns (key, near).  U1, dt_u, since as in advect."""
    U = np.ascontiguousarray(U, np.float64)
    key = np.zeros(max(st.n, 1), np.uint32)
    near = np.zeros(max(st.n, 1), np.uint8)
    if U1 is None:
        lib().orc_advect_odes(C.byref(mesh.c), _p(U), U.shape[1], float(dt), int(scheme), float(alpha),
                              float(beta), int(damage_prop), int(deform_prop), C.byref(st.c), _p(key), _p(near))
    else:
        U1 = np.ascontiguousarray(U1, np.float64)
        assert U1.shape == U.shape and dt_u is not None and dt_u > 0
        lib().orc_advect_odes_t(C.byref(mesh.c), _p(U), _p(U1), U.shape[1], float(dt_u), float(since), float(dt),
                                int(scheme), float(alpha), float(beta), int(damage_prop), int(deform_prop),
                                C.byref(st.c), _p(key), _p(near))
    return key[: st.n], near[: st.n]


def transfer(new_mesh: OracleMesh, src: OracleStore, cap=None):
    """Particles of src moved to the refined/coarsened mesh new_mesh (Sec. 2.5): located there, reference
    location recomputed, stable sort by new cell; returns the new store."""
    dst = OracleStore(new_mesh.dim, cap or max(src.n, 1), src.n_prop)
    cs = np.zeros(new_mesh.n_cells + 1, np.int64)
    if lib().orc_transfer(C.byref(new_mesh.c), C.byref(src.c), C.byref(dst.c), _p(cs)) != 0:
        raise ValueError("capacity too small")
    dst.cell_start = cs
    return dst


def stable_sort_perm(n_cells, old_cell, key):
    """Permutation of the stable sort by (new cell, moved), lost dropped (Sec. 2.4)."""
    old_cell = np.ascontiguousarray(old_cell, np.int32)
    key = np.ascontiguousarray(key, np.uint32)
    n = key.shape[0]
    perm = np.zeros(max(n, 1), np.int64)
    cs = np.zeros(n_cells + 1, np.int64)
    m = lib().orc_sort_perm(int(n_cells), n, _p(old_cell), _p(key), _p(perm), _p(cs))
    return perm[:m], cs


def seed_per_cell(mesh: OracleMesh, counts, seed_, first_id, n_prop, cap=None, init_position=True):
    """Reference-local generation with the counter hash (Sec. 2.2, remark on local generation):
    particle j of cell K at xhat_a = uniform01(seed, 2^64 - 1, K, j, a), ids first_id + position."""
    counts = np.ascontiguousarray(counts, np.int32)
    n = int(counts.sum())
    st = OracleStore(mesh.dim, cap or max(n, 1), n_prop)
    rc = lib().orc_seed_per_cell(C.byref(mesh.c), _p(counts), int(seed_), int(first_id), int(init_position),
                                 C.byref(st.c))
    if rc != 0:
        raise ValueError("capacity too small" if rc == -1 else "negative count")
    cs = np.zeros(mesh.n_cells + 1, np.int64)
    cs[1:] = np.cumsum(counts)
    st.cell_start = cs
    return st


def population(mesh: OracleMesh, st: OracleStore, pmin, pmax, seed_, step_, next_id):
    """Per-cell population management (Sec. 2.5, 2.6)."""
    nid = np.array([next_id], np.uint64)
    added = np.zeros(1, np.int64)
    deleted = np.zeros(1, np.int64)
    cs = np.ascontiguousarray(st.cell_start, np.int64)
    rc = lib().orc_population(C.byref(mesh.c), C.byref(st.c), _p(cs), int(pmin), int(pmax),
                              int(seed_), int(step_), _p(nid), _p(added), _p(deleted))
    if rc != 0:
        raise ValueError("capacity too small for population management")
    st.cell_start = cs
    return int(nid[0]), int(added[0]), int(deleted[0])


def cell_average(n_cells, st: OracleStore):
    """Arithmetic mean of each property over the particles of each cell (Sec. 2.7 (ii))."""
    out = np.zeros((n_cells, max(st.n_prop, 1)))
    cnt = np.zeros(n_cells, np.int32)
    cs = np.ascontiguousarray(st.cell_start, np.int64)
    lib().orc_cell_average(int(n_cells), _p(cs), C.byref(st.c), _p(out), _p(cnt))
    return out[:, : st.n_prop], cnt


def cell_mean(n_cells, st: OracleStore, mode):
    """Geometric (mode 1) or harmonic (mode 2) mean of each property per cell (Sec. 2.7 (ii))."""
    out = np.zeros((n_cells, max(st.n_prop, 1)))
    cnt = np.zeros(n_cells, np.int32)
    cs = np.ascontiguousarray(st.cell_start, np.int64)
    lib().orc_cell_mean(int(n_cells), _p(cs), C.byref(st.c), int(mode), _p(out), _p(cnt))
    return out[:, : st.n_prop], cnt


INTERP_NEAREST, INTERP_INV_DISTANCE, INTERP_SHAPE = 0, 1, 2


def interp_points(mesh: OracleMesh, st: OracleStore, kind, qhat):
    """Properties at the evaluation points qhat [dim][n_q] (reference coordinates, every cell) from the
    particles of the point's cell (Sec. 2.7 (i), (iii), (iv)); returns [n_cells][n_q][n_prop]."""
    qhat = np.ascontiguousarray(qhat, np.float64)
    n_q = qhat.shape[1]
    out = np.zeros((mesh.n_cells, n_q, max(st.n_prop, 1)))
    cs = np.ascontiguousarray(st.cell_start, np.int64)
    lib().orc_interp_points(C.byref(mesh.c), _p(cs), C.byref(st.c), int(kind), n_q, _p(qhat), _p(out))
    return out[:, :, : st.n_prop]


def seed_mh(mesh: OracleMesh, counts, rho, J, seed, first_id, n_prop, cap=None):
    """Metropolis-Hastings generation in the reference cells (Sec. 2.2); returns (store, longest run)."""
    counts = np.ascontiguousarray(counts, np.int32)
    rho = np.ascontiguousarray(rho, np.float64)
    n = int(counts.sum())
    st = OracleStore(mesh.dim, cap or max(n, 1), n_prop)
    longest = np.zeros(1, np.int64)
    rc = lib().orc_seed_mh(C.byref(mesh.c), _p(counts), _p(rho), int(J), int(seed), int(first_id), C.byref(st.c),
                           _p(longest))
    if rc != 0:
        raise ValueError("capacity too small")
    cs = np.zeros(mesh.n_cells + 1, np.int64)
    cs[1:] = np.cumsum(counts)
    st.cell_start = cs
    return st, int(longest[0])


def linear_least_squares(n_cells, dim, cell_start, xr, prop, rcond=1e-10):
    """Per-cell linear least-squares fit in centred reference coordinates (Sec. 2.7 (v)).

    For each cell minimise sum_k (c0 + sum_i c_i (xhat_ki - xbar_i) - phi_k)^2.
    Falls back to the constant fit (c0 = mean, c = 0) if n < dim + 1 or the
    design matrix has sigma_min / sigma_max < rcond.  Empty cells give NaN.
    Returns coef [n_cells][n_prop][dim+1] and xbar [n_cells][dim].
    """
    n_prop = prop.shape[0]
    cs = np.asarray(cell_start, np.int64)
    counts = np.diff(cs)
    coef = np.full((n_cells, n_prop, dim + 1), np.nan)
    xbar = np.full((n_cells, dim), np.nan)
    for cnt in np.unique(counts):
        if cnt == 0:
            continue
        cells = np.nonzero(counts == cnt)[0]
        idx = cs[cells][:, None] + np.arange(cnt)[None, :]            # [m][cnt]
        X = np.stack([xr[a][idx] for a in range(dim)], axis=-1)        # [m][cnt][dim]
        mean = X.mean(axis=1)                                          # [m][dim]
        Xc = X - mean[:, None, :]
        A = np.concatenate([np.ones((cells.size, cnt, 1)), Xc], axis=-1)   # [m][cnt][dim+1]
        B = np.stack([prop[j][idx] for j in range(n_prop)], axis=-1)   # [m][cnt][n_prop]
        xbar[cells] = mean
        const = B.mean(axis=1)                                         # [m][n_prop]
        if cnt < dim + 1:
            coef[cells, :, 0] = const
            coef[cells, :, 1:] = 0.0
            continue
        Uu, S, Vt = np.linalg.svd(A, full_matrices=False)
        ok = S[:, -1] >= rcond * S[:, 0]
        sol = np.einsum("mji,mj,mkj,mkp->mip", Vt, 1.0 / S, Uu, B)      # [m][dim+1][n_prop]
        c = np.transpose(sol, (0, 2, 1))
        c[~ok, :, 0] = const[~ok]
        c[~ok, :, 1:] = 0.0
        coef[cells] = c
    return coef, xbar


def adjoint(mesh: OracleMesh, U, dt, scheme, n_steps, x0, K0, xr0, target, mask):
    """Loss and dL/dU of the multi-step RK map by a per-particle reverse sweep."""
    U = np.ascontiguousarray(U, np.float64)
    x0 = np.ascontiguousarray(x0, np.float64)
    xr0 = np.ascontiguousarray(xr0, np.float64)
    K0 = np.ascontiguousarray(K0, np.int32)
    target = np.ascontiguousarray(target, np.float64)
    mask = np.ascontiguousarray(mask, np.uint8)
    dU = np.zeros_like(U)
    lost = np.zeros(1, np.int64)
    L = lib().orc_adjoint(C.byref(mesh.c), _p(U), U.shape[1], float(dt), int(scheme), int(n_steps),
                          x0.shape[1], _p(x0), _p(K0), _p(xr0), _p(target), _p(mask), _p(dU), _p(lost))
    return float(L), dU, int(lost[0])


def set_threads(n: int) -> int:
    """Threads of the oracle's OpenMP loops (0: keep); returns the number in use."""
    return int(lib().orc_set_threads(int(n)))


def splitmix64(state: int) -> int:
    return int(lib().orc_splitmix64(C.c_uint64(state & 0xFFFFFFFFFFFFFFFF)))


def uniform01(seed_, step_, cell, slot, coord) -> float:
    return float(lib().orc_uniform01(seed_, step_, cell, slot, coord))


def run(mesh: OracleMesh, U, dt, scheme, steps, st: OracleStore):
    s = Stats()
    for _ in range(steps):
        step(mesh, U, dt, scheme, st, s)
    return s
