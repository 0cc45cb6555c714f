"""Store invariants of uniform meshes after the step sequences (Sec. 2.1 store, Sec. 2.4 location).

On a uniform mesh the advect kernels derive a particle's cell from its place in the cell-sorted store and its
reference coordinates from its position (the closed form that located it), and only the re-sort's gather stores
the two.  After any sequence of steps the stored values must therefore be exactly what the closed form gives for
the stored positions: cell = floor((x - lo) / h) with the upper domain faces closed, x-hat = (x - (lo + i h)) / h.
With lo = 0 and h a power of two (the unit box with 2^k cells, or h = 1 on a box of n cells, which also gives cell
blocks that are ragged at the upper faces) every operation of that formula is exact or singly rounded in both NumPy
and the kernels, so the comparison is bit for bit.  The cell starts must count the cells' particles.
"""
import sys

import numpy as np
import pytest

from paper_1612_03369_amd import inputs as I

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def L():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1612_03369_amd import _lib
    _lib.load()
    return _lib


def _cfg(dim, n, seed, unit_cells=False):
    if unit_cells:                                          # box [0, n]^dim: h = 1
        mesh = I.UniformMesh(dim, (n,) * dim, (0.0,) * dim, (float(n),) * dim)
    else:
        mesh = I.UniformMesh(dim, (n,) * dim)
    f = I.FourierField(dim, seed=seed)
    nodes = I.uniform_q2_nodes(mesh)
    U = I.normalise_nodal(I.sample_nodes(f.velocity, nodes / np.asarray(mesh.hi[:dim])[:, None]))
    counts = np.random.default_rng(seed + 1).integers(0, 12, mesh.n_cells).astype(np.int32)
    counts, xr, ids = I.draw_reference_particles(counts, dim, seed=seed + 2)
    return mesh, U, counts, xr, ids


def _problem(mesh, U, counts, xr, ids):
    from paper_1612_03369_amd.api import Problem
    p = Problem(0)
    p.mesh_uniform(mesh.dim, mesh.n[: mesh.dim], mesh.lo[: mesh.dim], mesh.hi[: mesh.dim])
    p.set_velocity(U)
    p.allocate(xr.shape[1], n_prop=1, prop_dtype="float64")
    p.seed_reference(counts, xr, ids)
    return p


def _check_closed_form(mesh, g):
    dim, n = mesh.dim, np.array(mesh.n[: mesh.dim])
    x = g["x"][:dim]
    hi = np.asarray(mesh.hi[:dim], np.float64)[:, None]
    h = hi / n[:, None]                                      # a power of two, lo = 0
    s = x / h                                                # (x - lo) / h, exact
    ijk = np.minimum(np.floor(s).astype(np.int64), n[:, None] - 1)
    assert (ijk >= 0).all() and (x <= hi).all()
    cell = ijk[0] + n[0] * ijk[1] + (n[0] * n[1] * ijk[2] if dim == 3 else 0)
    assert np.array_equal(g["cell"].astype(np.int64), cell), "stored cell differs from the closed form"
    xr = (x - ijk * h) / h
    assert np.array_equal(g["xr"][:dim], xr), "stored reference coordinates differ from the closed form"
    cnt = np.bincount(cell, minlength=mesh.n_cells)
    cs = g["cell_start"].astype(np.int64)
    assert np.array_equal(np.diff(cs), cnt) and cs[0] == 0


@pytest.mark.parametrize("dim,n,prec,unit_cells", [(3, 16, "f32", False), (3, 16, "f64", False),
                                                   (2, 32, "f64", False), (2, 32, "f32", False),
                                                   (3, 13, "f32", True), (2, 37, "f32", True), (3, 11, "f64", True)])
def test_stored_cell_and_reference_coordinates_after_fused_steps(L, dim, n, prec, unit_cells):
    _say(f"case: store invariants after fused RK4 steps, {dim}D n={n} {prec}" + (", h = 1" if unit_cells else ""))
    mesh, U, counts, xr, ids = _cfg(dim, n, 300 + dim, unit_cells)
    p = _problem(mesh, U, counts, xr, ids)
    h = mesh.hi[0] / n
    p.advance(0.5 * h, 9, L.PIC_RK4, L.PIC_F32 if prec == "f32" else L.PIC_F64)
    g = p.numpy()
    assert g["id"].size > 0.7 * ids.size
    _check_closed_form(mesh, g)
    p.advance(0.5 * h, 1, L.PIC_RK2, L.PIC_F64)             # a single (unfused) step
    _check_closed_form(mesh, p.numpy())
    p.close()


def test_stored_cell_and_reference_coordinates_after_batched_steps(L):
    from paper_1612_03369_amd.api import Batch
    _say("case: store invariants after batched steps (2D and 3D, RK2 and RK4)")
    cfgs = [_cfg(2, 32, 310), _cfg(3, 8, 311), _cfg(3, 16, 312)]
    probs = [_problem(*c) for c in cfgs]
    b = Batch(probs)
    b.advance([0.5 / c[0].n[0] for c in cfgs], [4, 2, 4], 6)
    for c, p in zip(cfgs, probs):
        _check_closed_form(c[0], p.numpy())
    b.close()
    for p in probs:
        p.close()
