"""Edge cases of the property equations, the time-interpolated field, the point interpolators,
Metropolis-Hastings generation and the transfer between meshes: empty stores, all particles lost,
the maximum number of evaluation points, J = 1, zero counts."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
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


def _problem(dim, n, cap, n_prop=10, U=None):
    from paper_1612_03369_amd.api import Problem
    mesh = I.UniformMesh(dim, (n,) * dim)
    p = Problem(0)
    p.mesh_uniform(dim, mesh.n[:dim])
    p.set_velocity(np.zeros((dim, p.n_nodes)) if U is None else U)
    p.allocate(cap, n_prop=n_prop, prop_dtype="float64")
    return mesh, p


def test_empty_store_with_property_equations_and_time_field(L):
    _say("case: empty stores")
    for dim in (2, 3):
        mesh, p = _problem(dim, 4, 16, n_prop=1 + dim * dim)
        p.seed_reference(np.zeros(mesh.n_cells, np.int32), np.zeros((dim, 0)), np.zeros(0, np.uint32),
                         prop=np.zeros((1 + dim * dim, 0)))
        p.set_property_odes(0, 1, 1.0, 1.0)
        p.set_velocity_end(np.ones((dim, p.n_nodes)), 0.5)
        for prec in (L.PIC_F64, L.PIC_F32):
            for scheme in (L.PIC_EULER, L.PIC_RK2, L.PIC_RK4):
                p.advance(0.1, 3, scheme, prec)
        assert p.stats()["live"] == 0
        tau = 0.0
        for _ in range(18):                       # six advances of three steps
            tau = tau + 0.1
        assert p.field_time() == tau
        out, cnt = p.interpolate_points(L.PIC_INTERP_SHAPE_WEIGHTED, np.full((dim, 64), 0.25))
        assert out.shape == (mesh.n_cells, 64, 1 + dim * dim) and bool(out.isnan().all())
        p.close()


def test_everything_leaves_the_domain(L):
    """A uniform field that carries every particle out in one step: all lost, properties untouched."""
    _say("case: all particles lost with the property equations and a time-interpolated field")
    mesh, p = _problem(3, 4, 400, U=None)
    U = np.zeros((3, p.n_nodes))
    U[0] = 5.0
    p.set_velocity(U)
    p.set_velocity_end(U * 2, 1.0)
    counts = np.full(mesh.n_cells, 3, np.int32)
    counts, xr, ids = I.draw_reference_particles(counts, 3, seed=4500)
    P0 = np.zeros((10, xr.shape[1]))
    P0[[1, 5, 9]] = 1.0
    p.seed_reference(counts, xr, ids, prop=P0)
    p.set_property_odes(0, 1, 1.0, 1.0)
    p.advance(0.5, 2, L.PIC_RK4, L.PIC_F64)
    s = p.stats()
    assert s["live"] == 0 and s["lost"] == xr.shape[1]
    p.close()


def test_metropolis_hastings_zero_counts_and_every_state(L):
    _say("case: MH with zero counts and J = 1")
    mesh, p = _problem(2, 5, 300, n_prop=1)
    om = O.OracleMesh.uniform(mesh)
    rho = 1.0 + I.uniform_q2_nodes(mesh)[0]
    zero = np.zeros(mesh.n_cells, np.int32)
    assert p.seed_mh(zero, rho, 3, 1) == 0 and p.stats()["live"] == 0
    counts = np.arange(mesh.n_cells, dtype=np.int32) % 5
    longest = p.seed_mh(counts, rho, 1, 9, first_id=7)
    st, olongest = O.seed_mh(om, counts, rho, 1, 9, 7, 1)
    g = p.numpy()
    assert longest == olongest
    assert np.array_equal(g["xr"], st.view()["xr"]) and np.array_equal(g["id"], st.view()["id"])
    p.close()


def test_transfer_of_an_empty_store(L):
    from paper_1612_03369_amd.api import Problem
    _say("case: transfer of an empty store")
    mesh, a = _problem(2, 3, 10, n_prop=1)
    a.seed_reference(np.zeros(mesh.n_cells, np.int32), np.zeros((2, 0)), np.zeros(0, np.uint32))
    mesh2, b = _problem(2, 6, 10, n_prop=1)
    b.transfer_from(a)
    assert b.stats()["live"] == 0
    a.close()
    b.close()


@pytest.mark.parametrize("n_prop,dtype", [(0, "float32"), (1, "float32"), (4, "float32"), (6, "float32"),
                                          (2, "float64")])
def test_fused_steps_carry_any_number_of_properties(L, n_prop, dtype):
    """The fused kernels carry up to four single-precision properties in
    registers and copy the rest (and double-precision ones) one by one: for
    every count, fused = single steps bit for bit, and each surviving particle
    keeps its seeded values."""
    from paper_1612_03369_amd.api import Problem
    _say(f"case: fused steps with {n_prop} {dtype} properties")
    dim, n, steps = 3, 8, 4
    mesh = I.UniformMesh(dim, (n,) * dim)
    U = I.normalise_nodal(I.sample_nodes(I.FourierField(dim, seed=1600).velocity, I.uniform_q2_nodes(mesh)))
    counts = np.random.default_rng(1601).integers(0, 9, mesh.n_cells).astype(np.int32)
    counts, xr, ids = I.draw_reference_particles(counts, dim, seed=1602)
    npart = xr.shape[1]
    prop = np.random.default_rng(1603).standard_normal((n_prop, npart)).astype(dtype)
    dt = 0.6 / n
    outs = []
    for fused in (True, False):
        p = Problem(0)
        p.mesh_uniform(dim, mesh.n[:dim])
        p.set_velocity(U)
        p.allocate(npart, n_prop=n_prop, prop_dtype=dtype)
        p.seed_reference(counts, xr, ids, prop=prop if n_prop else None, init_position=False)
        if fused:
            p.advance(dt, steps, 4, 1)
        else:
            for _ in range(steps):
                p.advance(dt, 1, 4, 1)
        outs.append(p.numpy())
        p.close()
    g, g1 = outs
    keys = ("x", "xr", "cell", "id") + (("prop",) if n_prop else ())
    for k in keys:
        assert np.array_equal(g[k], g1[k]), k
    if n_prop:
        order = np.argsort(ids)
        pos = order[np.searchsorted(ids[order], g["id"])]
        assert np.array_equal(g["prop"], prop[:, pos])
    _say(f"  {g['id'].size} particles after {steps} fused steps")


@pytest.mark.parametrize("kind", ["uniform", "octree"])
def test_rejected_field_keeps_the_previous_one(L, kind):
    """A field with a NaN or an infinity is rejected (PIC_ENONFINITE) before anything is
    overwritten: the previous field, hanging nodes resolved, stays in use, in both precisions."""
    _say(f"case: rejected non-finite field, {kind}")
    from paper_1612_03369_amd._lib import PicError
    from paper_1612_03369_amd.api import Problem
    from helpers import oracle_run_tracking
    p = Problem(0)
    if kind == "octree":
        lv, an = I.octree_shell_leaves(base_level=1, max_level=4, r_in=0.0, r_out=0.2, width=1.0,
                                       centre=(0.3, 0.35, 0.4))
        lv, an = I.balance_octree(lv, an, 4)
        p.mesh_octree(lv, an, 4)
        om = O.OracleMesh.octree(lv, an, 4)
        nodes = om.q2_node_coords()
        dim = 3
    else:
        mesh = I.UniformMesh(3, (6, 5, 4))
        p.mesh_uniform(3, mesh.n)
        om = O.OracleMesh.uniform(mesh)
        nodes = I.uniform_q2_nodes(mesh)
        dim = 3
    Uraw = I.normalise_nodal(I.sample_nodes(I.FourierField(3, seed=88).velocity, nodes))
    U = om.resolve_hanging(Uraw) if kind == "octree" else Uraw
    p.set_velocity(Uraw)
    bad = Uraw.copy()
    bad[1, 7] = np.nan
    bad[2, -1] = np.inf
    for b in (bad, bad.astype(np.float32)):
        with pytest.raises(PicError) as e:
            p.set_velocity(b)
        assert e.value.status == L.PIC_ENONFINITE
    counts = np.full(om.n_cells, 4, np.int32)
    counts, xr, ids = I.draw_reference_particles(counts, dim, seed=89)
    p.allocate(xr.shape[1], n_prop=0)
    for prec in (L.PIC_F64, L.PIC_F32):
        p.seed_reference(counts, xr, ids)
        p.advance(0.02, 5, L.PIC_RK2, prec)
        g = p.numpy()
        st = O.seed(om, counts, xr, ids, 0)
        near, _ = oracle_run_tracking(om, U, 0.02, 2, 5, st)
        o = st.view()
        common, gi, oi = np.intersect1d(g["id"], o["id"], return_indices=True)
        assert len(common) > 0.9 * xr.shape[1]
        err = np.abs(g["x"][:, gi] - o["x"][:, oi]).max()
        assert err <= (1e-12 if prec == L.PIC_F64 else 1e-6), err
    p.close()


def test_crowded_cells_beyond_the_lds_sort(L):
    """Prescribed locations with thousands of particles in one cell (more than the LDS rank sort
    holds: 5,000 and 9,000 arrivals, one and two LDS tiles): sorted by (cell, input order)."""
    _say("case: 5,000 and 9,000 prescribed points in one cell each")
    from paper_1612_03369_amd.api import Problem
    mesh = I.UniformMesh(3, (4, 4, 4))
    rng = np.random.default_rng(90)
    n = 20000
    x = rng.uniform(0.0, 1.0, size=(3, n))
    x[:, 1000:6000] = rng.uniform(0.26, 0.49, size=(3, 5000))      # cell (1, 1, 1)
    x[:, 8000:17000] = rng.uniform(0.76, 0.99, size=(3, 9000))     # cell (3, 3, 3)
    perm = rng.permutation(n)
    x = np.ascontiguousarray(x[:, perm])
    ids = np.arange(n, dtype=np.uint32)
    p = Problem(0)
    p.mesh_uniform(3, mesh.n)
    p.set_velocity(np.zeros((3, mesh.n_nodes)))
    p.allocate(n, n_prop=1)
    p.seed_positions(x, ids)
    g = p.numpy()
    om = O.OracleMesh.uniform(mesh)
    cell = np.array([om.locate(x[:, i])[0] for i in range(n)])
    exp = np.lexsort((np.arange(n), cell))
    assert np.array_equal(g["id"], ids[exp])
    assert np.array_equal(g["cell"], cell[exp])
    big = np.bincount(cell, minlength=64)
    assert big.max() >= 9000 and np.sort(big)[-2] >= 5000
    # and a step of zero velocity keeps them (stayers in order)
    p.advance(0.01, 2, L.PIC_RK4, L.PIC_F64)
    assert np.array_equal(p.numpy()["id"], ids[exp])
    p.close()
