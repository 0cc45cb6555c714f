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
