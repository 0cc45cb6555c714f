"""GPU parity of the field that changes in time (Sec. 2.3): u^n and u^{n+1} evaluated at every stage
point and combined linearly in time, particle steps sub-dividing the field step, extrapolation past
its end, and the shift to the next field step; against the FP64 oracle on uniform, displaced and
octree meshes, with and without the property equations."""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1612_03369_amd import inputs as I

from helpers import compare_stores, oracle_run_tracking

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


def _fields(dim, nodes, seed, k=3):
    return [I.normalise_nodal(I.sample_nodes(I.FourierField(dim, seed=seed + j).velocity, nodes)) for j in range(k)]


def _uniform_case(dim, seed):
    n = 9 if dim == 3 else 19
    mesh = I.UniformMesh(dim, (n,) * dim)
    counts = np.random.default_rng(seed).integers(0, 9, mesh.n_cells).astype(np.int32)
    counts, xr, ids = I.draw_reference_particles(counts, dim, seed=seed + 1)
    return mesh, counts, xr, ids, 0.5 / n


def _gpu(mesh, counts, xr, ids, U, n_prop=1, displace=None, octree=None):
    from paper_1612_03369_amd.api import Problem
    p = Problem(0)
    if octree is not None:
        p.mesh_octree(*octree)
    else:
        p.mesh_uniform(mesh.dim, mesh.n[: mesh.dim])
        if displace is not None:
            p.mesh_displace(displace)
    p.set_velocity(U)
    p.allocate(xr.shape[1], n_prop=n_prop, prop_dtype="float64")
    p.seed_reference(counts, xr, ids)
    return p


def _tau_after(steps, dt, tau=0.0):
    for _ in range(steps):
        tau = tau + dt
    return tau


@pytest.mark.parametrize("dim,scheme,prec", [(3, 4, 0), (3, 2, 0), (3, 1, 0), (2, 4, 0), (2, 2, 0), (3, 4, 1),
                                             (2, 4, 1)])
def test_time_interpolated_field_uniform(L, dim, scheme, prec):
    _say(f"case: field changing in time, uniform dim={dim} scheme={scheme} prec={prec}")
    mesh, counts, xr, ids, dt = _uniform_case(dim, 3000 + 10 * dim + scheme)
    U0, U1, U2 = _fields(dim, I.uniform_q2_nodes(mesh), 3100 + dim)
    dt_u = 4 * dt                           # four particle steps per field step
    om = O.OracleMesh.uniform(mesh)
    results = []
    for fused in (True, False):
        p = _gpu(mesh, counts, xr, ids, U0)
        p.set_velocity_end(U1, dt_u)
        if fused:
            p.advance(dt, 6, scheme, prec)              # the last two steps extrapolate (theta up to 1.5)
        else:
            for _ in range(6):
                p.advance(dt, 1, scheme, prec)
        assert p.field_time() == _tau_after(6, dt)
        g1 = p.numpy()
        p.shift_velocity(U2, 2 * dt_u)                 # next field step, twice as long
        if fused:
            p.advance(dt, 3, scheme, prec)
        else:
            for _ in range(3):
                p.advance(dt, 1, scheme, prec)
        assert p.field_time() == _tau_after(3, dt)
        results.append((g1, p.numpy()))
        p.close()
    # fused steps = single steps, bit for bit
    for a, b in zip(results[0], results[1]):
        for k in ("x", "xr", "cell", "id"):
            assert np.array_equal(a[k], b[k]), k
    g1, g2 = results[0]
    st = O.seed(om, counts, xr, ids, 1)
    tf = dict(U1=U1, dt_u=dt_u, since=0.0)
    near, _ = oracle_run_tracking(om, U0, dt, scheme, 6, st, tfield=tf)
    if prec == 0:
        e1, _ = compare_stores(g1, st.view(), near)
    tf = dict(U1=U2, dt_u=2 * dt_u, since=0.0)
    near2, _ = oracle_run_tracking(om, U1, dt, scheme, 3, st, tfield=tf)
    if prec == 0:
        e2, _ = compare_stores(g2, st.view(), near | near2)
        _say(f"  max position err {e1:.2e} after the first field step, {e2:.2e} after the second")
    else:
        o = st.view()
        common, gi, oi = np.intersect1d(g2["id"], o["id"], return_indices=True)
        d = np.abs(g2["x"][:, gi] - o["x"][:, oi]).max()
        _say(f"  FP32 evaluation: max position err {d:.2e} on {common.size}")
        assert d <= 1e-5


@pytest.mark.parametrize("dim", [2, 3])
def test_equal_end_field_is_the_steady_field(L, dim):
    """u^{n+1} = u^n: every stage sees u^n exactly, so the run equals the steady one bit for bit."""
    from paper_1612_03369_amd import _lib
    _say(f"case: equal end field, dim={dim}")
    mesh, counts, xr, ids, dt = _uniform_case(dim, 3200 + dim)
    U0 = _fields(dim, I.uniform_q2_nodes(mesh), 3210 + dim, 1)[0]
    out = []
    for ti in (False, True):
        p = _gpu(mesh, counts, xr, ids, U0)
        if ti:
            p.set_velocity_end(U0.copy(), 3 * dt)
        p.advance(dt, 5, _lib.PIC_RK4, _lib.PIC_F64)
        out.append(p.numpy())
        p.close()
    for k in ("x", "xr", "cell", "id"):
        assert np.array_equal(out[0][k], out[1][k]), k


def test_time_interpolated_field_displaced_octree_and_property_equations(L):
    from paper_1612_03369_amd import _lib
    _say("case: field changing in time on a displaced mesh, an octree, and with the property equations")
    # displaced 3D, RK4, property equations on
    mesh = I.UniformMesh(3, (6, 5, 4))
    vert = I.displaced_vertices(mesh, 0.15, seed=3301)
    om = O.OracleMesh.displaced(mesh, vert)
    U0, U1, _ = _fields(3, om.q2_node_coords(), 3302)
    counts = np.random.default_rng(3303).integers(0, 7, mesh.n_cells).astype(np.int32)
    counts, xr, ids = I.draw_reference_particles(counts, 3, seed=3304)
    p = _gpu(mesh, counts, xr, ids, U0, n_prop=10, displace=vert)
    P0 = np.zeros((10, xr.shape[1]))
    P0[0] = 0.1
    P0[[1, 5, 9]] = 1.0
    p.seed_reference(counts, xr, ids, prop=P0)
    p.set_property_odes(0, 1, 0.8, 1.7)
    dt, dt_u = 0.06, 0.15
    p.set_velocity_end(U1, dt_u)
    p.advance(dt, 4, _lib.PIC_RK4, _lib.PIC_F64)
    g = p.numpy()
    p.close()
    st = O.seed(om, counts, xr, ids, 10)
    st.prop[:, : st.n] = P0
    near, _ = oracle_run_tracking(om, U0, dt, 4, 4, st, odes=(0.8, 1.7, 0, 1),
                                  tfield=dict(U1=U1, dt_u=dt_u, since=0.0))
    e, _ = compare_stores(g, st.view(), near, check_order=False)
    o = st.view()
    common, gi, oi = np.intersect1d(g["id"], o["id"], return_indices=True)
    keep = ~np.isin(common, np.array(sorted(near), dtype=np.uint32))
    perr = (np.abs(g["prop"][:, gi[keep]] - o["prop"][:, oi[keep]]) / np.maximum(1, np.abs(o["prop"][:, oi[keep]]))).max()
    _say(f"  displaced + property equations: position err {e:.2e}, property err {perr:.2e}")
    assert perr <= 4e-12
    # uniform 3D block kernel with the property equations
    mesh, counts, xr, ids, dt = _uniform_case(3, 3310)
    U0, U1, _ = _fields(3, I.uniform_q2_nodes(mesh), 3320)
    om = O.OracleMesh.uniform(mesh)
    p = _gpu(mesh, counts, xr, ids, U0, n_prop=10)
    P0 = np.zeros((10, xr.shape[1]))
    P0[[1, 5, 9]] = 1.0
    p.seed_reference(counts, xr, ids, prop=P0)
    p.set_property_odes(0, 1, 0.8, 1.7)
    p.set_velocity_end(U1, 3 * dt)
    p.advance(dt, 5, _lib.PIC_RK2, _lib.PIC_F64)
    g = p.numpy()
    p.close()
    st = O.seed(om, counts, xr, ids, 10)
    st.prop[:, : st.n] = P0
    near, _ = oracle_run_tracking(om, U0, dt, 2, 5, st, odes=(0.8, 1.7, 0, 1),
                                  tfield=dict(U1=U1, dt_u=3 * dt, since=0.0))
    e, _ = compare_stores(g, st.view(), near)
    o = st.view()
    common, gi, oi = np.intersect1d(g["id"], o["id"], return_indices=True)
    keep = ~np.isin(common, np.array(sorted(near), dtype=np.uint32))
    perr = (np.abs(g["prop"][:, gi[keep]] - o["prop"][:, oi[keep]]) / np.maximum(1, np.abs(o["prop"][:, oi[keep]]))).max()
    _say(f"  uniform + property equations: position err {e:.2e}, property err {perr:.2e}")
    assert perr <= 4e-12
    # octree, RK2
    level, anchor = I.octree_shell_leaves(base_level=1, max_level=4, r_in=0.0, r_out=0.3, width=1.0,
                                          centre=(0.3, 0.35, 0.4))
    level, anchor = I.balance_octree(level, anchor, 4)
    om = O.OracleMesh.octree(level, anchor, 4)
    nodes = om.q2_node_coords()
    R0, R1, _ = _fields(3, nodes, 3330)
    counts = np.random.default_rng(3334).integers(0, 6, level.size).astype(np.int32)
    counts, xr, ids = I.draw_reference_particles(counts, 3, seed=3335)
    p = _gpu(None, counts, xr, ids, R0, octree=(level, anchor, 4))
    p.set_velocity_end(R1, 0.1)
    dt = 0.5 / 16
    p.advance(dt, 6, _lib.PIC_RK2, _lib.PIC_F64)
    g = p.numpy()
    p.close()
    st = O.seed(om, counts, xr, ids, 1)
    near, _ = oracle_run_tracking(om, om.resolve_hanging(R0), dt, 2, 6, st,
                                  tfield=dict(U1=om.resolve_hanging(R1), dt_u=0.1, since=0.0))
    e, _ = compare_stores(g, st.view(), near, check_order=False)
    _say(f"  octree: position err {e:.2e}")


def test_time_field_argument_checks_and_state(L):
    from paper_1612_03369_amd import _lib
    from paper_1612_03369_amd._lib import PicError
    from paper_1612_03369_amd.api import Batch, Problem
    mesh, counts, xr, ids, dt = _uniform_case(2, 3400)
    U0, U1, _ = _fields(2, I.uniform_q2_nodes(mesh), 3410)
    p = Problem(0)
    p.mesh_uniform(2, mesh.n[:2])
    with pytest.raises(PicError):
        p.set_velocity_end(U1, 1.0)                     # no start field yet
    p.set_velocity(U0)
    p.allocate(xr.shape[1], n_prop=1)
    p.seed_reference(counts, xr, ids)
    with pytest.raises(PicError):
        p.field_time()                                  # steady field
    with pytest.raises(PicError):
        p.shift_velocity(U1, 1.0)
    for bad in (0.0, -1.0, float("nan"), float("inf")):
        with pytest.raises(PicError):
            p.set_velocity_end(U1, bad)
    bad_U = U1.copy()
    bad_U[0, 3] = np.nan
    with pytest.raises(PicError):
        p.set_velocity_end(bad_U, 1.0)
    p.set_velocity_end(U1, 1.0)
    p.set_field_time(0.25)
    assert p.field_time() == 0.25
    p.advance(dt, 2, _lib.PIC_RK2, _lib.PIC_F64)
    assert p.field_time() == (0.25 + dt) + dt
    ws = p.adjoint_workspace(2, 1)
    with pytest.raises(PicError):
        p.advance_checkpointed(dt, 2, _lib.PIC_RK4, 1, ws)
    with pytest.raises(PicError):
        Batch([p])
    p.set_velocity_end(None, 0.0)                       # back to the steady field
    with pytest.raises(PicError):
        p.field_time()
    p.close()


def test_changing_the_field_keeps_the_current_buffer(L):
    """Re-setting the field (or switching the property equations) between steps must keep the
    store's current buffer, which the step kernels flip on the device."""
    from paper_1612_03369_amd import _lib
    _say("case: field re-set after an odd number of steps")
    mesh, counts, xr, ids, dt = _uniform_case(3, 3500)
    U0 = _fields(3, I.uniform_q2_nodes(mesh), 3510, 1)[0]
    out = []
    for reset in (False, True):
        p = _gpu(mesh, counts, xr, ids, U0, n_prop=10)
        if reset:
            p.advance(dt, 3, _lib.PIC_RK4, _lib.PIC_F64)
            p.set_velocity(U0)
            p.set_property_odes(-1, -1)
            p.advance(dt, 2, _lib.PIC_RK4, _lib.PIC_F64)
        else:
            p.advance(dt, 5, _lib.PIC_RK4, _lib.PIC_F64)
        out.append(p.numpy())
        p.close()
    for k in ("x", "xr", "cell", "id"):
        assert np.array_equal(out[0][k], out[1][k]), k
