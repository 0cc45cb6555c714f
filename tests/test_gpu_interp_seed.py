"""GPU parity of the remaining particle->field interpolators (Sec. 2.7: geometric and harmonic cell
means; nearest-neighbour, inverse-distance and shape-function-weighted values at evaluation points)
and of Metropolis-Hastings generation (Sec. 2.2), against the FP64 oracle on the same stores."""
import math
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


def _gauss_points(dim):
    g = 1 / math.sqrt(3)
    pts = np.array(list(np.ndindex(*(2,) * dim)), float).T
    return np.concatenate([0.5 + (pts - 0.5) * g, np.full((dim, 1), 0.5), np.zeros((dim, 1))], axis=1)


def _case(kind, dim, seed):
    """(om, gpu mesh set-up, counts, xr, ids) for a uniform, displaced or octree mesh."""
    rng = np.random.default_rng(seed)
    if kind == "octree":
        level, anchor = I.octree_shell_leaves(base_level=1, max_level=4, r_in=0.0, r_out=0.3, width=1.0,
                                              centre=(0.3, 0.35, 0.4))
        level, anchor = I.balance_octree(level, anchor, 4)
        om = O.OracleMesh.octree(level, anchor, 4)
        setup = lambda p: p.mesh_octree(level, anchor, 4)
        n_cells = level.size
    else:
        mesh = I.UniformMesh(dim, (7, 6) if dim == 2 else (5, 4, 3))
        if kind == "displaced":
            vert = I.displaced_vertices(mesh, 0.2, seed=seed + 1)
            om = O.OracleMesh.displaced(mesh, vert)

            def setup(p):
                p.mesh_uniform(dim, mesh.n[:dim])
                p.mesh_displace(vert)
        else:
            om = O.OracleMesh.uniform(mesh)
            setup = lambda p: p.mesh_uniform(dim, mesh.n[:dim])
        n_cells = mesh.n_cells
    counts = rng.integers(0, 9, n_cells).astype(np.int32)
    counts[:3] = [0, 1, 40]                          # empty, single and crowded cells
    counts, xr, ids = I.draw_reference_particles(counts, om.dim, seed=seed + 2)
    P = rng.uniform(0.25, 3.0, (3, xr.shape[1]))
    return om, setup, counts, xr, ids, P


def _gpu_store(setup, counts, xr, ids, P, nn):
    from paper_1612_03369_amd.api import Problem
    p = Problem(0)
    setup(p)
    p.set_velocity(np.zeros((p.dim, p.n_nodes)))
    p.allocate(max(xr.shape[1], 1), n_prop=3, prop_dtype="float64")
    p.seed_reference(counts, xr, ids, prop=P)
    return p


@pytest.mark.parametrize("kind,dim", [("uniform", 2), ("uniform", 3), ("displaced", 2), ("displaced", 3),
                                      ("octree", 3)])
def test_interpolators_match_oracle(L, kind, dim):
    _say(f"case: interpolators on a {kind} {dim}D mesh")
    om, setup, counts, xr, ids, P = _case(kind, dim, 3600 + dim + (10 if kind == "displaced" else 0))
    p = _gpu_store(setup, counts, xr, ids, P, None)
    st = O.seed(om, counts, xr, ids, 3)
    st.prop[:, : st.n] = P
    for mode, gk in ((1, L.PIC_INTERP_GEOMETRIC_AVERAGE), (2, L.PIC_INTERP_HARMONIC_AVERAGE)):
        g, _, cnt = p.interpolate(gk)
        o, ocnt = O.cell_mean(om.n_cells, st, mode)
        g = g.cpu().numpy()
        assert np.array_equal(cnt.cpu().numpy(), ocnt)
        assert np.array_equal(np.isnan(g), np.isnan(o))
        ok = ~np.isnan(o)
        assert np.all(np.abs(g[ok] - o[ok]) <= 1e-13 * np.abs(o[ok])), np.abs(g[ok] - o[ok]).max()
    q = _gauss_points(om.dim)
    for ok_kind, gk, tol in ((O.INTERP_NEAREST, L.PIC_INTERP_NEAREST, 0.0),
                             (O.INTERP_INV_DISTANCE, L.PIC_INTERP_INV_DISTANCE, 1e-12),
                             (O.INTERP_SHAPE, L.PIC_INTERP_SHAPE_WEIGHTED, 1e-13)):
        g, cnt = p.interpolate_points(gk, q)
        g = g.cpu().numpy()
        o = O.interp_points(om, st, ok_kind, q)
        assert np.array_equal(np.isnan(g), np.isnan(o))
        ok = ~np.isnan(o)
        err = np.abs(g[ok] - o[ok]) / np.maximum(1.0, np.abs(o[ok]))
        assert err.max() <= tol, (gk, err.max())
        _say(f"  kind {gk}: max relative difference {err.max():.2e}")
    p.close()


def test_interpolators_full_size_benchmark_store(L):
    """The 64^3 benchmark workload's seeded store (5,242,880 particles, three f64 properties): every
    cell and 10 evaluation points against the oracle."""
    _say("case: interpolators on the 64^3 store")
    cfg = I.config2()
    mesh = cfg["mesh"]
    rng = np.random.default_rng(3700)
    n = cfg["xr"].shape[1]
    P = rng.uniform(0.25, 3.0, (3, n))
    p = _gpu_store(lambda q: q.mesh_uniform(3, mesh.n), cfg["counts"], cfg["xr"], cfg["ids"], P, None)
    om = O.OracleMesh.uniform(mesh)
    st = O.seed(om, cfg["counts"], cfg["xr"], cfg["ids"], 3)
    st.prop[:, :n] = P
    g, _, _ = p.interpolate(L.PIC_INTERP_HARMONIC_AVERAGE)
    o, _ = O.cell_mean(om.n_cells, st, 2)
    assert np.abs(g.cpu().numpy() - o).max() <= 1e-13 * np.abs(o).max()
    q = _gauss_points(3)
    for ok_kind, gk, tol in ((O.INTERP_NEAREST, L.PIC_INTERP_NEAREST, 0.0),
                             (O.INTERP_SHAPE, L.PIC_INTERP_SHAPE_WEIGHTED, 1e-13)):
        g, _ = p.interpolate_points(gk, q)
        o = O.interp_points(om, st, ok_kind, q)
        err = (np.abs(g.cpu().numpy() - o) / np.maximum(1.0, np.abs(o))).max()
        _say(f"  kind {gk}: max relative difference {err:.2e}")
        assert err <= tol
    p.close()


@pytest.mark.parametrize("kind,dim", [("uniform", 2), ("uniform", 3), ("displaced", 3), ("octree", 3)])
def test_metropolis_hastings_matches_oracle(L, kind, dim):
    _say(f"case: Metropolis-Hastings generation on a {kind} {dim}D mesh")
    from paper_1612_03369_amd.api import Problem
    om, setup, counts, _, _, _ = _case(kind, dim, 3800 + dim)
    nodes = om.q2_node_coords()
    # a density with zero and negative regions
    rho = np.sin(3.0 * nodes[0] + 1.0) + 0.6 * np.cos(2.0 * nodes[1]) + (0.3 * nodes[2] if om.dim == 3 else 0)
    J, seed, first = 7, 3810 + dim, 500
    p = Problem(0)
    setup(p)
    p.set_velocity(np.zeros((p.dim, p.n_nodes)))
    p.allocate(int(counts.sum()) + 5, n_prop=2, prop_dtype="float32")
    longest = p.seed_mh(counts, rho, J, seed, first)
    g = p.numpy()
    st, olongest = O.seed_mh(om, counts, rho, J, seed, first, 2)
    o = st.view()
    assert longest == olongest
    assert np.array_equal(g["cell_start"].cpu().numpy() if hasattr(g["cell_start"], "cpu") else g["cell_start"],
                          st.cell_start)
    for k in ("xr", "cell", "id"):
        assert np.array_equal(g[k], o[k]), k
    assert np.abs(g["x"] - o["x"]).max() <= 1e-15
    assert np.abs(g["prop"] - o["prop"]).max() <= 1e-6          # float32 properties
    _say(f"  {st.n} particles, longest run {longest}, positions bit-identical in reference coordinates")
    s = p.stats()
    assert s["live"] == st.n
    p.close()


def test_interpolation_and_generation_argument_checks(L):
    from paper_1612_03369_amd._lib import PicError
    om, setup, counts, xr, ids, P = _case("uniform", 2, 3900)
    p = _gpu_store(setup, counts, xr, ids, P, None)
    q = _gauss_points(2)
    with pytest.raises(PicError):
        p.interpolate_points(L.PIC_INTERP_CELL_AVERAGE, q)     # not a point interpolator
    with pytest.raises(PicError):
        p.interpolate_points(L.PIC_INTERP_NEAREST, np.full((2, 65), 0.5))
    with pytest.raises(PicError):
        p.interpolate_points(L.PIC_INTERP_NEAREST, np.array([[0.5], [1.5]]))
    rho = np.ones(p.n_nodes)
    with pytest.raises(PicError):
        p.seed_mh(counts, rho, 0, 1)                            # J < 1
    with pytest.raises(PicError):
        p.seed_mh(counts * 0 + 10 ** 6, rho, 1, 1)             # over capacity
    bad = rho.copy()
    bad[3] = np.inf
    with pytest.raises(PicError):
        p.seed_mh(counts, bad, 2, 1)
    with pytest.raises(PicError):
        p.seed_mh(counts, rho, 2, 1, first_id=2 ** 32 - 10)     # ids would overflow
    p.close()


# ----------------------------------------------------------------------------
# reference-local generation with the library's counter hash (Sec. 2.2)
# ----------------------------------------------------------------------------
@pytest.mark.parametrize("kind,dim", [("uniform", 2), ("uniform", 3), ("displaced", 3), ("octree", 3)])
def test_seed_per_cell_matches_oracle(L, kind, dim):
    """pic_seed_per_cell: reference coordinates, ids and cells bit-identical to the oracle's
    counter-hash generation; locations Phi_K(xhat) within a few ulps; properties = locations."""
    _say(f"case: seed per cell, {kind} {dim}D")
    from paper_1612_03369_amd.api import Problem
    p = Problem(0)
    if kind == "octree":
        lv, an = I.octree_shell_leaves(base_level=1, max_level=4, r_in=0.0, r_out=0.2, width=1.0,
                                       centre=(0.3, 0.35, 0.4))
        lv, an = I.balance_octree(lv, an, 4)
        p.mesh_octree(lv, an, 4)
        om = O.OracleMesh.octree(lv, an, 4)
    else:
        mesh = I.UniformMesh(dim, (9, 7, 6)[:dim])
        p.mesh_uniform(dim, mesh.n[:dim])
        om = O.OracleMesh.uniform(mesh)
        if kind == "displaced":
            vert = I.displaced_vertices(mesh, 0.2, seed=77)
            p.mesh_displace(vert)
            om = O.OracleMesh.displaced(mesh, vert)
    nc = om.n_cells
    counts = np.random.default_rng(78).integers(0, 25, nc).astype(np.int32)
    counts[::11] = 0
    n = int(counts.sum())
    p.set_velocity(np.zeros((dim, p.n_nodes)))
    p.allocate(30 * nc, n_prop=dim + 1, prop_dtype="float64")
    p.seed_per_cell(counts, seed=2024, first_id=17)
    g = p.numpy()
    st = O.seed_per_cell(om, counts, 2024, 17, dim + 1)
    o = st.view()
    assert g["n"] == n == st.n
    assert np.array_equal(g["id"], o["id"]) and np.array_equal(g["cell"], o["cell"])
    assert np.array_equal(g["xr"], o["xr"])
    assert np.array_equal(g["cell_start"], st.cell_start)
    err = (np.abs(g["x"] - o["x"]) / np.maximum(1.0, np.abs(o["x"]))).max()
    assert err <= 1e-15, err
    assert np.abs(g["prop"] - o["prop"]).max() <= 1e-15
    # the next id continues after the generated ones: population adds ids from there
    p.population(max(1, int(counts.max())), 1000, 5, 0)
    assert p.numpy()["id"].max() >= 17 + n
    _say(f"  {n} particles identical in reference coordinates, ids and cells; location err {err:.1e}")
    p.close()


def test_seed_per_cell_argument_checks(L):
    _say("case: seed per cell argument checks")
    from paper_1612_03369_amd._lib import PicError
    from paper_1612_03369_amd.api import Problem
    p = Problem(0)
    p.mesh_uniform(2, (4, 4))
    p.set_velocity(np.zeros((2, p.n_nodes)))
    p.allocate(50, n_prop=0)
    with pytest.raises(PicError) as e:
        p.seed_per_cell(np.full(16, 4, np.int32), seed=1)           # 64 > capacity 50
    assert e.value.status == L.PIC_ECAPACITY
    bad = np.full(16, 1, np.int32)
    bad[3] = -1
    with pytest.raises(PicError) as e:
        p.seed_per_cell(bad, seed=1)
    assert e.value.status == L.PIC_EINVAL
    with pytest.raises(PicError) as e:
        p.seed_per_cell(np.full(16, 1, np.int32), seed=1, first_id=0xFFFFFFF8)
    assert e.value.status == L.PIC_EINVAL
    p.seed_per_cell(np.zeros(16, np.int32), seed=1)
    assert p.numpy()["n"] == 0
    p.close()
