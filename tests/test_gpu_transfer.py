"""GPU parity of particle transfer after mesh refinement and coarsening (Sec. 2.5): particles of the
old mesh located in the new one (children of refined cells, parents of coarsened ones), reference
locations recomputed, stable by new cell; then population management on the new mesh, against the
FP64 oracle."""
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


def _octree_problem(level, anchor, cap, n_prop=2):
    from paper_1612_03369_amd.api import Problem
    p = Problem(0)
    p.mesh_octree(level, anchor, 4)
    p.set_velocity(np.zeros((3, p.n_nodes)))
    p.allocate(cap, n_prop=n_prop, prop_dtype="float64")
    return p


def _compare(g, o, tol_xr=4e-15):
    assert g["n"] == o["id"].size
    assert np.array_equal(g["cell_start"], o["cell_start"].astype(g["cell_start"].dtype))
    for k in ("id", "cell"):
        assert np.array_equal(g[k], o[k]), k
    # locations are copied, so they differ only as the two sides' seeding rounded them
    assert np.abs(g["x"] - o["x"]).max() <= 2e-16
    assert np.abs(g["prop"] - o["prop"]).max() <= 2e-16
    return np.abs(g["xr"] - o["xr"]).max()


def _numpy(p):
    g = p.numpy()
    g["cell_start"] = np.asarray(g["cell_start"])
    return g


@pytest.mark.parametrize("op", ["refine", "coarsen"])
def test_transfer_matches_oracle_then_population(L, op):
    _say(f"case: transfer after {op}")
    level, anchor = I.octree_shell_leaves(base_level=1, max_level=4, r_in=0.0, r_out=0.3, width=1.0,
                                          centre=(0.3, 0.35, 0.4))
    level, anchor = I.balance_octree(level, anchor, 4)
    # a 2:1-balanced refinement of every third leaf; coarsening is the way back
    fl, fa = I.refine_leaves(level, anchor, 4, (np.arange(level.size) % 3 == 0) & (level < 4))
    fl, fa = I.balance_octree(fl, fa, 4)
    if op == "refine":
        nl, na = fl, fa
    else:
        level, anchor, nl, na = fl, fa, level, anchor
    counts = np.random.default_rng(4100).integers(0, 12, level.size).astype(np.int32)
    counts, xr, ids = I.draw_reference_particles(counts, 3, seed=4101)
    n = xr.shape[1]
    cap = 12 * max(level.size, nl.size) + n
    old = _octree_problem(level, anchor, cap)
    rng = np.random.default_rng(4102)
    P0 = rng.uniform(0.0, 1.0, (2, n))
    old.seed_reference(counts, xr, ids, prop=P0)
    new = _octree_problem(nl, na, cap)
    new.transfer_from(old)
    g = _numpy(new)
    om = O.OracleMesh.octree(level, anchor, 4)
    nm = O.OracleMesh.octree(nl, na, 4)
    st = O.seed(om, counts, xr, ids, 2, cap=cap)
    st.prop[:, :n] = P0
    dst = O.transfer(nm, st, cap=cap)
    e = _compare(g, dst.view())
    _say(f"  {g['n']} particles on {nl.size} leaves (from {level.size}); reference locations within {e:.1e}")
    assert e <= 4e-15
    # the source is unchanged
    go = _numpy(old)
    assert np.array_equal(go["id"], ids) and go["n"] == n
    # more particles in the refined cells / fewer in the merged ones: population on the new mesh
    new.population(6, 10, 77, 0)
    nid, added, deleted = O.population(nm, dst, 6, 10, 77, 0, int(ids.max()) + 1)
    g = _numpy(new)
    o = dst.view()
    assert np.array_equal(g["id"], o["id"]) and np.array_equal(g["cell"], o["cell"])
    assert np.abs(g["x"] - o["x"]).max() <= 1e-15 and np.abs(g["prop"] - o["prop"]).max() <= 1e-15
    s = new.stats()
    _say(f"  population: added {s['added']} (oracle {added}), deleted {s['deleted']} (oracle {deleted})")
    assert s["added"] == added and s["deleted"] == deleted
    old.close()
    new.close()


def test_transfer_uniform_refinement_and_checks(L):
    from paper_1612_03369_amd._lib import PicError
    from paper_1612_03369_amd.api import Problem
    _say("case: transfer 2D 6x5 -> 12x10")
    a = I.UniformMesh(2, (6, 5))
    b = I.UniformMesh(2, (12, 10))
    counts = np.random.default_rng(4200).integers(0, 9, a.n_cells).astype(np.int32)
    counts, xr, ids = I.draw_reference_particles(counts, 2, seed=4201)
    n = xr.shape[1]
    pa, pb = Problem(0), Problem(0)
    pa.mesh_uniform(2, a.n[:2])
    pb.mesh_uniform(2, b.n[:2])
    for p in (pa, pb):
        p.set_velocity(np.zeros((2, p.n_nodes)))
        p.allocate(n, n_prop=1, prop_dtype="float64")
    pa.seed_reference(counts, xr, ids)
    pb.transfer_from(pa)
    g = _numpy(pb)
    st = O.seed(O.OracleMesh.uniform(a), counts, xr, ids, 1)
    dst = O.transfer(O.OracleMesh.uniform(b), st)
    e = _compare(g, dst.view())
    _say(f"  reference locations within {e:.1e}")
    assert e <= 4e-15
    # mismatches: property count, dimension, capacity
    pc = Problem(0)
    pc.mesh_uniform(2, b.n[:2])
    pc.set_velocity(np.zeros((2, pc.n_nodes)))
    pc.allocate(n, n_prop=2, prop_dtype="float64")
    with pytest.raises(PicError):
        pc.transfer_from(pa)
    pc.allocate(max(n // 2, 1), n_prop=1, prop_dtype="float64")
    with pytest.raises(PicError):
        pc.transfer_from(pa)
    p3 = Problem(0)
    p3.mesh_uniform(3, (3, 3, 3))
    p3.set_velocity(np.zeros((3, p3.n_nodes)))
    p3.allocate(n, n_prop=1, prop_dtype="float64")
    with pytest.raises(PicError):
        p3.transfer_from(pa)
    for p in (pa, pb, pc, p3):
        p.close()
