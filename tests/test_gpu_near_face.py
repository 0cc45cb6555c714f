"""The near-face counter of pic_stats against the oracle (Sec. 2.4: the owning cell of a point on a
face is decided by the half-open rule; particles within 1e-10 of a face, or of the domain boundary,
are counted and reported).

The lattice cases put every particle, every stage point and every end point on dyadic coordinates
(constant field with steps dt u = (3/64, 3/128, 3/256), so that even RK4's sixths and thirds of a
step are dyadic; reference coordinates in multiples of 1/16 on an 8^3 mesh), so both sides compute
them exactly and many particles sit on cell faces and on the boundary: the counts
must agree step for step on every kernel family (the uniform block kernel alone and fused with the
re-sort, single precision, the generic kernel on a displaced mesh, the octree kernel).  The random
cases check the counter where near-face particles are rare.
"""
import sys

import numpy as np
import pytest

from oracle import oracle as O
from paper_1612_03369_amd import inputs as I

from helpers import compare_stores, gpu_problem, oracle_run_tracking, oracle_store

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


N = 8
DT = 1.0 / 32.0
VEL = (1.5, 0.75, 0.375)


def _lattice_particles(seed=71):
    mesh = I.UniformMesh(3, (N, N, N))
    rng = np.random.default_rng(seed)
    counts = rng.integers(3, 9, mesh.n_cells).astype(np.int32)
    n = int(counts.sum())
    xr = rng.integers(0, 16, size=(3, n)) / 16.0
    xr[:, ::5] = 0.0                          # corners of cells (on three faces at once)
    ids = np.arange(n, dtype=np.uint32)
    return mesh, counts, xr, ids


def _oracle_steps(om, U, scheme, st, steps):
    """Per-step near counts and live id sets of the oracle."""
    out = []
    for _ in range(steps):
        tally = {}
        oracle_run_tracking(om, U, DT, scheme, 1, st, tally=tally)
        out.append((tally["near"], set(st.id[: st.n].tolist())))
    return out


def _gpu_problem_kind(kind, mesh, U, counts, xr, ids):
    from paper_1612_03369_amd.api import Problem
    p = Problem(0)
    if kind == "octree":
        g = np.stack(np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")).reshape(3, -1)
        level, anchor = I.morton_sort(np.full(N ** 3, 3), g, 3)
        p.mesh_octree(level, anchor, 3)
        om = O.OracleMesh.octree(level, anchor, 3)
    else:
        p.mesh_uniform(3, mesh.n)
        if kind == "displaced":
            p.mesh_displace(I.uniform_vertices(mesh))
            om = O.OracleMesh.displaced(mesh, I.uniform_vertices(mesh))
        else:
            om = O.OracleMesh.uniform(mesh)
    U = np.stack([np.full(p.n_nodes, v) for v in VEL])
    p.set_velocity(U)
    p.allocate(xr.shape[1], n_prop=0)
    if kind == "octree":
        # the octree numbers its leaves in Morton order: list the particles per leaf
        fine = om.anchor.astype(np.int64)
        leaf_of_uniform = np.empty(N ** 3, np.int64)
        leaf_of_uniform[fine[0] + N * (fine[1] + N * fine[2])] = np.arange(N ** 3)
        cell_u = np.repeat(np.arange(mesh.n_cells), counts)
        cell_o = leaf_of_uniform[cell_u]
        order = np.argsort(cell_o, kind="stable")
        counts = np.bincount(cell_o, minlength=N ** 3).astype(np.int32)
        xr, ids = np.ascontiguousarray(xr[:, order]), ids[order]
    p.seed_reference(counts, xr, ids)
    st = O.seed(om, counts, xr, ids, 0)
    return p, om, U, st


@pytest.mark.parametrize("scheme", [1, 2, 4])
@pytest.mark.parametrize("kind", ["uniform", "displaced", "octree"])
def test_near_face_lattice_single_steps(L, kind, scheme):
    """One step per call (block kernel alone on uniform meshes, the generic and octree kernels
    otherwise): the near-face count of every step equals the oracle's, the live sets agree."""
    _say(f"case: near-face lattice, {kind}, scheme {scheme}, single steps")
    mesh, counts, xr, ids = _lattice_particles()
    p, om, U, st = _gpu_problem_kind(kind, mesh, None, counts, xr, ids)
    steps = 12
    ref = _oracle_steps(om, U, scheme, st, steps)
    total = 0
    for k in range(steps):
        before = p.stats()["near_face"]
        p.advance(DT, 1, scheme, L.PIC_F64)
        got = p.stats()["near_face"] - before
        g = p.numpy()
        assert set(g["id"].tolist()) == ref[k][1], f"step {k}: live sets differ"
        assert got == ref[k][0], f"step {k}: near-face {got} vs oracle {ref[k][0]}"
        total += got
    s = p.stats()
    _say(f"  near-face {total} over {steps} steps, lost {s['lost']}, live {s['live']}")
    assert total > 100 and s["lost"] > 0
    p.close()


@pytest.mark.parametrize("prec", ["f64", "f32"])
@pytest.mark.parametrize("scheme", [1, 2, 4])
def test_near_face_lattice_fused_steps(L, scheme, prec):
    """Several steps per call: the fused re-sort + advect kernel; single precision evaluates the
    dyadic lattice exactly too."""
    _say(f"case: near-face lattice, fused, scheme {scheme}, {prec}")
    mesh, counts, xr, ids = _lattice_particles(seed=72)
    p, om, U, st = _gpu_problem_kind("uniform", mesh, None, counts, xr, ids)
    steps = 12
    ref = _oracle_steps(om, U, scheme, st, steps)
    p.advance(DT, steps, scheme, L.PIC_F64 if prec == "f64" else L.PIC_F32)
    g = p.numpy()
    s = p.stats()
    assert set(g["id"].tolist()) == ref[-1][1]
    want = sum(r[0] for r in ref)
    _say(f"  near-face {s['near_face']} (oracle {want}), lost {s['lost']}")
    assert s["near_face"] == want and want > 100
    p.close()


@pytest.mark.parametrize("case", ["config1", "fourier16_rk4"])
def test_near_face_counter_random_workloads(L, case):
    """Random workloads: the counter equals the oracle's summed per-step count, and lost particles
    are not counted as near-face unless a point of theirs was within the band."""
    _say(f"case: near-face counter, {case}")
    if case == "config1":
        cfg = I.config1()
        scheme, steps, dt = 2, cfg["steps"], cfg["dt"]
    else:
        mesh = I.UniformMesh(3, (16, 16, 16))
        f = I.FourierField(3, seed=17)
        U = I.normalise_nodal(I.sample_nodes(f.velocity, I.uniform_q2_nodes(mesh)))
        counts = np.full(mesh.n_cells, 6, np.int32)
        counts, xr, ids = I.draw_reference_particles(counts, 3, seed=18)
        cfg = dict(mesh=mesh, U=U, counts=counts, xr=xr, ids=ids, n_prop=1, prop_dtype=np.float64)
        scheme, steps, dt = 4, 20, 0.5 / 16
    p = gpu_problem(cfg)
    p.advance(dt, steps, scheme, L.PIC_F64)
    s = p.stats()
    om, st = oracle_store(cfg)
    tally = {}
    near, lost = oracle_run_tracking(om, cfg["U"], dt, scheme, steps, st, tally=tally)
    compare_stores(p.numpy(), st.view(), near)
    _say(f"  near-face {s['near_face']} (oracle {tally['near']}), lost {s['lost']} (oracle {lost})")
    assert s["near_face"] == tally["near"]
    assert s["lost"] > 100 and s["near_face"] < s["lost"] // 10
    p.close()
