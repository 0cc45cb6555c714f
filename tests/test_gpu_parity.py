"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Bars: positions within 1e-12 relative (FP64 evaluation), cells and sort
order bit-exact except for particles the oracle saw within 1e-10 of a face,
counts exact.  FP32 evaluation: p99 1e-6 / max 1e-5 absolute against the FP64
oracle.
"""
import math
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


def test_config1_rotation_rk2_full(L):
    """32x32 rigid rotation, 16 per cell, RK2 x 100 steps, cell average (full workload)."""
    _say("case: config1 full, 16384 particles, 100 RK2 steps")
    cfg = I.config1()
    p = gpu_problem(cfg)
    p.advance(cfg["dt"], cfg["steps"], L.PIC_RK2, L.PIC_F64)
    avg, _, cnt = p.interpolate(L.PIC_INTERP_CELL_AVERAGE)
    g = p.numpy()
    st_g = p.stats()
    om, st = oracle_store(cfg)
    near, lost = oracle_run_tracking(om, cfg["U"], cfg["dt"], 2, cfg["steps"], st)
    o = st.view()
    err, nn = compare_stores(g, o, near)
    _say(f"  live {g['n']} (oracle {st.n}), lost {st_g['lost']} (oracle {lost}), max err {err:.2e}, near {nn}")
    assert st_g["lost"] + g["n"] == cfg["xr"].shape[1]
    assert st_g["steps"] == cfg["steps"]
    # lost counts differ only through particles the oracle saw near a face (the live sets were
    # compared above); cell counts and averages are compared on every cell that holds no such
    # particle on either side
    assert abs(st_g["lost"] - lost) <= len(near)
    oavg, ocnt = O.cell_average(om.n_cells, st)
    nid = np.array(sorted(near), dtype=np.int64)
    touched = np.zeros(om.n_cells, bool)
    touched[g["cell"][np.isin(g["id"], nid)]] = True
    touched[o["cell"][np.isin(o["id"], nid)]] = True
    c = cnt.cpu().numpy()
    assert np.array_equal(c[~touched], ocnt[~touched])
    a = avg.cpu().numpy()[:, 0]
    ok = (ocnt > 0) & ~touched
    assert np.all(np.isnan(a[(ocnt == 0) & ~touched]))
    assert np.allclose(a[ok], oavg[ok, 0], rtol=1e-13, atol=1e-15)
    assert (~touched).sum() > 0.9 * om.n_cells
    p.close()


@pytest.mark.parametrize("scheme", [1, 2, 4])
@pytest.mark.parametrize("dim", [2, 3])
def test_fourier_small_fp64(L, scheme, dim):
    """Random divergence-free field, tiles and ragged tails, every scheme, FP64 evaluation."""
    _say(f"case: fourier dim={dim} scheme={scheme}")
    n = 21 if dim == 2 else 10                      # not multiples of the cell-block edges: ragged blocks
    mesh = I.UniformMesh(dim, (n,) * dim)
    f = I.FourierField(dim, seed=31 + dim)
    U = I.normalise_nodal(I.sample_nodes(f.velocity, I.uniform_q2_nodes(mesh)))
    rng = np.random.default_rng(40 + dim)
    counts = rng.integers(0, 13, mesh.n_cells).astype(np.int32)
    counts, xr, ids = I.draw_reference_particles(counts, dim, seed=50 + dim)
    cfg = dict(mesh=mesh, U=U, counts=counts, xr=xr, ids=ids, n_prop=2, prop_dtype=np.float64)
    p = gpu_problem(cfg, capacity=xr.shape[1] + 77)
    dt, steps = 0.5 / n, 12
    p.advance(dt, steps, scheme, L.PIC_F64)
    g = p.numpy()
    om, st = oracle_store(cfg)
    near, lost = oracle_run_tracking(om, U, dt, scheme, steps, st)
    err, nn = compare_stores(g, st.view(), near)
    # properties carried unchanged: initial position
    gi = np.argsort(g["id"])
    o = st.view()
    oi = np.argsort(o["id"])
    common = np.intersect1d(g["id"], o["id"])
    gsel = gi[np.searchsorted(g["id"][gi], common)]
    osel = oi[np.searchsorted(o["id"][oi], common)]
    # seeded from x = Phi_K(xr): equal up to the rounding of the map (FMA or not)
    assert np.abs(g["prop"][:, gsel] - o["prop"][:, osel]).max() <= 4e-16
    _say(f"  live {g['n']}, max err {err:.2e}, near {nn}")
    p.close()


@pytest.mark.parametrize("dim,cfl", [(3, 0.6), (3, 2.5), (2, 0.6), (2, 2.5)])
def test_box_domain_and_long_steps(L, dim, cfl):
    """Non-cubic cell counts, a box that is not the unit cube, anisotropic cells, and steps long
    enough (CFL 2.5) that stage points leave the cell block's node window: fused RK4, FP64,
    against the oracle."""
    _say(f"case: box domain dim={dim} cfl={cfl}")
    n = (9, 6, 5)[:dim]
    lo = (-1.0, 0.5, 2.0)[:dim]
    hi = (2.0, 1.5, 3.0)[:dim]
    mesh = I.UniformMesh(dim, n, lo, hi)
    f = I.FourierField(dim, seed=950 + dim)
    nodes = I.uniform_q2_nodes(mesh)
    # the field lives on the unit box: map the mesh nodes there first
    unit = (nodes - np.array(lo)[:, None]) / (np.array(hi) - np.array(lo))[:, None]
    U = I.normalise_nodal(I.sample_nodes(f.velocity, unit))
    counts = np.random.default_rng(951).integers(0, 11, mesh.n_cells).astype(np.int32)
    counts, xr, ids = I.draw_reference_particles(counts, dim, seed=952)
    cfg = dict(mesh=mesh, U=U, counts=counts, xr=xr, ids=ids, n_prop=1, prop_dtype=np.float64)
    h_min = min((b - a) / k for a, b, k in zip(lo, hi, n))
    dt, steps = cfl * h_min, 6
    p = gpu_problem(cfg)
    p.advance(dt, steps, L.PIC_RK4, L.PIC_F64)
    g = p.numpy()
    om, st = oracle_store(cfg)
    near, lost = oracle_run_tracking(om, U, dt, 4, steps, st)
    err, nn = compare_stores(g, st.view(), near)
    s = p.stats()
    _say(f"  live {g['n']}, lost {s['lost']} (oracle {lost}), moved {s['moved']}, max err {err:.2e}, near {nn}")
    assert s["moved"] > 0
    p.close()


@pytest.mark.parametrize("dim,n,per_cell,steps", [(3, 12, 9, 6),
                                                  # more than 2^19 cells: the scan's long chunks
                                                  (2, 768, 2, 3)])
def test_sort_is_pure_function_of_gpu_keys(L, dim, n, per_cell, steps):
    """Each step's new order = stable sort of the previous order by (new cell, moved): a property
    of the GPU's own keys, checked with NumPy's stable argsort (the oracle is not involved)."""
    _say(f"case: sort permutation vs a stable argsort of the GPU's own keys, {dim}D n={n}")
    mesh = I.UniformMesh(dim, (n,) * dim)
    f = I.FourierField(dim, seed=77)
    U = I.normalise_nodal(I.sample_nodes(f.velocity, I.uniform_q2_nodes(mesh)))
    counts = np.full(mesh.n_cells, per_cell, np.int32)
    counts, xr, ids = I.draw_reference_particles(counts, dim, seed=78)
    cfg = dict(mesh=mesh, U=U, counts=counts, xr=xr, ids=ids, n_prop=0, prop_dtype=np.float64)
    p = gpu_problem(cfg)
    for step in range(steps):
        a = p.numpy()
        p.advance(1.2 / n, 1, L.PIC_RK4, L.PIC_F64)         # CFL 1.2: many movers, some two cells away
        b = p.numpy()
        pos = {int(i): k for k, i in enumerate(b["id"])}
        lost = np.uint32(0xFFFFFFFF)
        key = np.array([b["cell"][pos[int(i)]] if int(i) in pos else lost for i in a["id"]], np.uint32)
        live = key != lost
        moved = live & (key != a["cell"].astype(np.uint32))
        sort_key = 2 * key.astype(np.int64) + moved              # (new cell, moved), lexicographic
        order = np.argsort(sort_key, kind="stable")
        perm = order[live[order]]
        assert np.array_equal(b["id"], a["id"][perm])
        cs = np.zeros(mesh.n_cells + 1, np.int64)
        cs[1:] = np.cumsum(np.bincount(key[live].astype(np.int64), minlength=mesh.n_cells))
        assert np.array_equal(b["cell_start"], cs.astype(np.int32))
        assert moved.sum() > 100
    p.close()


@pytest.mark.parametrize("tile", [1, 16, 100, 300])
def test_results_independent_of_the_tile(L, tile):
    """The work tiles (placement runs, fix ranges, generic advect) change the launch shape only: a
    run with tiles of 1, 16, 100 or 300 cells (partial placement runs, runs that cross no tile
    boundary) equals the run with the default tile bit for bit, single and fused steps."""
    _say(f"case: tile of {tile} cells vs the default tile")
    mesh = I.UniformMesh(3, (12, 12, 12))
    f = I.FourierField(3, seed=81)
    U = I.normalise_nodal(I.sample_nodes(f.velocity, I.uniform_q2_nodes(mesh)))
    counts = np.random.default_rng(82).integers(0, 14, mesh.n_cells).astype(np.int32)
    counts, xr, ids = I.draw_reference_particles(counts, 3, seed=83)
    cfg = dict(mesh=mesh, U=U, counts=counts, xr=xr, ids=ids, n_prop=1, prop_dtype=np.float64)
    out = []
    for t in (None, tile):
        p = gpu_problem(cfg)
        if t is not None:
            p.set_tile(t)
        p.advance(1.2 / 12, 1, L.PIC_RK4, L.PIC_F64)
        p.advance(1.2 / 12, 5, L.PIC_RK4, L.PIC_F32)
        out.append((p.numpy(), p.stats()))
        p.close()
    (a, sa), (b, sb) = out
    for k in ("x", "xr", "cell", "id", "prop", "cell_start"):
        assert np.array_equal(a[k], b[k]), k
    assert sa["moved"] == sb["moved"] and sa["lost"] == sb["lost"] and sa["moved"] > 100


def test_empty_single_and_all_lost(L):
    _say("case: empty store, one particle, everything lost")
    mesh = I.UniformMesh(2, (5, 3))
    U = np.zeros((2, mesh.n_nodes))
    U[0] = 1.0
    # empty
    cfg = dict(mesh=mesh, U=U, counts=np.zeros(mesh.n_cells, np.int32), xr=np.zeros((2, 0)),
               ids=np.zeros(0, np.uint32), n_prop=1, prop_dtype=np.float64)
    p = gpu_problem(cfg, capacity=8)
    p.advance(0.1, 3, L.PIC_RK4, L.PIC_F64)
    assert p.numpy()["n"] == 0
    avg, _, cnt = p.interpolate(L.PIC_INTERP_CELL_AVERAGE)
    assert int(cnt.sum()) == 0 and bool(avg.isnan().all())
    p.close()
    # one particle moving right
    counts = np.zeros(mesh.n_cells, np.int32)
    counts[5] = 1
    cfg.update(counts=counts, xr=np.array([[0.5], [0.25]]), ids=np.array([7], np.uint32))
    p = gpu_problem(cfg, capacity=3)
    p.advance(0.1, 4, L.PIC_RK2, L.PIC_F64)
    g = p.numpy()
    assert g["n"] == 1 and g["id"][0] == 7
    assert abs(g["x"][0, 0] - (0.1 + 0.4)) < 1e-15
    # everything lost: large step to the right
    p.advance(1.0, 1, L.PIC_EULER, L.PIC_F64)
    assert p.numpy()["n"] == 0 and p.stats()["lost"] == 1
    p.close()


def test_crowded_cell_many_arrivals(L):
    """A converging field sends > 32 arrivals into one cell (slow path of the arrival ordering)."""
    _say("case: many arrivals into one cell")
    mesh = I.UniformMesh(2, (8, 8))
    nodes = I.uniform_q2_nodes(mesh)
    # linear contraction toward (0.5625, 0.5625): exact in Q2
    U = -(nodes - 0.5625) * 4.0
    counts = np.full(mesh.n_cells, 20, np.int32)
    counts, xr, ids = I.draw_reference_particles(counts, 2, seed=90)
    cfg = dict(mesh=mesh, U=U, counts=counts, xr=xr, ids=ids, n_prop=1, prop_dtype=np.float32)
    p = gpu_problem(cfg)
    dt = 0.2
    p.advance(dt, 3, L.PIC_RK2, L.PIC_F64)
    g = p.numpy()
    assert np.diff(g["cell_start"]).max() > 64
    om, st = oracle_store(cfg)
    near, _ = oracle_run_tracking(om, U, dt, 2, 3, st)
    compare_stores(g, st.view(), near)
    p.close()


@pytest.mark.parametrize("n", [16, 13])
def test_fp32_evaluation_against_fp64_oracle(L, n):
    """16^3 and a mesh of 13^3 cells, whose cell blocks at the upper faces are ragged (the x-Horner window and
    the cell-from-row lookup of partial blocks)."""
    _say(f"case: FP32 field evaluation, {n}^3, RK4")
    cfg = I.config2(eval_f32=True, n=n, ppc=6, steps=20)
    p = gpu_problem(cfg)
    p.advance(cfg["dt"], cfg["steps"], L.PIC_RK4, L.PIC_F32)
    g = p.numpy()
    om, st = oracle_store(cfg)
    near, _ = oracle_run_tracking(om, cfg["U"], cfg["dt"], 4, cfg["steps"], st)
    o = st.view()
    common, gi, oi = np.intersect1d(g["id"], o["id"], return_indices=True)
    d = np.abs(g["x"][:, gi] - o["x"][:, oi]).max(axis=0)
    assert np.percentile(d, 99) <= 1e-6 and d.max() <= 1e-5, (np.percentile(d, 99), d.max())
    # cells: re-check with the oracle's own location of the GPU's positions
    for k in np.linspace(0, gi.size - 1, 300).astype(int):
        K, t = om.locate(g["x"][:, gi[k]])
        if min(t.min(), (1 - t).min()) > 1e-10:
            assert K == g["cell"][gi[k]]
    # live sets may differ only through particles that were near the boundary
    assert abs(g["n"] - st.n) <= max(5, len(near))
    p.close()


@pytest.mark.parametrize("dim,scheme,prec,dense", [(3, 4, 1, 0), (3, 2, 0, 0), (2, 4, 0, 0), (2, 2, 1, 0),
                                                   (3, 4, 1, 40), (3, 4, 0, 40), (3, 2, 1, 110), (2, 4, 1, 80)])
def test_fused_steps_bit_identical_to_single_steps(L, dim, scheme, prec, dense):
    """advance(n) fuses each re-sort with the next advect; the result must equal n separate
    one-step advances bit for bit (store, order, counters).  `dense` sets the particles per
    cell of the crowded cases (thousands of particles per cell block)."""
    _say(f"case: fused vs single steps dim={dim} scheme={scheme} prec={prec} dense={dense}")
    n = (20 if dim == 2 else 11) if not dense else (16 if dim == 2 else 8)
    mesh = I.UniformMesh(dim, (n,) * dim)
    f = I.FourierField(dim, seed=900 + dim)
    U = I.normalise_nodal(I.sample_nodes(f.velocity, I.uniform_q2_nodes(mesh)))
    hi = 15 if not dense else 2 * dense
    counts = np.random.default_rng(901).integers(0 if not dense else dense // 2, hi, mesh.n_cells).astype(np.int32)
    counts, xr, ids = I.draw_reference_particles(counts, dim, seed=902)
    cfg = dict(mesh=mesh, U=U, counts=counts, xr=xr, ids=ids, n_prop=2,
               prop_dtype=np.float32 if prec else np.float64)
    out = []
    for fused in (True, False):
        p = gpu_problem(cfg)
        if fused:
            p.advance(0.7 / n, 9, scheme, prec)
        else:
            for _ in range(9):
                p.advance(0.7 / n, 1, scheme, prec)
        out.append((p.numpy(), p.stats()))
        p.close()
    (a, sa), (b, sb) = out
    for k in ("x", "xr", "cell", "id", "prop", "cell_start"):
        assert np.array_equal(a[k], b[k]), k
    for k in ("lost", "moved", "particle_steps", "steps"):
        assert sa[k] == sb[k], k
    assert sa["moved"] > 0
