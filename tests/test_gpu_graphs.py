"""pic_advance from its captured HIP graph against the same calls launched kernel by kernel: the fused step
sequence is replayed several times with eager work and synchronisation in between (single steps, population,
statistics reads, a new step count and scheme that record new graphs, a rebind of the store), and every replay
must leave the store bit-identical to the eagerly launched twin."""
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


def _make(dim, n, seed, graphs, prop_dtype="float32"):
    from paper_1612_03369_amd.api import Problem
    mesh = I.UniformMesh(dim, (n,) * dim)
    f = I.FourierField(dim, seed=seed)
    U = I.normalise_nodal(I.sample_nodes(f.velocity, I.uniform_q2_nodes(mesh)))
    counts = np.random.default_rng(seed + 1).integers(0, 14, mesh.n_cells).astype(np.int32)
    counts, xr, ids = I.draw_reference_particles(counts, dim, seed=seed + 2)
    p = Problem(0)
    p.mesh_uniform(dim, mesh.n[:dim])
    p.set_velocity(U)
    p.allocate(int(xr.shape[1] * 1.5) + 16, n_prop=2, prop_dtype=prop_dtype)
    p.seed_reference(counts, xr, ids)
    p.set_launch_graphs(graphs)
    return p, (counts, xr, ids)


def _same(a, b, where):
    ga, gb = a.numpy(), b.numpy()
    for k in ("x", "xr", "cell", "id", "prop", "cell_start"):
        assert np.array_equal(ga[k], gb[k]), f"{where}: {k} differs"
    sa, sb = a.stats(), b.stats()
    for k in ("live", "lost", "moved", "near_face", "steps", "particle_steps"):
        assert sa[k] == sb[k], f"{where}: stats {k}"


@pytest.mark.parametrize("dim,n,prec", [(3, 16, "f32"), (3, 12, "f64"), (2, 40, "f64")])
def test_graph_replays_equal_eager_launches(L, dim, n, prec):
    _say(f"case: graph replays vs eager launches, {dim}D n={n} {prec}")
    P = L.PIC_F32 if prec == "f32" else L.PIC_F64
    g, seedargs = _make(dim, n, 400 + dim, True)
    e, _ = _make(dim, n, 400 + dim, False)
    dt = 0.5 / n
    for rep in range(4):                                  # the same graph, replayed
        g.advance(dt, 5, L.PIC_RK4, P)
        e.advance(dt, 5, L.PIC_RK4, P)
        _same(g, e, f"replay {rep}")
        g.advance(dt, 1, L.PIC_RK2, P)                    # eager work between replays
        e.advance(dt, 1, L.PIC_RK2, P)
        _same(g, e, f"single step after replay {rep}")
    for steps, scheme in ((3, L.PIC_RK2), (5, L.PIC_RK4), (2, L.PIC_EULER)):   # new keys record new graphs
        g.advance(dt, steps, scheme, P)
        e.advance(dt, steps, scheme, P)
        _same(g, e, f"{steps} steps scheme {scheme}")
    g.population(3, 9, 5, 1)
    e.population(3, 9, 5, 1)
    _same(g, e, "population")
    g.advance(dt, 5, L.PIC_RK4, P)
    e.advance(dt, 5, L.PIC_RK4, P)
    _same(g, e, "after population")
    # a rebind of the store rebuilds the work lists: the graph must be recorded anew
    for p in (g, e):
        p.allocate(seedargs[1].shape[1] + 16, n_prop=2, prop_dtype="float32")
        p.seed_reference(*seedargs)
    g.advance(dt, 5, L.PIC_RK4, P)
    e.advance(dt, 5, L.PIC_RK4, P)
    _same(g, e, "after rebinding")
    _say(f"  live {g.stats()['live']}, steps {g.stats()['steps']}")
    g.close()
    e.close()
