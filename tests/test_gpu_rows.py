"""GPU parity of the remaining hot-path rows: population management, least
squares, batched problems, the adjoint, displaced meshes, octree meshes and
prescribed-location seeding."""
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


def _fourier_cfg(dim, n, counts_hi, seed, n_prop=1, prop_dtype=np.float64, tangential=False):
    mesh = I.UniformMesh(dim, (n,) * dim)
    f = I.FourierField(dim, seed=seed, tangential=tangential)
    U = I.normalise_nodal(I.sample_nodes(f.velocity, I.uniform_q2_nodes(mesh)))
    rng = np.random.default_rng(seed + 1)
    counts = rng.integers(0, counts_hi, mesh.n_cells).astype(np.int32)
    counts, xr, ids = I.draw_reference_particles(counts, dim, seed=seed + 2)
    return dict(mesh=mesh, U=U, counts=counts, xr=xr, ids=ids, n_prop=n_prop, prop_dtype=prop_dtype)


# ----------------------------------------------------------------------------
def test_population_matches_oracle(L):
    """Advance + population each step (min 4 / max 9): ids, locations, properties."""
    _say("case: population 3D 8^3, counts 0..14, clamp [4, 9], 4 steps")
    cfg = _fourier_cfg(3, 8, 15, seed=101, n_prop=2)
    cap = 10 * cfg["mesh"].n_cells + 100
    p = gpu_problem(cfg, capacity=cap)
    om, st = oracle_store(cfg, cap=cap)
    nid = int(cfg["ids"].max()) + 1
    dt = 0.5 / 8
    near = set()
    for step in range(4):
        p.advance(dt, 1, L.PIC_RK2, L.PIC_F64)
        p.population(4, 9, 40, step)
        nr, _ = oracle_run_tracking(om, cfg["U"], dt, 2, 1, st)
        near |= nr
        nid, added, deleted = O.population(om, st, 4, 9, 40, step, nid)
    g = p.numpy()
    o = st.view()
    s = p.stats()
    cnt = np.diff(g["cell_start"])
    assert cnt.min() >= 4 and cnt.max() <= 9
    assert np.unique(g["id"]).size == g["n"]
    compare_stores(g, o, near, pos_tol=1e-12)
    if not near:
        assert np.array_equal(g["id"], o["id"])
        assert np.abs(g["prop"] - o["prop"]).max() < 1e-13
        # reference coordinates = (x - x_K)/h: the 1e-12 position bar scaled by 1/h
        assert np.abs(g["xr"] - o["xr"]).max() < 1e-12 * 8
    _say(f"  live {g['n']}, added {s['added']}, deleted {s['deleted']}, near {len(near)}")
    assert s["added"] > 0 and s["deleted"] > 0
    p.close()


def test_population_capacity_error(L):
    cfg = _fourier_cfg(2, 6, 3, seed=111)
    p = gpu_problem(cfg, capacity=cfg["xr"].shape[1] + 5)
    from paper_1612_03369_amd._lib import PicError
    with pytest.raises(PicError) as e:
        p.population(20, 30, 1, 0)
    assert e.value.status == L.PIC_ECAPACITY
    p.close()


def test_linear_least_squares_matches_oracle(L):
    _say("case: least squares 3D 6^3 after 3 RK2 steps")
    cfg = _fourier_cfg(3, 6, 12, seed=121, n_prop=2)
    p = gpu_problem(cfg)
    p.advance(0.5 / 6, 3, L.PIC_RK2, L.PIC_F64)
    out, xbar, cnt = p.interpolate(L.PIC_INTERP_LINEAR_LS)
    g = p.numpy()
    # the oracle fits its own store after its own 3 steps
    om, st = oracle_store(cfg)
    near, _ = oracle_run_tracking(om, cfg["U"], 0.5 / 6, 2, 3, st)
    o = st.view()
    compare_stores(g, o, near)
    coef_o, xbar_o = O.linear_least_squares(cfg["mesh"].n_cells, 3, st.cell_start, o["xr"], o["prop"])
    c = cnt.cpu().numpy()
    assert np.array_equal(c, np.diff(g["cell_start"]))
    og, xg = out.cpu().numpy(), xbar.cpu().numpy()
    # cells holding a near-face particle may hold different sets on the two sides
    skip = np.zeros(c.size, bool)
    near_arr = np.array(sorted(near), dtype=np.int64)
    skip[g["cell"][np.isin(g["id"].astype(np.int64), near_arr)]] = True
    skip[o["cell"][np.isin(o["id"].astype(np.int64), near_arr)]] = True
    ok = (c > 0) & ~skip
    assert np.array_equal(np.diff(st.cell_start)[~skip], c[~skip])
    assert np.all(np.isnan(og[c == 0]))
    assert np.allclose(xg[ok], xbar_o[ok], rtol=0, atol=1e-12)
    assert np.allclose(og[ok], coef_o[ok], rtol=1e-9, atol=1e-11)
    _say(f"  {ok.sum()} cells compared, {skip.sum()} skipped (near-face particles)")
    p.close()


def test_linear_least_squares_reproduces_linear_data(L):
    """Initial-position property is linear in the reference coordinates: exact recovery."""
    cfg = _fourier_cfg(2, 10, 9, seed=131, n_prop=2)
    p = gpu_problem(cfg)
    out, xbar, cnt = p.interpolate(L.PIC_INTERP_LINEAR_LS)
    c = cnt.cpu().numpy()
    o = out.cpu().numpy()
    h = 0.1
    full = c >= 3
    # property j = x_j = (i_j + xr_j) h: slope h along axis j, zero along the other
    assert np.allclose(o[full, 0, 1], h, atol=1e-12) and np.allclose(o[full, 0, 2], 0, atol=1e-12)
    assert np.allclose(o[full, 1, 2], h, atol=1e-12) and np.allclose(o[full, 1, 1], 0, atol=1e-12)
    p.close()


# ----------------------------------------------------------------------------
@pytest.mark.parametrize("schedule", ["default", "tuned", "shape2"])
def test_batch_bit_identical_to_single_runs(L, schedule):
    """Batched steps equal single runs bit for bit, whatever cell-block schedule the
    batch uses; the autotuner leaves the problems' state and statistics as they were."""
    _say(f"case: batch of 6 mixed problems vs single runs, schedule {schedule}")
    from paper_1612_03369_amd.api import Batch
    cfgs = []
    for q in range(6):
        dim = 2 + (q % 2)
        n = 20 if dim == 2 else 8
        c = _fourier_cfg(dim, n, 10, seed=200 + q)
        c["scheme"] = (2, 4)[(q // 2) % 2] if q != 5 else 1
        c["dt"] = 0.5 / n
        cfgs.append(c)
    singles, single_stats = [], []
    for c in cfgs:
        p = gpu_problem(c)
        p.advance(c["dt"], 7, c["scheme"], L.PIC_F64)
        singles.append(p.numpy())
        single_stats.append(p.stats())
        p.close()
    probs = [gpu_problem(c) for c in cfgs]
    b = Batch(probs, tile_cells=(16, 32, 8, 16))
    dts, schemes = [c["dt"] for c in cfgs], [c["scheme"] for c in cfgs]
    if schedule == "tuned":
        rec = b.tune(dts, schemes, trials=2)
        _say(f"  tuned variants {rec['variants']}")
        assert all(0 <= v <= 2 for v in rec["variants"])
        assert set(rec["times_ms"]) == {"2d-rk2", "2d-rk4", "3d-euler", "3d-rk2", "3d-rk4"}
    elif schedule == "shape2":
        b.set_schedule([2, 2, 2, 2, 2, 2])
    b.advance(dts, schemes, 4)
    b.advance(dts, schemes, 3)
    for p, s, ss in zip(probs, singles, single_stats):
        g = p.numpy()
        for k in ("x", "xr", "cell", "id", "prop", "cell_start"):
            assert np.array_equal(g[k], s[k]), k
        st = p.stats()
        assert st["steps"] == 7
        for k in ("particle_steps", "lost", "moved", "near_face"):
            assert st[k] == ss[k], k
    b.close()
    for p in probs:
        p.close()


def test_batch_with_long_and_short_scan_chunks(L):
    """A batch whose problems take different scan chunk widths (one mesh of more than 2^19
    cells, two small ones) equals the single runs bit for bit."""
    _say("case: batch with a 768^2 mesh (long scan chunks) and two small meshes vs single runs")
    from paper_1612_03369_amd.api import Batch
    cfgs = [_fourier_cfg(2, 768, 3, seed=251), _fourier_cfg(3, 8, 10, seed=252), _fourier_cfg(2, 20, 10, seed=253)]
    for c, sch in zip(cfgs, (4, 2, 4)):
        c["scheme"] = sch
        c["dt"] = 0.5 / c["mesh"].n[0]
    singles = []
    for c in cfgs:
        p = gpu_problem(c)
        p.advance(c["dt"], 5, c["scheme"], L.PIC_F64)
        singles.append(p.numpy())
        p.close()
    probs = [gpu_problem(c) for c in cfgs]
    b = Batch(probs)
    b.advance([c["dt"] for c in cfgs], [c["scheme"] for c in cfgs], 5)
    for p, s in zip(probs, singles):
        g = p.numpy()
        for k in ("x", "xr", "cell", "id", "prop", "cell_start"):
            assert np.array_equal(g[k], s[k]), k
    b.close()
    for p in probs:
        p.close()


# ----------------------------------------------------------------------------
def _adjoint_case(L, n=6, ppc=3, steps=8, scheme=4, ckpt=3, seed=301, dim=3):
    mesh = I.UniformMesh(dim, (n,) * dim)
    nodes = I.uniform_q2_nodes(mesh)
    U = I.normalise_nodal(I.sample_nodes(I.FourierField(dim, seed=seed, tangential=True).velocity, nodes))
    counts = np.full(mesh.n_cells, ppc, np.int32)
    counts, xr, ids = I.draw_reference_particles(counts, dim, seed=seed + 1)
    cfg = dict(mesh=mesh, U=U, counts=counts, xr=xr, ids=ids, n_prop=0, prop_dtype=np.float64)
    return cfg, 0.5 / n, steps, scheme, ckpt


@pytest.mark.parametrize("dim", [3, 2])
@pytest.mark.parametrize("scheme", [2, 4])
def test_adjoint_matches_oracle_gradient(L, scheme, dim):
    _say(f"case: adjoint vs oracle, {dim}D, scheme {scheme}")
    import torch
    from paper_1612_03369_amd.adjoint import ParticleFlow, advect
    cfg, dt, steps, _, ckpt = _adjoint_case(L, scheme=scheme, dim=dim, **({} if dim == 3 else dict(n=10, ppc=4)))
    p = gpu_problem(cfg)
    flow = ParticleFlow(p, cfg["counts"], cfg["xr"], cfg["ids"], dt, steps, scheme, ckpt)
    U = torch.tensor(cfg["U"], dtype=torch.float64, device=p.device, requires_grad=True)
    xT = advect(U, flow)
    # targets: the oracle's own forward run plus noise, indexed by id
    om, st = oracle_store(cfg)
    v = st.view()
    _, fin = oracle_store(cfg)
    O.run(om, cfg["U"], dt, scheme, steps, fin)
    f = fin.view()
    n_id = xT.shape[1]
    x_or = np.full((dim, n_id), np.nan)
    x_or[:, f["id"]] = f["x"]
    rng = np.random.default_rng(7)
    tgt_np = x_or + 0.01 * rng.standard_normal(x_or.shape)
    live_g = ~np.isnan(xT.detach().cpu().numpy()[0])
    m_id = live_g & ~np.isnan(x_or[0])
    tgt = torch.tensor(np.nan_to_num(tgt_np), device=p.device)
    mask = torch.tensor(m_id, device=p.device)
    nv = int(mask.sum())
    loss = ((xT - tgt)[:, mask] ** 2).sum() / nv
    loss.backward()
    g = U.grad.cpu().numpy()
    # oracle: per-particle reverse sweep from the initial state
    tg = np.nan_to_num(tgt_np)[:, v["id"]]
    m = m_id[v["id"]].astype(np.uint8)
    Lo, dUo, lost = O.adjoint(om, cfg["U"], dt, scheme, steps, v["x"], v["cell"], v["xr"], tg, m)
    assert abs(float(loss) - Lo) <= 1e-12 * abs(Lo)
    assert np.abs(g - dUo).max() <= 1e-10 * np.abs(dUo).max(), np.abs(g - dUo).max() / np.abs(dUo).max()
    p.close()


def test_adjoint_central_differences(L):
    _say("case: adjoint vs central differences (GPU forward)")
    import torch
    from paper_1612_03369_amd.adjoint import ParticleFlow, advect
    cfg, dt, steps, scheme, ckpt = _adjoint_case(L, n=5, ppc=4, steps=10, ckpt=4, seed=311)
    p = gpu_problem(cfg)
    flow = ParticleFlow(p, cfg["counts"], cfg["xr"], cfg["ids"], dt, steps, scheme, ckpt)
    U0 = torch.tensor(cfg["U"], dtype=torch.float64, device=p.device)
    with torch.no_grad():
        x0, _ = flow.run_forward(U0, checkpoint=False)
    tgt = x0 + 0.02
    mask = ~torch.isnan(x0[0])

    def loss_of(U):
        xT = advect(U, flow)
        return ((xT - tgt)[:, mask] ** 2).sum() / int(mask.sum())

    U = U0.clone().requires_grad_(True)
    loss_of(U).backward()
    g = U.grad.clone()
    rng = np.random.default_rng(8)
    for _ in range(6):
        d = torch.tensor(rng.standard_normal(cfg["U"].shape), device=p.device)
        d /= d.abs().max()
        eps = 1e-6
        with torch.no_grad():
            lp = float(loss_of(U0 + eps * d))
            lm = float(loss_of(U0 - eps * d))
        fd = (lp - lm) / (2 * eps)
        an = float((g * d).sum())
        assert abs(fd - an) <= 1e-6 * max(abs(an), 1e-12), (fd, an)
    p.close()


def test_adjoint_backward_after_a_later_forward(L):
    """Two forwards, then the backward of the first: the gradient is the first forward's (the flow
    re-runs it from its own field), equal to a lone forward + backward up to the order of the FP64
    atomic sums."""
    _say("case: adjoint, backward after a later forward")
    import torch
    from paper_1612_03369_amd.adjoint import ParticleFlow, advect
    cfg, dt, steps, scheme, ckpt = _adjoint_case(L, n=5, ppc=4, steps=9, ckpt=3, seed=321)
    p = gpu_problem(cfg)
    flow = ParticleFlow(p, cfg["counts"], cfg["xr"], cfg["ids"], dt, steps, scheme, ckpt)
    U0 = torch.tensor(cfg["U"], dtype=torch.float64, device=p.device)
    U2 = torch.tensor(I.normalise_nodal(I.sample_nodes(I.FourierField(3, seed=322, tangential=True).velocity,
                                                       I.uniform_q2_nodes(cfg["mesh"]))), device=p.device)
    tgt = torch.zeros((3, cfg["xr"].shape[1]), dtype=torch.float64, device=p.device) + 0.5

    def loss(xT):
        m = ~torch.isnan(xT[0])
        return ((xT - tgt)[:, m] ** 2).sum()

    Ua = U0.clone().requires_grad_(True)
    loss(advect(Ua, flow)).backward()
    ref = Ua.grad.clone()
    Ub = U0.clone().requires_grad_(True)
    lb = loss(advect(Ub, flow))
    Uc = U2.clone().requires_grad_(True)
    lc = loss(advect(Uc, flow))
    lb.backward()
    assert torch.allclose(Ub.grad, ref, rtol=0, atol=1e-12 * float(ref.abs().max()))
    lc.backward()
    Ud = U2.clone().requires_grad_(True)
    loss(advect(Ud, flow)).backward()
    assert torch.allclose(Uc.grad, Ud.grad, rtol=0, atol=1e-12 * float(Ud.grad.abs().max()))
    assert float((Uc.grad - ref).abs().max()) > 1e-6 * float(ref.abs().max())
    p.close()


# ----------------------------------------------------------------------------
@pytest.mark.parametrize("dim", [2, 3])
def test_displaced_mesh_newton_and_neighbour_search(L, dim):
    _say(f"case: displaced mesh dim {dim}")
    from paper_1612_03369_amd.api import Problem
    n = (6, 5) if dim == 2 else (4, 4, 3)
    mesh = I.UniformMesh(dim, n)
    vert = I.displaced_vertices(mesh, 0.2, seed=400 + dim)
    om = O.OracleMesh.displaced(mesh, vert)
    nodes = om.q2_node_coords()
    f = I.FourierField(dim, seed=410 + dim)
    U = I.normalise_nodal(I.sample_nodes(f.velocity, nodes))
    rng = np.random.default_rng(420 + dim)
    counts = rng.integers(0, 8, mesh.n_cells).astype(np.int32)
    counts, xr, ids = I.draw_reference_particles(counts, dim, seed=430 + dim)
    p = Problem(0)
    p.mesh_uniform(dim, n)
    p.mesh_displace(vert)
    gx, _ = p.q2_nodes()
    assert np.allclose(gx, nodes, atol=1e-15)
    p.set_velocity(U)
    p.allocate(xr.shape[1], n_prop=1)
    p.seed_reference(counts, xr, ids)
    dt = 0.3 / max(n)
    p.advance(dt, 6, L.PIC_RK4, L.PIC_F64)
    g = p.numpy()
    st = O.seed(om, counts, xr, ids, 1)
    near, _ = oracle_run_tracking(om, U, dt, 4, 6, st)
    err, nn = compare_stores(g, st.view(), near, pos_tol=1e-12)
    s = p.stats()
    _say(f"  moved {s['moved']}, first-try {s['first_try']}, fallback {s['fallback']}, newton_fail {s['newton_fail']}")
    assert s["first_try"] > 0
    p.close()


# ----------------------------------------------------------------------------
def _small_octree():
    """Base 2^3 refined toward a corner region (levels 1..4), 2:1 balanced."""
    level, anchor = I.octree_shell_leaves(base_level=1, max_level=4, r_in=0.0, r_out=0.3, width=1.0,
                                          centre=(0.3, 0.35, 0.4))
    return I.balance_octree(level, anchor, 4)


def test_octree_mesh_parity(L):
    _say("case: small octree, RK2")
    from paper_1612_03369_amd.api import Problem
    level, anchor = _small_octree()
    om = O.OracleMesh.octree(level, anchor, 4)
    nodes = om.q2_node_coords()
    f = I.FourierField(3, seed=501)
    U = om.resolve_hanging(I.normalise_nodal(I.sample_nodes(f.velocity, nodes)))
    counts = np.random.default_rng(502).integers(0, 9, level.size).astype(np.int32)
    counts, xr, ids = I.draw_reference_particles(counts, 3, seed=503)
    p = Problem(0)
    p.mesh_octree(level, anchor, 4)
    gx, ghang = p.q2_nodes()
    assert np.array_equal(gx, nodes)
    hang = np.zeros(nodes.shape[1], bool)
    hang[[nd for nd, _ in om.hanging_constraints()]] = True
    assert np.array_equal(ghang, hang)
    Uraw = I.normalise_nodal(I.sample_nodes(f.velocity, nodes))
    p.set_velocity(Uraw)                     # the library resolves hanging nodes itself
    p.allocate(xr.shape[1], n_prop=1)
    p.seed_reference(counts, xr, ids)
    dt = 0.5 / 16
    p.advance(dt, 8, L.PIC_RK2, L.PIC_F64)
    g = p.numpy()
    st = O.seed(om, counts, xr, ids, 1)
    near, _ = oracle_run_tracking(om, U, dt, 2, 8, st)
    compare_stores(g, st.view(), near, pos_tol=1e-12)
    s = p.stats()
    _say(f"  moved {s['moved']}, first-try {s['first_try']}, fallback {s['fallback']}")
    p.close()


def test_seed_positions_matches_oracle_locate(L):
    _say("case: prescribed locations")
    from paper_1612_03369_amd.api import Problem
    mesh = I.UniformMesh(3, (5, 4, 3))
    rng = np.random.default_rng(600)
    x = rng.uniform(-0.1, 1.1, size=(3, 3000))
    x[:, :50] = np.round(x[:, :50] * 4) / 4            # points on faces
    ids = np.arange(3000, dtype=np.uint32)
    p = Problem(0)
    p.mesh_uniform(3, mesh.n)
    p.set_velocity(np.zeros((3, mesh.n_nodes)))
    p.allocate(3000, n_prop=1)
    p.seed_positions(x, ids)
    g = p.numpy()
    om = O.OracleMesh.uniform(mesh)
    exp = []
    for i in range(3000):
        K, t = om.locate(x[:, i])
        if K is not None:
            exp.append((K, i))
    exp.sort()
    assert g["id"].tolist() == [i for _, i in exp]
    assert g["cell"].tolist() == [K for K, _ in exp]
    assert np.array_equal(g["x"], x[:, g["id"]])
    assert p.stats()["lost"] == 3000 - len(exp)
    p.close()


def test_batch_tune_cache(L, tmp_path):
    """The library's tune cache: the text written for a batch applies to the same problems and schemes,
    changes nothing for other schemes, rejects malformed text and out-of-range shapes; tune(cache=...)
    stores a choice and reuses it without timing."""
    import json
    from paper_1612_03369_amd._lib import PicError
    from paper_1612_03369_amd.api import Batch
    _say("case: batch tune cache")
    cfgs = [_fourier_cfg(2, 16, 6, seed=220), _fourier_cfg(3, 8, 6, seed=221), _fourier_cfg(3, 8, 6, seed=222)]
    probs = [gpu_problem(c) for c in cfgs]
    b = Batch(probs)
    schemes = [2, 4, 4]
    text = b.tune_cache(schemes)
    rec = json.loads(text)
    assert rec["variants"] == [0] * 6
    assert rec["signature"] == [[c["mesh"].dim, c["mesh"].n_cells, c["xr"].shape[1], s] for c, s in zip(cfgs, schemes)]
    rec["variants"] = [1, 2, 1, 0, 2, 1]
    assert b.apply_tune_cache(schemes, json.dumps(rec))
    assert json.loads(b.tune_cache(schemes))["variants"] == [1, 2, 1, 0, 2, 1]
    assert not b.apply_tune_cache([2, 2, 4], json.dumps(dict(rec, variants=[0] * 6)))   # other schemes
    assert json.loads(b.tune_cache(schemes))["variants"] == [1, 2, 1, 0, 2, 1]
    for bad in ("", "{}", text[:-1], text + "x", json.dumps(dict(rec, variants=[0, 0, 0, 0, 0, 3])),
                json.dumps(dict(rec, variants=[0, 0, 0]))):
        with pytest.raises(PicError) as e:
            b.apply_tune_cache(schemes, bad)
        assert e.value.status == L.PIC_EINVAL
    path = str(tmp_path / "tune.json")
    dts = [0.5 / c["mesh"].n[0] for c in cfgs]
    first = b.tune(dts, schemes, trials=1, cache=path)
    assert "times_ms" in first and not first.get("cached")
    b.set_schedule([2] * 6)
    again = b.tune(dts, schemes, trials=1, cache=path)
    assert again.get("cached") and again["variants"] == first["variants"]
    assert json.loads(b.tune_cache(schemes))["variants"] == first["variants"]
    b.close()
    for p in probs:
        p.close()
