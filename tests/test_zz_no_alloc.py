"""The generation call that allocates nothing (pic_seed_mh_static) against the one that allocates its
staging (pic_seed_mh): same particles bit for bit, on two calls in a row, the second on a smaller
problem, and a mesh beyond the fixed scratch rejected."""
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


def _problem(dim, n, cap):
    from paper_1612_03369_amd.api import Problem
    mesh = I.UniformMesh(dim, (n,) * dim)
    p = Problem(0)
    p.mesh_uniform(dim, mesh.n[:dim])
    p.set_velocity(np.zeros((dim, p.n_nodes)))
    p.allocate(cap, n_prop=dim, prop_dtype="float64")
    return mesh, p


def _inputs(mesh, seed):
    nodes = I.uniform_q2_nodes(mesh)
    rho = 1.0 + 0.5 * np.sin(6.0 * nodes[0]) * np.cos(4.0 * nodes[1])
    if mesh.dim == 3:
        rho = rho + 0.3 * nodes[2]
    counts = np.random.default_rng(seed).integers(0, 9, mesh.n_cells).astype(np.int32)
    return counts, rho


@pytest.mark.parametrize("dim,n1,n2", [(3, 12, 7), (2, 40, 17)])
def test_static_generation_matches_allocating_call(L, dim, n1, n2):
    import torch
    for n, seed in ((n1, 11), (n2, 12)):                   # the second call on a smaller problem
        _say(f"case: static MH generation {dim}D n={n}")
        mesh, p_ref = _problem(dim, n, 12 * n ** dim)
        _, p_st = _problem(dim, n, 12 * n ** dim)
        counts, rho = _inputs(mesh, seed)
        lr_ref = p_ref.seed_mh(counts, rho, 7, 99, first_id=5)
        c_t = torch.tensor(counts, device=p_st.device)
        r_t = torch.tensor(rho, device=p_st.device)
        torch.cuda.synchronize()
        lr_st = p_st.seed_mh_static(c_t, r_t, 7, 99, first_id=5)
        a, b = p_ref.numpy(), p_st.numpy()
        assert lr_st == lr_ref
        assert a["n"] == b["n"] == int(counts.sum())
        for k in ("x", "xr", "cell", "id", "prop", "cell_start"):
            assert np.array_equal(a[k], b[k]), k
        # the problems step on from the generated stores alike
        p_ref.population(2, 6, 3, 0)
        p_st.population(2, 6, 3, 0)
        assert np.array_equal(p_ref.numpy()["id"], p_st.numpy()["id"])
        p_ref.close()
        p_st.close()


def test_static_generation_rejects_what_does_not_fit(L):
    import torch
    from paper_1612_03369_amd._lib import PicError
    _say("case: static MH generation, mesh beyond the fixed scratch and bad counts")
    mesh, p = _problem(3, 41, 8)                           # 83^3 nodes x 32 B > 16 MiB
    c_t = torch.zeros(mesh.n_cells, dtype=torch.int32, device=p.device)
    r_t = torch.ones(p.n_nodes, dtype=torch.float64, device=p.device)
    with pytest.raises(PicError) as e:
        p.seed_mh_static(c_t, r_t, 3, 1)
    assert e.value.status == L.PIC_EINVAL
    p.close()
    mesh, p = _problem(2, 8, 10)
    counts, rho = _inputs(mesh, 13)
    c_t = torch.tensor(counts, device=p.device)
    r_t = torch.tensor(rho, device=p.device)
    with pytest.raises(PicError) as e:                     # more particles than the capacity
        p.seed_mh_static(c_t, r_t, 3, 1)
    assert e.value.status == L.PIC_ECAPACITY
    counts[5] = -1
    with pytest.raises(PicError) as e:
        p.seed_mh_static(torch.tensor(counts, device=p.device), r_t, 3, 1)
    assert e.value.status == L.PIC_EINVAL
    rho[3] = np.nan
    counts[5] = 0
    counts[:] = np.minimum(counts, 0)
    with pytest.raises(PicError) as e:
        p.seed_mh_static(torch.tensor(counts, device=p.device), torch.tensor(rho, device=p.device), 3, 1)
    assert e.value.status == L.PIC_ENONFINITE
    p.close()
