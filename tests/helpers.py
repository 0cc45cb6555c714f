"""Shared helpers of the GPU parity tests: run a workload on both sides and compare."""
from __future__ import annotations

import numpy as np

from oracle import oracle as O


def gpu_problem(cfg, capacity=None, n_prop=None, prop_dtype=None, U=None):
    from paper_1612_03369_amd.api import Problem
    mesh = cfg["mesh"]
    p = Problem(0)
    p.mesh_uniform(mesh.dim, mesh.n[: mesh.dim], mesh.lo[: mesh.dim], mesh.hi[: mesh.dim])
    p.set_velocity(cfg["U"] if U is None else U)
    n = cfg["xr"].shape[1]
    npr = cfg["n_prop"] if n_prop is None else n_prop
    pd = cfg["prop_dtype"] if prop_dtype is None else prop_dtype
    p.allocate(capacity or max(n, 1), n_prop=npr, prop_dtype="float64" if pd == np.float64 else "float32")
    p.seed_reference(cfg["counts"], cfg["xr"], cfg["ids"])
    return p


def oracle_store(cfg, n_prop=None, mesh=None, cap=None):
    om = mesh or O.OracleMesh.uniform(cfg["mesh"])
    npr = cfg["n_prop"] if n_prop is None else n_prop
    st = O.seed(om, cfg["counts"], cfg["xr"], cfg["ids"], npr, cap=cap)
    return om, st


def oracle_run_tracking(om, U, dt, scheme, steps, st, odes=None, tfield=None, tally=None):
    """Run the oracle step by step; return ids that were near a face at any step.
    odes = (alpha, beta, damage_prop, deform_prop) integrates the property equations too.
    tfield = dict(U1=..., dt_u=..., since=...): the field changes in time (U at t^n, U1 at
    t^n + dt_u); tfield["since"] is advanced by dt after every step.
    tally (dict): receives the summed per-step counts "near", "lost" and "moved"."""
    near_ids = set()
    lost = 0
    if tally is not None:
        for k in ("near", "lost", "moved"):
            tally.setdefault(k, 0)
    for _ in range(steps):
        n = st.n
        ids_before = st.id[:n].copy()
        tf = {} if tfield is None else dict(U1=tfield["U1"], dt_u=tfield["dt_u"], since=tfield["since"])
        if odes is None:
            key, near = O.advect(om, U, dt, scheme, st, **tf)
        else:
            key, near = O.advect_odes(om, U, dt, scheme, st, *odes, **tf)
        if tfield is not None:
            tfield["since"] = tfield["since"] + dt
        near_ids |= set(ids_before[near.astype(bool)].tolist())
        lost += int((key == O.LOST).sum())
        if tally is not None:
            tally["near"] += int(near.astype(bool).sum())
            tally["lost"] += int((key == O.LOST).sum())
            tally["moved"] += int(((key != O.LOST) & (key != st.cell[:n].astype(np.uint32))).sum())
        perm, cs = O.stable_sort_perm(om.n_cells, st.cell[:n], key)
        m = perm.size
        st.x[:, :m] = st.x[:, :n][:, perm]
        st.xr[:, :m] = st.xr[:, :n][:, perm]
        st.prop[:, :m] = st.prop[:, :n][:, perm]
        st.id[:m] = st.id[:n][perm]
        st.cell[:m] = key[perm].astype(np.int32)
        st.c.n = m
        st.cell_start = cs
    return near_ids, lost


def compare_stores(g, o, near_ids, pos_tol=1e-12, check_order=True):
    """Per-id comparison of GPU store g and oracle store o (dicts of numpy arrays)."""
    gid = g["id"].astype(np.int64)
    oid = o["id"].astype(np.int64)
    gs, os_ = set(gid.tolist()), set(oid.tolist())
    only_g, only_o = gs - os_, os_ - gs
    assert only_g <= near_ids and only_o <= near_ids, (
        f"live sets differ beyond near-face particles: {len(only_g - near_ids)} only on GPU, "
        f"{len(only_o - near_ids)} only in oracle")
    common = np.array(sorted(gs & os_), dtype=np.int64)
    gi = np.searchsorted(np.sort(gid), common)
    gidx = np.argsort(gid)[gi]
    oi = np.searchsorted(np.sort(oid), common)
    oidx = np.argsort(oid)[oi]
    scale = np.maximum(1.0, np.abs(o["x"][:, oidx]).max(axis=0))
    err = (np.abs(g["x"][:, gidx] - o["x"][:, oidx]).max(axis=0) / scale)
    assert err.max() <= pos_tol, f"max relative position error {err.max():.3e} > {pos_tol}"
    near_mask = np.isin(common, np.array(sorted(near_ids), dtype=np.int64)) if near_ids else np.zeros(common.size, bool)
    cell_ok = g["cell"][gidx] == o["cell"][oidx]
    assert np.all(cell_ok | near_mask), f"{(~cell_ok & ~near_mask).sum()} cells differ away from faces"
    if check_order:
        # order of the particles that never came near a face: a stable sort keeps their relative
        # order whatever happens to the others
        far = np.array(sorted(near_ids), dtype=np.int64) if near_ids else np.zeros(0, np.int64)
        assert np.array_equal(gid[~np.isin(gid, far)], oid[~np.isin(oid, far)]), "store order differs"
    return err.max(), int(near_mask.sum())
