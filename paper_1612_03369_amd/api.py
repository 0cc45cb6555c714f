"""Python front end of the C ABI: one ``Problem`` = one ``pic_ctx``.

Torch provides the device memory (the particle store, scratch, outputs) and
the stream; every computation happens in the HIP library.  This module only
allocates tensors, passes their pointers and shapes, and wraps results as
tensor views.
"""
from __future__ import annotations

import ctypes as C
from dataclasses import dataclass

import numpy as np

from . import _lib as L


def _torch():
    import torch
    return torch


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _np_ptr(a):
    return a.ctypes.data_as(C.c_void_p)


@dataclass
class StoreTensors:
    capacity: int
    x: list
    xr: list
    cell: list
    id: list
    prop: list
    cell_start: list
    scratch: object
    n_prop: int
    prop_dtype: object


class Problem:
    """A mesh + Q2 velocity field + particle store on one GPU."""

    def __init__(self, device: int = 0, stream=None):
        torch = _torch()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the particle library runs only on a HIP device")
        self.lib = L.load()
        self.device = torch.device("cuda", device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        L.check(self.lib.pic_create(C.byref(h), device, C.c_void_p(self.stream.cuda_stream)))
        self.h = h
        self.store = None
        self.dim = self.n_cells = self.n_nodes = None
        self._keep = []

    def close(self):
        if getattr(self, "h", None) is not None:
            self.lib.pic_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, status):
        L.check(status, ctx=self.h)

    # ------------------------------------------------------------------ mesh
    def _info(self):
        d = C.c_int32()
        nc = C.c_int64()
        nn = C.c_int64()
        self._chk(self.lib.pic_mesh_info(self.h, C.byref(d), C.byref(nc), C.byref(nn)))
        self.dim, self.n_cells, self.n_nodes = d.value, nc.value, nn.value

    def mesh_uniform(self, dim, n, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0)):
        n3 = np.array(list(n) + [1] * (3 - len(n)), np.int32)[:3]
        lo3 = np.array(list(lo) + [0.0] * (3 - len(lo)), np.float64)[:3]
        hi3 = np.array(list(hi) + [1.0] * (3 - len(hi)), np.float64)[:3]
        self._chk(self.lib.pic_mesh_uniform(self.h, dim, _np_ptr(n3), _np_ptr(lo3), _np_ptr(hi3)))
        self._info()

    def mesh_displace(self, vertices):
        v = np.ascontiguousarray(vertices, np.float64)
        self._chk(self.lib.pic_mesh_displace(self.h, _np_ptr(v)))
        self._info()

    def mesh_octree(self, level, anchor, max_level, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0)):
        lv = np.ascontiguousarray(level, np.uint8)
        an = np.ascontiguousarray(anchor, np.int32)
        lo3 = np.array(lo, np.float64)
        hi3 = np.array(hi, np.float64)
        self._chk(self.lib.pic_mesh_octree(self.h, _np_ptr(lo3), _np_ptr(hi3), int(max_level), lv.shape[0],
                                           _np_ptr(lv), _np_ptr(an)))
        self._info()

    def q2_nodes(self):
        xyz = np.zeros((self.dim, self.n_nodes), np.float64)
        hang = np.zeros(self.n_nodes, np.uint8)
        self._chk(self.lib.pic_q2_nodes(self.h, _np_ptr(xyz), _np_ptr(hang)))
        return xyz, hang.astype(bool)

    # ----------------------------------------------------------------- field
    def set_velocity(self, U):
        """U: [dim][n_nodes] float64 or float32 (numpy or torch); copied by the library."""
        torch = _torch()
        t = torch.as_tensor(U).to(self.device).contiguous()
        if t.dtype not in (torch.float64, torch.float32):
            t = t.to(torch.float64)
        if tuple(t.shape) != (self.dim, self.n_nodes):
            raise ValueError(f"U must have shape ({self.dim}, {self.n_nodes})")
        prec = L.PIC_F64 if t.dtype == torch.float64 else L.PIC_F32
        self._chk(self.lib.pic_set_velocity(self.h, _ptr(t), prec))

    def _field_tensor(self, U):
        torch = _torch()
        t = torch.as_tensor(U).to(self.device).contiguous()
        if t.dtype not in (torch.float64, torch.float32):
            t = t.to(torch.float64)
        if tuple(t.shape) != (self.dim, self.n_nodes):
            raise ValueError(f"U must have shape ({self.dim}, {self.n_nodes})")
        return t, (L.PIC_F64 if t.dtype == torch.float64 else L.PIC_F32)

    def set_velocity_end(self, U1, dt_u):
        """Field u^{n+1} at the end of the field step of length dt_u (Sec. 2.3): stages then use the
        field interpolated linearly in time; the elapsed time restarts at 0.  U1=None: steady field."""
        if U1 is None:
            self._chk(self.lib.pic_set_velocity_end(self.h, None, L.PIC_F64, 1.0))
            return
        t, prec = self._field_tensor(U1)
        self._chk(self.lib.pic_set_velocity_end(self.h, _ptr(t), prec, float(dt_u)))

    def shift_velocity(self, U_next, dt_u):
        """Next field step: the end field becomes the start field, U_next the end field."""
        t, prec = self._field_tensor(U_next)
        self._chk(self.lib.pic_shift_velocity(self.h, _ptr(t), prec, float(dt_u)))

    def set_field_time(self, tau):
        self._chk(self.lib.pic_set_field_time(self.h, float(tau)))

    def field_time(self) -> float:
        v = C.c_double()
        self._chk(self.lib.pic_field_time(self.h, C.byref(v)))
        return v.value

    # ----------------------------------------------------------------- store
    def allocate(self, capacity: int, n_prop: int = 0, prop_dtype="float64"):
        torch = _torch()
        dev = self.device
        pd = torch.float64 if str(prop_dtype).endswith("64") else torch.float32
        sb = C.c_int64()
        self._chk(self.lib.pic_scratch_bytes(self.h, int(capacity), C.byref(sb)))
        d = self.dim
        st = StoreTensors(
            capacity=int(capacity),
            x=[torch.zeros((d, capacity), dtype=torch.float64, device=dev) for _ in range(2)],
            xr=[torch.zeros((d, capacity), dtype=torch.float64, device=dev) for _ in range(2)],
            cell=[torch.zeros(capacity, dtype=torch.int32, device=dev) for _ in range(2)],
            id=[torch.zeros(capacity, dtype=torch.int32, device=dev) for _ in range(2)],
            prop=[torch.zeros((max(n_prop, 1), capacity), dtype=pd, device=dev) for _ in range(2)],
            cell_start=[torch.zeros(self.n_cells + 1, dtype=torch.int32, device=dev) for _ in range(2)],
            scratch=torch.zeros(int(sb.value), dtype=torch.uint8, device=dev),
            n_prop=int(n_prop), prop_dtype=pd)
        s = L.PicStore()
        s.capacity = int(capacity)
        for b in range(2):
            s.x[b] = st.x[b].data_ptr()
            s.xr[b] = st.xr[b].data_ptr()
            s.cell[b] = st.cell[b].data_ptr()
            s.id[b] = st.id[b].data_ptr()
            s.prop[b] = st.prop[b].data_ptr()
            s.cell_start[b] = st.cell_start[b].data_ptr()
        s.n_prop = int(n_prop)
        s.prop_prec = L.PIC_F64 if pd == torch.float64 else L.PIC_F32
        s.scratch = st.scratch.data_ptr()
        s.scratch_bytes = int(sb.value)
        self._chk(self.lib.pic_bind_store(self.h, C.byref(s)))
        self.store = st
        self._cstore = s
        return st

    def seed_reference(self, counts, xr, ids, prop=None, init_position=True):
        torch = _torch()
        dev = self.device
        c = torch.as_tensor(np.ascontiguousarray(counts, np.int32)).to(dev)
        x = torch.as_tensor(np.ascontiguousarray(xr, np.float64)).to(dev).contiguous()
        i = torch.as_tensor(np.ascontiguousarray(ids, np.uint32).view(np.int32)).to(dev)
        n = x.shape[1]
        p = None
        if prop is not None:
            p = torch.as_tensor(prop).to(dev).to(self.store.prop_dtype).contiguous()
        mode = L.PIC_PROP_INITIAL_POSITION if (init_position and prop is None) else L.PIC_PROP_GIVEN
        self._chk(self.lib.pic_seed_reference(self.h, _ptr(c), _ptr(x), _ptr(i), n, mode, _ptr(p)))

    def seed_per_cell(self, counts, seed, first_id=0, prop=None, init_position=True):
        """Reference-local generation with the library's counter hash (counts per cell)."""
        torch = _torch()
        dev = self.device
        c = torch.as_tensor(np.ascontiguousarray(counts, np.int32)).to(dev)
        p = None
        if prop is not None:
            p = torch.as_tensor(prop).to(dev).to(self.store.prop_dtype).contiguous()
        mode = L.PIC_PROP_INITIAL_POSITION if (init_position and prop is None) else L.PIC_PROP_GIVEN
        self._chk(self.lib.pic_seed_per_cell(self.h, _ptr(c), int(seed), int(first_id), mode, _ptr(p)))

    def seed_positions(self, x, ids, prop=None, init_position=True):
        torch = _torch()
        dev = self.device
        xt = torch.as_tensor(np.ascontiguousarray(x, np.float64)).to(dev).contiguous()
        i = torch.as_tensor(np.ascontiguousarray(ids, np.uint32).view(np.int32)).to(dev)
        p = None
        if prop is not None:
            p = torch.as_tensor(prop).to(dev).to(self.store.prop_dtype).contiguous()
        mode = L.PIC_PROP_INITIAL_POSITION if (init_position and prop is None) else L.PIC_PROP_GIVEN
        self._chk(self.lib.pic_seed_positions(self.h, _ptr(xt), _ptr(i), xt.shape[1], mode, _ptr(p)))

    def set_tile(self, tile_cells: int):
        self._chk(self.lib.pic_set_tile(self.h, int(tile_cells)))

    def current_index(self) -> int:
        w = C.c_int32()
        self._chk(self.lib.pic_current_buffer(self.h, C.byref(w)))
        return w.value

    def current(self, copy=True):
        """Current buffer as tensors sliced to the live count (synchronises)."""
        b = self.current_index()
        st = self.store
        cs = st.cell_start[b]
        n = int(cs[-1].item())
        out = dict(x=st.x[b][:, :n], xr=st.xr[b][:, :n], cell=st.cell[b][:n], id=st.id[b][:n],
                   prop=st.prop[b][: st.n_prop, :n], cell_start=cs, n=n, buffer=b)
        if copy:
            out = {k: (v.clone() if hasattr(v, "clone") else v) for k, v in out.items()}
        return out

    def numpy(self):
        cur = self.current(copy=False)
        out = {}
        for k, v in cur.items():
            if hasattr(v, "cpu"):
                a = v.cpu().numpy()
                if k == "id":
                    a = a.view(np.uint32)
                out[k] = a
            else:
                out[k] = v
        return out

    # -------------------------------------------------------------- hot path
    def advance(self, dt, n_steps=1, scheme=L.PIC_RK4, eval_prec=L.PIC_F64):
        self._chk(self.lib.pic_advance(self.h, float(dt), int(n_steps), int(scheme), int(eval_prec)))

    def set_property_odes(self, damage_prop=-1, deform_prop=-1, alpha=0.0, beta=0.0):
        """Integrate the damage (property damage_prop) and deformation-gradient (properties
        deform_prop .. + dim^2 - 1, row-major) equations with the positions; -1, -1 switches off."""
        self._chk(self.lib.pic_set_property_odes(self.h, int(damage_prop), int(deform_prop), float(alpha),
                                                 float(beta)))

    def population(self, pmin, pmax, seed, step):
        self._chk(self.lib.pic_population(self.h, int(pmin), int(pmax), int(seed), int(step)))

    def interpolate(self, kind=L.PIC_INTERP_CELL_AVERAGE):
        torch = _torch()
        dev = self.device
        npr = self.store.n_prop
        cnt = torch.zeros(self.n_cells, dtype=torch.int32, device=dev)
        if kind in (L.PIC_INTERP_CELL_AVERAGE, L.PIC_INTERP_GEOMETRIC_AVERAGE, L.PIC_INTERP_HARMONIC_AVERAGE):
            out = torch.zeros((self.n_cells, npr), dtype=torch.float64, device=dev)
            self._chk(self.lib.pic_interpolate(self.h, kind, _ptr(out), None, _ptr(cnt)))
            return out, None, cnt
        out = torch.zeros((self.n_cells, npr, self.dim + 1), dtype=torch.float64, device=dev)
        aux = torch.zeros((self.n_cells, self.dim), dtype=torch.float64, device=dev)
        self._chk(self.lib.pic_interpolate(self.h, kind, _ptr(out), _ptr(aux), _ptr(cnt)))
        return out, aux, cnt

    def interpolate_points(self, kind, qhat):
        """Properties at the evaluation points qhat [dim][n_q] (reference coordinates, the same in every
        cell) from the particles of each cell: returns out [n_cells][n_q][n_prop] and counts."""
        torch = _torch()
        q = np.ascontiguousarray(qhat, np.float64)
        if q.ndim != 2 or q.shape[0] != self.dim:
            raise ValueError(f"qhat must have shape ({self.dim}, n_q)")
        out = torch.empty((self.n_cells, q.shape[1], self.store.n_prop), dtype=torch.float64, device=self.device)
        cnt = torch.zeros(self.n_cells, dtype=torch.int32, device=self.device)
        self._chk(self.lib.pic_interpolate_points(self.h, int(kind), _np_ptr(q), q.shape[1], _ptr(out), _ptr(cnt)))
        return out, cnt

    def transfer_from(self, other: "Problem"):
        """Take the particles of `other` (the mesh before refinement or coarsening, Sec. 2.5): located in
        this mesh, reference locations recomputed, stable by new cell.  `other` is unchanged."""
        self._chk(self.lib.pic_transfer(other.h, self.h))

    def seed_mh(self, counts, rho, J, seed, first_id=0):
        """Metropolis-Hastings generation of counts[K] particles per cell from the nodal density rho
        (Sec. 2.2); returns the longest run of equal consecutive chain states."""
        torch = _torch()
        c = torch.as_tensor(np.ascontiguousarray(counts, np.int32)).to(self.device)
        r = torch.as_tensor(np.ascontiguousarray(rho, np.float64)).to(self.device).contiguous()
        if r.shape != (self.n_nodes,):
            raise ValueError(f"rho must have shape ({self.n_nodes},)")
        longest = C.c_int64()
        self._chk(self.lib.pic_seed_mh(self.h, _ptr(c), _ptr(r), int(J), int(seed), int(first_id),
                                       C.byref(longest)))
        return longest.value

    def seed_mh_static(self, counts, rho, J, seed, first_id=0):
        """seed_mh for callers that cannot allocate: counts (int32 [n_cells]) and rho (float64 [n_nodes])
        are device tensors already; the library stages everything in its fixed device scratch."""
        torch = _torch()
        if counts.dtype != torch.int32 or rho.dtype != torch.float64 or not (counts.is_cuda and rho.is_cuda):
            raise ValueError("counts must be int32 and rho float64 device tensors")
        if counts.numel() != self.n_cells or rho.numel() != self.n_nodes:
            raise ValueError("counts / rho sizes do not match the mesh")
        longest = C.c_int64()
        self._chk(self.lib.pic_seed_mh_static(self.h, _ptr(counts), _ptr(rho), int(J), int(seed), int(first_id),
                                              C.byref(longest)))
        return longest.value

    # ------------------------------------------------------------- adjoint
    def adjoint_workspace(self, n_steps, ckpt_every):
        torch = _torch()
        b = C.c_int64()
        self._chk(self.lib.pic_adjoint_workspace_bytes(self.h, int(n_steps), int(ckpt_every), C.byref(b)))
        return torch.zeros(int(b.value), dtype=torch.uint8, device=self.device)

    def advance_checkpointed(self, dt, n_steps, scheme, ckpt_every, workspace):
        self._chk(self.lib.pic_advance_checkpointed(self.h, float(dt), int(n_steps), int(scheme), int(ckpt_every),
                                                    _ptr(workspace)))

    def adjoint(self, dl_dx_full, workspace, dU):
        """dl_dx_full: [dim][capacity] float64 in the current buffer's order; dU accumulated."""
        self._chk(self.lib.pic_adjoint(self.h, _ptr(dl_dx_full), _ptr(workspace), _ptr(dU)))

    # --------------------------------------------------------- statistics
    def stats(self) -> dict:
        s = L.PicStats()
        self._chk(self.lib.pic_stats_read(self.h, C.byref(s)))
        return {n: getattr(s, n) for n, _ in L.PicStats._fields_}

    def stats_reset(self):
        self._chk(self.lib.pic_stats_reset(self.h))

    def set_launch_graphs(self, enable: bool):
        """Replay the fused step sequence of advance() from a captured HIP graph, or launch its kernels one by
        one (the default, measured faster)."""
        self._chk(self.lib.pic_set_launch_graphs(self.h, int(bool(enable))))

    def profile(self, enable: bool):
        self._chk(self.lib.pic_profile_enable(self.h, int(bool(enable))))

    def profile_read(self, kernel: str):
        ms = C.c_double()
        n = C.c_int64()
        self._chk(self.lib.pic_profile_read(self.h, kernel.encode(), C.byref(ms), C.byref(n)))
        return ms.value, n.value


class Batch:
    """Many problems stepped together from one HIP graph."""

    def __init__(self, problems, tile_cells=(0, 0, 0, 0), stream=None):
        torch = _torch()
        self.lib = L.load()
        self.problems = list(problems)
        # graphs cannot be captured on the legacy default stream: use a stream of our own
        self.stream = stream if stream is not None else torch.cuda.Stream(device=problems[0].device)
        arr = (C.c_void_p * len(self.problems))(*[p.h.value for p in self.problems])
        tiles = (C.c_int32 * 4)(*[int(t) for t in tile_cells])
        h = C.c_void_p()
        L.check(self.lib.pic_batch_create(C.byref(h), len(self.problems), arr, tiles,
                                          C.c_void_p(self.stream.cuda_stream)))
        self.h = h

    def advance(self, dts, schemes, n_steps):
        n = len(self.problems)
        dt = (C.c_double * n)(*[float(v) for v in dts])
        sc = (C.c_int32 * n)(*[int(v) for v in schemes])
        torch = _torch()
        cur = torch.cuda.current_stream(self.problems[0].device)
        self.stream.wait_stream(cur)
        L.check(self.lib.pic_batch_advance(self.h, dt, sc, int(n_steps)), batch=self.h)
        cur.wait_stream(self.stream)

    GROUPS = ("2d-euler", "2d-rk2", "2d-rk4", "3d-euler", "3d-rk2", "3d-rk4")
    SHAPES = {2: ((8, 8), (8, 4), (16, 8)), 3: ((4, 4, 4), (4, 2, 2), (4, 4, 2))}

    def set_schedule(self, variants):
        """Cell-block shape index (0..2) per group, in GROUPS order."""
        v = (C.c_int32 * 6)(*[int(x) for x in variants])
        L.check(self.lib.pic_batch_set_schedule(self.h, v), batch=self.h)

    def tune_cache(self, schemes):
        """The library's tune-cache text of the current schedule for these schemes."""
        n = len(self.problems)
        sc = (C.c_int32 * n)(*[int(v) for v in schemes])
        ln = C.c_int64()
        L.check(self.lib.pic_batch_tune_cache_write(self.h, sc, None, 0, C.byref(ln)), batch=self.h)
        buf = C.create_string_buffer(ln.value + 1)
        L.check(self.lib.pic_batch_tune_cache_write(self.h, sc, buf, ln.value + 1, C.byref(ln)), batch=self.h)
        return buf.value.decode()

    def apply_tune_cache(self, schemes, text):
        """Apply a tune-cache text when its signature matches these problems and schemes; True if applied."""
        n = len(self.problems)
        sc = (C.c_int32 * n)(*[int(v) for v in schemes])
        ok = C.c_int32()
        L.check(self.lib.pic_batch_tune_cache_apply(self.h, sc, text.encode(), C.byref(ok)), batch=self.h)
        return bool(ok.value)

    def tune(self, dts, schemes, trials=3, cache=None):
        """Pick the fastest cell-block shape per group (the library's autotuner) and return
        {"variants": [...], "times_ms": {...}}.  With `cache` (a file path) the library's tune-cache text
        stored there is applied without timing when its signature matches, and a new choice is stored."""
        import json
        import os
        if cache and os.path.exists(cache):
            with open(cache) as f:
                text = f.read()
            if self.apply_tune_cache(schemes, text):
                rec = json.loads(text)
                rec["cached"] = True
                return rec
        n = len(self.problems)
        dt = (C.c_double * n)(*[float(v) for v in dts])
        sc = (C.c_int32 * n)(*[int(v) for v in schemes])
        var = (C.c_int32 * 6)()
        tms = (C.c_double * 18)()
        torch = _torch()
        cur = torch.cuda.current_stream(self.problems[0].device)
        self.stream.wait_stream(cur)
        L.check(self.lib.pic_batch_tune(self.h, dt, sc, int(trials), var, tms), batch=self.h)
        cur.wait_stream(self.stream)
        times = {}
        for g, name in enumerate(self.GROUPS):
            if tms[3 * g] >= 0:
                d = 2 if g < 3 else 3
                times[name] = {"x".join(map(str, self.SHAPES[d][v])): tms[3 * g + v] for v in range(3)}
        rec = json.loads(self.tune_cache(schemes))
        rec["times_ms"] = times
        if cache:
            with open(cache, "w") as f:
                f.write(self.tune_cache(schemes))
        return rec

    def close(self):
        if getattr(self, "h", None) is not None:
            self.lib.pic_batch_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
