"""Python binding of the VBD library: topology handle, step, adjoint, autograd.

Every computation runs in libvbd.so (HIP kernels for gfx950).  torch is used
for device memory (state tensors, the workspace) and streams only.
"""
from __future__ import annotations

import ctypes as C
from typing import Optional

import numpy as np
import torch

from . import _native as N
from .workloads import StepParams, Workload


def _np_ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _t_ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _stream_handle(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def params_struct(p: StepParams, launch_mode: int = N.LAUNCH_PLAIN, backward_recorded: bool = False,
                  check_finite: bool = False):
    """StepParams -> (vbd_step_params, keep-alive arrays)."""
    sph = None if p.spheres is None else np.ascontiguousarray(p.spheres, np.float32).reshape(-1, 4)
    pl = None if p.planes is None else np.ascontiguousarray(p.planes, np.float32).reshape(-1, 4)
    s = N.StepParamsC(float(p.h), int(p.n_iters), (C.c_float * 3)(*[float(g) for g in p.gravity]),
                      int(p.init_mode), float(p.det_eps_rel), float(p.contact_k),
                      float(p.contact_thickness), 0 if sph is None else sph.shape[0], _np_ptr(sph),
                      0 if pl is None else pl.shape[0], _np_ptr(pl), float(p.kd), float(p.cheb_rho),
                      float(p.friction_mu), float(p.friction_eps_v),
                      int(bool(getattr(p, "spring_psd", False))), int(launch_mode),
                      int(bool(getattr(p, "mesh_contacts", False))),
                      float(getattr(p, "collision_radius", 0.0)), int(getattr(p, "n_col", 0)),
                      1 if backward_recorded else 0, 1 if check_finite else 0,
                      int(bool(getattr(p, "self_contact", False))), float(getattr(p, "self_exclusion", 0.0)),
                      int(bool(getattr(p, "edge_contacts", False))))
    return s, (sph, pl)


def _check_state(t, n, name):
    if not (t.is_cuda and t.dtype == torch.float32 and t.is_contiguous()):
        raise ValueError(f"{name} must be a contiguous float32 CUDA tensor")
    if t.numel() != 3 * n:
        raise ValueError(f"{name} must hold n_verts*3 = {3 * n} floats, got {t.numel()}")


class Topology:
    """Handle on a colored, device-resident VBD topology (one or many meshes)."""

    def __init__(self, rest, tets=None, *, springs=None, pinned=None, mass=None, density=1000.0,
                 nu=0.3, spring_k=0.0, spring_rest=None, vert_offsets=None, tet_offsets=None,
                 max_backward_iters: int = 0, device: Optional[torch.device] = None,
                 bind: bool = True, colors=None, coloring: str = "id"):
        """colors: optional caller-supplied vertex coloring; else greedy first fit
        in the vertex order `coloring` ("id", "smallest_last" or "dsatur")."""
        L = N.lib()
        self._keep = []

        def arr(a, dt):
            if a is None:
                return None
            a = np.ascontiguousarray(a, dt)
            self._keep.append(a)
            return a

        rest = arr(rest, np.float64).reshape(-1, 3)
        tets = arr(tets if tets is not None else np.zeros((0, 4)), np.int32).reshape(-1, 4)
        springs = arr(springs, np.int32)
        if springs is not None:
            springs = springs.reshape(-1, 2)
        n_meshes = 1 if vert_offsets is None else len(vert_offsets) - 1
        vo = arr(vert_offsets, np.int64)
        to = arr(tet_offsets, np.int64)
        desc = N.MeshDesc(rest.shape[0], tets.shape[0], 0 if springs is None else springs.shape[0],
                          n_meshes, _np_ptr(vo), _np_ptr(to), _np_ptr(tets), _np_ptr(springs),
                          _np_ptr(rest), _np_ptr(arr(spring_rest, np.float64)), float(spring_k),
                          _np_ptr(arr(mass, np.float64)), float(density), float(nu),
                          _np_ptr(arr(pinned, np.uint8)))
        h = C.c_void_p()
        N.check(L.vbd_build_topology(C.byref(desc), C.byref(h)))
        self._h = h
        self.n_verts = rest.shape[0]
        self.n_tets = tets.shape[0]
        self.n_springs = 0 if springs is None else springs.shape[0]
        self.max_backward_iters = int(max_backward_iters)
        if colors is not None:
            col = arr(colors, np.int32).reshape(-1)
            if col.shape[0] != self.n_verts:
                raise ValueError("colors must hold one entry per vertex")
            N.check(L.vbd_color_given(self._h, _np_ptr(col)))
            self.n_colors = int(col.max()) + 1 if col.size else 0
        else:
            order = {"id": N.COLOR_ID_ORDER, "smallest_last": N.COLOR_SMALLEST_LAST,
                     "dsatur": N.COLOR_DSATUR}[coloring]
            nc = C.c_int32()
            N.check(L.vbd_color_greedy(self._h, order, C.byref(nc), None))
            self.n_colors = nc.value
        self.workspace = None
        if bind:
            self.bind(device)

    @classmethod
    def from_workload(cls, w: Workload, **kw):
        kw.setdefault("colors", w.colors)
        kw.setdefault("coloring", w.coloring)
        return cls(w.rest, w.tets, springs=w.springs, pinned=w.pinned, mass=w.mass,
                   density=w.density, nu=w.nu, spring_k=w.spring_k, spring_rest=w.spring_rest,
                   vert_offsets=w.vert_offsets if w.n_meshes > 1 else None,
                   tet_offsets=w.tet_offsets if w.n_meshes > 1 else None, **kw)

    def bind(self, device=None, stream=None):
        L = N.lib()
        dev = torch.device(device) if device is not None else torch.device("cuda", torch.cuda.current_device())
        nbytes = C.c_size_t()
        N.check(L.vbd_workspace_size(self._h, self.max_backward_iters, C.byref(nbytes)))
        self.workspace = torch.empty(int(nbytes.value), dtype=torch.uint8, device=dev)
        with torch.cuda.device(dev):
            N.check(L.vbd_bind_workspace(self._h, _t_ptr(self.workspace), int(nbytes.value),
                                         _stream_handle(stream)))
        self.device = dev

    # ----------------------------------------------------------- queries --
    def counts(self):
        out = np.zeros(8, np.int64)
        N.check(N.lib().vbd_topology_query(self._h, N.Q_COUNTS, _np_ptr(out), out.nbytes))
        keys = ["n_verts", "n_tets", "n_springs", "n_colors", "n_free", "tet_entries",
                "spring_entries", "n_meshes"]
        return dict(zip(keys, out.tolist()))

    def query(self, what: int):
        c = self.counts()
        n_free = c["n_free"]
        spec = {N.Q_COLORS: (np.int32, c["n_verts"]), N.Q_PERM: (np.int32, c["n_verts"]),
                N.Q_COLOR_OFFSETS: (np.int32, c["n_colors"] + 1), N.Q_TET_ROWS: (np.int32, c["n_verts"] + 1),
                N.Q_TET_ENTRIES: (np.int32, c["tet_entries"]), N.Q_SPRING_ROWS: (np.int32, n_free + 1),
                N.Q_SPRING_NBRS: (np.int32, c["spring_entries"]), N.Q_MASS: (np.float64, c["n_verts"]),
                N.Q_DMINV: (np.float64, 9 * c["n_tets"]), N.Q_VOLUME: (np.float64, c["n_tets"]),
                N.Q_PHASE_BYTES: (np.float64, c["n_colors"]),
                N.Q_TET_ORDER: (np.int32, c["n_tets"]),
                N.Q_REST_FRAME: (np.float64, 6 * c["n_tets"]),
                N.Q_SURFACE_COUNTS: (np.int64, 3), N.Q_SNAPSHOT_REGION: (np.int64, 3),
                N.Q_ADJ_PHASE_BYTES: (np.float64, c["n_colors"]),
                N.Q_PHASE_COUNTS: (np.int64, 4 * c["n_colors"]),
                N.Q_XCD_SPLIT: (np.int32, 9 * c["n_colors"])}
        if what == N.Q_SURFACE:
            n_tri = int(self.query(N.Q_SURFACE_COUNTS)[0])
            out = np.zeros((n_tri, 3), np.int32)
            N.check(N.lib().vbd_topology_query(self._h, what, _np_ptr(out), out.nbytes))
            return out
        if what == N.Q_SURFACE_EDGES:
            n_edge = int(self.query(N.Q_SURFACE_COUNTS)[2])
            out = np.zeros((n_edge, 2), np.int32)
            N.check(N.lib().vbd_topology_query(self._h, what, _np_ptr(out), out.nbytes))
            return out
        spec = spec[what]
        out = np.zeros(spec[1], spec[0])
        N.check(N.lib().vbd_topology_query(self._h, what, _np_ptr(out), out.nbytes))
        return out

    # ----------------------------------------------------------- compute --
    def detect_contacts(self, x, params: StepParams, stream=None):
        """Mesh-mesh contact detection on positions x (device float32 [n_verts, 3]):
        int32 [n_verts] contact triangle (index into the Q_SURFACE rows) or -1."""
        _check_state(x, self.n_verts, "x")
        out = torch.empty(self.n_verts, dtype=torch.int32, device=x.device)
        ps, keep = params_struct(params)
        N.check(N.lib().vbd_detect_contacts(self._h, C.byref(ps), _t_ptr(x), _t_ptr(out),
                                            _stream_handle(stream)))
        return out

    def detect_edges(self, x, params: StepParams, x_t=None, stream=None):
        """Edge-edge detection with closest points on x and normals from x_t
        (default x), device float32 [n_verts, 3]: int32 [n_surf_edges], for
        each surface edge the second edge of the element kept from it, or -1."""
        _check_state(x, self.n_verts, "x")
        xt = x if x_t is None else x_t
        _check_state(xt, self.n_verts, "x_t")
        n_edge = int(self.query(N.Q_SURFACE_COUNTS)[2])
        out = torch.empty(max(n_edge, 1), dtype=torch.int32, device=x.device)
        ps, keep = params_struct(params)
        N.check(N.lib().vbd_detect_edges(self._h, C.byref(ps), _t_ptr(x), _t_ptr(xt), _t_ptr(out),
                                         _stream_handle(stream)))
        return out[:n_edge]

    def step(self, x, v, v_prev, tet_E, params: StepParams, launch_mode: int = N.LAUNCH_PLAIN,
             stream=None, check_finite: bool = False):
        """One time step in place on (x, v, v_prev): device float32 [n_verts, 3].
        check_finite: count non-finite outputs on the device (check() then
        raises VBD_E_NONFINITE)."""
        for t, name in ((x, "x"), (v, "v"), (v_prev, "v_prev")):
            _check_state(t, self.n_verts, name)
        if self.n_tets:
            if not (tet_E.is_cuda and tet_E.dtype == torch.float32 and tet_E.numel() == self.n_tets
                    and tet_E.is_contiguous()):
                raise ValueError("tet_E must be a contiguous float32 CUDA tensor of n_tets")
        ps, keep = params_struct(params, launch_mode, check_finite=check_finite)
        N.check(N.lib().vbd_step(self._h, C.byref(ps), _t_ptr(x), _t_ptr(v), _t_ptr(v_prev),
                                 _t_ptr(tet_E) if self.n_tets else None, _stream_handle(stream)))

    def step_static(self, x, v, v_prev, tet_E, params: StepParams, launch_mode: int = N.LAUNCH_PLAIN,
                    stream=None, check_finite: bool = False):
        """step() without allocation: the step's state buffers come from the
        library's fixed per-device scratch (vbd_step_static; PLAIN or
        PERSISTENT launches, no mesh contacts)."""
        for t, name in ((x, "x"), (v, "v"), (v_prev, "v_prev")):
            _check_state(t, self.n_verts, name)
        if self.n_tets:
            if not (tet_E.is_cuda and tet_E.dtype == torch.float32 and tet_E.numel() == self.n_tets
                    and tet_E.is_contiguous()):
                raise ValueError("tet_E must be a contiguous float32 CUDA tensor of n_tets")
        ps, keep = params_struct(params, launch_mode, check_finite=check_finite)
        N.check(N.lib().vbd_step_static(self._h, C.byref(ps), _t_ptr(x), _t_ptr(v), _t_ptr(v_prev),
                                        _t_ptr(tet_E) if self.n_tets else None,
                                        _stream_handle(stream)))

    def step_record(self, x, v, v_prev, tet_E, params: StepParams, launch_mode: int = N.LAUNCH_PLAIN,
                    stream=None):
        """step() for the differentiable path, leaving the step's iterates in
        the workspace snapshots (see snapshots())."""
        for t, name in ((x, "x"), (v, "v"), (v_prev, "v_prev")):
            _check_state(t, self.n_verts, name)
        ps, keep = params_struct(params, launch_mode)
        N.check(N.lib().vbd_step_record(self._h, C.byref(ps), _t_ptr(x), _t_ptr(v), _t_ptr(v_prev),
                                        _t_ptr(tet_E) if self.n_tets else None, _stream_handle(stream)))

    def snapshots(self, n_iters: int):
        """The workspace bytes holding a step's n_iters + 1 iterate snapshots
        (a uint8 view into the bound workspace tensor)."""
        off, per, cap = (int(a) for a in self.query(N.Q_SNAPSHOT_REGION))
        if off < 0 or n_iters > cap:
            raise ValueError(f"the workspace holds {cap} backward iterations, need {n_iters}")
        return self.workspace[off:off + per * (n_iters + 1)]

    def step_backward(self, x_t, v_t, v_prev, tet_E, gx_out, gv_out, gvp_out, gx_in, gv_in,
                      gvp_in, g_tet_E, params: StepParams, launch_mode: int = N.LAUNCH_PLAIN,
                      stream=None, recorded: bool = False):
        """recorded: the snapshots already hold this step's iterates (from
        step_record, or copied back into snapshots()); the recompute is skipped."""
        for t, name in ((x_t, "x_t"), (v_t, "v_t"), (v_prev, "v_prev"), (gx_out, "gx_out"),
                        (gv_out, "gv_out"), (gvp_out, "gvp_out"), (gx_in, "gx_in"),
                        (gv_in, "gv_in"), (gvp_in, "gvp_in")):
            _check_state(t, self.n_verts, name)
        ps, keep = params_struct(params, launch_mode, backward_recorded=recorded)
        N.check(N.lib().vbd_step_backward(self._h, C.byref(ps), _t_ptr(x_t), _t_ptr(v_t),
                                          _t_ptr(v_prev), _t_ptr(tet_E), _t_ptr(gx_out),
                                          _t_ptr(gv_out), _t_ptr(gvp_out), _t_ptr(gx_in),
                                          _t_ptr(gv_in), _t_ptr(gvp_in), _t_ptr(g_tet_E),
                                          _stream_handle(stream)))

    def autotune(self, x, v, v_prev, tet_E, params: StepParams, launch_mode=N.LAUNCH_PLAIN,
                 stream=None):
        ps, keep = params_struct(params, launch_mode)
        N.check(N.lib().vbd_autotune(self._h, C.byref(ps), _t_ptr(x), _t_ptr(v), _t_ptr(v_prev),
                                     _t_ptr(tet_E) if self.n_tets else None, _stream_handle(stream)))
        return self.launch_config

    @property
    def launch_config(self):
        c = N.LaunchConfig()
        N.check(N.lib().vbd_get_launch_config(self._h, C.byref(c)))
        return dict(lanes_per_vertex=c.lanes_per_vertex, block_size=c.block_size,
                    xcd_remap=c.xcd_remap, blocks_per_cu=c.blocks_per_cu, tet_unroll=c.tet_unroll,
                    compact_records=c.compact_records)

    @launch_config.setter
    def launch_config(self, cfg):
        cur = self.launch_config
        cur.update(cfg)
        c = N.LaunchConfig(cur["lanes_per_vertex"], cur["block_size"], cur["xcd_remap"],
                           cur["blocks_per_cu"], cur["tet_unroll"], cur["compact_records"])
        N.check(N.lib().vbd_set_launch_config(self._h, C.byref(c)))

    def profile_enable(self, on: bool = True):
        N.check(N.lib().vbd_profile_enable(self._h, 1 if on else 0))

    def profile_read(self, reset: bool = True):
        s = N.ProfileStats()
        N.check(N.lib().vbd_profile_read(self._h, C.byref(s), 1 if reset else 0))
        return dict(n_launches=s.n_launches, total_ms=s.total_ms, total_bytes=s.total_bytes,
                    n_vertex_updates=s.n_vertex_updates)

    def check(self, stream=None):
        N.check(N.lib().vbd_check(self._h, _stream_handle(stream)))

    def counters(self, reset: bool = False, stream=None):
        """Device event counters: determinant-rule skips and non-finite outputs."""
        c = N.Counters()
        N.check(N.lib().vbd_read_counters(self._h, C.byref(c), 1 if reset else 0,
                                          _stream_handle(stream)))
        return dict(n_skips=int(c.n_skips), n_nonfinite=int(c.n_nonfinite))

    def __del__(self):
        h = getattr(self, "_h", None)
        if h is not None and h.value:
            try:
                N.lib().vbd_topology_destroy(h)
            except Exception:
                pass
            self._h = None


def probe_read(src: torch.Tensor, partials: torch.Tensor, stream=None):
    """Read-only streaming probe over src; partials: float32 CUDA tensor, one
    entry per block (its length sets the grid)."""
    if not (partials.is_cuda and partials.dtype == torch.float32 and partials.is_contiguous()):
        raise ValueError("partials must be a contiguous float32 CUDA tensor")
    N.check(N.lib().vbd_probe_read(_t_ptr(src), src.numel() * src.element_size(), _t_ptr(partials),
                                   partials.numel(), _stream_handle(stream)))


def probe_copy(dst: torch.Tensor, src: torch.Tensor, stream=None):
    N.check(N.lib().vbd_probe_copy(_t_ptr(dst), _t_ptr(src), src.numel() * src.element_size(),
                                   _stream_handle(stream)))


class Rollout(torch.autograd.Function):
    """Unrolled VBD frames with per-frame checkpoints and the hand-written
    adjoint kernels in the backward.

    apply(x0, v0, tet_E, topo, params, frames, record_bytes=2**33) -> (x_T, v_T);
    the state before frame 0 has v^{-1} = v^0.  When the iterates of all
    frames fit in record_bytes of device memory, the forward keeps each
    frame's iterate snapshots and the backward skips its recompute; else the
    backward recomputes them frame by frame.  Both directions work on fixed
    buffers so that one captured hipGraph per direction is replayed for every
    frame.
    """

    @staticmethod
    def forward(ctx, x0, v0, tet_E, topo: Topology, params: StepParams, frames: int,
                record_bytes: int = 1 << 33):
        # x, v, v_prev as three views of one buffer: a frame's checkpoint is
        # one copy
        xvv = torch.empty((3,) + tuple(x0.shape), dtype=torch.float32, device=x0.device)
        xvv[0].copy_(x0.detach())
        xvv[1].copy_(v0.detach())
        xvv[2].copy_(v0.detach())
        x, v, vp = xvv[0], xvv[1], xvv[2]
        E = tet_E.detach().contiguous()
        states = torch.empty((frames,) + tuple(xvv.shape), dtype=torch.float32, device=x0.device)
        records = None
        snaps = topo.snapshots(params.n_iters) if topo.max_backward_iters >= params.n_iters else None
        if snaps is not None and frames * snaps.numel() <= record_bytes:
            records = torch.empty((frames, snaps.numel()), dtype=torch.uint8, device=x.device)
        for f in range(frames):
            states[f].copy_(xvv)
            if records is None:
                topo.step(x, v, vp, E, params, N.LAUNCH_GRAPH)
            else:
                topo.step_record(x, v, vp, E, params, N.LAUNCH_GRAPH)
                records[f].copy_(snaps)
        ctx.topo, ctx.params, ctx.states, ctx.records = topo, params, states, records
        ctx.save_for_backward(E)
        return x.clone(), v.clone()

    @staticmethod
    def backward(ctx, gx, gv):
        (E,) = ctx.saved_tensors
        topo, params, records, states = ctx.topo, ctx.params, ctx.records, ctx.states
        # fixed buffers (one captured graph serves every frame), each set of
        # three arrays one buffer so that a hand-over is one copy
        g_out = torch.zeros_like(states[0])
        for k, g in enumerate((gx, gv)):
            if g is not None:
                g_out[k].copy_(g)
        g_in = torch.empty_like(g_out)
        stage = torch.empty_like(g_out)
        gE = torch.zeros_like(E)
        snaps = topo.snapshots(params.n_iters) if records is not None else None
        for f in reversed(range(states.shape[0])):
            stage.copy_(states[f])
            if records is not None:
                snaps.copy_(records[f])
            topo.step_backward(*stage, E, *g_out, *g_in, gE, params, N.LAUNCH_GRAPH,
                               recorded=records is not None)
            g_out.copy_(g_in)
        gx0, gv0, gvp0 = g_out
        return gx0.clone(), gv0 + gvp0, gE, None, None, None, None
