"""ctypes wrapper of the FP64 VBD oracle.

TEST INFRASTRUCTURE ONLY: imported by the test suite, the smoke check and the
benchmark's CPU-baseline leg.  The product library never imports it.

Inputs are plain numpy arrays plus a parameter object with attributes
``h, n_iters, gravity, init_mode, det_eps_rel, contact_k, contact_thickness,
spheres, planes, kd, cheb_rho, friction_mu, friction_eps_v``.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        d, i32, p = C.c_double, C.c_int32, C.c_void_p
        L.oracle_color_greedy.argtypes = [i32, i32, p, i32, p, p]
        L.oracle_color_greedy.restype = i32
        L.oracle_color_smallest_last.argtypes = [i32, i32, p, i32, p, p]
        L.oracle_color_smallest_last.restype = i32
        L.oracle_color_dsatur.argtypes = [i32, i32, p, i32, p, p]
        L.oracle_color_dsatur.restype = i32
        L.oracle_tet_rest.argtypes = [i32, p, p, p, p]
        L.oracle_tet_rest.restype = i32
        L.oracle_lumped_mass.argtypes = [i32, i32, p, p, d, p]
        L.oracle_spring_rest.argtypes = [i32, p, p, p]
        L.oracle_lame.argtypes = [d, d, p, p]
        L.oracle_tet_energy.argtypes = [p, p, d, d, d]
        L.oracle_tet_energy.restype = d
        L.oracle_tet_derivs.argtypes = [p, p, d, d, d, p, p]
        L.oracle_spring_energy.argtypes = [p, p, d, d]
        L.oracle_spring_energy.restype = d
        L.oracle_spring_derivs.argtypes = [p, p, d, d, p, p]
        for name in ("oracle_step", "oracle_step_cs"):
            fn = getattr(L, name)
            fn.argtypes = [p, p, p, p, p, p, p, p, i32, p]
            fn.restype = i32
        L.oracle_predict.argtypes = [p, p, p, p, p]
        L.oracle_energy_G.argtypes = [p, p, p, p, p, p, p]
        L.oracle_energy_G.restype = d
        L.oracle_step_backward.argtypes = [p] * 13
        L.oracle_step_backward.restype = i32
        L.oracle_set_threads.argtypes = [i32]
        L.oracle_surface.argtypes = [i32, p, p, p]
        L.oracle_surface.restype = i32
        L.oracle_closest_point_triangle.argtypes = [p, p, p, p, p, p]
        L.oracle_detect_contacts.argtypes = [p, p, p, p]
        L.oracle_winding_number.argtypes = [p, C.c_int32, p, p]
        L.oracle_segment_closest.argtypes = [p, p, p, p, p, p]
        L.oracle_segment_closest.restype = d
        L.oracle_detect_edges.argtypes = [p, p, p, p, i32, p, p]
        L.oracle_detect_edges.restype = i32
        L.oracle_edge_element.argtypes = [p, p, d, d, p]
        L.oracle_edge_element.restype = d
        L.oracle_edge_element_friction.argtypes = [p, p, p, d, d, d, d, d, p]
        L.oracle_edge_element_friction.restype = d
        L.oracle_winding_number.restype = C.c_double
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


class _Model(C.Structure):
    _fields_ = [("n_verts", C.c_int32), ("n_tets", C.c_int32), ("n_springs", C.c_int32),
                ("n_colors", C.c_int32), ("tets", C.c_void_p), ("springs", C.c_void_p),
                ("Dminv", C.c_void_p), ("vol", C.c_void_p), ("spring_rest", C.c_void_p),
                ("mass", C.c_void_p), ("pinned", C.c_void_p), ("colors", C.c_void_p),
                ("nu", C.c_double), ("spring_k", C.c_double),
                ("n_surf_tris", C.c_int32), ("surf_tris", C.c_void_p), ("vert_mesh", C.c_void_p),
                ("rest_pos", C.c_void_p)]


class _Params(C.Structure):
    _fields_ = [("h", C.c_double), ("n_iters", C.c_int32), ("gravity", C.c_double * 3),
                ("init_mode", C.c_int32), ("det_eps_rel", C.c_double),
                ("contact_k", C.c_double), ("contact_thickness", C.c_double),
                ("n_spheres", C.c_int32), ("spheres", C.c_void_p),
                ("n_planes", C.c_int32), ("planes", C.c_void_p),
                ("kd", C.c_double), ("cheb_rho", C.c_double),
                ("friction_mu", C.c_double), ("friction_eps_v", C.c_double),
                ("spring_psd", C.c_int32), ("mesh_contacts", C.c_int32),
                ("collision_radius", C.c_double), ("n_col", C.c_int32),
                ("self_contact", C.c_int32), ("self_exclusion", C.c_double),
                ("edge_contacts", C.c_int32)]


class _Stats(C.Structure):
    _fields_ = [("n_updates", C.c_int64), ("n_skips", C.c_int64),
                ("max_local_grad", C.c_double), ("n_contacts", C.c_int64)]


def set_threads(n: int) -> None:
    lib().oracle_set_threads(int(n))


def color_greedy(n_verts, tets, springs=None, order="id"):
    """Greedy coloring; order "id" (first fit in ascending vertex id),
    "smallest_last" (first fit in Matula-Beck smallest-last order) or
    "dsatur" (Brelaz's saturation order)."""
    tets = np.ascontiguousarray(tets, np.int32)
    sp = None if springs is None or len(springs) == 0 else np.ascontiguousarray(springs, np.int32)
    colors = np.zeros(n_verts, np.int32)
    fn = {"id": lib().oracle_color_greedy, "smallest_last": lib().oracle_color_smallest_last,
          "dsatur": lib().oracle_color_dsatur}[order]
    nc = fn(n_verts, tets.shape[0], _ptr(tets), 0 if sp is None else sp.shape[0], _ptr(sp),
            _ptr(colors))
    return colors, int(nc)


def tet_rest(tets, rest):
    tets = np.ascontiguousarray(tets, np.int32)
    rest = np.ascontiguousarray(rest, np.float64)
    nt = tets.shape[0]
    Dminv = np.zeros((nt, 9)); vol = np.zeros(nt)
    r = lib().oracle_tet_rest(nt, _ptr(tets), _ptr(rest), _ptr(Dminv), _ptr(vol))
    if r != 0:
        raise ValueError(f"degenerate rest tet {-1 - r}")
    return Dminv, vol


def lumped_mass(n_verts, tets, vol, density):
    tets = np.ascontiguousarray(tets, np.int32)
    m = np.zeros(n_verts)
    lib().oracle_lumped_mass(n_verts, tets.shape[0], _ptr(tets), _ptr(np.ascontiguousarray(vol)),
                             float(density), _ptr(m))
    return m


def spring_rest(springs, rest):
    springs = np.ascontiguousarray(springs, np.int32)
    L = np.zeros(springs.shape[0])
    lib().oracle_spring_rest(springs.shape[0], _ptr(springs),
                             _ptr(np.ascontiguousarray(rest, np.float64)), _ptr(L))
    return L


def lame(E, nu):
    mu, lam = C.c_double(), C.c_double()
    lib().oracle_lame(float(E), float(nu), C.byref(mu), C.byref(lam))
    return mu.value, lam.value


def tet_energy(x12, Dminv9, vol, mu, lam):
    x = np.ascontiguousarray(x12, np.float64).ravel(); B = np.ascontiguousarray(Dminv9, np.float64).ravel()
    return lib().oracle_tet_energy(_ptr(x), _ptr(B), float(vol), float(mu), float(lam))


def tet_derivs(x12, Dminv9, vol, mu, lam):
    x = np.ascontiguousarray(x12, np.float64).ravel(); B = np.ascontiguousarray(Dminv9, np.float64).ravel()
    g = np.zeros(12); H = np.zeros((12, 12))
    lib().oracle_tet_derivs(_ptr(x), _ptr(B), float(vol), float(mu), float(lam), _ptr(g), _ptr(H))
    return g, H


def spring_energy(xa, xb, L, k):
    a = np.ascontiguousarray(xa, np.float64); b = np.ascontiguousarray(xb, np.float64)
    return lib().oracle_spring_energy(_ptr(a), _ptr(b), float(L), float(k))


def spring_derivs(xa, xb, L, k):
    a = np.ascontiguousarray(xa, np.float64); b = np.ascontiguousarray(xb, np.float64)
    g = np.zeros(6); H = np.zeros((6, 6))
    lib().oracle_spring_derivs(_ptr(a), _ptr(b), float(L), float(k), _ptr(g), _ptr(H))
    return g, H


def surface(tets, rest):
    tets = np.ascontiguousarray(tets, np.int32)
    out = np.zeros((4 * tets.shape[0], 3), np.int32)
    n = lib().oracle_surface(tets.shape[0], _ptr(tets), _ptr(np.ascontiguousarray(rest, np.float64)),
                             _ptr(out))
    return out[:n].copy()


def closest_point_triangle(p, a, b, c):
    arr = [np.ascontiguousarray(v, np.float64) for v in (p, a, b, c)]
    q = np.zeros(3); bary = np.zeros(3)
    lib().oracle_closest_point_triangle(*[_ptr(v) for v in arr], _ptr(q), _ptr(bary))
    return q, bary


class Model:
    """Oracle-side model: rest data, masses and coloring computed by the oracle."""

    def __init__(self, rest, tets, pinned, *, density=1000.0, nu=0.3, springs=None,
                 spring_rest_len=None, spring_k=0.0, mass=None, vert_offsets=None,
                 coloring="id"):
        self.rest = np.ascontiguousarray(rest, np.float64)
        self.n_verts = self.rest.shape[0]
        self.tets = np.ascontiguousarray(tets, np.int32).reshape(-1, 4)
        self.springs = (np.ascontiguousarray(springs, np.int32).reshape(-1, 2)
                        if springs is not None and len(springs) else np.zeros((0, 2), np.int32))
        self.pinned = np.ascontiguousarray(pinned, np.uint8)
        self.nu = float(nu)
        self.spring_k = float(spring_k)
        if self.tets.shape[0] and not (0.0 < self.nu < 0.5):
            # the energy's rest offset alpha = 1 + mu/lambda needs lambda > 0
            raise ValueError("nu must be in (0, 0.5)")
        if self.tets.shape[0]:
            self.Dminv, self.vol = tet_rest(self.tets, self.rest)
        else:
            self.Dminv, self.vol = np.zeros((0, 9)), np.zeros(0)
        if mass is None:
            self.mass = lumped_mass(self.n_verts, self.tets, self.vol, density)
        else:
            self.mass = np.ascontiguousarray(mass, np.float64)
        if self.springs.shape[0]:
            self.spring_rest = (spring_rest(self.springs, self.rest) if spring_rest_len is None
                                else np.ascontiguousarray(spring_rest_len, np.float64))
        else:
            self.spring_rest = np.zeros(0)
        self.colors, self.n_colors = color_greedy(self.n_verts, self.tets, self.springs, coloring)
        self.surf_tris = (surface(self.tets, self.rest) if self.tets.shape[0]
                          else np.zeros((0, 3), np.int32))
        self.vert_mesh = np.zeros(self.n_verts, np.int32)
        if vert_offsets is not None:
            for k in range(len(vert_offsets) - 1):
                self.vert_mesh[int(vert_offsets[k]):int(vert_offsets[k + 1])] = k
        self._s = _Model(self.n_verts, self.tets.shape[0], self.springs.shape[0], self.n_colors,
                         _ptr(self.tets), _ptr(self.springs), _ptr(self.Dminv), _ptr(self.vol),
                         _ptr(self.spring_rest), _ptr(self.mass), _ptr(self.pinned),
                         _ptr(self.colors), self.nu, self.spring_k, self.surf_tris.shape[0],
                         _ptr(self.surf_tris), _ptr(self.vert_mesh), _ptr(self.rest))

    @classmethod
    def from_workload(cls, w):
        m = cls(w.rest, w.tets, w.pinned, density=w.density, nu=w.nu, springs=w.springs,
                spring_rest_len=w.spring_rest, spring_k=w.spring_k, mass=w.mass,
                vert_offsets=w.vert_offsets, coloring=getattr(w, "coloring", "id"))
        if getattr(w, "colors", None) is not None:
            m.set_colors(w.colors)
        return m

    def set_colors(self, colors):
        """Replace the coloring (tests of coloring-dependent behaviour)."""
        self.colors = np.ascontiguousarray(colors, np.int32)
        self.n_colors = int(self.colors.max()) + 1 if self.colors.size else 0
        self._s.colors = _ptr(self.colors)
        self._s.n_colors = self.n_colors


def _params(p):
    sph = None if getattr(p, "spheres", None) is None else np.ascontiguousarray(p.spheres, np.float64).reshape(-1, 4)
    pl = None if getattr(p, "planes", None) is None else np.ascontiguousarray(p.planes, np.float64).reshape(-1, 4)
    s = _Params(float(p.h), int(p.n_iters), (C.c_double * 3)(*[float(g) for g in p.gravity]),
                int(p.init_mode), float(p.det_eps_rel), float(p.contact_k),
                float(p.contact_thickness), 0 if sph is None else sph.shape[0], _ptr(sph),
                0 if pl is None else pl.shape[0], _ptr(pl), float(p.kd), float(p.cheb_rho),
                float(p.friction_mu), float(p.friction_eps_v), int(bool(getattr(p, "spring_psd", False))),
                int(bool(getattr(p, "mesh_contacts", False))), float(getattr(p, "collision_radius", 0.0)),
                int(getattr(p, "n_col", 0)), int(bool(getattr(p, "self_contact", False))),
                float(getattr(p, "self_exclusion", 0.0)), int(bool(getattr(p, "edge_contacts", False))))
    return s, (sph, pl)


def step(model: Model, params, x, v, vprev, tet_E, *, order=None, G_trace=False,
         track_local_grad=False):
    """One step.  Returns (x, v, vprev, stats[, G_trace]) as new arrays."""
    x = np.array(x, np.float64, order="C"); v = np.array(v, np.float64, order="C")
    vp = np.array(vprev, np.float64, order="C")
    E = np.ascontiguousarray(tet_E, np.float64)
    ps, keep = _params(params)
    st = _Stats()
    gt = np.zeros(params.n_iters * model.n_colors) if G_trace else None
    od = None if order is None else np.ascontiguousarray(order, np.int32)
    r = lib().oracle_step(C.byref(model._s), C.byref(ps), _ptr(x), _ptr(v), _ptr(vp), _ptr(E),
                          _ptr(od), _ptr(gt), int(bool(track_local_grad)), C.byref(st))
    if r != 0:
        raise ValueError(f"oracle_step failed ({r})")
    stats = dict(n_updates=st.n_updates, n_skips=st.n_skips, max_local_grad=st.max_local_grad,
                 n_contacts=st.n_contacts)
    if G_trace:
        return x, v, vp, stats, gt
    return x, v, vp, stats


def step_cs(model: Model, params, x, v, vprev, tet_E):
    """Complex-step variant: complex128 arrays in and out."""
    x = np.array(x, np.complex128, order="C"); v = np.array(v, np.complex128, order="C")
    vp = np.array(vprev, np.complex128, order="C")
    E = np.ascontiguousarray(tet_E, np.complex128)
    ps, keep = _params(params)
    st = _Stats()
    r = lib().oracle_step_cs(C.byref(model._s), C.byref(ps), _ptr(x), _ptr(v), _ptr(vp), _ptr(E),
                             None, None, 0, C.byref(st))
    if r != 0:
        raise ValueError(f"oracle_step_cs failed ({r})")
    return x, v, vp


def detect_contacts(model: Model, params, x):
    x = np.ascontiguousarray(x, np.float64)
    out = np.zeros(model.n_verts, np.int32)
    ps, keep = _params(params)
    lib().oracle_detect_contacts(C.byref(model._s), C.byref(ps), _ptr(x), _ptr(out))
    return out


def segment_closest(p0, p1, q0, q1):
    """(distance, s, u) of the closest points p0 + s (p1 - p0), q0 + u (q1 - q0)."""
    a = [np.ascontiguousarray(v, np.float64) for v in (p0, p1, q0, q1)]
    s, u = C.c_double(), C.c_double()
    dist = lib().oracle_segment_closest(*[_ptr(v) for v in a], C.byref(s), C.byref(u))
    return dist, s.value, u.value


def detect_edges(model: Model, params, x, xt=None):
    """Edge-edge elements on positions x (normals from xt, default x):
    int32 [n, 4] vertex ids (first edge, second edge) and float64 [n, 3] normals."""
    x = np.ascontiguousarray(x, np.float64)
    xt = x if xt is None else np.ascontiguousarray(xt, np.float64)
    cap = 4 * max(1, model.surf_tris.shape[0])
    ov = np.zeros((cap, 4), np.int32); on = np.zeros((cap, 3))
    ps, keep = _params(params)
    n = lib().oracle_detect_edges(C.byref(model._s), C.byref(ps), _ptr(x), _ptr(xt), cap, _ptr(ov), _ptr(on))
    return ov[:n].copy(), on[:n].copy()


def edge_element(x4, n, k, delta, xt4=None, mu=0.0, eps_v=0.0, h=0.0):
    """(d, grad [4, 3]) of one edge-edge element at positions x4 [4, 3]; with
    xt4 (positions at the start of the step) its friction is included."""
    x4 = np.ascontiguousarray(x4, np.float64).reshape(12)
    nn = np.ascontiguousarray(n, np.float64)
    g = np.zeros(12)
    if xt4 is None:
        d = lib().oracle_edge_element(_ptr(x4), _ptr(nn), float(k), float(delta), _ptr(g))
    else:
        xt = np.ascontiguousarray(xt4, np.float64).reshape(12)
        d = lib().oracle_edge_element_friction(_ptr(x4), _ptr(xt), _ptr(nn), float(k), float(delta),
                                               float(mu), float(eps_v), float(h), _ptr(g))
    return d, g.reshape(4, 3)


def winding_number(model: Model, mesh, p, x):
    x = np.ascontiguousarray(x, np.float64)
    p = np.ascontiguousarray(p, np.float64)
    return lib().oracle_winding_number(C.byref(model._s), int(mesh), _ptr(p), _ptr(x))


def predict(model: Model, params, x, v):
    x = np.ascontiguousarray(x, np.float64); v = np.ascontiguousarray(v, np.float64)
    y = np.zeros_like(x)
    ps, keep = _params(params)
    lib().oracle_predict(C.byref(model._s), C.byref(ps), _ptr(x), _ptr(v), _ptr(y))
    return y


def energy_G(model: Model, params, x, y, tet_E, *, grad=False, hess=False):
    x = np.ascontiguousarray(x, np.float64); y = np.ascontiguousarray(y, np.float64)
    E = np.ascontiguousarray(tet_E, np.float64)
    n3 = 3 * model.n_verts
    g = np.zeros(n3) if grad else None
    H = np.zeros((n3, n3)) if hess else None
    ps, keep = _params(params)
    G = lib().oracle_energy_G(C.byref(model._s), C.byref(ps), _ptr(x), _ptr(y), _ptr(E),
                              _ptr(g), _ptr(H))
    out = [G]
    if grad:
        out.append(g)
    if hess:
        out.append(H)
    return out[0] if len(out) == 1 else tuple(out)


def step_backward(model: Model, params, x_t, v_t, v_prev, tet_E, gx_out, gv_out, gvp_out,
                  g_E=None):
    """Adjoint of one step.  Returns (gx_in, gv_in, gvp_in, g_E) with g_E accumulated."""
    arrs = [np.ascontiguousarray(a, np.float64) for a in (x_t, v_t, v_prev, tet_E, gx_out,
                                                           gv_out, gvp_out)]
    n3 = 3 * model.n_verts
    gx = np.zeros(n3); gv = np.zeros(n3); gvp = np.zeros(n3)
    gE = np.zeros(model.tets.shape[0]) if g_E is None else np.array(g_E, np.float64)
    ps, keep = _params(params)
    r = lib().oracle_step_backward(C.byref(model._s), C.byref(ps), *[_ptr(a) for a in arrs],
                                   _ptr(gx), _ptr(gv), _ptr(gvp), _ptr(gE))
    if r != 0:
        raise ValueError(f"oracle_step_backward failed ({r})")
    shp = np.shape(x_t)
    return gx.reshape(shp), gv.reshape(shp), gvp.reshape(shp), gE


def rollout(model: Model, params, x0, v0, tet_E, frames, vprev0=None):
    """Run ``frames`` steps; returns final (x, v, vprev) and the list of states."""
    x, v = np.array(x0, np.float64), np.array(v0, np.float64)
    vp = v.copy() if vprev0 is None else np.array(vprev0, np.float64)
    states = []
    for _ in range(frames):
        states.append((x.copy(), v.copy(), vp.copy()))
        x, v, vp, _ = step(model, params, x, v, vp, tet_E)
    return x, v, vp, states
