"""Pins of the oracle's mesh-mesh contacts (Sec. 3.5, 3.9): vertex-triangle
and edge-edge elements, between meshes and within one mesh."""
import dataclasses

import numpy as np
import pytest

import oracle as O
from paper_2403_06321_amd import workloads as W


def P(**kw):
    return dataclasses.replace(W.StepParams(), **kw)


@pytest.mark.parametrize("n", [3, 4, 6])
def test_surface_is_closed_and_encloses_the_volume(n):
    """Divergence theorem: V = 1/3 sum_T (c_T . n_T) A_T, sum_T n_T A_T = 0."""
    rest, tets = W.cube_lattice(n, n, n)
    tris = O.surface(tets, rest)
    assert tris.shape[0] == 2 * 6 * (n - 1) ** 2
    a, b, c = rest[tris[:, 0]], rest[tris[:, 1]], rest[tris[:, 2]]
    nA = 0.5 * np.cross(b - a, c - a)              # area-weighted outward normals
    cen = (a + b + c) / 3.0
    assert np.abs(nA.sum(0)).max() < 1e-12
    vol = (cen * nA).sum() / 3.0
    assert vol == pytest.approx((n - 1) ** 3 * W.EDGE ** 3, rel=1e-12)
    # every edge of a closed surface is shared by exactly two triangles
    edges = np.sort(np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]]), axis=1)
    _, counts = np.unique(edges, axis=0, return_counts=True)
    assert np.all(counts == 2)


def test_closest_point_matches_dense_sampling():
    rng = np.random.default_rng(0)
    s = np.linspace(0.0, 1.0, 401)
    u, v = np.meshgrid(s, s)
    keep = (u + v) <= 1.0
    u, v = u[keep], v[keep]
    for _ in range(40):
        a, b, c = rng.normal(size=(3, 3))
        p = rng.normal(size=3) * 2.0
        q, bary = O.closest_point_triangle(p, a, b, c)
        assert np.allclose(bary.sum(), 1.0) and np.all(bary >= -1e-12)
        assert np.allclose(q, bary[0] * a + bary[1] * b + bary[2] * c)
        pts = a + u[:, None] * (b - a) + v[:, None] * (c - a)
        dmin = np.linalg.norm(pts - p, axis=1).min()
        d = np.linalg.norm(q - p)
        assert d <= dmin + 1e-12
        assert d >= dmin - 5e-3 * np.linalg.norm(np.cross(b - a, c - a)) ** 0.5


def _two_blocks(dx=0.033, dy=0.041, gap=-0.003, n=4, pin_lower=True, E=1e5):
    """Lower block (mesh 0) and an upper block (mesh 1) whose bottom face lies
    `gap` above the lower block's top face, shifted by (dx, dy)."""
    r0, t0 = W.cube_lattice(n, n, n)
    r1, t1 = W.cube_lattice(n, n, n)
    top = r0[:, 2].max()
    r1 = r1 + np.array([dx, dy, top + gap])
    rest = np.concatenate([r0, r1])
    tets = np.concatenate([t0, t1 + r0.shape[0]]).astype(np.int32)
    pinned = np.zeros(rest.shape[0], np.uint8)
    if pin_lower:
        pinned[:r0.shape[0]] = 1
    vo = np.array([0, r0.shape[0], rest.shape[0]])
    return rest, tets, pinned, vo, np.full(tets.shape[0], E)


def _box(x):
    return x.min(0), x.max(0)


def _box_distance(p, lo, hi):
    """Distance from p to the boundary of the box [lo, hi] and whether p is inside."""
    inside = np.all((p > lo) & (p < hi), axis=-1)
    out = np.linalg.norm(np.maximum(np.maximum(lo - p, p - hi), 0.0), axis=-1)
    depth = np.minimum(p - lo, hi - p).min(-1)
    return np.where(inside, depth, out), inside


def test_winding_number_is_one_inside_and_zero_outside():
    rest, tets, pinned, vo, E = _two_blocks()
    m = O.Model(rest, tets, pinned, vert_offsets=vo)
    rng = np.random.default_rng(2)
    # a rigid motion changes nothing
    A = np.linalg.qr(rng.normal(size=(3, 3)))[0]
    A *= np.sign(np.linalg.det(A))
    x = rest @ A.T + np.array([0.3, -0.2, 0.1])
    for mesh in (0, 1):
        lo, hi = _box(rest[vo[mesh]:vo[mesh + 1]])
        pts = rng.uniform(lo - 0.1, hi + 0.1, size=(200, 3))
        d, inside = _box_distance(pts, lo, hi)
        keep = d > 1e-6
        for q, ins in zip(pts[keep], inside[keep]):
            w = O.winding_number(m, mesh, q @ A.T + np.array([0.3, -0.2, 0.1]), x)
            assert w == pytest.approx(1.0 if ins else 0.0, abs=1e-9)


def test_detection_matches_brute_force_on_boxes():
    """Both blocks are axis-aligned boxes at rest, so penetration and distance
    to the other block have closed forms: the detected set is exactly the
    surface vertices inside the other box or closer than the thickness."""
    rest, tets, pinned, vo, E = _two_blocks()
    m = O.Model(rest, tets, pinned, vert_offsets=vo)
    delta = 1e-3
    p = P(mesh_contacts=True, collision_radius=0.05, contact_thickness=delta)
    tri = O.detect_contacts(m, p, rest)
    surf = m.surf_tris
    on_surf = np.zeros(rest.shape[0], bool); on_surf[surf.ravel()] = True
    boxes = [_box(rest[vo[k]:vo[k + 1]]) for k in (0, 1)]
    for v in range(rest.shape[0]):
        other = 1 - m.vert_mesh[v]
        d, inside = _box_distance(rest[v], *boxes[other])
        expect = on_surf[v] and (inside or d < delta)
        assert (tri[v] >= 0) == expect, v
        if expect:
            T = surf[tri[v]]
            assert np.all(m.vert_mesh[T] == other)
            q, _ = O.closest_point_triangle(rest[v], *rest[T])
            assert np.linalg.norm(q - rest[v]) == pytest.approx(d, abs=1e-12)
    hit = np.flatnonzero(tri >= 0)
    assert set(m.vert_mesh[hit]) == {0, 1}


def test_vertex_on_triangle_interior_equals_plane_contact():
    """A free vertex pressing into the interior of a pinned mesh's top face
    behaves exactly like the analytic plane through that face (same penalty,
    same friction): the upper block hovers 1 cm above the lower one and only
    one of its bottom vertices, dipped 2 mm into the lower block, is free."""
    rest, tets, pinned, vo, E = _two_blocks(gap=0.01)
    pinned[:] = 1
    upper = np.arange(vo[1], vo[2])
    bottom = upper[np.abs(rest[upper, 2] - rest[upper, 2].min()) < 1e-9]
    v = bottom[len(bottom) // 2]
    pinned[v] = 0
    top = rest[:vo[1], 2].max()
    x0 = rest.copy()
    x0[v, 2] = top - 0.002
    m = O.Model(rest, tets, pinned, vert_offsets=vo)
    # friction in the sliding regime, and slow enough to stick (the static
    # branch of Eq. IPC_friction, |u| < h eps_v, which the plane contact's
    # closed-form pin fixes)
    for mu, tang in ((0.0, (0.05, -0.02)), (0.4, (0.05, -0.02)), (0.4, (0.004, -0.002))):
        base = dict(n_iters=5, contact_k=1e4, contact_thickness=1e-3, init_mode=W.INIT_PREV,
                    friction_mu=mu, friction_eps_v=1e-2)
        pm = P(mesh_contacts=True, collision_radius=0.05, **base)
        pp = P(planes=np.array([[0.0, 0.0, 1.0, top]]), **base)
        tri = O.detect_contacts(m, pm, x0)
        assert np.flatnonzero(tri >= 0).tolist() == [v]
        vel = np.zeros_like(rest); vel[v] = [tang[0], tang[1], -0.1]
        xm, vm, _, stm = O.step(m, pm, x0, vel, vel, E)
        xp, vp, _, stp = O.step(m, pp, x0, vel, vel, E)
        assert stm["n_contacts"] > 0 and stm["n_contacts"] == stp["n_contacts"]
        assert np.allclose(xm, xp, rtol=0, atol=1e-13)
        assert xm[v, 2] > x0[v, 2]
        slide = np.linalg.norm(xm[v, :2] - x0[v, :2])
        if tang[0] < 0.01:
            assert 0.0 < slide < pm.h * pm.friction_eps_v      # stuck: static branch
        elif mu > 0:
            assert slide > pm.h * pm.friction_eps_v            # sliding branch


def test_contact_forces_conserve_momentum_at_convergence():
    """Two free blocks in contact, no gravity, no pins: the converged implicit
    Euler step conserves linear momentum (contact gradients sum to zero over
    the four vertices of an element)."""
    rest, tets, pinned, vo, E = _two_blocks(gap=-0.002, pin_lower=False)
    m = O.Model(rest, tets, pinned, vert_offsets=vo)
    p = P(n_iters=3000, gravity=(0.0, 0.0, 0.0), mesh_contacts=True, collision_radius=0.05,
          contact_k=1e4, contact_thickness=1e-3)
    v0 = np.zeros_like(rest)
    v0[vo[1]:] = [0.0, 0.0, -0.3]
    x, v, _, st = O.step(m, p, rest, v0, v0, E)
    assert st["n_contacts"] > 0
    P0 = (m.mass[:, None] * v0).sum(0)
    P1 = (m.mass[:, None] * v).sum(0)
    assert np.abs(P1 - P0).max() <= 1e-8 * np.abs(m.mass[:, None] * v0).sum()
    # the contact pushed the blocks apart relative to free flight
    assert v[vo[1]:, 2].mean() > -0.3


# ---------------------------------------------------------------- edge-edge --
def test_segment_closest_points_match_dense_sampling():
    """Closest points of two segments: the distance equals the minimum over a
    dense grid of (s, u) up to the grid's resolution, never exceeds it, and the
    returned parameters attain it; includes nearly parallel pairs and pairs
    whose minimum lies at an end point."""
    rng = np.random.default_rng(1)
    g = np.linspace(0.0, 1.0, 801)
    for trial in range(60):
        p0, p1, q0, q1 = rng.normal(size=(4, 3))
        if trial % 3 == 1:                               # nearly parallel
            q1 = q0 + (p1 - p0) * 0.7 + rng.normal(size=3) * 1e-6
        if trial % 3 == 2:                               # far apart: end points win
            q0, q1 = q0 + 5.0, q1 + 5.0
        d, s, u = O.segment_closest(p0, p1, q0, q1)
        P_ = p0 + g[:, None] * (p1 - p0)
        Q_ = q0 + g[:, None] * (q1 - q0)
        D = np.linalg.norm(P_[:, None] - Q_[None], axis=2)
        assert d <= D.min() + 1e-12
        step = np.linalg.norm(p1 - p0) + np.linalg.norm(q1 - q0)
        assert D.min() - d <= step * (g[1] - g[0])
        assert 0.0 <= s <= 1.0 and 0.0 <= u <= 1.0
        assert np.linalg.norm(p0 + s * (p1 - p0) - q0 - u * (q1 - q0)) == pytest.approx(d, abs=1e-12)


def test_edge_element_gradient_and_momentum():
    """One edge-edge element: the analytic gradient equals central differences
    of E = k/2 d^2, d = delta - (x_a - x_b).n with the closest-point
    parameters and n held fixed (as Sec. 3.5 holds the normal), the four
    vertex forces sum to zero, and an element with d <= 0 exerts nothing."""
    rng = np.random.default_rng(2)
    k, delta = 1e4, 5e-3
    for _ in range(20):
        x = np.array([[-0.1, 0.0, 0.0], [0.1, 0.0, 0.0], [0.0, -0.1, 0.002], [0.0, 0.1, 0.002]])
        x = x + rng.normal(size=x.shape) * np.array([0.01, 0.01, 5e-4])
        n = np.array([0.0, 0.0, -1.0])
        d, grad = O.edge_element(x, n, k, delta)
        dd, s, u = O.segment_closest(*x)
        assert 0.0 < s < 1.0 and 0.0 < u < 1.0
        assert d > 0.0

        def energy(y):
            xa = y[0] + s * (y[1] - y[0])
            xb = y[2] + u * (y[3] - y[2])
            return 0.5 * k * max(0.0, delta - (xa - xb) @ n) ** 2
        fd = np.zeros_like(x)
        h = 1e-7
        for i in range(4):
            for a in range(3):
                e = np.zeros_like(x)
                e[i, a] = h
                fd[i, a] = (energy(x + e) - energy(x - e)) / (2 * h)
        assert np.abs(grad - fd).max() <= 1e-5 * np.abs(fd).max()
        assert np.abs(grad.sum(0)).max() <= 1e-12 * np.abs(grad).max()
    x[2:, 2] += 0.05                                      # separated by more than delta
    d, grad = O.edge_element(x, n, k, delta)
    assert d < 0.0 and not grad.any()


def test_edge_friction_is_the_gradient_of_the_smoothed_friction_potential():
    """Friction of one edge-edge element (Sec. 3.6, Eq. IPC_friction), with the
    contact force lambda = k d, the closest-point parameters and n held fixed:
    the friction forces on the four vertices are minus the gradient of
    mu lambda f0(|u|), u the tangential part of (x_a - x_a^t) - (x_b - x_b^t)
    and f0 the antiderivative of f1 (f0(y) = y above h eps_v and
    -y^3 / (3 (h eps_v)^2) + y^2 / (h eps_v) + h eps_v / 3 below), checked by
    central differences of that potential in the static and the sliding
    regime; with the penalty, the four forces sum to zero."""
    rng = np.random.default_rng(5)
    k, delta, mu, eps_v, h = 1e4, 5e-3, 0.3, 1e-2, 1.0 / 60.0
    ev = h * eps_v

    def f0(y):
        return y if y >= ev else -y ** 3 / (3 * ev ** 2) + y ** 2 / ev + ev / 3

    for scale, regime in ((2e-5, "static"), (2e-3, "sliding")):
        for _ in range(10):
            x = np.array([[-0.1, 0.0, 0.0], [0.1, 0.0, 0.0], [0.0, -0.1, 0.002], [0.0, 0.1, 0.002]])
            x = x + rng.normal(size=x.shape) * np.array([0.01, 0.01, 5e-4])
            n = np.array([0.0, 0.0, -1.0])
            disp = rng.normal(size=x.shape) * np.array([scale, scale, 0.1 * scale])
            xt = x - disp
            d, g_all = O.edge_element(x, n, k, delta, xt, mu, eps_v, h)
            _, g_pen = O.edge_element(x, n, k, delta)
            assert d > 0.0
            _, s, u = O.segment_closest(*x)
            lam = k * d
            w = np.array([1.0 - s, s, -(1.0 - u), -u])   # weights of x_a - x_b

            def potential(y):
                dx = w @ (y - xt)
                ut = dx - (dx @ n) * n
                return mu * lam * f0(np.linalg.norm(ut))
            ut0 = w @ disp
            ut0 = ut0 - (ut0 @ n) * n
            assert (np.linalg.norm(ut0) < ev) == (regime == "static")
            fd = np.zeros_like(x)
            step = 1e-9 if regime == "static" else 1e-7
            for i in range(4):
                for a in range(3):
                    e = np.zeros_like(x)
                    e[i, a] = step
                    fd[i, a] = (potential(x + e) - potential(x - e)) / (2 * step)
            g_fric = g_all - g_pen
            assert np.abs(g_fric - fd).max() <= 1e-5 * np.abs(fd).max(), regime
            assert np.abs(g_all.sum(0)).max() <= 1e-12 * np.abs(g_all).max()


def test_crossed_bars_detect_one_edge_element():
    """Two cubes crossed edge on edge: at rest the detection finds exactly one
    edge-edge element, between the middle segments of the two edges, with the
    normal -z (from the upper edge's contact point to the lower one's) and
    d = delta - gap; no vertex-triangle contact; nothing when edge contacts
    are off or the gap exceeds delta."""
    w = W.config_crossed_bars()
    m = O.Model.from_workload(w)
    ev, en = O.detect_edges(m, w.params, w.x0)
    assert ev.shape == (1, 4)
    lower, upper = ev[0, :2], ev[0, 2:]
    nl = int(w.vert_offsets[1])
    assert np.all(lower < nl) and np.all(upper >= nl)
    for seg in (lower, upper):                            # the middle segment of each edge
        mid = w.x0[seg].mean(0)
        assert np.hypot(mid[0], mid[1]) < 1e-9
    np.testing.assert_allclose(en[0], [0.0, 0.0, -1.0], atol=1e-12)
    d, _ = O.edge_element(w.x0[ev[0]], en[0], w.params.contact_k, w.params.contact_thickness)
    assert d == pytest.approx(w.params.contact_thickness - 2.5e-3, abs=1e-12)
    assert not np.any(O.detect_contacts(m, w.params, w.x0) >= 0)
    off = dataclasses.replace(w.params, edge_contacts=False)
    x, _, _, st = O.step(m, dataclasses.replace(off, n_iters=2), w.x0, w.v0, w.v0, w.tet_E)
    assert st["n_contacts"] == 0
    far = w.x0.copy()
    far[nl:, 2] += 0.01
    assert O.detect_edges(m, w.params, far)[0].shape[0] == 0


def test_crossed_bars_edge_contact_balances_the_weight():
    """Static equilibrium: steps started from rest (v = v_prev = 0 each time)
    are implicit gradient steps of the potential and converge to the static
    state, where the upper cube hangs on the single edge-edge element, whose
    force k_c d equals the upper cube's weight (the element's forces on the
    upper edge sum to k_c d, pointing up)."""
    w = W.config_crossed_bars(frames=1)
    p = dataclasses.replace(w.params, n_iters=60)
    m = O.Model.from_workload(w)
    O.set_threads(4)
    x, z = w.x0, np.zeros_like(w.x0)
    for _ in range(60):
        x, _, _, _ = O.step(m, p, x, z, z, w.tet_E)
    nl = int(w.vert_offsets[1])
    ev, en = O.detect_edges(m, p, x)
    assert ev.shape[0] == 1
    d, grad = O.edge_element(x[ev[0]], en[0], p.contact_k, p.contact_thickness)
    weight = m.mass[nl:].sum() * 9.8
    assert p.contact_k * d == pytest.approx(weight, rel=1e-3)
    np.testing.assert_allclose(-grad[2:].sum(0), [0.0, 0.0, p.contact_k * d], atol=1e-3 * weight)


def test_edge_contacts_conserve_momentum_at_convergence():
    """The crossed cubes free (no pins, no gravity), the upper one moving down
    into the lower: the converged step conserves linear momentum, and only
    edge-edge elements act."""
    w = W.config_crossed_bars()
    m = O.Model(w.rest, w.tets, np.zeros(w.n_verts, np.uint8), density=w.density,
                vert_offsets=w.vert_offsets)
    nl = int(w.vert_offsets[1])
    p = dataclasses.replace(w.params, n_iters=8000, gravity=(0.0, 0.0, 0.0))
    v0 = np.zeros_like(w.x0)
    v0[nl:] = [0.0, 0.0, -0.3]
    O.set_threads(4)
    x, v, _, st = O.step(m, p, w.x0, v0, v0, w.tet_E)
    assert st["n_contacts"] > 0
    assert not np.any(O.detect_contacts(m, p, w.x0) >= 0)
    P0 = (m.mass[:, None] * v0).sum(0)
    P1 = (m.mass[:, None] * v).sum(0)
    # the free cubes' rigid modes converge slowly: 8000 sweeps reach 1e-8
    assert np.abs(P1 - P0).max() <= 1e-7 * np.abs(m.mass[:, None] * v0).sum()
    assert v[nl:, 2].mean() > -0.3 and v[:nl, 2].mean() < 0.0


# ------------------------------------------------------------- self-contact --
def test_self_contact_detection_on_the_folding_c():
    """One C-shaped mesh: nothing at rest (the slabs are a gap apart, farther
    than the detection radius); with the upper slab lowered onto the lower
    one, its bottom vertices find lower-slab triangles of the same mesh and
    edge-edge pairs appear, but only with self-contact on; triangles that
    share a vertex or lie within the exclusion distance at rest are never
    taken (the wall's faces next to the slabs)."""
    w = W.config_folding_c()
    m = O.Model.from_workload(w)
    p = w.params
    assert not np.any(O.detect_contacts(m, p, w.x0) >= 0)
    x = w.x0.copy()
    up = w.rest[:, 2] > 1.5 * W.EDGE
    free_slab = up & (w.rest[:, 0] > 1.5 * W.EDGE)
    x[free_slab, 2] -= W.EDGE - 0.5 * p.contact_thickness
    tri = O.detect_contacts(m, p, x)
    hits = np.flatnonzero(tri >= 0)
    assert hits.size > 0
    # the facing faces find each other: upper-slab bottom vertices (rest z =
    # 2 cells) take lower-slab top triangles (rest z = 1 cell) and vice versa
    for v_ in hits:
        T = m.surf_tris[tri[v_]]
        assert v_ not in T
        zv, zT = round(w.rest[v_, 2] / W.EDGE), np.round(w.rest[T, 2] / W.EDGE)
        assert w.rest[v_, 0] > 0.5 * W.EDGE
        if zv == 2:      # upper slab bottom: a lower-slab triangle (top face or its edges)
            assert zT.max() == 1
        else:            # lower slab top: an upper-slab triangle
            assert zv == 1 and zT.min() == 2
    # the lowered faces are parallel lattices: their edge pairs are parallel
    # or meet at end points, which vertex-triangle elements cover
    assert O.detect_edges(m, p, x, w.x0)[0].shape[0] == 0
    off = dataclasses.replace(p, self_contact=False)
    assert not np.any(O.detect_contacts(m, off, x) >= 0)
    wide = dataclasses.replace(p, self_exclusion=2 * W.EDGE)
    assert not np.any(O.detect_contacts(m, wide, x) >= 0)


def test_folding_c_self_contact_stops_the_slab():
    """The sagging upper slab of the C: with self-contact, vertex-triangle and
    edge-edge elements of the one mesh appear (the slab's tip tilts, so its
    edges cross the lower slab's) and keep the slabs apart; without it, the
    upper slab falls through the lower one."""
    w = W.config_folding_c(frames=12)
    m = O.Model.from_workload(w)
    O.set_threads(4)
    upper_bottom = (np.abs(w.rest[:, 2] - 2 * W.EDGE) < 1e-9) & (w.rest[:, 0] > 1.5 * W.EDGE)
    lower_top = (np.abs(w.rest[:, 2] - W.EDGE) < 1e-9) & (w.rest[:, 0] > 1.5 * W.EDGE)
    for self_on in (True, False):
        p = dataclasses.replace(w.params, self_contact=self_on)
        x, v, vp = w.x0, w.v0, w.v0
        n_vt = n_ee = 0
        lowest = np.inf
        for _ in range(w.frames):
            xt = x
            x, v, vp, _ = O.step(m, p, x, v, vp, w.tet_E)
            n_vt += int((O.detect_contacts(m, p, x) >= 0).sum())
            n_ee += O.detect_edges(m, p, x, xt)[0].shape[0]
            lowest = min(lowest, x[upper_bottom, 2].min())
        if self_on:
            assert n_vt > 0 and n_ee > 0
            assert lowest > 0.5 * W.EDGE     # the impact dents less than half a cell
        else:
            assert n_vt == 0 and n_ee == 0
            assert lowest < 0.0              # through the lower slab
