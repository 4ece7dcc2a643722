"""Host-side checks of the C ABI (no GPU needed): the library loads and exports
every symbol declared in include/vbd.h; topology preprocessing (coloring,
permutation, incidence CSR) is bit-exact against the oracle and brute force;
FP64 rest data and masses agree with the oracle; bad inputs give the
documented error codes."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import oracle as O
from paper_2403_06321_amd import _native as N
from paper_2403_06321_amd import workloads as W
from paper_2403_06321_amd.api import Topology

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    header = open(os.path.join(ROOT, "include", "vbd.h")).read()
    declared = set(re.findall(r"\b(vbd_[a-z_]+)\s*\(", header))
    assert declared == set(N.EXPORTS)
    lib = N.lib()
    for name in declared:
        assert hasattr(lib, name), name


def test_library_opens_marker_ranges():
    """The entry points open ROCTx ranges: the library depends on the ROCTx
    runtime and imports its range push and pop."""
    import subprocess
    so = N.lib()._name
    dyn = subprocess.run(["readelf", "-d", so], capture_output=True, text=True, check=True).stdout
    assert "librocprofiler-sdk-roctx" in dyn
    und = subprocess.run(["nm", "-D", "--undefined-only", so], capture_output=True, text=True, check=True).stdout
    assert "roctxRangePushA" in und and "roctxRangePop" in und


@pytest.mark.parametrize("n", [3, 5, 11])
def test_coloring_matches_oracle_bit_exact(n):
    w = W.tet_cube(n, n)
    t = Topology.from_workload(w, bind=False)
    m = O.Model.from_workload(w)
    assert t.n_colors == m.n_colors
    assert np.array_equal(t.query(N.Q_COLORS), m.colors)


@pytest.mark.parametrize("order", ["smallest_last", "dsatur"])
@pytest.mark.parametrize("make", [lambda: W.tet_cube(9, 1), lambda: W.config_cloth(32),
                                  lambda: W.config_batch(n_meshes=6, lo=3, hi=7)])
def test_ordered_coloring_matches_oracle_bit_exact(make, order):
    w = make()
    w.coloring = order
    t = Topology.from_workload(w, bind=False)
    m = O.Model.from_workload(w)
    assert t.n_colors == m.n_colors
    assert np.array_equal(t.query(N.Q_COLORS), m.colors)


def test_cloth_coloring_matches_oracle():
    w = W.config_cloth(32)
    t = Topology.from_workload(w, bind=False)
    m = O.Model.from_workload(w)
    assert np.array_equal(t.query(N.Q_COLORS), m.colors)
    assert t.n_colors == 7


def test_batch_coloring_equals_per_mesh_coloring():
    w = W.config_batch(n_meshes=6, lo=3, hi=6)
    t = Topology.from_workload(w, bind=False)
    colors = t.query(N.Q_COLORS)
    vo, to = w.offsets()
    for k in range(w.n_meshes):
        sub = W.subset_meshes(w, [k])
        m = O.Model.from_workload(sub)
        assert np.array_equal(colors[vo[k]:vo[k + 1]], m.colors)


def _expected_layout(w, colors):
    nv = w.n_verts
    pinned = w.pinned.astype(bool)
    free = np.flatnonzero(~pinned)
    perm = np.concatenate([free[np.lexsort((free, colors[free]))], np.flatnonzero(pinned)])
    iperm = np.empty(nv, np.int64); iperm[perm] = np.arange(nv)
    rows, ents = [0], []
    for v in perm:
        inc = [(t << 2) | int(np.flatnonzero(w.tets[t] == v)[0])
               for t in np.flatnonzero((w.tets == v).any(1))]
        ents.extend(sorted(inc))
        rows.append(len(ents))
    return perm, np.array(rows), np.array(ents)


def test_permutation_and_csr_bit_exact():
    w = W.tet_cube(4, 1)
    t = Topology.from_workload(w, bind=False)
    colors = O.Model.from_workload(w).colors
    perm, rows, ents = _expected_layout(w, colors)
    assert np.array_equal(t.query(N.Q_PERM), perm)
    assert np.array_equal(t.query(N.Q_TET_ROWS), rows)
    assert np.array_equal(t.query(N.Q_TET_ENTRIES), ents)
    co = t.query(N.Q_COLOR_OFFSETS)
    free_colors = colors[perm[:co[-1]]]
    assert np.array_equal(np.searchsorted(free_colors, np.arange(t.n_colors + 1)), co)


def test_spring_csr():
    w = W.config_cloth(8)
    t = Topology.from_workload(w, bind=False)
    perm = t.query(N.Q_PERM)
    rows = t.query(N.Q_SPRING_ROWS)
    nbrs = t.query(N.Q_SPRING_NBRS)
    for s, v in enumerate(perm[:len(rows) - 1]):
        exp = [int(b if a == v else a) for a, b in w.springs if a == v or b == v]
        assert nbrs[rows[s]:rows[s + 1]].tolist() == exp


def test_rest_data_and_masses_match_oracle():
    w = W.config_large_cube() if os.environ.get("VBD_BIG_HOST_TESTS") else W.tet_cube(9, 2)
    t = Topology.from_workload(w, bind=False)
    m = O.Model.from_workload(w)
    assert np.allclose(t.query(N.Q_MASS), m.mass, rtol=1e-13, atol=0)
    assert np.allclose(t.query(N.Q_VOLUME), m.vol, rtol=1e-13, atol=0)
    assert np.allclose(t.query(N.Q_DMINV).reshape(-1, 9), m.Dminv, rtol=0, atol=1e-11)


def _status(fn):
    try:
        fn()
    except N.VBDError as e:
        return e.status
    return 0


def test_error_codes():
    rest, tets = W.cube_lattice(2, 2, 2)
    bad = tets.copy(); bad[0, 0] = 99
    assert _status(lambda: Topology(rest, bad, bind=False)) == -2          # out of range
    rep = tets.copy(); rep[0, 1] = rep[0, 0]
    assert _status(lambda: Topology(rest, rep, bind=False)) == -2          # repeated vertex
    flat = rest.copy(); flat[:, 2] = 0.0
    assert _status(lambda: Topology(flat, tets, bind=False)) == -2         # degenerate rest tet
    assert _status(lambda: Topology(rest, tets, nu=0.5, bind=False)) == -1  # bad Poisson ratio
    # nu = 0 gives lambda = 0 and an infinite rest offset alpha = 1 + mu/lambda
    assert _status(lambda: Topology(rest, tets, nu=0.0, bind=False)) == -1
    assert _status(lambda: Topology(rest, tets, nu=-0.1, bind=False)) == -1
    with pytest.raises(ValueError):
        O.Model(rest, tets, np.zeros(len(rest), np.uint8), nu=0.0)
    sp = np.array([[0, 0]], np.int32)
    assert _status(lambda: Topology(rest, None, springs=sp, mass=np.ones(8), bind=False)) == -2
    assert _status(lambda: Topology(rest, None, springs=np.array([[0, 1]]), spring_rest=[0.0],
                                    mass=np.ones(8), bind=False)) == -2
    # masses: finite and >= 0; a massless free vertex is accepted (skipped while singular)
    spr = np.array([[0, 1]], np.int32)
    for bad_m in (-1.0, float("nan"), float("inf")):
        mm = np.ones(8); mm[3] = bad_m
        assert _status(lambda: Topology(rest, None, springs=spr, mass=mm, bind=False)) == -1
    mm = np.ones(8); mm[1] = 0.0
    assert _status(lambda: Topology(rest, None, springs=spr, mass=mm, bind=False)) == 0


def test_step_before_color_and_bind():
    L = N.lib()
    rest, tets = W.cube_lattice(2, 2, 2)
    rest = np.ascontiguousarray(rest); tets = np.ascontiguousarray(tets)
    desc = N.MeshDesc(8, tets.shape[0], 0, 1, None, None, tets.ctypes.data, None, rest.ctypes.data,
                      None, 0.0, None, 1000.0, 0.3, None)
    h = C.c_void_p()
    assert L.vbd_build_topology(C.byref(desc), C.byref(h)) == 0
    ps, _ = __import__("paper_2403_06321_amd.api", fromlist=["params_struct"]).params_struct(W.StepParams())
    assert L.vbd_step(h, C.byref(ps), None, None, None, None, None) == -3   # not colored
    sz = C.c_size_t()
    assert L.vbd_workspace_size(h, 0, C.byref(sz)) == -3
    assert L.vbd_color(h, None, None) == 0
    assert L.vbd_step(h, C.byref(ps), None, None, None, None, None) == -4   # no workspace
    assert L.vbd_workspace_size(h, 0, C.byref(sz)) == 0 and sz.value > 0
    assert b"vbd_bind_workspace" in L.vbd_last_error()
    assert L.vbd_topology_destroy(h) == 0


def test_size_limits_rejected():
    """More than 2^28 vertices or 2^29 tets is refused before any array is read
    (the solve addresses positions by 32-bit byte offsets)."""
    L = N.lib()
    rest, tets = W.cube_lattice(2, 2, 2)
    rest = np.ascontiguousarray(rest); tets = np.ascontiguousarray(tets)
    h = C.c_void_p()
    for nv, nt in (((1 << 28) + 1, tets.shape[0]), (8, (1 << 29) + 1)):
        desc = N.MeshDesc(nv, nt, 0, 1, None, None, tets.ctypes.data, None, rest.ctypes.data,
                          None, 0.0, None, 1000.0, 0.3, None)
        assert L.vbd_build_topology(C.byref(desc), C.byref(h)) == -1
        assert b"too many" in L.vbd_last_error()
        assert not h.value


def test_batched_offsets_validated():
    w = W.config_batch(n_meshes=3, lo=3, hi=4)
    vo = w.vert_offsets.copy(); vo[-1] += 1
    assert _status(lambda: Topology(w.rest, w.tets, vert_offsets=vo, tet_offsets=w.tet_offsets,
                                    bind=False)) == -1
    tets = w.tets.copy(); tets[0, 0] = w.vert_offsets[1]   # crosses into mesh 1
    assert _status(lambda: Topology(w.rest, tets, vert_offsets=w.vert_offsets,
                                    tet_offsets=w.tet_offsets, bind=False)) == -2


def test_phase_bytes_model():
    w = W.tet_cube(4, 0)
    t = Topology.from_workload(w, bind=False)
    pb = t.query(N.Q_PHASE_BYTES)
    rows = t.query(N.Q_TET_ROWS)
    co = t.query(N.Q_COLOR_OFFSETS)
    for c in range(t.n_colors):
        pairs = rows[co[c + 1]] - rows[co[c]]
        nvc = co[c + 1] - co[c]
        assert pb[c] >= 36 * pairs + 48 * nvc
        assert pb[c] <= 36 * pairs + 48 * nvc + 16 * w.n_verts


def test_phase_counts_and_adjoint_bytes_model():
    """Per color: tet pairs, spring entries, distinct neighbours (brute force
    over the tets) and free vertices; the reverse phase's bytes follow them."""
    w = W.tet_cube(5, 0)
    t = Topology.from_workload(w, bind=False)
    q = t.query(N.Q_PHASE_COUNTS).reshape(-1, 4)
    ab = t.query(N.Q_ADJ_PHASE_BYTES)
    colors = t.query(N.Q_COLORS)
    free = w.pinned == 0
    for c in range(t.n_colors):
        verts = np.flatnonzero((colors == c) & free)
        inc = [tt for tt in w.tets if np.any(np.isin(tt, verts))]
        nbrs = set()
        for tt in inc:
            nbrs.update(int(u) for u in tt if u not in set(verts.tolist()))
        assert q[c, 0] == len(inc) and q[c, 1] == 0 and q[c, 3] == len(verts)
        assert q[c, 2] == len(nbrs)
        assert ab[c] == 124 * q[c, 0] + 96 * q[c, 3] + 16 * q[c, 2]


def test_phase_bytes_follow_the_record_layout():
    """Compact pair records are 32 B, full ones 36 B; nothing else changes."""
    w = W.tet_cube(4, 0)
    t = Topology.from_workload(w, bind=False)
    pb0 = t.query(N.Q_PHASE_BYTES).copy()
    rows = t.query(N.Q_TET_ROWS)
    co = t.query(N.Q_COLOR_OFFSETS)
    t.launch_config = dict(compact_records=1)
    assert t.launch_config["compact_records"] == 1
    pb1 = t.query(N.Q_PHASE_BYTES)
    for c in range(t.n_colors):
        assert pb0[c] - pb1[c] == 4 * (rows[co[c + 1]] - rows[co[c]])
    t.launch_config = dict(compact_records=0)
    assert np.array_equal(t.query(N.Q_PHASE_BYTES), pb0)
    with pytest.raises(N.VBDError):
        t.launch_config = dict(compact_records=2)


def test_launch_config_lanes_validation():
    w = W.tet_cube(3, 0)
    t = Topology.from_workload(w, bind=False)
    for lanes in (2, 4, 8, 16, 32):
        t.launch_config = dict(lanes_per_vertex=lanes)
        assert t.launch_config["lanes_per_vertex"] == lanes
    for lanes in (1, 3, 64):
        with pytest.raises(N.VBDError):
            t.launch_config = dict(lanes_per_vertex=lanes)


def test_launch_config_remap_validation():
    w = W.tet_cube(3, 0)
    t = Topology.from_workload(w, bind=False)
    for rm in (0, 1, 2, 3):
        t.launch_config = dict(xcd_remap=rm)
        assert t.launch_config["xcd_remap"] == rm
    for rm in (-1, 4):
        with pytest.raises(N.VBDError):
            t.launch_config = dict(xcd_remap=rm)


def test_xcd_split_cuts_colors_at_mesh_boundaries():
    """Launch mapping 3: each color's slot range in 8 contiguous parts that
    cover it, cut at mesh boundaries where that keeps each part within 1/16 of
    the color's work of its target (work = vertices: each walks the color's
    padded degree), else inside a mesh at the target; a single mesh is cut
    into about equal parts."""
    w = W.config_batch(n_meshes=40, frames=1, coloring="smallest_last")
    t = Topology.from_workload(w, bind=False)
    xs = t.query(N.Q_XCD_SPLIT).reshape(-1, 9)
    co, perm, rows = t.query(N.Q_COLOR_OFFSETS), t.query(N.Q_PERM), t.query(N.Q_TET_ROWS)
    mesh = np.searchsorted(w.vert_offsets, perm, side="right") - 1
    for c in range(t.n_colors):
        b, e = co[c], co[c + 1]
        assert xs[c, 0] == b and xs[c, 8] == e and np.all(np.diff(xs[c]) >= 0)
        work = np.arange(e - b + 1, dtype=np.float64)
        for k in range(1, 8):
            cut = xs[c, k] - b
            target = work[-1] * k / 8
            at_boundary = cut in (0, e - b) or mesh[b + cut] != mesh[b + cut - 1]
            assert at_boundary or abs(work[cut] - target) <= 1.0
            if at_boundary:
                assert abs(work[cut] - target) <= work[-1] / 16 + 1e-9 or cut == 0 or cut == e - b
    # one mesh: cut at the work targets, each part within one vertex's work of
    # an eighth
    t1 = Topology.from_workload(W.tet_cube(9, 0), bind=False)
    xs1 = t1.query(N.Q_XCD_SPLIT).reshape(-1, 9)
    co1, rows1 = t1.query(N.Q_COLOR_OFFSETS), t1.query(N.Q_TET_ROWS)
    for c in range(t1.n_colors):
        parts = np.diff(xs1[c])
        assert np.abs(parts - (co1[c + 1] - co1[c]) / 8).max() <= 1.0


def test_tet_order_groups_tets_by_vertex_colors():
    w = W.tet_cube(7, 2)
    t = Topology.from_workload(w, bind=False)
    order = t.query(N.Q_TET_ORDER)
    assert np.array_equal(np.sort(order), np.arange(w.n_tets))
    colors = t.query(N.Q_COLORS)
    keys = [tuple(sorted(colors[w.tets[o]])) for o in order]
    assert keys == sorted(keys)


def test_rest_frame_preserves_deformation_invariants():
    """F' = D_s R^{-1} = F Q (Q a proper rotation) must keep F F^T, tr(F^T F)
    and det F of F = D_s D_m^{-1}: the invariants the energy depends on."""
    w = W.tet_cube(4, 3)
    t = Topology.from_workload(w, bind=False)
    S6 = t.query(N.Q_REST_FRAME).reshape(-1, 6)
    Dminv = t.query(N.Q_DMINV).reshape(-1, 3, 3)
    rng = np.random.default_rng(0)
    x = w.rest + rng.normal(scale=0.02, size=w.rest.shape)
    for k in rng.choice(w.n_tets, 50, replace=False):
        S = np.array([[S6[k, 0], S6[k, 1], S6[k, 2]], [0, S6[k, 3], S6[k, 4]], [0, 0, S6[k, 5]]])
        q = w.tets[k]
        Ds = (x[q[1:]] - x[q[0]]).T
        F, Fp = Ds @ Dminv[k], Ds @ S
        assert np.allclose(Fp @ Fp.T, F @ F.T, rtol=1e-12, atol=1e-12)
        assert np.trace(Fp.T @ Fp) == pytest.approx(np.trace(F.T @ F), rel=1e-12)
        Q = np.linalg.solve(F, Fp)
        assert np.allclose(Q.T @ Q, np.eye(3), atol=1e-10)
        assert np.linalg.det(Fp) == pytest.approx(np.linalg.det(F), rel=1e-12)


def test_pair_frame_identities():
    """The identities the color solve and its reverse rest on, checked on the
    library's rest frames (vertex in slot 0 as origin) against full matrix
    algebra with F = D_s D_m^{-1}: with the rows s_k of S, m = -(s0 + s1 + s2),
    w = S m and sigma = det S,
      sum_k w_k = -|m|^2,   F m = sum_k w_k e_k,
      cof(F) m = -sigma (x_b - x_a) x (x_c - x_a),   J = e1 . sigma (x_b - x_a) x (x_c - x_a),
    and the gradient of (cof(F) m) . w with respect to x_a, x_b, x_c."""
    w_ = W.tet_cube(4, 3)
    t = Topology.from_workload(w_, bind=False)
    S6 = t.query(N.Q_REST_FRAME).reshape(-1, 6)
    Dminv = t.query(N.Q_DMINV).reshape(-1, 3, 3)
    rng = np.random.default_rng(1)
    x = w_.rest + rng.normal(scale=0.02, size=w_.rest.shape)
    for k in rng.choice(w_.n_tets, 40, replace=False):
        S = np.array([[S6[k, 0], S6[k, 1], S6[k, 2]], [0, S6[k, 3], S6[k, 4]], [0, 0, S6[k, 5]]])
        m = -S.sum(axis=0)
        wv = S @ m
        sig = np.linalg.det(S)
        assert wv.sum() == pytest.approx(-m @ m, rel=1e-12)
        q = w_.tets[k]
        xi, xa, xb, xc = x[q]
        e = np.stack([xa - xi, xb - xi, xc - xi], 1)
        F = e @ Dminv[k]
        # shape gradient of slot 0 for F = D_s D_m^{-1}
        m_true = -Dminv[k].sum(axis=0)
        cof = np.linalg.det(F) * np.linalg.inv(F).T
        n = sig * np.cross(xb - xa, xc - xa)
        # F' = F Q and m = Q^T m_true, so F' m = F m_true
        assert np.allclose(e @ wv, F @ m_true, rtol=1e-10, atol=1e-12)
        assert np.allclose(-n, cof @ m_true, rtol=1e-9, atol=1e-12)
        assert e[:, 0] @ n == pytest.approx(np.linalg.det(F), rel=1e-10)
        # d(n . u)/dx_q by central differences for a random u
        u = rng.normal(size=3)
        g = [sig * np.cross(u, xc - xb), sig * np.cross(xc - xa, u), sig * np.cross(u, xb - xa)]
        for j, idx in enumerate((1, 2, 3)):
            for d in range(3):
                h = 1e-6
                xp, xm = x[q].copy(), x[q].copy()
                xp[idx, d] += h
                xm[idx, d] -= h
                fp = sig * np.cross(xp[2] - xp[1], xp[3] - xp[1]) @ u
                fm = sig * np.cross(xm[2] - xm[1], xm[3] - xm[1]) @ u
                assert (fp - fm) / (2 * h) == pytest.approx(g[j][d], rel=1e-6, abs=1e-6 * abs(sig))


def test_surface_matches_oracle_with_outward_orientation():
    """The library's surface (extracted for batched topologies) is the
    oracle's set of boundary faces, each with the same outward orientation."""
    w = W.config_block_stack(cols=2, levels=2, n=4)
    t = Topology.from_workload(w, bind=False)
    surf = t.query(N.Q_SURFACE)
    n_tri, n_sv, n_edge = t.query(N.Q_SURFACE_COUNTS)
    m = O.Model.from_workload(w)
    assert n_tri == surf.shape[0] == m.surf_tris.shape[0] == w.n_meshes * 2 * 6 * 3 ** 2
    assert n_sv == np.unique(surf).size
    rot = {}
    for tri in m.surf_tris:
        k = int(np.argmin(tri))
        rot[tuple(np.roll(tri, -k))] = True
    for tri in surf:
        k = int(np.argmin(tri))
        assert tuple(np.roll(tri, -k)) in rot
    # surface edges: the distinct edges of the surface triangles, ascending
    edges = t.query(N.Q_SURFACE_EDGES)
    ref = np.unique(np.sort(np.concatenate([surf[:, [0, 1]], surf[:, [1, 2]], surf[:, [2, 0]]]), axis=1),
                    axis=0)
    assert n_edge == edges.shape[0] and np.array_equal(edges, ref)
    # a single mesh has its surface too (self-contact); springs alone have none
    w1 = W.tet_cube(4, 0)
    t1 = Topology.from_workload(w1, bind=False)
    n_f = 2 * 6 * 3 ** 2                       # closed surface: E = 3F/2, V = E - F + 2
    assert tuple(t1.query(N.Q_SURFACE_COUNTS)) == (n_f, n_f // 2 + 2, 3 * n_f // 2)
    t2 = Topology.from_workload(W.spring_net(n=4), bind=False)
    assert tuple(t2.query(N.Q_SURFACE_COUNTS)) == (0, 0, 0)


def test_given_coloring_layout_and_validation():
    w = W.tet_cube(5, 2)
    colors = W.lattice_colors(5, 5, 5)
    t = Topology.from_workload(w, bind=False, colors=colors)
    assert t.n_colors == 4
    assert np.array_equal(t.query(N.Q_COLORS), colors)
    perm, rows, ents = _expected_layout(w, colors)
    assert np.array_equal(t.query(N.Q_PERM), perm)
    assert np.array_equal(t.query(N.Q_TET_ROWS), rows)
    assert np.array_equal(t.query(N.Q_TET_ENTRIES), ents)
    bad = colors.copy()
    q = w.tets[17]
    bad[q[1]] = bad[q[0]]
    assert _status(lambda: Topology.from_workload(w, bind=False, colors=bad)) == -1
    neg = colors.copy(); neg[3] = -1
    assert _status(lambda: Topology.from_workload(w, bind=False, colors=neg)) == -1


def test_coloring_order_errors():
    L = N.lib()
    w = W.tet_cube(3, 0)
    t = Topology.from_workload(w, bind=False)
    nc = C.c_int32()
    assert L.vbd_color_greedy(t._h, 7, C.byref(nc), None) == -1
    assert b"order" in L.vbd_last_error()
    # switching the order before binding recolors
    assert L.vbd_color_greedy(t._h, N.COLOR_SMALLEST_LAST, C.byref(nc), None) == 0 and nc.value == 4
    assert L.vbd_color_greedy(t._h, N.COLOR_DSATUR, C.byref(nc), None) == 0 and nc.value == 4
    assert L.vbd_color_greedy(t._h, N.COLOR_ID_ORDER, C.byref(nc), None) == 0
    assert nc.value == O.color_greedy(w.n_verts, w.tets)[1]
    assert np.array_equal(t.query(N.Q_COLORS), O.color_greedy(w.n_verts, w.tets)[0])


@pytest.mark.parametrize("n", [4, 7])
def test_dsatur_on_crown_graph_matches_oracle(n):
    """Bipartite crown graph with interleaved ids: 2 colors for DSATUR, n for
    first fit in id order, on both sides."""
    sp = np.array([[2 * i, 2 * j + 1] for i in range(n) for j in range(n) if i != j], np.int32)
    rest = np.zeros((2 * n, 3))
    rest[:, 0] = np.arange(2 * n)
    for order, expect in (("dsatur", 2), ("id", n)):
        t = Topology(rest, None, springs=sp, mass=np.ones(2 * n), coloring=order, bind=False)
        c, nc = O.color_greedy(2 * n, np.zeros((0, 4)), sp, order=order)
        assert t.n_colors == nc == expect
        assert np.array_equal(t.query(N.Q_COLORS), c)
