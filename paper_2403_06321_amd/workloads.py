"""Seeded synthetic workloads for the VBD hot path.

This module only builds inputs: lattice and cloth topologies, rest shapes,
pins, jittered initial positions, velocities and per-tet Young's moduli, all
drawn from ``numpy.random.default_rng(seed)``.  It contains none of the
solver's arithmetic (no rest-shape inverses, masses, greedy colorings, forces
or Hessians); both the FP64 oracle and the HIP library consume what it
returns.  The one coloring built here, ``lattice_colors``, is an input: a
caller-supplied coloring handed to both sides as is.

Workload shapes follow the paper's setting (Sec. 5: fixed frame time 1/60 s,
fixed iteration count, stable Neo-Hookean tets, linear springs for mass-spring
systems, penalty contact of Sec. 3.5).  The paper's meshes are not available,
so Kuhn-split lattice cubes and a grid cloth stand in for them.

Conventions
-----------
* Lattice vertex id ``i + nx*(j + ny*k)``; cell edge 0.1 m; x and y centred on
  0, bottom face at z = 0.
* Each cell is split into 6 tets along its (0,0,0)->(1,1,1) diagonal: for the
  6 axis permutations in lexicographic order, ``v0`` is the cell corner and
  ``v[r+1] = v[r] + e[perm[r]]``; a tet with negative signed volume has
  ``v2`` and ``v3`` swapped.  Tet id = 6*cell + permutation index.
* Draw order for a seed: mesh dims / per-mesh E, per-tet E, jitter (vertex-id
  order, x,y,z), initial velocity, target point.
"""
from __future__ import annotations

import dataclasses
import itertools
from typing import List, Optional, Tuple

import numpy as np

EDGE = 0.1          # lattice cell edge [m]
DENSITY = 1000.0    # kg / m^3
NU = 0.3            # Poisson ratio
GRAVITY = (0.0, 0.0, -9.8)
FRAME_DT = 1.0 / 60.0

INIT_PREV, INIT_INERTIA, INIT_Y, INIT_ADAPTIVE = 0, 1, 2, 3


@dataclasses.dataclass
class StepParams:
    """Per-step solver parameters (plain data)."""
    h: float = FRAME_DT
    n_iters: int = 20
    gravity: Tuple[float, float, float] = GRAVITY
    init_mode: int = INIT_ADAPTIVE
    det_eps_rel: float = 1e-6
    contact_k: float = 0.0
    contact_thickness: float = 0.0
    spheres: Optional[np.ndarray] = None   # [n,4] cx, cy, cz, R
    planes: Optional[np.ndarray] = None    # [n,4] nx, ny, nz, offset (n.x = offset)
    kd: float = 0.0                        # Rayleigh damping coefficient
    cheb_rho: float = 0.0                  # Chebyshev spectral radius (0 = off)
    friction_mu: float = 0.0
    friction_eps_v: float = 1e-2
    spring_psd: bool = False               # clamp transverse spring stiffness at 0
    mesh_contacts: bool = False            # vertex-triangle contacts between meshes
    collision_radius: float = 0.0          # detection radius for mesh contacts
    n_col: int = 0                         # re-detect every n_col iterations (0: only at x^t)
    self_contact: bool = False             # contacts within one mesh too
    self_exclusion: float = 0.0            # same-mesh primitives closer at rest never collide
    edge_contacts: bool = False            # edge-edge elements


@dataclasses.dataclass
class Workload:
    """A (possibly batched) simulation input, host numpy arrays."""
    name: str
    rest: np.ndarray                 # [nv,3] float64 rest shape
    tets: np.ndarray                 # [nt,4] int32
    pinned: np.ndarray               # [nv] uint8
    x0: np.ndarray                   # [nv,3] float64 initial positions
    v0: np.ndarray                   # [nv,3] float64 initial velocities
    tet_E: np.ndarray                # [nt] float64 Young's modulus per tet
    density: float = DENSITY
    nu: float = NU
    springs: Optional[np.ndarray] = None      # [ns,2] int32
    spring_rest: Optional[np.ndarray] = None  # [ns] float64 or None (rest distance)
    spring_k: float = 0.0
    mass: Optional[np.ndarray] = None         # [nv] float64 or None (lumped from tets)
    vert_offsets: Optional[np.ndarray] = None  # [n_meshes+1] int64
    tet_offsets: Optional[np.ndarray] = None   # [n_meshes+1] int64
    params: StepParams = dataclasses.field(default_factory=StepParams)
    frames: int = 1
    target: Optional[np.ndarray] = None        # [3] loss target (differentiable workload)
    colors: Optional[np.ndarray] = None        # [nv] given vertex coloring (None: greedy)
    coloring: str = "id"                       # greedy vertex order: "id", "smallest_last", "dsatur"

    @property
    def n_verts(self) -> int:
        return int(self.rest.shape[0])

    @property
    def n_tets(self) -> int:
        return int(self.tets.shape[0])

    @property
    def n_springs(self) -> int:
        return 0 if self.springs is None else int(self.springs.shape[0])

    @property
    def n_meshes(self) -> int:
        return 1 if self.vert_offsets is None else int(len(self.vert_offsets) - 1)

    def offsets(self):
        vo = self.vert_offsets if self.vert_offsets is not None else np.array([0, self.n_verts], np.int64)
        to = self.tet_offsets if self.tet_offsets is not None else np.array([0, self.n_tets], np.int64)
        return vo.astype(np.int64), to.astype(np.int64)


# ---------------------------------------------------------------------------
# topology builders
# ---------------------------------------------------------------------------
_PERMS = list(itertools.permutations(range(3)))   # lexicographic order


def cube_lattice(nx: int, ny: int, nz: int, edge: float = EDGE):
    """Kuhn-split lattice: returns (rest [nv,3] f64, tets [nt,4] int32)."""
    if min(nx, ny, nz) < 2:
        raise ValueError("lattice needs at least 2 vertices per axis")
    ii, jj, kk = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    # vertex id = i + nx*(j + ny*k): flatten in (k, j, i) order
    ii = ii.transpose(2, 1, 0).ravel()
    jj = jj.transpose(2, 1, 0).ravel()
    kk = kk.transpose(2, 1, 0).ravel()
    rest = np.stack([ii * edge - (nx - 1) * edge / 2.0,
                     jj * edge - (ny - 1) * edge / 2.0,
                     kk * edge], axis=1).astype(np.float64)

    ci, cj, ck = np.meshgrid(np.arange(nx - 1), np.arange(ny - 1), np.arange(nz - 1), indexing="ij")
    ci = ci.transpose(2, 1, 0).ravel()
    cj = cj.transpose(2, 1, 0).ravel()
    ck = ck.transpose(2, 1, 0).ravel()
    n_cells = ci.size
    tets = np.empty((n_cells, 6, 4), np.int64)
    for p, perm in enumerate(_PERMS):
        pos = np.stack([ci, cj, ck], axis=1).copy()
        ids = [pos[:, 0] + nx * (pos[:, 1] + ny * pos[:, 2])]
        for r in range(3):
            pos[:, perm[r]] += 1
            ids.append(pos[:, 0] + nx * (pos[:, 1] + ny * pos[:, 2]))
        tets[:, p, :] = np.stack(ids, axis=1)
    tets = tets.reshape(-1, 4)
    # orientation: swap v2, v3 where the signed volume is negative
    X = rest[tets]
    d1, d2, d3 = X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]
    sv = np.einsum("ij,ij->i", d1, np.cross(d2, d3))
    neg = sv < 0
    tets[neg, 2], tets[neg, 3] = tets[neg, 3].copy(), tets[neg, 2].copy()
    return rest, tets.astype(np.int32)


def cloth_grid(n: int, spacing: float, z0: float):
    """n x n grid in the z = z0 plane, centred at the origin.

    Returns (rest [nv,3], springs [ns,2] int32, spring family offsets).
    Springs: structural (+x, +y), shear (diagonal, anti-diagonal), bend
    (+2x, +2y); each family in vertex-id order.  Vertex id = i + n*j.
    """
    i, j = np.meshgrid(np.arange(n), np.arange(n), indexing="xy")  # j rows
    i = i.ravel(); j = j.ravel()
    rest = np.stack([i * spacing - (n - 1) * spacing / 2.0,
                     j * spacing - (n - 1) * spacing / 2.0,
                     np.full(i.shape, z0)], axis=1).astype(np.float64)
    vid = lambda a, b: a + n * b
    fam = []
    m = i < n - 1; fam.append(np.stack([vid(i[m], j[m]), vid(i[m] + 1, j[m])], 1))
    m = j < n - 1; fam.append(np.stack([vid(i[m], j[m]), vid(i[m], j[m] + 1)], 1))
    m = (i < n - 1) & (j < n - 1); fam.append(np.stack([vid(i[m], j[m]), vid(i[m] + 1, j[m] + 1)], 1))
    m = (i < n - 1) & (j < n - 1); fam.append(np.stack([vid(i[m] + 1, j[m]), vid(i[m], j[m] + 1)], 1))
    m = i < n - 2; fam.append(np.stack([vid(i[m], j[m]), vid(i[m] + 2, j[m])], 1))
    m = j < n - 2; fam.append(np.stack([vid(i[m], j[m]), vid(i[m], j[m] + 2)], 1))
    springs = np.concatenate(fam, 0).astype(np.int32)
    return rest, springs


# ---------------------------------------------------------------------------
# workloads
# ---------------------------------------------------------------------------
def _log_uniform(rng, lo, hi, size):
    return np.exp(rng.uniform(np.log(lo), np.log(hi), size))


def tet_cube(n: int, seed: int, *, E: Optional[float] = 1e5, E_range=None,
             pin_bottom: bool = True, jitter: float = 0.01 * EDGE,
             n_iters: int = 20, frames: int = 10, name: str = "") -> Workload:
    """n^3-vertex Kuhn lattice cube, bottom face pinned, jittered start."""
    rng = np.random.default_rng(seed)
    rest, tets = cube_lattice(n, n, n)
    nv, nt = rest.shape[0], tets.shape[0]
    if E_range is not None:
        tet_E = _log_uniform(rng, E_range[0], E_range[1], nt)
    else:
        tet_E = np.full(nt, float(E))
    pinned = np.zeros(nv, np.uint8)
    if pin_bottom:
        pinned[rest[:, 2] == 0.0] = 1
    jit = rng.uniform(-jitter, jitter, size=(nv, 3))
    jit[pinned.astype(bool)] = 0.0
    x0 = rest + jit
    v0 = np.zeros((nv, 3))
    return Workload(name=name or f"tet cube {n}^3", rest=rest, tets=tets, pinned=pinned,
                    x0=x0, v0=v0, tet_E=tet_E,
                    params=StepParams(n_iters=n_iters), frames=frames)


def config_small_cube() -> Workload:
    """11^3 vertices, 6000 tets, E = 1e5 uniform, 20 iterations x 10 frames."""
    return tet_cube(11, 0, E=1e5, n_iters=20, frames=10, name="tet cube 11^3")


def lattice_colors(nx: int, ny: int, nz: int) -> np.ndarray:
    """(i + j + k) mod 4 for vertex i + nx*(j + ny*k) of cube_lattice: every
    Kuhn-split edge vector is a nonzero 0/1 vector (up to sign), so the two
    ends of an edge differ by 1..3 in i + j + k and never share a color; the
    four vertices of each tet take all four colors."""
    i, j, k = np.meshgrid(np.arange(nx), np.arange(ny), np.arange(nz), indexing="ij")
    s = (i + j + k).transpose(2, 1, 0).ravel()
    return (s % 4).astype(np.int32)


def config_large_cube(frames: int = 60, coloring: str = "id") -> Workload:
    """65^3 vertices, 1,572,864 tets, per-tet E log-uniform in [1e4, 1e6].
    coloring: greedy first fit in vertex-id order ("id", 8 colors) or in the
    smallest-last order ("smallest_last", 4 colors), or the given lattice
    coloring ("lattice4", 4 colors)."""
    w = tet_cube(65, 1, E_range=(1e4, 1e6), n_iters=100, frames=frames, name="tet cube 65^3")
    if coloring == "lattice4":
        w.colors = lattice_colors(65, 65, 65)
        w.name += ", 4-color lattice coloring"
    elif coloring in ("id", "smallest_last"):
        w.coloring = coloring
        if coloring == "smallest_last":
            w.name += ", smallest-last greedy coloring"
    else:
        raise ValueError(f"unknown coloring {coloring}")
    return w


def config_cloth(n: int = 1024, frames: int = 120, spacing: float = 1e-3,
                 mass: float = 1e-4, coloring: str = "id") -> Workload:
    """Mass-spring cloth (n x n, 1 mm spacing) over a sphere and a ground plane.
    coloring: greedy vertex order, "id" (7 colors), "smallest_last" or
    "dsatur" (5 colors)."""
    rest, springs = cloth_grid(n, spacing, 0.62)
    nv = rest.shape[0]
    pinned = np.zeros(nv, np.uint8)
    pinned[0] = 1
    pinned[n - 1] = 1
    p = StepParams(n_iters=50, contact_k=1e5, contact_thickness=1e-3, spring_psd=True,
                   spheres=np.array([[0.0, 0.0, 0.3, 0.3]]),
                   planes=np.array([[0.0, 0.0, 1.0, 0.0]]))
    name = f"cloth {n}^2" + ("" if coloring == "id" else f", {coloring.replace('_', '-')} coloring")
    return Workload(name=name, rest=rest, tets=np.zeros((0, 4), np.int32),
                    pinned=pinned, x0=rest.copy(), v0=np.zeros((nv, 3)),
                    tet_E=np.zeros(0), springs=springs, spring_k=1e3,
                    mass=np.full(nv, mass), params=p, frames=frames, coloring=coloring)


def config_cloth_coarse(n: int = 64, frames: int = 60, coloring: str = "id") -> Workload:
    """The cloth of config_cloth over the same 1.023 m square with n x n
    vertices: spacing 1.023/(n-1) m and the same total mass."""
    spacing = 1.023 / (n - 1)
    return config_cloth(n, frames, spacing=spacing, mass=1e-4 * (1024.0 / n) ** 2,
                        coloring=coloring)


def config_batch(n_meshes: int = 512, seed: int = 3, lo: int = 4, hi: int = 33,
                 frames: int = 60, n_iters: int = 40, coloring: str = "id") -> Workload:
    """Independent free cubes with per-axis dims U{lo..hi}, per-mesh E, rigid v0.
    coloring: greedy vertex order, "id" or "smallest_last"."""
    rng = np.random.default_rng(seed)
    dims = rng.integers(lo, hi + 1, size=(n_meshes, 3))
    Em = _log_uniform(rng, 1e4, 1e6, n_meshes)
    rests, tetss, Es, vo, to = [], [], [], [0], [0]
    for m in range(n_meshes):
        r, t = cube_lattice(*[int(d) for d in dims[m]])
        # every mesh's lattice starts at the origin
        r = r - r.min(axis=0)
        rests.append(r)
        tetss.append(t + vo[-1])
        Es.append(np.full(t.shape[0], Em[m]))
        vo.append(vo[-1] + r.shape[0])
        to.append(to[-1] + t.shape[0])
    rest = np.concatenate(rests)
    tets = np.concatenate(tetss).astype(np.int32)
    nv = rest.shape[0]
    jit = rng.uniform(-0.01 * EDGE, 0.01 * EDGE, size=(nv, 3))
    x0 = rest + jit
    d = rng.normal(size=(n_meshes, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    speed = rng.uniform(0.0, 2.0, size=n_meshes)
    v0 = np.repeat(d * speed[:, None], np.diff(vo), axis=0)
    return Workload(name=f"batch of {n_meshes} cubes", rest=rest, tets=tets,
                    pinned=np.zeros(nv, np.uint8), x0=x0, v0=v0,
                    tet_E=np.concatenate(Es), vert_offsets=np.array(vo, np.int64),
                    tet_offsets=np.array(to, np.int64),
                    params=StepParams(n_iters=n_iters), frames=frames, coloring=coloring)


def config_block_stack(cols: int = 2, levels: int = 3, n: int = 5, seed: int = 5,
                       overlap: float = 0.002, gap: float = 0.5 * EDGE, frames: int = 10,
                       n_iters: int = 20, contact_k: float = 1e4, coloring: str = "id") -> Workload:
    """cols x cols columns of `levels` stacked n^3 lattice cubes (separate
    meshes).  Each cube sinks `overlap` into the one below it; odd levels are
    shifted by (0.33, 0.41) lattice cells so no vertex lies above an edge of
    the surface under it.  The bottom face of the lowest level is pinned;
    per-block E log-uniform in [1e5, 1e6]; x0 = rest, v0 = 0; gravity.
    k_c = 1e4 keeps every contact element a few mm deep (its resting depth is
    about 4 mm), away from the d = 0 switch where the penalty Hessian jumps."""
    rng = np.random.default_rng(seed)
    side = (n - 1) * EDGE
    rests, tetss, Es, pins, vo, to = [], [], [], [], [0], [0]
    for lev in range(levels):
        shift = np.array([0.33, 0.41]) * EDGE if lev % 2 else np.zeros(2)
        z0 = lev * (side - overlap)
        for i in range(cols):
            for j in range(cols):
                r, t = cube_lattice(n, n, n)
                r = r - r.min(axis=0)
                r = r + np.array([i * (side + gap + EDGE) + shift[0],
                                  j * (side + gap + EDGE) + shift[1], z0])
                pin = np.zeros(r.shape[0], np.uint8)
                if lev == 0:
                    pin[np.abs(r[:, 2]) < 1e-12] = 1
                rests.append(r)
                tetss.append(t + vo[-1])
                Es.append(np.full(t.shape[0], _log_uniform(rng, 1e5, 1e6, 1)[0]))
                pins.append(pin)
                vo.append(vo[-1] + r.shape[0])
                to.append(to[-1] + t.shape[0])
    rest = np.concatenate(rests)
    tets = np.concatenate(tetss).astype(np.int32)
    nv = rest.shape[0]
    params = StepParams(n_iters=n_iters, contact_k=contact_k, contact_thickness=1e-3,
                        mesh_contacts=True, collision_radius=0.5 * EDGE)
    return Workload(name=f"stack of {levels} x {cols}x{cols} cubes {n}^3", rest=rest, tets=tets,
                    pinned=np.concatenate(pins), x0=rest.copy(), v0=np.zeros((nv, 3)),
                    tet_E=np.concatenate(Es), vert_offsets=np.array(vo, np.int64),
                    tet_offsets=np.array(to, np.int64), params=params, frames=frames,
                    coloring=coloring)


def masked_lattice(mask: np.ndarray, edge: float = EDGE):
    """Kuhn-split lattice of the cells where mask[i, j, k] is true (the
    neighbouring cells' splits agree on every shared face); unused vertices
    are dropped and the rest renumbered in lattice order.  Returns
    (rest [nv, 3] f64 with the lattice origin at 0, tets [nt, 4] int32)."""
    cx, cy, cz = mask.shape
    rest, tets = cube_lattice(cx + 1, cy + 1, cz + 1, edge)
    # cube_lattice emits 6 tets per cell, cells in (k, j, i) order
    keep_cell = mask.transpose(2, 1, 0).ravel()
    tets = tets.reshape(-1, 6, 4)[keep_cell].reshape(-1, 4)
    used = np.zeros(rest.shape[0], bool)
    used[tets.ravel()] = True
    new_id = np.cumsum(used) - 1
    rest = rest[used] - rest.min(axis=0)
    return rest, new_id[tets].astype(np.int32)


def _rotate(rest, axis: int, angle: float):
    c, s = np.cos(angle), np.sin(angle)
    i, j = [a for a in range(3) if a != axis]
    out = rest.copy()
    out[:, i] = c * rest[:, i] - s * rest[:, j]
    out[:, j] = s * rest[:, i] + c * rest[:, j]
    return out


def config_crossed_bars(n: int = 4, gap: float = 0.5 * 5e-3, density: float = 100.0,
                        E: float = 1e6, frames: int = 12, n_iters: int = 20,
                        contact_k: float = 1e4, coloring: str = "id") -> Workload:
    """Edge-on-edge contact: two n^3 lattice cubes turned 45 degrees, the
    lower one about y (its top is an edge along y), the upper one about x
    (its bottom is an edge along x), the upper edge `gap` above the lower one
    and crossing it at both edges' midpoints (odd segment counts: the
    crossing is interior to a segment of each edge).  The lower cube's lowest
    vertices are pinned.  Only edge-edge elements can hold the upper cube:
    every vertex is farther from the other cube than the detection radius."""
    if n % 2:
        raise ValueError("n must be even: the crossing must be interior to a segment")
    side = (n - 1) * EDGE
    r0, t0 = cube_lattice(n, n, n)
    r0 = r0 - r0.mean(axis=0)
    lower = _rotate(r0, 1, np.pi / 4)
    lower[:, 2] -= lower[:, 2].max()
    upper = _rotate(r0, 0, np.pi / 4)
    upper[:, 2] += gap - upper[:, 2].min()
    rest = np.concatenate([lower, upper])
    tets = np.concatenate([t0, t0 + r0.shape[0]]).astype(np.int32)
    pinned = np.zeros(rest.shape[0], np.uint8)
    pinned[:r0.shape[0]][lower[:, 2] < lower[:, 2].min() + 0.3 * side] = 1
    nv = rest.shape[0]
    params = StepParams(n_iters=n_iters, contact_k=contact_k, contact_thickness=5e-3,
                        mesh_contacts=True, collision_radius=0.2 * EDGE, edge_contacts=True)
    vo = np.array([0, r0.shape[0], nv], np.int64)
    to = np.array([0, t0.shape[0], 2 * t0.shape[0]], np.int64)
    return Workload(name=f"crossed bars {n}^3", rest=rest, tets=tets, pinned=pinned,
                    x0=rest.copy(), v0=np.zeros((nv, 3)), tet_E=np.full(tets.shape[0], E),
                    density=density, vert_offsets=vo, tet_offsets=to, params=params,
                    frames=frames, coloring=coloring)


def config_folding_c(length: int = 7, width: int = 2, slab: int = 1, gap: int = 1,
                     E: float = 3e4, frames: int = 24, n_iters: int = 20,
                     contact_k: float = 1e4, coloring: str = "id") -> Workload:
    """Self-contact: one mesh shaped like a C lying on its side, a lower and
    an upper slab (`slab` cells thick, `length` cells long, `width` deep)
    joined by a wall at x = 0, `gap` cells apart.  The lower slab's bottom is
    pinned; the soft upper slab sags onto the lower one, so its bottom face
    meets the lower slab's top face: surfaces of the same mesh that are a gap
    apart in the rest shape (the self-contact exclusion distance is half of
    it)."""
    nz = 2 * slab + gap
    mask = np.ones((length, width, nz), bool)
    mask[1:, :, slab:slab + gap] = False
    rest, tets = masked_lattice(mask)
    pinned = (rest[:, 2] < 1e-12).astype(np.uint8)
    nv = rest.shape[0]
    params = StepParams(n_iters=n_iters, contact_k=contact_k, contact_thickness=5e-3,
                        mesh_contacts=True, collision_radius=0.2 * EDGE, edge_contacts=True,
                        self_contact=True, self_exclusion=0.5 * gap * EDGE, n_col=10)
    return Workload(name=f"folding C {length}x{width}", rest=rest, tets=tets, pinned=pinned,
                    x0=rest.copy(), v0=np.zeros((nv, 3)), tet_E=np.full(tets.shape[0], E),
                    params=params, frames=frames, coloring=coloring)


def config_differentiable(n: int = 33, seed: int = 4, frames: int = 30, n_iters: int = 20,
                          coloring: str = "id") -> Workload:
    """n^3 cube, per-tet E log-uniform, v0 = 0, seeded target for a centroid loss."""
    rng = np.random.default_rng(seed)
    rest, tets = cube_lattice(n, n, n)
    nv, nt = rest.shape[0], tets.shape[0]
    tet_E = _log_uniform(rng, 1e4, 1e6, nt)
    pinned = np.zeros(nv, np.uint8)
    pinned[rest[:, 2] == 0.0] = 1
    jit = rng.uniform(-0.01 * EDGE, 0.01 * EDGE, size=(nv, 3))
    jit[pinned.astype(bool)] = 0.0
    x0 = rest + jit
    v0 = np.zeros((nv, 3))
    target = x0.mean(axis=0) + rng.uniform(-0.5, 0.5, size=3)
    return Workload(name=f"differentiable cube {n}^3", rest=rest, tets=tets, pinned=pinned,
                    x0=x0, v0=v0, tet_E=tet_E, params=StepParams(n_iters=n_iters),
                    frames=frames, target=target, coloring=coloring)


def spring_net(n: int = 24, seed: int = 9, spacing: float = 0.05, k: float = 100.0,
               m: float = 0.01, rest_scale=(0.92, 1.08), n_massless: int = 6,
               frames: int = 12, n_iters: int = 3) -> Workload:
    """A hanging mass-spring net for the unprojected spring Hessian: an n x n
    grid in the xz-plane (structural + shear springs) with its top row pinned,
    jittered by U(+-10% spacing), each spring's rest length its jittered
    length times U[rest_scale] (about half the springs start compressed, whose
    transverse stiffness k(1 - L/l) is then negative).  Plus n_massless
    massless particles, each hung from its own pinned anchor by one spring at
    its rest length: their local Hessian k d d^T has rank one, so the
    determinant rule skips them in every iteration.  The light vertices
    (m/h^2 = 36 N/m against k = 100 N/m) and the few iterations per frame
    keep the step far from converged, so the Hessian used shapes the answer."""
    rng = np.random.default_rng(seed)
    ii, kk = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    ii, kk = ii.T.ravel(), kk.T.ravel()                 # vertex id = i + n k
    grid = np.stack([ii * spacing, np.zeros(ii.size), 1.0 - kk * spacing], 1)
    grid += rng.uniform(-0.1 * spacing, 0.1 * spacing, size=grid.shape)
    sp = []
    for k_ in range(n):
        for i in range(n):
            v = i + n * k_
            if i + 1 < n:
                sp.append((v, v + 1))
            if k_ + 1 < n:
                sp.append((v, v + n))
            if i + 1 < n and k_ + 1 < n:
                sp.append((v, v + n + 1))
            if i > 0 and k_ + 1 < n:
                sp.append((v, v + n - 1))
    sp = np.array(sp, np.int64)
    L = np.linalg.norm(grid[sp[:, 0]] - grid[sp[:, 1]], axis=1) * rng.uniform(*rest_scale, size=len(sp))
    pinned = np.zeros(n * n, np.uint8)
    pinned[np.flatnonzero(kk == 0)] = 1
    mass = np.full(n * n, m)
    # massless particles below the net, each on one spring from a pinned anchor
    anchors = np.stack([np.arange(n_massless) * 2 * spacing, np.full(n_massless, 0.3),
                        np.full(n_massless, 0.0)], 1)
    hang = anchors + np.array([0.0, 0.0, -spacing])
    base = n * n
    ids_a = base + 2 * np.arange(n_massless)
    extra_sp = np.stack([ids_a, ids_a + 1], 1)
    extra_pos = np.empty((2 * n_massless, 3))
    extra_pos[0::2], extra_pos[1::2] = anchors, hang
    rest = np.concatenate([grid, extra_pos])
    springs = np.concatenate([sp, extra_sp]).astype(np.int32)
    spring_rest = np.concatenate([L, np.full(n_massless, spacing)])
    pinned = np.concatenate([pinned, np.tile(np.array([1, 0], np.uint8), n_massless)])
    mass = np.concatenate([mass, np.tile(np.array([m, 0.0]), n_massless)])
    nv = rest.shape[0]
    return Workload(name=f"spring net {n}^2", rest=rest, tets=np.zeros((0, 4), np.int32),
                    pinned=pinned, x0=rest.copy(), v0=np.zeros((nv, 3)), tet_E=np.zeros(0),
                    springs=springs, spring_rest=spring_rest, spring_k=k, mass=mass,
                    params=StepParams(n_iters=n_iters), frames=frames)


def single_particle_chain(n: int = 2, length: float = 0.1, k: float = 100.0, m: float = 0.01):
    """n particles on a vertical line joined by springs, the top one pinned."""
    rest = np.zeros((n, 3))
    rest[:, 2] = -length * np.arange(n)
    springs = np.stack([np.arange(n - 1), np.arange(1, n)], 1).astype(np.int32)
    pinned = np.zeros(n, np.uint8); pinned[0] = 1
    return Workload(name=f"spring chain {n}", rest=rest, tets=np.zeros((0, 4), np.int32),
                    pinned=pinned, x0=rest.copy(), v0=np.zeros((n, 3)), tet_E=np.zeros(0),
                    springs=springs, spring_k=k, mass=np.full(n, m))


def subset_meshes(w: Workload, ids: List[int]) -> Workload:
    """Extract meshes ``ids`` of a batched workload as a new batched workload."""
    vo, to = w.offsets()
    rests, tetss, x0s, v0s, Es, pins = [], [], [], [], [], []
    nvo, nto = [0], [0]
    for m in ids:
        a, b = int(vo[m]), int(vo[m + 1])
        ta, tb = int(to[m]), int(to[m + 1])
        rests.append(w.rest[a:b]); x0s.append(w.x0[a:b]); v0s.append(w.v0[a:b])
        pins.append(w.pinned[a:b])
        tetss.append(w.tets[ta:tb] - a + nvo[-1]); Es.append(w.tet_E[ta:tb])
        nvo.append(nvo[-1] + b - a); nto.append(nto[-1] + tb - ta)
    colors = None
    if w.colors is not None:
        colors = np.concatenate([w.colors[int(vo[m]):int(vo[m + 1])] for m in ids])
    return dataclasses.replace(
        w, name=f"{w.name} [meshes {ids}]", rest=np.concatenate(rests), colors=colors,
        tets=np.concatenate(tetss).astype(np.int32), pinned=np.concatenate(pins),
        x0=np.concatenate(x0s), v0=np.concatenate(v0s), tet_E=np.concatenate(Es),
        vert_offsets=np.array(nvo, np.int64), tet_offsets=np.array(nto, np.int64))
