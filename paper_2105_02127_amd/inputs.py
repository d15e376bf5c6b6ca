"""Seeded synthetic inputs: jittered periodic triangle meshes and initial states.

This module holds no arithmetic of the reconstruction or flux method. It only
builds meshes (vertex coordinates and triangle lists) and cell-average initial
states, which both the CPU oracle and the HIP path consume unchanged.

Mesh recipe (periodic unit square, N x N squares, two triangles each):
  * h = 1/N; vertex (i, j) has id j*N + i and sits at (i*h + jx, j*h + jy),
    where jx and jy are drawn U[-0.2h, 0.2h]: first all jx, then all jy, each
    as an (N, N) array indexed [j, i] from ``np.random.default_rng(seed)``.
  * square (i, j) has corners v00=(i,j), v10=(i+1,j), v11=(i+1,j+1),
    v01=(i,j+1) (indices mod N) and is split along v00-v11 into cells
    2(jN+i) = (v00, v10, v11) and 2(jN+i)+1 = (v00, v11, v01).
  * the initial-state parameters are drawn from the same generator afterwards.

Initial states (conservative variables rho, rho*u, rho*v, E; gamma = 1.4):
  * ``smooth_wave``: rho = 1 + 0.2 sin(2 pi (x + y)), u = v = p = 1, as exact
    cell averages up to a 64-point product Gauss rule per triangle.  This is an
    exact Euler solution translating with velocity (1, 1).
  * ``random_lines``: two random lines split the torus into four regions with
    piecewise-constant states rho ~ U[0.1, 1.5], u, v ~ U[-1, 1],
    p ~ U[0.03, 1.5], sampled at cell centroids wrapped into [0, 1)^2.
  * ``wave_plus_jump``: the smooth wave with p multiplied by a ratio
    ~ U[2, 10] on the positive side of one random line.
  * ``kelvin_helmholtz``: the paper's single-mode KHI state (Sec. 5.7).

Meshes with boundaries (``jittered_box_mesh``): the same construction on
[x0, x0 + Lx] x [y0, y0 + Ly] with (Nx + 1) x (Ny + 1) vertices and no wrap;
interior vertices are jittered on both axes, boundary vertices only along
their side, corners stay put.  Boundary conditions are assigned per side
from each boundary face's midpoint:
  * ``double_mach``: the paper's double Mach reflection (Sec. 5.8) on
    [0, 4] x [0, 1]: a Mach 10 shock at x = 1/6 + y/sqrt(3) (60 degrees to
    the wall), post-shock (8, 8.25 cos 30deg, -8.25 sin 30deg, 116.5) to its
    left, (1.4, 0, 0, 1) to its right; bottom prescribed post-shock for
    x < 1/6 and reflective after it, left prescribed post-shock, right
    transmissive, top prescribed with the exact shock position
    1/6 + (1 + 20 t)/sqrt(3) at time t.
  * ``sod_x``: Sod's shock tube along x on [0, 1] x [0, Ly] (left state
    (1, 0, 1), right state (0.125, 0, 0.1), jump at x = 0.5), transmissive
    ends and reflective side walls.
  * ``shu_osher``: the paper's shock-density wave interaction (Sec. 5.5)
    along x on [0, 10] x [0, Ly], post-shock inflow on the left.

Disc meshes (``disc_mesh``): rings of points about a centre, jittered inside,
triangulated by Delaunay; every boundary face is transmissive (the library's
default).  ``ep01`` and ``ep02`` are the paper's explosion problems (Sec. 5.6)
on the unit disc about (1, 1).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

GAMMA = 1.4


@dataclass
class MeshData:
    n: int
    xy: np.ndarray          # [n_vert, 2] float64
    tri: np.ndarray         # [n_cell, 3] int32 (counter-clockwise)
    period: tuple = (1.0, 1.0)
    seed: int = 0
    rng: np.random.Generator = field(default=None, repr=False)
    box: tuple = None       # (x0, y0, lx, ly) of a mesh with open sides

    @property
    def n_cell(self) -> int:
        return int(self.tri.shape[0])

    @property
    def n_vert(self) -> int:
        return int(self.xy.shape[0])


def jittered_periodic_mesh(n: int, seed: int, jitter: float = 0.2) -> MeshData:
    """N x N x 2 jittered periodic triangulation of the unit torus."""
    if n < 2:
        raise ValueError("n must be >= 2")
    rng = np.random.default_rng(seed)
    h = 1.0 / n
    jx = rng.uniform(-jitter * h, jitter * h, size=(n, n))
    jy = rng.uniform(-jitter * h, jitter * h, size=(n, n))
    jj, ii = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    xy = np.stack([ii * h + jx, jj * h + jy], axis=-1).reshape(-1, 2)
    ip = (ii + 1) % n
    jp = (jj + 1) % n
    v00 = jj * n + ii
    v10 = jj * n + ip
    v11 = jp * n + ip
    v01 = jp * n + ii
    tri = np.empty((n * n, 2, 3), dtype=np.int32)
    tri[:, 0, 0] = v00.ravel()
    tri[:, 0, 1] = v10.ravel()
    tri[:, 0, 2] = v11.ravel()
    tri[:, 1, 0] = v00.ravel()
    tri[:, 1, 1] = v11.ravel()
    tri[:, 1, 2] = v01.ravel()
    return MeshData(n=n, xy=np.ascontiguousarray(xy, dtype=np.float64),
                    tri=np.ascontiguousarray(tri.reshape(-1, 3)), seed=seed, rng=rng)


def jittered_box_mesh(nx: int, ny: int, seed: int, lx: float = 1.0, ly: float = 1.0,
                      x0: float = 0.0, y0: float = 0.0, jitter: float = 0.2) -> MeshData:
    """Nx x Ny x 2 jittered triangulation of a rectangle with open sides."""
    if nx < 2 or ny < 2:
        raise ValueError("nx, ny must be >= 2")
    rng = np.random.default_rng(seed)
    hx, hy = lx / nx, ly / ny
    jx = rng.uniform(-jitter * hx, jitter * hx, size=(ny + 1, nx + 1))
    jy = rng.uniform(-jitter * hy, jitter * hy, size=(ny + 1, nx + 1))
    jx[:, 0] = jx[:, -1] = 0.0          # left and right sides keep their x
    jy[0, :] = jy[-1, :] = 0.0          # bottom and top keep their y
    jj, ii = np.meshgrid(np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    xy = np.stack([x0 + ii * hx + jx, y0 + jj * hy + jy], axis=-1).reshape(-1, 2)
    cj, ci = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    w = nx + 1
    v00 = cj * w + ci
    v10 = cj * w + ci + 1
    v11 = (cj + 1) * w + ci + 1
    v01 = (cj + 1) * w + ci
    tri = np.empty((nx * ny, 2, 3), dtype=np.int32)
    tri[:, 0, 0] = v00.ravel()
    tri[:, 0, 1] = v10.ravel()
    tri[:, 0, 2] = v11.ravel()
    tri[:, 1, 0] = v00.ravel()
    tri[:, 1, 1] = v11.ravel()
    tri[:, 1, 2] = v01.ravel()
    return MeshData(n=nx, xy=np.ascontiguousarray(xy, dtype=np.float64),
                    tri=np.ascontiguousarray(tri.reshape(-1, 3)), period=(0.0, 0.0),
                    seed=seed, rng=rng, box=(x0, y0, lx, ly))


def unwrapped_vertices(mesh: MeshData) -> np.ndarray:
    """[n_cell, 3, 2] vertex coordinates with v1, v2 moved to the periodic
    image nearest to v0 (on the periodic axes)."""
    p = np.asarray(mesh.period, dtype=np.float64)
    v = mesh.xy[mesh.tri]                      # [nc, 3, 2]
    d = v - v[:, :1, :]
    safe = np.where(p > 0, p, 1.0)
    v = v - np.where(p > 0, np.round(d / safe) * safe, 0.0)
    return v


def centroids(mesh: MeshData, wrap: bool = True) -> np.ndarray:
    c = unwrapped_vertices(mesh).mean(axis=1)
    if wrap:
        p = np.asarray(mesh.period)
        safe = np.where(p > 0, p, 1.0)
        c = c - np.where(p > 0, np.floor(c / safe) * safe, 0.0)
    return c


def _gauss01(n: int):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def triangle_average(mesh: MeshData, f, npts: int = 8) -> np.ndarray:
    """Cell averages of f(x, y) (vectorised) by a collapsed product Gauss rule."""
    v = unwrapped_vertices(mesh)
    t, w = _gauss01(npts)
    uu, ww = np.meshgrid(t, t, indexing="ij")
    wgt = (w[:, None] * w[None, :]) * uu * 2.0        # sums to 1 over the triangle
    q0, q1, q2 = v[:, 0], v[:, 1], v[:, 2]
    x = (q0[:, None, None, :] + uu[None, :, :, None] * (q1 - q0)[:, None, None, :]
         + (uu * ww)[None, :, :, None] * (q2 - q1)[:, None, None, :])
    vals = f(x[..., 0], x[..., 1])
    return (vals * wgt[None]).sum(axis=(1, 2))


def conservative(rho, u, v, p, gamma: float = GAMMA) -> np.ndarray:
    rho = np.asarray(rho, dtype=np.float64)
    u = np.broadcast_to(np.asarray(u, dtype=np.float64), rho.shape)
    v = np.broadcast_to(np.asarray(v, dtype=np.float64), rho.shape)
    p = np.broadcast_to(np.asarray(p, dtype=np.float64), rho.shape)
    e = p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)
    return np.ascontiguousarray(np.stack([rho, rho * u, rho * v, e], axis=-1))


def smooth_wave_density(x, y, t: float = 0.0):
    return 1.0 + 0.2 * np.sin(2.0 * math.pi * (x + y - 2.0 * t))


def smooth_wave(mesh: MeshData, t: float = 0.0, npts: int = 8) -> np.ndarray:
    """Exact cell averages of the translating density wave at time t."""
    rho = triangle_average(mesh, lambda x, y: smooth_wave_density(x, y, t), npts)
    return conservative(rho, 1.0, 1.0, 1.0)


def _random_line(rng):
    c = rng.uniform(0.0, 1.0, size=2)
    th = rng.uniform(0.0, math.pi)
    return c, np.array([math.cos(th), math.sin(th)])


def random_lines(mesh: MeshData, rng: np.random.Generator | None = None) -> np.ndarray:
    rng = mesh.rng if rng is None else rng
    c1, n1 = _random_line(rng)
    c2, n2 = _random_line(rng)
    states = []
    for _ in range(4):
        rho = rng.uniform(0.1, 1.5)
        u = rng.uniform(-1.0, 1.0)
        v = rng.uniform(-1.0, 1.0)
        p = rng.uniform(0.03, 1.5)
        states.append((rho, u, v, p))
    states = np.array(states)
    x = centroids(mesh, wrap=True)
    reg = 2 * (((x - c1) @ n1) >= 0.0).astype(np.int64) + (((x - c2) @ n2) >= 0.0).astype(np.int64)
    s = states[reg]
    return conservative(s[:, 0], s[:, 1], s[:, 2], s[:, 3])


def wave_plus_jump(mesh: MeshData, rng: np.random.Generator | None = None) -> np.ndarray:
    rng = mesh.rng if rng is None else rng
    c, nrm = _random_line(rng)
    ratio = rng.uniform(2.0, 10.0)
    rho = triangle_average(mesh, lambda x, y: smooth_wave_density(x, y), 8)
    x = centroids(mesh, wrap=True)
    p = np.where(((x - c) @ nrm) >= 0.0, ratio, 1.0)
    return conservative(rho, 1.0, 1.0, p)


def kelvin_helmholtz(mesh: MeshData) -> np.ndarray:
    """The single-mode Kelvin-Helmholtz state of the paper's KHI test on the
    periodic square [-0.5, 0.5]^2 (the unit torus shifted by -0.5), sampled
    at cell centroids: (rho, u) = (2, -0.5) for |y| <= 0.25, (1, 0.5)
    otherwise; v = 0.01 sin(2 pi x); p = 2.5."""
    x = centroids(mesh, wrap=True) - 0.5
    inner = np.abs(x[:, 1]) <= 0.25
    rho = np.where(inner, 2.0, 1.0)
    u = np.where(inner, -0.5, 0.5)
    v = 0.01 * np.sin(2.0 * math.pi * x[:, 0])
    return conservative(rho, u, v, np.full(mesh.n_cell, 2.5))


# ---------------------------------------------------------------------------
# states and boundary conditions on meshes with open sides
# ---------------------------------------------------------------------------
BC_TRANSMISSIVE, BC_REFLECTIVE, BC_PRESCRIBED = 1, 2, 3
def disc_mesh(h: float, seed: int, radius: float = 1.0, center=(1.0, 1.0),
              jitter: float = 0.2) -> MeshData:
    """Jittered Delaunay triangulation of a disc with open sides.

    Points: the centre, then rings k = 1..K at radius k R / K with
    K = round(R / (h sqrt(3) / 2)) and round(2 pi r / h) points each (at least
    6), spaced evenly from a random phase; all but the outer ring are moved by
    U[-jitter h, jitter h] on both axes, the outer ring stays on the circle.
    The draws come from ``np.random.default_rng(seed)`` in that order (ring
    phases, then the jitter).  Triangles are scipy's Delaunay simplices,
    turned counter-clockwise."""
    from scipy.spatial import Delaunay
    if not h > 0.0 or h > radius:
        raise ValueError("need 0 < h <= radius")
    rng = np.random.default_rng(seed)
    k_rings = max(1, round(radius / (h * math.sqrt(3.0) / 2.0)))
    rings = [np.zeros((1, 2))]
    for k in range(1, k_rings + 1):
        r = radius * k / k_rings
        n = max(6, round(2.0 * math.pi * r / h))
        th = 2.0 * math.pi * (np.arange(n) + rng.uniform(0.0, 1.0)) / n
        rings.append(np.stack([r * np.cos(th), r * np.sin(th)], 1))
    xy = np.concatenate(rings)
    n_in = len(xy) - len(rings[-1])
    xy[:n_in] += rng.uniform(-jitter * h, jitter * h, size=(n_in, 2))
    xy += np.asarray(center, dtype=np.float64)
    tri = Delaunay(xy).simplices.astype(np.int32)
    a = xy[tri]
    cw = ((a[:, 1, 0] - a[:, 0, 0]) * (a[:, 2, 1] - a[:, 0, 1])
          - (a[:, 2, 0] - a[:, 0, 0]) * (a[:, 1, 1] - a[:, 0, 1])) < 0.0
    tri[cw] = tri[cw][:, [0, 2, 1]]
    return MeshData(n=k_rings, xy=np.ascontiguousarray(xy), tri=np.ascontiguousarray(tri),
                    period=(0.0, 0.0), seed=seed, rng=rng)


DMR_PRE = (1.4, 0.0, 0.0, 1.0)
DMR_POST = (8.0, 8.25 * math.cos(math.pi / 6), -8.25 * math.sin(math.pi / 6), 116.5)


def face_sides(mesh: MeshData, verts: np.ndarray):
    """Midpoints [nb, 2] of boundary faces (vertex pairs) and their side:
    0 left, 1 right, 2 bottom, 3 top."""
    x0, y0, lx, ly = mesh.box
    mid = 0.5 * (mesh.xy[verts[:, 0]] + mesh.xy[verts[:, 1]])
    tol = 1e-9 * max(lx, ly)
    side = np.full(len(verts), -1, dtype=np.int64)
    side[np.abs(mid[:, 0] - x0) <= tol] = 0
    side[np.abs(mid[:, 0] - (x0 + lx)) <= tol] = 1
    side[np.abs(mid[:, 1] - y0) <= tol] = 2
    side[np.abs(mid[:, 1] - (y0 + ly)) <= tol] = 3
    if (side < 0).any():
        raise ValueError("a boundary face lies on no side of the box")
    return mid, side


def double_mach(mesh: MeshData) -> np.ndarray:
    """Initial state of the double Mach reflection at cell centroids."""
    x = centroids(mesh, wrap=False)
    post = x[:, 0] < 1.0 / 6.0 + x[:, 1] / math.sqrt(3.0)
    s = np.where(post[:, None], np.array(DMR_POST), np.array(DMR_PRE))
    return conservative(s[:, 0], s[:, 1], s[:, 2], s[:, 3])


def double_mach_boundary(mesh: MeshData, verts: np.ndarray, t: float = 0.0):
    """(kind [nb], state [nb, 4]) of the double Mach reflection at time t."""
    mid, side = face_sides(mesh, verts)
    post = conservative(*DMR_POST)
    pre = conservative(*DMR_PRE)
    kind = np.full(len(verts), BC_PRESCRIBED, dtype=np.int32)
    state = np.tile(post, (len(verts), 1))
    kind[side == 1] = BC_TRANSMISSIVE
    wall = (side == 2) & (mid[:, 0] >= 1.0 / 6.0)
    kind[wall] = BC_REFLECTIVE
    top = side == 3
    xs = 1.0 / 6.0 + (1.0 + 20.0 * t) / math.sqrt(3.0)
    state[top & (mid[:, 0] >= xs)] = pre
    return kind, np.ascontiguousarray(state)


def sod_x(mesh: MeshData) -> np.ndarray:
    """Sod's shock tube along x: (1, 0, 1) left of x = 0.5, (0.125, 0, 0.1) right."""
    x = centroids(mesh, wrap=False)
    left = x[:, 0] < 0.5
    return conservative(np.where(left, 1.0, 0.125), 0.0, 0.0, np.where(left, 1.0, 0.1))


SHU_OSHER_LEFT = (3.857, 2.629, 0.0, 10.333)


def shu_osher(mesh: MeshData) -> np.ndarray:
    """The shock-density wave interaction of the paper (Sec. 5.5) along x on
    [0, 10] x [0, Ly]: (3.857, 2.629, 10.333) for x < 1, (1 + 0.2 sin(5(x -
    5)), 0, 1) after it, at cell centroids."""
    x = centroids(mesh, wrap=False)[:, 0]
    left = x < 1.0
    rho = np.where(left, SHU_OSHER_LEFT[0], 1.0 + 0.2 * np.sin(5.0 * (x - 5.0)))
    return conservative(rho, np.where(left, SHU_OSHER_LEFT[1], 0.0), 0.0,
                        np.where(left, SHU_OSHER_LEFT[3], 1.0))


def shu_osher_boundary(mesh: MeshData, verts: np.ndarray):
    """Post-shock inflow on the left, transmissive right, reflective side walls."""
    _, side = face_sides(mesh, verts)
    kind = np.full(len(verts), BC_REFLECTIVE, dtype=np.int32)
    kind[side == 0] = BC_PRESCRIBED
    kind[side == 1] = BC_TRANSMISSIVE
    state = np.tile(conservative(*SHU_OSHER_LEFT), (len(verts), 1))
    return kind, np.ascontiguousarray(state)


def tube_boundary(mesh: MeshData, verts: np.ndarray):
    """Transmissive ends (left, right), reflective side walls."""
    _, side = face_sides(mesh, verts)
    kind = np.where(side <= 1, BC_TRANSMISSIVE, BC_REFLECTIVE).astype(np.int32)
    return kind, None


EXPLOSIONS = {
    # (inside r <= 0.5, outside) as (rho, u, v, p)
    "ep01": ((1.0, 0.0, 0.0, 1.0), (0.125, 0.0, 0.0, 0.1)),
    "ep02": ((1.0, 0.0, 0.0, 2.0), (1.0, 0.0, 0.0, 1.0)),
}


def explosion(mesh: MeshData, which: str = "ep01") -> np.ndarray:
    """The paper's 2D explosion problems (Sec. 5.6) on the disc of radius 1
    about (1, 1): one state inside the circle of radius 0.5 about the centre,
    another outside, at cell centroids."""
    inner, outer = EXPLOSIONS[which]
    x = centroids(mesh, wrap=False) - 1.0
    s = np.where(((x * x).sum(1) <= 0.25)[:, None], np.array(inner), np.array(outer))
    return conservative(s[:, 0], s[:, 1], s[:, 2], s[:, 3])


def disc_mask(mesh: MeshData, center, radius: float) -> np.ndarray:
    """Cells whose centroid lies within `radius` of `center` (periodic distance)."""
    x = centroids(mesh, wrap=True)
    d = x - np.asarray(center)
    p = np.asarray(mesh.period)
    d = d - np.round(d / p) * p
    return (d * d).sum(axis=1) <= radius * radius


# ---------------------------------------------------------------------------
# Named workloads: (order, mesh size, seed, initial state, steps); the batch
# workload is batch_specs below
# ---------------------------------------------------------------------------
WORKLOADS = {
    1: dict(name="teno3_wave_N32", order=3, n=32, seed=1, ic="smooth_wave", steps=10),
    2: dict(name="teno5_lines_N512", order=5, n=512, seed=2, ic="random_lines", steps=100),
    3: dict(name="teno6_wavejump_N1024", order=6, n=1024, seed=3, ic="wave_plus_jump", steps=50),
    4: dict(name="teno4_adjoint_N256", order=4, n=256, seed=4, ic="random_lines", steps=200),
    # the paper's KHI timing workload at its size (576,738 ~ 577,416 triangles)
    6: dict(name="teno5_khi_N537", order=5, n=537, seed=6, ic="kelvin_helmholtz", steps=100),
    # the paper's DMR timing workload at its size (369,800 ~ 369,794 triangles)
    7: dict(name="teno5_dmr_860x215", order=5, n=860, ny=215, lx=4.0, ly=1.0, seed=7,
            ic="double_mach", steps=100),
    # the paper's explosion problems at h = 1/50 (18,218 ~ 18,464 triangles)
    8: dict(name="teno5_ep01_h50", order=5, h=1.0 / 50.0, seed=8, ic="ep01", steps=100),
    9: dict(name="teno5_ep02_h50", order=5, h=1.0 / 50.0, seed=9, ic="ep02", steps=100),
}


def make_state(mesh: MeshData, ic: str) -> np.ndarray:
    if ic == "smooth_wave":
        return smooth_wave(mesh)
    if ic == "random_lines":
        return random_lines(mesh)
    if ic == "wave_plus_jump":
        return wave_plus_jump(mesh)
    if ic == "kelvin_helmholtz":
        return kelvin_helmholtz(mesh)
    if ic == "double_mach":
        return double_mach(mesh)
    if ic == "sod_x":
        return sod_x(mesh)
    if ic == "shu_osher":
        return shu_osher(mesh)
    if ic in EXPLOSIONS:
        return explosion(mesh, ic)
    raise ValueError(ic)


def make_workload(key: int, n: int | None = None):
    """Mesh + initial state of a named workload (optionally at another size)."""
    w = dict(WORKLOADS[key])
    if n is not None:
        w["n"] = n
    if "h" in w:
        if n is not None:
            w["h"] = 1.0 / n
        mesh = disc_mesh(w["h"], w["seed"])
    elif "ny" in w:
        if n is not None:
            w["ny"] = max(2, round(n * w["ly"] / w["lx"]))
        mesh = jittered_box_mesh(w["n"], w["ny"], w["seed"], w["lx"], w["ly"])
    else:
        mesh = jittered_periodic_mesh(w["n"], w["seed"])
    u0 = make_state(mesh, w["ic"])
    return w, mesh, u0


def adjoint_loss_disc(mesh: MeshData):
    """Disc of radius 0.1 with a seeded centre (drawn after the initial state)."""
    center = mesh.rng.uniform(0.0, 1.0, size=2)
    return center, 0.1


def batch_specs(n_mesh: int = 64, seed: int = 5, nmin: int = 32, nmax: int = 316):
    """(N, order, seed) of each mesh of the batched workload."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(nmin, nmax + 1, size=n_mesh)
    ps = rng.integers(3, 7, size=n_mesh)
    return [(int(ns[m]), int(ps[m]), 5000 + m) for m in range(n_mesh)]
