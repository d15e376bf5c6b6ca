"""Seeded synthetic inputs on tetrahedral meshes: jittered Kuhn subdivisions
of a periodic cube or of a box with open sides, and initial states.

This module holds no arithmetic of the reconstruction or flux method.  It only
builds meshes (vertex coordinates and tetrahedron lists) and cell-average
initial states, which both the CPU oracle and the HIP path consume unchanged.

Mesh recipe (N x N x N cubes of edge h = 1/N, six tetrahedra each):
  * vertex (i, j, k) has id (k N + j) N + i and sits at (i h, j h, k h)
    plus a jitter drawn U[-0.12 h, 0.12 h]: first all x jitters, then all y,
    then all z, each as an (N, N, N) array indexed [k, j, i] from
    ``np.random.default_rng(seed)``.
  * cube (i, j, k) (user cells 6c .. 6c+5, c = (k N + j) N + i) is split
    along its main diagonal from corner 0 = (i, j, k) to corner 7 =
    (i+1, j+1, k+1) into the six tetrahedra (0, a, b, 7) that follow the
    cube's edges (corner bits: 1 = +x, 2 = +y, 4 = +z), in the order of the
    axis permutations xyz, xzy, yxz, yzx, zxy, zyx (the Kuhn subdivision,
    conforming between neighbouring cubes); indices wrap modulo N.
  * the initial-state parameters are drawn from the same generator afterwards.

Boxes with open sides (``jittered_box3``) use (N+1)^3 vertices and no wrap;
a vertex on a side keeps its coordinate across that side.

Initial states (conservative variables rho, rho u, rho v, rho w, E;
gamma = 1.4):
  * ``smooth_wave3``: rho = 1 + 0.2 sin(2 pi (x + y + z - 3 t)),
    u = v = w = p = 1, as cell averages (a 64-point collapsed Gauss rule per
    tetrahedron): an exact Euler solution translating with (1, 1, 1).
  * ``random_planes3``: two random planes split the torus into four regions
    with rho ~ U[0.1, 1.5], u, v, w ~ U[-1, 1], p ~ U[0.03, 1.5], sampled at
    centroids wrapped into the unit cube.
  * ``explosion3``: the paper's 3D explosion (Sec. 5.9): (1, 0, 0, 0, 1)
    inside the ball of radius 0.5 about the centre, (0.125, 0, 0, 0, 0.1)
    outside, sampled at centroids.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

GAMMA = 1.4

# corners (bit 1 = +x, 2 = +y, 4 = +z) of the six Kuhn tetrahedra of a cube
KUHN = np.array([[0, 1, 3, 7], [0, 1, 5, 7], [0, 2, 3, 7], [0, 2, 6, 7], [0, 4, 5, 7],
                 [0, 4, 6, 7]], dtype=np.int64)


@dataclass
class TetMesh:
    n: tuple                  # cubes per axis
    xyz: np.ndarray           # [n_vert, 3] float64
    tet: np.ndarray           # [n_cell, 4] int32
    period: tuple = (1.0, 1.0, 1.0)   # 0 on an open axis
    seed: int = 0
    rng: np.random.Generator = field(default=None, repr=False)
    box: tuple = None         # (lo[3], hi[3]) of a box with open sides

    @property
    def n_cell(self) -> int:
        return int(self.tet.shape[0])

    @property
    def n_vert(self) -> int:
        return int(self.xyz.shape[0])


def _kuhn_cells(nx, ny, nz, vid):
    """[nx*ny*nz*6, 4] tetrahedra; vid(i, j, k) gives vertex ids (arrays)."""
    k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    corners = np.stack([vid(i + (c & 1), j + ((c >> 1) & 1), k + ((c >> 2) & 1)).ravel()
                        for c in range(8)], axis=1)           # [cubes, 8]
    return np.ascontiguousarray(corners[:, KUHN].reshape(-1, 4).astype(np.int32))


def jittered_periodic_cube(n: int, seed: int, jitter: float = 0.12) -> TetMesh:
    """N^3 x 6 jittered Kuhn tetrahedra of the unit 3-torus."""
    if n < 3:
        raise ValueError("n must be >= 3")
    rng = np.random.default_rng(seed)
    h = 1.0 / n
    jx = rng.uniform(-jitter * h, jitter * h, size=(n, n, n))
    jy = rng.uniform(-jitter * h, jitter * h, size=(n, n, n))
    jz = rng.uniform(-jitter * h, jitter * h, size=(n, n, n))
    k, j, i = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    xyz = np.stack([i * h + jx, j * h + jy, k * h + jz], axis=-1).reshape(-1, 3)
    tet = _kuhn_cells(n, n, n, lambda a, b, c: ((c % n) * n + (b % n)) * n + (a % n))
    return TetMesh(n=(n, n, n), xyz=np.ascontiguousarray(xyz, dtype=np.float64), tet=tet,
                   seed=seed, rng=rng)


def jittered_box3(nx: int, ny: int, nz: int, seed: int, lo=(0.0, 0.0, 0.0), hi=(1.0, 1.0, 1.0),
                  jitter: float = 0.12) -> TetMesh:
    """Nx x Ny x Nz x 6 jittered Kuhn tetrahedra of a box with open sides."""
    rng = np.random.default_rng(seed)
    lo, hi = np.asarray(lo, float), np.asarray(hi, float)
    h = (hi - lo) / np.array([nx, ny, nz])
    shape = (nz + 1, ny + 1, nx + 1)
    jit = [rng.uniform(-jitter * h[a], jitter * h[a], size=shape) for a in range(3)]
    jit[0][:, :, 0] = jit[0][:, :, -1] = 0.0
    jit[1][:, 0, :] = jit[1][:, -1, :] = 0.0
    jit[2][0, :, :] = jit[2][-1, :, :] = 0.0
    k, j, i = np.meshgrid(np.arange(nz + 1), np.arange(ny + 1), np.arange(nx + 1), indexing="ij")
    xyz = np.stack([lo[0] + i * h[0] + jit[0], lo[1] + j * h[1] + jit[1],
                    lo[2] + k * h[2] + jit[2]], axis=-1).reshape(-1, 3)
    tet = _kuhn_cells(nx, ny, nz, lambda a, b, c: (c * (ny + 1) + b) * (nx + 1) + a)
    return TetMesh(n=(nx, ny, nz), xyz=np.ascontiguousarray(xyz, dtype=np.float64), tet=tet,
                   period=(0.0, 0.0, 0.0), seed=seed, rng=rng, box=(tuple(lo), tuple(hi)))


def unwrapped_vertices(mesh: TetMesh) -> np.ndarray:
    """[n_cell, 4, 3] vertex coordinates of each cell, unwrapped about its
    first vertex on periodic axes."""
    v = mesh.xyz[mesh.tet]
    d = v - v[:, :1]
    for a in range(3):
        if mesh.period[a] > 0:
            d[..., a] -= mesh.period[a] * np.round(d[..., a] / mesh.period[a])
    return v[:, :1] + d


def centroids(mesh: TetMesh, wrap: bool = True) -> np.ndarray:
    c = unwrapped_vertices(mesh).mean(1)
    if wrap:
        for a in range(3):
            if mesh.period[a] > 0:
                c[:, a] -= mesh.period[a] * np.floor(c[:, a] / mesh.period[a])
    return c


def tet_average(mesh: TetMesh, f, npts: int = 4) -> np.ndarray:
    """Cell averages of f(x, y, z) by a collapsed Gauss-Legendre rule
    (npts^3 points per tetrahedron)."""
    t, w = np.polynomial.legendre.leggauss(npts)
    t, w = 0.5 * (t + 1.0), 0.5 * w
    u, v, s = np.meshgrid(t, t, t, indexing="ij")
    wu, wv, ws = np.meshgrid(w, w, w, indexing="ij")
    xi = (u * (1 - v) * (1 - s)).ravel()
    eta = (v * (1 - s)).ravel()
    zeta = s.ravel()
    wt = (wu * wv * ws * (1 - v) * (1 - s) ** 2).ravel() * 6.0   # sums to 1
    V = unwrapped_vertices(mesh)
    e1, e2, e3 = V[:, 1] - V[:, 0], V[:, 2] - V[:, 0], V[:, 3] - V[:, 0]
    pts = (V[:, None, 0] + xi[None, :, None] * e1[:, None] + eta[None, :, None] * e2[:, None]
           + zeta[None, :, None] * e3[:, None])
    return (f(pts[..., 0], pts[..., 1], pts[..., 2]) * wt[None]).sum(1)


def conservative(rho, u, v, w, p, gamma: float = GAMMA) -> np.ndarray:
    rho = np.asarray(rho, dtype=np.float64)
    n = rho.shape
    u = np.broadcast_to(np.asarray(u, dtype=np.float64), n)
    v = np.broadcast_to(np.asarray(v, dtype=np.float64), n)
    w = np.broadcast_to(np.asarray(w, dtype=np.float64), n)
    p = np.broadcast_to(np.asarray(p, dtype=np.float64), n)
    return np.stack([rho, rho * u, rho * v, rho * w,
                     p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v + w * w)], axis=-1)


def smooth_wave3_density(x, y, z, t: float = 0.0):
    return 1.0 + 0.2 * np.sin(2.0 * math.pi * (x + y + z - 3.0 * t))


def smooth_wave3(mesh: TetMesh, t: float = 0.0, npts: int = 4) -> np.ndarray:
    """Cell averages of the translating density wave at time t (momentum
    and energy are affine in rho here, so their averages follow)."""
    rho = tet_average(mesh, lambda x, y, z: smooth_wave3_density(x, y, z, t), npts)
    return conservative(rho, 1.0, 1.0, 1.0, 1.0)


def _random_plane(rng):
    c = rng.uniform(0.0, 1.0, size=3)
    nrm = rng.normal(size=3)
    return c, nrm / np.linalg.norm(nrm)


def random_planes3(mesh: TetMesh, rng: np.random.Generator | None = None) -> np.ndarray:
    rng = mesh.rng if rng is None else rng
    c1, n1 = _random_plane(rng)
    c2, n2 = _random_plane(rng)
    states = np.array([[rng.uniform(0.1, 1.5), rng.uniform(-1.0, 1.0), rng.uniform(-1.0, 1.0),
                        rng.uniform(-1.0, 1.0), rng.uniform(0.03, 1.5)] for _ in range(4)])
    x = centroids(mesh, wrap=True)
    if mesh.box is not None:
        lo, hi = np.asarray(mesh.box[0]), np.asarray(mesh.box[1])
        x = (x - lo) / (hi - lo)
    reg = 2 * (((x - c1) @ n1) >= 0).astype(int) + (((x - c2) @ n2) >= 0).astype(int)
    s = states[reg]
    return conservative(s[:, 0], s[:, 1], s[:, 2], s[:, 3], s[:, 4])


def explosion3(mesh: TetMesh, centre=(0.0, 0.0, 0.0), radius: float = 0.5) -> np.ndarray:
    x = centroids(mesh, wrap=False)
    inside = np.linalg.norm(x - np.asarray(centre), axis=1) <= radius
    return conservative(np.where(inside, 1.0, 0.125), 0.0, 0.0, 0.0, np.where(inside, 1.0, 0.1))


# Workloads on tetrahedra: TENO on the jittered periodic cube (random planes
# or the smooth wave), and the paper's 3D explosion (Sec. 5.9: edge h ~ 1/30)
# on [-1, 1]^3 with transmissive sides, 60^3 x 6 = 1,296,000 cells.  fallback:
# cells whose reconstruction leaves the physical states at a face point use
# their average there (the strong jumps need it).
WORKLOADS3 = {
    "teno4_planes_N32": dict(order=4, n=32, seed=31, ic="random_planes", fallback=1),
    "teno3_wave_N12": dict(order=3, n=12, seed=32, ic="smooth_wave", fallback=0),
    "explosion3_N60": dict(order=4, n=60, seed=33, ic="explosion", box=((-1.0,) * 3, (1.0,) * 3),
                           fallback=1),
}


def make_workload3(name: str, n: int | None = None):
    w = dict(WORKLOADS3[name])
    n = n or w["n"]
    if "box" in w:
        m = jittered_box3(n, n, n, w["seed"], w["box"][0], w["box"][1])
    else:
        m = jittered_periodic_cube(n, w["seed"])
    if w["ic"] == "random_planes":
        U = random_planes3(m)
    elif w["ic"] == "smooth_wave":
        U = smooth_wave3(m)
    else:
        U = explosion3(m)
    return w, m, U
