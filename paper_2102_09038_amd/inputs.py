"""Seeded synthetic problem instances for the even-parity RTE solver.

This module only *describes* problem instances: a spatial simplicial mesh, an
antipodally symmetric triangulation of the unit sphere, piecewise-constant optical
parameters and a nodal source.  It contains none of the discretisation or solver
arithmetic, so it can feed both the HIP library and the independent CPU oracle.

Shapes follow the paper's setting (Sec. 1: the RTE, its inflow condition and the HG
phase function; Sec. 4: the spatial and angular meshes; Sec. 6: how the sphere mesh is
refined and projected):

* spatial mesh: structured N x N squares of [0,1]^2, each cut along the "/" diagonal
  (P1 vertices (N+1)^2, P0 cells 2N^2), or N^3 cubes of [0,1]^3 cut into 6 Kuhn
  tetrahedra;
* sphere mesh: the octahedron refined r times by edge midpoints projected to the
  sphere (8*4^r geodesic triangles); the upper half (centroid z > 0) is listed
  first and triangle n_tri/2 + k is the antipode of triangle k;
* media: sigma_t drawn U[lo, hi] per block of 8x8 (or 8x8x8) squares, sigma_s a fixed
  fraction of sigma_t;
* sources: the closed disk/ball indicator or a Gaussian bump, sampled at vertices.

All random draws use ``numpy.random.Generator(PCG64(seed))``.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

__all__ = [
    "Instance", "octahedral_sphere", "grid2d", "grid3d", "blockwise_sigma_t",
    "disk_source", "bump_source", "make_instance", "config_small", "config_realistic",
    "instance_distribution", "tiny_instance",
]


# --------------------------------------------------------------------------- sphere
def octahedral_sphere(level: int):
    """Octahedron refined ``level`` times, vertices projected to the unit sphere.

    Returns ``(svert [nv,3] float64, stri [nt,3] int32)``.  Triangles ``0..nt/2-1`` have
    centroids with z > 0; triangle ``nt/2 + k`` is the antipode of triangle ``k`` (its
    vertices are the negated vertices of triangle k, listed so that both are
    counter-clockwise seen from outside).
    """
    if level < 0:
        raise ValueError("level must be >= 0")
    verts: list[np.ndarray] = []
    index: dict[tuple, int] = {}

    def vid(p):
        key = tuple(np.round(p, 12) + 0.0)
        if key not in index:
            index[key] = len(verts)
            verts.append(np.asarray(p, dtype=np.float64))
        return index[key]

    px, py, pz = np.eye(3)
    # the four upper faces of the octahedron, counter-clockwise seen from outside
    faces = [(px, py, pz), (py, -px, pz), (-px, -py, pz), (-py, px, pz)]
    tris = [tuple(np.array(v) for v in f) for f in faces]
    for _ in range(level):
        nxt = []
        for a, b, c in tris:
            ab = (a + b); ab /= np.linalg.norm(ab)
            bc = (b + c); bc /= np.linalg.norm(bc)
            ca = (c + a); ca /= np.linalg.norm(ca)
            nxt += [(a, ab, ca), (ab, b, bc), (ca, bc, c), (ab, bc, ca)]
        tris = nxt
    upper = [(vid(a), vid(b), vid(c)) for a, b, c in tris]
    lower = [(vid(-a), vid(-c), vid(-b)) for a, b, c in tris]
    svert = np.array(verts, dtype=np.float64)
    stri = np.array(upper + lower, dtype=np.int32)
    return svert, stri


# --------------------------------------------------------------------------- spatial
def grid2d(n: int):
    """[0,1]^2 cut into n x n squares, each split along the "/" diagonal.

    Vertex (i, j) -> index i + (n+1) j at (i/n, j/n).  Square (i, j) gives cells
    2(i + n j) (lower right) and 2(i + n j) + 1 (upper left).  Returns
    ``(vert [(n+1)^2, 2], cell [2n^2, 3] int32, square_of_cell [2n^2, 2] int32)``.
    """
    xs = np.arange(n + 1, dtype=np.float64) / n
    X, Y = np.meshgrid(xs, xs, indexing="xy")
    vert = np.stack([X.ravel(), Y.ravel()], axis=1)
    cells, sq = [], []
    for j in range(n):
        for i in range(n):
            v00 = i + (n + 1) * j
            v10, v01, v11 = v00 + 1, v00 + n + 1, v00 + n + 2
            cells += [(v00, v10, v11), (v00, v11, v01)]
            sq += [(i, j), (i, j)]
    return vert, np.array(cells, dtype=np.int32), np.array(sq, dtype=np.int32)


def grid3d(n: int):
    """[0,1]^3 cut into n^3 cubes, each split into the 6 Kuhn tetrahedra that share
    the cube's main diagonal (all cubes in the same orientation).

    Vertex (i, j, k) -> i + (n+1)(j + (n+1) k).  Returns ``(vert, cell [6n^3, 4],
    cube_of_cell [6n^3, 3])``.
    """
    xs = np.arange(n + 1, dtype=np.float64) / n
    Z, Y, X = np.meshgrid(xs, xs, xs, indexing="ij")
    vert = np.stack([X.ravel(), Y.ravel(), Z.ravel()], axis=1)
    m = n + 1

    def v(i, j, k):
        return i + m * (j + m * k)

    perms = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]
    cells, cub = [], []
    for k in range(n):
        for j in range(n):
            for i in range(n):
                for p in perms:
                    o = [0, 0, 0]
                    path = [v(i, j, k)]
                    for axis in p[:2]:
                        o[axis] = 1
                        path.append(v(i + o[0], j + o[1], k + o[2]))
                    path.append(v(i + 1, j + 1, k + 1))
                    cells.append(path)
                    cub.append((i, j, k))
    return vert, np.array(cells, dtype=np.int32), np.array(cub, dtype=np.int32)


# --------------------------------------------------------------------------- media / sources
def blockwise_sigma_t(block_of_cell: np.ndarray, block: int, seed: int,
                      lo: float = 1.0, hi: float = 10.0) -> np.ndarray:
    """sigma_t ~ U[lo, hi], one draw per block of ``block`` squares (cubes) per axis.

    ``block_of_cell`` holds each cell's square/cube integer coordinates.  Blocks are
    drawn in lexicographic order with the first coordinate fastest.
    """
    bc = np.asarray(block_of_cell) // block
    nb = bc.max(axis=0) + 1
    rng = np.random.Generator(np.random.PCG64(seed))
    vals = rng.uniform(lo, hi, size=int(np.prod(nb)))
    flat = np.zeros(len(bc), dtype=np.int64)
    stride = 1
    for a in range(bc.shape[1]):
        flat += bc[:, a] * stride
        stride *= nb[a]
    return vals[flat].astype(np.float64)


def disk_source(vert: np.ndarray, radius: float = 0.2, centre: Optional[np.ndarray] = None):
    """q = 1 on the closed disk/ball |x - centre| <= radius, 0 elsewhere (at vertices)."""
    c = np.full(vert.shape[1], 0.5) if centre is None else np.asarray(centre, float)
    return (np.linalg.norm(vert - c, axis=1) <= radius + 1e-14).astype(np.float64)


def bump_source(vert: np.ndarray, width: float = 0.1, centre: Optional[np.ndarray] = None):
    """q = exp(-|x - centre|^2 / (2 width^2)) at vertices."""
    c = np.full(vert.shape[1], 0.5) if centre is None else np.asarray(centre, float)
    r2 = np.sum((vert - c) ** 2, axis=1)
    return np.exp(-r2 / (2.0 * width * width))


# --------------------------------------------------------------------------- instances
@dataclasses.dataclass
class Instance:
    """One RTE problem instance plus the method parameters it is solved with."""
    name: str
    vert: np.ndarray          # [n_vert, dim] float64
    cell: np.ndarray          # [n_cell, dim+1] int32
    sigma_t: np.ndarray       # [n_cell] float64
    sigma_s: np.ndarray       # [n_cell] float64
    g: float                  # Henyey-Greenstein anisotropy, 0 <= g < 1
    svert: np.ndarray         # [n_svert, 3] float64 unit vectors
    stri: np.ndarray          # [n_stri, 3] int32
    q_nodal: np.ndarray       # [n_vert] float64 isotropic source at vertices
    quad_level: int = 2       # sub-triangle refinement of the angular quadrature
    n_even: int = 0           # N+ : even subspace-correction degree
    n_odd: int = 5            # N- : degree of the odd PCG preconditioner
    l: int = 4                # inner Richardson steps of P1
    tol: float = 1e-8         # outer relative-residual tolerance

    @property
    def dim(self) -> int:
        return int(self.vert.shape[1])

    @property
    def n_sphere_pairs(self) -> int:
        return int(self.stri.shape[0] // 2)


def default_quad_level(svert, stri, g: float) -> int:
    """r_q = max(2, 1 + ceil(log2(2 h_S / (1 - g)))), h_S = longest geodesic edge."""
    e = []
    for a, b in ((0, 1), (1, 2), (2, 0)):
        dots = np.clip(np.sum(svert[stri[:, a]] * svert[stri[:, b]], axis=1), -1, 1)
        e.append(np.arccos(dots))
    h = float(np.max(e))
    return max(2, 1 + int(math.ceil(math.log2(2.0 * h / (1.0 - g)))))


def make_instance(name, dim, n, sphere_level, g, ratio, sigma_t=None, block=8, seed=1,
                  source="bump", quad_level=None, **kw) -> Instance:
    if dim == 2:
        vert, cell, blk = grid2d(n)
    elif dim == 3:
        vert, cell, blk = grid3d(n)
    else:
        raise ValueError("dim must be 2 or 3")
    if sigma_t is None:
        st = blockwise_sigma_t(blk, block, seed)
    else:
        st = np.full(len(cell), float(sigma_t))
    ss = ratio * st
    svert, stri = octahedral_sphere(sphere_level)
    q = disk_source(vert) if source == "disk" else bump_source(vert)
    if quad_level is None:
        quad_level = default_quad_level(svert, stri, g)
    return Instance(name=name, vert=vert, cell=cell, sigma_t=st, sigma_s=ss, g=float(g),
                    svert=svert, stri=stri, q_nodal=q, quad_level=int(quad_level), **kw)


def lattice_standin(cells_per_unit: int = 8, sphere_level: int = 2, g: float = 0.5, n_even: int = 4,
                    l: int = 4, n_odd: int = 5, seed: int = 11, n_absorbers: int = 12,
                    quad_level=None) -> Instance:
    """Stand-in for the lattice problem of the paper's numerical section (its block layout is
    in a figure that is not available): R = (0,7)^2 as 7 x 7 unit blocks, each cut into
    cells_per_unit^2 squares ("/" diagonal).  n_absorbers blocks (sigma_s = 0, sigma_a = 1),
    drawn with the seed from the 24 interior blocks other than the centre; the centre block
    holds the source q = 1 (nodal values on its closed square, 0 elsewhere); every other
    block scatters (sigma_s = 10, sigma_a = 0.01, so c = 10 / 10.01).  cells_per_unit = 8
    gives the paper's coarsest n_R+ = 57^2 = 3249."""
    n = 7 * cells_per_unit
    vert, cell, sq = grid2d(n)
    vert = 7.0 * vert
    blk = sq // cells_per_unit
    interior = [(i, j) for j in range(1, 6) for i in range(1, 6) if (i, j) != (3, 3)]
    rng = np.random.Generator(np.random.PCG64(seed))
    pick = rng.choice(len(interior), size=n_absorbers, replace=False)
    absorbing = {interior[int(t)] for t in pick}
    is_abs = np.array([(int(a), int(b)) in absorbing for a, b in blk])
    sigma_s = np.where(is_abs, 0.0, 10.0)
    sigma_t = np.where(is_abs, 1.0, 10.01)
    q = ((vert[:, 0] >= 3.0) & (vert[:, 0] <= 4.0) & (vert[:, 1] >= 3.0) & (vert[:, 1] <= 4.0)).astype(np.float64)
    svert, stri = octahedral_sphere(sphere_level)
    if quad_level is None:
        quad_level = default_quad_level(svert, stri, g)
    return Instance(name=f"lattice-standin-{n}x{n}-s{8 * 4 ** sphere_level}-g{g}", vert=vert, cell=cell,
                    sigma_t=sigma_t, sigma_s=sigma_s, g=float(g), svert=svert, stri=stri, q_nodal=q,
                    quad_level=int(quad_level), n_even=n_even, n_odd=n_odd, l=l, tol=1e-8)


def config_small() -> Instance:
    """16x16 grid, 128 sphere triangles, g=0.5, sigma_t=1, sigma_s=0.9, disk source,
    l=4, N+=4, N-=5, tol 1e-8 (the paper's benchmark method settings, Sec. 6.4)."""
    return make_instance("small-16x16-s128-g0.5", 2, 16, 2, 0.5, 0.9, sigma_t=1.0,
                         source="disk", quad_level=2, n_even=4, n_odd=5, l=4, tol=1e-8)


def config_realistic(n_even: int = 0) -> Instance:
    """128x128 grid, 2048 sphere triangles, g=0.9, sigma_t ~ U[1,10] per 8x8 block
    (seed 1), sigma_s = 0.99 sigma_t, Gaussian bump, l=4, N+=0 ("P1" correction), N-=5."""
    return make_instance("realistic-128x128-s2048-g0.9", 2, 128, 4, 0.9, 0.99, seed=1,
                         source="bump", quad_level=2, n_even=n_even, n_odd=5, l=4, tol=1e-8)


def tiny_instance(n=4, sphere_level=1, g=0.5, ratio=0.9, sigma_t=1.0, dim=2, quad_level=2,
                  n_even=2, n_odd=3, l=2, source="bump", seed=7) -> Instance:
    """A mesh small enough for a direct LU of the full mixed system."""
    return make_instance(f"tiny-{dim}d-{n}-s{8*4**sphere_level}-g{g}", dim, n, sphere_level, g,
                         ratio, sigma_t=sigma_t, seed=seed, source=source,
                         quad_level=quad_level, n_even=n_even, n_odd=n_odd, l=l, block=2)


def instance_distribution(count: int = 64, seed: int = 3, tol: float = 1e-8,
                          large_3d_fraction: float = 0.0, max_n: int = 128):
    """Instances of uneven size: N ~ U{32..max_n}, sphere level ~ U{2,3,4},
    g ~ U[0,0.95], sigma_s/sigma_t ~ U[0.5,0.999], sigma_t blockwise U[1,10] with
    per-instance seed 1000+i, Gaussian bump, N+=0, l=4.  With ``large_3d_fraction`` > 0
    that share of instances is replaced by 3D cube problems (32^3 Kuhn tets, 512
    sphere triangles, g=0.8)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    for i in range(count):
        n = int(rng.integers(32, max_n + 1))
        lev = int(rng.integers(2, 5))
        g = float(rng.uniform(0.0, 0.95))
        ratio = float(rng.uniform(0.5, 0.999))
        big = bool(rng.uniform() < large_3d_fraction)
        if big:
            inst = make_instance(f"req{i}-3d-32-s512", 3, 32, 3, 0.8, ratio, seed=1000 + i,
                                 n_even=0, n_odd=5, l=4, tol=tol)
        else:
            inst = make_instance(f"inst{i}-{n}x{n}-s{8*4**lev}-g{g:.3f}", 2, n, lev, g, ratio,
                                 seed=1000 + i, n_even=0, n_odd=5, l=4, tol=tol)
        out.append(inst)
    return out
