"""Seeded synthetic workloads for the explicit phase-field + concentration step.

This module is shared by the tests, the benchmark and the smoke check: it
builds parameter sets and initial fields only.  It contains none of the
method's arithmetic (no right-hand side, integrator, projection or norm); both
the CPU oracle and the HIP library consume what it returns.

Initial conditions follow Sec. 4 of Seiz & Takaki (arXiv 2601.16522): a
phase-field value is the equilibrium profile (eq. profile) of a distance
field, and where several distance fields overlap one phase is kept and the
rest are rescaled to fill the remainder of the simplex (eq. distfix, which for
ratio-preserving fields is a proportional rescaling).  Random numbers come
from ``numpy.random.default_rng(seed)`` (PCG64).

Fields are float64 arrays of shape (F, nz, ny, nx), F = n_phi + with_c, phi
planes first, then c.  Coordinates are cell indices (cell-centred grid, the
cell spacing dx only scales the physics).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import List, Sequence

import numpy as np

# -----------------------------------------------------------------------------
# Parameter sets
# -----------------------------------------------------------------------------


@dataclass
class Workload:
    """Grid, parameters and initial state of one simulation."""
    name: str
    dim: int
    nx: int
    ny: int
    nz: int
    n_phi: int
    type_of: List[int]
    n_types: int
    dx: float
    W: float
    gamma: List[float]
    mob: List[float]
    k: List[float]
    c0: List[float]
    D: List[float]
    with_c: bool
    u0: np.ndarray = field(repr=False, default=None)
    # boundaries (default periodic): per axis 0 periodic / 1 zero-gradient
    # walls; per face (x-, x+, y-, y+, z-, z+) a fixed c in the ghost cell
    bc: List[int] = field(default_factory=lambda: [0, 0, 0])
    c_fixed: List[int] = field(default_factory=lambda: [0] * 6)
    c_bc: List[float] = field(default_factory=lambda: [0.0] * 6)

    @property
    def F(self) -> int:
        return self.n_phi + (1 if self.with_c else 0)

    @property
    def cells(self) -> int:
        return self.nx * self.ny * self.nz

    def param_dict(self) -> dict:
        d = dict(dim=self.dim, nx=self.nx, ny=self.ny, nz=self.nz, n_phi=self.n_phi,
                 type_of=list(self.type_of), n_types=self.n_types, dx=self.dx, W=self.W,
                 gamma=list(self.gamma), mob=list(self.mob), k=list(self.k),
                 c0=list(self.c0), D=list(self.D), with_c=bool(self.with_c))
        if any(self.bc):
            d.update(bc=list(self.bc), c_fixed=list(self.c_fixed), c_bc=list(self.c_bc))
        return d


def profile(d: np.ndarray, W: float) -> np.ndarray:
    """Equilibrium obstacle profile of a signed distance d (eq. profile)."""
    x = np.clip(d / W, -0.5 * math.pi, 0.5 * math.pi)
    return 0.5 * (1.0 + np.sin(x))


def tanh_profile(d: np.ndarray, W: float) -> np.ndarray:
    """Smooth profile with the same centre slope 1/(2W) as eq. profile."""
    return 0.5 * (1.0 + np.tanh(d / W))


# -----------------------------------------------------------------------------
# Geometries
# -----------------------------------------------------------------------------


def circle_fields(nx: int, ny: int, R: float, W: float, kind: str = "tanh",
                  center=None) -> np.ndarray:
    """Two phases: a disc of radius R (phase 1) inside a matrix (phase 0).
    Distance field d = R - |X - C| (eq. centersphere)."""
    cx, cy = (nx / 2.0, ny / 2.0) if center is None else center
    y, x = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nx, dtype=np.float64),
                       indexing="ij")
    d = R - np.sqrt((x - cx) ** 2 + (y - cy) ** 2)
    p1 = tanh_profile(d, W) if kind == "tanh" else profile(d, W)
    phi = np.stack([1.0 - p1, p1])
    return phi[:, None, :, :]


def seeds_min_distance(n: int, box: Sequence[int], dmin: float, rng) -> np.ndarray:
    """n uniform points in a periodic box with pairwise (minimum-image) distance
    >= dmin, by dart throwing (falls back to accepting after many misses)."""
    box = np.asarray(box, dtype=np.float64)
    pts = []
    tries = 0
    while len(pts) < n:
        p = rng.random(len(box)) * box
        tries += 1
        if pts and dmin > 0 and tries < 200000:
            q = np.asarray(pts)
            dd = np.abs(q - p)
            dd = np.minimum(dd, box - dd)
            if np.min(np.sum(dd * dd, axis=1)) < dmin * dmin:
                continue
        pts.append(p)
    return np.asarray(pts)


def _grid_coords(shape_zyx, z0=0, z1=None):
    nz, ny, nx = shape_zyx
    z1 = nz if z1 is None else z1
    zz, yy, xx = np.meshgrid(np.arange(z0, z1, dtype=np.float64),
                             np.arange(ny, dtype=np.float64),
                             np.arange(nx, dtype=np.float64), indexing="ij")
    return zz, yy, xx


def _parallel_slabs(fn, starts) -> None:
    """Run fn over independent z slabs on a thread pool (numpy and the k-d tree
    release the GIL); results are identical to a sequential loop."""
    import os
    from concurrent.futures import ThreadPoolExecutor
    starts = list(starts)
    workers = max(1, min(16, os.cpu_count() or 1, len(starts)))
    if workers == 1:
        for z0 in starts:
            fn(z0)
        return
    with ThreadPoolExecutor(workers) as ex:
        list(ex.map(fn, starts))


def voronoi_fields(shape_zyx, seeds: np.ndarray, n_fields: int, W: float,
                   knear: int = 4, slab: int = 16) -> np.ndarray:
    """Periodic Voronoi grains smoothed by eq. profile.

    For a cell X with nearest seed p1, the grain of p1 gets the profile of the
    distance to the nearest bisector, every other near grain j the profile of
    minus its bisector distance; the nearest grain is kept and the others are
    rescaled to fill 1 - phi_1 (eq. distfix).  Grain g is stored in field
    g mod n_fields (round-robin; same-field neighbours merge).
    """
    from scipy.spatial import cKDTree

    nz, ny, nx = shape_zyx
    dim = 2 if nz == 1 and seeds.shape[1] == 2 else 3
    box = np.array([nx, ny] if dim == 2 else [nx, ny, nz], dtype=np.float64)
    tree = cKDTree(seeds, boxsize=box)
    k = min(knear, len(seeds))
    out = np.zeros((n_fields, nz, ny, nx))
    zstep = slab if dim == 3 else 1

    def one(z0):
        z1 = min(nz, z0 + zstep)
        zz, yy, xx = _grid_coords(shape_zyx, z0, z1)
        X = np.stack([xx.ravel(), yy.ravel()] + ([zz.ravel()] if dim == 3 else []), axis=1)
        _, idx = tree.query(X, k=k, workers=1)
        idx = idx.reshape(len(X), k)
        # minimum-image displacement from X to each of the k seeds
        disp = seeds[idx] - X[:, None, :]
        disp -= box * np.round(disp / box)
        d2 = np.sum(disp * disp, axis=2)
        p1 = disp[:, 0, :]
        bis = np.full((len(X), k), np.inf)
        for j in range(1, k):
            pj = disp[:, j, :]
            sep = np.sqrt(np.sum((pj - p1) ** 2, axis=1))
            sep = np.maximum(sep, 1e-12)
            bis[:, j] = (d2[:, j] - d2[:, 0]) / (2.0 * sep)
        d1 = np.min(bis[:, 1:], axis=1) if k > 1 else np.full(len(X), np.inf)
        phi1 = profile(d1, W)
        trial = np.zeros((len(X), k))
        for j in range(1, k):
            trial[:, j] = profile(-bis[:, j], W)
        rest = np.sum(trial, axis=1)
        scale = np.where(rest > 0.0, (1.0 - phi1) / np.where(rest > 0, rest, 1.0), 0.0)
        vals = trial * scale[:, None]
        vals[:, 0] = phi1
        fld = idx % n_fields
        plane = np.zeros((n_fields, len(X)))
        rows = np.arange(len(X))
        for j in range(k):
            # rows are distinct within one j, so plain fancy-index accumulation is exact
            plane[fld[:, j], rows] += vals[:, j]
        out[:, z0:z1] = plane.reshape(n_fields, z1 - z0, ny, nx)

    _parallel_slabs(one, range(0, nz, zstep))
    return out


def add_spheres(phi_grains: np.ndarray, centers: np.ndarray, radii: np.ndarray, W: float,
                slab: int = 16) -> np.ndarray:
    """Append a pore phase made of spheres: phi_pore = max_k profile(r_k - |X - C_k|)
    (periodic minimum image), grains rescaled to 1 - phi_pore (eq. distfix)."""
    nf, nz, ny, nx = phi_grains.shape
    dim = 3 if centers.shape[1] == 3 else 2
    box = np.array([nx, ny, nz][:dim], dtype=np.float64)
    out = np.zeros((nf + 1, nz, ny, nx))
    zstep = slab if dim == 3 else nz
    from scipy.spatial import cKDTree
    tree = cKDTree(centers, boxsize=box)
    kq = min(8, len(centers))

    def one(z0):
        z1 = min(nz, z0 + zstep)
        zz, yy, xx = _grid_coords((nz, ny, nx), z0, z1)
        X = np.stack([xx.ravel(), yy.ravel()] + ([zz.ravel()] if dim == 3 else []), axis=1)
        dist, idx = tree.query(X, k=kq, workers=1)
        dist = dist.reshape(len(X), kq)
        idx = idx.reshape(len(X), kq)
        pore = np.max(profile(radii[idx] - dist, W), axis=1)
        g = phi_grains[:, z0:z1].reshape(nf, -1)
        s = np.sum(g, axis=0)
        scale = np.where(s > 0, (1.0 - pore) / np.where(s > 0, s, 1.0), 0.0)
        out[:nf, z0:z1] = (g * scale).reshape(nf, z1 - z0, ny, nx)
        out[nf, z0:z1] = pore.reshape(z1 - z0, ny, nx)

    _parallel_slabs(one, range(0, nz, zstep))
    return out


# -----------------------------------------------------------------------------
# The five workloads (reduced sizes allowed through the keyword arguments)
# -----------------------------------------------------------------------------


def single_grain(n: int = 128, R: float = 40.0, W: float = 4.0, M: float = 1.0,
                 seed: int = 1, with_c: bool = True, profile_kind: str = "tanh",
                 ny: int = None) -> Workload:
    """Circular grain in a matrix, Table tab:params values (M = gamma = D = 1,
    dx = 1, k = 500), one thermodynamic type whose c0 equals the mean c;
    c = 0.5 + U(-1e-3, 1e-3)."""
    ny = n if ny is None else ny
    rng = np.random.default_rng(seed)
    phi = circle_fields(n, ny, R, W, kind=profile_kind)
    fields = [phi]
    if with_c:
        c = 0.5 + rng.uniform(-1e-3, 1e-3, size=(1, 1, ny, n))
        fields.append(c)
    u0 = np.concatenate(fields, axis=0)
    return Workload("single_grain_%dx%d" % (n, ny), 2, n, ny, 1, 2, [0, 0], 1, 1.0, W,
                    [1.0], [M], [500.0], [0.5], [1.0], with_c, u0)


def phase_embedding(n: int = 128, r: float = 32.0, W: float = 2.5, D: float = 100.0) -> Workload:
    """Phase embedding (Sec. 5.1.1): a disc of phase beta (type 1, c0 = 0.98)
    of radius r (d = r - |X - C|, eq. centersphere, eq. profile) embedded in
    phase alpha (type 0, c0 = 0.02) on a periodic n^2 grid; Table tab:params
    otherwise (gamma = M = 1, dx = 1, k = 500) with D = 100 as the paper uses
    for equilibrium runs.  c is the local equilibrium at mu = 0 (eq. cadef:
    sum phi c0), shifted uniformly so that its total equals the sharp-interface
    total pi r^2 c0_beta + (n^2 - pi r^2) c0_alpha (Sec. 4)."""
    c0a, c0b = 0.02, 0.98
    phi = circle_fields(n, n, r, W, kind="profile")
    c = phi[0:1] * c0a + phi[1:2] * c0b
    area = math.pi * r * r
    c = c + (area * c0b + (n * n - area) * c0a - c.sum()) / (n * n)
    u0 = np.concatenate([phi, c], axis=0)
    return Workload("phase_embedding_%dx%d_r%g" % (n, n, r), 2, n, n, 1, 2, [0, 1], 2, 1.0, W,
                    [1.0] * 4, [1.0] * 4, [500.0, 500.0], [c0a, c0b], [D, D], True, u0)


def double_triple_junction(nx: int = 96, ny: int = 192, r: float = 32.0, W: float = 3.0,
                           D: float = 100.0, g_ab: float = 2.0, g_bb: float = 1.0) -> Workload:
    """Double triple junction (Sec. 5.1.2): a disc of phase alpha (field 0,
    type 0, c0 = 0.02) of radius r (eq. centersphere, eq. profile) on the
    grain boundary x = nx / 2 between two grains of phase beta (fields 1 and 2,
    type 1, c0 = 0.98; d = C_x - x and its complement), the beta fields
    rescaled to fill 1 - phi_alpha with their ratio kept (eq. distfix).  The
    long side runs along the grain boundary; x ends in zero-gradient walls (so
    the boundary meets no second one), y is periodic.  gamma_ab = g_ab,
    gamma_bb = g_bb, M = 1, k = 500, D for both types (the paper's equilibrium
    value), W = 3 (its coarsest resolution, dx = 1).  c is the local
    equilibrium at mu = 0, shifted uniformly so that its total equals the
    sharp-interface total pi r^2 c0_alpha + (nx ny - pi r^2) c0_beta (Sec. 4)."""
    c0a, c0b = 0.02, 0.98
    cx, cy = nx / 2.0, ny / 2.0
    y, x = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nx, dtype=np.float64), indexing="ij")
    pa = profile(r - np.sqrt((x - cx) ** 2 + (y - cy) ** 2), W)
    b1, b2 = profile(cx - x, W), profile(x - cx, W)
    rest = b1 + b2
    scale = np.where(rest > 0.0, (1.0 - pa) / np.where(rest > 0.0, rest, 1.0), 0.0)
    phi = np.stack([pa, b1 * scale, b2 * scale])[:, None]
    c = phi[0:1] * c0a + (phi[1:2] + phi[2:3]) * c0b
    area = math.pi * r * r
    c = c + (area * c0a + (nx * ny - area) * c0b - c.sum()) / (nx * ny)
    u0 = np.concatenate([phi, c], axis=0)
    return Workload("double_triple_junction_%dx%d" % (nx, ny), 2, nx, ny, 1, 3, [0, 1, 1], 2, 1.0, W,
                    [1.0, g_ab, g_ab, g_bb], [1.0] * 4, [500.0, 500.0], [c0a, c0b], [D, D], True, u0,
                    bc=[1, 0, 0])


# M + F of the thin-interface relation for the phase-field mobility (Sec. 5.2.2)
STEFAN_MF = 0.3084251


def stefan_1d(nx: int = 1800, h: float = 400.0, W: float = 2.5, D: float = 1.0) -> Workload:
    """Solutal Stefan problem (Sec. 5.2.2) on an nx x 1 grid: phase beta
    (type 1, c0 = 0.98) on the left up to h (d = h - x, eq. profile), phase
    alpha (type 0, c0 = 0.02) beyond; k = 1, gamma = 1, D for both; the pair
    mobility from the thin-interface relation with K = 0 (eq. thin-interface:
    L = pi^2 / (16 W^2) D dc/dmu / ((c_beta - c_alpha)^2 (M + F)), dc/dmu =
    1/k, L = pi M / (4 W)).  c = phi_alpha 0.2 + phi_beta 0.98 (the far-field
    compositions); x ends in walls (zero-gradient phi) with c held at 0.98 on
    the left and 0.2 on the right; y is periodic (one row)."""
    c0a, c0b, ca, cb, k = 0.02, 0.98, 0.2, 0.98, 1.0
    L = math.pi ** 2 / (16 * W * W) * D * (1.0 / k) / ((c0b - c0a) ** 2 * STEFAN_MF)
    M = 4 * W * L / math.pi
    x = np.arange(nx, dtype=np.float64)[None, None, None, :]
    pb = profile(h - x, W)
    phi = np.concatenate([1.0 - pb, pb], axis=0)
    c = (1.0 - pb) * ca + pb * cb
    u0 = np.concatenate([phi, c], axis=0)
    return Workload("stefan1d_%d" % nx, 2, nx, 1, 1, 2, [0, 1], 2, 1.0, W, [1.0] * 4, [M] * 4,
                    [k, k], [c0a, c0b], [D, D], True, u0, bc=[1, 0, 0],
                    c_fixed=[1, 1, 0, 0, 0, 0], c_bc=[cb, ca, 0.0, 0.0, 0.0, 0.0])


def voronoi_2d(n: int = 1024, n_grains: int = 200, n_phi: int = 8, W: float = 5.0,
               seed: int = 2, c_seed: int = 3, dmin: float = 12.0, ny: int = None) -> Workload:
    """Periodic 2D Voronoi tessellation, grain g -> field g mod n_phi, eq. profile
    of width W from the bisector distances, eq. distfix; c = 0.3 + N(0, 0.01^2).
    One type (c0 = 0.3), Table tab:params values."""
    ny = n if ny is None else ny
    rng = np.random.default_rng(seed)
    seeds = seeds_min_distance(n_grains, (n, ny), dmin, rng)
    phi = voronoi_fields((1, ny, n), seeds, n_phi, W)
    crng = np.random.default_rng(c_seed)
    c = 0.3 + crng.normal(0.0, 0.01, size=(1, 1, ny, n))
    u0 = np.concatenate([phi, c], axis=0)
    return Workload("voronoi2d_%dx%d_N%d" % (n, ny, n_phi), 2, n, ny, 1, n_phi, [0] * n_phi, 1,
                    1.0, W, [1.0], [1.0], [500.0], [0.3], [1.0], True, u0)


def _pore_params(n_grain_fields: int):
    dx = 0.005
    W = 2.5 * dx
    type_of = [0] * n_grain_fields + [1]
    # types: 0 grain, 1 pore (the paper's mobile-pore set in its own units)
    gamma = [1.0, 1.0, 1.0, 1.0]
    mob = [5e-3, 5e-3, 5e-3, 5e-3]
    k = [1e5, 1e5]
    c0 = [0.0, 1.0]
    D = [5e-8, 10.0]
    return dx, W, type_of, gamma, mob, k, c0, D


def grains_pores_3d(n: int = 256, n_grains: int = 12, n_grain_fields: int = 12,
                    n_pores: int = 40, r_range=(4.0, 10.0), seed_grains: int = 4,
                    seed_pores: int = 5, dmin: float = 12.0, nyz=None) -> Workload:
    """3D Voronoi grains (round-robin to n_grain_fields fields) plus one pore
    phase of spheres (radius uniform in r_range cells); c = phi_pore, i.e. 1 in
    pores and 0 in solid.  Mobile-pore parameter set of Sec. 5.3:
    dx = 0.005, W = 2.5 dx, gamma = 1, M = 5e-3, D_pore = 10, D_grain = 5e-8,
    k = 1e5, c0 = 0 (grain) / 1 (pore)."""
    ny, nz = (n, n) if nyz is None else nyz
    dx, W, type_of, gamma, mob, k, c0, D = _pore_params(n_grain_fields)
    Wc = W / dx  # interface parameter in cells
    rng = np.random.default_rng(seed_grains)
    seeds = seeds_min_distance(n_grains, (n, ny, nz), dmin, rng)
    phi = voronoi_fields((nz, ny, n), seeds, n_grain_fields, Wc)
    prng = np.random.default_rng(seed_pores)
    centers = prng.random((n_pores, 3)) * np.array([n, ny, nz], dtype=np.float64)
    radii = prng.uniform(r_range[0], r_range[1], size=n_pores)
    phi = add_spheres(phi, centers, radii, Wc)
    c = phi[-1:].copy()
    u0 = np.concatenate([phi, c], axis=0)
    N = n_grain_fields + 1
    return Workload("grains_pores3d_%dx%dx%d_N%d" % (n, ny, nz, N), 3, n, ny, nz, N, type_of, 2,
                    dx, W, gamma, mob, k, c0, D, True, u0)


def batch_instances(count: int = 96, seed: int = 6, sides=(64, 96, 128, 192, 256, 384, 512),
                    W: float = 4.0) -> List[Workload]:
    """Independent 2D shrinking-grain instances: side drawn from `sides`,
    radius uniform in [0.2, 0.4] side, mobility uniform in [0.5, 2]; c as in
    single_grain.  Instance i uses generator seed (seed, i)."""
    out = []
    for i in range(count):
        rng = np.random.default_rng([seed, i])
        side = int(rng.choice(np.asarray(sides)))
        R = float(rng.uniform(0.2, 0.4)) * side
        M = float(rng.uniform(0.5, 2.0))
        phi = circle_fields(side, side, R, W, kind="tanh")
        c = 0.5 + rng.uniform(-1e-3, 1e-3, size=(1, 1, side, side))
        u0 = np.concatenate([phi, c], axis=0)
        out.append(Workload("batch%02d_%d" % (i, side), 2, side, side, 1, 2, [0, 0], 1, 1.0, W,
                            [1.0], [M], [500.0], [0.5], [1.0], True, u0))
    return out


def grain_growth_pores_3d(n: int = 512, n_grains: int = 2000, n_grain_fields: int = 8,
                          n_pores: int = 400, r_range=(3.0, 8.0), seed_grains: int = 7,
                          seed_pores: int = 8, dmin: float = 4.0, nyz=None) -> Workload:
    """Large 3D grain growth with pores: 2000 Voronoi grains round-robin onto 8
    fields plus a pore field of 400 spheres (radius 3-8 cells); c = phi_pore."""
    wl = grains_pores_3d(n=n, n_grains=n_grains, n_grain_fields=n_grain_fields,
                         n_pores=n_pores, r_range=r_range, seed_grains=seed_grains,
                         seed_pores=seed_pores, dmin=dmin, nyz=nyz)
    wl.name = "grain_growth_pores3d_%dx%dx%d_N%d" % (wl.nx, wl.ny, wl.nz, wl.n_phi)
    return wl
