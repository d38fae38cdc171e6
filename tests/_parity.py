"""Shared checks of the GPU parity tests (no GPU needed to import).

FP32 against the FP64 oracle.  Where every cell has at most two phases whose
values stay away from exact zeros, the bar is max |diff| <= 1e-4.  On
multi-grain states an FP32 value can also differ from the FP64 one by an
activity decision: phase a is active at a cell when phi_a > 0 at some point
of its stencil (reading R1), and where a third phase has a vanishing tail the
two precisions can decide it differently, which changes N_z and the pairwise
terms of eq. phieq by O(L B dt).  Such a change made in stage j spreads at
most one cell per later stage, so every value above 1e-4 must lie within
`reach` cells (the step's stage count) of a cell where three or more phases
are > 0 in either result; the count of such values is reported and bounded
by the caller.
"""
import math

import numpy as np
from scipy import ndimage

import oracle
import pf_inputs as pi


def mixed_2d(nx=70, ny=45, seed=21):
    """Three phases of two thermodynamic types with c: Voronoi grains (6 seeds,
    round-robin to 3 fields), ragged grid, c near the local equilibrium."""
    rng = np.random.default_rng(seed)
    seeds = pi.seeds_min_distance(6, (nx, ny), 8.0, rng)
    phi = pi.voronoi_fields((1, ny, nx), seeds, 3, 3.0)
    c0 = [0.1, 0.9]
    tof = [0, 1, 1]
    c = sum(phi[a] * c0[tof[a]] for a in range(3)) + rng.normal(0, 0.01, size=phi[0].shape)
    u0 = np.concatenate([phi, c[None]])
    return pi.Workload("mixed2d", 2, nx, ny, 1, 3, tof, 2, 1.0, 3.0, [1.0, 0.8, 0.8, 1.2],
                       [1.0, 2.0, 2.0, 0.5], [500.0, 300.0], c0, [1.0, 0.3], True, u0)


def multi_phase_cells(ref, u32, N):
    return ((ref[:N] > 0).sum(axis=0) >= 3) | ((u32[:N] > 0).sum(axis=0) >= 3)


def periodic_distance(mask, reach):
    """Euclidean distance (cells) to the nearest True cell of a periodic grid,
    exact up to reach + 1 cells."""
    pad = [(0, 0)] * mask.ndim
    for ax in range(mask.ndim):
        if mask.shape[ax] > 1:
            pad[ax] = (reach + 1, reach + 1)
    m = np.pad(mask, pad, mode="wrap")
    d = ndimage.distance_transform_edt(~m)
    sl = tuple(slice(p[0], p[0] + n) for p, n in zip(pad, mask.shape))
    return d[sl]


def fp32_stats(wl, u32, ref, reach):
    """(max, rms, count above 1e-4, farthest such value from a multi-phase
    cell) over all fields; c is compared relative to max(1, max |c|)."""
    N = wl.n_phi
    d = np.abs(u32 - ref)
    if wl.with_c:
        d[N] = d[N] / max(1.0, float(np.abs(ref[N]).max()))
    bad = (d > 1e-4).any(axis=0)
    far = 0.0
    if bad.any():
        mp = multi_phase_cells(ref, u32, N)
        far = float(periodic_distance(mp, reach)[bad].max()) if mp.any() else math.inf
    return float(d.max()), float(math.sqrt((d ** 2).mean())), int((d > 1e-4).sum()), far


def check_fp32_two_phase(wl, u32, ref, what):
    mx, rms, cnt, _ = fp32_stats(wl, u32, ref, 0)
    print(f"\n{what}: FP32 vs oracle max {mx:.2e} rms {rms:.2e}", flush=True)
    assert mx <= 1e-4, (what, mx)


def check_fp32_multi(wl, u32, ref, reach, what, max_count_frac):
    mx, rms, cnt, far = fp32_stats(wl, u32, ref, reach)
    print(f"\n{what}: FP32 vs oracle max {mx:.2e} rms {rms:.2e}, {cnt} values > 1e-4 "
          f"of {u32.size}, farthest {far:.2f} cells from a three-phase cell (reach {reach})",
          flush=True)
    assert far <= reach, (what, far, reach)
    assert cnt <= max_count_frac * u32.size, (what, cnt)
    assert rms <= 1e-5, (what, rms)
    assert mx <= 1e-2, (what, mx)


def window(u, wl, cell, s):
    """The (2s + 1)^3 periodic window of u (F planes of wl's 3D grid) centred
    on the flat cell index `cell`."""
    z, rest = divmod(cell, wl.ny * wl.nx)
    y, x = divmod(rest, wl.nx)
    off = np.arange(-s, s + 1)
    return u[np.ix_(np.arange(u.shape[0]), (z + off) % wl.nz, (y + off) % wl.ny, (x + off) % wl.nx)]


def windowed_step(wl, u, cells, dt, s, radius=None, integ=oracle.RKL2, extra=None):
    """The oracle's step of s stages (RKL2 unless integ says otherwise) at each
    of `cells`, computed on the cell's periodic window of (2 radius + 1)^3
    cells (radius s by default): after s stages a cell depends only on cells
    at most s stencil steps away (every stage reads the six neighbours, and a
    fixed step has no global coupling), so with radius s the window's centre
    equals the cell's value in a step of the whole grid.  extra: further
    oracle parameters (n_p for sparse storage)."""
    h = s if radius is None else radius
    w = 2 * h + 1
    P = oracle.Params(**dict(wl.param_dict(), nx=w, ny=w, nz=w, **(extra or {})))
    out = np.empty((len(cells), wl.F))
    for k, cell in enumerate(cells):
        ref, _, _ = oracle.step(P, integ, dt, window(u, wl, int(cell), h), s=s)
        out[k] = ref[:, h, h, h]
    return out
