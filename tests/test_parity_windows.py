"""The sampled full-size parity tests take the oracle's step at a cell from
the cell's periodic window of (2s + 1)^3 cells.  On 3D grids small enough for
a whole-grid oracle step, the window's centre equals the whole-grid result bit
for bit (s = 3: first stage, two inner stages and the R0 correction; two
thermodynamic types with c; pores and grains of both 3D workloads)."""
import numpy as np
import pytest

import oracle
import pf_inputs as pi
from _parity import windowed_step


@pytest.mark.parametrize("nphi", [4, 9])
def test_windowed_step_equals_whole_grid_step(nphi):
    wl = pi.grains_pores_3d(n=20, nyz=(18, 13), n_grains=nphi + 2, n_grain_fields=nphi - 1, n_pores=3,
                            r_range=(2.0, 4.0), dmin=4.0)
    assert wl.n_phi == nphi
    P = oracle.Params(**wl.param_dict())
    dte = oracle.stable_dt(P)
    dt = 2.0 * dte
    s = oracle.stage_count(2, dt, dte)
    assert s == 3
    full, _, _ = oracle.step(P, oracle.RKL2, dt, wl.u0, s=s)
    assert np.abs(full - wl.u0).max() > 1e-5          # the step moves the state
    rng = np.random.default_rng(nphi)
    iface = np.flatnonzero((wl.u0[:nphi] > 0).sum(axis=0).ravel() >= 3)
    cells = np.unique(np.concatenate([rng.choice(wl.cells, 120, replace=False),
                                      rng.choice(iface, min(120, iface.size), replace=False)]))
    got = windowed_step(wl, wl.u0, cells, dt, s)
    ref = full.reshape(wl.F, -1)[:, cells].T
    assert np.array_equal(got, ref)
    # a window one cell narrower misses part of the dependence
    assert not np.array_equal(windowed_step(wl, wl.u0, cells, dt, s, radius=s - 1), ref)
