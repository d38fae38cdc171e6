"""The sampled full-size parity tests take the oracle's step at a cell from
the cell's periodic window of (2s + 1)^3 cells.  On 3D grids small enough for
a whole-grid oracle step, the window's centre equals the whole-grid result bit
for bit (s = 3: first stage, two inner stages and the R0 correction; two
thermodynamic types with c; pores and grains of both 3D workloads; and with
sparse storage that cuts cells, n_p = 2 of 4 phases)."""
import numpy as np
import pytest

import oracle
import pf_inputs as pi
from _parity import windowed_step


@pytest.mark.parametrize("nphi,n_p", [(4, 0), (9, 0), (4, 2)])
def test_windowed_step_equals_whole_grid_step(nphi, n_p):
    wl = pi.grains_pores_3d(n=20, nyz=(18, 13), n_grains=nphi + 2, n_grain_fields=nphi - 1, n_pores=3,
                            r_range=(2.0, 4.0), dmin=4.0)
    assert wl.n_phi == nphi
    P = oracle.Params(**wl.param_dict(), n_p=n_p)
    dte = oracle.stable_dt(P)
    dt = 2.0 * dte
    s = oracle.stage_count(2, dt, dte)
    assert s == 3
    oracle.store_truncations()
    full, _, _ = oracle.step(P, oracle.RKL2, dt, wl.u0, s=s)
    assert (oracle.store_truncations() > 0) == (n_p > 0)   # the sparse case does cut cells
    assert np.abs(full - wl.u0).max() > 1e-5          # the step moves the state
    rng = np.random.default_rng(nphi)
    iface = np.flatnonzero((wl.u0[:nphi] > 0).sum(axis=0).ravel() >= 3)
    cells = np.unique(np.concatenate([rng.choice(wl.cells, 120, replace=False),
                                      rng.choice(iface, min(120, iface.size), replace=False)]))
    extra = {"n_p": n_p} if n_p else None
    got = windowed_step(wl, wl.u0, cells, dt, s, extra=extra)
    ref = full.reshape(wl.F, -1)[:, cells].T
    assert np.array_equal(got, ref)
    # a window one cell narrower misses part of the dependence
    assert not np.array_equal(windowed_step(wl, wl.u0, cells, dt, s, radius=s - 1, extra=extra), ref)
