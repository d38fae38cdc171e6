"""Sparse phase storage (Sec. 3.1 "Phase-field details") through the C-ABI
(-m gpu).  A state vector holds c, at most n_p nonzero phase values and their
phase ids per cell; the kernels compute on the scattered dense values, so:

* with n_p at least the largest count of nonzero phases any stored stage
  reaches (no cell cut), FE, RKL1 and RKL2 steps and the RHS equal dense
  storage bit for bit, in FP32 and FP64, 2D and 3D, one and two buffer groups;
  a stage can make every phase present on a cell's stencil nonzero there, so
  that count can exceed the initial one (up to 8 of 9 phases on the 3D
  grain-growth state below);
* with a smaller n_p, cells are cut by the storage rule (the n_p largest kept
  and renormalised); FP64 runs cut exactly the cells the oracle cuts with the
  same n_p and match it within 1e-10;
* fields round-trip through the dense host and device layouts, the
  diagnostics read the sparse layout, and what the mode does not run is
  refused.
"""
import numpy as np
import pytest

import oracle
import pf_inputs as pi
from _parity import check_fp32_multi, mixed_2d

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pf = pytest.importorskip("paper_2601_16522_amd")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    oracle.build(force=False)
    pf.lib()


def voronoi8():
    return pi.voronoi_2d(n=150, ny=70, n_grains=24, n_phi=8, W=4.0, dmin=8.0)


def gg9():
    return pi.grain_growth_pores_3d(n=40, nyz=(30, 20), n_grains=40, n_pores=4)


def pores4():
    return pi.grains_pores_3d(n=45, nyz=(19, 13), n_grains=6, n_grain_fields=3, n_pores=4,
                              r_range=(2.0, 4.0), dmin=4.0)


CASES = {
    "voronoi8_np5_fp32": (voronoi8, "fp32", 5, 0),
    "voronoi8_np5_fp64": (voronoi8, "fp64", 5, 0),
    # on this state stages spread up to 8 of the 9 phases into some cells
    "gg9_np8_fp32": (gg9, "fp32", 8, 0),
    "gg9_np8_fp32_g2": (gg9, "fp32", 8, 2),
    "gg9_np8_fp64": (gg9, "fp64", 8, 0),
    "pores4_np4_fp32": (pores4, "fp32", 4, 0),
    "mixed3_np3_fp64": (mixed_2d, "fp64", 3, 0),
}


def make(wl, prec, n_p, groups=0):
    sim = pf.Sim(wl.param_dict(), prec=prec)
    if groups:
        sim.set_field_groups(groups)
    if n_p:
        sim.set_sparse_storage(n_p)
        assert sim.sparse_storage() == n_p
    sim.init_fields(wl.u0)
    return sim


@pytest.mark.parametrize("name", list(CASES))
def test_sparse_equals_dense_without_cuts(name):
    gen, prec, n_p, groups = CASES[name]
    wl = gen()
    dte = pf.params_stable_dt(wl.param_dict())
    runs = [("fe", 0.9, 4), ("rkl1", 12.0, 2), ("rkl2", 25.0, 2)]
    d0 = make(wl, prec, 0, groups)
    s0 = make(wl, prec, n_p, groups)
    assert s0.sparse_cuts() == 0                 # the initial state fits
    np.testing.assert_array_equal(s0.rhs(), d0.rhs())
    u_in, _ = s0.get_fields()
    np.testing.assert_array_equal(u_in, d0.get_fields()[0])
    d0.close(); s0.close()
    for integ, mult, nsteps in runs:
        out = {}
        for sp in (0, n_p):
            sim = make(wl, prec, sp, groups)
            for _ in range(nsteps):
                sim.step(integ, mult * dte)
            u, t = sim.get_fields()
            out[sp] = (u, t, sim.sparse_cuts() if sp else 0, sim.diagnostics())
            sim.close()
        assert out[n_p][2] == 0, (name, integ, out[n_p][2])
        np.testing.assert_array_equal(out[n_p][0], out[0][0], err_msg=f"{name} {integ}")
        assert out[n_p][1] == out[0][1]
        dd, ds = out[0][3], out[n_p][3]
        assert ds["sum_c"] == pytest.approx(dd["sum_c"], rel=1e-12, abs=1e-12)
        assert ds["max_sum_dev"] == pytest.approx(dd["max_sum_dev"], abs=1e-12)
        assert ds["max_phi"] == dd["max_phi"] and ds["nonfinite"] == 0
    print(f"{name}: FE, RKL1, RKL2 and the RHS equal dense storage bit for bit", flush=True)


@pytest.mark.parametrize("wlname,n_p,integ,mult", [("mixed3", 2, "fe", 0.9), ("mixed3", 2, "rkl2", 20.0),
                                                   ("mixed3", 2, "rkl1", 10.0), ("gg9", 6, "fe", 0.9),
                                                   ("gg9", 5, "rkl2", 25.0)])
def test_sparse_with_cuts_matches_oracle_fp64(wlname, n_p, integ, mult):
    """Three phases of two types at n_p = 2 (cells with a third phase are cut),
    and the 3D grain-growth state at n_p = 6 and 5: the oracle applies the same
    storage rule; the same cells are cut and the fields agree."""
    wl = mixed_2d() if wlname == "mixed3" else gg9()
    P = oracle.Params(**wl.param_dict(), n_p=n_p)
    dte = oracle.stable_dt(P)
    dt = mult * dte
    oracle.store_truncations()
    ref, _, rc = oracle.run_to(P, INTEG[integ], wl.u0, 3 * dt, dt_fixed=dt)
    assert rc == 0
    ref_cuts = oracle.store_truncations()
    sim = make(wl, "fp64", n_p)
    sim.run_to(integ, 3 * dt, dt_fixed=dt)
    u, t = sim.get_fields()
    cuts = sim.sparse_cuts()
    print(f"\n{wlname} n_p = {n_p}, {integ}: {cuts} cells cut on the GPU, {ref_cuts} in the oracle",
          flush=True)
    assert cuts > 0 and cuts == ref_cuts
    N = wl.n_phi
    assert (u[:N] > 0).sum(axis=0).max() <= n_p
    assert np.abs(u[:N] - ref[:N]).max() <= 1e-10
    assert np.abs(u[N] - ref[N]).max() <= 1e-10


INTEG = {"fe": oracle.FE, "rkl1": oracle.RKL1, "rkl2": oracle.RKL2}


def test_sparse_device_round_trip_and_fp32_against_oracle():
    wl = gg9()
    sim = make(wl, "fp32", 8)
    dev = sim.empty_device()
    sim.get_fields_device(dev)
    host, _ = sim.get_fields()
    np.testing.assert_array_equal(dev.cpu().numpy().astype(np.float64), host)
    sim.init_fields_device(dev)
    again, _ = sim.get_fields()
    np.testing.assert_array_equal(again, host)
    P = oracle.Params(**wl.param_dict())
    dte = oracle.stable_dt(P)
    dt = 25.0 * dte
    sim.step("rkl2", dt)
    u, _ = sim.get_fields()
    assert sim.sparse_cuts() == 0
    s = oracle.stage_count(2, dt, dte)
    ref, _, _ = oracle.step(P, oracle.RKL2, dt, wl.u0, s=s)
    check_fp32_multi(wl, u, ref, s, "sparse FP32 RKL2 step", 2e-5)


def test_sparse_refusals():
    wl = mixed_2d()
    sim = pf.Sim(wl.param_dict(), prec="fp32")
    for bad in (-1, 4, 9):
        with pytest.raises(pf.PFError) as e:
            sim.set_sparse_storage(bad)
        assert e.value.code == -1
    sim.set_sparse_storage(2)
    with pytest.raises(pf.PFError) as e:
        sim.step("rkl2", 1.0)
    assert e.value.code == -6          # the fields were cleared
    sim.init_fields(wl.u0)
    for integ in ("ssp2", "ssp104"):
        with pytest.raises(pf.PFError) as e:
            sim.step(integ, 0.1)
        assert e.value.code == -7
    with pytest.raises(pf.PFError) as e:
        sim.run_to("rkl2", 10.0, tol=pf.Tol())
    assert e.value.code == -7
    with pytest.raises(pf.PFError) as e:
        sim.get_state()
    assert e.value.code == -7
    with pytest.raises(pf.PFError) as e:
        sim.set_stage_fusion(2)
    assert e.value.code == -7
    sim.set_sparse_storage(0)
    sim.init_fields(wl.u0)
    sim.set_stage_fusion(2)
    walled = dict(wl.param_dict())
    walled["bc"] = (1, 0, 0)
    sw = pf.Sim(walled, prec="fp64")
    with pytest.raises(pf.PFError) as e:
        sw.set_sparse_storage(2)
    assert e.value.code == -7
