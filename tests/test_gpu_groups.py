"""Stage kernels compiled for two and four buffer groups per state vector (the
addressing of the 512^3 workloads) on small grids: pf_set_field_groups forces
the group count, every stage kind runs (RHS, Euler and SSP sub-steps, SSP(s)2
and SSP(10)4 finals, RKL1 and RKL2 stages, the first RKL2 stage with its R0
correction, the estimator), and the results equal the one-group kernels' bit
for bit and the oracle to 1e-10 in FP64."""
import numpy as np
import pytest

import oracle
import pf_inputs as pi
from _parity import mixed_2d

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pf = pytest.importorskip("paper_2601_16522_amd")

INTEG = {"fe": oracle.FE, "ssp2": oracle.SSP2, "ssp104": oracle.SSP104, "rkl1": oracle.RKL1,
         "rkl2": oracle.RKL2}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    oracle.build(force=False)
    pf.lib()


def workloads():
    mixed = mixed_2d()
    p3 = pi.grains_pores_3d(n=20, nyz=(18, 13), n_grains=5, n_grain_fields=3, n_pores=3,
                            r_range=(2.0, 4.0), dmin=5.0)
    gg = pi.grain_growth_pores_3d(n=24, n_grains=20, n_pores=3, dmin=4.0)
    return {"mixed2d": mixed, "pores3d": p3, "gg3d_N9": gg}


def run(wl, prec, ng, fn):
    sim = pf.Sim(wl.param_dict(), prec=prec, ssp_stages=3)
    sim.set_field_groups(ng)
    assert sim.field_groups() == ng
    sim.set_tiling(0, 5)
    sim.init_fields(wl.u0)
    out = fn(sim)
    u, t = sim.get_fields()
    return u, out


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("wlname", ["mixed2d", "pores3d", "gg3d_N9"])
def test_every_stage_kind_at_two_and_four_groups(wlname, prec):
    wl = workloads()[wlname]
    P = oracle.Params(**wl.param_dict())
    dte = oracle.stable_dt(P)
    tol = pf.Tol(r_phi=1e-4, a_phi=1e-3, r_c=1e-4, a_c=1e-4)
    cases = {
        "rhs": lambda s: s.rhs(),
        "fe": lambda s: s.step("fe", 0.9 * dte),
        "ssp2": lambda s: s.step("ssp2", 1.5 * dte),
        "ssp104": lambda s: s.step("ssp104", 4.0 * dte),
        "rkl1": lambda s: s.step("rkl1", 12.0 * dte),
        "rkl2": lambda s: s.step("rkl2", 25.0 * dte),
        "rkl2_adaptive": lambda s: (s.run_to("rkl2", 120.0 * dte, tol=tol), s.trace()),
        "rkl1_adaptive": lambda s: (s.run_to("rkl1", 60.0 * dte, tol=tol), s.trace()),
    }
    for name, fn in cases.items():
        u1, o1 = run(wl, prec, 1, fn)
        for ng in (2, 4):
            ug, og = run(wl, prec, ng, fn)
            assert np.array_equal(u1, ug), (name, ng)
            if name == "rhs":
                assert np.array_equal(o1, og), (name, ng)
            if name.endswith("adaptive"):
                assert np.array_equal(o1[1], og[1]), (name, ng)
        if prec == "fp64" and name in INTEG:
            s = {"ssp2": 3, "ssp104": 0}.get(name, 0)
            dt = {"fe": 0.9, "ssp2": 1.5, "ssp104": 4.0, "rkl1": 12.0, "rkl2": 25.0}[name] * dte
            if name in ("rkl1", "rkl2"):
                s = oracle.stage_count(1 if name == "rkl1" else 2, dt, dte)
            ref, _, _ = oracle.step(P, INTEG[name], dt, wl.u0, s=s)
            sim4 = pf.Sim(wl.param_dict(), prec=prec, ssp_stages=3)
            sim4.set_field_groups(4)
            sim4.init_fields(wl.u0)
            sim4.step(name, dt)
            u4, _ = sim4.get_fields()
            N = wl.n_phi
            assert np.abs(u4[:N] - ref[:N]).max() <= 1e-10, name
            assert np.abs(u4[N] - ref[N]).max() <= 1e-10 * max(1.0, np.abs(ref[N]).max()), name
        if prec == "fp64" and name == "rhs":
            ref = oracle.rhs(P, wl.u0)
            scale = np.abs(ref).max(axis=(1, 2, 3), keepdims=True)
            assert (np.abs(o1 - ref) / np.maximum(scale, 1e-300)).max() <= 1e-12


def test_group_count_errors():
    wl = workloads()["mixed2d"]
    sim = pf.Sim(wl.param_dict(), prec="fp32")
    for bad in (3, 5, -1):
        with pytest.raises(pf.PFError):
            sim.set_field_groups(bad)
    sim.set_field_groups(2)
    # fused stage pairs run with one group only
    with pytest.raises(pf.PFError):
        sim.set_stage_fusion(2)
    sim.set_field_groups(0)
    assert sim.field_groups() == 1
    sim.set_stage_fusion(2)
    walled = dict(wl.param_dict())
    walled["bc"] = (1, 0, 0)
    sw = pf.Sim(walled, prec="fp64")
    with pytest.raises(pf.PFError) as ei:
        sw.set_field_groups(2)
    assert ei.value.code == -7
