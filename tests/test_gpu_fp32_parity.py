"""The FP32 chosen form against the FP64 oracle, element by element, for every
integrator in 2D and 3D, and FP32 adaptive runs replayed step for step in the
oracle.  Bars (see tests/_parity.py): two-phase states with smooth profiles
max |diff| <= 1e-4; multi-grain states 1e-4 except for values within the
step's stage count of a cell with three phases > 0 (activity decisions at
vanishing tails, reading R1), whose count is bounded per test."""
import math

import numpy as np
import pytest

import oracle
import pf_inputs as pi
from _parity import check_fp32_multi, check_fp32_two_phase

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pf = pytest.importorskip("paper_2601_16522_amd")

INTEG = {"fe": oracle.FE, "ssp2": oracle.SSP2, "ssp104": oracle.SSP104, "rkl1": oracle.RKL1,
         "rkl2": oracle.RKL2}
DT = {"fe": 0.9, "ssp2": 1.8, "ssp104": 5.0, "rkl1": 20.0, "rkl2": 50.0}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    oracle.build(force=False)
    pf.lib()


def sphere_3d(n=40, r=11.0):
    """Two phases in 3D: a pore sphere (tanh profile, every phi > 0) in one
    grain, the mobile-pore parameter set, c = phi_pore."""
    dx, W, _, gamma, mob, k, c0, D = pi._pore_params(1)
    Wc = W / dx
    z, y, x = np.meshgrid(*(np.arange(n, dtype=np.float64),) * 3, indexing="ij")
    d = r - np.sqrt((x - n / 2) ** 2 + (y - n / 2) ** 2 + (z - n / 2) ** 2)
    pore = pi.tanh_profile(d, Wc)
    u0 = np.stack([1.0 - pore, pore, pore.copy()])[:, :, :, :]
    return pi.Workload("sphere3d", 3, n, n, n, 2, [0, 1], 2, dx, W, gamma, mob, k, c0, D, True, u0)


def stages(integ, dt, dte, ssp):
    if integ in ("rkl1", "rkl2"):
        return oracle.stage_count(1 if integ == "rkl1" else 2, dt, dte)
    return {"fe": 1, "ssp2": ssp, "ssp104": 10}[integ]


def one_step(wl, integ, ssp=3):
    P = oracle.Params(**wl.param_dict())
    dte = oracle.stable_dt(P)
    dt = DT[integ] * dte
    if integ == "ssp2":
        dt = min(dt, 0.9 * (ssp - 1) * dte)
    sim = pf.Sim(wl.param_dict(), prec="fp32", ssp_stages=ssp)
    sim.init_fields(wl.u0)
    sim.step(integ, dt)
    u32, _ = sim.get_fields()
    s = stages(integ, dt, dte, ssp)
    ref, _, _ = oracle.step(P, INTEG[integ], dt, wl.u0, s=s if integ != "ssp104" else 0)
    return u32, ref, s


@pytest.mark.parametrize("integ", ["fe", "ssp2", "ssp104", "rkl1", "rkl2"])
@pytest.mark.parametrize("dim", [2, 3])
def test_one_step_fp32_two_phase_every_integrator(integ, dim):
    wl = pi.single_grain(n=96, R=30.0) if dim == 2 else sphere_3d()
    for ssp in ((3, 5) if integ == "ssp2" else (3,)):
        u32, ref, _ = one_step(wl, integ, ssp)
        check_fp32_two_phase(wl, u32, ref, f"{integ} ssp={ssp} {dim}D two-phase")


def voronoi_small():
    return pi.voronoi_2d(n=160, n_grains=24, n_phi=8, dmin=12.0)


def sintering_small():
    """The sintering generator (12 grains on 12 fields plus the pore phase,
    radii 4-10 cells) at 48^3."""
    return pi.grains_pores_3d(n=48, n_grains=12, n_grain_fields=12, n_pores=6, dmin=12.0)


def graingrowth_small():
    """The grain-growth generator (grains round-robin on 8 fields plus the pore
    field, radii 3-8 cells) at 56^3."""
    return pi.grain_growth_pores_3d(n=56, n_grains=60, n_pores=8, dmin=4.0)


WORKLOADS = {"voronoi2d": voronoi_small, "sintering3d": sintering_small, "graingrowth3d": graingrowth_small}


@pytest.mark.parametrize("integ", ["fe", "ssp2", "ssp104", "rkl1", "rkl2"])
@pytest.mark.parametrize("wlname", ["voronoi2d", "sintering3d", "graingrowth3d"])
def test_one_step_fp32_multi_grain_every_integrator(integ, wlname):
    wl = WORKLOADS[wlname]()
    u32, ref, s = one_step(wl, integ, 5)
    check_fp32_multi(wl, u32, ref, s, f"{integ} {wlname}", 2e-5)


def replay(P, integ, u0, trace, ssp):
    """The oracle takes the accepted steps (dt, s) of a GPU run's trace."""
    u = u0
    for h, s, _, acc in trace:
        if acc:
            u, _, _ = oracle.step(P, INTEG[integ], h, u, s=int(s) if integ != "ssp104" else 0)
    return u


@pytest.mark.parametrize("wlname,integ,tolv,tmul", [
    ("sphere3d", "rkl2", 1e-4, 600.0),
    ("sintering3d", "rkl2", 1e-4, 600.0),
    ("graingrowth3d", "rkl2", 1e-4, 600.0),
    ("graingrowth3d", "rkl1", 1e-4, 200.0),
    ("voronoi2d", "ssp2", 1e-4, 30.0),
    ("sintering3d", "ssp104", 1e-4, 40.0),
])
def test_adaptive_fp32_replayed_in_oracle(wlname, integ, tolv, tmul):
    """An FP32 adaptive run (Sec. 3.3) and the oracle taking the same accepted
    steps: the FP32 fields against the FP64 fields, by the bars above."""
    wl = sphere_3d() if wlname == "sphere3d" else WORKLOADS[wlname]()
    P = oracle.Params(**wl.param_dict())
    t_end = tmul * oracle.stable_dt(P)
    sim = pf.Sim(wl.param_dict(), prec="fp32", ssp_stages=3)
    sim.init_fields(wl.u0)
    tol = pf.Tol(r_phi=tolv, a_phi=tolv, r_c=tolv, a_c=tolv)
    st = sim.run_to(integ, t_end, tol=tol)
    u32, t = sim.get_fields()
    tr = sim.trace()
    assert t == t_end and st.accepted >= 3
    ref = replay(P, integ, wl.u0, tr, 3)
    smax = int(tr[tr[:, 3] == 1, 1].max())
    what = f"adaptive {integ} {wlname} ({st.accepted} accepted, {st.rejected} rejected)"
    if wlname == "sphere3d":
        check_fp32_two_phase(wl, u32, ref, what)
    else:
        check_fp32_multi(wl, u32, ref, smax, what, 2e-5)
