"""Walls through the C-ABI against the FP64 oracle (-m gpu): axes that end in
zero-gradient walls for phi and c, and wall faces that hold c fixed in their
ghost cell (the Dirichlet walls of the solutal Stefan problem, Sec. 5.2.2).

* The right-hand side and one step of several integrators on a ragged
  three-phase 2D grid (walls in x and y, fixed c on two faces; walls in x
  only) and on a 3D grains + pores grid (walls in x and z, fixed c on both z
  faces, also with z chunks smaller than the grid), FP64 within 1e-10.
* The Stefan workload: adaptive RKL2, FP64 against the oracle replaying the
  GPU's accepted steps, FP32 interface position against FP64.
* Parameter checks: walls on z of a 2D grid, a fixed c on a periodic axis, and
  a batch of walled instances are refused.
"""
import dataclasses

import numpy as np
import pytest

import oracle
import pf_inputs as pi

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pf = pytest.importorskip("paper_2601_16522_amd")

from test_gpu_parity import check_fp64, mixed_2d, pores_3d  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    oracle.build(force=False)
    pf.lib()


def walled(wl, bc, fixed=(), values=None):
    cf = [0] * 6
    cb = [0.0] * 6
    for f in fixed:
        cf[f] = 1
        cb[f] = values[f]
    return dataclasses.replace(wl, bc=list(bc), c_fixed=cf, c_bc=cb)


CASES = {
    "2d_xy_fixed": lambda: walled(mixed_2d(), (1, 1, 0), (0, 3), {0: 0.3, 3: 0.7}),
    "2d_x": lambda: walled(mixed_2d(), (1, 0, 0)),
    "2d_small_y_fixed": lambda: walled(mixed_2d(nx=33, ny=50, seed=5), (0, 1, 0), (2, 3), {2: 0.2, 3: 0.8}),
    "3d_xz_fixed": lambda: walled(pores_3d(), (1, 0, 1), (4, 5), {4: 0.0, 5: 1.0}),
}


def make(wl, prec="fp64", zchunk=0):
    sim = pf.Sim(wl.param_dict(), prec=prec, ssp_stages=3)
    sim.init_fields(wl.u0)
    if zchunk:
        sim.set_tiling(0, zchunk)
    return sim


@pytest.mark.parametrize("case", list(CASES))
def test_rhs_with_walls_fp64(case):
    wl = CASES[case]()
    for zc in ((0, 4) if wl.dim == 3 else (0,)):
        sim = make(wl, zchunk=zc)
        r = sim.rhs()
        sim.close()
        ref = oracle.rhs(oracle.Params(**wl.param_dict()), wl.u0)
        scale = np.abs(ref).max(axis=(1, 2, 3), keepdims=True)
        err = np.abs(r - ref) / np.maximum(scale, 1e-300)
        assert err.max() <= 1e-12, (case, zc, err.max())


@pytest.mark.parametrize("integ", ["fe", "rkl2", "ssp104"])
@pytest.mark.parametrize("case", list(CASES))
def test_one_step_with_walls_fp64(case, integ):
    wl = CASES[case]()
    P = oracle.Params(**wl.param_dict())
    dte = oracle.stable_dt(P)
    dt = {"fe": 0.9, "rkl2": 25.0, "ssp104": 4.0}[integ] * dte
    s = oracle.stage_count(2, dt, dte) if integ == "rkl2" else 0
    ref, _, _ = oracle.step(P, {"fe": oracle.FE, "rkl2": oracle.RKL2, "ssp104": oracle.SSP104}[integ],
                            dt, wl.u0, s=s)
    for zc in ((0, 4) if wl.dim == 3 else (0,)):
        sim = make(wl, zchunk=zc)
        sim.step(integ, dt)
        u, _ = sim.get_fields()
        sim.close()
        check_fp64(wl, u, ref, (case, integ, zc))


def _position(u):
    a = u[0, 0, 0]
    i = int(np.where((a[:-1] - 0.5) * (a[1:] - 0.5) <= 0)[0][0])
    return i + (0.5 - a[i]) / (a[i + 1] - a[i])


def test_stefan_adaptive_rkl2():
    """The solutal Stefan workload to t = 6000.  Its first steps are rejected
    often, so norms a few ulps apart may take a decision the other way;
    the FP64 run is therefore checked in replay: the oracle takes the GPU's
    accepted (dt, s) sequence and must end within 1e-10 of the GPU's fields,
    and the counts of accepted and rejected steps must agree with the
    oracle's own adaptive run to within 10%.  FP32 puts the interface within
    0.02 cells of FP64's."""
    wl = pi.stefan_1d()
    P = oracle.Params(**wl.param_dict())
    tol = dict(r_phi=1e-4, a_phi=1e-2, r_c=1e-4, a_c=1e-4)
    _, st_ref, rc = oracle.run_to(P, oracle.RKL2, wl.u0, 6000.0, tol=oracle.Tol(**tol))
    assert rc == 0
    pos = {}
    for prec in ("fp64", "fp32"):
        sim = make(wl, prec=prec)
        st = sim.run_to("rkl2", 6000.0, tol=pf.Tol(**tol))
        u, t = sim.get_fields()
        tr = sim.trace()
        sim.close()
        assert t == 6000.0
        pos[prec] = _position(u)
        if prec == "fp64":
            assert abs(st.accepted - st_ref.accepted) <= max(2, st_ref.accepted // 10)
            assert abs(st.rejected - st_ref.rejected) <= max(2, st_ref.rejected // 10)
            ref = oracle._state(P, wl.u0).copy()
            for h, s, _, acc in tr:
                if acc:
                    ref, _, _ = oracle.step(P, oracle.RKL2, float(h), ref, s=int(s))
            check_fp64(wl, u, ref, "stefan replay")
    print(f"\nStefan interface at t = 6000: FP64 {pos['fp64']:.5f}, FP32 {pos['fp32']:.5f}", flush=True)
    assert abs(pos["fp32"] - pos["fp64"]) < 0.02


def test_wall_parameters_checked():
    wl = mixed_2d()
    with pytest.raises(pf.PFError) as e:
        pf.Sim(walled(wl, (0, 0, 1)).param_dict())
    assert e.value.code == -1
    bad = dict(walled(wl, (1, 0, 0)).param_dict(), c_fixed=[0, 0, 1, 0, 0, 0])
    with pytest.raises(pf.PFError) as e:
        pf.Sim(bad)
    assert e.value.code == -1
    one = pi.single_grain(n=64, R=20.0)
    with pytest.raises(pf.PFError) as e:
        pf.Batch([walled(one, (1, 0, 0)).param_dict()], prec="fp32")
    assert e.value.code == -7
