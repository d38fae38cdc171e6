"""LDS poison: the debug library libpf_poison.so holds the same kernels as
libpf.so for N in {2, 4, 9} and one or two buffer groups, built so that every
LDS region (plane tiles, halo regions, the stage pairs' ring planes, the
tables) is filled with NaN before the block writes it.  A kernel that reads an
LDS element no thread wrote for the current tile or plane -- a halo cell
missed on a ragged edge, a stale plane of the z march -- would carry that NaN
into its results.  Every case runs on both libraries from the same input; the
results must agree bit for bit and be finite (FP64 cases are also held to the
oracle at 1e-10).  Cases cover every stage kind (FE, SSP(3)2, SSP(10)4, RKL1,
RKL2 first and inner stages, the estimator), the 64 x 8 and 64 x 4 tiles on
ragged 2D grids, 3D z chunks that do not divide nz, fused RKL2 stage pairs in
2D and 3D, the 3D stages that recompute R0, two buffer groups, sparse phase
storage and the batched kernels at both fusion depths."""
import os

import numpy as np
import pytest

import oracle
import pf_inputs as pi

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pf = pytest.importorskip("paper_2601_16522_amd")

POISON = os.path.join(os.path.dirname(pf.LIB_PATH), "libpf_poison.so")
INTEG = {"fe": oracle.FE, "ssp2": oracle.SSP2, "ssp104": oracle.SSP104, "rkl1": oracle.RKL1,
         "rkl2": oracle.RKL2}
MULT = {"fe": 0.9, "ssp2": 1.5, "ssp104": 4.0, "rkl1": 12.0, "rkl2": 40.0}


@pytest.fixture(scope="module")
def libs():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(POISON):
        pytest.fail(f"{POISON} is not built; run paper_2601_16522_amd/build.py")
    regular = pf.lib()
    mp = pytest.MonkeyPatch()
    mp.setattr(pf, "LIB_PATH", POISON)
    mp.setattr(pf, "_lib", None)
    poisoned = pf.lib()
    assert pf.supported_nphi() == [2, 4, 9]
    mp.setattr(pf, "_lib", regular)  # new handles use libpf.so unless a case switches
    yield regular, poisoned
    mp.undo()


def _on(lib, fn):
    """Runs fn() with new handles made on lib."""
    old = pf._lib
    pf._lib = lib
    try:
        return fn()
    finally:
        pf._lib = old


def four_phase_2d(nx=70, ny=45, seed=5):
    rng = np.random.default_rng(seed)
    seeds = pi.seeds_min_distance(8, (nx, ny), 8.0, rng)
    phi = pi.voronoi_fields((1, ny, nx), seeds, 4, 3.0)
    c0 = [0.1, 0.9]
    tof = [0, 1, 0, 1]
    c = sum(phi[a] * c0[tof[a]] for a in range(4)) + rng.normal(0, 0.01, size=phi[0].shape)
    return pi.Workload("four2d", 2, nx, ny, 1, 4, tof, 2, 1.0, 3.0, [1.0, 0.8, 0.8, 1.2],
                       [1.0, 2.0, 2.0, 0.5], [500.0, 300.0], c0, [1.0, 0.3], True,
                       np.concatenate([phi, c[None]]))


def nine_phase_3d():
    return pi.grain_growth_pores_3d(n=36, n_grains=40, n_grain_fields=8, n_pores=6, r_range=(2.0, 4.0),
                                    dmin=4.0, nyz=(30, 23))


def four_phase_3d():
    return pi.grains_pores_3d(n=20, nyz=(18, 13), n_grains=5, n_grain_fields=3, n_pores=3,
                              r_range=(2.0, 4.0), dmin=5.0)


def _both(libs, wl, prec, run):
    out = []
    for L in libs:
        def go():
            sim = pf.Sim(wl.param_dict(), prec=prec, ssp_stages=3)
            sim.init_fields(wl.u0)
            run(sim)
            return sim.get_fields()[0], sim.diagnostics()["nonfinite"]
        out.append(_on(L, go))
    (a, na), (b, nb) = out
    assert na == 0 and nb == 0, (na, nb)
    assert np.array_equal(a, b), np.abs(a - b).max()
    return a


CASES = [("two2d", lambda: pi.single_grain(n=40, R=12.0)), ("four2d", four_phase_2d),
         ("four3d", four_phase_3d), ("nine3d", nine_phase_3d)]


@pytest.mark.parametrize("integ", list(INTEG))
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", [c[0] for c in CASES])
def test_every_stage_kind_sees_no_unwritten_lds(libs, case, prec, integ):
    wl = dict(CASES)[case]()
    P = oracle.Params(**wl.param_dict())
    dte = oracle.stable_dt(P)
    dt = MULT[integ] * dte
    zc = {"four3d": 5, "nine3d": 7}.get(case)

    def run(sim):
        if zc:
            sim.set_tiling(0, zc)  # z chunks that do not divide nz
        sim.step(integ, dt)

    u = _both(libs, wl, prec, run)
    if prec == "fp64":
        s = {"ssp2": 3}.get(integ, 0)
        if integ in ("rkl1", "rkl2"):
            s = oracle.stage_count(1 if integ == "rkl1" else 2, dt, dte)
        ref, _, _ = oracle.step(P, INTEG[integ], dt, wl.u0, s=s)
        assert np.abs(u - ref).max() <= 1e-10 * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("case", ["two2d", "four3d"])
def test_estimator_sees_no_unwritten_lds(libs, case, prec):
    wl = dict(CASES)[case]()
    tol = pf.Tol(1e-4, 1e-2, 1e-4, 1e-4)
    t_end = 30.0 * oracle.stable_dt(oracle.Params(**wl.param_dict()))
    traces = []

    def run(sim):
        sim.run_to("rkl2", t_end, tol=tol)
        traces.append(sim.trace())

    _both(libs, wl, prec, run)
    assert np.array_equal(traces[0], traces[1])


@pytest.mark.parametrize("prec,case", [("fp32", "four2d"), ("fp64", "two2d"), ("fp32", "nine3d"),
                                       ("fp64", "four3d")])
def test_fused_stage_pairs_see_no_unwritten_lds(libs, prec, case):
    wl = dict(CASES)[case]()
    dt = 60.0 * oracle.stable_dt(oracle.Params(**wl.param_dict()))

    def run(sim):
        sim.set_stage_fusion(2)
        if wl.dim == 3:
            sim.set_pair_zchunk(6)
        sim.step("rkl2", dt)

    _both(libs, wl, prec, run)


@pytest.mark.parametrize("prec,case", [("fp32", "nine3d"), ("fp64", "four3d"), ("fp32", "four3d")])
def test_r0_recompute_stages_see_no_unwritten_lds(libs, prec, case):
    """The 3D stages that recompute R0 stage two planes (Y_{j-1} and u0) in LDS."""
    wl = dict(CASES)[case]()
    dt = 40.0 * oracle.stable_dt(oracle.Params(**wl.param_dict()))

    def run(sim):
        sim.set_r0_recompute(True)
        sim.set_tiling(0, 5)  # z chunks that do not divide nz
        sim.step("rkl2", dt)

    u = _both(libs, wl, prec, run)

    def stored(sim):
        sim.set_tiling(0, 5)
        sim.step("rkl2", dt)

    assert np.array_equal(u, _both(libs, wl, prec, stored))


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_two_buffer_groups_see_no_unwritten_lds(libs, prec):
    wl = nine_phase_3d()
    dt = 40.0 * oracle.stable_dt(oracle.Params(**wl.param_dict()))

    def run(sim):
        sim.set_field_groups(2)
        sim.step("rkl2", dt)
        sim.step("ssp104", 4.0 * dt / 40.0)

    _both(libs, wl, prec, run)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_sparse_storage_sees_no_unwritten_lds(libs, prec):
    wl = four_phase_3d()
    dt = 40.0 * oracle.stable_dt(oracle.Params(**wl.param_dict()))

    def run(sim):
        sim.set_sparse_storage(2)
        sim.init_fields(wl.u0)
        sim.step("rkl2", dt)
        sim.step("fe", 0.9 * dt / 40.0)

    _both(libs, wl, prec, run)


@pytest.mark.parametrize("depth", [1, 2])
def test_batch_kernels_see_no_unwritten_lds(libs, depth):
    wls = pi.batch_instances(count=5, seed=3, sides=(40, 72, 100))
    res = []
    for L in libs:
        def go():
            b = pf.Batch([w.param_dict() for w in wls], prec="fp32")
            for i, w in enumerate(wls):
                b.init_fields(i, w.u0)
            b.set_fusion(depth)
            dts = np.array([b.stable_dt(i) for i in range(len(wls))])
            b.run_to(7.5 * 0.9 * dts)
            b.run_to(7.5 * 0.9 * dts + 3.5 * 30 * dts, dt=30 * dts, integ="rkl2")
            te = 7.5 * 0.9 * dts + 3.5 * 30 * dts + 20 * dts
            b.run_adaptive(te, pf.Tol(1e-4, 1e-2, 1e-4, 1e-4))
            out = [b.get_fields(i)[0] for i in range(len(wls))]
            b.close()
            return out
        res.append(_on(L, go))
    for a, b in zip(*res):
        assert np.isfinite(a).all() and np.array_equal(a, b)
