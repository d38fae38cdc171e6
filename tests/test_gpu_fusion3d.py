"""Fused RKL2 stage pairs in 3D through the C-ABI (-m gpu).

The 3D pair kernel computes stage j on a 32 x 8 tile and its one-cell ring
one plane ahead of stage j + 1 on the tile, marching a z extent, with the
single-stage arithmetic; every result must equal depth 1 bit for bit:

* fixed RKL2 steps of 3, 5 and 9 stages, two steps each, on grids ragged in
  x and y against the tile, grids thinner than the tile and the two-cell
  halo in y and z, z extents of 1, 2, 3, 5 and more than the grid, two to
  nine phases in single precision, two and four in double precision, without
  c, and with the vectors forced into two and four buffer groups;
* a whole adaptive RKL2 run;
* single-precision steps against the FP64 oracle, double-precision steps
  within 1e-10 of it.
"""
import dataclasses

import numpy as np
import pytest

import oracle
import pf_inputs as pi
from _parity import check_fp32_multi, check_fp32_two_phase

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pf = pytest.importorskip("paper_2601_16522_amd")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    oracle.build(force=False)
    pf.lib()


def pores(n=45, nyz=(19, 13), nphi=4, seed=4):
    return pi.grains_pores_3d(n=n, nyz=nyz, n_grains=6 if nphi <= 4 else 14,
                              n_grain_fields=nphi - 1, n_pores=4, r_range=(2.0, 4.0), dmin=4.0,
                              seed_grains=seed)


def sphere(n=36, nyz=None, r=9.0):
    """Two phases: a pore sphere (tanh profile) in one grain, mobile-pore
    parameters, c = phi_pore."""
    ny, nz = (n, n) if nyz is None else nyz
    dx, W, _, gamma, mob, k, c0, D = pi._pore_params(1)
    z, y, x = np.meshgrid(np.arange(nz, dtype=float), np.arange(ny, dtype=float),
                          np.arange(n, dtype=float), indexing="ij")
    d = r - np.sqrt((x - n / 2) ** 2 + (y - ny / 2) ** 2 + (z - nz / 2) ** 2)
    pore = pi.tanh_profile(d, W / dx)
    u0 = np.stack([1.0 - pore, pore, pore.copy()])
    return pi.Workload("sphere3d", 3, n, ny, nz, 2, [0, 1], 2, dx, W, gamma, mob, k, c0, D, True, u0)


def no_c(wl):
    return dataclasses.replace(wl, with_c=False, u0=wl.u0[:wl.n_phi].copy())


WORKLOADS = {
    "pores4_fp32": (lambda: pores(), "fp32", 0),
    "gg9_fp32": (lambda: pi.grain_growth_pores_3d(n=40, nyz=(24, 20), n_grains=40, n_pores=4), "fp32", 0),
    "gg9_fp32_g2": (lambda: pi.grain_growth_pores_3d(n=40, nyz=(24, 20), n_grains=40, n_pores=4), "fp32", 2),
    "gg9_fp32_g4": (lambda: pi.grain_growth_pores_3d(n=33, nyz=(17, 9), n_grains=30, n_pores=3), "fp32", 4),
    "sphere2_fp32": (lambda: sphere(), "fp32", 0),
    "sphere2_fp64": (lambda: sphere(), "fp64", 0),
    "pores4_fp64": (lambda: pores(n=37, nyz=(11, 10)), "fp64", 0),
    "pores3_noc_fp32": (lambda: no_c(pores(nphi=3)), "fp32", 0),
    "pores8_fp32": (lambda: pores(n=34, nyz=(16, 12), nphi=8), "fp32", 0),
    # thinner than the tile and the two-cell halo: 5 rows, 2 planes, 1 plane
    "thin_y5_fp32": (lambda: pores(n=40, nyz=(5, 12)), "fp32", 0),
    "thin_z2_fp32": (lambda: pores(n=40, nyz=(20, 2)), "fp32", 0),
    "thin_z1_fp64": (lambda: sphere(n=40, nyz=(20, 1)), "fp64", 0),
}


def dt_for_stages(dte, s):
    best = None
    for k in np.linspace(0.2, 60.0, 1200):
        if pf.rkl_stage_count("rkl2", k * dte, dte) == s:
            best = k * dte
    assert best is not None, s
    return best


def make(wl, prec, depth, groups=0, zc=None):
    sim = pf.Sim(wl.param_dict(), prec=prec)
    if groups:
        sim.set_field_groups(groups)
    sim.init_fields(wl.u0)
    sim.set_stage_fusion(depth)
    assert sim.get_stage_fusion() == depth
    if zc is not None:
        sim.set_pair_zchunk(zc)
    return sim


@pytest.mark.parametrize("name", list(WORKLOADS))
def test_pairs_equal_single_stages_3d(name):
    gen, prec, groups = WORKLOADS[name]
    wl = gen()
    for s in (3, 5, 9):
        ref = make(wl, prec, 1, groups)
        dt = dt_for_stages(ref.stable_dt(), s)
        st_ref = [ref.step("rkl2", dt) for _ in range(2)]
        u_ref, t_ref = ref.get_fields()
        ref.close()
        for zc in (1, 2, 3, 5, 64):
            sim = make(wl, prec, 2, groups, zc)
            sts = [sim.step("rkl2", dt) for _ in range(2)]
            u, t = sim.get_fields()
            sim.close()
            np.testing.assert_array_equal(u, u_ref, err_msg=f"{name} s={s} zchunk={zc}")
            assert t == t_ref
            assert [(x.rhs_evals, x.stages) for x in sts] == [(x.rhs_evals, x.stages) for x in st_ref]
    print(f"{name}: pairs equal single stages at s = 3, 5, 9, z extents 1, 2, 3, 5, 64", flush=True)


def test_adaptive_run_equal_single_stages_3d():
    wl = pi.grain_growth_pores_3d(n=48, n_grains=50, n_pores=5)
    tol = pf.Tol(r_phi=1e-4, a_phi=1e-4, r_c=1e-4, a_c=1e-4)
    dte = pf.params_stable_dt(wl.param_dict())
    out = {}
    for depth in (1, 2):
        sim = make(wl, "fp32", depth, zc=16)
        st = sim.run_to("rkl2", 800 * dte, tol=tol)
        u, t = sim.get_fields()
        sim.close()
        out[depth] = (u, t, st)
    a, b = out[1][2], out[2][2]
    print(f"adaptive 3D: {a.accepted} accepted, {a.rejected} rejected, {a.rhs_evals} RHS", flush=True)
    assert (a.accepted, a.rejected, a.rhs_evals, a.stages) == (b.accepted, b.rejected, b.rhs_evals, b.stages)
    assert a.accepted > 2
    np.testing.assert_array_equal(out[2][0], out[1][0])
    assert out[2][1] == out[1][1]


@pytest.mark.parametrize("name", ["sphere2_fp32", "gg9_fp32", "sphere2_fp64", "pores4_fp64"])
def test_pairs_3d_against_oracle(name):
    gen, prec, groups = WORKLOADS[name]
    wl = gen()
    P = oracle.Params(**wl.param_dict())
    dte = oracle.stable_dt(P)
    dt = dt_for_stages(dte, 9)
    s = oracle.stage_count(2, dt, dte)
    assert s == 9
    sim = make(wl, prec, 2, groups, 4)
    sim.step("rkl2", dt)
    u, _ = sim.get_fields()
    sim.close()
    ref, _, _ = oracle.step(P, oracle.RKL2, dt, wl.u0, s=s)
    N = wl.n_phi
    if prec == "fp64":
        assert np.abs(u[:N] - ref[:N]).max() <= 1e-10
        assert np.abs(u[N] - ref[N]).max() <= 1e-10 * max(1.0, np.abs(ref[N]).max())
    elif N == 2:
        check_fp32_two_phase(wl, u, ref, f"3D pairs {name}")
    else:
        check_fp32_multi(wl, u, ref, s, f"3D pairs {name}", 2e-5)


def test_pair_zchunk_setting():
    wl = pores()
    sim = pf.Sim(wl.param_dict(), prec="fp32")
    assert sim.get_stage_fusion() == 1  # in 3D the autotuner decides
    sim.set_stage_fusion(2)
    assert sim.get_pair_zchunk() == 32
    sim.set_pair_zchunk(7)
    assert sim.get_pair_zchunk() == 7
    with pytest.raises(pf.PFError) as e:
        sim.set_pair_zchunk(0)
    assert e.value.code == -1
    sim.close()


def test_autotune_keeps_bits_3d():
    wl = pi.grain_growth_pores_3d(n=64, n_grains=60, n_pores=6)
    sim = pf.Sim(wl.param_dict(), prec="fp32")
    sim.init_fields(wl.u0)
    tx, zc, ms = sim.autotune()
    depth, zc2 = sim.get_stage_fusion(), sim.get_pair_zchunk()
    print(f"autotune 3D: depth {depth}, z extents {zc} / {zc2}, {ms * 1e3:.1f} us per stage", flush=True)
    assert depth in (1, 2) and ms > 0
    dt = dt_for_stages(sim.stable_dt(), 7)
    sim.step("rkl2", dt)
    u, _ = sim.get_fields()
    sim.close()
    ref = make(wl, "fp32", 1)
    ref.step("rkl2", dt)
    v, _ = ref.get_fields()
    ref.close()
    np.testing.assert_array_equal(u, v)
