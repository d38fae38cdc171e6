"""Fused RKL2 stage pairs through the C-ABI (-m gpu).

Depth 2 computes the inner stages j and j + 1 of eq. sts in one launch with the
single-stage arithmetic, so every result must equal depth 1 bit for bit:

* fixed steps of 3, 5, 9 and 15 stages (the stage count of eq. sts-limit is
  odd, so the inner stages always form pairs), on ragged grids of several
  tiles, grids smaller than one tile (the general wrapping path; one and
  three rows, thinner than the two-cell halo), two- to
  eight-phase workloads in single precision, two-phase in double precision,
  and without c;
* a whole adaptive RKL2 run (same accepted / rejected steps, same fields);
* a single-precision step against the FP64 oracle (1e-4);
* the setting's checks, and the autotuner's choice keeping the bits.
"""
import dataclasses

import numpy as np
import pytest

import oracle
import pf_inputs as pi

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pf = pytest.importorskip("paper_2601_16522_amd")

from _parity import mixed_2d  # noqa: E402


def pores_3d(n=20, nyz=(18, 13), nphi=4):
    return pi.grains_pores_3d(n=n, nyz=nyz, n_grains=5 if nphi <= 4 else 12,
                              n_grain_fields=nphi - 1, n_pores=3, r_range=(2.0, 4.0), dmin=4.0)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    oracle.build(force=False)
    pf.lib()


def voronoi8(n=200, ny=75):
    return pi.voronoi_2d(n=n, ny=ny, n_grains=30, dmin=8.0, seed=4, c_seed=5)


def small4():
    return pi.voronoi_2d(n=24, ny=14, n_grains=4, n_phi=4, dmin=5.0, seed=7, c_seed=8)


def no_c(wl):
    return dataclasses.replace(wl, with_c=False, u0=wl.u0[:wl.n_phi].copy())


WORKLOADS = {
    "voronoi8_fp32": (voronoi8, "fp32"),
    "mixed3_fp32": (mixed_2d, "fp32"),
    "small4_fp32": (small4, "fp32"),
    "grain2_fp32": (lambda: pi.single_grain(n=130, R=40.0, ny=70), "fp32"),
    "grain2_fp64": (lambda: pi.single_grain(n=130, R=40.0, ny=70), "fp64"),
    "voronoi8_noc_fp32": (lambda: no_c(voronoi8(n=150, ny=40)), "fp32"),
    # grids thinner than the two-cell halo: one row, three rows
    "strip2_fp32": (lambda: pi.single_grain(n=97, R=30.0, ny=1), "fp32"),
    "thin4_fp32": (lambda: pi.voronoi_2d(n=70, ny=3, n_grains=5, n_phi=4, dmin=6.0, seed=9, c_seed=10),
                   "fp32"),
}


def dt_for_stages(dte, s):
    """The largest sampled multiple of dt_e whose RKL2 stage count is s."""
    best = None
    for k in np.linspace(0.2, 120.0, 2400):
        if pf.rkl_stage_count("rkl2", k * dte, dte) == s:
            best = k * dte
    assert best is not None, s
    return best


def make(wl, prec, depth):
    sim = pf.Sim(wl.param_dict(), prec=prec)
    sim.init_fields(wl.u0)
    sim.set_stage_fusion(depth)
    assert sim.get_stage_fusion() == depth
    return sim


@pytest.mark.parametrize("s", [3, 5, 9, 15])
@pytest.mark.parametrize("name", list(WORKLOADS))
def test_pairs_equal_single_stages(name, s):
    gen, prec = WORKLOADS[name]
    wl = gen()
    out = {}
    for depth in (1, 2):
        sim = make(wl, prec, depth)
        dt = dt_for_stages(sim.stable_dt(), s)
        sts = [sim.step("rkl2", dt) for _ in range(2)]
        u, t = sim.get_fields()
        sim.close()
        out[depth] = (u, t, [(x.rhs_evals, x.stages) for x in sts])
    print(f"{name} s={s}", flush=True)
    np.testing.assert_array_equal(out[2][0], out[1][0])
    assert out[2][1] == out[1][1]
    assert out[2][2] == out[1][2]


def test_adaptive_run_equal_single_stages():
    wl = voronoi8(n=256, ny=136)
    tol = pf.Tol(r_phi=1e-4, a_phi=1e-2, r_c=1e-4, a_c=1e-4)
    out = {}
    for depth in (1, 2):
        sim = make(wl, "fp32", depth)
        st = sim.run_to("rkl2", 40.0, tol=tol)
        u, t = sim.get_fields()
        sim.close()
        out[depth] = (u, t, st)
    a, b = out[1][2], out[2][2]
    print(f"adaptive: {a.accepted} accepted, {a.rejected} rejected, {a.rhs_evals} RHS", flush=True)
    assert (a.accepted, a.rejected, a.rhs_evals, a.stages) == (b.accepted, b.rejected, b.rhs_evals, b.stages)
    assert a.accepted > 2
    np.testing.assert_array_equal(out[2][0], out[1][0])
    assert out[2][1] == out[1][1] == 40.0


def test_pairs_fp32_against_oracle():
    wl = voronoi8()
    P = oracle.Params(**wl.param_dict())
    dte = oracle.stable_dt(P)
    dt = dt_for_stages(dte, 9)
    s = oracle.stage_count(2, dt, dte)
    assert s == 9
    sim = make(wl, "fp32", 2)
    sim.step("rkl2", dt)
    u, _ = sim.get_fields()
    sim.close()
    ref, _, _ = oracle.step(P, oracle.RKL2, dt, wl.u0, s=s)
    N = wl.n_phi
    assert np.abs(u[:N] - ref[:N]).max() <= 1e-4
    assert np.abs(u[N] - ref[N]).max() <= 1e-4


def test_fusion_setting_checked():
    wl = voronoi8(n=64, ny=16)
    sim = pf.Sim(wl.param_dict(), prec="fp32")
    assert sim.get_stage_fusion() == 2  # the default where pairs are built
    sim.close()
    sim = make(wl, "fp32", 1)
    for bad in (0, 3):
        with pytest.raises(pf.PFError) as e:
            sim.set_stage_fusion(bad)
        assert e.value.code == -1
    sim.set_stage_fusion(2)
    sim.set_stage_fusion(1)
    assert sim.get_stage_fusion() == 1
    sim.close()
    walls = dataclasses.replace(mixed_2d(), bc=[1, 0, 0], c_fixed=[0] * 6, c_bc=[0.0] * 6)
    p13 = pi.grains_pores_3d(n=20, nyz=(18, 13), n_grains=14, n_grain_fields=12, n_pores=3,
                             r_range=(2.0, 4.0), dmin=4.0)
    refused = [(p13, "fp32"), (pores_3d(n=20, nyz=(18, 13), nphi=8), "fp64"), (walls, "fp32"),
               (mixed_2d(), "fp64"), (pi.voronoi_2d(n=64, ny=16, n_grains=12, n_phi=9, dmin=4.0), "fp32")]
    for wl, prec in refused:
        sim = pf.Sim(wl.param_dict(), prec=prec)
        with pytest.raises(pf.PFError) as e:
            sim.set_stage_fusion(2)
        assert e.value.code == -7, (wl.name, prec)
        assert sim.get_stage_fusion() == 1
        sim.close()


def test_autotune_keeps_bits():
    wl = voronoi8(n=256, ny=256)
    sim = pf.Sim(wl.param_dict(), prec="fp32")
    sim.init_fields(wl.u0)
    tx, zc, ms = sim.autotune()
    depth = sim.get_stage_fusion()
    print(f"autotune: depth {depth}, {ms * 1e3:.1f} us per stage", flush=True)
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
