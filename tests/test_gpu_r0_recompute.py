"""RKL2 inner stages of 3D grids that recompute R0 from u^{n,0} read as a
stencil (pf_set_r0_recompute) against the stages that read the stored R0:
the same bits for every supported N, both precisions, 1, 2 and 4 buffer
groups, z extents from 1 to the whole grid, ragged and tiny grids, fixed and
adaptive RKL2 runs (traces included); FP64 against the oracle; the mode's
error paths."""
import numpy as np
import pytest

import oracle
import pf_inputs as pi

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pf = pytest.importorskip("paper_2601_16522_amd")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    oracle.build(force=False)
    pf.lib()


def pores(nphi, n=20, nyz=(18, 13)):
    return pi.grains_pores_3d(n=n, nyz=nyz, n_grains=max(2, nphi + 1), n_grain_fields=nphi - 1, n_pores=3,
                              r_range=(2.0, 4.0), dmin=4.0)


def run(wl, prec, recompute, fn, groups=0, zchunk=5):
    s = pf.Sim(wl.param_dict(), prec=prec)
    if groups:
        s.set_field_groups(groups)
    s.set_tiling(0, zchunk)
    s.set_r0_recompute(recompute)
    assert s.get_r0_recompute() == recompute
    s.init_fields(wl.u0)
    out = fn(s)
    u, t = s.get_fields()
    return u, t, out


def step25(s):
    return s.step("rkl2", 25.0 * s.stable_dt())


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("nphi", [2, 3, 4, 8, 9, 13])
def test_recompute_equals_stored_r0_every_n(nphi, prec):
    wl = pores(nphi)
    assert wl.n_phi == nphi
    if nphi > (9 if prec == "fp32" else 4):  # not built: the mode is refused
        s = pf.Sim(wl.param_dict(), prec=prec)
        with pytest.raises(pf.PFError) as ei:
            s.set_r0_recompute(True)
        assert ei.value.code == -7
        return
    u0, _, st0 = run(wl, prec, False, step25)
    u1, _, st1 = run(wl, prec, True, step25)
    assert np.array_equal(u0, u1), (nphi, prec)
    assert st0.rhs_evals == st1.rhs_evals and st0.stages == st1.stages


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("groups,zchunk", [(1, 1), (2, 4), (4, 64), (2, 1000)])
def test_recompute_any_groups_and_z_extent(groups, zchunk, prec):
    wl = pi.grain_growth_pores_3d(n=24, n_grains=20, n_pores=3, dmin=4.0) if prec == "fp32" else pores(4)
    ref, _, _ = run(wl, prec, False, step25, groups=1, zchunk=5)
    u, _, _ = run(wl, prec, True, step25, groups=groups, zchunk=zchunk)
    assert np.array_equal(ref, u), (groups, zchunk, prec)


@pytest.mark.parametrize("shape", [(1, 1, 1), (2, 1, 3), (1, 4, 1), (5, 2, 2), (3, 70, 1)],
                         ids=lambda s: "x".join(map(str, s)))
def test_recompute_tiny_and_ragged_grids(shape):
    """Grids smaller than a tile or its halo in every direction (general wrap)."""
    nz, ny, nx = shape
    rng = np.random.default_rng(sum(shape))
    cuts = np.sort(rng.integers(0, 9, size=(2,) + shape), axis=0)
    edges = np.concatenate([np.zeros((1,) + shape, int), cuts, np.full((1,) + shape, 8)])
    u0 = np.concatenate([np.diff(edges, axis=0) / 8.0, rng.uniform(0.2, 0.8, (1,) + shape)])
    d = dict(dim=3, nx=nx, ny=ny, nz=nz, n_phi=3, type_of=[0, 1, 1], n_types=2, dx=1.0, W=3.0,
             gamma=[1.0, 0.8, 0.8, 1.2], mob=[1.0, 2.0, 2.0, 0.5], k=[500.0, 300.0], c0=[0.1, 0.9],
             D=[1.0, 0.3], with_c=True)
    wl = pi.Workload("tiny", 3, nx, ny, nz, 3, [0, 1, 1], 2, 1.0, 3.0, [1.0, 0.8, 0.8, 1.2],
                     [1.0, 2.0, 2.0, 0.5], [500.0, 300.0], [0.1, 0.9], [1.0, 0.3], True, u0)
    assert wl.param_dict() == d
    for prec in ("fp32", "fp64"):
        for zc in (1, 4):
            ref, _, _ = run(wl, prec, False, step25, zchunk=zc)
            u, _, _ = run(wl, prec, True, step25, zchunk=zc)
            assert np.array_equal(ref, u), (shape, prec, zc)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_recompute_adaptive_run_same_trace(prec):
    wl = pores(4)
    tol = pf.Tol(r_phi=1e-4, a_phi=1e-4, r_c=1e-4, a_c=1e-4)

    def adaptive(s):
        st = s.run_to("rkl2", 150.0 * s.stable_dt(), tol=tol)
        return st, s.trace()

    u0, t0, (st0, tr0) = run(wl, prec, False, adaptive)
    u1, t1, (st1, tr1) = run(wl, prec, True, adaptive)
    assert st0.accepted > 3 and t0 == t1
    assert np.array_equal(tr0, tr1) and np.array_equal(u0, u1)
    assert st0.rhs_evals == st1.rhs_evals


def test_recompute_fp64_matches_oracle():
    wl = pores(4)
    P = oracle.Params(**wl.param_dict())
    dte = oracle.stable_dt(P)
    dt = 25.0 * dte
    ref, _, _ = oracle.step(P, oracle.RKL2, dt, wl.u0, s=oracle.stage_count(2, dt, dte))
    u, _, _ = run(wl, "fp64", True, step25)
    N = wl.n_phi
    assert np.abs(u[:N] - ref[:N]).max() <= 1e-10
    assert np.abs(u[N] - ref[N]).max() <= 1e-10 * max(1.0, np.abs(ref[N]).max())


def test_recompute_errors_and_autotune():
    s2 = pf.Sim(pi.single_grain(n=32, R=10.0).param_dict(), prec="fp32")
    with pytest.raises(pf.PFError) as ei:
        s2.set_r0_recompute(True)
    assert ei.value.code == -7
    walled = dict(pores(3).param_dict(), bc=[1, 0, 0], c_fixed=[0] * 6, c_bc=[0.0] * 6)
    sw = pf.Sim(walled, prec="fp32")
    with pytest.raises(pf.PFError) as ei:
        sw.set_r0_recompute(True)
    assert ei.value.code == -7
    # the autotuner may pick either form; the result bits do not depend on it
    wl = pores(4)
    ref, _, _ = run(wl, "fp32", False, step25)
    s = pf.Sim(wl.param_dict(), prec="fp32")
    s.init_fields(wl.u0)
    s.autotune()
    step25(s)
    u, _ = s.get_fields()
    assert np.array_equal(ref, u), s.get_r0_recompute()
    # sparse storage turns the mode off in effect (dense stages only)
    a = pf.Sim(wl.param_dict(), prec="fp32")
    a.set_r0_recompute(True)
    a.set_sparse_storage(4)
    a.init_fields(wl.u0)
    step25(a)
    b = pf.Sim(wl.param_dict(), prec="fp32")
    b.set_sparse_storage(4)
    b.init_fields(wl.u0)
    step25(b)
    assert np.array_equal(a.get_fields()[0], b.get_fields()[0])
