"""The allocation-free error norm (pf_error_norm_device_noalloc) against the
device error norm it mirrors (pf_error_norm_device): the same kernels and the
same partial-sum order, so the same norm and degree-of-freedom count bit for
bit.  Two calls in a row per case, the second on a smaller grid, share the
static scratch the first left behind."""
import numpy as np
import pytest

import pf_inputs as pi

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pf = pytest.importorskip("paper_2601_16522_amd")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pf.lib()


def _vectors(wl, prec, zchunk):
    sim = pf.Sim(wl.param_dict(), prec=prec, ssp_stages=3)
    if wl.dim == 3:
        sim.set_tiling(0, zchunk)
    sim.init_fields(wl.u0)
    u_old, aux, u_new = sim.empty_device(), sim.empty_device(), sim.empty_device()
    sim.get_fields_device(u_old)
    sim.rhs_device(aux)
    dt = 40.0 * sim.stable_dt()
    sim.step("rkl2", dt)
    sim.get_fields_device(u_new)
    return sim, dt, u_old, u_new, aux


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_noalloc_norm_equals_device_norm(prec):
    big = pi.grains_pores_3d(n=64, n_grains=12, n_grain_fields=12, n_pores=8, dmin=10.0)
    small = pi.single_grain(n=40, R=12.0)
    tol = pf.Tol(r_phi=1e-4, a_phi=1e-3, r_c=1e-4, a_c=1e-4)
    for kind in (0, 1):
        for wl, zc in ((big, 1), (small, 1)):   # z extent 1: 1024 tiles at 64^3
            sim, dt, u_old, u_new, aux = _vectors(wl, prec, zc)
            ref = sim.error_norm(kind, dt, u_old, u_new, aux, tol)
            got = sim.error_norm_noalloc(kind, dt, u_old, u_new, aux, tol)
            again = sim.error_norm_noalloc(kind, dt, u_old, u_new, aux, tol)
            print(f"\n{prec} kind {kind} {wl.name}: norm {got[0]!r} ({got[1]} DoF)", flush=True)
            assert got == ref and again == ref, (kind, wl.name, got, ref)
            assert np.isfinite(got[0]) and got[0] > 0 and got[1] > 0


def test_noalloc_norm_refuses_more_partials_than_the_scratch_holds():
    # 2 x 65537 tiles of 64 x 4 cells at z extent 1: two more partials than
    # 2 MiB holds
    p = dict(pi.grains_pores_3d(n=16, n_grains=2, n_grain_fields=1, n_pores=1,
                                r_range=(2.0, 3.0), dmin=4.0).param_dict())
    p.update(nx=128, ny=4, nz=65537)
    sim = pf.Sim(p, prec="fp32")
    sim.set_tiling(0, 1)
    vec = sim.empty_device()
    tol = pf.Tol()
    with pytest.raises(pf.PFError) as ei:
        sim.error_norm_noalloc(0, 1.0, vec, vec, vec, tol)
    assert ei.value.code == -1 and "static scratch" in str(ei.value)
    # the embedded estimate needs 1024 partials whatever the grid
    vec.copy_(torch.zeros_like(vec))
    n, ndof = sim.error_norm_noalloc(1, 1.0, vec, vec, vec, tol)
    assert n == 0.0 and ndof == 2 * sim.V + sim.V
