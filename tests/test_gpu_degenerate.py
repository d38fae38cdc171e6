"""Degenerate grids, states and parameters on the GPU, through the C-ABI.

* Grids of one cell, one row or one column (2D) and of one cell or a few cells
  per axis (3D): every periodic neighbour is the cell itself or wraps onto the
  same few cells, and the tile, halo and z-march logic meets its smallest
  cases.  FP64 against the oracle (1e-10); both precisions against the same
  state tiled periodically onto a grid of ordinary size, whose cells must
  evolve bit for bit like the tiny grid's (translation invariance of the
  periodic stencil: every cell sees the same neighbour values in the same
  order).
* A state in pure bulk (one phase per cell, uniform c): the right-hand side is
  exactly zero and every integrator keeps phi; c moves by rounding at most.
* Zero pair mobility and diffusivity: dt_e is infinite, the right-hand side
  zero, and runs land on t_end in one clipped step (reading R18); a single
  step of infinite size and a non-finite t_end are refused.
"""
import math

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
pf = pytest.importorskip("paper_2601_16522_amd")

INTEG = {"fe": oracle.FE, "ssp2": oracle.SSP2, "ssp104": oracle.SSP104, "rkl1": oracle.RKL1,
         "rkl2": oracle.RKL2}
DT_OVER_DTE = {"fe": 0.9, "ssp2": 1.5, "ssp104": 4.0, "rkl1": 12.0, "rkl2": 25.0}

# (dim, (nz, ny, nx))
TINY = [(2, (1, 1, 1)), (2, (1, 1, 5)), (2, (1, 6, 1)), (2, (1, 3, 2)), (2, (1, 2, 67)),
        (3, (1, 1, 1)), (3, (2, 1, 3)), (3, (1, 4, 1)), (3, (5, 2, 2)), (3, (3, 1, 1))]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    oracle.build(force=False)
    pf.lib()


def params(dim, shape, n_phi=3, mob=None, D=None):
    nz, ny, nx = shape
    return dict(dim=dim, nx=nx, ny=ny, nz=nz, n_phi=n_phi, type_of=[0] + [1] * (n_phi - 1),
                n_types=2, dx=1.0, W=3.0, gamma=[1.0, 0.8, 0.8, 1.2],
                mob=mob if mob is not None else [1.0, 2.0, 2.0, 0.5], k=[500.0, 300.0],
                c0=[0.1, 0.9], D=D if D is not None else [1.0, 0.3], with_c=True)


def state(rng, n_phi, shape):
    """phi in multiples of 1/8 summing to 1 exactly per cell (exact zeros in
    places), c in [0.2, 0.8]."""
    cuts = np.sort(rng.integers(0, 9, size=(n_phi - 1,) + shape), axis=0)
    edges = np.concatenate([np.zeros((1,) + shape, int), cuts, np.full((1,) + shape, 8)])
    phi = np.diff(edges, axis=0) / 8.0
    return np.concatenate([phi, rng.uniform(0.2, 0.8, (1,) + shape)])


def pairs_built(d, prec):
    """Whether fused RKL2 stage pairs are built for these parameters."""
    s = pf.Sim(d, prec=prec, ssp_stages=3)
    try:
        s.set_stage_fusion(2)
        return True
    except pf.PFError as e:
        assert e.code == -7
        return False


def sim_of(d, u, prec, fusion=1):
    s = pf.Sim(d, prec=prec, ssp_stages=3)
    s.set_tiling(0, 4)
    s.set_stage_fusion(fusion)
    s.init_fields(u)
    return s


def check_fp64(u, ref, n_phi, what):
    assert np.abs(u[:n_phi] - ref[:n_phi]).max() <= 1e-10, what
    scale = max(1.0, np.abs(ref[n_phi]).max())
    assert np.abs(u[n_phi] - ref[n_phi]).max() <= 1e-10 * scale, what


@pytest.mark.parametrize("dim,shape", TINY, ids=[f"{d}d_" + "x".join(map(str, s)) for d, s in TINY])
def test_tiny_grid_fp64_matches_oracle(dim, shape):
    d = params(dim, shape)
    rng = np.random.default_rng(100 * dim + 10 * sum(shape) + shape[2])
    u0 = state(rng, 3, shape)
    P = oracle.Params(**d)
    dte = oracle.stable_dt(P)
    s = sim_of(d, u0, "fp64")
    assert s.stable_dt() == dte
    ref_r = oracle.rhs(P, u0)
    r = s.rhs()
    scale = np.maximum(np.abs(ref_r).max(axis=(1, 2, 3), keepdims=True), 1e-300)
    assert (np.abs(r - ref_r) / scale).max() <= 1e-12, shape
    for name, integ in INTEG.items():
        dt = DT_OVER_DTE[name] * dte
        ns = {"ssp2": 3, "ssp104": 0}.get(name, 0)
        if name in ("rkl1", "rkl2"):
            ns = oracle.stage_count(1 if name == "rkl1" else 2, dt, dte)
        ref, _, _ = oracle.step(P, integ, dt, u0, s=ns)
        fusions = (1, 2) if name == "rkl2" and pairs_built(d, "fp64") else (1,)
        for fu in fusions:
            g = sim_of(d, u0, "fp64", fusion=fu)
            g.step(name, dt)
            u, _ = g.get_fields()
            check_fp64(u, ref, 3, (shape, name, fu))


def tile_up(u, reps):
    return np.tile(u, (1,) + reps)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("dim,shape,reps", [
    (2, (1, 1, 1), (1, 9, 70)), (2, (1, 1, 5), (1, 9, 14)), (2, (1, 6, 1), (1, 2, 66)),
    (2, (1, 3, 2), (1, 4, 35)), (3, (1, 1, 1), (6, 9, 70)), (3, (2, 1, 3), (3, 9, 23)),
    (3, (5, 2, 2), (1, 5, 33))], ids=lambda v: "x".join(map(str, v)) if isinstance(v, tuple) else str(v))
def test_tiny_grid_equals_its_periodic_tiling(dim, shape, reps, prec):
    """The tiny grid's cells evolve bit for bit like the cells of the same state
    repeated periodically on a grid of ordinary size, for every stage kind and
    for fused RKL2 stage pairs."""
    d = params(dim, shape)
    rng = np.random.default_rng(7 + sum(shape))
    u0 = state(rng, 3, shape)
    big_shape = tuple(a * b for a, b in zip(shape, reps))
    dbig = dict(d, nz=big_shape[0], ny=big_shape[1], nx=big_shape[2])
    ubig = tile_up(u0, reps)
    dte = pf.params_stable_dt(d)
    assert pf.params_stable_dt(dbig) == dte
    cases = [(name, 1) for name in INTEG] + ([("rkl2", 2)] if pairs_built(d, prec) else [])
    for name, fu in cases:
        dt = DT_OVER_DTE[name] * dte
        a = sim_of(d, u0, prec, fusion=fu)
        b = sim_of(dbig, ubig, prec, fusion=fu)
        a.step(name, dt)
        b.step(name, dt)
        ua, _ = a.get_fields()
        ub, _ = b.get_fields()
        assert np.array_equal(tile_up(ua, reps), ub), (shape, name, fu, prec)
    a, b = sim_of(d, u0, prec), sim_of(dbig, ubig, prec)
    assert np.array_equal(tile_up(a.rhs(), reps), b.rhs()), (shape, "rhs", prec)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("dim", [2, 3])
def test_bulk_state_is_stationary(dim, prec):
    """Pure bulk: phase 1 everywhere, the other phases zero, uniform c.  N_z = 1
    at every cell and mu is uniform, so the right-hand side is exactly zero;
    every integrator keeps phi bit for bit (values 0 and 1) and c to rounding,
    and an adaptive run accepts every step with an error at rounding level."""
    shape = (6, 10, 12) if dim == 3 else (1, 16, 20)
    d = params(dim, shape)
    u0 = np.zeros((4,) + shape)
    u0[1] = 1.0
    u0[3] = 0.37
    s = sim_of(d, u0, prec)
    assert np.abs(s.rhs()).max() == 0.0
    dte = s.stable_dt()
    ctol = 1e-14 if prec == "fp64" else 1e-6
    for name in INTEG:
        g = sim_of(d, u0, prec)
        g.step(name, DT_OVER_DTE[name] * dte)
        u, _ = g.get_fields()
        assert np.array_equal(u[:3], u0[:3]), (name, prec)
        assert np.abs(u[3] - 0.37).max() <= ctol, (name, prec)
    g = sim_of(d, u0, prec)
    t_end = 400.0 * dte
    st = g.run_to("rkl2", t_end, tol=pf.Tol(r_phi=1e-4, a_phi=1e-2, r_c=1e-4, a_c=1e-4))
    tr = g.trace()
    u, t = g.get_fields()
    assert t == t_end and st.rejected == 0 and np.all(tr[:, 3] == 1.0)
    assert tr[:, 2].max() <= 1e-6
    assert np.array_equal(u[:3], u0[:3])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_no_mobility_no_diffusion_lands_on_t_end(prec):
    shape = (1, 7, 9)
    d = params(2, shape, mob=[0.0] * 4, D=[0.0, 0.0])
    rng = np.random.default_rng(31)
    u0 = state(rng, 3, shape)
    P = oracle.Params(**d)
    s = sim_of(d, u0, prec)
    assert math.isinf(s.stable_dt()) and math.isinf(oracle.stable_dt(P))
    assert np.abs(s.rhs()).max() == 0.0
    t_end = 7.5
    tol = pf.Tol(r_phi=1e-4, a_phi=1e-2, r_c=1e-4, a_c=1e-4)
    otol = oracle.Tol(r_phi=1e-4, a_phi=1e-2, r_c=1e-4, a_c=1e-4)
    atol = 1e-14 if prec == "fp64" else 1e-6
    for name in ("rkl1", "rkl2", "ssp2", "ssp104"):
        g = sim_of(d, u0, prec)
        st = g.run_to(name, t_end, tol=tol)
        u, t = g.get_fields()
        assert t == t_end and st.accepted == 1 and st.rejected == 0, (name, prec)
        assert np.abs(u - u0).max() <= atol, (name, prec)
        if prec == "fp64":
            ref, st_ref, rc = oracle.run_to(P, INTEG[name], u0, t_end, tol=otol, s=3)
            assert rc == 0 and st_ref.accepted == 1
            check_fp64(u, ref, 3, name)
    for name in ("fe", "rkl2"):
        g = sim_of(d, u0, prec)
        st = g.run_to(name, t_end, dt_fixed=math.inf)
        u, t = g.get_fields()
        assert t == t_end and st.accepted == 1, (name, prec)
        assert np.abs(u - u0).max() <= atol, (name, prec)
    g = sim_of(d, u0, prec)
    for bad in (math.inf, math.nan):
        with pytest.raises(pf.PFError) as ei:
            g.step("fe", bad)
        assert ei.value.code == -1
        with pytest.raises(pf.PFError) as ei:
            g.run_to("rkl2", bad, tol=tol)
        assert ei.value.code == -1
    u, t = g.get_fields()
    # the refused calls changed nothing (FP32 holds u0 rounded to single precision)
    assert t == 0.0 and np.abs(u - u0).max() <= (0.0 if prec == "fp64" else 1e-7)
