"""Host logic of the library against the oracle, on the CPU (no device).

The library's scalar computations (stable step, RKL stage count, step-size
controller, clipping to exact output times) are exported as host-only calls
that run the engine's own functions; the oracle implements each of them
independently from the paper (Sec. 3.2, eq. sts-limit, Sec. 3.3, Sec. 5).
"""
import math

import numpy as np
import pytest

import oracle
import pf_inputs as pi
import paper_2601_16522_amd as pf


@pytest.fixture(scope="module", autouse=True)
def _libs():
    oracle.build(force=False)
    pf.lib()


def _param_sets():
    wls = [pi.single_grain(n=32, R=8.0), pi.voronoi_2d(n=48, n_grains=6, n_phi=4, dmin=5.0),
           pi.grains_pores_3d(n=16, n_grains=5, n_grain_fields=3, n_pores=3, r_range=(2.0, 3.0)),
           pi.grains_pores_3d(n=16, n_grains=9, n_grain_fields=8, n_pores=3, r_range=(2.0, 3.0),
                              dmin=3.0),
           pi.single_grain(n=32, R=8.0, with_c=False)]
    wls += pi.batch_instances(count=4)
    mixed = dict(pi.voronoi_2d(n=40, n_grains=4, n_phi=3, dmin=5.0).param_dict())
    mixed.update(type_of=[0, 1, 1], n_types=2, gamma=[1.0, 0.8, 0.8, 1.2], mob=[1.0, 2.0, 2.0, 0.5],
                 k=[500.0, 300.0], c0=[0.1, 0.9], D=[1.0, 0.3])
    return [w.param_dict() for w in wls] + [mixed]


def test_stable_dt_matches_oracle():
    for p in _param_sets():
        ref = oracle.stable_dt(oracle.Params(**p))
        got = pf.params_stable_dt(p)
        assert abs(got - ref) <= 1e-14 * ref, (p["dim"], got, ref)


def test_stage_count_matches_oracle():
    ratios = np.concatenate([np.geomspace(0.01, 500.0, 400), [0.9, 2.7, 5.4, 9.0, 13.5, 100.0, 200.0]])
    for integ, order in (("rkl1", 1), ("rkl2", 2)):
        for r in ratios:
            assert pf.rkl_stage_count(integ, r, 1.0) == oracle.stage_count(order, r, 1.0), (integ, r)
    with pytest.raises(pf.PFError):
        pf.rkl_stage_count("fe", 1.0, 1.0)


@pytest.mark.parametrize("order", [1, 2, 4])
def test_controller_matches_oracle(order):
    """Random error sequences with rejections, tiny errors and non-finite
    values: identical accept decisions, steps and bias."""
    rng = np.random.default_rng(order)
    mine, ref = pf.Controller(), oracle.Controller()
    h = 1.0
    for k in range(400):
        e = float(10.0 ** rng.uniform(-4, 1.5))
        if k % 97 == 13:
            e = float("nan")
        if k % 89 == 7:
            e = float("inf")
        if k % 71 == 5:
            e = 0.0
        acc, hn = mine.update(order, e, h)
        hn_ref, acc_ref = ref.update(order, e, h)
        assert acc == acc_ref, (k, e)
        assert hn == hn_ref or abs(hn - hn_ref) <= 1e-15 * abs(hn_ref), (k, e, hn, hn_ref)
        assert mine.bias == ref.bias, k
        h = hn if hn > 0 else 1e-3


def test_clip_step_matches_oracle_run():
    """The steps of a fixed-dt run to t_end: the oracle's FE run (its trace of
    step sizes) against iterating pf_clip_step; includes ends within the
    1e-10 relative tolerance of a full step and remainders below 1e-12 dt."""
    wl = pi.single_grain(n=8, R=2.0)
    P = oracle.Params(**wl.param_dict())
    dt = 0.5 * oracle.stable_dt(P)
    for n_full, frac in [(7, 0.0), (7, 0.3), (7, 1.0 - 1e-11), (7, 1e-13), (0, 0.5), (3, 1.0 + 5e-11)]:
        t_end = (n_full + frac) * dt
        _, st, rc = oracle.run_to(P, oracle.FE, wl.u0, t_end, dt_fixed=dt)
        assert rc == 0
        steps = []
        t = 0.0
        while True:
            r = pf.clip_step(t, t_end, dt)
            if r is None:
                break
            h, last = r
            steps.append(h)
            t = t_end if last else t + h
        assert len(steps) == st.accepted, (n_full, frac)
        assert np.array_equal(np.asarray(steps), st.trace[:, 0]), (n_full, frac)


def test_clip_step_infinite_step_lands_on_t_end():
    """An infinite step (0.9 dt_e without mobility and diffusion) is clipped to
    the remainder; at or past t_end there is no step."""
    assert pf.clip_step(0.0, 5.0, math.inf) == (5.0, True)
    assert pf.clip_step(2.5, 5.0, math.inf) == (2.5, True)
    assert pf.clip_step(5.0, 5.0, math.inf) is None
    assert pf.clip_step(6.0, 5.0, math.inf) is None
    assert pf.clip_step(0.0, 5.0, 2.0) == (2.0, False)


def test_tolerance_marshalling():
    """pf.Tol keyword construction and its C struct (every adaptive call uses it)."""
    t = pf.Tol(r_phi=1e-5, a_phi=2e-5, r_c=3e-5, a_c=4e-5, dt_max_over_dte=50.0, dt0=1e-3)
    c = t._c()
    assert (c.r_phi, c.a_phi, c.r_c, c.a_c, c.dt_max_over_dte, c.dt0) == (1e-5, 2e-5, 3e-5, 4e-5, 50.0, 1e-3)
    d = pf.Tol()
    assert (d.r_phi, d.a_phi, d.r_c, d.a_c) == (1e-4, 1e-2, 1e-4, 1e-4)


def test_host_error_norm_matches_oracle_embedded():
    """pf_error_norm (host arrays, a given estimate e) against the oracle's norm
    of the embedded estimate e = u^{n+1} - z (Sec. 3.3, eq. error_norm): the
    same cells, weights, degree-of-freedom rule and summation order, so the
    same bits.  Phi entries with e = 0 are left out and bulk cells count two."""
    rng = np.random.default_rng(11)
    for p in _param_sets()[:4]:
        P = oracle.Params(**p)
        shape = P.shape
        un = rng.uniform(0.0, 1.0, size=shape)
        unp1 = un + rng.normal(0.0, 1e-3, size=shape)
        z = unp1 - rng.normal(0.0, 1e-4, size=shape)
        # entries without error: whole cells, and single phi entries
        N = P.n_phi
        z[:N, ..., ::3] = unp1[:N, ..., ::3]
        z[0, ..., 1::5] = unp1[0, ..., 1::5]
        tol = oracle.Tol(r_phi=1e-3, a_phi=1e-2, r_c=2e-4, a_c=1e-4)
        ref, ndof, _ = oracle.error_norm(P, 1, 0.1, un, unp1, z, tol)
        got = pf.error_norm(p, unp1 - z, un, unp1, pf.Tol(1e-3, 1e-2, 2e-4, 1e-4))
        assert got == ref, (got, ref)


def test_host_error_norm_hand_worked():
    """The hand-worked 2 x 1 case of the oracle's pins: one nontrivial phi entry
    in cell 0, none in cell 1 (2 DoF), one c entry per cell."""
    p = dict(pi.single_grain(n=2, R=1.0).param_dict())
    p.update(nx=2, ny=1)
    e = np.zeros((3, 1, 1, 2))
    un = np.zeros_like(e)
    unp1 = np.zeros_like(e)
    unp1[0] = 1.0
    unp1[2] = 0.5
    un[:] = unp1
    un[0, 0, 0, 0], un[1, 0, 0, 0], un[2, 0, 0, 0] = 0.98, 0.02, 0.51
    e[0, 0, 0, 0] = (12 * (0.98 - 1.0) + 6 * 0.5 * 0.01) / 15
    e[2, 0, 0, 0] = (12 * (0.51 - 0.5)) / 15
    e[2, 0, 0, 1] = (6 * 0.5 * 0.02) / 15
    got = pf.error_norm(p, e, un, unp1, pf.Tol(0.1, 0.01, 0.2, 0.001))
    ss = (e[0, 0, 0, 0] / (0.1 * 1.0 + 0.01)) ** 2 + (e[2, 0, 0, 0] / (0.2 * 0.51 + 0.001)) ** 2 \
        + (e[2, 0, 0, 1] / (0.2 * 0.5 + 0.001)) ** 2
    assert got == pytest.approx(math.sqrt(ss / 5), rel=1e-14)


def test_host_error_norm_errors():
    p = pi.single_grain(n=4, R=1.0).param_dict()
    a = np.zeros((3, 1, 4, 4))
    with pytest.raises(pf.PFError):
        pf.error_norm(p, a, a, a, pf.Tol(-1.0, 1e-2, 1e-4, 1e-4))
    L = pf.lib()
    assert L.pf_error_norm(None, 16, None, None, None, None, None) == -1
