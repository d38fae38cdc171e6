"""Error budget of reduced-precision stage storage (CPU, oracle only).

The RKL2 recurrence (eq. sts, with the first-stage R0 correction of Sec. 3.2)
is re-run here from the oracle's RHS and simplex projection S, once exactly
and once with every intermediate stage vector rounded to BF16 (round to
nearest even) as a BF16 stage ring would store it.  The exact re-run must equal
the oracle's own step bit for bit, which pins the emulation; the BF16 run
shows what such storage costs: on the shrinking grain (Sec. 5.2.1) it moves
the sharp-interface error of the area rate by an order of magnitude, so the
stage buffers stay in the compute precision.
"""
import math

import numpy as np
import pytest

import oracle
import pf_inputs as pi


@pytest.fixture(scope="module", autouse=True)
def _oracle():
    oracle.build(force=False)


def bf16_round(x):
    u = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32)
    r = (u + np.uint32(0x7FFF) + ((u >> 16) & np.uint32(1))) & np.uint32(0xFFFF0000)
    return r.view(np.float32).astype(np.float64).reshape(np.shape(x))


def rkl2_step(P, u, dt, s, bf16_stages):
    """One RKL2 step from the oracle's building blocks; intermediate stages
    1..s-1 optionally stored in BF16 (u^n, R0 and the result stay FP64)."""
    N = P.n_phi
    store = bf16_round if bf16_stages else (lambda q: q)
    r0 = oracle.rhs(P, u)
    mu, nu, mut, gam = oracle.rkl_coeffs(2, s, 1)
    q1, changed = oracle.simplex(P, u + mut * dt * r0)
    r0[:N][:, changed] = (q1[:N][:, changed] - u[:N][:, changed]) / (mut * dt)
    q = {0: u, 1: store(q1)}
    for j in range(2, s + 1):
        r = oracle.rhs(P, q[j - 1])
        mu, nu, mut, gam = oracle.rkl_coeffs(2, s, j)
        qj, _ = oracle.simplex(P, (1 - mu - nu) * u + mu * q[j - 1] + nu * q[j - 2] +
                               dt * (mut * r + gam * r0))
        q[j] = store(qj) if j < s else qj
    return q[s]


def test_emulated_rkl2_step_equals_oracle():
    wl = pi.voronoi_2d(n=96, n_grains=12)
    P = oracle.Params(**wl.param_dict())
    dte = oracle.stable_dt(P)
    s = oracle.stage_count(2, 100 * dte, dte)
    ref, _, _ = oracle.step(P, oracle.RKL2, 100 * dte, wl.u0, s=s)
    u = rkl2_step(P, oracle._state(P, wl.u0).copy(), 100 * dte, s, bf16_stages=False)
    assert np.array_equal(u, ref)


def test_bf16_stage_storage_exceeds_the_error_budget():
    """Shrinking grain, 100 RKL2 steps at 20 dt_e: the area-rate error against
    dA/dt = -2 pi M gamma with FP64 stages vs with BF16 stages."""
    wl = pi.single_grain()
    P = oracle.Params(**wl.param_dict())
    dte = oracle.stable_dt(P)
    dt = 20 * dte
    s = oracle.stage_count(2, dt, dte)
    A0 = oracle._state(P, wl.u0)[1].sum()
    err = {}
    for bf in (False, True):
        u = oracle._state(P, wl.u0).copy()
        for _ in range(100):
            u = rkl2_step(P, u, dt, s, bf16_stages=bf)
        rate = (u[1].sum() - A0) / (100 * dt)
        err[bf] = abs(rate / (-2 * math.pi * wl.mob[0]) - 1.0)
    # FP64 stages: ~2.6e-3 (discretisation); BF16 stages: ~2.5e-2
    assert err[False] < 5e-3
    assert err[True] > 5 * err[False]
