"""Pins of the PID step-size controller of Sec. 3.3 (after Soederlind), for the
oracle's controller and for the engine's own host controller (pf_controller_*).

The paper prints the controller as
  F = (E_n^-k1 E_{n-1}^-k2 E_{n-2}^-k3)^(1/(P+1)) (dt_n/dt_{n-1})^k4 (dt_{n-1}/dt_{n-2})^k5
with E = e/b, k = (1.25, 0.5, -0.6, 0.25, 0) and the limiter
dt_{n+1} = dt_n (1 + 5 atan((F - 1)/5)); on a rejection where F would grow
the step, F = e_n^(-k1/(P+1)) instead.  These tests invert the limiter and
check each exponent separately, by the ratio of two factors that differ in a
single input: a dropped term, a flipped sign or exponent, or E in place of e
in the fallback changes that ratio.  All on the CPU.
"""
import math

import pytest

import oracle

K1, K2, K3, K4 = 1.25, 0.5, -0.6, 0.25


class _Oracle:
    def __init__(self):
        self.c = oracle.Controller()

    def update(self, order, e, h):
        hn, acc = self.c.update(order, e, h)
        return acc, hn

    @property
    def bias(self):
        return self.c.bias


class _Engine:
    def __init__(self):
        import paper_2601_16522_amd as pf
        self.c = pf.Controller()

    def update(self, order, e, h):
        return self.c.update(order, e, h)

    @property
    def bias(self):
        return self.c.bias


@pytest.fixture(params=["oracle", "engine"])
def make(request):
    if request.param == "oracle":
        oracle.build(force=False)
        return _Oracle
    return _Engine


def _factor(hn, h):
    """F from the limited step hn = h (1 + 5 atan((F - 1)/5))."""
    return 1.0 + 5.0 * math.tan((hn / h - 1.0) / 5.0)


def _run(make, order, history, e, h):
    """Accept every (e, h) of history, then propose from (e, h); returns
    (accepted, F, bias before the last update)."""
    c = make()
    for ei, hi in history:
        acc, _ = c.update(order, ei, hi)
        assert acc
    b = c.bias
    acc, hn = c.update(order, e, h)
    return acc, _factor(hn, h), b


@pytest.mark.parametrize("order", [1, 2, 4])
def test_error_exponent_k1(make, order):
    a = _run(make, order, [], 0.02, 1.0)
    b = _run(make, order, [], 0.3, 1.0)
    assert a[0] and b[0]
    assert a[1] / b[1] == pytest.approx((0.02 / 0.3) ** (-K1 / (order + 1)), rel=1e-12)


@pytest.mark.parametrize("order", [1, 2])
def test_error_exponent_k2(make, order):
    a = _run(make, order, [(0.01, 1.0)], 0.4, 1.0)
    b = _run(make, order, [(0.5, 1.0)], 0.4, 1.0)
    assert a[2] == b[2]
    assert a[1] / b[1] == pytest.approx((0.01 / 0.5) ** (-K2 / (order + 1)), rel=1e-12)


@pytest.mark.parametrize("order", [1, 2])
def test_error_exponent_k3(make, order):
    a = _run(make, order, [(0.01, 1.0), (0.3, 1.0)], 0.4, 1.0)
    b = _run(make, order, [(0.6, 1.0), (0.3, 1.0)], 0.4, 1.0)
    assert a[2] == b[2]
    assert a[1] / b[1] == pytest.approx((0.01 / 0.6) ** (-K3 / (order + 1)), rel=1e-12)


def test_step_ratio_exponent_k4(make):
    """(dt_n / dt_{n-1})^k4 with k4 = +0.25: after a step half as long as the
    current one the factor is 4^0.25 times that after a step twice as long."""
    a = _run(make, 2, [(0.3, 0.5)], 0.3, 1.0)
    b = _run(make, 2, [(0.3, 2.0)], 0.3, 1.0)
    assert a[1] / b[1] == pytest.approx(4.0 ** K4, rel=1e-12)
    assert a[1] > b[1]


def test_step_ratio_exponent_k5_is_zero(make):
    """k5 = 0: the step before the previous one does not enter the factor."""
    a = _run(make, 2, [(0.3, 0.25), (0.3, 1.0)], 0.3, 1.0)
    b = _run(make, 2, [(0.3, 4.0), (0.3, 1.0)], 0.3, 1.0)
    assert a[1] == b[1]


@pytest.mark.parametrize("order,e", [(1, 1.05), (2, 1.05), (2, 1.3), (4, 1.2)])
def test_reject_fallback_uses_e_not_E(make, order, e):
    """A rejection after a very accurate accepted step: the full formula would
    grow the step (E_{n-1}^-k2 is large), so the factor is e_n^(-k1/(P+1)) of
    the unscaled norm, which shrinks the step; with E_n = e_n/b it would shrink
    it by another (1/b)^(k1/(P+1))."""
    acc, F, b = _run(make, order, [(1e-9, 1.0)], e, 1.0)
    assert not acc
    assert b < 1.0
    full = ((e / b) ** -K1 * (1e-9 / 0.9) ** -K2) ** (1.0 / (order + 1))
    assert full > 1.0                      # the case the fallback is for
    assert F == pytest.approx(e ** (-K1 / (order + 1)), rel=1e-12)
    assert abs(F / (e / b) ** (-K1 / (order + 1)) - 1) > 1e-3
    assert F < 1.0
