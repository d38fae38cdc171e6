"""Handles on HIP streams of their own (pf_set_stream, pf_batch_set_stream):
two handles whose steps are queued on two streams at once, and an adaptive run
of one handle while the other's fixed steps are in flight, give the same bits
as each handle run alone on the null stream; a handle moved from stream to
stream between steps, with its work still queued, keeps those bits (the
change of stream waits for the previous stream's work)."""
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


def voronoi():
    return pi.voronoi_2d(n=160, ny=96, n_grains=20, n_phi=8, W=4.0, dmin=8.0)


def pores():
    return pi.grains_pores_3d(n=40, nyz=(36, 28), n_grains=8, n_grain_fields=3, n_pores=4,
                              r_range=(2.0, 4.0), dmin=4.0)


TOL = pf.Tol(r_phi=1e-4, a_phi=1e-4, r_c=1e-4, a_c=1e-4)


def make(wl, prec, stream=None):
    s = pf.Sim(wl.param_dict(), prec=prec)
    if stream is not None:
        s.set_stream(stream)
    s.init_fields(wl.u0)
    return s


def fixed_steps(s, n, mult=20.0):
    dt = mult * s.stable_dt()
    for _ in range(n):
        s.step("rkl2", dt)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_two_handles_on_two_streams(prec):
    wa, wb = voronoi(), pores()
    a0, b0 = make(wa, prec), make(wb, prec)
    fixed_steps(a0, 6)
    fixed_steps(b0, 6)
    ref_a, ref_b = a0.get_fields()[0], b0.get_fields()[0]
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    a, b = make(wa, prec, sa), make(wb, prec, sb)
    dta, dtb = 20.0 * a.stable_dt(), 20.0 * b.stable_dt()
    for _ in range(6):  # queued alternately on the two streams, no wait between
        a.step("rkl2", dta)
        b.step("rkl2", dtb)
    assert np.array_equal(a.get_fields()[0], ref_a)
    assert np.array_equal(b.get_fields()[0], ref_b)


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_adaptive_run_while_another_stream_is_busy(prec):
    wa, wb = pores(), voronoi()
    a0 = make(wa, prec)
    st0 = a0.run_to("rkl2", 60.0 * a0.stable_dt(), tol=TOL)
    ref_a, tr0 = a0.get_fields()[0], a0.trace()
    b0 = make(wb, prec)
    fixed_steps(b0, 12)
    ref_b = b0.get_fields()[0]
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    a, b = make(wa, prec, sa), make(wb, prec, sb)
    fixed_steps(b, 12)  # in flight on stream b while a runs its adaptive loop
    st = a.run_to("rkl2", 60.0 * a.stable_dt(), tol=TOL)
    assert st.accepted == st0.accepted and st.rejected == st0.rejected and st0.accepted > 3
    assert np.array_equal(a.trace(), tr0)
    assert np.array_equal(a.get_fields()[0], ref_a)
    assert np.array_equal(b.get_fields()[0], ref_b)


def test_handle_moved_between_streams():
    wl = pores()
    s0 = make(wl, "fp32")
    fixed_steps(s0, 9)
    ref = s0.get_fields()[0]
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    s = make(wl, "fp32", s1)
    fixed_steps(s, 3)
    s.set_stream(s2)  # the three steps may still be running on s1
    fixed_steps(s, 3)
    s.set_stream(None)
    fixed_steps(s, 3)
    assert np.array_equal(s.get_fields()[0], ref)


def test_batch_moved_between_streams():
    wls = pi.batch_instances(count=6)

    def run(streams):
        b = pf.Batch([w.param_dict() for w in wls], prec="fp32")
        for i, w in enumerate(wls):
            b.init_fields(i, w.u0)
        dts = [0.9 * b.stable_dt(i) for i in range(len(wls))]
        for k, st in enumerate(streams):
            b.set_stream(st)
            b.run_to([(k + 1) * 40 * d for d in dts], dt=dts, graph_steps=10)
        return [b.get_fields(i)[0] for i in range(len(wls))]
    one = torch.cuda.Stream()
    ref = run([one] * 3)
    got = run([torch.cuda.Stream(), torch.cuda.Stream(), torch.cuda.Stream()])
    assert all(np.array_equal(x, y) for x, y in zip(ref, got))
