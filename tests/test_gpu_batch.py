"""Batched 2D instances (one fused launch per step, hipGraph replay) against
single-instance runs and the FP64 oracle, through the C-ABI."""
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


def small_batch():
    """Six two-phase instances of uneven (partly ragged) size, radius and mobility."""
    out = []
    shapes = [(64, 64), (70, 45), (96, 96), (33, 50), (128, 64), (40, 200)]
    rng = np.random.default_rng(9)
    for k, (nx, ny) in enumerate(shapes):
        R = float(rng.uniform(0.2, 0.4)) * min(nx, ny)
        M = float(rng.uniform(0.5, 2.0))
        wl = pi.single_grain(n=nx, ny=ny, R=R, W=4.0, M=M, seed=30 + k)
        out.append(wl)
    return out


@pytest.mark.parametrize("prec,blocks,depth", [("fp32", None, 1), ("fp64", None, 1), ("fp32", 8, 1),
                                                ("fp64", 24, 1), ("fp32", None, 2), ("fp64", None, 2),
                                                ("fp32", 8, 2), ("fp64", 16, 2)])
def test_batch_equals_single_runs_bitwise(prec, blocks, depth):
    """blocks: persistent grid size; a small grid makes each block walk tiles of
    several instances, entering and skipping (finished) instances mid-range.
    depth: steps per launch; at depth 2 the odd step counts end with a launch
    that takes one step."""
    wls = small_batch()
    b = pf.Batch([w.param_dict() for w in wls], prec=prec)
    if blocks is not None:
        b.set_blocks(blocks)
    b.set_fusion(depth)
    assert b.config()[1] == depth
    for i, w in enumerate(wls):
        b.init_fields(i, w.u0)
    dts = [0.9 * b.stable_dt(i) for i in range(len(wls))]
    # uneven step counts (odd and even) and clipped last steps
    t_end = [dts[i] * (17 + 3 * i) + 0.3 * dts[i] * (i % 2) for i in range(len(wls))]
    st = b.run_to(t_end, graph_steps=4)
    for i, w in enumerate(wls):
        u_b, t_b = b.get_fields(i)
        s = pf.Sim(w.param_dict(), prec=prec)
        s.init_fields(w.u0)
        st1 = s.run_to("fe", t_end[i], dt_fixed=dts[i])
        u_s, t_s = s.get_fields()
        assert st[i].accepted == st1.accepted and t_b == t_s == t_end[i]
        assert np.array_equal(u_b, u_s), (i, np.abs(u_b - u_s).max())


@pytest.mark.parametrize("depth", [1, 2])
def test_batch_graph_replays_equal_eager_runs(depth):
    """Replay one captured graph across several runs, with eager work and
    synchronisation in between, and compare every run with direct launches."""
    wls = small_batch()[:4]
    g = pf.Batch([w.param_dict() for w in wls], prec="fp32")
    e = pf.Batch([w.param_dict() for w in wls], prec="fp32")
    g.set_fusion(depth)
    e.set_fusion(depth)
    for i, w in enumerate(wls):
        g.init_fields(i, w.u0)
        e.init_fields(i, w.u0)
    dts = [0.9 * g.stable_dt(i) for i in range(len(wls))]
    t = [0.0] * len(wls)
    for rep in range(4):
        t = [t[i] + 12 * dts[i] for i in range(len(wls))]
        g.run_to(t, dt=dts, graph_steps=6)
        e.run_to(t, dt=dts, graph_steps=0)
        _ = torch.ones(1024, device="cuda").sum().item()  # unrelated eager work + sync
        for i in range(len(wls)):
            ug, _ = g.get_fields(i)
            ue, _ = e.get_fields(i)
            assert np.array_equal(ug, ue), (rep, i)


def test_batch_fp64_matches_oracle():
    wls = small_batch()[:3]
    b = pf.Batch([w.param_dict() for w in wls], prec="fp64")
    for i, w in enumerate(wls):
        b.init_fields(i, w.u0)
    dts = [0.9 * b.stable_dt(i) for i in range(len(wls))]
    t_end = [40 * d for d in dts]
    b.run_to(t_end, graph_steps=8)
    for i, w in enumerate(wls):
        P = oracle.Params(**w.param_dict())
        ref, st, rc = oracle.run_to(P, oracle.FE, w.u0, t_end[i], dt_fixed=dts[i])
        u, t = b.get_fields(i)
        assert rc == 0 and np.abs(u - ref).max() <= 1e-10


def test_batch_autotune_keeps_state():
    wls = small_batch()[:3]
    b = pf.Batch([w.param_dict() for w in wls], prec="fp32")
    for i, w in enumerate(wls):
        b.init_fields(i, w.u0)
    before = [b.get_fields(i)[0] for i in range(3)]
    nb, ms = b.autotune()
    assert nb % 8 == 0 and ms > 0
    assert b.config() == (nb, b.config()[1]) and b.config()[1] in (1, 2)
    for i in range(3):
        assert np.array_equal(b.get_fields(i)[0], before[i])


def test_batch_fusion_depth_limits():
    """Depth 2 is built for N <= 4 where (N + 3) LDS planes of the two regions
    of a 64 x 8 tile fit one workgroup's 64 KiB: N = 2 in both precisions and
    N = 4 in single precision take it; N = 4 in double precision, N = 8 and 9
    are refused; bad depths are refused."""
    def batch(n_phi, prec):
        wl = pi.voronoi_2d(n=64, n_grains=2 * n_phi, n_phi=n_phi, dmin=5.0)
        return pf.Batch([wl.param_dict()], prec=prec)
    for n_phi, prec in [(9, "fp32"), (8, "fp64"), (8, "fp32"), (4, "fp64")]:
        b = batch(n_phi, prec)
        with pytest.raises(pf.PFError) as e:
            b.set_fusion(2)
        assert e.value.code == -7, (n_phi, prec)
        assert b.config()[1] == 1
        b.close()
    for n_phi, prec in [(4, "fp32"), (2, "fp32"), (2, "fp64")]:
        b = batch(n_phi, prec)
        b.set_fusion(2)
        with pytest.raises(pf.PFError):
            b.set_fusion(3)
        assert b.config()[1] == 2, (n_phi, prec)
        b.close()


@pytest.mark.parametrize("prec,dt0", [("fp32", 0.0), ("fp64", 0.0), ("fp32", 30.0), ("fp64", 30.0)])
def test_batch_adaptive_equals_single_runs_bitwise(prec, dt0):
    """Adaptive RKL2 of six uneven instances in one batch against fresh
    single-instance adaptive runs (pf_run_to with the same tolerances): the
    same accepted and rejected steps, stages, RHS evaluations, end time and
    last norm, and the same fields bit for bit.  dt0 = 30 starts every
    instance at 120-240 dt_e, which forces rejections."""
    wls = small_batch()
    tol = pf.Tol(r_phi=1e-4, a_phi=1e-3, r_c=1e-4, a_c=1e-4, dt0=dt0)
    b = pf.Batch([w.param_dict() for w in wls], prec=prec)
    for i, w in enumerate(wls):
        b.init_fields(i, w.u0)
    t_end = [40.0 + 7.5 * i for i in range(len(wls))]
    st = b.run_adaptive(t_end, tol)
    rejected = 0
    for i, w in enumerate(wls):
        s = pf.Sim(w.param_dict(), prec=prec)
        s.init_fields(w.u0)
        ss = s.run_to("rkl2", t_end[i], tol=tol)
        u, t = s.get_fields()
        ub, tb = b.get_fields(i)
        got = (st[i].accepted, st[i].rejected, st[i].stages, st[i].rhs_evals, st[i].last_err)
        assert got == (ss.accepted, ss.rejected, ss.stages, ss.rhs_evals, ss.last_err), (i, got, ss)
        assert tb == t == t_end[i]
        assert np.array_equal(ub, u), i
        rejected += ss.rejected
        s.close()
    print(f"\nbatch adaptive {prec} dt0={dt0}: accepted {[x.accepted for x in st]}, "
          f"rejected {[x.rejected for x in st]}", flush=True)
    if dt0 > 0:
        assert rejected > 0
    b.close()


def test_batch_adaptive_fp64_matches_oracle():
    """One instance of the adaptive batch against the oracle's adaptive RKL2
    run: the same accepted and rejected steps, fields to 1e-10."""
    wls = small_batch()[:3]
    tol = dict(r_phi=1e-4, a_phi=1e-3, r_c=1e-4, a_c=1e-4)
    b = pf.Batch([w.param_dict() for w in wls], prec="fp64")
    for i, w in enumerate(wls):
        b.init_fields(i, w.u0)
    t_end = [30.0, 45.0, 25.0]
    st = b.run_adaptive(t_end, pf.Tol(**tol))
    for i in (1, 2):
        P = oracle.Params(**wls[i].param_dict())
        ref, st_ref, rc = oracle.run_to(P, oracle.RKL2, wls[i].u0, t_end[i], tol=oracle.Tol(**tol))
        assert rc == 0
        assert (st[i].accepted, st[i].rejected) == (st_ref.accepted, st_ref.rejected), i
        u, _ = b.get_fields(i)
        assert np.abs(u - ref).max() <= 1e-10, i
    b.close()


def test_batch_adaptive_rejects_bad_calls():
    wls = small_batch()[:2]
    b = pf.Batch([w.param_dict() for w in wls], prec="fp32")
    for i, w in enumerate(wls):
        b.init_fields(i, w.u0)
    with pytest.raises(pf.PFError) as e:
        b.run_adaptive([1.0, 1.0], pf.Tol(), integ="fe")
    assert e.value.code == -7
    with pytest.raises(pf.PFError) as e:
        b.run_adaptive([1.0, 1.0], pf.Tol(r_phi=0.0, a_phi=0.0))
    assert e.value.code == -1
    st = b.run_adaptive([0.0, 0.0], pf.Tol())  # nothing to do
    assert all(x.accepted == 0 and x.rejected == 0 for x in st)
    b.close()


def test_batch_rejects_mixed_instances():
    a = pi.single_grain(n=32, R=8.0).param_dict()
    c = dict(pi.voronoi_2d(n=40, n_grains=4, n_phi=3, dmin=5.0).param_dict())
    with pytest.raises(pf.PFError):
        pf.Batch([a, c])


@pytest.mark.parametrize("prec,blocks,graph", [("fp32", None, 2), ("fp64", None, 0), ("fp32", 8, 3),
                                               ("fp64", 16, 2)])
def test_batch_rkl2_equals_single_runs_bitwise(prec, blocks, graph):
    """RKL2 steps of 20 dt_e (eq. sts; 11 stages) with uneven step counts and
    clipped last steps whose stage count differs: every instance equals its
    single-instance run bit for bit, stage counts included."""
    wls = small_batch()
    b = pf.Batch([w.param_dict() for w in wls], prec=prec)
    if blocks is not None:
        b.set_blocks(blocks)
    for i, w in enumerate(wls):
        b.init_fields(i, w.u0)
    dts = [20.0 * b.stable_dt(i) for i in range(len(wls))]
    t_end = [dts[i] * (2 + i) + 0.15 * dts[i] * (i % 2) for i in range(len(wls))]
    st = b.run_to(t_end, dt=dts, graph_steps=graph, integ="rkl2")
    for i, w in enumerate(wls):
        u_b, t_b = b.get_fields(i)
        s = pf.Sim(w.param_dict(), prec=prec)
        s.init_fields(w.u0)
        st1 = s.run_to("rkl2", t_end[i], dt_fixed=dts[i])
        u_s, t_s = s.get_fields()
        assert (st[i].accepted, st[i].rhs_evals) == (st1.accepted, st1.rhs_evals), i
        assert t_b == t_s == t_end[i]
        assert np.array_equal(u_b, u_s), (i, np.abs(u_b - u_s).max())
        s.close()
    # a second run continues from the reached state (ring and table reused)
    t2 = [t + 2.5 * d for t, d in zip(t_end, dts)]
    b.run_to(t2, dt=dts, graph_steps=graph, integ="rkl2")
    for i, w in enumerate(wls[:2]):
        s = pf.Sim(w.param_dict(), prec=prec)
        s.init_fields(w.u0)
        s.run_to("rkl2", t_end[i], dt_fixed=dts[i])
        s.run_to("rkl2", t2[i], dt_fixed=dts[i])
        assert np.array_equal(b.get_fields(i)[0], s.get_fields()[0]), i
        s.close()


def test_batch_rkl2_fp64_matches_oracle():
    wls = small_batch()[:3]
    b = pf.Batch([w.param_dict() for w in wls], prec="fp64")
    for i, w in enumerate(wls):
        b.init_fields(i, w.u0)
    dts = [25.0 * b.stable_dt(i) for i in range(len(wls))]
    t_end = [3.4 * d for d in dts]
    b.run_to(t_end, dt=dts, graph_steps=2, integ="rkl2")
    for i, w in enumerate(wls):
        P = oracle.Params(**w.param_dict())
        ref, st, rc = oracle.run_to(P, oracle.RKL2, w.u0, t_end[i], dt_fixed=dts[i])
        assert rc == 0
        assert np.abs(b.get_fields(i)[0] - ref).max() <= 1e-10, i
