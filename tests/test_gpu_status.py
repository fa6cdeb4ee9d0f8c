"""GPU checks of the C ABI's status reporting and of repeatability.

Failure statuses: refinement that misses rtol (NOT_CONVERGED), a NaN in the
right-hand side (NONFINITE), a failed device allocation (NOMEM, forced from
the host through MPOIS_FAULT_ALLOC).  Repeatability: two executes of one plan
on one input give bit-identical results (no race in the LDS stages or the
reductions), for single grids and batches, eager and graph-replayed.
"""

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1409_8116_amd as mp
    mp.load_library()
    yield


def _mp():
    import paper_1409_8116_amd as mp
    return mp


def test_not_converged_is_reported():
    mp = _mp()
    shape = (30, 28, 26)
    plan = mp.Plan(shape, (0.1,) * 3, ("N", "P", "D"), ("v", "v", "s"), prec="f32r", rtol=1e-30, max_iter=1)
    g = torch.as_tensor(np.random.default_rng(0).standard_normal(shape)).cuda()
    phi = plan.solve(g)
    info = plan.info()
    assert info["status"] == 5, info  # NOT_CONVERGED
    assert 0 < info["rel_resid"] < 1e-6  # phi still holds the refined iterate
    with pytest.raises(mp.MpoisError) as e:
        plan.info(check=True)
    assert e.value.status == 5
    assert torch.isfinite(phi).all()
    plan.close()


@pytest.mark.parametrize("prec", ["f64", "f32r"])
def test_nonfinite_rhs_is_reported(prec):
    mp = _mp()
    shape = (20, 24)
    plan = mp.Plan(shape, (0.1, 0.1), ("D", "N"), ("v", "s"), prec=prec, max_iter=1)
    g = np.random.default_rng(1).standard_normal(shape)
    g[3, 5] = np.nan
    plan.solve(torch.as_tensor(g).cuda())
    info = plan.info()
    assert info["status"] == 6, info  # NONFINITE
    plan.close()


def test_failed_allocation_is_nomem(monkeypatch):
    mp = _mp()
    monkeypatch.setenv("MPOIS_FAULT_ALLOC", "1")
    for kw in ({"prec": "f64"}, {"prec": "f32r"}):
        with pytest.raises(mp.MpoisError) as e:
            mp.Plan((16, 16, 16), (0.1,) * 3, ("P", "P", "P"), ("v",) * 3, **kw)
        assert e.value.status == 3
    with pytest.raises(mp.MpoisError) as e:
        mp.BatchPlan(workloads.batch_2d(count=4, lo=8, hi=20, seed=3), prec="f32r")
    assert e.value.status == 3
    monkeypatch.delenv("MPOIS_FAULT_ALLOC")
    mp.Plan((16, 16, 16), (0.1,) * 3, ("P", "P", "P"), ("v",) * 3).close()  # and recovers


@pytest.mark.parametrize("prec", ["f64", "f32", "f32r"])
def test_repeat_execute_is_bitwise_identical(prec):
    """Rader (DCT-I 512 per line: 1022 = 73 x 14), Bluestein (DST-I n = 100: 202 = 2 x 101)
    and plain Stockham lengths, on every axis."""
    mp = _mp()
    dt = torch.float32 if prec == "f32" else torch.float64
    for shape, bc, grid in (((24, 40, 512), ("N",) * 3, ("v",) * 3),
                            ((512, 12, 20), ("N", "P", "D"), ("v", "v", "s")),
                            ((33, 100, 45), ("P", "D", "N"), ("v", "v", "s"))):
        print(f"[repeat] {prec} {shape} {bc} {grid}", flush=True)
        plan = mp.Plan(shape, [1.0 / n for n in shape], bc, grid, prec=prec, max_iter=2)
        g = torch.as_tensor(np.random.default_rng(2).standard_normal(shape), dtype=dt).cuda()
        a = plan.solve(g).clone()
        b = plan.solve(g)
        torch.cuda.synchronize()
        assert torch.equal(a, b), (shape, prec)
        plan.close()


@pytest.mark.parametrize("prec", ["f64", "f32r"])
def test_batch_graph_replay_equals_eager(prec):
    """A batch plan with MPOIS_FLAG_GRAPH: replays (with new pointer tables and
    eager work in between) equal the eager batch bit for bit."""
    mp = _mp()
    descs = workloads.batch_2d(count=24, lo=20, hi=150, seed=31)
    eager = mp.BatchPlan(descs, prec=prec, max_iter=2)
    graph = mp.BatchPlan(descs, prec=prec, max_iter=2, graph=True)
    for rep in range(3):
        print(f"[batch graph] {prec} replay {rep}", flush=True)
        rhs = [torch.as_tensor(workloads.batch_rhs(d, i, seed=40 + rep)).cuda() for i, d in enumerate(descs)]
        pe = [torch.empty_like(r) for r in rhs]
        pg = [torch.empty_like(r) for r in rhs]  # new output pointers every replay
        eager.solve(rhs, pe)
        graph.solve(rhs, pg)
        graph.solve(rhs, pg)  # same pointers: tables are not re-uploaded
        torch.cuda.synchronize()
        for i in range(len(descs)):
            assert torch.equal(pe[i], pg[i]), (rep, i)
        _ = sum(float(r.abs().sum()) for r in rhs[:3])  # unrelated eager work between replays
    d = descs[5]
    ref = oracle.solve(rhs[5].cpu().numpy(), oracle.axes_from(d["shape"], d["h"], d["bc"], d["grid"]), "fd")
    assert np.linalg.norm(pg[5].cpu().numpy() - ref) <= 1e-12 * np.linalg.norm(ref)


def test_single_and_batch_executes_keep_their_own_report():
    """mpois_get_info reports on the entry point that ran last (single or batch)."""
    mp = _mp()
    descs = workloads.batch_2d(count=1, lo=30, hi=40, seed=5)
    plan = mp.BatchPlan(descs, prec="f64")
    d = descs[0]
    g = torch.as_tensor(workloads.batch_rhs(d, 0)).cuda()
    phi = torch.empty_like(g)
    plan.solve([g], [phi])
    assert plan.info()["rel_resid"] < 1e-12
    del g, phi
    torch.cuda.synchronize()
    single = mp.Plan.from_desc(d, prec="f64")
    g2 = torch.as_tensor(workloads.batch_rhs(d, 1)).cuda()
    out = single.solve(g2)
    assert single.info()["rel_resid"] < 1e-12
    # a one-grid batch plan run through mpois_execute reports on that call's arrays
    out2 = torch.empty_like(g2)
    st = plan.lib.mpois_execute(plan._h, __import__("ctypes").c_void_p(g2.data_ptr()),
                                __import__("ctypes").c_void_p(out2.data_ptr()), None)
    assert st == 0
    torch.cuda.synchronize()
    assert plan.info()["rel_resid"] < 1e-12
    assert torch.equal(out, out2)


def test_trace_ranges_leave_results_unchanged(monkeypatch):
    """MPOIS_TRACE=1 wraps the calls and solve phases in roctx ranges (for
    rocprofv3 --marker-trace); the results are bit for bit the same."""
    mp = _mp()
    shape, h, bc, grid = (20, 24, 18), (0.05, 0.04, 0.06), ("P", "N", "D"), ("v", "s", "s")
    g = torch.tensor(np.random.default_rng(7).standard_normal(shape), device="cuda")
    outs = []
    for trace in ("0", "1"):
        monkeypatch.setenv("MPOIS_TRACE", trace)
        plan = mp.Plan(shape, h, bc, grid, prec="f32r", max_iter=2)
        outs.append(plan.solve(g).clone())
        plan.info()
        plan.close()
    torch.cuda.synchronize()
    assert torch.equal(outs[0], outs[1])
