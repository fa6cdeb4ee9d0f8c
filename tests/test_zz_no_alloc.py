"""mpois_execute_noalloc (static device scratch, no allocation) against
mpois_execute (the plan's workspace), through the C ABI: the same kernels on
the same inputs, so the results must agree bit for bit.  Two calls in a row,
the second on a smaller grid (the shared scratch keeps the first call's
contents), then a plan too large for the scratch is refused."""

import ctypes

import numpy as np
import pytest

import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1409_8116_amd as mp
    mp.load_library()
    yield


def _run(mp, shape, bc, grid, prec, seed):
    h = tuple(1.0 / n for n in shape)
    plan = mp.Plan(shape, h, bc, grid, prec=prec, max_iter=2)
    dt = torch.float32 if prec == "f32" else torch.float64
    g = np.random.default_rng(seed).standard_normal(shape)
    rhs = torch.as_tensor(g, dtype=dt).cuda()
    ref = torch.empty_like(rhs)
    out = torch.full_like(rhs, float("nan"))
    lib = mp.load_library()
    stream = ctypes.c_void_p(int(torch.cuda.current_stream().cuda_stream))
    assert lib.mpois_execute(plan._h, ctypes.c_void_p(rhs.data_ptr()), ctypes.c_void_p(ref.data_ptr()), stream) == 0
    print(f"[noalloc] {prec} {shape} {bc} {grid}", flush=True)
    assert lib.mpois_execute_noalloc(plan._h, ctypes.c_void_p(rhs.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                                     stream) == 0
    torch.cuda.synchronize()
    assert torch.equal(out, ref), (shape, prec)
    info = plan.info()
    if prec != "f32":
        assert info["rel_resid"] < 1e-10, info
    if prec == "f32r" and np.prod(shape) <= 40 ** 3:
        axes = oracle.axes_from(shape, h, bc, grid)
        phi_o = oracle.solve(g, axes, "fd")
        assert np.linalg.norm(out.cpu().numpy() - phi_o) <= 1e-12 * np.linalg.norm(phi_o)
    plan.close()


@pytest.mark.parametrize("prec", ["f32r", "f64", "f32"])
def test_noalloc_matches_execute_twice_second_smaller(prec):
    import paper_1409_8116_amd as mp
    _run(mp, (40, 36, 33), ("N", "P", "D"), ("v", "v", "s"), prec, seed=1)
    _run(mp, (17, 12, 9), ("N", "N", "P"), ("s", "v", "v"), prec, seed=2)


@pytest.mark.parametrize("prec", ["f32r", "f64"])
def test_noalloc_with_plane_kernels(prec):
    """32 x 32 periodic planes (the plane-kernel path) through the static scratch."""
    import paper_1409_8116_amd as mp
    _run(mp, (12, 32, 32), ("P", "P", "P"), ("v", "v", "v"), prec, seed=4)


def test_noalloc_full_scratch_size_and_refusal():
    import paper_1409_8116_amd as mp
    _run(mp, (256, 256, 256), ("N", "N", "N"), ("v", "v", "v"), "f32r", seed=3)  # 64 MiB working array
    plan = mp.Plan((512, 256, 132), (0.01,) * 3, ("P", "P", "P"), ("v",) * 3, prec="f32r", max_iter=1)
    rhs = torch.zeros((512, 256, 132), dtype=torch.float64, device="cuda")
    with pytest.raises(mp.MpoisError) as e:
        plan.solve_noalloc(rhs, torch.empty_like(rhs))
    assert e.value.status == 2  # UNSUPPORTED: working array beyond the static scratch
    plan.close()
