"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Error metric: ||phi_gpu - phi_oracle||_2 / ||phi_oracle||_2 over the grid, both
in the zero-weighted-mean gauge.  Bars: 1e-12 for FP64 and for FP32 with FP64
refinement, 1e-5 for single-pass FP32.
"""

import itertools

import numpy as np
import pytest

import oracle
import workloads

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

TOL = {"f64": 1e-12, "f32": 1e-5, "f32r": 1e-12}
KINDS = [("P", "v"), ("D", "v"), ("D", "s"), ("N", "v"), ("N", "s")]


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


def rel_err(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def gpu_solve(g, shape, h, bc, grid, approx, prec, max_iter=2, graph=False, tune=False, shift=0.0):
    mp = _mp()
    plan = mp.Plan(shape, h, bc, grid, approx=approx, prec=prec, max_iter=max_iter, graph=graph, tune=tune,
                   shift=shift)
    dt = torch.float32 if prec == "f32" else torch.float64
    rhs = torch.as_tensor(np.ascontiguousarray(g), dtype=dt).cuda()
    phi = torch.empty_like(rhs)
    plan.solve(rhs, phi)
    torch.cuda.synchronize()
    out = phi.double().cpu().numpy()
    info = plan.info()
    plan.close()
    return out, info


def oracle_solve(g, shape, h, bc, grid, approx, shift=0.0):
    axes = oracle.axes_from(shape, h, bc, grid)
    return oracle.solve(g, axes, approx, shift=shift)


def check(shape, kinds, approx, prec, seed=0, h=None, max_iter=2, shift=0.0):
    bc = tuple(k[0] for k in kinds)
    grid = tuple(k[1] for k in kinds)
    h = h or tuple(1.0 / (n + 1) for n in shape)
    print(f"[parity] shape={shape} kinds={kinds} approx={approx} prec={prec} seed={seed} shift={shift}", flush=True)
    g = np.random.default_rng(seed).standard_normal(shape)
    ref = oracle_solve(g, shape, h, bc, grid, approx, shift)
    out, info = gpu_solve(g, shape, h, bc, grid, approx, prec, max_iter=max_iter, shift=shift)
    err = rel_err(out, ref)
    assert err <= TOL[prec], (shape, kinds, approx, prec, err)
    return err, info


# ------------------------------------------------------------------ 1D: every kind, many lengths
# Rader stage then Stockham stages: DST-I n = 72 and DCT-I n = 74 (146 = 73 x 2), DCT-I n = 147
# (292 = 73 x 4) and n = 439 (876 = 73 x 12); DCT-I n = 512: 1022 = 73 x 14 (the radix-14 stage)
# includes lengths whose DFTs take the prime codelets 17..31 of the wide shapes
# (19, 23, 29, 38 = 2*19, 46, 58, 62, 341 = 11*31, 527 = 17*31, 986 = 2*17*29)
LENGTHS = [1, 2, 3, 4, 5, 6, 7, 8, 9, 11, 12, 13, 16, 17, 19, 23, 25, 29, 31, 32, 37, 38, 46, 49, 58, 62, 64, 72, 74,
           100, 121, 127, 128, 143, 147, 169, 255, 256, 257, 341, 343, 439, 509, 511, 512, 513, 527, 986, 1000, 1021,
           1024]


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_1d_all_lengths(kind, prec):
    for n in LENGTHS:
        if kind == ("N", "v") and n < 2:
            continue
        for approx in ("fd", "ps"):
            check((n,), [kind], approx, prec, seed=n)


# ------------------------------------------------------------------ 2D / 3D: every kind pair, ragged tiles
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_2d_all_kind_pairs(prec):
    for k0, k1 in itertools.product(KINDS, repeat=2):
        check((37, 45), [k0, k1], "fd", prec, seed=3)
        check((20, 33), [k0, k1], "ps", prec, seed=4)


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_3d_mixed_kinds(prec):
    combos = [[("P", "v"), ("D", "s"), ("N", "s")], [("N", "v")] * 3, [("D", "v"), ("P", "v"), ("N", "v")],
              [("P", "v")] * 3, [("D", "s"), ("N", "v"), ("P", "v")], [("N", "s"), ("D", "v"), ("D", "s")]]
    for kinds in combos:
        for approx in ("fd", "ps"):
            check((19, 24, 35), kinds, approx, prec, seed=5)


def test_3d_several_tiles_and_tails():
    # lines per tile are 2-32; these shapes leave partial tiles on every axis
    for shape in [(33, 17, 65), (3, 50, 7), (1, 1, 40), (40, 1, 1), (2, 2, 2)]:
        for kinds in ([("P", "v"), ("D", "s"), ("N", "s")], [("N", "v"), ("N", "v"), ("D", "v")]):
            if any(k == ("N", "v") and n < 2 for k, n in zip(kinds, shape)):
                continue  # a vertex Neumann axis needs two nodes
            check(shape, kinds, "fd", "f64", seed=6)
            check(shape, kinds, "fd", "f32", seed=6)


def test_invalid_plans_are_refused():
    mp = _mp()
    with pytest.raises(mp.MpoisError) as e:
        mp.Plan((40, 1), (0.1, 0.1), ("P", "N"), ("v", "v"))
    assert e.value.status == 1
    with pytest.raises(mp.MpoisError) as e:
        mp.Plan((8, 8), (0.1, 0.1), ("P", "D"), ("v", "v"), approx="ps", prec="f32r")
    assert e.value.status == 2


# ------------------------------------------------------------------ refinement
@pytest.mark.parametrize("kinds", [[("N", "v")] * 3, [("P", "v")] * 3, [("P", "v"), ("D", "s"), ("N", "s")],
                                   [("D", "v"), ("N", "s"), ("P", "v")]])
def test_refinement_reaches_fp64(kinds):
    err, info = check((24, 31, 20), kinds, "fd", "f32r", seed=7, max_iter=2)
    assert info["iters"] == 3
    assert info["rel_resid"] < 1e-11


def test_refinement_2d_1d():
    check((45, 64), [("N", "v"), ("P", "v")], "fd", "f32r", seed=8, max_iter=2)
    check((200,), [("N", "s")], "fd", "f32r", seed=9, max_iter=2)
    check((201,), [("D", "v")], "fd", "f32r", seed=10, max_iter=2)


def test_refinement_incompatible_rhs_is_projected():
    """A right-hand side with a large mean on a singular problem: solved for g - m_g."""
    shape = (20, 18, 22)
    kinds = [("N", "v"), ("N", "s"), ("P", "v")]
    bc = tuple(k[0] for k in kinds)
    grid = tuple(k[1] for k in kinds)
    h = (0.05, 0.05, 0.05)
    g = np.random.default_rng(1).standard_normal(shape) + 5.0
    ref = oracle_solve(g, shape, h, bc, grid, "fd")
    out, info = gpu_solve(g, shape, h, bc, grid, "fd", "f32r", max_iter=2)
    assert rel_err(out, ref) <= 1e-12
    axes = oracle.axes_from(shape, h, bc, grid)
    assert abs(info["zero_mode_rhs"] - oracle.weighted_mean(g, axes)) <= 1e-12 * 5


# ------------------------------------------------------------------ configurations at full size
def test_periodic_box_32():
    d, g = workloads.periodic_noise(32, seed=1)
    ref = oracle_solve(g, d["shape"], d["h"], d["bc"], d["grid"], d["approx"])
    out, _ = gpu_solve(g, d["shape"], d["h"], d["bc"], d["grid"], d["approx"], "f64")
    assert rel_err(out, ref) <= 1e-12
    assert abs(out.mean()) <= 1e-14 * np.abs(out).max()


@pytest.mark.parametrize("prec", ["f64", "f32", "f32r"])
def test_plane_kernels_match_oracle_and_per_axis_sweeps(prec, monkeypatch):
    """32 x 32 periodic planes in one sweep (three launches per solve): the
    oracle on the 32^3 box and on a 7 x 32 x 32 box, the same results as the
    per-axis sweeps (MPOIS_NO_PLANE=1), and the profile names the plane
    kernels."""
    mp = _mp()
    for shape in ((32, 32, 32), (7, 32, 32)):
        d, g = workloads.periodic_noise(32, seed=1)
        g = g[: shape[0]] - g[: shape[0]].mean()
        h = d["h"]
        print(f"[parity] planes {prec} {shape}", flush=True)
        ref = oracle_solve(g, shape, h, d["bc"], d["grid"], "fd")
        out, info = gpu_solve(g, shape, h, d["bc"], d["grid"], "fd", prec)
        assert rel_err(out, ref) <= TOL[prec], (shape, prec)
        monkeypatch.setenv("MPOIS_NO_PLANE", "1")
        per_axis, _ = gpu_solve(g, shape, h, d["bc"], d["grid"], "fd", prec)
        monkeypatch.delenv("MPOIS_NO_PLANE")
        assert rel_err(out, per_axis) <= (1e-6 if prec == "f32" else 1e-14), (shape, prec)
    plan = mp.Plan((32, 32, 32), d["h"], d["bc"], d["grid"], prec=prec, profile=True)
    dt = torch.float32 if prec == "f32" else torch.float64
    rhs = torch.zeros((32, 32, 32), dtype=dt, device="cuda")
    plan.solve(rhs, torch.empty_like(rhs))
    kernels = [r["kernel"] for r in plan.profile()]
    plan.close()
    line_kernels = [k for k in kernels if k not in (100, 101)]
    planes = sum(k >= 300 for k in line_kernels)
    # every solve: forward planes, the fused axis-0 sweep, inverse planes
    assert planes > 0 and 3 * planes == 2 * len(line_kernels), kernels


@pytest.mark.parametrize("approx,prec", [("fd", "f64"), ("ps", "f64"), ("fd", "f32"), ("ps", "f32")])
def test_mixed_box_256(approx, prec):
    d, g, modes = workloads.mixed_modes(256, seed=2, approx=approx)
    ref = oracle_solve(g, d["shape"], d["h"], d["bc"], d["grid"], approx)
    out, _ = gpu_solve(g, d["shape"], d["h"], d["bc"], d["grid"], approx, prec)
    assert rel_err(out, ref) <= TOL[prec]


@pytest.mark.parametrize("prec,max_iter", [("f64", 0), ("f32r", 2)])
def test_neumann_cube_512(prec, max_iter):
    d, g = workloads.neumann_blobs(512, seed=3)
    axes = oracle.axes_from(d["shape"], d["h"], d["bc"], d["grid"])
    ref = oracle.solve(g, axes, "fd")
    out, info = gpu_solve(g, d["shape"], d["h"], d["bc"], d["grid"], "fd", prec, max_iter=max(max_iter, 1))
    err = rel_err(out, ref)
    print(f"[parity] neumann cube 512 {prec}: rel err {err:.3e} resid {info['rel_resid']:.3e}", flush=True)
    assert err <= 1e-12
    # the generated right-hand side is compatible: its weighted mean is rounding-level
    assert abs(info["zero_mode_rhs"]) <= 1e-14 * np.abs(g).max(), info


# ------------------------------------------------------------------ batches of independent grids
def _batch_check(descs, prec, max_iter=2, n_oracle=None):
    mp = _mp()
    dt = torch.float32 if prec == "f32" else torch.float64
    rhs = [torch.as_tensor(workloads.batch_rhs(d, i, seed=11), dtype=dt).cuda() for i, d in enumerate(descs)]
    phi = [torch.empty_like(r) for r in rhs]
    plan = mp.BatchPlan(descs, prec=prec, max_iter=max_iter)
    plan.solve(rhs, phi)
    torch.cuda.synchronize()
    worst = 0.0
    idx = range(len(descs)) if n_oracle is None else range(0, len(descs), max(1, len(descs) // n_oracle))
    for i in idx:
        d = descs[i]
        ref = oracle_solve(rhs[i].double().cpu().numpy(), d["shape"], d["h"], d["bc"], d["grid"], d["approx"])
        worst = max(worst, rel_err(phi[i].double().cpu().numpy(), ref))
    info = plan.info()
    plan.close()
    return worst, info


@pytest.mark.parametrize("prec", ["f64", "f32", "f32r"])
def test_batch_small_mixed(prec):
    print(f"[parity] batch of 60 small 2D grids, {prec}", flush=True)
    descs = workloads.batch_2d(count=60, lo=5, hi=90, seed=21)
    worst, info = _batch_check(descs, prec)
    assert worst <= TOL[prec], worst
    if prec != "f32":
        assert info["rel_resid"] < 1e-10


def test_batch_matches_single_plans():
    descs = workloads.batch_2d(count=12, lo=30, hi=140, seed=22)
    mp = _mp()
    rhs = [torch.as_tensor(workloads.batch_rhs(d, i), dtype=torch.float64).cuda() for i, d in enumerate(descs)]
    phi_b = [torch.empty_like(r) for r in rhs]
    mp.BatchPlan(descs, prec="f64").solve(rhs, phi_b)
    for i, d in enumerate(descs):
        single = mp.Plan.from_desc(d, prec="f64").solve(rhs[i])
        torch.cuda.synchronize()
        assert torch.allclose(single, phi_b[i], rtol=0, atol=0), i  # same kernels, same tables: bit-identical


def test_batch_full_size_subset():
    """The 2048-grid workload (sides 64..1024) as configured: autotuned plans,
    FP32 + refinement.  Every grid's residual, and every 32nd grid (64 grids)
    against the oracle."""
    print("[parity] batch 2048 grids, sides 64..1024, f32r, tuned plans", flush=True)
    descs = workloads.batch_2d(count=2048, seed=4)
    mp = _mp()
    rhs = [torch.as_tensor(workloads.batch_rhs(d, i), dtype=torch.float64).cuda() for i, d in enumerate(descs)]
    phi = [torch.empty_like(r) for r in rhs]
    plan = mp.BatchPlan(descs, prec="f32r", max_iter=2, tune=True)
    print("[parity] batch plan built", flush=True)
    plan.solve(rhs, phi)
    info = plan.info()
    assert info["rel_resid"] < 1e-11, info
    worst = 0.0
    for i in range(0, 2048, 32):
        d = descs[i]
        ref = oracle_solve(rhs[i].cpu().numpy(), d["shape"], d["h"], d["bc"], d["grid"], "fd")
        err = rel_err(phi[i].cpu().numpy(), ref)
        worst = max(worst, err)
        assert err <= 1e-12, (i, d, err)
    print(f"[parity] batch 2048: worst rel err over 64 grids {worst:.3e}", flush=True)
    plan.close()


# ------------------------------------------------------------------ captured graphs, autotuned plans
def test_graph_replay_matches_eager_and_oracle():
    """A graph-captured refinement plan replayed several times, with eager work and
    synchronisation between replays: every replay equals the eager result bit for bit
    and matches the oracle."""
    d = workloads.channel_desc(64, 32, 16)
    mp = _mp()
    eager = mp.Plan.from_desc(d, prec="f32r", max_iter=1)
    graph = mp.Plan.from_desc(d, prec="f32r", max_iter=1, graph=True)
    rhs = torch.empty(d["shape"], dtype=torch.float64, device="cuda")
    phi_g = torch.empty_like(rhs)
    for s in range(4):
        print(f"[parity] graph replay {s}", flush=True)
        rhs.copy_(workloads.channel_divergence(d, s, device="cuda"))
        ref_eager = eager.solve(rhs)
        graph.solve(rhs, phi_g)
        torch.cuda.synchronize()
        assert torch.equal(ref_eager, phi_g), s
        ref = oracle_solve(rhs.cpu().numpy(), d["shape"], d["h"], d["bc"], d["grid"], "fd")
        assert rel_err(phi_g.cpu().numpy(), ref) <= 1e-10
        _ = (rhs * 2.0).sum().item()  # unrelated eager work between replays


def test_graph_replay_new_buffers_recaptures():
    d = workloads.channel_desc(32, 16, 8)
    mp = _mp()
    graph = mp.Plan.from_desc(d, prec="f64", graph=True)
    for s in range(3):
        rhs = workloads.channel_divergence(d, s, device="cuda")
        out = graph.solve(rhs)  # a new phi every call
        torch.cuda.synchronize()
        ref = oracle_solve(rhs.cpu().numpy(), d["shape"], d["h"], d["bc"], d["grid"], "fd")
        assert rel_err(out.cpu().numpy(), ref) <= 1e-12


def test_autotuned_plan_matches_default():
    for kinds, shape in (([("N", "v")] * 3, (40, 66, 34)), ([("P", "v"), ("D", "s"), ("N", "s")], (64, 48, 80))):
        bc = tuple(k[0] for k in kinds)
        grid = tuple(k[1] for k in kinds)
        h = tuple(1.0 / n for n in shape)
        g = np.random.default_rng(12).standard_normal(shape)
        ref = oracle_solve(g, shape, h, bc, grid, "fd")
        for prec in ("f64", "f32r", "f32"):
            out, _ = gpu_solve(g, shape, h, bc, grid, "fd", prec, tune=True)
            assert rel_err(out, ref) <= TOL[prec], (kinds, prec)


def test_channel_full_size_first_and_last_rhs():
    """The 1024x512x256 channel with a graph-captured FP32+refinement plan, as
    streamed: right-hand sides #0 and #199 written into the captured buffer in
    turn, each against the oracle."""
    d = workloads.channel_desc()
    mp = _mp()
    plan = mp.Plan.from_desc(d, prec="f32r", max_iter=2, graph=True)
    rhs = torch.empty(d["shape"], dtype=torch.float64, device="cuda")
    phi = torch.empty_like(rhs)
    for s in (0, 199):
        print(f"[parity] channel 1024x512x256 rhs #{s}", flush=True)
        rhs.copy_(workloads.channel_divergence(d, s, device="cuda"))
        plan.solve(rhs, phi)
        info = plan.info()
        ref = oracle_solve(rhs.cpu().numpy(), d["shape"], d["h"], d["bc"], d["grid"], "fd")
        err = rel_err(phi.cpu().numpy(), ref)
        print(f"[parity] channel rhs #{s} rel err {err:.3e} resid {info['rel_resid']:.3e}", flush=True)
        assert err <= 1e-12, (s, err)


@pytest.mark.parametrize("variant", [0, 1, 2, 3])
def test_every_tuner_radix_plan_matches_oracle(variant, monkeypatch):
    """Each candidate radix plan the autotuner can choose (stage order reversed,
    one more power-of-two stage, Bluestein in place of Rader / radix 11-13),
    forced through MPOIS_TUNE_VARIANT, on lengths that have such variants."""
    monkeypatch.setenv("MPOIS_TUNE_VARIANT", str(variant))
    cases = [((147,), [("N", "v")]), ((512,), [("N", "v")]), ((74,), [("N", "v")]), ((72,), [("D", "v")]),
             ((143,), [("P", "v")]), ((1000,), [("N", "s")]), ((1024,), [("P", "v")]), ((120,), [("D", "s")]),
             ((40, 147, 26), [("N", "s"), ("N", "v"), ("P", "v")]), ((64, 52), [("D", "v"), ("N", "v")])]
    for shape, kinds in cases:
        bc = tuple(k[0] for k in kinds)
        grid = tuple(k[1] for k in kinds)
        h = tuple(1.0 / n for n in shape)
        g = np.random.default_rng(13).standard_normal(shape)
        ref = oracle_solve(g, shape, h, bc, grid, "fd")
        for prec in ("f64", "f32r", "f32"):
            print(f"[tuner variant {variant}] {shape} {kinds} {prec}", flush=True)
            out, _ = gpu_solve(g, shape, h, bc, grid, "fd", prec, tune=True)
            assert rel_err(out, ref) <= TOL[prec], (variant, shape, kinds, prec)


# ------------------------------------------------------------------ kernels specialised for one transform
SPEC_CASES = [
    ((512, 6, 512), ("N", "N", "N"), ("v", "v", "v")),      # 512-point DCT-I: forward and fused
    ((256, 4, 256), ("P", "D", "N"), ("v", "s", "s")),      # 256: DCT-II/III, fused real DFT
    ((4, 256, 256), ("P", "D", "N"), ("v", "s", "s")),      # 256: DST-II/III
    ((1024, 4, 256), ("P", "N", "P"), ("v", "s", "v")),     # 1024 fused real DFT, 256 real DFT
    ((4, 512, 256), ("P", "N", "P"), ("v", "s", "v")),      # 512: DCT-II/III
    ((32, 32, 32), ("P", "P", "P"), ("v", "v", "v")),       # 32-point real DFT
]


@pytest.mark.parametrize("prec", ["f64", "f32", "f32r"])
def test_specialised_kernels_match_generic_and_oracle(prec, monkeypatch):
    """Plans that use the kernels compiled for one transform against plans
    forced onto the generic shapes (MPOIS_NO_SPEC=1), and both against the oracle."""
    for shape, bc, grid in SPEC_CASES:
        h = tuple(1.0 / n for n in shape)
        g = np.random.default_rng(17).standard_normal(shape)
        print(f"[spec] {prec} {shape} {bc} {grid}", flush=True)
        monkeypatch.delenv("MPOIS_NO_SPEC", raising=False)
        out_s, _ = gpu_solve(g, shape, h, bc, grid, "fd", prec)
        monkeypatch.setenv("MPOIS_NO_SPEC", "1")
        out_g, _ = gpu_solve(g, shape, h, bc, grid, "fd", prec)
        monkeypatch.delenv("MPOIS_NO_SPEC")
        assert rel_err(out_s, out_g) <= (1e-5 if prec == "f32" else 1e-13), (shape, prec)
        ref = oracle_solve(g, shape, h, bc, grid, "fd")
        assert rel_err(out_s, ref) <= TOL[prec], (shape, prec)



# ------------------------------------------------------------------ different faces on one axis, Helmholtz shift
MIXED = [("DN", "v"), ("DN", "s"), ("ND", "v"), ("ND", "s")]
MIXED_LENGTHS = [1, 2, 3, 4, 5, 7, 8, 12, 16, 31, 32, 37, 64, 100, 127, 128, 255, 256, 257, 511, 512, 1000, 1024]


@pytest.mark.parametrize("kind", MIXED)
@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_1d_mixed_faces_all_lengths(kind, prec):
    """Dirichlet on one face and Neumann on the other: vertex DST-III/II and DCT-III/II,
    staggered DST-IV / DCT-IV (length-2n DFT of the modulated pair), FD and PS."""
    for n in MIXED_LENGTHS:
        for approx in ("fd", "ps"):
            check((n,), [kind], approx, prec, seed=n + 3)


@pytest.mark.parametrize("prec", ["f64", "f32", "f32r"])
def test_mixed_faces_2d_3d(prec):
    for k0, k1 in itertools.product(MIXED + [("P", "v"), ("N", "s")], repeat=2):
        check((21, 34), [k0, k1], "fd", prec, seed=5)
    for kinds in ([("DN", "s"), ("P", "v"), ("ND", "v")], [("ND", "s")] * 3, [("N", "v"), ("DN", "v"), ("D", "s")]):
        check((19, 24, 35), kinds, "fd", prec, seed=6)
        if prec != "f32r":
            check((19, 24, 35), kinds, "ps", prec, seed=6)


@pytest.mark.parametrize("prec", ["f64", "f32", "f32r"])
def test_helmholtz_shift(prec):
    """(Lap - sigma) phi = g: the shift joins the eigenvalue divisor (and the FP64
    residual of refinement); with sigma > 0 periodic / Neumann problems are not singular."""
    for kinds in ([("P", "v")] * 3, [("N", "v"), ("N", "s"), ("P", "v")], [("D", "s"), ("DN", "v"), ("N", "s")]):
        for shift in (0.5, 40.0):
            check((18, 23, 30), kinds, "fd", prec, seed=8, shift=shift)
            if prec != "f32r":
                check((18, 23, 30), kinds, "ps", prec, seed=9, shift=shift)
    # 512-point DCT-I axes (the specialised kernels) with a shift
    check((512, 6, 512), [("N", "v")] * 3, "fd", prec, seed=10, shift=3.0, h=(1 / 511,) * 3)


def test_batch_mixed_faces_and_shift():
    """Batch entries with mixed faces and their own shifts, FP32 + refinement."""
    rng = np.random.default_rng(12)
    descs = []
    for i in range(16):
        n0, n1 = int(rng.integers(8, 120)), int(rng.integers(8, 120))
        k0 = MIXED[i % 4]
        k1 = [("P", "v"), ("N", "s"), ("D", "v"), ("ND", "s")][i % 4]
        descs.append({"shape": (n0, n1), "h": (1.0 / n0, 1.0 / n1), "bc": (k0[0], k1[0]),
                      "grid": (k0[1], k1[1]), "approx": "fd", "shift": float(i % 3) * 2.0})
    mp = _mp()
    rhs = [torch.as_tensor(np.random.default_rng([12, i]).standard_normal(d["shape"])).cuda() for i, d in enumerate(descs)]
    phi = [torch.empty_like(r) for r in rhs]
    plan = mp.BatchPlan(descs, prec="f32r", max_iter=2)
    plan.solve(rhs, phi)
    torch.cuda.synchronize()
    for i, d in enumerate(descs):
        ref = oracle_solve(rhs[i].cpu().numpy(), d["shape"], d["h"], d["bc"], d["grid"], "fd", d["shift"])
        assert rel_err(phi[i].cpu().numpy(), ref) <= 1e-12, (i, d)
    assert plan.info()["rel_resid"] < 1e-11
    plan.close()
