"""GPU parity of the projection and the plain GPSS solver against the FP64
oracle, through the C ABI.

Tolerances (stated per dtype):
  * projection: FP64 vectors 1e-12 relative to max|v| (the threshold comes
    from a different summation order); FP32 vectors: output rounded to FP32,
    4 ulp of max|v|.
  * FP64 solver: relative objective gap <= 1e-10 and
    ||x - x_oracle|| / ||x_oracle|| <= 1e-6.  Both runs stop at the FP64
    stationarity floor, where either is ~1e-8 from the exact minimiser.
  * FP32 / BF16-storage solver: gap <= 1e-6 and x error <= 1e-4 against the
    oracle run on the same stored K (widened to FP64).
The gap is (f(x) - f*)/f* with f(x) recomputed in FP64 on the CPU from the
returned x, and f* the oracle's objective at its tight run.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import gpss, project_l1_mu
from paper_0902_4424_amd import gpl1, instances

pytestmark = pytest.mark.gpu

DEV = "cuda:0"


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def H():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    h = gpl1.Handle(0)
    yield h
    h.close()


def _dev(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(DEV)


def _K_tensor(inst):
    if inst.dtype == "bf16":
        return _dev(inst.K_store.view(np.int16))
    return _dev(inst.K_store)


def _gap_err(inst, x, ref):
    K, y = inst.K64, inst.y64
    x = np.asarray(x, dtype=np.float64)
    fx = float(np.sum((K @ x - y) ** 2))
    gap = (fx - ref["f"]) / ref["f"]
    err = np.linalg.norm(x - ref["x"]) / max(np.linalg.norm(ref["x"]), 1e-300)
    return gap, err, fx


# ---------------------------------------------------------------------------
# projection
# ---------------------------------------------------------------------------
PROJ_CASES = [
    # (p, scale of rho relative to ||v||_1, kind)
    (1, 0.5, "gauss"), (7, 0.3, "gauss"), (1000, 0.1, "gauss"), (1025, 0.5, "gauss"),
    (4096, 0.05, "ties"), (16384, 0.2, "wide"), (16384, 2.0, "gauss"),
    (40000, 0.3, "gauss"), (3000, 0.0, "gauss"), (5000, 1e-9, "wide"),
    (2048, 0.5, "zeros"), (20000, 0.2, "gauss"), (16383, 0.1, "wide"),
]


@pytest.mark.parametrize("p,frac,kind", PROJ_CASES)
@pytest.mark.parametrize("vdt", ["f64", "f32"])
def test_projection_matches_oracle(H, p, frac, kind, vdt):
    say(f"[proj] p={p} frac={frac} kind={kind} dtype={vdt}")
    rng = np.random.default_rng(p + int(frac * 1000))
    v = rng.standard_normal(p)
    if kind == "wide":
        v *= np.exp(rng.uniform(-12, 12, p))
    elif kind == "ties":
        v = rng.choice([-2.0, -1.0, 0.5, 1.0, 3.0], size=p)
    elif kind == "zeros":
        v[rng.random(p) < 0.7] = 0.0
    if vdt == "f32":
        v = v.astype(np.float32).astype(np.float64)
    rho = frac * np.abs(v).sum()
    want, mu_want = project_l1_mu(v, rho)
    vt = _dev(v, torch.float64 if vdt == "f64" else torch.float32)
    h, mu = H.project(vt, rho)
    got = h.cpu().double().numpy()
    scale = max(np.abs(v).max(), 1e-300)
    tol = 1e-12 * scale if vdt == "f64" else 4 * np.finfo(np.float32).eps * scale
    assert np.abs(got - want).max() <= tol
    assert abs(mu - mu_want) <= 1e-12 * scale
    assert np.abs(got).sum() <= rho * (1 + 1e-6) + 1e-300


def test_projection_inplace_and_empty(H):
    say("[proj] in-place and p=0")
    v = torch.tensor([3.0, 1.0], dtype=torch.float64, device=DEV)
    H.project(v, 1.0, out=v)
    assert v.cpu().tolist() == [1.0, 0.0]
    e = torch.empty(0, dtype=torch.float64, device=DEV)
    _, mu = H.project(e, 1.0)
    assert mu == 0.0
    with pytest.raises(gpl1.GPError):
        H.project(v, -1.0)


# ---------------------------------------------------------------------------
# hand-derived trajectories (same fixtures as the oracle pins)
# ---------------------------------------------------------------------------
def test_hand_examples_on_gpu(H):
    say("[solve] hand examples 2x2")
    for K, y, rho, iters, want in (
            ([[1.0, 0.0], [0.0, 0.5]], [1.0, 1.0], 100.0, 1, [1.0, 0.5]),
            ([[1.0, 0.0], [0.0, 0.5]], [1.0, 1.0], 100.0, 2, [1.0, 16 / 17]),
            ([[1.0, 0.0], [0.0, 0.1]], [1.0, 100.0], 1000.0, 2, [190.1 / 101, 2099 / 101]),
            ([[2.0]], [1.0], 10.0, 1, [0.5])):
        Kt = _dev(np.array(K))
        yt = _dev(np.array(y))
        x, res = H.solve(Kt, yt, rho, tol=0.0, max_iter=iters)
        np.testing.assert_allclose(x.cpu().numpy(), want, rtol=1e-13)
        assert res["iters"] == iters


# ---------------------------------------------------------------------------
# full solves
# ---------------------------------------------------------------------------
def test_fp64_gaussian_256x1024(H):
    say("[solve] gauss 256x1024 f64 tol=0 (stationary)")
    inst = instances.plain_small(seed=1, dtype="f64")
    ref = gpss(inst.K64, inst.y64, inst.rho, tol=0.0, max_iter=100000)
    x, res = H.solve(_K_tensor(inst), _dev(inst.y_store), inst.rho, tol=0.0)
    gap, err, fx = _gap_err(inst, x.cpu().numpy(), ref)
    say(f"   gpu iters={res['iters']} status={res['status_name']} oracle iters={ref['iters']} "
        f"gap={gap:.2e} err={err:.2e}")
    assert res["status_name"] == "stationary"
    assert gap <= 1e-10 and err <= 1e-6
    assert abs(res["f"] - fx) <= 1e-9 * fx
    assert res["l1norm"] <= inst.rho * (1 + 1e-12)
    lam = np.abs(inst.K64.T @ (inst.y64 - inst.K64 @ x.cpu().numpy())).max()
    assert res["lambda_est"] == pytest.approx(lam, rel=1e-6)


def test_fp64_tol_stop_matches_oracle_iteration_count(H):
    say("[solve] gauss 256x1024 f64 tol=1e-10")
    inst = instances.plain_small(seed=1, dtype="f64")
    ref = gpss(inst.K64, inst.y64, inst.rho, tol=1e-10)
    x, res = H.solve(_K_tensor(inst), _dev(inst.y_store), inst.rho, tol=1e-10)
    assert res["status_name"] == "ok_tol"
    # same trajectory up to rounding: the stop lands within a few iterations
    assert abs(res["iters"] - ref["iters"]) <= 5
    gap, err, _ = _gap_err(inst, x.cpu().numpy(), ref)
    assert abs(gap) <= 1e-8


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_reduced_precision_gaussian(H, dtype):
    say(f"[solve] gauss 1024x4096 {dtype}")
    inst = instances.gaussian_instance(1024, 4096, 50, amp="pm1", sigma=1e-2, dtype=dtype,
                                       seed=21)
    ref = gpss(inst.K64, inst.y64, inst.rho, tol=0.0, max_iter=100000)
    x, res = H.solve(_K_tensor(inst), _dev(inst.y_store), inst.rho, tol=1e-12,
                     refresh_every=50, max_iter=5000)
    gap, err, _ = _gap_err(inst, x.cpu().numpy(), ref)
    say(f"   gpu iters={res['iters']} status={res['status_name']} oracle iters={ref['iters']} "
        f"gap={gap:.2e} err={err:.2e}")
    assert gap <= 1e-6 and err <= 1e-4


def test_fp32_illconditioned(H):
    say("[solve] illcond 512 f32, 2000 iterations")
    inst = instances.plain_illcond(seed=3, dtype="f32", m=512)
    ref = gpss(inst.K64, inst.y64, inst.rho, tol=0.0, max_iter=2000)
    x, res = H.solve(_K_tensor(inst), _dev(inst.y_store), inst.rho, tol=0.0, max_iter=2000,
                     refresh_every=50)
    gap, err, _ = _gap_err(inst, x.cpu().numpy(), ref)
    tight = gpss(inst.K64, inst.y64, inst.rho, tol=0.0, max_iter=50000)
    g_gpu = (np.sum((inst.K64 @ x.cpu().numpy() - inst.y64) ** 2) - tight["f"]) / tight["f"]
    g_ora = (ref["f"] - tight["f"]) / tight["f"]
    say(f"   gpu gap={g_gpu:.2e} oracle gap={g_ora:.2e} at 2000 iterations")
    # ill-conditioned: both at a fixed budget; the GPU must be as close to f*
    # as the oracle is, within a factor 10 (or both at the 1e-6 target)
    assert g_gpu <= max(10 * g_ora, 1e-6)


# p covers every projection shape: 512 threads with 2..16 register slots,
# 1024 threads with 16 and 22 slots (ragged tails included), and the
# streamed form
@pytest.mark.parametrize("p", [1, 3, 1001, 4097, 8191, 16383, 20001, 30001])
def test_ragged_and_padded_shapes(H, p):
    say(f"[solve] ragged p={p}")
    n = 37
    inst = instances.gaussian_instance(n, p, min(3, p), dtype="f32", seed=100 + p)
    ref = gpss(inst.K64, inst.y64, inst.rho, tol=1e-13, max_iter=20000)
    # padded leading dimension (ldk = p + 3) exercises the unaligned loads
    Kp = np.zeros((n, p + 3), dtype=np.float32)
    Kp[:, :p] = inst.K_store
    Kt = _dev(Kp)[:, :p]
    # with n << p the ball's image can contain y (f* = 0 up to rounding, as
    # for p = 8191 here): the gap is then taken relative to 1e-3 ||y||^2
    scale = max(ref["f"], 1e-3 * float(inst.y64 @ inst.y64))
    x, res = H.solve(Kt, _dev(inst.y_store), inst.rho, tol=1e-13, max_iter=20000)
    _, _, fx = _gap_err(inst, x.cpu().numpy(), ref)
    assert (fx - ref["f"]) / scale <= 1e-6, (fx, ref["f"], res)
    x2, _ = H.solve(_dev(inst.K_store), _dev(inst.y_store), inst.rho, tol=1e-13, max_iter=20000)
    _, _, f2 = _gap_err(inst, x2.cpu().numpy(), ref)
    assert (f2 - ref["f"]) / scale <= 1e-6


# bf16 rows of p + 3 elements are 8-byte (p = 1001, 4097) or 4-byte (16383)
# aligned, unpadded rows of odd p only 2-byte aligned: every load width of
# the fused kernel's unaligned path
@pytest.mark.parametrize("p", [1001, 4097, 16383])
def test_bf16_ragged_and_unaligned_rows(H, p):
    say(f"[solve] bf16 ragged p={p}, padded and unpadded rows")
    n = 37
    inst = instances.gaussian_instance(n, p, 3, dtype="bf16", seed=300 + p)
    ref = gpss(inst.K64, inst.y64, inst.rho, tol=1e-13, max_iter=20000)
    scale = max(ref["f"], 1e-3 * float(inst.y64 @ inst.y64))
    Kp = np.zeros((n, p + 3), dtype=np.uint16)
    Kp[:, :p] = inst.K_store
    for Kt in (_dev(Kp.view(np.int16))[:, :p], _dev(inst.K_store.view(np.int16))):
        x, res = H.solve(Kt, _dev(inst.y_store), inst.rho, tol=1e-13, max_iter=20000)
        _, _, fx = _gap_err(inst, x.cpu().numpy(), ref)
        assert (fx - ref["f"]) / scale <= 1e-6, (fx, ref["f"], res)


def test_special_cases(H):
    say("[solve] special cases")
    inst = instances.gaussian_instance(64, 256, 5, dtype="f64", seed=9)
    K, y = _K_tensor(inst), _dev(inst.y_store)
    x, res = H.solve(K, y, 0.0)
    assert res["status_name"] == "stationary" and not x.any().item()
    x, res = H.solve(K, torch.zeros_like(y), 2.0)
    assert res["status_name"] == "stationary" and res["iters"] == 0
    x0 = _dev(np.random.default_rng(0).standard_normal(256) * 10)
    x, res = H.solve(K, y, 1.0, x0=x0, max_iter=1, tol=0.0)
    assert res["projected_x0"] == 1 and res["l1norm"] <= 1.0 + 1e-12
    x, res = H.solve(K, y, 1.0, max_iter=0)
    assert res["status_name"] == "max_iter" and res["iters"] == 0
    ref = gpss(inst.K64, inst.y64, 1.0, max_iter=3, tol=0.0)
    x, res = H.solve(K, y, 1.0, max_iter=3, tol=0.0)
    np.testing.assert_allclose(x.cpu().numpy(), ref["x"], atol=1e-12)
    # warm start from the oracle's answer stops almost at once
    ref = gpss(inst.K64, inst.y64, inst.rho, tol=0.0)
    x, res = H.solve(K, y, inst.rho, x0=_dev(ref["x"]), tol=1e-12)
    assert res["iters"] <= 3
    # f_target stop
    x, res = H.solve(K, y, inst.rho, tol=0.0, f_target=ref["f"] * 1.01)
    assert res["status_name"] == "reached_target" and res["f"] <= ref["f"] * 1.01


def test_errors(H):
    say("[solve] argument errors and non-finite data")
    inst = instances.gaussian_instance(16, 32, 2, dtype="f64", seed=2)
    K, y = _K_tensor(inst), _dev(inst.y_store)
    for bad in (dict(rho=-1.0), dict(rho=float("nan")), dict(tol=-1.0)):
        kw = dict(rho=1.0, tol=1e-10)
        kw.update(bad)
        with pytest.raises(gpl1.GPError) as e:
            H.solve(K, y, kw["rho"], tol=kw["tol"])
        assert e.value.code == -1
    with pytest.raises(gpl1.GPError):
        H.solve(K, y, 1.0, M=0)
    ybad = y.clone()
    ybad[3] = float("nan")
    with pytest.raises(gpl1.GPError) as e:
        H.solve(K, ybad, 1.0)
    assert e.value.code == -2
    # the handle still works after an error
    x, res = H.solve(K, y, 1.0)
    assert res["status"] >= 0


def test_deterministic(H):
    say("[solve] determinism")
    inst = instances.gaussian_instance(512, 2048, 20, dtype="f32", seed=5)
    K, y = _K_tensor(inst), _dev(inst.y_store)
    a, ra = H.solve(K, y, inst.rho, tol=0.0, max_iter=200)
    b, rb = H.solve(K, y, inst.rho, tol=0.0, max_iter=200)
    assert torch.equal(a, b) and ra == rb


def test_nonmonotone_memory(H):
    say("[solve] M=5 non-monotone line search")
    inst = instances.plain_small(seed=1, dtype="f64")
    from oracle import GPSSParams
    ref = gpss(inst.K64, inst.y64, inst.rho, tol=0.0, params=GPSSParams(M=5))
    x, res = H.solve(_K_tensor(inst), _dev(inst.y_store), inst.rho, tol=0.0, M=5)
    gap, err, _ = _gap_err(inst, x.cpu().numpy(), ref)
    assert gap <= 1e-10 and err <= 1e-6


def _golden(name):
    import os
    path = os.path.join(os.path.dirname(__file__), "golden", name)
    vals = {}
    for line in open(path):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        k, v = line.split("=")
        vals[k.strip()] = [float(t) for t in v.split()]
    return vals


@pytest.mark.parametrize("M", [1, 2, 3])
def test_nonmonotone_hand_example_on_gpu(H, M):
    """Algorithm 1 step 4 on the device, pinned by the hand-derived example
    (tests/golden/nonmonotone_hand_example.txt): K = diag(1, 3, 5), y = (5, 2, 1),
    rho = 100.  The second step raises f from 28.39 to 29.09; M = 1 rejects
    it (one reduction to lambda = 1/2), M = 2 and 3 accept it (f0 = 30 is
    still in the window)."""
    say(f"[solve] hand nonmonotone example M={M}")
    g = _golden("nonmonotone_hand_example.txt")
    K = torch.tensor(np.diag([1.0, 3.0, 5.0]), device=DEV)
    y = torch.tensor([5.0, 2.0, 1.0], dtype=torch.float64, device=DEV)
    x1, r1 = H.solve(K, y, 100.0, tol=0.0, max_iter=1, M=M)
    np.testing.assert_allclose(x1.cpu().numpy(), g["C.x1"], rtol=1e-14)
    assert r1["f"] == pytest.approx(g["C.f1"][0], rel=1e-14) and r1["backtracks"] == 0
    x2, r2 = H.solve(K, y, 100.0, tol=0.0, max_iter=2, M=M)
    assert r2["iters"] == 2
    if M == 1:
        assert r2["backtracks"] == 1
        assert r2["f"] == pytest.approx(g["C.f2_M1"][0], rel=1e-13)
        np.testing.assert_allclose(x2.cpu().numpy(), g["C.x2_M1"], rtol=1e-13)
    else:
        assert r2["backtracks"] == 0
        assert r2["f"] == pytest.approx(g["C.f2_M2"][0], rel=1e-13)
        assert r2["f"] > r1["f"]
        np.testing.assert_allclose(x2.cpu().numpy(), g["C.x2_M2"], rtol=1e-13)


# An ill-conditioned 32 x 32 problem (singular values 1 .. 1e-3) on which the
# line-search memory changes the path early: at k = 9 the step raises f by
# 16 % (M = 3) or 3x (M = 5); M = 1 needs two reductions there, M = 3 one,
# M = 5 none, and the iterates then stay apart by 1-10 %.
def _nonmono_instance():
    return instances.illcond_instance(32, 5, dtype="f64", seed=4, cond=1e3)


@pytest.mark.parametrize("k", [8, 10, 12, 16, 20])
def test_nonmonotone_trajectory_matches_oracle(H, k):
    """Trajectory level for M = 1, 3, 5: after k accepted updates the FP64
    iterate, objective and backtrack count equal the oracle's, and the three
    memories give different iterates once the memory matters (k > 9)."""
    from oracle import GPSSParams
    inst = _nonmono_instance()
    K, y = _K_tensor(inst), _dev(inst.y_store)
    xs, bts = {}, {}
    for M in (1, 3, 5):
        say(f"[solve] FP64 nonmonotone trajectory M={M} after {k} iterations")
        ref = gpss(inst.K64, inst.y64, inst.rho, tol=0.0, max_iter=k, params=GPSSParams(M=M))
        x, res = H.solve(K, y, inst.rho, tol=0.0, max_iter=k, M=M)
        assert res["iters"] == ref["iters"] == k
        assert res["backtracks"] == ref["backtracks"]
        xn = x.cpu().numpy()
        err = np.linalg.norm(xn - ref["x"]) / np.linalg.norm(ref["x"])
        assert err <= 1e-10, (M, err)
        assert abs(res["f"] - ref["f"]) <= 1e-10 * ref["f"]
        xs[M], bts[M] = xn, res["backtracks"]
    nx = np.linalg.norm(xs[1])
    if k > 9:
        assert bts[1] > bts[3] > bts[5]
        assert np.linalg.norm(xs[1] - xs[3]) > 1e-3 * nx
        assert np.linalg.norm(xs[3] - xs[5]) > 1e-3 * nx
    else:
        assert bts[1] == bts[3] == bts[5]
        assert np.array_equal(xs[1], xs[3]) and np.array_equal(xs[3], xs[5])


def test_sampled_profiling(H):
    say("[solve] timing every k-th fused launch; x unchanged by it")
    inst = instances.gaussian_instance(512, 2048, 20, dtype="f32", seed=5)
    K, y = _K_tensor(inst), _dev(inst.y_store)
    x0, r0 = H.solve(K, y, inst.rho, tol=0.0, max_iter=20)
    assert r0["iters"] == 20 and r0["n_fused"] == 0
    for k, want in ((1, 20), (4, 5), (7, 3), (25, 1)):
        x, r = H.solve(K, y, inst.rho, tol=0.0, max_iter=20, profile=k)
        assert r["n_fused"] == want and r["t_fused_ms"] > 0.0
        assert torch.equal(x, x0)
    with pytest.raises(gpl1.GPError):
        H.solve(K, y, inst.rho, profile=-1)


@pytest.mark.parametrize("k", [1, 2, 3, 5, 8, 13, 21, 34])
def test_fp64_trajectory_matches_oracle(H, k):
    """Trajectory level: after k accepted updates the FP64 iterate, objective
    and backtrack count equal the oracle's (the steplength branches and the
    line search take the same decisions while rounding stays far below the
    branch margins)."""
    say(f"[solve] FP64 trajectory after {k} iterations")
    inst = instances.plain_small(seed=1, dtype="f64")
    ref = gpss(inst.K64, inst.y64, inst.rho, tol=0.0, max_iter=k)
    x, res = H.solve(_K_tensor(inst), _dev(inst.y_store), inst.rho, tol=0.0, max_iter=k)
    assert res["iters"] == ref["iters"] == k
    assert res["backtracks"] == ref["backtracks"]
    xn = x.cpu().numpy()
    err = np.linalg.norm(xn - ref["x"]) / np.linalg.norm(ref["x"])
    say(f"   x rel err {err:.2e}, f rel diff {abs(res['f'] - ref['f']) / ref['f']:.2e}")
    assert err <= 1e-10
    assert abs(res["f"] - ref["f"]) <= 1e-10 * ref["f"]


def test_every_fused_shape_matches_oracle(H):
    """Every fused-kernel shape the autotuner may choose (threads, column
    chunks, row blocks, buffers, partial w in registers or LDS) and both row
    orders give the oracle's solution at the FP32 bar."""
    from paper_0902_4424_amd import tune
    inst = instances.gaussian_instance(1024, 4096, 50, dtype="f32", seed=15)
    ref = gpss(inst.K64, inst.y64, inst.rho, tol=0.0, max_iter=100000)
    K, y = _K_tensor(inst), _dev(inst.y_store)
    shapes = [c for c, (T, cpt) in tune.CFG_COVER.items() if T * cpt * 4 >= 4096]
    assert {10, 11, 12} <= set(shapes)
    for cfg in shapes:
        for grid, il in ((64, 0), (256, 1)):
            x, res = H.solve(K, y, inst.rho, tol=0.0, max_iter=5000, refresh_every=50,
                             fused_cfg=cfg, fused_grid=grid, fused_interleave=il)
            gap, err, _ = _gap_err(inst, x.cpu().numpy(), ref)
            assert gap <= 1e-6 and err <= 1e-4, (cfg, grid, il, gap, err)
    say(f"   {len(shapes)} shapes x 2 grids match")


def test_graph_mode_matches_plain(H):
    """Replaying captured chunks of iterations gives bit-identical results to
    plain launches: on the caller's null stream and on a stream of its own,
    with and without periodic refreshes, with a ragged last chunk, after a
    switch to another problem (re-capture) and back, and with plain solves
    in between the replays."""
    say("[solve] graph mode vs plain launches")
    a = instances.gaussian_instance(512, 2048, 20, dtype="f32", seed=5)
    b = instances.gaussian_instance(300, 1100, 9, dtype="f64", seed=6)
    Ka, ya = _K_tensor(a), _dev(a.y_store)
    Kb, yb = _K_tensor(b), _dev(b.y_store)
    side = torch.cuda.Stream()
    cases = [
        (Ka, ya, a.rho, dict(tol=0.0, max_iter=300), None),
        (Ka, ya, a.rho, dict(tol=0.0, max_iter=203, refresh_every=25), None),
        (Kb, yb, b.rho, dict(tol=1e-12, max_iter=5000, chunk=16), None),
        (Ka, ya, a.rho, dict(tol=0.0, max_iter=300), side),
        (Ka, ya, a.rho, dict(tol=1e-9, max_iter=100000), None),
    ]
    want = []
    for K, y, rho, kw, s in cases:
        with torch.cuda.stream(s or torch.cuda.current_stream()):
            want.append(H.solve(K, y, rho, stream=s, **kw))
        torch.cuda.synchronize()
    for rep in range(3):
        for i, (K, y, rho, kw, s) in enumerate(cases):
            with torch.cuda.stream(s or torch.cuda.current_stream()):
                x, r = H.solve(K, y, rho, stream=s, graph=1, **kw)
                xp, rp = H.solve(K, y, rho, stream=s, **kw)   # plain solve between replays
            torch.cuda.synchronize()
            x0, r0 = want[i]
            assert torch.equal(x, x0) and r == r0, (rep, i, r, r0)
            assert torch.equal(xp, x0) and rp == r0
    say(f"   {len(cases)} cases x 3 replays bit-identical")
    with pytest.raises(gpl1.GPError) as e:
        H.solve(Ka, ya, a.rho, graph=1, profile=4)
    assert e.value.code == -1


def test_lookahead_matches_chunked_polls(H):
    """Pacing the launches by the progress word the update kernel posts
    (lookahead k) changes only when the host enqueues: every stop kind (the
    tolerance, the budget, stationarity, an objective target checked in
    double) gives the bits of the chunked polls, for several k, through both
    entry points, with profiling and refreshes, and an invalid k is refused."""
    say("[solve] lookahead pacing vs chunked polls")
    a = instances.gaussian_instance(512, 2048, 20, dtype="f32", seed=5)
    b = instances.gaussian_instance(300, 1100, 9, dtype="f64", seed=6)
    Ka, ya = _K_tensor(a), _dev(a.y_store)
    Kb, yb = _K_tensor(b), _dev(b.y_store)
    xs, rs = H.solve(Ka, ya, a.rho, tol=0.0, max_iter=3000, lookahead=0)
    target = rs["f"] * (1 + 1e-7)
    cases = [
        (Ka, ya, a.rho, dict(tol=0.0, max_iter=300)),
        (Ka, ya, a.rho, dict(tol=0.0, max_iter=203, refresh_every=25, profile=4)),
        (Kb, yb, b.rho, dict(tol=1e-12, max_iter=5000)),
        (Ka, ya, a.rho, dict(tol=1e-9, max_iter=100000)),
        (Ka, ya, a.rho, dict(tol=0.0, max_iter=5000, refresh_every=50, f_target=target)),
        (Ka, ya, a.rho, dict(tol=0.0, max_iter=1)),
        (Ka, ya, a.rho, dict(tol=0.0, max_iter=0)),
    ]
    timing = ("t_fused_ms",)
    for i, (K, y, rho, kw) in enumerate(cases):
        x0, r0 = H.solve(K, y, rho, lookahead=0, **kw)
        x1, r1 = H.solve(K, y, rho, lookahead=0, chunk=1, **kw)
        assert torch.equal(x1, x0)
        for la in (1, 2, 5):
            # (the allocation-free entry point takes no profiling)
            for fn in (H.solve,) if "profile" in kw else (H.solve, H.solve_noalloc):
                x, r = fn(K, y, rho, lookahead=la, **kw)
                torch.cuda.synchronize()
                assert torch.equal(x, x0), (i, la)
                assert {k: v for k, v in r.items() if k not in timing} == \
                    {k: v for k, v in r0.items() if k not in timing}, (i, la, r, r0)
        say(f"   case {i}: {r0['iters']} iterations, {r0['status_name']}, reopened {r0['reopened']}")
    with pytest.raises(gpl1.GPError) as e:
        H.solve(Ka, ya, a.rho, lookahead=-1)
    assert e.value.code == -1
