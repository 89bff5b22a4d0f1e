"""GPU parity of the batched solvers against the FP64 oracle (through the C ABI).

Shared K (bf16 storage, matrix-core GEMMs with three-plane bf16 operands):
every column must meet the FP32-path bar against the oracle run on the same
stored K widened to FP64: relative objective gap <= 1e-6 and
||x - x_oracle|| / ||x_oracle|| <= 1e-4.
"""
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import gpss
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


def _kt(batch):
    return torch.from_numpy(batch.K_store.view(np.int16)).to(DEV)


def _check_columns(batch, X, res, cols, tight_iters=100000, gap_tol=1e-6, err_tol=1e-4):
    K64 = batch.K64
    Xn = X.cpu().double().numpy()
    worst_gap = worst_err = 0.0
    for b in cols:
        y = batch.Y_store[b].astype(np.float64)
        ref = gpss(K64, y, float(batch.rho[b]), tol=0.0, max_iter=tight_iters)
        x = Xn[b]
        fx = float(np.sum((K64 @ x - y) ** 2))
        gap = (fx - ref["f"]) / ref["f"]
        err = np.linalg.norm(x - ref["x"]) / np.linalg.norm(ref["x"])
        worst_gap, worst_err = max(worst_gap, gap), max(worst_err, err)
        assert res[b]["status"] >= 0
        assert abs(res[b]["l1norm"] - np.abs(x).sum()) <= 1e-6 * max(1.0, batch.rho[b])
        assert np.abs(x).sum() <= batch.rho[b] * (1 + 1e-6)
    say(f"   worst gap {worst_gap:.2e}, worst x err {worst_err:.2e} over {len(cols)} columns")
    assert worst_gap <= gap_tol and worst_err <= err_tol


# p = 3001 and 5001 take the 512-thread column kernel with 8 and 16 slots
# per thread, both with a ragged last pair
@pytest.mark.parametrize("n,p,B", [(256, 1024, 5), (200, 700, 3), (130, 260, 129), (300, 3001, 5),
                                   (260, 5001, 3)])
def test_shared_small_matches_oracle(H, n, p, B):
    say(f"[batched-shared] n={n} p={p} B={B} bf16")
    batch = instances.shared_batch(n, p, B, max(1, n // 20), dtype="bf16", seed=31 + n,
                                   rhs_seed_base=700 + p)
    Y = torch.from_numpy(batch.Y_store).to(DEV)
    X, res = H.solve_batched_shared(_kt(batch), Y, batch.rho, tol=1e-12, max_iter=3000,
                                    refresh_every=50)
    cols = list(range(B)) if B <= 8 else [0, 1, B // 2, B - 1]
    _check_columns(batch, X, res, cols)


@pytest.mark.parametrize("n,p", [(128, 2048), (128, 2049), (160, 4096), (160, 4097), (256, 8192),
                                 (256, 8193), (1024, 600), (1025, 600), (2048, 600), (2049, 600)])
def test_shared_column_shape_boundaries(H, n, p):
    """Both sides of every switch of the per-problem kernels' shapes (columns:
    256 x 8, 512 x 8, 512 x 16 and 1024 x 16 threads x slots; rows: 4 or 8
    rows per thread in registers, or q parked in memory above n = 2048) meet
    the FP32-path bar."""
    say(f"[batched-shared] shape boundary n={n} p={p} B=2 bf16")
    batch = instances.shared_batch(n, p, 2, max(1, n // 20), dtype="bf16", seed=31 + n,
                                   rhs_seed_base=900 + p)
    Y = torch.from_numpy(batch.Y_store).to(DEV)
    X, res = H.solve_batched_shared(_kt(batch), Y, batch.rho, tol=1e-12, max_iter=3000,
                                    refresh_every=50)
    assert all(r["status"] >= 0 for r in res)
    _check_columns(batch, X, res, [0, 1])


def test_shared_refresh_and_warm_start(H):
    say("[batched-shared] refresh every 7, warm start from the answer")
    batch = instances.shared_batch(256, 1024, 4, 12, dtype="bf16", seed=8, rhs_seed_base=80)
    Y = torch.from_numpy(batch.Y_store).to(DEV)
    X, res = H.solve_batched_shared(_kt(batch), Y, batch.rho, tol=1e-12, max_iter=3000,
                                    refresh_every=7)
    _check_columns(batch, X, res, range(4))
    X2, res2 = H.solve_batched_shared(_kt(batch), Y, batch.rho, X0=X.clone(), tol=1e-12,
                                      max_iter=3000, refresh_every=50)
    assert max(r["iters"] for r in res2) <= max(5, min(r["iters"] for r in res) // 2)
    _check_columns(batch, X2, res2, range(4))


def test_shared_agrees_with_single_solves(H):
    say("[batched-shared] vs plain solver on each column")
    batch = instances.shared_batch(512, 2048, 3, 25, dtype="bf16", seed=9, rhs_seed_base=90)
    Kt = _kt(batch)
    Y = torch.from_numpy(batch.Y_store).to(DEV)
    X, res = H.solve_batched_shared(Kt, Y, batch.rho, tol=1e-13, max_iter=5000, refresh_every=50)
    K64 = batch.K64
    for b in range(3):
        xs, rs = H.solve(Kt, Y[b].contiguous(), float(batch.rho[b]), tol=1e-13, max_iter=5000,
                         refresh_every=50)
        y = batch.Y_store[b].astype(np.float64)
        fb = np.sum((K64 @ X[b].cpu().double().numpy() - y) ** 2)
        fs = np.sum((K64 @ xs.cpu().double().numpy() - y) ** 2)
        assert abs(fb - fs) <= 1e-6 * fs


def test_shared_special_columns(H):
    say("[batched-shared] rho = 0, y = 0 and max_iter stop in one batch")
    batch = instances.shared_batch(128, 512, 4, 6, dtype="bf16", seed=10, rhs_seed_base=100)
    Y = torch.from_numpy(batch.Y_store).to(DEV)
    Y[1] = 0.0
    rho = list(batch.rho)
    rho[0] = 0.0
    X, res = H.solve_batched_shared(_kt(batch), Y, rho, tol=0.0, max_iter=4)
    assert res[0]["status_name"] == "stationary" and not X[0].any().item()
    assert res[1]["status_name"] == "stationary" and res[1]["iters"] == 0
    assert res[2]["status_name"] == "max_iter" and res[2]["iters"] == 4
    ref = gpss(batch.K64, batch.Y_store[2].astype(np.float64), float(batch.rho[2]), tol=0.0,
               max_iter=4)
    np.testing.assert_allclose(X[2].cpu().double().numpy(), ref["x"], rtol=0, atol=1e-5)


def test_shared_large_sampled(H):
    say("[batched-shared] 2048 x 8192 bf16, 64 right-hand sides, 3 sampled columns")
    batch = instances.shared_batch(2048, 8192, 64, 102, dtype="bf16", seed=5, rhs_seed_base=5000)
    Y = torch.from_numpy(batch.Y_store).to(DEV)
    X, res = H.solve_batched_shared(_kt(batch), Y, batch.rho, tol=1e-12, max_iter=5000,
                                    refresh_every=50)
    assert all(r["status"] >= 0 for r in res)
    _check_columns(batch, X, res, [0, 31, 63], tight_iters=20000)


@pytest.mark.parametrize("n,p,B", [(256, 1024, 4), (190, 650, 130), (300, 3001, 4)])
def test_shared_f32_matches_oracle(H, n, p, B):
    say(f"[batched-shared] FP32 K as three bf16 planes n={n} p={p} B={B}")
    batch = instances.shared_batch(n, p, B, max(1, n // 20), dtype="f32", seed=61 + n,
                                   rhs_seed_base=610 + p)
    Kt = torch.from_numpy(batch.K_store).to(DEV)
    Y = torch.from_numpy(batch.Y_store).to(DEV)
    X, res = H.solve_batched_shared(Kt, Y, batch.rho, tol=1e-12, max_iter=4000, refresh_every=50)
    cols = list(range(B)) if B <= 8 else [0, 1, B // 2, B - 1]
    _check_columns(batch, X, res, cols)


def test_shared_per_problem_targets(H):
    say("[batched-shared] one f_target per problem")
    batch = instances.shared_batch(200, 800, 6, 10, dtype="f32", seed=71, rhs_seed_base=710)
    Kt = torch.from_numpy(batch.K_store).to(DEV)
    Y = torch.from_numpy(batch.Y_store).to(DEV)
    K64 = batch.K64
    fref = [gpss(K64, batch.Y_store[b].astype(np.float64), float(batch.rho[b]), tol=0.0,
                 max_iter=20000)["f"] for b in range(6)]
    gaps = [1e-2, 1e-4, 1e-6, 1e-3, 1e-5, 1e-6]
    targets = [f * (1 + g) for f, g in zip(fref, gaps)]
    X, res = H.solve_batched_shared(Kt, Y, batch.rho, tol=0.0, max_iter=20000, refresh_every=50,
                                    f_targets=targets)
    for b in range(6):
        assert res[b]["status_name"] == "reached_target", res[b]
        fx = float(np.sum((K64 @ X[b].cpu().double().numpy() - batch.Y_store[b]) ** 2))
        # a target stop is checked on the device in double from the returned
        # x: the host's FP64 value agrees to summation order and meets it
        assert fx <= targets[b] * (1 + 1e-13)
        assert abs(res[b]["f"] - fx) <= 1e-12 * fx
    its = [r["iters"] for r in res]
    say(f"   iterations per target gap: {list(zip(gaps, its))}")
    assert its[0] < its[2] and its[3] < its[1]
    # the same targets through the uneven-batch entry point
    probs = [(Kt, Y[b], float(batch.rho[b])) for b in range(6)]
    Xv, rv = H.solve_batched_var(probs, tol=0.0, max_iter=20000, refresh_every=50, f_targets=targets)
    assert all(r["status_name"] == "reached_target" for r in rv)
    for b in range(6):
        fx = float(np.sum((K64 @ Xv[b].cpu().double().numpy() - batch.Y_store[b]) ** 2))
        assert fx <= targets[b] * (1 + 1e-13)
        assert abs(rv[b]["f"] - fx) <= 1e-12 * fx
    with pytest.raises(ValueError):
        H.solve_batched_shared(Kt, Y, batch.rho, f_targets=targets[:5])


def _nonmono_batch():
    # the ill-conditioned 32 x 32 operator on which M changes the path at
    # k = 9, stored FP32, with three right-hand sides: the instance's own y
    # and two more from fresh 5-sparse signals
    inst = instances.illcond_instance(32, 5, dtype="f32", seed=4, cond=1e3)
    rng = np.random.default_rng(44)
    ys, rhos = [inst.y_store], [inst.rho]
    for _ in range(2):
        x = np.zeros(32)
        x[rng.choice(32, 5, replace=False)] = rng.choice([-1.0, 1.0], 5)
        ys.append((inst.K64 @ x + 1e-3 * rng.standard_normal(32)).astype(np.float32))
        rhos.append(float(np.abs(x).sum()))
    return inst, np.stack(ys), rhos


@pytest.mark.parametrize("k", [12, 16])
def test_shared_nonmonotone_trajectory(H, k):
    """Line-search memory M = 1, 3, 5 in the shared-K batch (FP32 K as three
    bf16 planes): after k iterations every column's backtrack count equals the
    oracle's and its iterate is within the FP32 bar of the oracle's k-th
    iterate; on the first column M changes the path (the iterates differ by
    far more than that bar)."""
    from oracle import GPSSParams
    inst, Ys, rhos = _nonmono_batch()
    Kt = torch.from_numpy(inst.K_store).to(DEV)
    Y = torch.from_numpy(Ys).to(DEV)
    xs = {}
    for M in (1, 3, 5):
        say(f"[batched-shared] nonmonotone M={M}, {k} iterations, 3 columns")
        X, res = H.solve_batched_shared(Kt, Y, rhos, tol=0.0, max_iter=k, M=M)
        Xn = X.cpu().double().numpy()
        for b in range(3):
            ref = gpss(inst.K64, Ys[b].astype(np.float64), rhos[b], tol=0.0, max_iter=k,
                       params=GPSSParams(M=M))
            assert res[b]["iters"] == ref["iters"] == k
            assert res[b]["backtracks"] == ref["backtracks"], (M, b)
            err = np.linalg.norm(Xn[b] - ref["x"]) / np.linalg.norm(ref["x"])
            assert err <= 1e-4, (M, b, err)
        xs[M] = Xn[0]
    nx = np.linalg.norm(xs[1])
    assert np.linalg.norm(xs[1] - xs[3]) > 1e-3 * nx
    assert np.linalg.norm(xs[3] - xs[5]) > 1e-3 * nx


@pytest.mark.parametrize("k", [10, 16])
def test_var_nonmonotone_trajectory(H, k):
    """M = 1, 3, 5 in the uneven batch (FP64): the hand-derived 3 x 3 example
    of Algorithm 1 step 4, the ill-conditioned 32 x 32 problem and a Gaussian
    problem in one batch; after k iterations iterates and backtrack counts
    equal the oracle's."""
    from oracle import GPSSParams
    ill = instances.illcond_instance(32, 5, dtype="f64", seed=4, cond=1e3)
    gau = instances.gaussian_instance(96, 384, 6, dtype="f64", seed=45)
    Kc = np.diag([1.0, 3.0, 5.0])
    yc = np.array([5.0, 2.0, 1.0])
    cases = [(Kc, yc, 100.0), (ill.K64, ill.y64, ill.rho), (gau.K64, gau.y64, gau.rho)]
    probs = [(torch.from_numpy(np.ascontiguousarray(K)).to(DEV), torch.from_numpy(y).to(DEV), r)
             for K, y, r in cases]
    xs = {}
    for M in (1, 3, 5):
        say(f"[batched-var] nonmonotone M={M}, {k} iterations")
        X, res = H.solve_batched_var(probs, tol=0.0, max_iter=k, M=M)
        for i, (K, y, r) in enumerate(cases):
            ref = gpss(K, y, r, tol=0.0, max_iter=k, params=GPSSParams(M=M))
            assert res[i]["iters"] == ref["iters"], (M, i)
            assert res[i]["backtracks"] == ref["backtracks"], (M, i)
            x = X[i].cpu().numpy()
            err = np.linalg.norm(x - ref["x"]) / np.linalg.norm(ref["x"])
            assert err <= 1e-10, (M, i, err)
        xs[M] = X[1].cpu().numpy()
    nx = np.linalg.norm(xs[1])
    assert np.linalg.norm(xs[1] - xs[3]) > 1e-3 * nx
    assert np.linalg.norm(xs[3] - xs[5]) > 1e-3 * nx


def _warm_like_batch(B, seed):
    # the learned-start workload's regime: K 1024 x 4096 FP32 N(0, 1/1024),
    # 50-sparse +-1 signals, noise 1e-2 (residual about 1 % of K x)
    return instances.shared_batch(1024, 4096, B, 50, dtype="f32", seed=seed, rhs_seed_base=100 * seed)


@pytest.mark.parametrize("entry", ["shared", "var"])
def test_target_stops_hold_in_double(H, entry):
    """A stop at f <= f_target holds for f recomputed in FP64 on the host from
    the returned x, at a 1e-6 gap above the oracle's f*, on the workload where
    the tracked f undershoots most (residual ~1 % of K x).  Stops that the
    device's double check overturns iterate on (result.reopened counts them)."""
    say(f"[target] 1e-6 gap, 24 problems, {entry} entry point")
    batch = _warm_like_batch(24, 12)
    Kt = torch.from_numpy(batch.K_store).to(DEV)
    Y = torch.from_numpy(batch.Y_store).to(DEV)
    K64 = batch.K64
    fstar = [gpss(K64, batch.Y_store[b].astype(np.float64), float(batch.rho[b]), tol=0.0,
                  max_iter=20000)["f"] for b in range(24)]
    targets = [f * (1 + 1e-6) for f in fstar]
    if entry == "shared":
        X, res = H.solve_batched_shared(Kt, Y, batch.rho, tol=0.0, max_iter=5000, refresh_every=50,
                                        f_targets=targets)
    else:
        probs = [(Kt, Y[b], float(batch.rho[b])) for b in range(24)]
        X, res = H.solve_batched_var(probs, tol=0.0, max_iter=5000, refresh_every=50, f_targets=targets)
    worst = 0.0
    for b in range(24):
        assert res[b]["status_name"] == "reached_target", (b, res[b])
        x = X[b].cpu().double().numpy()
        fx = float(np.sum((K64 @ x - batch.Y_store[b]) ** 2))
        assert fx <= targets[b] * (1 + 1e-13), (b, (fx - fstar[b]) / fstar[b])
        assert abs(res[b]["f"] - fx) <= 1e-12 * fx
        worst = max(worst, (fx - fstar[b]) / fstar[b])
    say(f"   worst host gap {worst:.3e}; reopened {sum(r['reopened'] for r in res)} stops")
    assert worst <= 1e-6


def test_target_stop_holds_single(H):
    """The single-problem solver's target stop, checked the same way, on
    several right-hand sides of the same workload (FP32 K)."""
    batch = _warm_like_batch(6, 13)
    Kt = torch.from_numpy(batch.K_store).to(DEV)
    K64 = batch.K64
    reopened = 0
    for b in range(6):
        say(f"[target] single solve, right-hand side {b}")
        y = torch.from_numpy(np.ascontiguousarray(batch.Y_store[b])).to(DEV)
        fstar = gpss(K64, batch.Y_store[b].astype(np.float64), float(batch.rho[b]), tol=0.0,
                     max_iter=20000)["f"]
        target = fstar * (1 + 1e-6)
        x, res = H.solve(Kt, y, float(batch.rho[b]), tol=0.0, max_iter=5000, refresh_every=50,
                         f_target=target)
        assert res["status_name"] == "reached_target", res
        fx = float(np.sum((K64 @ x.cpu().double().numpy() - batch.Y_store[b]) ** 2))
        assert fx <= target * (1 + 1e-13)
        assert abs(res["f"] - fx) <= 1e-12 * fx
        reopened += res["reopened"]
        # the same through the allocation-free entry point: the same bits
        x2, res2 = H.solve_noalloc(Kt, y, float(batch.rho[b]), tol=0.0, max_iter=5000,
                                   refresh_every=50, f_target=target)
        assert torch.equal(x, x2) and res2 == res
    say(f"   reopened {reopened} stops")


@pytest.mark.parametrize("dtype", ["bf16", "f32"])
def test_shared_active_set_is_exact(H, dtype):
    say(f"[batched-shared] finished problems dropped from the launches ({dtype}): same bits")
    batch = instances.shared_batch(192, 700, 300, 8, dtype=dtype, seed=81, rhs_seed_base=810)
    Kt = _kt(batch) if dtype == "bf16" else torch.from_numpy(batch.K_store).to(DEV)
    Y = torch.from_numpy(batch.Y_store).to(DEV)
    rho = list(batch.rho)
    rho[3] = 0.0                       # finishes at once
    Y[7] = 0.0
    kw = dict(tol=1e-9, max_iter=3000, refresh_every=20)
    Xa, ra = H.solve_batched_shared(Kt, Y, rho, chunk=3, **kw)       # polls (and compacts) often
    Xb, rb = H.solve_batched_shared(Kt, Y, rho, chunk=10 ** 6, **kw)  # never compacts
    assert torch.equal(Xa, Xb)
    assert [r["iters"] for r in ra] == [r["iters"] for r in rb]
    its = [r["iters"] for r in ra]
    say(f"   iterations min {min(its)} mean {np.mean(its):.1f} max {max(its)}")
    assert min(its) < max(its)
    _check_columns(batch, Xa, ra, [0, 150, 299])


# ---------------------------------------------------------------------------
# independent problems of different sizes (lockstep batch)
# ---------------------------------------------------------------------------
def _var_problems(insts, dtype):
    probs = []
    for inst in insts:
        if dtype == "bf16":
            K = torch.from_numpy(inst.K_store.view(np.int16)).to(DEV)
        else:
            K = torch.from_numpy(inst.K_store).to(DEV)
        probs.append((K, torch.from_numpy(inst.y_store).to(DEV), inst.rho))
    return probs


def _check_var(insts, X, res, idx, gap_tol, err_tol):
    worst = [0.0, 0.0]
    for i in idx:
        inst = insts[i]
        ref = gpss(inst.K64, inst.y64, inst.rho, tol=0.0, max_iter=100000)
        x = X[i].cpu().double().numpy()
        fx = float(np.sum((inst.K64 @ x - inst.y64) ** 2))
        gap = (fx - ref["f"]) / ref["f"]
        err = np.linalg.norm(x - ref["x"]) / np.linalg.norm(ref["x"])
        worst = [max(worst[0], gap), max(worst[1], err)]
        assert res[i]["status"] >= 0
        assert np.abs(x).sum() <= inst.rho * (1 + 1e-6)
    say(f"   worst gap {worst[0]:.2e}, worst x err {worst[1]:.2e}")
    assert worst[0] <= gap_tol and worst[1] <= err_tol


@pytest.mark.parametrize("dtype", ["bf16", "f32", "f64"])
def test_var_small_matches_oracle(H, dtype):
    say(f"[batched-var] 7 uneven problems {dtype}")
    rng = np.random.default_rng(77)
    ns = rng.integers(16, 300, size=7)
    # odd and even n: with p = 4n, bf16 rows are 8-byte aligned for odd n
    # (read as four-element chunks) and 16-byte aligned for even n
    assert (ns % 2 == 1).any() and (ns % 2 == 0).any()
    insts = [instances.gaussian_instance(int(n), 4 * int(n), max(1, int(n) // 20), sigma=1e-2,
                                         dtype=dtype, seed=900 + i)
             for i, n in enumerate(ns)]
    X, res = H.solve_batched_var(_var_problems(insts, dtype), tol=1e-13, max_iter=5000,
                                 refresh_every=0 if dtype == "f64" else 50)
    tol = (1e-10, 1e-6) if dtype == "f64" else (1e-6, 1e-4)
    _check_var(insts, X, res, range(7), *tol)


@pytest.mark.parametrize("dtype", ["bf16", "f32"])
def test_var_wave_pass_matches_oracle(H, dtype):
    """Narrow problems (p <= 1024) run the fused pass one row per wave, each
    wave leaving its own partial vector: checked against the oracle when every
    problem is narrow (one column chunk per thread), beside a wide problem (two
    chunks), with items of 16 rows and with items whose last rows leave waves
    empty (n = 130, 131 at 64-row items), and beside the workgroup-wide pass
    (var_wave_rows = -1) on the same problems."""
    rng = np.random.default_rng(79)
    narrow = [130, 131] + [int(n) for n in rng.integers(20, 257, size=4)]
    for label, ns, kw in (("all narrow", narrow, {}), ("all narrow, 16-row items", narrow, dict(var_item_rows=16)),
                          ("beside a wide problem", narrow + [700], {}),
                          ("workgroup pass", narrow, dict(var_wave_rows=-1))):
        say(f"[batched-var] wave pass {dtype}: {label}")
        insts = [instances.gaussian_instance(n, 4 * n, max(1, n // 20), sigma=1e-2, dtype=dtype, seed=970 + i)
                 for i, n in enumerate(ns)]
        X, res = H.solve_batched_var(_var_problems(insts, dtype), tol=1e-13, max_iter=5000, refresh_every=50, **kw)
        _check_var(insts, X, res, range(len(ns)), 1e-6, 1e-4)


def test_var_uneven_sampled(H):
    say("[batched-var] 64 problems, n in [128, 1024], p = 4n, bf16; 4 sampled")
    insts = instances.uneven_batch(64, dtype="bf16", seed=4)
    X, res = H.solve_batched_var(_var_problems(insts, "bf16"), tol=1e-12, max_iter=5000,
                                 refresh_every=50)
    assert all(r["status"] >= 0 for r in res)
    big = int(np.argmax([i.n for i in insts]))
    # problems 0 and 17 have odd n (8-byte aligned bf16 rows), 40 and the
    # largest even n
    assert insts[0].n % 2 == 1 and insts[17].n % 2 == 1 and insts[40].n % 2 == 0
    _check_var(insts, X, res, [0, 17, 40, big], 1e-6, 1e-4)


def test_var_special_and_padded(H):
    say("[batched-var] rho = 0, y = 0, padded leading dimension, warm start")
    insts = [instances.gaussian_instance(40, 160, 3, dtype="f32", seed=1000 + i) for i in range(4)]
    probs = _var_problems(insts, "f32")
    Kp = torch.zeros(40, 163, dtype=torch.float32, device=DEV)
    Kp[:, :160] = probs[2][0]
    probs[2] = (Kp[:, :160], probs[2][1], probs[2][2])
    probs[0] = (probs[0][0], probs[0][1], 0.0)
    probs[1] = (probs[1][0], torch.zeros_like(probs[1][1]), probs[1][2])
    X, res = H.solve_batched_var(probs, tol=1e-13, max_iter=5000, refresh_every=50)
    assert res[0]["status_name"] == "stationary" and not X[0].any().item()
    assert res[1]["status_name"] == "stationary" and res[1]["iters"] == 0
    _check_var(insts, X, res, [2, 3], 1e-6, 1e-4)
    # warm start from the answer
    probs3 = [(probs[3][0], probs[3][1], probs[3][2], X[3].clone())]
    X2, res2 = H.solve_batched_var(probs3, tol=1e-13, max_iter=5000, refresh_every=50)
    assert res2[0]["iters"] <= max(5, res[3]["iters"] // 2)


def test_binding_rejects_bad_shapes_before_launch(H):
    """The binding's argument checks: a short or wrongly typed y or x0, a
    column-major K, a radius list of the wrong length and a mis-shaped out are
    refused (ValueError) before the library reads any device memory."""
    K = torch.zeros(8, 32, dtype=torch.float32, device=DEV)
    y = torch.zeros(8, dtype=torch.float32, device=DEV)
    with pytest.raises(ValueError):
        H.solve_batched_var([(K, y[:7], 1.0)])
    with pytest.raises(ValueError):
        H.solve_batched_var([(K, y.double(), 1.0)])
    with pytest.raises(ValueError):
        H.solve_batched_var([(K, y, 1.0, torch.zeros(31, device=DEV))])
    Y = torch.zeros(3, 8, dtype=torch.float32, device=DEV)
    with pytest.raises(ValueError):
        H.solve_batched_shared(K, Y, [1.0, 1.0])
    with pytest.raises(ValueError):
        H.solve_batched_shared(K.t().contiguous().t(), Y, [1.0] * 3)
    with pytest.raises(ValueError):
        H.solve_batched_shared(K, Y, [1.0] * 3, out=torch.zeros(3, 31, device=DEV))


def test_batched_graph_replay_is_bit_identical(H):
    """opts.graph = 1 in both batched solvers: captured chunks (re-captured in
    the shared-K solver whenever finished problems leave the launches) give the
    same bits and counters as plain launches, on the null stream and on a
    stream of the caller's, with refreshes, per-problem targets (whose checks
    may reopen problems between chunks) and a ragged last chunk."""
    batch = instances.shared_batch(192, 700, 40, 8, dtype="f32", seed=83, rhs_seed_base=830)
    Kt = torch.from_numpy(batch.K_store).to(DEV)
    Y = torch.from_numpy(batch.Y_store).to(DEV)
    K64 = batch.K64
    fref = [gpss(K64, batch.Y_store[b].astype(np.float64), float(batch.rho[b]), tol=0.0,
                 max_iter=20000)["f"] for b in range(0, 40, 8)]
    # targets for every 8th problem (the others run to their floor)
    targets = [fref[b // 8] * (1 + 1e-6) if b % 8 == 0 else -1.0 for b in range(40)]
    side = torch.cuda.Stream()
    cases = [dict(tol=1e-9, max_iter=3000, refresh_every=20),
             dict(tol=0.0, max_iter=3000, refresh_every=20, f_targets=targets),
             dict(tol=1e-9, max_iter=203, refresh_every=0, chunk=16)]
    for i, kw in enumerate(cases):
        for s in (None, side):
            say(f"[graph] shared-K case {i}, {'caller stream' if s else 'null stream'}")
            with torch.cuda.stream(s or torch.cuda.current_stream()):
                Xa, ra = H.solve_batched_shared(Kt, Y, batch.rho, stream=s, **kw)
                Xb, rb = H.solve_batched_shared(Kt, Y, batch.rho, stream=s, graph=1, **kw)
            torch.cuda.synchronize()
            assert torch.equal(Xa, Xb) and ra == rb, i
    insts = [instances.gaussian_instance(int(n), 4 * int(n), max(1, int(n) // 20), dtype="f32", seed=940 + i)
             for i, n in enumerate((40, 97, 160, 33))]
    probs = [(torch.from_numpy(i.K_store).to(DEV), torch.from_numpy(i.y_store).to(DEV), i.rho) for i in insts]
    for kw in (dict(tol=1e-10, max_iter=3000, refresh_every=20), dict(tol=1e-10, max_iter=77, chunk=8)):
        say(f"[graph] uneven batch {kw}")
        Xa, ra = H.solve_batched_var(probs, **kw)
        Xb, rb = H.solve_batched_var(probs, graph=1, **kw)
        assert all(torch.equal(a, b) for a, b in zip(Xa, Xb)) and ra == rb


def test_batched_tuning_options(H):
    """Every shape the batched tuner may pick meets the FP32 bar against the
    oracle: shared-K split-K chunks, row- and column-kernel widths (a width
    without a compiled shape for p is refused), uneven-batch rows per item."""
    batch = instances.shared_batch(300, 2100, 5, 15, dtype="bf16", seed=84, rhs_seed_base=840)
    Kt = _kt(batch)
    Y = torch.from_numpy(batch.Y_store).to(DEV)
    base = dict(tol=1e-12, max_iter=4000, refresh_every=50)
    for kw in (dict(batch_splitk=256), dict(batch_splitk=2048), dict(batch_rows_t=512),
               dict(batch_rows_t=1024), dict(batch_cols_t=512), dict(batch_cols_t=1024)):
        say(f"[tuning] shared {kw}")
        X, res = H.solve_batched_shared(Kt, Y, batch.rho, **base, **kw)
        _check_columns(batch, X, res, range(5))
    # GEMM variants on a batch of 150 right-hand sides, so that the launches
    # span two 128-column tiles until problems finish: loads two k-steps
    # ahead, 256 x 128 and 128 x 64 tiles take the same products in the same
    # order as the 128 x 128 tile, so the same bits (and 128 x 64 tiles, used
    # by all of them once at most 128 problems run, too); chunks of 1, 2 and 3
    # k-steps (split-K 32 and 96) cover the loop's odd and early exits; both
    # padded sizes (384 and 2176 rows) end in half a 256-row tile
    wide = instances.shared_batch(300, 2100, 150, 15, dtype="bf16", seed=86, rhs_seed_base=860)
    Kw = _kt(wide)
    Yw = torch.from_numpy(wide.Y_store).to(DEV)
    for sk in (512, 96, 32):   # explicit chunks: the automatic one differs with the tile
        say(f"[tuning] shared GEMM variants, split-K {sk}")
        X1, r1 = H.solve_batched_shared(Kw, Yw, wide.rho, batch_splitk=sk, **base)
        for kw in (dict(batch_gemm_depth=2), dict(batch_gemm_tile=256), dict(batch_gemm_tile=64)):
            X2, r2 = H.solve_batched_shared(Kw, Yw, wide.rho, batch_splitk=sk, **base, **kw)
            assert torch.equal(X1, X2) and r1 == r2, (sk, kw)
    _check_columns(wide, X2, r2, (0, 77, 149))
    # p = 2100 needs 16 slots at 256 threads: not a compiled shape
    with pytest.raises(gpl1.GPError) as e:
        H.solve_batched_shared(Kt, Y, batch.rho, batch_cols_t=256, **base)
    assert e.value.code == -1
    for bad in (dict(batch_splitk=100), dict(batch_rows_t=300), dict(var_item_rows=8), dict(batch_gemm_depth=3),
                dict(var_wave_rows=2),
                dict(batch_gemm_tile=100), dict(batch_gemm_tile=256, batch_gemm_depth=2),
                dict(batch_gemm_tile=64, batch_gemm_depth=2)):
        with pytest.raises(gpl1.GPError):
            H.solve_batched_shared(Kt, Y, batch.rho, **base, **bad)
    rng = np.random.default_rng(85)
    insts = [instances.gaussian_instance(int(n), 4 * int(n), max(1, int(n) // 20), dtype="bf16", seed=950 + i)
             for i, n in enumerate(rng.integers(40, 400, size=5))]
    for rows in (16, 32, 128, 256):
        say(f"[tuning] uneven rows per item {rows}")
        X, res = H.solve_batched_var(_var_problems(insts, "bf16"), tol=1e-13, max_iter=5000,
                                     refresh_every=50, var_item_rows=rows)
        _check_var(insts, X, res, range(5), 1e-6, 1e-4)
