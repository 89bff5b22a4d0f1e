"""CPU pins of the FP64 oracle against facts the paper and the mathematics fix.

Every pin here is independent of the oracle's own code path: hand-derived
trajectories, brute-force enumeration, closed forms, a library lasso-path
solver, finite differences, and optimality certificates.
"""
import os

import numpy as np
import pytest

from oracle import (GPSSParams, gpss, project_l1, project_l1_mu, ss_update,
                    soft_threshold)
from oracle.gpss import SSState
from oracle import exact, lista
from paper_0902_4424_amd import instances

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    vals = {}
    with open(os.path.join(GOLDEN, name)) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            k, v = line.split("=")
            vals[k.strip()] = np.array([float(t) for t in v.split()])
    return vals


# --------------------------------------------------------------------------
# projection onto the l1 ball
# --------------------------------------------------------------------------

def test_projection_hand_cases():
    np.testing.assert_allclose(project_l1([3.0, 1.0], 1.0), [1.0, 0.0])
    np.testing.assert_allclose(project_l1([1.0, 1.0], 1.0), [0.5, 0.5])
    np.testing.assert_allclose(project_l1([-1.0, 1.0], 1.0), [-0.5, 0.5])
    np.testing.assert_allclose(project_l1([0.2, -0.3], 1.0), [0.2, -0.3])
    h, mu = project_l1_mu([2.0, -2.0, 1.0], 2.0)   # mu = (4 - 2)/2 = 1
    assert mu == pytest.approx(1.0)
    np.testing.assert_allclose(h, [1.0, -1.0, 0.0])
    np.testing.assert_allclose(project_l1([5.0, -7.0], 0.0), [0.0, 0.0])
    # radius far below the size of v: the answer is rho at the largest entry
    np.testing.assert_allclose(project_l1([3e9, -1e9, 2.0], 1e-9), [1e-9, 0, 0],
                               rtol=1e-15, atol=0)
    np.testing.assert_allclose(project_l1([1e9, -1e9 + 1.0, 0.0], 3.0),
                               [2.0, -1.0, 0.0], rtol=1e-15, atol=0)


@pytest.mark.parametrize("seed", range(40))
def test_projection_vs_bruteforce(seed):
    rng = np.random.default_rng(seed)
    p = int(rng.integers(1, 7))
    v = rng.standard_normal(p) * rng.choice([0.1, 1.0, 10.0])
    if seed % 5 == 0 and p > 1:       # ties in |v|
        v[1] = -v[0]
    if seed % 7 == 0:                 # exact zeros
        v[0] = 0.0
    rho = float(rng.uniform(0.05, 1.2) * np.abs(v).sum())
    want = exact.project_l1_bruteforce(v, rho)
    got = project_l1(v, rho)
    np.testing.assert_allclose(got, want, atol=1e-12, rtol=1e-12)


@pytest.mark.parametrize("seed", range(10))
def test_projection_optimality_certificate(seed):
    """h = P(v) iff ||h||_1 <= rho and (v-h)^T (h - u) >= 0 for all u in the
    ball; the worst u is a vertex +-rho e_i, giving rho ||v-h||_inf <= (v-h)^T h."""
    rng = np.random.default_rng(100 + seed)
    p = int(rng.integers(10, 5000))
    v = rng.standard_normal(p) * np.exp(rng.uniform(-5, 5, p))
    rho = float(rng.uniform(0.01, 0.9) * np.abs(v).sum())
    h = project_l1(v, rho)
    w = v - h
    assert np.abs(h).sum() <= rho * (1 + 1e-12)
    assert np.abs(h).sum() >= rho * (1 - 1e-12)   # v outside -> on the sphere
    assert rho * np.abs(w).max() <= w @ h + 1e-9 * rho * np.abs(w).max()


# --------------------------------------------------------------------------
# Algorithm 2 in isolation
# --------------------------------------------------------------------------

def test_ss_update_branches():
    p = GPSSParams()
    st = SSState(tau=0.5)
    # s^T z <= 0 -> alpha_max, tau unchanged, nothing recorded
    a, rule = ss_update(1, 1.0, 0.0, 1.0, st, p)
    assert (a, rule, st.tau, st.a2_hist) == (1e10, "max", 0.5, [])
    a, rule = ss_update(2, 1.0, -3.0, 1.0, st, p)
    assert (a, rule, st.tau) == (1e10, "max", 0.5)
    # a1 = ss/sz = 4, a2 = sz/zz = 0.5, ratio 0.125 <= 0.5 -> min window
    a, rule = ss_update(3, 4.0, 1.0, 2.0, st, p)
    assert rule == "bb2min" and a == 0.5 and st.tau == pytest.approx(0.45)
    # a1 = 1, a2 = 0.8, ratio 0.8 > 0.45 -> BB1, tau * 1.1
    a, rule = ss_update(4, 1.0, 1.0, 1.25, st, p)
    assert rule == "bb1" and a == 1.0 and st.tau == pytest.approx(0.495)
    # a1 = 10, a2 = 0.9, ratio 0.09 <= 0.495 -> min over k = 3,4,5 -> 0.5
    a, rule = ss_update(5, 10.0, 1.0, 1 / 0.9, st, p)
    assert rule == "bb2min" and a == pytest.approx(0.5)
    # window is iterations max(1, k-2)..k: at k=6 the value from k=3 drops out
    a, rule = ss_update(6, 10.0, 1.0, 1 / 0.95, st, p)
    assert rule == "bb2min" and a == pytest.approx(0.8)
    # clamps: ss/sz above alpha_max and sz/zz below alpha_min
    st2 = SSState(tau=0.5)
    a, rule = ss_update(1, 1e12, 1e-3, 1e12, st2, p)
    assert rule == "bb2min" and a == 1e-10


# --------------------------------------------------------------------------
# hand-derived trajectories (golden)
# --------------------------------------------------------------------------

def test_gpss_hand_examples():
    g = _golden("ss_hand_examples.txt")
    for tag, K, y, rho in (("A", np.diag([1.0, 0.5]), np.array([1.0, 1.0]), 100.0),
                           ("B", np.diag([1.0, 0.1]), np.array([1.0, 100.0]), 1000.0)):
        out = gpss(K, y, rho, tol=0.0, max_iter=2, trace=True)
        tr = out["trace"]
        assert tr[0]["alpha"] == pytest.approx(g[f"{tag}.alpha0"][0], rel=1e-14)
        assert tr[0]["f"] == pytest.approx(g[f"{tag}.f0"][0], rel=1e-14)
        assert tr[0]["f_new"] == pytest.approx(g[f"{tag}.f1"][0], rel=1e-12)
        assert tr[0]["lam"] == 1.0 and tr[1]["lam"] == 1.0
        assert tr[1]["alpha"] == pytest.approx(g[f"{tag}.alpha1"][0], rel=1e-12)
        assert tr[0]["tau"] == pytest.approx(g[f"{tag}.tau2"][0], rel=1e-14)
        assert tr[1]["alpha_next"] == pytest.approx(g[f"{tag}.alpha2"][0], rel=1e-12)
        assert tr[1]["tau"] == pytest.approx(g[f"{tag}.tau3"][0], rel=1e-14)
        np.testing.assert_allclose(out["x"], g[f"{tag}.x2"], rtol=1e-12)
    assert gpss(np.diag([1.0, 0.5]), np.array([1.0, 1.0]), 100.0,
                tol=0.0, max_iter=2, trace=True)["trace"][1]["f_new"] == \
        pytest.approx(g["A.f2"][0], rel=1e-12)
    out = gpss(np.diag([1.0, 0.5]), np.array([1.0, 1.0]), 100.0, tol=0.0, max_iter=3)
    np.testing.assert_allclose(out["x"], g["A.x3"], rtol=1e-12)
    out = gpss(np.diag([1.0, 0.1]), np.array([1.0, 100.0]), 1000.0, tol=0.0,
               max_iter=1, trace=True)
    np.testing.assert_allclose(out["x"], g["B.x1"], rtol=1e-14)


def test_gpss_backtracking_hand_example():
    """K = [2], y = [1], rho = 10, x0 = 0.  grad f(0) = 2*2*(0 - 1) = -4,
    P(0 + 4) = 4 -> alpha_0 = 1/4, h = 1, d = 1.  f(0) = 1 and f(1) = (2-1)^2 = 1,
    so with grad'd = -4 the Armijo test 1 <= 1 - 4e-4 fails at lambda = 1 and
    holds at lambda = theta = 1/2: x_1 = 1/2 = K^{-1} y, f = 0."""
    out = gpss(np.array([[2.0]]), np.array([1.0]), 10.0, tol=0.0, max_iter=1,
               trace=True)
    r = out["trace"][0]
    assert r["alpha"] == 0.25 and r["gd"] == -4.0
    assert r["lam"] == 0.5 and r["nb"] == 1
    assert out["x"][0] == 0.5 and out["f"] == 0.0


def test_gpss_nonmonotone_hand_example():
    """Algorithm 1, step 4 with M > 1 (tests/golden/nonmonotone_hand_example.txt):
    at k = 1 the BB1 step raises f from 28.39 to 29.09.  With M = 1 the trial
    is rejected and one reduction gives lambda = 1/2; with M = 2 or 3 the
    window still holds f0 = 30 and the increase is accepted at lambda = 1.
    At k = 2 the window of M = 2 has dropped f0, the one of M = 3 has not."""
    g = _golden("nonmonotone_hand_example.txt")
    K, y, rho = np.diag([1.0, 3.0, 5.0]), np.array([5.0, 2.0, 1.0]), 100.0
    runs = {M: gpss(K, y, rho, tol=0.0, max_iter=3, trace=True,
                    params=GPSSParams(M=M))["trace"] for M in (1, 2, 3)}
    for M, tr in runs.items():
        assert tr[0]["f"] == pytest.approx(g["C.f0"][0], rel=1e-15)
        assert tr[0]["alpha"] == pytest.approx(g["C.alpha0"][0], rel=1e-15)
        assert tr[0]["lam"] == 1.0 and tr[0]["fmax"] == g["C.f0"][0]
        assert tr[0]["f_new"] == pytest.approx(g["C.f1"][0], rel=1e-14)
        assert tr[1]["alpha"] == pytest.approx(g["C.alpha1"][0], rel=1e-13)
        assert tr[1]["gd"] == pytest.approx(g["C.gd1"][0], rel=1e-13)
        for r in tr:
            assert r["l1"] < rho
    # M = 1: monotone Armijo, one reduction
    r = runs[1][1]
    assert r["fmax"] == pytest.approx(g["C.f1"][0], rel=1e-14)
    assert (r["lam"], r["nb"]) == (0.5, 1)
    assert r["f_new"] == pytest.approx(g["C.f2_M1"][0], rel=1e-13)
    np.testing.assert_allclose(gpss(K, y, rho, tol=0.0, max_iter=2)["x"], g["C.x2_M1"],
                               rtol=1e-13)
    # M = 2, 3: the increase is accepted at lambda = 1
    for M in (2, 3):
        r = runs[M][1]
        assert r["fmax"] == pytest.approx(g["C.fmax1_M2"][0], rel=1e-15)
        assert (r["lam"], r["nb"]) == (1.0, 0)
        assert r["f_new"] == pytest.approx(g["C.f2_M2"][0], rel=1e-13)
        assert r["f_new"] > r["f"]
        x2 = gpss(K, y, rho, tol=0.0, max_iter=2, params=GPSSParams(M=M))["x"]
        np.testing.assert_allclose(x2, g["C.x2_M2"], rtol=1e-13)
    assert runs[2][2]["fmax"] == pytest.approx(g["C.fmax2_M2"][0], rel=1e-13)
    assert runs[3][2]["fmax"] == pytest.approx(g["C.fmax2_M3"][0], rel=1e-15)


# --------------------------------------------------------------------------
# full solutions against exact references
# --------------------------------------------------------------------------

@pytest.mark.parametrize("seed", range(12))
def test_gpss_vs_bruteforce(seed):
    rng = np.random.default_rng(200 + seed)
    n, p = 8, int(rng.integers(2, 6))
    K = rng.standard_normal((n, p))
    x_ls = np.linalg.lstsq(K, y := rng.standard_normal(n), rcond=None)[0]
    rho = float(rng.uniform(0.1, 1.3) * np.abs(x_ls).sum())
    want = exact.constrained_ls_bruteforce(K, y, rho)
    out = gpss(K, y, rho, tol=1e-15, max_iter=20000)
    np.testing.assert_allclose(out["x"], want, atol=1e-7)


def _lasso_path_solution(K, y, rho):
    """x~(rho) from the exact piecewise-linear lasso path (sklearn LARS-lasso):
    the path is linear between knots, so interpolate where ||x||_1 = rho."""
    from sklearn.linear_model import lars_path
    _, _, coefs = lars_path(K, y, method="lasso", alpha_min=0.0, eps=1e-15,
                            max_iter=2000)
    l1 = np.abs(coefs).sum(axis=0)
    j = int(np.searchsorted(l1, rho))
    assert 0 < j < coefs.shape[1], "rho outside the computed path"
    t = (rho - l1[j - 1]) / (l1[j] - l1[j - 1])
    return (1 - t) * coefs[:, j - 1] + t * coefs[:, j]


@pytest.mark.parametrize("seed", [11, 12, 13])
def test_gpss_vs_lars_path(seed):
    inst = instances.gaussian_instance(64, 256, 6, amp="pm1", sigma=1e-2,
                                       rho_scale=0.8, dtype="f64", seed=seed)
    K, y = inst.K64, inst.y64
    want = _lasso_path_solution(K, y, inst.rho)
    out = gpss(K, y, inst.rho, tol=0.0, max_iter=20000)
    assert out["status"] == "stationary"
    # FP64 stationarity floor of the iteration: ~1e-8 relative in x
    assert np.linalg.norm(out["x"] - want) <= 1e-7 * np.linalg.norm(want)
    fw = np.sum((K @ want - y) ** 2)
    assert abs(out["f"] - fw) <= 1e-12 * fw


def test_gpss_orthonormal_closed_form():
    """K^T K = I: f = ||x - K^T y||^2 + const, so x~ = P_rho(K^T y)."""
    rng = np.random.default_rng(7)
    Q, _ = np.linalg.qr(rng.standard_normal((80, 30)))
    y = rng.standard_normal(80)
    rho = 0.5 * np.abs(Q.T @ y).sum()
    out = gpss(Q, y, rho, tol=0.0, max_iter=50)
    np.testing.assert_allclose(out["x"], project_l1(Q.T @ y, rho), atol=1e-13)


def test_gpss_kkt_and_lambda_rho():
    """Section 1: lambda = ||K^T (y - K x~)||_inf; on the support the
    correlation equals lambda sgn(x_i), off it |.| <= lambda; and x~ is a
    fixed point of the soft-thresholding step of ISTA (Section 2)."""
    inst = instances.plain_small(seed=1)
    K, y = inst.K64, inst.y64
    out = gpss(K, y, inst.rho, tol=0.0, max_iter=100000)
    assert out["status"] == "stationary"
    x = out["x"]
    corr = K.T @ (y - K @ x)
    lam = exact.lambda_of_rho(K, y, x)
    assert out["lambda_est"] == pytest.approx(lam, rel=1e-12)
    assert lam > 0
    supp = np.abs(x) > 1e-9 * np.abs(x).max()
    # FP64 stationarity floor: x is exact to ~1e-8 relative, which moves the
    # correlations by ~||K^T K|| * 1e-8 ~ 1e-5 lambda
    assert np.abs(corr[supp] - lam * np.sign(x[supp])).max() <= 1e-4 * lam
    assert np.abs(corr[~supp]).max() <= lam * (1 + 1e-9)
    assert np.abs(x).sum() == pytest.approx(inst.rho, rel=1e-12)
    t = 0.3
    fixed = soft_threshold(x + t * corr, t * lam)
    assert np.abs(fixed - x).max() <= 1e-6 * np.abs(x).max()
    # exact solution from the piecewise-linear lasso path at the same rho
    want = _lasso_path_solution(K, y, inst.rho)
    fw = np.sum((K @ want - y) ** 2)
    assert np.linalg.norm(x - want) <= 1e-7 * np.linalg.norm(want)
    assert (out["f"] - fw) / fw <= 1e-10


def test_gpss_monotone_feasible_and_bb_order():
    inst = instances.plain_small(seed=1)
    out = gpss(inst.K64, inst.y64, inst.rho, tol=1e-12, trace=True)
    assert out["status"] == "tol"
    fs = [r["f"] for r in out["trace"]] + [out["f"]]
    tr = out["trace"]
    for r in tr:
        # Armijo with M = 1 (monotone): f_new <= f + beta lam g'd < f
        assert r["f_new"] <= r["f"] + 1e-4 * r["lam"] * r["gd"] + 1e-12 * r["f"]
        assert r["gd"] < 0
        assert r["l1"] <= inst.rho * (1 + 1e-12)
        # s'z = 2 lam^2 ||Kd||^2 >= 0 for this quadratic f, so BB2 <= BB1
        assert r["sz"] > 0 and r["sz"] ** 2 <= r["ss"] * r["zz"] * (1 + 1e-12)
    assert all(b < a for a, b in zip(fs, fs[1:]))
    rules = {r["rule"] for r in tr}
    assert {"bb1", "bb2min"} <= rules


def test_gpss_special_cases():
    rng = np.random.default_rng(3)
    K = rng.standard_normal((20, 40))
    y = rng.standard_normal(20)
    out = gpss(K, y, 0.0)
    assert out["status"] == "stationary" and out["iters"] == 0
    assert not out["x"].any()
    out = gpss(K, np.zeros(20), 3.0)
    assert out["status"] == "stationary" and out["iters"] == 0
    # square full-rank K and a radius above ||K^{-1} y||_1: unconstrained LS
    Ks = rng.standard_normal((12, 12)) + 4 * np.eye(12)
    ys = rng.standard_normal(12)
    xs = np.linalg.solve(Ks, ys)
    out = gpss(Ks, ys, 10 * np.abs(xs).sum(), tol=0.0, max_iter=5000)
    np.testing.assert_allclose(out["x"], xs, atol=1e-10)
    # infeasible start is projected first
    x0 = rng.standard_normal(40) * 10
    out = gpss(K, y, 1.0, x0=x0, max_iter=1, tol=0.0)
    assert out["projected_x0"] and out["l1norm"] <= 1.0 + 1e-12
    out = gpss(K, y, 1.0, max_iter=1, tol=0.0)
    assert out["status"] == "max_iter" and out["iters"] == 1


def test_lambda_max_gives_zero():
    """Section 1: x_bar(lambda) = 0 for lambda >= lambda_max = ||K^T y||_inf;
    in the constrained form rho -> 0 drives x -> 0 and lambda -> lambda_max."""
    inst = instances.gaussian_instance(30, 60, 3, dtype="f64", seed=5)
    K, y = inst.K64, inst.y64
    out = gpss(K, y, 1e-9, tol=0.0, max_iter=200)
    assert out["l1norm"] <= 1e-9 * (1 + 1e-9)
    assert out["lambda_est"] == pytest.approx(np.abs(K.T @ y).max(), rel=1e-6)


# --------------------------------------------------------------------------
# unrolled network
# --------------------------------------------------------------------------

def test_lista_ista_init_matches_ista_iterations():
    """With W_e = K^T/L, S = I - K^T K/L, theta = lam/L the network computes T
    ISTA steps x <- S_{lam/L}[x + K^T (y - K x)/L] from x = 0 (Section 2)."""
    rng = np.random.default_rng(4)
    K = rng.standard_normal((12, 30)) / np.sqrt(12)
    Y = rng.standard_normal((12, 5))
    lam = 0.05
    We, S, th = lista.ista_init(K, lam)
    L = np.linalg.norm(K, 2) ** 2
    x_net, _, _ = lista.forward(We, S, [th] * 6, Y)
    X = np.zeros((30, 5))
    for _ in range(6):
        X = soft_threshold(X + K.T @ (Y - K @ X) / L, lam / L)
    np.testing.assert_allclose(x_net, X, atol=1e-13)


def test_lista_gradients_finite_differences():
    rng = np.random.default_rng(5)
    n, p, B, T = 6, 10, 4, 3
    We = rng.standard_normal((p, n)) * 0.3
    S = rng.standard_normal((p, p)) * 0.2
    th = np.array([0.05, 0.08, 0.03])
    Y = rng.standard_normal((n, B))
    Xs = rng.standard_normal((p, B)) * 0.5
    L, dWe, dS, dth = lista.backward(We, S, th, Y, Xs)
    eps = 1e-6

    def fd(f, A, idx):
        A0 = A[idx]
        A[idx] = A0 + eps
        lp = f()
        A[idx] = A0 - eps
        lm = f()
        A[idx] = A0
        return (lp - lm) / (2 * eps)

    f = lambda: lista.loss(We, S, th, Y, Xs)  # noqa: E731
    for idx in [(0, 0), (3, 2), (9, 5)]:
        assert dWe[idx] == pytest.approx(fd(f, We, idx), rel=1e-5, abs=1e-9)
    for idx in [(0, 0), (4, 7), (9, 9)]:
        assert dS[idx] == pytest.approx(fd(f, S, idx), rel=1e-5, abs=1e-9)
    for t in range(T):
        assert dth[t] == pytest.approx(fd(f, th, t), rel=1e-5, abs=1e-9)


# --------------------------------------------------------------------------
# instance construction
# --------------------------------------------------------------------------

def test_bf16_rounding_matches_torch():
    import torch
    rng = np.random.default_rng(0)
    a = (rng.standard_normal(100000) * np.exp(rng.uniform(-20, 20, 100000))).astype(np.float32)
    a[:4] = [0.0, -0.0, 1.00390625, 1.01171875]   # exact ties between bf16 values
    ours = instances.f32_to_bf16_bits(a)
    ref = torch.from_numpy(a).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    np.testing.assert_array_equal(ours, ref)
    back = instances.bf16_bits_to_f32(ours)
    np.testing.assert_array_equal(back, torch.from_numpy(a).to(torch.bfloat16).float().numpy())


def test_instances_deterministic_and_shaped():
    a = instances.plain_small(seed=1)
    b = instances.plain_small(seed=1)
    assert a.K_store.dtype == np.float64 and a.K_store.shape == (256, 1024)
    np.testing.assert_array_equal(a.K_store, b.K_store)
    np.testing.assert_array_equal(a.y_store, b.y_store)
    assert a.rho == 20.0 and np.count_nonzero(a.x_true) == 20
    c = instances.gaussian_instance(50, 200, 5, dtype="bf16", seed=2)
    assert c.K_store.dtype == np.uint16 and c.y_store.dtype == np.float32
