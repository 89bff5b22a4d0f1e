"""The per-update trace ring of gp_l1_solve (gp_opts.trace) against the FP64
oracle: for every accepted update, the objective after it, the steplength
alpha its projection used and the Algorithm 2 branch and tau that produced
that alpha, the line-search lambda and backtracks (Algorithm 1), and the
projection's threshold mu and active set, recomputed from the oracle's
iterate before the update.  Also: the ring keeps the last trace_cap records,
and tracing leaves the iterates unchanged."""
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
from oracle import GPSSParams, gpss, project_l1_mu
from paper_0902_4424_amd import gpl1, instances

pytestmark = pytest.mark.gpu

DEV = "cuda:0"
RULE = {"max": 0, "bb1": 1, "bb2min": 2}
COL = {c: i for i, c in enumerate(gpl1.TRACE_COLUMNS)}


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


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


@pytest.mark.parametrize("M", [1, 5])
def test_trace_matches_oracle(H, M):
    k = 20
    say(f"[trace] FP64 ill-conditioned 32x32, {k} updates, M = {M}")
    # backtracks, projections inside and outside the ball, active sets of
    # 18-32 of the 32 entries within these 20 updates
    inst = instances.illcond_instance(32, 5, dtype="f64", seed=4, cond=1e3)
    prm = GPSSParams(M=M)
    ref = gpss(inst.K64, inst.y64, inst.rho, tol=0.0, max_iter=k, params=prm, trace=True)
    rec = ref["trace"]
    K, y = _dev(inst.K_store), _dev(inst.y_store)
    x, res = H.solve(K, y, inst.rho, tol=0.0, max_iter=k, M=M, trace=64)
    T = res["trace"]
    assert res["iters"] == k and T.shape == (k, gpl1.TRACE_FIELDS)
    xs, _ = H.solve(K, y, inst.rho, tol=0.0, max_iter=k, M=M)
    assert torch.equal(x, xs)                  # tracing changes nothing
    assert sum(r["nb"] for r in rec) > 0       # the line search backtracks here
    for i in range(k):
        row, r = T[i], rec[i]
        assert row[COL["k"]] == i + 1
        assert row[COL["f"]] == pytest.approx(r["f_new"], rel=1e-10)
        assert row[COL["alpha"]] == pytest.approx(r["alpha"], rel=1e-10)
        assert row[COL["lam"]] == r["lam"] and row[COL["backtracks"]] == r["nb"]
        if i == 0:
            assert row[COL["rule"]] == -1
        else:
            assert row[COL["rule"]] == RULE[rec[i - 1]["rule"]]
            assert row[COL["tau"]] == pytest.approx(rec[i - 1]["tau"], rel=1e-12)
        assert row[COL["passes"]] >= 0
    # mu and the active set of each projection, from the oracle's iterate
    # before the update (x_i and its gradient) and the recorded alpha
    for i in (0, 1, 5, 11, 19):
        xi = gpss(inst.K64, inst.y64, inst.rho, tol=0.0, max_iter=i, params=prm)["x"]
        gi = 2.0 * inst.K64.T @ (inst.K64 @ xi - inst.y64)
        v = xi - rec[i]["alpha"] * gi
        _, mu = project_l1_mu(v, inst.rho)
        row = T[i]
        if np.abs(v).sum() <= inst.rho:
            assert row[COL["mu"]] == 0.0 and row[COL["nactive"]] == -1
        else:
            assert row[COL["mu"]] == pytest.approx(mu, rel=1e-9)
            assert row[COL["nactive"]] == int(np.sum(np.abs(v) > mu))


def test_trace_ring_keeps_the_last_records(H):
    say("[trace] ring of 5 over 17 updates, f32")
    inst = instances.gaussian_instance(512, 2048, 20, dtype="f32", seed=5)
    K, y = _dev(inst.K_store), _dev(inst.y_store)
    _, full = H.solve(K, y, inst.rho, tol=0.0, max_iter=17, trace=32)
    _, ring = H.solve(K, y, inst.rho, tol=0.0, max_iter=17, trace=5)
    assert full["trace"].shape == (17, gpl1.TRACE_FIELDS) and ring["trace"].shape == (5, gpl1.TRACE_FIELDS)
    assert np.array_equal(ring["trace"], full["trace"][-5:])
    assert list(ring["trace"][:, COL["k"]]) == [13, 14, 15, 16, 17]
    f = full["trace"][:, COL["f"]]
    assert f[-1] == pytest.approx(full["f"], rel=1e-5)
    with pytest.raises(ValueError):
        H.solve(K, y, inst.rho, trace=-1)


def test_trace_same_under_graph_replay_and_noalloc(H):
    """Captured-graph chunks and the allocation-free entry point write the
    same records, bit for bit, as plain launches."""
    say("[trace] FP64 256x1024: plain, graph chunks of 8, allocation-free")
    inst = instances.plain_small(seed=2, dtype="f64")
    K, y = _dev(inst.K_store), _dev(inst.y_store)
    _, a = H.solve(K, y, inst.rho, tol=0.0, max_iter=30, trace=32)
    _, b = H.solve(K, y, inst.rho, tol=0.0, max_iter=30, trace=32, graph=1, chunk=8)
    _, c = H.solve_noalloc(K, y, inst.rho, tol=0.0, max_iter=30, trace=32)
    assert a["trace"].shape == (30, gpl1.TRACE_FIELDS)
    assert np.array_equal(a["trace"], b["trace"]) and np.array_equal(a["trace"], c["trace"])
