"""Wide problems on the GPU: p beyond the columns that one workgroup of the
fused K pass holds at full speed (8192 for double K, 16384 for float and
bf16), where the pass runs as two launches over column panels (8192 / 16384
columns).

Parity against the FP64 oracle: trajectory level in FP64 (iterate, objective
and backtrack count after k updates, as for narrow problems), the FP32/bf16
solution bar on float and bf16 K with aligned, padded and odd rows, several
row slabs, the first-order methods on the same pass, and the entry points
that share it (allocation-free, captured graphs) bit for bit.
"""
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
from oracle import gpss
from oracle.fom import fista, ista, psd
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


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def _K(inst, pad=0):
    """K on the device; with `pad`, rows of p + pad elements (a strided view)."""
    Ks = inst.K_store.view(np.int16) if inst.dtype == "bf16" else inst.K_store
    if not pad:
        return _dev(Ks)
    n, p = Ks.shape
    Kp = np.zeros((n, p + pad), dtype=Ks.dtype)
    Kp[:, :p] = Ks
    return _dev(Kp)[:, :p]


def _rel_gap(inst, x, ref):
    """(f(x) - f*) relative to f*, or to 1e-3 ||y||^2 where the ball's image
    nearly contains y (n << p, f* close to 0)."""
    x = np.asarray(x, dtype=np.float64)
    fx = float(np.sum((inst.K64 @ x - inst.y64) ** 2))
    scale = max(ref["f"], 1e-3 * float(inst.y64 @ inst.y64))
    return (fx - ref["f"]) / scale


@pytest.mark.parametrize("k", [1, 3, 8, 21])
def test_fp64_wide_trajectory_matches_oracle(H, k):
    """Three panels of 8192 columns, the last ragged (p = 20001)."""
    say(f"[wide] FP64 48x20001 trajectory after {k} iterations")
    inst = instances.gaussian_instance(48, 20001, 6, dtype="f64", seed=600)
    ref = gpss(inst.K64, inst.y64, inst.rho, tol=0.0, max_iter=k)
    x, res = H.solve(_K(inst), _dev(inst.y_store), inst.rho, tol=0.0, max_iter=k)
    assert res["iters"] == ref["iters"] == k
    assert res["backtracks"] == ref["backtracks"]
    err = np.linalg.norm(x.cpu().numpy() - ref["x"]) / np.linalg.norm(ref["x"])
    say(f"   x rel err {err:.2e}")
    assert err <= 1e-10
    assert abs(res["f"] - ref["f"]) <= 1e-10 * ref["f"]


@pytest.mark.parametrize("p,pad", [(40000, 0), (40000, 3), (49153, 0), (32769, 1)])
def test_fp32_wide_matches_oracle(H, p, pad):
    """Float K: 3-4 panels of 16384 columns, aligned rows, padded rows whose
    starts are only 4-byte aligned, odd p (element-wise tails)."""
    say(f"[wide] FP32 64x{p} pad={pad}")
    inst = instances.gaussian_instance(64, p, 4, dtype="f32", seed=610 + p + pad)
    ref = gpss(inst.K64, inst.y64, inst.rho, tol=1e-13, max_iter=20000)
    x, res = H.solve(_K(inst, pad), _dev(inst.y_store), inst.rho, tol=1e-13, max_iter=20000)
    gap = _rel_gap(inst, x.cpu().numpy(), ref)
    say(f"   gpu iters={res['iters']} status={res['status_name']} oracle iters={ref['iters']} gap={gap:.2e}")
    assert gap <= 1e-6, (gap, res)


@pytest.mark.parametrize("p,pad", [(70000, 0), (70001, 0), (70000, 3)])
def test_bf16_wide_matches_oracle(H, p, pad):
    """bf16 K: five panels of 16384 columns; the oracle runs on the rounded K."""
    say(f"[wide] bf16 40x{p} pad={pad}")
    inst = instances.gaussian_instance(40, p, 4, dtype="bf16", seed=620 + p + pad)
    ref = gpss(inst.K64, inst.y64, inst.rho, tol=1e-13, max_iter=20000)
    x, res = H.solve(_K(inst, pad), _dev(inst.y_store), inst.rho, tol=1e-13, max_iter=20000)
    gap = _rel_gap(inst, x.cpu().numpy(), ref)
    say(f"   gpu iters={res['iters']} status={res['status_name']} gap={gap:.2e}")
    assert gap <= 1e-6, (gap, res)


def test_fp32_wide_many_slabs(H):
    """1024 rows over 128 slabs and three panels: every slab's partial w and
    dots, the panels' t summed in one order, at the FP32 solution bar."""
    say("[wide] FP32 1024x33000")
    inst = instances.gaussian_instance(1024, 33000, 40, dtype="f32", seed=630)
    ref = gpss(inst.K64, inst.y64, inst.rho, tol=0.0, max_iter=100000)
    x, res = H.solve(_K(inst), _dev(inst.y_store), inst.rho, tol=1e-12, refresh_every=50, max_iter=5000)
    xn = x.cpu().numpy()
    gap = _rel_gap(inst, xn, ref)
    err = np.linalg.norm(xn - ref["x"]) / np.linalg.norm(ref["x"])
    say(f"   gpu iters={res['iters']} oracle iters={ref['iters']} gap={gap:.2e} err={err:.2e}")
    assert gap <= 1e-6 and err <= 1e-4


def test_wide_entry_points_agree(H):
    """The allocation-free solve, captured-graph chunks and a second run give
    the same bits as the plain solve; the pass is deterministic."""
    say("[wide] FP64 48x20001: solve, noalloc, graph, repeat")
    inst = instances.gaussian_instance(48, 20001, 6, dtype="f64", seed=640)
    K, y = _K(inst), _dev(inst.y_store)
    a, ra = H.solve(K, y, inst.rho, tol=0.0, max_iter=40)
    b, rb = H.solve(K, y, inst.rho, tol=0.0, max_iter=40)
    c, rc = H.solve_noalloc(K, y, inst.rho, tol=0.0, max_iter=40)
    d, rd = H.solve(K, y, inst.rho, tol=0.0, max_iter=40, graph=1, chunk=16)
    for other, r in ((b, rb), (c, rc), (d, rd)):
        assert torch.equal(a, other)
        assert r["iters"] == ra["iters"] and r["f"] == ra["f"]


def test_wide_first_order_methods_match_oracle(H):
    """ISTA and FISTA on double K with p = 20001 run their K and K^T passes
    through the panels: the FP64 iterates equal the oracle's."""
    say("[wide] FP64 48x20001: ISTA and FISTA, 10 steps")
    inst = instances.gaussian_instance(48, 20001, 6, dtype="f64", seed=650)
    L = float(np.linalg.norm(inst.K64, 2) ** 2)
    lam = 0.05 * float(np.abs(inst.K64.T @ inst.y64).max())
    K, y = _K(inst), _dev(inst.y_store)
    for name, fn in (("ista", ista), ("fista", fista)):
        ref = fn(inst.K64, inst.y64, lam, tau=1.0 / L, max_iter=10)
        x, r = H.fom(name, K, y, lam, 10, tau=1.0 / L)
        err = np.linalg.norm(x.cpu().numpy() - ref["x"]) / max(np.linalg.norm(ref["x"]), 1e-300)
        say(f"   {name} x rel err {err:.2e}")
        assert err <= 1e-10, (name, err)


def test_explicit_narrow_shape_is_refused(H):
    inst = instances.gaussian_instance(8, 20001, 2, dtype="f64", seed=660)
    with pytest.raises(gpl1.GPError) as e:
        H.solve(_K(inst), _dev(inst.y_store), inst.rho, fused_cfg=6, fused_grid=4)
    assert e.value.code == -5


@pytest.mark.parametrize("k", [2, 13])
def test_panels_on_a_narrow_problem_match_oracle(H, k):
    """The panel pass asked for where one panel holds every column (p = 1000,
    double K) keeps the oracle's FP64 trajectory."""
    say(f"[wide] FP64 200x1000 with GP_FUSED_PANELS, {k} iterations")
    inst = instances.gaussian_instance(200, 1000, 10, dtype="f64", seed=670)
    ref = gpss(inst.K64, inst.y64, inst.rho, tol=0.0, max_iter=k)
    x, res = H.solve(_K(inst), _dev(inst.y_store), inst.rho, tol=0.0, max_iter=k,
                     fused_cfg=gpl1.GP_FUSED_PANELS, fused_grid=16)
    assert res["iters"] == k and res["backtracks"] == ref["backtracks"]
    err = np.linalg.norm(x.cpu().numpy() - ref["x"]) / np.linalg.norm(ref["x"])
    assert err <= 1e-10
    assert abs(res["f"] - ref["f"]) <= 1e-10 * ref["f"]


@pytest.mark.parametrize("dt,p", [("f32", 30001), ("bf16", 40001), ("f64", 12001)])
def test_explicit_one_pass_beyond_the_panel_width(H, dt, p):
    """The widest one-pass shape (1024 threads, 8 chunks) stays available by
    explicit choice past the automatic limit, at the solution bar."""
    say(f"[wide] {dt} 48x{p}, one-pass shape 6")
    inst = instances.gaussian_instance(48, p, 4, dtype=dt, seed=680 + p)
    ref = gpss(inst.K64, inst.y64, inst.rho, tol=1e-13, max_iter=20000)
    x, res = H.solve(_K(inst), _dev(inst.y_store), inst.rho, tol=1e-13, max_iter=20000,
                     fused_cfg=6, fused_grid=16)
    gap = _rel_gap(inst, x.cpu().numpy(), ref)
    say(f"   gpu iters={res['iters']} status={res['status_name']} gap={gap:.2e}")
    assert gap <= 1e-6, (gap, res)


def test_first_order_methods_past_32768_columns(H):
    """ISTA, FISTA and PSD take any p (double K, p = 40001: five panels; PSD's
    projection in its streamed form past 32768 columns): the FP64 iterates
    equal the oracle's."""
    say("[wide] FP64 24x40001: ISTA, FISTA and PSD, 6 steps")
    inst = instances.gaussian_instance(24, 40001, 4, dtype="f64", seed=690)
    L = float(np.linalg.norm(inst.K64, 2) ** 2)
    lam = 0.05 * float(np.abs(inst.K64.T @ inst.y64).max())
    K, y = _K(inst), _dev(inst.y_store)
    for name, fn in (("ista", ista), ("fista", fista)):
        ref = fn(inst.K64, inst.y64, lam, tau=1.0 / L, max_iter=6)
        x, r = H.fom(name, K, y, lam, 6, tau=1.0 / L)
        err = np.linalg.norm(x.cpu().numpy() - ref["x"]) / max(np.linalg.norm(ref["x"]), 1e-300)
        say(f"   {name} x rel err {err:.2e}")
        assert r["iters"] == 6 and err <= 1e-10, (name, err)
    for rho in (inst.rho, 0.2 * inst.rho):
        ref = psd(inst.K64, inst.y64, rho, max_iter=6)
        x, r = H.fom("psd", K, y, rho, 6)
        xn = x.cpu().numpy()
        err = np.linalg.norm(xn - ref["x"]) / np.linalg.norm(ref["x"])
        say(f"   psd rho={rho:.3g} x rel err {err:.2e}")
        assert r["iters"] == ref["iters"] == 6 and err <= 1e-10
        assert r["f"] == pytest.approx(ref["f"], rel=1e-10)
        assert np.abs(xn).sum() <= rho * (1 + 1e-12)
    # from an x0 outside the ball (projected first), and a stationary start
    x0 = np.random.default_rng(3).standard_normal(40001)
    ref = psd(inst.K64, inst.y64, inst.rho, x0=x0, max_iter=4)
    x, r = H.fom("psd", K, y, inst.rho, 4, x0=_dev(x0))
    err = np.linalg.norm(x.cpu().numpy() - ref["x"]) / np.linalg.norm(ref["x"])
    assert err <= 1e-10
    x, r = H.fom("psd", K, torch.zeros_like(y), inst.rho, 5)
    assert r["status_name"] == "stationary" and r["iters"] == 0 and not x.any().item()


def test_batched_forms_route_wide_problems_through_the_panels(H):
    """A shared-K batch past the matrix-core path's 16384 columns, and an
    uneven batch holding a wide problem, run each problem on the single solver
    and so on the panel pass: every solution at the FP32 bar."""
    say("[wide] shared-K batch 32x20001 f32, B = 3; uneven batch with a 32x40000 problem")
    inst = instances.gaussian_instance(32, 20001, 3, dtype="f32", seed=700)
    rng = np.random.default_rng(701)
    ys = [inst.y64.astype(np.float32)]
    for _ in range(2):
        xt = np.zeros(20001)
        xt[rng.choice(20001, 3, replace=False)] = rng.choice([-1.0, 1.0], 3)
        ys.append((inst.K64 @ xt + 1e-2 * rng.standard_normal(32)).astype(np.float32))
    rhos = [inst.rho, 2.0, 3.0]
    K = _K(inst)
    X, rs = H.solve_batched_shared(K, _dev(np.stack(ys)), rhos, tol=1e-13, max_iter=20000)
    for b in range(3):
        y64 = ys[b].astype(np.float64)
        ref = gpss(inst.K64, y64, rhos[b], tol=1e-13, max_iter=20000)
        x = X[b].cpu().numpy().astype(np.float64)
        fx = float(np.sum((inst.K64 @ x - y64) ** 2))
        scale = max(ref["f"], 1e-3 * float(y64 @ y64))
        assert (fx - ref["f"]) / scale <= 1e-6, (b, fx, ref["f"], rs[b])
    wide = instances.gaussian_instance(32, 40000, 3, dtype="f32", seed=702)
    small = instances.gaussian_instance(16, 500, 3, dtype="f32", seed=703)
    probs = [(_K(i), _dev(i.y_store), i.rho) for i in (wide, small)]
    xs, rv = H.solve_batched_var(probs, tol=1e-13, max_iter=20000)
    for i, x, r in zip((wide, small), xs, rv):
        ref = gpss(i.K64, i.y64, i.rho, tol=1e-13, max_iter=20000)
        assert _rel_gap(i, x.cpu().numpy(), ref) <= 1e-6, r


@pytest.mark.parametrize("dt", ["f32", "bf16"])
def test_panels_and_one_pass_agree_at_the_same_width(H, dt):
    """At p = 16384 (one panel) the panel pass asked for and the automatic
    one-pass kernel both reach the oracle's solution at the FP32 bar."""
    say(f"[wide] {dt} 96x16384: one pass against GP_FUSED_PANELS")
    inst = instances.gaussian_instance(96, 16384, 5, dtype=dt, seed=710)
    ref = gpss(inst.K64, inst.y64, inst.rho, tol=1e-13, max_iter=20000)
    K, y = _K(inst), _dev(inst.y_store)
    x1, r1 = H.solve(K, y, inst.rho, tol=1e-13, max_iter=20000)
    x2, r2 = H.solve(K, y, inst.rho, tol=1e-13, max_iter=20000, fused_cfg=gpl1.GP_FUSED_PANELS, fused_grid=32)
    for x, r in ((x1, r1), (x2, r2)):
        assert _rel_gap(inst, x.cpu().numpy(), ref) <= 1e-6, r
