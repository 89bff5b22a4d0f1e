"""gp_l1_solve_noalloc (the solver on a fixed device scratch, for callers that
cannot allocate) against gp_l1_solve on the same inputs, through the C ABI.

Both entry points run the same kernels with the same launch shapes, so the
solutions, the objective and the counters must agree exactly; they are also
held to the FP32 parity bar against the FP64 oracle (relative gap <= 1e-6,
||x - x_oracle|| / ||x_oracle|| <= 1e-4).  Two calls run in a row, the second on a
smaller problem, so the second reuses a scratch that still holds the first
call's larger state.
"""
import ctypes as C
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


def _pair(H, inst, tol, **kw):
    K = torch.from_numpy(inst.K_store).to(DEV)
    y = torch.from_numpy(inst.y_store).to(DEV)
    out_a = torch.full((inst.p,), float("nan"), dtype=y.dtype, device=DEV)
    out_b = torch.full((inst.p,), float("nan"), dtype=y.dtype, device=DEV)
    xa, ra = H.solve(K, y, inst.rho, tol=tol, out=out_a, **kw)
    xb, rb = H.solve_noalloc(K, y, inst.rho, tol=tol, out=out_b, **kw)
    torch.cuda.synchronize()
    return xa.cpu().numpy(), ra, xb.cpu().numpy(), rb


def _check(inst, tol, xa, ra, xb, rb, gap_bar, err_bar):
    assert ra["status"] >= 0 and rb["status"] == ra["status"]
    for k in ("iters", "backtracks", "f", "lambda_est", "l1norm", "proj_passes"):
        assert rb[k] == ra[k], (k, ra[k], rb[k])
    assert np.array_equal(xa, xb)
    ref = gpss(inst.K64, inst.y64, inst.rho, tol=tol)
    x = xb.astype(np.float64)
    fx = float(np.sum((inst.K64 @ x - inst.y64) ** 2))
    gap = (fx - ref["f"]) / ref["f"]
    err = np.linalg.norm(x - ref["x"]) / np.linalg.norm(ref["x"])
    say(f"    iters={rb['iters']} oracle_iters={ref['iters']} gap={gap:.2e} x_err={err:.2e}")
    assert gap <= gap_bar and err <= err_bar


def test_noalloc_matches_solve_two_calls_second_smaller(H):
    # first call: 1024 x 4096 FP32 K (several row slabs and a multi-pass
    # threshold search); second call: 200 x 777 (ragged p) on the same scratch
    big = instances.gaussian_instance(1024, 4096, 40, amp="pm1", sigma=1e-2, dtype="f32",
                                      seed=31, name="noalloc_big")
    small = instances.gaussian_instance(200, 777, 9, amp="pm1", sigma=1e-2, dtype="f32",
                                        seed=32, name="noalloc_small")
    for inst in (big, small):
        say(f"[noalloc] n={inst.n} p={inst.p} f32 refresh_every=50")
        xa, ra, xb, rb = _pair(H, inst, 1e-10, refresh_every=50)
        _check(inst, 1e-10, xa, ra, xb, rb, 1e-6, 1e-4)


def test_noalloc_fp64_then_smaller_with_x0(H):
    big = instances.gaussian_instance(256, 1024, 20, amp="pm1", sigma=1e-3, dtype="f64",
                                      seed=33, name="noalloc_f64")
    small = instances.gaussian_instance(64, 130, 5, amp="pm1", sigma=1e-3, dtype="f64",
                                        seed=34, name="noalloc_f64_small")
    say(f"[noalloc] n={big.n} p={big.p} f64")
    xa, ra, xb, rb = _pair(H, big, 1e-12)
    _check(big, 1e-12, xa, ra, xb, rb, 1e-10, 1e-6)
    # a warm start outside the ball (projected on entry) on the smaller problem
    rng = np.random.default_rng(35)
    x0 = torch.from_numpy(rng.standard_normal(small.p)).to(DEV)
    K = torch.from_numpy(small.K_store).to(DEV)
    y = torch.from_numpy(small.y_store).to(DEV)
    say(f"[noalloc] n={small.n} p={small.p} f64 x0 outside the ball")
    xa, ra = H.solve(K, y, small.rho, x0=x0, tol=1e-12)
    xb, rb = H.solve_noalloc(K, y, small.rho, x0=x0, tol=1e-12)
    torch.cuda.synchronize()
    assert ra["projected_x0"] == 1 and rb["projected_x0"] == 1
    _check(small, 1e-12, xa.cpu().numpy(), ra, xb.cpu().numpy(), rb, 1e-10, 1e-6)


def test_noalloc_refuses_what_does_not_fit(H):
    # 8192 x 16384 float K needs 256 partial vectors of 64 KiB (16 MiB) plus
    # vectors: fits; 8192 x 32768 needs about 34 MB: refused before any launch
    lib = gpl1.load()
    res = gpl1.GPResult()
    o = gpl1.default_opts()
    dummy = torch.zeros(8, dtype=torch.float32, device=DEV)
    p = dummy.data_ptr()
    rc = lib.gp_l1_solve_noalloc(H.h, gpl1.GP_F32, p, 8192, 32768, 32768, p, 1.0, None, 0.0, p,
                                 C.byref(o), C.byref(res), None)
    assert rc == -5 and "scratch" in H.error()
    o.graph = 1
    rc = lib.gp_l1_solve_noalloc(H.h, gpl1.GP_F32, p, 16, 64, 64, p, 1.0, None, 0.0, p,
                                 C.byref(o), C.byref(res), None)
    assert rc == -1
    assert torch.all(dummy == 0)
