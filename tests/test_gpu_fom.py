"""GPU parity of the comparison methods of Section 2 (ISTA, item 1; FISTA,
item 2 and equation (3); projected steepest descent, item 5) against the FP64
oracle, through the C ABI (gp_fom_solve).

Tolerances: FP64 K -- iterates after k steps within 1e-10 of the oracle's
(relative), the hand-derived steps within 1e-14; FP32 K -- 1e-5 relative
after 30 steps (the products are FP32, the oracle's FP64 on the same stored
K); the reported objective equals the host's FP64 value of the returned x to
1e-12.  Fixed point: FISTA at lambda = lambda_est of a GPSS solution reaches
that solution (Section 1 pairs rho and lambda).
"""
import ctypes as C
import os
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import gpss
from oracle.fom import fista, ista, penalised_objective, psd
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


def _golden(name):
    vals = {}
    for line in open(os.path.join(os.path.dirname(__file__), "golden", name)):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        k, v = line.split("=")
        vals[k.strip()] = [float(t) for t in v.split()]
    return vals


def _t(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    return (t.to(dtype) if dtype is not None else t).to(DEV)


def test_hand_examples(H):
    """Example F (ISTA and FISTA on K = [1/2], y = [1], lambda = 1/10) and
    example P (PSD on K = diag(1, 1/2), y = (1, 1)) of
    tests/golden/fom_hand_examples.txt."""
    g = _golden("fom_hand_examples.txt")
    K, y = _t(np.array([[0.5]])), _t(np.array([1.0]))
    for k in (1, 2, 3):
        say(f"[fom] hand example F, {k} steps")
        x, r = H.fom("ista", K, y, 0.1, k)
        assert r["iters"] == k and r["status_name"] == "max_iter"
        assert x.item() == pytest.approx(g["F.ista_x"][k - 1], rel=1e-14)
        x, r = H.fom("fista", K, y, 0.1, k)
        assert x.item() == pytest.approx(g["F.fista_x"][k - 1], rel=1e-14)
        # F(x) = ||Kx - y||^2 + 2 lambda |x|
        assert r["f"] == pytest.approx((0.5 * x.item() - 1.0) ** 2 + 0.2 * abs(x.item()), rel=1e-14)
    Kp, yp = _t(np.diag([1.0, 0.5])), _t(np.array([1.0, 1.0]))
    say("[fom] hand example P")
    x1, r1 = H.fom("psd", Kp, yp, 100.0, 1)
    np.testing.assert_allclose(x1.cpu().numpy(), g["P.x1"], rtol=1e-14)
    x2, _ = H.fom("psd", Kp, yp, 100.0, 2)
    np.testing.assert_allclose(x2.cpu().numpy(), g["P.x2"], rtol=1e-14)
    xr, rr = H.fom("psd", Kp, yp, 1.0, 1)
    np.testing.assert_allclose(xr.cpu().numpy(), g["P.x1_rho1"], rtol=1e-14)
    assert rr["l1norm"] == pytest.approx(1.0, rel=1e-14)


def _small():
    inst = instances.gaussian_instance(200, 700, 12, amp="pm1", sigma=1e-2, dtype="f64", seed=77)
    L = float(np.linalg.norm(inst.K64, 2) ** 2)
    lam = 0.05 * float(np.abs(inst.K64.T @ inst.y64).max())
    return inst, 1.0 / L, lam


@pytest.mark.parametrize("k", [1, 5, 20, 60])
def test_fp64_trajectories_match_oracle(H, k):
    inst, tau, lam = _small()
    K, y = _t(inst.K_store), _t(inst.y_store)
    say(f"[fom] FP64 200x700, {k} steps of ISTA, FISTA (tau = 1/||K||^2) and PSD")
    for name, fn, arg in (("ista", ista, lam), ("fista", fista, lam)):
        ref = fn(inst.K64, inst.y64, lam, tau=tau, max_iter=k)
        x, r = H.fom(name, K, y, arg, k, tau=tau)
        assert r["iters"] == k
        xn = x.cpu().numpy()
        err = np.linalg.norm(xn - ref["x"]) / max(np.linalg.norm(ref["x"]), 1e-300)
        assert err <= 1e-10, (name, err)
        assert r["f"] == pytest.approx(penalised_objective(inst.K64, inst.y64, xn, lam), rel=1e-12)
    ref = psd(inst.K64, inst.y64, inst.rho, max_iter=k)
    x, r = H.fom("psd", K, y, inst.rho, k)
    assert r["iters"] == ref["iters"] == k
    err = np.linalg.norm(x.cpu().numpy() - ref["x"]) / np.linalg.norm(ref["x"])
    assert err <= 1e-10, ("psd", err)
    assert r["f"] == pytest.approx(ref["f"], rel=1e-10)
    assert np.abs(x.cpu().numpy()).sum() <= inst.rho * (1 + 1e-12)


@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_reduced_precision_matches_oracle(H, dtype):
    """FP32 / bf16 K (vectors FP32 on return), 30 steps, against the oracle on
    the same stored K; a ragged p across several row slabs."""
    inst = instances.gaussian_instance(1000, 3001, 40, amp="pm1", sigma=1e-2, dtype=dtype, seed=78)
    K = _t(inst.K_store.view(np.int16) if dtype == "bf16" else inst.K_store)
    y = _t(inst.y_store)
    tau = 1.0 / float(np.linalg.norm(inst.K64, 2) ** 2)
    lam = 0.05 * float(np.abs(inst.K64.T @ inst.y64).max())
    for name in ("ista", "fista", "psd"):
        say(f"[fom] {dtype} 1000x3001, 30 steps of {name}")
        if name == "psd":
            ref = psd(inst.K64, inst.y64, inst.rho, max_iter=30)
            x, r = H.fom(name, K, y, inst.rho, 30)
        else:
            ref = (ista if name == "ista" else fista)(inst.K64, inst.y64, lam, tau=tau, max_iter=30)
            x, r = H.fom(name, K, y, lam, 30, tau=tau)
        xn = x.cpu().double().numpy()
        err = np.linalg.norm(xn - ref["x"]) / np.linalg.norm(ref["x"])
        say(f"   x err {err:.2e}")
        assert err <= 1e-5, (name, err)
        fh = float(np.sum((inst.K64 @ xn - inst.y64) ** 2))
        if name != "psd":
            fh += 2 * lam * float(np.abs(xn).sum())
        assert r["f"] == pytest.approx(fh, rel=1e-12)


def test_fista_fixed_point_is_the_gpss_solution(H):
    """Section 1: the solution of (2) at radius rho solves (1) at
    lambda = ||K^T (y - K x)||_inf.  GPSS at rho gives x~ and lambda_est;
    FISTA at that lambda (tau = 1/||K||^2) converges to x~."""
    inst = instances.gaussian_instance(64, 256, 6, amp="pm1", sigma=1e-2, dtype="f64", seed=79)
    K, y = _t(inst.K_store), _t(inst.y_store)
    rho = 0.7 * inst.rho
    xg, rg = H.solve(K, y, rho, tol=0.0)
    lam = rg["lambda_est"]
    tau = 1.0 / float(np.linalg.norm(inst.K64, 2) ** 2)
    say(f"[fom] fixed point: GPSS at rho {rho:.3f} -> lambda {lam:.4e}; FISTA 20000 steps")
    xf, rf = H.fom("fista", K, y, lam, 20000, tau=tau)
    err = np.linalg.norm(xf.cpu().numpy() - xg.cpu().numpy()) / np.linalg.norm(xg.cpu().numpy())
    say(f"   ||x_fista - x_gpss|| / ||x_gpss|| = {err:.2e}, ||x_fista||_1 / rho = {rf['l1norm'] / rho:.8f}")
    assert err <= 1e-6
    assert rf["l1norm"] == pytest.approx(rho, rel=1e-6)


def test_psd_stationary_and_errors(H):
    K = _t(np.eye(3))
    y = _t(np.zeros(3))
    x, r = H.fom("psd", K, y, 1.0, 10)              # y = 0: r = 0 at x = 0
    assert r["status_name"] == "stationary" and r["iters"] == 0 and not x.any().item()
    with pytest.raises(ValueError):
        H.fom("gpsr", K, y, 1.0, 10)
    lib = gpl1.load()
    res = gpl1.GPResult()
    o = gpl1.default_opts()
    p = K.data_ptr()
    ro, rr = C.byref(o), C.byref(res)
    assert lib.gp_fom_solve(H.h, 7, gpl1.GP_F64, p, 3, 3, 3, p, 1.0, 1.0, None, 5, p, ro, rr, None) == -1
    assert lib.gp_fom_solve(H.h, gpl1.GP_ISTA, gpl1.GP_F64, p, 3, 3, 3, p, -1.0, 1.0, None, 5, p, ro, rr,
                            None) == -1
    # ldk < p: refused before any launch
    assert lib.gp_fom_solve(H.h, gpl1.GP_PSD, gpl1.GP_F64, p, 3, 3, 2, p, 1.0, 1.0, None, 5, p, ro,
                            rr, None) == -1
