"""The rho sweep of the Section 4 experiment, reduced in size: one batched
call with a radius per column (one shared y), against exact references from
the homotopy (LARS-lasso) path, which the FP64 oracle confirms on sampled
points (the solution of (2) at rho = ||x_bar(lambda)||_1 is x_bar(lambda),
Section 1).

Bars: homotopy reference vs oracle 1e-7 (relative x error; both FP64, the
oracle at its stationarity floor); GPU columns vs reference 1e-4 (the FP32
bar); the same columns through the plain solver, and the isochrone methods
run to convergence at the grid's middle point, to the same bar.
"""
import sys
import warnings

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


def test_rho_sweep_matches_homotopy_references(H):
    import bench
    inst = instances.paper_gaussian(n=240, p=960, s=12, seed=19)
    K64, y64 = inst.K64, inst.y64
    lam_max = float(np.abs(K64.T @ y64).max())
    l2 = 6.0 * (np.arange(12) + 1) / 12
    lams = lam_max * 2.0 ** (-l2)
    with warnings.catch_warnings():
        warnings.simplefilter("ignore")
        xbar = bench.lasso_references(K64, y64, lams)
    kkt = [abs(float(np.abs(K64.T @ (y64 - K64 @ x)).max()) - l) / l for x, l in zip(xbar, lams)]
    assert max(kkt) <= 1e-9
    rhos = np.abs(xbar).sum(axis=1)
    for j in (0, 5, 11):
        o = gpss(K64, y64, float(rhos[j]), tol=0.0, max_iter=100000)
        assert np.linalg.norm(o["x"] - xbar[j]) / np.linalg.norm(xbar[j]) <= 1e-7
    K = torch.from_numpy(inst.K_store).to(DEV)
    y = torch.from_numpy(inst.y_store).to(DEV)
    Y = y.unsqueeze(0).repeat(len(lams), 1).contiguous()
    say(f"[sweep] 240x960 unit-norm K, {len(lams)} radii as columns of one batch")
    X, res = H.solve_batched_shared(K, Y, rhos, tol=1e-12, max_iter=20000, refresh_every=50)
    errs = [float(np.linalg.norm(X[j].cpu().double().numpy() - xbar[j]) / np.linalg.norm(xbar[j]))
            for j in range(len(lams))]
    say(f"   worst column error {max(errs):.2e}")
    assert all(r["status"] >= 0 for r in res) and max(errs) <= 1e-4
    # the middle radius through the plain solver and the isochrone methods
    j = 5
    xs, _ = H.solve(K, y, float(rhos[j]), tol=1e-12, max_iter=20000, refresh_every=50)
    xi, _ = H.fom("fista", K, y, float(lams[j]), 3000)
    xp, _ = H.fom("psd", K, y, float(rhos[j]), 3000)
    for name, xt in (("gpss", xs), ("fista", xi), ("psd", xp)):
        e = float(np.linalg.norm(xt.cpu().double().numpy() - xbar[j]) / np.linalg.norm(xbar[j]))
        say(f"   {name}: e = {e:.2e}")
        assert e <= 1e-4, name
