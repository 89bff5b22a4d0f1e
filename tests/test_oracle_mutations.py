"""Planted mistakes in the oracle must be caught by its pins.

Each case rewrites one line of the oracle's source (on the CPU, in a private
module copy), then runs a pin from test_oracle against it and expects it to
fail.  This shows the pins are sensitive to the plausible mistakes: a dropped
factor, a swapped ratio, a wrong sign, an off-by-one window or threshold.
"""
import os
import sys
import types

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _load_mutant(module, old, new):
    """Fresh copy of the oracle package with one textual change in `module`."""
    pkg = types.ModuleType("oracle_mut")
    pkg.__path__ = [os.path.join(ROOT, "oracle")]
    sys.modules["oracle_mut"] = pkg
    mods = {}
    for name in ("projection", "gpss", "fom"):
        path = os.path.join(ROOT, "oracle", f"{name}.py")
        src = open(path).read()
        if name == module:
            assert old in src, f"mutation anchor not found: {old!r}"
            src = src.replace(old, new)
        m = types.ModuleType(f"oracle_mut.{name}")
        m.__package__ = "oracle_mut"
        m.__file__ = path
        sys.modules[f"oracle_mut.{name}"] = m
        exec(compile(src, path, "exec"), m.__dict__)
        mods[name] = m
    return mods


def _pins_pass(mods):
    """Run a subset of the pins against a (possibly mutated) oracle; an
    exception counts as a failed pin."""
    try:
        return _pins(mods)
    except Exception:
        return False


def _pins(mods):
    gp = mods["gpss"]
    pj = mods["projection"]
    from oracle import exact
    ok = True
    # hand-derived trajectories
    for K, y, rho, a0, a1, a2 in (
            (np.diag([1.0, 0.5]), np.array([1.0, 1.0]), 100.0, 0.5, 10 / 17, 2.0),
            (np.diag([1.0, 0.1]), np.array([1.0, 100.0]), 1000.0, 0.05, 100 / 101, 100 / 101)):
        out = gp.gpss(K, y, rho, tol=0.0, max_iter=2, trace=True)
        tr = out["trace"]
        ok &= len(tr) == 2
        if len(tr) == 2:
            ok &= np.isclose(tr[0]["alpha"], a0, rtol=1e-12)
            ok &= np.isclose(tr[1]["alpha"], a1, rtol=1e-12)
            ok &= np.isclose(tr[1]["alpha_next"], a2, rtol=1e-12)
    # hand example with one backtracking step (test_gpss_backtracking_hand_example)
    out = gp.gpss(np.array([[2.0]]), np.array([1.0]), 10.0, tol=0.0, max_iter=1,
                  trace=True)
    ok &= out["trace"][0]["lam"] == 0.5 and np.isclose(out["x"][0], 0.5)
    # brute-force projections
    for seed in range(20):
        rng = np.random.default_rng(seed)
        v = rng.standard_normal(5)
        rho = float(rng.uniform(0.1, 0.9) * np.abs(v).sum())
        ok &= np.allclose(pj.project_l1(v, rho), exact.project_l1_bruteforce(v, rho),
                          atol=1e-12)
    # brute-force constrained least squares
    for seed in range(6):
        rng = np.random.default_rng(300 + seed)
        K = rng.standard_normal((8, 4))
        y = rng.standard_normal(8)
        rho = 0.5 * np.abs(np.linalg.lstsq(K, y, rcond=None)[0]).sum()
        try:
            out = gp.gpss(K, y, rho, tol=1e-15, max_iter=3000)
            ok &= np.allclose(out["x"], exact.constrained_ls_bruteforce(K, y, rho), atol=1e-7)
        except Exception:
            ok = False
    # the alternation rule in isolation (window and tau updates)
    st = gp.SSState(tau=0.5)
    P = gp.GPSSParams()
    gp.ss_update(3, 4.0, 1.0, 2.0, st, P)
    gp.ss_update(4, 1.0, 1.0, 1.25, st, P)
    gp.ss_update(5, 10.0, 1.0, 1 / 0.9, st, P)
    a, _ = gp.ss_update(6, 10.0, 1.0, 1 / 0.95, st, P)
    ok &= np.isclose(a, 0.8) and np.isclose(st.tau, 0.5 * 0.9 * 1.1 * 0.9 * 0.9)
    # nonmonotone window (test_gpss_nonmonotone_hand_example): at k = 1 the
    # window of M = 2 still holds f0 = 30 and accepts the rise to 29.09; at
    # k = 2 it holds only f1, f2
    K, y = np.diag([1.0, 3.0, 5.0]), np.array([5.0, 2.0, 1.0])
    tr1 = gp.gpss(K, y, 100.0, tol=0.0, max_iter=2, trace=True,
                  params=gp.GPSSParams(M=1))["trace"]
    ok &= tr1[1]["lam"] == 0.5 and tr1[1]["nb"] == 1
    tr2 = gp.gpss(K, y, 100.0, tol=0.0, max_iter=3, trace=True,
                  params=gp.GPSSParams(M=2))["trace"]
    ok &= tr2[1]["lam"] == 1.0 and np.isclose(tr2[1]["f_new"], 29.091255602545022, rtol=1e-13)
    ok &= np.isclose(tr2[2]["fmax"], 29.091255602545022, rtol=1e-13)
    # comparison methods (test_oracle_fom, tests/golden/fom_hand_examples.txt)
    fm = mods["fom"]
    K1, y1 = np.array([[0.5]]), np.array([1.0])
    tr = fm.ista(K1, y1, 0.1, max_iter=3, trace=True)["trace"]
    ok &= np.allclose([r["x"][0] for r in tr], [0.4, 0.7, 0.925], rtol=1e-14)
    tr = fm.fista(K1, y1, 0.1, max_iter=3, trace=True)["trace"]
    ok &= np.allclose([r["x"][0] for r in tr], [0.4, 0.7845260575375963, 1.1135701132020648], rtol=1e-13)
    K2, y2 = np.diag([1.0, 0.5]), np.array([1.0, 1.0])
    tr = fm.psd(K2, y2, 100.0, max_iter=2, trace=True)["trace"]
    ok &= np.allclose(tr[1]["x"], [25 / 34, 25 / 17], rtol=1e-13)
    tr = fm.psd(K2, y2, 1.0, max_iter=1, trace=True)["trace"]
    ok &= np.allclose(tr[0]["x"], [27 / 34, 7 / 34], rtol=1e-13)
    return bool(ok)


def test_unmutated_oracle_passes_pins():
    assert _pins_pass(_load_mutant("gpss", "", ""))


MUTATIONS = [
    ("gpss", "g = 2.0 * (K.T @ r)\n", "g = (K.T @ r)\n"),                 # dropped factor 2
    ("gpss", "a1 = _clamp(ss / sz, p)", "a1 = _clamp(sz / ss, p)"),        # inverted BB1
    ("gpss", "a2 = _clamp(sz / zz, p)", "a2 = _clamp(zz / sz, p)"),        # inverted BB2
    ("gpss", "state.tau *= 0.9", "state.tau *= 1.1"),                      # wrong tau update
    ("gpss", "first = max(1, k - p.M_alpha)", "first = max(1, k - p.M_alpha + 1)"),  # window
    ("gpss", "if a2 / a1 <= state.tau:", "if a1 / a2 <= state.tau:"),      # ratio flipped
    ("gpss", "ft <= fmax + p.beta * lam * gd", "ft <= fmax - p.beta * lam * gd"),  # Armijo sign
    ("gpss", "z = g_new - g\n", "z = g - g_new\n"),                         # sign of z
    ("gpss", "alpha = p.alpha_max if nrm == 0.0 else _clamp(1.0 / nrm, p)",
             "alpha = p.alpha_max if nrm == 0.0 else _clamp(nrm, p)"),     # alpha_0
    ("gpss", "fmax = max(f_hist[-p.M:])", "fmax = f_hist[-1]"),         # memory M ignored
    ("gpss", "fmax = max(f_hist[-p.M:])", "fmax = max(f_hist[-(p.M + 1):])"),  # window too long
    ("gpss", "fmax = max(f_hist[-p.M:])", "fmax = max(f_hist[-p.M:][1:] or f_hist[-1:])"),  # too short
    ("gpss", "f_hist.append(f)", "f_hist.append(f_hist[-1])"),             # stale history
    ("fom", "z = x + ((t - 1.0) / t_next) * (x - x_prev)", "z = x + (t / t_next) * (x - x_prev)"),  # momentum
    ("fom", "t_next = (1.0 + math.sqrt(1.0 + 4.0 * t * t)) / 2.0",
            "t_next = (1.0 + math.sqrt(1.0 + 2.0 * t * t)) / 2.0"),           # t recursion
    ("fom", "x = soft_threshold(x + tau * r, tau * lam)",
            "x = soft_threshold(x + tau * r, 2.0 * tau * lam)"),             # ISTA threshold
    ("fom", "r = K.T @ (y - K @ x)                      # the residual of step k",
            "r = K.T @ (K @ x - y)"),                                        # residual sign
    ("fom", "beta = rr / kk", "beta = kk / rr"),                              # PSD step inverted
    ("fom", "x = project_l1(x + beta * r, rho)", "x = x + beta * r"),        # PSD without P
    ("projection", "t = (cw[jstar] - rho) / (jstar + 1)", "t = (cw[jstar] - rho) / (jstar + 2)"),
    ("projection", "positive = w - (cw - rho) / j > 0", "positive = w - (cw + rho) / j > 0"),
]


@pytest.mark.parametrize("module,old,new", MUTATIONS)
def test_planted_mistake_is_caught(module, old, new):
    assert not _pins_pass(_load_mutant(module, old, new))
