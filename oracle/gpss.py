"""GPSS in FP64: Algorithm 1 (gradient projection, GP) with the steplength
rule of Algorithm 2 (SS), Section 3 of the paper.  TEST INFRASTRUCTURE ONLY.

Problem (2), Section 1:  minimise f(x) = ||K x - y||^2  over ||x||_1 <= rho.
f carries no 1/2 factor, so grad f(x) = 2 K^T (K x - y).

One iteration k, in the paper's order:
  * choose alpha_k (Algorithm 2; alpha_0 from the parameter list that closes
    Section 3);
  * h = P_Omega(x - alpha_k grad f(x)); stop (stationary) when h == x;
  * d = h - x;
  * lambda = 1, f_max = max of the last M objective values;
  * backtrack lambda <- theta*lambda until
        f(x + lambda d) <= f_max + beta * lambda * grad f(x)^T d;
  * x <- x + lambda d.
Algorithm 2 then uses s = x_new - x_old and z = grad f(x_new) - grad f(x_old)
in the two Barzilai-Borwein ratios of equation (5).

Readings where the paper is silent (each is also listed with the design notes):
  * f(x + lambda d) is evaluated as ||r + lambda K d||^2 with r = K x - y, which
    equals ||K(x + lambda d) - y||^2 by linearity; r is carried along.
  * backtracking is capped (default 60 reductions); hitting the cap stops the
    run with status "backtrack_limit" and x unchanged.
  * when s^T z <= 0 the threshold tau is left unchanged and no alpha^(2) is
    recorded for that iteration; the minimum over the alpha^(2) window runs
    over the recorded values of iterations max(1, k - M_alpha) .. k.
  * the ratio test and the window minimum use the clamped alpha^(1), alpha^(2).
  * alpha_0 uses ||P_Omega(x0 - grad f(x0))||_inf literally; if that norm is 0,
    alpha_0 = alpha_max.
  * an infeasible x0 is projected onto Omega first (Algorithm 1 requires x0 in
    Omega).
  * stationarity: besides h == x, a direction with grad f(x)^T d >= 0 also
    stops the run as stationary.  In exact arithmetic d != 0 is a descent
    direction (Section 3), so a non-negative slope only arises from rounding
    at a point that is stationary to working precision; continuing would let
    the Armijo test accept increases and drift off the ball.
  * besides the stationarity stop, runs stop on a relative objective change
    (f_old - f_new)/f_old < tol, on f_new <= f_target, or on max_iter.
"""
from dataclasses import dataclass, field
import numpy as np

from .projection import project_l1

STATUS_NAMES = ("tol", "stationary", "max_iter", "target", "backtrack_limit")


@dataclass
class GPSSParams:
    """Parameter values the paper uses for GPSS in all its experiments."""
    M: int = 1               # line-search memory (1 = monotone Armijo)
    theta: float = 0.5       # backtracking reduction factor
    beta: float = 1e-4       # sufficient-decrease constant
    alpha_min: float = 1e-10
    alpha_max: float = 1e10
    tau1: float = 0.5        # initial alternation threshold
    M_alpha: int = 2         # alpha^(2) window is the last M_alpha + 1 iterations
    backtrack_cap: int = 60


def _clamp(a, p: GPSSParams):
    return max(p.alpha_min, min(a, p.alpha_max))


@dataclass
class SSState:
    """State Algorithm 2 carries between iterations."""
    tau: float
    a2_hist: list = field(default_factory=list)   # (iteration index j, alpha_j^(2))


def ss_update(k, ss, sz, zz, state: SSState, p: GPSSParams):
    """Algorithm 2 for iteration k >= 1, given s^T s, s^T z, z^T z of the step
    from iteration k-1 to k.  Returns (alpha_k, rule) and updates `state`.

    rule is "max" (s^T z <= 0), "bb2min" or "bb1"."""
    if sz <= 0.0:
        return p.alpha_max, "max"
    a1 = _clamp(ss / sz, p)
    a2 = _clamp(sz / zz, p) if zz > 0.0 else p.alpha_max
    state.a2_hist.append((k, a2))
    first = max(1, k - p.M_alpha)
    state.a2_hist = [(j, v) for (j, v) in state.a2_hist if j >= first]
    if a2 / a1 <= state.tau:
        alpha = min(v for (_, v) in state.a2_hist)
        state.tau *= 0.9
        return alpha, "bb2min"
    state.tau *= 1.1
    return a1, "bb1"


def gpss(K, y, rho, x0=None, *, tol=1e-10, max_iter=100000, f_target=None,
         params: GPSSParams = None, trace=False):
    """Run GPSS on min ||Kx - y||^2 s.t. ||x||_1 <= rho, all in float64.

    Returns a dict with x, f, status (one of STATUS_NAMES), iters (accepted
    updates), backtracks, lambda_est = ||K^T (y - K x)||_inf (the lambda that
    Section 1 pairs with rho), l1norm, projected_x0 and, if `trace`, a list of
    per-iteration records."""
    p = params or GPSSParams()
    K = np.asarray(K, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    n, pdim = K.shape
    if rho < 0 or not np.isfinite(rho):
        raise ValueError("rho must be finite and >= 0")
    x = np.zeros(pdim) if x0 is None else np.array(x0, dtype=np.float64)
    projected = False
    if np.abs(x).sum() > rho:
        x = project_l1(x, rho)
        projected = True

    r = K @ x - y
    g = 2.0 * (K.T @ r)
    f = float(r @ r)
    nrm = np.abs(project_l1(x - g, rho)).max() if pdim else 0.0
    alpha = p.alpha_max if nrm == 0.0 else _clamp(1.0 / nrm, p)
    st = SSState(tau=p.tau1)
    f_hist = [f]
    rec = []
    status = "max_iter"
    iters = 0
    backtracks = 0
    rel = np.inf
    for k in range(max_iter):
        h = project_l1(x - alpha * g, rho)
        d = h - x
        gd = float(g @ d)
        if not np.any(d) or gd >= 0.0:
            status = "stationary"
            break
        q = K @ d
        fmax = max(f_hist[-p.M:])
        lam = 1.0
        nb = 0
        while True:
            rt = r + lam * q
            ft = float(rt @ rt)
            if ft <= fmax + p.beta * lam * gd:
                break
            nb += 1
            if nb > p.backtrack_cap:
                break
            lam *= p.theta
        if nb > p.backtrack_cap:
            status = "backtrack_limit"
            break
        backtracks += nb
        x_new = x + lam * d
        r_new = r + lam * q
        g_new = 2.0 * (K.T @ r_new)
        s = x_new - x
        z = g_new - g
        ss, sz, zz = float(s @ s), float(s @ z), float(z @ z)
        alpha_used = alpha
        alpha, rule = ss_update(k + 1, ss, sz, zz, st, p)
        rel = (f - ft) / f
        if trace:
            rec.append(dict(k=k, f=f, f_new=ft, alpha=alpha_used, lam=lam,
                            nb=nb, gd=gd, fmax=fmax, ss=ss, sz=sz, zz=zz, rule=rule,
                            tau=st.tau, alpha_next=alpha,
                            l1=float(np.abs(x_new).sum())))
        x, r, g, f = x_new, r_new, g_new, ft
        f_hist.append(f)
        iters = k + 1
        if f_target is not None and f <= f_target:
            status = "target"
            break
        if tol > 0 and rel < tol:
            status = "tol"
            break
    else:
        status = "max_iter"
    out = dict(x=x, f=f, status=status, iters=iters, backtracks=backtracks,
               lambda_est=float(np.abs(g).max() / 2.0) if pdim else 0.0,
               l1norm=float(np.abs(x).sum()), projected_x0=projected,
               rel_change=float(rel), alpha_next=alpha, tau=st.tau)
    if trace:
        out["trace"] = rec
    return out
