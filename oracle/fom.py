"""The paper's fully specified comparison methods in FP64 (Section 2, items 1,
2 and 5).  TEST INFRASTRUCTURE ONLY.

ISTA and FISTA minimise the penalised functional (1) of Section 1,
    F(x) = ||K x - y||^2 + 2 lambda ||x||_1;
PSD minimises f(x) = ||K x - y||^2 over the l1 ball of radius rho, problem (2).

  * ISTA (item 1):  x <- S_lambda[x + K^T (y - K x)], with the soft
    threshold (S_t[v])_i = v_i - t sgn(v_i) for |v_i| > t, else 0.  The paper
    states it for ||K|| < sqrt(2).  `tau` scales the step for other operators:
    x <- S_{tau lambda}[x + tau K^T (y - K x)] is the same forward-backward
    step applied to F (tau = 1 is the paper's form; it converges for
    tau < 2 / ||K||^2).
  * FISTA (item 2, equation (3)):  with T(x) = S_lambda[x + K^T (y - K x)],
        x^(k+1) = T(x^(k) + ((t^(k) - 1) / t^(k+1)) (x^(k) - x^(k-1))),
        t^(0) = 1,  t^(k+1) = (1 + sqrt(1 + 4 (t^(k))^2)) / 2,
    started at x^(0) = 0 (the momentum factor is 0 at k = 0).  `tau` as for
    ISTA (the paper's form is tau = 1, for ||K|| <= 1).
  * PSD (item 5):  x <- P_Omega[x + beta r] with r = K^T (y - K x) and
    beta = ||r||^2 / ||K r||^2 (the exact minimiser of f along r).

Readings where the paper is silent (also in the design notes): every method
stops after `max_iter` iterations, or earlier when `tol` > 0 and the relative
change of its objective, (F_old - F_new) / F_old, falls below tol; PSD stops
when r = 0 (x is then the unconstrained minimiser) or K r = 0 (beta
undefined); ISTA and FISTA start from x0 (default 0), PSD from P_Omega(x0).
"""
import math

import numpy as np

from .projection import project_l1, soft_threshold


def penalised_objective(K, y, x, lam):
    """F(x) = ||K x - y||^2 + 2 lambda ||x||_1, functional (1) of Section 1."""
    r = K @ x - y
    return float(r @ r) + 2.0 * lam * float(np.abs(x).sum())


def ista(K, y, lam, x0=None, *, tau=1.0, max_iter=1000, tol=0.0, trace=False):
    """ISTA of Section 2, item 1.  Returns dict(x, F, iters, status[, trace])."""
    K = np.asarray(K, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    x = np.zeros(K.shape[1]) if x0 is None else np.array(x0, dtype=np.float64)
    F = penalised_objective(K, y, x, lam)
    rec = []
    status = "max_iter"
    it = 0
    for it in range(1, max_iter + 1):
        r = K.T @ (y - K @ x)                      # the residual of step k
        x = soft_threshold(x + tau * r, tau * lam)
        Fn = penalised_objective(K, y, x, lam)
        if trace:
            rec.append(dict(k=it - 1, F=Fn, x=x.copy()))
        rel = (F - Fn) / F if F > 0 else 0.0
        F = Fn
        if tol > 0 and rel < tol:
            status = "tol"
            break
    out = dict(x=x, F=F, iters=it, status=status)
    if trace:
        out["trace"] = rec
    return out


def fista_t(k):
    """t^(k) of equation (3): t^(0) = 1, t^(j+1) = (1 + sqrt(1 + 4 t^(j)^2)) / 2."""
    t = 1.0
    for _ in range(k):
        t = (1.0 + math.sqrt(1.0 + 4.0 * t * t)) / 2.0
    return t


def fista(K, y, lam, x0=None, *, tau=1.0, max_iter=1000, tol=0.0, trace=False):
    """FISTA, equation (3).  Returns dict(x, F, iters, status[, trace])."""
    K = np.asarray(K, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    x = np.zeros(K.shape[1]) if x0 is None else np.array(x0, dtype=np.float64)
    x_prev = x.copy()
    t = 1.0
    F = penalised_objective(K, y, x, lam)
    rec = []
    status = "max_iter"
    it = 0
    for it in range(1, max_iter + 1):
        t_next = (1.0 + math.sqrt(1.0 + 4.0 * t * t)) / 2.0
        z = x + ((t - 1.0) / t_next) * (x - x_prev)
        x_new = soft_threshold(z + tau * (K.T @ (y - K @ z)), tau * lam)
        Fn = penalised_objective(K, y, x_new, lam)
        if trace:
            rec.append(dict(k=it - 1, t=t, t_next=t_next, z=z.copy(), F=Fn, x=x_new.copy()))
        x_prev, x, t = x, x_new, t_next
        rel = (F - Fn) / F if F > 0 else 0.0
        F = Fn
        if tol > 0 and abs(rel) < tol:
            status = "tol"
            break
    out = dict(x=x, F=F, iters=it, status=status)
    if trace:
        out["trace"] = rec
    return out


def psd(K, y, rho, x0=None, *, max_iter=1000, tol=0.0, trace=False):
    """Projected steepest descent of Section 2, item 5, on problem (2).
    Returns dict(x, f, iters, status[, trace])."""
    K = np.asarray(K, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    x = np.zeros(K.shape[1]) if x0 is None else np.array(x0, dtype=np.float64)
    if np.abs(x).sum() > rho:
        x = project_l1(x, rho)
    res = K @ x - y
    f = float(res @ res)
    rec = []
    status = "max_iter"
    it = 0
    for it in range(1, max_iter + 1):
        r = K.T @ (y - K @ x)
        Kr = K @ r
        rr, kk = float(r @ r), float(Kr @ Kr)
        if rr == 0.0 or kk == 0.0:
            status = "stationary"
            it -= 1
            break
        beta = rr / kk
        x = project_l1(x + beta * r, rho)
        res = K @ x - y
        fn = float(res @ res)
        if trace:
            rec.append(dict(k=it - 1, beta=beta, f=fn, x=x.copy()))
        rel = (f - fn) / f if f > 0 else 0.0
        f = fn
        if tol > 0 and abs(rel) < tol:
            status = "tol"
            break
    out = dict(x=x, f=f, iters=it, status=status)
    if trace:
        out["trace"] = rec
    return out
