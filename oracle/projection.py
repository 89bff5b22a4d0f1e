"""Euclidean projection onto the l1 ball, FP64 (test infrastructure only).

The paper uses the projection P_Omega onto Omega = {x : ||x||_1 <= rho}
(Section 2, item 5, and Algorithm 1) without spelling out how it is computed.
The textbook method is the sort-based one (Duchi, Shalev-Shwartz, Singer,
Chandra, ICML 2008), written out here step by step:

    if ||v||_1 <= rho:  P(v) = v
    else: u = |v| sorted decreasingly, c_j = u_1 + ... + u_j,
          j* = max{ j : u_j - (c_j - rho)/j > 0 },
          mu = (c_{j*} - rho) / j*,
          P(v)_i = sgn(v_i) * max(|v_i| - mu, 0)      (= S_mu[v], Section 2)

The result is the soft-thresholding S_mu of Section 2 with the threshold mu
chosen so that ||S_mu[v]||_1 = rho.

Rounding order: every quantity is taken relative to m = max|v| (w_j = u_j - m,
t = mu - m, h_i = (|v_i| - m) - t).  This is the same formula, but it stays
exact when rho is far below the size of v (GP can use alpha up to 1e10), where
c_j - rho would round to c_j.  With w_1 = 0 the first test reads rho > 0, so
j* >= 1 always.
"""
import numpy as np


def soft_threshold(v, t):
    """(S_t[v])_i = v_i - t sgn(v_i) if |v_i| > t else 0  (Section 2, item 1)."""
    v = np.asarray(v, dtype=np.float64)
    return np.sign(v) * np.maximum(np.abs(v) - t, 0.0)


def project_l1_mu(v, rho):
    """Return (P_Omega(v), mu) with mu the threshold (0 when v is inside)."""
    v = np.asarray(v, dtype=np.float64)
    if rho < 0 or not np.isfinite(rho):
        raise ValueError("rho must be finite and >= 0")
    if rho == 0.0:
        return np.zeros_like(v), (float(np.abs(v).max()) if v.size else 0.0)
    a = np.abs(v)
    if a.sum() <= rho:
        return v.copy(), 0.0
    m = a.max()
    w = np.sort(a)[::-1] - m                  # u_j - m  (<= 0)
    cw = np.cumsum(w)                         # c_j - j m
    j = np.arange(1, w.size + 1)
    positive = w - (cw - rho) / j > 0         # u_j - (c_j - rho)/j > 0
    jstar = int(np.nonzero(positive)[0][-1])  # 0-based index of j*
    t = (cw[jstar] - rho) / (jstar + 1)       # mu - m
    h = np.sign(v) * np.maximum((a - m) - t, 0.0)
    return h, float(m + t)


def project_l1(v, rho):
    return project_l1_mu(v, rho)[0]
