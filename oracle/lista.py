"""Unrolled soft-thresholding network in FP64 (test infrastructure only).

ISTA (Section 2, item 1) iterates x <- S_lambda[x + K^T (y - K x)].  With a
step 1/L that is x <- S_{lambda/L}[(I - K^T K / L) x + K^T y / L], i.e. a fixed
affine map followed by soft thresholding.  The learned variant keeps the same
shape but treats the two matrices and the per-layer thresholds as parameters:

    c        = W_e y                       (W_e : p x n)
    u^1      = c,            x^1 = S_{theta_1}[u^1]
    u^t      = c + S x^{t-1}, x^t = S_{theta_t}[u^t]     t = 2..T  (S : p x p)

Columns of Y (n x B) are independent samples.  The training loss is
    loss = 1/(2B) sum_b ||x^T_b - x*_b||^2.
The soft threshold's derivative is taken as 1[|u| > theta] for u and
-sgn(u) 1[|u| > theta] for theta (0 at the kink).
"""
import numpy as np

from .projection import soft_threshold


def ista_init(K, lam):
    """ISTA weights for step 1/L, L = ||K||_2^2: W_e = K^T/L, S = I - K^T K/L,
    theta_t = lam/L for every layer."""
    K = np.asarray(K, dtype=np.float64)
    L = np.linalg.norm(K, 2) ** 2
    We = K.T / L
    S = np.eye(K.shape[1]) - (K.T @ K) / L
    return We, S, lam / L


def forward(We, S, thetas, Y):
    """Return the list of (u^t, x^t) for t = 1..T and the output x^T."""
    We = np.asarray(We, dtype=np.float64)
    S = np.asarray(S, dtype=np.float64)
    Y = np.asarray(Y, dtype=np.float64)
    c = We @ Y
    cache = []
    x = None
    for t, th in enumerate(thetas):
        u = c if t == 0 else c + S @ x
        x = soft_threshold(u, th)
        cache.append((u, x))
    return x, cache, c


def loss(We, S, thetas, Y, Xstar):
    x, _, _ = forward(We, S, thetas, Y)
    B = Y.shape[1]
    return 0.5 * np.sum((x - Xstar) ** 2) / B


def backward(We, S, thetas, Y, Xstar):
    """Loss and gradients (dWe, dS, dthetas) by reverse accumulation."""
    x, cache, c = forward(We, S, thetas, Y)
    B = Y.shape[1]
    T = len(thetas)
    L = 0.5 * np.sum((x - Xstar) ** 2) / B
    dx = (x - Xstar) / B
    dS = np.zeros_like(S, dtype=np.float64)
    dc = np.zeros_like(c)
    dth = np.zeros(T)
    for t in range(T - 1, -1, -1):
        u, _ = cache[t]
        active = np.abs(u) > thetas[t]
        du = dx * active
        dth[t] = -np.sum(dx * np.sign(u) * active)
        dc += du
        if t > 0:
            x_prev = cache[t - 1][1]
            dS += du @ x_prev.T
            dx = S.T @ du
    dWe = dc @ Y.T
    return L, dWe, dS, dth
