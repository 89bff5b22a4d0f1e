"""Exact references that pin the oracle (test infrastructure only).

* `constrained_ls_bruteforce` solves problem (2) of Section 1 exactly for tiny
  full-column-rank K by enumerating supports and sign patterns.  If the
  unconstrained least-squares solution is inside the ball it is the answer;
  otherwise the minimiser lies on the sphere ||x||_1 = rho, where on its support
  S with signs sigma it solves the equality-constrained least-squares problem
      min ||K_S x_S - y||^2  s.t.  sigma^T x_S = rho,
  whose KKT system is  [2 K_S^T K_S  sigma; sigma^T 0] [x_S; nu] = [2 K_S^T y; rho].
  Every sign-consistent candidate is feasible; the smallest objective wins.
* `project_l1_bruteforce` does the same for the projection of a vector.
* `lambda_of_rho` is the relation of Section 1:
  lambda = max_i |(K^T (y - K x~(rho)))_i|.
"""
import itertools
import numpy as np


def _candidates_on_sphere(G, b, rho, p):
    """Yield x on ||x||_1 = rho minimising 0.5 x^T G x - b^T x on each
    (support, sign) face, when the face minimiser is sign consistent."""
    for size in range(1, p + 1):
        for S in itertools.combinations(range(p), size):
            S = list(S)
            for signs in itertools.product((-1.0, 1.0), repeat=size):
                sg = np.array(signs)
                A = np.zeros((size + 1, size + 1))
                A[:size, :size] = G[np.ix_(S, S)]
                A[:size, size] = sg
                A[size, :size] = sg
                rhs = np.concatenate([b[S], [rho]])
                try:
                    sol = np.linalg.solve(A, rhs)
                except np.linalg.LinAlgError:
                    continue
                xs = sol[:size]
                if np.all(sg * xs >= -1e-12):
                    x = np.zeros(p)
                    x[S] = xs
                    yield x


def constrained_ls_bruteforce(K, y, rho):
    """Exact argmin_{||x||_1 <= rho} ||Kx - y||^2 for tiny K with full column rank."""
    K = np.asarray(K, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    p = K.shape[1]
    if np.linalg.matrix_rank(K) < p:
        raise ValueError("brute force needs full column rank")
    x_ls = np.linalg.lstsq(K, y, rcond=None)[0]
    if np.abs(x_ls).sum() <= rho:
        return x_ls
    G = 2.0 * K.T @ K
    b = 2.0 * K.T @ y
    best, best_f = None, np.inf
    for x in _candidates_on_sphere(G, b, rho, p):
        r = K @ x - y
        fx = r @ r
        if fx < best_f:
            best, best_f = x, fx
    return best


def project_l1_bruteforce(v, rho):
    """Exact nearest point of {||h||_1 <= rho} to v by enumeration (p <= 8)."""
    v = np.asarray(v, dtype=np.float64)
    p = v.size
    if np.abs(v).sum() <= rho:
        return v.copy()
    if rho == 0:
        return np.zeros(p)
    # minimise ||h - v||^2 = h^T h - 2 v^T h + const: G = 2I, b = 2v
    G = 2.0 * np.eye(p)
    b = 2.0 * v
    best, best_d = None, np.inf
    for h in _candidates_on_sphere(G, b, rho, p):
        dist = np.sum((h - v) ** 2)
        if dist < best_d:
            best, best_d = h, dist
    return best


def lambda_of_rho(K, y, x):
    """lambda = ||K^T (y - K x)||_inf at a solution x of problem (2)."""
    return float(np.abs(K.T @ (y - K @ x)).max())

