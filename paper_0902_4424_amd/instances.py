"""Seeded synthetic problem instances for l1-constrained least squares.

This module only *builds* inputs: it draws K, a sparse x_true and noisy data
y = K x_true + noise, fixes the radius rho of the l1 ball, and rounds K and y to
a storage dtype.  It contains none of the solver's arithmetic, so both the
FP64 oracle and the HIP path can be fed from it.

Problem (the constrained form (2) of the paper, Section 1):
    x~(rho) = argmin_{||x||_1 <= rho} ||K x - y||^2,   K is n x p, row-major.

Draw order for every instance, from one numpy PCG64 stream seeded by `seed`:
    1. K (row-major, n x p), 2. support (without replacement), 3. amplitudes,
    4. noise.  Then y = K_fp64 @ x_true + noise in FP64, then K and y are rounded
    to the storage dtype.  The rounded arrays are the problem both sides solve.

Storage dtypes: "f64"; "f32" (IEEE round-to-nearest-even); "bf16" (K only,
round-to-nearest-even on the FP32 bits, NaN kept quiet; vectors stay FP32).
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np

DTYPES = ("f64", "f32", "bf16")


def f32_to_bf16_bits(a: np.ndarray) -> np.ndarray:
    """Round float32 values to bfloat16 (round to nearest, ties to even).

    Returns the 16-bit patterns as uint16.  NaNs stay NaN (quiet bit set)."""
    a = np.ascontiguousarray(a, dtype=np.float32)
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    rounded = ((u + 0x7FFF + lsb) >> 16).astype(np.uint32)
    nan = np.isnan(a)
    if nan.any():
        rounded = np.where(nan, ((u >> 16) | 0x40).astype(np.uint32), rounded)
    return rounded.astype(np.uint16)


def bf16_bits_to_f32(b: np.ndarray) -> np.ndarray:
    """Widen bfloat16 bit patterns (uint16) to float32 exactly."""
    b = np.ascontiguousarray(b, dtype=np.uint16)
    return (b.astype(np.uint32) << 16).view(np.float32)


@dataclass
class Instance:
    """One stored problem.  `K_store`/`y_store` are exactly what a solver sees.

    K_store: float64 / float32 array, or uint16 bf16 bit patterns, shape (n, p).
    y_store: float64 for dtype "f64", else float32, shape (n,).
    """
    name: str
    dtype: str
    K_store: np.ndarray
    y_store: np.ndarray
    rho: float
    x_true: np.ndarray
    seed: int
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return self.K_store.shape[0]

    @property
    def p(self) -> int:
        return self.K_store.shape[1]

    @property
    def K64(self) -> np.ndarray:
        """The stored K widened exactly to float64."""
        if self.dtype == "bf16":
            return bf16_bits_to_f32(self.K_store).astype(np.float64)
        return self.K_store.astype(np.float64)

    @property
    def y64(self) -> np.ndarray:
        return self.y_store.astype(np.float64)

    @property
    def K32(self) -> np.ndarray:
        """The stored K as float32 (exact for f32 and bf16 storage)."""
        if self.dtype == "bf16":
            return bf16_bits_to_f32(self.K_store)
        return self.K_store.astype(np.float32)


def _store(K64: np.ndarray, y64: np.ndarray, dtype: str):
    if dtype == "f64":
        return np.ascontiguousarray(K64), np.ascontiguousarray(y64)
    K32 = np.ascontiguousarray(K64, dtype=np.float32)
    y32 = np.ascontiguousarray(y64, dtype=np.float32)
    if dtype == "f32":
        return K32, y32
    if dtype == "bf16":
        return f32_to_bf16_bits(K32), y32
    raise ValueError(f"unknown dtype {dtype!r}")


def _sparse_signal(rng, p, s, amp):
    support = rng.choice(p, size=s, replace=False)
    if amp == "pm1":
        vals = rng.choice(np.array([-1.0, 1.0]), size=s)
    elif amp == "normal":
        vals = rng.standard_normal(s)
    else:
        raise ValueError(amp)
    x = np.zeros(p)
    x[support] = vals
    return x


def gaussian_instance(n, p, s, *, amp="pm1", sigma=1e-2, rho_scale=1.0,
                      kscale=None, dtype="f32", seed=0, name="gauss",
                      unit_norm=False) -> Instance:
    """Gaussian compressed-sensing instance (the paper's first test operator).

    K_ij ~ N(0, kscale^2) with kscale = 1/sqrt(n) unless given; with
    `unit_norm` K is rescaled to spectral norm 1 as in Section 4.
    rho = rho_scale * ||x_true||_1."""
    rng = np.random.default_rng(seed)
    if kscale is None:
        kscale = 1.0 / np.sqrt(n)
    K = rng.standard_normal((n, p)) * kscale
    if unit_norm:
        K = K / np.linalg.norm(K, 2)
    x_true = _sparse_signal(rng, p, s, amp)
    noise = sigma * rng.standard_normal(n)
    y = K @ x_true + noise
    Ks, ys = _store(K, y, dtype)
    rho = float(rho_scale * np.abs(x_true).sum())
    return Instance(name, dtype, Ks, ys, rho, x_true, seed,
                    dict(n=n, p=p, s=s, sigma=sigma, amp=amp, kscale=kscale))


def haar_orthogonal(rng, m) -> np.ndarray:
    """Haar-distributed orthogonal matrix: QR of a Gaussian matrix with the
    signs of diag(R) folded into Q (Mezzadri, Notices AMS 2007)."""
    A = rng.standard_normal((m, m))
    Q, R = np.linalg.qr(A)
    return Q * np.sign(np.diag(R))[None, :]


def illcond_instance(m, s, *, cond=1e4, sigma=1e-3, amp="pm1", dtype="f32",
                     seed=0, name="illcond") -> Instance:
    """Square ill-conditioned operator K = U diag(sv) V^T with Haar U, V and
    singular values geometric from 1 down to 1/cond (a synthetic stand-in for
    the paper's severely ill-conditioned seismic operator)."""
    rng = np.random.default_rng(seed)
    U = haar_orthogonal(rng, m)
    V = haar_orthogonal(rng, m)
    sv = cond ** (-np.arange(m) / max(m - 1, 1))
    K = (U * sv[None, :]) @ V.T
    x_true = _sparse_signal(rng, m, s, amp)
    noise = sigma * rng.standard_normal(m)
    y = K @ x_true + noise
    Ks, ys = _store(K, y, dtype)
    rho = float(np.abs(x_true).sum())
    return Instance(name, dtype, Ks, ys, rho, x_true, seed,
                    dict(n=m, p=m, s=s, sigma=sigma, cond=cond))


@dataclass
class SharedBatch:
    """Many right-hand sides sharing one stored K.

    Y_store is (B, n): row b is the data vector of column problem b (so each
    right-hand side is contiguous).  rho is (B,)."""
    name: str
    dtype: str
    K_store: np.ndarray
    Y_store: np.ndarray
    rho: np.ndarray
    X_true: np.ndarray
    seed: int
    meta: dict = field(default_factory=dict)

    @property
    def n(self):
        return self.K_store.shape[0]

    @property
    def p(self):
        return self.K_store.shape[1]

    @property
    def B(self):
        return self.Y_store.shape[0]

    @property
    def K64(self):
        if self.dtype == "bf16":
            return bf16_bits_to_f32(self.K_store).astype(np.float64)
        return self.K_store.astype(np.float64)

    @property
    def K32(self):
        if self.dtype == "bf16":
            return bf16_bits_to_f32(self.K_store)
        return self.K_store.astype(np.float32)

    def instance(self, b: int) -> Instance:
        return Instance(f"{self.name}[{b}]", self.dtype, self.K_store,
                        self.Y_store[b], float(self.rho[b]), self.X_true[b],
                        self.seed, dict(self.meta, column=b))


def shared_batch(n, p, B, s, *, amp="pm1", sigma=1e-2, dtype="bf16", seed=0,
                 rhs_seed_base=None, kscale=None, name="shared") -> SharedBatch:
    """One Gaussian K (seed `seed`) and B right-hand sides; right-hand side b
    draws its support, amplitudes and noise from seed rhs_seed_base + b."""
    rng = np.random.default_rng(seed)
    if kscale is None:
        kscale = 1.0 / np.sqrt(n)
    K = rng.standard_normal((n, p)) * kscale
    if rhs_seed_base is None:
        rhs_seed_base = 1000 * seed
    Xt = np.zeros((B, p))
    Y = np.zeros((B, n))
    for b in range(B):
        rb = np.random.default_rng(rhs_seed_base + b)
        Xt[b] = _sparse_signal(rb, p, s, amp)
        Y[b] = K @ Xt[b] + sigma * rb.standard_normal(n)
    Ks, _ = _store(K, Y[0], dtype)
    Ys = Y.astype(np.float64 if dtype == "f64" else np.float32)
    rho = np.abs(Xt).sum(axis=1)
    return SharedBatch(name, dtype, Ks, np.ascontiguousarray(Ys), rho, Xt, seed,
                       dict(n=n, p=p, B=B, s=s, sigma=sigma, kscale=kscale))


def uneven_batch(B, *, nmin=128, nmax=1024, ratio=4, sigma=1e-2, dtype="bf16",
                 seed=4, inst_seed_base=4000, name="uneven"):
    """B independent Gaussian instances with n_i uniform in [nmin, nmax],
    p_i = ratio * n_i, sparsity n_i // 20, +/-1 amplitudes, rho_i = s_i."""
    rng = np.random.default_rng(seed)
    ns = rng.integers(nmin, nmax + 1, size=B)
    out = []
    for i, n in enumerate(ns):
        n = int(n)
        p = ratio * n
        s = max(1, n // 20)
        out.append(gaussian_instance(n, p, s, amp="pm1", sigma=sigma,
                                     rho_scale=1.0, dtype=dtype,
                                     seed=inst_seed_base + i, name=f"{name}[{i}]"))
    return out


# ---------------------------------------------------------------------------
# The named workloads.  Sizes follow the problem families of the paper's
# Section 4 (Gaussian compressed sensing; ill-conditioned inverse problem).
# ---------------------------------------------------------------------------

def plain_small(seed=1, dtype="f64") -> Instance:
    """K 256x1024, N(0, 1/256), 20-sparse +/-1, sigma 1e-3, rho = ||x_true||_1."""
    return gaussian_instance(256, 1024, 20, amp="pm1", sigma=1e-3,
                             rho_scale=1.0, kscale=1 / 16, dtype=dtype,
                             seed=seed, name="gauss_256x1024")


def plain_large(seed=2, dtype="f32") -> Instance:
    """K 4096x16384, N(0, 1/4096), 400-sparse N(0,1), sigma 1e-2,
    rho = 0.9 ||x_true||_1."""
    return gaussian_instance(4096, 16384, 400, amp="normal", sigma=1e-2,
                             rho_scale=0.9, kscale=1 / 64, dtype=dtype,
                             seed=seed, name="gauss_4096x16384")


def plain_illcond(seed=3, dtype="f32", m=4096) -> Instance:
    """K = U diag(s) V^T, m x m, s geometric 1 .. 1e-4, 200-sparse +/-1,
    sigma 1e-3, rho = ||x_true||_1."""
    return illcond_instance(m, 200 if m >= 4096 else max(4, m // 20),
                            cond=1e4, sigma=1e-3, dtype=dtype, seed=seed,
                            name=f"illcond_{m}")


def shared_rhs(seed=5, dtype="bf16", n=2048, p=8192, B=256) -> SharedBatch:
    """One K 2048x8192 N(0, 1/2048), 256 right-hand sides, each n//20-sparse
    +/-1, sigma 1e-2, rho_b = ||x_true_b||_1."""
    return shared_batch(n, p, B, max(1, n // 20), amp="pm1", sigma=1e-2,
                        dtype=dtype, seed=seed, rhs_seed_base=5000,
                        name=f"shared_{n}x{p}x{B}")


def paper_gaussian(n=1848, p=8192, s=100, noise=0.02, seed=9, dtype="f32") -> Instance:
    """The Gaussian test problem of Section 4 in shape: K 1848x8192 with
    N(0,1) entries rescaled to spectral norm 1 (the norm from the largest
    eigenvalue of K K^T, FP64), x_true s-sparse with N(0,1) amplitudes (the
    paper gives no sparsity: 100), and noise of about 2 %:
    sigma = noise * ||K x_true|| / sqrt(n).  rho = ||x_true||_1 (the sweep sets
    its own radii)."""
    rng = np.random.default_rng(seed)
    K = rng.standard_normal((n, p))
    K /= np.sqrt(np.linalg.eigvalsh(K @ K.T)[-1])
    x_true = _sparse_signal(rng, p, s, "normal")
    Kx = K @ x_true
    sigma = noise * float(np.linalg.norm(Kx)) / np.sqrt(n)
    y = Kx + sigma * rng.standard_normal(n)
    Ks, ys = _store(K, y, dtype)
    return Instance(f"paper_gauss_{n}x{p}", dtype, Ks, ys, float(np.abs(x_true).sum()), x_true, seed,
                    dict(n=n, p=p, s=s, sigma=sigma, noise=noise))


@dataclass
class WarmStartSet:
    """Right-hand sides for one fixed K: Y (B x n, FP32), rho (B), and the
    sparse x_true of each row as (support B x s, signs B x s)."""
    Y: np.ndarray
    rho: np.ndarray
    support: np.ndarray
    signs: np.ndarray


def warm_start_matrix(n=1024, p=4096, seed=6):
    """The fixed K of the learned warm-start workload: N(0, 1/n) entries,
    rounded to FP32 (returned as FP32, the stored problem)."""
    rng = np.random.default_rng(seed)
    return (rng.standard_normal((n, p)) / np.sqrt(n)).astype(np.float32)


def warm_start_rhs(K32, B, s=50, sigma=1e-2, seed=0, chunk=1024) -> WarmStartSet:
    """B data vectors y = K x_true + noise for one stored K: x_true s-sparse
    with a uniformly random support and +/-1 amplitudes, noise N(0, sigma^2),
    rho = ||x_true||_1 = s.  Drawn in chunks from one PCG64 stream (support
    keys, signs, noise per chunk); y formed in FP64 and rounded to FP32."""
    n, p = K32.shape
    rng = np.random.default_rng(seed)
    K64 = K32.astype(np.float64)
    Y = np.empty((B, n), dtype=np.float32)
    sup = np.empty((B, s), dtype=np.int64)
    sg = np.empty((B, s), dtype=np.float64)
    for b0 in range(0, B, chunk):
        m = min(chunk, B - b0)
        keys = rng.random((m, p))
        sp = np.argpartition(keys, s, axis=1)[:, :s]
        sv = rng.choice(np.array([-1.0, 1.0]), size=(m, s))
        noise = sigma * rng.standard_normal((m, n))
        Xc = np.zeros((m, p))
        np.put_along_axis(Xc, sp, sv, axis=1)
        Yc = Xc @ K64.T + noise
        Y[b0:b0 + m] = Yc.astype(np.float32)
        sup[b0:b0 + m] = sp
        sg[b0:b0 + m] = sv
    return WarmStartSet(Y, np.full(B, float(s)), sup, sg)
