"""ctypes binding of libgpl1.so (the C ABI declared in include/gp_l1.h).

Argument marshalling only: torch tensors supply device memory (data_ptr())
and the current HIP stream; every step of the solver runs in the library's
kernels.  Importing this module does not load the library; the first call
does, and raises if it is missing (there is no fallback path).
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "lib", "libgpl1.so")

GP_F64, GP_F32, GP_BF16 = 0, 1, 2
GP_ISTA, GP_FISTA, GP_PSD = 0, 1, 2
GP_FUSED_PANELS = 13          # gp_opts.fused_cfg: the K pass over column panels
TRACE_FIELDS = 10             # GP_TRACE_FIELDS: doubles per record of gp_opts.trace
TRACE_COLUMNS = ("k", "f", "alpha", "lam", "backtracks", "tau", "rule", "mu", "nactive", "passes")
FOM_METHODS = {"ista": GP_ISTA, "fista": GP_FISTA, "psd": GP_PSD}
STATUS = {0: "ok_tol", 1: "stationary", 2: "max_iter", 3: "reached_target",
          4: "backtrack_limit", -1: "bad_argument", -2: "nonfinite",
          -3: "hip_error", -4: "out_of_memory", -5: "unsupported"}

SYMBOLS = ("gp_opts_default", "gp_create", "gp_destroy", "gp_last_error",
           "gp_l1_project", "gp_l1_solve", "gp_l1_solve_noalloc", "gp_l1_solve_batched_shared",
           "gp_l1_solve_batched_var", "gp_fom_solve", "gp_lista_create", "gp_lista_destroy",
           "gp_lista_init_from_K", "gp_lista_set_weights", "gp_lista_get_weights",
           "gp_lista_forward", "gp_lista_train_step", "gp_lista_gradients", "gp_lista_save",
           "gp_lista_load", "gp_lista_set_forward_planes")


class GPOpts(C.Structure):
    _fields_ = [("M", C.c_int32), ("theta", C.c_double), ("beta", C.c_double),
                ("alpha_min", C.c_double), ("alpha_max", C.c_double),
                ("tau1", C.c_double), ("M_alpha", C.c_int32),
                ("max_iter", C.c_int32), ("f_target", C.c_double),
                ("refresh_every", C.c_int32), ("backtrack_cap", C.c_int32),
                ("chunk", C.c_int32), ("fused_cfg", C.c_int32),
                ("fused_grid", C.c_int32), ("profile", C.c_int32),
                ("fused_interleave", C.c_int32), ("f_targets", C.POINTER(C.c_double)),
                ("x0_fallback", C.c_int32), ("graph", C.c_int32),
                ("batch_splitk", C.c_int32), ("batch_rows_t", C.c_int32),
                ("batch_cols_t", C.c_int32), ("var_item_rows", C.c_int32),
                ("batch_gemm_depth", C.c_int32), ("batch_gemm_tile", C.c_int32),
                ("lookahead", C.c_int32), ("var_wave_rows", C.c_int32),
                ("trace", C.POINTER(C.c_double)), ("trace_cap", C.c_int32)]


class GPResult(C.Structure):
    _fields_ = [("status", C.c_int32), ("iters", C.c_int32),
                ("backtracks", C.c_int32), ("projected_x0", C.c_int32),
                ("f", C.c_double), ("rel_change", C.c_double),
                ("lambda_est", C.c_double), ("l1norm", C.c_double),
                ("t_fused_ms", C.c_double), ("n_fused", C.c_int32),
                ("proj_passes", C.c_int32), ("x0_rejected", C.c_int32),
                ("reopened", C.c_int32), ("reserved_", C.c_int32)]

    def as_dict(self):
        d = {k: getattr(self, k) for k, _ in self._fields_}
        d["status_name"] = STATUS.get(self.status, str(self.status))
        return d


class GPInstance(C.Structure):
    _fields_ = [("K", C.c_void_p), ("y", C.c_void_p), ("x0", C.c_void_p),
                ("x_out", C.c_void_p), ("n", C.c_int64), ("p", C.c_int64),
                ("ldk", C.c_int64), ("rho", C.c_double)]


_lib = None


def load():
    """Load libgpl1.so and declare the signatures.  Raises if it is absent."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_0902_4424_amd.build`")
    lib = C.CDLL(LIB_PATH)
    vp, i64, dbl, i32 = C.c_void_p, C.c_int64, C.c_double, C.c_int
    lib.gp_opts_default.argtypes = [C.POINTER(GPOpts)]
    lib.gp_opts_default.restype = None
    lib.gp_create.argtypes = [C.POINTER(vp), i32]
    lib.gp_create.restype = i32
    lib.gp_destroy.argtypes = [vp]
    lib.gp_destroy.restype = i32
    lib.gp_last_error.argtypes = [vp]
    lib.gp_last_error.restype = C.c_char_p
    lib.gp_l1_project.argtypes = [vp, i32, vp, i64, dbl, vp, C.POINTER(dbl), vp]
    lib.gp_l1_project.restype = i32
    lib.gp_l1_solve.argtypes = [vp, i32, vp, i64, i64, i64, vp, dbl, vp, dbl, vp,
                                C.POINTER(GPOpts), C.POINTER(GPResult), vp]
    lib.gp_l1_solve.restype = i32
    lib.gp_l1_solve_noalloc.argtypes = lib.gp_l1_solve.argtypes
    lib.gp_l1_solve_noalloc.restype = i32
    lib.gp_l1_solve_batched_shared.argtypes = [
        vp, i32, vp, i64, i64, i64, vp, i64, i64, C.POINTER(dbl), vp, i64, dbl,
        vp, C.POINTER(GPOpts), C.POINTER(GPResult), vp]
    lib.gp_l1_solve_batched_shared.restype = i32
    lib.gp_l1_solve_batched_var.argtypes = [vp, i32, C.POINTER(GPInstance), i64,
                                            dbl, C.POINTER(GPOpts),
                                            C.POINTER(GPResult), vp]
    lib.gp_l1_solve_batched_var.restype = i32
    lib.gp_fom_solve.argtypes = [vp, C.c_int32, i32, vp, i64, i64, i64, vp, dbl, dbl, vp, C.c_int32, vp,
                                 C.POINTER(GPOpts), C.POINTER(GPResult), vp]
    lib.gp_fom_solve.restype = i32
    fp = C.c_void_p
    lib.gp_lista_create.argtypes = [vp, C.POINTER(vp), i64, i64, C.c_int32]
    lib.gp_lista_create.restype = i32
    lib.gp_lista_destroy.argtypes = [vp]
    lib.gp_lista_destroy.restype = i32
    lib.gp_lista_init_from_K.argtypes = [vp, fp, i64, dbl, dbl, vp]
    lib.gp_lista_init_from_K.restype = i32
    lib.gp_lista_set_weights.argtypes = [vp, fp, fp, fp, vp]
    lib.gp_lista_set_weights.restype = i32
    lib.gp_lista_get_weights.argtypes = [vp, fp, fp, fp, vp]
    lib.gp_lista_get_weights.restype = i32
    lib.gp_lista_forward.argtypes = [vp, fp, i64, i64, C.POINTER(dbl), fp, i64, vp]
    lib.gp_lista_forward.restype = i32
    lib.gp_lista_train_step.argtypes = [vp, fp, i64, fp, i64, i64, dbl, C.POINTER(dbl), vp]
    lib.gp_lista_train_step.restype = i32
    lib.gp_lista_gradients.argtypes = [vp, fp, i64, fp, i64, i64, fp, fp, fp, C.POINTER(dbl), vp]
    lib.gp_lista_gradients.restype = i32
    lib.gp_lista_set_forward_planes.argtypes = [vp, C.c_int32]
    lib.gp_lista_set_forward_planes.restype = i32
    lib.gp_lista_save.argtypes = [vp, C.c_char_p]
    lib.gp_lista_save.restype = i32
    lib.gp_lista_load.argtypes = [vp, C.c_char_p]
    lib.gp_lista_load.restype = i32
    _lib = lib
    return lib


def default_opts(**kw) -> GPOpts:
    o = GPOpts()
    load().gp_opts_default(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown option {k!r}")
        if k == "f_targets":
            if v is None:
                continue
            arr = (C.c_double * len(v))(*[float(t) for t in v])
            o._targets = arr                     # keeps the host array alive with the struct
            o.f_targets = C.cast(arr, C.POINTER(C.c_double))
            continue
        setattr(o, k, v)
    return o


def _check_targets(o: GPOpts, B: int):
    t = getattr(o, "_targets", None)
    if t is not None and len(t) != B:
        raise ValueError(f"f_targets holds {len(t)} values for {B} problems")


class GPError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{STATUS.get(code, code)}: {msg}")
        self.code = code


# ---------------------------------------------------------------------------
# torch helpers (torch is only a source of device memory and streams)
# ---------------------------------------------------------------------------
def _torch():
    import torch
    return torch


def _stream(stream=None):
    torch = _torch()
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def k_dtype(K) -> int:
    torch = _torch()
    if K.dtype == torch.float64:
        return GP_F64
    if K.dtype == torch.float32:
        return GP_F32
    if K.dtype in (torch.bfloat16, torch.int16, torch.uint16):
        return GP_BF16
    raise TypeError(f"unsupported K dtype {K.dtype}")


def vec_dtype(kdt: int):
    torch = _torch()
    return torch.float64 if kdt == GP_F64 else torch.float32


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else C.c_void_p(0)


def _check_dev(*ts):
    for t in ts:
        if t is not None and not t.is_cuda:
            raise ValueError("all tensors must live on the GPU")


class Handle:
    """Owns one gp_handle (device workspace).  Use as a context manager or
    keep it alive for many solves; the library reuses its workspace."""

    def __init__(self, device: int = 0):
        self.lib = load()
        h = C.c_void_p()
        rc = self.lib.gp_create(C.byref(h), int(device))
        if rc != 0:
            raise GPError(rc, f"gp_create(device={device}) failed")
        self.h = h
        self.device = device

    def close(self):
        if getattr(self, "h", None):
            self.lib.gp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def error(self) -> str:
        return self.lib.gp_last_error(self.h).decode()

    def _raise(self, rc):
        if rc < 0:
            raise GPError(rc, self.error())

    # -- projection -----------------------------------------------------
    def project(self, v, rho: float, out=None, want_mu=True, stream=None):
        torch = _torch()
        _check_dev(v)
        if v.dtype not in (torch.float64, torch.float32):
            raise TypeError("v must be float64 or float32")
        v = v.contiguous()
        out = torch.empty_like(v) if out is None else out
        mu = C.c_double(0.0)
        rc = self.lib.gp_l1_project(self.h, GP_F64 if v.dtype == torch.float64 else GP_F32,
                                    _ptr(v), v.numel(), float(rho), _ptr(out),
                                    C.byref(mu) if want_mu else None, _stream(stream))
        self._raise(rc)
        return out, (mu.value if want_mu else None)

    # -- one problem ----------------------------------------------------
    def solve(self, K, y, rho: float, x0=None, tol: float = 1e-10, out=None,
              opts: GPOpts | None = None, stream=None, **kw):
        """gp_l1_solve: the handle's workspace grows as needed.  `trace=N`
        keeps the device's last N per-update records (gp_opts.trace) in
        result["trace"], rows in update order, columns TRACE_COLUMNS."""
        return self._solve(self.lib.gp_l1_solve, K, y, rho, x0, tol, out, opts, stream, kw)

    def solve_noalloc(self, K, y, rho: float, x0=None, tol: float = 1e-10, out=None,
                      opts: GPOpts | None = None, stream=None, **kw):
        """gp_l1_solve_noalloc: the device's fixed scratch, no allocation in the
        library (`out` should be given by callers that cannot allocate)."""
        return self._solve(self.lib.gp_l1_solve_noalloc, K, y, rho, x0, tol, out, opts, stream, kw)

    def _solve(self, fn, K, y, rho, x0, tol, out, opts, stream, kw):
        torch = _torch()
        _check_dev(K, y, x0)
        kdt = k_dtype(K)
        vdt = vec_dtype(kdt)
        if K.dim() != 2 or K.stride(1) != 1:
            raise ValueError("K must be a row-major 2-D tensor")
        n, p = K.shape
        ldk = K.stride(0)
        if y.dtype != vdt or y.numel() != n or not y.is_contiguous():
            raise ValueError(f"y must be contiguous {vdt} of length {n}")
        if x0 is not None and (x0.dtype != vdt or x0.numel() != p or not x0.is_contiguous()):
            raise ValueError(f"x0 must be contiguous {vdt} of length {p}")
        if out is None:
            out = torch.empty(p, dtype=vdt, device=K.device)
        elif out.dtype != vdt or out.numel() != p or not out.is_contiguous() or not out.is_cuda:
            raise ValueError(f"out must be a contiguous device {vdt} tensor of length {p}")
        kw = dict(kw)
        cap = int(kw.pop("trace", 0) or 0)
        if cap < 0:
            raise ValueError("trace must be >= 0 (records kept)")
        o = opts if opts is not None else default_opts(**_tuned(kdt, n, p, kw))
        tbuf = None
        if cap:
            # the device ring of per-update records (gp_opts.trace)
            tbuf = torch.full((cap, TRACE_FIELDS), float("nan"), dtype=torch.float64, device=K.device)
            o.trace = C.cast(C.c_void_p(tbuf.data_ptr()), C.POINTER(C.c_double))
            o.trace_cap = cap
        res = GPResult()
        rc = fn(self.h, kdt, _ptr(K), n, p, ldk, _ptr(y), float(rho), _ptr(x0), float(tol),
                _ptr(out), C.byref(o), C.byref(res), _stream(stream))
        self._raise(rc)
        d = res.as_dict()
        if tbuf is not None:
            # the last min(iters, cap) records in update order
            it = d["iters"]
            rows = tbuf.cpu().numpy()
            keep = min(it, cap)
            order = [(k - 1) % cap for k in range(it - keep + 1, it + 1)]
            d["trace"] = rows[order] if keep else rows[:0]
        return out, d

    # -- the comparison methods of Section 2 ------------------------------
    def fom(self, method: str, K, y, param: float, iters: int, tau: float = 1.0, x0=None, out=None,
            opts: GPOpts | None = None, stream=None, **kw):
        """gp_fom_solve: `iters` iterations of ISTA / FISTA (param = lambda)
        or PSD (param = rho).  Returns (x, result dict)."""
        torch = _torch()
        if method not in FOM_METHODS:
            raise ValueError(f"method must be one of {sorted(FOM_METHODS)}")
        _check_dev(K, y, x0)
        kdt = k_dtype(K)
        vdt = vec_dtype(kdt)
        if K.dim() != 2 or K.stride(1) != 1:
            raise ValueError("K must be a row-major 2-D tensor")
        n, p = K.shape
        if y.dtype != vdt or y.numel() != n or not y.is_contiguous():
            raise ValueError(f"y must be contiguous {vdt} of length {n}")
        if x0 is not None and (x0.dtype != vdt or x0.numel() != p or not x0.is_contiguous()):
            raise ValueError(f"x0 must be contiguous {vdt} of length {p}")
        if out is None:
            out = torch.empty(p, dtype=vdt, device=K.device)
        elif out.dtype != vdt or out.numel() != p or not out.is_contiguous() or not out.is_cuda:
            raise ValueError(f"out must be a contiguous device {vdt} tensor of length {p}")
        o = opts if opts is not None else default_opts(**_tuned(kdt, n, p, kw))
        res = GPResult()
        rc = self.lib.gp_fom_solve(self.h, FOM_METHODS[method], kdt, _ptr(K), n, p, K.stride(0), _ptr(y),
                                   float(param), float(tau), _ptr(x0), int(iters), _ptr(out), C.byref(o),
                                   C.byref(res), _stream(stream))
        self._raise(rc)
        return out, res.as_dict()

    # -- many right-hand sides, one K -------------------------------------
    def solve_batched_shared(self, K, Y, rho, X0=None, tol: float = 1e-10, out=None,
                             opts: GPOpts | None = None, stream=None, **kw):
        torch = _torch()
        _check_dev(K, Y, X0)
        kdt = k_dtype(K)
        vdt = vec_dtype(kdt)
        if K.dim() != 2 or K.stride(1) != 1:
            raise ValueError("K must be a row-major 2-D tensor")
        n, p = K.shape
        if Y.dim() != 2 or Y.shape[1] != n or Y.dtype != vdt or Y.stride(1) != 1:
            raise ValueError(f"Y must be a row-major B x {n} {vdt} tensor")
        B = Y.shape[0]
        rho = [float(r) for r in rho]
        if len(rho) != B:
            raise ValueError(f"rho holds {len(rho)} radii for {B} right-hand sides")
        rho_arr = (C.c_double * B)(*rho)
        if X0 is not None and (tuple(X0.shape) != (B, p) or X0.dtype != vdt or X0.stride(1) != 1):
            raise ValueError("X0 must be a row-major B x p tensor of the vector dtype")
        if out is None:
            out = torch.empty(B, p, dtype=vdt, device=K.device)
        elif tuple(out.shape) != (B, p) or out.dtype != vdt or out.stride(1) != 1 or not out.is_cuda:
            raise ValueError(f"out must be a row-major device B x p tensor of dtype {vdt}")
        ldx = out.stride(0)
        if X0 is not None and X0.stride(0) != ldx:
            raise ValueError("X0 and out must share a leading dimension")
        o = opts if opts is not None else default_opts(**_tuned_shared(kdt, n, p, B, kw))
        _check_targets(o, B)
        res = (GPResult * B)()
        rc = self.lib.gp_l1_solve_batched_shared(
            self.h, kdt, _ptr(K), n, p, K.stride(0), _ptr(Y), Y.stride(0), B, rho_arr,
            _ptr(X0), ldx, float(tol), _ptr(out), C.byref(o), res, _stream(stream))
        self._raise(rc)
        return out, [r.as_dict() for r in res]

    # -- many independent problems of different sizes ---------------------
    def solve_batched_var(self, problems, tol: float = 1e-10, opts: GPOpts | None = None,
                          stream=None, **kw):
        """problems: list of (K, y, rho[, x0]) with device tensors of one K dtype.
        Returns (list of solution tensors, list of result dicts)."""
        torch = _torch()
        B = len(problems)
        if B == 0:
            return [], []
        kdt = k_dtype(problems[0][0])
        vdt = vec_dtype(kdt)
        inst = (GPInstance * B)()
        outs = []
        for b, prob in enumerate(problems):
            K, y, rho = prob[0], prob[1], prob[2]
            x0 = prob[3] if len(prob) > 3 else None
            _check_dev(K, y, x0)
            if k_dtype(K) != kdt or K.dim() != 2 or K.stride(1) != 1:
                raise ValueError("all K must share one dtype and be row-major")
            n, p = K.shape
            if y.dtype != vdt or y.numel() != n or not y.is_contiguous():
                raise ValueError(f"problem {b}: y must be contiguous {vdt} of length {n}")
            if x0 is not None and (x0.dtype != vdt or x0.numel() != p or not x0.is_contiguous()):
                raise ValueError(f"problem {b}: x0 must be contiguous {vdt} of length {p}")
            out = torch.empty(p, dtype=vdt, device=K.device)
            outs.append(out)
            inst[b] = GPInstance(K.data_ptr(), y.data_ptr(),
                                 x0.data_ptr() if x0 is not None else None,
                                 out.data_ptr(), n, p, K.stride(0), float(rho))
        o = opts if opts is not None else default_opts(**_tuned_var(kdt, kw))
        _check_targets(o, B)
        res = (GPResult * B)()
        rc = self.lib.gp_l1_solve_batched_var(self.h, kdt, inst, B, float(tol), C.byref(o),
                                              res, _stream(stream))
        self._raise(rc)
        return outs, [r.as_dict() for r in res]


class Lista:
    """Unrolled soft-thresholding network on the device (learned warm start).

    Weights: We (p x n), S (p x p), theta (layers), FP32 masters with Adam
    state, used as bf16 on the matrix cores.  Samples are rows: Y (B x n),
    X (B x p), float32 device tensors."""

    def __init__(self, handle: "Handle", n: int, p: int, layers: int = 8):
        self.H = handle
        self.lib = handle.lib
        self.n, self.p, self.layers = n, p, layers
        net = C.c_void_p()
        rc = self.lib.gp_lista_create(handle.h, C.byref(net), n, p, layers)
        handle._raise(rc)
        self.net = net

    def close(self):
        if getattr(self, "net", None):
            self.lib.gp_lista_destroy(self.net)
            self.net = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _f32(self, t, shape):
        torch = _torch()
        _check_dev(t)
        if t.dtype != torch.float32 or tuple(t.shape) != tuple(shape) or t.stride(-1) != 1:
            raise ValueError(f"expected a row-major float32 tensor of shape {shape}")
        return t

    def init_from_K(self, K, L: float, lam: float, stream=None):
        """ISTA start: We = K^T/L, S = I - K^T K/L, theta = lam/L (L >= ||K||^2)."""
        self._f32(K, (self.n, self.p))
        self.H._raise(self.lib.gp_lista_init_from_K(self.net, _ptr(K), K.stride(0), float(L),
                                                    float(lam), _stream(stream)))

    def set_weights(self, We, S, theta, stream=None):
        self._f32(We, (self.p, self.n))
        self._f32(S, (self.p, self.p))
        self._f32(theta, (self.layers,))
        self.H._raise(self.lib.gp_lista_set_weights(self.net, _ptr(We.contiguous()), _ptr(S.contiguous()),
                                                    _ptr(theta.contiguous()), _stream(stream)))

    def get_weights(self, stream=None):
        torch = _torch()
        dev = torch.device("cuda", self.H.device)
        We = torch.empty(self.p, self.n, dtype=torch.float32, device=dev)
        S = torch.empty(self.p, self.p, dtype=torch.float32, device=dev)
        th = torch.empty(self.layers, dtype=torch.float32, device=dev)
        self.H._raise(self.lib.gp_lista_get_weights(self.net, _ptr(We), _ptr(S), _ptr(th), _stream(stream)))
        return We, S, th

    def set_forward_planes(self, planes: int):
        """bf16 planes of the activations in forward(): 3 = FP32-accurate, 1 = bf16."""
        self.H._raise(self.lib.gp_lista_set_forward_planes(self.net, int(planes)))

    def save(self, path: str):
        self.H._raise(self.lib.gp_lista_save(self.net, os.fsencode(path)))

    def load(self, path: str):
        self.H._raise(self.lib.gp_lista_load(self.net, os.fsencode(path)))

    def forward(self, Y, rho=None, out=None, stream=None):
        """Network output for each row of Y; with rho (sequence of B radii)
        each row is projected onto its l1 ball."""
        torch = _torch()
        B = Y.shape[0]
        self._f32(Y, (B, self.n))
        out = torch.empty(B, self.p, dtype=torch.float32, device=Y.device) if out is None else out
        r = (C.c_double * B)(*[float(v) for v in rho]) if rho is not None else None
        self.H._raise(self.lib.gp_lista_forward(self.net, _ptr(Y), Y.stride(0), B, r, _ptr(out),
                                                out.stride(0), _stream(stream)))
        return out

    def train_step(self, Y, Xstar, lr: float, stream=None) -> float:
        B = Y.shape[0]
        self._f32(Y, (B, self.n))
        self._f32(Xstar, (B, self.p))
        loss = C.c_double(0.0)
        self.H._raise(self.lib.gp_lista_train_step(self.net, _ptr(Y), Y.stride(0), _ptr(Xstar),
                                                   Xstar.stride(0), B, float(lr), C.byref(loss),
                                                   _stream(stream)))
        return loss.value

    def gradients(self, Y, Xstar, stream=None):
        torch = _torch()
        B = Y.shape[0]
        self._f32(Y, (B, self.n))
        self._f32(Xstar, (B, self.p))
        dev = Y.device
        dWe = torch.empty(self.p, self.n, dtype=torch.float32, device=dev)
        dS = torch.empty(self.p, self.p, dtype=torch.float32, device=dev)
        dth = torch.empty(self.layers, dtype=torch.float32, device=dev)
        loss = C.c_double(0.0)
        self.H._raise(self.lib.gp_lista_gradients(self.net, _ptr(Y), Y.stride(0), _ptr(Xstar),
                                                  Xstar.stride(0), B, _ptr(dWe), _ptr(dS), _ptr(dth),
                                                  C.byref(loss), _stream(stream)))
        return loss.value, dWe, dS, dth


_DT_NAME = {GP_F64: "f64", GP_F32: "f32", GP_BF16: "bf16"}


def _tuned(kdt, n, p, kw):
    """Add the autotuned kernel shape for this problem shape (tuned.json),
    unless the caller chose one."""
    if "fused_cfg" in kw or "fused_grid" in kw:
        return kw
    from . import tune
    t = tune.lookup(_DT_NAME[kdt], n, p)
    if not t:
        return kw
    kw = dict(kw)
    kw["fused_cfg"] = int(t["fused_cfg"])
    kw["fused_grid"] = int(t["fused_grid"])
    kw["fused_interleave"] = int(t.get("fused_interleave", 0))
    return kw


_SHARED_KEYS = ("batch_splitk", "batch_rows_t", "batch_cols_t", "batch_gemm_depth", "batch_gemm_tile", "graph")


def _tuned_shared(kdt, n, p, B, kw):
    """Add the tuned shared-K batch options (tuned.json, nearest batch size)
    unless the caller chose any of them."""
    if any(k in kw for k in _SHARED_KEYS):
        return kw
    from . import tune
    t = tune.lookup_shared(_DT_NAME[kdt], n, p, B)
    if not t:
        return kw
    kw = dict(kw)
    for k in _SHARED_KEYS:
        if t.get(k):
            kw[k] = int(t[k])
    return kw


def _tuned_var(kdt, kw):
    """Add the tuned uneven-batch options unless the caller chose any."""
    if "var_item_rows" in kw or "graph" in kw or "var_wave_rows" in kw:
        return kw
    from . import tune
    t = tune.lookup_var(_DT_NAME[kdt])
    if not t:
        return kw
    kw = dict(kw)
    for k in ("var_item_rows", "graph", "var_wave_rows"):
        if t.get(k):
            kw[k] = int(t[k])
    return kw


def opts_for(K, **kw) -> GPOpts:
    """Options for solving with this K: the autotuned kernel shape of its
    (dtype, n, p) from tuned.json (unless given) plus the caller's options."""
    n, p = K.shape
    return default_opts(**_tuned(k_dtype(K), n, p, kw))


_default_handles = {}


def handle(device: int = 0) -> Handle:
    if device not in _default_handles:
        _default_handles[device] = Handle(device)
    return _default_handles[device]


def solve(K, y, rho, x0=None, tol=1e-10, **kw):
    """x, result = solve(K, y, rho): GPSS on min ||Kx-y||^2 s.t. ||x||_1 <= rho."""
    return handle(K.device.index or 0).solve(K, y, rho, x0=x0, tol=tol, **kw)


def project(v, rho, **kw):
    return handle(v.device.index or 0).project(v, rho, **kw)
