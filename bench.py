#!/usr/bin/env python3
"""Benchmark of the plain GPSS solver on MI355X.

Workload: Gaussian compressed sensing, K 4096 x 16384 stored in FP32
(N(0, 1/4096) entries, 256 MiB), x_true 400-sparse with N(0,1) amplitudes,
noise sigma = 1e-2, rho = 0.9 ||x_true||_1, x0 = 0, exactly 500 iterations
per solve (residual refreshed every 50).  One step = one full solve.
Inputs are resident in HBM before the timed region starts.

Prints ONE JSON line: iterations/s (whole job), the fused K/K^T kernel's
roofline (algorithmic bytes per launch / its HIP-event-timed duration inside
the timed solves), wall time to a 1e-6 relative objective gap, parity of the
returned x against the FP64 CPU oracle, and the oracle's own iteration rate
on this host as a reported CPU baseline.  Further legs, each reported in its
own key: BF16 storage of the same instance, 256 right-hand sides sharing a
bf16 K 2048x8192, 512 uneven problems, and the learned warm start (an
unrolled network trained on 100000 batched solutions for a fixed FP32 K
1024x4096, then 10000 fresh problems to a 1e-6 gap).
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
ITERS = 500
REFRESH = 50
# the fused launch of every 16th iteration is timed with HIP events inside the
# timed solves; a launch that stamps events leaves about 11 us of idle time
# around it on the GPU, so timing every launch would slow the iterations being
# measured (every 16th: under 1 us per iteration)
PROFILE_EVERY = 16
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "fused_traffic_gauss_4096x16384.json")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_0902_4424_amd", "csrc", f)
                  for f in ("gp_kernels.hpp", "gp_device.hpp")]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def kernel_hash():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per fused launch from committed rocprofv3 counter runs,
    valid only while the kernel sources are unchanged."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    if t.get("kernel_hash") != kernel_hash():
        return None
    return t.get("bytes_per_launch")


def host_info():
    """CPU model and core counts of the machine the bench runs on."""
    model = None
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"cpu_model": model, "logical_cpus": os.cpu_count(), "usable_cpus": usable,
            "blas_threads": blas_threads()}


def blas_threads():
    try:
        from threadpoolctl import threadpool_info
        n = [i.get("num_threads") for i in threadpool_info() if i.get("user_api") == "blas"]
        if n:
            return int(max(n))
    except Exception:
        pass
    return os.cpu_count()


def _gap(K64, y64, x, f_ref):
    import numpy as np
    r = K64 @ np.asarray(x, dtype=np.float64) - y64
    return (float(r @ r) - f_ref) / f_ref


def forms_legs(H, inst, np, torch, gpl1, instances, out, with_cpu):
    """BF16 storage of the same instance, and many right-hand sides sharing one
    bf16 K, each timed to a tight stop and checked in FP64 on the host (with
    the CPU leg: against the FP64 oracle, on the stored K and on the FP64 K
    before rounding)."""
    if with_cpu:
        from oracle import gpss
    res = {}
    dev = torch.device("cuda:0")
    # BF16 storage of the benchmark instance: parity against the oracle is
    # judged on the bf16 K (widened), the error against the FP32-stored K is
    # reported
    b16 = instances.plain_large(seed=2, dtype="bf16")
    Kb = torch.from_numpy(b16.K_store.view(np.int16)).to(dev)
    yb = torch.from_numpy(b16.y_store).to(dev)
    ob = gpl1.opts_for(Kb, max_iter=ITERS, refresh_every=REFRESH, profile=PROFILE_EVERY)
    H.solve(Kb, yb, b16.rho, tol=0.0, opts=ob)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xb, rb = H.solve(Kb, yb, b16.rho, tol=0.0, opts=ob)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    K64b = b16.K64
    y64 = b16.y64
    xbn = xb.cpu().double().numpy()
    fused_us = rb["t_fused_ms"] * 1e3 / max(rb["n_fused"], 1)
    alg = inst.n * inst.p * 2 + 8 * inst.p + 16 * inst.n + 4 * inst.p
    e = {"workload": "same instance, K stored bf16 (128 MiB)", "iterations": rb["iters"],
         "status": rb["status_name"], "seconds": round(tb, 5),
         "iterations_per_s": round(rb["iters"] / tb, 1),
         "fused_avg_us": round(fused_us, 2), "fused_GBps": round(alg / fused_us / 1e3, 1),
         "x_rel_diff_vs_fp32_storage_solution": float(
             np.linalg.norm(xbn - out.get("_x_fp32", xbn)) / max(np.linalg.norm(out.get("_x_fp32", xbn)), 1e-300))}
    if with_cpu:
        # parity: the FP64 oracle on the bf16-rounded K (the problem solved)
        ob16 = gpss(K64b, y64, b16.rho, tol=0.0, max_iter=100000)
        e["parity_vs_oracle_on_bf16_K"] = {
            "gap": _gap(K64b, y64, xbn, ob16["f"]),
            "x_rel_err": float(np.linalg.norm(xbn - ob16["x"]) / np.linalg.norm(ob16["x"]))}
        del K64b
        # storage error: the FP64 oracle on K before rounding (the same draw)
        f64i = instances.plain_large(seed=2, dtype="f64")
        K64f, y64f = f64i.K_store, f64i.y_store
        o64 = gpss(K64f, y64f, f64i.rho, tol=0.0, max_iter=100000)
        xf32 = out.get("_x_fp32")
        e["error_vs_oracle_on_fp64_K"] = {
            "bf16_storage": {"gap": _gap(K64f, y64f, xbn, o64["f"]),
                             "x_rel_err": float(np.linalg.norm(xbn - o64["x"]) / np.linalg.norm(o64["x"]))},
            "fp32_storage": {"gap": _gap(K64f, y64f, xf32, o64["f"]),
                             "x_rel_err": float(np.linalg.norm(xf32 - o64["x"]) / np.linalg.norm(o64["x"]))},
            "note": "stated, not thresholded: the stored K differs from the FP64 draw"}
        del K64f, f64i
    else:
        xl, _ = H.solve(Kb, yb, b16.rho, tol=0.0, max_iter=3000, refresh_every=REFRESH)
        f_ref = float(np.sum((K64b @ xl.cpu().double().numpy() - y64) ** 2))
        e["gap_vs_bf16_gpu_ref"] = _gap(K64b, y64, xbn, f_ref)
        del K64b
    res["bf16_storage"] = e
    log(f"bf16 storage: {rb['iters']} iterations in {tb * 1e3:.2f} ms; fused {fused_us:.1f} us")
    del Kb

    # many right-hand sides sharing one bf16 K (matrix-core GEMMs)
    batch = instances.shared_rhs(seed=5, dtype="bf16")
    Ks = torch.from_numpy(batch.K_store.view(np.int16)).to(dev)
    Y = torch.from_numpy(batch.Y_store).to(dev)
    kw = dict(tol=1e-10, max_iter=5000, refresh_every=REFRESH, chunk=8)
    H.solve_batched_shared(Ks, Y, batch.rho, **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    X, rs = H.solve_batched_shared(Ks, Y, batch.rho, **kw)
    torch.cuda.synchronize()
    tbat = time.perf_counter() - t0
    its = [r["iters"] for r in rs]
    # plain solver on 8 of the columns, one at a time
    t0 = time.perf_counter()
    pits = 0
    for b in range(8):
        _, r1 = H.solve(Ks, Y[b].contiguous(), float(batch.rho[b]), tol=1e-10, max_iter=5000,
                        refresh_every=REFRESH)
        pits += r1["iters"]
    torch.cuda.synchronize()
    tpl = (time.perf_counter() - t0) / 8
    K64 = batch.K64
    Xn = X.cpu().double().numpy()
    gaps, xerrs = [], []
    cols = list(range(0, batch.B, 32))
    if with_cpu:
        # parity of 8 sampled columns against the FP64 oracle on the bf16 K
        for b in cols:
            y = batch.Y_store[b].astype(np.float64)
            ob = gpss(K64, y, float(batch.rho[b]), tol=0.0, max_iter=100000)
            gaps.append(_gap(K64, y, Xn[b], ob["f"]))
            xerrs.append(float(np.linalg.norm(Xn[b] - ob["x"]) / np.linalg.norm(ob["x"])))
        ref_src = "FP64 oracle on the bf16 K, 8 sampled columns"
    else:
        Xl, _ = H.solve_batched_shared(Ks, Y, batch.rho, tol=0.0, max_iter=3000, refresh_every=REFRESH)
        Xln = Xl.cpu().double().numpy()
        for b in cols:
            y = batch.Y_store[b].astype(np.float64)
            gaps.append(_gap(K64, y, Xn[b], float(np.sum((K64 @ Xln[b] - y) ** 2))))
        ref_src = "3000-iteration batched GPU run, 8 sampled columns"
    e = {"workload": "K 2048x8192 bf16 shared by 256 right-hand sides (102-sparse +-1, sigma 1e-2), "
                     "each to relative change < 1e-10",
         "seconds": round(tbat, 5), "rhs_iterations_per_s": round(sum(its) / tbat, 1),
         "iterations_min_mean_max": [min(its), round(float(np.mean(its)), 1), max(its)],
         "statuses": sorted(set(r["status_name"] for r in rs)),
         "max_gap_sampled": max(gaps), "reference": ref_src,
         "plain_solver_seconds_per_column": round(tpl, 6),
         "plain_solver_seconds_for_256_extrapolated": round(256 * tpl, 4),
         "speedup_vs_plain_per_column": round(256 * tpl / tbat, 2)}
    if xerrs:
        e["max_x_rel_err_sampled"] = max(xerrs)
        # storage error of 2 columns against the oracle on the FP64 K before rounding
        f64b = instances.shared_rhs(seed=5, dtype="f64")
        serr = []
        for b in cols[:2]:
            y = f64b.Y_store[b].astype(np.float64)
            o64 = gpss(f64b.K_store, y, float(f64b.rho[b]), tol=0.0, max_iter=100000)
            serr.append({"column": b, "gap": _gap(f64b.K_store, y, Xn[b], o64["f"]),
                         "x_rel_err": float(np.linalg.norm(Xn[b] - o64["x"]) / np.linalg.norm(o64["x"]))})
        e["bf16_error_vs_oracle_on_fp64_K"] = serr
        del f64b
    res["batched_shared"] = e
    log(f"batched shared: {tbat * 1e3:.1f} ms for 256 columns; plain {tpl * 1e3:.2f} ms/column; "
        f"max sampled gap {max(gaps):.2e}")
    del Ks, Y, X, K64

    # 512 independent problems of uneven size in one lockstep batch
    t0 = time.time()
    insts = instances.uneven_batch(512, dtype="bf16", seed=4)
    probs = [(torch.from_numpy(i.K_store.view(np.int16)).to(dev), torch.from_numpy(i.y_store).to(dev),
              i.rho) for i in insts]
    log(f"uneven batch generated in {time.time() - t0:.1f}s")
    kv = dict(tol=1e-10, max_iter=5000, refresh_every=REFRESH)
    H.solve_batched_var(probs, **kv)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    Xv, rv = H.solve_batched_var(probs, **kv)
    torch.cuda.synchronize()
    tvar = time.perf_counter() - t0
    sample = list(range(0, 512, 32))
    t0 = time.perf_counter()
    for i in sample:
        H.solve(probs[i][0], probs[i][1], probs[i][2], **kv)
    torch.cuda.synchronize()
    tseq = (time.perf_counter() - t0) / len(sample)
    vgaps = []
    for i in sample[:6]:
        inst = insts[i]
        if with_cpu:
            fr = gpss(inst.K64, inst.y64, inst.rho, tol=0.0, max_iter=100000)["f"]
        else:
            xl, _ = H.solve(probs[i][0], probs[i][1], probs[i][2], tol=0.0, max_iter=3000,
                            refresh_every=REFRESH)
            fr = float(np.sum((inst.K64 @ xl.cpu().double().numpy() - inst.y64) ** 2))
        vgaps.append(_gap(inst.K64, inst.y64, Xv[i].cpu().double().numpy(), fr))
    vits = [r["iters"] for r in rv]
    kbytes = sum(2 * i.n * i.p for i in insts)
    # bytes of K the iterations that ran streamed (problem i reads its K once
    # per iteration), plus one K read per refresh
    streamed = sum(2 * i.n * i.p * (r["iters"] + r["iters"] // REFRESH) for i, r in zip(insts, rv))
    res["batched_uneven"] = {
        "workload": "512 problems, n uniform in [128,1024], p = 4n, K bf16 (%.2f GB), each to "
                    "relative change < 1e-10" % (kbytes / 1e9),
        "seconds": round(tvar, 5), "problem_iterations_per_s": round(sum(vits) / tvar, 1),
        "iterations_min_mean_max": [min(vits), round(float(np.mean(vits)), 1), max(vits)],
        "statuses": sorted(set(r["status_name"] for r in rv)),
        "max_gap_sampled_6": max(vgaps),
        "reference": "FP64 oracle" if with_cpu else "3000-iteration GPU runs",
        "plain_solver_seconds_per_problem": round(tseq, 6),
        "plain_solver_seconds_for_512_extrapolated": round(512 * tseq, 4),
        "speedup_vs_plain_per_problem": round(512 * tseq / tvar, 2),
        "K_GB_per_sweep": round(kbytes / 1e9, 3),
        "K_GBps_streamed": round(streamed / tvar / 1e9, 1)}
    log(f"batched uneven: {tvar * 1e3:.1f} ms for 512 problems; plain {tseq * 1e3:.2f} ms/problem")
    res["wide_fp32"] = wide_leg(H, np, torch, gpl1, instances)
    return res


def wide_leg(H, np, torch, gpl1, instances):
    """A problem past the fused kernel's width: 4096 x 65536 FP32 K (1 GiB),
    whose K pass runs over four column panels in two launches (K read twice per
    iteration); a fixed budget of iterations, the pass timed by its own events."""
    dev = torch.device("cuda:0")
    n, p = 4096, 65536
    t0 = time.time()
    inst = instances.gaussian_instance(n, p, 400, amp="normal", sigma=1e-2, rho_scale=0.9,
                                       kscale=1 / 64, dtype="f32", seed=23, name="gauss_4096x65536")
    log(f"{n}x{p} instance generated in {time.time() - t0:.1f}s")
    K = torch.from_numpy(inst.K_store).to(dev)
    y = torch.from_numpy(inst.y_store).to(dev)
    rho = inst.rho
    del inst
    iters = 60
    o = gpl1.opts_for(K, max_iter=iters, refresh_every=REFRESH, profile=PROFILE_EVERY)
    H.solve(K, y, rho, tol=0.0, opts=o)
    torch.cuda.synchronize()
    _, r = H.solve(K, y, rho, tol=0.0, opts=o)
    us = r["t_fused_ms"] * 1e3 / max(r["n_fused"], 1)
    o2 = gpl1.opts_for(K, max_iter=iters, refresh_every=REFRESH)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, r2 = H.solve(K, y, rho, tol=0.0, opts=o2)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kb = n * p * 4
    alg = 2 * kb + 8 * p + 16 * n + 4 * p
    res = {"workload": f"gauss {n}x{p} fp32 (1 GiB), 400-sparse N(0,1), rho = 0.9 ||x_true||_1, "
                       f"{iters} iterations",
           "panels": (p + 16383) // 16384, "iterations": r2["iters"], "status": r2["status_name"],
           "iterations_per_s": round(r2["iters"] / dt, 1), "pass_avg_us": round(us, 2),
           "K_read_GBps": round(2 * kb / us / 1e3, 1), "alg_bytes_per_pass": alg,
           "frac_of_8TBps": round(alg / us / 1e3 / HBM_PEAK_GBS, 4)}
    log(f"wide 4096x65536: pass {us:.1f} us ({2 * kb / us / 1e3:.0f} GB/s of K reads), "
        f"{r2['iters'] / dt:.0f} it/s")
    del K
    torch.cuda.empty_cache()
    return res


def configs_leg(H, np, torch, gpl1, instances, with_cpu):
    """The other single-instance workloads: K 256x1024 FP64 to a relative
    change of 1e-10, and the ill-conditioned 4096x4096 FP32 operator for 2000
    iterations; iteration rate, wall time to a 1e-6 gap, and the oracle beside
    them (timed on a bounded sample for the large one)."""
    dev = torch.device("cuda:0")
    out = {}

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            r = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps, r

    def fval(K64, y64, x):
        r = K64 @ x.cpu().double().numpy() - y64
        return float(r @ r)

    # ---- K 256x1024 FP64, tol 1e-10 ----
    a = instances.plain_small(seed=1, dtype="f64")
    K = torch.from_numpy(a.K_store).to(dev)
    y = torch.from_numpy(a.y_store).to(dev)
    ts, (x, r) = timed(lambda: H.solve(K, y, a.rho, tol=1e-10, max_iter=100000), 20)
    if with_cpu:
        from oracle import gpss
        ref = gpss(a.K64, a.y64, a.rho, tol=0.0, max_iter=100000)   # tight reference (stationary)
        ref_src = "FP64 oracle, stationary"
    else:
        xr, _ = H.solve(K, y, a.rho, tol=0.0, max_iter=100000)
        ref = {"x": xr.cpu().numpy(), "f": fval(a.K64, a.y64, xr)}
        ref_src = "GPU FP64 run to its stationarity floor (oracle leg off)"
    f_ref = ref["f"]
    tg, (xg, rg) = timed(lambda: H.solve(K, y, a.rho, tol=0.0, max_iter=100000,
                                         f_target=f_ref * (1 + 1e-6)), 20)
    e = {"workload": "K 256x1024 N(0,1/256) FP64, 20-sparse +-1, sigma 1e-3, rho = ||x_true||_1, "
                     "stop at relative change < 1e-10",
         "iterations": r["iters"], "status": r["status_name"], "seconds_per_solve": round(ts, 6),
         "iterations_per_s": round(r["iters"] / ts, 1),
         "gap_vs_oracle_tight": (fval(a.K64, a.y64, x) - f_ref) / f_ref,
         "x_rel_err_vs_oracle_tight": float(np.linalg.norm(x.cpu().numpy() - ref["x"]) /
                                            np.linalg.norm(ref["x"])),
         "reference": ref_src,
         "time_to_gap_1e-6": {"seconds": round(tg, 6), "iterations": rg["iters"], "status": rg["status_name"],
                              "gap": (fval(a.K64, a.y64, xg) - f_ref) / f_ref}}
    if with_cpu:
        t0 = time.perf_counter()
        n_it = nsol = 0
        while time.perf_counter() - t0 < 3.0:
            n_it += gpss(a.K64, a.y64, a.rho, tol=1e-10, max_iter=100000)["iters"]
            nsol += 1
        e["oracle_iterations_per_s"] = round(n_it / (time.perf_counter() - t0), 1)
        e["oracle_sample"] = f"{nsol} solves to relative change < 1e-10"
    out["fp64_256x1024"] = e
    log(f"256x1024 fp64: {r['iters']} it in {ts * 1e3:.2f} ms ({r['iters'] / ts:.0f} it/s); "
        f"gap {e['gap_vs_oracle_tight']:.1e}")

    # ---- ill-conditioned 4096x4096 FP32, 2000 iterations ----
    t0 = time.time()
    c = instances.plain_illcond(seed=3, dtype="f32")
    log(f"ill-conditioned instance generated in {time.time() - t0:.1f}s")
    K = torch.from_numpy(c.K_store).to(dev)
    y = torch.from_numpy(c.y_store).to(dev)
    o2000 = gpl1.opts_for(K, max_iter=2000, refresh_every=REFRESH)
    ts, (x, r) = timed(lambda: H.solve(K, y, c.rho, tol=0.0, opts=o2000), 3)
    K64, y64 = c.K64, c.y64
    if with_cpu:
        # f* and the oracle's own iterate after the same 2000-iteration budget
        t0 = time.perf_counter()
        o2 = gpss(K64, y64, c.rho, tol=0.0, max_iter=2000)
        tcpu = time.perf_counter() - t0
        oref = o2 if o2["status"] == "stationary" else gpss(K64, y64, c.rho, tol=0.0, max_iter=100000)
        f_ref = oref["f"]
        f_src = f"FP64 oracle, {oref['status']} after {oref['iters']} iterations"
    else:
        xl, _ = H.solve(K, y, c.rho, tol=0.0, max_iter=40000, refresh_every=REFRESH)
        f_ref = fval(K64, y64, xl)
        f_src = "40000-iteration GPU run, f recomputed in FP64 on the host (oracle leg off)"
    og = gpl1.opts_for(K, max_iter=40000, refresh_every=REFRESH, f_target=f_ref * (1 + 1e-6))
    tg, (xg, rg) = timed(lambda: H.solve(K, y, c.rho, tol=0.0, opts=og), 1)
    gg = (fval(K64, y64, xg) - f_ref) / f_ref
    e = {"workload": "K = U diag(s) V^T 4096x4096 FP32, s geometric 1..1e-4, 200-sparse +-1, "
                     "sigma 1e-3, rho = ||x_true||_1, 2000-iteration budget",
         "iterations": r["iters"], "status": r["status_name"], "seconds_per_solve": round(ts, 5),
         "iterations_per_s": round(r["iters"] / ts, 1),
         "gap_at_budget": (fval(K64, y64, x) - f_ref) / f_ref,
         "f_ref_source": f_src,
         "time_to_gap_1e-6": {"seconds": round(tg, 5), "iterations": rg["iters"], "status": rg["status_name"],
                              "gap": gg, "passed": bool(rg["status_name"] == "reached_target" and gg <= 1e-6)}}
    if with_cpu:
        e["oracle_gap_at_budget"] = (o2["f"] - f_ref) / f_ref
        e["oracle_status_at_budget"] = f"{o2['status']} after {o2['iters']} iterations"
        e["x_rel_err_vs_oracle"] = float(np.linalg.norm(x.cpu().double().numpy() - oref["x"]) /
                                         np.linalg.norm(oref["x"]))
        e["oracle_iterations_per_s"] = round(o2["iters"] / tcpu, 1)
        e["oracle_sample"] = f"{o2['iters']} iterations ({tcpu:.1f} s)"
    out["illcond_4096"] = e
    log(f"illcond 4096: {r['iters']} it in {ts * 1e3:.1f} ms ({r['iters'] / ts:.0f} it/s); gap at 2000 "
        f"{e['gap_at_budget']:.2e}; to 1e-6: {tg * 1e3:.1f} ms, {rg['iters']} it")
    return out


def mall_leg(H, np, torch, gpl1, instances):
    """The fused kernel on a K twice the size of the 256 MB Infinity Cache
    (8192 x 16384 FP32, 512 MiB), so that no part of K can stay cached between
    iterations: its rate is the HBM rate."""
    dev = torch.device("cuda:0")
    t0 = time.time()
    inst = instances.gaussian_instance(8192, 16384, 400, amp="normal", sigma=1e-2, rho_scale=0.9,
                                       kscale=1 / np.sqrt(8192), dtype="f32", seed=22, name="gauss_8192x16384")
    log(f"8192x16384 instance generated in {time.time() - t0:.1f}s")
    K = torch.from_numpy(inst.K_store).to(dev)
    y = torch.from_numpy(inst.y_store).to(dev)
    o = gpl1.opts_for(K, max_iter=ITERS, refresh_every=REFRESH, profile=PROFILE_EVERY)
    H.solve(K, y, inst.rho, tol=0.0, opts=o)
    torch.cuda.synchronize()
    _, r = H.solve(K, y, inst.rho, tol=0.0, opts=o)
    us = r["t_fused_ms"] * 1e3 / max(r["n_fused"], 1)
    alg = 8192 * 16384 * 4 + 8 * 16384 + 16 * 8192 + 4 * 16384
    res = {"workload": "gauss 8192x16384 fp32 (512 MiB, twice the Infinity Cache)",
           "fused_avg_us": round(us, 2), "fused_GBps": round(alg / us / 1e3, 1),
           "frac_of_8TBps": round(alg / us / 1e3 / HBM_PEAK_GBS, 4), "timed_launches": r["n_fused"]}
    log(f"512 MiB K: fused {us:.1f} us -> {alg / us / 1e3:.0f} GB/s")
    return res


def lasso_references(K64, y64, lams):
    import numpy as np
    """Exact minimisers x_bar(lambda) of the penalised functional (1),
    ||K x - y||^2 + 2 lambda ||x||_1, at each lambda: the homotopy (LARS-lasso)
    path of the stored problem in FP64, linear between its breakpoints (the
    path is piecewise linear in lambda, Section 1).  scikit-learn scales the
    functional by 1/(2n), so its alpha is lambda / n."""
    from sklearn.linear_model import lars_path
    n = K64.shape[0]
    lams = np.asarray(lams, dtype=np.float64)
    alphas, _, coefs = lars_path(K64, y64, method="lasso", alpha_min=float(lams.min()) / n * 0.999,
                                 max_iter=50 * n, return_path=True)
    out = []
    for lam in lams:
        a = lam / n
        k = int(np.searchsorted(-alphas, -a))          # alphas decrease
        if k == 0:
            out.append(coefs[:, 0].copy())
            continue
        k = min(k, len(alphas) - 1)
        a0, a1 = alphas[k - 1], alphas[k]
        w = 0.0 if a0 == a1 else (a0 - a) / (a0 - a1)
        out.append((1.0 - w) * coefs[:, k - 1] + w * coefs[:, k])
    return np.array(out)


def isochrone_leg(H, np, torch, gpl1, instances, nlam=50, lrange=9.0, budgets_ms=(0.5, 1.0, 2.0, 4.0, 8.0)):
    """The experiment of Section 4 on the Gaussian operator, in shape: K
    1848x8192 (spectral norm 1, FP32 storage), 100-sparse signal, about 2 %
    noise; lambda_j = lambda_max 2^(-L (j+1)/nlam), rho_j = ||x_bar(lambda_j)||_1
    with x_bar from the homotopy path.  L = 9: near lambda_max / 2^9 the
    solution has about a thousand nonzeros and the FP64 homotopy path ends at
    a degeneracy, so no exact reference exists below it; grid points whose
    reference misses the KKT relation ||K^T (y - K x_bar)||_inf = lambda by
    more than 1e-9 (relative) are dropped and counted.  Two measurements:
      * the rho sweep: one batched GPSS call with the nlam radii as columns
        sharing K and y, against the same nlam plain solves one after another;
      * approximation isochrones: GPSS, ISTA, FISTA (lambda_j, step 1 as in
        the paper, ||K|| = 1) and PSD (rho_j), one problem at a time, each run
        for the iterations that fit a wall-time budget on this GPU (its own
        measured time per iteration); e = ||x - x_bar|| / ||x_bar|| per
        (method, budget, lambda_j)."""
    dev = torch.device("cuda:0")
    t0 = time.time()
    inst = instances.paper_gaussian()
    K64, y64 = inst.K64, inst.y64
    lam_max = float(np.abs(K64.T @ y64).max())
    l2 = lrange * (np.arange(nlam) + 1) / nlam
    lams = lam_max * 2.0 ** (-l2)
    tl = time.time()
    xbar = lasso_references(K64, y64, lams)
    t_lars = time.time() - tl
    kkts = np.array([abs(float(np.abs(K64.T @ (y64 - K64 @ xb)).max()) - lam) / lam for xb, lam in zip(xbar, lams)])
    keep = np.nonzero(kkts <= 1e-9)[0]
    dropped = nlam - len(keep)
    lams, l2, xbar = lams[keep], l2[keep], xbar[keep]
    nlam = len(keep)
    kkt = float(kkts[keep].max())
    rhos = np.abs(xbar).sum(axis=1)
    log(f"isochrones: instance and homotopy references in {time.time() - t0:.1f}s (LARS {t_lars:.1f}s); "
        f"{nlam} grid points kept (max KKT rel err {kkt:.1e}), {dropped} dropped")
    K = torch.from_numpy(inst.K_store).to(dev)
    y = torch.from_numpy(inst.y_store).to(dev)
    nx = np.linalg.norm(xbar, axis=1)

    def err(xt, j):
        return float(np.linalg.norm(xt.cpu().double().numpy() - xbar[j]) / nx[j])

    # ---- the rho sweep as one batched call -------------------------------
    Y = y.unsqueeze(0).repeat(nlam, 1).contiguous()
    kw = dict(tol=1e-10, max_iter=5000, refresh_every=REFRESH)
    H.solve_batched_shared(K, Y, rhos, **kw)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    X, rs = H.solve_batched_shared(K, Y, rhos, **kw)
    torch.cuda.synchronize()
    t_batch = time.perf_counter() - t1
    e_batch = [err(X[j], j) for j in range(nlam)]
    t1 = time.perf_counter()
    e_seq = []
    for j in range(nlam):
        xs, _ = H.solve(K, y, float(rhos[j]), **kw)
        e_seq.append(xs)
    torch.cuda.synchronize()
    t_seq = time.perf_counter() - t1
    e_seq = [err(e_seq[j], j) for j in range(nlam)]
    sweep = {"batched_seconds": round(t_batch, 5), "sequential_plain_seconds": round(t_seq, 5),
             "speedup": round(t_seq / t_batch, 2),
             "iterations_min_mean_max": [min(r["iters"] for r in rs), round(float(np.mean([r["iters"] for r in rs])), 1),
                                         max(r["iters"] for r in rs)],
             "max_e_batched": max(e_batch), "max_e_sequential": max(e_seq)}
    log(f"  rho sweep: batched {t_batch * 1e3:.1f} ms, sequential {t_seq * 1e3:.1f} ms; "
        f"max e {max(e_batch):.1e} / {max(e_seq):.1e}")

    # ---- isochrones: iterations per budget from each method's own rate -----
    jm = nlam // 2

    def run(method, j, k):
        if method == "gpss":
            return H.solve(K, y, float(rhos[j]), tol=0.0, max_iter=max(k, 1), refresh_every=REFRESH)
        if method == "psd":
            return H.fom("psd", K, y, float(rhos[j]), k)
        return H.fom(method, K, y, float(lams[j]), k, tau=1.0)

    per_it = {}
    for m in ("gpss", "ista", "fista", "psd"):
        run(m, jm, 50)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        _, r = run(m, jm, 400)
        torch.cuda.synchronize()
        per_it[m] = (time.perf_counter() - t1) / max(r["iters"], 1)
    table = {}
    for m in ("gpss", "ista", "fista", "psd"):
        table[m] = {}
        for b in budgets_ms:
            k = max(1, int(b * 1e-3 / per_it[m]))
            table[m][str(b)] = {"iterations": k,
                                "e": [float("%.3e" % err(run(m, j, k)[0], j)) for j in range(nlam)]}
    # the method with the smallest e at each (budget, lambda)
    best = {str(b): [min(table, key=lambda m: table[m][str(b)]["e"][j]) for j in range(nlam)] for b in budgets_ms}
    wins = {str(b): {m: best[str(b)].count(m) for m in table} for b in budgets_ms}
    log(f"  per-iteration us: " + ", ".join(f"{m} {v * 1e6:.1f}" for m, v in per_it.items()))
    for b in budgets_ms:
        log(f"  budget {b} ms: lowest e per lambda -> {wins[str(b)]}")
    return {"workload": "Gaussian K 1848x8192, spectral norm 1, fp32; 100-sparse N(0,1) signal, 2 % noise; "
                        f"lambda grid log2(lambda_max/lambda) = {lrange:g} (j+1)/50, j < 50",
            "reference": f"homotopy (LARS-lasso) path in FP64, linear between breakpoints; max KKT rel err {kkt:.1e}; "
                         f"{dropped} grid points without an exact reference dropped",
            "log2_lambda_max_over_lambda": [round(v, 3) for v in l2],
            "rho": [round(float(v), 6) for v in rhos],
            "rho_sweep": sweep,
            "per_iteration_us": {m: round(v * 1e6, 2) for m, v in per_it.items()},
            "budgets_ms": list(budgets_ms), "e": table, "lowest_e_count": wins}


def ingest_counters(fetch_dir, write_dir):
    """Write the fused kernel's measured HBM bytes per live launch from two
    rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE; KiB per dispatch) of
    `bench.py --steps 1 --warmup 0 --no-gap --no-cpu-baseline --no-forms
    --no-learned --no-configs --no-mall --no-cold --no-isochrone --calibrate-copy`.  Each counter is scaled by what it reads for
    the 256 MiB reference copy; launches below half the largest fetch (those
    that exited at once after the solve stopped) are left out."""
    import csv
    import glob
    from collections import defaultdict

    def per_dispatch(d, counter):
        path = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)[0]
        val, name = defaultdict(float), {}
        with open(path) as fh:
            for r in csv.DictReader(fh):
                if r["Counter_Name"] == counter:
                    k = int(r["Dispatch_Id"])
                    val[k] += float(r["Counter_Value"])
                    name[k] = r["Kernel_Name"]
        return val, name

    fv, fname = per_dispatch(fetch_dir, "FETCH_SIZE")
    wv, wname = per_dispatch(write_dir, "WRITE_SIZE")
    copy_f = max(v for k, v in fv.items() if "copyBuffer" in fname[k])
    copy_w = max(v for k, v in wv.items() if "copyBuffer" in wname[k])
    ref_kib = 256 * 1024
    fs, ws = ref_kib / copy_f, ref_kib / copy_w
    fused_f = [v for k, v in fv.items() if "k_fused" in fname[k]]
    fused_w = [v for k, v in wv.items() if "k_fused" in wname[k]]
    kname = next(fname[k] for k in fv if "k_fused" in fname[k])
    if len({fname[k] for k in fv if "k_fused" in fname[k]}) != 1:
        raise SystemExit("counter runs hold more than one fused-kernel shape: profile the main leg only "
                         "(--no-forms --no-learned --no-configs --no-mall --no-cold --no-isochrone)")
    lf = [v for v in fused_f if v > 0.5 * max(fused_f)]
    lw = sorted(fused_w)[-len(lf):]
    fb = sum(lf) / len(lf) * 1024 * fs
    wb = sum(lw) / len(lw) * 1024 * ws
    t = {"kernel": kname.split("(")[0].replace("void ", ""), "workload": "gauss 4096x16384 fp32",
         "kernel_hash": kernel_hash(), "fetch_scale": fs, "write_scale": ws, "live_launches": len(lf),
         "fetch_bytes_per_launch": int(fb), "write_bytes_per_launch": int(wb),
         "bytes_per_launch": int(fb + wb), "algorithmic_bytes_per_launch": 4096 * 16384 * 4 + 8 * 16384 +
         16 * 4096 + 4 * 16384,
         "command": "cd /tmp && export TMPDIR=/tmp && timeout -s KILL 120 rocprofv3 --pmc "
                    "<FETCH_SIZE|WRITE_SIZE> -f csv -d <out> -o run -- python3 <repo>/bench.py --steps 1 "
                    "--warmup 0 --no-gap --no-cpu-baseline --no-forms --no-learned --no-configs --no-mall --no-cold "
                    "--no-isochrone --calibrate-copy"}
    with open(TRAFFIC_FILE, "w") as fh:
        json.dump(t, fh, indent=1)
        fh.write("\n")
    print(json.dumps(t, indent=1))


def learned_leg(H, np, torch, gpl1, instances, ntrain, neval, epochs, batch=256, lr=3e-4,
                layers=8, oracle_check=0):
    """Learned warm start + batched GP refinement on one fixed FP32 K 1024x4096.

    Training pairs (y, x*) come from the batched shared-K solver; the unrolled
    network is trained by the library's own kernels; on fresh y, three ways of
    reaching a 1e-6 relative objective gap are timed: the plain solver one
    problem at a time (timed on a sample), the batched solver from x0 = 0, and
    the batched solver from the network's projected output."""
    dev = torch.device("cuda:0")
    res = {}
    K32 = instances.warm_start_matrix()
    n, p = K32.shape
    K64 = K32.astype(np.float64)
    Kd = torch.from_numpy(K32).to(dev)
    t0 = time.time()
    tr = instances.warm_start_rhs(K32, ntrain, seed=61)
    ev = instances.warm_start_rhs(K32, neval, seed=62)
    log(f"learned leg: {ntrain} training and {neval} evaluation right-hand sides drawn "
        f"({time.time() - t0:.1f}s)")
    CH = 10000
    # batched calls poll every 8 iterations: finished problems leave the launches
    kw = dict(refresh_every=REFRESH, chunk=8)

    # 1. training targets from the batched solver (matrix cores, FP32 K as bf16 planes)
    Ytr = torch.from_numpy(tr.Y).to(dev)
    Xstar = torch.empty(ntrain, p, dtype=torch.float32, device=dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    its = []
    for b0 in range(0, ntrain, CH):
        m = min(CH, ntrain - b0)
        X, r = H.solve_batched_shared(Kd, Ytr[b0:b0 + m], tr.rho[b0:b0 + m], tol=1e-9,
                                      max_iter=3000, out=Xstar[b0:b0 + m], **kw)
        its += [q["iters"] for q in r]
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t0
    log(f"  targets: {ntrain} solves in {t_gen:.2f}s (mean {np.mean(its):.1f} iterations)")

    # 2. training
    Lk = float(np.linalg.norm(K64, 2) ** 2) * 1.01
    lam = 0.1 * float(np.median(np.abs(tr.Y[:256].astype(np.float64) @ K64).max(axis=1)))
    net = gpl1.Lista(H, n, p, layers)
    net.init_from_K(Kd, Lk, lam)
    net.set_forward_planes(1)            # bf16 activations suffice for a warm start
    # each pair also enters negated: the solution of (2) is odd in y, so
    # (-y, -x*) is an exact pair of the same problem
    Ytr2 = torch.cat([Ytr, -Ytr]).contiguous()
    Xs2 = torch.cat([Xstar, -Xstar]).contiguous()
    n2 = Ytr2.shape[0]
    gen = torch.Generator(device="cpu").manual_seed(7)
    steps = 0
    losses = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for ep in range(epochs):
        perm = torch.randperm(n2, generator=gen).to(dev)
        el = []
        lr_ep = lr * (0.5 ** (ep // max(1, epochs // 3)))
        for b0 in range(0, n2 - batch + 1, batch):
            idx = perm[b0:b0 + batch]
            el.append(net.train_step(Ytr2[idx].contiguous(), Xs2[idx].contiguous(), lr_ep))
            steps += 1
        losses.append(float(np.mean(el)))
        log(f"  epoch {ep}: mean loss {losses[-1]:.4e} (lr {lr_ep:.1e})")
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0

    # 3. evaluation on fresh right-hand sides
    del Ytr, Xstar, Ytr2, Xs2
    Yev = torch.from_numpy(ev.Y).to(dev)
    # reference optimum of each problem: a long batched run, f recomputed in FP64 on the host
    f_ref = np.empty(neval)
    for b0 in range(0, neval, CH):
        m = min(CH, neval - b0)
        Xl, _ = H.solve_batched_shared(Kd, Yev[b0:b0 + m], ev.rho[b0:b0 + m], tol=0.0,
                                       max_iter=3000, **kw)
        R = Xl.cpu().double().numpy() @ K64.T - ev.Y[b0:b0 + m].astype(np.float64)
        f_ref[b0:b0 + m] = np.einsum("ij,ij->i", R, R)
    targets = f_ref * (1 + 1e-6)
    # the FP64 oracle, run to stationarity on a random subset, checks these optima
    oracle_f = None
    if oracle_check:
        from oracle import gpss
        pick = np.random.default_rng(63).choice(neval, size=min(oracle_check, neval), replace=False)
        t0 = time.perf_counter()
        rel = [(gpss(K64, ev.Y[b].astype(np.float64), float(ev.rho[b]), tol=0.0, max_iter=100000)["f"]
                - f_ref[b]) / f_ref[b] for b in pick]
        oracle_f = {"instances": len(pick), "max_rel_diff_f_ref_vs_oracle": float(np.max(np.abs(rel))),
                    "seconds": round(time.perf_counter() - t0, 1)}
        log(f"  oracle check of f_ref on {len(pick)} problems: max rel diff {np.max(np.abs(rel)):.2e}")

    def host_gaps(X, b0, m):
        R = X.cpu().double().numpy() @ K64.T - ev.Y[b0:b0 + m].astype(np.float64)
        return (np.einsum("ij,ij->i", R, R) - f_ref[b0:b0 + m]) / f_ref[b0:b0 + m]

    def batched(warm):
        its, gaps, reached, x0err, kept = [], [], 0, [], 0
        stats = {}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        outs = []
        for b0 in range(0, neval, CH):
            m = min(CH, neval - b0)
            Yc = Yev[b0:b0 + m]
            # x0 = P_Omega(net(y)); the solver keeps 0 where x0 is no better
            X0 = net.forward(Yc, rho=ev.rho[b0:b0 + m]) if warm else None
            X, r = H.solve_batched_shared(Kd, Yc, ev.rho[b0:b0 + m], X0=X0, tol=0.0, x0_fallback=1,
                                          max_iter=20000, f_targets=targets[b0:b0 + m], **kw)
            outs.append((b0, m, X, X0, r))
        torch.cuda.synchronize()
        t = time.perf_counter() - t0
        for b0, m, X, X0, r in outs:
            its += [q["iters"] for q in r]
            kept += sum(q["x0_rejected"] == 0 for q in r) if X0 is not None else 0
            reached += sum(q["status_name"] == "reached_target" for q in r)
            for q in r:
                stats[q["status_name"]] = stats.get(q["status_name"], 0) + 1
            gaps += list(host_gaps(X, b0, m))
            if X0 is not None:
                ref = X.cpu().double().numpy()
                x0 = X0.cpu().double().numpy()
                x0err += list(np.linalg.norm(x0 - ref, axis=1) / np.linalg.norm(ref, axis=1))
        return t, its, gaps, reached, x0err, kept, stats

    batched(False)                       # warm-up of the code paths
    batched(True)
    tc, itc, gc, rc_, _, _, stc = batched(False)
    tw, itw, gw, rw, x0err, kept, stw = batched(True)
    # the network's share of the learned time: projected forward passes alone
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for b0 in range(0, neval, CH):
        m = min(CH, neval - b0)
        net.forward(Yev[b0:b0 + m], rho=ev.rho[b0:b0 + m])
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    # generalisation: the raw network output against the solutions, first chunk
    m0 = min(CH, neval)
    Xs0, _ = H.solve_batched_shared(Kd, Yev[:m0], ev.rho[:m0], tol=0.0, f_targets=targets[:m0],
                                    max_iter=20000, **kw)
    Xr = net.forward(Yev[:m0]).cpu().double().numpy()
    Xs0 = Xs0.cpu().double().numpy()
    raw_err = float(np.mean(np.linalg.norm(Xr - Xs0, axis=1) / np.linalg.norm(Xs0, axis=1)))
    Ytr0 = torch.from_numpy(tr.Y[:m0]).to(dev)
    Xt0, _ = H.solve_batched_shared(Kd, Ytr0, tr.rho[:m0], tol=1e-9, max_iter=3000, **kw)
    Xt0 = Xt0.cpu().double().numpy()
    Xrt = net.forward(Ytr0).cpu().double().numpy()
    raw_err_train = float(np.mean(np.linalg.norm(Xrt - Xt0, axis=1) / np.linalg.norm(Xt0, axis=1)))
    # plain solver, one problem at a time, on a sample
    sample = list(range(0, neval, max(1, neval // 32)))[:32]
    # (its own default host-poll interval: one poll per 64 iterations)
    H.solve(Kd, Yev[0], float(ev.rho[0]), tol=0.0, f_target=float(targets[0]), max_iter=20000,
            refresh_every=REFRESH)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pits = []
    for b in sample:
        _, r = H.solve(Kd, Yev[b], float(ev.rho[b]), tol=0.0, f_target=float(targets[b]),
                       max_iter=20000, refresh_every=REFRESH)
        pits.append(r["iters"])
    torch.cuda.synchronize()
    tp = (time.perf_counter() - t0) / len(sample)
    t_plain_all = tp * neval
    res = {
        "workload": f"fixed Gaussian K {n}x{p} fp32; {layers}-layer unrolled network (bf16 weights "
                    f"on the matrix cores); {ntrain} training pairs from the batched solver (each also "
                    "negated), "
                    f"{epochs} epochs of batch {batch}; {neval} fresh y (50-sparse +-1, sigma 1e-2, "
                    "rho = ||x_true||_1), each run to f <= 1.000001 f_ref",
        "f_ref_source": "3000-iteration batched GPU run per problem, f recomputed in FP64 on the host "
                        "(checked against the FP64 oracle on a sample, f_ref_oracle_check)",
        "target_check": "a stop at the target is confirmed on the device with f recomputed in double "
                        "from the returned x, else the problem iterates on",
        "f_ref_oracle_check": oracle_f,
        "training": {"target_generation_s": round(t_gen, 3), "train_s": round(t_train, 3),
                     "steps": steps, "loss_per_epoch": [round(v, 6) for v in losses]},
        "plain_solver": {"seconds_per_problem": round(tp, 6), "sample": len(sample),
                         "iterations_mean": round(float(np.mean(pits)), 1),
                         "seconds_all_extrapolated": round(t_plain_all, 4)},
        "batched_cold": {"seconds": round(tc, 4), "iterations_mean_max": [round(float(np.mean(itc)), 1), max(itc)],
                         "statuses": stc, "reached_target": int(rc_), "max_gap_host": float(max(gc)),
                         "host_confirmed_le_1e-6": int(np.sum(np.asarray(gc) <= 1e-6)),
                         "passed": bool(rc_ == neval and max(gc) <= 1e-6)},
        "batched_learned": {"seconds": round(tw, 4), "network_forward_seconds": round(t_fwd, 4),
                            "iterations_mean_max": [round(float(np.mean(itw)), 1), max(itw)],
                            "statuses": stw, "reached_target": int(rw), "max_gap_host": float(max(gw)),
                            "host_confirmed_le_1e-6": int(np.sum(np.asarray(gw) <= 1e-6)),
                            "passed": bool(rw == neval and max(gw) <= 1e-6),
                            "warm_start_kept": kept,
                            "x0_rel_err_mean": round(float(np.mean(x0err)), 4),
                            "net_raw_rel_err_fresh": round(raw_err, 4),
                            "net_raw_rel_err_training": round(raw_err_train, 4)},
        "speedup_learned_vs_plain": round(t_plain_all / tw, 2),
        "speedup_learned_vs_batched_cold": round(tc / tw, 3),
    }
    log(f"  plain {tp * 1e3:.2f} ms/problem ({np.mean(pits):.1f} it) -> {t_plain_all:.2f}s for {neval}; "
        f"batched cold {tc:.3f}s ({np.mean(itc):.1f} it, max {max(itc)}); learned {tw:.3f}s "
        f"({np.mean(itw):.1f} it, max {max(itw)}, x0 err {np.mean(x0err):.3f}, kept {kept}, "
        f"network {t_fwd * 1e3:.1f} ms); "
        f"raw net error fresh {raw_err:.3f} / training {raw_err_train:.3f}")
    net.close()
    return res


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-gap", action="store_true", help="skip the time-to-gap leg")
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the BF16-storage and batched legs")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned warm-start leg")
    ap.add_argument("--no-configs", action="store_true",
                    help="skip the FP64 256x1024 and ill-conditioned 4096x4096 legs")
    ap.add_argument("--no-mall", action="store_true", help="skip the 512 MiB K check")
    ap.add_argument("--no-cold", action="store_true",
                    help="skip the solves timed after an Infinity Cache flush")
    ap.add_argument("--no-isochrone", action="store_true",
                    help="skip the rho sweep and approximation isochrones on the 1848x8192 operator")
    ap.add_argument("--learned-train", type=int, default=100000,
                    help="training pairs of the learned leg")
    ap.add_argument("--learned-eval", type=int, default=10000,
                    help="fresh right-hand sides of the learned leg")
    ap.add_argument("--learned-epochs", type=int, default=6)
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="first run one plain 256 MiB device-to-device copy (a reference "
                         "kernel of known traffic for hardware-counter scaling)")
    ap.add_argument("--ingest-counters", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="write the fused kernel's measured traffic from two rocprofv3 --pmc "
                         "output folders and exit (no GPU needed)")
    args = ap.parse_args()
    if args.ingest_counters:
        ingest_counters(*args.ingest_counters)
        return
    if args.gpus != 1:
        print(f"bench.py: this solver runs on one GPU; --gpus {args.gpus} is not supported "
              "(independent problems shard across GPUs without exchange, see the design notes)",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_0902_4424_amd import gpl1, instances

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    t = time.time()
    inst = instances.plain_large(seed=2, dtype="f32")
    n, p = inst.n, inst.p
    log(f"instance {inst.name}: n={n} p={p} rho={inst.rho:.4f} ({time.time() - t:.1f}s)")
    K = torch.from_numpy(inst.K_store).to(dev)
    y = torch.from_numpy(inst.y_store).to(dev)
    torch.cuda.synchronize()
    H = gpl1.Handle(0)
    opts = gpl1.opts_for(K, max_iter=ITERS, refresh_every=REFRESH, profile=PROFILE_EVERY)
    if args.calibrate_copy:
        src = torch.ones(64 << 20, dtype=torch.float32, device=dev)   # 256 MiB
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: 256 MiB read + 256 MiB written")
        del src, dst

    for i in range(args.warmup):
        H.solve(K, y, inst.rho, tol=0.0, opts=opts)
        log(f"warmup {i} done")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    results = []
    for _ in range(args.steps):
        x, res = H.solve(K, y, inst.rho, tol=0.0, opts=opts)
        results.append(res)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    elapsed = t1 - t0
    iters = sum(r["iters"] for r in results)
    value = iters / elapsed
    ms_per_step = 1e3 * elapsed / args.steps
    fused_ms = sum(r["t_fused_ms"] for r in results)
    fused_n = sum(r["n_fused"] for r in results)
    avg_fused_s = fused_ms / max(fused_n, 1) / 1e3
    # algorithmic bytes of one fused launch: K once, d (p doubles) in,
    # q (n doubles) out, r (n doubles) in, w (p floats) out
    alg_bytes = n * p * 4 + 8 * p + 16 * n + 4 * p
    achieved = alg_bytes / avg_fused_s / 1e9
    log(f"timed: {args.steps} solves, {iters} iterations in {elapsed:.3f}s -> {value:.1f} it/s; "
        f"fused avg {avg_fused_s * 1e6:.1f} us -> {achieved:.0f} GB/s")
    x_gpu = x.cpu().double().numpy()
    status = results[-1]["status_name"]

    out = {
        "metric": "GP iterations/s (plain GPSS, FP32 K, FP64 scalars)",
        "value": round(value, 2),
        "unit": "iterations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded Gaussian compressed-sensing instance)",
        "config": {"workload": "plain GPSS, Gaussian K 4096x16384 fp32, 400-sparse x, "
                               "sigma 1e-2, rho 0.9||x||_1; each solve runs to the stationarity "
                               f"floor ({iters / args.steps:.0f} iterations) within a "
                               f"{ITERS}-iteration budget",
                   "n": n, "p": p, "iterations_per_step": round(iters / args.steps, 2),
                   "iteration_budget": ITERS, "refresh_every": REFRESH,
                   "status": status,
                   "threshold_passes_per_iter": round(results[-1]["proj_passes"] /
                                                      max(results[-1]["iters"], 1), 2)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": measured_traffic(),
                     "kernel": "k_fused (K d and K^T (K d), one read of K)",
                     "alg_bytes_per_launch": alg_bytes,
                     "avg_launch_us": round(avg_fused_s * 1e6, 2)},
    }

    # ---- the same solves with the Infinity Cache flushed first -------------
    # (outside the timed region above: a 512 MiB scratch write before each
    # solve, then the solve alone is timed)
    if not args.no_cold:
        scratch = torch.empty(128 << 20, dtype=torch.float32, device=dev)
        tcold = 0.0
        icold = 0
        for i in range(3):
            scratch.fill_(float(i))
            torch.cuda.synchronize()
            t0c = time.perf_counter()
            _, rc = H.solve(K, y, inst.rho, tol=0.0, opts=opts)
            torch.cuda.synchronize()
            tcold += time.perf_counter() - t0c
            icold += rc["iters"]
        del scratch
        out["cold_cache"] = {"value": round(icold / tcold, 2), "unit": "iterations/s",
                             "sample": "3 solves, each after a 512 MiB scratch write that evicts the "
                                       "256 MB Infinity Cache"}
        log(f"cold cache: {icold / tcold:.1f} it/s")
    out["host"] = host_info()

    # ---- wall time to a 1e-6 relative objective gap ----------------------
    K64 = y64 = None
    if not args.no_gap:
        K64 = inst.K64
        y64 = inst.y64
        if not args.no_cpu_baseline:
            # f* of the stored instance from the FP64 oracle, run to its
            # stationarity floor
            from oracle import gpss
            to = time.perf_counter()
            oref = gpss(K64, y64, inst.rho, tol=0.0, max_iter=100000)
            xl, f_ref = oref["x"], oref["f"]
            f_src = (f"FP64 oracle on the stored K, {oref['status']} after {oref['iters']} iterations "
                     f"({time.perf_counter() - to:.1f} s)")
        else:
            xl, _ = H.solve(K, y, inst.rho, tol=0.0, max_iter=3000, refresh_every=REFRESH)
            xl = xl.cpu().double().numpy()
            f_ref = float(np.sum((K64 @ xl - y64) ** 2))
            f_src = "3000-iteration GPU run, f recomputed in FP64 on the host (oracle leg off)"
        rl64 = K64 @ xl - y64
        g = 2.0 * (K64.T @ rl64)
        fw = float(g @ xl + inst.rho * np.abs(g).max())
        target = f_ref * (1 + 1e-6)
        gopts = gpl1.opts_for(K, max_iter=20000, refresh_every=REFRESH, f_target=target, chunk=16)
        H.solve(K, y, inst.rho, tol=0.0, opts=gopts)       # warm
        torch.cuda.synchronize()
        tg0 = time.perf_counter()
        xg, rg = H.solve(K, y, inst.rho, tol=0.0, opts=gopts)
        torch.cuda.synchronize()
        tg = time.perf_counter() - tg0
        xg = xg.cpu().double().numpy()
        fg = float(np.sum((K64 @ xg - y64) ** 2))
        out["time_to_gap_1e-6"] = {
            "seconds": round(tg, 5), "iterations": rg["iters"], "status": rg["status_name"],
            "gap_vs_ref": (fg - f_ref) / f_ref,
            "passed": bool(rg["status_name"] == "reached_target" and (fg - f_ref) / f_ref <= 1e-6),
            "target_stops_reopened": rg["reopened"],
            "f_ref_source": f_src,
            "f_ref_frank_wolfe_bound_rel": fw / f_ref}
        log(f"time to 1e-6 gap: {tg * 1e3:.2f} ms, {rg['iters']} iterations, "
            f"gap {(fg - f_ref) / f_ref:.2e} (FW bound of ref {fw / f_ref:.1e})")

    # ---- the other forms: BF16 storage, batched shared K --------------------
    if not args.no_forms:
        out["_x_fp32"] = x_gpu
        out["forms"] = forms_legs(H, inst, np, torch, gpl1, instances, out, not args.no_cpu_baseline)
        del out["_x_fp32"]

    # ---- the other single-instance workloads; a K larger than the cache ----
    if not args.no_configs:
        out["other_configs"] = configs_leg(H, np, torch, gpl1, instances, not args.no_cpu_baseline)
    if not args.no_mall:
        out["hbm_check_512MiB"] = mall_leg(H, np, torch, gpl1, instances)

    # ---- rho sweep and approximation isochrones (Section 4, in shape) ------
    if not args.no_isochrone:
        out["isochrone"] = isochrone_leg(H, np, torch, gpl1, instances)

    # ---- learned warm start + batched refinement --------------------------
    if not args.no_learned:
        out["learned_warm_start"] = learned_leg(H, np, torch, gpl1, instances, args.learned_train,
                                                args.learned_eval, args.learned_epochs,
                                                oracle_check=0 if args.no_cpu_baseline else 100)

    # ---- CPU oracle baseline + parity at 500 iterations --------------------
    if not args.no_cpu_baseline:
        from oracle import gpss
        if K64 is None:
            K64, y64 = inst.K64, inst.y64
        threads = blas_threads()
        # the same solve as one timed step, repeated until about 10 s of CPU
        # work (each solve stops at the stationarity floor, as the GPU's does)
        tc0 = time.perf_counter()
        nsolve = cpu_iters = 0
        while True:
            ref = gpss(K64, y64, inst.rho, tol=0.0, max_iter=ITERS)
            nsolve += 1
            cpu_iters += ref["iters"]
            if time.perf_counter() - tc0 >= 10.0 or nsolve >= 200:
                break
        tc = time.perf_counter() - tc0
        out["cpu_baseline"] = {"value": round(cpu_iters / tc, 3), "unit": "iterations/s",
                               "cores": threads, "kind": "oracle",
                               "sample": f"{nsolve} full solves ({ITERS}-iteration budget, "
                                         f"{cpu_iters} iterations) of the same stored instance by "
                                         f"the FP64 numpy oracle, {tc:.1f} s"}
        # the same oracle on one BLAS thread, a shorter sample
        try:
            from threadpoolctl import threadpool_limits
            with threadpool_limits(limits=1, user_api="blas"):
                t1 = time.perf_counter()
                n1 = 0
                while time.perf_counter() - t1 < 5.0:
                    n1 += gpss(K64, y64, inst.rho, tol=0.0, max_iter=ITERS)["iters"]
                t1 = time.perf_counter() - t1
            out["cpu_oracle_1_thread"] = {"value": round(n1 / t1, 3), "unit": "iterations/s",
                                          "sample": f"{n1} iterations in {t1:.1f} s"}
        except ImportError:
            pass
        fx = float(np.sum((K64 @ x_gpu - y64) ** 2))
        out["parity"] = {"rel_objective_diff_vs_oracle_500": (fx - ref["f"]) / ref["f"],
                         "x_rel_err_vs_oracle_500":
                             float(np.linalg.norm(x_gpu - ref["x"]) / np.linalg.norm(ref["x"])),
                         "oracle_status": ref["status"], "oracle_iters": ref["iters"]}
        log(f"cpu oracle: {cpu_iters / tc:.2f} it/s on {threads} threads; parity "
            f"{out['parity']}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
