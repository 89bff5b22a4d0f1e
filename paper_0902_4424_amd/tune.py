"""Autotuner of the solvers' kernel shapes, results in tuned.json.

Single problems (K dtype, n, p): it times the fused K / K^T kernel (HIP
events around every 4th launch, `profile` option) and the whole iteration
over the candidate kernel shapes (threads, column chunks per thread, rows
per block, or the two-launch pass over column panels) and grid sizes (row
slabs), and records the fastest; the binding
passes it through gp_opts.fused_cfg / fused_grid / fused_interleave.

Shared-K batches (dtype, n, p, B): the whole batched solve to a relative
change of 1e-10 over the GEMM output tile and split-K chunk, the per-problem row and column
kernel widths and graph replay, one option at a time (coordinate search from
the automatic choice).  Uneven batches (dtype, the 512-problem workload of n
in [128, 1024], p = 4n): rows per work item, the wave-per-row pass of the
narrow problems and graph replay.

    python -m paper_0902_4424_amd.tune f32:4096x16384 shared:bf16:2048x8192:256 var:bf16:512 ...
"""
import json
import os
import sys
import time

PKG = os.path.dirname(os.path.abspath(__file__))
TABLE = os.path.join(PKG, "tuned.json")

# (threads, chunks per thread) of the library's configurations 1..12; a
# configuration covers T * CPT * (16 / element size) columns.  Shape 6 spills
# registers and is tried only when nothing else covers p.
CFG_COVER = {1: (256, 1), 2: (256, 2), 3: (256, 4), 4: (512, 4), 5: (512, 8), 6: (1024, 8),
             7: (256, 4), 8: (512, 4), 9: (512, 8), 10: (1024, 4), 11: (1024, 4), 12: (1024, 2)}
ESIZE = {"f64": 8, "f32": 4, "bf16": 2}
PANELS = 13   # gp_opts.fused_cfg of the pass over column panels (GP_FUSED_PANELS)
GRIDS = (64, 128, 192, 256, 384, 512)


def key(dtype, n, p):
    return f"{dtype}:{n}x{p}"


def load_table():
    try:
        with open(TABLE) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def lookup(dtype, n, p):
    return load_table().get(key(dtype, n, p))


def candidates(dtype, n, p):
    vec = 16 // ESIZE[dtype]
    out = []
    covering = [c for c, (T, cpt) in CFG_COVER.items() if T * cpt * vec >= p]
    for c, (T, cpt) in CFG_COVER.items():
        if c == 6 and len(covering) > 1:
            continue
        if T * cpt * vec >= p and T * cpt * vec < 4 * max(p, 1):
            for g in GRIDS:
                if g <= n:
                    for il in (0, 1):
                        out.append((c, g, il))
    # the pass over column panels (two launches, K read twice): the automatic
    # choice past 8192 / 16384 columns, a candidate from 4096 on
    if p > 4096:
        out += [(PANELS, g, 0) for g in GRIDS if g <= n]
    return out


def tune_shape(H, dtype, n, p, iters=40, reps=3, log=print):
    import numpy as np
    import torch
    from . import gpl1, instances
    inst = instances.gaussian_instance(n, p, max(1, n // 20), dtype=dtype, seed=12345)
    if dtype == "bf16":
        K = torch.from_numpy(inst.K_store.view(np.int16)).cuda()
    else:
        K = torch.from_numpy(inst.K_store).cuda()
    y = torch.from_numpy(inst.y_store).cuda()
    best = None
    for cfg, grid, il in candidates(dtype, n, p):
        opts = gpl1.default_opts(max_iter=iters, profile=4, fused_cfg=cfg, fused_grid=grid,
                                 fused_interleave=il)
        H.solve(K, y, inst.rho, tol=0.0, opts=opts)          # warm
        torch.cuda.synchronize()
        fused, it_us = [], []
        for _ in range(reps):
            t0 = time.perf_counter()
            _, res = H.solve(K, y, inst.rho, tol=0.0, opts=opts)
            dt = time.perf_counter() - t0
            fused.append(res["t_fused_ms"] * 1e3 / max(res["n_fused"], 1))
            it_us.append(dt * 1e6 / max(res["iters"], 1))
        f_us, i_us = min(fused), min(it_us)
        log(f"  {key(dtype, n, p)} cfg={cfg} grid={grid} interleave={il}: fused {f_us:8.2f} us  "
            f"iteration {i_us:8.2f} us")
        if best is None or i_us < best["iter_us"]:
            best = {"fused_cfg": cfg, "fused_grid": grid, "fused_interleave": il,
                    "fused_us": round(f_us, 3), "iter_us": round(i_us, 3)}
    return best


def shared_key(dtype, n, p, B):
    return f"shared:{dtype}:{n}x{p}:{B}"


def var_key(dtype):
    return f"var:{dtype}"


def lookup_shared(dtype, n, p, B):
    """The tuned options of the shared-K batch with this (dtype, n, p) and the
    nearest batch size (log scale), or None."""
    import math
    best, dist = None, None
    pre = f"shared:{dtype}:{n}x{p}:"
    for k, v in load_table().items():
        if k.startswith(pre):
            d = abs(math.log2(int(k[len(pre):])) - math.log2(max(B, 1)))
            if dist is None or d < dist:
                best, dist = v, d
    return best


def lookup_var(dtype):
    return load_table().get(var_key(dtype))


def _coordinate_search(space, run, log):
    """Minimise run(opts) one option at a time, from the automatic choice."""
    cur = {k: 0 for k in space}
    best_t = run(dict(cur))
    for k, values in space.items():
        for v in values:
            if v == cur[k]:
                continue
            trial = dict(cur, **{k: v})
            t = run(trial)
            if t is not None and (best_t is None or t < best_t):
                best_t, cur = t, trial
        log(f"  {k} -> {cur[k]} ({best_t * 1e3:.3f} ms)")
    return cur, best_t


def tune_shared(H, dtype, n, p, B, reps=3, log=print):
    import numpy as np
    import torch
    from . import gpl1, instances
    batch = instances.shared_batch(n, p, B, max(1, n // 20), dtype=dtype, seed=12346, rhs_seed_base=70000)
    K = torch.from_numpy(batch.K_store.view(np.int16) if dtype == "bf16" else batch.K_store).cuda()
    Y = torch.from_numpy(batch.Y_store).cuda()

    def run(o):
        kw = {k: v for k, v in o.items() if v}
        try:
            H.solve_batched_shared(K, Y, batch.rho, tol=1e-10, max_iter=5000, refresh_every=50, chunk=8, **kw)
        except gpl1.GPError:
            return None
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            H.solve_batched_shared(K, Y, batch.rho, tol=1e-10, max_iter=5000, refresh_every=50, chunk=8, **kw)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        log(f"  {shared_key(dtype, n, p, B)} {kw or 'automatic'}: {min(ts) * 1e3:.3f} ms")
        return min(ts)

    space = {"batch_gemm_tile": (256, 64) if dtype == "bf16" else (), "batch_splitk": (256, 512, 1024, 2048),
             "batch_rows_t": (512, 1024), "batch_cols_t": (256, 512, 1024),
             "batch_gemm_depth": (2,) if dtype == "bf16" else (), "graph": (1,)}
    best, t = _coordinate_search(space, run, log)
    return dict(best, solve_ms=round(t * 1e3, 3))


def tune_var(H, dtype, B, reps=3, log=print):
    import numpy as np
    import torch
    from . import gpl1, instances
    insts = instances.uneven_batch(B, dtype=dtype, seed=4)
    probs = [(torch.from_numpy(i.K_store.view(np.int16) if dtype == "bf16" else i.K_store).cuda(),
              torch.from_numpy(i.y_store).cuda(), i.rho) for i in insts]

    def run(o):
        kw = {k: v for k, v in o.items() if v}
        H.solve_batched_var(probs, tol=1e-10, max_iter=5000, refresh_every=50, **kw)
        torch.cuda.synchronize()
        ts = []
        for _ in range(reps):
            t0 = time.perf_counter()
            H.solve_batched_var(probs, tol=1e-10, max_iter=5000, refresh_every=50, **kw)
            torch.cuda.synchronize()
            ts.append(time.perf_counter() - t0)
        log(f"  {var_key(dtype)} ({B} problems) {kw or 'automatic'}: {min(ts) * 1e3:.3f} ms")
        return min(ts)

    best, t = _coordinate_search({"var_item_rows": (16, 32, 128, 256), "var_wave_rows": (-1,), "graph": (1,)},
                                 run, log)
    return dict(best, solve_ms=round(t * 1e3, 3), problems=B)


def main(argv):
    import torch
    from . import gpl1
    if not torch.cuda.is_available():
        print("tune: needs a GPU", file=sys.stderr)
        return 2
    table = load_table()
    H = gpl1.Handle(0)
    say = lambda m: print(m, flush=True)   # noqa: E731
    for a in argv:
        parts = a.split(":")
        if parts[0] == "shared":
            dt, nm, B = parts[1], parts[2], int(parts[3])
            n, p = (int(v) for v in nm.split("x"))
            say(f"tuning {shared_key(dt, n, p, B)}")
            table[shared_key(dt, n, p, B)] = best = tune_shared(H, dt, n, p, B, log=say)
        elif parts[0] == "var":
            dt, B = parts[1], int(parts[2])
            say(f"tuning {var_key(dt)}")
            table[var_key(dt)] = best = tune_var(H, dt, B, log=say)
        else:
            dt, nm = parts
            n, p = (int(v) for v in nm.split("x"))
            say(f"tuning {key(dt, n, p)}")
            best = tune_shape(H, dt, n, p, log=say)
            if best:
                table[key(dt, n, p)] = best
        say(f"  -> {best}")
    with open(TABLE, "w") as fh:
        json.dump(table, fh, indent=1, sort_keys=True)
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
