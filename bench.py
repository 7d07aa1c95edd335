#!/usr/bin/env python3
"""Benchmark of the GeMSLR preconditioner apply on one MI355X.

Workload: 3-D 7-point convection-diffusion on a 128^3 grid (n = 2,097,152,
beta = 0.1/h), 3 levels, 512 subdomains, ILUT(1e-3, lfil 10), rank 32.

A step is one application of M^{-1} (the hot path of every FGMRES iteration:
gather, block triangular solves, interface products, low-rank corrections,
scatter) on a right-hand side already resident in HBM.  `value` is applies/s.
The level-0 block triangular solve (the dominant kernel) is bracketed with
HIP events on the library's stream during the timed steps, giving its
compulsory bytes / duration for the roofline.  After the timed region the
script reports time-to-1e-8 relative residual for the float64, float32 and
bfloat16 storage forms (setup of the low-rank terms + FGMRES, same partition
and factorisation) and times the CPU oracle on a bounded sample.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("time-to-1e-8 rel. residual + M^-1 applies/s (HBM GB/s), "
          "mixed/learned vs FP64")
HBM_PEAK_GBPS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def measured_traffic():
    """HBM bytes per level-0 trisolve launch from the committed rocprofv3
    counter summary (FETCH_SIZE and WRITE_SIZE, calibrated on a copy of known
    size), or None when the kernel sources differ from the ones it was
    measured with."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "trisolve_l0_convdiff3d_128.md")
    if not os.path.exists(path):
        return None
    fields = {}
    for line in open(path):
        k, _, v = line.strip().partition(": ")
        if k in ("traffic_bytes_per_launch", "source_sha256"):
            fields[k] = v.strip()
    h = hashlib.sha256()
    for f in ("kernels.hip", "device.h", "engine.hip"):
        with open(os.path.join(ROOT, "paper_2205_03224_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if fields.get("source_sha256") != h.hexdigest() or "traffic_bytes_per_launch" not in fields:
        return None
    return float(fields["traffic_bytes_per_launch"])


def oracle_setup_like(ctx, seed=7):
    """An oracle Setup with the structure of the installed preconditioner:
    permutation, per-level blocks, ILU factors, E_l and F_l as the library's
    host stages produced them (gs_get_level; the host ILU equals the oracle's
    bit for bit), and seeded synthetic W_l, H_l of the same ranks (W_l with
    orthonormal columns), so that no value computed on the GPU enters the
    oracle.  Only the time of the oracle's apply on it is used."""
    import numpy as np
    import scipy.sparse as sp

    from oracle import gemslr as og
    info = ctx.info()
    L = info["nlevels"]
    rng = np.random.default_rng(seed)
    levels, start = [], 0
    for l in range(L + 1):
        lv = ctx.level(l)
        d, s, k = lv["d"], lv["s"], lv["k"]
        mk = lambda m, r, c: sp.csr_matrix((m[2], m[1], m[0]), shape=(r, c))
        Lf, Uf = mk(lv["L"], d, d), mk(lv["U"], d, d)
        E, F = mk(lv["E"], s, d), mk(lv["F"], d, s)
        W = H = None
        if l < L and k > 0:
            W, _ = np.linalg.qr(rng.standard_normal((s, k)))
            H = 0.1 * rng.standard_normal((k, k))
        levels.append(og.Level(start, d, s, lv["block_ptr"],
                               Lf, Uf, E, F, W=W, H=H))
        start += d
    return og.Setup(ctx.n, ctx.perm(), levels, None, True)


def cpu_baseline(ctx, x, reps=2):
    """The oracle's apply (oracle.gemslr.apply, unmodified) timed on the host
    on the benchmark's own preconditioner structure (oracle_setup_like): a
    bounded sample of `reps` full applies, once on one thread and once with
    every host thread available to NumPy/SciPy."""
    import numpy as np
    from threadpoolctl import threadpool_info, threadpool_limits

    from oracle import gemslr as og
    st = oracle_setup_like(ctx)
    res = {}
    for label, limit in (("1", 1), ("all", None)):
        with threadpool_limits(limits=limit):
            used = max([t.get("num_threads", 1) for t in threadpool_info()] or [1])
            ts = []
            for _ in range(reps):
                t0 = time.perf_counter()
                og.apply(st, x)
                ts.append(time.perf_counter() - t0)
        res[label] = {"s_per_apply": float(np.median(ts)), "threads": int(used)}
    try:
        import subprocess
        model = [ln.split(":", 1)[1].strip() for ln in subprocess.run(
            ["lscpu"], capture_output=True, text=True).stdout.splitlines()
            if ln.startswith("Model name")][0]
    except Exception:
        model = "unknown"
    one, allc = res["1"], res["all"]
    return {"value": 1.0 / one["s_per_apply"], "unit": "applies/s", "cores": 1, "kind": "oracle",
            "sample": (f"{reps} full oracle applies (oracle.gemslr.apply) on the benchmark's "
                       f"128^3 preconditioner structure (library host-stage factors, E, F; "
                       f"seeded W, H of the same ranks), median {one['s_per_apply']:.2f} s on 1 "
                       f"thread; host {model}, os.cpu_count() {os.cpu_count()}"),
            "all_threads": {"value": 1.0 / allc["s_per_apply"], "threads": allc["threads"],
                            "s_per_apply": allc["s_per_apply"]},
            "host_cpu": model, "host_cpu_count": os.cpu_count()}


def copy_bandwidth(mib=1024, reps=10):
    """Device-to-device copy of `mib` MiB with torch (read + write bytes / time)."""
    import torch
    src = torch.ones((mib << 20) // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(2):
        dst.copy_(src)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    s = e0.elapsed_time(e1) * 1e-3 / reps
    del src, dst
    return 2.0 * (mib << 20) / s / 1e9


def timed_applies(ctx, b, K, warmup=10):
    """K applies after `warmup`: us per apply and the level-0 trisolve launch
    time and compulsory bytes from the library's probe (HIP events on its
    stream)."""
    import torch
    y = torch.empty_like(b)
    for _ in range(warmup):
        ctx.apply(b, y)
    torch.cuda.synchronize()
    ctx.probe_enable(0, 2 * K + 8)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        ctx.apply(b, y)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    launches, kms, kbytes = ctx.probe_read()
    ctx.probe_enable(-1, 0)
    k_ms = kms / max(launches, 1)
    k_bytes = kbytes / max(launches, 1)
    return dt * 1e6 / K, k_ms * 1e3, k_bytes


def convdiff64(K, log):
    """The 64^3 convection-diffusion configuration (n = 262,144, 64
    subdomains of ~16^3, 3 levels, ILUT(1e-3, 10), rank 32): apply rate,
    level-0 roofline and time to 1e-8 (low-rank setup + FGMRES(50))."""
    import numpy as np
    import torch

    from paper_2205_03224_amd import gemslr, workloads as wl
    w = wl.convdiff3d_64()
    ctx = gemslr.Context(0)
    ctx.setup(w.rowptr, w.col, w.val, w.levels, w.nparts, w.rank, w.drop_tol, lfil=w.lfil,
              grid_dims=w.dims, fgmres_restart=w.restart)
    info = ctx.info()
    b = torch.from_numpy(w.b).cuda()
    us, k_us, k_b = timed_applies(ctx, b, K)
    x = torch.zeros_like(b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = ctx.solve(b, x, 1e-8)
    ts = time.perf_counter() - t0
    xh = x.cpu().numpy()
    out = {"workload": "convdiff3d_64 (beta=0.1/h, 64 subdomains)", "n": w.n,
           "us_per_apply": us, "applies_per_s": 1e6 / us, "apply_bytes": info["apply_bytes"],
           "apply_GBps": info["apply_bytes"] / (us * 1e-6) / 1e9,
           "level0_us_per_launch": k_us, "level0_GBps": k_b / (k_us * 1e-6) / 1e9,
           "level0_frac": k_b / (k_us * 1e-6) / 1e9 / HBM_PEAK_GBPS,
           "its": res["its"], "relres": res["relres"], "t_lowrank_s": info["t_lowrank"],
           "t_solve_s": ts, "time_to_tol_s": info["t_lowrank"] + ts,
           "err_vs_x_true": float(np.linalg.norm(xh - w.x_true) / np.linalg.norm(w.x_true))}
    log(f"[bench] 64^3: {us:.1f} us/apply, level-0 {k_us:.1f} us ({out['level0_GBps']:.0f} GB/s); "
        f"time to 1e-8 {out['time_to_tol_s']:.3f} s ({res['its']} its)")
    ctx.close()
    return out


def helmholtz(N, K, log, ilu_shift=0.0):
    """Complex128 path: the shifted Helmholtz operator at N^3 (512 subdomains,
    ILUT(1e-4, 10), rank 64): applies/s and its HBM rate, time to 1e-8;
    ilu_shift s factors the blocks as B + i s mean|a_ii| I."""
    import numpy as np
    import torch

    from paper_2205_03224_amd import gemslr, workloads as wl
    w = wl.helmholtz3d_128(N=N, nparts=512 if N >= 64 else 8)
    ctx = gemslr.Context(0)
    t0 = time.perf_counter()
    ctx.setup(w.rowptr, w.col, w.val, w.levels, w.nparts, w.rank, w.drop_tol, lfil=w.lfil,
              grid_dims=w.dims, fgmres_restart=w.restart, ilu_shift=ilu_shift)
    t_setup = time.perf_counter() - t0
    info = ctx.info()
    b = torch.from_numpy(w.b).cuda()
    y = torch.empty_like(b)
    for _ in range(10):
        ctx.apply(b, y)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        ctx.apply(b, y)
    torch.cuda.synchronize()
    us = (time.perf_counter() - t0) * 1e6 / K
    x = torch.zeros_like(b)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    res = ctx.solve(b, x, 1e-8)
    ts = time.perf_counter() - t0
    xh = x.cpu().numpy()
    out = {"workload": f"helmholtz3d_{N} (complex128, k^2h^2=(2pi/10)^2, damping 0.05)",
           "ilu_shift": ilu_shift,
           "n": w.n, "levels": info["nlevels"], "rank": w.rank, "ilu": f"ILUT({w.drop_tol},{w.lfil})",
           "setup_s": t_setup, "t_lowrank_s": info["t_lowrank"], "fill": info["fill"],
           "us_per_apply": us, "applies_per_s": 1e6 / us, "apply_bytes": info["apply_bytes"],
           "apply_GBps": info["apply_bytes"] / (us * 1e-6) / 1e9,
           "its": res["its"], "relres": res["relres"], "converged": bool(res["converged"]),
           "t_solve_s": ts, "time_to_tol_s": info["t_lowrank"] + ts,
           "err_vs_x_true": float(np.linalg.norm(xh - w.x_true) / np.linalg.norm(w.x_true)),
           "arnoldi_cycles": list(info["arnoldi_cycles"][:info["nlevels"]]),
           "arnoldi_matvecs": list(info["arnoldi_matvecs"][:info["nlevels"]])}
    log(f"[bench] c128 (ilu_shift {ilu_shift}): {us:.1f} us/apply, {out['apply_GBps']:.0f} GB/s; solve its {res['its']} "
        f"relres {res['relres']:.2e} in {ts:.2f} s (+ lowrank {info['t_lowrank']:.2f} s; Arnoldi "
        f"cycles {out['arnoldi_cycles']} products {out['arnoldi_matvecs']})")
    ctx.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--N", type=int, default=128)
    ap.add_argument("--no-forms", action="store_true",
                    help="skip the time-to-tolerance runs of the three storage forms")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-c128", action="store_true",
                    help="skip the complex Helmholtz apply rate and time to tolerance")
    ap.add_argument("--breakdown", action="store_true", help="print per-launch profile")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the timed applies (no distribution, several right-hand sides, "
                         "mixed storage or copy measurement): for profiler runs")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="after the timed steps, copy a MIB-sized float64 buffer once (a plain "
                         "copy kernel of known traffic for counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        log("bench.py measures one GPU: the library holds all subdomains on a single "
            "MI355X and has no multi-GPU path; run it with --gpus 1.")
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2205_03224_amd import gemslr, workloads as wl

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    N = args.N
    w = wl.convdiff3d_128(N=N, nparts=512 if N >= 64 else 8)
    log(f"[bench] workload {w.name}: n={w.n} nnz={w.nnz}")
    setup_kw = dict(lfil=w.lfil, grid_dims=w.dims, fgmres_restart=w.restart)

    ctx = gemslr.Context(0)
    t0 = time.perf_counter()
    ctx.setup(w.rowptr, w.col, w.val, w.levels, w.nparts, w.rank, w.drop_tol, **setup_kw)
    setup_s = time.perf_counter() - t0
    info = ctx.info()
    log(f"[bench] setup {time.perf_counter() - t0:.1f} s: partition {info['t_partition']:.2f} "
        f"factor {info['t_factor']:.2f} layout {info['t_layout']:.2f} lowrank "
        f"{info['t_lowrank']:.2f}; d={info['d']} s={info['s']} k={info['k']} "
        f"depth L/U={info['depth_l']}/{info['depth_u']} fill={info['fill']:.3f}; Arnoldi "
        f"cycles {info['arnoldi_cycles'][:info['nlevels']]} products "
        f"{info['arnoldi_matvecs'][:info['nlevels']]}")

    b = torch.from_numpy(w.b).cuda()
    y = torch.empty_like(b)
    for _ in range(args.warmup):
        ctx.apply(b, y)
    torch.cuda.synchronize()

    K = args.steps
    ctx.probe_enable(0, 2 * K + 8)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        ctx.apply(b, y)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    launches, kms, kbytes = ctx.probe_read()
    ctx.probe_enable(-1, 0)
    ms_per_apply = dt * 1e3 / K
    applies_per_s = K / dt
    apply_bytes = info["apply_bytes"]
    k_ms = kms / max(launches, 1)
    k_bytes = kbytes / max(launches, 1)
    achieved = k_bytes / (k_ms * 1e-3) / 1e9
    log(f"[bench] {K} applies: {ms_per_apply * 1e3:.1f} us/apply, whole-apply "
        f"{apply_bytes / (ms_per_apply * 1e-3) / 1e9:.0f} GB/s; level-0 trisolve "
        f"{k_ms * 1e3:.1f} us/launch, {achieved:.0f} GB/s ({launches} launches)")

    dist, multi, mixed, copy_gbps = None, None, None, None
    if not args.no_extras:
        # per-apply distribution with events on the library's stream (torch's
        # current stream): warm = back-to-back applies on one setup; cold = a
        # 1 GiB buffer written between applies, which evicts the 256 MiB
        # last-level cache, so every factor byte comes from HBM
        def distribution(reps, flush=None):
            ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
                  for _ in range(reps)]
            for e0, e1 in ev:
                if flush is not None:
                    flush.fill_(1.0)
                e0.record()
                ctx.apply(b, y)
                e1.record()
            torch.cuda.synchronize()
            us = np.array([e0.elapsed_time(e1) * 1e3 for e0, e1 in ev])
            return {"median_us": float(np.median(us)), "p10_us": float(np.percentile(us, 10)),
                    "p90_us": float(np.percentile(us, 90)), "reps": reps}

        dist = {"warm": distribution(100)}
        flush = torch.empty((1 << 30) // 8, dtype=torch.float64, device="cuda")
        dist["cold"] = distribution(50, flush)
        del flush
        for key in ("warm", "cold"):
            d = dist[key]
            d["GBps_at_median"] = apply_bytes / (d["median_us"] * 1e-6) / 1e9
            log(f"[bench] {key}: median {d['median_us']:.1f} us (p10 {d['p10_us']:.1f}, "
                f"p90 {d['p90_us']:.1f}), {d['GBps_at_median']:.0f} GB/s")

        # several right-hand sides per call (gs_apply_many): every launch of
        # a level covers all vectors; in the level-0 sweeps workgroups sweep
        # groups of vectors over the same staged factor entries, so the
        # level-0 sweep time per vector falls where groups fit in LDS
        multi = {}
        for nb_ in (2, 3, 4, 8):
            Bm = torch.stack([torch.roll(b, 7919 * j) for j in range(nb_)])
            Ym = torch.empty_like(Bm)
            for _ in range(3):
                ctx.apply_many(nb_, Bm, Ym)
            torch.cuda.synchronize()
            kp = max(K // nb_, 4)
            t0 = time.perf_counter()
            for _ in range(kp):
                ctx.apply_many(nb_, Bm, Ym)
            torch.cuda.synchronize()
            us_call = (time.perf_counter() - t0) * 1e6 / kp
            # level-0 sweeps (down and up) of a few calls, per vector
            ctx.probe_enable(0, 2 * 4 + 8)
            for _ in range(4):
                ctx.apply_many(nb_, Bm, Ym)
            l0_launches, l0_ms, _ = ctx.probe_read()
            ctx.probe_enable(-1, 0)
            l0_us_vec = l0_ms * 1e3 / max(l0_launches, 1) / nb_
            multi[str(nb_)] = {"nrhs": nb_, "us_per_call": us_call,
                               "applies_per_s": nb_ * 1e6 / us_call,
                               "speedup_vs_single": (nb_ * 1e6 / us_call) / applies_per_s,
                               "level0_sweep_us_per_vector": l0_us_vec,
                               "calls": kp}
            log(f"[bench] {nb_} right-hand sides per call: {us_call:.1f} us per call, "
                f"{multi[str(nb_)]['applies_per_s']:.0f} applies/s "
                f"({multi[str(nb_)]['speedup_vs_single']:.2f}x single); level-0 sweep "
                f"{l0_us_vec:.1f} us per vector")
            del Bm, Ym

        # the float32 and bfloat16 storage forms of the same preconditioner:
        # apply rate and level-0 trisolve roofline (factors, E, F, W stored in
        # the narrow type, sweeps in float32)
        mixed = {}
        for prec in ("f32", "bf16"):
            ctx.set_precision(prec)
            us_m, k_us, k_b = timed_applies(ctx, b, K)
            mixed[prec] = {"us_per_apply": us_m, "applies_per_s": 1e6 / us_m,
                           "apply_bytes": ctx.info()["apply_bytes"],
                           "level0_us_per_launch": k_us, "level0_bytes_per_launch": k_b,
                           "level0_GBps": k_b / (k_us * 1e-6) / 1e9,
                           "level0_frac": k_b / (k_us * 1e-6) / 1e9 / HBM_PEAK_GBPS}
            log(f"[bench] {prec} storage: {us_m:.1f} us/apply ({1e6 / us_m:.0f} applies/s); level-0 "
                f"trisolve {k_us:.1f} us/launch, {mixed[prec]['level0_GBps']:.0f} GB/s")
        ctx.set_precision("f64")
        copy_gbps = copy_bandwidth()
        log(f"[bench] device copy (torch, 1 GiB): {copy_gbps:.0f} GB/s read + write")

    if args.calibrate_copy:
        nel = args.calibrate_copy * (1 << 20) // 8
        src = torch.ones(nel, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"[bench] calibration copy: {nel * 8} bytes read, {nel * 8} bytes written")
        del src, dst

    breakdown = None
    if args.breakdown:
        breakdown = ctx.apply_profile(b, y, reps=5)
        for st in breakdown:
            log(f"   {st['label']:<22s} {st['ms'] * 1e3:9.1f} us  {st['bytes'] / 1e6:9.2f} MB  "
                f"{st['bytes'] / max(st['ms'], 1e-9) / 1e6:8.0f} GB/s")

    out = {
        "metric": METRIC, "value": applies_per_s, "unit": "applies/s", "n_gpus": 1,
        "steps": K, "warmup": args.warmup, "ms_per_step": ms_per_apply,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"convdiff3d_{N} (7-pt convection-diffusion, beta=0.1/h)",
                   "n": w.n, "levels": info["nlevels"], "nparts": w.nparts, "rank": w.rank,
                   "ilu": f"ILUT({w.drop_tol},{w.lfil})", "parallelism": "single GPU"},
        "apply_GBps": apply_bytes / (ms_per_apply * 1e-3) / 1e9,
        "multi_rhs": multi,
        "mixed_storage": mixed,
        "copy_GBps_measured": copy_gbps,
        "apply_bytes": apply_bytes,
        "apply_distribution": dist,
        "setup": {"total_s": setup_s, "partition_s": info["t_partition"],
                  "factor_s": info["t_factor"], "layout_s": info["t_layout"],
                  "lowrank_s": info["t_lowrank"], "fill": info["fill"],
                  "depth_L": list(info["depth_l"][:info["nlevels"] + 1]),
                  "depth_U": list(info["depth_u"][:info["nlevels"] + 1]),
                  "arnoldi_cycles": list(info["arnoldi_cycles"][:info["nlevels"]]),
                  "arnoldi_matvecs": list(info["arnoldi_matvecs"][:info["nlevels"]]),
                  "host_threads": os.cpu_count()},
        "roofline": {"bound": "hbm", "kernel": "k_trisolve level 0 (down + up)",
                     "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS, "traffic": measured_traffic(),
                     "bytes_per_launch": k_bytes, "us_per_launch": k_ms * 1e3},
    }
    del y

    if not args.no_forms:
        forms = {}
        x64 = None
        for prec in ("f64", "f32", "bf16"):
            c2 = gemslr.Context(0)
            c2.setup(w.rowptr, w.col, w.val, w.levels, w.nparts, w.rank, w.drop_tol,
                     precision=prec, **setup_kw)
            i2 = c2.info()
            x = torch.zeros_like(b)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = c2.solve(b, x, 1e-8)
            ts = time.perf_counter() - t0
            xh = x.cpu().numpy()
            if prec == "f64":
                x64 = xh
            forms[prec] = {"t_lowrank_s": i2["t_lowrank"], "t_solve_s": ts,
                           "time_to_tol_s": i2["t_lowrank"] + ts, "its": res["its"],
                           "relres": res["relres"], "converged": bool(res["converged"]),
                           "err_vs_x_true": float(np.linalg.norm(xh - w.x_true) /
                                                  np.linalg.norm(w.x_true)),
                           "diff_vs_f64": float(np.linalg.norm(xh - x64) / np.linalg.norm(x64)),
                           "arnoldi_cycles": list(i2["arnoldi_cycles"][:i2["nlevels"]]),
                           "arnoldi_matvecs": list(i2["arnoldi_matvecs"][:i2["nlevels"]])}
            log(f"[bench] form {prec}: lowrank {i2['t_lowrank']:.2f} s + solve {ts:.2f} s, "
                f"its {res['its']}, relres {res['relres']:.2e}; Arnoldi cycles "
                f"{forms[prec]['arnoldi_cycles']} products {forms[prec]['arnoldi_matvecs']}")
            c2.close()
            del x
        out["time_to_tol"] = forms

    if not args.no_cpu_baseline:
        log("[bench] timing the CPU oracle on its bounded sample ...")
        out["cpu_baseline"] = cpu_baseline(ctx, w.b)
        log(f"[bench] cpu baseline: {out['cpu_baseline']['value']:.3f} applies/s on 1 thread, "
            f"{out['cpu_baseline']['all_threads']['value']:.3f} on "
            f"{out['cpu_baseline']['all_threads']['threads']} threads")
    ctx.close()
    if not args.no_forms:
        out["cfg2"] = convdiff64(args.steps, log)
    if not args.no_forms and not args.no_c128:
        out["c128"] = helmholtz(args.N, args.steps // 2, log)
        out["c128_shifted"] = helmholtz(args.N, args.steps // 2, log, ilu_shift=0.05)
    params = os.path.join(ROOT, "paper_2205_03224_amd", "data", "mlp_lognormal64.npz")
    if not args.no_forms and os.path.exists(params):
        # learned warm start on held-out members of the log-normal family it
        # was trained on (64^3, 64 subdomains, rank 32): Arnoldi vs learned
        # vs random-start block iteration, time to 1e-8 each
        from paper_2205_03224_amd import learned
        z = np.load(params)
        mlp = gemslr.Mlp(*[int(v) for v in z["dims"]])
        mlp.set_params(z["params"])
        rows = learned.evaluate(range(100000, 100004), mlp, N=64, nparts=64, rank=32,
                                levels=tuple(int(v) for v in z["levels"]))
        out["learned"] = learned.summarise(rows)
        out["learned"]["workload"] = "lognormal_convdiff3d_64, held-out members 100000-100003"
        log(f"[bench] learned: {json.dumps(out['learned'])}")
        mlp.close()
    if breakdown is not None:
        out["breakdown"] = [{"label": s["label"], "us": round(s["ms"] * 1e3, 2),
                             "MB": round(s["bytes"] / 1e6, 3)} for s in breakdown]
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
