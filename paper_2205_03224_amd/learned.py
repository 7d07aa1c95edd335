"""Learned warm start for the low-rank setup (not in the paper; the paper
names a block or randomised-subspace setup as future work, Sec. 6).

Pipeline, all device arithmetic in libgemslr:
  * training data: for each member of a parametric matrix family, a plain
    setup (thick-restart Arnoldi) gives the bases W_l; gs_features gives the
    per-node features X_l of the interface unknowns;
  * training: the 3-layer perceptron (gs_mlp_*) minimises the subspace loss
    ||Y^T Y||^2 - 2 ||W^T Y||^2 + k with Adam, one (instance, level) pair per
    step;
  * use: setup with the low-rank stage deferred, Y_l = network(X_l) on the
    GPU, then gs_lowrank runs the block Rayleigh-Ritz iteration from Y_l with
    Arnoldi as the fallback.
This module only orders those calls and moves arrays between them.
"""
import time

import numpy as np

from . import gemslr
from . import workloads as wl

NFEAT = 38
HIDDEN = 64


def init_params(seed, dims):
    """Glorot-uniform weights, zero biases, from default_rng(seed)."""
    rng = np.random.default_rng(seed)
    i, h, o = dims
    out = []
    for a, b in ((i, h), (h, h), (h, o)):
        lim = np.sqrt(6.0 / (a + b))
        out.append(rng.uniform(-lim, lim, (a, b)))
        out.append(np.zeros(b))
    return out


def family_member(instance, N=64, nparts=64):
    return wl.lognormal_convdiff3d_64(instance, N=N, nparts=nparts)


def setup_kwargs(w):
    return dict(lfil=w.lfil, grid_dims=w.dims, fgmres_restart=w.restart)


def collect(instances, N=64, nparts=64, rank=32, levels=(0, 1), log=None):
    """Per (instance, level): features X (s x 38) and the Arnoldi basis W
    (s x k), both float32 row-major numpy arrays."""
    data = []
    for i in instances:
        w = family_member(i, N, nparts)
        ctx = gemslr.Context(0)
        ctx.setup(w.rowptr, w.col, w.val, w.levels, w.nparts, rank, w.drop_tol,
                  **setup_kwargs(w))
        for l in levels:
            if l >= ctx.info()["nlevels"]:
                continue
            X = ctx.features(l)
            W = ctx.level(l)["W"]
            # same subspace, entries O(1) like the network's outputs: the loss
            # is minimised at Y = sqrt(s) W Q for any orthogonal Q
            Wt = np.ascontiguousarray(W * np.sqrt(W.shape[0]), dtype=np.float32)
            data.append({"instance": i, "level": l, "X": X, "W": Wt})
        ctx.close()
        if log:
            log(f"[learned] collected instance {i}")
    return data


def train(data, epochs=30, lr=1e-3, seed=0, out_dim=32, log=None):
    """Train the network on the GPU; returns (Mlp, loss history per epoch)."""
    import torch
    dims = (NFEAT, HIDDEN, out_dim)
    mlp = gemslr.Mlp(*dims)
    mlp.set_params(gemslr.pack_params(init_params(seed, dims)))
    Xs = [torch.from_numpy(d["X"]).cuda() for d in data]
    Ws = [torch.from_numpy(d["W"]).cuda() for d in data]
    rng = np.random.default_rng(seed + 1)
    hist = []
    for ep in range(epochs):
        tot = 0.0
        for j in rng.permutation(len(data)):
            mlp.zero_grad()
            loss = mlp.loss_backward(Xs[j], Ws[j])
            mlp.adam_step(lr)
            s, kw = Ws[j].shape
            # back to ||Y Y^T - W W^T||^2 / k for Y scaled by 1/sqrt(s)
            tot += ((loss - kw) / float(s) ** 2 + kw) / kw
        hist.append(tot / max(1, len(data)))
        if log and (ep % 5 == 0 or ep == epochs - 1):
            log(f"[learned] epoch {ep}: mean normalised loss {hist[-1]:.4f}")
    return mlp, hist


def predicted_bases(ctx, mlp, levels, out_dim):
    import torch
    warm = [None] * ctx.info()["nlevels"]
    for l in levels:
        if l >= len(warm):
            continue
        X = torch.from_numpy(ctx.features(l)).cuda()
        Y = torch.empty((X.shape[0], out_dim), dtype=torch.float32, device="cuda")
        mlp.forward(X, Y)
        warm[l] = Y
    return warm


def random_bases(ctx, levels, out_dim, seed):
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    warm = [None] * ctx.info()["nlevels"]
    for l in levels:
        if l >= len(warm):
            continue
        s = ctx.level_size(l)[1]
        warm[l] = torch.randn((s, out_dim), generator=g, device="cuda", dtype=torch.float32)
    return warm


def setup_with(w, rank, mode, mlp=None, levels=(0, 1), seed=0, **extra):
    """Setup with the low-rank stage run by `mode`: "arnoldi" (plain),
    "learned" (block iteration from the network's bases), "learned_arnoldi"
    (the thick-restart Arnoldi started from a vector of the network's
    subspace) or "random" (block iteration from random bases, the control).
    Returns (ctx, seconds spent on the low-rank stage incl. the network)."""
    import torch
    ctx = gemslr.Context(0)
    kw = setup_kwargs(w)
    kw.update(extra)
    if mode == "learned_arnoldi":
        kw["warm_start"] = 1
    ctx.setup(w.rowptr, w.col, w.val, w.levels, w.nparts, rank, w.drop_tol, defer_lowrank=1,
              **kw)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    if mode == "arnoldi":
        ctx.lowrank(rank)
    elif mode in ("learned", "learned_arnoldi"):
        ctx.lowrank(rank, predicted_bases(ctx, mlp, levels, rank))
    elif mode == "random":
        ctx.lowrank(rank, random_bases(ctx, levels, rank, seed))
    else:
        raise ValueError(mode)
    torch.cuda.synchronize()
    return ctx, time.perf_counter() - t0


def evaluate(instances, mlp, N=64, nparts=64, rank=32, tol=1e-8, levels=(0, 1), log=None):
    """Per held-out instance and mode: matvecs of the low-rank stage, its
    time, FGMRES iterations, true relative residual and time to tol."""
    import torch
    rows = []
    for i in instances:
        w = family_member(i, N, nparts)
        for mode in MODES:
            ctx, t_lr = setup_with(w, rank, mode, mlp, levels, seed=1000 + i)
            info = ctx.info()
            b = torch.from_numpy(w.b).cuda()
            x = torch.zeros_like(b)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            res = ctx.solve(b, x, tol)
            t_s = time.perf_counter() - t0
            rows.append({"instance": i, "mode": mode,
                         "matvecs": int(sum(info["arnoldi_matvecs"])),
                         "methods": info["lowrank_method"], "t_lowrank_s": t_lr,
                         "its": res["its"], "relres": res["relres"],
                         "converged": bool(res["converged"]), "t_solve_s": t_s,
                         "time_to_tol_s": t_lr + t_s})
            ctx.close()
            if log:
                r = rows[-1]
                log(f"[learned] instance {i} {mode}: matvecs {r['matvecs']} lowrank "
                    f"{r['t_lowrank_s']:.3f} s its {r['its']} time-to-tol {r['time_to_tol_s']:.3f} s")
    return rows


MODES = ("arnoldi", "learned", "learned_arnoldi", "random")


def summarise(rows):
    out = {}
    for mode in MODES:
        r = [x for x in rows if x["mode"] == mode]
        if not r:
            continue
        out[mode] = {k: float(np.mean([x[k] for x in r]))
                     for k in ("matvecs", "t_lowrank_s", "its", "relres", "time_to_tol_s")}
        out[mode]["median_time_to_tol_s"] = float(np.median([x["time_to_tol_s"] for x in r]))
    ar = {x["instance"]: x for x in rows if x["mode"] == "arnoldi"}
    for mode in ("learned", "learned_arnoldi"):
        if mode in out and ar:
            lr = {x["instance"]: x for x in rows if x["mode"] == mode}
            wins = [lr[i]["time_to_tol_s"] < ar[i]["time_to_tol_s"] for i in lr if i in ar]
            out[f"{mode}_win_fraction_vs_arnoldi"] = float(np.mean(wins)) if wins else None
    return out


def main(argv=None):
    """python -m paper_2205_03224_amd.learned train|evaluate ...

    train:    collect bases of members 0..n_train-1, train, save the
              parameters (npz) and the loss history.
    evaluate: load the parameters and compare Arnoldi / learned / random
              starts on held-out members 100000.. (JSON report)."""
    import argparse
    import json
    import sys

    ap = argparse.ArgumentParser()
    ap.add_argument("cmd", choices=["train", "evaluate"])
    ap.add_argument("--N", type=int, default=64)
    ap.add_argument("--nparts", type=int, default=64)
    ap.add_argument("--rank", type=int, default=32)
    ap.add_argument("--n-train", type=int, default=512)
    ap.add_argument("--n-heldout", type=int, default=64)
    ap.add_argument("--epochs", type=int, default=30)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--levels", default="0,1")
    ap.add_argument("--params", required=True, help="npz file to write (train) / read")
    ap.add_argument("--report", default=None)
    a = ap.parse_args(argv)

    def log(m):
        print(m, file=sys.stderr, flush=True)

    levels = tuple(int(x) for x in a.levels.split(","))
    if a.cmd == "train":
        t0 = time.perf_counter()
        data = collect(range(a.n_train), a.N, a.nparts, a.rank, levels, log=log)
        t1 = time.perf_counter()
        mlp, hist = train(data, a.epochs, a.lr, seed=0, out_dim=a.rank, log=log)
        t2 = time.perf_counter()
        np.savez(a.params, params=mlp.get_params(), dims=np.array(mlp.dims),
                 loss=np.array(hist), n_train=a.n_train, N=a.N, nparts=a.nparts,
                 rank=a.rank, levels=np.array(levels))
        rep = {"collect_s": t1 - t0, "train_s": t2 - t1, "loss_first": hist[0],
               "loss_last": hist[-1], "pairs": len(data)}
        log(f"[learned] trained: {rep}")
    else:
        z = np.load(a.params)
        dims = tuple(int(x) for x in z["dims"])
        mlp = gemslr.Mlp(*dims)
        mlp.set_params(z["params"])
        rows = evaluate(range(100000, 100000 + a.n_heldout), mlp, a.N, a.nparts, a.rank,
                        levels=levels, log=log)
        rep = {"summary": summarise(rows), "rows": rows}
        log(f"[learned] summary: {json.dumps(rep['summary'])}")
    if a.report:
        with open(a.report, "w") as f:
            json.dump(rep, f, indent=1, default=float)


if __name__ == "__main__":
    main()
