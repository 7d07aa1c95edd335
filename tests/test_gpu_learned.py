"""Learned warm start on the GPU.

* the network's forward pass, subspace loss, gradients and Adam update (own
  HIP kernels, float32) against the float64 CPU oracle: float32 arithmetic
  with fixed-order row sums of a few hundred terms gives relative errors of
  order 1e-6; bounds 1e-4 (gradients) and 1e-5 (forward, loss, Adam);
* the block Rayleigh-Ritz setup from a given basis: from the Arnoldi basis
  itself it accepts after one block of products; from a random basis it
  converges or falls back, and the preconditioner still solves;
* the gain: a network trained on a small family of log-normal problems
  needs fewer Ĝ products than the same block iteration from random bases.
"""
import numpy as np
import pytest

from oracle import mlp as omlp
from paper_2205_03224_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def _rel(a, b):
    return float(np.linalg.norm(np.asarray(a, float) - np.asarray(b, float)) /
                 max(np.linalg.norm(np.asarray(b, float)), 1e-30))


def test_mlp_matches_oracle(torch_dev):
    torch = torch_dev
    from paper_2205_03224_amd import gemslr, learned
    dims = (38, 64, 8)
    rs = np.random.default_rng(4)
    params = learned.init_params(7, dims)
    params = [p + 0.05 * rs.standard_normal(p.shape) for p in params]  # nonzero biases
    s = 333
    X = rs.standard_normal((s, 38)).astype(np.float32)
    W, _ = np.linalg.qr(rs.standard_normal((s, 10)))
    W = W.astype(np.float32)
    mlp = gemslr.Mlp(*dims)
    mlp.set_params(gemslr.pack_params(params))
    P64 = [p.astype(np.float32).astype(np.float64) for p in params]
    Xd = torch.from_numpy(X).cuda()
    Wd = torch.from_numpy(W).cuda()
    Yd = torch.empty((s, 8), dtype=torch.float32, device="cuda")
    mlp.forward(Xd, Yd)
    Yo, _ = omlp.forward(P64, X.astype(np.float64))
    assert _rel(Yd.cpu().numpy(), Yo) < 1e-5
    mlp.zero_grad()
    loss = mlp.loss_backward(Xd, Wd)
    lo, go = omlp.loss_and_grad(P64, X.astype(np.float64), W.astype(np.float64))
    assert abs(loss - lo) <= 1e-5 * max(1.0, abs(lo))
    g = gemslr.unpack_params(mlp.get_grads(), dims)
    for a, b in zip(g, go):
        assert _rel(a, b) < 1e-4
    # gradients accumulate over calls
    mlp.loss_backward(Xd, Wd)
    g2 = gemslr.unpack_params(mlp.get_grads(), dims)
    assert _rel(g2[0], 2 * go[0]) < 1e-4
    # Adam from zero moments
    mlp.set_params(gemslr.pack_params(params))
    mlp.zero_grad()
    mlp.loss_backward(Xd, Wd)
    mlp.adam_step(1e-3, 0.9, 0.999, 1e-8)
    new = gemslr.unpack_params(mlp.get_params(), dims)
    g32 = gemslr.unpack_params(mlp.get_grads(), dims)
    ref, _, _ = omlp.adam_step(P64, [x.astype(np.float64) for x in g32],
                               [np.zeros_like(p) for p in P64], [np.zeros_like(p) for p in P64], 1,
                               lr=1e-3)
    for a, b in zip(new, ref):
        assert np.max(np.abs(a - b)) < 1e-5
    mlp.close()


def test_mlp_loss_backward_as_first_call(torch_dev):
    """Regression: a fresh network whose first call is loss_backward (no
    forward before it) must size its buffers before using them."""
    torch = torch_dev
    from paper_2205_03224_amd import gemslr, learned
    dims = (38, 64, 6)
    params = learned.init_params(3, dims)
    rs = np.random.default_rng(9)
    X = rs.standard_normal((1141, 38)).astype(np.float32)
    W, _ = np.linalg.qr(rs.standard_normal((1141, 7)))
    W = W.astype(np.float32)
    mlp = gemslr.Mlp(*dims)
    mlp.set_params(gemslr.pack_params(params))
    loss = mlp.loss_backward(torch.from_numpy(X).cuda(), torch.from_numpy(W).cuda())
    P64 = [p.astype(np.float32).astype(np.float64) for p in params]
    lo, _ = omlp.loss_and_grad(P64, X.astype(np.float64), W.astype(np.float64))
    assert abs(loss - lo) <= 1e-5 * max(1.0, abs(lo))
    mlp.close()


def _small():
    return wl.lognormal_convdiff3d_64(3, N=20, nparts=8)


def test_block_setup_from_arnoldi_basis(torch_dev):
    torch = torch_dev
    from paper_2205_03224_amd import gemslr, learned
    w = _small()
    rank = 6
    ref = gemslr.Context(0)
    ref.setup(w.rowptr, w.col, w.val, w.levels, w.nparts, rank, w.drop_tol,
              **learned.setup_kwargs(w))
    W0 = ref.level(0)["W"]
    k0 = W0.shape[1]
    ctx = gemslr.Context(0)
    ctx.setup(w.rowptr, w.col, w.val, w.levels, w.nparts, rank, w.drop_tol, defer_lowrank=1,
              **learned.setup_kwargs(w))
    warm = [torch.from_numpy(np.ascontiguousarray(W0, dtype=np.float32)).cuda(),
            None, None][:ctx.info()["nlevels"]]
    info = ctx.lowrank(k0, warm)
    print("  methods", info["lowrank_method"], "matvecs", info["arnoldi_matvecs"], flush=True)
    assert info["lowrank_method"][0] == 1
    assert info["arnoldi_matvecs"][0] == k0  # accepted after one block of products
    b = torch.from_numpy(w.b).cuda()
    x = torch.zeros_like(b)
    res = ctx.solve(b, x, 1e-8)
    xr = torch.zeros_like(b)
    res_ref = ref.solve(b, xr, 1e-8)
    assert res["converged"] and abs(res["its"] - res_ref["its"]) <= 2
    ref.close()
    ctx.close()


def test_block_setup_from_random_basis(torch_dev):
    torch = torch_dev
    from paper_2205_03224_amd import gemslr, learned
    w = _small()
    ctx = gemslr.Context(0)
    ctx.setup(w.rowptr, w.col, w.val, w.levels, w.nparts, 6, w.drop_tol, defer_lowrank=1,
              block_max_iters=3, **learned.setup_kwargs(w))
    info = ctx.lowrank(6, learned.random_bases(ctx, (0, 1), 6, seed=5))
    print("  methods", info["lowrank_method"], "matvecs", info["arnoldi_matvecs"], flush=True)
    assert info["lowrank_method"][0] in (1, 2)
    b = torch.from_numpy(w.b).cuda()
    x = torch.zeros_like(b)
    res = ctx.solve(b, x, 1e-8)
    assert res["converged"]
    ctx.close()


@pytest.mark.slow
def test_learned_gain_small_family(torch_dev):
    """Train on 24 members of the log-normal family (20^3, 8 parts, rank 6)
    and score on 6 held-out members against the method without the network,
    plain thick-restart Arnoldi (the baseline it has to beat), with the block
    iteration from random bases as a second control.  Reported per mode: Ĝ products,
    low-rank setup time, FGMRES iterations, true residual, time to 1e-8.

    What the network buys on this family: fewer Ĝ products than the same
    block iteration from random bases, and a preconditioner as good as
    Arnoldi's (FGMRES iterations within 3).  What it does not buy: a time
    to 1e-8 clearly below plain Arnoldi's.  At this size the two are within
    a few percent in products and in time (measured: 65.3 against 67.0
    products, time ratio 0.99-1.02); on the benchmark's 64^3 family the
    learned start loses clearly (the single-vector Krylov-Schur needs fewer
    products on those clustered spectra, and the block iteration spends its
    time in per-iteration host work).  The test states this instead of
    asserting a gain that does not hold: every mode's figures are reported,
    the times are printed beside Arnoldi's, and the finding is asserted on
    the G_hat products, which timing noise does not move: no cut beyond 15 %
    against Arnoldi's (measured ~3 %); it fails if that changes, so that the
    finding gets re-examined."""
    from paper_2205_03224_amd import learned
    rank = 6
    data = learned.collect(range(24), N=20, nparts=8, rank=rank, levels=(0,))
    mlp, hist = learned.train(data, epochs=40, lr=3e-3, seed=0, out_dim=rank)
    print("  loss", [round(h, 3) for h in hist[::10]], flush=True)
    assert hist[-1] < hist[0]
    rows = learned.evaluate(range(100000, 100006), mlp, N=20, nparts=8, rank=rank,
                            levels=(0,))
    summ = learned.summarise(rows)
    for mode in learned.MODES:
        m = summ[mode]
        print(f"  {mode:16s} products {m['matvecs']:6.1f}  low-rank {m['t_lowrank_s']:.4f} s  "
              f"its {m['its']:5.1f}  time to 1e-8 {m['time_to_tol_s']:.4f} s", flush=True)
    assert all(r["converged"] and r["relres"] <= 1.5e-8 for r in rows)
    # gain over the random-basis control, same preconditioner quality
    assert summ["learned"]["matvecs"] < summ["random"]["matvecs"]
    assert summ["learned"]["its"] <= summ["arnoldi"]["its"] + 3
    # against plain Arnoldi: the measured finding on this family
    ar = summ["arnoldi"]
    for mode in learned.MODES:
        for key in ("matvecs", "t_lowrank_s", "its", "time_to_tol_s"):
            assert np.isfinite(summ[mode][key]) and summ[mode][key] > 0, (mode, key)
    print(f"  learned / Arnoldi time to 1e-8: "
          f"{summ['learned']['time_to_tol_s'] / ar['time_to_tol_s']:.2f} (block), "
          f"{summ['learned_arnoldi']['time_to_tol_s'] / ar['time_to_tol_s']:.2f} "
          f"(Arnoldi from the predicted subspace)", flush=True)
    assert summ["learned"]["matvecs"] >= 0.85 * ar["matvecs"]
    mlp.close()
