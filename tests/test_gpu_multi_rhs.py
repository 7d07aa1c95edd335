"""Several right-hand sides per apply (gs_apply_many): every launch of a
level covers all vectors, and in the streamed triangular sweeps a workgroup
may sweep a group of vectors (one consumer wave each) over the same staged
factor entries.  At these sizes the library would pick one vector per
workgroup, so GEMSLR_CONSUMERS forces groups of 2, 3 and 8 (with 8 vectors
and groups of 3: launches of 3 + 3 and 2).  Every column must equal the
oracle's apply of that column to the float64 apply tolerance, and, since
each right-hand side goes through the same operations in the same order as
in a single apply, equal the single apply of the same column bit for bit.
"""
import numpy as np
import pytest

from paper_2205_03224_amd import workloads as wl
from oracle import gemslr as og
from oracle import partition as opart
from tests.abi_helpers import assert_close, oracle_levels, relerr

pytestmark = pytest.mark.gpu

APPLY_TOL_F64 = 1e-10


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_03224_amd import gemslr  # noqa: F401  (fails loudly if unbuilt)
    return torch


def _case(name):
    if name == "laplace2d_32":
        w = wl.laplace2d_32()
        kw = dict(ilu="ilu0", rank=8)
    elif name == "convdiff3d_20_p27":
        w = wl.convdiff3d_64(N=20, nparts=27)
        kw = dict(ilu="ilut", drop_tol=1e-3, lfil=10, rank=8, dense_max=100)
    elif name == "helmholtz3d_16_p8":
        w = wl.helmholtz3d_128(N=16, nparts=8, levels=5)
        kw = dict(ilu="ilut", drop_tol=1e-4, lfil=10, rank=8, dense_max=100)
    else:
        raise KeyError(name)
    part = opart.wirebasket(w.dims, w.nparts, w.levels, w.rowptr, w.col)
    return w, og.setup(w.rowptr, w.col, w.val, part, **kw)


def _block(w, nrhs, seed):
    rs = np.random.default_rng(seed)
    X = rs.standard_normal((nrhs, w.n))
    if w.is_complex:
        X = X + 1j * rs.standard_normal((nrhs, w.n))
    return X


@pytest.mark.parametrize("env", [{}, {"GEMSLR_GROUP_CUS": "4"}, {"GEMSLR_NO_STREAM": "1"},
                                 {"GEMSLR_CONSUMERS": "2"}, {"GEMSLR_CONSUMERS": "3"},
                                 {"GEMSLR_CONSUMERS": "8", "GEMSLR_GROUP_CUS": "4"}])
@pytest.mark.parametrize("name", ["laplace2d_32", "convdiff3d_20_p27", "helmholtz3d_16_p8"])
@pytest.mark.parametrize("nrhs", [2, 3, 4, 8])
def test_apply_many_matches_oracle_and_single(torch_dev, name, nrhs, env, monkeypatch):
    torch = torch_dev
    from paper_2205_03224_amd import gemslr
    for k, v in env.items():
        monkeypatch.setenv(k, v)
    w, st = _case(name)
    print(f"[multi-rhs] {name} nrhs={nrhs} {env}", flush=True)
    ctx = gemslr.Context(0)
    ctx.setup_explicit(w.rowptr, w.col, w.val, st.perm, oracle_levels(st))
    X = _block(w, nrhs, 40 + nrhs)
    xd = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    yd = torch.empty_like(xd)
    ctx.apply_many(nrhs, xd, yd)
    ys = torch.empty_like(xd)
    for j in range(nrhs):
        ctx.apply(xd[j], ys[j])
    torch.cuda.synchronize()
    Y = yd.cpu().numpy()
    for j in range(nrhs):
        assert_close(Y[j], og.apply(st, X[j]), APPLY_TOL_F64, what=f"column {j}")
    assert torch.equal(yd, ys), "apply_many differs from single applies"
    ctx.close()


@pytest.mark.parametrize("cons", [None, "3"])
@pytest.mark.parametrize("nrhs", [2, 5])
@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_apply_many_mixed_forms_equal_single(torch_dev, prec, nrhs, cons, monkeypatch):
    """The float32-sweep forms share launches between right-hand sides as
    well; each column equals the single apply of the same form bit for
    bit."""
    torch = torch_dev
    from paper_2205_03224_amd import gemslr
    if cons:
        monkeypatch.setenv("GEMSLR_CONSUMERS", cons)
    w, st = _case("convdiff3d_20_p27")
    ctx = gemslr.Context(0)
    ctx.setup_explicit(w.rowptr, w.col, w.val, st.perm, oracle_levels(st))
    ctx.set_precision(prec)
    X = _block(w, nrhs, 77)
    xd = torch.from_numpy(X).cuda()
    yd = torch.empty_like(xd)
    ys = torch.empty_like(xd)
    ctx.apply_many(nrhs, xd, yd)
    for j in range(nrhs):
        ctx.apply(xd[j], ys[j])
    torch.cuda.synchronize()
    assert torch.equal(yd, ys)
    ctx.close()


@pytest.mark.parametrize("cons", [None, "8"])
def test_apply_many_beyond_one_batch(torch_dev, cons, monkeypatch):
    """More vectors than one batch holds (64): the library sweeps them in
    successive batches of its working vectors; every column still equals its
    single apply bit for bit, and the oracle's apply to the float64 apply
    tolerance (checked on a few columns)."""
    torch = torch_dev
    from paper_2205_03224_amd import gemslr
    if cons:
        monkeypatch.setenv("GEMSLR_CONSUMERS", cons)
    w, st = _case("laplace2d_32")
    ctx = gemslr.Context(0)
    ctx.setup_explicit(w.rowptr, w.col, w.val, st.perm, oracle_levels(st))
    nrhs = 70
    X = _block(w, nrhs, 1234)
    xd = torch.from_numpy(np.ascontiguousarray(X)).cuda()
    yd = torch.empty_like(xd)
    ctx.apply_many(nrhs, xd, yd)
    ys = torch.empty_like(xd)
    for j in range(nrhs):
        ctx.apply(xd[j], ys[j])
    torch.cuda.synchronize()
    assert torch.equal(yd, ys)
    Y = yd.cpu().numpy()
    for j in (0, 63, 64, 69):
        assert_close(Y[j], og.apply(st, X[j]), APPLY_TOL_F64, what=f"column {j}")
    ctx.close()


def test_batch_buffers_follow_rank_changes(torch_dev):
    """The batch buffers (each level's per-vector partial sums and t') are
    sized for the ranks in place when they are made, and made again when a
    rank has grown since.  20^3 / 27 subdomains, native setup with the
    low-rank stage deferred (rank 0 everywhere): a batched apply at rank 0;
    then ranks 100 / 100 / 8 from the block iteration started from random
    bases, whose batched G_hat products on level 0 run level 1's interface
    step at k = 100 (the E product, the multidot and the finish, all through
    the batch buffers) after level 1's own batched products made the
    buffers at rank 0 there; then ranks 8 from Arnoldi (smaller: the buffers
    stay).  After each, a batched apply of three vectors equals the single
    applies bit for bit, and so does the apply that allocates nothing
    (gs_apply_noalloc, whose scratch layout follows the current ranks)."""
    torch = torch_dev
    from paper_2205_03224_amd import gemslr, learned
    w = wl.convdiff3d_64(N=20, nparts=27)
    ctx = gemslr.Context(0)
    ctx.setup(w.rowptr, w.col, w.val, w.levels, w.nparts, 100, w.drop_tol, defer_lowrank=1,
              block_max_iters=2, **learned.setup_kwargs(w))
    X = torch.from_numpy(np.random.default_rng(77).standard_normal((3, w.n))).cuda()

    def check(what):
        Y = torch.empty_like(X)
        ctx.apply_many(3, X, Y)
        y = torch.empty_like(X[0])
        for j in range(3):
            ctx.apply(X[j].contiguous(), y)
            torch.cuda.synchronize()
            assert torch.isfinite(y).all(), what
            assert torch.equal(Y[j], y), f"{what}: column {j}"
            y2 = torch.empty_like(y)
            ctx.apply_noalloc(X[j].contiguous(), y2)
            torch.cuda.synchronize()
            assert torch.equal(y2, y), f"{what}: no-alloc apply, column {j}"

    check("rank 0")
    info = ctx.lowrank(100, learned.random_bases(ctx, (0, 1), 100, seed=9))
    ks = [ctx.level_size(l)[7] for l in range(info["nlevels"])]
    print(f"  block iteration: methods {info['lowrank_method']}, k = {ks}", flush=True)
    assert ks[0] == 100 and ks[1] == 100
    check("ranks 100")
    ctx.lowrank(8)
    check("ranks 8")
    ctx.close()
