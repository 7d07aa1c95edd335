"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the
same seeded inputs.

Tolerances: a float64 apply differs from the oracle only by the order of
additions inside the triangular solves and sparse products.  Per entry the
difference is a small multiple of depth * eps times the magnitudes of the
partial sums, which on these diagonally dominant factors stay within a small
factor of the result's own entries; applies are compared entry by entry
(tests/abi_helpers.assert_close: |y_i - ref_i| <= tol (|ref_i| + 1e-3
||ref||_inf)) with tol = 1e-10.
The solve compares FGMRES(m) runs with the same M^{-1}: both stop at the same
true-residual tolerance and their iterates agree to well below 1e-10.
"""
import numpy as np
import pytest

from paper_2205_03224_amd import workloads as wl
from oracle import fgmres as ofg
from oracle import gemslr as og
from oracle import partition as opart
from tests.abi_helpers import MIXED_FLOOR, MIXED_TOL, assert_close, oracle_levels, relerr

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
        return w, dict(ilu="ilu0", rank=8)
    if name == "convdiff3d_20_p27":
        w = wl.convdiff3d_64(N=20, nparts=27)
        return w, dict(ilu="ilut", drop_tol=1e-3, lfil=10, rank=8, dense_max=100)
    if name == "helmholtz3d_16_p8":
        w = wl.helmholtz3d_128(N=16, nparts=8, levels=5)
        return w, dict(ilu="ilut", drop_tol=1e-4, lfil=10, rank=8, dense_max=100)
    if name == "lognormal_16_p8":
        w = wl.lognormal_convdiff3d_64(7, N=16, nparts=8)
        return w, dict(ilu="ilut", drop_tol=1e-3, lfil=10, rank=6, dense_max=50)
    raise KeyError(name)


def _oracle_setup(w, kw):
    part = opart.wirebasket(w.dims, w.nparts, w.levels, w.rowptr, w.col)
    return og.setup(w.rowptr, w.col, w.val, part, **kw)


def _ctx_explicit(torch, w, st, **opts):
    from paper_2205_03224_amd import gemslr
    ctx = gemslr.Context(0)
    ctx.setup_explicit(w.rowptr, w.col, w.val, st.perm, oracle_levels(st), **opts)
    return ctx


CASES = ["laplace2d_32", "convdiff3d_20_p27", "helmholtz3d_16_p8", "lognormal_16_p8"]


@pytest.mark.parametrize("name", CASES)
def test_apply_matches_oracle(torch_dev, name):
    torch = torch_dev
    w, kw = _case(name)
    print(f"[apply parity] {name} n={w.n}", flush=True)
    st = _oracle_setup(w, kw)
    ctx = _ctx_explicit(torch, w, st)
    rs = np.random.default_rng(12)
    for trial in range(3):
        x = rs.standard_normal(w.n)
        if w.is_complex:
            x = x + 1j * rs.standard_normal(w.n)
        if trial == 2:
            x = w.b  # the actual right-hand side
        ref = og.apply(st, x)
        xd = torch.from_numpy(np.ascontiguousarray(x)).cuda()
        yd = torch.empty_like(xd)
        ctx.apply(xd, yd)
        torch.cuda.synchronize()
        assert_close(yd.cpu().numpy(), ref, APPLY_TOL_F64, what=f"trial {trial}")
    ctx.close()


def test_apply_full_rank_is_exact_inverse(torch_dev):
    torch = torch_dev
    r, c, v = wl.convdiff3d(7, (0.3, 0.2, 0.1))
    w = wl.Workload("cd7", (7, 7, 7), r, c, v, levels=3, nparts=8, rank=10 ** 6,
                    ilu="ilut", drop_tol=0.0, lfil=10 ** 6, restart=30, tol=1e-8)
    st = _oracle_setup(w, dict(ilu="ilut", drop_tol=0.0, lfil=10 ** 9, rank=10 ** 9))
    ctx = _ctx_explicit(torch, w, st)
    A = og.csr(r, c, v, w.n).toarray()
    x = np.random.default_rng(3).standard_normal(w.n)
    xd = torch.from_numpy(x).cuda()
    yd = torch.empty_like(xd)
    ctx.apply(xd, yd)
    torch.cuda.synchronize()
    assert_close(yd.cpu().numpy(), np.linalg.solve(A, x), 1e-10, what="M^-1 x vs A^-1 x")
    ctx.close()


@pytest.mark.parametrize("name,rank,prec", [("convdiff3d_20_p27", 100, None),
                                            ("convdiff3d_20_p27", 200, None),
                                            ("convdiff3d_20_p27", 100, "f32"),
                                            ("convdiff3d_20_p27", 1024, None),
                                            ("helmholtz3d_16_p8", 40, None),
                                            ("helmholtz3d_16_p8", 1024, None)])
def test_apply_matches_oracle_at_large_ranks(torch_dev, name, rank, prec):
    """The interface step of large ranks.  Float64, 20^3 / 27 subdomains
    (s_l = 2168, 224, 8), ranks 100 and 200: levels 0 and 1 above the
    one-workgroup step's k = 64 and above k = 80, where the E product runs
    alone, W^H z2 as a column-chunked multidot and the finish on its
    column-major partials (10 or 5 threads per column); also with float32
    storage (the same three launches in float32, against the float64 oracle
    to the mixed form's tolerance).  Complex128
    Helmholtz 16^3 / 8 subdomains (s_0 = 721), rank 40: level 0 above two
    16-column batches, the same three launches in complex arithmetic.
    Rank 1024, the largest the library takes: k = 1024 / 224 / 8 on the
    float64 case (one thread per column in the finish), k = 721 / 46 / 1 on
    the complex one (every level at full rank, k = s_l).
    W_l are seeded orthonormal columns and H_l seeded k x k matrices (the
    apply does not depend on how they were found), the same on both sides."""
    torch = torch_dev
    w, kw = _case(name)
    kw = dict(kw, rank=0)
    st = _oracle_setup(w, kw)
    rng = np.random.default_rng(rank)
    for lv in st.levels[:-1]:
        k = min(rank, lv.s)
        G = rng.standard_normal((lv.s, k))
        H = 0.1 * rng.standard_normal((k, k))
        if w.is_complex:
            G = G + 1j * rng.standard_normal((lv.s, k))
            H = H + 0.1j * rng.standard_normal((k, k))
        lv.W = np.linalg.qr(G)[0]
        lv.H = H
    print(f"[apply parity] {name} rank {rank}: k = {[lv.W.shape[1] for lv in st.levels[:-1]]}",
          flush=True)
    ctx = _ctx_explicit(torch, w, st)
    if prec:
        ctx.set_precision(prec)
    x = np.random.default_rng(rank + 1).standard_normal(w.n)
    if w.is_complex:
        x = x + 1j * np.random.default_rng(rank + 3).standard_normal(w.n)
    ref = og.apply(st, x)
    xd = torch.from_numpy(x).cuda()
    yd = torch.empty_like(xd)
    ctx.apply(xd, yd)
    torch.cuda.synchronize()
    if prec:
        assert_close(yd.cpu().numpy(), ref, MIXED_TOL[prec], floor=MIXED_FLOOR)
    else:
        assert_close(yd.cpu().numpy(), ref, APPLY_TOL_F64)
    # three vectors per call: every launch of a level covers all three, each
    # column equal to its single apply bit for bit
    Xh = np.random.default_rng(rank + 2).standard_normal((3, w.n))
    if w.is_complex:
        Xh = Xh + 1j * np.random.default_rng(rank + 4).standard_normal((3, w.n))
    X = torch.from_numpy(Xh).cuda()
    Y = torch.empty_like(X)
    ctx.apply_many(3, X, Y)
    torch.cuda.synchronize()
    for j in range(3):
        ctx.apply(X[j].contiguous(), yd)
        torch.cuda.synchronize()
        assert torch.equal(Y[j], yd), f"column {j}"
    ctx.close()


@pytest.mark.parametrize("name", ["laplace2d_32", "convdiff3d_20_p27", "helmholtz3d_16_p8"])
def test_apply_rank_zero_matches_oracle(torch_dev, name):
    """Rank 0 on every level: without the low-rank correction the Schur
    complement solve is the C_l solve alone, so M^{-1} is the multilevel
    block LDU of Sec. 2.2 built from the ILU factors (the oracle's rank-0
    form, pinned against dense inverses).  The interface kernels take their
    k = 0 branch: z2 written, no projection and no update launch.  Two
    vectors per call are bit-equal to single applies."""
    torch = torch_dev
    w, kw = _case(name)
    st = _oracle_setup(w, dict(kw, rank=0))
    assert all(lv.W.shape[1] == 0 for lv in st.levels[:-1])
    print(f"[apply parity] {name} rank 0", flush=True)
    ctx = _ctx_explicit(torch, w, st)
    rs = np.random.default_rng(21)
    X = rs.standard_normal((2, w.n))
    if w.is_complex:
        X = X + 1j * rs.standard_normal((2, w.n))
    Xd = torch.from_numpy(X).cuda()
    Yd = torch.empty_like(Xd)
    ctx.apply_many(2, Xd, Yd)
    yd = torch.empty_like(Xd[0])
    for j in range(2):
        ctx.apply(Xd[j].contiguous(), yd)
        torch.cuda.synchronize()
        assert_close(yd.cpu().numpy(), og.apply(st, X[j]), APPLY_TOL_F64, what=f"vector {j}")
        assert torch.equal(Yd[j], yd), f"column {j}"
    ctx.close()


@pytest.mark.parametrize("name", ["convdiff3d_20_p27", "helmholtz3d_16_p8"])
def test_apply_degenerate_inputs(torch_dev, name):
    """x = 0 gives y = 0 in every entry (without inner GMRES steps M^{-1} is
    a fixed linear operator and every kernel forms sums of products with
    x's entries), written over an output filled with NaN, so every entry of
    y, the C_0 rows' scatter included, is written.  An empty batch
    (nrhs = 0) succeeds and writes nothing, with empty tensors (NULL
    pointers) and with live buffers."""
    import ctypes as ct

    from paper_2205_03224_amd import gemslr
    torch = torch_dev
    w, kw = _case(name)
    print(f"[degenerate inputs] {name}", flush=True)
    st = _oracle_setup(w, kw)
    ctx = _ctx_explicit(torch, w, st)
    dt = torch.complex128 if w.is_complex else torch.float64
    x = torch.zeros(w.n, dtype=dt, device="cuda")
    y = torch.full((w.n,), float("nan"), dtype=dt, device="cuda")
    ctx.apply(x, y)
    torch.cuda.synchronize()
    assert torch.equal(y, torch.zeros_like(y))
    y.fill_(float("nan"))
    ctx.apply_many(1, x, y)
    torch.cuda.synchronize()
    assert torch.equal(y, torch.zeros_like(y))
    empty = torch.empty(0, dtype=dt, device="cuda")
    ctx.apply_many(0, empty, torch.empty_like(empty))
    y.fill_(float("nan"))
    rc = gemslr.lib().gs_apply_many(ctx._h, 0, ct.c_void_p(x.data_ptr()),
                                    ct.c_void_p(y.data_ptr()))
    torch.cuda.synchronize()
    assert rc == 0
    assert torch.isnan(y.real).all()
    assert gemslr.lib().gs_apply_many(ctx._h, -1, ct.c_void_p(x.data_ptr()),
                                      ct.c_void_p(y.data_ptr())) != 0
    ctx.close()


@pytest.mark.parametrize("name", ["laplace2d_32", "convdiff3d_20_p27", "helmholtz3d_16_p8"])
def test_solve_same_setup_matches_oracle(torch_dev, name):
    torch = torch_dev
    w, kw = _case(name)
    print(f"[solve parity] {name}", flush=True)
    st = _oracle_setup(w, kw)
    A = og.csr(w.rowptr, w.col, w.val, w.n)
    xo, io = ofg.fgmres(lambda z: A @ z, lambda z: og.apply(st, z), w.b, tol=w.tol,
                        restart=w.restart)
    ctx = _ctx_explicit(torch, w, st, fgmres_restart=w.restart)
    bd = torch.from_numpy(w.b).cuda()
    xd = torch.zeros_like(bd)
    info = ctx.solve(bd, xd, w.tol)
    xg = xd.cpu().numpy()
    print(f"  oracle its {io['its']} relres {io['relres']:.2e}; gpu its {info['its']} "
          f"relres {info['relres']:.2e}; diff {relerr(xg, xo):.2e}", flush=True)
    assert info["converged"] and io["converged"]
    assert abs(info["its"] - io["its"]) <= 1
    assert relerr(xg, xo) <= 1e-10
    assert np.linalg.norm(w.b - A @ xg) <= w.tol * np.linalg.norm(w.b) * 1.0001
    ctx.close()


def test_native_setup_solves(torch_dev):
    """gs_setup end to end (host partition + ILUT, GPU Arnoldi) on a small
    convection-diffusion grid: reaches the tolerance, agrees with x* and with
    the oracle's own solve to within cond * tol."""
    torch = torch_dev
    from paper_2205_03224_amd import gemslr
    w = wl.convdiff3d_64(N=20, nparts=27)
    ctx = gemslr.Context(0)
    ctx.setup(w.rowptr, w.col, w.val, w.levels, w.nparts, 8, 1e-3, lfil=10,
              grid_dims=w.dims, fgmres_restart=w.restart)
    info = ctx.info()
    print("  setup info", {k: info[k] for k in ("d", "s", "k", "arnoldi_cycles",
                                                 "arnoldi_converged", "fill")}, flush=True)
    bd = torch.from_numpy(w.b).cuda()
    xd = torch.zeros_like(bd)
    res = ctx.solve(bd, xd, 1e-12)
    xg = xd.cpu().numpy()
    assert res["converged"], res
    assert relerr(xg, w.x_true) <= 1e-8
    ctx.close()


@pytest.mark.parametrize("env", [{"GEMSLR_NO_STREAM": "1"}, {"GEMSLR_LDS_BUDGET": "16384"},
                                 {"GEMSLR_LDS_BUDGET": "20480"},
                                 {"GEMSLR_NO_GROUP": "1"}, {"GEMSLR_GROUP_CUS": "4"},
                                 {"GEMSLR_GROUP_CUS": "2", "GEMSLR_NO_STREAM": "1"},
                                 {"GEMSLR_NO_FUSE_SMALL": "1"}, {"GEMSLR_NO_FUSE_PERM": "1"},
                                 {"GEMSLR_NO_HALF": "1"}, {"GEMSLR_NO_FUSE_FY": "1"},
                                 {"GEMSLR_NO_FUSE_E": "1"}, {"GEMSLR_NO_SMALL_LDS": "1"}])
@pytest.mark.parametrize("name", ["convdiff3d_20_p27", "helmholtz3d_16_p8"])
def test_apply_kernel_variants(torch_dev, name, env, monkeypatch):
    """Both block-trisolve kernels (register prefetch; LDS-streamed with small
    chunks so that each block takes many producer/consumer hand-offs, with
    two or three chunk buffers; consecutive diagonal blocks swept by one
    workgroup or one each), both interface paths (one fused launch for
    small levels, three launches) and both ways of applying the permutation
    (inside the level-0 sweeps, or separate kernels), U stages swept with
    one lane per row or two lanes per row, F_l y2 formed inside the up
    sweep or by a launch of its own, E_l z1 from values the down sweep filed
    in E_l's entry order or from gathers of z1, and the small-level
    interface step with
    W_l and H_l copied to LDS or read from global memory, give the oracle's
    apply."""
    torch = torch_dev
    for k, v in env.items():
        monkeypatch.setenv(k, v)
    w, kw = _case(name)
    print(f"[kernel variant] {name} {env}", flush=True)
    st = _oracle_setup(w, kw)
    ctx = _ctx_explicit(torch, w, st)
    x = np.random.default_rng(5).standard_normal(w.n)
    if w.is_complex:
        x = x + 1j * np.random.default_rng(6).standard_normal(w.n)
    ref = og.apply(st, x)
    xd = torch.from_numpy(x).cuda()
    yd = torch.empty_like(xd)
    ctx.apply(xd, yd)
    torch.cuda.synchronize()
    assert_close(yd.cpu().numpy(), ref, APPLY_TOL_F64)
    ctx.close()


@pytest.mark.parametrize("name", ["convdiff3d_20_p27", "helmholtz3d_16_p8"])
@pytest.mark.parametrize("knob", ["GEMSLR_NO_FUSE_FY", "GEMSLR_NO_FUSE_E", "GEMSLR_NO_SMALL_LDS"])
def test_fused_paths_bit_equal(torch_dev, name, knob, monkeypatch):
    """F_l y2 formed in the up sweep's prologue adds every row's entries in
    the same order as the separate launch (the 27-point case has F rows
    longer than one batch of four entries), E_l z1 from the values the down
    sweep filed in E_l's entry order equals the product over gathers of z1,
    and the small-level interface
    step computes the same sums from LDS copies of W_l and H_l as from
    global memory: the applies agree bit for bit."""
    torch = torch_dev
    w, kw = _case(name)
    st = _oracle_setup(w, kw)
    x = np.random.default_rng(9).standard_normal(w.n)
    if w.is_complex:
        x = x + 1j * np.random.default_rng(10).standard_normal(w.n)
    xd = torch.from_numpy(x).cuda()
    out = []
    for env in ({}, {knob: "1"}):
        for k, v in env.items():
            monkeypatch.setenv(k, v)
        ctx = _ctx_explicit(torch, w, st)
        yd = torch.empty_like(xd)
        ctx.apply(xd, yd)
        torch.cuda.synchronize()
        out.append(yd.clone())
        ctx.close()
    assert torch.equal(out[0], out[1])


@pytest.mark.parametrize("lfil", [2, 6, 12, 16, 24])
def test_apply_matches_oracle_across_row_lengths(torch_dev, lfil):
    """ILUT fill caps that put the longest factor row in each slot bucket of
    the streamed layout (4, 8, 12, 16) and past it (register-prefetch
    kernel), on a nonsymmetric 3-D operator with 27 subdomains."""
    torch = torch_dev
    r, c, v = wl.convdiff3d(14, (0.3, 0.2, 0.1))
    w = wl.Workload("cd14", (14, 14, 14), r, c, v, levels=3, nparts=27, rank=6, ilu="ilut",
                    drop_tol=0.0, lfil=lfil, restart=30, tol=1e-8)
    st = _oracle_setup(w, dict(ilu="ilut", drop_tol=0.0, lfil=lfil, rank=6, dense_max=400))
    maxrow = max(int(np.max(np.diff(lv.Lf.indptr))) if lv.d else 0 for lv in st.levels)
    print(f"[apply parity] lfil={lfil} longest L row {maxrow}", flush=True)
    ctx = _ctx_explicit(torch, w, st)
    x = np.random.default_rng(30 + lfil).standard_normal(w.n)
    ref = og.apply(st, x)
    xd = torch.from_numpy(x).cuda()
    yd = torch.empty_like(xd)
    ctx.apply(xd, yd)
    torch.cuda.synchronize()
    assert_close(yd.cpu().numpy(), ref, APPLY_TOL_F64)
    ctx.close()
