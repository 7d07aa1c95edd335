"""Error behaviour of the C ABI on a device context.  Every failure here is
forced from the host with a crafted input; no kernel is made to fault."""
import numpy as np
import pytest
import scipy.sparse as sp

from paper_2205_03224_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def G():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_03224_amd import gemslr
    return gemslr


def test_apply_and_solve_before_setup(G):
    import torch
    ctx = G.Context(0)
    x = torch.zeros(16, dtype=torch.float64, device="cuda")
    y = torch.zeros_like(x)
    with pytest.raises(G.GemslrError) as e:
        ctx.apply(x, y)
    assert e.value.code == G.GS_ESTATE
    with pytest.raises(G.GemslrError) as e:
        ctx.solve(x, y, 1e-8)
    assert e.value.code == G.GS_ESTATE
    ctx.close()


def test_aliasing_and_bad_csr(G):
    import torch
    r, c, v = wl.laplace2d(8)
    ctx = G.Context(0)
    ctx.setup(r, c, v, 2, 4, 4, 0.0, ilu="ilu0", grid_dims=(8, 8))
    x = torch.ones(64, dtype=torch.float64, device="cuda")
    with pytest.raises(G.GemslrError) as e:
        ctx.apply(x, x)
    assert e.value.code == G.GS_EINVAL
    for wrong in (torch.ones(63, dtype=torch.float64, device="cuda"),
                  torch.ones(64, dtype=torch.float32, device="cuda"),
                  torch.ones(64, dtype=torch.float64)):
        with pytest.raises(ValueError):   # extent / dtype / device checked in the binding
            ctx.apply(wrong, torch.empty(64, dtype=torch.float64, device="cuda"))
    bad = c.copy()
    bad[0] = 63  # first row's columns no longer ascending
    with pytest.raises(G.GemslrError) as e:
        ctx.setup(r, bad, v, 2, 4, 4, 0.0, ilu="ilu0", grid_dims=(8, 8))
    assert e.value.code == G.GS_EINVAL
    with pytest.raises(G.GemslrError) as e:   # grid does not match n
        ctx.setup(r, c, v, 2, 4, 4, 0.0, ilu="ilu0", grid_dims=(8, 9))
    assert e.value.code == G.GS_EINVAL
    ctx.close()


def test_zero_pivot(G):
    r, c, v = wl.laplace2d(8)
    v = v.copy()
    v[r[0]] = 0.0  # A[0,0] = 0: first row of the first subdomain block
    ctx = G.Context(0)
    with pytest.raises(G.GemslrError) as e:
        ctx.setup(r, c, v, 2, 4, 4, 0.0, ilu="ilu0", grid_dims=(8, 8))
    assert e.value.code == G.GS_EZEROPIVOT
    ctx.close()


def test_singular_correction(G):
    # 1-D chain of 5 points, 2 parts: cut at x = 3, B = {0,1,2} u {4}, C = {3}.
    # E B^{-1} F = (B1^{-1})_{22} + (B2^{-1})_{00} = 3/4 + 1/2; choosing
    # a_33 = 5/4 makes the Schur complement zero, so G = E B^{-1} F C^{-1} = 1
    # and I - R is singular.
    n = 5
    A = sp.diags([[-1.0] * 4, [2.0, 2.0, 2.0, 1.25, 2.0], [-1.0] * 4], [-1, 0, 1]).tocsr()
    A.sort_indices()
    ctx = G.Context(0)
    with pytest.raises(G.GemslrError) as e:
        ctx.setup(A.indptr, A.indices, A.data, 1, 2, 1, 0.0, ilu="ilu0", grid_dims=(n,))
    assert e.value.code == G.GS_ESINGULAR
    ctx.close()


def test_not_converged_status(G):
    import torch
    w = wl.laplace2d_32()
    ctx = G.Context(0)
    ctx.setup(w.rowptr, w.col, w.val, w.levels, w.nparts, 2, 0.0, ilu="ilu0",
              grid_dims=w.dims, maxit=2, fgmres_restart=30)
    b = torch.from_numpy(w.b).cuda()
    x = torch.zeros_like(b)
    info = ctx.solve(b, x, 1e-12)
    assert info["status"] == G.GS_NOT_CONVERGED and info["its"] == 2
    assert not info["converged"] and info["relres"] > 1e-12
    ctx.close()


def test_rank_limit_rejected_before_setup_work(G):
    """k = min(rank, s_l) above 1024 on some level is refused right after the
    partition (before factorisation or Arnoldi)."""
    import time
    w = wl.convdiff3d_64(N=20, nparts=8)
    ctx = G.Context(0)
    t0 = time.perf_counter()
    with pytest.raises(G.GemslrError) as e:
        ctx.setup(w.rowptr, w.col, w.val, w.levels, w.nparts, 1100, w.drop_tol, lfil=w.lfil,
                  grid_dims=w.dims)
    assert e.value.code == G.GS_EINVAL and "1024" in str(e.value)
    assert time.perf_counter() - t0 < 5.0
    ctx.close()
