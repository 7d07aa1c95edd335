"""Setup without grid coordinates (nested-dissection partition) on a
randomly relabelled 3-D convection-diffusion operator: the library's native
setup against an oracle setup built on the oracle's own algebraic partition
(identical partitions, so identical ILUT factors and -- with dense low-rank
terms at these sizes -- M^{-1} to rounding), and a full solve."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import gemslr as og
from oracle import partition as op
from paper_2205_03224_amd import workloads as wl
from tests.abi_helpers import assert_close, oracle_levels, relerr

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_03224_amd import gemslr  # noqa: F401
    return torch


def _relabelled(N, seed):
    r, c, v = wl.convdiff3d(N, (0.1, 0.2, 0.3))
    n = N ** 3
    A = sp.csr_matrix((v, c, r), shape=(n, n))
    p = np.random.default_rng(seed).permutation(n)
    B = A[p][:, p].tocsr()
    B.sort_indices()
    return B.indptr.astype(np.int64), B.indices.astype(np.int32), B.data


def test_algebraic_setup_apply_matches_oracle(torch_dev):
    torch = torch_dev
    from paper_2205_03224_amd import gemslr
    N, p, lev = 14, 8, 3
    rp, ci, v = _relabelled(N, 11)
    n = N ** 3
    part = op.algebraic(n, p, lev, rp, ci)
    print(f"[algebraic] n={n} L={part.nlevels} starts={part.level_start.tolist()}", flush=True)
    st = og.setup(rp, ci, v, part, ilu="ilut", drop_tol=1e-3, lfil=10, rank=6)
    # the library's own partition and factors ...
    ctx = gemslr.Context(0)
    ctx.setup(rp, ci, v, lev, p, 6, 1e-3, lfil=10)
    assert np.array_equal(ctx.perm(), part.perm)
    for l, lv in enumerate(st.levels):
        got = ctx.level(l)
        assert np.array_equal(got["U"][0], lv.Uf.indptr)
        assert_close(got["U"][2], lv.Uf.data, 1e-12, what=f"U values level {l}")
    # ... and the same M^{-1} when the low-rank terms are the oracle's
    ctx2 = gemslr.Context(0)
    ctx2.setup_explicit(rp, ci, v, st.perm, oracle_levels(st))
    x = np.random.default_rng(3).standard_normal(n)
    xd = torch.from_numpy(x).cuda()
    yd = torch.empty_like(xd)
    ctx2.apply(xd, yd)
    torch.cuda.synchronize()
    assert_close(yd.cpu().numpy(), og.apply(st, x), 1e-10, what="apply")
    # full solve with the native setup
    b = torch.from_numpy(sp.csr_matrix((v, ci, rp)) @ np.ones(n)).cuda()
    xs = torch.zeros_like(b)
    res = ctx.solve(b, xs, 1e-8)
    print(f"  solve its {res['its']} relres {res['relres']:.2e}", flush=True)
    assert res["converged"]
    assert relerr(xs.cpu().numpy(), np.ones(n)) <= 1e-5
    ctx.close()
    ctx2.close()
