"""gs_apply_noalloc: the apply with every scratch buffer in the library's
static device region, for callers that cannot allocate.  Checked through the
C ABI against gs_apply of the same context (the same kernels, so bit for bit)
and against the oracle entry by entry, on two calls in a row where the second
runs a smaller system (the region then holds the first call's leftovers), and
with a system whose scratch exceeds the region (rejected, nothing run)."""
import numpy as np
import pytest

from oracle import gemslr as og
from oracle import partition as opart
from paper_2205_03224_amd import workloads as wl
from tests.abi_helpers import assert_close, oracle_levels

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_03224_amd import gemslr  # noqa: F401  (fails loudly if unbuilt)
    return torch


def _explicit(w, kw):
    from paper_2205_03224_amd import gemslr
    part = opart.wirebasket(w.dims, w.nparts, w.levels, w.rowptr, w.col)
    st = og.setup(w.rowptr, w.col, w.val, part, **kw)
    ctx = gemslr.Context(0)
    ctx.setup_explicit(w.rowptr, w.col, w.val, st.perm, oracle_levels(st))
    return ctx, st


def test_noalloc_matches_apply_two_calls(torch_dev):
    torch = torch_dev
    cases = [
        (wl.convdiff3d_64(N=24, nparts=8),
         dict(ilu="ilut", drop_tol=1e-3, lfil=10, rank=8, dense_max=100)),
        (wl.helmholtz3d_128(N=16, nparts=8, levels=5),
         dict(ilu="ilut", drop_tol=1e-4, lfil=10, rank=8, dense_max=100)),
        (wl.laplace2d_32(), dict(ilu="ilu0", rank=8)),
    ]
    assert cases[1][0].n < cases[0][0].n and cases[2][0].n < cases[1][0].n
    for i, (w, kw) in enumerate(cases):
        print(f"[noalloc] call {i}: {w.name} n={w.n}", flush=True)
        ctx, st = _explicit(w, kw)
        rs = np.random.default_rng(70 + i)
        x = rs.standard_normal(w.n)
        if w.is_complex:
            x = x + 1j * rs.standard_normal(w.n)
        xd = torch.from_numpy(x).cuda()
        y0 = torch.empty_like(xd)
        y1 = torch.full_like(xd, float("nan"))
        ctx.apply_noalloc(xd, y1)
        ctx.apply(xd, y0)
        torch.cuda.synchronize()
        assert torch.equal(y0, y1), "gs_apply_noalloc differs from gs_apply"
        assert_close(y1.cpu().numpy(), og.apply(st, x), 1e-10, what=f"call {i} vs oracle")
        ctx.close()


def test_noalloc_rejects_scratch_beyond_region(torch_dev):
    """A one-level block-diagonal preconditioner of 9.6M float64 unknowns
    needs a 77 MB working vector: rejected with GS_EINVAL, while gs_apply of
    the same context still runs."""
    torch = torch_dev
    from paper_2205_03224_amd import gemslr
    nb, bs = 1200, 8000
    n = nb * bs
    rp = np.arange(n + 1, dtype=np.int64)
    ci = np.arange(n, dtype=np.int32)
    val = np.full(n, 2.0)
    lev = {"d": n, "block_ptr": np.arange(0, n + 1, bs, dtype=np.int64),
           "L": (np.zeros(n + 1, np.int64), np.zeros(0, np.int32), np.zeros(0)),
           "U": (rp, ci, val)}
    ctx = gemslr.Context(0)
    ctx.setup_explicit(rp, ci, val, np.arange(n, dtype=np.int64), [lev])
    xd = torch.ones(n, dtype=torch.float64, device="cuda")
    yd = torch.empty_like(xd)
    with pytest.raises(gemslr.GemslrError) as e:
        ctx.apply_noalloc(xd, yd)
    assert e.value.code == gemslr.GS_EINVAL and "static region" in str(e.value)
    ctx.apply(xd, yd)
    torch.cuda.synchronize()
    assert torch.all(yd == 0.5)
    ctx.close()
