"""GPU parity of the inner GMRES at the root level (Alg. 2, l = 0): the apply
with m inner steps on S_hat_0 against the oracle's, on the same setup data.

The oracle takes the GMRES minimiser from its definition (least squares over
an orthonormal Krylov basis), the device path from Arnoldi plus plane
rotations, so the two agree up to rounding amplified by the conditioning of
the small least-squares problem; entry by entry (tests/abi_helpers.assert_close)
1e-8 bounds that with margin for m <= 5 on these operators (observed
differences in norm are near 1e-13).
"""
import numpy as np
import pytest

from oracle import gemslr as og
from tests.abi_helpers import assert_close, relerr
from tests.test_gpu_parity import _case, _ctx_explicit, _oracle_setup

pytestmark = pytest.mark.gpu

INNER_TOL = 1e-8


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_03224_amd import gemslr  # noqa: F401
    return torch


@pytest.mark.parametrize("name", ["laplace2d_32", "convdiff3d_20_p27", "helmholtz3d_16_p8"])
@pytest.mark.parametrize("its", [1, 3, 5])
def test_inner_apply_matches_oracle(torch_dev, name, its):
    torch = torch_dev
    w, kw = _case(name)
    print(f"[inner parity] {name} its={its} n={w.n}", flush=True)
    st = _oracle_setup(w, kw)
    ctx = _ctx_explicit(torch, w, st, inner_gmres_its=its)
    rs = np.random.default_rng(20 + its)
    for trial in range(2):
        x = rs.standard_normal(w.n)
        if w.is_complex:
            x = x + 1j * rs.standard_normal(w.n)
        ref = og.apply(st, x, inner_its=its)
        xd = torch.from_numpy(np.ascontiguousarray(x)).cuda()
        yd = torch.empty_like(xd)
        ctx.apply(xd, yd)
        torch.cuda.synchronize()
        assert_close(yd.cpu().numpy(), ref, INNER_TOL, what=f"trial {trial}")
    ctx.close()


def test_inner_exact_case_breaks_down_cleanly(torch_dev):
    """Exact factors and full rank: one inner step is exact and the next
    Arnoldi direction vanishes; the device path must stop the space there
    (no division by the vanished norm) and return A^{-1} x."""
    torch = torch_dev
    from paper_2205_03224_amd import workloads as wl
    from oracle import partition as opart
    import scipy.sparse as sp
    r, c, v = wl.convdiff3d(7, (.3, .2, .1))
    part = opart.wirebasket((7,) * 3, 8, 3, r, c)
    st = og.setup(r, c, v, part, ilu="ilut", drop_tol=0.0, lfil=10 ** 9, rank=10 ** 9)

    class W:
        pass
    w = W()
    w.rowptr, w.col, w.val = r, c, v
    ctx = _ctx_explicit(torch, w, st, inner_gmres_its=4)
    x = np.random.default_rng(8).standard_normal(len(r) - 1)
    xd = torch.from_numpy(x).cuda()
    yd = torch.empty_like(xd)
    ctx.apply(xd, yd)
    torch.cuda.synchronize()
    A = sp.csr_matrix((v, c, r)).toarray()
    y = yd.cpu().numpy()
    assert np.all(np.isfinite(y))
    assert_close(y, np.linalg.solve(A, x), 1e-8, what="exact case vs A^-1 x")
    ctx.close()


def test_inner_solve_converges_native_setup(torch_dev):
    torch = torch_dev
    from paper_2205_03224_amd import gemslr
    from paper_2205_03224_amd import workloads as wl
    w = wl.convdiff3d_64(N=24, nparts=8)
    its = {}
    for m in (0, 3):
        ctx = gemslr.Context(0)
        ctx.setup(w.rowptr, w.col, w.val, w.levels, w.nparts, 8, w.drop_tol, lfil=w.lfil,
                  grid_dims=w.dims, inner_gmres_its=m)
        b = torch.from_numpy(w.b).cuda()
        x = torch.zeros_like(b)
        res = ctx.solve(b, x, 1e-8)
        print(f"  inner {m}: its {res['its']} relres {res['relres']:.2e}", flush=True)
        assert res["converged"] and res["relres"] <= 1e-8
        its[m] = res["its"]
        ctx.close()
    assert its[3] <= its[0] + 2


def test_inner_rejected_in_mixed_form_and_above_limit(torch_dev):
    from paper_2205_03224_amd import gemslr
    from paper_2205_03224_amd import workloads as wl
    w = wl.laplace2d_32()
    ctx = gemslr.Context(0)
    with pytest.raises(gemslr.GemslrError) as e:
        ctx.setup(w.rowptr, w.col, w.val, w.levels, w.nparts, w.rank, 0.0, ilu="ilu0",
                  grid_dims=w.dims, inner_gmres_its=3, precision="f32")
    assert e.value.code == gemslr.GS_EINVAL
    with pytest.raises(gemslr.GemslrError) as e:
        ctx.setup(w.rowptr, w.col, w.val, w.levels, w.nparts, w.rank, 0.0, ilu="ilu0",
                  grid_dims=w.dims, inner_gmres_its=17)
    assert e.value.code == gemslr.GS_EINVAL
    # a float64 setup with inner steps refuses a switch to float32 and keeps working
    ctx.setup(w.rowptr, w.col, w.val, w.levels, w.nparts, w.rank, 0.0, ilu="ilu0",
              grid_dims=w.dims, inner_gmres_its=2)
    with pytest.raises(gemslr.GemslrError):
        ctx.set_precision("f32")
    import torch
    b = torch.from_numpy(w.b).cuda()
    x = torch.zeros_like(b)
    assert ctx.solve(b, x, 1e-8)["converged"]
    ctx.close()
