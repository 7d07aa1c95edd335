"""gs_setup with a partition given by the caller (gs_opts.part_*): the
library's own grid partition handed back to it, with its block lists or with
the blocks left to be derived (connected components), gives the same
permutation and bit-identical applies as the native setup, which partitions
by itself; a partition whose B_0 blocks are coupled is refused.  Also the
seeded start of the learned-start network (gs_mlp_create)."""
import numpy as np
import pytest

from paper_2205_03224_amd import workloads as wl

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2205_03224_amd import gemslr  # noqa: F401  (fails loudly if unbuilt)
    return torch


def test_user_partition_matches_native_setup(torch_dev):
    torch = torch_dev
    from paper_2205_03224_amd import gemslr
    w = wl.convdiff3d_64(N=20, nparts=27)
    kw = dict(lfil=10)
    native = gemslr.Context(0)
    native.setup(w.rowptr, w.col, w.val, w.levels, w.nparts, 8, 1e-3, grid_dims=w.dims, **kw)
    perm, ls, L, blocks = gemslr.partition_grid(w.dims, w.nparts, w.levels, w.rowptr, w.col)
    rs = np.random.default_rng(3)
    x = torch.from_numpy(rs.standard_normal(w.n)).cuda()
    y0 = torch.empty_like(x)
    native.apply(x, y0)
    for part in ((perm, ls, L, blocks), (perm, ls, L)):
        print(f"[user-partition] blocks given: {len(part) == 4}", flush=True)
        ctx = gemslr.Context(0)
        ctx.setup(w.rowptr, w.col, w.val, 0, 0, 8, 1e-3, partition=part, **kw)
        assert np.array_equal(ctx.perm(), perm)
        y = torch.empty_like(x)
        ctx.apply(x, y)
        torch.cuda.synchronize()
        assert torch.equal(y, y0)
        ctx.close()
    native.close()


def test_user_partition_with_coupled_blocks_is_refused(torch_dev):
    from paper_2205_03224_amd import gemslr
    w = wl.convdiff3d_64(N=12, nparts=8)
    perm, ls, L, blocks = gemslr.partition_grid(w.dims, w.nparts, w.levels, w.rowptr, w.col)
    split = [b.copy() for b in blocks]
    split[0] = np.sort(np.append(split[0], (split[0][0] + split[0][1]) // 2))
    ctx = gemslr.Context(0)
    with pytest.raises(gemslr.GemslrError) as e:
        ctx.setup(w.rowptr, w.col, w.val, 0, 0, 8, 1e-3, partition=(perm, ls, L, split))
    assert "coupled" in str(e.value)
    # the context stays usable: a valid setup afterwards works
    ctx.setup(w.rowptr, w.col, w.val, 0, 0, 8, 1e-3, partition=(perm, ls, L, blocks))
    ctx.close()


def test_mlp_seeded_start(torch_dev):
    from paper_2205_03224_amd import gemslr
    dims = (38, 64, 32)
    a = gemslr.Mlp(*dims, seed=5).get_params()
    b = gemslr.Mlp(*dims, seed=5).get_params()
    c = gemslr.Mlp(*dims, seed=6).get_params()
    assert np.array_equal(a, b)
    assert not np.array_equal(a, c)
    o = 0
    for fan_in, fan_out in ((38, 64), (64, 64), (64, 32)):
        lim = np.sqrt(6.0 / (fan_in + fan_out))
        W = a[o:o + fan_in * fan_out]
        o += fan_in * fan_out
        bias = a[o:o + fan_out]
        o += fan_out
        assert np.all(np.abs(W) <= lim * (1 + 1e-6))
        assert np.all(bias == 0)
        # uniform on [-lim, lim): mean 0, variance lim^2 / 3 (loose, sampling)
        assert abs(W.mean()) < 0.1 * lim
        assert abs(W.var() / (lim * lim / 3) - 1) < 0.15
    assert o == len(a)
