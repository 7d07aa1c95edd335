"""A partition given by the caller (gs_opts.part_*, checked by
gs_partition_check; host only, no device).  On the library's own
partitions the blocks derived as connected components of every segment are
the partitioner's blocks, and every malformed partition is rejected with a
message: perm not a permutation, level starts not rising from 0 to n, an
empty segment, blocks that do not tile their segment, a block of B_l split
in two (coupled by entries of A: B_l must be block diagonal), and a
component that is not contiguous in perm."""
import numpy as np
import pytest

from paper_2205_03224_amd import workloads as wl


@pytest.fixture(scope="module")
def gm():
    from paper_2205_03224_amd import gemslr
    return gemslr


def _grid_case(gm, N=12, nparts=8, levels=3):
    rp, ci, _ = wl.convdiff3d(N)
    perm, ls, L, blocks = gm.partition_grid((N, N, N), nparts, levels, rp, ci)
    return rp, ci, perm, ls, L, blocks


@pytest.mark.parametrize("N,nparts,levels", [(12, 8, 3), (16, 8, 2), (10, 27, 3)])
def test_components_reproduce_the_partitioner_blocks(gm, N, nparts, levels):
    rp, ci, perm, ls, L, blocks = _grid_case(gm, N, nparts, levels)
    got = gm.partition_check(rp, ci, perm, ls, L)
    for l in range(L):
        assert np.array_equal(got[l], blocks[l]), l
    # C_last: the derived blocks tile the segment and refine or equal the
    # partitioner's block-Jacobi cut
    assert got[L][0] == ls[L] and got[L][-1] == ls[L + 1]
    assert set(blocks[L].tolist()) <= set(got[L].tolist())
    # the given blocks pass unchanged
    same = gm.partition_check(rp, ci, perm, ls, L, blocks)
    for l in range(L + 1):
        assert np.array_equal(same[l], blocks[l])


def test_graph_partition_blocks(gm):
    rp, ci, _ = wl.convdiff3d(10)
    perm, ls, L, blocks = gm.partition_graph(8, 3, rp, ci)
    got = gm.partition_check(rp, ci, perm, ls, L, blocks)
    for l in range(L + 1):
        assert np.array_equal(got[l], blocks[l])


def _expect_error(gm, text, *args):
    with pytest.raises(gm.GemslrError) as e:
        gm.partition_check(*args)
    assert text in str(e.value), str(e.value)


def test_rejects_malformed_partitions(gm):
    rp, ci, perm, ls, L, blocks = _grid_case(gm)
    n = len(perm)
    bad = perm.copy()
    bad[1] = bad[0]
    _expect_error(gm, "not a permutation", rp, ci, bad, ls, L)
    bad_ls = ls.copy()
    bad_ls[-1] = n - 1
    _expect_error(gm, "from 0 to n", rp, ci, perm, bad_ls, L)
    empty = ls.copy()
    empty[2] = empty[1]
    _expect_error(gm, "at least one row", rp, ci, perm, empty, L)
    short = [b.copy() for b in blocks]
    short[0] = short[0][:-1]
    _expect_error(gm, "cover their segment", rp, ci, perm, ls, L, short)
    # a subdomain of B_0 cut in half: its halves are coupled through A
    split = [b.copy() for b in blocks]
    b0 = split[0]
    split[0] = np.sort(np.append(b0, (b0[0] + b0[1]) // 2))
    _expect_error(gm, "coupled", rp, ci, perm, ls, L, split)
    # two rows of different subdomains swapped: their components interleave
    sw = perm.copy()
    i, j = blocks[0][0], blocks[0][1]
    sw[i], sw[j] = sw[j], sw[i]
    _expect_error(gm, "not contiguous", rp, ci, sw, ls, L)
