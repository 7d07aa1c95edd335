"""Algebraic (nested-dissection) partitioner: the oracle's bisection pinned
to closed forms, the level structure's invariants, and the library's host
implementation equal to the oracle's, integer for integer."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import partition as op
from paper_2205_03224_amd import workloads as wl


def _path(n):
    rows = np.arange(n)
    A = sp.diags([np.full(n - 1, -1.0), np.full(n, 2.0), np.full(n - 1, -1.0)], [-1, 0, 1]).tocsr()
    A.sort_indices()
    return A.indptr.astype(np.int64), A.indices.astype(np.int32), A.data


def _bisect(rp, ci, verts):
    n = len(rp) - 1
    adj = op._adjacency(n, rp, ci)
    inP = np.zeros(n, dtype=bool)
    inP[verts] = True
    return op._bisect(adj, inP, list(verts))


def test_bisect_path_closed_form():
    # BFS from vertex 0 (already peripheral): levels are the indices, the
    # median vertex n//2 is the separator
    for n in (2, 7, 10, 31):
        rp, ci, _ = _path(n)
        A, B, S = _bisect(rp, ci, np.arange(n))
        m = n // 2 if n // 2 < n - 1 else n - 2
        assert S == [m] and A == list(range(m)) and B == list(range(m + 1, n))


def test_bisect_grid_diagonal_separator():
    # 2-D grid: BFS levels from the corner are i + j; the separator is the
    # anti-diagonal i + j = m (all of it has a neighbour at m + 1)
    N = 9
    r, c, _ = wl.laplace2d(N)
    A, B, S = _bisect(r, c, np.arange(N * N))
    lev = np.add.outer(np.arange(N), np.arange(N)).ravel()  # index = x + N y
    order = sorted(range(N * N), key=lambda v: (lev[v], v))
    m = lev[order[N * N // 2]]
    assert S == [v for v in range(N * N) if lev[v] == m]
    assert A == [v for v in range(N * N) if lev[v] < m]
    assert B == [v for v in range(N * N) if lev[v] > m]


def test_bisect_disconnected_balances_components():
    # chains of lengths 5, 3, 4 (vertices 0-4, 5-7, 8-11), no separator:
    # 5 -> first half, 4 -> second, 3 -> second (4 < 5)
    blocks = [_path(k)[0:2] for k in (5, 3, 4)]
    A = sp.block_diag([sp.csr_matrix((np.ones(len(ci)), ci, rp)) for rp, ci in blocks]).tocsr()
    A.sort_indices()
    a, b, s = _bisect(A.indptr, A.indices, np.arange(12))
    assert s == [] and a == list(range(5)) and b == list(range(5, 12))


def _relabelled_grid(N, seed):
    r, c, v = wl.convdiff3d(N, (0.1, 0.2, 0.3))
    n = N ** 3
    A = sp.csr_matrix((v, c, r), shape=(n, n))
    p = np.random.default_rng(seed).permutation(n)
    B = A[p][:, p].tocsr()
    B.sort_indices()
    return B.indptr.astype(np.int64), B.indices.astype(np.int32), B.data


@pytest.mark.parametrize("N,p,lev", [(12, 8, 3), (14, 16, 3), (10, 4, 2)])
def test_algebraic_structure_invariants(N, p, lev):
    rp, ci, _ = _relabelled_grid(N, N)
    n = N ** 3
    P = op.algebraic(n, p, lev, rp, ci)
    assert np.array_equal(np.sort(P.perm), np.arange(n))
    assert P.level_start[0] == 0 and P.level_start[-1] == n
    assert P.level_start[-2] < n  # C_last is not empty
    A = sp.csr_matrix((np.ones(len(ci)), ci, rp), shape=(n, n))
    Ap = (abs(A) + abs(A.T))[P.perm][:, P.perm].tocoo()
    # no edge between two different blocks of one level (p-way separator)
    lab = np.full(n, -1)
    for l in range(P.nlevels + 1):
        b = P.blocks[l]
        for i in range(len(b) - 1):
            lab[b[i]:b[i + 1]] = 1000000 * l + i
    lvl = np.searchsorted(P.level_start, np.arange(n), side="right") - 1
    same_level = lvl[Ap.row] == lvl[Ap.col]
    assert np.all(lab[Ap.row][same_level] == lab[Ap.col][same_level])


@pytest.mark.parametrize("N,p,lev,seed", [(12, 8, 3, 1), (16, 16, 3, 2), (11, 32, 4, 3),
                                          (9, 1, 2, 4), (13, 2, 3, 5)])
def test_library_partition_equals_oracle(N, p, lev, seed):
    from paper_2205_03224_amd import gemslr
    rp, ci, _ = _relabelled_grid(N, seed)
    perm, ls, L, blocks = gemslr.partition_graph(p, lev, rp, ci)
    P = op.algebraic(N ** 3, p, lev, rp, ci)
    assert L == P.nlevels
    assert np.array_equal(perm, P.perm)
    assert np.array_equal(ls, P.level_start)
    for a, b in zip(blocks, P.blocks):
        assert np.array_equal(a, b)


def test_partition_graph_rejects_non_power_of_two():
    from paper_2205_03224_amd import gemslr
    rp, ci, _ = _path(20)
    with pytest.raises(gemslr.GemslrError):
        gemslr.partition_graph(3, 2, rp, ci)
    with pytest.raises(ValueError):
        op.algebraic(20, 6, 2, rp, ci)
