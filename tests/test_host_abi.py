"""CPU-only checks of the C-ABI library: it loads, exports every symbol that
include/gemslr.h declares, and its host stages (geometric partition, ILU)
agree with the oracle -- bit for bit on integer structure, to rounding on
values.  No device call is made here."""
import os
import re

import numpy as np
import pytest
import scipy.sparse as sp

from paper_2205_03224_amd import gemslr as G
from paper_2205_03224_amd import workloads as wl
from oracle import ilu as oilu
from oracle import partition as opart

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    src = open(os.path.join(ROOT, "include", "gemslr.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gs_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = G.lib()
    names = _declared_symbols()
    assert len(names) >= 15
    for name in names:
        assert hasattr(L, name), name
    # the binding declares a signature for every exported entry point
    assert sorted(n for n, _, _ in G.SIGNATURES) == names


@pytest.mark.parametrize("dims,p,lev", [((32, 32), 4, 2), ((20, 20, 20), 27, 3),
                                        ((17, 13, 11), 8, 5), ((16, 16), 1, 3)])
def test_partition_bit_exact(dims, p, lev):
    if len(dims) == 2:
        r, c, v = wl.laplace2d(dims[0])
    else:
        r, c, v = wl._assemble(dims, np.full(int(np.prod(dims)), 6.0),
                               [np.full(int(np.prod(dims)), -1.0)] * 3,
                               [np.full(int(np.prod(dims)), -1.0)] * 3)
    perm, ls, L, blocks = G.partition_grid(dims, p, lev, r, c)
    ref = opart.wirebasket(dims, p, lev, r, c)
    assert L == ref.nlevels
    assert np.array_equal(perm, ref.perm)
    assert np.array_equal(ls, ref.level_start)
    assert len(blocks) == len(ref.blocks)
    for a, b in zip(blocks, ref.blocks):
        assert np.array_equal(a, b)


def _block(w, size):
    A = sp.csr_matrix((w[2], w[1], w[0]))
    B = A[:size, :size].tocsr()
    B.sort_indices()
    return B


@pytest.mark.parametrize("kind,tau,lfil", [("ilu0", 0, 0), ("ilut", 1e-3, 10),
                                           ("ilut", 1e-2, 3), ("ilut", 0.0, 10 ** 6)])
def test_ilu_matches_oracle_real(kind, tau, lfil):
    B = _block(wl.convdiff3d(10, (0.1, 0.2, 0.3)), 1000)
    (lr, lc, lv), (ur, uc, uv) = G.ilu(B.indptr, B.indices, B.data, kind, tau, lfil)
    Lo, Uo = oilu.factor(B, kind, tau, lfil)
    assert np.array_equal(lr, Lo.indptr) and np.array_equal(lc, Lo.indices)
    assert np.array_equal(ur, Uo.indptr) and np.array_equal(uc, Uo.indices)
    # same operation order on both sides: equal to the last bit
    assert np.array_equal(lv, Lo.data) and np.array_equal(uv, Uo.data)


def test_ilu_matches_oracle_complex():
    B = _block(wl.helmholtz3d(9, 0.39), 729)
    (lr, lc, lv), (ur, uc, uv) = G.ilu(B.indptr, B.indices, B.data, "ilut", 1e-4, 10)
    Lo, Uo = oilu.factor(B, "ilut", 1e-4, 10)
    assert np.array_equal(lc, Lo.indices) and np.array_equal(uc, Uo.indices)
    np.testing.assert_allclose(lv, Lo.data, rtol=1e-13, atol=1e-15)
    np.testing.assert_allclose(uv, Uo.data, rtol=1e-13, atol=1e-15)


def test_host_errors():
    r, c, v = wl.laplace2d(4)
    with pytest.raises(G.GemslrError) as e:
        G.partition_grid((4, 4), 3, 2, r, c)      # 3 is not a square
    assert e.value.code == G.GS_EINVAL
    bad_c = c.copy()
    bad_c[1], bad_c[2] = bad_c[2], bad_c[1]       # unsorted row
    with pytest.raises(G.GemslrError) as e:
        G.partition_grid((4, 4), 4, 2, r, bad_c)
    assert e.value.code == G.GS_EINVAL
    D = sp.csr_matrix(np.array([[1.0, 1.0], [1.0, 1.0]]))
    with pytest.raises(G.GemslrError) as e:
        G.ilu(D.indptr, D.indices, D.data, "ilu0")
    assert e.value.code == G.GS_EZEROPIVOT


def test_host_only_context_refuses_device_work():
    ctx = G.Context(device=-1, stream=0)
    r, c, v = wl.laplace2d(8)
    with pytest.raises(G.GemslrError) as e:
        ctx.setup(r, c, v, 2, 4, 4, 0.0, grid_dims=(8, 8))
    assert e.value.code == G.GS_ESTATE
    ctx.close()


def _diag_level(d, s, k):
    """One level of an explicit setup with identity factors and empty E, F;
    W zero (s x k), H zero (k x k)."""
    eye = (np.arange(d + 1, dtype=np.int64), np.arange(d, dtype=np.int32), np.ones(d))
    empty = (np.zeros(d + 1, np.int64), np.zeros(0, np.int32), np.zeros(0))
    lv = {"d": d, "block_ptr": np.array([0, d], np.int64), "L": empty, "U": eye}
    if s > 0:
        lv.update(E=(np.zeros(s + 1, np.int64), np.zeros(0, np.int32), np.zeros(0)),
                  F=(np.zeros(d + 1, np.int64), np.zeros(0, np.int32), np.zeros(0)),
                  W=np.zeros((s, k)), H=np.zeros((k, k)))
    return lv


@pytest.mark.parametrize("block,csr,msg", [
    ("E", ([0, 2, 1, 2], [0, 1], [1.0, 1.0]), "E of level 0: rowptr not monotone"),
    ("E", ([1, 1, 1, 1], [], []), "E of level 0: rowptr[0] != 0"),
    ("F", ([0, 1, 1, 1, 1], [3], [1.0]), "F of level 0: column out of range"),
    ("L", ([0, 0, 2, 1, 2], [0, 1], [1.0, 1.0]), "L of level 0: rowptr not monotone"),
    ("E", ([0, 1, 1, 2], [0, 3], [1.0, 2.0]), None),
    ("F", ([0, 1, 1, 1, 2], [2, 0], [1.0, 2.0]), None),
])
def test_explicit_setup_checks_level_blocks(block, csr, msg):
    """Every CSR block of an explicit level is checked before anything reads
    it (rowptr from 0 and monotone, columns within the block's width: d for
    E_l, s for F_l), so a malformed one is refused with GS_EINVAL naming the
    block and level rather than read out of bounds; well-formed E_l and F_l
    with entries are accepted (host-only context: validation only)."""
    d, s = 4, 3
    n = d + s
    A = sp.identity(n, format="csr")
    perm = np.arange(n, dtype=np.int64)
    lv0 = _diag_level(d, s, 0)
    lv0[block] = tuple(np.asarray(a, dt) for a, dt in zip(csr, (np.int64, np.int32, float)))
    ctx = G.Context(-1)
    try:
        levels = [lv0, _diag_level(s, 0, 0)]
        if msg is None:
            ctx.setup_explicit(A.indptr, A.indices, A.data, perm, levels)
        else:
            with pytest.raises(G.GemslrError) as e:
                ctx.setup_explicit(A.indptr, A.indices, A.data, perm, levels)
            assert e.value.code == G.GS_EINVAL
            assert msg in str(e.value)
    finally:
        ctx.close()


def test_explicit_setup_rejects_rank_above_1024():
    """The low-rank kernels take k <= 1024 per level (as gs_setup's rank check
    says); an explicit level with k = 1025 <= s is refused with GS_EINVAL,
    k = 1024 is accepted (host-only context: validation only)."""
    d, s = 8, 1100
    n = d + s
    A = sp.identity(n, format="csr")
    perm = np.arange(n, dtype=np.int64)
    for k, ok in ((1024, True), (1025, False)):
        ctx = G.Context(-1)
        try:
            levels = [_diag_level(d, s, k), _diag_level(s, 0, 0)]
            if ok:
                ctx.setup_explicit(A.indptr, A.indices, A.data, perm, levels)
            else:
                with pytest.raises(G.GemslrError) as e:
                    ctx.setup_explicit(A.indptr, A.indices, A.data, perm, levels)
                assert e.value.code == G.GS_EINVAL
                assert "1024" in str(e.value)
        finally:
            ctx.close()
