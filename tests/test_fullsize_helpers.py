"""The full-size test's oracle setup factors each level a run of blocks at a
time in worker processes; on a smaller grid that must give exactly the
factors of oracle.gemslr.setup (the same rows, the same operations)."""
import numpy as np

from oracle import gemslr as og
from oracle import partition as opart
from paper_2205_03224_amd import workloads as wl
from tests.fullsize_helpers import oracle_setup_parallel


def test_parallel_factors_equal_oracle_setup():
    w = wl.convdiff3d_64(N=24, nparts=27)
    part = opart.wirebasket(w.dims, w.nparts, w.levels, w.rowptr, w.col)
    st = oracle_setup_parallel(w.rowptr, w.col, w.val, part, (8, 8, 8), tau=w.drop_tol,
                               lfil=w.lfil, seed=3, workers=4, run_rows=500)
    ref = og.setup(w.rowptr, w.col, w.val, part, ilu="ilut", drop_tol=w.drop_tol, lfil=w.lfil,
                   rank=8, dense_max=100)
    assert len(st.levels) == len(ref.levels)
    for a, b in zip(st.levels, ref.levels):
        assert (a.start, a.d, a.s) == (b.start, b.d, b.s)
        for x, y in ((a.Lf, b.Lf), (a.Uf, b.Uf), (a.E, b.E), (a.F, b.F)):
            assert np.array_equal(x.indptr, y.indptr)
            assert np.array_equal(x.indices, y.indices)
            assert np.array_equal(x.data, y.data)
    for lv in st.levels[:-1]:
        k = lv.W.shape[1]
        assert np.allclose(lv.W.T @ lv.W, np.eye(k), atol=1e-12)
        assert np.max(np.abs(np.linalg.eigvals(lv.R))) < 0.5
