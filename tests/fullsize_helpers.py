"""Oracle state for the full-size parity test (the 128^3 convection-diffusion
workload the benchmark times).

The factors are the oracle's own ILU (oracle.ilu.factor) of every level's
diagonal blocks, computed in worker processes a run of consecutive blocks at
a time.  Rows of different blocks never reference each other, so factoring
a run of blocks alone performs, row by row, the operations the whole-level
factorisation performs: the assembled factors are the oracle's.  E_l, F_l
and the permuted matrix are taken from the input matrix exactly as
oracle.gemslr.setup takes them.

The low-rank terms are seeded synthetic data (W_l with orthonormal columns,
R_l with spectral radius below one half, H_l = (I - R_l)^{-1} - I) of the
ranks the benchmark's Arnoldi setup yields, because the oracle's
Krylov-Schur iteration at this size would take far longer than a test may:
the apply (Alg. 2) is defined for any such terms, and the device kernels see
the same shapes as in the benchmark.
"""
from concurrent.futures import ProcessPoolExecutor
import multiprocessing as mp

import numpy as np
import scipy.sparse as sp

from oracle import gemslr as og
from oracle import ilu as oilu
from oracle import lowrank as olr


def _factor_run(args):
    indptr, indices, data, n, kind, tau, lfil = args
    B = sp.csr_matrix((data, indices, indptr), shape=(n, n))
    L, U = oilu.factor(B, kind, tau, lfil)
    return (L.indptr, L.indices, L.data), (U.indptr, U.indices, U.data)


def _runs(blocks, target):
    """Split block boundaries into runs of consecutive blocks of about
    `target` rows; returns row boundaries of the runs."""
    cuts = [0]
    for b in blocks[1:]:
        if b - cuts[-1] >= target or b == blocks[-1]:
            cuts.append(int(b))
    return cuts


def _assemble(pieces, n, dtype):
    Ls, Us = [], []
    for (lp, up), m in pieces:
        Ls.append(sp.csr_matrix((lp[2], lp[1], lp[0]), shape=(m, m)))
        Us.append(sp.csr_matrix((up[2], up[1], up[0]), shape=(m, m)))
    L = sp.block_diag(Ls, format="csr", dtype=dtype)
    U = sp.block_diag(Us, format="csr", dtype=dtype)
    L.sort_indices()
    U.sort_indices()
    assert L.shape == (n, n) and U.shape == (n, n)
    return L, U


def oracle_setup_parallel(rowptr, col, val, part, ks, kind="ilut", tau=1e-3, lfil=10,
                          seed=0, workers=16, run_rows=20000):
    n = len(rowptr) - 1
    A = og.csr(rowptr, col, val, n)
    real = not np.iscomplexobj(val)
    perm = part.perm
    Ap = A[perm][:, perm].tocsr()
    Ap.sort_indices()
    ls = part.level_start
    nl = part.nlevels
    levels = []
    ctx = mp.get_context("spawn")
    with ProcessPoolExecutor(max_workers=workers, mp_context=ctx) as ex:
        for l in range(nl + 1):
            a = int(ls[l])
            b = int(ls[l + 1]) if l < nl else n
            B = Ap[a:b, a:b].tocsr()
            blocks = np.asarray(part.blocks[l]) - a
            if l == nl:
                B = og._block_diag_part(B, blocks)
                E = sp.csr_matrix((0, b - a), dtype=Ap.dtype)
                F = sp.csr_matrix((b - a, 0), dtype=Ap.dtype)
            else:
                E = Ap[b:, a:b].tocsr()
                F = Ap[a:b, b:].tocsr()
            cuts = _runs(blocks, run_rows)
            jobs, sizes = [], []
            for r0, r1 in zip(cuts[:-1], cuts[1:]):
                Bc = B[r0:r1, r0:r1].tocsr()
                Bc.sort_indices()
                jobs.append((Bc.indptr, Bc.indices, Bc.data, r1 - r0, kind, tau, lfil))
                sizes.append(r1 - r0)
            pieces = list(zip(ex.map(_factor_run, jobs), sizes))
            Lf, Uf = _assemble(pieces, b - a, Ap.dtype)
            levels.append(og.Level(a, b - a, n - b, blocks, Lf, Uf, E, F))
    dt = np.float64 if real else np.complex128
    rs = np.random.default_rng(seed)
    for l in range(nl):
        lv = levels[l]
        k = min(ks[l], lv.s)
        X = rs.standard_normal((lv.s, k))
        W, _ = np.linalg.qr(X)
        R = 0.5 * rs.standard_normal((k, k)) / np.sqrt(max(k, 1))
        R *= 0.45 / max(np.max(np.abs(np.linalg.eigvals(R))), 1e-300)
        lv.W = W.astype(dt)
        lv.R = R.astype(dt)
        lv.H = olr.finish(lv.W, lv.R)
        lv.info = {"mode": "synthetic"}
    return og.Setup(n, perm, levels, Ap, real)
