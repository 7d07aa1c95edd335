"""Incomplete LU factorisations of the diagonal blocks B_l (Sec. 2.1, Alg. 1).

Both routines factor a square sparse matrix row by row in the IKJ order and
return (L, U): L strictly lower triangular (its unit diagonal implied) and U
upper triangular including the diagonal, both scipy CSR with sorted columns.
Applied to a block-diagonal B_l they factor every block independently, since
no row references a column of another block.

ILU(0): L and U keep exactly the pattern of B; for every (i, j) in that
pattern (L U)_ij = B_ij.

ILUT(tau, lfil): the dual-threshold factorisation of Saad (1994), cited in
Sec. 2.1.  For row i with tau_i = tau * ||b_i||_2 (original row):
  * eliminate columns k < i in increasing order, including fill created on
    the way: w_k <- w_k / u_kk; if |w_k| < tau_i the multiplier is dropped,
    otherwise w <- w - w_k * u_k (strict upper part of row k of U);
  * afterwards drop every remaining entry with |w_j| < tau_i (the diagonal
    is always kept), then keep the lfil largest-magnitude entries of the L
    part and of the U part separately (ties: lower column index first).
With tau = 0 and lfil >= n this is exact Gaussian elimination without
pivoting.

A zero or non-finite pivot raises ZeroPivotError (no pivot modification).
"""
import heapq

import numpy as np
import scipy.sparse as sp


class ZeroPivotError(ArithmeticError):
    pass


def _rows(B):
    B = sp.csr_matrix(B)
    B.sort_indices()
    return [dict(zip(B.indices[B.indptr[i]:B.indptr[i + 1]].tolist(),
                     B.data[B.indptr[i]:B.indptr[i + 1]].tolist()))
            for i in range(B.shape[0])]


def _to_csr(rows, n, dtype):
    indptr = [0]
    idx, dat = [], []
    for r in rows:
        ks = sorted(r)
        idx.extend(ks)
        dat.extend(r[k] for k in ks)
        indptr.append(len(idx))
    return sp.csr_matrix((np.array(dat, dtype=dtype),
                          np.array(idx, dtype=np.int64),
                          np.array(indptr, dtype=np.int64)), shape=(n, n))


def _check_pivot(i, piv):
    if piv == 0 or not np.isfinite(piv):
        raise ZeroPivotError(f"zero or non-finite pivot in row {i}")


def ilu0(B):
    n = B.shape[0]
    dtype = np.result_type(B.dtype, np.float64)
    A = _rows(B)
    Lr, Ur = [], []
    for i in range(n):
        w = dict(A[i])
        for k in sorted(c for c in w if c < i):
            w[k] = w[k] / Ur[k][k]
            for j, ukj in Ur[k].items():
                if j > k and j in w:
                    w[j] = w[j] - w[k] * ukj
        Lr.append({j: v for j, v in w.items() if j < i})
        Ur.append({j: v for j, v in w.items() if j >= i})
        _check_pivot(i, Ur[i].get(i, 0.0))
    return _to_csr(Lr, n, dtype), _to_csr(Ur, n, dtype)


def _keep_largest(part, lfil):
    if len(part) <= lfil:
        return part
    order = sorted(part.items(), key=lambda kv: (-abs(kv[1]), kv[0]))
    return dict(order[:lfil])


def ilut(B, tau, lfil):
    n = B.shape[0]
    dtype = np.result_type(B.dtype, np.float64)
    A = _rows(B)
    Lr, Ur = [], []
    for i in range(n):
        w = dict(A[i])
        tau_i = tau * np.sqrt(sum(abs(v) ** 2 for v in A[i].values()))
        heap = [c for c in w if c < i]
        heapq.heapify(heap)
        while heap:
            k = heapq.heappop(heap)
            wk = w[k] / Ur[k][k]
            if abs(wk) < tau_i:
                del w[k]
                continue
            w[k] = wk
            for j, ukj in Ur[k].items():
                if j <= k:
                    continue
                if j in w:
                    w[j] = w[j] - wk * ukj
                else:
                    w[j] = -wk * ukj
                    if j < i:
                        heapq.heappush(heap, j)
        lpart = {j: v for j, v in w.items() if j < i and abs(v) >= tau_i}
        upart = {j: v for j, v in w.items() if j > i and abs(v) >= tau_i}
        diag = w.get(i, 0.0)
        _check_pivot(i, diag)
        lpart = _keep_largest(lpart, lfil)
        upart = _keep_largest(upart, lfil)
        upart[i] = diag
        Lr.append(lpart)
        Ur.append(upart)
    return _to_csr(Lr, n, dtype), _to_csr(Ur, n, dtype)


def factor(B, kind, tau=0.0, lfil=0):
    if kind == "ilu0":
        return ilu0(B)
    if kind == "ilut":
        return ilut(B, tau, lfil)
    raise ValueError(kind)
