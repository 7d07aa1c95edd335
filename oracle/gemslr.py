"""GeMSLR setup (Alg. 1) and preconditioner apply M^{-1} (Alg. 2).

Level structure (Sec. 2.4): A_l = [[B_l, F_l], [E_l, C_l]] with A_0 = P^T A P
and A_{l+1} = C_l.  With the composed permutation of partition.py every C_l
is the tail of the permuted vector, so level l acts on the index range
[start_l, n) and splits it into B_l = [start_l, start_{l+1}) and
C_l = [start_{l+1}, n).

Setup (Alg. 1): ILU of every B_l, then the rank-k terms W_l, R_l built
bottom-up (l = L-1 ... 0) because G_hat_l needs C_l^{-1}, which is the apply
of the levels below l (Sec. 4.2).  The last separator C_{L-1} is kept only
on its diagonal blocks (block Jacobi) and factored the same way (Sec. 4.3);
it is stored here as level L with no interface (s = 0).

Apply (Alg. 2) with a low-rank term at every level, the last one included,
and by default zero inner GMRES iterations at level 0: M_l^{-1} is the
inverse of the block LDU factorisation of A_l (Sec. 2.2) with B_l^{-1} taken
as the ILU solve and the Schur complement inverse as the low-rank corrected
next-level preconditioner of eq. gemslr6 (see apply_level).
"""
from dataclasses import dataclass

import numpy as np
import scipy.sparse as sp
from scipy.sparse.linalg import spsolve_triangular

from . import ilu as ilu_mod
from . import lowrank


@dataclass
class Level:
    start: int
    d: int
    s: int
    blocks: np.ndarray      # block boundaries relative to start, nb+1 entries
    Lf: sp.csr_matrix       # strictly lower ILU factor (unit diagonal implied)
    Uf: sp.csr_matrix       # upper ILU factor including the diagonal
    E: sp.csr_matrix        # s x d
    F: sp.csr_matrix        # d x s
    W: np.ndarray = None    # s x k
    R: np.ndarray = None    # k x k
    H: np.ndarray = None    # k x k, (I - R)^{-1} - I
    info: dict = None


@dataclass
class Setup:
    n: int
    perm: np.ndarray
    levels: list            # L+1 entries; the last is C_last with s = 0
    Ap: sp.csr_matrix       # P^T A P
    real: bool

    @property
    def nlevels(self):
        return len(self.levels) - 1


def csr(rowptr, col, val, n):
    a = sp.csr_matrix((val, col, rowptr), shape=(n, n))
    a.sort_indices()
    return a


def _block_diag_part(B, blocks):
    """Keep only the entries of B inside its diagonal blocks."""
    B = B.tocoo()
    lab = np.zeros(B.shape[0], dtype=np.int64)
    for i in range(len(blocks) - 1):
        lab[blocks[i]:blocks[i + 1]] = i
    keep = lab[B.row] == lab[B.col]
    return sp.csr_matrix((B.data[keep], (B.row[keep], B.col[keep])),
                         shape=B.shape)


def trisolve(lv, b):
    """U^{-1} L^{-1} b for one level (b may hold several columns)."""
    if lv.d == 0:
        return b.copy()
    I = sp.identity(lv.d, dtype=lv.Lf.dtype, format="csr")
    y = spsolve_triangular((lv.Lf + I).tocsr(), b, lower=True)
    return spsolve_triangular(lv.Uf, y, lower=False)


def lowrank_then_lower(st, l, z2):
    """The interface branch of Alg. 2 for l > 0: M_{l+1}^{-1} (z2 + u2) with
    u2 = W_l [(I - R_l)^{-1} - I] W_l^H z2."""
    lv = st.levels[l]
    if lv.W is not None and lv.W.shape[1] > 0:
        u2 = lv.W @ (lv.H @ (lv.W.conj().T @ z2))
    else:
        u2 = np.zeros_like(z2)
    return apply_level(st, l + 1, u2 + z2)


def schur_matvec(st, v):
    """S_hat_0 v = C_0 v - E_0 U_0^{-1} L_0^{-1} F_0 v: the root-level Schur
    complement with B_0^{-1} replaced by the ILU solve (Sec. 3, the operator
    of the inner iteration of Alg. 2 at l = 0)."""
    lv = st.levels[0]
    C = st.Ap[lv.d:, lv.d:]
    return C @ v - lv.E @ trisolve(lv, lv.F @ v)


def inner_gmres(st, z2, its):
    """`its` steps of right-preconditioned GMRES for S_hat_0 y = z2 from
    y = 0 (Alg. 2, l = 0), preconditioned by the l > 0 branch of Alg. 2
    applied at level 0, P v = M_1^{-1}(v + W_0 H_0 W_0^H v).

    Written from the definition of GMRES (Saad and Schultz 1986): with K an
    orthonormal basis of the Krylov space span{z2, (S P) z2, ...,
    (S P)^{its-1} z2}, y = P K c where c minimises ||z2 - S P K c||_2.  The
    basis stops early when the space becomes invariant."""
    beta = np.linalg.norm(z2)
    if beta == 0:
        return np.zeros_like(z2)

    def P(v):
        return lowrank_then_lower(st, 0, v)

    basis = [z2 / beta]
    for _ in range(1, its):
        w = schur_matvec(st, P(basis[-1]))
        wn = np.linalg.norm(w)
        K = np.column_stack(basis)
        for _ in range(2):
            w = w - K @ (K.conj().T @ w)
        if np.linalg.norm(w) <= 1e-12 * wn:
            break
        basis.append(w / np.linalg.norm(w))
    PK = np.column_stack([P(k) for k in basis])
    SPK = np.column_stack([schur_matvec(st, PK[:, j]) for j in range(PK.shape[1])])
    c = np.linalg.lstsq(SPK, z2, rcond=None)[0]
    return PK @ c


def ilu_solve(lv, b):
    """B_l^{-1} b with B_l replaced by its incomplete factors, U_l^{-1} L_l^{-1} b."""
    return trisolve(lv, b)


def schur_solve(st, l, r, inner_its=0):
    """S_l^{-1} r for the Schur complement S_l = C_l - E_l B_l^{-1} F_l.

    eq. gemslr6 (with eq. gemslr4): S_l^{-1} ~ C_l^{-1} (I + W_l H_l W_l^H)
    with H_l = (I - R_l)^{-1} - I, and C_l^{-1} is the preconditioner of the
    next level (C_last^{-1} below the last one).  At the root level with
    inner_its > 0 the system S_hat_0 y = r is instead solved by that many
    GMRES steps preconditioned by this approximation (Alg. 2, l = 0)."""
    if l == 0 and inner_its > 0:
        return inner_gmres(st, r, inner_its)
    return lowrank_then_lower(st, l, r)


def apply_level(st, l, b, inner_its=0):
    """M_l^{-1} b on the index range of level l.

    A_l = [[B, F], [E, C]] factors into block unit-lower, block diagonal and
    block unit-upper parts (Sec. 2.2),
        A_l = [[I, 0], [E B^{-1}, I]] [[B, 0], [0, S]] [[I, B^{-1} F], [0, I]],
    and M_l^{-1} is the inverse of that product, taken factor by factor, with
    B^{-1} replaced by the ILU solve and S^{-1} by schur_solve -- the
    recursion of Alg. 2.  The last level is the block-Jacobi ILU of C_last
    (Sec. 4.3)."""
    lv = st.levels[l]
    if l == st.nlevels:
        return ilu_solve(lv, b)
    d = lv.d
    # inverse of the block unit-lower factor: [b1; b2 - E B^{-1} b1]
    u = b.copy()
    u[d:] = b[d:] - lv.E @ ilu_solve(lv, b[:d])
    # inverse of the block diagonal: [B^{-1} u1; S^{-1} u2]
    v = np.empty_like(u)
    v[:d] = ilu_solve(lv, u[:d])
    v[d:] = schur_solve(st, l, u[d:], inner_its)
    # inverse of the block unit-upper factor: [v1 - B^{-1} F v2; v2]
    y = v.copy()
    y[:d] = v[:d] - ilu_solve(lv, lv.F @ v[d:])
    return y


def _promote(st, x):
    """x in the type of x and of the setup's scalars together: apply_level's
    work vectors copy the input's type, so a real vector on a complex setup
    must be made complex first (and a complex one on a real setup stays
    complex, M^{-1} being real and linear there)."""
    x = np.asarray(x)
    return x.astype(np.result_type(x.dtype, np.float64 if st.real else np.complex128),
                    copy=False)


def apply(st, x, inner_its=0):
    """y = M^{-1} x in the original ordering."""
    q = apply_level(st, 0, _promote(st, x)[st.perm], inner_its)
    y = np.empty_like(q)
    y[st.perm] = q
    return y


def apply_permuted(st, xp, inner_its=0):
    return apply_level(st, 0, _promote(st, xp), inner_its)


def ghat_matvec(st, l, v):
    """G_hat_l v = E_l U_l^{-1} L_l^{-1} F_l C_l^{-1} v (Sec. 2.3; E_l, not
    its transpose -- the transpose in the multilevel formula does not
    conform)."""
    lv = st.levels[l]
    c = apply_level(st, l + 1, v)
    return lv.E @ trisolve(lv, lv.F @ c)


def setup(rowptr, col, val, part, ilu="ilut", drop_tol=1e-3, lfil=10,
          rank=32, seed=0, lowrank_last_level=True, dense_max=2000,
          arnoldi_tol=1e-2, max_cycles=20, ilu_shift=0.0):
    """ilu_shift s: each on-diagonal block is factored as B + i s m I with m
    the mean of |a_ii| over A (the complex shift of the Helmholtz tests,
    Sec. 5); E, F and C keep A's entries."""
    n = len(rowptr) - 1
    A = csr(rowptr, col, val, n)
    real = not np.iscomplexobj(val)
    if ilu_shift != 0.0 and real:
        raise ValueError("a complex shift needs a complex matrix")
    sigma = ilu_shift * np.mean(np.abs(A.diagonal()))
    perm = part.perm
    Ap = A[perm][:, perm].tocsr()
    Ap.sort_indices()
    ls = part.level_start
    L = part.nlevels
    levels = []
    for l in range(L + 1):
        a = ls[l]
        b = ls[l + 1] if l < L else n
        B = Ap[a:b, a:b]
        blocks = part.blocks[l] - a
        if l == L:
            B = _block_diag_part(B, blocks)
            E = sp.csr_matrix((0, b - a), dtype=Ap.dtype)
            F = sp.csr_matrix((b - a, 0), dtype=Ap.dtype)
        else:
            E = Ap[b:, a:b].tocsr()
            F = Ap[a:b, b:].tocsr()
        Bf = B if ilu_shift == 0.0 else (B + 1j * sigma * sp.identity(B.shape[0])).tocsr()
        Lf, Uf = ilu_mod.factor(Bf, ilu, drop_tol, lfil)
        levels.append(Level(int(a), int(b - a), int(n - b), blocks, Lf, Uf,
                            E, F))
    st = Setup(n, perm, levels, Ap, real)
    # low-rank terms, bottom-up
    for l in range(L - 1, -1, -1):
        lv = levels[l]
        k = min(rank, lv.s)
        if l == L - 1 and not lowrank_last_level:
            k = 0
        dt = np.float64 if real else np.complex128
        if k == 0:
            lv.W = np.zeros((lv.s, 0), dtype=dt)
            lv.R = np.zeros((0, 0), dtype=dt)
            lv.info = {"mode": "none"}
        elif lv.s <= dense_max:
            G = ghat_matvec(st, l, np.eye(lv.s, dtype=dt))
            lv.W, lv.R = lowrank.dense_lowrank(G, k, real)
            lv.info = {"mode": "dense"}
        else:
            lv.W, lv.R, lv.info = lowrank.krylov_schur(
                lambda v: ghat_matvec(st, l, v), lv.s, k, real,
                seed=seed + l, tol=arnoldi_tol, max_cycles=max_cycles)
            lv.info["mode"] = "krylov-schur"
        lv.H = lowrank.finish(lv.W, lv.R)
    return st
