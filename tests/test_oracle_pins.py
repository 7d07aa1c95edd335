"""Pins of the CPU oracle against facts fixed outside the oracle itself:
closed-form counts, textbook/library factorizations, dense linear algebra,
hand-worked fixtures, published test vectors and brute force on tiny inputs.
CPU only."""
import json
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from paper_2205_03224_amd import workloads as wl
from oracle import fgmres, gemslr, ilu, lowrank, mlp, partition, rng

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- rng

def test_splitmix64_published_vector():
    # First outputs of SplitMix64 seeded with 1234567 (the test vector that
    # accompanies Vigna's reference implementation).
    assert rng.splitmix64_outputs(1234567, 5) == [
        6457827717110365317, 3203168211198807973, 9817491932198370423,
        4593380528125082431, 16408922859458223821]


def test_start_vector_matches_scalar_definition():
    outs = rng.splitmix64_outputs(42, 7)
    v = rng.start_vector(42, 7)
    ref = [2.0 * ((o >> 11) * 2.0 ** -53) - 1.0 for o in outs]
    assert np.array_equal(v, np.array(ref))


# ---------------------------------------------------------------- partition

def _sizes(p):
    L = p.nlevels
    ls = p.level_start
    return [int(ls[l + 1] - ls[l]) for l in range(L + 1)]


def test_partition_2d_closed_form():
    w = wl.laplace2d_32()
    p = partition.wirebasket(w.dims, 4, 2, w.rowptr, w.col)
    # cut at 16 on both axes: 31^2 interior, 2*31 arm vertices, 1 centre
    assert p.nlevels == 2
    assert _sizes(p) == [31 * 31, 2 * 31, 1]
    assert [len(b) - 1 for b in p.blocks] == [4, 4, 1]
    box = np.diff(p.blocks[0]).tolist()
    assert sorted(box) == sorted([16 * 16, 16 * 15, 15 * 16, 15 * 15])


@pytest.mark.parametrize("N,q", [(64, 4), (20, 3)])
def test_partition_3d_closed_form(N, q):
    r, c, v = wl.convdiff3d(N)
    p = partition.wirebasket((N, N, N), q ** 3, 5, r, c)
    m = N - (q - 1)  # points per axis not on a cut
    # class l = l coordinates on a cut: C(3,l) (q-1)^l m^(3-l)
    assert p.nlevels == 3
    assert _sizes(p) == [m ** 3, 3 * (q - 1) * m * m, 3 * (q - 1) ** 2 * m,
                         (q - 1) ** 3]
    # boxes, faces, edges, corners
    assert [len(b) - 1 for b in p.blocks] == [
        q ** 3, 3 * (q - 1) * q * q, 3 * (q - 1) ** 2 * q, (q - 1) ** 3]


def test_partition_is_vertex_separator():
    r, c, v = wl.convdiff3d(12)
    n = 12 ** 3
    p = partition.wirebasket((12, 12, 12), 27, 3, r, c)
    assert sorted(p.perm.tolist()) == list(range(n))
    inv = np.empty(n, dtype=np.int64)
    inv[p.perm] = np.arange(n)
    # block label and level of every permuted position
    blk = np.empty(n, dtype=np.int64)
    lev = np.empty(n, dtype=np.int64)
    nb = 0
    for l, b in enumerate(p.blocks):
        for i in range(len(b) - 1):
            blk[b[i]:b[i + 1]] = nb
            lev[b[i]:b[i + 1]] = l
            nb += 1
    A = sp.csr_matrix((v, c, r), shape=(n, n)).tocoo()
    pi, pj = inv[A.row], inv[A.col]
    same_level = lev[pi] == lev[pj]
    # no edge joins two different diagonal blocks of the same level
    assert np.all(blk[pi][same_level] == blk[pj][same_level])


def test_partition_stop_rule():
    # 2-D grid asked for 5 levels stops at dim = 2 levels
    r, c, v = wl.laplace2d(16)
    p = partition.wirebasket((16, 16), 4, 5, r, c)
    assert p.nlevels == 2
    # one part: no separator at all
    p1 = partition.wirebasket((16, 16), 1, 3, r, c)
    assert p1.nlevels == 1 and _sizes(p1) == [256, 0]


# ---------------------------------------------------------------- ILU

def _csr_from_dense(D):
    return sp.csr_matrix(np.asarray(D, dtype=float))


def test_ilut_hand_worked_cases():
    cases = json.load(open(os.path.join(GOLDEN, "ilut_hand.json")))["cases"]
    for case in cases:
        B = _csr_from_dense(case["B"])
        Lf, Uf = ilu.ilut(B, case["tau"], case["lfil"])
        n = B.shape[0]
        for i in range(n):
            got_l = list(zip(Lf.indices[Lf.indptr[i]:Lf.indptr[i + 1]].tolist(),
                             Lf.data[Lf.indptr[i]:Lf.indptr[i + 1]].tolist()))
            got_u = list(zip(Uf.indices[Uf.indptr[i]:Uf.indptr[i + 1]].tolist(),
                             Uf.data[Uf.indptr[i]:Uf.indptr[i + 1]].tolist()))
            exp_l = [tuple(e) for e in case["L"][i]]
            exp_u = [tuple(e) for e in case["U"][i]]
            assert [c for c, _ in got_l] == [c for c, _ in exp_l], case["name"]
            assert [c for c, _ in got_u] == [c for c, _ in exp_u], case["name"]
            np.testing.assert_allclose([x for _, x in got_l],
                                       [x for _, x in exp_l], rtol=1e-15)
            np.testing.assert_allclose([x for _, x in got_u],
                                       [x for _, x in exp_u], rtol=1e-15)


@pytest.mark.parametrize("kind", ["ilu0", "ilut"])
def test_tridiagonal_factor_is_exact_lu(kind):
    # a tridiagonal matrix has no fill, so ILU(0) and ILUT(0, inf) are its LU
    n = 30
    rs = np.random.default_rng(3)
    D = np.diag(4 + rs.random(n)) + np.diag(-1 - rs.random(n - 1), 1) + \
        np.diag(-1 + 0.3 * rs.random(n - 1), -1)
    P, Ld, Ud = sla.lu(D)
    assert np.array_equal(P, np.eye(n))  # diagonally dominant: no pivoting
    Lf, Uf = ilu.factor(sp.csr_matrix(D), kind, 0.0, 10 ** 9)
    np.testing.assert_allclose(Lf.toarray() + np.eye(n), Ld, rtol=0, atol=1e-14)
    np.testing.assert_allclose(Uf.toarray(), Ud, rtol=0, atol=1e-13)


def test_ilut_no_dropping_is_exact_lu():
    r, c, v = wl.convdiff3d(5, (0.2, 0.1, 0.05))
    B = sp.csr_matrix((v, c, r), shape=(125, 125))
    Lf, Uf = ilu.ilut(B, 0.0, 10 ** 9)
    LU = (Lf.toarray() + np.eye(125)) @ Uf.toarray()
    np.testing.assert_allclose(LU, B.toarray(), atol=1e-13)
    P, Ld, Ud = sla.lu(B.toarray())
    np.testing.assert_allclose(Uf.toarray(), Ud, atol=1e-12)


def test_ilu0_pattern_identity():
    # (L U)_ij = b_ij on the pattern of B, and L, U stay inside it
    r, c, v = wl.lognormal_convdiff3d(6, seed=5)[:3]
    n = 216
    B = sp.csr_matrix((v, c, r), shape=(n, n))
    Lf, Uf = ilu.ilu0(B)
    pat = B.toarray() != 0
    LU = (Lf.toarray() + np.eye(n)) @ Uf.toarray()
    np.testing.assert_allclose(LU[pat], B.toarray()[pat], rtol=1e-13,
                               atol=1e-13)
    assert np.all(pat[Lf.toarray() != 0]) and np.all(pat[Uf.toarray() != 0])
    assert abs(LU[~pat]).max() > 0  # genuinely incomplete


def test_ilut_caps_and_threshold():
    r, c, v = wl.convdiff3d(8)
    n = 512
    B = sp.csr_matrix((v, c, r), shape=(n, n))
    tau, lfil = 1e-2, 4
    Lf, Uf = ilu.ilut(B, tau, lfil)
    rown = np.sqrt(np.asarray(abs(B).power(2).sum(axis=1)).ravel())
    for i in range(n):
        li = Lf.data[Lf.indptr[i]:Lf.indptr[i + 1]]
        cols = Uf.indices[Uf.indptr[i]:Uf.indptr[i + 1]]
        ui = Uf.data[Uf.indptr[i]:Uf.indptr[i + 1]][cols != i]
        assert len(li) <= lfil and len(ui) <= lfil
        assert np.all(abs(li) >= tau * rown[i]) and np.all(abs(ui) >= tau * rown[i])
        assert i in cols


def test_zero_pivot_raises():
    D = np.array([[1.0, 1.0], [1.0, 1.0]])
    with pytest.raises(ilu.ZeroPivotError):
        ilu.ilu0(sp.csr_matrix(D))
    with pytest.raises(ilu.ZeroPivotError):
        ilu.ilut(sp.csr_matrix(D), 0.0, 5)


# ---------------------------------------------------------------- low-rank

def test_selection_uses_correction_weight():
    # |theta/(1-theta)|: 0.9 -> 9, 0.5 -> 1, -0.95 -> 0.487; "largest
    # |theta|" would wrongly take -0.95 second.
    th = np.array([-0.95, 0.5, 0.9, 0.1], dtype=complex)
    m = lowrank.select_wanted(th, 2, real=True)
    assert m.tolist() == [False, True, True, False]


def test_selection_completes_conjugate_pairs():
    th = np.array([0.9, 0.5 + 0.4j, 0.5 - 0.4j, 0.1], dtype=complex)
    m = lowrank.select_wanted(th, 2, real=True)
    assert m.sum() == 3 and m[0] and m[1] and m[2]
    mc = lowrank.select_wanted(th, 2, real=False)
    assert mc.sum() == 2


def test_smw_identity_dense():
    # S^{-1} = C^{-1} + C^{-1} W [(I-R)^{-1} - I] W^H with G = E B^{-1} F C^{-1}
    rs = np.random.default_rng(7)
    d, s = 12, 6
    B = np.eye(d) * 5 + rs.standard_normal((d, d))
    C = np.eye(s) * 5 + rs.standard_normal((s, s))
    E = rs.standard_normal((s, d))
    F = rs.standard_normal((d, s))
    G = E @ np.linalg.solve(B, F) @ np.linalg.inv(C)
    W, R = lowrank.dense_lowrank(G, s, real=False)
    H = lowrank.finish(W, R)
    S = C - E @ np.linalg.solve(B, F)
    Ci = np.linalg.inv(C)
    np.testing.assert_allclose(Ci + Ci @ W @ H @ W.conj().T, np.linalg.inv(S),
                               atol=1e-12)
    # eigenvalues of the correction are gamma/(1-gamma)
    gam = np.linalg.eigvals(G)
    corr = np.linalg.eigvals(W @ H @ W.conj().T)
    want = gam / (1 - gam)
    dist = np.abs(corr[:, None] - want[None, :])
    assert dist.min(axis=0).max() < 1e-11 and dist.min(axis=1).max() < 1e-11


def _laplace1d_scaled(m):
    T = 2 * np.eye(m) - np.eye(m, k=1) - np.eye(m, k=-1)
    return T / 4.0   # eigenvalues (2 - 2 cos(j pi/(m+1)))/4 in (0, 1)


def test_krylov_schur_closed_form_eigenvalues():
    m = 100
    T = _laplace1d_scaled(m)
    exact = (2 - 2 * np.cos(np.arange(1, m + 1) * np.pi / (m + 1))) / 4
    k = 6
    W, R, info = lowrank.krylov_schur(lambda v: T @ v, m, k, real=True,
                                      seed=1, tol=1e-10, max_cycles=400)
    assert info["converged"] and info["cycles"] > 1   # needed restarts
    want = np.sort(exact)[::-1][:k]   # weight grows with theta on (0, 1)
    np.testing.assert_allclose(np.sort(np.linalg.eigvals(R).real)[::-1], want,
                               rtol=1e-8)
    np.testing.assert_allclose(W.T @ W, np.eye(W.shape[1]), atol=1e-12)
    np.testing.assert_allclose(W.T @ T @ W, R, atol=1e-12)


def test_krylov_schur_complex_spectrum():
    # real operator with conjugate pairs: block-diagonal rotations, hidden by
    # an orthogonal similarity.  The three wanted pairs sit near theta = 1
    # (largest |theta/(1-theta)|), the rest inside |theta| < 0.5.
    rs = np.random.default_rng(11)
    m = 120
    D = np.zeros((m, m))
    vals = []
    fixed = [(0.9, 0.05), (0.85, 0.1), (0.8, 0.02)]
    for i in range(0, m, 2):
        if i // 2 < len(fixed):
            a, b = fixed[i // 2]
        else:
            r_, t_ = 0.5 * rs.random(), rs.random() * np.pi
            a, b = r_ * np.cos(t_), r_ * np.sin(t_)
        D[i:i + 2, i:i + 2] = [[a, b], [-b, a]]
        vals += [a + 1j * b, a - 1j * b]
    Q, _ = np.linalg.qr(rs.standard_normal((m, m)))
    G = Q @ D @ Q.T
    k = 5
    W, R, info = lowrank.krylov_schur(lambda v: G @ v, m, k, real=True,
                                      seed=3, tol=1e-10, max_cycles=300)
    assert info["converged"]
    assert W.shape[1] == 6        # k raised to keep the pair together
    got = np.linalg.eigvals(R)
    want = np.array([a + s * 1j * b for a, b in fixed for s in (1, -1)])
    dist = np.abs(got[:, None] - want[None, :])
    assert dist.min(axis=0).max() < 1e-9
    np.testing.assert_allclose(W.T @ W, np.eye(6), atol=1e-12)
    np.testing.assert_allclose(W.T @ G @ W, R, atol=1e-11)


def test_krylov_schur_breakdown_invariant_subspace():
    # G = a I + U diag(lam) U^T with U of rank 3: the Krylov space of any
    # start vector is span{v0} + range(U) (4-dimensional), so with k = 3
    # (m = 6) the step on v_3 finds nothing new; the fresh direction v_4 is
    # orthogonal to range(U), so G v_4 = a v_4 is in the basis again, and so
    # is G v_5: the breakdown branch runs three times.  The wanted Ritz values
    # are then exactly a + lam (largest theta/(1 - theta)), W spans range(U),
    # and the Krylov relation has no remainder.
    rs = np.random.default_rng(21)
    s = 40
    U, _ = np.linalg.qr(rs.standard_normal((s, 3)))
    a, lam = 0.1, np.array([0.6, 0.4, 0.2])
    G = a * np.eye(s) + U @ np.diag(lam) @ U.T
    for real in (True, False):
        W, R, info = lowrank.krylov_schur(lambda v: G @ v, s, 3, real=real, seed=5)
        assert info["breakdowns"] == 3
        assert info["converged"] and info["cycles"] == 1 and info["matvecs"] == 6
        np.testing.assert_allclose(np.sort(np.linalg.eigvals(R).real)[::-1], a + lam,
                                   atol=1e-13)
        np.testing.assert_allclose(W.conj().T @ W, np.eye(3), atol=1e-13)
        np.testing.assert_allclose(W.conj().T @ G @ W, R, atol=1e-13)
        # span(W) = range(U): the projector difference vanishes
        assert np.linalg.norm(W @ W.conj().T - U @ U.T) < 1e-12


def test_singular_correction_raises():
    R = np.array([[1.0, 0.3], [0.0, 0.5]])
    with pytest.raises(lowrank.SingularCorrectionError):
        lowrank.finish(np.eye(2), R)


# ---------------------------------------------------------------- apply

FULL = dict(ilu="ilut", drop_tol=0.0, lfil=10 ** 9, rank=10 ** 9)


@pytest.mark.parametrize("case", ["lap2d8", "lap2d32", "cd3d", "helm3d",
                                  "cd3d27"])
def test_full_rank_apply_is_exact_inverse(case):
    # exact factors + full rank at every level => M^{-1} = A^{-1}
    if case == "lap2d8":
        (r, c, v), dims, p, lev = wl.laplace2d(8), (8, 8), 4, 2
    elif case == "lap2d32":
        (r, c, v), dims, p, lev = wl.laplace2d(32), (32, 32), 4, 2
    elif case == "cd3d":
        (r, c, v), dims, p, lev = wl.convdiff3d(6, (.3, .2, .1)), (6,) * 3, 8, 3
    elif case == "helm3d":
        (r, c, v), dims, p, lev = wl.helmholtz3d(6, 0.39), (6,) * 3, 8, 3
    else:
        (r, c, v), dims, p, lev = wl.convdiff3d(9, (.3, .2, .1)), (9,) * 3, 27, 3
    n = len(r) - 1
    part = partition.wirebasket(dims, p, lev, r, c)
    st = gemslr.setup(r, c, v, part, **FULL)
    A = sp.csr_matrix((v, c, r), shape=(n, n)).toarray()
    rs = np.random.default_rng(0)
    x = rs.standard_normal(n)
    if np.iscomplexobj(v):
        x = x + 1j * rs.standard_normal(n)
    y = gemslr.apply(st, x)
    ref = sla.lu_solve(sla.lu_factor(A), x)
    assert np.linalg.norm(y - ref) <= 1e-12 * np.linalg.norm(ref)
    # a vector of the other kind: real on a complex setup (its result is
    # complex, not the real part of one), complex on a real setup
    x2 = rs.standard_normal(n)
    if not np.iscomplexobj(v):
        x2 = x2 + 1j * rs.standard_normal(n)
    y2 = gemslr.apply(st, x2)
    ref2 = np.linalg.solve(A, x2)
    assert np.iscomplexobj(y2)
    assert np.linalg.norm(y2 - ref2) <= 1e-12 * np.linalg.norm(ref2)


def test_full_rank_via_krylov_schur_is_exact():
    # same identity when the rank-s terms come from Arnoldi (m = s)
    r, c, v = wl.convdiff3d(6, (.3, .2, .1))
    part = partition.wirebasket((6,) * 3, 8, 3, r, c)
    st = gemslr.setup(r, c, v, part, dense_max=0, **FULL)
    assert st.levels[0].info["mode"] == "krylov-schur"
    A = sp.csr_matrix((v, c, r), shape=(216, 216)).toarray()
    x = np.random.default_rng(2).standard_normal(216)
    y = gemslr.apply(st, x)
    ref = np.linalg.solve(A, x)
    assert np.linalg.norm(y - ref) <= 1e-10 * np.linalg.norm(ref)


def _dense_block_ldu(Ap, ls, L):
    """Rank-0 multilevel preconditioner written with dense inverses:
    M_l^{-1} = [[I, -B^{-1}F], [0, I]] diag(B^{-1}, M_{l+1}^{-1})
               [[I, 0], [-E B^{-1}, I]],   M_L^{-1} = C_last^{-1}."""
    n = Ap.shape[0]

    def minv(l):
        a = ls[l]
        if l == L:
            return np.linalg.inv(Ap[a:, a:])
        b = ls[l + 1]
        B, F, E = Ap[a:b, a:b], Ap[a:b, b:], Ap[b:, a:b]
        Bi = np.linalg.inv(B)
        d, s = b - a, n - b
        up = np.block([[np.eye(d), -Bi @ F], [np.zeros((s, d)), np.eye(s)]])
        lo = np.block([[np.eye(d), np.zeros((d, s))], [-E @ Bi, np.eye(s)]])
        mid = np.block([[Bi, np.zeros((d, s))], [np.zeros((s, d)), minv(l + 1)]])
        return up @ mid @ lo

    return minv(0)


def test_rank_zero_apply_is_block_ldu():
    r, c, v = wl.convdiff3d(7, (.3, .2, .1))
    n = 343
    part = partition.wirebasket((7,) * 3, 8, 3, r, c)
    st = gemslr.setup(r, c, v, part, ilu="ilut", drop_tol=0.0, lfil=10 ** 9,
                      rank=0)
    A = sp.csr_matrix((v, c, r), shape=(n, n)).toarray()
    Ap = A[np.ix_(part.perm, part.perm)]
    Mi = _dense_block_ldu(Ap, part.level_start, part.nlevels)
    x = np.random.default_rng(4).standard_normal(n)
    yp = gemslr.apply_permuted(st, x[part.perm])
    np.testing.assert_allclose(yp, Mi @ x[part.perm], rtol=1e-12, atol=1e-12)
    # and it is not the exact inverse (the Schur complement was replaced)
    assert np.linalg.norm(yp - np.linalg.solve(Ap, x[part.perm])) > 1e-6


def test_lowrank_terms_properties_krylov():
    w = wl.convdiff3d_64(N=24, nparts=8)
    part = partition.wirebasket(w.dims, 8, 3, w.rowptr, w.col)
    st = gemslr.setup(w.rowptr, w.col, w.val, part, ilu="ilut", drop_tol=1e-3,
                      lfil=10, rank=8, dense_max=100)
    lv = st.levels[0]
    assert lv.info["mode"] == "krylov-schur"
    k = lv.W.shape[1]
    np.testing.assert_allclose(lv.W.T @ lv.W, np.eye(k), atol=1e-12)
    GW = np.column_stack([gemslr.ghat_matvec(st, 0, lv.W[:, i])
                          for i in range(k)])
    np.testing.assert_allclose(lv.W.T @ GW, lv.R, atol=1e-11)
    # Ritz pairs accurate to two digits
    ev, Y = np.linalg.eig(lv.R)
    X = lv.W @ Y
    GX = np.column_stack([gemslr.ghat_matvec(st, 0, X[:, i]) for i in range(k)])
    res = np.linalg.norm(GX - X * ev, axis=0) / np.linalg.norm(X, axis=0)
    assert np.all(res <= 1e-2 * np.abs(ev) + 1e-12)


# ---------------------------------------------------------------- inner GMRES (level 0)

def _inner_case(rank, exact=False):
    r, c, v = wl.convdiff3d(7, (.3, .2, .1))
    part = partition.wirebasket((7,) * 3, 8, 3, r, c)
    kw = FULL if exact else dict(ilu="ilut", drop_tol=1e-2, lfil=3, rank=rank)
    return gemslr.setup(r, c, v, part, **kw), r, c, v, part


def _dense_schur_hat(st):
    """C_0 - E_0 U^{-1} L^{-1} F_0 from dense copies of the factors."""
    lv = st.levels[0]
    Ld = lv.Lf.toarray() + np.eye(lv.d)
    Ud = lv.Uf.toarray()
    X = sla.solve_triangular(Ud, sla.solve_triangular(Ld, lv.F.toarray(), lower=True,
                                                      unit_diagonal=True))
    C = st.Ap.toarray()[lv.d:, lv.d:]
    return C - lv.E.toarray() @ X


def test_schur_hat_with_exact_factors_is_schur_complement():
    st, r, c, v, part = _inner_case(0, exact=True)
    A = sp.csr_matrix((v, c, r)).toarray()[np.ix_(part.perm, part.perm)]
    d = st.levels[0].d
    S = A[d:, d:] - A[d:, :d] @ np.linalg.solve(A[:d, :d], A[:d, d:])
    x = np.random.default_rng(1).standard_normal(S.shape[0])
    np.testing.assert_allclose(gemslr.schur_matvec(st, x), S @ x, rtol=1e-11, atol=1e-11)


def test_inner_gmres_one_step_closed_form():
    st, *_ = _inner_case(4)
    s = st.levels[0].s
    z = np.random.default_rng(2).standard_normal(s)
    pz = gemslr.lowrank_then_lower(st, 0, z)
    spz = _dense_schur_hat(st) @ pz
    alpha = (spz @ z) / (spz @ spz)
    np.testing.assert_allclose(gemslr.inner_gmres(st, z, 1), alpha * pz, rtol=1e-11)


def test_inner_gmres_full_space_solves_schur_hat():
    st, *_ = _inner_case(4)
    s = st.levels[0].s
    z = np.random.default_rng(3).standard_normal(s)
    Sh = _dense_schur_hat(st)
    y = gemslr.inner_gmres(st, z, s)
    np.testing.assert_allclose(y, np.linalg.solve(Sh, z), rtol=1e-8, atol=1e-10)


def test_inner_gmres_residual_does_not_grow():
    st, *_ = _inner_case(2)
    s = st.levels[0].s
    z = np.random.default_rng(4).standard_normal(s)
    Sh = _dense_schur_hat(st)
    res = [np.linalg.norm(z - Sh @ gemslr.inner_gmres(st, z, m)) for m in range(1, 6)]
    assert all(b <= a * (1 + 1e-12) for a, b in zip(res, res[1:]))
    assert res[-1] < res[0]


def test_inner_gmres_exact_case_is_exact_inverse():
    # exact factors and full rank: the preconditioner of the inner iteration is
    # S^{-1} itself, one step is exact and the space is then invariant
    st, r, c, v, part = _inner_case(0, exact=True)
    A = sp.csr_matrix((v, c, r)).toarray()
    x = np.random.default_rng(5).standard_normal(A.shape[0])
    for its in (1, 3):
        y = gemslr.apply(st, x, inner_its=its)
        np.testing.assert_allclose(y, np.linalg.solve(A, x), rtol=1e-10, atol=1e-12)


# ---------------------------------------------------------------- complex shift

def test_shifted_exact_factors_reproduce_shifted_blocks():
    """With exact factors, L U of every block equals B + i s m I, m = mean
    |a_ii| of A; E and F keep A's entries."""
    r, c, v = wl.helmholtz3d(6, 0.39)
    part = partition.wirebasket((6,) * 3, 8, 3, r, c)
    st = gemslr.setup(r, c, v, part, ilu_shift=0.05, **FULL)
    A = sp.csr_matrix((v, c, r)).toarray()
    m = np.mean(np.abs(np.diag(A)))
    Ap = A[np.ix_(part.perm, part.perm)]
    for l, lv in enumerate(st.levels):
        a, b = lv.start, lv.start + lv.d
        B = Ap[a:b, a:b].copy()
        if l == st.nlevels:
            lab = np.repeat(np.arange(len(lv.blocks) - 1), np.diff(lv.blocks))
            B[lab[:, None] != lab[None, :]] = 0
        LU = (lv.Lf.toarray() + np.eye(lv.d)) @ lv.Uf.toarray()
        np.testing.assert_allclose(LU, B + 1j * 0.05 * m * np.eye(lv.d), atol=1e-12)
        if lv.s:
            np.testing.assert_array_equal(lv.E.toarray(), Ap[b:, a:b])


def test_zero_shift_is_unshifted_setup():
    r, c, v = wl.helmholtz3d(6, 0.39)
    part = partition.wirebasket((6,) * 3, 8, 3, r, c)
    a = gemslr.setup(r, c, v, part, ilu="ilut", drop_tol=1e-4, lfil=10, rank=4)
    b = gemslr.setup(r, c, v, part, ilu="ilut", drop_tol=1e-4, lfil=10, rank=4, ilu_shift=0.0)
    for la, lb in zip(a.levels, b.levels):
        np.testing.assert_array_equal(la.Uf.toarray(), lb.Uf.toarray())
    with pytest.raises(ValueError):
        rr, cc, vv = wl.laplace2d(8)
        gemslr.setup(rr, cc, vv, partition.wirebasket((8, 8), 4, 2, rr, cc), ilu_shift=0.05)


# ---------------------------------------------------------------- FGMRES

def test_fgmres_identity_preconditioner_full_space():
    rs = np.random.default_rng(5)
    n = 40
    A = np.eye(n) * 3 + rs.standard_normal((n, n)) * 0.3
    b = rs.standard_normal(n)
    x, info = fgmres.fgmres(lambda z: A @ z, lambda z: z, b, tol=1e-13,
                            restart=n)
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-11)
    assert info["converged"] and info["its"] <= n


def test_fgmres_complex_restarted():
    rs = np.random.default_rng(6)
    n = 60
    A = np.eye(n) * (2 + 1j) + (rs.standard_normal((n, n)) +
                                1j * rs.standard_normal((n, n))) * 0.15
    b = rs.standard_normal(n) + 1j * rs.standard_normal(n)
    x, info = fgmres.fgmres(lambda z: A @ z, lambda z: z, b, tol=1e-12,
                            restart=7)
    assert info["converged"]
    np.testing.assert_allclose(x, np.linalg.solve(A, b), rtol=1e-10)
    assert np.linalg.norm(b - A @ x) <= 1e-12 * np.linalg.norm(b)


def test_gemslr_solve_matches_dense_lu_laplace32():
    w = wl.laplace2d_32()
    part = partition.wirebasket(w.dims, w.nparts, w.levels, w.rowptr, w.col)
    st = gemslr.setup(w.rowptr, w.col, w.val, part, ilu=w.ilu, rank=w.rank)
    A = sp.csr_matrix((w.val, w.col, w.rowptr), shape=(w.n, w.n))
    x, info = fgmres.fgmres(lambda z: A @ z, lambda z: gemslr.apply(st, z),
                            w.b, tol=1e-13, restart=w.restart)
    ref = sla.lu_solve(sla.lu_factor(A.toarray()), w.b)
    assert info["converged"]
    cond = np.linalg.cond(A.toarray())
    assert np.linalg.norm(x - ref) <= cond * 1e-13 * np.linalg.norm(ref)
    assert np.linalg.norm(x - w.x_true) <= 1e-10 * np.linalg.norm(w.x_true)
    # the preconditioner must actually help
    _, plain = fgmres.fgmres(lambda z: A @ z, lambda z: z, w.b, tol=1e-8,
                             restart=w.restart)
    _, prec = fgmres.fgmres(lambda z: A @ z, lambda z: gemslr.apply(st, z),
                            w.b, tol=1e-8, restart=w.restart)
    assert prec["its"] < plain["its"] / 3


# ---------------------------------------------------------------- MLP

def _params(rs, F, Hd, K):
    return [rs.standard_normal((F, Hd)) / np.sqrt(F), rs.standard_normal(Hd) * .1,
            rs.standard_normal((Hd, Hd)) / np.sqrt(Hd), rs.standard_normal(Hd) * .1,
            rs.standard_normal((Hd, K)) / np.sqrt(Hd), rs.standard_normal(K) * .1]


def test_mlp_gradient_central_differences():
    rs = np.random.default_rng(8)
    F, Hd, K, s = 5, 7, 3, 11
    P = _params(rs, F, Hd, K)
    X = rs.standard_normal((s, F))
    W, _ = np.linalg.qr(rs.standard_normal((s, K)))
    _, g = mlp.loss_and_grad(P, X, W)
    h = 1e-6
    for pi in range(len(P)):
        flat = P[pi].reshape(-1)
        for idx in range(0, flat.size, max(1, flat.size // 6)):
            old = flat[idx]
            flat[idx] = old + h
            lp = mlp.loss(mlp.forward(P, X)[0], W)
            flat[idx] = old - h
            lm = mlp.loss(mlp.forward(P, X)[0], W)
            flat[idx] = old
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[pi].reshape(-1)[idx]) <= 1e-6 * max(1, abs(fd))


def test_mlp_loss_zero_on_rotated_basis():
    rs = np.random.default_rng(9)
    W, _ = np.linalg.qr(rs.standard_normal((50, 4)))
    Q, _ = np.linalg.qr(rs.standard_normal((4, 4)))
    assert abs(mlp.loss(W @ Q, W)) < 1e-12
    assert mlp.loss(rs.standard_normal((50, 4)), W) > 1


def test_adam_first_step_closed_form():
    # from zero moments the bias-corrected first step is lr * g/(|g| + eps)
    g = [np.array([0.5, -2.0, 1e-3])]
    p = [np.zeros(3)]
    p1, m1, v1 = mlp.adam_step(p, g, [np.zeros(3)], [np.zeros(3)], 1,
                               lr=0.01, eps=1e-8)
    np.testing.assert_allclose(p1[0], -0.01 * g[0] / (np.abs(g[0]) + 1e-8),
                               rtol=1e-12)
