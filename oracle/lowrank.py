"""Low-rank correction of the Schur complement (Sec. 2.2-2.3).

For G = E B^{-1} F C^{-1} with complex Schur form G = W R W^H the paper
writes S = (I - G) C and, by Sherman-Morrison-Woodbury,
    S^{-1} = C^{-1} + C^{-1} W [(I - R)^{-1} - I] W^H        (eq. gemslr4)
and truncates to the k leading Schur vectors (eq. gemslr6).  In practice G
is replaced by G_hat = E (U^{-1} L^{-1}) F C^{-1} and its leading Schur
vectors are approximated from an m-step Arnoldi relation
G_hat V_m = V_m H_m + beta v_{m+1} e_m^H with H_m = Q T Q^H,
W_k = V_m Q_k, R_k = T_k (Sec. 2.3), using thick-restart Arnoldi with cycle
length m = 2k and Ritz values accurate to two digits (Sec. 4.2, Sec. 5).

Readings of points the paper leaves open (each listed in the design notes):
  * "leading" Schur vectors: Ritz values ordered by |theta/(1-theta)|
    descending -- the magnitude of the correction's eigenvalue
    gamma/(1-gamma) (Sec. 2.2) -- ties to larger |theta|, then lower index;
  * real A uses the real Schur form; k is raised by one rather than split a
    complex-conjugate pair;
  * convergence: every wanted Ritz pair has residual |b^H y| <= 1e-2 |theta|;
    at most 20 cycles, after which the current Ritz vectors are kept;
  * Gram-Schmidt: classical, always with one re-orthogonalisation pass;
  * restart: Krylov-Schur (Stewart 2001) truncation to the wanted Schur
    vectors, which keeps a Krylov decomposition G V = V S + v b^H;
  * Arnoldi breakdown (||w|| <= 1e-12 ||G v_j|| after orthogonalisation):
    the subspace is invariant, the subdiagonal entry is set to 0 and the
    basis continues from a fresh generator vector orthogonalised against it;
  * small problems (s <= dense_max) take the Schur form of the
    explicitly formed G_hat instead of Arnoldi.

The multiplier actually applied at run time is H = (I - R_k)^{-1} - I.
"""
import numpy as np
import scipy.linalg as sla
from scipy.linalg import lapack

from .rng import start_vector

SINGULAR_TOL = 1e-12
BREAKDOWN = 1e-12


def _fresh_direction(V, seed, salt):
    """Unit vector orthogonal to the columns of V, drawn from the start
    vector generator with seed + 0x5DEECE66D * salt."""
    s = V.shape[0]
    v = start_vector(seed + 0x5DEECE66D * salt, s).astype(V.dtype)
    for _ in range(2):
        v = v - V @ (V.conj().T @ v)
    return v / np.linalg.norm(v)


class SingularCorrectionError(ArithmeticError):
    pass


def correction_weight(theta):
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.abs(theta / (1.0 - theta))


def select_wanted(theta, k, real):
    """Boolean mask of the k wanted Ritz values (k+1 if a real-arithmetic
    conjugate pair would be split)."""
    m = len(theta)
    k = min(k, m)
    if k <= 0:
        return np.zeros(m, dtype=bool)
    wgt = correction_weight(theta)
    order = sorted(range(m), key=lambda i: (-wgt[i], -abs(theta[i]), i))
    mask = np.zeros(m, dtype=bool)
    mask[order[:k]] = True
    if real:
        # complete conjugate pairs
        for i in np.nonzero(mask)[0]:
            if abs(theta[i].imag) > 0:
                j = int(np.argmin(np.abs(theta - np.conj(theta[i]))
                                  + np.where(np.arange(m) == i, np.inf, 0)))
                mask[j] = True
    return mask


def _diag_eigs(T, real):
    """Eigenvalue belonging to each diagonal position of a (quasi-)triangular
    Schur factor."""
    m = T.shape[0]
    ev = np.zeros(m, dtype=np.complex128)
    if not real:
        return np.diag(T).astype(np.complex128)
    j = 0
    while j < m:
        if j + 1 < m and T[j + 1, j] != 0.0:
            ev[j:j + 2] = np.linalg.eigvals(T[j:j + 2, j:j + 2])
            j += 2
        else:
            ev[j] = T[j, j]
            j += 1
    return ev


def ordered_schur(Hm, k, real):
    """Schur form Hm = Q T Q^H reordered so the wanted values lead.

    Returns (T, Q, kk, theta_wanted) with kk = number of wanted values."""
    if real:
        T, Q = sla.schur(Hm, output="real")
    else:
        T, Q = sla.schur(Hm.astype(np.complex128), output="complex")
    ev = _diag_eigs(T, real)
    sel = select_wanted(ev, k, real)
    kk = int(sel.sum())
    if kk == 0:
        return T, Q, 0, np.zeros(0, np.complex128)
    fn = lapack.dtrsen if real else lapack.ztrsen
    res = fn(sel.astype(np.int32), T, Q, job="N", wantq=1)
    T, Q, info = res[0], res[1], res[-1]
    if info != 0:
        raise RuntimeError(f"trsen failed: {info}")
    return T, Q, kk, _diag_eigs(T, real)[:kk]


def finish(W, R):
    """H = (I - R)^{-1} - I for the k x k block R."""
    k = R.shape[0]
    if k == 0:
        return np.zeros((0, 0), dtype=R.dtype)
    theta = np.linalg.eigvals(R) if k else np.zeros(0)
    if np.any(np.abs(1.0 - theta) < SINGULAR_TOL):
        raise SingularCorrectionError("(I - R_k) is singular")
    I = np.eye(k, dtype=R.dtype)
    return np.linalg.solve(I - R, I) - I


def dense_lowrank(G, k, real):
    """Leading k Schur vectors of an explicitly formed G."""
    T, Q, kk, theta = ordered_schur(G, k, real)
    return Q[:, :kk], T[:kk, :kk]


def krylov_schur(matvec, s, k, real, seed=0, tol=1e-2, max_cycles=20):
    """Thick-restart (Krylov-Schur) Arnoldi for the k wanted Schur vectors of
    the s x s operator `matvec`.  Returns (W, R, info)."""
    dtype = np.float64 if real else np.complex128
    k = min(k, s)
    m = min(2 * k, s)
    if m <= k:
        m = min(k + 1, s)
    V = np.zeros((s, m + 1), dtype=dtype)
    S = np.zeros((m + 1, m), dtype=dtype)
    v0 = start_vector(seed, s).astype(dtype)
    V[:, 0] = v0 / np.linalg.norm(v0)
    j0 = 0
    nmv = 0
    info = {"cycles": 0, "converged": False, "breakdowns": 0}
    for cycle in range(max_cycles):
        for j in range(j0, m):
            w = matvec(V[:, j])
            nmv += 1
            wnorm = np.linalg.norm(w)
            h = V[:, :j + 1].conj().T @ w
            w = w - V[:, :j + 1] @ h
            h2 = V[:, :j + 1].conj().T @ w
            w = w - V[:, :j + 1] @ h2
            h = h + h2
            beta = np.linalg.norm(w)
            S[:j + 1, j] = h
            if beta > BREAKDOWN * wnorm:
                S[j + 1, j] = beta
                V[:, j + 1] = w / beta
            else:
                # invariant subspace found: continue from a fresh direction
                info["breakdowns"] += 1
                S[j + 1, j] = 0.0
                V[:, j + 1] = _fresh_direction(V[:, :j + 1], seed, nmv) \
                    if j + 1 < m else 0.0
        info["cycles"] = cycle + 1
        Sm = S[:m, :m]
        b = S[m, :m]                       # G V_m = V_m S_m + v_{m+1} b
        T, Q, kk, theta = ordered_schur(Sm, k, real)
        ev, Y = np.linalg.eig(T[:kk, :kk])
        bq = b @ Q[:, :kk]
        res = np.abs(bq @ Y) / np.linalg.norm(Y, axis=0)
        conv = bool(np.all(res <= tol * np.abs(ev)))
        if conv or cycle == max_cycles - 1 or kk >= m:
            info["converged"] = conv
            info["matvecs"] = nmv
            info["ritz"] = ev
            W = V[:, :m] @ Q[:, :kk]
            return W, T[:kk, :kk], info
        # thick restart: keep the wanted Schur vectors
        Vk = V[:, :m] @ Q[:, :kk]
        vnext = V[:, m].copy()
        S[:] = 0
        S[:kk, :kk] = T[:kk, :kk]
        S[kk, :kk] = bq
        V[:] = 0
        V[:, :kk] = Vk
        V[:, kk] = vnext
        j0 = kk
    raise AssertionError("unreachable")
