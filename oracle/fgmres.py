"""Right-preconditioned flexible GMRES(m) (Saad 1993), the outer accelerator
the paper runs around the GeMSLR apply (Sec. 4.1 and the FGMRES settings of
Sec. 5: restart 50, relative-residual stop, x0 = 0).

Each iteration j: z_j = M^{-1} v_j (the preconditioner may change between
iterations), w = A z_j, classical Gram-Schmidt against v_0..v_j with one
re-orthogonalisation pass, h_{j+1,j} = ||w||, v_{j+1} = w / h_{j+1,j}; the
least-squares problem min ||beta e_1 - H_j y|| is kept triangular with
Givens rotations, so |g_{j+1}| is the residual-norm estimate.  At the end of
a cycle x += Z_j y.  The iteration stops when the estimate is <= tol ||b||
and the true residual ||b - A x|| / ||b|| is <= tol, or after maxit
iterations (the paper flags failure at 1000).

Complex Givens rotation G = [[c, s], [-conj(s), c]] with c real:
c = |a|/t, s = (a/|a|) conj(b)/t, t = sqrt(|a|^2 + |b|^2), so G [a; b] =
[(a/|a|) t; 0]; for a = 0: c = 0, s = conj(b)/|b|.
"""
import numpy as np


def givens(a, b):
    if b == 0:
        return 1.0, 0.0 * a, a
    if a == 0:
        return 0.0, np.conj(b) / abs(b), abs(b) + 0.0 * a
    t = np.hypot(abs(a), abs(b))
    ph = a / abs(a)
    return abs(a) / t, ph * np.conj(b) / t, ph * t


def fgmres(matvec, precond, b, x0=None, tol=1e-8, restart=50, maxit=1000):
    n = len(b)
    dtype = np.result_type(b, np.float64)
    x = np.zeros(n, dtype=dtype) if x0 is None else np.array(x0, dtype=dtype)
    nb = np.linalg.norm(b)
    if nb == 0:
        return np.zeros(n, dtype=dtype), {"its": 0, "relres": 0.0,
                                          "converged": True, "history": []}
    its = 0
    history = []
    while True:
        r = b - matvec(x)
        beta = np.linalg.norm(r)
        relres = beta / nb
        if relres <= tol:
            return x, {"its": its, "relres": relres, "converged": True,
                       "history": history}
        if its >= maxit:
            return x, {"its": its, "relres": relres, "converged": False,
                       "history": history}
        m = restart
        V = np.zeros((n, m + 1), dtype=dtype)
        Z = np.zeros((n, m), dtype=dtype)
        Hh = np.zeros((m + 1, m), dtype=dtype)
        cs = np.zeros(m)
        sn = np.zeros(m, dtype=dtype)
        g = np.zeros(m + 1, dtype=dtype)
        g[0] = beta
        V[:, 0] = r / beta
        jend = 0
        for j in range(m):
            Z[:, j] = precond(V[:, j])
            w = matvec(Z[:, j])
            h = V[:, :j + 1].conj().T @ w
            w = w - V[:, :j + 1] @ h
            h2 = V[:, :j + 1].conj().T @ w
            w = w - V[:, :j + 1] @ h2
            h = h + h2
            hn = np.linalg.norm(w)
            Hh[:j + 1, j] = h
            Hh[j + 1, j] = hn
            if hn > 0:
                V[:, j + 1] = w / hn
            for i in range(j):
                t1 = cs[i] * Hh[i, j] + sn[i] * Hh[i + 1, j]
                t2 = -np.conj(sn[i]) * Hh[i, j] + cs[i] * Hh[i + 1, j]
                Hh[i, j], Hh[i + 1, j] = t1, t2
            c, s, rr = givens(Hh[j, j], Hh[j + 1, j])
            cs[j], sn[j] = c, s
            Hh[j, j] = rr
            Hh[j + 1, j] = 0
            g[j + 1] = -np.conj(s) * g[j]
            g[j] = c * g[j]
            its += 1
            jend = j + 1
            history.append(abs(g[j + 1]) / nb)
            if abs(g[j + 1]) <= tol * nb or its >= maxit or hn == 0:
                break
        # back substitution for y
        y = np.zeros(jend, dtype=dtype)
        for i in range(jend - 1, -1, -1):
            y[i] = (g[i] - Hh[i, i + 1:jend] @ y[i + 1:jend]) / Hh[i, i]
        x = x + Z[:, :jend] @ y
