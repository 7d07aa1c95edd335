"""Seeded synthetic inputs: the sparse systems the solver is exercised on.

This module builds the test matrices and right-hand sides only.  It holds
none of the preconditioner's arithmetic (no partitioning, factorisation,
low-rank or Krylov step), so both the GPU path and the CPU oracle can be fed
from it.

Every operator is a finite-difference discretisation on the open unit square
or cube with homogeneous Dirichlet boundary conditions eliminated, rows scaled
by h^2 with h = 1/(N+1).  Unknowns are numbered lexicographically,
index = x + N*y + N^2*z (x fastest).  The model problem of the paper's
experiments is the 7-point stencil on (0,1)^3 (Sec. 5.1); the variants below
(convection, complex shift, log-normal diffusion) are the synthetic
stand-ins for its convection-diffusion and Helmholtz workloads.

Matrices are returned as plain CSR arrays: rowptr (int64, n+1), col (int32,
sorted within each row), val (float64 or complex128).
"""
from __future__ import annotations

from dataclasses import dataclass, field
import numpy as np


# ----------------------------------------------------------------------------
# stencil assembly
# ----------------------------------------------------------------------------

def _assemble(dims, diag, coef_minus, coef_plus):
    """Assemble a nearest-neighbour stencil on a lexicographic grid.

    diag: (n,) diagonal values.
    coef_minus[a], coef_plus[a]: (n,) coupling of row i to its -a / +a
    neighbour (ignored where the neighbour is outside the grid).
    """
    dims = tuple(int(d) for d in dims)
    n = int(np.prod(dims))
    coords = np.indices(dims[::-1]).reshape(len(dims), -1)[::-1]  # coords[a][i]
    strides = [int(np.prod(dims[:a])) for a in range(len(dims))]
    rows, cols, vals = [np.arange(n)], [np.arange(n)], [diag]
    for a in range(len(dims)):
        c = coords[a]
        m = c > 0
        rows.append(np.nonzero(m)[0])
        cols.append(np.nonzero(m)[0] - strides[a])
        vals.append(coef_minus[a][m])
        m = c < dims[a] - 1
        rows.append(np.nonzero(m)[0])
        cols.append(np.nonzero(m)[0] + strides[a])
        vals.append(coef_plus[a][m])
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    vals = np.concatenate([np.asarray(v) for v in vals])
    order = np.lexsort((cols, rows))
    rows, cols, vals = rows[order], cols[order], vals[order]
    rowptr = np.zeros(n + 1, dtype=np.int64)
    np.add.at(rowptr, rows + 1, 1)
    rowptr = np.cumsum(rowptr)
    return rowptr, cols.astype(np.int32), vals


def _const(n, v, dtype=np.float64):
    return np.full(n, v, dtype=dtype)


def laplace2d(N):
    """5-point Laplacian on an N x N grid: diagonal 4, neighbours -1."""
    n = N * N
    return _assemble((N, N), _const(n, 4.0), [_const(n, -1.0)] * 2,
                     [_const(n, -1.0)] * 2)


def convdiff3d(N, c=(0.05, 0.05, 0.05)):
    """-Lap(u) + beta.grad(u), central differences, times h^2.

    c[a] = beta_a * h / 2 is the scaled convection coefficient on axis a, so
    the -a neighbour gets -1 - c[a] and the +a neighbour -1 + c[a]
    (beta = 0.1/h gives c = 0.05: -1.05 / -0.95).
    """
    n = N ** 3
    return _assemble((N, N, N), _const(n, 6.0),
                     [_const(n, -1.0 - c[a]) for a in range(3)],
                     [_const(n, -1.0 + c[a]) for a in range(3)])


def helmholtz3d(N, kh2, damping=0.05):
    """-Lap(u) - k^2 (1 + i*damping) u, times h^2; kh2 = (k h)^2."""
    n = N ** 3
    d = 6.0 - kh2 * (1.0 + 1j * damping)
    return _assemble((N, N, N), _const(n, d, np.complex128),
                     [_const(n, -1.0 + 0j, np.complex128)] * 3,
                     [_const(n, -1.0 + 0j, np.complex128)] * 3)


def gaussian_field(N, corr_len_h, rng):
    """Zero-mean, unit-variance Gaussian field on an N^3 grid.

    White noise is filtered in Fourier space with a Gaussian kernel of
    standard deviation corr_len/sqrt(2) (grid units), which gives a
    squared-exponential covariance of length corr_len; the result is
    normalised to zero mean and unit sample variance.
    """
    w = rng.standard_normal((N, N, N))
    s = corr_len_h / np.sqrt(2.0)
    k = np.fft.fftfreq(N) * 2.0 * np.pi
    kx, ky, kz = np.meshgrid(k, k, k, indexing="ij")
    filt = np.exp(-0.5 * s * s * (kx ** 2 + ky ** 2 + kz ** 2))
    g = np.real(np.fft.ifftn(np.fft.fftn(w) * filt))
    g = g - g.mean()
    return g / g.std()


def lognormal_convdiff3d(N, seed, sigma=1.0, corr_len_h=8.0):
    """-div(kappa grad u) + v.grad(u) times h^2 with kappa = exp(sigma*g).

    g is gaussian_field(N, corr_len_h) drawn from default_rng(seed) first,
    then v ~ U[-1,1]^3 from the same generator.  Face coefficients are the
    harmonic mean of the two cell values (the cell's own value on a boundary
    face); the convection term uses v literally (scaled coefficient v*h/2).
    Returns (rowptr, col, val, kappa, v).
    """
    rng = np.random.default_rng(seed)
    g = gaussian_field(N, corr_len_h, rng)
    v = rng.uniform(-1.0, 1.0, 3)
    h = 1.0 / (N + 1)
    kap = np.exp(sigma * g)  # indexed [x, y, z]
    kflat = kap.transpose(2, 1, 0).reshape(-1)  # lexicographic, x fastest
    n = N ** 3
    strides = [1, N, N * N]
    coords = np.indices((N, N, N)).reshape(3, -1)[::-1]
    diag = np.zeros(n)
    cm, cp = [], []
    for a in range(3):
        c = coords[a]
        nb_m = np.where(c > 0, np.arange(n) - strides[a], np.arange(n))
        nb_p = np.where(c < N - 1, np.arange(n) + strides[a], np.arange(n))
        km = 2 * kflat * kflat[nb_m] / (kflat + kflat[nb_m])
        kp = 2 * kflat * kflat[nb_p] / (kflat + kflat[nb_p])
        diag += km + kp
        ca = v[a] * h / 2.0
        cm.append(-km - ca)
        cp.append(-kp + ca)
    rowptr, col, val = _assemble((N, N, N), diag, cm, cp)
    return rowptr, col, val, kflat, v


# ----------------------------------------------------------------------------
# right-hand side
# ----------------------------------------------------------------------------

def csr_matvec(rowptr, col, val, x):
    """y = A x for CSR arrays (used only to form b = A x*)."""
    prod = val * x[col]
    y = np.zeros(len(rowptr) - 1, dtype=np.result_type(val, x))
    nz = np.diff(rowptr) > 0
    y[nz] = np.add.reduceat(prod, rowptr[:-1][nz])
    return y


def exact_solution(n, seed, complex_=False):
    """x* ~ U(-1,1) from default_rng(seed); real part drawn first."""
    rng = np.random.default_rng(seed)
    xr = rng.uniform(-1.0, 1.0, n)
    if not complex_:
        return xr
    xi = rng.uniform(-1.0, 1.0, n)
    return xr + 1j * xi


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------

@dataclass
class Workload:
    name: str
    dims: tuple
    rowptr: np.ndarray
    col: np.ndarray
    val: np.ndarray
    levels: int
    nparts: int
    rank: int
    ilu: str            # "ilu0" or "ilut"
    drop_tol: float
    lfil: int
    restart: int
    tol: float
    x_true: np.ndarray = None
    b: np.ndarray = None
    extra: dict = field(default_factory=dict)

    @property
    def n(self):
        return len(self.rowptr) - 1

    @property
    def nnz(self):
        return int(self.rowptr[-1])

    @property
    def is_complex(self):
        return np.iscomplexobj(self.val)


def _finish(w, seed):
    w.x_true = exact_solution(w.n, seed, w.is_complex)
    w.b = csr_matvec(w.rowptr, w.col, w.val, w.x_true)
    return w


def laplace2d_32(N=32, seed=0):
    """2-D 5-point Laplacian, 2 levels, 4 subdomains, ILU(0), rank 8."""
    r, c, v = laplace2d(N)
    return _finish(Workload(f"laplace2d_{N}", (N, N), r, c, v, levels=2,
                            nparts=4, rank=8, ilu="ilu0", drop_tol=0.0,
                            lfil=0, restart=30, tol=1e-8), seed)


def convdiff3d_64(N=64, nparts=64, seed=0):
    """3-D 7-point convection-diffusion, beta = 0.1/h on every axis, 3 levels,
    ILUT(1e-3, lfil 10), rank 32."""
    r, c, v = convdiff3d(N, (0.05, 0.05, 0.05))
    return _finish(Workload(f"convdiff3d_{N}", (N, N, N), r, c, v, levels=3,
                            nparts=nparts, rank=32, ilu="ilut",
                            drop_tol=1e-3, lfil=10, restart=50, tol=1e-8),
                   seed)


def convdiff3d_128(N=128, nparts=512, seed=0):
    """The convection-diffusion operator at 128^3 (beta = 0.1/h, h = 1/129),
    512 subdomains; the roofline and mixed-precision workload."""
    w = convdiff3d_64(N, nparts, seed)
    return w


def helmholtz3d_128(N=128, nparts=512, seed=0, levels=5):
    """Complex-shifted Helmholtz, 10 points per wavelength: (kh)^2 = (2pi/10)^2,
    damping 0.05; 5 levels requested, ILUT(1e-4, lfil 10), rank 64."""
    kh2 = (2.0 * np.pi / 10.0) ** 2
    r, c, v = helmholtz3d(N, kh2, 0.05)
    return _finish(Workload(f"helmholtz3d_{N}", (N, N, N), r, c, v,
                            levels=levels, nparts=nparts, rank=64, ilu="ilut",
                            drop_tol=1e-4, lfil=10, restart=100, tol=1e-8),
                   seed)


def lognormal_convdiff3d_64(instance, N=64, nparts=64, seed_rhs=0):
    """One member of the log-normal-diffusion / random-convection family."""
    r, c, v, kap, vel = lognormal_convdiff3d(N, instance)
    w = Workload(f"lognormal_convdiff3d_{N}_i{instance}", (N, N, N), r, c, v,
                 levels=3, nparts=nparts, rank=32, ilu="ilut", drop_tol=1e-3,
                 lfil=10, restart=50, tol=1e-8,
                 extra={"kappa": kap, "velocity": vel, "instance": instance})
    return _finish(w, seed_rhs)


TRAIN_INSTANCES = range(0, 512)
HELDOUT_INSTANCES = range(100000, 100064)
