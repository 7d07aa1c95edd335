"""Host Schur forms of the low-rank setup (the m x m Rayleigh matrices of
thick-restart Arnoldi, Sec. 2.3): schur_real (double-shift QR on real
matrices, then complex-triangular 2x2 blocks) and schur_complex.  The
library's host source is compiled into a small driver with g++; its factors
must satisfy A = Q T Q^H, Q^H Q = I, T upper triangular exactly, and diag(T)
must be the eigenvalues numpy's LAPACK computes, on random matrices, on
spectra fixed by construction (conjugate pairs, repeated and real-split
2x2 blocks, hidden by an orthogonal similarity) and on the degenerate cases
(1x1, zero, identity, already triangular, an arrow-row restart matrix)."""
import os
import shutil
import struct
import subprocess

import numpy as np
import pytest
from scipy.optimize import linear_sum_assignment

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2205_03224_amd", "csrc")


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    if not shutil.which("g++"):
        pytest.skip("no g++")
    d = tmp_path_factory.mktemp("schur")
    exe = str(d / "schur_driver")
    subprocess.run(["g++", "-O2", "-std=c++17", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC,
                    os.path.join(ROOT, "tests", "host", "schur_driver.cpp"),
                    os.path.join(CSRC, "host_dense.cpp"), "-o", exe], check=True)
    return exe, d


def run(driver, mats):
    exe, d = driver
    fin, fout = str(d / "in.bin"), str(d / "out.bin")
    with open(fin, "wb") as f:
        f.write(struct.pack("i", len(mats)))
        for A in mats:
            cx = np.iscomplexobj(A)
            f.write(struct.pack("ii", A.shape[0], int(cx)))
            a = np.asfortranarray(A)
            if cx:
                f.write(np.ascontiguousarray(a.T.reshape(-1).view(np.float64)).tobytes())
            else:
                f.write(np.ascontiguousarray(a.T.reshape(-1)).tobytes())
    subprocess.run([exe, fin, fout], check=True)
    raw = np.fromfile(fout, dtype=np.complex128)
    out, o = [], 0
    for A in mats:
        m = A.shape[0]
        T = raw[o:o + m * m].reshape(m, m).T
        Q = raw[o + m * m:o + 2 * m * m].reshape(m, m).T
        out.append((T, Q))
        o += 2 * m * m
    return out


def check(A, T, Q, eig_tol=1e-9):
    m = A.shape[0]
    an = max(np.abs(A).max(), 1.0)
    assert np.abs(Q @ T @ Q.conj().T - A).max() <= 1e-13 * m * an
    assert np.abs(Q.conj().T @ Q - np.eye(m)).max() <= 1e-13 * m
    assert np.all(np.tril(T, -1) == 0)
    ref = np.linalg.eigvals(A) if m else np.zeros(0)
    got = np.diag(T)
    # every eigenvalue matched to a distinct diagonal entry (optimal
    # assignment on the distances)
    cost = np.abs(ref[:, None] - got[None, :])
    r, c = linear_sum_assignment(cost)
    assert cost[r, c].max(initial=0.0) <= eig_tol * an


def hidden(D, seed):
    """D under a random orthogonal similarity."""
    rs = np.random.default_rng(seed)
    Qo, _ = np.linalg.qr(rs.standard_normal(D.shape))
    return Qo @ D @ Qo.T


def rotations(pairs, reals):
    blocks = [np.array([[a, b], [-b, a]]) for a, b in pairs] + [np.array([[r]]) for r in reals]
    m = sum(b.shape[0] for b in blocks)
    D = np.zeros((m, m))
    i = 0
    for b in blocks:
        k = b.shape[0]
        D[i:i + k, i:i + k] = b
        i += k
    return D


@pytest.mark.parametrize("m", [1, 2, 3, 4, 7, 33, 66, 130])
def test_real_random(driver, m):
    A = np.random.default_rng(m).standard_normal((m, m))
    (T, Q), = run(driver, [A])
    check(A, T, Q)


def test_real_constructed_spectra(driver):
    mats = [
        # conjugate pairs and real values, known exactly
        hidden(rotations([(1.0, 2.0), (0.5, 0.25), (-3.0, 1.0)], [2.0, -1.0, 0.1]), 1),
        # a 2x2 block with real eigenvalues (must be split): [[1, 4], [1, 1]]
        # has eigenvalues 3 and -1
        hidden(np.block([[np.array([[1.0, 4.0], [1.0, 1.0]]), np.zeros((2, 3))],
                         [np.zeros((3, 2)), np.diag([5.0, 6.0, 7.0])]]), 2),
        # repeated conjugate pair
        hidden(rotations([(0.3, 0.7), (0.3, 0.7), (0.3, 0.7)], [0.3]), 3),
        # pure rotations (eigenvalues on the unit circle)
        hidden(rotations([(np.cos(t), np.sin(t)) for t in (0.1, 0.9, 2.0)], []), 4),
    ]
    expect = [
        [1 + 2j, 1 - 2j, 0.5 + 0.25j, 0.5 - 0.25j, -3 + 1j, -3 - 1j, 2, -1, 0.1],
        [3, -1, 5, 6, 7],
    ]
    res = run(driver, mats)
    for A, (T, Q) in zip(mats, res):
        check(A, T, Q, eig_tol=1e-8)
    for e, (T, _) in zip(expect, res):
        got = sorted(np.diag(T), key=lambda z: (round(z.real, 6), round(z.imag, 6)))
        want = sorted(np.array(e, dtype=complex), key=lambda z: (round(z.real, 6), round(z.imag, 6)))
        assert np.allclose(got, want, atol=1e-10)


def test_real_degenerate(driver):
    rs = np.random.default_rng(9)
    m = 12
    arrow = np.triu(rs.standard_normal((m, m)), -1)
    arrow[:5, :5] = np.triu(rs.standard_normal((5, 5)))
    arrow[5, :5] = rs.standard_normal(5)       # the restart's arrow row
    mats = [np.zeros((1, 1)), np.array([[2.5]]), np.zeros((6, 6)), np.eye(7),
            np.triu(rs.standard_normal((9, 9))), arrow]
    for A, (T, Q) in zip(mats, run(driver, mats)):
        check(A, T, Q)


def test_real_clustered_spectrum(driver):
    """A tight cluster, c I + 1e-6 N: the shifts sit within 1e-6 of the
    diagonal, where the expanded shift polynomial h00^2 - (s1 + s2) h00 +
    s1 s2 cancels to rounding noise and the double-shift steps stop making
    progress (the form the last level's Rayleigh matrix takes when C_last is
    a scaled identity).  N: coupling of 3 x 3 x 3 grid neighbours in a
    lexicographic order (block lower and upper parts, zero subdiagonal
    entries between lines), and a dense random N."""
    rs = np.random.default_rng(27)
    g = 3
    idx = np.arange(g ** 3).reshape(g, g, g)
    N = np.zeros((g ** 3, g ** 3))
    for ax in range(3):
        a0 = np.take(idx, range(g - 1), axis=ax).ravel()
        a1 = np.take(idx, range(1, g), axis=ax).ravel()
        N[a0, a1] = rs.uniform(0.5, 1.0, a0.size)
        N[a1, a0] = rs.uniform(0.5, 1.0, a0.size)
    mats = [0.171 * np.eye(g ** 3) + 1e-6 * N,
            0.171 * np.eye(30) + 1e-6 * rs.standard_normal((30, 30)),
            -2.0 * np.eye(12) + 1e-9 * np.triu(rs.standard_normal((12, 12)), -1)]
    for A, (T, Q) in zip(mats, run(driver, mats)):
        check(A, T, Q, eig_tol=1e-8)


@pytest.mark.parametrize("m", [1, 2, 5, 40])
def test_complex_random(driver, m):
    rs = np.random.default_rng(100 + m)
    A = rs.standard_normal((m, m)) + 1j * rs.standard_normal((m, m))
    (T, Q), = run(driver, [A])
    check(A, T, Q)
