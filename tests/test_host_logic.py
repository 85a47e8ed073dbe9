"""Host-side logic of the library checked on the CPU: the symmetric
tridiagonal eigensolver behind the Lanczos sign function (tridiag.h),
compiled here with g++, against LAPACK (numpy.linalg.eigh)."""
import ctypes
import os
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


@pytest.fixture(scope="module")
def lib(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("host") / "libtri.so")
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-fPIC", "-shared", os.path.join(HERE, "host_tridiag.cpp"),
                           "-o", out])
    lib = ctypes.CDLL(out)
    P = ctypes.c_void_p
    lib.tri_eig.argtypes = [ctypes.c_int, P, P, P, P]
    lib.tri_sign_e1.argtypes = [ctypes.c_int, P, P, ctypes.c_double, P]
    lib.herm_eig.argtypes = [ctypes.c_int, P, P, P]
    return lib


def ptr(a):
    return a.ctypes.data


@pytest.mark.parametrize("n,seed", [(1, 0), (2, 1), (7, 2), (64, 3), (300, 4)])
def test_tridiag_eig_matches_lapack(lib, n, seed):
    rng = np.random.default_rng(seed)
    d = rng.standard_normal(n)
    e = rng.standard_normal(max(n - 1, 0))
    if n > 10:
        e[n // 3] = 0.0        # a split into independent blocks
    w = np.empty(n)
    z = np.empty(n * n)
    assert lib.tri_eig(n, ptr(d), ptr(e), ptr(w), ptr(z)) == 0
    T = np.diag(d) + np.diag(e, 1) + np.diag(e, -1)
    Z = z.reshape(n, n)
    ref = np.linalg.eigvalsh(T)
    assert np.allclose(np.sort(w), ref, atol=1e-12 * max(1.0, np.abs(ref).max()))
    assert np.allclose(T @ Z, Z * w, atol=1e-11 * max(1.0, np.abs(ref).max()))
    assert np.allclose(Z.T @ Z, np.eye(n), atol=1e-12)


@pytest.mark.parametrize("n,seed", [(1, 8), (2, 10), (120, 9), (700, 11)])
def test_tridiag_sign_e1_matches_lapack(lib, n, seed):
    """sign(T) e_1 from the first eigenvector row and the logged rotations
    (O(n^2)) equals Z sign(theta) Z^T e_1 from LAPACK."""
    rng = np.random.default_rng(seed)
    a = rng.standard_normal(n)
    b = np.abs(rng.standard_normal(n - 1)) + 0.1
    c = np.empty(n)
    assert lib.tri_sign_e1(n, ptr(a), ptr(b), 2.5, ptr(c)) == 0
    T = np.diag(a) + np.diag(b, 1) + np.diag(b, -1)
    th, Z = np.linalg.eigh(T)
    ref = 2.5 * (Z @ (np.sign(th) * Z[0]))
    assert np.allclose(c, ref, atol=1e-12)


@pytest.mark.parametrize("n,seed,degenerate", [(1, 0, False), (2, 1, False), (7, 2, False), (40, 3, False),
                                               (40, 4, True), (128, 5, False)])
def test_hermitian_jacobi_matches_lapack(lib, n, seed, degenerate):
    """The Rayleigh-Ritz step's Hermitian Jacobi solver: eigenvalues as LAPACK,
    A V = V diag(w) and V unitary, also with a spectrum of +-lambda pairs
    (the degeneracy of Q^2 that the step resolves)."""
    rng = np.random.default_rng(seed)
    if degenerate:
        Qm, _ = np.linalg.qr(rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)))
        lam = np.repeat(rng.uniform(0.5, 2.0, n // 2), 2) * np.tile([1.0, -1.0], n // 2)
        lam[:4] = [0.7, 0.7, -0.7, 1e-3]
        A = (Qm * lam) @ Qm.conj().T
    else:
        X = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n))
        A = X + X.conj().T
    A = 0.5 * (A + A.conj().T)
    a = np.ascontiguousarray(A).view(np.float64).copy()
    w = np.empty(n)
    v = np.empty(2 * n * n)
    assert lib.herm_eig(n, ptr(a), ptr(w), ptr(v)) == 0
    V = v.view(np.complex128).reshape(n, n)
    ref = np.linalg.eigvalsh(A)
    scale = max(1.0, np.abs(ref).max())
    assert np.allclose(np.sort(w), ref, atol=1e-12 * scale)
    assert np.abs(A @ V - V * w).max() < 1e-11 * scale
    assert np.abs(V.conj().T @ V - np.eye(n)).max() < 1e-12
