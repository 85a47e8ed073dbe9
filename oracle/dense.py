"""Dense small-lattice checks (numpy/LAPACK) -- TEST INFRASTRUCTURE.

On a 4^4 lattice D_W is a 3072 x 3072 matrix, small enough that its spectrum
and the exact matrix sign function are available from standard dense
routines (Section 2, discussion of Fig. 1).  The matrix is assembled column
by column from the oracle's stencil; everything after that is LAPACK.
"""
from __future__ import annotations

import numpy as np

from . import Lattice, dw, gamma


def dense_dw(lat: Lattice, U, m0: float) -> np.ndarray:
    """The matrix of D_W(m0) in the canonical (site, spin, colour) order."""
    n = 12 * lat.V
    M = np.empty((n, n), dtype=np.complex128)
    e = np.zeros((lat.V, 4, 3), dtype=np.complex128)
    for k in range(n):
        e.reshape(-1)[k] = 1.0
        M[:, k] = dw(lat, U, m0, e).reshape(-1)
        e.reshape(-1)[k] = 0.0
    return M


def gamma5_matrix(V: int) -> np.ndarray:
    """Gamma_5 = I_{n_L} (x) gamma_5 (x) I_3 (the Kronecker order of Section 2)."""
    return np.kron(np.kron(np.eye(V), gamma(4)), np.eye(3))


def sign_hermitian(H: np.ndarray) -> np.ndarray:
    """Exact sign of a Hermitian matrix: W sign(Delta) W^H from eigh."""
    w, W = np.linalg.eigh(H)
    return (W * np.sign(w)) @ W.conj().T


def sign_q_exact(lat: Lattice, U, m0: float):
    """(sign(Q), eigenvalues of Q) with Q = Gamma_5 D_W(m0)."""
    D = dense_dw(lat, U, m0)
    Q = gamma5_matrix(lat.V) @ D
    w, W = np.linalg.eigh(Q)
    return (W * np.sign(w)) @ W.conj().T, w


def sign_q_polar(lat: Lattice, U, m0: float) -> np.ndarray:
    """sign(Q) from the polar factor of D_W (Lemma 2): with D_W = U S V^H,
    Gamma_5 sign(Gamma_5 D_W) = U V^H, so sign(Q) = Gamma_5 U V^H."""
    D = dense_dw(lat, U, m0)
    u, s, vh = np.linalg.svd(D)
    return gamma5_matrix(lat.V) @ (u @ vh)


def overlap_exact(lat: Lattice, U, rho: float) -> np.ndarray:
    """D_ov = rho (I + Gamma_5 sign(Gamma_5 D_W(-rho))) as a dense matrix."""
    S, _ = sign_q_exact(lat, U, -rho)
    n = S.shape[0]
    return rho * (np.eye(n) + gamma5_matrix(lat.V) @ S)
