"""Low-mode deflation of sign(Q) -- TEST INFRASTRUCTURE.

Only tests/ and bench.py's cpu_baseline leg may use this module; it shares no
code with the GPU library.

Section 5.2 (deflation): with the k eigenvalues lambda_1..lambda_k of
Q = Gamma_5 D_W smallest in modulus and their normalised eigenvectors
xi_1..xi_k, Xi = [xi_1 | .. | xi_k] and Pi = I - Xi Xi^H,

    sign(Q) chi = sum_i sign(lambda_i) (xi_i^H chi) xi_i + sign(Q) Pi chi,

(the paper prints xi^H in the sum; the i-th eigenvector is meant).  The
first term is exact; the second is left to any approximation of the sign
function, which then only has to be accurate for |lambda| >= |lambda_{k+1}|.

`low_modes_dense` is the definition of the eigenpairs written out with a
dense LAPACK eigendecomposition (small lattices only); `deflated_sign` and
`deflated_overlap` take the formula's steps in the paper's order with any
callable for the remaining sign(Q) Pi chi.
"""
from __future__ import annotations

import numpy as np

from . import Lattice, gamma5
from .dense import dense_dw, gamma5_matrix


def low_modes_dense(lat: Lattice, U, m0: float, k: int):
    """The k eigenpairs of Q = Gamma_5 D_W(m0) smallest in |lambda| (dense
    eigh; orthonormal eigenvectors).  Returns (lambda[k], xi (k, V, 4, 3),
    all eigenvalues sorted by modulus)."""
    Q = gamma5_matrix(lat.V) @ dense_dw(lat, U, m0)
    w, W = np.linalg.eigh(0.5 * (Q + Q.conj().T))
    order = np.argsort(np.abs(w), kind="stable")
    lam = w[order[:k]]
    xi = W[:, order[:k]].T.reshape(k, lat.V, 4, 3)
    return lam, xi, w[order]


def deflated_sign(apply_sign, xi, lam, chi):
    """sum_i sign(lambda_i) (xi_i^H chi) xi_i + apply_sign(Pi chi)."""
    chi = np.asarray(chi, dtype=np.complex128)
    c = np.array([np.vdot(x, chi) for x in xi])          # xi_i^H chi
    proj = chi - np.tensordot(c, xi, axes=1)             # Pi chi
    return np.tensordot(np.sign(lam) * c, xi, axes=1) + apply_sign(proj)


def deflated_overlap(apply_sign, xi, lam, chi, rho: float):
    """rho (chi + Gamma_5 sign(Q) chi) with the deflated sign function
    (eq. (overlap_def), massless normalisation, Q = Gamma_5 D_W(-rho))."""
    chi = np.asarray(chi, dtype=np.complex128)
    return rho * (chi + gamma5(deflated_sign(apply_sign, xi, lam, chi)))
