"""Outer-solver oracle: restarted GMRES for D_ov psi = eta -- TEST INFRASTRUCTURE.

Only tests/ and bench.py's cpu_baseline leg may use this module; it shares no
code with the GPU library.  The paper solves eq. (linsys), D_N psi = eta, with
GMRES(100), restarted GMRES with cycle length 100 (Section 5, "Accuracy of the
preconditioner"), and with flexible GMRES when a preconditioner is used.  The
solution does not depend on the method, so the oracle is plain GMRES(m): the
Arnoldi process with modified Gram-Schmidt, and at each restart the small
Hessenberg least-squares problem min |beta e_1 - H y| solved by a library
least-squares routine.  Vectors are numpy complex128 arrays of any shape;
`apply` is any linear operator on them (for D_ov: oracle.overlap at a fixed,
tight multishift tolerance).
"""
from __future__ import annotations

import numpy as np


def gmres(apply, b, tol: float, restart: int = 100, maxiter: int = 10000):
    """x with |b - A x| <= tol |b| by GMRES(restart).  Returns (x, iterations,
    true relative residual |b - A x|/|b| recomputed at the end)."""
    b = np.asarray(b, dtype=np.complex128)
    shape = b.shape
    bv = b.reshape(-1)
    n = bv.size
    x = np.zeros(n, dtype=np.complex128)
    bnorm = np.linalg.norm(bv)
    if bnorm == 0.0:
        return x.reshape(shape), 0, 0.0
    A = lambda v: np.asarray(apply(v.reshape(shape)), dtype=np.complex128).reshape(-1)
    r = bv.copy()
    beta = bnorm
    it = 0
    while it < maxiter and beta > tol * bnorm:
        m = min(restart, maxiter - it)
        Vb = np.zeros((m + 1, n), dtype=np.complex128)
        H = np.zeros((m + 1, m), dtype=np.complex128)
        Vb[0] = r / beta
        k_used = 0
        for k in range(m):
            w = A(Vb[k])
            it += 1
            for i in range(k + 1):          # modified Gram-Schmidt
                H[i, k] = np.vdot(Vb[i], w)
                w = w - H[i, k] * Vb[i]
            H[k + 1, k] = np.linalg.norm(w)
            k_used = k + 1
            e1 = np.zeros(k + 2, dtype=np.complex128)
            e1[0] = beta
            y, *_ = np.linalg.lstsq(H[:k + 2, :k + 1], e1, rcond=None)
            res = np.linalg.norm(e1 - H[:k + 2, :k + 1] @ y)
            if H[k + 1, k] == 0.0 or res <= tol * bnorm:
                break
            Vb[k + 1] = w / H[k + 1, k]
        e1 = np.zeros(k_used + 1, dtype=np.complex128)
        e1[0] = beta
        y, *_ = np.linalg.lstsq(H[:k_used + 1, :k_used], e1, rcond=None)
        x = x + Vb[:k_used].T @ y
        r = bv - A(x)
        beta = np.linalg.norm(r)
    return x.reshape(shape), it, float(beta / bnorm)


def lanczos_sign(apply_q, b, steps: int):
    """The Lanczos approximation of sign(Q) b for Hermitian Q after `steps`
    steps: |b| V_k sign(T_k) e_1, with V_k the Lanczos basis (kept whole) and
    sign(T_k) from the eigen-decomposition of the tridiagonal T_k (a Krylov
    method for the sign function, the kind the paper uses in Section 5).  An
    exact breakdown stops early.  Returns (approximation, steps taken)."""
    b = np.asarray(b, dtype=np.complex128)
    shape = b.shape
    bn = np.linalg.norm(b)
    if bn == 0.0:
        return np.zeros_like(b), 0
    Q = lambda v: np.asarray(apply_q(v.reshape(shape)), dtype=np.complex128).reshape(-1)
    V = [b.reshape(-1) / bn]
    a, bt = [], []
    v_prev = np.zeros_like(V[0])
    beta = 0.0
    for k in range(steps):
        w = Q(V[k]) - beta * v_prev
        alpha = np.vdot(V[k], w).real
        w = w - alpha * V[k]
        a.append(alpha)
        beta = np.linalg.norm(w)
        if beta <= 1e-14 * abs(alpha) or k == steps - 1:
            break
        bt.append(beta)
        v_prev = V[k]
        V.append(w / beta)
    n = len(a)
    T = np.diag(a) + np.diag(bt[:n - 1], 1) + np.diag(bt[:n - 1], -1)
    th, Z = np.linalg.eigh(T)
    c = bn * (Z @ (np.where(th >= 0, 1.0, -1.0) * Z[0]))
    return (np.array(V[:n]).T @ c).reshape(shape), n
