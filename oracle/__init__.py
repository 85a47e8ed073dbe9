"""FP64 CPU oracle for the overlap-operator apply -- TEST INFRASTRUCTURE.

Only ``tests/``, the smoke check in ``__graft_entry__`` and the ``cpu_baseline``
leg of ``bench.py`` may import this package.  It shares no code with the GPU
library (``paper_1410_7170_amd``) and never imports it; the GPU library never
imports this package.  The only code both sides use is the seeded input
generator ``synth``.

The arithmetic lives in ``oracle.c`` (plain C99 complex128 loops, OpenMP over
sites); this module only marshals numpy arrays.  The 4^4 dense checks are in
``oracle.dense``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

DEFAULT_BC = (-1, 1, 1, 1)   # antiperiodic time, periodic space


def build(force: bool = True) -> str:
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        # -O3 on the x86-64-v3 baseline (AVX2, FMA): the library is built once
        # and may run on another host's CPU, so not -march=native.  ISO C mode
        # (-std=c11) keeps floating-point contraction off, so the arithmetic is
        # the plain loops' whatever the vector width.
        subprocess.check_call([
            "gcc", "-O3", "-march=x86-64-v3", "-std=c11", "-fopenmp", "-fPIC", "-shared",
            os.path.join(_HERE, "oracle.c"), "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        P, D, I, I64 = ctypes.c_void_p, ctypes.c_double, ctypes.c_int, ctypes.c_int64
        lib.orc_gamma.argtypes = [I, P]
        lib.orc_dw.argtypes = [P, P, P, D, P, P]
        lib.orc_gamma5.argtypes = [I64, P, P]
        lib.orc_q.argtypes = [P, P, P, D, P, P]
        lib.orc_q2.argtypes = [P, P, P, D, D, P, P, P]
        lib.orc_norm2.argtypes = [I64, P]
        lib.orc_norm2.restype = D
        lib.orc_dot.argtypes = [I64, P, P, P]
        lib.orc_cg.argtypes = [P, P, P, D, D, P, P, D, I]
        lib.orc_cg.restype = I
        lib.orc_mscg.argtypes = [P, P, P, D, I, P, P, P, D, I, P]
        lib.orc_mscg.restype = I
        lib.orc_true_residual.argtypes = [P, P, P, D, D, P, P]
        lib.orc_true_residual.restype = D
        lib.orc_zolotarev.argtypes = [D, I, P, P, P, P]
        lib.orc_lanczos_q2.argtypes = [P, P, P, D, P, I, P, P]
        lib.orc_lanczos_q2.restype = I
        lib.orc_overlap.argtypes = [P, P, P, D, I, P, P, P, P, P, D, I, P]
        lib.orc_overlap.restype = I
        lib.orc_sign_q.argtypes = [P, P, P, D, I, P, P, P, P, D, I, P]
        lib.orc_sign_q.restype = I
        lib.orc_plaquette_sum.argtypes = [P, P]
        lib.orc_plaquette_sum.restype = D
        lib.orc_set_threads.argtypes = [I]
        lib.orc_max_threads.restype = I
        _lib = lib
    return _lib


def _i32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.int32))


def _c(a):
    a = np.ascontiguousarray(a, dtype=np.complex128)
    return a


def _f(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


class Lattice:
    """Lattice extents (L0 = time, L1, L2, L3) and boundary phases."""

    def __init__(self, dims, bc=DEFAULT_BC):
        self.dims = _i32(dims)
        self.bc = _i32(bc)
        self.V = int(np.prod(self.dims.astype(np.int64)))

    def spinor_shape(self):
        return (self.V, 4, 3)


def gamma(mu: int) -> np.ndarray:
    """gamma_mu for mu = 0..3 and gamma_5 for mu = 4 (chiral basis)."""
    out = np.empty((4, 4), dtype=np.complex128)
    _load().orc_gamma(int(mu), out.ctypes.data)
    return out


def dw(lat: Lattice, U, m0: float, psi) -> np.ndarray:
    """D_W(m0) psi (eq. (Wilson-Dirac))."""
    U, psi = _c(U), _c(psi)
    out = np.empty_like(psi)
    _load().orc_dw(lat.dims.ctypes.data, lat.bc.ctypes.data, U.ctypes.data, float(m0),
                   psi.ctypes.data, out.ctypes.data)
    return out


def gamma5(psi) -> np.ndarray:
    psi = _c(psi)
    out = np.empty_like(psi)
    _load().orc_gamma5(psi.size // 12, psi.ctypes.data, out.ctypes.data)
    return out


def q(lat: Lattice, U, m0: float, psi) -> np.ndarray:
    """Q psi = Gamma_5 D_W(m0) psi."""
    U, psi = _c(U), _c(psi)
    out = np.empty_like(psi)
    _load().orc_q(lat.dims.ctypes.data, lat.bc.ctypes.data, U.ctypes.data, float(m0),
                  psi.ctypes.data, out.ctypes.data)
    return out


def q2(lat: Lattice, U, m0: float, psi, shift: float = 0.0) -> np.ndarray:
    """(Q^2 + shift) psi."""
    U, psi = _c(U), _c(psi)
    out = np.empty_like(psi)
    tmp = np.empty_like(psi)
    _load().orc_q2(lat.dims.ctypes.data, lat.bc.ctypes.data, U.ctypes.data, float(m0), float(shift),
                   psi.ctypes.data, out.ctypes.data, tmp.ctypes.data)
    return out


def norm2(a) -> float:
    a = _c(a)
    return _load().orc_norm2(a.size, a.ctypes.data)


def cg(lat: Lattice, U, m0: float, shift: float, b, tol: float, maxit: int):
    U, b = _c(U), _c(b)
    x = np.empty_like(b)
    it = _load().orc_cg(lat.dims.ctypes.data, lat.bc.ctypes.data, U.ctypes.data, float(m0),
                        float(shift), b.ctypes.data, x.ctypes.data, float(tol), int(maxit))
    return x, it


def mscg(lat: Lattice, U, m0: float, shifts, b, tol: float, maxit: int):
    """Solve (Q^2 + s_j) x_j = b for every shift; returns (x[ns], iters[ns], base_iters)."""
    U, b, shifts = _c(U), _c(b), _f(shifts)
    ns = shifts.size
    x = np.empty((ns,) + b.shape, dtype=np.complex128)
    iters = np.zeros(ns, dtype=np.int32)
    it = _load().orc_mscg(lat.dims.ctypes.data, lat.bc.ctypes.data, U.ctypes.data, float(m0), ns,
                          shifts.ctypes.data, b.ctypes.data, x.ctypes.data, float(tol), int(maxit),
                          iters.ctypes.data)
    return x, iters, it


def true_residual(lat: Lattice, U, m0: float, shift: float, b, x) -> float:
    U, b, x = _c(U), _c(b), _c(x)
    return _load().orc_true_residual(lat.dims.ctypes.data, lat.bc.ctypes.data, U.ctypes.data,
                                     float(m0), float(shift), b.ctypes.data, x.ctypes.data)


def zolotarev_unit(k: float, n: int):
    """Zolotarev coefficients on [k, 1]: (sigma[n], a[n], D, delta)."""
    sig = np.empty(n)
    a = np.empty(n)
    D = ctypes.c_double()
    delta = ctypes.c_double()
    _load().orc_zolotarev(float(k), int(n), sig.ctypes.data, a.ctypes.data,
                          ctypes.byref(D), ctypes.byref(delta))
    return sig, a, D.value, delta.value


def zolotarev(lmin: float, lmax: float, n: int):
    """Shifts s_j and weights w_j with sign(x) ~ x sum_j w_j / (x^2 + s_j)
    for lmin <= |x| <= lmax, plus the relative error bound delta."""
    sig, a, D, delta = zolotarev_unit(lmin / lmax, n)
    return sig * lmax ** 2, D * a * lmax, delta


def lanczos_q2(lat: Lattice, U, m0: float, v0, m: int):
    """Extreme Ritz values (theta_min, theta_max) of Q^2 after m Lanczos steps."""
    U, v0 = _c(U), _c(v0)
    lo = ctypes.c_double()
    hi = ctypes.c_double()
    _load().orc_lanczos_q2(lat.dims.ctypes.data, lat.bc.ctypes.data, U.ctypes.data, float(m0),
                           v0.ctypes.data, int(m), ctypes.byref(lo), ctypes.byref(hi))
    return lo.value, hi.value


def spectral_interval(lat: Lattice, U, m0: float, v0, m: int = 300,
                      lo_margin: float = 0.9, hi_margin: float = 1.05):
    """[lambda_min, lambda_max] of |Q| from Lanczos on Q^2, widened by the margins
    (Ritz values lie inside the spectrum)."""
    t0, t1 = lanczos_q2(lat, U, m0, v0, m)
    return lo_margin * np.sqrt(max(t0, 0.0)), hi_margin * np.sqrt(t1)


def overlap(lat: Lattice, U, rho: float, shifts, weights, b, tol: float, maxit: int,
            return_y: bool = False):
    """D_ov b = rho (b + Gamma_5 sign(Gamma_5 D_W(-rho)) b) via Zolotarev + multishift CG."""
    U, b, shifts, weights = _c(U), _c(b), _f(shifts), _f(weights)
    out = np.empty_like(b)
    y = np.empty_like(b)
    iters = np.zeros(shifts.size, dtype=np.int32)
    it = _load().orc_overlap(lat.dims.ctypes.data, lat.bc.ctypes.data, U.ctypes.data, float(rho),
                             shifts.size, shifts.ctypes.data, weights.ctypes.data, b.ctypes.data,
                             out.ctypes.data, y.ctypes.data, float(tol), int(maxit),
                             iters.ctypes.data)
    if return_y:
        return out, y, iters, it
    return out, iters, it


def sign_q(lat: Lattice, U, m0: float, shifts, weights, b, tol: float, maxit: int):
    U, b, shifts, weights = _c(U), _c(b), _f(shifts), _f(weights)
    out = np.empty_like(b)
    iters = np.zeros(shifts.size, dtype=np.int32)
    it = _load().orc_sign_q(lat.dims.ctypes.data, lat.bc.ctypes.data, U.ctypes.data, float(m0),
                            shifts.size, shifts.ctypes.data, weights.ctypes.data, b.ctypes.data,
                            out.ctypes.data, float(tol), int(maxit), iters.ctypes.data)
    return out, iters, it


def set_threads(n: int) -> None:
    """OpenMP threads of the oracle's site loops (for timing runs)."""
    _load().orc_set_threads(int(n))


def max_threads() -> int:
    return int(_load().orc_max_threads())


def plaquette_sum(lat: Lattice, U) -> float:
    """sum_x sum_{mu<nu} Re tr P^{mu,nu}_x (eq. (plaquette_def1))."""
    U = _c(U)
    return _load().orc_plaquette_sum(lat.dims.ctypes.data, U.ctypes.data)


def average_plaquette(lat: Lattice, U) -> float:
    """Q_avg of eq. (avgplaquette): mean of Re tr P over the 6V plaquettes."""
    return plaquette_sum(lat, U) / (6 * lat.V)
