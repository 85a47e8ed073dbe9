"""Seeded synthetic inputs shared by the FP64 oracle and the GPU library.

This module draws gauge fields and sources; it holds none of the overlap
operator's arithmetic.  Both sides receive the same canonical complex128
bytes:

* gauge ``U[site, mu, row, col]`` with ``U_mu(x)`` the link x -> x+mu,
* spinor ``psi[site, spin, colour]`` (``[rhs, site, spin, colour]`` for several),
* ``site = ((x0*L1 + x1)*L2 + x2)*L3 + x3`` with x0 the (antiperiodic) time axis.

Workload recipes (the benchmark workloads, WORKLOADS): links
``exp(i*eps0*H)`` with H a seeded traceless Hermitian Gaussian matrix, then
``n_stout`` stout-smearing steps at ``rho_stout = 0.1`` (Section "Smearing and
Normality", eq. (stout)), Gaussian or spin-colour point sources.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libsynth.so")
_lib = None

# per-purpose seeds: gauge 1410717 + 10*cfg, source +1, point site +2
SEED_BASE = 1410717


def build(force: bool = True) -> str:
    """Compile the generator with gcc (OpenMP)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call([
            "gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared",
            os.path.join(_HERE, "gen.c"), "-o", tmp, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        lib.synth_gauge.argtypes = [P, ctypes.c_double, ctypes.c_uint64, P]
        lib.synth_stout.argtypes = [P, ctypes.c_double, ctypes.c_int, P, P]
        lib.synth_gaussian_spinor.argtypes = [ctypes.c_int64, ctypes.c_int, ctypes.c_uint64, P]
        lib.synth_randint.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64]
        lib.synth_randint.restype = ctypes.c_int64
        _lib = lib
    return _lib


def _dims(dims):
    d = np.ascontiguousarray(np.asarray(dims, dtype=np.int32))
    assert d.shape == (4,) and (d > 0).all()
    return d


def volume(dims) -> int:
    return int(np.prod(np.asarray(dims, dtype=np.int64)))


def gauge(dims, eps0: float, seed: int, n_stout: int = 0, rho_stout: float = 0.1) -> np.ndarray:
    """SU(3) gauge field, shape (V, 4, 3, 3) complex128."""
    lib = _load()
    d = _dims(dims)
    V = volume(d)
    U = np.empty((V, 4, 3, 3), dtype=np.complex128)
    lib.synth_gauge(d.ctypes.data, float(eps0), ctypes.c_uint64(seed), U.ctypes.data)
    if n_stout > 0:
        work = np.empty_like(U)
        lib.synth_stout(d.ctypes.data, float(rho_stout), int(n_stout), U.ctypes.data, work.ctypes.data)
        del work
    return U


def stout(dims, U: np.ndarray, rho_stout: float, n_steps: int) -> np.ndarray:
    """Return a smeared copy of U (simultaneous update of all links)."""
    lib = _load()
    d = _dims(dims)
    out = np.ascontiguousarray(U, dtype=np.complex128).copy()
    work = np.empty_like(out)
    lib.synth_stout(d.ctypes.data, float(rho_stout), int(n_steps), out.ctypes.data, work.ctypes.data)
    return out


def unit_gauge(dims) -> np.ndarray:
    """Free field: every link the identity."""
    V = volume(dims)
    U = np.zeros((V, 4, 3, 3), dtype=np.complex128)
    U[:, :, 0, 0] = U[:, :, 1, 1] = U[:, :, 2, 2] = 1.0
    return U


def gaussian_spinor(V: int, seed: int, nrhs: int = 1) -> np.ndarray:
    """Complex Gaussian spinors, shape (nrhs, V, 4, 3)."""
    lib = _load()
    out = np.empty((nrhs, V, 4, 3), dtype=np.complex128)
    lib.synth_gaussian_spinor(ctypes.c_int64(V), int(nrhs), ctypes.c_uint64(seed), out.ctypes.data)
    return out


def random_site(V: int, seed: int) -> int:
    return int(_load().synth_randint(ctypes.c_uint64(seed), ctypes.c_uint64(0), ctypes.c_int64(V)))


def point_sources(V: int, site: int) -> np.ndarray:
    """The 12 spin-colour point sources e_{site,s,c}, shape (12, V, 4, 3)."""
    out = np.zeros((12, V, 4, 3), dtype=np.complex128)
    for s in range(4):
        for c in range(3):
            out[3 * s + c, site, s, c] = 1.0
    return out


# Workload recipes: lattice (L0=t, L1, L2, L3), link eps0, stout steps,
# sources, Zolotarev poles.
WORKLOADS = {
    0: dict(name="4^4 fp64 dense check", dims=(4, 4, 4, 4), eps0=0.5, n_stout=0,
            source="gaussian", nrhs=1, poles=20),
    1: dict(name="16^3x32 fp64/fp32", dims=(32, 16, 16, 16), eps0=0.3, n_stout=2,
            source="gaussian", nrhs=1, poles=20),
    2: dict(name="32^3x64 mixed", dims=(64, 32, 32, 32), eps0=0.3, n_stout=2,
            source="gaussian", nrhs=1, poles=20),
    3: dict(name="24^3x48 12 point sources", dims=(48, 24, 24, 24), eps0=0.3, n_stout=2,
            source="point", nrhs=12, poles=20),
    4: dict(name="48^3x96 4 rhs 24 poles", dims=(96, 48, 48, 48), eps0=0.3, n_stout=3,
            source="gaussian", nrhs=4, poles=24),
}


def workload_gauge(cfg: int, dims=None) -> np.ndarray:
    c = WORKLOADS[cfg]
    return gauge(dims or c["dims"], c["eps0"], SEED_BASE + 10 * cfg, c["n_stout"])


def workload_sources(cfg: int, dims=None) -> np.ndarray:
    c = WORKLOADS[cfg]
    V = volume(dims or c["dims"])
    if c["source"] == "point":
        return point_sources(V, random_site(V, SEED_BASE + 10 * cfg + 2))
    return gaussian_spinor(V, SEED_BASE + 10 * cfg + 1, c["nrhs"])
