"""Python binding of libovl.so, the gfx950 overlap-operator library.

Argument marshalling only: every step of the computation runs in the HIP
kernels behind the C ABI declared in ``include/ovl.h``.  PyTorch provides
device memory (uint8 / float32 tensors) and the current HIP stream.  There is
no fallback: if ``libovl.so`` is missing or fails to load, importing this
package raises.

torch is imported first on purpose: libovl.so then binds to the HIP runtime
torch already loaded, so both share one runtime, one context and one set of
streams.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libovl.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run paper_1410_7170_amd/build.py "
                      "(or __graft_entry__.build())")
_lib = ctypes.CDLL(LIB_PATH)

# ---------------------------------------------------------------- constants
OK, NOT_CONVERGED = 0, 1
ERR_INVALID, ERR_WORKSPACE, ERR_HIP, ERR_NONFINITE = -1, -2, -3, -4
F64, F32, F16S, F48 = 0, 1, 2, 3
SOLVE_F64, SOLVE_MIXED, SOLVE_LANCZOS = 0, 1, 2
OP_Q2, OP_LANCZOS, OP_MSCG, OP_TUNE, OP_WILSON_SOLVE = 0, 1, 2, 3, 4
K_STENCIL, K_UPDATE, K_SCALAR, K_OTHER = 0, 1, 2, 3
MAX_SHIFTS, MAX_RHS, MAX_BLOCK = 32, 16, 32
PREC_NAMES = {F64: "f64", F32: "f32", F16S: "f16s", F48: "f48"}

c_i32, c_i64, c_dbl, c_vp = ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_void_p


class ovl_lattice(ctypes.Structure):
    _fields_ = [("dims", c_i32 * 4), ("bc", c_i32 * 4), ("vol", c_i64), ("tile_t", c_i32), ("stream_t", c_i32),
                ("stream_t64", c_i32), ("rhs_tile", c_i32), ("mfma", c_i32)]


class ovl_gauge(ctypes.Structure):
    _fields_ = [("f64", c_vp), ("f32", c_vp), ("f16", c_vp)]


class ovl_spinor(ctypes.Structure):
    _fields_ = [("d", c_vp), ("scale", c_vp), ("prec", c_i32), ("nrhs", c_i32)]


class ovl_zolo(ctypes.Structure):
    _fields_ = [("npoles", c_i32), ("shifts", ctypes.POINTER(c_dbl)), ("weights", ctypes.POINTER(c_dbl))]


class ovl_deflation(ctypes.Structure):
    _fields_ = [("evecs", ovl_spinor), ("evals", ctypes.POINTER(c_dbl))]


class ovl_solver_params(ctypes.Structure):
    _fields_ = [("tol", c_dbl), ("maxiter", c_i32), ("mode", c_i32), ("reliable_delta", c_dbl),
                ("check_every", c_i32), ("refine", c_i32), ("verify", c_i32), ("profile", c_i32),
                ("block", c_i32), ("sloppy_below", c_dbl), ("block_f64", c_i32), ("rhs_group", c_i32),
                ("deflation", ctypes.POINTER(ovl_deflation)), ("sloppy_f16", c_i32),
                ("even_odd", c_i32), ("store48", c_i32)]


class ovl_eig_params(ctypes.Structure):
    _fields_ = [("nev", c_i32), ("extra", c_i32), ("tol", c_dbl), ("degree", c_i32), ("steps", c_i32),
                ("stages", c_i32), ("check_every", c_i32)]


class ovl_eig_stats(ctypes.Structure):
    _fields_ = [("steps", c_i32), ("stages", c_i32), ("q2_applies", ctypes.c_int64), ("converged", c_i32),
                ("reserved", c_i32), ("max_residual", c_dbl), ("lambda_next", c_dbl), ("theta_cut", c_dbl),
                ("mean_degree", c_dbl), ("seconds", c_dbl)]


class ovl_solver_stats(ctypes.Structure):
    _fields_ = [("iterations", c_i32 * MAX_RHS),
                ("shift_iters", (c_i32 * MAX_SHIFTS) * MAX_RHS),
                ("true_residual", (c_dbl * MAX_SHIFTS) * MAX_RHS),
                ("reliable_updates", c_i32), ("refine_iterations", c_i32), ("stencil_applies", c_i32),
                ("algorithmic_bytes", c_dbl), ("seconds", c_dbl),
                ("kernel_seconds", c_dbl * 4), ("kernel_bytes", c_dbl * 4), ("kernel_launches", c_i32 * 4)]

    def to_dict(self, nrhs: int = 1, nshift: int = 0) -> dict:
        return dict(
            iterations=[int(self.iterations[r]) for r in range(nrhs)],
            shift_iters=[[int(self.shift_iters[r][j]) for j in range(nshift)] for r in range(nrhs)],
            true_residual=[[float(self.true_residual[r][j]) for j in range(nshift)] for r in range(nrhs)],
            reliable_updates=int(self.reliable_updates), refine_iterations=int(self.refine_iterations),
            stencil_applies=int(self.stencil_applies), algorithmic_bytes=float(self.algorithmic_bytes),
            seconds=float(self.seconds),
            kernel_seconds=[float(v) for v in self.kernel_seconds],
            kernel_bytes=[float(v) for v in self.kernel_bytes],
            kernel_launches=[int(v) for v in self.kernel_launches])


class ovl_outer_params(ctypes.Structure):
    _fields_ = [("tol", c_dbl), ("restart", c_i32), ("maxiter", c_i32), ("relax", c_i32),
                ("relax_factor", c_dbl), ("sign_tol_max", c_dbl), ("inner", ovl_solver_params),
                ("precondition", c_i32), ("prec_m0", c_dbl), ("prec_tol", c_dbl), ("prec_maxiter", c_i32),
                ("prec_block", c_i32), ("prec_even_odd", c_i32)]


class ovl_outer_stats(ctypes.Structure):
    _fields_ = [("iterations", c_i32), ("restarts", c_i32), ("overlap_applies", c_i32),
                ("mscg_iterations", c_i32), ("prec_iterations", c_i32), ("residual", c_dbl),
                ("estimated_residual", c_dbl), ("seconds", c_dbl)]

    def to_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


P = ctypes.POINTER
_sig = {
    "ovl_lattice_init": (c_i32, [P(ovl_lattice), P(c_i32), P(c_i32)]),
    "ovl_spinor_bytes": (ctypes.c_size_t, [P(ovl_lattice), c_i32]),
    "ovl_scale_bytes": (ctypes.c_size_t, [P(ovl_lattice)]),
    "ovl_gauge_bytes": (ctypes.c_size_t, [P(ovl_lattice), c_i32]),
    "ovl_pack_spinor": (c_i32, [P(ovl_lattice), c_vp, P(ovl_spinor), c_vp]),
    "ovl_unpack_spinor": (c_i32, [P(ovl_lattice), P(ovl_spinor), c_vp, c_vp]),
    "ovl_pack_gauge": (c_i32, [P(ovl_lattice), c_vp, c_i32, c_vp, c_vp]),
    "ovl_wilson_apply": (c_i32, [P(ovl_lattice), P(ovl_gauge), c_dbl, P(ovl_spinor), P(ovl_spinor), c_vp]),
    "ovl_q_apply": (c_i32, [P(ovl_lattice), P(ovl_gauge), c_dbl, P(ovl_spinor), P(ovl_spinor), c_vp]),
    "ovl_q2_apply": (c_i32, [P(ovl_lattice), P(ovl_gauge), c_dbl, c_dbl, P(ovl_spinor), P(ovl_spinor),
                             c_vp, ctypes.c_size_t, c_vp]),
    "ovl_q2_apply_noalloc": (c_i32, [P(ovl_lattice), P(ovl_gauge), c_dbl, c_dbl, P(ovl_spinor), P(ovl_spinor),
                                     c_vp]),
    "ovl_zolotarev": (c_i32, [c_dbl, c_dbl, c_i32, P(c_dbl), P(c_dbl), P(c_dbl)]),
    "ovl_spectral_bounds": (c_i32, [P(ovl_lattice), P(ovl_gauge), c_dbl, c_i32, P(ovl_spinor), c_dbl, c_dbl,
                                    P(c_dbl), P(c_dbl), c_vp, ctypes.c_size_t, c_vp]),
    "ovl_multishift_cg": (c_i32, [P(ovl_lattice), P(ovl_gauge), c_dbl, c_i32, P(c_dbl), P(c_dbl),
                                  P(ovl_spinor), P(ovl_spinor), P(ovl_solver_params), P(ovl_solver_stats),
                                  c_vp, ctypes.c_size_t, c_vp]),
    "ovl_sign_q_apply": (c_i32, [P(ovl_lattice), P(ovl_gauge), c_dbl, P(ovl_zolo), P(ovl_spinor), P(ovl_spinor),
                                 P(ovl_solver_params), P(ovl_solver_stats), c_vp, ctypes.c_size_t, c_vp]),
    "ovl_overlap_apply": (c_i32, [P(ovl_lattice), P(ovl_gauge), c_dbl, P(ovl_zolo), P(ovl_spinor), P(ovl_spinor),
                                  P(ovl_solver_params), P(ovl_solver_stats), c_vp, ctypes.c_size_t, c_vp]),
    "ovl_workspace_bytes": (ctypes.c_size_t, [P(ovl_lattice), c_i32, c_i32, c_i32, c_i32, P(ovl_solver_params)]),
    "ovl_default_params": (None, [P(ovl_solver_params)]),
    "ovl_autotune_stencil": (c_i32, [P(ovl_lattice), P(ovl_gauge), c_i32, c_vp, ctypes.c_size_t, P(c_i32),
                                     P(ctypes.c_float), c_i32, c_vp]),
    "ovl_autotune_stencil_cached": (c_i32, [P(ovl_lattice), P(ovl_gauge), c_i32, c_vp, ctypes.c_size_t,
                                            ctypes.c_char_p, P(c_i32), P(ctypes.c_float), c_i32, c_vp]),
    "ovl_default_outer_params": (None, [P(ovl_outer_params)]),
    "ovl_overlap_solve_workspace_bytes": (ctypes.c_size_t, [P(ovl_lattice), c_i32, P(ovl_outer_params)]),
    "ovl_overlap_solve": (c_i32, [P(ovl_lattice), P(ovl_gauge), c_dbl, P(ovl_zolo), P(ovl_spinor), P(ovl_spinor),
                                  P(ovl_outer_params), P(ovl_outer_stats), c_vp, ctypes.c_size_t, c_vp]),
    "ovl_wilson_solve": (c_i32, [P(ovl_lattice), P(ovl_gauge), c_dbl, P(ovl_spinor), P(ovl_spinor),
                                 P(ovl_solver_params), P(ovl_solver_stats), c_vp, ctypes.c_size_t, c_vp]),
    "ovl_default_eig_params": (None, [P(ovl_eig_params)]),
    "ovl_low_modes_workspace_bytes": (ctypes.c_size_t, [P(ovl_lattice), P(ovl_eig_params)]),
    "ovl_low_modes": (c_i32, [P(ovl_lattice), P(ovl_gauge), c_dbl, P(ovl_spinor), P(ovl_eig_params),
                              P(ovl_spinor), P(c_dbl), P(c_dbl), P(ovl_eig_stats), c_vp, ctypes.c_size_t, c_vp]),
    "ovl_status_string": (ctypes.c_char_p, [c_i32]),
    "ovl_last_hip_error": (c_i32, []),
    "ovl_version": (ctypes.c_char_p, []),
}
for _name, (_res, _args) in _sig.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = tuple(_sig)


class OvlError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = _lib.ovl_status_string(status).decode()
        if status == ERR_HIP:
            msg += f" (hipError {_lib.ovl_last_hip_error()})"
        super().__init__(f"{where}: {msg} [{status}]")
        self.status = status


def _check(status: int, where: str, allow_not_converged: bool = False) -> int:
    if status < 0 or (status == NOT_CONVERGED and not allow_not_converged):
        raise OvlError(status, where)
    return status


def _stream(stream):
    if stream is None:
        return c_vp(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return c_vp(stream.cuda_stream)
    return c_vp(stream)


def version() -> str:
    return _lib.ovl_version().decode()


# ---------------------------------------------------------------- lattice
class Lattice:
    def __init__(self, dims, bc=(-1, 1, 1, 1)):
        self.c = ovl_lattice()
        d = (c_i32 * 4)(*[int(v) for v in dims])
        b = (c_i32 * 4)(*[int(v) for v in bc])
        _check(_lib.ovl_lattice_init(ctypes.byref(self.c), d, b), "ovl_lattice_init")
        self.dims = tuple(int(v) for v in dims)
        self.bc = tuple(int(v) for v in bc)
        self.V = int(self.c.vol)

    @property
    def tile_t(self) -> int:
        return int(self.c.tile_t)

    @tile_t.setter
    def tile_t(self, t: int):
        if t < 1 or self.dims[0] % t:
            raise ValueError(f"tile_t must divide L0={self.dims[0]}")
        self.c.tile_t = int(t)

    @property
    def stream_t(self) -> int:
        return int(self.c.stream_t)

    @stream_t.setter
    def stream_t(self, s: int):
        if s and (s < 0 or s > 256 or self.dims[0] % s or (self.dims[1] * self.dims[2] * self.dims[3]) % 256):
            raise ValueError(f"stream_t={s} needs s | L0 and L1*L2*L3 % 256 == 0")
        self.c.stream_t = int(s)

    @property
    def stream_t64(self) -> int:
        return int(self.c.stream_t64)

    @stream_t64.setter
    def stream_t64(self, s: int):
        if s and (s < 0 or s > 256 or self.dims[0] % s or (self.dims[1] * self.dims[2] * self.dims[3]) % 256):
            raise ValueError(f"stream_t64={s} needs s | L0 and L1*L2*L3 % 256 == 0")
        self.c.stream_t64 = int(s)

    @property
    def rhs_tile(self) -> int:
        return int(self.c.rhs_tile)

    @rhs_tile.setter
    def rhs_tile(self, k: int):
        if k not in (1, 2, 4, 8):
            raise ValueError("rhs_tile must be 1, 2, 4 or 8")
        self.c.rhs_tile = int(k)

    @property
    def mfma(self) -> int:
        return int(self.c.mfma)

    @mfma.setter
    def mfma(self, v: int):
        self.c.mfma = 1 if v else 0

    @property
    def ref(self):
        return ctypes.byref(self.c)

    def spinor_bytes(self, prec: int) -> int:
        return int(_lib.ovl_spinor_bytes(self.ref, prec))

    def gauge_bytes(self, prec: int) -> int:
        return int(_lib.ovl_gauge_bytes(self.ref, prec))

    def scale_bytes(self) -> int:
        return int(_lib.ovl_scale_bytes(self.ref))


def _dev_buffer(nbytes: int, device) -> torch.Tensor:
    # 256-byte granularity keeps every field 16-byte aligned
    return torch.empty(max(int(nbytes), 1), dtype=torch.uint8, device=device)


class Spinor:
    """nrhs packed fields of one storage precision (device memory from torch)."""

    def __init__(self, lat: Lattice, prec: int, nrhs: int = 1, device="cuda"):
        self.lat, self.prec, self.nrhs = lat, prec, nrhs
        self.data = _dev_buffer(lat.spinor_bytes(prec) * nrhs, device)
        self.scale = (torch.empty(lat.scale_bytes() // 4 * nrhs, dtype=torch.float32, device=device)
                      if prec == F16S else None)
        self.c = ovl_spinor(self.data.data_ptr(), self.scale.data_ptr() if self.scale is not None else None,
                            prec, nrhs)

    @property
    def ref(self):
        return ctypes.byref(self.c)

    @classmethod
    def from_canonical(cls, lat: Lattice, canon: torch.Tensor, prec: int, stream=None) -> "Spinor":
        """canon: complex128 device tensor (nrhs, V, 4, 3) or (V, 4, 3)."""
        if canon.dim() == 3:
            canon = canon.unsqueeze(0)
        canon = canon.contiguous()
        assert canon.dtype == torch.complex128 and canon.shape[1:] == (lat.V, 4, 3) and canon.is_cuda
        s = cls(lat, prec, canon.shape[0], canon.device)
        pack_spinor(lat, canon, s, stream)
        return s

    def to_canonical(self, stream=None) -> torch.Tensor:
        out = torch.empty((self.nrhs, self.lat.V, 4, 3), dtype=torch.complex128, device=self.data.device)
        unpack_spinor(self.lat, self, out, stream)
        return out


class Gauge:
    """A gauge field packed in FP64, FP32 and FP16, 12 reals per link (rows 0
    and 1; row 2 is rebuilt in the kernels)."""

    def __init__(self, lat: Lattice, canon: torch.Tensor, precs=(F64, F32, F16S), stream=None):
        canon = canon.contiguous()
        assert canon.dtype == torch.complex128 and canon.shape == (lat.V, 4, 3, 3) and canon.is_cuda
        self.lat = lat
        self.bufs = {}
        for p in precs:
            buf = _dev_buffer(lat.gauge_bytes(p), canon.device)
            _check(_lib.ovl_pack_gauge(lat.ref, c_vp(canon.data_ptr()), p, c_vp(buf.data_ptr()),
                                       _stream(stream)), "ovl_pack_gauge")
            self.bufs[p] = buf
        ptr = lambda p: c_vp(self.bufs[p].data_ptr()) if p in self.bufs else None
        self.c = ovl_gauge(ptr(F64), ptr(F32), ptr(F16S))

    @property
    def ref(self):
        return ctypes.byref(self.c)


def default_params(**kw) -> ovl_solver_params:
    """ovl_default_params, then keyword overrides; deflation=Deflation(...)
    points the parameters at its low modes (the Deflation object is kept
    alive by the returned structure)."""
    p = ovl_solver_params()
    _lib.ovl_default_params(ctypes.byref(p))
    for k, v in kw.items():
        if k == "deflation":
            set_deflation(p, v)
        else:
            setattr(p, k, v)
    return p


class Deflation:
    """Low modes of Q for deflated sign/overlap applies: eigenvectors evecs
    (an FP64 Spinor with nrhs = k) and eigenvalues evals (float64, k)."""

    def __init__(self, evecs: "Spinor", evals, residuals=None, stats=None):
        assert evecs.prec == F64 and len(evals) == evecs.nrhs
        self.evecs = evecs
        self.evals = np.ascontiguousarray(np.asarray(evals, dtype=np.float64))
        self.residuals = residuals
        self.stats = stats
        self.c = ovl_deflation(evecs.c, self.evals.ctypes.data_as(ctypes.POINTER(c_dbl)))

    @property
    def nev(self) -> int:
        return self.evecs.nrhs


def set_deflation(params: ovl_solver_params, defl):
    """Point params (an ovl_solver_params, e.g. outer params' .inner) at a
    Deflation, or clear it with None."""
    if defl is None:
        params.deflation = ctypes.POINTER(ovl_deflation)()
        params._defl = None
    else:
        params.deflation = ctypes.pointer(defl.c)
        params._defl = defl


# ---------------------------------------------------------------- C ABI
def pack_spinor(lat: Lattice, canon: torch.Tensor, out: Spinor, stream=None):
    _check(_lib.ovl_pack_spinor(lat.ref, c_vp(canon.data_ptr()), out.ref, _stream(stream)), "ovl_pack_spinor")


def unpack_spinor(lat: Lattice, inp: Spinor, canon: torch.Tensor, stream=None):
    _check(_lib.ovl_unpack_spinor(lat.ref, inp.ref, c_vp(canon.data_ptr()), _stream(stream)), "ovl_unpack_spinor")


def wilson_apply(lat: Lattice, U: Gauge, m0: float, inp: Spinor, out: Spinor, stream=None):
    _check(_lib.ovl_wilson_apply(lat.ref, U.ref, float(m0), inp.ref, out.ref, _stream(stream)), "ovl_wilson_apply")


def q_apply(lat: Lattice, U: Gauge, m0: float, inp: Spinor, out: Spinor, stream=None):
    _check(_lib.ovl_q_apply(lat.ref, U.ref, float(m0), inp.ref, out.ref, _stream(stream)), "ovl_q_apply")


def workspace_bytes(lat: Lattice, op: int, prec: int, nrhs: int, nshift: int = 0, params=None) -> int:
    return int(_lib.ovl_workspace_bytes(lat.ref, op, prec, nrhs, nshift,
                                        ctypes.byref(params) if params is not None else None))


def workspace(lat: Lattice, op: int, prec: int, nrhs: int, nshift: int = 0, params=None, device="cuda"):
    return _dev_buffer(workspace_bytes(lat, op, prec, nrhs, nshift, params), device)


def q2_apply(lat: Lattice, U: Gauge, m0: float, shift: float, inp: Spinor, out: Spinor, ws=None, stream=None):
    if ws is None:
        ws = workspace(lat, OP_Q2, inp.prec, inp.nrhs, device=inp.data.device)
    _check(_lib.ovl_q2_apply(lat.ref, U.ref, float(m0), float(shift), inp.ref, out.ref, c_vp(ws.data_ptr()),
                             ws.numel(), _stream(stream)), "ovl_q2_apply")


def q2_apply_noalloc(lat: Lattice, U: Gauge, m0: float, shift: float, inp: Spinor, out: Spinor, stream=None):
    """(Q^2 + shift) inp with the library's own scratch array (no workspace)."""
    _check(_lib.ovl_q2_apply_noalloc(lat.ref, U.ref, float(m0), float(shift), inp.ref, out.ref, _stream(stream)),
           "ovl_q2_apply_noalloc")


NOALLOC_SCRATCH_BYTES = 256 << 20


def zolotarev(lambda_min: float, lambda_max: float, npoles: int):
    """Host-only: (shifts, weights, delta) with sign(x) ~ x sum w/(x^2+s)."""
    s = (c_dbl * npoles)()
    w = (c_dbl * npoles)()
    d = c_dbl()
    _check(_lib.ovl_zolotarev(float(lambda_min), float(lambda_max), int(npoles), s, w, ctypes.byref(d)),
           "ovl_zolotarev")
    return np.array(s[:]), np.array(w[:]), d.value


def autotune_stencil(lat: Lattice, U: Gauge, nrhs: int = 1, ws=None, stream=None, cache=None) -> dict:
    """Time the stencil's candidate site orders and RHS tiles
    (ovl_autotune_stencil) and keep the fastest in `lat`; with `cache` (a file
    path) earlier choices for the same device, lattice, RHS count and links are
    reused (ovl_autotune_stencil_cached).  Returns the choices and every
    timing (microseconds): (what, rhs tile, value, us)."""
    if ws is None:
        ws = workspace(lat, OP_TUNE, F64, nrhs)
    n = 256
    tried = (c_i32 * n)()
    times = (ctypes.c_float * n)()
    if cache is not None:
        rc = _lib.ovl_autotune_stencil_cached(lat.ref, U.ref, int(nrhs), c_vp(ws.data_ptr()), ws.numel(),
                                              os.fsencode(cache), tried, times, n, _stream(stream))
    else:
        rc = _lib.ovl_autotune_stencil(lat.ref, U.ref, int(nrhs), c_vp(ws.data_ptr()), ws.numel(), tried, times, n,
                                       _stream(stream))
    _check(rc, "ovl_autotune_stencil")
    names = ("tile_t", "stream_t", "stream_t64", "mfma")
    table = [(names[tried[k] // 10000], (tried[k] // 100) % 100, tried[k] % 100, round(float(times[k]), 2))
             for k in range(min(rc, n))]
    return dict(tile_t=lat.tile_t, stream_t=lat.stream_t, stream_t64=lat.stream_t64, rhs_tile=lat.rhs_tile,
                mfma=lat.mfma, timings=table if rc > 0 or cache is None else "cache")


def spectral_bounds(lat: Lattice, U: Gauge, m0: float, iters: int, start: Spinor,
                    lo_margin: float = 0.9, hi_margin: float = 1.05, ws=None, stream=None):
    if ws is None:
        ws = workspace(lat, OP_LANCZOS, F64, 1, device=start.data.device)
    lo, hi = c_dbl(), c_dbl()
    _check(_lib.ovl_spectral_bounds(lat.ref, U.ref, float(m0), int(iters), start.ref, float(lo_margin),
                                    float(hi_margin), ctypes.byref(lo), ctypes.byref(hi), c_vp(ws.data_ptr()),
                                    ws.numel(), _stream(stream)), "ovl_spectral_bounds")
    return lo.value, hi.value


def low_modes(lat: Lattice, U: Gauge, m0: float, start: Spinor, nev: int = 16, ws=None, stream=None,
              allow_not_converged=False, **kw) -> Deflation:
    """ovl_low_modes: the nev eigenpairs of Q = Gamma_5 D_W(m0) smallest in
    |lambda|, as a Deflation (evals ascending in |lambda|, residuals
    |Q xi - lambda xi|, stats).  Keywords override ovl_eig_params fields
    (extra, tol, degree, steps, stages, check_every)."""
    p = ovl_eig_params()
    _lib.ovl_default_eig_params(ctypes.byref(p))
    p.nev = int(nev)
    for k, v in kw.items():
        setattr(p, k, v)
    if ws is None:
        nbytes = int(_lib.ovl_low_modes_workspace_bytes(lat.ref, ctypes.byref(p)))
        if nbytes == 0:
            raise OvlError(ERR_INVALID, "ovl_low_modes_workspace_bytes")
        ws = _dev_buffer(nbytes, start.data.device)
    evecs = Spinor(lat, F64, int(nev), start.data.device)
    evals = np.zeros(int(nev))
    res = np.zeros(int(nev))
    st = ovl_eig_stats()
    rc = _lib.ovl_low_modes(lat.ref, U.ref, float(m0), start.ref, ctypes.byref(p), evecs.ref,
                            evals.ctypes.data_as(P(c_dbl)), res.ctypes.data_as(P(c_dbl)), ctypes.byref(st),
                            c_vp(ws.data_ptr()), ws.numel(), _stream(stream))
    _check(rc, "ovl_low_modes", allow_not_converged)
    return Deflation(evecs, evals, res, {k: getattr(st, k) for k, _ in st._fields_})


def _dvec(a):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    return a, a.ctypes.data_as(P(c_dbl))


def multishift_cg(lat: Lattice, U: Gauge, m0: float, shifts, weights, b: Spinor, x: Spinor, params=None,
                  ws=None, stream=None, allow_not_converged=False):
    params = params or default_params()
    s_arr, s_ptr = _dvec(shifts)
    w_arr, w_ptr = _dvec(weights) if weights is not None else (None, None)
    if ws is None:
        ws = workspace(lat, OP_MSCG, F64, b.nrhs, len(s_arr), params, device=b.data.device)
    st = ovl_solver_stats()
    rc = _lib.ovl_multishift_cg(lat.ref, U.ref, float(m0), len(s_arr), s_ptr, w_ptr, b.ref, x.ref,
                                ctypes.byref(params), ctypes.byref(st), c_vp(ws.data_ptr()), ws.numel(),
                                _stream(stream))
    _check(rc, "ovl_multishift_cg", allow_not_converged)
    return st.to_dict(b.nrhs, len(s_arr))


def _zolo(shifts, weights):
    s_arr, s_ptr = _dvec(shifts)
    w_arr, w_ptr = _dvec(weights)
    return ovl_zolo(len(s_arr), s_ptr, w_ptr), (s_arr, w_arr)


def sign_q_apply(lat: Lattice, U: Gauge, m0: float, shifts, weights, b: Spinor, out: Spinor, params=None,
                 ws=None, stream=None, allow_not_converged=False):
    params = params or default_params()
    z, keep = _zolo(shifts, weights)
    if ws is None:
        ws = workspace(lat, OP_MSCG, F64, b.nrhs, z.npoles, params, device=b.data.device)
    st = ovl_solver_stats()
    rc = _lib.ovl_sign_q_apply(lat.ref, U.ref, float(m0), ctypes.byref(z), b.ref, out.ref, ctypes.byref(params),
                               ctypes.byref(st), c_vp(ws.data_ptr()), ws.numel(), _stream(stream))
    _check(rc, "ovl_sign_q_apply", allow_not_converged)
    return st.to_dict(b.nrhs, z.npoles)


def overlap_apply(lat: Lattice, U: Gauge, rho: float, shifts, weights, b: Spinor, out: Spinor, params=None,
                  ws=None, stream=None, allow_not_converged=False):
    params = params or default_params()
    z, keep = _zolo(shifts, weights)
    if ws is None:
        ws = workspace(lat, OP_MSCG, F64, b.nrhs, z.npoles, params, device=b.data.device)
    st = ovl_solver_stats()
    rc = _lib.ovl_overlap_apply(lat.ref, U.ref, float(rho), ctypes.byref(z), b.ref, out.ref, ctypes.byref(params),
                                ctypes.byref(st), c_vp(ws.data_ptr()), ws.numel(), _stream(stream))
    _check(rc, "ovl_overlap_apply", allow_not_converged)
    return st.to_dict(b.nrhs, z.npoles)


def default_outer_params(**kw) -> ovl_outer_params:
    """ovl_default_outer_params, then keyword overrides; inner=dict(...)
    overrides fields of the D_ov applications' solver parameters."""
    p = ovl_outer_params()
    _lib.ovl_default_outer_params(ctypes.byref(p))
    for k, v in kw.items():
        if k == "inner":
            for ik, iv in v.items():
                if ik == "deflation":
                    set_deflation(p.inner, iv)
                    p._defl = iv
                else:
                    setattr(p.inner, ik, iv)
        else:
            setattr(p, k, v)
    return p


def overlap_solve(lat: Lattice, U: Gauge, rho: float, shifts, weights, eta: Spinor, psi: Spinor, params=None,
                  ws=None, stream=None, allow_not_converged=False) -> dict:
    """psi = D_ov^{-1} eta by FGMRES (ovl_overlap_solve); returns the stats."""
    params = params or default_outer_params()
    z, keep = _zolo(shifts, weights)
    if ws is None:
        ws = _dev_buffer(_lib.ovl_overlap_solve_workspace_bytes(lat.ref, z.npoles, ctypes.byref(params)),
                         eta.data.device)
    st = ovl_outer_stats()
    rc = _lib.ovl_overlap_solve(lat.ref, U.ref, float(rho), ctypes.byref(z), eta.ref, psi.ref, ctypes.byref(params),
                                ctypes.byref(st), c_vp(ws.data_ptr()), ws.numel(), _stream(stream))
    _check(rc, "ovl_overlap_solve", allow_not_converged)
    return st.to_dict()


def wilson_solve(lat: Lattice, U: Gauge, m0: float, b: Spinor, x: Spinor, params=None, ws=None, stream=None,
                 allow_not_converged=False) -> dict:
    """x = D_W(m0)^{-1} b (ovl_wilson_solve); returns iterations and the FP64
    true residual |b - D_W x|/|b| per RHS."""
    params = params or default_params()
    if ws is None:
        ws = workspace(lat, OP_WILSON_SOLVE, F64, b.nrhs, 0, params, device=b.data.device)
    st = ovl_solver_stats()
    rc = _lib.ovl_wilson_solve(lat.ref, U.ref, float(m0), b.ref, x.ref, ctypes.byref(params), ctypes.byref(st),
                               c_vp(ws.data_ptr()), ws.numel(), _stream(stream))
    _check(rc, "ovl_wilson_solve", allow_not_converged)
    d = st.to_dict(b.nrhs, 1)
    return dict(iterations=d["iterations"], true_residual=[r[0] for r in d["true_residual"]], seconds=d["seconds"])
