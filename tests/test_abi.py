"""Host-side checks of the C ABI (no GPU needed): the library loads, exports
every symbol include/ovl.h declares, validates arguments before touching the
device, and its host-only Zolotarev routine agrees with the oracle's."""
import ctypes
import os
import re

import numpy as np
import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def ovl():
    import paper_1410_7170_amd as m
    return m


def header_symbols():
    text = open(os.path.join(ROOT, "include", "ovl.h")).read()
    return sorted(set(re.findall(r"OVL_API[^;(]*?\b(ovl_\w+)\s*\(", text)))


def test_header_declares_entry_points():
    names = header_symbols()
    for need in ("ovl_wilson_apply", "ovl_q_apply", "ovl_q2_apply", "ovl_multishift_cg", "ovl_sign_q_apply",
                 "ovl_overlap_apply", "ovl_zolotarev", "ovl_spectral_bounds", "ovl_pack_spinor",
                 "ovl_unpack_spinor", "ovl_pack_gauge", "ovl_workspace_bytes", "ovl_lattice_init"):
        assert need in names


def test_library_exports_every_declared_symbol(ovl):
    lib = ctypes.CDLL(ovl.LIB_PATH)
    for name in header_symbols():
        assert hasattr(lib, name), name
    assert set(header_symbols()) == set(ovl.EXPORTED)


def test_lattice_validation(ovl):
    lat = ovl.Lattice((4, 4, 4, 8))
    assert lat.V == 512
    for dims, bc in [((3, 4, 4, 4), (-1, 1, 1, 1)), ((4, 4, 4, 0), (-1, 1, 1, 1)),
                     ((4, 4, 4, 4), (2, 1, 1, 1)), ((2048, 1024, 1024, 2), (1, 1, 1, 1))]:
        with pytest.raises(ovl.OvlError) as e:
            ovl.Lattice(dims, bc)
        assert e.value.status == ovl.ERR_INVALID


def test_sizes(ovl):
    lat = ovl.Lattice((4, 4, 4, 4))
    # component arrays are S = round_up(V/2, 16) + 24 sites long
    S = (128 + 15) // 16 * 16 + 24
    assert lat.spinor_bytes(ovl.F64) == 2 * 12 * S * 16
    assert lat.spinor_bytes(ovl.F32) == 2 * 6 * S * 16
    assert lat.spinor_bytes(ovl.F16S) == 2 * 3 * S * 16
    assert lat.scale_bytes() == 2 * S * 4
    assert lat.gauge_bytes(ovl.F64) == 2 * 4 * 6 * S * 16
    assert lat.gauge_bytes(ovl.F32) == 2 * 4 * 3 * S * 16
    assert lat.gauge_bytes(ovl.F16S) == 2 * 4 * 3 * S * 8
    big = ovl.Lattice((64, 32, 32, 32))
    Sb = 2 ** 20 + 24
    assert big.spinor_bytes(ovl.F64) == 24 * Sb * 16 and (Sb * 16) % (1 << 18) != 0
    p = ovl.default_params()
    assert p.tol == 1e-10 and p.mode == ovl.SOLVE_F64
    assert ovl.workspace_bytes(lat, ovl.OP_MSCG, ovl.F64, 1, 20, p) > 40 * 256 * 192
    assert ovl.workspace_bytes(lat, ovl.OP_MSCG, ovl.F64, 1, 0, p) == 0
    assert ovl.workspace_bytes(lat, ovl.OP_MSCG, ovl.F64, 17, 4, p) == 0
    # the block length runs up to OVL_MAX_BLOCK; a longer one is rejected
    pm = ovl.default_params(mode=ovl.SOLVE_MIXED, block=16)
    w16 = ovl.workspace_bytes(lat, ovl.OP_MSCG, ovl.F64, 1, 20, pm)
    pm.block = ovl.MAX_BLOCK
    assert ovl.workspace_bytes(lat, ovl.OP_MSCG, ovl.F64, 1, 20, pm) > w16 > 0
    pm.block = ovl.MAX_BLOCK + 1
    assert ovl.workspace_bytes(lat, ovl.OP_MSCG, ovl.F64, 1, 20, pm) == 0
    # the FP64 phase's block length of the mixed form, likewise
    pm.block = 0
    w0 = ovl.workspace_bytes(lat, ovl.OP_MSCG, ovl.F64, 1, 20, pm)
    pm.block_f64 = ovl.MAX_BLOCK
    assert ovl.workspace_bytes(lat, ovl.OP_MSCG, ovl.F64, 1, 20, pm) > w0 > 0
    pm.block_f64 = -1
    assert ovl.workspace_bytes(lat, ovl.OP_MSCG, ovl.F64, 1, 20, pm) == 0


def test_null_and_alias_rejected_before_launch(ovl):
    lat = ovl.Lattice((4, 4, 4, 4))
    lib = ovl._lib
    s = ovl.ovl_spinor(None, None, ovl.F64, 1)
    g = ovl.ovl_gauge(None, None, None)
    assert lib.ovl_wilson_apply(lat.ref, ctypes.byref(g), -1.6, ctypes.byref(s), ctypes.byref(s), None) == ovl.ERR_INVALID
    fake = ovl.ovl_spinor(ctypes.c_void_p(4096), None, ovl.F64, 1)
    gf = ovl.ovl_gauge(ctypes.c_void_p(8192), None, None)
    # in == out
    assert lib.ovl_wilson_apply(lat.ref, ctypes.byref(gf), -1.6, ctypes.byref(fake), ctypes.byref(fake), None) == ovl.ERR_INVALID
    # F16S needs scales; nrhs range; precision mismatch
    h = ovl.ovl_spinor(ctypes.c_void_p(4096), None, ovl.F16S, 1)
    o = ovl.ovl_spinor(ctypes.c_void_p(1 << 20), None, ovl.F64, 1)
    assert lib.ovl_wilson_apply(lat.ref, ctypes.byref(gf), -1.6, ctypes.byref(h), ctypes.byref(o), None) == ovl.ERR_INVALID
    big = ovl.ovl_spinor(ctypes.c_void_p(4096), None, ovl.F64, 17)
    assert lib.ovl_q_apply(lat.ref, ctypes.byref(gf), -1.6, ctypes.byref(big), ctypes.byref(o), None) == ovl.ERR_INVALID
    o32 = ovl.ovl_spinor(ctypes.c_void_p(1 << 20), None, ovl.F32, 1)
    assert lib.ovl_q_apply(lat.ref, ctypes.byref(gf), -1.6, ctypes.byref(fake), ctypes.byref(o32), None) == ovl.ERR_INVALID
    # missing gauge precision
    assert lib.ovl_q_apply(lat.ref, ctypes.byref(gf), -1.6, ctypes.byref(o32),
                           ctypes.byref(ovl.ovl_spinor(ctypes.c_void_p(1 << 22), None, ovl.F32, 1)), None) == ovl.ERR_INVALID
    # workspace too small for q2
    assert lib.ovl_q2_apply(lat.ref, ctypes.byref(gf), -1.6, 0.1, ctypes.byref(fake), ctypes.byref(o),
                            ctypes.c_void_p(1 << 24), 16, None) == ovl.ERR_WORKSPACE


def test_autotune_rejected_before_launch(ovl):
    lat = ovl.Lattice((4, 4, 4, 4))
    lib = ovl._lib
    g0 = ovl.ovl_gauge(None, None, None)
    gf = ovl.ovl_gauge(ctypes.c_void_p(8192), None, None)
    ws = ctypes.c_void_p(1 << 24)
    need = lib.ovl_workspace_bytes(lat.ref, ovl.OP_TUNE, 0, 1, 0, None)
    assert need > 6 * lat.spinor_bytes(ovl.F16S)
    # no links, no workspace, bad RHS count, too small a workspace
    assert lib.ovl_autotune_stencil(lat.ref, ctypes.byref(g0), 1, ws, need, None, None, 0, None) == ovl.ERR_INVALID
    assert lib.ovl_autotune_stencil(lat.ref, ctypes.byref(gf), 1, None, need, None, None, 0, None) == ovl.ERR_INVALID
    assert lib.ovl_autotune_stencil(lat.ref, ctypes.byref(gf), 0, ws, need, None, None, 0, None) == ovl.ERR_INVALID
    assert lib.ovl_autotune_stencil(lat.ref, ctypes.byref(gf), 17, ws, need, None, None, 0, None) == ovl.ERR_INVALID
    assert lib.ovl_autotune_stencil(lat.ref, ctypes.byref(gf), 1, ws, 64, None, None, 0, None) == ovl.ERR_WORKSPACE


def test_solver_params_rejected(ovl):
    lat = ovl.Lattice((4, 4, 4, 4))
    lib = ovl._lib
    b = ovl.ovl_spinor(ctypes.c_void_p(4096), None, ovl.F64, 1)
    o = ovl.ovl_spinor(ctypes.c_void_p(1 << 20), None, ovl.F64, 1)
    gf = ovl.ovl_gauge(ctypes.c_void_p(8192), None, None)
    s = (ctypes.c_double * 2)(0.1, 0.2)
    w = (ctypes.c_double * 2)(1.0, 1.0)
    z = ovl.ovl_zolo(2, s, w)
    st = ovl.ovl_solver_stats()
    for bad in [dict(tol=0.0), dict(tol=float("nan")), dict(maxiter=0), dict(mode=7), dict(reliable_delta=1.5)]:
        p = ovl.default_params(**bad)
        rc = lib.ovl_overlap_apply(lat.ref, ctypes.byref(gf), 1.6, ctypes.byref(z), ctypes.byref(b), ctypes.byref(o),
                                   ctypes.byref(p), ctypes.byref(st), ctypes.c_void_p(1 << 26), 1 << 30, None)
        assert rc == ovl.ERR_INVALID, bad
    p = ovl.default_params()
    rc = lib.ovl_overlap_apply(lat.ref, ctypes.byref(gf), -1.0, ctypes.byref(z), ctypes.byref(b), ctypes.byref(o),
                               ctypes.byref(p), ctypes.byref(st), ctypes.c_void_p(1 << 26), 1 << 30, None)
    assert rc == ovl.ERR_INVALID
    nz = ovl.ovl_zolo(0, s, w)
    rc = lib.ovl_overlap_apply(lat.ref, ctypes.byref(gf), 1.6, ctypes.byref(nz), ctypes.byref(b), ctypes.byref(o),
                               ctypes.byref(p), ctypes.byref(st), ctypes.c_void_p(1 << 26), 1 << 30, None)
    assert rc == ovl.ERR_INVALID
    rc = lib.ovl_overlap_apply(lat.ref, ctypes.byref(gf), 1.6, ctypes.byref(z), ctypes.byref(b), ctypes.byref(o),
                               ctypes.byref(p), ctypes.byref(st), ctypes.c_void_p(1 << 26), 64, None)
    assert rc == ovl.ERR_WORKSPACE


def test_status_strings(ovl):
    for s in (0, 1, -1, -2, -3, -4):
        assert ovl._lib.ovl_status_string(s).decode()
    assert ovl.version().startswith("ovl")


@pytest.mark.parametrize("k", [0.001, 0.01, 0.05, 0.075, 0.3, 0.9])
@pytest.mark.parametrize("n", [1, 4, 12, 20, 24, 32])
def test_zolotarev_library_matches_oracle(ovl, k, n):
    """The library derives sn/cn from theta functions, the oracle from the
    descending Landen scheme; both give the same Zolotarev coefficients."""
    s, w, d = ovl.zolotarev(k, 1.0, n)
    s2, w2, d2 = oracle.zolotarev(k, 1.0, n)
    tol = 1e-13 if k >= 0.05 else 1e-11
    assert np.max(np.abs(s - s2) / s2) < tol
    assert np.max(np.abs(w - w2) / w2) < tol
    # delta near 1e-12 is at the rounding level of evaluating R itself
    assert abs(d - d2) < 5e-13 + 1e-6 * d2
    # scaling to [lmin, lmax]
    s3, w3, d3 = ovl.zolotarev(0.5 * k, 0.5, n)
    assert np.allclose(s3, s * 0.25, rtol=1e-13) and np.allclose(w3, w * 0.5, rtol=1e-13)


def test_zolotarev_rejects(ovl):
    for args in [(0.0, 1.0, 4), (1.0, 0.5, 4), (0.1, 1.0, 0), (0.1, 1.0, 33), (0.1, float("inf"), 4)]:
        with pytest.raises(ovl.OvlError):
            ovl.zolotarev(*args)


def test_deflation_rejected_before_launch(ovl):
    """ovl_deflation: FP64 eigenvectors, 1..OVL_MAX_NEV of them, finite
    eigenvalues, no aliasing with the call's fields; its bytes count in the
    workspace."""
    lat = ovl.Lattice((4, 4, 4, 4))
    lib = ovl._lib
    b = ovl.ovl_spinor(ctypes.c_void_p(4096), None, ovl.F64, 1)
    o = ovl.ovl_spinor(ctypes.c_void_p(1 << 20), None, ovl.F64, 1)
    gf = ovl.ovl_gauge(ctypes.c_void_p(8192), None, None)
    s = (ctypes.c_double * 2)(0.1, 0.2)
    w = (ctypes.c_double * 2)(1.0, 1.0)
    z = ovl.ovl_zolo(2, s, w)
    st = ovl.ovl_solver_stats()
    ev = (ctypes.c_double * 4)(0.1, -0.2, 0.3, -0.4)
    bad_ev = (ctypes.c_double * 4)(0.1, float("nan"), 0.3, -0.4)
    cases = [ovl.ovl_deflation(ovl.ovl_spinor(ctypes.c_void_p(1 << 24), None, ovl.F32, 4), ev),
             ovl.ovl_deflation(ovl.ovl_spinor(ctypes.c_void_p(1 << 24), None, ovl.F64, 0), ev),
             ovl.ovl_deflation(ovl.ovl_spinor(ctypes.c_void_p(1 << 24), None, ovl.F64, 257), ev),
             ovl.ovl_deflation(ovl.ovl_spinor(ctypes.c_void_p(1 << 24), None, ovl.F64, 4), bad_ev),
             ovl.ovl_deflation(ovl.ovl_spinor(ctypes.c_void_p(1 << 24), None, ovl.F64, 4), None),
             ovl.ovl_deflation(ovl.ovl_spinor(ctypes.c_void_p(4096), None, ovl.F64, 4), ev)]   # aliases b
    for d in cases:
        p = ovl.default_params()
        p.deflation = ctypes.pointer(d)
        for fn in (lib.ovl_overlap_apply, lib.ovl_sign_q_apply):
            rc = fn(lat.ref, ctypes.byref(gf), 1.6 if fn is lib.ovl_overlap_apply else -1.6, ctypes.byref(z),
                    ctypes.byref(b), ctypes.byref(o), ctypes.byref(p), ctypes.byref(st), ctypes.c_void_p(1 << 26),
                    1 << 30, None)
            assert rc == ovl.ERR_INVALID
    good = ovl.ovl_deflation(ovl.ovl_spinor(ctypes.c_void_p(1 << 24), None, ovl.F64, 4), ev)
    p = ovl.default_params()
    base = lib.ovl_workspace_bytes(lat.ref, ovl.OP_MSCG, ovl.F64, 1, 2, ctypes.byref(p))
    p.deflation = ctypes.pointer(good)
    need = lib.ovl_workspace_bytes(lat.ref, ovl.OP_MSCG, ovl.F64, 1, 2, ctypes.byref(p))
    assert need >= base + lat.spinor_bytes(ovl.F64)
    rc = lib.ovl_overlap_apply(lat.ref, ctypes.byref(gf), 1.6, ctypes.byref(z), ctypes.byref(b), ctypes.byref(o),
                               ctypes.byref(p), ctypes.byref(st), ctypes.c_void_p(1 << 26), need - 1, None)
    assert rc == ovl.ERR_WORKSPACE


def test_low_modes_rejected_before_launch(ovl):
    lat = ovl.Lattice((4, 4, 4, 4))
    lib = ovl._lib
    gf = ovl.ovl_gauge(ctypes.c_void_p(8192), None, None)
    start = ovl.ovl_spinor(ctypes.c_void_p(4096), None, ovl.F64, 1)
    ev = (ctypes.c_double * 8)()
    res = (ctypes.c_double * 8)()
    st = ovl.ovl_eig_stats()
    ws = ctypes.c_void_p(1 << 26)

    def call(p, evecs, start=start, g=gf, nbytes=1 << 40):
        return lib.ovl_low_modes(lat.ref, ctypes.byref(g), -1.6, ctypes.byref(start), ctypes.byref(p),
                                 ctypes.byref(evecs), ev, res, ctypes.byref(st), ws, nbytes, None)

    ok = ovl.ovl_spinor(ctypes.c_void_p(1 << 24), None, ovl.F64, 8)
    for field, value in (("nev", 0), ("nev", 300), ("degree", 0), ("degree", 201), ("stages", 0), ("steps", 5),
                         ("tol", 0.0), ("extra", -1)):
        p = ovl.ovl_eig_params()
        lib.ovl_default_eig_params(ctypes.byref(p))
        p.nev = 8
        setattr(p, field, value)
        assert lib.ovl_low_modes_workspace_bytes(lat.ref, ctypes.byref(p)) == 0, field
        assert call(p, ok) == ovl.ERR_INVALID, field
    p = ovl.ovl_eig_params()
    lib.ovl_default_eig_params(ctypes.byref(p))
    p.nev = 8
    need = lib.ovl_low_modes_workspace_bytes(lat.ref, ctypes.byref(p))
    assert need > 40 * lat.spinor_bytes(ovl.F64)
    # evecs count, precision and aliasing; start count; missing FP64 links; workspace
    assert call(p, ovl.ovl_spinor(ctypes.c_void_p(1 << 24), None, ovl.F64, 7)) == ovl.ERR_INVALID
    assert call(p, ovl.ovl_spinor(ctypes.c_void_p(1 << 24), None, ovl.F32, 8)) == ovl.ERR_INVALID
    assert call(p, ovl.ovl_spinor(ctypes.c_void_p(4096), None, ovl.F64, 8)) == ovl.ERR_INVALID
    assert call(p, ok, start=ovl.ovl_spinor(ctypes.c_void_p(4096), None, ovl.F64, 2)) == ovl.ERR_INVALID
    assert call(p, ok, g=ovl.ovl_gauge(None, ctypes.c_void_p(8192), None)) == ovl.ERR_INVALID
    assert call(p, ok, nbytes=need - 1) == ovl.ERR_WORKSPACE


def test_new_descriptor_fields_validated(ovl):
    """rhs_tile in {1, 2, 4, 8}, mfma in {0, 1}, sloppy_f16 in {0, 1}."""
    lat = ovl.Lattice((4, 4, 4, 4))
    lib = ovl._lib
    gf = ovl.ovl_gauge(ctypes.c_void_p(8192), ctypes.c_void_p(8192), None)
    i = ovl.ovl_spinor(ctypes.c_void_p(4096), None, ovl.F32, 2)
    o = ovl.ovl_spinor(ctypes.c_void_p(1 << 20), None, ovl.F32, 2)
    for field, value in (("rhs_tile", 3), ("rhs_tile", 16), ("mfma", 2), ("mfma", -1)):
        l2 = ovl.Lattice((4, 4, 4, 4))
        setattr(l2.c, field, value)
        assert lib.ovl_wilson_apply(l2.ref, ctypes.byref(gf), -1.6, ctypes.byref(i), ctypes.byref(o), None) \
            == ovl.ERR_INVALID, field
    p = ovl.default_params(mode=ovl.SOLVE_MIXED, sloppy_f16=2)
    assert lib.ovl_workspace_bytes(lat.ref, ovl.OP_MSCG, ovl.F64, 1, 2, ctypes.byref(p)) == 0


def test_even_odd_wilson_solve_fields(ovl):
    """even_odd in {0, 1} (default 0) for ovl_wilson_solve, with its own
    workspace size; prec_even_odd in {0, 1} (default 1) for the outer solve.
    Both are checked before any device work."""
    lat = ovl.Lattice((4, 4, 4, 8))
    lib = ovl._lib
    assert ovl.default_params().even_odd == 0 and ovl.default_outer_params().prec_even_odd == 1
    ws = [lib.ovl_workspace_bytes(lat.ref, ovl.OP_WILSON_SOLVE, ovl.F64, 1, 0,
                                  ctypes.byref(ovl.default_params(even_odd=eo))) for eo in (0, 1)]
    assert ws[0] > 0 and ws[1] > 0 and ws[0] != ws[1]
    gf = ovl.ovl_gauge(ctypes.c_void_p(8192), ctypes.c_void_p(8192), None)
    b = ovl.ovl_spinor(ctypes.c_void_p(4096), None, ovl.F64, 1)
    x = ovl.ovl_spinor(ctypes.c_void_p(1 << 20), None, ovl.F64, 1)
    st = ovl.ovl_solver_stats()
    for eo in (2, -1):
        p = ovl.default_params(even_odd=eo)
        assert lib.ovl_wilson_solve(lat.ref, ctypes.byref(gf), -0.5, ctypes.byref(b), ctypes.byref(x),
                                    ctypes.byref(p), ctypes.byref(st), ctypes.c_void_p(1 << 24), 1 << 30,
                                    None) == ovl.ERR_INVALID
        assert lib.ovl_workspace_bytes(lat.ref, ovl.OP_WILSON_SOLVE, ovl.F64, 1, 0, ctypes.byref(p)) == 0
        q = ovl.default_outer_params(precondition=1, prec_m0=-0.5, prec_even_odd=eo)
        assert lib.ovl_overlap_solve_workspace_bytes(lat.ref, 12, ctypes.byref(q)) == 0
    q = ovl.default_outer_params(precondition=1, prec_m0=-0.5, prec_even_odd=1)
    assert lib.ovl_overlap_solve_workspace_bytes(lat.ref, 12, ctypes.byref(q)) > 0


def test_store48_field_and_f48_sizes(ovl):
    """store48 in {0, 1} (default 1, hand-over default 3e-5); a 48-bit field
    takes 3/4 of an FP64 one; the mixed workspace with 48-bit storage is sized
    for either form of the FP64 phase (it falls back to FP64 storage without
    an unshifted base), so it is at least the FP64-storage size."""
    lat = ovl.Lattice((8, 4, 4, 8))
    lib = ovl._lib
    p = ovl.default_params()
    assert p.store48 == 1 and p.sloppy_below == 3e-5
    assert lib.ovl_spinor_bytes(lat.ref, ovl.F48) * 4 == lib.ovl_spinor_bytes(lat.ref, ovl.F64) * 3
    assert lib.ovl_gauge_bytes(lat.ref, ovl.F48) == 0    # links exist in F64, F32 and F16 only
    ws = {s: lib.ovl_workspace_bytes(lat.ref, ovl.OP_MSCG, ovl.F64, 1, 20,
                                     ctypes.byref(ovl.default_params(mode=ovl.SOLVE_MIXED, store48=s)))
          for s in (0, 1)}
    assert ws[0] > 0 and ws[1] >= ws[0]
    for bad in (2, -1):
        q = ovl.default_params(mode=ovl.SOLVE_MIXED, store48=bad)
        assert lib.ovl_workspace_bytes(lat.ref, ovl.OP_MSCG, ovl.F64, 1, 20, ctypes.byref(q)) == 0
