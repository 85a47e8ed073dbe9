"""GPU checks of the 48-bit storage format (OVL_F48) and of the mixed solver's
FP64 phase on it (store48).

The format keeps the top 48 bits of a double after rounding the dropped 16
to nearest, ties away from zero: ``r48`` (tests/parity.py) writes that
definition out with integer operations on the IEEE bit pattern, and packing
must reproduce it bit for bit.  Stencils on 48-bit fields compute in FP64 from the stored
values and round their outputs, so each output component lies within
1e-11 M_x of the oracle applied to the rounded input (tests/parity.py: M_x
bounds the terms summed at x; the output rounding is at most 2^-37 of the
component, and a CPU emulation of the format, Q^2 included, stays at 0.15 of
that bound).  The mixed solver with 48-bit storage must meet the FP64
storage's bar: every shifted system's FP64 true residual <= 1e-10 (library
verification, which aims at 0.9e-10 with 48-bit storage), D_ov within 1e-8 of
the oracle, and within 1e-9 of the FP64-storage form, with the same iteration
count up to one.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
import synth
from parity import field_check, r48, stencil_check

pytestmark = pytest.mark.gpu

RHO = 1.6
M0 = -RHO
TOL48 = 1e-11


def note(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ovl():
    import paper_1410_7170_amd as m
    assert torch.cuda.is_available()
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def setup(ovl, dims, eps0=0.5, seed=3, n_stout=0, bc=(-1, 1, 1, 1)):
    lat = ovl.Lattice(dims, bc)
    olat = oracle.Lattice(dims, bc)
    U = synth.gauge(dims, eps0, seed, n_stout)
    G = ovl.Gauge(lat, dev(U))
    return lat, olat, U, G


def check(got, ref, psi, dims, shift=None):
    ratio, r2 = stencil_check(got, ref, psi, dims, M0, TOL48, shift)
    assert ratio <= 1.0, (dims, ratio, r2)
    return ratio


def test_f48_pack_roundtrip_bit_exact(ovl):
    dims = (6, 4, 2, 4)
    note(f"f48 pack roundtrip dims={dims}")
    lat = ovl.Lattice(dims)
    psi = synth.gaussian_spinor(lat.V, 5, 3)
    # plant ties, carries into the exponent, zeros and tiny values
    bits = psi.view(np.uint64).reshape(-1)
    bits[0:40:4] = (bits[0:40:4] & np.uint64(0xFFFFFFFFFFFF0000)) | np.uint64(0x8000)
    bits[1:40:4] = bits[1:40:4] | np.uint64(0x000FFFFFFFFFFFFF)
    bits[2] = 0
    bits[6] = 0x0000000000012345
    s = ovl.Spinor.from_canonical(lat, dev(psi), ovl.F48)
    back = s.to_canonical().cpu().numpy()
    assert np.array_equal(back.view(np.uint64), r48(psi).view(np.uint64))


@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (2, 2, 2, 2), (6, 4, 2, 4), (10, 8, 6, 4)])
def test_f48_wilson_apply_matches_oracle(ovl, dims):
    note(f"f48 wilson_apply dims={dims}")
    lat, olat, U, G = setup(ovl, dims, seed=7)
    psi = r48(synth.gaussian_spinor(lat.V, 8, 2))
    inp = ovl.Spinor.from_canonical(lat, dev(psi), ovl.F48)
    out = ovl.Spinor(lat, ovl.F48, 2)
    ovl.wilson_apply(lat, G, M0, inp, out)
    got = out.to_canonical().cpu().numpy()
    for r in range(2):
        check(got[r], oracle.dw(olat, U, M0, psi[r]), psi[r], dims)
    ovl.q2_apply(lat, G, M0, 0.29, inp, out)
    got = out.to_canonical().cpu().numpy()
    for r in range(2):
        check(got[r], oracle.q2(olat, U, M0, psi[r], 0.29), psi[r], dims, shift=0.29)


# the time-streaming form (48-bit fields take the FP64 stream length, halved
# while the launch has fewer than 512 blocks), with and without the LDS
# staging of each slice, RHS tiles, and the two-wave staged build of launches
# above 256 blocks (the last two lattices: 1 and 2 slices per thread)
STREAM48 = [((4, 4, 8, 8), 2, 1, 2), ((16, 8, 8, 8), 4, 1, 2), ((4, 2, 16, 16), 2, 1, 2),
            ((8, 4, 24, 24), 4, 1, 2), ((4, 4, 48, 48), 2, 1, 1), ((8, 2, 16, 16), 8, 4, 5),
            ((8, 16, 32, 32), 2, 1, 1), ((16, 16, 32, 32), 4, 1, 2)]


@pytest.mark.parametrize("dims,ts,tile,nrhs", STREAM48)
def test_f48_streaming_forms_match_oracle(ovl, dims, ts, tile, nrhs):
    note(f"f48 streaming dims={dims} stream={ts} tile={tile} nrhs={nrhs}")
    lat, olat, U, G = setup(ovl, dims, seed=31, n_stout=1, bc=(-1, 1, -1, 1))
    lat.stream_t = ts
    lat.stream_t64 = ts
    lat.rhs_tile = tile
    psi = r48(synth.gaussian_spinor(lat.V, 32, nrhs))
    inp = ovl.Spinor.from_canonical(lat, dev(psi), ovl.F48)
    out = ovl.Spinor(lat, ovl.F48, nrhs)
    ovl.wilson_apply(lat, G, M0, inp, out)
    got = out.to_canonical().cpu().numpy()
    for r in range(nrhs):
        check(got[r], oracle.dw(olat, U, M0, psi[r]), psi[r], dims)
    ovl.q2_apply(lat, G, M0, 0.23, inp, out)
    got = out.to_canonical().cpu().numpy()
    for r in range(nrhs):
        check(got[r], oracle.q2(olat, U, M0, psi[r], 0.23), psi[r], dims, shift=0.23)


def test_f48_stencils_full_32x64(ovl):
    """Every site of the 32^3x64 workload field: D_W and Q^2 + s on 48-bit
    fields in the lattice's default launch (16 slices, two waves per SIMD)."""
    dims = synth.WORKLOADS[2]["dims"]
    note(f"f48 full-lattice stencils {dims}")
    lat = ovl.Lattice(dims)
    olat = oracle.Lattice(dims)
    U = synth.workload_gauge(2)
    G = ovl.Gauge(lat, dev(U))
    psi = r48(synth.workload_sources(2)[0])
    inp = ovl.Spinor.from_canonical(lat, dev(psi), ovl.F48)
    out = ovl.Spinor(lat, ovl.F48)
    ovl.wilson_apply(lat, G, M0, inp, out)
    check(out.to_canonical().cpu().numpy()[0], oracle.dw(olat, U, M0, psi), psi, dims)
    ovl.q2_apply(lat, G, M0, 0.31, inp, out)
    check(out.to_canonical().cpu().numpy()[0], oracle.q2(olat, U, M0, psi, 0.31), psi, dims, shift=0.31)


def mixed_setup(ovl, dims, seed, npoles=20):
    U = synth.gauge(dims, 0.3, seed, n_stout=2)
    lat = ovl.Lattice(dims)
    olat = oracle.Lattice(dims)
    G = ovl.Gauge(lat, dev(U))
    v0 = synth.gaussian_spinor(lat.V, seed + 1)[0]
    lo, hi = ovl.spectral_bounds(lat, G, M0, 300, ovl.Spinor.from_canonical(lat, dev(v0), 0))
    s, w, _ = ovl.zolotarev(lo, hi, npoles)
    olo, ohi = oracle.spectral_interval(olat, U, M0, v0, 300)
    os_, ow, _ = oracle.zolotarev(olo, ohi, npoles)
    return U, lat, olat, G, (s, w), (os_, ow)


def overlap(ovl, lat, G, s, w, b, nrhs, **kw):
    B = ovl.Spinor.from_canonical(lat, dev(b), 0)
    O = ovl.Spinor(lat, 0, nrhs)
    prm = ovl.default_params(tol=1e-10, maxiter=5000, mode=ovl.SOLVE_MIXED, **kw)
    st = ovl.overlap_apply(lat, G, RHO, s, w, B, O, prm)
    return O.to_canonical().cpu().numpy(), st


@pytest.mark.parametrize("dims,nrhs,sloppy_below", [((16, 8, 8, 8), 1, 1e-5), ((8, 8, 8, 8), 2, 1e-3),
                                                    ((8, 4, 4, 6), 1, 1e-7)])
def test_mixed_store48_matches_fp64_storage_and_oracle(ovl, dims, nrhs, sloppy_below):
    note(f"mixed store48 dims={dims} nrhs={nrhs} sloppy_below={sloppy_below}")
    U, lat, olat, G, (s, w), (os_, ow) = mixed_setup(ovl, dims, 401)
    b = synth.gaussian_spinor(lat.V, 402, nrhs)
    got48, st48 = overlap(ovl, lat, G, s, w, b, nrhs, sloppy_below=sloppy_below, store48=1)
    got64, st64 = overlap(ovl, lat, G, s, w, b, nrhs, sloppy_below=sloppy_below, store48=0)
    for r in range(nrhs):
        # with 48-bit storage the solve aims at 0.9 tol (the rounding's gap
        # between recursive and true residuals stays below the tenth left)
        tr = np.array(st48["true_residual"][r])
        assert (tr > 0).all() and (tr <= 0.9e-10 * (1 + 1e-9)).all(), (r, tr)
        assert abs(st48["iterations"][r] - st64["iterations"][r]) <= 1, (st48["iterations"], st64["iterations"])
        ratio, _ = field_check(got48[r], got64[r], dims, 1e-9)
        assert ratio <= 1.0, ("vs FP64 storage", r, ratio)
        ref, _, _ = oracle.overlap(olat, U, RHO, os_, ow, b[r], 1e-13, 5000)
        ratio, _ = field_check(got48[r], ref, dims, 1e-8)
        assert ratio <= 1.0, ("vs oracle", r, ratio)
    # the FP64 phase's stencils and block passes move fewer bytes
    assert st48["algorithmic_bytes"] < st64["algorithmic_bytes"]


def test_mixed_store48_falls_back_without_base(ovl):
    """With OVL_MAX_SHIFTS caller shifts there is no room for the unshifted
    base, so the FP64 phase keeps FP64 storage: the result equals the
    store48 = 0 result bit for bit."""
    dims = (8, 4, 4, 6)
    note(f"mixed store48 fallback dims={dims}")
    U, lat, olat, G, (s, w), _ = mixed_setup(ovl, dims, 411, npoles=32)
    b = synth.gaussian_spinor(lat.V, 412, 1)
    got48, st48 = overlap(ovl, lat, G, s, w, b, 1, store48=1)
    got64, st64 = overlap(ovl, lat, G, s, w, b, 1, store48=0)
    assert np.array_equal(got48, got64)
    assert (np.array(st48["true_residual"][0]) <= 1e-10).all()
