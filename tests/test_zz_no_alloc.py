"""The entry point without allocation, ovl_q2_apply_noalloc, against
ovl_q2_apply (caller workspace) through the C ABI: two calls in a row, the
second on a smaller lattice, in each storage precision; the results must be
bit-identical to the workspace form (same kernels, same launch shapes) and
meet the oracle's element-wise bound.  An input whose intermediate field does
not fit the scratch array is refused before any device work."""
import sys

import numpy as np
import pytest
import torch

import oracle
import synth
from parity import f16s_stencil_check, stencil_check

pytestmark = pytest.mark.gpu

M0 = -1.6


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


def one_case(ovl, dims, nrhs, prec, shift, seed):
    note(f"q2 noalloc dims={dims} nrhs={nrhs} prec={prec}")
    lat = ovl.Lattice(dims)
    U = synth.gauge(dims, 0.3, seed, n_stout=1)
    G = ovl.Gauge(lat, dev(U))
    psi = synth.gaussian_spinor(lat.V, seed + 1, nrhs)
    inp = ovl.Spinor.from_canonical(lat, dev(psi), prec)
    a, b = ovl.Spinor(lat, prec, nrhs), ovl.Spinor(lat, prec, nrhs)
    ovl.q2_apply_noalloc(lat, G, M0, shift, inp, a)
    ovl.q2_apply(lat, G, M0, shift, inp, b)
    ga, gb = a.to_canonical().cpu().numpy(), b.to_canonical().cpu().numpy()
    assert np.array_equal(ga, gb)
    olat = oracle.Lattice(dims)
    for r in range(nrhs):
        ref = oracle.q2(olat, U, M0, psi[r], shift)
        if prec == ovl.F16S:
            ratio, _ = f16s_stencil_check(ga[r], ref, psi[r], dims, M0, shift=shift,
                                          ref_mid=oracle.q(olat, U, M0, psi[r]))
        else:
            ratio, _ = stencil_check(ga[r], ref, psi[r], dims, M0, 1e-12 if prec == ovl.F64 else 1e-6, shift=shift)
        assert ratio <= 1.0, (dims, prec, r, ratio)


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_noalloc_q2_matches_workspace_form(ovl, prec):
    one_case(ovl, (32, 16, 16, 16), 2, prec, 0.37, 401)
    one_case(ovl, (8, 4, 4, 8), 1, prec, 0.19, 403)


def test_noalloc_q2_refuses_oversized_input(ovl):
    # 16 FP64 fields at 16^3x32 need 403 MB of scratch, above the 256 MiB
    # array: refused before any device work (the small buffers below are never
    # touched)
    lat = ovl.Lattice((32, 16, 16, 16))
    need = ovl.workspace_bytes(lat, ovl.OP_Q2, ovl.F64, 16)
    assert need > ovl.NOALLOC_SCRATCH_BYTES
    small = ovl.Spinor(ovl.Lattice((4, 4, 4, 4)), ovl.F64)
    fake_in = ovl.ovl_spinor(small.c.d, None, ovl.F64, 16)
    fake_out = ovl.ovl_spinor(small.c.d + 256, None, ovl.F64, 16)
    G = ovl.Gauge(ovl.Lattice((4, 4, 4, 4)), dev(synth.unit_gauge((4, 4, 4, 4))))
    import ctypes
    rc = ovl._lib.ovl_q2_apply_noalloc(lat.ref, G.ref, M0, 0.1, ctypes.byref(fake_in), ctypes.byref(fake_out),
                                       ovl._stream(None))
    assert rc == ovl.ERR_WORKSPACE
