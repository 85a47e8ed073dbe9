"""CPU checks of the element-wise parity bounds in tests/parity.py.

The GPU's storage rounding is emulated on the oracle: inputs rounded to FP32,
or to FP16 with one scale per site and FP16 links whose third row is rebuilt
as conj(row0 x row1), the oracle's FP64 stencil applied to the rounded
inputs, and the output rounded again.  The derived per-site bounds must hold
for these emulated results, must not be loose by orders of magnitude, and must
reject a result with a single wrong site (a mistake planted here, on the CPU).
"""
import numpy as np
import pytest

import oracle
import synth
from parity import f16s_stencil_check, field_check, r48, stencil_check

M0 = -1.6
DIMS = (4, 4, 6, 4)


def round_f16s(psi):
    """FP16 storage with one FP32 scale per site (largest |real or imag|)."""
    v = np.asarray(psi).reshape(-1, 12).astype(np.complex64)
    re, im = v.real, v.imag
    sc = np.maximum(np.abs(re), np.abs(im)).max(axis=1).astype(np.float32)
    sc = np.where(sc > 0, sc, np.float32(1.0))
    inv = (np.float32(1.0) / sc)[:, None]
    hr = (re * inv).astype(np.float16).astype(np.float32) * sc[:, None]
    hi = (im * inv).astype(np.float16).astype(np.float32) * sc[:, None]
    return (hr.astype(np.float64) + 1j * hi.astype(np.float64)).reshape(np.shape(psi))


def round_links_f16(U):
    r = U[..., :2, :]
    r16 = r.real.astype(np.float16).astype(np.float64) + 1j * r.imag.astype(np.float16).astype(np.float64)
    out = np.empty_like(U)
    out[..., :2, :] = r16
    out[..., 2, :] = np.conj(np.cross(r16[..., 0, :], r16[..., 1, :]))
    return out


@pytest.fixture(scope="module")
def field():
    U = synth.gauge(DIMS, 0.5, 3, n_stout=1)
    psi = synth.gaussian_spinor(synth.volume(DIMS), 4)[0]
    return oracle.Lattice(DIMS), U, psi


def test_fp32_rounded_inputs_within_bound_and_planted_site_fails(field):
    olat, U, psi = field
    ref = oracle.dw(olat, U, M0, psi)
    emu = oracle.dw(olat, U.astype(np.complex64).astype(np.complex128), M0,
                    psi.astype(np.complex64).astype(np.complex128))
    ratio, r2 = stencil_check(emu, ref, psi, DIMS, M0, 1e-6)
    assert 1e-4 < ratio <= 1.0, ratio
    bad = emu.copy()
    bad[37, 2, 1] += 1e-3 * np.abs(ref[37]).max()
    assert stencil_check(bad, ref, psi, DIMS, M0, 1e-6)[0] > 1.0


def test_f16s_emulated_stencil_within_bound_and_planted_site_fails(field):
    olat, U, psi = field
    ref = oracle.dw(olat, U, M0, psi)
    emu = round_f16s(oracle.dw(olat, round_links_f16(U), M0, round_f16s(psi)))
    ratio, r2 = f16s_stencil_check(emu, ref, psi, DIMS, M0)
    assert 0.02 < ratio <= 1.0, ratio
    # a single site off by 5% of its own size, far above the storage rounding
    bad = emu.copy()
    bad[101] *= 1.05
    assert f16s_stencil_check(bad, ref, psi, DIMS, M0)[0] > 1.0


def test_f16s_emulated_q2_within_bound(field):
    olat, U, psi = field
    s = 0.37
    qref = oracle.q(olat, U, M0, psi)
    ref = oracle.q2(olat, U, M0, psi, s)
    U16 = round_links_f16(U)
    p16 = round_f16s(psi)
    t16 = round_f16s(oracle.q(olat, U16, M0, p16))
    emu = round_f16s(oracle.q(olat, U16, M0, t16) + s * p16)
    ratio, _ = f16s_stencil_check(emu, ref, psi, DIMS, M0, shift=s, ref_mid=qref)
    assert 0.01 < ratio <= 1.0, ratio


def test_field_check_spread_error_passes_single_site_fails(field):
    olat, U, psi = field
    rng = np.random.default_rng(5)
    ref = psi
    noise = rng.standard_normal(ref.shape) + 1j * rng.standard_normal(ref.shape)
    got = ref + 1e-11 * np.linalg.norm(ref) / np.linalg.norm(noise) * noise   # field-wide 1e-11
    assert field_check(got, ref, DIMS, 1e-10)[0] <= 1.0
    bad = got.copy()
    bad[5, 0, 0] += 1e-6 * np.abs(ref).max()
    assert field_check(bad, ref, DIMS, 1e-10)[0] > 1.0


def test_r48_definition_on_hand_values():
    """The 48-bit rounding emulation of the GPU tests, on values whose
    rounding is known by hand."""
    def d(bits):
        return np.array([bits], dtype=np.uint64).view(np.float64)[0]
    one = 0x3FF0000000000000
    cases = [
        (one | 0x7FFF, one),                       # below half an ulp: down
        (one | 0x8000, one | 0x10000),             # a tie: away from zero
        (one | 0x18000, one | 0x20000),            # a tie above an odd unit: away from zero
        (0x3FFFFFFFFFFF8000, 0x4000000000000000),  # the carry moves into the exponent
        (0xBFF0000000008000, 0xBFF0000000010000),  # negative tie: larger magnitude
        (0x7FF0000000000000, 0x7FF0000000000000),  # infinity stays
    ]
    for src, want in cases:
        got = r48(np.array([complex(d(src), 0.0)]))[0].real
        assert np.array([got]).view(np.uint64)[0] == want, (hex(src), got)
