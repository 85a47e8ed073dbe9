"""GPU parity of the Wilson stencil family (wilson_apply, q_apply, q2_apply,
pack/unpack) against the FP64 oracle, through the C ABI.

Every comparison is element by element (tests/parity.py): each component at
site x lies within tol * M_x of the oracle, M_x = |m0+4| |psi(x)| + sum of the
8 neighbours' |psi(y)| (the size of the terms summed at x), with tol 1e-12
for the FP64 path and 1e-6 for FP32 links and spinors; FP16 storage with
per-site scales meets a per-site bound derived from the storage rounding of
inputs, links and output.  The field-wide relative L2 difference is reported
beside it.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
import synth
from parity import f16s_stencil_check, stencil_check

pytestmark = pytest.mark.gpu

RHO = 1.6
M0 = -RHO
# element-wise tolerance relative to M_x per storage precision (F16S: the
# derived per-site bound instead)
TOL = {0: 1e-12, 1: 1e-6}


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


def check(prec, got, ref, psi, dims, shift=None, ref_mid=None, tol=None):
    """Element-wise GPU vs oracle check of one stencil output; returns the
    worst site's error over its bound and the relative L2 difference."""
    if prec == 2:
        ratio, r2 = f16s_stencil_check(got, ref, psi, dims, M0, shift, ref_mid)
    else:
        ratio, r2 = stencil_check(got, ref, psi, dims, M0, tol or TOL[prec], shift)
    assert ratio <= 1.0, (prec, dims, ratio, r2)
    return ratio, r2


def setup(ovl, dims, eps0=0.5, seed=3, n_stout=0, bc=(-1, 1, 1, 1)):
    lat = ovl.Lattice(dims, bc)
    olat = oracle.Lattice(dims, bc)
    U = synth.gauge(dims, eps0, seed, n_stout)
    G = ovl.Gauge(lat, dev(U))
    return lat, olat, U, G


LATTICES = [(4, 4, 4, 4), (2, 2, 2, 2), (6, 4, 2, 4), (8, 4, 4, 6), (4, 6, 6, 8), (10, 8, 6, 4)]


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_pack_roundtrip(ovl, prec):
    dims = (6, 4, 2, 4)
    note(f"pack roundtrip prec={prec} dims={dims}")
    lat = ovl.Lattice(dims)
    psi = synth.gaussian_spinor(lat.V, 5, 3)
    s = ovl.Spinor.from_canonical(lat, dev(psi), prec)
    back = s.to_canonical().cpu().numpy()
    if prec == 0:
        assert np.array_equal(back, psi)
    elif prec == 1:
        assert np.abs(back - psi).max() <= 6e-8 * np.abs(psi).max()
    else:
        site_max = np.maximum(np.abs(psi.real), np.abs(psi.imag)).reshape(3, lat.V, 12).max(-1)
        err = np.abs(back - psi).reshape(3, lat.V, 12).max(-1)
        assert (err <= 2 ** -11 * site_max * 1.01).all()


@pytest.mark.parametrize("dims", LATTICES)
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_wilson_apply_matches_oracle(ovl, dims, prec):
    note(f"wilson_apply prec={prec} dims={dims}")
    lat, olat, U, G = setup(ovl, dims, seed=7)
    psi = synth.gaussian_spinor(lat.V, 8, 2)
    inp = ovl.Spinor.from_canonical(lat, dev(psi), prec)
    out = ovl.Spinor(lat, prec, 2)
    ovl.wilson_apply(lat, G, M0, inp, out)
    got = out.to_canonical().cpu().numpy()
    for r in range(2):
        check(prec, got[r], oracle.dw(olat, U, M0, psi[r]), psi[r], dims)


@pytest.mark.parametrize("bc", [(1, 1, 1, 1), (-1, -1, 1, -1)])
def test_boundary_phases(ovl, bc):
    dims = (4, 4, 6, 4)
    note(f"boundary phases bc={bc}")
    lat, olat, U, G = setup(ovl, dims, seed=9, bc=bc)
    psi = synth.gaussian_spinor(lat.V, 10)[0]
    inp = ovl.Spinor.from_canonical(lat, dev(psi), 0)
    out = ovl.Spinor(lat, 0)
    ovl.wilson_apply(lat, G, M0, inp, out)
    check(0, out.to_canonical().cpu().numpy()[0], oracle.dw(olat, U, M0, psi), psi, dims)


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_q_and_q2_match_oracle(ovl, prec):
    dims = (8, 4, 4, 6)
    note(f"q/q2 prec={prec}")
    lat, olat, U, G = setup(ovl, dims, seed=11, n_stout=1)
    psi = synth.gaussian_spinor(lat.V, 12)[0]
    inp = ovl.Spinor.from_canonical(lat, dev(psi), prec)
    out = ovl.Spinor(lat, prec)
    ovl.q_apply(lat, G, M0, inp, out)
    qref = oracle.q(olat, U, M0, psi)
    check(prec, out.to_canonical().cpu().numpy()[0], qref, psi, dims)
    ovl.q2_apply(lat, G, M0, 0.37, inp, out)
    check(prec, out.to_canonical().cpu().numpy()[0], oracle.q2(olat, U, M0, psi, 0.37), psi, dims, shift=0.37,
          ref_mid=qref)


def test_gamma5_hermiticity_gpu(ovl):
    """<phi, Q psi> = <Q phi, psi> for the GPU operator (eq. (gamma_5_symmetry))."""
    dims = (8, 6, 4, 4)
    lat, olat, U, G = setup(ovl, dims, seed=13)
    phi, psi = synth.gaussian_spinor(lat.V, 14, 2)
    a = ovl.Spinor.from_canonical(lat, dev(np.stack([phi, psi])), 0)
    out = ovl.Spinor(lat, 0, 2)
    ovl.q_apply(lat, G, M0, a, out)
    q = out.to_canonical().cpu().numpy()
    x = np.vdot(phi, q[1])
    y = np.vdot(q[0], psi)
    assert abs(x - y) / abs(x) < 1e-14


def test_free_field_plane_wave_gpu(ovl):
    """Unit links: the GPU stencil multiplies a plane wave by
    m0 + sum(1 - cos p) + i sum sin(p) gamma (closed form from eq. (Wilson-Dirac))."""
    dims = (8, 4, 6, 4)
    lat = ovl.Lattice(dims)
    U = synth.unit_gauge(dims)
    G = ovl.Gauge(lat, dev(U))
    rng = np.random.default_rng(3)
    chi = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    n = (3, 1, 2, 1)
    p = np.array([(2 * n[0] + 1) * np.pi / dims[0]] + [2 * np.pi * n[k] / dims[k] for k in (1, 2, 3)])
    x = np.stack(np.meshgrid(*[np.arange(l) for l in dims], indexing="ij"), -1).reshape(-1, 4)
    psi = np.exp(1j * (x @ p))[:, None, None] * chi[None]
    A = (M0 + np.sum(1 - np.cos(p))) * np.eye(4, dtype=complex)
    for mu in range(4):
        A = A + 1j * np.sin(p[mu]) * oracle.gamma(mu)
    expect = np.einsum("ab,xbc->xac", A, psi)
    for prec in (0, 1, 2):
        inp = ovl.Spinor.from_canonical(lat, dev(psi), prec)
        out = ovl.Spinor(lat, prec)
        ovl.wilson_apply(lat, G, M0, inp, out)
        check(prec, out.to_canonical().cpu().numpy()[0], expect, psi, dims)


def test_q2_diagonal_gpu(ovl):
    """<e, Q^2 e> = (m0+4)^2 + 4 for point sources on any SU(3) field."""
    dims = (4, 4, 6, 8)
    lat, olat, U, G = setup(ovl, dims, seed=15)
    rng = np.random.default_rng(2)
    e = np.zeros((4, lat.V, 4, 3), dtype=complex)
    for r in range(4):
        e[r, rng.integers(lat.V), rng.integers(4), rng.integers(3)] = 1.0
    inp = ovl.Spinor.from_canonical(lat, dev(e), 0)
    out = ovl.Spinor(lat, 0, 4)
    ovl.q2_apply(lat, G, M0, 0.0, inp, out)
    q = out.to_canonical().cpu().numpy()
    for r in range(4):
        assert abs(np.vdot(e[r], q[r]) - ((M0 + 4) ** 2 + 4)) < 1e-13


def test_wilson_apply_16x32_full(ovl):
    """The 16^3x32 workload (links exp(i 0.3 H), 2 stout steps), every site."""
    dims = synth.WORKLOADS[1]["dims"]
    note(f"wilson_apply full {dims}")
    lat = ovl.Lattice(dims)
    olat = oracle.Lattice(dims)
    U = synth.workload_gauge(1)
    G = ovl.Gauge(lat, dev(U))
    psi = synth.workload_sources(1)[0]
    ref = oracle.dw(olat, U, M0, psi)
    for prec in (0, 1, 2):
        inp = ovl.Spinor.from_canonical(lat, dev(psi), prec)
        out = ovl.Spinor(lat, prec)
        ovl.wilson_apply(lat, G, M0, inp, out)
        ratio, r2 = check(prec, out.to_canonical().cpu().numpy()[0], ref, psi, dims)
        note(f"  prec={prec} worst site / bound {ratio:.3g}, rel L2 {r2:.3g}")


def test_wilson_apply_32x64_full(ovl):
    """The 32^3x64 workload in the benchmark's launch shape, every site against
    the oracle."""
    dims = synth.WORKLOADS[2]["dims"]
    note(f"wilson_apply sampled {dims}")
    lat = ovl.Lattice(dims)
    U = synth.workload_gauge(2)
    G = ovl.Gauge(lat, dev(U))
    psi = synth.workload_sources(2)[0]
    inp = ovl.Spinor.from_canonical(lat, dev(psi), 0)
    out = ovl.Spinor(lat, 0)
    ovl.wilson_apply(lat, G, M0, inp, out)
    got = out.to_canonical().cpu().numpy()[0]
    olat = oracle.Lattice(dims)
    ref = oracle.dw(olat, U, M0, psi)
    ratio, r2 = check(0, got, ref, psi, dims)
    note(f"  worst site / bound {ratio:.3g}, rel L2 {r2:.3g}")


# time-streaming form: lattices whose spatial volume is a multiple of 256
STREAM_CASES = [((4, 4, 8, 8), 1), ((4, 4, 8, 8), 2), ((4, 4, 8, 8), 4), ((6, 4, 8, 8), 3),
                ((8, 8, 8, 4), 8), ((16, 8, 8, 8), 4), ((2, 8, 4, 8), 2)]


@pytest.mark.parametrize("dims,ts", STREAM_CASES)
@pytest.mark.parametrize("prec", [0, 1, 2])
def test_wilson_stream_matches_oracle(ovl, dims, ts, prec):
    note(f"wilson_apply streaming prec={prec} dims={dims} stream_t={ts}")
    lat, olat, U, G = setup(ovl, dims, seed=17)
    lat.stream_t = ts
    psi = synth.gaussian_spinor(lat.V, 18, 2)
    inp = ovl.Spinor.from_canonical(lat, dev(psi), prec)
    out = ovl.Spinor(lat, prec, 2)
    ovl.wilson_apply(lat, G, M0, inp, out)
    got = out.to_canonical().cpu().numpy()
    for r in range(2):
        check(prec, got[r], oracle.dw(olat, U, M0, psi[r]), psi[r], dims)


@pytest.mark.parametrize("bc", [(1, 1, 1, 1), (-1, -1, 1, -1)])
@pytest.mark.parametrize("ts", [1, 2, 4])
def test_stream_boundary_phases_and_q2(ovl, bc, ts):
    dims = (4, 4, 8, 8)
    note(f"streaming boundary phases bc={bc} stream_t={ts}")
    lat, olat, U, G = setup(ovl, dims, seed=19, bc=bc, n_stout=1)
    lat.stream_t = ts
    psi = synth.gaussian_spinor(lat.V, 20)[0]
    inp = ovl.Spinor.from_canonical(lat, dev(psi), 0)
    out = ovl.Spinor(lat, 0)
    ovl.wilson_apply(lat, G, M0, inp, out)
    check(0, out.to_canonical().cpu().numpy()[0], oracle.dw(olat, U, M0, psi), psi, dims)
    ovl.q_apply(lat, G, M0, inp, out)
    check(0, out.to_canonical().cpu().numpy()[0], oracle.q(olat, U, M0, psi), psi, dims)
    ovl.q2_apply(lat, G, M0, 0.37, inp, out)
    check(0, out.to_canonical().cpu().numpy()[0], oracle.q2(olat, U, M0, psi, 0.37), psi, dims, shift=0.37)


@pytest.mark.parametrize("cfg,ts", [(1, 4), (2, 8), (2, 16)])
def test_wilson_stream_full_workloads(ovl, cfg, ts):
    """Every site of the 16^3x32 and 32^3x64 fields in the streaming form, all
    three precisions against the oracle."""
    dims = synth.WORKLOADS[cfg]["dims"]
    note(f"wilson_apply streaming full {dims} stream_t={ts}")
    lat = ovl.Lattice(dims)
    lat.stream_t = ts
    olat = oracle.Lattice(dims)
    U = synth.workload_gauge(cfg)
    G = ovl.Gauge(lat, dev(U))
    psi = synth.workload_sources(cfg)[0]
    ref = oracle.dw(olat, U, M0, psi)
    for prec in (0, 1, 2):
        inp = ovl.Spinor.from_canonical(lat, dev(psi), prec)
        out = ovl.Spinor(lat, prec)
        ovl.wilson_apply(lat, G, M0, inp, out)
        check(prec, out.to_canonical().cpu().numpy()[0], ref, psi, dims)


@pytest.mark.parametrize("dims,ts,ts64", [((4, 4, 8, 8), 2, 4), ((8, 8, 8, 4), 4, 8), ((16, 8, 8, 8), 8, 16)])
def test_stream_t64_selects_fp64_length(ovl, dims, ts, ts64):
    """FP64 follows stream_t64 and FP32 stream_t when both are set."""
    note(f"stream_t64 dims={dims} stream_t={ts} stream_t64={ts64}")
    lat, olat, U, G = setup(ovl, dims, seed=27, n_stout=1)
    lat.stream_t = ts
    lat.stream_t64 = ts64
    psi = synth.gaussian_spinor(lat.V, 28)[0]
    ref = oracle.dw(olat, U, M0, psi)
    for prec in (0, 1):
        inp = ovl.Spinor.from_canonical(lat, dev(psi), prec)
        out = ovl.Spinor(lat, prec)
        ovl.wilson_apply(lat, G, M0, inp, out)
        check(prec, out.to_canonical().cpu().numpy()[0], ref, psi, dims)


@pytest.mark.parametrize("dims,nrhs", [((8, 8, 8, 4), 1), ((16, 8, 8, 8), 3)])
def test_autotune_keeps_results(ovl, dims, nrhs):
    """The autotuner only reorders summation: after it, the stencil still
    matches the oracle in every precision, and its choices are valid."""
    note(f"autotune dims={dims} nrhs={nrhs}")
    lat, olat, U, G = setup(ovl, dims, seed=29, n_stout=1)
    res = ovl.autotune_stencil(lat, G, nrhs)
    assert len(res["timings"]) > 3 and all(t > 0 for _, _, _, t in res["timings"])
    assert dims[0] % lat.tile_t == 0
    assert lat.rhs_tile in (1, 2, 4, 8) and (nrhs > 1 or lat.rhs_tile == 1)
    assert lat.mfma in (0, 1) and (nrhs > 1 or lat.mfma == 0)
    assert lat.stream_t == 0 or dims[0] % lat.stream_t == 0
    assert lat.stream_t64 == 0 or dims[0] % lat.stream_t64 == 0
    psi = synth.gaussian_spinor(lat.V, 30, nrhs)
    for prec in (0, 1, 2):
        inp = ovl.Spinor.from_canonical(lat, dev(psi), prec)
        out = ovl.Spinor(lat, prec, nrhs)
        ovl.wilson_apply(lat, G, M0, inp, out)
        got = out.to_canonical().cpu().numpy()
        for r in range(nrhs):
            check(prec, got[r], oracle.dw(olat, U, M0, psi[r]), psi[r], dims)


def test_autotune_cache_round_trip(ovl, tmp_path):
    """The cached autotuner times once, writes its choice as a JSON line and
    returns it unchanged on the next call for the same lattice and RHS count
    without timing; another RHS count is tuned anew."""
    dims = (16, 8, 8, 8)
    note("autotune cache")
    lat, olat, U, G = setup(ovl, dims, seed=33, n_stout=1)
    cache = str(tmp_path / "tune.json")
    first = ovl.autotune_stencil(lat, G, 3, cache=cache)
    assert first["timings"] != "cache" and len(first["timings"]) > 3
    lat2 = ovl.Lattice(dims)
    again = ovl.autotune_stencil(lat2, G, 3, cache=cache)
    assert again["timings"] == "cache"
    for k in ("tile_t", "stream_t", "stream_t64", "rhs_tile", "mfma"):
        assert again[k] == first[k]
    other = ovl.autotune_stencil(ovl.Lattice(dims), G, 1, cache=cache)
    assert other["timings"] != "cache"
    assert len(open(cache).read().splitlines()) == 2


# LDS-staged streaming form: blocks of whole x3 rows of consecutive x2 at one
# x1 (256 % L3 == 0, L2*L3 % 256 == 0) and launches of at most 512 blocks
# the last three have x3 extents (24, 48) whose rows tile 192-site blocks, not 256
STAGED_CASES = [((4, 2, 16, 16), 2), ((4, 4, 8, 32), 4), ((6, 2, 32, 8), 3), ((8, 2, 16, 16), 8), ((4, 4, 16, 16), 1),
                ((4, 8, 24, 24), 2), ((4, 4, 48, 48), 2), ((8, 4, 24, 24), 4)]


@pytest.mark.parametrize("dims,ts", STAGED_CASES)
@pytest.mark.parametrize("bc", [(-1, 1, 1, 1), (1, -1, -1, -1)])
def test_staged_stream_matches_oracle(ovl, dims, ts, bc):
    note(f"staged streaming dims={dims} stream={ts} bc={bc}")
    lat, olat, U, G = setup(ovl, dims, seed=31, n_stout=1, bc=bc)
    lat.stream_t = ts
    lat.stream_t64 = ts
    psi = synth.gaussian_spinor(lat.V, 32, 2)
    for prec in (0, 1):
        inp = ovl.Spinor.from_canonical(lat, dev(psi), prec)
        out = ovl.Spinor(lat, prec, 2)
        ovl.wilson_apply(lat, G, M0, inp, out)
        got = out.to_canonical().cpu().numpy()
        for r in range(2):
            check(prec, got[r], oracle.dw(olat, U, M0, psi[r]), psi[r], dims)
        ovl.q2_apply(lat, G, M0, 0.29, inp, out)
        got = out.to_canonical().cpu().numpy()
        for r in range(2):
            check(prec, got[r], oracle.q2(olat, U, M0, psi[r], 0.29), psi[r], dims, shift=0.29)


# RHS tiles of the streaming form: K lanes per site hold K RHS (one link load
# serves them); tiles need whole x3 rows per block and at least 256
# site-slices per block, else the launcher halves K.  nrhs not a multiple of K
# leaves idle lanes in the last tile.
TILE_CASES = [((8, 2, 16, 16), 8, 2, 3), ((8, 2, 16, 16), 8, 4, 5), ((8, 2, 16, 16), 8, 8, 12),
              ((8, 4, 24, 24), 4, 2, 3), ((8, 4, 24, 24), 8, 4, 6), ((16, 4, 24, 24), 16, 8, 9),
              ((4, 4, 16, 16), 4, 4, 4)]


@pytest.mark.parametrize("dims,ts,tile,nrhs", TILE_CASES)
def test_rhs_tiles_match_oracle(ovl, dims, ts, tile, nrhs):
    note(f"rhs tiles dims={dims} stream={ts} tile={tile} nrhs={nrhs}")
    lat, olat, U, G = setup(ovl, dims, seed=41, n_stout=1, bc=(-1, 1, -1, 1))
    lat.stream_t = ts
    lat.stream_t64 = ts
    lat.rhs_tile = tile
    psi = synth.gaussian_spinor(lat.V, 42, nrhs)
    for prec in (0, 1):
        inp = ovl.Spinor.from_canonical(lat, dev(psi), prec)
        out = ovl.Spinor(lat, prec, nrhs)
        ovl.wilson_apply(lat, G, M0, inp, out)
        got = out.to_canonical().cpu().numpy()
        for r in range(nrhs):
            check(prec, got[r], oracle.dw(olat, U, M0, psi[r]), psi[r], dims)
        ovl.q2_apply(lat, G, M0, 0.23, inp, out)
        got = out.to_canonical().cpu().numpy()
        for r in range(nrhs):
            check(prec, got[r], oracle.q2(olat, U, M0, psi[r], 0.23), psi[r], dims, shift=0.23)


# The matrix-core FP32 stencil (lat.mfma): two sites and four RHS per wave,
# used for FP32 D_W and Gamma_5 D_W on two or more RHS; a ragged last RHS tile
# (nrhs not a multiple of 4) and both boundary-phase patterns.  FP64, FP16S and
# single-RHS applies keep the vector form.
MFMA_CASES = [((4, 4, 4, 4), 2, (-1, 1, 1, 1)), ((6, 4, 2, 4), 3, (1, -1, -1, -1)),
              ((8, 4, 4, 6), 5, (-1, 1, -1, 1)), ((4, 6, 6, 8), 8, (-1, 1, 1, 1)),
              ((8, 4, 24, 24), 12, (-1, 1, 1, 1))]


@pytest.mark.parametrize("dims,nrhs,bc", MFMA_CASES)
def test_mfma_stencil_matches_oracle(ovl, dims, nrhs, bc):
    note(f"mfma stencil dims={dims} nrhs={nrhs} bc={bc}")
    lat, olat, U, G = setup(ovl, dims, seed=43, n_stout=1, bc=bc)
    lat.mfma = 1
    psi = synth.gaussian_spinor(lat.V, 44, nrhs)
    inp = ovl.Spinor.from_canonical(lat, dev(psi), 1)
    out = ovl.Spinor(lat, 1, nrhs)
    ovl.wilson_apply(lat, G, M0, inp, out)
    got = out.to_canonical().cpu().numpy()
    for r in range(nrhs):
        check(1, got[r], oracle.dw(olat, U, M0, psi[r]), psi[r], dims)
    ovl.q_apply(lat, G, M0, inp, out)
    got = out.to_canonical().cpu().numpy()
    for r in range(nrhs):
        check(1, got[r], oracle.q(olat, U, M0, psi[r]), psi[r], dims)
    ovl.q2_apply(lat, G, M0, 0.31, inp, out)
    got = out.to_canonical().cpu().numpy()
    for r in range(nrhs):
        check(1, got[r], oracle.q2(olat, U, M0, psi[r], 0.31), psi[r], dims, shift=0.31)
    # the vector form on the same input agrees to FP32 rounding
    lat.mfma = 0
    ref = ovl.Spinor(lat, 1, nrhs)
    ovl.wilson_apply(lat, G, M0, inp, ref)
    lat.mfma = 1
    ovl.wilson_apply(lat, G, M0, inp, out)
    a, b = out.to_canonical().cpu().numpy(), ref.to_canonical().cpu().numpy()
    assert np.abs(a - b).max() <= 1e-5 * np.abs(b).max()


@pytest.mark.parametrize("prec,nrhs", [(0, 3), (2, 3), (1, 1)])
def test_mfma_flag_other_forms(ovl, prec, nrhs):
    """With lat.mfma set, FP64, FP16S and single-RHS applies still run the
    vector stencil and match the oracle."""
    dims = (6, 4, 2, 4)
    note(f"mfma flag prec={prec} nrhs={nrhs}")
    lat, olat, U, G = setup(ovl, dims, seed=45)
    lat.mfma = 1
    psi = synth.gaussian_spinor(lat.V, 46, nrhs)
    inp = ovl.Spinor.from_canonical(lat, dev(psi), prec)
    out = ovl.Spinor(lat, prec, nrhs)
    ovl.wilson_apply(lat, G, M0, inp, out)
    got = out.to_canonical().cpu().numpy()
    for r in range(nrhs):
        check(prec, got[r], oracle.dw(olat, U, M0, psi[r]), psi[r], dims)
