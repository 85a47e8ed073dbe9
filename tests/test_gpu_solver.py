"""GPU parity of the sign function and the overlap apply (FP64 path) against
the oracle, through the C ABI: Lanczos bounds, multishift CG, sign_q_apply,
overlap_apply, plus the solver's failure paths.

Each side builds its own Zolotarev coefficients (the library from theta
functions, the oracle from the Landen scheme) and its own Lanczos bounds; the
FP64 path must agree with the oracle to 1e-12 relative.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
import synth
from parity import field_check
from oracle import dense

pytestmark = pytest.mark.gpu

RHO = 1.6
M0 = -RHO


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


def close(got, ref, dims, tol):
    """Site-wise check of a solver output against its reference
    (tests/parity.py field_check); returns the worst site's error over its
    bound and the relative L2 difference."""
    ratio, r2 = field_check(got, ref, dims, tol)
    assert ratio <= 1.0, (ratio, r2)
    return ratio, r2


def both_sides(ovl, dims, U, npoles=20, start_seed=99):
    """Each side's own spectral interval and Zolotarev data."""
    lat = ovl.Lattice(dims)
    olat = oracle.Lattice(dims)
    G = ovl.Gauge(lat, dev(U))
    v0 = synth.gaussian_spinor(lat.V, start_seed)[0]
    lo, hi = ovl.spectral_bounds(lat, G, M0, 300, ovl.Spinor.from_canonical(lat, dev(v0), 0))
    s, w, d = ovl.zolotarev(lo, hi, npoles)
    olo, ohi = oracle.spectral_interval(olat, U, M0, v0, 300)
    os_, ow, od = oracle.zolotarev(olo, ohi, npoles)
    return lat, olat, G, (s, w, d, lo, hi), (os_, ow, od, olo, ohi)


def test_spectral_bounds_bracket_exact_spectrum(ovl):
    dims = (4, 4, 4, 4)
    note("spectral bounds 4^4")
    U = synth.workload_gauge(0)
    lat = ovl.Lattice(dims)
    G = ovl.Gauge(lat, dev(U))
    v0 = synth.gaussian_spinor(lat.V, 5)[0]
    lo, hi = ovl.spectral_bounds(lat, G, M0, 300, ovl.Spinor.from_canonical(lat, dev(v0), 0), 1.0, 1.0)
    _, w = dense.sign_q_exact(oracle.Lattice(dims), U, M0)
    aw = np.abs(w)
    assert abs(lo - aw.min()) < 1e-6 * aw.min() and abs(hi - aw.max()) < 1e-9 * aw.max()
    lo2, hi2 = ovl.spectral_bounds(lat, G, M0, 300, ovl.Spinor.from_canonical(lat, dev(v0), 0))
    assert lo2 < aw.min() and hi2 > aw.max()


@pytest.mark.parametrize("block", [0, 1, 5, 8, 16, 32])
def test_multishift_cg_matches_oracle(ovl, block):
    """Per-shift solutions of the plain (block 0) and blocked shift updates
    against the oracle's multishift CG and its true residuals."""
    dims = (8, 4, 4, 6)
    note(f"multishift cg vs oracle block={block}")
    U = synth.gauge(dims, 0.3, 21, n_stout=1)
    lat, olat, G, (s, w, d, lo, hi), _ = both_sides(ovl, dims, U)
    b = synth.gaussian_spinor(lat.V, 22)[0]
    x_ref, it_ref, _ = oracle.mscg(olat, U, M0, s, b, 1e-12, 3000)
    B = ovl.Spinor.from_canonical(lat, dev(b), 0)
    X = ovl.Spinor(lat, 0, len(s))
    st = ovl.multishift_cg(lat, G, M0, s, None, B, X,
                           ovl.default_params(tol=1e-12, verify=1, check_every=7, block=block))
    x = X.to_canonical().cpu().numpy()
    for j in range(len(s)):
        close(x[j], x_ref[j], dims, 1e-10)
        assert abs(st["shift_iters"][0][j] - it_ref[j]) <= 1
        assert st["true_residual"][0][j] < 1e-11
    assert st["iterations"][0] == max(st["shift_iters"][0])


def test_sign_q_matches_exact_dense_sign(ovl):
    """4^4 workload: Zolotarev + multishift CG on the GPU against W sign(Delta) W^H."""
    dims = (4, 4, 4, 4)
    note("sign(Q) vs dense 4^4")
    U = synth.workload_gauge(0)
    lat = ovl.Lattice(dims)
    G = ovl.Gauge(lat, dev(U))
    S, w = dense.sign_q_exact(oracle.Lattice(dims), U, M0)
    aw = np.abs(w)
    s, wt, delta = ovl.zolotarev(0.99 * aw.min(), 1.01 * aw.max(), 20)
    b = synth.workload_sources(0)[0]
    B = ovl.Spinor.from_canonical(lat, dev(b), 0)
    O = ovl.Spinor(lat, 0)
    ovl.sign_q_apply(lat, G, M0, s, wt, B, O, ovl.default_params(tol=1e-13))
    exact = (S @ b.reshape(-1)).reshape(b.shape)
    close(O.to_canonical().cpu().numpy()[0], exact, dims, 1e-12 + 2 * delta)
    # overlap against the dense overlap matrix
    Dov = RHO * (np.eye(3072) + dense.gamma5_matrix(lat.V) @ S)
    ovl.overlap_apply(lat, G, RHO, s, wt, B, O, ovl.default_params(tol=1e-13))
    close(O.to_canonical().cpu().numpy()[0], (Dov @ b.reshape(-1)).reshape(b.shape), dims, 1e-12)


@pytest.mark.parametrize("block", [0, 8])
@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 4, 2, 4), (8, 4, 4, 6), (8, 8, 8, 8)])
def test_overlap_apply_matches_oracle(ovl, dims, block):
    note(f"overlap fp64 vs oracle {dims} block={block}")
    U = synth.gauge(dims, 0.3, 31, n_stout=2)
    lat, olat, G, (s, w, d, lo, hi), (os_, ow, od, olo, ohi) = both_sides(ovl, dims, U)
    # the smallest Ritz value is not fully converged after 300 steps, so two
    # implementations with different rounding agree on it only to a few
    # parts in 1e8 here; the bound leaves a factor of about 100
    assert abs(lo - olo) < 1e-6 * lo and abs(hi - ohi) < 1e-8 * hi
    b = synth.gaussian_spinor(lat.V, 32)[0]
    ref, _, _ = oracle.overlap(olat, U, RHO, os_, ow, b, 1e-13, 5000)
    B = ovl.Spinor.from_canonical(lat, dev(b), 0)
    O = ovl.Spinor(lat, 0)
    st = ovl.overlap_apply(lat, G, RHO, s, w, B, O, ovl.default_params(tol=1e-13, maxiter=5000, block=block))
    close(O.to_canonical().cpu().numpy()[0], ref, dims, 1e-12)
    assert st["iterations"][0] > 10


@pytest.mark.parametrize("block", [0, 6])
def test_overlap_multi_rhs(ovl, block):
    dims = (8, 4, 4, 4)
    note(f"overlap multi-rhs block={block}")
    U = synth.gauge(dims, 0.3, 41, n_stout=2)
    lat, olat, G, (s, w, d, lo, hi), (os_, ow, od, olo, ohi) = both_sides(ovl, dims, U)
    b = synth.gaussian_spinor(lat.V, 42, 3)
    b[2] *= 1e-3   # a RHS with a different scale converges on its own schedule
    B = ovl.Spinor.from_canonical(lat, dev(b), 0)
    O = ovl.Spinor(lat, 0, 3)
    st = ovl.overlap_apply(lat, G, RHO, s, w, B, O, ovl.default_params(tol=1e-13, maxiter=5000, block=block))
    got = O.to_canonical().cpu().numpy()
    for r in range(3):
        ref, _, _ = oracle.overlap(olat, U, RHO, os_, ow, b[r], 1e-13, 5000)
        close(got[r], ref, dims, 1e-12)


@pytest.mark.parametrize("block", [0, 16])
def test_point_sources_batch(ovl, block):
    """All 12 spin-colour point sources in one batched solve (the multi-RHS
    workload shape), each against the oracle at the FP64 path's 1e-12."""
    dims = (8, 4, 4, 4)
    note(f"point sources block={block}")
    U = synth.gauge(dims, 0.3, 51, n_stout=2)
    lat, olat, G, (s, w, d, lo, hi), (os_, ow, od, olo, ohi) = both_sides(ovl, dims, U)
    site = synth.random_site(lat.V, 52)
    b = synth.point_sources(lat.V, site)
    B = ovl.Spinor.from_canonical(lat, dev(b), 0)
    O = ovl.Spinor(lat, 0, 12)
    ovl.overlap_apply(lat, G, RHO, s, w, B, O, ovl.default_params(tol=1e-13, maxiter=5000, block=block))
    got = O.to_canonical().cpu().numpy()
    for r in range(12):
        ref, _, _ = oracle.overlap(olat, U, RHO, os_, ow, b[r], 1e-13, 5000)
        close(got[r], ref, dims, 1e-12)


def test_ginsparg_wilson_gpu(ovl):
    """Gamma_5 D + D Gamma_5 = (1/rho) D Gamma_5 D for the GPU overlap (eq. (GW))."""
    dims = (8, 4, 4, 4)
    note("GW relation")
    U = synth.gauge(dims, 0.3, 61, n_stout=2)
    lat, olat, G, (s, w, d, lo, hi), _ = both_sides(ovl, dims, U)
    b = synth.gaussian_spinor(lat.V, 62)[0]
    g5 = oracle.gamma5
    prm = ovl.default_params(tol=1e-13, maxiter=5000)

    def D(v):
        B = ovl.Spinor.from_canonical(lat, dev(v), 0)
        O = ovl.Spinor(lat, 0)
        ovl.overlap_apply(lat, G, RHO, s, w, B, O, prm)
        return O.to_canonical().cpu().numpy()[0]

    Db = D(b)
    lhs = g5(Db) + D(g5(b))
    rhs = D(g5(Db)) / RHO
    assert np.linalg.norm(lhs - rhs) / np.linalg.norm(b) < 1e-11


def test_not_converged_and_zero_rhs(ovl):
    dims = (4, 4, 4, 4)
    U = synth.workload_gauge(0)
    lat = ovl.Lattice(dims)
    G = ovl.Gauge(lat, dev(U))
    s, w, d = ovl.zolotarev(0.4, 6.0, 12)
    b = synth.gaussian_spinor(lat.V, 71)[0]
    B = ovl.Spinor.from_canonical(lat, dev(b), 0)
    O = ovl.Spinor(lat, 0)
    st = ovl.overlap_apply(lat, G, RHO, s, w, B, O, ovl.default_params(tol=1e-12, maxiter=5),
                           allow_not_converged=True)
    assert st["iterations"][0] == 5
    with pytest.raises(ovl.OvlError) as e:
        ovl.overlap_apply(lat, G, RHO, s, w, B, O, ovl.default_params(tol=1e-12, maxiter=5))
    assert e.value.status == ovl.NOT_CONVERGED
    Z = ovl.Spinor.from_canonical(lat, dev(np.zeros_like(b)), 0)
    st = ovl.overlap_apply(lat, G, RHO, s, w, Z, O, ovl.default_params())
    assert np.abs(O.to_canonical().cpu().numpy()).max() == 0.0
    assert st["iterations"][0] == 0


def test_nonfinite_input_reported(ovl):
    dims = (4, 4, 4, 4)
    U = synth.workload_gauge(0)
    lat = ovl.Lattice(dims)
    G = ovl.Gauge(lat, dev(U))
    s, w, d = ovl.zolotarev(0.4, 6.0, 8)
    b = synth.gaussian_spinor(lat.V, 72)[0]
    b[3, 1, 2] = np.nan
    B = ovl.Spinor.from_canonical(lat, dev(b), 0)
    O = ovl.Spinor(lat, 0)
    with pytest.raises(ovl.OvlError) as e:
        ovl.overlap_apply(lat, G, RHO, s, w, B, O, ovl.default_params())
    assert e.value.status == ovl.ERR_NONFINITE


@pytest.mark.parametrize("dims,block,ts,ts64", [((8, 8, 8, 8), 0, 2, 0), ((8, 8, 8, 8), 8, 4, 0),
                                               ((8, 8, 8, 8), 16, 8, 0), ((8, 8, 8, 8), 0, 2, 4),
                                               ((8, 8, 8, 8), 16, 4, 8), ((8, 4, 8, 32), 16, 4, 8),
                                               ((8, 2, 16, 16), 0, 2, 8), ((4, 4, 24, 24), 16, 2, 4)])
def test_solvers_with_streaming_stencil(ovl, dims, block, ts, ts64):
    """Multishift CG and the overlap apply with the time-streaming stencil: its
    partial sums (fewer blocks than slots) feed the same reductions.  The
    last three lattices take the LDS-staged form, the last one with blocks of
    192 sites (rows of 24)."""
    note(f"solvers with streaming stencil block={block} stream_t={ts} stream_t64={ts64}")
    U = synth.gauge(dims, 0.3, 61, n_stout=2)
    lat, olat, G, (s, w, d, lo, hi), (os_, ow, od, olo, ohi) = both_sides(ovl, dims, U)
    lat.stream_t = ts
    lat.stream_t64 = ts64
    b = synth.gaussian_spinor(lat.V, 62, 2)
    x_ref, it_ref, _ = oracle.mscg(olat, U, M0, s, b[0], 1e-12, 3000)
    B = ovl.Spinor.from_canonical(lat, dev(b[:1]), 0)
    X = ovl.Spinor(lat, 0, len(s))
    st = ovl.multishift_cg(lat, G, M0, s, None, B, X, ovl.default_params(tol=1e-12, verify=1, block=block))
    x = X.to_canonical().cpu().numpy()
    for j in range(len(s)):
        close(x[j], x_ref[j], dims, 1e-10)
        assert abs(st["shift_iters"][0][j] - it_ref[j]) <= 1
    B2 = ovl.Spinor.from_canonical(lat, dev(b), 0)
    O = ovl.Spinor(lat, 0, 2)
    ovl.overlap_apply(lat, G, RHO, s, w, B2, O, ovl.default_params(tol=1e-13, maxiter=5000, block=block))
    got = O.to_canonical().cpu().numpy()
    for r in range(2):
        ref, _, _ = oracle.overlap(olat, U, RHO, os_, ow, b[r], 1e-13, 5000)
        close(got[r], ref, dims, 1e-12)
    # mixed form on the streaming stencil: every shift verified at 1e-10
    O3 = ovl.Spinor(lat, 0, 2)
    st3 = ovl.overlap_apply(lat, G, RHO, s, w, B2, O3, ovl.default_params(tol=1e-10, maxiter=5000,
                                                                          mode=ovl.SOLVE_MIXED, block=block))
    for r in range(2):
        assert max(st3["true_residual"][r][:len(s)]) <= 1e-10
        close(O3.to_canonical().cpu().numpy()[r], got[r], dims, 1e-8)


@pytest.mark.parametrize("dims,ts,tile,block", [((8, 2, 16, 16), 8, 4, 8), ((8, 4, 24, 24), 8, 4, 16),
                                                ((8, 2, 16, 16), 8, 8, 0)])
def test_solvers_with_rhs_tiles(ovl, dims, ts, tile, block):
    """Multishift CG and the overlap apply on a lattice whose streaming stencil
    runs RHS tiles: five RHS (two Gaussian, one scaled by 1e-3, a point source
    and a zero field) finish at different iterations, so tiles hold lanes of
    finished RHS, which must store nothing and add no norms."""
    note(f"solvers with rhs tiles dims={dims} stream={ts} tile={tile} block={block}")
    U = synth.gauge(dims, 0.3, 71, n_stout=2)
    lat, olat, G, (s, w, d, lo, hi), (os_, ow, od, olo, ohi) = both_sides(ovl, dims, U)
    lat.stream_t = ts
    lat.stream_t64 = ts
    lat.rhs_tile = tile
    V = lat.V
    b = np.concatenate([synth.gaussian_spinor(V, 72, 3), synth.point_sources(V, synth.random_site(V, 73))[:1],
                        np.zeros((1, V, 4, 3), dtype=complex)])
    b[1] *= 1e-3
    B = ovl.Spinor.from_canonical(lat, dev(b), 0)
    O = ovl.Spinor(lat, 0, 5)
    st = ovl.overlap_apply(lat, G, RHO, s, w, B, O, ovl.default_params(tol=1e-13, maxiter=5000, block=block))
    got = O.to_canonical().cpu().numpy()
    assert st["iterations"][4] == 0 and not np.any(got[4])
    for r in range(4):
        ref, _, _ = oracle.overlap(olat, U, RHO, os_, ow, b[r], 1e-13, 5000)
        close(got[r], ref, dims, 1e-12)
    O2 = ovl.Spinor(lat, 0, 5)
    st2 = ovl.overlap_apply(lat, G, RHO, s, w, B, O2, ovl.default_params(tol=1e-10, maxiter=5000,
                                                                        mode=ovl.SOLVE_MIXED))
    got2 = O2.to_canonical().cpu().numpy()
    assert not np.any(got2[4])
    for r in range(4):
        assert max(st2["true_residual"][r][:len(s)]) <= 1e-10, r
        close(got2[r], got[r], dims, 1e-8)


@pytest.mark.parametrize("mode", ["fp64", "fp64_blocked", "mixed"])
def test_rhs_groups_match_whole_batch(ovl, mode):
    """rhs_group = 2 on five RHS (groups of 2, 2, 1 in one workspace sized for
    one group).  The FP64 forms treat every RHS independently, so the groups
    give the whole batch's D_ov bit for bit and the same iteration counts; the
    mixed form replaces the base residuals of a batch together and verifies
    shifts batch-wise, so there the results agree to the solver tolerance and
    every shifted residual meets it in both runs."""
    dims = (8, 4, 4, 8)
    note(f"rhs groups {mode}")
    U = synth.gauge(dims, 0.3, 81, n_stout=2)
    lat, olat, G, (s, w, d, lo, hi), _ = both_sides(ovl, dims, U)
    b = synth.gaussian_spinor(lat.V, 82, 5)
    b[3] = synth.point_sources(lat.V, synth.random_site(lat.V, 83))[4]
    B = ovl.Spinor.from_canonical(lat, dev(b), 0)
    kw = dict(tol=1e-10, maxiter=5000)
    if mode == "fp64_blocked":
        kw["block"] = 8
    if mode == "mixed":
        kw["mode"] = ovl.SOLVE_MIXED
    p_all = ovl.default_params(**kw)
    p_grp = ovl.default_params(rhs_group=2, **kw)
    assert ovl.workspace_bytes(lat, ovl.OP_MSCG, ovl.F64, 5, len(s), p_grp) < \
        ovl.workspace_bytes(lat, ovl.OP_MSCG, ovl.F64, 5, len(s), p_all)
    O1, O2 = ovl.Spinor(lat, 0, 5), ovl.Spinor(lat, 0, 5)
    st1 = ovl.overlap_apply(lat, G, RHO, s, w, B, O1, p_all)
    st2 = ovl.overlap_apply(lat, G, RHO, s, w, B, O2, p_grp)
    g1, g2 = O1.to_canonical().cpu().numpy(), O2.to_canonical().cpu().numpy()
    if mode == "mixed":
        for r in range(5):
            assert max(st1["true_residual"][r][:len(s)]) <= 1e-10 and max(st2["true_residual"][r][:len(s)]) <= 1e-10
            close(g2[r], g1[r], dims, 1e-8)
    else:
        assert np.array_equal(g1, g2)
        assert st1["iterations"] == st2["iterations"] and st1["shift_iters"] == st2["shift_iters"]


@pytest.mark.parametrize("mode", ["fp64", "fp64_blocked", "mixed"])
def test_profile_stats_are_consistent(ovl, mode):
    """profile = 1 times the solver's kernels with HIP events: one stencil
    span per stencil launched in the iterations, one scalar span each for
    alpha and beta, block passes (or the plain form's shift updates) as update
    spans, every class timed; profile = 2 times the same stencil launches and
    nothing else; the result equals the unprofiled one bit for bit."""
    dims = (8, 4, 4, 8)
    note(f"profile stats {mode} {dims}")
    U = synth.gauge(dims, 0.3, 41, n_stout=2)
    lat, olat, G, (s, w, d, lo, hi), _ = both_sides(ovl, dims, U)
    b = synth.gaussian_spinor(lat.V, 42)[0]
    B = ovl.Spinor.from_canonical(lat, dev(b), 0)
    kw = dict(tol=1e-10, maxiter=5000, block=0 if mode == "fp64" else 8)
    if mode == "mixed":
        kw["mode"] = ovl.SOLVE_MIXED
    out = {}
    for prof in (0, 1, 2):
        O = ovl.Spinor(lat, 0)
        st = ovl.overlap_apply(lat, G, RHO, s, w, B, O, ovl.default_params(profile=prof, **kw))
        out[prof] = (O.to_canonical().cpu().numpy(), st)
    assert np.array_equal(out[0][0], out[1][0]) and np.array_equal(out[0][0], out[2][0])
    st = out[1][1]
    launches, secs = st["kernel_launches"], st["kernel_seconds"]
    assert launches[0] > 0 and launches[0] % 2 == 0
    assert launches[2] == launches[0]                 # alpha and beta per pair of stencils
    assert launches[1] >= 1                          # block passes
    assert all(t > 0 for t in secs[:3])
    if mode != "mixed":
        # every stencil but the overlap's final D_W (no residual replacements)
        assert launches[0] == st["stencil_applies"] - 1
    assert out[0][1]["kernel_launches"] == [0, 0, 0, 0]
    light = out[2][1]
    assert light["kernel_launches"] == [launches[0], 0, 0, 0]
    assert light["kernel_seconds"][0] > 0 and light["kernel_seconds"][1:] == [0.0, 0.0, 0.0]
