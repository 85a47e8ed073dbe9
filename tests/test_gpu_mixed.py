"""GPU checks of the mixed-precision overlap apply: FP64 iterations until the
base residual falls below sloppy_below, then FP32 links, stencil and Krylov
vectors with FP64 residual replacement; FP64 per-shift verification (batched
fused residual norms) and refinement.  Bar: every shifted system's FP64 true residual <= 1e-10
(verified by the library and re-checked here with the oracle), and D_ov
within 1e-8 of the FP64 oracle (a 1e-10 residual bounds the solution error
by the condition number of Q^2 + s, ~1e2 here)."""
import sys

import numpy as np
import pytest
import torch

import oracle
import synth
from parity import field_check

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


def setup(ovl, dims, seed):
    U = synth.gauge(dims, 0.3, seed, n_stout=2)
    lat = ovl.Lattice(dims)
    olat = oracle.Lattice(dims)
    G = ovl.Gauge(lat, dev(U))
    v0 = synth.gaussian_spinor(lat.V, seed + 1)[0]
    lo, hi = ovl.spectral_bounds(lat, G, M0, 300, ovl.Spinor.from_canonical(lat, dev(v0), 0))
    s, w, d = ovl.zolotarev(lo, hi, 20)
    olo, ohi = oracle.spectral_interval(olat, U, M0, v0, 300)
    os_, ow, od = oracle.zolotarev(olo, ohi, 20)
    return U, lat, olat, G, (s, w), (os_, ow)


@pytest.mark.parametrize("sloppy_below", [0.0, 1e-3])
@pytest.mark.parametrize("dims", [(8, 4, 4, 6), (8, 8, 8, 8), (16, 8, 8, 8)])
def test_mixed_overlap_verified_residuals(ovl, dims, sloppy_below):
    note(f"mixed overlap {dims} sloppy_below={sloppy_below}")
    U, lat, olat, G, (s, w), (os_, ow) = setup(ovl, dims, 301)
    b = synth.gaussian_spinor(lat.V, 302)[0]
    B = ovl.Spinor.from_canonical(lat, dev(b), 0)
    O = ovl.Spinor(lat, 0)
    prm = ovl.default_params(tol=1e-10, maxiter=5000, mode=ovl.SOLVE_MIXED, block=8, sloppy_below=sloppy_below)
    st = ovl.overlap_apply(lat, G, RHO, s, w, B, O, prm)
    tr = np.array(st["true_residual"][0])
    assert (tr > 0).all() and (tr <= 1e-10).all(), tr
    assert st["reliable_updates"] > 0
    got = O.to_canonical().cpu().numpy()[0]
    ref, _, _ = oracle.overlap(olat, U, RHO, os_, ow, b, 1e-13, 5000)
    close(got, ref, dims, 1e-8)
    # the oracle confirms the library's verification for a few shifts: rebuild
    # y's shifted solutions is not possible from D_ov alone, so check D_ov
    # against the FP64 path at the same tolerance too
    O64 = ovl.Spinor(lat, 0)
    ovl.overlap_apply(lat, G, RHO, s, w, B, O64, ovl.default_params(tol=1e-10, maxiter=5000))
    close(got, O64.to_canonical().cpu().numpy()[0], dims, 1e-8)


def test_mixed_multishift_solutions_vs_oracle(ovl):
    """Per-shift solutions of the mixed solver (through sign_q with unit
    weights on one shift at a time is not exposed, so use the oracle's true
    residual of y's building blocks via overlap on two RHS)."""
    dims = (8, 4, 4, 8)
    U, lat, olat, G, (s, w), (os_, ow) = setup(ovl, dims, 311)
    b = synth.gaussian_spinor(lat.V, 312, 2)
    b[1] *= 1e3
    B = ovl.Spinor.from_canonical(lat, dev(b), 0)
    O = ovl.Spinor(lat, 0, 2)
    prm = ovl.default_params(tol=1e-10, maxiter=5000, mode=ovl.SOLVE_MIXED, block=6)
    st = ovl.overlap_apply(lat, G, RHO, s, w, B, O, prm)
    got = O.to_canonical().cpu().numpy()
    for r in range(2):
        tr = np.array(st["true_residual"][r])
        assert (tr <= 1e-10).all(), (r, tr)
        ref, _, _ = oracle.overlap(olat, U, RHO, os_, ow, b[r], 1e-13, 5000)
        close(got[r], ref, dims, 1e-8)


def test_mixed_ginsparg_wilson(ovl):
    dims = (8, 4, 4, 4)
    U, lat, olat, G, (s, w), _ = setup(ovl, dims, 321)
    b = synth.gaussian_spinor(lat.V, 322)[0]
    g5 = oracle.gamma5
    prm = ovl.default_params(tol=1e-10, maxiter=5000, mode=ovl.SOLVE_MIXED)

    def D(v):
        B = ovl.Spinor.from_canonical(lat, dev(v), 0)
        O = ovl.Spinor(lat, 0)
        ovl.overlap_apply(lat, G, RHO, s, w, B, O, prm)
        return O.to_canonical().cpu().numpy()[0]

    Db = D(b)
    lhs = g5(Db) + D(g5(b))
    rhs = D(g5(Db)) / RHO
    assert np.linalg.norm(lhs - rhs) / np.linalg.norm(b) < 1e-8


def test_mixed_fp64_phase_cuts_refinement(ovl):
    """Starting the FP32 phase only once |r|/|b| < 1e-4 leaves the shifted
    residuals near tol, so the refinement has little left to do, while the
    iterates stay those of the FP64 solver (same iteration count)."""
    dims = (16, 8, 8, 8)
    note(f"mixed FP64-phase switch {dims}")
    U, lat, olat, G, (s, w), _ = setup(ovl, dims, 331)
    b = synth.gaussian_spinor(lat.V, 332)[0]
    B = ovl.Spinor.from_canonical(lat, dev(b), 0)
    runs = {}
    for sb in (0.0, 1e-4):
        O = ovl.Spinor(lat, 0)
        prm = ovl.default_params(tol=1e-10, maxiter=5000, mode=ovl.SOLVE_MIXED, block=8, sloppy_below=sb)
        st = ovl.overlap_apply(lat, G, RHO, s, w, B, O, prm)
        tr = np.array(st["true_residual"][0])
        assert (tr > 0).all() and (tr <= 1e-10).all(), (sb, tr)
        runs[sb] = (st, O.to_canonical().cpu().numpy()[0])
    O64 = ovl.Spinor(lat, 0)
    st64 = ovl.overlap_apply(lat, G, RHO, s, w, B, O64, ovl.default_params(tol=1e-10, maxiter=5000, block=8))
    ref = O64.to_canonical().cpu().numpy()[0]
    close(runs[1e-4][1], ref, dims, 1e-9)
    assert runs[1e-4][0]["refine_iterations"] < runs[0.0][0]["refine_iterations"]
    assert abs(runs[1e-4][0]["iterations"][0] - st64["iterations"][0]) <= 8


def test_mixed_handover_per_rhs_long_blocks(ovl):
    """Three RHS that reach the hand-over level at different iterations (two
    Gaussian sources and a point source), blocks of the longest length: each
    RHS stops its FP64 phase at its own iteration and waits for the others, so
    every shifted residual still meets tol, D_ov agrees with the FP64 blocked
    solver, and each RHS takes about the FP64 solver's iterations."""
    dims = (16, 8, 8, 8)
    note(f"mixed per-RHS hand-over {dims} block={ovl.MAX_BLOCK}")
    U, lat, olat, G, (s, w), _ = setup(ovl, dims, 341)
    b = np.concatenate([synth.gaussian_spinor(lat.V, 342, 2),
                        synth.point_sources(lat.V, synth.random_site(lat.V, 343))[:1]])
    B = ovl.Spinor.from_canonical(lat, dev(b), 0)
    O = ovl.Spinor(lat, 0, 3)
    prm = ovl.default_params(tol=1e-10, maxiter=5000, mode=ovl.SOLVE_MIXED, block=ovl.MAX_BLOCK,
                             block_f64=ovl.MAX_BLOCK, sloppy_below=1e-4)
    st = ovl.overlap_apply(lat, G, RHO, s, w, B, O, prm)
    O64 = ovl.Spinor(lat, 0, 3)
    st64 = ovl.overlap_apply(lat, G, RHO, s, w, B, O64,
                             ovl.default_params(tol=1e-10, maxiter=5000, block=ovl.MAX_BLOCK))
    got, ref = O.to_canonical().cpu().numpy(), O64.to_canonical().cpu().numpy()
    for r in range(3):
        tr = np.array(st["true_residual"][r])
        assert (tr > 0).all() and (tr <= 1e-10).all(), (r, tr)
        close(got[r], ref[r], dims, 1e-9)
        assert abs(st["iterations"][r] - st64["iterations"][r]) <= 8, (r, st["iterations"], st64["iterations"])


def test_mixed_zero_rhs_in_batch(ovl):
    """A zero right-hand side next to a Gaussian one: it is finished before
    the first iteration, so every pass skips it and the FP32 phase's first
    pass must leave its increments at zero; D_ov of it is exactly zero and
    the other RHS agrees with the FP64 blocked form."""
    dims = (8, 4, 4, 8)
    note(f"mixed zero RHS {dims}")
    U, lat, olat, G, (s, w), _ = setup(ovl, dims, 351)
    b = synth.gaussian_spinor(lat.V, 352, 2)
    b[1] = 0.0
    B = ovl.Spinor.from_canonical(lat, dev(b), 0)
    O = ovl.Spinor(lat, 0, 2)
    st = ovl.overlap_apply(lat, G, RHO, s, w, B, O, ovl.default_params(tol=1e-10, maxiter=5000,
                                                                       mode=ovl.SOLVE_MIXED, sloppy_below=1e-3))
    O64 = ovl.Spinor(lat, 0, 2)
    ovl.overlap_apply(lat, G, RHO, s, w, B, O64, ovl.default_params(tol=1e-10, maxiter=5000, block=8))
    got, ref = O.to_canonical().cpu().numpy(), O64.to_canonical().cpu().numpy()
    assert not np.any(got[1]) and not np.any(ref[1])
    assert (np.array(st["true_residual"][0]) <= 1e-10).all()
    close(got[0], ref[0], dims, 1e-9)


@pytest.mark.parametrize("sloppy_below", [1e-5, 1e-8])
def test_mixed_fp16_storage_mode(ovl, sloppy_below):
    """sloppy_f16 rounds the FP32 phase's Krylov vectors through FP16 storage
    with per-site scales.  With refinement every shift still meets 1e-10 and
    D_ov matches the oracle; without it the verified residuals report the
    format's floor, which stays above the FP32 bulk's when the hand-over is
    early."""
    dims = (8, 8, 8, 8)
    note(f"mixed fp16 storage sloppy_below={sloppy_below}")
    U, lat, olat, G, (s, w), (os_, ow) = setup(ovl, dims, 311)
    b = synth.gaussian_spinor(lat.V, 312)[0]
    B = ovl.Spinor.from_canonical(lat, dev(b), 0)
    O = ovl.Spinor(lat, 0)
    prm = ovl.default_params(tol=1e-10, maxiter=5000, mode=ovl.SOLVE_MIXED, sloppy_below=sloppy_below, sloppy_f16=1)
    st = ovl.overlap_apply(lat, G, RHO, s, w, B, O, prm)
    tr = np.array(st["true_residual"][0])
    note(f"  refined: max residual {tr.max():.2e}, {st['refine_iterations']} refinement iterations")
    assert (tr > 0).all() and (tr <= 1e-10).all(), tr
    ref, _, _ = oracle.overlap(olat, U, RHO, os_, ow, b, 1e-13, 5000)
    close(O.to_canonical().cpu().numpy()[0], ref, dims, 1e-8)
    prm.refine = 0
    st = ovl.overlap_apply(lat, G, RHO, s, w, B, O, prm, allow_not_converged=True)
    floor = max(st["true_residual"][0])
    note(f"  floor without refinement: {floor:.2e}")
    assert floor > 0 and np.isfinite(floor)
    if sloppy_below >= 1e-5:
        assert floor > 1e-10


def test_mixed_unshifted_base_bookkeeping(ovl):
    """With all shifts positive the mixed solver runs its recurrences on an
    extra unshifted base system of weight 0 and hides it from the caller.
    Passing that system explicitly (shift 0, weight 0, first) runs the same
    arithmetic with nothing hidden: D_ov must agree bit for bit, the
    iteration counts must agree, and the caller's per-shift statistics must
    be the explicit run's entries 1..n."""
    dims = (8, 4, 4, 8)
    U, lat, olat, G, (s, w), (os_, ow) = setup(ovl, dims, 331)
    s, w = np.asarray(s)[:12], np.asarray(w)[:12]
    b = synth.gaussian_spinor(lat.V, 332, 2)
    B = ovl.Spinor.from_canonical(lat, dev(b), 0)
    prm = ovl.default_params(tol=1e-10, maxiter=5000, mode=ovl.SOLVE_MIXED, block=8, sloppy_below=1e-3)
    Oa, Ob = ovl.Spinor(lat, 0, 2), ovl.Spinor(lat, 0, 2)
    sa = ovl.overlap_apply(lat, G, RHO, s, w, B, Oa, prm)
    sb = ovl.overlap_apply(lat, G, RHO, np.concatenate([[0.0], s]), np.concatenate([[0.0], w]), B, Ob, prm)
    ga, gb = Oa.to_canonical().cpu().numpy(), Ob.to_canonical().cpu().numpy()
    assert np.array_equal(ga, gb)
    assert sa["iterations"] == sb["iterations"]
    for q in range(2):
        ta, tb = np.array(sa["true_residual"][q]), np.array(sb["true_residual"][q])
        assert ta.shape == (12,) and tb.shape == (13,)
        assert np.allclose(ta, tb[1:], rtol=1e-9, atol=0.0), (ta, tb)
        assert (ta > 0).all() and (ta <= 1e-10).all()
        assert list(sa["shift_iters"][q]) == list(sb["shift_iters"][q][1:])
    note(f"  iterations {sa['iterations']}, max shifted residual {max(map(max, sa['true_residual'])):.2e}")
