"""GPU checks of low-mode deflation (Section 5.2): ovl_low_modes against the
dense eigendecomposition on 4^4 and against the oracle stencil on larger
lattices, and sign/overlap applies with the modes deflated against the dense
exact sign and against the oracle's undeflated overlap, in every solver mode.
All comparisons are element-wise (tests/parity.py field_check)."""
import sys

import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import deflation, dense
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


@pytest.fixture(scope="module")
def w44(ovl):
    """4^4 workload field on the GPU, its 16 GPU low modes and the dense
    reference modes."""
    dims = (4, 4, 4, 4)
    lat, olat = ovl.Lattice(dims), oracle.Lattice(dims)
    U = synth.workload_gauge(0)
    G = ovl.Gauge(lat, dev(U))
    start = ovl.Spinor.from_canonical(lat, dev(synth.gaussian_spinor(lat.V, 301)), 0)
    note("low modes 4^4, nev 16")
    D = ovl.low_modes(lat, G, M0, start, nev=16, tol=1e-10)
    lam, xi, wsorted = deflation.low_modes_dense(olat, U, M0, 17)
    return dict(dims=dims, lat=lat, olat=olat, U=U, G=G, D=D, lam=lam, xi=xi, wsorted=wsorted)


def test_low_modes_match_dense_eigenpairs(ovl, w44):
    D, lam, xi = w44["D"], w44["lam"], w44["xi"]
    st = D.stats
    note(f"  {st['steps']} Lanczos steps in {st['stages']} stages, {st['q2_applies']} Q^2 applies, "
         f"max residual {st['max_residual']:.2e}, next |lambda| {st['lambda_next']:.6f}, cut {st['theta_cut']:.4f}")
    assert st["converged"] == 1 and st["max_residual"] <= 1e-10
    assert np.abs(D.evals - lam[:16]).max() < 1e-10
    assert abs(lam[15]) <= st["lambda_next"] < abs(lam[16]) + 0.05
    got = D.evecs.to_canonical().cpu().numpy()
    G = np.array([[np.vdot(a, b) for b in got] for a in got])
    assert np.abs(G - np.eye(16)).max() < 1e-10
    for i in range(16):
        # the GPU eigenvector up to a phase: its component outside the dense
        # eigenvector's span, and its residual with the oracle's Q
        c = np.vdot(xi[i], got[i])
        assert np.linalg.norm(got[i] - c * xi[i]) < 1e-8
        r = np.linalg.norm(oracle.q(w44["olat"], w44["U"], M0, got[i]) - D.evals[i] * got[i])
        assert r < 2e-10 and abs(D.residuals[i] - r) < 1e-11


@pytest.mark.parametrize("mode", ["f64", "blocked", "mixed", "lanczos"])
def test_deflated_apply_vs_dense_exact(ovl, w44, mode):
    """sign(Q) b and D_ov b with the 16 GPU modes deflated and 10 Zolotarev
    poles on [|lambda_17|, lambda_max] only: within the rational bound of that
    interval of the exact dense results."""
    lat, dims = w44["lat"], w44["dims"]
    ws = w44["wsorted"]
    lo, hi = abs(w44["D"].evals[-1]), 1.001 * abs(ws[-1])
    s, wt, delta = ovl.zolotarev(lo, hi, 10)
    kw = dict(tol=1e-12, maxiter=4000, deflation=w44["D"])
    if mode == "blocked":
        kw["block"] = 8
    elif mode == "mixed":
        kw.update(mode=ovl.SOLVE_MIXED, tol=1e-11)
    elif mode == "lanczos":
        kw.update(mode=ovl.SOLVE_LANCZOS)
    prm = ovl.default_params(**kw)
    b = np.concatenate([synth.gaussian_spinor(lat.V, 302, 2), np.zeros((1, lat.V, 4, 3), complex)])
    B = ovl.Spinor.from_canonical(lat, dev(b), 0)
    O = ovl.Spinor(lat, 0, 3)
    S, _ = dense.sign_q_exact(w44["olat"], w44["U"], M0)
    Dov = RHO * (np.eye(3072) + dense.gamma5_matrix(lat.V) @ S)
    # the remainder's error is delta (Zolotarev mode) or the Lanczos tolerance,
    # plus the eigenvector error; 10x delta of head room
    tol = max(10 * delta, 1e-9)
    ovl.sign_q_apply(lat, w44["G"], M0, s, wt, B, O, prm)
    got = O.to_canonical().cpu().numpy()
    assert not np.any(got[2])
    for r in range(2):
        ratio, r2 = field_check(got[r], (S @ b[r].reshape(-1)).reshape(b[r].shape), dims, tol)
        note(f"  {mode} sign rhs {r}: worst/bound {ratio:.3g}, L2 {r2:.2e} (delta {delta:.1e})")
        assert ratio <= 1.0
    ovl.overlap_apply(lat, w44["G"], RHO, s, wt, B, O, prm)
    got = O.to_canonical().cpu().numpy()
    assert not np.any(got[2])
    for r in range(2):
        ratio, r2 = field_check(got[r], (Dov @ b[r].reshape(-1)).reshape(b[r].shape), dims, tol)
        assert ratio <= 1.0


def test_deflation_changes_nothing_but_the_interval(ovl, w44):
    """Undeflated with the same 10 poles, the low modes fall outside the
    Zolotarev interval and the error is far above the deflated one."""
    lat, dims = w44["lat"], w44["dims"]
    ws = w44["wsorted"]
    lo, hi = abs(w44["D"].evals[-1]), 1.001 * abs(ws[-1])
    s, wt, delta = ovl.zolotarev(lo, hi, 10)
    b = synth.gaussian_spinor(lat.V, 303)
    B = ovl.Spinor.from_canonical(lat, dev(b), 0)
    O = ovl.Spinor(lat, 0)
    S, _ = dense.sign_q_exact(w44["olat"], w44["U"], M0)
    exact = (S @ b[0].reshape(-1)).reshape(b[0].shape)
    errs = []
    for defl in (w44["D"], None):
        prm = ovl.default_params(tol=1e-12, maxiter=4000, deflation=defl)
        ovl.sign_q_apply(lat, w44["G"], M0, s, wt, B, O, prm)
        got = O.to_canonical().cpu().numpy()[0]
        errs.append(np.linalg.norm(got - exact) / np.linalg.norm(exact))
    note(f"  deflated {errs[0]:.2e}, undeflated {errs[1]:.2e}")
    assert errs[0] < 10 * delta and errs[1] > 100 * errs[0]


@pytest.mark.parametrize("dims,nev", [((8, 4, 4, 8), 12), ((8, 8, 8, 8), 20)])
def test_deflated_overlap_vs_oracle(ovl, dims, nev):
    """Larger lattices: the GPU modes are eigenpairs of the oracle's Q, and the
    deflated mixed and FP64 D_ov (poles on the deflated interval) match the
    oracle's undeflated D_ov (20 poles on the full interval) element-wise."""
    note(f"deflated overlap {dims} nev {nev}")
    lat, olat = ovl.Lattice(dims), oracle.Lattice(dims)
    U = synth.gauge(dims, 0.3, 311, n_stout=2)
    G = ovl.Gauge(lat, dev(U))
    start = ovl.Spinor.from_canonical(lat, dev(synth.gaussian_spinor(lat.V, 312)), 0)
    D = ovl.low_modes(lat, G, M0, start, nev=nev, tol=1e-10)
    note(f"  {D.stats['steps']} steps, {D.stats['q2_applies']} Q^2 applies, max residual {D.stats['max_residual']:.2e}, "
         f"|lambda| {abs(D.evals[0]):.4f}..{abs(D.evals[-1]):.4f}, next {D.stats['lambda_next']:.4f}")
    vecs = D.evecs.to_canonical().cpu().numpy()
    for i in (0, nev // 2, nev - 1):
        assert np.linalg.norm(oracle.q(olat, U, M0, vecs[i]) - D.evals[i] * vecs[i]) < 2e-10
    v0 = synth.gaussian_spinor(lat.V, 313)[0]
    olo, ohi = oracle.spectral_interval(olat, U, M0, v0, 300)
    assert abs(D.evals[0]) >= olo
    os_, ow, _ = oracle.zolotarev(olo, ohi, 20)
    b = synth.gaussian_spinor(lat.V, 314, 2)
    refs = [oracle.overlap(olat, U, RHO, os_, ow, b[r], 1e-13, 5000)[0] for r in range(2)]
    s, wt, delta = ovl.zolotarev(abs(D.evals[-1]), ohi, 14)
    B = ovl.Spinor.from_canonical(lat, dev(b), 0)
    O = ovl.Spinor(lat, 0, 2)
    for mode in (ovl.SOLVE_F64, ovl.SOLVE_MIXED):
        prm = ovl.default_params(tol=1e-12, maxiter=4000, mode=mode, deflation=D)
        st = ovl.overlap_apply(lat, G, RHO, s, wt, B, O, prm)
        got = O.to_canonical().cpu().numpy()
        for r in range(2):
            ratio, r2 = field_check(got[r], refs[r], dims, 1e-9)
            note(f"  mode {mode} rhs {r}: {st['iterations'][r]} iterations, worst/bound {ratio:.3g}, L2 {r2:.2e}")
            assert ratio <= 1.0


def test_low_modes_rejects_bad_arguments(ovl, w44):
    lat = w44["lat"]
    start = ovl.Spinor(lat, 0)
    with pytest.raises(ovl.OvlError):
        ovl.low_modes(lat, w44["G"], M0, start, nev=16, steps=16)      # steps below nev + extra
    with pytest.raises(ovl.OvlError):
        ovl.low_modes(lat, w44["G"], M0, start, nev=0)
    # an all-zero start vector is rejected
    start.data.zero_()
    with pytest.raises(ovl.OvlError):
        ovl.low_modes(lat, w44["G"], M0, start, nev=4)


def test_outer_solve_with_deflated_inner_applies(ovl, w44):
    """The outer FGMRES with its D_ov applications deflated (16 modes, poles on
    the deflated interval) reaches the same solution as without deflation."""
    lat, dims = w44["lat"], w44["dims"]
    ws = w44["wsorted"]
    eta = synth.gaussian_spinor(lat.V, 321)
    E = ovl.Spinor.from_canonical(lat, dev(eta), 0)
    sols = []
    for defl in (w44["D"], None):
        lo = abs(w44["D"].evals[-1]) if defl is not None else 0.999 * abs(ws[0])
        s, wt, _ = ovl.zolotarev(lo, 1.001 * abs(ws[-1]), 16)
        P = ovl.Spinor(lat, 0)
        prm = ovl.default_outer_params(tol=1e-9, inner=dict(deflation=defl) if defl is not None else {})
        st = ovl.overlap_solve(lat, w44["G"], RHO, s, wt, E, P, prm)
        note(f"  deflated={defl is not None}: {st['iterations']} steps, {st['mscg_iterations']} multishift "
             f"iterations, residual {st['residual']:.2e}")
        assert st["residual"] <= 1e-9
        sols.append(P.to_canonical().cpu().numpy()[0])
    ratio, r2 = field_check(sols[0], sols[1], dims, 1e-7)
    assert ratio <= 1.0
