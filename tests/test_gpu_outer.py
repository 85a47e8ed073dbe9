"""GPU checks of the outer solver for D_ov psi = eta (eq. (linsys)) and of the
Wilson solve behind its preconditioner, through the C ABI, against the FP64
oracle.

* ovl_wilson_solve: the returned true residual |b - D_W x|/|b| is recomputed
  with the oracle's D_W, and x is compared site by site with the oracle's
  GMRES solution.
* ovl_overlap_solve (FGMRES with relaxed D_ov applications): the GPU solution
  psi satisfies |eta - D_ov psi| <= tol |eta| with the oracle's D_ov (Zolotarev
  + multishift CG at a 1e-13 tolerance), agrees site by site with the oracle's
  GMRES solution to the condition number times tol, and the same holds with
  the paper's Wilson preconditioner D_W(m0^prec) at the default mass of
  eq. (default_m), which must cut the number of D_ov applications.
"""
import sys

import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import dense, krylov
from parity import field_check, rel_l2

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


@pytest.mark.parametrize("m0", [-0.6, 0.3])
def test_wilson_solve_matches_oracle(ovl, m0):
    dims = (8, 4, 4, 8)
    note(f"wilson solve m0={m0}")
    lat, olat = ovl.Lattice(dims), oracle.Lattice(dims)
    U = synth.gauge(dims, 0.3, 91, n_stout=2)
    G = ovl.Gauge(lat, dev(U))
    b = synth.gaussian_spinor(lat.V, 92, 2)
    B = ovl.Spinor.from_canonical(lat, dev(b), 0)
    X = ovl.Spinor(lat, 0, 2)
    st = ovl.wilson_solve(lat, G, m0, B, X, ovl.default_params(tol=1e-11, maxiter=3000))
    x = X.to_canonical().cpu().numpy()
    for r in range(2):
        res = np.linalg.norm(b[r] - oracle.dw(olat, U, m0, x[r])) / np.linalg.norm(b[r])
        assert abs(res - st["true_residual"][r]) <= 1e-3 * res + 1e-14, (res, st["true_residual"][r])
        assert res < 1e-9, res
        ref, it, ores = krylov.gmres(lambda v: oracle.dw(olat, U, m0, v), b[r], 1e-12, restart=100)
        ratio, r2 = field_check(x[r], ref, dims, 1e-8)
        note(f"  rhs {r}: {st['iterations'][r]} CG iterations, residual {res:.2e}, worst/bound {ratio:.3g}")
        assert ratio <= 1.0


@pytest.mark.parametrize("m0", [-0.6, 0.3, -1.2])
def test_wilson_solve_even_odd_matches_oracle(ovl, m0):
    """The even-odd form (Schur complement on the even sites, FP32 CGLS in
    FP64 defect correction): x against the oracle's GMRES solution site by
    site, the returned true residual against the oracle's D_W, and fewer
    Krylov iterations than the normal-equations CG on the full lattice."""
    dims = (8, 4, 4, 8)
    note(f"wilson solve even-odd m0={m0}")
    lat, olat = ovl.Lattice(dims), oracle.Lattice(dims)
    U = synth.gauge(dims, 0.3, 91, n_stout=2)
    G = ovl.Gauge(lat, dev(U))
    b = synth.gaussian_spinor(lat.V, 92, 2)
    B = ovl.Spinor.from_canonical(lat, dev(b), 0)
    X = ovl.Spinor(lat, 0, 2)
    st = ovl.wilson_solve(lat, G, m0, B, X, ovl.default_params(tol=1e-11, maxiter=3000, even_odd=1))
    full = ovl.wilson_solve(lat, G, m0, B, ovl.Spinor(lat, 0, 2), ovl.default_params(tol=1e-11, maxiter=3000))
    x = X.to_canonical().cpu().numpy()
    for r in range(2):
        res = np.linalg.norm(b[r] - oracle.dw(olat, U, m0, x[r])) / np.linalg.norm(b[r])
        assert abs(res - st["true_residual"][r]) <= 1e-3 * res + 1e-14, (res, st["true_residual"][r])
        assert res <= 1e-11, res
        ref, it, ores = krylov.gmres(lambda v: oracle.dw(olat, U, m0, v), b[r], 1e-13, restart=100)
        ratio, r2 = field_check(x[r], ref, dims, 1e-8)
        note(f"  rhs {r}: {st['iterations'][r]} CGLS iterations (normal equations on the full lattice: "
             f"{full['iterations'][r]}), residual {res:.2e}, worst/bound {ratio:.3g}")
        assert ratio <= 1.0
        assert st["iterations"][r] < full["iterations"][r]


@pytest.mark.parametrize("dims", [(6, 4, 4, 6), (2, 2, 4, 2)])
def test_wilson_solve_even_odd_ragged_and_tiny(ovl, dims):
    """Lattices whose half volume is not a multiple of the 256-thread blocks
    (288 sites per parity), and the smallest one (extent 2, where the forward
    and backward neighbour coincide): x against the oracle's GMRES solution."""
    note(f"wilson solve even-odd {dims}")
    lat, olat = ovl.Lattice(dims), oracle.Lattice(dims)
    U = synth.gauge(dims, 0.3, 96, n_stout=1)
    G = ovl.Gauge(lat, dev(U))
    b = synth.gaussian_spinor(lat.V, 97)
    B = ovl.Spinor.from_canonical(lat, dev(b), 0)
    X = ovl.Spinor(lat, 0)
    st = ovl.wilson_solve(lat, G, -0.7, B, X, ovl.default_params(tol=1e-11, maxiter=3000, even_odd=1))
    x = X.to_canonical().cpu().numpy()[0]
    res = np.linalg.norm(b[0] - oracle.dw(olat, U, -0.7, x)) / np.linalg.norm(b[0])
    ref, it, _ = krylov.gmres(lambda v: oracle.dw(olat, U, -0.7, v), b[0], 1e-13, restart=100)
    ratio, r2 = field_check(x, ref, dims, 1e-8)
    note(f"  {st['iterations'][0]} iterations, residual {res:.2e}, worst/bound {ratio:.3g}")
    assert res <= 1e-11 and abs(res - st["true_residual"][0]) <= 1e-3 * res + 1e-15 and ratio <= 1.0


def test_wilson_solve_even_odd_edge_cases(ovl):
    """A zero RHS returns x = 0 with no iterations; a loose tolerance (the
    preconditioner's 1e-1) stops after one defect-correction step with the
    true residual below it; a capped run reports OVL_NOT_CONVERGED with its
    iterations at the cap; m0 = -4 (no diagonal to divide by) is rejected; a
    NaN in the source returns OVL_ERR_NONFINITE."""
    dims = (4, 4, 4, 8)
    lat, olat = ovl.Lattice(dims), oracle.Lattice(dims)
    U = synth.gauge(dims, 0.3, 94, n_stout=1)
    G = ovl.Gauge(lat, dev(U))
    b = np.concatenate([synth.gaussian_spinor(lat.V, 95, 1), np.zeros((1, lat.V, 4, 3), complex)])
    B = ovl.Spinor.from_canonical(lat, dev(b), 0)
    X = ovl.Spinor(lat, 0, 2)
    st = ovl.wilson_solve(lat, G, -0.8, B, X, ovl.default_params(tol=1e-1, even_odd=1))
    x = X.to_canonical().cpu().numpy()
    assert st["iterations"][1] == 0 and st["true_residual"][1] == 0.0 and not np.any(x[1])
    res = np.linalg.norm(b[0] - oracle.dw(olat, U, -0.8, x[0])) / np.linalg.norm(b[0])
    note(f"  tol 1e-1: {st['iterations'][0]} iterations, residual {res:.3e}")
    assert 0 < res <= 1e-1 and abs(res - st["true_residual"][0]) <= 1e-6 * res
    st = ovl.wilson_solve(lat, G, -0.8, B, X, ovl.default_params(tol=1e-12, maxiter=5, even_odd=1),
                          allow_not_converged=True)
    assert st["iterations"][0] == 5 and st["true_residual"][0] > 1e-12
    with pytest.raises(ovl.OvlError):
        ovl.wilson_solve(lat, G, -4.0, B, X, ovl.default_params(even_odd=1))
    # a NaN in the source is reported, not iterated on
    bn = b.copy()
    bn[0, 5, 2, 1] = np.nan
    with pytest.raises(ovl.OvlError) as e:
        ovl.wilson_solve(lat, G, -0.8, ovl.Spinor.from_canonical(lat, dev(bn), 0), X,
                         ovl.default_params(even_odd=1))
    assert e.value.status == ovl.ERR_NONFINITE


@pytest.mark.parametrize("dims,m0", [((32, 16, 16, 16), -0.5), ((64, 32, 32, 32), -0.5)])
def test_wilson_solve_even_odd_workload_sizes(ovl, dims, m0):
    """At the workload sizes the oracle's D_W checks the true residual of the
    even-odd solve (a property that holds at any size)."""
    note(f"wilson solve even-odd {dims} m0={m0}")
    lat, olat = ovl.Lattice(dims), oracle.Lattice(dims)
    U = synth.gauge(dims, 0.3, 97, n_stout=1) if dims[0] <= 32 else synth.workload_gauge(2)
    G = ovl.Gauge(lat, dev(U))
    b = synth.gaussian_spinor(lat.V, 98)
    B = ovl.Spinor.from_canonical(lat, dev(b), 0)
    X = ovl.Spinor(lat, 0)
    st = ovl.wilson_solve(lat, G, m0, B, X, ovl.default_params(tol=1e-10, maxiter=5000, even_odd=1))
    x = X.to_canonical().cpu().numpy()[0]
    res = np.linalg.norm(b[0] - oracle.dw(olat, U, m0, x)) / np.linalg.norm(b[0])
    note(f"  {st['iterations'][0]} CGLS iterations, {st['seconds']:.3f} s, oracle residual {res:.2e}")
    assert res <= 1e-10 and abs(res - st["true_residual"][0]) <= 1e-3 * res


def sigma_min_4x4(U):
    """Smallest real part of the eigenvalues of D_W(0) on 4^4 (dense)."""
    D = dense.dense_dw(oracle.Lattice((4, 4, 4, 4)), U, 0.0)
    return float(np.linalg.eigvals(D).real.min())


@pytest.mark.parametrize("n_stout", [0, 2])
def test_overlap_solve_4x4_with_and_without_wilson_preconditioner(ovl, n_stout):
    dims = (4, 4, 4, 4)
    note(f"overlap solve 4^4 n_stout={n_stout}")
    lat, olat = ovl.Lattice(dims), oracle.Lattice(dims)
    U = synth.gauge(dims, 0.5, synth.SEED_BASE, n_stout=n_stout)
    G = ovl.Gauge(lat, dev(U))
    S, w = dense.sign_q_exact(olat, U, M0)
    aw = np.abs(w)
    s, wt, delta = ovl.zolotarev(0.99 * aw.min(), 1.01 * aw.max(), 20)
    Dov = RHO * (np.eye(3072) + dense.gamma5_matrix(lat.V) @ S)
    cond = np.linalg.cond(Dov)
    eta = synth.gaussian_spinor(lat.V, 93)[0]
    exact = np.linalg.solve(Dov, eta.reshape(-1)).reshape(eta.shape)
    E = ovl.Spinor.from_canonical(lat, dev(eta), 0)
    tol = 1e-8
    # the paper's default preconditioner mass (eq. (default_m)) in the
    # normalisation rho (I + Gamma_5 sign(Q)) = rho D_N with m0^ovl = -rho:
    # omega = -m0^ovl - sigma_min, m0^prec = omega * 1 + m0^ovl = -sigma_min
    sig = sigma_min_4x4(U)
    m0_prec = (-M0 - sig) + M0
    runs = {}
    for prec, eo in ((0, 1), (1, 0), (1, 1)):
        Psi = ovl.Spinor(lat, 0)
        prm = ovl.default_outer_params(tol=tol, precondition=prec, prec_m0=m0_prec, prec_even_odd=eo)
        st = ovl.overlap_solve(lat, G, RHO, s, wt, E, Psi, prm)
        psi = Psi.to_canonical().cpu().numpy()[0]
        ores = np.linalg.norm(eta - oracle.overlap(olat, U, RHO, s, wt, psi, 1e-13, 5000)[0]) / np.linalg.norm(eta)
        err = rel_l2(psi, exact)
        note(f"  precondition={prec} even_odd={eo}: {st['iterations']} steps, {st['restarts']} restarts, {st['mscg_iterations']} "
             f"MSCG iterations, {st['prec_iterations']} preconditioner iterations, residual {st['residual']:.2e} "
             f"(oracle {ores:.2e}), error {err:.2e}, cond {cond:.1f}")
        assert st["residual"] <= tol and ores <= 2 * tol, (st, ores)
        assert err <= cond * (2 * tol + 10 * delta), err
        runs[(prec, eo)] = st
    assert runs[(1, 0)]["iterations"] < runs[(0, 1)]["iterations"], runs
    assert runs[(1, 1)]["iterations"] < runs[(0, 1)]["iterations"], runs


def test_overlap_solve_matches_oracle_gmres_and_relaxation_saves_work(ovl):
    dims = (8, 4, 4, 8)
    note("overlap solve 8x4x4x8 vs oracle GMRES, relaxed and fixed sign tolerance")
    lat, olat = ovl.Lattice(dims), oracle.Lattice(dims)
    U = synth.gauge(dims, 0.3, 95, n_stout=2)
    G = ovl.Gauge(lat, dev(U))
    v0 = synth.gaussian_spinor(lat.V, 96)[0]
    lo, hi = ovl.spectral_bounds(lat, G, M0, 300, ovl.Spinor.from_canonical(lat, dev(v0), 0))
    s, wt, delta = ovl.zolotarev(lo, hi, 20)
    eta = synth.gaussian_spinor(lat.V, 97)[0]
    E = ovl.Spinor.from_canonical(lat, dev(eta), 0)
    tol = 1e-8
    olo, ohi = oracle.spectral_interval(olat, U, M0, v0, 300)
    os_, ow, _ = oracle.zolotarev(olo, ohi, 20)
    D = lambda v: oracle.overlap(olat, U, RHO, os_, ow, v, 1e-13, 5000)[0]
    ref, oit, ores = krylov.gmres(D, eta, 1e-11, restart=100)
    stats = {}
    for relax in (1, 0):
        for mode in (ovl.SOLVE_MIXED, ovl.SOLVE_F64):
            Psi = ovl.Spinor(lat, 0)
            prm = ovl.default_outer_params(tol=tol, relax=relax, inner=dict(mode=mode))
            st = ovl.overlap_solve(lat, G, RHO, s, wt, E, Psi, prm)
            psi = Psi.to_canonical().cpu().numpy()[0]
            res = np.linalg.norm(eta - D(psi)) / np.linalg.norm(eta)
            ratio, r2 = field_check(psi, ref, dims, 1e-6)
            note(f"  relax={relax} mode={mode}: {st['iterations']} steps, {st['mscg_iterations']} MSCG iterations, "
                 f"oracle residual {res:.2e}, worst/bound {ratio:.3g}, L2 {r2:.2e} (oracle GMRES {oit} steps)")
            assert res <= 2 * tol and ratio <= 1.0
            stats[(relax, mode)] = st
    # relaxation: about the same number of steps, fewer multishift iterations
    for mode in (ovl.SOLVE_MIXED, ovl.SOLVE_F64):
        assert abs(stats[(1, mode)]["iterations"] - stats[(0, mode)]["iterations"]) <= 3
        assert stats[(1, mode)]["mscg_iterations"] < stats[(0, mode)]["mscg_iterations"]


def test_overlap_solve_zero_rhs_and_not_converged(ovl):
    dims = (4, 4, 4, 4)
    lat = ovl.Lattice(dims)
    G = ovl.Gauge(lat, dev(synth.workload_gauge(0)))
    s, w, _ = ovl.zolotarev(0.4, 6.0, 12)
    Z = ovl.Spinor.from_canonical(lat, dev(np.zeros((lat.V, 4, 3), dtype=complex)), 0)
    Psi = ovl.Spinor(lat, 0)
    st = ovl.overlap_solve(lat, G, RHO, s, w, Z, Psi)
    assert st["iterations"] == 0 and not np.any(Psi.to_canonical().cpu().numpy())
    E = ovl.Spinor.from_canonical(lat, dev(synth.gaussian_spinor(lat.V, 98)[0]), 0)
    st = ovl.overlap_solve(lat, G, RHO, s, w, E, Psi, ovl.default_outer_params(tol=1e-12, maxiter=3),
                           allow_not_converged=True)
    assert st["iterations"] == 3 and st["residual"] > 1e-12
    with pytest.raises(ovl.OvlError) as e:
        ovl.overlap_solve(lat, G, RHO, s, w, E, Psi, ovl.default_outer_params(tol=1e-12, maxiter=3))
    assert e.value.status == ovl.NOT_CONVERGED
