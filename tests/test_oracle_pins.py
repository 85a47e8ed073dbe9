"""Pins for the FP64 oracle: closed forms, identities and brute force that
fix what the oracle must compute, independent of the oracle's own formulas.

Each test names the paper passage (Brannick et al., arXiv:1410.7170) or the
mathematical fact it rests on.
"""
import numpy as np
import pytest

import oracle
import synth
from oracle import dense

RHO = 1.6
M0 = -RHO


def rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(np.asarray(b))


@pytest.fixture(scope="module")
def lat44():
    return oracle.Lattice((4, 4, 4, 4))


@pytest.fixture(scope="module")
def U44():
    # the dense-check workload: 4^4, links exp(i 0.5 H), no smearing
    return synth.workload_gauge(0)


@pytest.fixture(scope="module")
def dense44(lat44, U44):
    D = dense.dense_dw(lat44, U44, M0)
    G5 = dense.gamma5_matrix(lat44.V)
    Q = G5 @ D
    w, W = np.linalg.eigh(Q)
    S = (W * np.sign(w)) @ W.conj().T
    return dict(D=D, G5=G5, Q=Q, w=w, S=S)


# ---------------------------------------------------------------- T1
def test_gamma_algebra():
    """Clifford relation eq. (commutativity_rel); gamma_5 = g0 g1 g2 g3 is
    Hermitian, squares to I and anticommutes with every gamma_mu
    (eq. (gamma_commutativity))."""
    g = [oracle.gamma(m) for m in range(5)]
    I4 = np.eye(4)
    for m in range(4):
        assert np.allclose(g[m], g[m].conj().T, atol=0)
        for n in range(4):
            ac = g[m] @ g[n] + g[n] @ g[m]
            assert np.abs(ac - (2 * I4 if m == n else 0)).max() == 0
        assert np.abs(g[4] @ g[m] + g[m] @ g[4]).max() == 0
    assert np.abs(g[4] - g[0] @ g[1] @ g[2] @ g[3]).max() == 0
    assert np.abs(g[4] @ g[4] - I4).max() == 0
    assert np.abs(g[4] - g[4].conj().T).max() == 0


# ---------------------------------------------------------------- T2
def test_links_are_su3(U44):
    """Gauge links lie in SU(3) (Section 2, below eq. (Wilson-Dirac))."""
    u = U44.reshape(-1, 3, 3)
    assert np.abs(u @ u.conj().transpose(0, 2, 1) - np.eye(3)).max() < 1e-14
    assert np.abs(np.linalg.det(u) - 1).max() < 1e-14


# ---------------------------------------------------------------- T3
@pytest.mark.parametrize("dims", [(4, 4, 4, 4), (6, 4, 2, 4), (8, 4, 4, 6)])
def test_gamma5_hermiticity(dims):
    """(Gamma_5 D_W)^H = Gamma_5 D_W, eq. (gamma_5_symmetry)."""
    lat = oracle.Lattice(dims)
    U = synth.gauge(dims, 0.5, 11)
    phi, psi = synth.gaussian_spinor(lat.V, 12, 2)
    a = np.vdot(phi, oracle.q(lat, U, M0, psi))
    b = np.vdot(oracle.q(lat, U, M0, phi), psi)
    assert abs(a - b) / abs(a) < 1e-14


def test_dense_q_hermitian(dense44):
    Q = dense44["Q"]
    assert np.abs(Q - Q.conj().T).max() < 1e-15


# ---------------------------------------------------------------- T4
def _plane_wave(dims, n, chi):
    """psi(x) = exp(i p.x) chi with p0 = (2 n0 + 1) pi / L0 (antiperiodic
    time) and p_k = 2 pi n_k / L_k."""
    L = np.asarray(dims)
    p = np.array([(2 * n[0] + 1) * np.pi / L[0]] + [2 * np.pi * n[k] / L[k] for k in (1, 2, 3)])
    x = np.stack(np.meshgrid(*[np.arange(l) for l in L], indexing="ij"), -1).reshape(-1, 4)
    ph = np.exp(1j * (x @ p))
    return p, ph[:, None, None] * chi[None, :, :]


def _free_symbol(p, m0):
    """b(p) + i sum_mu sin(p_mu) gamma_mu as a 4x4 matrix."""
    b = m0 + np.sum(1 - np.cos(p))
    A = b * np.eye(4, dtype=complex)
    for mu in range(4):
        A = A + 1j * np.sin(p[mu]) * oracle.gamma(mu)
    return A


@pytest.mark.parametrize("n", [(0, 0, 0, 0), (1, 2, 0, 3), (3, 1, 1, 1), (7, 3, 2, 1)])
def test_free_field_plane_wave(n):
    """Unit links: D_W on a plane wave is multiplication by
    m0 + sum(1 - cos p) + i sum sin(p_mu) gamma_mu (from eq. (Wilson-Dirac);
    the 1/2 and the (I -+ gamma) projectors fix the cos and sin terms)."""
    dims = (8, 4, 4, 6)
    lat = oracle.Lattice(dims)
    U = synth.unit_gauge(dims)
    rng = np.random.default_rng(5)
    chi = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    p, psi = _plane_wave(dims, n, chi)
    A = _free_symbol(p, M0)
    expect = np.einsum("ab,xbc->xac", A, psi)
    assert rel(oracle.dw(lat, U, M0, psi), expect) < 1e-14


# ---------------------------------------------------------------- T5
def test_free_field_overlap_plane_wave():
    """Unit links: D_W is normal and Theorem 1 gives D_ov on a plane wave as
    rho (I + A(p)/|A(p)|), A(p) = b(p) + i sum sin(p) gamma, |A|^2 = b^2 + sum sin^2."""
    dims = (8, 4, 4, 4)
    lat = oracle.Lattice(dims)
    U = synth.unit_gauge(dims)
    # exact |Q| spectrum: omega(p) over every allowed momentum
    om = []
    for n0 in range(8):
        for n1 in range(4):
            for n2 in range(4):
                for n3 in range(4):
                    p = np.array([(2 * n0 + 1) * np.pi / 8, 2 * np.pi * n1 / 4, 2 * np.pi * n2 / 4,
                                  2 * np.pi * n3 / 4])
                    b = M0 + np.sum(1 - np.cos(p))
                    om.append(np.sqrt(b * b + np.sum(np.sin(p) ** 2)))
    s, w, delta = oracle.zolotarev(0.99 * min(om), 1.01 * max(om), 20)
    rng = np.random.default_rng(9)
    chi = rng.standard_normal((4, 3)) + 1j * rng.standard_normal((4, 3))
    for n in [(0, 0, 0, 0), (2, 1, 3, 0), (5, 2, 2, 1)]:
        p, psi = _plane_wave(dims, n, chi)
        A = _free_symbol(p, M0)
        om_p = np.sqrt(np.real(np.linalg.eigvals(A.conj().T @ A))[0])
        Dn = RHO * (np.eye(4) + A / om_p)
        expect = np.einsum("ab,xbc->xac", Dn, psi)
        out, iters, _ = oracle.overlap(lat, U, RHO, s, w, psi, 1e-13, 5000)
        assert rel(out, expect) < 1e-12 + 2 * delta


# ---------------------------------------------------------------- T6
def test_lemma1_spectral_symmetries():
    """Lemma 1(i): spec D_W is symmetric to the real axis and to the line
    Re z = m0 + 4; D_W(-4) has zero red-red and black-black blocks."""
    dims = (4, 2, 2, 4)
    lat = oracle.Lattice(dims)
    U = synth.gauge(dims, 0.5, 21)
    D = dense.dense_dw(lat, U, M0)
    ev = np.linalg.eigvals(D)
    for lam in (np.conj(ev), 2 * (M0 + 4) - ev):
        d = np.abs(ev[:, None] - lam[None, :]).min(axis=0)
        assert d.max() < 1e-10
    x = np.stack(np.meshgrid(*[np.arange(l) for l in dims], indexing="ij"), -1).reshape(-1, 4)
    par = np.repeat(x.sum(1) % 2, 12)
    D4 = dense.dense_dw(lat, U, -4.0)
    assert np.abs(D4[np.ix_(par == 0, par == 0)]).max() == 0
    assert np.abs(D4[np.ix_(par == 1, par == 1)]).max() == 0


# ---------------------------------------------------------------- T7
def test_prop2_non_normality(lat44, U44, dense44):
    """Prop. 2: ||D^H D - D D^H||_F^2 = 16 sum_x sum_{mu<nu} Re tr(I - P_x^{mu,nu}),
    independent of the mass.  Only holds with the 1/2 in the hopping term and
    the link orientation of eq. (Wilson-Dirac)."""
    D = dense44["D"]
    C = D.conj().T @ D - D @ D.conj().T
    lhs = np.sum(np.abs(C) ** 2)
    rhs = 16 * (3 * 6 * lat44.V - oracle.plaquette_sum(lat44, U44))
    assert abs(lhs - rhs) / rhs < 1e-12


def test_prop2_pure_gauge_is_normal():
    """Pure-gauge links U_mu(x) = g(x) g(x+mu)^H give a normal D_W (after Prop. 2)."""
    dims = (4, 4, 4, 4)
    lat = oracle.Lattice(dims)
    g = synth.gauge(dims, 0.7, 31)[:, 0]
    x = np.stack(np.meshgrid(*[np.arange(l) for l in dims], indexing="ij"), -1).reshape(-1, 4)
    U = np.empty((lat.V, 4, 3, 3), dtype=complex)
    for mu in range(4):
        y = x.copy()
        y[:, mu] = (y[:, mu] + 1) % dims[mu]
        n = ((y[:, 0] * 4 + y[:, 1]) * 4 + y[:, 2]) * 4 + y[:, 3]
        U[:, mu] = g @ g[n].conj().transpose(0, 2, 1)
    assert abs(oracle.plaquette_sum(lat, U) - 18 * lat.V) < 1e-10
    # ||(D^H D - D D^H) z|| for a random z vanishes
    z = synth.gaussian_spinor(lat.V, 32)[0]
    g5 = oracle.gamma5
    Dz = oracle.dw(lat, U, M0, z)
    a = g5(oracle.dw(lat, U, M0, g5(Dz)))
    b = oracle.dw(lat, U, M0, g5(oracle.dw(lat, U, M0, g5(z))))
    assert rel(a, b) < 1e-14 * 1e2 or np.linalg.norm(a - b) < 1e-12


# ---------------------------------------------------------------- T8
@pytest.mark.parametrize("dims,m0", [((4, 4, 4, 4), -1.6), ((6, 4, 4, 8), -1.6), ((4, 4, 4, 4), 0.3)])
def test_q2_diagonal(dims, m0):
    """<e, Q^2 e> = (m0+4)^2 + 4 for every point source e and any SU(3) field:
    the 8 hops each contribute |1/2 (I -+ gamma) u|^2 summed to 4 (the diagonal
    of D_W^H D_W in the appendix, with the hop paths included)."""
    lat = oracle.Lattice(dims)
    U = synth.gauge(dims, 0.5, 41)
    rng = np.random.default_rng(1)
    for _ in range(6):
        e = np.zeros((lat.V, 4, 3), dtype=complex)
        e[rng.integers(lat.V), rng.integers(4), rng.integers(3)] = 1
        val = np.vdot(e, oracle.q2(lat, U, m0, e))
        assert abs(val - ((m0 + 4) ** 2 + 4)) < 1e-13


# ---------------------------------------------------------------- T9
def test_prop2_stochastic():
    """E||(D^H D - D D^H) z||^2 = ||D^H D - D D^H||_F^2 for E[z z^H] = I; with
    Prop. 2 this checks the stencil at a size where no dense matrix exists."""
    dims = (8, 8, 8, 8)
    lat = oracle.Lattice(dims)
    U = synth.gauge(dims, 0.3, 51, n_stout=1)
    g5 = oracle.gamma5
    vals = []
    for z in synth.gaussian_spinor(lat.V, 52, 12):
        Dz = oracle.dw(lat, U, M0, z)
        a = g5(oracle.dw(lat, U, M0, g5(Dz)))
        b = oracle.dw(lat, U, M0, g5(oracle.dw(lat, U, M0, g5(z))))
        vals.append(np.sum(np.abs(a - b) ** 2))
    vals = np.array(vals)
    expect = 16 * (18 * lat.V - oracle.plaquette_sum(lat, U))
    assert abs(vals.mean() - expect) < 4 * vals.std(ddof=1) / np.sqrt(len(vals)) + 1e-9 * expect


# ---------------------------------------------------------------- T10
def test_gauge_covariance():
    """D_W[U^g](g psi) = g D_W[U] psi for U^g_mu(x) = g(x) U_mu(x) g(x+mu)^H."""
    dims = (4, 4, 6, 4)
    lat = oracle.Lattice(dims)
    U = synth.gauge(dims, 0.5, 61)
    g = synth.gauge(dims, 0.9, 62)[:, 0]
    x = np.stack(np.meshgrid(*[np.arange(l) for l in dims], indexing="ij"), -1).reshape(-1, 4)
    Ug = np.empty_like(U)
    for mu in range(4):
        y = x.copy()
        y[:, mu] = (y[:, mu] + 1) % dims[mu]
        n = ((y[:, 0] * dims[1] + y[:, 1]) * dims[2] + y[:, 2]) * dims[3] + y[:, 3]
        Ug[:, mu] = g @ U[:, mu] @ g[n].conj().transpose(0, 2, 1)
    psi = synth.gaussian_spinor(lat.V, 63)[0]
    gpsi = np.einsum("xcd,xad->xac", g, psi)
    lhs = oracle.dw(lat, Ug, M0, gpsi)
    rhs = np.einsum("xcd,xad->xac", g, oracle.dw(lat, U, M0, psi))
    assert rel(lhs, rhs) < 1e-14


# ---------------------------------------------------------------- T11
def test_exact_sign_two_routes(lat44, U44, dense44):
    """sign(Q) from eigh(Q) equals Gamma_5 times the polar factor of D_W (Lemma 2)."""
    Sp = dense.sign_q_polar(lat44, U44, M0)
    assert np.abs(dense44["S"] - Sp).max() < 1e-12


def test_zolotarev_mscg_matches_exact_sign(lat44, U44, dense44):
    """Zolotarev + multishift CG reproduces the exact sign(Q) b on 4^4 within
    the rational error delta plus the solver tolerance."""
    w = np.abs(dense44["w"])
    s, wt, delta = oracle.zolotarev(0.99 * w.min(), 1.01 * w.max(), 20)
    assert delta < 1e-13
    b = synth.workload_sources(0)[0]
    out, iters, _ = oracle.sign_q(lat44, U44, M0, s, wt, b, 1e-13, 5000)
    exact = (dense44["S"] @ b.reshape(-1)).reshape(b.shape)
    assert rel(out, exact) < 1e-12
    # D_ov itself against the dense overlap matrix
    Dov = RHO * (np.eye(3072) + dense44["G5"] @ dense44["S"])
    out2, _, _ = oracle.overlap(lat44, U44, RHO, s, wt, b, 1e-13, 5000)
    assert rel(out2, (Dov @ b.reshape(-1)).reshape(b.shape)) < 1e-12


# ---------------------------------------------------------------- T12
def test_sign_squared_and_ginsparg_wilson(lat44, U44, dense44):
    """sign(Q)^2 = I (the sign function is its own inverse, proof of Lemma 1(ii))
    and the Ginsparg-Wilson relation eq. (GW), which in the normalisation
    D = rho (I + Gamma_5 sign(Q)) reads Gamma_5 D + D Gamma_5 = (1/rho) D Gamma_5 D."""
    w = np.abs(dense44["w"])
    s, wt, delta = oracle.zolotarev(0.99 * w.min(), 1.01 * w.max(), 20)
    b = synth.gaussian_spinor(lat44.V, 71)[0]
    Sb, _, _ = oracle.sign_q(lat44, U44, M0, s, wt, b, 1e-13, 5000)
    SSb, _, _ = oracle.sign_q(lat44, U44, M0, s, wt, Sb, 1e-13, 5000)
    assert rel(SSb, b) < 1e-12
    g5 = oracle.gamma5
    D = lambda v: oracle.overlap(lat44, U44, RHO, s, wt, v, 1e-13, 5000)[0]
    lhs = g5(D(b)) + D(g5(b))
    rhs = D(g5(D(b))) / RHO
    assert np.linalg.norm(lhs - rhs) / np.linalg.norm(b) < 1e-11


# ---------------------------------------------------------------- T13
def test_overlap_normal_and_on_circle():
    """Lemma 1(ii) in this normalisation: D_ov is normal and its spectrum lies
    on |lambda - rho| = rho, symmetric to the real axis."""
    dims = (4, 2, 2, 4)
    lat = oracle.Lattice(dims)
    U = synth.gauge(dims, 0.5, 81)
    Dov = dense.overlap_exact(lat, U, RHO)
    assert np.abs(Dov @ Dov.conj().T - Dov.conj().T @ Dov).max() < 1e-12
    ev = np.linalg.eigvals(Dov)
    assert np.abs(np.abs(ev - RHO) - RHO).max() < 1e-12
    d = np.abs(ev[:, None] - np.conj(ev)[None, :]).min(axis=0)
    assert d.max() < 1e-10


# ---------------------------------------------------------------- T14
def test_zolotarev_n1_closed_form():
    """n = 1: sigma_1 = k and D = 2 / (1/(1+k) + 1/(2 sqrt k)) (x/(x^2+k) has
    equal endpoint values 1/(1+k) and its maximum 1/(2 sqrt k) at sqrt k)."""
    for k in (0.01, 0.075, 0.3, 0.8):
        sig, a, D, delta = oracle.zolotarev_unit(k, 1)
        assert abs(sig[0] - k) < 1e-14 * max(1, k)
        assert abs(a[0] - 1) < 1e-15
        lo, hi = 1 / (1 + k), 1 / (2 * np.sqrt(k))
        assert abs(D - 2 / (lo + hi)) < 1e-13
        assert abs(delta - (hi - lo) / (hi + lo)) < 1e-13


@pytest.mark.parametrize("k,n", [(0.075, 4), (0.075, 8), (0.2, 6), (0.01, 10)])
def test_zolotarev_equioscillation(k, n):
    """Chebyshev alternation of the optimal approximant: the relative error
    D R(x) - 1 on [k,1] has 2n+1 extrema of alternating sign and equal size
    delta (the two endpoints and 2n-1 interior ones), all a_j, sigma_j > 0."""
    sig, a, D, delta = oracle.zolotarev_unit(k, n)
    assert (sig > 0).all() and (a > 0).all()
    x = np.exp(np.linspace(np.log(k), 0, 400001))
    err = D * x * np.sum(a[None, :] / (x[:, None] ** 2 + sig[None, :]), axis=1) - 1
    # 2n+1 alternating extrema <=> 2n zero crossings; the extreme of each
    # stretch between crossings must have size delta
    cross = np.where(np.sign(err[1:]) != np.sign(err[:-1]))[0] + 1
    assert len(cross) == 2 * n
    seg = np.split(err, cross)
    vals = np.array([sg[np.argmax(np.abs(sg))] for sg in seg])
    assert np.all(np.sign(vals[1:]) == -np.sign(vals[:-1]))
    assert vals[0] < 0 and vals[-1] < 0
    assert np.abs(np.abs(vals) - delta).max() < 1e-6 * delta + 1e-15
    assert np.abs(err).max() <= delta * (1 + 1e-6) + 1e-15


def test_zolotarev_error_decreases():
    ds = [oracle.zolotarev_unit(0.075, n)[3] for n in (2, 4, 6, 8, 10, 12)]
    assert all(b < a for a, b in zip(ds, ds[1:]))
    assert ds[-1] < 1e-12


# ---------------------------------------------------------------- T15
def test_multishift_cg_matches_single_shift_cg():
    """Every shifted solution from the shared Krylov space equals an
    independent CG solve of that shifted system."""
    dims = (4, 4, 4, 8)
    lat = oracle.Lattice(dims)
    U = synth.gauge(dims, 0.3, 91, n_stout=1)
    b = synth.gaussian_spinor(lat.V, 92)[0]
    shifts = np.array([0.003, 0.05, 0.4, 3.0, 25.0, 400.0])
    x, iters, it = oracle.mscg(lat, U, M0, shifts, b, 1e-12, 3000)
    assert np.all(np.diff(iters) <= 0)
    for j, s in enumerate(shifts):
        xr, _ = oracle.cg(lat, U, M0, s, b, 1e-13, 3000)
        assert rel(x[j], xr) < 1e-10
        assert oracle.true_residual(lat, U, M0, s, b, x[j]) < 1e-11


def test_multishift_cg_frozen_shifts_stay_finite():
    """A shift that converges in a few iterations is frozen; otherwise its
    zeta underflows and the next ratio is 0/0."""
    dims = (4, 4, 4, 4)
    lat = oracle.Lattice(dims)
    U = synth.gauge(dims, 0.5, 93)
    b = synth.gaussian_spinor(lat.V, 94)[0]
    shifts = np.array([1e-4, 1e8, 1e12])
    x, iters, it = oracle.mscg(lat, U, M0, shifts, b, 1e-15, 4000)
    assert np.isfinite(x).all()
    assert iters[2] <= 3 and iters[1] <= 4
    for j, s in enumerate(shifts):
        assert oracle.true_residual(lat, U, M0, s, b, x[j]) < 1e-13


# ---------------------------------------------------------------- Lanczos
def test_lanczos_bounds_bracket_spectrum(lat44, U44, dense44):
    """Extreme Ritz values of Q^2 converge to the extreme eigenvalues from inside."""
    ev = dense44["w"] ** 2
    v0 = synth.gaussian_spinor(lat44.V, 101)[0]
    t0, t1 = oracle.lanczos_q2(lat44, U44, M0, v0, 300)
    assert ev.min() - 1e-12 <= t0 and t1 <= ev.max() + 1e-10
    assert abs(t0 - ev.min()) < 1e-6 * ev.min() and abs(t1 - ev.max()) < 1e-9 * ev.max()
    lo, hi = oracle.spectral_interval(lat44, U44, M0, v0)
    w = np.abs(dense44["w"])
    assert lo < w.min() and hi > w.max()


# ---------------------------------------------------------------- T16
def test_stout_smearing_lowers_action():
    """Stout smearing (eq. (stout)) is a Lie-Euler step of the Wilson flow, so it
    lowers the Wilson action: <Re tr P> rises at every step, the links stay in
    SU(3), and the Prop. 2 non-normality falls.  The opposite orientation of Z
    (the literal sign of eq. (Zdef)) raises the action instead."""
    dims = (4, 4, 4, 4)
    lat = oracle.Lattice(dims)
    U = synth.gauge(dims, 0.3, 111)
    plaq = [oracle.average_plaquette(lat, U)]
    V = U
    for _ in range(3):
        V = synth.stout(dims, V, 0.1, 1)
        u = V.reshape(-1, 3, 3)
        assert np.abs(u @ u.conj().transpose(0, 2, 1) - np.eye(3)).max() < 1e-14
        assert np.abs(np.linalg.det(u) - 1).max() < 1e-14
        plaq.append(oracle.average_plaquette(lat, V))
    assert all(b > a for a, b in zip(plaq, plaq[1:]))
    assert synth.gauge(dims, 0.3, 111, n_stout=3).tobytes() == V.tobytes()
    W = synth.stout(dims, U, -0.1, 1)
    assert oracle.average_plaquette(lat, W) < plaq[0]


# ---------------------------------------------------------------- outer solver
def test_gmres_dense_random_and_restart():
    """oracle.krylov.gmres against a direct dense solve (LAPACK), for short and
    long restart cycles: the solution of A x = b does not depend on them."""
    from oracle import krylov
    rng = np.random.default_rng(7)
    n = 80
    # eigenvalues in a disk of radius about 13 around 30: restarted GMRES converges
    A = rng.standard_normal((n, n)) + 1j * rng.standard_normal((n, n)) + 30.0 * np.eye(n)
    b = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    exact = np.linalg.solve(A, b)
    for m in (5, 30, 100):
        x, it, res = krylov.gmres(lambda v: A @ v, b, 1e-12, restart=m)
        assert res <= 1e-12
        assert rel(x, exact) < 1e-10, (m, rel(x, exact))
    x0, it0, _ = krylov.gmres(lambda v: A @ v, np.zeros(n), 1e-12)
    assert it0 == 0 and not np.any(x0)


def test_gmres_overlap_system_vs_dense_solve(lat44, U44, dense44):
    """eq. (linsys) on the 4^4 dense-check workload: GMRES on the oracle's
    Zolotarev D_ov against a dense solve with the exact sign (Lemma 2's
    operator); the difference is bounded by the condition number times the
    GMRES tolerance plus the Zolotarev error."""
    from oracle import krylov
    aw = np.abs(dense44["w"])
    s, wt, delta = oracle.zolotarev(0.99 * aw.min(), 1.01 * aw.max(), 20)
    Dov = RHO * (np.eye(3072) + dense44["G5"] @ dense44["S"])
    b = synth.workload_sources(0)[0]
    exact = np.linalg.solve(Dov, b.reshape(-1)).reshape(b.shape)
    cond = np.linalg.cond(Dov)
    tol = 1e-10
    x, it, res = krylov.gmres(lambda v: oracle.overlap(lat44, U44, RHO, s, wt, v, 1e-13, 5000)[0], b, tol,
                              restart=100)
    assert res <= tol and it > 5
    assert rel(x, exact) < cond * (tol + 10 * delta) * 10, (rel(x, exact), cond)


def test_lanczos_sign_converges_to_exact_sign(lat44, U44, dense44):
    """The Lanczos approximation of sign(Q) b (oracle.krylov.lanczos_sign)
    converges to the exact sign from the dense eigen-decomposition, and with
    a full Krylov space it is exact."""
    from oracle import krylov
    b = synth.workload_sources(0)[0]
    exact = (dense44["S"] @ b.reshape(-1)).reshape(b.shape)
    qop = lambda v: oracle.q(lat44, U44, M0, v)
    errs = [rel(krylov.lanczos_sign(qop, b, k)[0], exact) for k in (50, 150, 400)]
    assert errs[0] > errs[1] > errs[2] and errs[2] < 1e-10, errs
    # a 2x2 diagonal check: sign of diag(3, -2) applied to (1, 1)
    x, n = krylov.lanczos_sign(lambda v: np.array([3.0, -2.0]) * v, np.array([1.0 + 0j, 1.0]), 5)
    assert n == 2 and np.allclose(x, [1.0, -1.0], atol=1e-14)


# ---------------------------------------------------------------- deflation (Section 5.2)
@pytest.fixture(scope="module")
def modes44(lat44, U44):
    from oracle import deflation
    return deflation.low_modes_dense(lat44, U44, M0, 16)


def test_low_modes_dense_are_the_smallest_eigenpairs(lat44, U44, dense44, modes44):
    """The k = 16 pairs are eigenpairs of the stencil's Q (residual through
    oracle.q), orthonormal, and carry the 16 smallest moduli of the spectrum;
    the smallest modulus squared is the oracle Lanczos's lowest Ritz value of
    Q^2 (an independent routine)."""
    lam, xi, wsorted = modes44
    assert np.allclose(np.abs(lam), np.sort(np.abs(dense44["w"]))[:16], rtol=0, atol=1e-12)
    assert np.all(np.diff(np.abs(lam)) >= -1e-14)
    G = np.array([[np.vdot(a, b) for b in xi] for a in xi])
    assert np.abs(G - np.eye(16)).max() < 1e-12
    for l, x in zip(lam, xi):
        assert np.linalg.norm(oracle.q(lat44, U44, M0, x) - l * x) < 1e-11
    v0 = synth.gaussian_spinor(lat44.V, 101)[0]
    t0, _ = oracle.lanczos_q2(lat44, U44, M0, v0, 300)
    assert abs(np.sqrt(t0) - abs(lam[0])) < 1e-6 * abs(lam[0])


def test_deflated_sign_with_exact_sign_is_exact(lat44, U44, dense44, modes44):
    """With the exact sign(Q) for the remainder, the deflation formula gives
    sign(Q) chi itself: sign(Q) xi_i = sign(lambda_i) xi_i, so any dropped or
    doubled term (no projector, wrong sign of a mode, xi^H chi vs chi^H xi)
    shows.  D_ov with the deflated sign is the dense overlap matrix."""
    from oracle import deflation
    lam, xi, _ = modes44
    S = dense44["S"]
    exact_sign = lambda v: (S @ v.reshape(-1)).reshape(v.shape)
    chi = synth.gaussian_spinor(lat44.V, 211)[0]
    got = deflation.deflated_sign(exact_sign, xi, lam, chi)
    assert rel(got, exact_sign(chi)) < 1e-13
    Dov = RHO * (np.eye(3072) + dense44["G5"] @ S)
    got = deflation.deflated_overlap(exact_sign, xi, lam, chi, RHO)
    assert rel(got, (Dov @ chi.reshape(-1)).reshape(chi.shape)) < 1e-13


def test_deflated_zolotarev_meets_the_deflated_bound(lat44, U44, dense44, modes44):
    """Zolotarev + multishift CG built on [|lambda_17|, lambda_max] only: with
    the 16 modes deflated the sign(Q) chi error stays within the rational
    bound delta of that interval; without deflation the same approximation
    misses the low modes by far more."""
    from oracle import deflation
    lam, xi, wsorted = modes44
    lo, hi = 0.999 * abs(wsorted[16]), 1.001 * abs(wsorted[-1])
    s, wt, delta = oracle.zolotarev(lo, hi, 8)
    apply = lambda v: oracle.sign_q(lat44, U44, M0, s, wt, v, 1e-13, 5000)[0]
    chi = synth.gaussian_spinor(lat44.V, 212)[0]
    exact = (dense44["S"] @ chi.reshape(-1)).reshape(chi.shape)
    err_defl = rel(deflation.deflated_sign(apply, xi, lam, chi), exact)
    err_plain = rel(apply(chi), exact)
    assert err_defl <= 1.05 * delta + 1e-12
    assert err_plain > 10 * err_defl


def test_even_odd_reduction_of_the_wilson_system(lat44, U44, dense44):
    """The even-odd reduction behind ovl_wilson_solve's even_odd form, on the
    dense 4^4 D_W of eq. (Wilson-Dirac): the hops join opposite parities, so
    the parity-diagonal blocks are (m0+4) I; the solution of D_W x = b has
    x_e solving the Schur complement system M x_e = b_e - D_eo D_oo^{-1} b_o
    and x_o = D_oo^{-1}(b_o - D_oe x_e); Gamma_5 M Gamma_5 = M^H (the form of
    M^H the CGLS applies); and for any x_e with that x_o the full residual
    has the norm of the reduced one."""
    L = lat44.dims
    x = np.indices(L).reshape(4, -1)                   # canonical sites, x3 fastest
    par = np.repeat(x.sum(0) % 2, 12)                  # parity of each (site, spin, colour)
    e, o = np.flatnonzero(par == 0), np.flatnonzero(par == 1)
    D, G5 = dense44["D"], dense44["G5"]
    A = M0 + 4.0
    assert np.array_equal(D[np.ix_(e, e)], A * np.eye(e.size))
    assert np.array_equal(D[np.ix_(o, o)], A * np.eye(o.size))
    Deo, Doe = D[np.ix_(e, o)], D[np.ix_(o, e)]
    M = A * np.eye(e.size) - Deo @ Doe / A
    # with D_eo = -H_eo / 2: M = A - H_eo H_oe / (4A) and c = b_e + H_eo b_o / (2A)
    b = synth.gaussian_spinor(lat44.V, 931)[0].reshape(-1)
    xs = np.linalg.solve(D, b)
    c = b[e] - Deo @ b[o] / A
    assert rel(M @ xs[e], c) < 1e-12
    assert rel((b[o] - Doe @ xs[e]) / A, xs[o]) < 1e-12
    G5e = G5[np.ix_(e, e)]
    assert np.abs(G5e @ M @ G5e - M.conj().T).max() < 1e-13
    xe = synth.gaussian_spinor(lat44.V, 932)[0].reshape(-1)[e]
    full = np.empty_like(b)
    full[e], full[o] = xe, (b[o] - Doe @ xe) / A
    assert abs(np.linalg.norm(b - D @ full) - np.linalg.norm(c - M @ xe)) < 1e-12 * np.linalg.norm(b)
