"""GPU checks of the Lanczos sign-function mode (OVL_SOLVE_LANCZOS): sign(Q) b
as |b| V_k sign(T_k) e_1 in two passes, against the exact dense sign on 4^4,
against the oracle's Lanczos approximation after the same number of steps,
and the overlap apply against the oracle's Zolotarev form."""
import sys

import numpy as np
import pytest
import torch

import oracle
import synth
from oracle import dense, krylov
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


def test_lanczos_sign_vs_exact_dense_4x4(ovl):
    dims = (4, 4, 4, 4)
    note("lanczos sign vs dense 4^4")
    lat, olat = ovl.Lattice(dims), oracle.Lattice(dims)
    U = synth.workload_gauge(0)
    G = ovl.Gauge(lat, dev(U))
    S, w = dense.sign_q_exact(olat, U, M0)
    b = synth.gaussian_spinor(lat.V, 101, 2)
    B = ovl.Spinor.from_canonical(lat, dev(b), 0)
    O = ovl.Spinor(lat, 0, 2)
    s, wt, _ = ovl.zolotarev(0.4, 6.0, 12)   # ignored by the Lanczos mode
    prm = ovl.default_params(tol=1e-13, maxiter=3000, mode=ovl.SOLVE_LANCZOS)
    st = ovl.sign_q_apply(lat, G, M0, s, wt, B, O, prm)
    got = O.to_canonical().cpu().numpy()
    Dov = RHO * (np.eye(3072) + dense.gamma5_matrix(lat.V) @ S)
    for r in range(2):
        exact = (S @ b[r].reshape(-1)).reshape(b[r].shape)
        ratio, r2 = field_check(got[r], exact, dims, 1e-10)
        note(f"  rhs {r}: {st['iterations'][r]} steps, worst/bound {ratio:.3g}, L2 {r2:.2e}")
        assert ratio <= 1.0
        # the oracle's Lanczos approximation with the same number of steps
        ref, n = krylov.lanczos_sign(lambda v: oracle.q(olat, U, M0, v), b[r], st["iterations"][r])
        assert field_check(got[r], ref, dims, 1e-9)[0] <= 1.0
    st = ovl.overlap_apply(lat, G, RHO, s, wt, B, O, prm)
    got = O.to_canonical().cpu().numpy()
    for r in range(2):
        assert field_check(got[r], (Dov @ b[r].reshape(-1)).reshape(b[r].shape), dims, 1e-10)[0] <= 1.0


def test_lanczos_overlap_vs_oracle_zolotarev(ovl):
    dims = (8, 4, 4, 8)
    note("lanczos overlap vs oracle Zolotarev 8x4x4x8")
    lat, olat = ovl.Lattice(dims), oracle.Lattice(dims)
    U = synth.gauge(dims, 0.3, 103, n_stout=2)
    G = ovl.Gauge(lat, dev(U))
    b = np.concatenate([synth.gaussian_spinor(lat.V, 104, 2), np.zeros((1, lat.V, 4, 3), dtype=complex)])
    B = ovl.Spinor.from_canonical(lat, dev(b), 0)
    O = ovl.Spinor(lat, 0, 3)
    v0 = synth.gaussian_spinor(lat.V, 105)[0]
    olo, ohi = oracle.spectral_interval(olat, U, M0, v0, 300)
    os_, ow, _ = oracle.zolotarev(olo, ohi, 20)
    prm = ovl.default_params(tol=1e-12, maxiter=3000, mode=ovl.SOLVE_LANCZOS)
    st = ovl.overlap_apply(lat, G, RHO, os_, ow, B, O, prm)
    got = O.to_canonical().cpu().numpy()
    assert st["iterations"][2] == 0 and not np.any(got[2])
    for r in range(2):
        ref, _, _ = oracle.overlap(olat, U, RHO, os_, ow, b[r], 1e-13, 5000)
        ratio, r2 = field_check(got[r], ref, dims, 1e-9)
        note(f"  rhs {r}: {st['iterations'][r]} Lanczos steps, worst/bound {ratio:.3g}, L2 {r2:.2e}")
        assert ratio <= 1.0
