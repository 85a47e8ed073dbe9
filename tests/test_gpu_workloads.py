"""GPU checks at the full sizes of the two largest workloads: the batched
24^3x48 point-source solve and the 48^3x96, 24-pole overlap apply of all four
Gaussian sources in one call (solved one after another in one workspace).  Bars: the oracle's stencil at every site (1e-12 FP64, 1e-6
FP32), every shifted system's FP64 true residual <= 1e-10 as verified by the
library, and D_ov within 1e-8 of the FP64 blocked form."""
import sys

import numpy as np
import pytest
import torch

import oracle
import synth
from parity import field_check, stencil_check

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


@pytest.fixture(autouse=True)
def release_cached_memory():
    # these workloads take most of the GPU's memory: start each from an empty cache
    torch.cuda.empty_cache()
    yield
    torch.cuda.empty_cache()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def close(got, ref, dims, tol):
    """Site-wise check of a solver output against its reference
    (tests/parity.py field_check); returns the worst site's error over its
    bound and the relative L2 difference."""
    ratio, r2 = field_check(got, ref, dims, tol)
    assert ratio <= 1.0, (ratio, r2)
    return ratio, r2


def bounds(ovl, lat, G, cfg, npoles):
    v0 = synth.gaussian_spinor(lat.V, synth.SEED_BASE + 10 * cfg + 3)[0]
    lo, hi = ovl.spectral_bounds(lat, G, M0, 300, ovl.Spinor.from_canonical(lat, dev(v0), 0))
    return ovl.zolotarev(lo, hi, npoles)


def test_point_sources_24x48_batched(ovl):
    cfg = 3
    dims = synth.WORKLOADS[cfg]["dims"]
    note(f"12 point sources {dims}, mixed vs FP64 blocked")
    lat = ovl.Lattice(dims)
    G = ovl.Gauge(lat, dev(synth.workload_gauge(cfg)))
    s, w, d = bounds(ovl, lat, G, cfg, 20)
    b = synth.workload_sources(cfg)
    B = ovl.Spinor.from_canonical(lat, dev(b), 0)
    O = ovl.Spinor(lat, 0, 12)
    st = ovl.overlap_apply(lat, G, RHO, s, w, B, O, ovl.default_params(tol=1e-10, maxiter=5000,
                                                                      mode=ovl.SOLVE_MIXED))
    for r in range(12):
        assert max(st["true_residual"][r][:20]) <= 1e-10, r
    O64 = ovl.Spinor(lat, 0, 12)
    ovl.overlap_apply(lat, G, RHO, s, w, B, O64, ovl.default_params(tol=1e-10, maxiter=5000, block=16))
    got, ref = O.to_canonical().cpu().numpy(), O64.to_canonical().cpu().numpy()
    for r in range(12):
        close(got[r], ref[r], dims, 1e-8)


def test_48x96_stencil_and_overlap(ovl):
    cfg = 4
    dims = synth.WORKLOADS[cfg]["dims"]
    note(f"full-size workload {dims}: stencil vs oracle, 24-pole overlap")
    lat = ovl.Lattice(dims)
    U = synth.workload_gauge(cfg)
    G = ovl.Gauge(lat, dev(U))
    psi = synth.workload_sources(cfg)[0]
    ref = oracle.dw(oracle.Lattice(dims), U, M0, psi)
    del U
    for prec, tol in ((0, 1e-12), (1, 1e-6)):
        inp = ovl.Spinor.from_canonical(lat, dev(psi), prec)
        out = ovl.Spinor(lat, prec)
        ovl.wilson_apply(lat, G, M0, inp, out)
        ratio, r2 = stencil_check(out.to_canonical().cpu().numpy()[0], ref, psi, dims, M0, tol)
        assert ratio <= 1.0, (prec, ratio, r2)
        del inp, out
    del ref
    s, w, d = bounds(ovl, lat, G, cfg, 24)
    # all four Gaussian sources in one call, solved one after another in a
    # workspace sized for one (rhs_group = 1)
    b = synth.workload_sources(cfg)
    assert b.shape[0] == 4
    B = ovl.Spinor.from_canonical(lat, dev(b), 0)
    del b
    pm = ovl.default_params(tol=1e-10, maxiter=5000, mode=ovl.SOLVE_MIXED, rhs_group=1)
    p64 = ovl.default_params(tol=1e-10, maxiter=5000, block=16, rhs_group=1)
    nb = max(ovl.workspace_bytes(lat, ovl.OP_MSCG, ovl.F64, 4, 24, pm),
             ovl.workspace_bytes(lat, ovl.OP_MSCG, ovl.F64, 4, 24, p64))
    note(f"  workspace {nb / 2**30:.1f} GiB (mixed {ovl.workspace_bytes(lat, ovl.OP_MSCG, ovl.F64, 4, 24, pm) / 2**30:.1f})")
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    O = ovl.Spinor(lat, 0, 4)
    st = ovl.overlap_apply(lat, G, RHO, s, w, B, O, pm, ws=ws)
    for r in range(4):
        tr = np.array(st["true_residual"][r][:24])
        assert (tr > 0).all() and (tr <= 1e-10).all(), (r, tr)
    got = O.to_canonical().cpu().numpy()
    del O
    O64 = ovl.Spinor(lat, 0, 4)
    ovl.overlap_apply(lat, G, RHO, s, w, B, O64, p64, ws=ws)
    ref = O64.to_canonical().cpu().numpy()
    for r in range(4):
        ratio, r2 = close(got[r], ref[r], dims, 1e-8)
        note(f"  RHS {r}: {st['iterations'][r]} iterations, worst site / bound {ratio:.3g}, rel L2 {r2:.2e}")
