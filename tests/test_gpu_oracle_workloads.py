"""GPU overlap applies at the workload sizes against the FP64 oracle, site by
site (tests/parity.py).

* 16^3x32 (links exp(i 0.3 H), 2 stout steps, one Gaussian source, 20 poles):
  the oracle runs here on the whole field -- wilson_apply and q2_apply in
  every precision, the FP64 overlap apply at 1e-12 and the mixed one at 1e-8
  with every shifted system's FP64 true residual <= 1e-10.
* 32^3x64 (the benchmark workload) and 24^3x48 (12 spin-colour point sources,
  all of them): the oracle's overlap applies at sampled sites, written by
  tests/golden/make_golden.py from the oracle alone (too slow to run inside a
  GPU test); FP64 form at 1e-12, mixed form at 1e-8.

The oracle and the library each take their own Lanczos interval and Zolotarev
coefficients (error bound about 1e-15 on both sides).  FP64 comparisons run
both solvers to a 1e-13 residual, so that an iteration more or less on either
side stays below the 1e-12 bar.
"""
import os
import sys

import numpy as np
import pytest
import torch

import oracle
import synth
from parity import f16s_stencil_check, field_check, load_golden, sample_check, stencil_check

pytestmark = pytest.mark.gpu

RHO = 1.6
M0 = -RHO
GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


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
    torch.cuda.empty_cache()
    yield
    torch.cuda.empty_cache()


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def gpu_zolo(ovl, lat, G, cfg):
    v0 = synth.gaussian_spinor(lat.V, synth.SEED_BASE + 10 * cfg + 3)[0]
    lo, hi = ovl.spectral_bounds(lat, G, M0, 300, ovl.Spinor.from_canonical(lat, dev(v0), 0))
    return ovl.zolotarev(lo, hi, synth.WORKLOADS[cfg]["poles"])


def test_16x32_operators_and_overlap_vs_oracle(ovl):
    cfg = 1
    dims = synth.WORKLOADS[cfg]["dims"]
    note(f"16^3x32 operators and overlap vs oracle {dims}")
    lat = ovl.Lattice(dims)
    olat = oracle.Lattice(dims)
    U = synth.workload_gauge(cfg)
    G = ovl.Gauge(lat, dev(U))
    b = synth.workload_sources(cfg)[0]
    # wilson_apply and q2_apply, every precision, every site
    ref_w = oracle.dw(olat, U, M0, b)
    ref_q = oracle.q(olat, U, M0, b)
    s = 0.41
    ref_q2 = oracle.q2(olat, U, M0, b, s)
    for prec in (0, 1, 2):
        inp = ovl.Spinor.from_canonical(lat, dev(b), prec)
        out = ovl.Spinor(lat, prec)
        ovl.wilson_apply(lat, G, M0, inp, out)
        got_w = out.to_canonical().cpu().numpy()[0]
        ovl.q2_apply(lat, G, M0, s, inp, out)
        got_q2 = out.to_canonical().cpu().numpy()[0]
        if prec == 2:
            rw = f16s_stencil_check(got_w, ref_w, b, dims, M0)
            rq = f16s_stencil_check(got_q2, ref_q2, b, dims, M0, shift=s, ref_mid=ref_q)
        else:
            tol = 1e-12 if prec == 0 else 1e-6
            rw = stencil_check(got_w, ref_w, b, dims, M0, tol)
            rq = stencil_check(got_q2, ref_q2, b, dims, M0, tol, shift=s)
        note(f"  prec {prec}: D_W worst/bound {rw[0]:.3g} (L2 {rw[1]:.2e}), Q^2+s worst/bound {rq[0]:.3g} "
             f"(L2 {rq[1]:.2e})")
        assert rw[0] <= 1.0 and rq[0] <= 1.0, (prec, rw, rq)
    # overlap apply: oracle on the whole field
    v0 = synth.gaussian_spinor(lat.V, synth.SEED_BASE + 10 * cfg + 3)[0]
    olo, ohi = oracle.spectral_interval(olat, U, M0, v0, 300)
    os_, ow, _ = oracle.zolotarev(olo, ohi, 20)
    ref, _, oit = oracle.overlap(olat, U, RHO, os_, ow, b, 1e-13, 5000)
    shifts, weights, delta = gpu_zolo(ovl, lat, G, cfg)
    B = ovl.Spinor.from_canonical(lat, dev(b), 0)
    O = ovl.Spinor(lat, 0)
    for block in (0, 16):
        st = ovl.overlap_apply(lat, G, RHO, shifts, weights, B, O,
                               ovl.default_params(tol=1e-13, maxiter=5000, block=block))
        ratio, r2 = field_check(O.to_canonical().cpu().numpy()[0], ref, dims, 1e-12)
        note(f"  FP64 block={block}: {st['iterations'][0]} iterations (oracle {oit}), worst/bound {ratio:.3g}, "
             f"L2 {r2:.2e}")
        assert ratio <= 1.0
    st = ovl.overlap_apply(lat, G, RHO, shifts, weights, B, O,
                           ovl.default_params(tol=1e-10, maxiter=5000, mode=ovl.SOLVE_MIXED))
    tr = np.array(st["true_residual"][0][:20])
    ratio, r2 = field_check(O.to_canonical().cpu().numpy()[0], ref, dims, 1e-8)
    note(f"  mixed: {st['iterations'][0]} iterations, max shifted residual {tr.max():.2e}, worst/bound {ratio:.3g}, "
         f"L2 {r2:.2e}")
    assert (tr > 0).all() and (tr <= 1e-10).all(), tr
    assert ratio <= 1.0


def golden_case(ovl, cfg, name):
    path = os.path.join(GOLDEN, f"{name}.txt")
    gold = load_golden(path)
    dims = synth.WORKLOADS[cfg]["dims"]
    assert tuple(int(v) for v in gold["meta"]["dims"].split()) == tuple(dims)
    lat = ovl.Lattice(dims)
    G = ovl.Gauge(lat, dev(synth.workload_gauge(cfg)))
    b = synth.workload_sources(cfg)
    assert len(gold["rhs"]) == len(b)
    return gold, dims, lat, G, b


def compare_samples(got, gold, tol, what):
    sites = gold["sites"]
    worst = 0.0
    for r, g in enumerate(gold["rhs"]):
        ratio = sample_check(got[r].reshape(-1, 12)[sites], g["vals"], g["rms"], tol)
        worst = max(worst, ratio)
        assert ratio <= 1.0, (what, r, ratio)
    note(f"  {what}: worst sampled site / bound {worst:.3g} over {len(gold['rhs'])} RHS x {len(sites)} sites")


def test_32x64_overlap_vs_oracle_samples(ovl):
    cfg = 2
    gold, dims, lat, G, b = golden_case(ovl, cfg, "overlap_32x32x32x64_gaussian")
    note(f"32^3x64 overlap vs oracle samples {dims}")
    shifts, weights, delta = gpu_zolo(ovl, lat, G, cfg)
    B = ovl.Spinor.from_canonical(lat, dev(b), 0)
    O = ovl.Spinor(lat, 0)
    st = ovl.overlap_apply(lat, G, RHO, shifts, weights, B, O,
                           ovl.default_params(tol=1e-10, maxiter=5000, mode=ovl.SOLVE_MIXED))
    tr = np.array(st["true_residual"][0][:20])
    assert (tr > 0).all() and (tr <= 1e-10).all(), tr
    compare_samples(O.to_canonical().cpu().numpy(), gold, 1e-8, "mixed, tol 1e-10")
    st = ovl.overlap_apply(lat, G, RHO, shifts, weights, B, O, ovl.default_params(tol=1e-13, maxiter=5000, block=16))
    compare_samples(O.to_canonical().cpu().numpy(), gold, 1e-12, f"FP64 blocked, tol 1e-13 ({st['iterations'][0]} it)")


def test_24x48_point_sources_vs_oracle_samples(ovl):
    cfg = 3
    gold, dims, lat, G, b = golden_case(ovl, cfg, "overlap_24x24x24x48_points")
    note(f"24^3x48, all 12 point sources, vs oracle samples {dims}")
    shifts, weights, delta = gpu_zolo(ovl, lat, G, cfg)
    B = ovl.Spinor.from_canonical(lat, dev(b), 0)
    O = ovl.Spinor(lat, 0, 12)
    st = ovl.overlap_apply(lat, G, RHO, shifts, weights, B, O,
                           ovl.default_params(tol=1e-10, maxiter=5000, mode=ovl.SOLVE_MIXED))
    for r in range(12):
        tr = np.array(st["true_residual"][r][:20])
        assert (tr > 0).all() and (tr <= 1e-10).all(), (r, tr)
    compare_samples(O.to_canonical().cpu().numpy(), gold, 1e-8, "mixed batch of 12, tol 1e-10")
    ovl.overlap_apply(lat, G, RHO, shifts, weights, B, O, ovl.default_params(tol=1e-13, maxiter=5000, block=16))
    compare_samples(O.to_canonical().cpu().numpy(), gold, 1e-12, "FP64 blocked batch of 12, tol 1e-13")


def test_mixed_mode_needs_no_fp16_links(ovl):
    """The mixed solver reads FP64 and FP32 links only: a gauge field packed
    without its FP16 copy is accepted and gives the same D_ov."""
    dims = (8, 4, 4, 8)
    lat = ovl.Lattice(dims)
    U = synth.gauge(dims, 0.3, 361, n_stout=2)
    G3 = ovl.Gauge(lat, dev(U))
    G2 = ovl.Gauge(lat, dev(U), precs=(ovl.F64, ovl.F32))
    assert G2.c.f16 is None
    s, w, _ = ovl.zolotarev(0.3, 7.0, 16)
    b = synth.gaussian_spinor(lat.V, 362)[0]
    B = ovl.Spinor.from_canonical(lat, dev(b), 0)
    O2, O3 = ovl.Spinor(lat, 0), ovl.Spinor(lat, 0)
    prm = ovl.default_params(tol=1e-10, maxiter=5000, mode=ovl.SOLVE_MIXED)
    ovl.overlap_apply(lat, G2, RHO, s, w, B, O2, prm)
    ovl.overlap_apply(lat, G3, RHO, s, w, B, O3, prm)
    assert np.array_equal(O2.to_canonical().cpu().numpy(), O3.to_canonical().cpu().numpy())
