"""Benchmark: Wilson stencil HBM bandwidth and overlap applies per second.

One step = one overlap apply D_ov b = rho (b + D_W(-rho) sum_l w_l (Q^2+s_l)^{-1} b)
on the 32^3x64 workload (links exp(i 0.3 H) with 2 stout steps, one Gaussian
source, 20 Zolotarev poles over Lanczos bounds of |Q|, multishift CG to a
1e-10 relative residual on every shifted system): the whole hot path -- field
packing is done once, the stencil, Q^2, the multishift iteration with its
reductions, the combination and the final FP64 stencil run inside every step.
Inputs are synthetic and seeded; nothing is read from disk except the
oracle's stored samples of the same apply (tests/golden), for the error line.

Besides the timed steps the line reports: the stencil's bandwidth in each
precision; the FP64 forms' applies/s (the speedups are against the fastest of
them, with the plain form's ratio kept as a second key); the timed result's
error against the FP64 oracle at the sampled sites and its Ginsparg-Wilson
residual; the 16^3x32 workload (operator bandwidth, overlap applies); the
batched 24^3x48 point-source workload; and the oracle's own speed on the
host cores.

Prints one JSON line.  Single GPU only.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import platform
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
RHO = 1.6
GOLDEN = os.path.join(ROOT, "tests", "golden")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", type=int, default=2, help="workload recipe index (2 = 32^3x64)")
    ap.add_argument("--form", default="auto", help="overlap form for the timed steps")
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-iters", type=int, default=2)
    ap.add_argument("--forms", default="fp64,fp64_blocked",
                    help="comma-separated forms timed besides the timed form")
    ap.add_argument("--form-steps", type=int, default=2, help="timed applies of each form in --forms")
    ap.add_argument("--no-checks", action="store_true",
                    help="skip the Ginsparg-Wilson residual and the oracle-sample error")
    ap.add_argument("--small", type=int, default=1,
                    help="workload recipe of the small line (1 = 16^3x32); -1 skips it")
    ap.add_argument("--multi-rhs", type=int, default=3,
                    help="workload recipe of the batched multi-RHS line (3 = 24^3x48, 12 point "
                         "sources); -1 skips it")
    ap.add_argument("--multi-rhs-steps", type=int, default=2)
    ap.add_argument("--no-outer", action="store_true", help="skip the outer-solve line (16^3x32)")
    ap.add_argument("--deflate-nev", type=int, default=16,
                    help="low modes deflated in the small line's deflation entry (0 skips it)")
    ap.add_argument("--big", type=int, default=-1,
                    help="workload recipe of the largest line (4 = 48^3x96, 4 Gaussian sources, 24 poles, "
                         "one call); -1 skips it")
    ap.add_argument("--stencil-forms-only", action="store_true",
                    help="run only the multi-RHS stencil comparison (vector form, RHS tiles, matrix cores) "
                         "on the batched workload's lattice and print it as the JSON line (profiling runs)")
    ap.add_argument("--outer-only", action="store_true",
                    help="run only the outer-solve line on the small workload and print it as the JSON line "
                         "(profiling runs)")
    ap.add_argument("--outer-cases", default="",
                    help="comma-separated indices of the outer-solve cases to run (default all)")
    ap.add_argument("--stencil-order", default="",
                    help="tile_t,stream_t,stream_t64[,rhs_tile] for the main workload instead of autotuning "
                         "(profiling runs pin the order the timed run chose)")
    return ap.parse_args()


# sources that define each kernel class's kernels and launches
# (the stencils themselves, and the solvers that choose which of their modes an
# apply launches)
CLASS_SOURCES = {"wilson_stencil_q2": ("device.h", "wilson.h", "wilson.hip", "blocked.hip", "mixed.hip")}


def source_hash(kernel: str = "") -> str:
    h = hashlib.sha1()
    d = os.path.join(ROOT, "paper_1410_7170_amd", "csrc")
    files = CLASS_SOURCES.get(kernel) or sorted(f for f in os.listdir(d) if f.endswith((".h", ".hip", ".cpp")))
    for f in files:
        h.update(open(os.path.join(d, f), "rb").read())
    return h.hexdigest()[:12]


def load_traffic(kernel: str, src: str, workload: str):
    """HBM bytes per launch (calibrated FETCH_SIZE + WRITE_SIZE) measured with
    rocprofv3 counters, if recorded for these exact kernel sources and this
    workload (profiles/hbm_traffic.txt: kernel source workload fetch write)."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.txt")
    if not os.path.exists(path):
        return None
    for line in open(path):
        parts = line.split()
        if (len(parts) >= 5 and not line.startswith("#") and parts[0] == kernel and parts[1] == src
                and parts[2] == workload):
            return float(parts[3]) + float(parts[4])
    return None


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def median_event_us(torch, fn, n=20, warm=3):
    """Median over n launches of fn, each bracketed by HIP events on the
    current stream (the library launches on it)."""
    stream = torch.cuda.current_stream()
    for _ in range(warm):
        fn()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(n)]
    for a, b in ev:
        a.record(stream)
        fn()
        b.record(stream)
    torch.cuda.synchronize()
    return statistics.median(a.elapsed_time(b) for a, b in ev) * 1e3


# compulsory bytes per site of one stencil (12-real links): in + out + 4 links
SITE_BYTES = {0: 192 + 192 + 4 * 96, 1: 96 + 96 + 4 * 48, 2: 52 + 52 + 4 * 24}


def operator_bandwidth(ovl, torch, lat, G, b, q2=False):
    """Median time and algorithmic GB/s of wilson_apply (and q2_apply: two
    stencils, the second also reading the input for the shift term) per
    storage precision."""
    out = {}
    for prec in (ovl.F64, ovl.F32, ovl.F16S):
        inp = ovl.Spinor.from_canonical(lat, torch.from_numpy(b[:1]).cuda(), prec)
        o = ovl.Spinor(lat, prec)
        us = median_event_us(torch, lambda: ovl.wilson_apply(lat, G, -RHO, inp, o))
        gbps = SITE_BYTES[prec] * lat.V / (us * 1e-6) / 1e9
        d = dict(us=round(us, 2), GBps=round(gbps, 1), frac=round(gbps / HBM_PEAK_GBPS, 4),
                 bytes_per_site=SITE_BYTES[prec])
        if q2:
            ws = ovl.workspace(lat, ovl.OP_Q2, prec, 1)
            us2 = median_event_us(torch, lambda: ovl.q2_apply(lat, G, -RHO, 0.41, inp, o, ws))
            # two stencils, plus the second's read of the input for the shift term
            b2 = 2 * SITE_BYTES[prec] + (192 >> prec if prec < 2 else 52)
            g2 = b2 * lat.V / (us2 * 1e-6) / 1e9
            d["q2"] = dict(us=round(us2, 2), GBps=round(g2, 1), frac=round(g2 / HBM_PEAK_GBPS, 4), bytes_per_site=b2)
        out[ovl.PREC_NAMES[prec]] = d
        log(f"{lat.dims} stencil {ovl.PREC_NAMES[prec]}: {us:.1f} us {gbps:.0f} GB/s")
    return out


def params_for(ovl, form, tol, profile=False):
    # an optional ":f<k>" suffix sets the mixed form's FP64-phase block length
    if ":f" in form:
        form, m = form.split(":f", 1)
        prm = params_for(ovl, form, tol, profile)
        prm.block_f64 = int(m)
        return prm
    # an optional ":m<k>" suffix sets the block length of the blocked forms
    if ":m" in form:
        form, m = form.split(":m", 1)
        prm = params_for(ovl, form, tol, profile)
        prm.block = int(m)
        return prm
    if form == "fp64":       # plain FP64: every shifted vector updated every iteration
        return ovl.default_params(tol=tol, maxiter=5000, profile=int(profile))
    if form == "fp64_blocked":
        return ovl.default_params(tol=tol, maxiter=5000, profile=int(profile), block=16)
    if form == "lanczos":    # the Lanczos sign function in two passes (no poles, no per-shift vectors)
        return ovl.default_params(tol=tol, maxiter=4000, profile=int(profile), mode=ovl.SOLVE_LANCZOS)
    if form.startswith("mixed"):
        # FP64 iterations until |r|/|b| < sloppy_below ("mixed@<value>", default
        # the library's), then the FP32 bulk with FP64 residual replacement;
        # FP64 verification and refinement of every shift.  Block lengths: the
        # library's (FP64 phase 16, FP32 phase 32) unless ":m<k>" sets the FP32
        # phase's
        prm = ovl.default_params(tol=tol, maxiter=5000, profile=int(profile), mode=ovl.SOLVE_MIXED)
        if "@" in form:
            prm.sloppy_below = float(form.split("@", 1)[1])
        # "_f16": the FP32 phase's vectors rounded through FP16 storage (a
        # measurement of that format's floor); "_s64": the FP64 phase's
        # vectors stored in FP64 instead of 48 bits; "_norefine": report the
        # verified residuals without refining them
        if "_f16" in form:
            prm.sloppy_f16 = 1
        if "_s64" in form:
            prm.store48 = 0
        if "_norefine" in form:
            prm.refine = 0
        return prm
    raise ValueError(form)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "the overlap path here has no multi-GPU form.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import synth
    import paper_1410_7170_amd as ovl

    torch.cuda.set_device(0)
    if args.stencil_forms_only:
        print(json.dumps(dict(metric="multi-RHS stencil forms", data="synthetic",
                              stencil_forms=stencil_forms(args, ovl, synth, np, torch))))
        return
    if args.outer_only:
        lat, G, shifts, weights, B = small_setup(args, ovl, synth, torch)
        print(json.dumps(dict(metric="outer solve", data="synthetic",
                              outer_solve=outer_line(ovl, torch, lat, G, shifts, weights, B,
                                                     args.outer_cases))))
        return
    cfg = synth.WORKLOADS[args.workload]
    dims = cfg["dims"]
    npoles = cfg["poles"]
    t_setup = time.time()
    U = synth.workload_gauge(args.workload)
    b = synth.workload_sources(args.workload)
    lat = ovl.Lattice(dims)
    V = lat.V
    G = ovl.Gauge(lat, torch.from_numpy(U).cuda())
    v0 = synth.gaussian_spinor(V, synth.SEED_BASE + 10 * args.workload + 3)[0]
    start = ovl.Spinor.from_canonical(lat, torch.from_numpy(v0).cuda(), ovl.F64)
    lo, hi = ovl.spectral_bounds(lat, G, -RHO, 300, start)
    shifts, weights, delta = ovl.zolotarev(lo, hi, npoles)
    B = ovl.Spinor.from_canonical(lat, torch.from_numpy(b).cuda(), ovl.F64)
    out = ovl.Spinor(lat, ovl.F64, B.nrhs)
    if args.stencil_order:
        vals = [int(v) for v in args.stencil_order.split(",")]
        lat.tile_t, lat.stream_t, lat.stream_t64 = vals[:3]
        if len(vals) > 3:
            lat.rhs_tile = vals[3]
        tune = dict(tile_t=lat.tile_t, stream_t=lat.stream_t, stream_t64=lat.stream_t64, rhs_tile=lat.rhs_tile,
                    timings="fixed")
    else:
        tune = ovl.autotune_stencil(lat, G, B.nrhs)
    log(f"setup {time.time() - t_setup:.1f}s dims={dims} |Q| in [{lo:.4f}, {hi:.4f}] delta={delta:.2e}")

    # ---- Wilson stencil bandwidth, one launch = D_W on every site
    stencil = operator_bandwidth(ovl, torch, lat, G, b)

    def overlap(form, profile=False, src=B, dst=out):
        # forms that only report their verified residuals may miss the tolerance
        return ovl.overlap_apply(lat, G, RHO, shifts, weights, src, dst, params_for(ovl, form, args.tol, profile),
                                 allow_not_converged="_norefine" in form)

    # ---- the reference forms, each timed over a few applies
    forms = [f for f in args.forms.split(",") if f]
    timed_form = "mixed" if args.form == "auto" else args.form
    if "fp64" not in forms:
        forms.insert(0, "fp64")
    results, outputs = {}, {}
    for form in forms:
        st = overlap(form)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.form_steps):
            st = overlap(form)
        torch.cuda.synchronize()
        results[form] = dict(seconds=(time.perf_counter() - t0) / args.form_steps, iterations=st["iterations"],
                             shift_iters=st["shift_iters"][0], reliable_updates=st["reliable_updates"],
                             refine_iterations=st["refine_iterations"],
                             max_true_residual=max(st["true_residual"][0]))
        outputs[form] = out.to_canonical().cpu().numpy()
        log(f"form {form}: {len(b) / results[form]['seconds']:.3f} applies/s, {st['iterations']} iterations")
    ref = outputs["fp64"]
    for form in forms:
        results[form]["rel_diff_vs_fp64"] = float(np.linalg.norm(outputs[form] - ref) / np.linalg.norm(ref))

    # ---- timed region: K steps of the timed form, kernels bracketed by HIP events
    for _ in range(args.warmup):
        overlap(timed_form)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ksec = [0.0] * 4
    kbytes = [0.0] * 4
    klaunch = [0] * 4
    last = None
    for _ in range(args.steps):
        # profile level 2: HIP events on the stencil launches (the dominant
        # class) only, as each timed launch costs a little
        st = overlap(timed_form, profile=2)
        for c in range(4):
            ksec[c] += st["kernel_seconds"][c]
            kbytes[c] += st["kernel_bytes"][c]
            klaunch[c] += st["kernel_launches"][c]
        last = st
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    ms_per_step = elapsed / args.steps * 1e3
    applies_per_s = len(b) * args.steps / elapsed

    got = out.to_canonical().cpu().numpy()
    timed_diff = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))

    # dominant kernel of the timed step
    names = {0: "wilson_stencil_q2", 1: "multishift_update", 2: "scalar_reductions", 3: "other"}
    dom = max(range(4), key=lambda c: ksec[c])
    avg = ksec[dom] / max(klaunch[dom], 1)
    bytes_per_launch = kbytes[dom] / max(klaunch[dom], 1)
    achieved = bytes_per_launch / avg / 1e9 if avg > 0 else 0.0
    src = source_hash(names[dom])
    wl = f"{timed_form}@{'x'.join(str(d) for d in dims)}@s{lat.stream_t}-{lat.stream_t64}"
    traffic = load_traffic(names[dom], src, wl)
    roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBPS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBPS, 4),
                    traffic=(round(traffic) if traffic else None),
                    kernel=names[dom], avg_launch_us=round(avg * 1e6, 2),
                    algorithmic_bytes_per_launch=round(bytes_per_launch),
                    share_of_step=round(ksec[dom] / (elapsed), 3), source=src)

    # ---- accuracy of the timed form: oracle samples and the Ginsparg-Wilson relation
    checks = None
    if not args.no_checks:
        checks = accuracy_checks(args, ovl, torch, np, lat, B, out, got, overlap, timed_form)

    nrhs = len(b)
    fp64_rate = nrhs / results["fp64"]["seconds"]
    best64 = min((f for f in results if f.startswith("fp64")), key=lambda f: results[f]["seconds"])
    best64_rate = nrhs / results[best64]["seconds"]

    wsolve = wilson_solves(ovl, torch, lat, G, B) if not args.no_checks else None

    # ---- the small workload and the batched multi-RHS workload (own lattices)
    del G, B, out, start
    torch.cuda.empty_cache()
    small = small_line(args, ovl, synth, np, torch) if args.small >= 0 else None
    torch.cuda.empty_cache()
    mrhs = multi_rhs_line(args, ovl, synth, np, torch) if args.multi_rhs >= 0 else None
    torch.cuda.empty_cache()
    big = big_line(args, ovl, synth, np, torch) if args.big >= 0 else None

    # ---- CPU baseline: the FP64 oracle on a bounded sample of the same workload
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args, dims, U, b[0], shifts, weights, results["fp64"]["shift_iters"])

    # one unpack and one pack of a packed FP64 field: plain streaming kernels
    # of known size for counter calibration
    lat2 = ovl.Lattice(dims)
    Bc = ovl.Spinor.from_canonical(lat2, torch.from_numpy(b[:1]).cuda(), ovl.F64)
    ovl.unpack_spinor(lat2, Bc, torch.empty((1, V, 4, 3), dtype=torch.complex128, device="cuda"))
    torch.cuda.synchronize()
    line = {
        "metric": "Wilson stencil HBM GB/s + D_ov applies/sec @32^3x64, mixed vs FP64, 1e-10 res",
        "value": round(applies_per_s, 4),
        "unit": "D_ov applies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if timed_form.startswith("fp64") else "f64+f32",
        "data": "synthetic (seeded SU(3) links exp(i 0.3 H), 2 stout steps; Gaussian source)",
        "config": {"workload": f"overlap apply {dims[1]}^3x{dims[0]}, {npoles} Zolotarev poles, "
                               f"tol {args.tol:g}, rho {RHO}",
                   "lattice": list(dims), "nrhs": nrhs, "poles": npoles, "form": timed_form,
                   "stencil_order": {k: tune[k] for k in ("tile_t", "stream_t", "stream_t64", "rhs_tile")},
                   "spectral_interval": [lo, hi], "zolotarev_delta": delta},
        "stencil": stencil,
        "forms": {k: dict(applies_per_s=round(nrhs / v["seconds"], 4), iterations=v["iterations"],
                          rel_diff_vs_fp64=v["rel_diff_vs_fp64"], reliable_updates=v["reliable_updates"],
                          refine_iterations=v["refine_iterations"], max_true_residual=v["max_true_residual"])
                  for k, v in results.items()},
        "timed_rel_diff_vs_fp64": timed_diff,
        "fp64_applies_per_s": round(best64_rate, 4),
        "fp64_form": best64,
        "speedup_vs_fp64": round(applies_per_s / best64_rate, 3),
        "speedup_vs_fp64_plain": round(applies_per_s / fp64_rate, 3),
        "iterations": last["iterations"],
        "timed_max_true_residual": max(max(r) for r in last["true_residual"][:nrhs]),
        "timed_refine_iterations": last["refine_iterations"],
        "accuracy": checks,
        "roofline": roofline,
        "cpu_baseline": cpu,
        "wilson_solve": wsolve,
        "small": small,
        "multi_rhs": mrhs,
        "big": big,
        "autotune": tune["timings"],
    }
    print(json.dumps(line))


def golden_errors(np, lat, got, kind):
    """Every RHS of got (nrhs, V, 4, 3) against the oracle's D_ov at the sampled
    sites stored in tests/golden (written from the oracle alone): the worst
    site error over the field's rms site norm, over all RHS."""
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from parity import load_golden
    path = os.path.join(GOLDEN, f"overlap_{lat.dims[1]}x{lat.dims[2]}x{lat.dims[3]}x{lat.dims[0]}_{kind}.txt")
    if not os.path.exists(path):
        return None
    gold = load_golden(path)
    sites = gold["sites"]
    worst, worst_rel = 0.0, 0.0
    for q, g in enumerate(gold["rhs"]):
        err = np.linalg.norm(got[q].reshape(-1, 12)[sites] - g["vals"], axis=-1)
        worst = max(worst, float(err.max() / g["rms"]))
        worst_rel = max(worst_rel, float(np.linalg.norm(err) / np.linalg.norm(g["vals"])))
    return dict(rhs=len(gold["rhs"]), sites=len(sites), max_site_err_over_rms=worst, max_rel_l2_sampled=worst_rel,
                oracle_tol=float(gold["meta"].get("tol", "nan")))


def accuracy_checks(args, ovl, torch, np, lat, B, out, got, overlap, form):
    """Error of the timed form's D_ov b against the oracle's at the sampled
    sites (tests/golden, written from the oracle alone), and the
    Ginsparg-Wilson residual |g5 D b + D g5 b - (1/rho) D g5 D b| / |b| of
    eq. (GW) in this normalisation."""
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from parity import load_golden

    res = {}
    path = os.path.join(GOLDEN, f"overlap_{lat.dims[1]}x{lat.dims[2]}x{lat.dims[3]}x{lat.dims[0]}_gaussian.txt")
    if os.path.exists(path):
        gold = load_golden(path)
        sites = gold["sites"]
        g = gold["rhs"][0]
        mine = got[0].reshape(-1, 12)[sites]
        err = np.linalg.norm(mine - g["vals"], axis=-1)
        res["oracle_samples"] = dict(
            sites=len(sites), max_site_err_over_rms=float(err.max() / g["rms"]),
            max_site_rel_err=float((err / np.linalg.norm(g["vals"], axis=-1)).max()),
            rel_l2_sampled=float(np.linalg.norm(mine - g["vals"]) / np.linalg.norm(g["vals"])),
            oracle_tol=float(gold["meta"].get("tol", "nan")))
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()

    def g5(v):
        w = v.copy()
        w[..., :2, :] *= -1
        return w

    def D(v):
        src = ovl.Spinor.from_canonical(lat, dev(v), ovl.F64)
        overlap(form, src=src, dst=out)
        return out.to_canonical().cpu().numpy()

    b = B.to_canonical().cpu().numpy()
    Db = got
    lhs = g5(Db) + D(g5(b))
    rhs = D(g5(Db)) / RHO
    res["ginsparg_wilson_residual"] = float(np.linalg.norm(lhs - rhs) / np.linalg.norm(b))
    log(f"accuracy: {res}")
    return res


def small_setup(args, ovl, synth, torch):
    """Lattice, links, Zolotarev poles on the Lanczos interval and the source
    of the small workload (16^3x32)."""
    cfg = args.small
    c = synth.WORKLOADS[cfg]
    lat = ovl.Lattice(c["dims"])
    G = ovl.Gauge(lat, torch.from_numpy(synth.workload_gauge(cfg)).cuda())
    v0 = synth.gaussian_spinor(lat.V, synth.SEED_BASE + 10 * cfg + 3)[0]
    lo, hi = ovl.spectral_bounds(lat, G, -RHO, 300, ovl.Spinor.from_canonical(lat, torch.from_numpy(v0).cuda(),
                                                                                ovl.F64))
    shifts, weights, delta = ovl.zolotarev(lo, hi, c["poles"])
    ovl.autotune_stencil(lat, G, 1)
    B = ovl.Spinor.from_canonical(lat, torch.from_numpy(synth.workload_sources(cfg)).cuda(), ovl.F64)
    return lat, G, shifts, weights, B


def small_line(args, ovl, synth, np, torch):
    """The 16^3x32 workload: wilson_apply and q2_apply bandwidth in every
    precision and the overlap apply's rate in the FP64 and mixed forms."""
    cfg = args.small
    c = synth.WORKLOADS[cfg]
    dims = c["dims"]
    lat = ovl.Lattice(dims)
    G = ovl.Gauge(lat, torch.from_numpy(synth.workload_gauge(cfg)).cuda())
    b = synth.workload_sources(cfg)
    v0 = synth.gaussian_spinor(lat.V, synth.SEED_BASE + 10 * cfg + 3)[0]
    lo, hi = ovl.spectral_bounds(lat, G, -RHO, 300, ovl.Spinor.from_canonical(lat, torch.from_numpy(v0).cuda(),
                                                                                ovl.F64))
    shifts, weights, delta = ovl.zolotarev(lo, hi, c["poles"])
    ovl.autotune_stencil(lat, G, 1)
    ops = operator_bandwidth(ovl, torch, lat, G, b, q2=True)
    B = ovl.Spinor.from_canonical(lat, torch.from_numpy(b).cuda(), ovl.F64)
    out = ovl.Spinor(lat, ovl.F64)
    rates = {}
    for form in ("fp64", "fp64_blocked", "mixed", "lanczos"):
        prm = params_for(ovl, form, args.tol)
        ovl.overlap_apply(lat, G, RHO, shifts, weights, B, out, prm)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        n = 3
        for _ in range(n):
            st = ovl.overlap_apply(lat, G, RHO, shifts, weights, B, out, prm)
        torch.cuda.synchronize()
        rates[form] = dict(applies_per_s=round(n / (time.perf_counter() - t0), 3), iterations=st["iterations"][0],
                           max_true_residual=max(st["true_residual"][0]))
        if form == "lanczos":
            # iterations: Lanczos steps per pass (two passes); the result against the mixed form's
            got = out.to_canonical()
            rates[form]["rel_diff_vs_mixed"] = float(torch.linalg.vector_norm(got - ref_mixed) /
                                                     torch.linalg.vector_norm(ref_mixed))
        if form == "mixed":
            ref_mixed = out.to_canonical()
    log(f"small {dims}: {rates}")
    wsolve = wilson_solves(ovl, torch, lat, G, B)
    outer = None if args.no_outer else outer_line(ovl, torch, lat, G, shifts, weights, B)
    defl = None
    if args.deflate_nev > 0:
        defl = deflation_line(args, ovl, synth, torch, lat, G, B, ref_mixed, hi, delta, rates["mixed"]["applies_per_s"],
                              cfg)
    return dict(workload=f"{dims[1]}^3x{dims[0]}, {c['poles']} Zolotarev poles, tol {args.tol:g}",
                operators=ops, overlap=rates, wilson_solve=wsolve, outer_solve=outer, deflation=defl)


def deflation_line(args, ovl, synth, torch, lat, G, B, ref, hi, delta, rate_plain, cfg):
    import numpy as np
    """Low-mode deflation on the small workload: the nev lowest modes of Q
    (ovl_low_modes), then the mixed overlap apply with them deflated and the
    Zolotarev interval raised to [|lambda_nev|, lambda_max], with the fewest
    poles whose error bound does not exceed the undeflated one."""
    nev = args.deflate_nev
    start = ovl.Spinor.from_canonical(lat, torch.from_numpy(synth.gaussian_spinor(lat.V, synth.SEED_BASE + 10 * cfg
                                                                                  + 5)).cuda(), ovl.F64)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    D = ovl.low_modes(lat, G, -RHO, start, nev=nev, stages=120, allow_not_converged=True)
    setup = time.perf_counter() - t0
    lo = abs(D.evals[-1])
    eig = dict(nev=nev, setup_seconds=round(setup, 3), q2_applies=int(D.stats["q2_applies"]),
               seed_lanczos_steps=int(D.stats["steps"]), filter_iterations=int(D.stats["stages"]),
               mean_filter_degree=round(float(D.stats["mean_degree"]), 1),
               max_eig_residual=float(D.stats["max_residual"]), converged=bool(D.stats["converged"]),
               abs_lambda=[round(float(v), 6) for v in np.abs(D.evals)])
    if not D.stats["converged"]:
        # approximate eigenvectors would leave errors of their residual size
        # in the deflated apply: no timing
        log(f"deflation nev {nev}: eigenpairs not converged ({D.stats['max_residual']:.1e}), apply not timed")
        return dict(eig, applied=False)
    npoles = None
    # the rational bound saturates near 1e-15: compare at the larger of the two
    for n in range(4, 33):
        s2, w2, d2 = ovl.zolotarev(lo, hi, n)
        if d2 <= max(delta, 1e-14):
            npoles = n
            break
    if npoles is None:
        npoles, (s2, w2, d2) = 32, ovl.zolotarev(lo, hi, 32)
    out = ovl.Spinor(lat, ovl.F64)
    prm = params_for(ovl, "mixed", args.tol)
    ovl.set_deflation(prm, D)
    ovl.overlap_apply(lat, G, RHO, s2, w2, B, out, prm)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    n = 3
    for _ in range(n):
        st = ovl.overlap_apply(lat, G, RHO, s2, w2, B, out, prm)
    torch.cuda.synchronize()
    rate = n / (time.perf_counter() - t1)
    got = out.to_canonical()
    diff = float(torch.linalg.vector_norm(got - ref) / torch.linalg.vector_norm(ref))
    gain = 1.0 / rate_plain - 1.0 / rate
    line = dict(eig, applied=True, lambda_min=float(abs(D.evals[0])), lambda_nev=lo, poles=npoles, delta=d2,
                mixed_applies_per_s=round(rate, 3), undeflated_mixed_applies_per_s=rate_plain,
                speedup=round(rate / rate_plain, 3), iterations=st["iterations"][0],
                max_true_residual=max(st["true_residual"][0]),
                rel_diff_vs_undeflated=diff,
                break_even_applies=(round(setup / gain, 1) if gain > 0 else None))
    log(f"deflation nev {nev}: setup {setup:.2f}s, {rate:.2f} vs {rate_plain:.2f} applies/s, poles {npoles}")
    return line


def outer_line(ovl, torch, lat, G, shifts, weights, E, only=""):
    """D_ov psi = eta (eq. (linsys)) by FGMRES(100) to 1e-8: with the relaxed
    sign accuracy of Table (allparms1) and without it, and with the Wilson
    preconditioner D_W(m0^prec)^{-1} (eps_prec 0.1) at a few masses m0^prec
    (the paper scans m0^prec, Fig. (prec_eff_m0w)), solved in the even-odd
    form and, at one mass, through the full-lattice normal equations."""
    psi = ovl.Spinor(lat, ovl.F64)
    runs = []
    cases = [dict(relax=1), dict(relax=0)] + [dict(relax=1, precondition=1, prec_m0=m) for m in (-0.1, 0.0, 0.1)]
    # the same preconditioner solved through the normal equations of the full lattice
    cases.append(dict(relax=1, precondition=1, prec_m0=0.0, prec_even_odd=0))
    if only:
        cases = [cases[int(k)] for k in only.split(",")]
    for kw in cases:
        prm = ovl.default_outer_params(tol=1e-8, **kw)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = ovl.overlap_solve(lat, G, RHO, shifts, weights, E, psi, prm, allow_not_converged=True)
        sec = time.perf_counter() - t0
        runs.append(dict(kw, seconds=round(sec, 3), steps=st["iterations"], overlap_applies=st["overlap_applies"],
                         mscg_iterations=st["mscg_iterations"], prec_iterations=st["prec_iterations"],
                         residual=st["residual"]))
        log(f"outer solve {kw}: {sec:.2f}s, {st['iterations']} steps, {st['mscg_iterations']} MSCG iterations, "
            f"{st['prec_iterations']} CG iterations, residual {st['residual']:.2e}")
    return dict(tol=1e-8, restart=100, inner="mixed", runs=runs)


def wilson_solves(ovl, torch, lat, G, B):
    """ovl_wilson_solve in its two forms (normal equations on the full
    lattice, even-odd reduced system) at a tight tolerance and at the
    preconditioner's eps_prec, average of 3 solves each."""
    X = ovl.Spinor(lat, ovl.F64)
    runs = []
    for m0, tol in ((-0.5, 1e-10), (0.0, 1e-1)):
        for eo in (0, 1):
            prm = ovl.default_params(tol=tol, maxiter=20000, even_odd=eo)
            ws = ovl.workspace(lat, ovl.OP_WILSON_SOLVE, ovl.F64, 1, 0, prm, device="cuda")
            ovl.wilson_solve(lat, G, m0, B, X, prm, ws=ws)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(3):
                st = ovl.wilson_solve(lat, G, m0, B, X, prm, ws=ws)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t0) / 3 * 1e3
            runs.append(dict(m0=m0, tol=tol, form="even_odd" if eo else "normal_equations", ms=round(ms, 3),
                             iterations=st["iterations"][0], true_residual=st["true_residual"][0]))
            log(f"wilson solve m0 {m0} tol {tol:g} {runs[-1]['form']}: {ms:.2f} ms, {st['iterations'][0]} it, "
                f"true residual {st['true_residual'][0]:.2e}")
    return runs


def big_line(args, ovl, synth, np, torch):
    """The 48^3x96 workload: its 4 Gaussian sources in one overlap_apply call
    (24 poles, groups of one RHS in one workspace), mixed and FP64 blocked."""
    cfg = args.big
    c = synth.WORKLOADS[cfg]
    dims = c["dims"]
    lat = ovl.Lattice(dims)
    G = ovl.Gauge(lat, torch.from_numpy(synth.workload_gauge(cfg)).cuda())
    v0 = synth.gaussian_spinor(lat.V, synth.SEED_BASE + 10 * cfg + 3)[0]
    lo, hi = ovl.spectral_bounds(lat, G, -RHO, 300, ovl.Spinor.from_canonical(lat, torch.from_numpy(v0).cuda(),
                                                                                ovl.F64))
    shifts, weights, delta = ovl.zolotarev(lo, hi, c["poles"])
    b = synth.workload_sources(cfg)
    B = ovl.Spinor.from_canonical(lat, torch.from_numpy(b).cuda(), ovl.F64)
    del b
    ovl.autotune_stencil(lat, G, 1)
    out = ovl.Spinor(lat, ovl.F64, B.nrhs)
    pm = ovl.default_params(tol=args.tol, maxiter=5000, mode=ovl.SOLVE_MIXED, rhs_group=1)
    p64 = ovl.default_params(tol=args.tol, maxiter=5000, block=16, rhs_group=1)
    nb = max(ovl.workspace_bytes(lat, ovl.OP_MSCG, ovl.F64, B.nrhs, c["poles"], p) for p in (pm, p64))
    ws = torch.empty(nb, dtype=torch.uint8, device="cuda")
    res = {}
    for name, prm in (("mixed", pm), ("fp64_blocked", p64)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = ovl.overlap_apply(lat, G, RHO, shifts, weights, B, out, prm, ws=ws)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        res[name] = dict(seconds=round(el, 3), rhs_applies_per_s=round(B.nrhs / el, 4), iterations=st["iterations"],
                         max_true_residual=max(max(r) for r in st["true_residual"][:B.nrhs]))
        log(f"big {dims} {name}: {el:.2f}s for {B.nrhs} RHS")
    return dict(workload=f"overlap apply {dims[1]}^3x{dims[0]}, {B.nrhs} Gaussian sources in one call, "
                         f"{c['poles']} Zolotarev poles, tol {args.tol:g}",
                workspace_GiB=round(nb / 2 ** 30, 1), forms=res)


def multi_rhs_line(args, ovl, synth, np, torch):
    """The batched multi-RHS workload: the 12 spin-colour point sources of one
    seeded site on 24^3x48 (20 poles), solved together in one mixed overlap
    apply, against the FP64 single-RHS forms (blocked, the faster, and plain)
    on the first of them."""
    cfg = args.multi_rhs
    c = synth.WORKLOADS[cfg]
    dims = c["dims"]
    lat = ovl.Lattice(dims)
    U = synth.workload_gauge(cfg)
    G = ovl.Gauge(lat, torch.from_numpy(U).cuda())
    del U
    v0 = synth.gaussian_spinor(lat.V, synth.SEED_BASE + 10 * cfg + 3)[0]
    lo, hi = ovl.spectral_bounds(lat, G, -RHO, 300, ovl.Spinor.from_canonical(lat, torch.from_numpy(v0).cuda(),
                                                                                ovl.F64))
    shifts, weights, delta = ovl.zolotarev(lo, hi, c["poles"])
    b = synth.workload_sources(cfg)
    B = ovl.Spinor.from_canonical(lat, torch.from_numpy(b).cuda(), ovl.F64)
    out = ovl.Spinor(lat, ovl.F64, B.nrhs)
    tune = ovl.autotune_stencil(lat, G, B.nrhs)
    prm = params_for(ovl, "mixed", args.tol)
    ovl.overlap_apply(lat, G, RHO, shifts, weights, B, out, prm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.multi_rhs_steps):
        st = ovl.overlap_apply(lat, G, RHO, shifts, weights, B, out, prm)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    rate = B.nrhs * args.multi_rhs_steps / el
    got_all = out.to_canonical().cpu().numpy()
    got = got_all[0]
    del out
    oracle_samples = golden_errors(np, lat, got_all, "points")
    # FP64, one RHS at a time: both FP64 forms, each over two applies
    B1 = ovl.Spinor.from_canonical(lat, torch.from_numpy(b[:1]).cuda(), ovl.F64)
    out1 = ovl.Spinor(lat, ovl.F64)
    single = {}
    for form in ("fp64_blocked", "fp64"):
        p64 = params_for(ovl, form, args.tol)
        ovl.overlap_apply(lat, G, RHO, shifts, weights, B1, out1, p64)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(2):
            ovl.overlap_apply(lat, G, RHO, shifts, weights, B1, out1, p64)
        torch.cuda.synchronize()
        single[form] = 2.0 / (time.perf_counter() - t1)
    ref = out1.to_canonical().cpu().numpy()[0]
    line = dict(workload=f"overlap apply {dims[1]}^3x{dims[0]}, 12 spin-colour point sources at one site, "
                         f"{c['poles']} Zolotarev poles, tol {args.tol:g}",
                nrhs=B.nrhs, form="mixed (FP64 until the hand-over, FP32 bulk, FP64 verification)",
                applies_per_s=round(rate, 4), seconds_per_batch=round(el / args.multi_rhs_steps, 4),
                fp64_single_rhs_applies_per_s=round(single["fp64_blocked"], 4),
                fp64_plain_single_rhs_applies_per_s=round(single["fp64"], 4),
                speedup_vs_fp64_single_rhs=round(rate / single["fp64_blocked"], 3),
                speedup_vs_fp64_plain_single_rhs=round(rate / single["fp64"], 3),
                iterations=st["iterations"], max_true_residual=max(max(r) for r in st["true_residual"]),
                refine_iterations=st["refine_iterations"],
                rel_diff_rhs0_vs_fp64=float(np.linalg.norm(got - ref) / np.linalg.norm(ref)),
                oracle_samples=oracle_samples,
                stencil_order={k: tune[k] for k in ("tile_t", "stream_t", "stream_t64", "rhs_tile", "mfma")},
                autotune=tune["timings"],
                stencil_forms=stencil_forms(args, ovl, synth, np, torch, lat, G))
    log(f"multi-rhs {dims}: {rate:.3f} RHS-applies/s, FP64 single {single}, "
        f"max residual {line['max_true_residual']:.2e}")
    return line


def stencil_forms(args, ovl, synth, np, torch, lat=None, G=None):
    """D_W on the batched workload's 12 RHS in one launch, per stencil form:
    one RHS per block (vector ALUs), RHS tiles of 2 and 4 lanes per site
    sharing each link load, and the matrix-core FP32 form (two sites x four
    RHS per v_mfma_f32_16x16x4f32).  Algorithmic bytes per site: 12 RHS x
    (in + out) + the 12-real links once."""
    cfg = args.multi_rhs if args.multi_rhs >= 0 else 3
    c = synth.WORKLOADS[cfg]
    dims = c["dims"]
    standalone = lat is None
    if standalone:
        lat = ovl.Lattice(dims)
        G = ovl.Gauge(lat, torch.from_numpy(synth.workload_gauge(cfg)).cuda())
    nrhs = 12
    psi = torch.from_numpy(synth.gaussian_spinor(lat.V, synth.SEED_BASE + 10 * cfg + 7, nrhs)).cuda()
    if standalone:
        ovl.autotune_stencil(lat, G, nrhs)
    saved = (lat.rhs_tile, lat.mfma)   # the autotuner's choice for 12 RHS
    res = {}
    for prec in (ovl.F64, ovl.F32):
        inp = ovl.Spinor.from_canonical(lat, psi, prec)
        out = ovl.Spinor(lat, prec, nrhs)
        algo = lat.V * (nrhs * (SITE_BYTES[prec] - 4 * (96 >> prec)) + 4 * (96 >> prec))
        forms = [("vector", 1, 0), ("vector_tile2", 2, 0), ("vector_tile4", 4, 0)]
        if prec == ovl.F32:
            forms.append(("mfma", 1, 1))
        for name, tile, mf in forms:
            lat.rhs_tile, lat.mfma = tile, mf
            us = median_event_us(torch, lambda: ovl.wilson_apply(lat, G, -RHO, inp, out), n=10, warm=2)
            res[f"{ovl.PREC_NAMES[prec]}_{name}"] = dict(
                us=round(us, 1), us_per_rhs=round(us / nrhs, 2),
                frac=round(algo / (us * 1e-6) / 1e9 / HBM_PEAK_GBPS, 4))
            log(f"stencil form {ovl.PREC_NAMES[prec]} {name}: {us:.1f} us ({us / nrhs:.1f} us/RHS)")
        del inp, out
    lat.rhs_tile, lat.mfma = saved
    return dict(workload=f"D_W on {nrhs} RHS in one launch, {dims[1]}^3x{dims[0]}", nrhs=nrhs,
                bytes_per_site={ovl.PREC_NAMES[p]: nrhs * (SITE_BYTES[p] - 4 * (96 >> p)) + 4 * (96 >> p)
                                for p in (ovl.F64, ovl.F32)},
                stream_t=lat.stream_t, stream_t64=lat.stream_t64,
                autotune_choice=dict(rhs_tile=saved[0], mfma=saved[1]), forms=res)


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def cpu_baseline(args, dims, U, b, shifts, weights, shift_iters):
    """The oracle as it stands, timed on the host cores (medians).  At 32^3x64
    one oracle apply takes minutes, so the sample is: Q^2 (5 runs) and k
    multishift iterations with every shift active (3 runs) on the full
    32^3x64 field, which price one apply from the per-shift iteration counts of
    the same solve; whole oracle applies at 16^3x32 (median of 5) check that
    pricing; Q^2 at 16^3x32 on one core gives the single-core rate."""
    import numpy as np
    import oracle
    import synth

    lat = oracle.Lattice(dims)
    cores = oracle.max_threads()
    med = lambda f, n: statistics.median(_t(f) for _ in range(n))
    s0 = float(min(shifts))
    k = args.cpu_sample_iters
    t_q2 = med(lambda: oracle.q2(lat, U, -RHO, b, s0), 5)
    t_k = med(lambda: oracle.mscg(lat, U, -RHO, shifts, b, 1e-300, k), 3)
    t_shift = max(t_k / k - t_q2, 0.0) / len(shifts)

    def price(t_q2, t_shift, shift_iters):
        return max(shift_iters) * t_q2 + sum(shift_iters) * t_shift + t_q2 / 2

    est = price(t_q2, t_shift, shift_iters)
    # the 16^3x32 workload: a whole oracle apply against its pricing
    c1 = synth.WORKLOADS[1]
    lat1 = oracle.Lattice(c1["dims"])
    U1 = synth.workload_gauge(1)
    b1 = synth.workload_sources(1)[0]
    v1 = synth.gaussian_spinor(lat1.V, synth.SEED_BASE + 13)[0]
    lo1, hi1 = oracle.spectral_interval(lat1, U1, -RHO, v1, 100)
    s1, w1, _ = oracle.zolotarev(lo1, hi1, c1["poles"])
    full = []
    for _ in range(5):
        t0 = time.perf_counter()
        _, it1, _ = oracle.overlap(lat1, U1, RHO, s1, w1, b1, args.tol, 5000)
        full.append(time.perf_counter() - t0)
    t_full1 = statistics.median(full)
    t_q2_1 = med(lambda: oracle.q2(lat1, U1, -RHO, b1, float(min(s1))), 3)
    t_k1 = med(lambda: oracle.mscg(lat1, U1, -RHO, s1, b1, 1e-300, k), 3)
    est1 = price(t_q2_1, max(t_k1 / k - t_q2_1, 0.0) / len(s1), list(it1))
    # one core
    oracle.set_threads(1)
    try:
        t_q2_1c = med(lambda: oracle.q2(lat1, U1, -RHO, b1, float(min(s1))), 3)
    finally:
        oracle.set_threads(cores)
    return dict(value=round(1.0 / est, 6), unit="D_ov applies/s", cores=cores, kind="oracle",
                cpu_model=cpu_model(),
                sample=f"oracle Q^2 (median of 5, {t_q2:.2f}s) and {k} multishift iterations with all "
                       f"{len(shifts)} shifts active (median of 3, {t_k:.1f}s) on the full {dims[1]}^3x{dims[0]} "
                       f"field; one apply priced as {max(shift_iters)} Q^2 + {sum(shift_iters)} shift updates + "
                       f"1 stencil",
                seconds_per_apply=round(est, 2),
                check_16x32=dict(measured_apply_s=round(t_full1, 2), runs=5, priced_apply_s=round(est1, 2),
                                 iterations=int(max(it1))),
                single_core=dict(q2_16x32_s=round(t_q2_1c, 3), q2_16x32_all_cores_s=round(t_q2_1, 3),
                                 parallel_speedup=round(t_q2_1c / t_q2_1, 2)))


def _t(f):
    t0 = time.perf_counter()
    f()
    return time.perf_counter() - t0


if __name__ == "__main__":
    main()
