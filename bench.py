"""Benchmark: Wilson stencil HBM bandwidth and overlap applies per second.

One step = one overlap apply D_ov b = rho (b + D_W(-rho) sum_l w_l (Q^2+s_l)^{-1} b)
on the 32^3x64 workload (links exp(i 0.3 H) with 2 stout steps, one Gaussian
source, 20 Zolotarev poles over Lanczos bounds of |Q|, multishift CG to a
1e-10 relative residual on every shifted system): the whole hot path -- field
packing is done once, the stencil, Q^2, the multishift iteration with its
reductions, the combination and the final FP64 stencil run inside every step.
Inputs are synthetic and seeded; nothing is read from disk.

Prints one JSON line.  Single GPU only.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
RHO = 1.6


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
                    help="comma-separated forms timed once each besides the timed form")
    ap.add_argument("--multi-rhs", type=int, default=3,
                    help="workload recipe of the batched multi-RHS line (3 = 24^3x48, 12 point "
                         "sources); -1 skips it")
    ap.add_argument("--multi-rhs-steps", type=int, default=2)
    ap.add_argument("--stencil-order", default="",
                    help="tile_t,stream_t,stream_t64 for the main workload instead of autotuning "
                         "(profiling runs pin the order the timed run chose)")
    return ap.parse_args()


# sources that define each kernel class's kernels and launches
CLASS_SOURCES = {"wilson_stencil_q2": ("device.h", "wilson.h", "wilson.hip")}


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
        lat.tile_t, lat.stream_t, lat.stream_t64 = (int(v) for v in args.stencil_order.split(","))
        tune = dict(tile_t=lat.tile_t, stream_t=lat.stream_t, stream_t64=lat.stream_t64, timings="fixed")
    else:
        tune = ovl.autotune_stencil(lat, G, B.nrhs)
    setup_s = time.time() - t_setup
    print(f"[bench] setup {setup_s:.1f}s dims={dims} |Q| in [{lo:.4f}, {hi:.4f}] delta={delta:.2e}",
          file=sys.stderr, flush=True)

    stream = torch.cuda.current_stream()

    # ---- Wilson stencil bandwidth, one launch = D_W on every site
    site_bytes = {ovl.F64: 192 + 192 + 4 * 96, ovl.F32: 96 + 96 + 4 * 48, ovl.F16S: 52 + 52 + 4 * 24}
    stencil = {}
    for prec in (ovl.F64, ovl.F32, ovl.F16S):
        inp = ovl.Spinor.from_canonical(lat, torch.from_numpy(b[:1]).cuda(), prec)
        o = ovl.Spinor(lat, prec)
        for _ in range(3):
            ovl.wilson_apply(lat, G, -RHO, inp, o)
        n = 20
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(n):
            ovl.wilson_apply(lat, G, -RHO, inp, o)
        e1.record(stream)
        torch.cuda.synchronize()
        sec = e0.elapsed_time(e1) * 1e-3 / n
        gbps = site_bytes[prec] * V / sec / 1e9
        stencil[ovl.PREC_NAMES[prec]] = dict(us=round(sec * 1e6, 2), GBps=round(gbps, 1),
                                             frac=round(gbps / HBM_PEAK_GBPS, 4),
                                             bytes_per_site=site_bytes[prec])
        print(f"[bench] stencil {ovl.PREC_NAMES[prec]}: {sec*1e6:.1f} us {gbps:.0f} GB/s", file=sys.stderr, flush=True)

    # ---- overlap applies
    def params(form, profile=False):
        # an optional ":m<k>" suffix sets the block length of the blocked forms
        if ":m" in form:
            form, m = form.split(":m", 1)
            prm = params(form, profile)
            prm.block = int(m)
            return prm
        if form == "fp64":       # plain FP64: every shifted vector updated every iteration
            return ovl.default_params(tol=args.tol, maxiter=5000, profile=int(profile))
        if form == "fp64_blocked":
            return ovl.default_params(tol=args.tol, maxiter=5000, profile=int(profile), block=16)
        if form.startswith("mixed"):
            # FP64 iterations until |r|/|b| < sloppy_below ("mixed@<value>", default
            # the library's), then the FP32 bulk with FP64 residual replacement;
            # FP64 verification and refinement of every shift
            # block lengths: the library's (FP64 phase 16, FP32 phase 32) unless ":m<k>"
            # sets the FP32 phase's
            prm = ovl.default_params(tol=args.tol, maxiter=5000, profile=int(profile), mode=ovl.SOLVE_MIXED)
            if "@" in form:
                prm.sloppy_below = float(form.split("@", 1)[1])
            return prm
        raise ValueError(form)

    def overlap(form, profile=False):
        return ovl.overlap_apply(lat, G, RHO, shifts, weights, B, out, params(form, profile))

    forms = [f for f in args.forms.split(",") if f]
    timed_form = "mixed" if args.form == "auto" else args.form
    if "fp64" not in forms:
        forms.insert(0, "fp64")
    results = {}
    outputs = {}
    for form in forms:
        st = overlap(form)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = overlap(form)
        torch.cuda.synchronize()
        results[form] = dict(seconds=time.perf_counter() - t0, iterations=st["iterations"],
                             shift_iters=st["shift_iters"][0], reliable_updates=st["reliable_updates"],
                             refine_iterations=st["refine_iterations"],
                             max_true_residual=max(st["true_residual"][0]))
        outputs[form] = out.to_canonical().cpu().numpy()
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
        st = overlap(timed_form, profile=True)
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

    # ---- batched multi-RHS workload (its own lattice, after the timed region)
    mrhs = None
    if args.multi_rhs >= 0:
        del G, B, out
        torch.cuda.empty_cache()
        mrhs = multi_rhs_line(args, ovl, synth, np, torch)

    # ---- CPU baseline: the FP64 oracle on a bounded sample of the same workload
    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(args, dims, U, b[0], shifts, weights, results["fp64"]["shift_iters"])

    nrhs = len(b)
    fp64_rate = nrhs / results["fp64"]["seconds"]
    # one unpack and one pack of a packed FP64 field: plain streaming kernels
    # of known size for counter calibration
    Bc = ovl.Spinor.from_canonical(lat, torch.from_numpy(b[:1]).cuda(), ovl.F64)
    ovl.unpack_spinor(lat, Bc, torch.empty((1, V, 4, 3), dtype=torch.complex128, device="cuda"))
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
                   "stencil_order": {k: tune[k] for k in ("tile_t", "stream_t", "stream_t64")},
                   "spectral_interval": [lo, hi], "zolotarev_delta": delta},
        "stencil": stencil,
        "forms": {k: dict(applies_per_s=round(nrhs / v["seconds"], 4), iterations=v["iterations"],
                          rel_diff_vs_fp64=v["rel_diff_vs_fp64"], reliable_updates=v["reliable_updates"],
                          refine_iterations=v["refine_iterations"], max_true_residual=v["max_true_residual"])
                  for k, v in results.items()},
        "timed_rel_diff_vs_fp64": timed_diff,
        "fp64_applies_per_s": round(fp64_rate, 4),
        "speedup_vs_fp64": round(applies_per_s / fp64_rate, 3),
        "speedup_vs_fp64_blocked": (round(applies_per_s * results["fp64_blocked"]["seconds"] / nrhs, 3)
                                    if "fp64_blocked" in results else None),
        "iterations": last["iterations"],
        "timed_max_true_residual": max(max(r) for r in last["true_residual"][:nrhs]),
        "timed_refine_iterations": last["refine_iterations"],
        "roofline": roofline,
        "cpu_baseline": cpu,
        "multi_rhs": mrhs,
        "autotune": tune["timings"],
    }
    print(json.dumps(line))


def multi_rhs_line(args, ovl, synth, np, torch):
    """The batched multi-RHS workload: the 12 spin-colour point sources of one
    seeded site on 24^3x48 (20 poles), solved together in one mixed overlap
    apply (one link load serves all 12 RHS in every stencil), against the
    plain FP64 single-RHS form on the first of them."""
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
    prm = ovl.default_params(tol=args.tol, maxiter=5000, mode=ovl.SOLVE_MIXED)
    ovl.overlap_apply(lat, G, RHO, shifts, weights, B, out, prm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.multi_rhs_steps):
        st = ovl.overlap_apply(lat, G, RHO, shifts, weights, B, out, prm)
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    rate = B.nrhs * args.multi_rhs_steps / el
    # plain FP64, one RHS at a time
    B1 = ovl.Spinor.from_canonical(lat, torch.from_numpy(b[:1]).cuda(), ovl.F64)
    out1 = ovl.Spinor(lat, ovl.F64)
    p64 = ovl.default_params(tol=args.tol, maxiter=5000)
    ovl.overlap_apply(lat, G, RHO, shifts, weights, B1, out1, p64)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    st64 = ovl.overlap_apply(lat, G, RHO, shifts, weights, B1, out1, p64)
    torch.cuda.synchronize()
    el64 = time.perf_counter() - t1
    got = out.to_canonical().cpu().numpy()[0]
    ref = out1.to_canonical().cpu().numpy()[0]
    line = dict(workload=f"overlap apply {dims[1]}^3x{dims[0]}, 12 spin-colour point sources at one site, "
                         f"{c['poles']} Zolotarev poles, tol {args.tol:g}",
                nrhs=B.nrhs, form="mixed (FP64 until 1e-5, FP32 bulk, FP64 verification)",
                applies_per_s=round(rate, 4), seconds_per_batch=round(el / args.multi_rhs_steps, 4),
                fp64_single_rhs_applies_per_s=round(1.0 / el64, 4),
                speedup_vs_fp64_single_rhs=round(rate * el64, 3),
                iterations=st["iterations"], max_true_residual=max(max(r) for r in st["true_residual"]),
                refine_iterations=st["refine_iterations"],
                rel_diff_rhs0_vs_fp64=float(np.linalg.norm(got - ref) / np.linalg.norm(ref)),
                stencil_order={k: tune[k] for k in ("tile_t", "stream_t", "stream_t64")},
                autotune=tune["timings"])
    print(f"[bench] multi-rhs {dims}: {rate:.3f} RHS-applies/s, FP64 single {1.0/el64:.3f}/s, "
          f"max residual {line['max_true_residual']:.2e}", file=sys.stderr, flush=True)
    return line


def cpu_baseline(args, dims, U, b, shifts, weights, shift_iters):
    """Oracle timing on a bounded sample: the FP64 oracle's multishift CG on
    the full 32^3x64 field, capped at a few iterations with every shift
    active, plus one oracle stencil; the full apply is then priced with the
    per-shift iteration counts of the same solve."""
    import numpy as np
    import oracle

    lat = oracle.Lattice(dims)
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    k = args.cpu_sample_iters
    t0 = time.perf_counter()
    oracle.q2(lat, U, -RHO, b, float(min(shifts)))
    t_q2 = time.perf_counter() - t0
    t0 = time.perf_counter()
    oracle.mscg(lat, U, -RHO, shifts, b, 1e-300, k)
    t_k = time.perf_counter() - t0
    t_shift = max(t_k / k - t_q2, 0.0) / len(shifts)
    n_iter = max(shift_iters)
    act_iters = sum(shift_iters)
    est = n_iter * t_q2 + act_iters * t_shift + t_q2 / 2
    return dict(value=round(1.0 / est, 6), unit="D_ov applies/s", cores=cores, kind="oracle",
                sample=f"oracle multishift CG, {k} iterations with all {len(shifts)} shifts active on the "
                       f"full {dims[1]}^3x{dims[0]} field ({t_k:.1f}s) and one oracle Q^2 ({t_q2:.2f}s); "
                       f"apply priced as {n_iter} Q^2 + {act_iters} shift updates + 1 stencil",
                seconds_per_apply=round(est, 2))


if __name__ == "__main__":
    main()
