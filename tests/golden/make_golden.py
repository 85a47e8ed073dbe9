"""Write the oracle's overlap applies at the full workload sizes, sampled at a
fixed set of sites, for the GPU parity tests and the benchmark's error line.

Calls only the FP64 oracle (oracle/) on the seeded inputs of synth/; nothing
here comes from the GPU library.  Each file holds, per right-hand side, the
oracle's D_ov b = rho (b + D_W(-rho) y), y = sum_l w_l (Q^2 + s_l)^{-1} b
(eq. (overlap_def) in the massless normalisation, Zolotarev shifts and weights
over the oracle's own Lanczos interval of |Q|, multishift CG to tol), at the
listed sites, plus the root mean square site norm of the whole field (the
floor of the site-wise check).

Usage:  python tests/golden/make_golden.py [gauss32|points24|all]
        (32^3x64 takes about 10 minutes on 8 cores, 24^3x48 with its 12 point
        sources about 40.)
"""
from __future__ import annotations

import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import synth  # noqa: E402

RHO = 1.6
TOL = 1e-13
LANCZOS = 300


def sample_sites(V, n, seed, must=()):
    rng = np.random.default_rng(seed)
    extra = [int(s) for s in rng.choice(V, size=n, replace=False)]
    out = list(dict.fromkeys(list(must) + extra))
    return out[:max(n, len(must))]


def neighbours(dims, site):
    L = dims
    x = np.unravel_index(site, L)
    out = []
    for mu in range(4):
        for d in (-1, 1):
            y = list(x)
            y[mu] = (y[mu] + d) % L[mu]
            out.append(int(np.ravel_multi_index(y, L)))
    return out


def write(path, cfg, sites, results, meta):
    with open(path, "w") as f:
        f.write(f"# oracle D_ov b at sampled sites, workload {cfg} ({synth.WORKLOADS[cfg]['name']})\n")
        f.write("# written by tests/golden/make_golden.py (FP64 oracle only)\n")
        for k, v in meta.items():
            f.write(f"# {k} {v}\n")
        f.write("sites " + " ".join(str(s) for s in sites) + "\n")
        for r, (vals, rms, iters) in enumerate(results):
            f.write(f"rhs {r} rms {rms!r} iterations {iters}\n")
            for s, v in zip(sites, vals):
                nums = " ".join(f"{float(z.real)!r} {float(z.imag)!r}" for z in v.reshape(12))
                f.write(f"{s} {nums}\n")


def run(cfg, name, nsample, seed):
    t0 = time.time()
    c = synth.WORKLOADS[cfg]
    dims = c["dims"]
    lat = oracle.Lattice(dims)
    U = synth.workload_gauge(cfg)
    b = synth.workload_sources(cfg)
    v0 = synth.gaussian_spinor(lat.V, synth.SEED_BASE + 10 * cfg + 3)[0]
    lo, hi = oracle.spectral_interval(lat, U, -RHO, v0, LANCZOS)
    shifts, weights, delta = oracle.zolotarev(lo, hi, c["poles"])
    print(f"[{name}] interval [{lo:.6f}, {hi:.6f}] delta {delta:.2e} ({time.time() - t0:.0f}s)", flush=True)
    must = []
    if c["source"] == "point":
        src = synth.random_site(lat.V, synth.SEED_BASE + 10 * cfg + 2)
        must = [src] + neighbours(dims, src)
    sites = sample_sites(lat.V, nsample, seed, must)
    results = []
    for r in range(len(b)):
        out, iters, it = oracle.overlap(lat, U, RHO, shifts, weights, b[r], TOL, 20000)
        rms = float(np.sqrt(np.mean(np.sum(np.abs(out) ** 2, axis=(1, 2)))))
        results.append((out[sites], rms, int(it)))
        print(f"[{name}] rhs {r}: {it} iterations, rms site norm {rms:.6e} ({time.time() - t0:.0f}s)", flush=True)
        del out
    meta = dict(dims=" ".join(map(str, dims)), rho=RHO, poles=c["poles"], tol=TOL,
                interval=f"{float(lo)!r} {float(hi)!r}", lanczos=LANCZOS, delta=repr(float(delta)))
    write(os.path.join(HERE, f"{name}.txt"), cfg, sites, results, meta)


def main():
    what = sys.argv[1] if len(sys.argv) > 1 else "all"
    if what in ("gauss32", "all"):
        run(2, "overlap_32x32x32x64_gaussian", 128, 11)
    if what in ("points24", "all"):
        run(3, "overlap_24x24x24x48_points", 40, 12)


if __name__ == "__main__":
    main()
