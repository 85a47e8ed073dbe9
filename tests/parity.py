"""Element-wise parity checks of GPU results against the FP64 oracle.

Every check compares site by site (each site's 12 complex components) and
returns the largest ratio of a site's error to its bound, plus the field-wide
relative L2 difference as a second, reported number.

Stencil outputs (D_W, Q, Q^2 + s).  With 1/2 (I -+ gamma_mu) a projector and
unitary links, eq. (Wilson-Dirac) gives at every site
    |(D_W psi)(x)| <= M_x = |m0+4| |psi(x)| + sum over the 8 neighbours |psi(y)|,
so M_x is the size of the terms the kernel adds at x and every component of
the FP64 or FP32 result must lie within tol * M_x of the oracle's (Q^2 + s:
M applied twice, plus |s| |psi(x)|).  A wrong site has an error of order M_x
and fails by a factor 1/tol.

FP16 storage with per-site scales (F16S): each stored real is within
2^-11 * s_x of its value (s_x the site's largest |real or imaginary part|, an
11-bit significand, round to nearest), and each FP16 link entry within 2^-11
of its value (entries are at most 1), so a rebuilt SU(3) link differs from
the true one by at most 2^-11 sqrt(6) in Frobenius norm (rows 0 and 1: sqrt(2),
row 2 = conj(row0 x row1): 2).  Propagating these through eq. (Wilson-Dirac)
site by site, with the FP32 arithmetic and the rounding of the stored output,
gives a per-site bound on |GPU - oracle| (f16s_stencil_bound).

Solver outputs (multishift solutions, sign(Q) b, D_ov b) are global functions
of the input, so their error is spread over the lattice: site x must satisfy
|got_x - ref_x| <= tol (|ref_x| + rms), rms the root mean square of the
site norms |ref_x|.  A single wrong site fails; a field that meets the
field-wide relative tolerance tol/3 everywhere passes.
"""
from __future__ import annotations

import numpy as np

EPS16 = 2.0 ** -11          # half-ulp of FP16 relative to the site scale
LINK16 = 3.0 * EPS16        # >= sqrt(6) * 2^-11: Frobenius error of a rebuilt FP16 link
FP32_ARITH = 1e-6           # FP32 arithmetic of one stencil, relative to M_x
SQRT24 = 24 ** 0.5


def _grid(a, dims):
    """(..., V, 4, 3) -> (..., L0, L1, L2, L3, 12)."""
    a = np.asarray(a)
    return a.reshape(a.shape[:-3] + tuple(dims) + (12,))


def site_norms(psi, dims):
    return np.linalg.norm(_grid(psi, dims), axis=-1)


def site_max(psi, dims):
    g = _grid(psi, dims)
    return np.maximum(np.abs(g.real), np.abs(g.imag)).max(axis=-1)


def neighbour_sum(n):
    """sum over the 8 nearest neighbours of a per-site quantity on the last
    four axes (periodic; boundary phases do not change magnitudes)."""
    out = np.zeros_like(n)
    for ax in range(-4, 0):
        out += np.roll(n, 1, axis=ax) + np.roll(n, -1, axis=ax)
    return out


def stencil_mag(n, m0):
    """M_x of a field with site norms n: |m0+4| n_x + sum of the neighbours."""
    return abs(m0 + 4.0) * n + neighbour_sum(n)


def _ratio(err, bound):
    with np.errstate(divide="ignore", invalid="ignore"):
        r = np.where(bound > 0, err / bound, np.where(err > 0, np.inf, 0.0))
    return float(r.max())


def rel_l2(got, ref):
    got, ref = np.asarray(got), np.asarray(ref)
    nr = np.linalg.norm(ref)
    return float(np.linalg.norm(got - ref) / nr) if nr > 0 else float(np.linalg.norm(got))


def stencil_check(got, ref, psi, dims, m0, tol, shift=None):
    """Element-wise check of D_W psi / Q psi (shift None) or (Q^2 + shift) psi
    against the oracle.  Returns (max site error / (tol M_x), relative L2)."""
    n = site_norms(psi, dims)
    M = stencil_mag(n, m0)
    if shift is not None:
        M = stencil_mag(M, m0) + abs(shift) * n
    err = np.abs(_grid(got, dims) - _grid(ref, dims)).max(axis=-1)
    return _ratio(err, tol * M), rel_l2(got, ref)


def f16s_stencil_bound(psi, dims, m0, ref_out, shift=None, ref_mid=None):
    """Per-site bound on |GPU - oracle| for a stencil on FP16S storage and FP16
    links (see the module docstring).  psi: the unrounded input; ref_out: the
    oracle's output.  For Q^2 + shift, ref_mid is the oracle's Q psi (stored in
    FP16S between the two stencils)."""
    n = site_norms(psi, dims)
    e_in = SQRT24 * EPS16 * site_max(psi, dims)   # stored input, per site

    def one(err_in, norm_in):
        # error of one stencil on inputs with per-site errors err_in and norms
        # norm_in: diagonal term, hops (input error plus link error), FP32 arithmetic
        return (abs(m0 + 4.0) * err_in + neighbour_sum(err_in + LINK16 * norm_in)
                + FP32_ARITH * stencil_mag(norm_in, m0))

    if shift is None:
        e = one(e_in, n)
    else:
        e1 = one(e_in, n)
        e1 = e1 + SQRT24 * EPS16 * (site_max(ref_mid, dims) + e1)   # t stored in FP16S
        e = one(e1, site_norms(ref_mid, dims)) + abs(shift) * e_in
    return e + SQRT24 * EPS16 * (site_max(ref_out, dims) + e)


def f16s_stencil_check(got, ref, psi, dims, m0, shift=None, ref_mid=None):
    """Site-wise check of an F16S stencil result: max over sites of
    |GPU_x - oracle_x| / bound_x (<= 1 passes), and the relative L2 difference."""
    B = f16s_stencil_bound(psi, dims, m0, ref, shift, ref_mid)
    err = np.linalg.norm(_grid(got, dims) - _grid(ref, dims), axis=-1)
    return _ratio(err, B), rel_l2(got, ref)


def field_check(got, ref, dims, tol):
    """Site-wise check of a solver output: max over sites of
    |got_x - ref_x| / (tol (|ref_x| + rms)) (<= 1 passes), and the relative L2
    difference."""
    nr = site_norms(ref, dims)
    rms = float(np.sqrt(np.mean(nr ** 2)))
    err = np.linalg.norm(_grid(got, dims) - _grid(ref, dims), axis=-1)
    return _ratio(err, tol * (nr + rms)), rel_l2(got, ref)


def sample_check(got_sites, ref_sites, rms, tol):
    """The same check on sampled sites: got_sites, ref_sites (n, 12) complex,
    rms the root mean square site norm of the whole reference field."""
    nr = np.linalg.norm(ref_sites, axis=-1)
    err = np.linalg.norm(np.asarray(got_sites) - np.asarray(ref_sites), axis=-1)
    return _ratio(err, tol * (nr + rms))


def load_golden(path):
    """Read a file written by tests/golden/make_golden.py: dict with 'meta'
    (header fields), 'sites' (site indices) and 'rhs' (per RHS: rms site norm,
    oracle iterations, (nsites, 12) complex values)."""
    meta, sites, rhs = {}, None, []
    cur = None
    with open(path) as f:
        for line in f:
            parts = line.split()
            if not parts:
                continue
            if parts[0] == "#":
                if len(parts) >= 3:
                    meta[parts[1]] = " ".join(parts[2:])
            elif parts[0] == "sites":
                sites = [int(v) for v in parts[1:]]
            elif parts[0] == "rhs":
                cur = dict(rms=float(parts[3]), iterations=int(parts[5]), vals=[])
                rhs.append(cur)
            else:
                v = np.array([float(t) for t in parts[1:]])
                cur["vals"].append(v[0::2] + 1j * v[1::2])
    for r in rhs:
        r["vals"] = np.array(r["vals"])
    return dict(meta=meta, sites=sites, rhs=rhs)


def r48(a):
    """Each real of a complex128 array rounded to the 48-bit storage format:
    the top 48 bits of its IEEE pattern after rounding the dropped 16 to
    nearest, ties away from zero (adding half a unit of the kept part to the
    magnitude bits); infinities and NaNs keep their top bits."""
    a = np.ascontiguousarray(a, dtype=np.complex128)
    x = a.view(np.uint64).copy()
    special = (x & np.uint64(0x7FF0000000000000)) == np.uint64(0x7FF0000000000000)
    y = np.where(special, x, x + np.uint64(0x8000)) & np.uint64(0xFFFFFFFFFFFF0000)
    return y.view(np.complex128).reshape(a.shape)
