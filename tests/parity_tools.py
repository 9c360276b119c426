"""Comparison helpers of the GPU parity tests (no arithmetic of the method).

``rel_l2`` is the per-component relative L2 norm of the density difference.
``site_check`` bounds the error of every single site: max |rho_gpu - rho_ref| over the
sites, divided by the largest reference density of that component, and reports the
worst site with its label and its distance from the nearest wall plane, so that an error
localised at a membrane- or wall-adjacent site is seen even where the norm hides it."""
import sys

import numpy as np


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel_l2(a, b):
    return [float(np.linalg.norm(a[c] - b[c]) / np.linalg.norm(b[c])) for c in range(2)]


def site_errors(a, b, labels=None, wall=True, lz=None):
    """Per component: (max |a - b| / max |b|, worst site (z, y, x), its label, its distance
    from the nearest wall plane of its slab, or None without a wall)."""
    out = []
    nz = a.shape[1]
    lz = lz or nz
    for c in range(2):
        d = np.abs(np.asarray(a[c], np.float64) - np.asarray(b[c], np.float64))
        k = np.unravel_index(int(np.argmax(d)), d.shape)
        scale = float(np.abs(b[c]).max())
        lab = int(labels[k]) if labels is not None else None
        zs = k[0] % lz
        wd = min(zs - 0.5, lz - 0.5 - zs) if wall else None
        out.append((float(d[k]) / scale, tuple(int(v) for v in k), lab, wd))
    return out


def site_check(a, b, bound, what="", labels=None, wall=True, lz=None):
    """Assert the per-site bound on both components; print the worst sites."""
    errs = site_errors(a, b, labels, wall, lz)
    for c, (e, k, lab, wd) in enumerate(errs):
        say(f"{what} component {c}: max site error {e:.3e} (of max rho) at (z, y, x) = {k}, "
            f"label {lab}, wall distance {wd}")
    worst = max(e[0] for e in errs)
    assert worst <= bound, (what, errs)
    return worst
