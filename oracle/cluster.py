"""CPU reference of the surrogate-driven cluster evolution and of its analysis (test
infrastructure only: imported by tests/, never by the library).

Many capsules at a flat interface (section "Clustering of soft particles in a thin film")
are reduced to their centres of mass in the plane of the interface, in a periodic square
of side `box`.  Each pair interacts through the lateral capillary force the learned
surrogate predicts for its separation (oracle/mlp.py, mixed precision); the motion is
overdamped, p_i <- p_i + mobility * sum_j f(r_ij) e_ij with e_ij the unit vector from j
to i (minimum image).  Pairs closer than r_contact radii are outside the surrogate's
domain and repel with k_contact (r_contact - r / R); pairs farther than r_cut radii
exert no force.

Precision: the separations, the network's inputs, the forces and the update are float64,
written as defined (minimum image d - box rint(d / box), inputs (raw - mean) / scale);
the network is oracle/mlp.py's mixed mode, which rounds its inputs to bfloat16 as the
kernels do; the positions are stored as float32 between steps.  A kernel that forms the
inputs in float32 may round an input lying within a few float32 units of a bfloat16
rounding boundary to the other neighbour: ``input_flip_allowance`` bounds what that can
change, from the network itself.

Analysis: clusters (capsules in one cluster when their centres are at most `cutoff`
apart, transitively; the criterion of the clustering section), cluster sizes, and the
radial distribution function g(r) = (A / N) n(r) / (2 pi r dr) of the same section, with
n(r) the mean number of other centres in the shell [r - dr/2, r + dr/2) around a centre.
"""
from collections import deque

import numpy as np

from oracle import mlp

F32 = np.float32


def _separations(p, box, rows=None):
    """d[i, j] = p_i - p_j (minimum image, float64) and |d| for the capsules i of ``rows``
    (all by default)."""
    p = np.asarray(p, F32).astype(np.float64)
    b = float(F32(box))
    q = p if rows is None else p[rows]
    d = q[:, None, :] - p[None, :, :]
    d = d - b * np.rint(d / b)
    r = np.sqrt(d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1])
    return d, r


def _inputs(r, c):
    """Network inputs (raw - mean) / scale of every pair, float64: the separation in radii
    and the three fixed features."""
    raw = np.empty(r.shape + (4,))
    raw[..., 0] = r / float(F32(c["radius"]))
    raw[..., 1:] = np.asarray(c["features"], F32).astype(np.float64)
    xm = np.asarray(c["in_mean"], F32).astype(np.float64)
    xs = np.asarray(c["in_scale"], F32).astype(np.float64)
    return raw[..., 0], (raw - xm) / xs


def _pair_forces(theta, p, c, rows):
    """Pair force magnitudes f [m][n], separations d [m][n][2], |d| and the mask of
    interacting pairs for the capsules of ``rows``."""
    n = len(p)
    d, r = _separations(p, c["box"], rows)
    m = len(rows)
    rr, x = _inputs(r, c)
    y, _ = mlp.forward(theta, x.reshape(-1, 4), mixed=True)
    f_net = y[:, 0].reshape(m, n) * float(c["out_scale"][0]) + float(c["out_mean"][0])
    rc, rcut = float(F32(c["r_contact"])), float(F32(c["r_cut"]))
    f = np.where(rr < rc, float(c["k_contact"]) * (rc - rr), f_net)
    act = (r > 0) & (rr <= rcut) & (rows[:, None] != np.arange(n)[None, :])
    return f, d, r, act


def step(theta, p, c, rows=None):
    """One overdamped step of all capsules; c: dict with box, radius, features (raw log10
    ks, film / 2R, contact angle), in_mean, in_scale, out_mean, out_scale, r_contact,
    r_cut, k_contact, mobility.  Returns the new float32 positions (of the capsules in
    ``rows`` only, if given)."""
    p = np.asarray(p, F32)
    n = len(p)
    rows = np.arange(n) if rows is None else np.asarray(rows)
    f, d, r, act = _pair_forces(theta, p, c, rows)
    w = np.where(act, f / np.where(act, r, 1.0), 0.0)
    force = np.einsum("ij,ijk->ik", w, d)
    q = p[rows].astype(np.float64) + float(c["mobility"]) * force
    box = float(F32(c["box"]))
    q = q - box * np.floor(q / box)
    return q.astype(F32)


def pair_forces_abs(theta, p, c, rows=None):
    """sum_j |f(r_ij)| per capsule (of ``rows``) over the interacting partners: the scale
    of the rounding error of the summed force."""
    p = np.asarray(p, F32)
    rows = np.arange(len(p)) if rows is None else np.asarray(rows)
    f, _, _, act = _pair_forces(theta, p, c, rows)
    return np.where(act, np.abs(f), 0.0).sum(1)


def input_flip_allowance(theta, p, c, rows=None, ulps=32):
    """Per capsule (of ``rows``): the largest change of its summed pair force that rounding
    the separation input to the other bfloat16 neighbour can make.  A pair qualifies when
    its float64 input lies within ``ulps`` float32 units (of the larger of |rr| and
    |mean|, divided by |scale|) of a point where the float32-then-bfloat16 rounding changes
    value; its allowance is |f(x - t) - f(x + t)| of the network at the two ends, t that
    distance.  The fixed features must not lie that close to a rounding point (checked:
    ValueError), unless they equal their mean, which gives exactly 0 in any precision."""
    p = np.asarray(p, F32)
    n = len(p)
    rows = np.arange(n) if rows is None else np.asarray(rows)
    _, r = _separations(p, c["box"], rows)
    rr, x = _inputs(r, c)
    xm = np.asarray(c["in_mean"], F32).astype(np.float64)
    xs = np.abs(np.asarray(c["in_scale"], F32).astype(np.float64))
    raw_abs = np.concatenate([[0.0], np.abs(np.asarray(c["features"], F32))])
    feats = np.asarray(c["features"], F32).astype(np.float64)
    for k in range(1, 4):
        if feats[k - 1] == xm[k]:
            continue                    # (raw - mean) is exactly 0 in any precision
        t = ulps * 2.0 ** -24 * max(raw_abs[k], abs(xm[k])) / xs[k]
        v = x[0, 0, k] if x.size else 0.0
        if mlp.bf16(v - t) != mlp.bf16(v + t):
            raise ValueError(f"fixed input {k} lies within float32 rounding of a bfloat16 boundary")
    rc, rcut = float(F32(c["r_contact"])), float(F32(c["r_cut"]))
    net = (r > 0) & (rr >= rc) & (rr <= rcut) & (rows[:, None] != np.arange(n)[None, :])
    t0 = ulps * 2.0 ** -24 * np.maximum(rr, abs(xm[0])) / xs[0]
    x0 = x[..., 0]
    near = net & (mlp.bf16(x0 - t0) != mlp.bf16(x0 + t0))
    out = np.zeros(len(rows))
    if not near.any():
        return out
    xa = x[near].copy()
    xb = x[near].copy()
    xa[:, 0] -= t0[near]
    xb[:, 0] += t0[near]
    ya, _ = mlp.forward(theta, xa, mixed=True)
    yb, _ = mlp.forward(theta, xb, mixed=True)
    dy = np.abs(ya[:, 0] - yb[:, 0]) * abs(float(c["out_scale"][0]))
    ii = np.nonzero(near)[0]
    np.add.at(out, ii, dy)
    return out


def network_partners(p, c, rows=None):
    """Number of partners of each capsule (of ``rows``) whose force comes from the network
    (separation in [r_contact, r_cut] radii)."""
    p = np.asarray(p, F32)
    n = len(p)
    rows = np.arange(n) if rows is None else np.asarray(rows)
    _, r = _separations(p, c["box"], rows)
    rr = r / float(F32(c["radius"]))
    act = (r > 0) & (rr <= float(F32(c["r_cut"]))) & (rr >= float(F32(c["r_contact"]))) & \
        (rows[:, None] != np.arange(n)[None, :])
    return act.sum(1)


def clusters(p, box, cutoff):
    """Cluster index per capsule: connected components of the graph joining centres at
    most `cutoff` apart (minimum image), by breadth-first search in float64; clusters
    numbered by their smallest member."""
    p = np.asarray(p, np.float64)
    n = len(p)
    label = [-1] * n
    for s in range(n):
        if label[s] >= 0:
            continue
        label[s] = s
        todo = deque([s])
        while todo:
            i = todo.popleft()
            for j in range(n):
                if label[j] >= 0:
                    continue
                dx = p[i, 0] - p[j, 0]
                dy = p[i, 1] - p[j, 1]
                dx -= box * round(dx / box)
                dy -= box * round(dy / box)
                if (dx * dx + dy * dy) ** 0.5 <= cutoff:
                    label[j] = s
                    todo.append(j)
    return np.array(label)


def rdf(p, box, dr, r_max):
    """Shell centres r_k = (k + 1/2) dr below r_max and g(r_k) = (A / N) n(r_k) /
    (2 pi r_k dr), n the mean over centres of the others in the shell (minimum image)."""
    p = np.asarray(p, np.float64)
    n = len(p)
    nb = int(r_max / dr)
    count = np.zeros(nb)
    for i in range(n):
        for j in range(n):
            if i == j:
                continue
            dx = p[i, 0] - p[j, 0]
            dy = p[i, 1] - p[j, 1]
            dx -= box * round(dx / box)
            dy -= box * round(dy / box)
            k = int((dx * dx + dy * dy) ** 0.5 // dr)
            if k < nb:
                count[k] += 1
    rk = (np.arange(nb) + 0.5) * dr
    return rk, (box * box / n) * (count / n) / (2 * np.pi * rk * dr)
