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

Precision: the separations (the minimum image through the float32 reciprocal of the box)
and the network's inputs (scaled by the float32 reciprocals of the input scales) are
float32, each operation rounded as written (the inputs are then rounded to bfloat16 inside
the network, so that decision is taken in float32 on both sides); the network is oracle/mlp.py's mixed mode; the forces
and the update are float64; the positions are stored as float32 between steps.

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
    """d[i, j] = p_i - p_j (minimum image) and |d| for the capsules i of ``rows`` (all by
    default), float32 as the operations are written."""
    p = np.asarray(p, F32)
    b = F32(box)
    q = p if rows is None else p[rows]
    d = q[:, None, :] - p[None, :, :]
    d = d - b * np.rint(d * (F32(1) / b))
    r = np.sqrt(d[..., 0] * d[..., 0] + d[..., 1] * d[..., 1])
    return d, r


def step(theta, p, c, rows=None):
    """One overdamped step of all capsules; c: dict with box, radius, features (raw log10
    ks, film / 2R, contact angle), in_mean, in_scale, out_mean, out_scale, r_contact,
    r_cut, k_contact, mobility.  Returns the new float32 positions (of the capsules in
    ``rows`` only, if given)."""
    p = np.asarray(p, F32)
    n = len(p)
    rows = np.arange(n) if rows is None else np.asarray(rows)
    d, r = _separations(p, c["box"], rows)
    m = len(rows)
    rr = r * (F32(1) / F32(c["radius"]))
    xm = np.asarray(c["in_mean"], F32)
    ixs = F32(1) / np.asarray(c["in_scale"], F32)
    raw = np.empty((m, n, 4), F32)
    raw[..., 0] = rr
    raw[..., 1:] = np.asarray(c["features"], F32)
    x = (raw - xm) * ixs
    y, _ = mlp.forward(theta, x.reshape(-1, 4), mixed=True)
    f_net = y[:, 0].reshape(m, n) * float(c["out_scale"][0]) + float(c["out_mean"][0])
    rc, rcut = F32(c["r_contact"]), F32(c["r_cut"])
    f = np.where(rr < rc, float(c["k_contact"]) * (float(rc) - rr.astype(np.float64)), f_net)
    act = (r > 0) & (rr <= rcut) & (rows[:, None] != np.arange(n)[None, :])
    d64, r64 = d.astype(np.float64), np.where(act, r, 1).astype(np.float64)
    w = np.where(act, f / r64, 0.0)
    force = np.einsum("ij,ijk->ik", w, d64)
    q = p[rows].astype(np.float64) + float(c["mobility"]) * force
    box = float(F32(c["box"]))
    q = q - box * np.floor(q / box)
    return q.astype(F32)


def pair_forces_abs(theta, p, c, rows=None):
    """sum_j |f(r_ij)| per capsule (of ``rows``) over the interacting partners: the scale
    of the rounding error of the summed force."""
    p = np.asarray(p, F32)
    n = len(p)
    rows = np.arange(n) if rows is None else np.asarray(rows)
    _, r = _separations(p, c["box"], rows)
    m = len(rows)
    rr = r * (F32(1) / F32(c["radius"]))
    raw = np.empty((m, n, 4), F32)
    raw[..., 0] = rr
    raw[..., 1:] = np.asarray(c["features"], F32)
    x = (raw - np.asarray(c["in_mean"], F32)) * (F32(1) / np.asarray(c["in_scale"], F32))
    y, _ = mlp.forward(theta, x.reshape(-1, 4), mixed=True)
    f_net = y[:, 0].reshape(m, n) * float(c["out_scale"][0]) + float(c["out_mean"][0])
    f = np.where(rr < F32(c["r_contact"]), float(c["k_contact"]) *
                 (float(F32(c["r_contact"])) - rr.astype(np.float64)), f_net)
    act = (r > 0) & (rr <= F32(c["r_cut"])) & (rows[:, None] != np.arange(n)[None, :])
    return np.where(act, np.abs(f), 0.0).sum(1)


def network_partners(p, c, rows=None):
    """Number of partners of each capsule (of ``rows``) whose force comes from the network
    (separation in [r_contact, r_cut] radii)."""
    p = np.asarray(p, F32)
    n = len(p)
    rows = np.arange(n) if rows is None else np.asarray(rows)
    _, r = _separations(p, c["box"], rows)
    rr = r * (F32(1) / F32(c["radius"]))
    act = (r > 0) & (rr <= F32(c["r_cut"])) & (rr >= F32(c["r_contact"])) & \
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
