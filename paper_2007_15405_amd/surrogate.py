"""Training data for the learned surrogate from the batched solver, and its training.

One sample per capsule-pair run (``synth.batch_instances``): inputs (separation L / R,
log10 of the shear modulus, film height above the repulsive plane / 2R, contact angle in
degrees; 90 without a wetting offset), outputs after ``steps`` steps of the batched
solver: the lateral capillary force (each anchored capsule's anchor force, which at rest
balances the force of the fluid, projected on the unit vector pointing away from the other
capsule in the film plane, averaged over the two; negative = attraction) and the meniscus
deformation (the meniscus height at the column midway between the capsules minus the
median height along the box edge farthest from the pair axis).  Everything here reads the
library's observables; the solver and the network run in the library's kernels.
"""
from __future__ import annotations

import numpy as np

import synth

from .lbm import Batch, Sim, Surrogate

RADIUS = 10.0
PLANE = 10.5          # repulsive plane of the batch instances (0.5 + 10 above the wall)
CONTACT = 2.4         # L / R below which the pair comes into contact during the run: the
                      # force then grows by an order of magnitude; such pairs are left to
                      # the solver (outside the surrogate's domain)


def pair_inputs(inst: dict, angles=None) -> np.ndarray:
    """(L / R, log10 ks, film above the plane / 2R, contact angle in degrees); the angle
    of the capsules' wetting offset is interpolated in ``angles`` = (offsets, angles) of
    ``contact_angle_table`` (90 for a neutral capsule)."""
    film_above_plane = inst["film_height"] + 0.5 - PLANE
    w = inst.get("wet_drho", 0.0)
    if angles is None and w != 0.0:
        raise ValueError("a wetting capsule needs the contact-angle table (contact_angle_table)")
    theta = 90.0 if angles is None else float(np.interp(w, *angles))
    return np.array([inst["L"] / RADIUS, np.log10(inst["ks"]),
                     film_above_plane / (2 * RADIUS), theta])


# --------------------------------------------------------------------------------------
# Contact angle of a wetting offset: a sessile drop on the substrate, run by the library
# --------------------------------------------------------------------------------------

DROP_BOX = (80, 3, 40)      # quasi-two-dimensional: periodic in x and y, wall at z = 0
WALL_PLANE = 0.5            # half-way bounce-back between the solid layer and z = 1


def drop_density(radius: float) -> np.ndarray:
    """Initial densities [2][nz][ny][nx] of a half-cylinder of component 0 (radius
    ``radius``) resting on the wall, component 1 around it."""
    nx, ny, nz = DROP_BOX
    x, z = np.meshgrid(np.arange(nx), np.arange(nz))
    inside = ((x - (nx - 1) / 2) ** 2 + (z - WALL_PLANE) ** 2 < radius * radius) & (z >= 1)
    rho = np.empty((2, nz, ny, nx))
    rho[0] = np.where(inside, 0.72, 0.036)[:, None, :]
    rho[1] = np.where(inside, 0.036, 0.72)[:, None, :]
    return rho


def contact_angle(r0, r1, wall: float = WALL_PLANE) -> float:
    """Contact angle (degrees, inside component 0) of a drop on the wall from density
    planes [nz][nx]: a least-squares circle through the points where the densities are
    equal (interpolated along rows and columns, 3 or more sites above the wall), met
    with the wall plane."""
    phi = np.asarray(r0, np.float64) - np.asarray(r1, np.float64)
    nz = phi.shape[0]
    zs = np.arange(3, nz // 2)
    a, b = phi[zs, :-1], phi[zs, 1:]
    zi, xi = np.nonzero(a * b < 0)
    px = [xi + a[zi, xi] / (a[zi, xi] - b[zi, xi])]
    pz = [zs[zi].astype(np.float64)]
    a, b = phi[zs, :], phi[zs + 1, :]
    zi, xi = np.nonzero(a * b < 0)
    px.append(xi.astype(np.float64))
    pz.append(zs[zi] + a[zi, xi] / (a[zi, xi] - b[zi, xi]))
    x, z = np.concatenate(px), np.concatenate(pz)
    M = np.column_stack([2 * x, 2 * z, np.ones_like(x)])
    (xc, zc, c), *_ = np.linalg.lstsq(M, x * x + z * z, rcond=None)
    rc = np.sqrt(c + xc * xc + zc * zc)
    return float(np.degrees(np.arccos(np.clip((wall - zc) / rc, -1.0, 1.0))))


def wall_contact_angle(drho: float, radius: float = 14.0, steps: int = 4000,
                       storage: str = "f32") -> float:
    """Contact angle of the wetting offset ``drho``: a sessile drop on a wall with that
    offset, run ``steps`` steps on the GPU and measured with ``contact_angle``."""
    nx, ny, nz = DROP_BOX
    cfg = synth.workload("pf", capsules=[], wall_z0=1, nx=nx, ny=ny, nz=nz, init_mode=2,
                         init_rho_array=drop_density(radius), wall_drho=float(drho))
    sim = Sim(cfg, storage=storage)
    sim.step(steps)
    r = sim.observables(rho=True, capsules=False)["rho"][:, :, ny // 2, :]
    sim.close()
    return contact_angle(r[0], r[1])


def contact_angle_table(drhos) -> tuple:
    """(offsets, angles) for interpolation: the wall contact angle of each offset.  A
    capsule surface takes the offset through the same substitution as the wall, so its
    contact angle is read from this table."""
    d = np.sort(np.asarray(drhos, np.float64))
    return d, np.array([wall_contact_angle(v) for v in d])


def run_pairs(instances: list, steps: int, average: int = 0, every: int = 200,
              storage: str = "f32", parts: int = 3, angles=None):
    """Run the instances with one batch (stacked by box size) and return
    (inputs [n][4], outputs [n][2]) in the order of ``instances``; the outputs are
    averaged over samples taken every ``every`` steps during the last ``average`` steps
    (0: the final state only)."""
    angles = _angles_for(instances) if angles is None else angles
    groups = synth.batch_groups(instances)
    sims = [Sim(g, storage=storage, meshes=synth.capsule_meshes(g["capsules"])) for g in groups]
    bt = Batch(sims, tile=13, zchunk=16, parts=parts)
    X = np.array([pair_inputs(i, angles) for i in instances])
    Y = np.zeros((len(instances), 2))
    nsamp = max(1, average // every) if average else 1
    bt.step(steps - (nsamp - 1) * every if average else steps)
    for j in range(nsamp):
        if j:
            bt.step(every)
        bt.sync()
        Y += _outputs(groups, sims, len(instances)) / nsamp
    bt.close()
    for x in sims:
        x.close()
    return X, Y


def _outputs(groups, sims, n):
    Y = np.zeros((n, 2))
    for g, sim in zip(groups, sims):
        ob = sim.observables(meniscus=True)
        men = ob["meniscus"].reshape(-1, g["ny"], g["nx"])
        for s, k in enumerate(g["instances"]):
            c = [ob["capsules"][2 * s + j] for j in range(2)]
            d = c[0]["centroid"][:2] - c[1]["centroid"][:2]
            e = d / np.linalg.norm(d)
            Y[k, 0] = 0.5 * (c[0]["f_anchor"][:2] @ e - c[1]["f_anchor"][:2] @ e)
            mid = 0.5 * (c[0]["centroid"][:2] + c[1]["centroid"][:2])
            h = men[s]
            hm = h[int(round(mid[1])) % g["ny"], int(round(mid[0])) % g["nx"]]
            edge = h[0][~np.isnan(h[0])]
            Y[k, 1] = hm - np.median(edge) if edge.size else np.nan
    return Y


def _angles_for(instances):
    wmax = max(abs(i.get("wet_drho", 0.0)) for i in instances)
    return contact_angle_table(np.linspace(-wmax, wmax, 5)) if wmax > 0 else None


def in_hull(points, queries, tol: float = 1e-9) -> np.ndarray:
    """Exact membership of each query in the convex hull of ``points``: the query is a
    convex combination of the points, lambda >= 0, sum lambda = 1, sum lambda p = q, a
    linear feasibility problem solved with scipy's HiGHS.  Coordinates are scaled to
    unit spread first; queries outside the points' bounding box are outside without a
    solve."""
    from scipy.optimize import linprog
    P = np.asarray(points, np.float64)
    Q = np.atleast_2d(np.asarray(queries, np.float64))
    lo, hi = P.min(0), P.max(0)
    span = np.where(hi > lo, hi - lo, 1.0)
    Ps, Qs = (P - lo) / span, (Q - lo) / span
    inbox = np.all((Qs >= -tol) & (Qs <= 1 + tol), axis=1)
    A = np.vstack([Ps.T, np.ones(len(Ps))])
    out = np.zeros(len(Q), bool)
    for k in np.nonzero(inbox)[0]:
        r = linprog(np.zeros(len(Ps)), A_eq=A, b_eq=np.append(Qs[k], 1.0), bounds=(0, None),
                    method="highs")
        out[k] = r.status == 0
    return out


class Fitted:
    """A trained surrogate with the normalisation of its inputs and outputs and its
    training inputs, whose convex hull (with separations of at least CONTACT radii) is
    its domain; queries outside go to the solver."""

    def __init__(self, net: Surrogate, xm, xs, ym, ys, lo, hi, train_x=None):
        self.net, self.xm, self.xs, self.ym, self.ys = net, xm, xs, ym, ys
        self.lo, self.hi = lo, hi
        self.train_x = train_x

    def inside(self, X) -> np.ndarray:
        X = np.atleast_2d(np.asarray(X, np.float64))
        ok = X[:, 0] >= CONTACT
        if self.train_x is None:
            return ok & np.all((X >= self.lo) & (X <= self.hi), axis=1)
        return ok & in_hull(self.train_x, X)

    def predict(self, X) -> np.ndarray:
        x = (np.asarray(X, np.float64) - self.xm) / self.xs
        return self.net.predict(x.astype(np.float32)) * self.ys + self.ym


def in_domain(X) -> np.ndarray:
    """Samples the surrogate is trained on: pairs that stay out of contact."""
    return np.asarray(X)[:, 0] >= CONTACT


def fit(X, Y, steps: int = 500, lr: float = 1e-3, seed: int = synth.SEED,
        max_queries: int = 65536) -> Fitted:
    """Train on (X, Y), columns normalised to zero mean and unit variance (constant
    columns left centred).  Full-batch Adam; few steps, since a few hundred samples of
    solver output are fitted to their noise level quickly and then overfitted.  The
    network takes up to max_queries inputs per prediction call."""
    X, Y = np.asarray(X, np.float64), np.asarray(Y, np.float64)
    xm, xs = X.mean(0), X.std(0)
    xs[xs == 0] = 1.0
    ym, ys = Y.mean(0), Y.std(0)
    ys[ys == 0] = 1.0
    net = Surrogate(synth.surrogate_init(seed), max(len(X), max_queries))
    net.set_data(((X - xm) / xs).astype(np.float32), ((Y - ym) / ys).astype(np.float32))
    net.train(steps, lr)
    return Fitted(net, xm, xs, ym, ys, X.min(0), X.max(0), X)


def predict_or_solve(fitted: Fitted, instances: list, steps: int, average: int = 0,
                     every: int = 200, angles=None):
    """Outputs of capsule-pair instances: the network's prediction where the pair's inputs
    lie in the surrogate's domain (``Fitted.inside``), the batched solver's run
    (``run_pairs``) elsewhere.  Returns (inputs, outputs, solved mask)."""
    angles = _angles_for(instances) if angles is None else angles
    X = np.array([pair_inputs(i, angles) for i in instances])
    Y = np.zeros((len(instances), 2))
    inside = fitted.inside(X)
    if inside.any():
        Y[inside] = fitted.predict(X[inside])
    out = np.nonzero(~inside)[0]
    if len(out):
        _, Ys = run_pairs([instances[k] for k in out], steps, average, every, angles=angles)
        Y[out] = Ys
    return X, Y, ~inside


# --------------------------------------------------------------------------------------
# Cluster evolution driven by the network, and its analysis
# --------------------------------------------------------------------------------------


def cluster_params(fitted: Fitted, features, box: float, radius: float = RADIUS,
                   k_contact: float = 0.05, mobility: float = 1.0) -> dict:
    """Arguments of ``Surrogate.cluster`` for a trained surrogate: the network is used
    from the contact separation up to the largest training separation; beyond that the
    capillary force is taken as zero, closer the pair repels with ``k_contact`` per
    radius of overlap (the solver is the fallback for contact, not a per-step option in
    a many-capsule run)."""
    return dict(box=float(box), radius=float(radius), features=[float(v) for v in features],
                in_mean=fitted.xm, in_scale=fitted.xs, out_mean=fitted.ym,
                out_scale=fitted.ys, r_contact=CONTACT, r_cut=float(fitted.hi[0]),
                k_contact=float(k_contact), mobility=float(mobility))


def _pairs_within(xy, box: float, cutoff: float):
    p = np.asarray(xy, np.float64)
    d = p[:, None, :] - p[None, :, :]
    d -= box * np.round(d / box)
    r = np.sqrt((d * d).sum(-1))
    i, j = np.nonzero(np.triu(r <= cutoff, 1))
    return i, j, r


def cluster_labels(xy, box: float, cutoff: float) -> np.ndarray:
    """Cluster of each capsule: centres at most ``cutoff`` apart (minimum image) are in
    one cluster, transitively (union-find with path halving and union by size); each
    cluster is labelled by its smallest member."""
    n = len(xy)
    parent = np.arange(n)
    size = np.ones(n, int)

    def root(a):
        while parent[a] != a:
            parent[a] = parent[parent[a]]
            a = parent[a]
        return a

    i, j, _ = _pairs_within(xy, box, cutoff)
    for a, b in zip(i.tolist(), j.tolist()):
        ra, rb = root(a), root(b)
        if ra != rb:
            if size[ra] < size[rb]:
                ra, rb = rb, ra
            parent[rb] = ra
            size[ra] += size[rb]
    roots = np.array([root(a) for a in range(n)])
    first = {}
    for a in range(n):
        first.setdefault(roots[a], a)
    return np.array([first[r] for r in roots])


def cluster_sizes(labels) -> tuple:
    """(mean, largest) number of capsules per cluster, single capsules counted as
    clusters of one."""
    counts = np.unique(np.asarray(labels), return_counts=True)[1]
    return float(counts.mean()), int(counts.max())


def rdf(xy, box: float, dr: float, r_max: float):
    """Radial distribution function of the centres, g(r) = (A / N) n(r) / (2 pi r dr):
    shell centres and g over shells of width ``dr`` below ``r_max`` (minimum image)."""
    n = len(xy)
    _, _, r = _pairs_within(xy, box, 0.0)
    nb = int(r_max / dr)
    off = r[~np.eye(n, dtype=bool)]
    count = np.bincount(np.minimum((off // dr).astype(int), nb), minlength=nb + 1)[:nb]
    rk = (np.arange(nb) + 0.5) * dr
    return rk, (box * box / n) * (count / n) / (2 * np.pi * rk * dr)


def evolve(fitted: Fitted, xy, steps: int, every: int, features, box: float,
           radius: float = RADIUS, k_contact: float = 0.05, mobility: float = 1.0,
           delta0: float = 1.0):
    """Run the cluster evolution for ``steps`` steps on the GPU, sampling every ``every``
    steps: returns the final positions and a list of (step, mean cluster size, largest
    cluster size) with clusters of centres at most d + delta0 apart, d the in-plane
    contact separation (CONTACT radii: the closest approach of two capsules in the
    solver's pair runs, the reduced model's particle diameter in the plane)."""
    cp = cluster_params(fitted, features, box, radius, k_contact, mobility)
    p = np.asarray(xy, np.float32)
    cut = CONTACT * radius + delta0
    hist = [(0, *cluster_sizes(cluster_labels(p, box, cut)))]
    done = 0
    while done < steps:
        k = min(every, steps - done)
        p = fitted.net.cluster(p, k, **cp)
        done += k
        hist.append((done, *cluster_sizes(cluster_labels(p, box, cut))))
    return p, hist
