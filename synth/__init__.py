"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the benchmark.

This module holds no arithmetic of the simulation method itself: it only produces
inputs (lattice sizes, initial density arrays with seeded noise, capsule meshes and
capsule placements).  Both the CPU oracle and the HIP library receive the same
arrays from here, so their initial states are bit-identical.

Workloads (lattice units, dx = dt = 1):

* ``c1``   32^3 box, wall at z=0, two-component mixture rho^c = 1*(1 + 0.02*xi),
           xi uniform in [-1, 1), one capsule R=6 (icosphere level 3, 1280
           triangles), ks=0.01, C=9, 200 steps.
* ``pf``   the same box as ``c1`` with a flat film (film layers 1..10, one mixed
           layer, gas above) and the same capsule centred at z=10, straddling
           the interface; 1000 steps.  Non-chaotic parity geometry.
* ``c2``   128x128x64 film-drying geometry: film 12 lu above the wall, repulsive
           plane 10 lu above the wall, two capsules R=10 (level 4, 5120 triangles)
           at separation 3R, anchored, ks in {0.005, 0.05, 5.0}.
* ``c3``   256x256x96 film with 16 capsules R=10 at seeded random non-overlapping
           positions (periodic centre distance >= 2R + delta0 + 1), ks=0.05.
* batch    64 independent capsule-pair boxes from 64x48x40 to 128x96x48
           (``batch_instances``), stacked by box size into slabs (``batch_groups``).

The film layout follows the paper's setup (Section 3.2): majority density 0.7,
minority 0.04, and one interface layer where both components have density 0.3.
"""
from __future__ import annotations

import copy
import math
from typing import Dict, List, Tuple

import numpy as np

SEED = 15405

# --------------------------------------------------------------------------------------
# Icosphere meshes
# --------------------------------------------------------------------------------------


def _icosahedron() -> Tuple[np.ndarray, List[Tuple[int, int, int]]]:
    t = (1.0 + math.sqrt(5.0)) / 2.0
    v = [(-1, t, 0), (1, t, 0), (-1, -t, 0), (1, -t, 0),
         (0, -1, t), (0, 1, t), (0, -1, -t), (0, 1, -t),
         (t, 0, -1), (t, 0, 1), (-t, 0, -1), (-t, 0, 1)]
    f = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11),
         (1, 5, 9), (5, 11, 4), (11, 10, 2), (10, 7, 6), (7, 1, 8),
         (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8), (3, 8, 9),
         (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    verts = np.array(v, dtype=np.float64)
    verts /= np.linalg.norm(verts, axis=1, keepdims=True)
    return verts, f


def icosphere(level: int, radius: float = 1.0,
              center=(0.0, 0.0, 0.0)) -> Tuple[np.ndarray, np.ndarray]:
    """Geodesic sphere: the icosahedron with every edge split at its midpoint
    ``level`` times, each new vertex projected back onto the sphere.

    Returns ``(nodes, tris)``: nodes (n, 3) float64, tris (m, 3) int32 with an
    outward counter-clockwise orientation.  Level L has 10*4^L + 2 nodes and
    20*4^L triangles (level 3: 642/1280, level 4: 2562/5120).
    """
    verts, faces = _icosahedron()
    vlist = [tuple(p) for p in verts]
    for _ in range(level):
        cache: Dict[Tuple[int, int], int] = {}
        new_faces = []

        def mid(a: int, b: int) -> int:
            key = (a, b) if a < b else (b, a)
            if key in cache:
                return cache[key]
            p = np.add(vlist[a], vlist[b]) * 0.5
            p = p / np.linalg.norm(p)
            vlist.append(tuple(p))
            cache[key] = len(vlist) - 1
            return cache[key]

        for (a, b, c) in faces:
            ab, bc, ca = mid(a, b), mid(b, c), mid(c, a)
            new_faces += [(a, ab, ca), (b, bc, ab), (c, ca, bc), (ab, bc, ca)]
        faces = new_faces
    nodes = np.array(vlist, dtype=np.float64)
    tris = np.array(faces, dtype=np.int32)
    # outward orientation: normal . centroid > 0
    p0, p1, p2 = nodes[tris[:, 0]], nodes[tris[:, 1]], nodes[tris[:, 2]]
    nrm = np.cross(p1 - p0, p2 - p0)
    flip = np.einsum("ij,ij->i", nrm, p0 + p1 + p2) < 0
    tris[flip] = tris[flip][:, [0, 2, 1]]
    nodes = nodes * float(radius) + np.asarray(center, dtype=np.float64)
    return np.ascontiguousarray(nodes), np.ascontiguousarray(tris)


def level_for_triangles(n_tri: int) -> int:
    lev = int(round(math.log(n_tri / 20.0, 4)))
    if 20 * 4 ** lev != n_tri:
        raise ValueError(f"{n_tri} is not 20*4^L")
    return lev


# --------------------------------------------------------------------------------------
# Initial density arrays
# --------------------------------------------------------------------------------------


def noise_rho(nx: int, ny: int, nz: int, base=(1.0, 1.0), amp: float = 0.02,
              seed: int = SEED) -> np.ndarray:
    """rho^c(x) = base_c * (1 + amp * xi), xi i.i.d. uniform in [-1, 1).

    Layout [2][nz][ny][nx], float64, C-contiguous."""
    rng = np.random.default_rng(seed)
    xi = rng.uniform(-1.0, 1.0, size=(2, nz, ny, nx))
    b = np.asarray(base, dtype=np.float64).reshape(2, 1, 1, 1)
    return np.ascontiguousarray(b * (1.0 + amp * xi))


# --------------------------------------------------------------------------------------
# Capsule placement
# --------------------------------------------------------------------------------------


def place_capsules(n: int, radius: float, nx: int, ny: int, z: float,
                   min_dist: float, seed: int = SEED, max_tries: int = 200000):
    """Seeded rejection sampling of ``n`` capsule centres, x and y uniform in the
    periodic box, every periodic centre distance >= ``min_dist``."""
    rng = np.random.default_rng(seed)
    out: List[Tuple[float, float, float]] = []
    tries = 0
    while len(out) < n:
        tries += 1
        if tries > max_tries:
            raise RuntimeError("could not place capsules")
        x, y = rng.uniform(0.0, nx), rng.uniform(0.0, ny)
        ok = True
        for (px, py, _) in out:
            dx = abs(x - px); dx = min(dx, nx - dx)
            dy = abs(y - py); dy = min(dy, ny - dy)
            if dx * dx + dy * dy < min_dist * min_dist:
                ok = False
                break
        if ok:
            out.append((float(x), float(y), float(z)))
    return out


# --------------------------------------------------------------------------------------
# Workloads
# --------------------------------------------------------------------------------------

_BASE = dict(
    nx=32, ny=32, nz=32, wall_z0=1,
    tau=[1.0, 1.0], G=3.6, rho0=1.0, sc_norm=1.0,
    body_force=[0.0, 0.0, 0.0], wall_drho=0.0,
    init_mode=0, init_rho=[1.0, 1.0],
    film_height=0.0, rho_maj=0.7, rho_min=0.04, rho_iface=0.3,
    init_rho_array=None,
    hertz_xi=1.5, hertz_delta0=1.5, plane_dz=0.0,
    slab_nz=0, slab_film_height=None,
    coupling=0, node_mass=25.0,
    capsules=[], steps=1,
)


def capsule(center, radius, n_tri, ks, C=9.0, kb=0.0, kv=0.0, wet_drho=0.0,
            anchor_k=0.0) -> dict:
    return dict(center=[float(c) for c in center], radius=float(radius),
                n_tri=int(n_tri), ks=float(ks), C=float(C), kb=float(kb),
                kv=float(kv), wet_drho=float(wet_drho), anchor_k=float(anchor_k))


def workload(name: str, **over) -> dict:
    """Return a configuration dict; keyword overrides replace top-level keys."""
    cfg = copy.deepcopy(_BASE)
    if name == "c1":
        cfg.update(nx=32, ny=32, nz=32, wall_z0=1, init_mode=2, steps=200,
                   init_rho_array=noise_rho(32, 32, 32, (1.0, 1.0), 0.02, SEED),
                   capsules=[capsule((16.0, 16.0, 16.0), 6.0, 1280, 0.01)])
    elif name == "pf":
        cfg.update(nx=32, ny=32, nz=32, wall_z0=1, init_mode=1, film_height=10.0,
                   steps=1000,
                   capsules=[capsule((16.0, 16.0, 10.0), 6.0, 1280, 0.01)])
    elif name == "c2":
        ks = over.pop("ks", 0.05)
        cfg.update(nx=128, ny=128, nz=64, wall_z0=1, init_mode=1, film_height=12.0,
                   plane_dz=10.0, steps=20000,
                   capsules=[capsule((49.0, 64.0, 22.0), 10.0, 5120, ks, anchor_k=1.0),
                             capsule((79.0, 64.0, 22.0), 10.0, 5120, ks, anchor_k=1.0)])
    elif name == "c3":
        R = 10.0
        cen = place_capsules(16, R, 256, 256, 22.0, 2 * R + 1.5 + 1.0, SEED)
        cfg.update(nx=256, ny=256, nz=96, wall_z0=1, init_mode=1, film_height=12.0,
                   plane_dz=10.0, steps=10000,
                   capsules=[capsule(c, R, 5120, 0.05, anchor_k=1.0) for c in cen])
    else:
        raise KeyError(name)
    for k, v in over.items():
        if k not in cfg:
            raise KeyError(k)
        cfg[k] = v
    return cfg


def batch_instances(n: int = 64, seed: int = SEED, radius: float = 10.0,
                    n_tri: int = 5120, ks_max: float = 0.2, wet_max: float = 0.0) -> List[dict]:
    """Independent capsule-pair runs for the batched form: separation L uniform in
    [2.2 R, 6 R], shear modulus log-uniform in [0.002, ks_max], film height (above the
    repulsive plane) uniform in [0.4, 0.9] of the capsule diameter.  ks_max = 0.2: with
    the explicit immersed-boundary coupling (nodes move with the fluid, no node inertia)
    a R = 10 capsule of 5120 triangles diverges from ks ~ 0.3 on, in the oracle and the
    library alike; the paper's stiffer capsules (up to 5) rely on its own coupling.  Box
    Lx = clamp(16 * ceil((2 L + 2 R) / 16), 64, 128), Ly = 3 Lx / 4, Lz 40 or 48; wall at
    z = 0, repulsive plane 10 lu above it, the two anchored capsules resting delta0
    above the plane on the x axis of the box, centred in x and y.  wet_max > 0: both
    capsules of an instance get the wetting offset wet_drho uniform in [-wet_max,
    wet_max] (drawn after the other parameters, so wet_max = 0 leaves every other draw
    as it was)."""
    rng = np.random.default_rng(seed)
    out = []
    z_plane, delta0 = 0.5 + 10.0, 1.5
    for _ in range(n):
        L = rng.uniform(2.2 * radius, 6.0 * radius)
        ks = float(np.exp(rng.uniform(np.log(0.002), np.log(ks_max))))
        film = rng.uniform(0.4, 0.9) * 2.0 * radius
        lx = int(min(max(16 * math.ceil((2.0 * L + 2.0 * radius) / 16.0), 64), 128))
        ly = 3 * lx // 4
        lz = int(rng.choice([40, 48]))
        wet = float(rng.uniform(-wet_max, wet_max)) if wet_max > 0 else 0.0
        zc = z_plane + delta0 + radius
        caps = [capsule((lx / 2.0 + sgn * L / 2.0, ly / 2.0, zc), radius, n_tri, ks,
                        wet_drho=wet, anchor_k=1.0) for sgn in (-1.0, 1.0)]
        out.append(dict(nx=lx, ny=ly, nz=lz, L=float(L), ks=ks, wet_drho=wet,
                        film_height=float(round(z_plane - 0.5 + film)), capsules=caps))
    return out


def batch_groups(instances: List[dict]) -> List[dict]:
    """Stack the instances of equal box size along z: one workload per (Lx, Ly, Lz) with
    slab_nz = Lz, per-slab film heights and the capsules moved into their slabs.  Each
    group dict also lists the indices of its instances, in slab order."""
    keys = sorted({(i["nx"], i["ny"], i["nz"]) for i in instances})
    groups = []
    for (lx, ly, lz) in keys:
        idx = [k for k, i in enumerate(instances) if (i["nx"], i["ny"], i["nz"]) == (lx, ly, lz)]
        caps, films = [], []
        for s, k in enumerate(idx):
            films.append(instances[k]["film_height"])
            for c in instances[k]["capsules"]:
                c2 = dict(c)
                c2["center"] = [c["center"][0], c["center"][1], c["center"][2] + s * lz]
                caps.append(c2)
        cfg = workload("c2", nx=lx, ny=ly, nz=lz * len(idx), slab_nz=lz, film_height=0.0,
                       slab_film_height=films, capsules=caps, steps=5000)
        cfg["instances"] = idx
        groups.append(cfg)
    return groups


def capsule_mesh(cap: dict) -> Tuple[np.ndarray, np.ndarray]:
    """Icosphere mesh for a capsule dict (radius, centre, triangle count)."""
    return icosphere(level_for_triangles(cap["n_tri"]), cap["radius"], cap["center"])


_UNIT: Dict[int, Tuple[np.ndarray, np.ndarray]] = {}


def capsule_meshes(caps: List[dict]) -> List[Tuple[np.ndarray, np.ndarray]]:
    """``capsule_mesh`` of many capsules from one unit sphere per level (the same
    arithmetic, so the same bits, without rebuilding the sphere each time)."""
    out = []
    for c in caps:
        lev = level_for_triangles(c["n_tri"])
        if lev not in _UNIT:
            _UNIT[lev] = icosphere(lev, 1.0)
        nodes, tris = _UNIT[lev]
        out.append((nodes * float(c["radius"]) + np.asarray(c["center"], dtype=np.float64),
                    tris.copy()))
    return out


def fluid_sites(cfg: dict) -> int:
    """Number of fluid sites (the wall layer z=0 is solid when present)."""
    return cfg["nx"] * cfg["ny"] * (cfg["nz"] - (1 if cfg["wall_z0"] else 0))


def surrogate_init(seed: int = SEED) -> np.ndarray:
    """Initial parameters of the surrogate network 4 -> 64 -> 64 -> 64 -> 2 (layout of
    ``lbm_surrogate_*``): weights N(0, 1 / fan_in), biases 0, float32."""
    rng = np.random.default_rng(seed)
    dims = (4, 64, 64, 64, 2)
    out = []
    for i in range(4):
        out.append(rng.normal(0.0, 1.0 / math.sqrt(dims[i]), dims[i] * dims[i + 1]))
        out.append(np.zeros(dims[i + 1]))
    return np.concatenate(out).astype(np.float32)


def cluster_film(n: int = 512, radius: float = 10.0, packing: float = 0.25,
                 min_sep: float = 2.4, seed: int = SEED):
    """Capsule centres in the plane of a film for the cluster evolution: ``n`` capsules of
    radius ``radius`` in a periodic square whose side gives the area fraction ``packing``
    (n pi R^2 / box^2), placed uniformly at random at least ``min_sep`` radii apart.
    Returns (box, float32 positions [n][2])."""
    box = math.sqrt(n * math.pi * radius * radius / packing)
    pts = place_capsules(n, radius, box, box, 0.0, min_sep * radius, seed)
    return box, np.array([(x, y) for x, y, _ in pts], np.float32)
