"""ctypes wrapper of the CPU oracle (``lbmref.c``).

TEST INFRASTRUCTURE ONLY: imported by ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py``.  The product library never imports this module.

``Oracle(cfg)`` takes the same configuration dict as the product binding (see
``synth.workload``); meshes come from ``synth.capsule_mesh``.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))


class Params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("wall_z0", C.c_int32),
        ("tau", C.c_double * 2), ("G", C.c_double), ("rho0", C.c_double),
        ("sc_norm", C.c_double), ("body_force", C.c_double * 3), ("wall_drho", C.c_double),
        ("init_mode", C.c_int32), ("n_threads", C.c_int32), ("init_rho", C.c_double * 2),
        ("film_height", C.c_double), ("rho_maj", C.c_double), ("rho_min", C.c_double),
        ("rho_iface", C.c_double), ("init_rho_array", C.POINTER(C.c_double)),
        ("hertz_xi", C.c_double), ("hertz_delta0", C.c_double), ("plane_dz", C.c_double),
        ("coupling", C.c_int32), ("node_mass", C.c_double),
    ]


class CapsuleParams(C.Structure):
    _fields_ = [("ks", C.c_double), ("C", C.c_double), ("kb", C.c_double), ("kv", C.c_double),
                ("wet_drho", C.c_double), ("anchor_k", C.c_double)]


class CapsuleObs(C.Structure):
    _fields_ = [("centroid", C.c_double * 3), ("volume", C.c_double),
                ("f_anchor", C.c_double * 3), ("f_capillary", C.c_double * 3),
                ("f_hertz", C.c_double * 3), ("f_fluid", C.c_double * 3)]


class Summary(C.Structure):
    _fields_ = [("mass", C.c_double * 2), ("momentum", C.c_double * 3),
                ("pending", C.c_double * 3), ("step", C.c_int64),
                ("lost_reaction", C.c_int64), ("n_capsules", C.c_int32),
                ("unstable", C.c_int32), ("node_momentum", C.c_double * 3),
                ("lost_links", C.c_int64), ("links", C.c_int64)]


_LIBS = {}


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _ip(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_int32))


def lib(precision: str = "f64"):
    """Load ``liblbmref_<precision>.so`` (built by ``oracle/build.py``)."""
    if precision in _LIBS:
        return _LIBS[precision]
    path = os.path.join(HERE, f"liblbmref_{precision}.so")
    if not os.path.exists(path):
        from . import build as _b
        _b.build()
    L = C.CDLL(path)
    H = C.c_void_p
    L.lbmref_error.restype = C.c_char_p
    L.lbmref_create.restype = H
    L.lbmref_create.argtypes = [C.POINTER(Params)]
    L.lbmref_add_capsule.argtypes = [H, C.POINTER(CapsuleParams), C.c_int32,
                                     C.POINTER(C.c_double), C.c_int32, C.POINTER(C.c_int32)]
    L.lbmref_step.argtypes = [H, C.c_int64]
    for fn in ("lbmref_rho", "lbmref_velocity", "lbmref_meniscus"):
        getattr(L, fn).argtypes = [H, C.POINTER(C.c_double)]
    L.lbmref_labels.argtypes = [H, C.POINTER(C.c_uint8)]
    L.lbmref_capsule_nodes.argtypes = [H, C.c_int32, C.POINTER(C.c_double)]
    L.lbmref_capsule_observe.argtypes = [H, C.c_int32, C.POINTER(CapsuleObs)]
    L.lbmref_get_summary.argtypes = [H, C.POINTER(Summary)]
    L.lbmref_destroy.argtypes = [H]
    L.lbmref_lattice.argtypes = [C.POINTER(C.c_int32), C.POINTER(C.c_double),
                                 C.POINTER(C.c_int32)]
    L.lbmref_feq.argtypes = [C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    L.lbmref_phi4.restype = C.c_double
    L.lbmref_phi4.argtypes = [C.c_double]
    L.lbmref_sc_sum.argtypes = [C.POINTER(C.c_double), C.c_double, C.POINTER(C.c_double)]
    L.lbmref_reference_geometry.argtypes = [C.c_int32, C.POINTER(C.c_double), C.c_int32,
                                            C.POINTER(C.c_int32), C.POINTER(C.c_double),
                                            C.POINTER(C.c_double)]
    L.lbmref_skalak.restype = C.c_double
    L.lbmref_skalak.argtypes = [C.c_int32, C.POINTER(C.c_double), C.c_int32,
                                C.POINTER(C.c_int32), C.POINTER(C.c_double),
                                C.POINTER(C.c_double), C.c_double, C.c_double,
                                C.POINTER(C.c_double)]
    L.lbmref_bending.restype = C.c_double
    L.lbmref_bending.argtypes = [C.c_int32, C.POINTER(C.c_double), C.c_int32,
                                 C.POINTER(C.c_int32), C.POINTER(C.c_double), C.c_double,
                                 C.POINTER(C.c_double)]
    L.lbmref_volume.restype = C.c_double
    L.lbmref_volume.argtypes = [C.c_int32, C.POINTER(C.c_double), C.c_int32,
                                C.POINTER(C.c_int32)]
    L.lbmref_volume_force.argtypes = [C.c_int32, C.POINTER(C.c_double), C.c_int32,
                                      C.POINTER(C.c_int32), C.c_double, C.c_double,
                                      C.POINTER(C.c_double)]
    L.lbmref_miss_distance.restype = C.c_double
    L.lbmref_miss_distance.argtypes = [C.POINTER(C.c_double)] * 5
    L.lbmref_hertz.restype = C.c_double
    L.lbmref_hertz.argtypes = [C.c_double, C.c_double, C.c_double]
    L.lbmref_column_labels.argtypes = [C.c_int32, C.POINTER(C.c_double), C.c_int32,
                                       C.POINTER(C.c_int32)] + [C.c_int32] * 6 + \
                                      [C.POINTER(C.c_uint8)]
    _LIBS[precision] = L
    return L


# ---------------------------------------------------------------------------------------
# Pure helpers (pins)
# ---------------------------------------------------------------------------------------


def lattice(precision="f64"):
    L = lib(precision)
    e = np.zeros(57, np.int32); w = np.zeros(19); o = np.zeros(19, np.int32)
    L.lbmref_lattice(_ip(e), _dp(w), _ip(o))
    return e.reshape(19, 3), w, o


def feq(rho, u, precision="f64"):
    out = np.zeros(19); uu = np.ascontiguousarray(u, dtype=np.float64)
    lib(precision).lbmref_feq(float(rho), _dp(uu), _dp(out))
    return out


def phi4(r):
    return lib().lbmref_phi4(float(r))


def sc_sum(psi27, sc_norm=3.0):
    p = np.ascontiguousarray(psi27, dtype=np.float64).reshape(27)
    out = np.zeros(3)
    lib().lbmref_sc_sum(_dp(p), float(sc_norm), _dp(out))
    return out


def reference_geometry(nodes, tris):
    x = np.ascontiguousarray(nodes, dtype=np.float64); t = np.ascontiguousarray(tris, np.int32)
    minv = np.zeros((len(t), 4)); a0 = np.zeros(len(t))
    lib().lbmref_reference_geometry(len(x), _dp(x), len(t), _ip(t), _dp(minv), _dp(a0))
    return minv, a0


def skalak(nodes, tris, minv, a0, ks, Cs, precision="f64"):
    x = np.ascontiguousarray(nodes, dtype=np.float64); t = np.ascontiguousarray(tris, np.int32)
    f = np.zeros_like(x)
    E = lib(precision).lbmref_skalak(len(x), _dp(x), len(t), _ip(t),
                                     _dp(np.ascontiguousarray(minv)),
                                     _dp(np.ascontiguousarray(a0)), float(ks), float(Cs), _dp(f))
    return E, f


def bending(nodes, tris, ref, kb, precision="f64"):
    """Edge-form Helfrich energy and node forces (eq. method:curvature); ``ref`` the
    reference node positions (None: flat reference angles)."""
    x = np.ascontiguousarray(nodes, dtype=np.float64)
    t = np.ascontiguousarray(tris, dtype=np.int32)
    f = np.zeros_like(x)
    r = None if ref is None else np.ascontiguousarray(ref, dtype=np.float64)
    E = lib(precision).lbmref_bending(len(x), _dp(x), len(t), _ip(t),
                                      None if r is None else _dp(r), float(kb), _dp(f))
    return E, f


def volume(nodes, tris):
    x = np.ascontiguousarray(nodes, dtype=np.float64); t = np.ascontiguousarray(tris, np.int32)
    return lib().lbmref_volume(len(x), _dp(x), len(t), _ip(t))


def volume_force(nodes, tris, kv, v0):
    x = np.ascontiguousarray(nodes, dtype=np.float64); t = np.ascontiguousarray(tris, np.int32)
    f = np.zeros_like(x)
    lib().lbmref_volume_force(len(x), _dp(x), len(t), _ip(t), float(kv), float(v0), _dp(f))
    return f


def hertz(d, xi=1.5, delta0=1.5):
    return lib().lbmref_hertz(float(d), float(xi), float(delta0))


def miss_distance(p0, p1, a, b, c):
    """Miss distance of the segment p0 -> p1 from triangle (a, b, c) (0: they meet)."""
    v = [np.ascontiguousarray(x, dtype=np.float64) for x in (p0, p1, a, b, c)]
    return lib().lbmref_miss_distance(*[_dp(x) for x in v])


def column_labels(nodes, tris, origin, dims):
    x = np.ascontiguousarray(nodes, dtype=np.float64); t = np.ascontiguousarray(tris, np.int32)
    out = np.zeros(int(np.prod(dims)), np.uint8)
    lib().lbmref_column_labels(len(x), _dp(x), len(t), _ip(t), *[int(v) for v in origin],
                               *[int(v) for v in dims], out.ctypes.data_as(C.POINTER(C.c_uint8)))
    return out.reshape(dims[2], dims[1], dims[0])


# ---------------------------------------------------------------------------------------
# Simulation handle
# ---------------------------------------------------------------------------------------


def make_params(cfg: dict, n_threads: int = 0):
    if cfg.get("slab_nz", 0) not in (0, cfg["nz"]):
        raise ValueError("the oracle simulates one box; run each stacked slab as a box of its own")
    p = Params()
    p.nx, p.ny, p.nz, p.wall_z0 = cfg["nx"], cfg["ny"], cfg["nz"], int(cfg["wall_z0"])
    p.tau[0], p.tau[1] = cfg["tau"]
    p.G, p.rho0, p.sc_norm = cfg["G"], cfg["rho0"], cfg["sc_norm"]
    for d in range(3):
        p.body_force[d] = cfg["body_force"][d]
    p.wall_drho = cfg["wall_drho"]
    p.init_mode = int(cfg["init_mode"])
    p.n_threads = int(n_threads)
    p.init_rho[0], p.init_rho[1] = cfg["init_rho"]
    p.film_height, p.rho_maj = cfg["film_height"], cfg["rho_maj"]
    p.rho_min, p.rho_iface = cfg["rho_min"], cfg["rho_iface"]
    keep = None
    if cfg.get("init_rho_array") is not None:
        keep = np.ascontiguousarray(cfg["init_rho_array"], dtype=np.float64)
        assert keep.shape == (2, cfg["nz"], cfg["ny"], cfg["nx"])
        p.init_rho_array = _dp(keep)
    p.hertz_xi, p.hertz_delta0, p.plane_dz = cfg["hertz_xi"], cfg["hertz_delta0"], cfg["plane_dz"]
    p.coupling = int(cfg.get("coupling", 0))
    p.node_mass = float(cfg.get("node_mass", 25.0))
    return p, keep


class Oracle:
    """One oracle simulation.  ``precision`` is ``"f64"`` (the oracle) or ``"f32"``
    (diagnostic build of the same code)."""

    def __init__(self, cfg: dict, precision: str = "f64", n_threads: int = 0,
                 meshes: Optional[list] = None):
        import synth
        self.cfg = cfg
        self.L = lib(precision)
        p, keep = make_params(cfg, n_threads)
        self.h = self.L.lbmref_create(C.byref(p))
        del keep
        if not self.h:
            raise ValueError(self.L.lbmref_error().decode())
        self.nx, self.ny, self.nz = cfg["nx"], cfg["ny"], cfg["nz"]
        self.meshes = []
        for i, cp in enumerate(cfg["capsules"]):
            nodes, tris = meshes[i] if meshes is not None else synth.capsule_mesh(cp)
            self.add_capsule(cp, nodes, tris)

    def add_capsule(self, cp: dict, nodes, tris) -> int:
        q = CapsuleParams(cp["ks"], cp["C"], cp["kb"], cp["kv"], cp["wet_drho"], cp["anchor_k"])
        x = np.ascontiguousarray(nodes, dtype=np.float64)
        t = np.ascontiguousarray(tris, dtype=np.int32)
        r = self.L.lbmref_add_capsule(self.h, C.byref(q), len(x), _dp(x), len(t), _ip(t))
        if r < 0:
            raise ValueError(self.L.lbmref_error().decode())
        self.meshes.append((x, t))
        return r

    def step(self, n: int = 1) -> int:
        return self.L.lbmref_step(self.h, int(n))

    def rho(self) -> np.ndarray:
        out = np.zeros((2, self.nz, self.ny, self.nx))
        self.L.lbmref_rho(self.h, _dp(out))
        return out

    def velocity(self) -> np.ndarray:
        out = np.zeros((3, self.nz, self.ny, self.nx))
        self.L.lbmref_velocity(self.h, _dp(out))
        return out

    def meniscus(self) -> np.ndarray:
        out = np.zeros((self.ny, self.nx))
        self.L.lbmref_meniscus(self.h, _dp(out))
        return out

    def labels(self) -> np.ndarray:
        out = np.zeros((self.nz, self.ny, self.nx), np.uint8)
        self.L.lbmref_labels(self.h, out.ctypes.data_as(C.POINTER(C.c_uint8)))
        return out

    def nodes(self, k: int) -> np.ndarray:
        out = np.zeros((len(self.meshes[k][0]), 3))
        if self.L.lbmref_capsule_nodes(self.h, k, _dp(out)) < 0:
            raise IndexError(k)
        return out

    def capsule(self, k: int) -> dict:
        o = CapsuleObs()
        if self.L.lbmref_capsule_observe(self.h, k, C.byref(o)) < 0:
            raise IndexError(k)
        return dict(centroid=np.array(o.centroid), volume=o.volume,
                    f_anchor=np.array(o.f_anchor), f_capillary=np.array(o.f_capillary),
                    f_hertz=np.array(o.f_hertz), f_fluid=np.array(o.f_fluid))

    def summary(self) -> dict:
        s = Summary()
        self.L.lbmref_get_summary(self.h, C.byref(s))
        return dict(mass=np.array(s.mass), momentum=np.array(s.momentum),
                    pending=np.array(s.pending), step=s.step, lost_reaction=s.lost_reaction,
                    n_capsules=s.n_capsules, unstable=s.unstable,
                    node_momentum=np.array(s.node_momentum), lost_links=s.lost_links,
                    links=s.links)

    def close(self):
        if getattr(self, "h", None):
            self.L.lbmref_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
