"""ctypes binding of ``liblbm.so`` (the C ABI declared in ``include/lbm.h``).

Argument marshalling only: every step of the simulation runs in the library's HIP
kernels.  PyTorch is used, when present, for the stream the library enqueues on and for
device buffers (``Sim.rho_device``).  The library must have been built
(``python -m paper_2007_15405_amd.build``); there is no fallback path.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblbm.so")

STORAGE = {"f32": 0, "f16": 1, "bf16": 2, "f16site": 3}

LBM_OK, LBM_E_INVAL, LBM_E_NOMEM, LBM_E_DEVICE, LBM_E_UNSTABLE, LBM_E_STATE = 0, -1, -2, -3, -4, -5


class LbmError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"lbm status {status}: {msg}")
        self.status = status


class Params(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32), ("wall_z0", C.c_int32),
        ("tau", C.c_double * 2), ("G", C.c_double), ("rho0", C.c_double),
        ("sc_norm", C.c_double), ("body_force", C.c_double * 3), ("wall_drho", C.c_double),
        ("init_mode", C.c_int32), ("storage", C.c_int32), ("init_rho", C.c_double * 2),
        ("film_height", C.c_double), ("rho_maj", C.c_double), ("rho_min", C.c_double),
        ("rho_iface", C.c_double), ("init_rho_array", C.POINTER(C.c_double)),
        ("hertz_xi", C.c_double), ("hertz_delta0", C.c_double), ("plane_dz", C.c_double),
        ("rho_shift", C.c_double * 2), ("stream", C.c_void_p), ("device", C.c_int32),
        ("stream_given", C.c_int32), ("slab_nz", C.c_int32),
        ("slab_film_height", C.POINTER(C.c_double)),
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
                ("links", C.c_int64), ("lost_links", C.c_int64)]


class Obs(C.Structure):
    _fields_ = [("rho", C.POINTER(C.c_float)), ("meniscus", C.POINTER(C.c_float)),
                ("capsules", C.POINTER(CapsuleObs)), ("slab_mass", C.POINTER(C.c_double)),
                ("summary", Summary)]


class KernelStat(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("launches", C.c_int64), ("total_ms", C.c_double)]


class ClusterParams(C.Structure):
    _fields_ = [("box", C.c_float), ("radius", C.c_float), ("log10_ks", C.c_float),
                ("film", C.c_float), ("angle", C.c_float), ("in_mean", C.c_float * 4),
                ("in_scale", C.c_float * 4), ("out_mean", C.c_float * 2),
                ("out_scale", C.c_float * 2), ("r_contact", C.c_float), ("r_cut", C.c_float),
                ("k_contact", C.c_float), ("mobility", C.c_float)]


# entry point -> (restype, argtypes); every function declared in include/lbm.h
H = C.c_void_p
SIGNATURES = {
    "lbm_init": (C.c_int, [C.POINTER(Params), C.POINTER(C.c_void_p)]),
    "lbm_add_capsule": (C.c_int, [H, C.POINTER(CapsuleParams), C.c_int32, C.POINTER(C.c_double),
                                  C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32)]),
    "lbm_add_sphere_capsule": (C.c_int, [H, C.POINTER(CapsuleParams), C.POINTER(C.c_double),
                                         C.c_double, C.c_int32, C.POINTER(C.c_int32)]),
    "lbm_step": (C.c_int, [H, C.c_int64]),
    "lbm_sync": (C.c_int, [H]),
    "lbm_observables": (C.c_int, [H, C.POINTER(Obs)]),
    "lbm_rho_device": (C.c_int, [H, C.c_void_p]),
    "lbm_capsule_nodes": (C.c_int, [H, C.c_int32, C.POINTER(C.c_double)]),
    "lbm_labels": (C.c_int, [H, C.POINTER(C.c_uint8)]),
    "lbm_save": (C.c_int, [H, C.c_char_p]),
    "lbm_load": (C.c_int, [H, C.c_char_p]),
    "lbm_set_profiling": (C.c_int, [H, C.c_int32]),
    "lbm_kernel_stats": (C.c_int, [H, C.POINTER(KernelStat), C.c_int32, C.POINTER(C.c_int32)]),
    "lbm_set_launch": (C.c_int, [H, C.c_int32, C.c_int32]),
    "lbm_set_zoffset": (C.c_int, [H, C.c_int32]),
    "lbm_zoffset": (C.c_int32, [H]),
    "lbm_autotune": (C.c_int, [H, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                               C.POINTER(C.c_double)]),
    "lbm_bytes_per_site": (C.c_double, [H]),
    "lbm_fluid_sites": (C.c_int64, [H]),
    "lbm_last_error": (C.c_char_p, [H]),
    "lbm_destroy": (None, [H]),
    "lbm_batch_create": (C.c_int, [C.POINTER(C.c_void_p), C.c_int32, C.POINTER(C.c_void_p)]),
    "lbm_batch_set_launch": (C.c_int, [H, C.c_int32, C.c_int32]),
    "lbm_batch_set_parts": (C.c_int, [H, C.c_int32]),
    "lbm_batch_autotune": (C.c_int, [H, C.c_int32, C.POINTER(C.c_int32), C.POINTER(C.c_int32),
                                     C.POINTER(C.c_double)]),
    "lbm_batch_step": (C.c_int, [H, C.c_int64]),
    "lbm_batch_set_profiling": (C.c_int, [H, C.c_int32]),
    "lbm_batch_set_graph": (C.c_int, [H, C.c_int32]),
    "lbm_batch_set_schedule": (C.c_int, [H, C.c_int32]),
    "lbm_batch_kernel_stats": (C.c_int, [H, C.POINTER(KernelStat), C.c_int32, C.POINTER(C.c_int32)]),
    "lbm_batch_last_error": (C.c_char_p, [H]),
    "lbm_batch_destroy": (None, [H]),
    "lbm_surrogate_create": (C.c_int, [C.c_int32, C.POINTER(C.c_float), C.POINTER(C.c_void_p)]),
    "lbm_surrogate_set_data": (C.c_int, [H, C.c_int32, C.POINTER(C.c_float), C.POINTER(C.c_float),
                                         C.POINTER(C.c_float)]),
    "lbm_surrogate_gradient": (C.c_int, [H, C.POINTER(C.c_float), C.POINTER(C.c_float)]),
    "lbm_surrogate_train": (C.c_int, [H, C.c_int32, C.c_float]),
    "lbm_surrogate_predict": (C.c_int, [H, C.c_int32, C.POINTER(C.c_float), C.POINTER(C.c_float)]),
    "lbm_surrogate_params": (C.c_int, [H, C.POINTER(C.c_float)]),
    "lbm_surrogate_cluster": (C.c_int, [H, C.c_int32, C.POINTER(C.c_float), C.c_int32,
                                        C.POINTER(ClusterParams)]),
    "lbm_surrogate_cluster_noalloc": (C.c_int, [H, C.c_int32, C.c_void_p, C.c_int32,
                                                C.POINTER(ClusterParams)]),
    "lbm_surrogate_last_error": (C.c_char_p, [H]),
    "lbm_surrogate_destroy": (None, [H]),
}

_LIB = None


def load_library(path: str = LIB_PATH):
    """Load liblbm.so; raises if it has not been built.

    PyTorch-ROCm ships its own HIP runtime; importing torch first makes liblbm bind to
    that already-loaded runtime, so one process never holds two HSA runtimes."""
    global _LIB
    if _LIB is not None:
        return _LIB
    try:
        import torch  # noqa: F401
    except Exception:
        pass
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with "
                           f"'python -m paper_2007_15405_amd.build' (no fallback exists)")
    L = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = L
    return L


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _torch_stream():
    """Handle of torch's current stream (0 for the null stream), or None."""
    try:
        import torch
        if torch.cuda.is_available():
            return int(torch.cuda.current_stream().cuda_stream)
    except Exception:
        pass
    return None


class Sim:
    """One simulation on the GPU, configured by a dict as made by ``synth.workload``.

    ``storage`` is ``"f32"``, ``"f16"`` or ``"bf16"`` (16-bit modes store f - w rho_shift).
    ``cfg["slab_nz"]`` (0: one box) stacks independent boxes of that height along z, with
    ``cfg["slab_film_height"]`` (or None) their film heights.
    ``stream``: ``"torch"`` (default: torch's current stream if a GPU is visible), ``None``
    (a stream of the library's own) or a raw hipStream_t integer."""

    def __init__(self, cfg: dict, storage: str = "f32", rho_shift=(1.0, 1.0),
                 stream="torch", device: int = 0, meshes: Optional[list] = None,
                 library_meshes: bool = False):
        import synth
        self.L = load_library()
        self.cfg = cfg
        self.nx, self.ny, self.nz = cfg["nx"], cfg["ny"], cfg["nz"]
        self.lz = cfg.get("slab_nz", 0) or self.nz
        self.n_slabs = self.nz // self.lz
        p = Params()
        p.nx, p.ny, p.nz, p.wall_z0 = self.nx, self.ny, self.nz, int(cfg["wall_z0"])
        p.tau[0], p.tau[1] = cfg["tau"]
        p.G, p.rho0, p.sc_norm = cfg["G"], cfg["rho0"], cfg["sc_norm"]
        for d in range(3):
            p.body_force[d] = cfg["body_force"][d]
        p.wall_drho = cfg["wall_drho"]
        p.init_mode = int(cfg["init_mode"])
        p.storage = STORAGE[storage]
        p.init_rho[0], p.init_rho[1] = cfg["init_rho"]
        p.film_height, p.rho_maj = cfg["film_height"], cfg["rho_maj"]
        p.rho_min, p.rho_iface = cfg["rho_min"], cfg["rho_iface"]
        keep = None
        if cfg.get("init_rho_array") is not None:
            keep = np.ascontiguousarray(cfg["init_rho_array"], dtype=np.float64)
            if keep.shape != (2, self.nz, self.ny, self.nx):
                raise ValueError("init_rho_array must be [2][nz][ny][nx]")
            p.init_rho_array = _dp(keep)
        p.slab_nz = int(cfg.get("slab_nz", 0))
        films = None
        if cfg.get("slab_film_height") is not None:
            films = np.ascontiguousarray(cfg["slab_film_height"], dtype=np.float64)
            if films.shape != (self.n_slabs,):
                raise ValueError("slab_film_height needs one value per slab")
            p.slab_film_height = _dp(films)
        p.hertz_xi, p.hertz_delta0 = cfg["hertz_xi"], cfg["hertz_delta0"]
        p.plane_dz = cfg["plane_dz"]
        p.coupling = int(cfg.get("coupling", 0))
        p.node_mass = float(cfg.get("node_mass", 25.0))
        p.rho_shift[0], p.rho_shift[1] = rho_shift
        if stream == "torch":
            s = _torch_stream()
            if s is not None:
                p.stream, p.stream_given = (s or None), 1
        elif stream is not None:
            p.stream, p.stream_given = (int(stream) or None), 1
        p.device = device
        h = C.c_void_p()
        st = self.L.lbm_init(C.byref(p), C.byref(h))
        if st != LBM_OK:
            raise LbmError(st, self.L.lbm_last_error(None).decode())
        self.h = h
        self.storage = storage
        self.n_nodes = []
        for i, cp in enumerate(cfg["capsules"]):
            if library_meshes:     # the library builds the geodesic sphere itself
                self.add_sphere_capsule(cp)
                continue
            nodes, tris = meshes[i] if meshes is not None else synth.capsule_mesh(cp)
            self.add_capsule(cp, nodes, tris)

    # -- plumbing --------------------------------------------------------------------------
    def _check(self, st: int):
        if st != LBM_OK:
            raise LbmError(st, self.L.lbm_last_error(self.h).decode())

    def add_capsule(self, cp: dict, nodes, tris) -> int:
        q = CapsuleParams(cp["ks"], cp["C"], cp["kb"], cp["kv"], cp["wet_drho"], cp["anchor_k"])
        x = np.ascontiguousarray(nodes, dtype=np.float64)
        t = np.ascontiguousarray(tris, dtype=np.int32)
        out = C.c_int32()
        self._check(self.L.lbm_add_capsule(self.h, C.byref(q), len(x), _dp(x), len(t),
                                           t.ctypes.data_as(C.POINTER(C.c_int32)), C.byref(out)))
        self.n_nodes.append(len(x))
        return out.value

    def add_sphere_capsule(self, cp: dict, n_nodes: int = None) -> int:
        """A spherical capsule of cp["center"], cp["radius"], cp["n_tri"] whose mesh the library
        builds (``lbm_add_sphere_capsule``)."""
        q = CapsuleParams(cp["ks"], cp["C"], cp["kb"], cp["kv"], cp["wet_drho"], cp["anchor_k"])
        cen = np.ascontiguousarray(cp["center"], dtype=np.float64)
        out = C.c_int32()
        self._check(self.L.lbm_add_sphere_capsule(self.h, C.byref(q), _dp(cen), float(cp["radius"]),
                                                  int(cp["n_tri"]), C.byref(out)))
        self.n_nodes.append(10 * int(cp["n_tri"]) // 20 + 2)
        return out.value

    def step(self, n: int = 1):
        self._check(self.L.lbm_step(self.h, int(n)))

    def sync(self):
        self._check(self.L.lbm_sync(self.h))

    # -- observables -------------------------------------------------------------------------
    def observables(self, rho: bool = False, meniscus: bool = False, capsules: bool = True,
                    check: bool = True) -> dict:
        o = Obs()
        r = m = caps = None
        if rho:
            r = np.zeros((2, self.nz, self.ny, self.nx), np.float32)
            o.rho = r.ctypes.data_as(C.POINTER(C.c_float))
        if meniscus:
            m = np.zeros((self.n_slabs, self.ny, self.nx), np.float32)
            o.meniscus = m.ctypes.data_as(C.POINTER(C.c_float))
        sm = np.zeros((self.n_slabs, 2))
        o.slab_mass = _dp(sm)
        nc = len(self.n_nodes)
        if capsules and nc:
            caps = (CapsuleObs * nc)()
            o.capsules = caps
        st = self.L.lbm_observables(self.h, C.byref(o))
        if check:
            self._check(st)
        s = o.summary
        out = dict(status=st, summary=dict(
            mass=np.array(s.mass), momentum=np.array(s.momentum), pending=np.array(s.pending),
            step=s.step, lost_reaction=s.lost_reaction, n_capsules=s.n_capsules,
            unstable=s.unstable, node_momentum=np.array(s.node_momentum), links=s.links,
            lost_links=s.lost_links))
        out["slab_mass"] = sm
        if rho:
            out["rho"] = r
        if meniscus:
            # one box: [ny][nx]; stacked slabs: [n_slabs][ny][nx], heights above each wall
            out["meniscus"] = m[0] if self.n_slabs == 1 else m
        if caps is not None:
            out["capsules"] = [dict(centroid=np.array(c.centroid), volume=c.volume,
                                    f_anchor=np.array(c.f_anchor),
                                    f_capillary=np.array(c.f_capillary),
                                    f_hertz=np.array(c.f_hertz), f_fluid=np.array(c.f_fluid))
                               for c in caps]
        return out

    def rho(self) -> np.ndarray:
        return self.observables(rho=True, capsules=False)["rho"]

    def meniscus(self) -> np.ndarray:
        return self.observables(meniscus=True, capsules=False)["meniscus"]

    def summary(self) -> dict:
        return self.observables(capsules=False)["summary"]

    def capsule(self, k: int) -> dict:
        return self.observables()["capsules"][k]

    def rho_device(self):
        """Densities into a new torch CUDA tensor [2][nz][ny][nx] (library stream)."""
        import torch
        out = torch.empty((2, self.nz, self.ny, self.nx), dtype=torch.float32, device="cuda")
        self._check(self.L.lbm_rho_device(self.h, C.c_void_p(out.data_ptr())))
        return out

    def nodes(self, k: int) -> np.ndarray:
        out = np.zeros((self.n_nodes[k], 3))
        self._check(self.L.lbm_capsule_nodes(self.h, k, _dp(out)))
        return out

    def labels(self) -> np.ndarray:
        out = np.zeros((self.nz, self.ny, self.nx), np.uint8)
        self._check(self.L.lbm_labels(self.h, out.ctypes.data_as(C.POINTER(C.c_uint8))))
        return out

    # -- checkpoints, profiling ------------------------------------------------------------
    def save(self, path: str):
        self._check(self.L.lbm_save(self.h, path.encode()))

    def load(self, path: str):
        self._check(self.L.lbm_load(self.h, path.encode()))

    def set_profiling(self, on=True):
        """on: True/1 times every kernel, 2 only the fluid kernel, False/0 stops."""
        self._check(self.L.lbm_set_profiling(self.h, int(on)))

    def kernel_stats(self) -> dict:
        arr = (KernelStat * 32)()
        n = C.c_int32()
        self._check(self.L.lbm_kernel_stats(self.h, arr, 32, C.byref(n)))
        return {arr[i].name.decode(): (arr[i].launches, arr[i].total_ms) for i in range(n.value)}

    def set_launch(self, tile: int = 1, zchunk: int = 0):
        """Fluid-step launch shape (tile 0: two-kernel variant; 1..5: fused kernel)."""
        self._check(self.L.lbm_set_launch(self.h, int(tile), int(zchunk)))

    def autotune(self, reps: int = 10) -> dict:
        """Time the fluid kernel in every applicable launch shape on the current state and
        keep the fastest (``lbm_autotune``; the simulation is not advanced)."""
        t, z, ms = C.c_int32(), C.c_int32(), C.c_double()
        self._check(self.L.lbm_autotune(self.h, int(reps), C.byref(t), C.byref(z), C.byref(ms)))
        return dict(tile=t.value, zchunk=z.value, zoff=self.zoffset, fluid_ms=ms.value)

    def set_zoffset(self, planes: int = 0):
        """Shorten the fluid launch's first z-chunk by ``planes`` planes (``lbm_set_zoffset``)."""
        self._check(self.L.lbm_set_zoffset(self.h, int(planes)))

    @property
    def zoffset(self) -> int:
        return int(self.L.lbm_zoffset(self.h))

    @property
    def bytes_per_site(self) -> float:
        return self.L.lbm_bytes_per_site(self.h)

    @property
    def fluid_sites(self) -> int:
        return self.L.lbm_fluid_sites(self.h)

    def close(self):
        if getattr(self, "h", None):
            self.L.lbm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Batch:
    """Several ``Sim`` objects stepped together, one fluid launch per step over all their
    lattices (``lbm_batch_*``).  The sims must share stream and storage and have tau = 1;
    close the batch before them."""

    def __init__(self, sims: list, tile: int = 10, zchunk: int = 0, parts: int = 1):
        self.L = load_library()
        self.sims = list(sims)
        arr = (C.c_void_p * len(self.sims))(*[s.h.value for s in self.sims])
        b = C.c_void_p()
        st = self.L.lbm_batch_create(arr, len(self.sims), C.byref(b))
        if st != LBM_OK:
            raise LbmError(st, self.L.lbm_batch_last_error(None).decode())
        self.b = b
        self.set_launch(tile, zchunk)
        self.set_parts(parts)

    def _check(self, st: int):
        if st != LBM_OK:
            raise LbmError(st, self.L.lbm_batch_last_error(self.b).decode())

    def set_launch(self, tile: int = 10, zchunk: int = 0):
        self._check(self.L.lbm_batch_set_launch(self.b, int(tile), int(zchunk)))

    def set_parts(self, parts: int = 1):
        """Advance the sims in ``parts`` sets on streams of their own (overlap)."""
        self._check(self.L.lbm_batch_set_parts(self.b, int(parts)))

    def step(self, n: int = 1):
        self._check(self.L.lbm_batch_step(self.b, int(n)))

    def autotune(self, reps: int = 10) -> dict:
        """``lbm_batch_autotune``: the fastest batched fluid launch shape (not advancing)."""
        t, z, ms = C.c_int32(), C.c_int32(), C.c_double()
        self._check(self.L.lbm_batch_autotune(self.b, int(reps), C.byref(t), C.byref(z),
                                              C.byref(ms)))
        return dict(tile=t.value, zchunk=z.value, fluid_ms=ms.value)

    def sync(self):
        for s in self.sims:
            s.sync()

    def set_profiling(self, on=True):
        self._check(self.L.lbm_batch_set_profiling(self.b, int(on)))

    def set_schedule(self, queue=True):
        """``lbm_batch_set_schedule``: the fluid launch as a resident grid with a work queue
        (True) or one workgroup per tile in the static order (False)."""
        self._check(self.L.lbm_batch_set_schedule(self.b, int(bool(queue))))

    def set_graph(self, on=True):
        """``lbm_batch_set_graph``: replay pairs of steps from a captured HIP graph."""
        self._check(self.L.lbm_batch_set_graph(self.b, int(bool(on))))

    def kernel_stats(self) -> dict:
        arr = (KernelStat * 32)()
        n = C.c_int32()
        self._check(self.L.lbm_batch_kernel_stats(self.b, arr, 32, C.byref(n)))
        return {arr[i].name.decode(): (arr[i].launches, arr[i].total_ms) for i in range(n.value)}

    @property
    def fluid_sites(self) -> int:
        return sum(s.fluid_sites for s in self.sims)

    @property
    def bytes_per_site(self) -> float:
        return self.sims[0].bytes_per_site

    def close(self):
        if getattr(self, "b", None):
            self.L.lbm_batch_destroy(self.b)
            self.b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


SURROGATE_PARAMS = 8770
CLUSTER_NOALLOC_MAX = 16384      # LBM_CLUSTER_NOALLOC_MAX


def _fp(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


class Surrogate:
    """The learned surrogate network (``lbm_surrogate_*``): 4 -> 64 -> 64 -> 64 -> 2, tanh,
    trained by Adam with the matrix products on the matrix cores (bfloat16 operands,
    float32 sums).  Inputs and targets are passed normalised."""

    def __init__(self, theta0, max_samples: int):
        self.L = load_library()
        th = np.ascontiguousarray(theta0, dtype=np.float32)
        if th.shape != (SURROGATE_PARAMS,):
            raise ValueError(f"theta0 must have {SURROGATE_PARAMS} entries")
        s = C.c_void_p()
        st = self.L.lbm_surrogate_create(int(max_samples), _fp(th), C.byref(s))
        if st != LBM_OK:
            raise LbmError(st, self.L.lbm_surrogate_last_error(None).decode())
        self.s = s
        self.max_samples = int(max_samples)

    def _check(self, st: int):
        if st != LBM_OK:
            raise LbmError(st, self.L.lbm_surrogate_last_error(self.s).decode())

    def set_data(self, x, t, w=None):
        x = np.ascontiguousarray(x, dtype=np.float32)
        t = np.ascontiguousarray(t, dtype=np.float32)
        wp = None
        if w is not None:
            w = np.ascontiguousarray(w, dtype=np.float32)
            wp = _fp(w)
        if x.ndim != 2 or x.shape[1] != 4 or t.shape != (len(x), 2):
            raise ValueError("x must be [n][4] and t [n][2]")
        self._check(self.L.lbm_surrogate_set_data(self.s, len(x), _fp(x), _fp(t), wp))

    def gradient(self):
        g = np.zeros(SURROGATE_PARAMS, np.float32)
        loss = C.c_float()
        self._check(self.L.lbm_surrogate_gradient(self.s, C.byref(loss), _fp(g)))
        return float(loss.value), g

    def train(self, steps: int, lr: float = 1e-3):
        self._check(self.L.lbm_surrogate_train(self.s, int(steps), float(lr)))

    def predict(self, x) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.float32)
        y = np.zeros((len(x), 2), np.float32)
        self._check(self.L.lbm_surrogate_predict(self.s, len(x), _fp(x), _fp(y)))
        return y

    def params(self) -> np.ndarray:
        th = np.zeros(SURROGATE_PARAMS, np.float32)
        self._check(self.L.lbm_surrogate_params(self.s, _fp(th)))
        return th

    def cluster(self, xy, steps: int, *, box, radius, features, in_mean, in_scale, out_mean,
                out_scale, r_contact, r_cut, k_contact, mobility) -> np.ndarray:
        """Positions [n][2] after ``steps`` overdamped steps driven by the network's pair
        forces (``lbm_surrogate_cluster``); ``features`` = raw (log10 ks, film / 2R,
        contact angle)."""
        p = np.ascontiguousarray(xy, dtype=np.float32).copy()
        if p.ndim != 2 or p.shape[1] != 2:
            raise ValueError("xy must be [n][2]")
        cp = ClusterParams(box=box, radius=radius, log10_ks=features[0], film=features[1],
                           angle=features[2], r_contact=r_contact, r_cut=r_cut,
                           k_contact=k_contact, mobility=mobility)
        cp.in_mean[:] = [float(v) for v in in_mean]
        cp.in_scale[:] = [float(v) for v in in_scale]
        cp.out_mean[:] = [float(v) for v in out_mean]
        cp.out_scale[:] = [float(v) for v in out_scale]
        self._check(self.L.lbm_surrogate_cluster(self.s, len(p), _fp(p), int(steps),
                                                 C.byref(cp)))
        return p

    def cluster_noalloc(self, xy_device, steps: int, *, box, radius, features, in_mean,
                        in_scale, out_mean, out_scale, r_contact, r_cut, k_contact,
                        mobility):
        """``lbm_surrogate_cluster_noalloc``: advance a device tensor of positions [n][2]
        (float32, contiguous, on the GPU) in place, with no device allocation."""
        import torch
        if xy_device.dtype != torch.float32 or xy_device.dim() != 2 or xy_device.shape[1] != 2 \
                or not xy_device.is_contiguous() or not xy_device.is_cuda:
            raise ValueError("xy_device must be a contiguous float32 [n][2] GPU tensor")
        cp = ClusterParams(box=box, radius=radius, log10_ks=features[0], film=features[1],
                           angle=features[2], r_contact=r_contact, r_cut=r_cut,
                           k_contact=k_contact, mobility=mobility)
        cp.in_mean[:] = [float(v) for v in in_mean]
        cp.in_scale[:] = [float(v) for v in in_scale]
        cp.out_mean[:] = [float(v) for v in out_mean]
        cp.out_scale[:] = [float(v) for v in out_scale]
        self._check(self.L.lbm_surrogate_cluster_noalloc(
            self.s, int(xy_device.shape[0]), C.c_void_p(xy_device.data_ptr()), int(steps),
            C.byref(cp)))
        return xy_device

    def close(self):
        if getattr(self, "s", None):
            self.L.lbm_surrogate_destroy(self.s)
            self.s = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
