"""The C-ABI library: it loads without a GPU, exports every entry point that
include/lbm.h declares, the ctypes structures of the binding match the C layout, and
parameter validation rejects bad input before any device call."""
import ctypes as C
import os
import re
import subprocess

import pytest

import paper_2007_15405_amd as pkg
from paper_2007_15405_amd import lbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbm.h")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lbm_[a-z_]+)\s*\(", text)))


def test_library_exports_every_declared_entry_point():
    L = pkg.load_library()
    names = declared_functions()
    assert len(names) >= 16
    for n in names:
        assert hasattr(L, n), n
    assert sorted(pkg.SIGNATURES) == names


def test_binding_structs_match_c_layout(tmp_path):
    structs = {
        "lbm_params": lbm.Params, "lbm_capsule_params": lbm.CapsuleParams,
        "lbm_capsule_obs": lbm.CapsuleObs, "lbm_summary": lbm.Summary, "lbm_obs": lbm.Obs,
        "lbm_kernel_stat": lbm.KernelStat,
    }
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "lbm.h"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {}
    for ln in out:
        if ln:
            a, b, v = ln.split()
            got[(a, b)] = int(v)
    for cname, py in structs.items():
        assert got[(cname, "size")] == C.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


@pytest.mark.parametrize("field,value,msg", [
    ("nx", 2, "nx, ny, nz"),
    ("tau", (0.5, 1.0), "tau"),
    ("init_mode", 7, "init_mode"),
    ("storage", 4, "storage"),
    ("rho0", 0.0, "rho0"),
])
def test_invalid_parameters_are_rejected_on_the_host(field, value, msg):
    L = pkg.load_library()
    p = lbm.Params()
    p.nx = p.ny = p.nz = 8
    p.tau[0] = p.tau[1] = 1.0
    p.rho0, p.G = 1.0, 3.6
    if field == "tau":
        p.tau[0], p.tau[1] = value
    else:
        setattr(p, field, value)
    h = C.c_void_p()
    st = L.lbm_init(C.byref(p), C.byref(h))
    assert st == lbm.LBM_E_INVAL and not h.value
    assert msg in L.lbm_last_error(None).decode()


def test_mode2_without_array_is_rejected():
    L = pkg.load_library()
    p = lbm.Params()
    p.nx = p.ny = p.nz = 8
    p.tau[0] = p.tau[1] = 1.0
    p.rho0 = 1.0
    p.init_mode = 2
    h = C.c_void_p()
    assert L.lbm_init(C.byref(p), C.byref(h)) == lbm.LBM_E_INVAL


def test_null_handles_are_rejected():
    L = pkg.load_library()
    assert L.lbm_step(None, 1) == lbm.LBM_E_INVAL
    assert L.lbm_sync(None) == lbm.LBM_E_INVAL
    assert L.lbm_observables(None, None) == lbm.LBM_E_INVAL
    assert L.lbm_bytes_per_site(None) == 0.0
    L.lbm_destroy(None)


@pytest.mark.parametrize("nz,slab,wall,msg", [
    (30, 7, 1, "slab_nz"),       # does not divide nz
    (30, 2, 1, "slab_nz"),       # too thin
    (30, 10, 0, "wall_z0"),      # stacked slabs need their wall layers
])
def test_invalid_slabs_are_rejected_on_the_host(nz, slab, wall, msg):
    L = pkg.load_library()
    p = lbm.Params()
    p.nx = p.ny = 8
    p.nz, p.slab_nz, p.wall_z0 = nz, slab, wall
    p.tau[0] = p.tau[1] = 1.0
    p.rho0 = 1.0
    h = C.c_void_p()
    assert L.lbm_init(C.byref(p), C.byref(h)) == lbm.LBM_E_INVAL and not h.value
    assert msg in L.lbm_last_error(None).decode()


def test_lattice_beyond_32_bit_population_offsets_is_rejected():
    L = pkg.load_library()
    p = lbm.Params()
    p.nx, p.ny, p.nz = 1024, 512, 216     # 113 M sites: 10 x 4 B x N > 4 GiB
    p.tau[0] = p.tau[1] = 1.0
    p.rho0 = 1.0
    h = C.c_void_p()
    assert L.lbm_init(C.byref(p), C.byref(h)) == lbm.LBM_E_INVAL
    assert "too large" in L.lbm_last_error(None).decode()


def test_batch_without_handles_is_rejected():
    L = pkg.load_library()
    b = C.c_void_p()
    assert L.lbm_batch_create(None, 0, C.byref(b)) == lbm.LBM_E_INVAL and not b.value
    arr = (C.c_void_p * 2)(None, None)
    assert L.lbm_batch_create(arr, 2, C.byref(b)) == lbm.LBM_E_INVAL
    assert "NULL" in L.lbm_batch_last_error(None).decode()
    assert L.lbm_batch_step(None, 1) == lbm.LBM_E_INVAL
    assert L.lbm_batch_set_graph(None, 1) == lbm.LBM_E_INVAL
    assert L.lbm_batch_set_schedule(None, 1) == lbm.LBM_E_INVAL
    L.lbm_batch_destroy(None)


def test_surrogate_entry_points_reject_bad_input_on_the_host():
    import numpy as np
    L = pkg.load_library()
    out = C.c_void_p()
    th = np.zeros(lbm.SURROGATE_PARAMS, np.float32)
    thp = th.ctypes.data_as(C.POINTER(C.c_float))
    assert L.lbm_surrogate_create(0, thp, C.byref(out)) == lbm.LBM_E_INVAL
    assert L.lbm_surrogate_create((1 << 20) + 1, thp, C.byref(out)) == lbm.LBM_E_INVAL
    assert L.lbm_surrogate_create(16, None, C.byref(out)) == lbm.LBM_E_INVAL
    assert b"max_samples" in L.lbm_surrogate_last_error(None)
    assert L.lbm_surrogate_create(16, thp, None) == lbm.LBM_E_INVAL
    assert L.lbm_surrogate_train(None, 1, 1e-3) == lbm.LBM_E_INVAL
    assert L.lbm_surrogate_predict(None, 1, None, None) == lbm.LBM_E_INVAL
    assert L.lbm_surrogate_cluster(None, 2, None, 1, None) == lbm.LBM_E_INVAL
    L.lbm_surrogate_destroy(None)
