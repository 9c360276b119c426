"""The CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host code only):
the driver ``oracle/lbmref_sanitize`` runs a film box with two capsules exercising every
membrane term (Skalak, bending, volume penalty, wetting offsets, Hertz contact between the
capsules and with the plane, anchor) and every pure helper, with the immersed-boundary and
with the bounce-back coupling, and must finish without a finding; its observables must
equal those of the regular build of the same oracle."""
import os
import subprocess

import numpy as np
import pytest

import oracle
import synth
from oracle import build as oracle_build

STEPS = 12


def _case(coupling):
    caps = [synth.capsule((7.5, 12.0, 7.0), 4.0, 320, 0.05, kb=0.03, kv=0.3, wet_drho=0.05,
                          anchor_k=0.5),
            synth.capsule((16.4, 12.3, 7.2), 4.0, 320, 0.02, kb=0.0, kv=0.0, wet_drho=-0.03)]
    return synth.workload("pf", nx=24, ny=24, nz=20, film_height=6.0, plane_dz=2.0,
                          wall_drho=0.02, tau=[1.0, 0.9], coupling=coupling, capsules=caps)


def _write(cfg, path):
    lines = [f"{cfg['nx']} {cfg['ny']} {cfg['nz']} {cfg['wall_z0']} {cfg['init_mode']} "
             f"{cfg['film_height']!r} {STEPS} {len(cfg['capsules'])} {cfg['body_force'][0]!r} "
             f"{cfg['wall_drho']!r} {cfg['tau'][0]!r} {cfg['tau'][1]!r} {cfg['coupling']} "
             f"{cfg['node_mass']!r}"]
    for cap in cfg["capsules"]:
        x, t = synth.capsule_mesh(cap)
        lines.append(f"{len(x)} {len(t)} {cap['ks']!r} {cap['C']!r} {cap['kb']!r} {cap['kv']!r} "
                     f"{cap['wet_drho']!r} {cap['anchor_k']!r}")
        lines += [" ".join(repr(float(v)) for v in row) for row in x]
        lines += [" ".join(str(int(v)) for v in row) for row in t]
    path.write_text("\n".join(lines) + "\n")


@pytest.mark.parametrize("coupling", [0, 1])
def test_oracle_runs_clean_under_sanitizers(tmp_path, coupling):
    exe = oracle_build.build_sanitized()
    cfg = _case(coupling)
    case = tmp_path / "case.txt"
    _write(cfg, case)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1", OMP_NUM_THREADS="2")
    r = subprocess.run([exe, str(case)], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
    got = dict(ln.split() for ln in r.stdout.strip().split("\n"))
    assert int(got["status"]) == 0 and int(got["step"]) == STEPS
    # the same observables from the regular build
    o = oracle.Oracle(cfg)
    o.step(STEPS)
    s = o.summary()
    assert float(got["mass0"]) == pytest.approx(s["mass"][0], rel=1e-13)
    assert float(got["mass1"]) == pytest.approx(s["mass"][1], rel=1e-13)
    for k in range(2):
        c = o.capsule(k)
        for d in range(3):
            assert float(got[f"cap{k}_centroid{d}"]) == pytest.approx(c["centroid"][d], abs=1e-12)
            for f in ("f_anchor", "f_capillary", "f_hertz", "f_fluid"):
                assert float(got[f"cap{k}_{f}{d}"]) == pytest.approx(c[f][d], abs=1e-12)
        assert float(got[f"cap{k}_volume"]) == pytest.approx(c["volume"], rel=1e-12)
    m = o.meniscus()
    assert int(got["meniscus_count"]) == int(np.isfinite(m).sum())
    assert float(got["meniscus_sum"]) == pytest.approx(float(np.nansum(m)), rel=1e-12)
    if coupling == 0:
        assert abs(o.capsule(0)["f_hertz"]).max() > 1e-4  # the contact terms ran
    for d in range(3):
        assert float(got[f"node_momentum{d}"]) == pytest.approx(s["node_momentum"][d], abs=1e-12)
    assert int(got["links"]) == s["links"]
    if coupling == 1:
        assert s["links"] > 500
