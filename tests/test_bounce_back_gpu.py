"""GPU parity of the bounce-back coupling (Section 3.1: half-way bounce-back on the moving
membrane with momentum exchange, homogeneous weighting, two-step smoothing, Newtonian
nodes of mass 25 rho0) against the oracle's bounce-back coupling.

Tolerances (FP32 kernels against the FP64 oracle): densities relative L2 and every single
site within 1e-5 of the component's largest density; node positions within 1e-3 lattice
units (as for the immersed boundary's film and capsule run); the labels and the link count
equal (both sides take every geometric decision on the FP32-rounded node positions, in
double precision, with the same rules); the fluid force on the capsule within 1e-3 of its
size.

Which triangle a link crosses, and on which side of the membrane a site lies, are discrete
decisions.  The kernels keep the nodes in FP64 but sum their forces in FP32, so their node
positions drift from the oracle's by 1e-7 .. 1e-6 lattice units; a link that passes within
that distance of a triangle edge can then be credited to the neighbouring triangle (both are
valid choices), which moves the three nodes of each by about 1e-3 of a lattice unit.  A
capsule centred on a lattice point has mirror planes that contain lattice links, whose
crossings lie exactly on edges; the capsules here are placed off those planes, and the run
lengths are such that no such event occurs (measured: with the centre at a lattice point the
node error jumps to 1e-3 within 20 steps; off it, ks = 0.3 stays at 2e-6 over 300 steps).
The node sums are fixed point on the GPU, so runs are bitwise reproducible and a checkpoint
resumes bit for bit.
"""
import numpy as np
import pytest

import oracle
import synth
from parity_tools import rel_l2, say, site_check

pytestmark = pytest.mark.gpu


def _sim(cfg, **kw):
    from paper_2007_15405_amd import Sim
    return Sim(cfg, **kw)


def run_pair(cfg, steps, **kw):
    say("bounce-back case", {k: cfg[k] for k in ("nx", "ny", "nz", "wall_z0", "init_mode")},
        "caps", [(c["radius"], c["n_tri"], c["ks"]) for c in cfg["capsules"]], "steps", steps)
    g = _sim(cfg, **kw)
    o = oracle.Oracle(cfg)
    g.step(steps)
    o.step(steps)
    return g, o


def check_capsules(g, o, n, node_tol=1e-3):
    for k in range(n):
        cg, co = g.capsule(k), o.capsule(k)
        err = float(np.abs(g.nodes(k) - o.nodes(k)).max())
        say("capsule", k, "node error", err, "f_fluid gpu", cg["f_fluid"].round(6),
            "oracle", co["f_fluid"].round(6))
        assert err <= node_tol
        assert np.abs(cg["centroid"] - co["centroid"]).max() <= node_tol
        assert abs(cg["volume"] - co["volume"]) / co["volume"] <= 1e-5
        for f in ("f_fluid", "f_capillary", "f_hertz", "f_anchor"):
            assert np.linalg.norm(cg[f] - co[f]) <= 1e-3 * max(np.linalg.norm(co[f]), 1e-3), f


def test_labels_and_links_after_the_first_step():
    cfg = synth.workload("pf", coupling=1)      # centred on a lattice point: exact ties
    g, o = run_pair(cfg, 1)
    assert np.array_equal(g.labels(), o.labels())
    sg, so = g.summary(), o.summary()
    say("links gpu", sg["links"], "oracle", so["links"])
    assert sg["links"] == so["links"] > 2000
    assert sg["lost_links"] == so["lost_links"] == 0


CENTRE = (16.23, 15.81, 10.17)    # off the lattice's symmetry planes


@pytest.mark.parametrize("ks,steps", [(0.01, 100), (0.3, 300), (1.0, 100)])
def test_film_with_capsule(ks, steps):
    """The film with a capsule straddling its interface (32^3): a soft capsule that the
    interface deforms, a stiffer one beyond the immersed boundary's reach, and the stiffest
    the explicit node update of the paper's scheme keeps stable at node mass 25."""
    cfg = synth.workload("pf", coupling=1, capsules=[synth.capsule(CENTRE, 6.0, 1280, ks)])
    g, o = run_pair(cfg, steps)
    rg, ro = g.rho(), o.rho()
    e = rel_l2(rg, ro)
    say("bounce-back film rel-L2", e)
    assert max(e) <= 1e-5
    site_check(rg, ro, 1e-5, f"bounce-back film ks={ks} {steps} steps", g.labels())
    check_capsules(g, o, 1)
    assert np.array_equal(g.labels(), o.labels())
    sg, so = g.summary(), o.summary()
    assert sg["links"] == so["links"]
    assert sg["lost_links"] == 0 and sg["unstable"] == 0
    assert np.abs(sg["mass"] - so["mass"]).max() <= 1e-5 * so["mass"].max()
    mg, mo = g.meniscus(), o.meniscus()
    assert np.array_equal(np.isnan(mg), np.isnan(mo))
    ok = ~np.isnan(mo)
    assert np.abs(mg[ok] - mo[ok]).max() <= 1e-3


def test_wide_window_sorts_its_triangles_in_passes():
    """An R = 20 capsule of 5120 triangles on a 64 x 64 x 56 film: its window (floor of the
    node extent + 4 sites per axis, 44^3 = 85,184 cells) holds more than five times the 16384
    cell counters the triangle sort keeps in LDS, so the sort takes six passes over cell
    ranges.  Labels, link counts, densities and nodes against the oracle after 10 steps."""
    cfg = synth.workload("pf", nx=64, ny=64, nz=56, coupling=1,
                         capsules=[synth.capsule((32.23, 31.81, 22.17), 20.0, 5120, 0.05)])
    g, o = run_pair(cfg, 10)
    n = o.nodes(0)
    cells = int(np.prod(np.floor(n.max(0)) - np.floor(n.min(0)) + 4))
    say("window cells", cells)
    assert cells > 5 * 16384
    rg, ro = g.rho(), o.rho()
    assert max(rel_l2(rg, ro)) <= 1e-5
    site_check(rg, ro, 1e-5, "bounce-back wide window 10 steps", g.labels())
    check_capsules(g, o, 1)
    assert np.array_equal(g.labels(), o.labels())
    sg, so = g.summary(), o.summary()
    say("links gpu", sg["links"], "oracle", so["links"])
    assert sg["links"] == so["links"] > 20000
    assert sg["lost_links"] == 0 and sg["unstable"] == 0


def test_wetting_capsules_in_contact_on_a_ragged_periodic_box():
    """Two wetting capsules with a volume penalty pressed into Hertz contact, on a box
    whose sizes are no tile multiples, one capsule across the periodic boundary."""
    rho = synth.noise_rho(27, 21, 22, (0.7, 0.04), 0.02, seed=9)
    caps = [synth.capsule((2.1, 10.3, 11.2), 4.0, 320, 0.05, kv=0.3, wet_drho=0.05),
            synth.capsule((11.0, 10.6, 11.0), 4.0, 320, 0.02, wet_drho=-0.04)]
    cfg = synth.workload("pf", nx=27, ny=21, nz=22, wall_z0=0, init_mode=2, init_rho_array=rho,
                         coupling=1, capsules=caps)
    g, o = run_pair(cfg, 100)
    rg, ro = g.rho(), o.rho()
    assert max(rel_l2(rg, ro)) <= 1e-5
    site_check(rg, ro, 1e-5, "bounce-back ragged", g.labels(), wall=False)
    check_capsules(g, o, 2)
    assert g.summary()["links"] == o.summary()["links"]


def test_momentum_of_fluid_and_nodes_is_conserved_on_gpu():
    rho = synth.noise_rho(24, 24, 24, (0.7, 0.04), 0.05, seed=11)
    cfg = synth.workload("pf", wall_z0=0, nx=24, ny=24, nz=24, init_mode=2, init_rho_array=rho,
                         coupling=1, capsules=[synth.capsule((12.2, 11.7, 12.4), 5.0, 1280, 0.05,
                                                             kv=0.5, wet_drho=0.05)])
    g = _sim(cfg)
    s = g.summary()

    def total(s):
        return s["momentum"] + s["node_momentum"] + s["pending"]

    P0 = total(s)
    g.step(200)
    s = g.summary()
    say("momentum drift", total(s) - P0, "node momentum", s["node_momentum"])
    assert np.abs(total(s) - P0).max() < 1e-5 * s["mass"].sum() / 1000
    assert np.abs(s["node_momentum"]).max() > 1e-7


def test_film_drying_box_two_capsules():
    """The film box of two R = 10 capsules (5120 triangles each) at separation 3R, anchored,
    with the shear modulus 0.5 (above the immersed boundary's limit of about 0.3)."""
    cfg = synth.workload("c2", ks=0.5, coupling=1)
    for c, dc in zip(cfg["capsules"], ((0.31, 0.22, 0.13), (0.17, -0.29, 0.13))):
        c["center"] = [c["center"][d] + dc[d] for d in range(3)]   # off the symmetry planes
    g, o = run_pair(cfg, 40)
    rg, ro = g.rho(), o.rho()
    assert max(rel_l2(rg, ro)) <= 1e-5
    site_check(rg, ro, 1e-5, "bounce-back c2", g.labels())
    check_capsules(g, o, 2)
    assert g.summary()["links"] == o.summary()["links"]


def test_bounce_back_runs_are_bitwise_deterministic_and_resume(tmp_path):
    cfg = synth.workload("pf", coupling=1,
                         capsules=[synth.capsule(CENTRE, 6.0, 1280, 0.05, kv=0.2)])
    a, b = _sim(cfg), _sim(cfg)
    a.step(80)
    b.step(80)
    assert np.array_equal(a.rho(), b.rho()) and np.array_equal(a.nodes(0), b.nodes(0))
    path = str(tmp_path / "bb.bin")
    a.save(path)
    a.step(60)
    c = _sim(cfg)
    c.step(2)
    c.load(path)
    c.step(60)
    assert np.array_equal(a.rho(), c.rho())
    assert np.array_equal(a.nodes(0), c.nodes(0))
    sa, sc = a.summary(), c.summary()
    assert np.array_equal(sa["node_momentum"], sc["node_momentum"])


@pytest.mark.parametrize("storage,tol", [("f16", 1e-2)])
def test_bounce_back_with_16bit_storage_tracks_the_oracle(storage, tol):
    cfg = synth.workload("pf", coupling=1, capsules=[synth.capsule(CENTRE, 6.0, 1280, 0.01)])
    g, o = run_pair(cfg, 100, storage=storage)
    e = rel_l2(g.rho(), o.rho())
    say(storage, "bounce-back rel-L2", e, "node error", np.abs(g.nodes(0) - o.nodes(0)).max())
    assert max(e) <= tol
    assert np.abs(g.nodes(0) - o.nodes(0)).max() <= 5e-2


def test_batches_refuse_bounce_back_handles():
    from paper_2007_15405_amd import Batch, LbmError
    a = _sim(synth.workload("pf", nx=8, ny=8, nz=8, capsules=[], coupling=1))
    with pytest.raises(LbmError):
        Batch([a])
