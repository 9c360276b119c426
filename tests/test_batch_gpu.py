"""GPU parity of the batched form: independent runs stacked as slabs of one lattice, and
several lattices advanced by one fluid launch (lbm_batch_*).

* Stacked slabs: each slab of a stacked lattice is compared with the oracle running that
  slab as a box of its own (same film, capsule shifted to the box's frame), to the
  tolerances of the plain parity tests (densities relative L2 <= 1e-5 after 200 steps,
  nodes 1e-4, meniscus 1e-3, mass 1e-5).  It is also compared with the library running
  the same box alone: the per-site arithmetic is the same, so results agree bit for bit.
* Batches: a batch of three lattices of different sizes (one with stacked slabs) ends in
  the state each handle reaches when stepped alone, also across a handle stepped outside
  the batch in between; one member is checked against the oracle.  The batched kernel is
  a separately compiled copy of the same per-site arithmetic, and the backend may fuse a
  few multiply-adds differently in it (about one ulp): densities agree to 1e-6 relative,
  as between the launch shapes of the fluid kernel, and nodes to 1e-5.
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


def shifted(cap, dz):
    c = dict(cap)
    c["center"] = [cap["center"][0], cap["center"][1], cap["center"][2] + dz]
    return c


# three slabs of 32 x 28 x 20 (28 is not a multiple of the tile height): films of 6, 9
# and 12 layers; a wetting capsule straddling the film in slab 0, none in slab 1, and a
# capsule pressed against its repulsive plane (Hertz active) in slab 2
NX, NY, LZ = 32, 28, 20
FILMS = [6.0, 9.0, 12.0]
SLAB_CAPS = {0: [synth.capsule((10.3, 14.2, 7.6), 4.0, 320, 0.02, wet_drho=0.05)],
             1: [],
             2: [synth.capsule((20.6, 9.1, 7.4), 4.0, 320, 0.05, anchor_k=0.5)]}


def box_cfg(s):
    """Slab s as a box of its own."""
    return synth.workload("pf", nx=NX, ny=NY, nz=LZ, film_height=FILMS[s], plane_dz=2.0,
                          capsules=SLAB_CAPS[s])


def stacked_cfg():
    caps = [shifted(c, s * LZ) for s in range(3) for c in SLAB_CAPS[s]]
    return synth.workload("pf", nx=NX, ny=NY, nz=3 * LZ, slab_nz=LZ, slab_film_height=FILMS,
                          plane_dz=2.0, capsules=caps)


@pytest.mark.parametrize("tile", [10, 1])
def test_stacked_slabs_match_the_oracle_box_by_box(tile):
    steps = 200
    say("stacked 3 x", (NX, NY, LZ), "tile", tile, "steps", steps)
    g = _sim(stacked_cfg())
    g.set_launch(tile, 4)     # z chunks of 4 planes: slab boundaries are chunk boundaries
    g.step(steps)
    ob = g.observables(rho=True, meniscus=True)
    assert ob["summary"]["unstable"] == 0 and ob["summary"]["lost_reaction"] == 0
    rho = ob["rho"].reshape(2, 3, LZ, NY, NX)
    k = 0
    for s in range(3):
        cfg = box_cfg(s)
        o = oracle.Oracle(cfg)
        o.step(steps)
        ro = o.rho()
        e = rel_l2(rho[:, s], ro)
        say("slab", s, "rel-L2 vs oracle", e)
        assert max(e) <= 1e-5
        site_check(rho[:, s], ro, 1e-5, f"slab {s} tile {tile}")
        so = o.summary()
        assert np.all(np.abs(ob["slab_mass"][s] - so["mass"]) / so["mass"] < 1e-5)
        mo, mg = o.meniscus(), ob["meniscus"][s]
        assert np.array_equal(np.isnan(mg), np.isnan(mo))
        ok = ~np.isnan(mo)
        assert ok.sum() > 100 and np.abs(mg[ok] - mo[ok]).max() <= 1e-3
        for j in range(len(SLAB_CAPS[s])):
            cg, co = ob["capsules"][k], o.capsule(j)
            dz = np.array([0.0, 0.0, s * LZ])
            assert np.abs(cg["centroid"] - dz - co["centroid"]).max() <= 1e-4
            assert np.abs(g.nodes(k) - dz - o.nodes(j)).max() <= 1e-4
            for f in ("f_capillary", "f_hertz", "f_anchor"):
                assert np.linalg.norm(cg[f] - co[f]) <= 1e-3 * max(np.linalg.norm(co[f]), 1e-3)
            if s == 2:
                assert abs(co["f_hertz"][2]) > 1e-3       # the plane contact is active
            k += 1
        # the same box run alone by the library: identical arithmetic, identical result
        a = _sim(cfg)
        a.set_launch(tile, 4)
        a.step(steps)
        assert np.array_equal(rho[:, s], a.rho())
        a.close()
    lab = g.labels().reshape(3, LZ, NY, NX)
    assert np.all(lab[:, 0] == 255)
    g.close()


def test_capsule_window_must_stay_inside_its_slab():
    from paper_2007_15405_amd import LbmError
    g = _sim(synth.workload("pf", nx=NX, ny=NY, nz=2 * LZ, slab_nz=LZ, capsules=[]))
    for cz in (LZ - 3.0, LZ + 2.5):     # window through the wall layer above / below
        cap = synth.capsule((16.0, 14.0, cz), 3.0, 320, 0.02)
        nodes, tris = synth.capsule_mesh(cap)
        with pytest.raises(LbmError) as ei:
            g.add_capsule(cap, nodes, tris)
        assert ei.value.status == -1
    cap = synth.capsule((16.0, 14.0, LZ + 8.0), 3.0, 320, 0.02)
    g.add_capsule(cap, *synth.capsule_mesh(cap))
    g.close()


def batch_members():
    a = stacked_cfg()                                      # 32 x 28 x 60, three slabs
    b = synth.workload("pf", nx=48, ny=40, nz=24, film_height=8.0, plane_dz=2.0,
                       capsules=[synth.capsule((30.5, 12.2, 8.3), 4.0, 320, 0.05,
                                               anchor_k=0.5),
                                 synth.capsule((20.1, 20.7, 9.1), 4.0, 320, 0.02)])
    c = synth.workload("pf", nx=40, ny=16, nz=36, slab_nz=12, film_height=5.0, capsules=[])
    return [a, b, c]


def test_batch_equals_handles_stepped_alone():
    from paper_2007_15405_amd import Batch
    cfgs = batch_members()
    sims = [_sim(c) for c in cfgs]
    refs = [_sim(c) for c in cfgs]
    for x in sims + refs:
        x.set_launch(10, 4)   # for the step taken outside the batch, and the references
    bt = Batch(sims, tile=10, zchunk=4)
    say("batch of", [(c["nx"], c["ny"], c["nz"], c["slab_nz"]) for c in cfgs])
    bt.step(31)
    sims[1].step(1)           # a member stepped on its own: the batch rebuilds its tables
    bt.step(30)
    for i, r in enumerate(refs):
        r.step(62 if i == 1 else 61)
    for i, (s, r) in enumerate(zip(sims, refs)):
        a, b = s.rho(), r.rho()
        d = float(np.abs(a - b).max())
        say("member", i, "max |diff| vs alone", d)
        assert d <= 1e-6 * float(np.abs(b).max())
        for k in range(len(cfgs[i]["capsules"])):
            assert np.abs(s.nodes(k) - r.nodes(k)).max() <= 1e-5
        assert s.summary()["step"] == r.summary()["step"]
    o = oracle.Oracle(cfgs[1])
    o.step(62)
    e = rel_l2(sims[1].rho(), o.rho())
    say("member 1 vs oracle", e)
    assert max(e) <= 1e-5
    for k in range(2):
        assert np.abs(sims[1].nodes(k) - o.nodes(k)).max() <= 1e-4
    for tile, zc in ((6, 8), (13, 8), (13, 0)):   # other tiles and z chunks: the same
        bt.set_launch(tile, zc)                   # result up to rounding
        bt.step(5)
        for i, r in enumerate(refs):
            r.step(5)
            a, b = sims[i].rho(), r.rho()
            d = float(np.abs(a - b).max())
            say("member", i, "tile", tile, "zchunk", zc, "max |diff|", d)
            assert d <= 1e-6 * float(np.abs(b).max())
    for parts in (2, 3):      # members split over streams of the batch's own
        bt.set_parts(parts)
        bt.step(7)
        for i, r in enumerate(refs):
            r.step(7)
            a, b = sims[i].rho(), r.rho()
            d = float(np.abs(a - b).max())
            say("parts", parts, "member", i, "max |diff|", d)
            assert d <= 1e-6 * float(np.abs(b).max())
            for k in range(len(cfgs[i]["capsules"])):
                assert np.abs(sims[i].nodes(k) - r.nodes(k)).max() <= 1e-5
            assert sims[i].summary()["step"] == r.summary()["step"]
    bt.close()


def test_batch_rejects_unequal_relaxation_times():
    from paper_2007_15405_amd import Batch, LbmError
    a = _sim(synth.workload("pf", nx=8, ny=8, nz=8, capsules=[]))
    b = _sim(synth.workload("pf", nx=8, ny=8, nz=8, capsules=[], tau=[0.8, 1.0]))
    with pytest.raises(LbmError):
        Batch([a, b])
    with pytest.raises(LbmError):
        Batch([a, a])


def test_full_batch_workload_sampled_instances():
    """The batched workload the benchmark times (64 capsule-pair boxes in 8 groups of
    stacked slabs, one batch), a few steps, in its default launch shape; the first and the
    last instance against the oracle running them as boxes of their own."""
    from paper_2007_15405_amd import Batch
    inst = synth.batch_instances()
    groups = synth.batch_groups(inst)
    say("batch workload:", len(inst), "instances in", len(groups), "groups")
    sims = [_sim(g, meshes=synth.capsule_meshes(g["capsules"])) for g in groups]
    bt = Batch(sims)
    steps = 3
    bt.step(steps)
    bt.sync()
    for k in (0, len(inst) - 1):
        gi = next(j for j, g in enumerate(groups) if k in g["instances"])
        g, sim = groups[gi], sims[gi]
        s = g["instances"].index(k)
        lz = g["slab_nz"]
        ob = sim.observables(rho=True)
        rho = ob["rho"].reshape(2, -1, lz, g["ny"], g["nx"])[:, s]
        i = inst[k]
        cfg = synth.workload("c2", nx=i["nx"], ny=i["ny"], nz=i["nz"],
                             film_height=i["film_height"], capsules=i["capsules"])
        o = oracle.Oracle(cfg)
        o.step(steps)
        e = rel_l2(rho, o.rho())
        say("instance", k, "box", (i["nx"], i["ny"], i["nz"]), "slab", s, "of group", gi,
            "rel-L2", e)
        assert max(e) <= 1e-6
        for j in range(2):
            cg = ob["capsules"][2 * s + j]
            co = o.capsule(j)
            assert np.abs(cg["centroid"] - np.array([0, 0, s * lz]) - co["centroid"]).max() <= 1e-5
            assert np.linalg.norm(cg["f_capillary"] - co["f_capillary"]) <= \
                1e-3 * max(np.linalg.norm(co["f_capillary"]), 1e-3)
        assert ob["summary"]["lost_reaction"] == 0
    bt.close()


BENCH_STEPS = 200


@pytest.fixture(scope="module")
def batch_reference():
    """The oracle running the first and the last instance of the batched workload as boxes
    of their own for BENCH_STEPS steps."""
    inst = synth.batch_instances()
    ref = {}
    for k in (0, len(inst) - 1):
        i = inst[k]
        cfg = synth.workload("c2", nx=i["nx"], ny=i["ny"], nz=i["nz"],
                             film_height=i["film_height"], capsules=i["capsules"])
        say("oracle: batch instance", k, (i["nx"], i["ny"], i["nz"]), BENCH_STEPS, "steps")
        o = oracle.Oracle(cfg)
        o.step(BENCH_STEPS)
        ref[k] = dict(rho=o.rho(), meniscus=o.meniscus(), caps=[o.capsule(j) for j in range(2)],
                      mass=o.summary()["mass"])
        o.close()
    return inst, ref


@pytest.mark.parametrize("launch", [(13, 16, 3), "tuned"])
def test_batch_instances_in_benchmark_launch_match_the_oracle(batch_reference, launch):
    """The batched workload in the launch shape behind the batched figures and the
    surrogate's training data (whole rows of the box width, z-chunks of 16 planes, three
    parts), and in the shape the library's autotuner picks: 200 steps, then the first and
    the last instance against the oracle, every site checked."""
    from paper_2007_15405_amd import Batch
    inst, ref = batch_reference
    groups = synth.batch_groups(inst)
    sims = [_sim(g, meshes=synth.capsule_meshes(g["capsules"])) for g in groups]
    if launch == "tuned":
        bt = Batch(sims, parts=1)
        bt.step(1)
        t = bt.autotune(3)
        say("batch autotuner choice:", t)
        bt.step(BENCH_STEPS - 1)
    else:
        bt = Batch(sims, tile=launch[0], zchunk=launch[1], parts=launch[2])
        bt.step(BENCH_STEPS)
    bt.sync()
    for k, r in ref.items():
        gi = next(j for j, g in enumerate(groups) if k in g["instances"])
        g, sim = groups[gi], sims[gi]
        s = g["instances"].index(k)
        lz = g["slab_nz"]
        ob = sim.observables(rho=True, meniscus=True)
        rho = ob["rho"].reshape(2, -1, lz, g["ny"], g["nx"])[:, s]
        lab = sim.labels().reshape(-1, lz, g["ny"], g["nx"])[s]
        e = rel_l2(rho, r["rho"])
        say("instance", k, "launch", launch, "rel-L2", e)
        assert max(e) <= 1e-5
        site_check(rho, r["rho"], 1e-5, f"batch instance {k} launch {launch}", lab)
        assert np.all(np.abs(ob["slab_mass"][s] - r["mass"]) / r["mass"] < 1e-5)
        men = ob["meniscus"].reshape(-1, g["ny"], g["nx"])[s]
        assert np.array_equal(np.isnan(men), np.isnan(r["meniscus"]))
        ok = ~np.isnan(men)
        assert np.abs(men[ok] - r["meniscus"][ok]).max() <= 1e-3
        for j in range(2):
            cg, co = ob["capsules"][2 * s + j], r["caps"][j]
            assert np.abs(cg["centroid"] - np.array([0, 0, s * lz]) - co["centroid"]).max() <= 1e-4
            for f in ("f_capillary", "f_anchor"):
                assert np.linalg.norm(cg[f] - co[f]) <= 1e-3 * max(np.linalg.norm(co[f]), 1e-3)
        assert ob["summary"]["lost_reaction"] == 0
    bt.close()
    for x in sims:
        x.close()


def test_checkpoint_resume_with_slabs_is_bitwise(tmp_path):
    a = _sim(stacked_cfg())
    a.step(40)
    path = str(tmp_path / "slabs.bin")
    a.save(path)
    a.step(40)
    b = _sim(stacked_cfg())
    b.step(2)
    b.load(path)
    b.step(40)
    assert np.array_equal(a.rho(), b.rho())
    for k in range(2):
        assert np.array_equal(a.nodes(k), b.nodes(k))
    oa, ob = a.observables(meniscus=True), b.observables(meniscus=True)
    assert np.array_equal(oa["slab_mass"], ob["slab_mass"])
    assert np.array_equal(np.nan_to_num(oa["meniscus"], nan=-1), np.nan_to_num(ob["meniscus"], nan=-1))
    # a handle with another slab height refuses the checkpoint
    from paper_2007_15405_amd import LbmError
    c = _sim(synth.workload("pf", nx=NX, ny=NY, nz=3 * LZ, slab_nz=3 * LZ, capsules=[]))
    with pytest.raises(LbmError):
        c.load(path)


@pytest.mark.parametrize("storage,tol", [("f16", 1e-3), ("bf16", 8e-3)])
def test_batch_with_16bit_storage_tracks_handles_stepped_alone(storage, tol):
    """16-bit storage: the one-ulp FP32 differences between the batched and the single
    kernel can flip the rounding of a stored population by one 16-bit ulp (2^-11
    relative for FP16, 2^-8 for BF16), which then spreads; the bound is set on that
    scale (relative L2 after 40 steps)."""
    from paper_2007_15405_amd import Batch
    cfgs = batch_members()[:2]
    sims = [_sim(c, storage=storage) for c in cfgs]
    refs = [_sim(c, storage=storage) for c in cfgs]
    for r in refs:
        r.set_launch(10, 4)
    bt = Batch(sims, tile=10, zchunk=4, parts=2)
    bt.step(40)
    for i, r in enumerate(refs):
        r.step(40)
        e = rel_l2(sims[i].rho(), r.rho())
        say(storage, "member", i, "rel-L2 vs alone", e)
        assert max(e) <= tol
        assert sims[i].summary()["unstable"] == 0
    bt.close()


@pytest.mark.parametrize("parts", [1, 2])
def test_graph_replay_equals_enqueued_steps(parts):
    """lbm_batch_set_graph: pairs of steps replayed from a captured graph give the same bits
    as the same steps enqueued one by one.  Replays are checked one at a time, with the
    program's own work (observables, synchronisation) between them; an odd step count, a
    member stepped alone (the graphs are recorded again) and event timing (steps enqueued
    as usual) are covered."""
    from paper_2007_15405_amd import Batch
    cfgs = batch_members()
    sims = [_sim(c) for c in cfgs]
    refs = [_sim(c) for c in cfgs]
    for x in sims + refs:
        x.set_launch(10, 4)
    bg = Batch(sims, tile=10, zchunk=4, parts=parts)
    br = Batch(refs, tile=10, zchunk=4, parts=parts)
    bg.set_graph(True)

    def same(tag):
        for i, (s, r) in enumerate(zip(sims, refs)):
            assert np.array_equal(s.rho(), r.rho()), f"{tag}: member {i} densities"
            for k in range(len(cfgs[i]["capsules"])):
                assert np.array_equal(s.nodes(k), r.nodes(k)), f"{tag}: member {i} nodes"
            ss = s.summary()
            assert ss["step"] == r.summary()["step"] and ss["unstable"] == 0, tag

    for rep in range(4):          # one graph launch per call, checked after each
        bg.step(2)
        br.step(2)
        same(f"replay {rep}")
    bg.step(5)                    # two replays and an enqueued step: the other parity next
    br.step(5)
    same("odd count")
    bg.step(4)
    br.step(4)
    same("replays from parity 1")
    sims[1].step(1)               # tables rewritten: graphs recorded again
    refs[1].step(1)
    bg.step(6)
    br.step(6)
    same("after a member stepped alone")
    bg.set_profiling(1)           # timed steps are enqueued
    bg.step(2)
    br.step(2)
    bg.set_profiling(0)
    same("timed")
    say("graph replay, parts", parts, ": bit-identical after", sims[0].summary()["step"], "steps")
    bg.close()
    br.close()


@pytest.mark.parametrize("tile", [10, 13])
def test_work_queue_schedule_gives_the_same_bits(tile):
    """lbm_batch_set_schedule(1): the fluid launch as a resident grid taking tiles from a
    device work queue (the queue clears itself at the end of each launch, also inside a
    replayed graph) gives the same bits as one workgroup per tile."""
    from paper_2007_15405_amd import Batch
    cfgs = batch_members()
    sims = [_sim(c) for c in cfgs]
    refs = [_sim(c) for c in cfgs]
    bq = Batch(sims, tile=tile, zchunk=4, parts=2)
    br = Batch(refs, tile=tile, zchunk=4, parts=2)
    bq.set_schedule(True)
    bq.step(9)
    br.step(9)
    bq.set_graph(True)
    bq.step(6)
    br.step(6)
    for i, (s, r) in enumerate(zip(sims, refs)):
        assert np.array_equal(s.rho(), r.rho()), f"member {i}"
        for k in range(len(cfgs[i]["capsules"])):
            assert np.array_equal(s.nodes(k), r.nodes(k))
    say("work queue, tile", tile, ": bit-identical after 15 steps")
    bq.close()
    br.close()
