"""Host-side logic of the batched form (no GPU): the sampled capsule-pair instances stay
inside their stated ranges, stacking them by box size keeps every instance once with its
film and capsules moved into its slab, and every capsule's site window lies between the
wall layers of its slab (the condition the library enforces when a capsule is added)."""
import math

import numpy as np
import pytest

import oracle
import synth


def test_instances_follow_the_sampling_ranges():
    inst = synth.batch_instances()
    assert len(inst) == 64
    R = 10.0
    for i in inst:
        assert 2.2 * R <= i["L"] <= 6.0 * R
        assert 0.002 <= i["ks"] <= 0.2
        film_above_plane = i["film_height"] - 10.0
        assert 0.4 * 2 * R - 0.5 <= film_above_plane <= 0.9 * 2 * R + 0.5
        assert i["nx"] == min(max(16 * math.ceil((2 * i["L"] + 2 * R) / 16), 64), 128)
        assert i["ny"] == 3 * i["nx"] // 4 and i["nz"] in (40, 48)
        a, b = (np.array(c["center"]) for c in i["capsules"])
        assert abs(np.linalg.norm(a - b) - i["L"]) < 1e-9
        assert all(c["ks"] == i["ks"] and c["anchor_k"] == 1.0 for c in i["capsules"])
    assert synth.batch_instances() == inst          # seeded


def test_groups_stack_every_instance_once():
    inst = synth.batch_instances()
    groups = synth.batch_groups(inst)
    seen = sorted(k for g in groups for k in g["instances"])
    assert seen == list(range(len(inst)))
    for g in groups:
        lz = g["slab_nz"]
        assert g["nz"] == lz * len(g["instances"]) and g["wall_z0"] == 1
        assert len(g["capsules"]) == 2 * len(g["instances"]) <= 125
        for s, k in enumerate(g["instances"]):
            i = inst[k]
            assert (i["nx"], i["ny"], i["nz"]) == (g["nx"], g["ny"], lz)
            assert g["slab_film_height"][s] == i["film_height"]
            for j in range(2):
                cg, ci = g["capsules"][2 * s + j], i["capsules"][j]
                assert cg["center"][2] == ci["center"][2] + s * lz
                assert cg["center"][:2] == ci["center"][:2]


def test_capsule_windows_stay_inside_their_slabs():
    inst = synth.batch_instances()
    groups = synth.batch_groups(inst)
    for g in groups:
        lz = g["slab_nz"]
        for c, (nodes, _) in zip(g["capsules"], synth.capsule_meshes(g["capsules"])):
            z = nodes[:, 2].astype(np.float32)
            base = int(math.floor(float(np.mean(nodes[:, 2])) / lz)) * lz
            assert math.floor(z.min()) - 1 >= base and math.floor(z.max()) + 2 <= base + lz
            for d, n in ((0, g["nx"]), (1, g["ny"])):
                v = nodes[:, d].astype(np.float32)
                assert math.floor(v.max()) - math.floor(v.min()) + 4 <= min(64, n)


def test_shared_unit_sphere_meshes_are_the_same_bits():
    caps = synth.batch_instances()[5]["capsules"]
    for c, (n, t) in zip(caps, synth.capsule_meshes(caps)):
        n0, t0 = synth.capsule_mesh(c)
        assert np.array_equal(n, n0) and np.array_equal(t, t0)


def test_oracle_runs_one_box_only():
    cfg = synth.workload("pf", nz=64, slab_nz=32, capsules=[])
    with pytest.raises(ValueError):
        oracle.Oracle(cfg)
