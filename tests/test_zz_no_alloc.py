"""The allocation-free cluster evolution (lbm_surrogate_cluster_noalloc) against the
allocating entry point (lbm_surrogate_cluster): the same kernels on the same inputs, so
the positions must agree bit for bit.  Two calls in a row on one GPU (the file-scope
scratch keeps the first call's contents), the second with fewer capsules and an odd step
count (its result then passes through the scratch); and the size limit is refused."""
import math

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _theta(seed):
    rng = np.random.default_rng(seed)
    out = []
    for k, n in ((4, 64), (64, 64), (64, 64), (64, 2)):
        out.append(rng.normal(0, 1 / math.sqrt(k), k * n))
        out.append(0.1 * rng.normal(size=n))
    return np.concatenate(out).astype(np.float32)


def _cfg(box):
    return dict(box=box, radius=10.0, features=[-1.2, 0.18, 90.0], in_mean=[4.0, -1.5, 0.2, 90.0],
                in_scale=[1.1, 0.5, 0.1, 1.0], out_mean=[0.0, 0.4], out_scale=[0.02, 0.3],
                r_contact=2.4, r_cut=6.0, k_contact=0.05, mobility=10.0)


def test_noalloc_matches_the_allocating_entry_point_twice():
    import torch

    from paper_2007_15405_amd import Surrogate
    s = Surrogate(_theta(21), 16)
    for n, steps, seed in ((700, 6, 21), (96, 5, 22)):   # second call: smaller, odd steps
        box, p = synth.cluster_film(n=n, packing=0.25, min_sep=2.0, seed=seed)
        c = _cfg(box)
        want = s.cluster(p, steps, **c)
        dev = torch.from_numpy(p.copy()).cuda()
        got = s.cluster_noalloc(dev, steps, **c).cpu().numpy()
        print("n", n, "steps", steps, "max |diff|", float(np.abs(got - want).max()), flush=True)
        assert np.abs(want - p).max() > 1e-3          # the capsules moved
        assert np.array_equal(got, want)
    s.close()


def test_noalloc_refuses_more_capsules_than_its_scratch_holds():
    import torch

    from paper_2007_15405_amd import LbmError, Surrogate, lbm
    s = Surrogate(_theta(23), 16)
    n = lbm.CLUSTER_NOALLOC_MAX + 1
    dev = torch.zeros((n, 2), dtype=torch.float32, device="cuda")
    with pytest.raises(LbmError) as ei:
        s.cluster_noalloc(dev, 1, **_cfg(4000.0))
    assert ei.value.status == -1
    s.close()
