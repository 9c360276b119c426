"""GPU parity of the cluster evolution driven by the network (lbm_surrogate_cluster)
against the CPU reference oracle/cluster.py.

The reference forms the separations and the network's inputs in float64 as defined; the
kernel forms them in float32 (reciprocals of the box and of the input scales), a few
float32 units away.  Both round the inputs to bfloat16 before the first product, so an
input lying within that distance of a bfloat16 rounding point may round to different
neighbours: ``cluster.input_flip_allowance`` takes the network's own output change across
that distance for each such pair (rare: about one pair in 10^4).  The kernel's network sums
in float32 on the matrix cores and takes tanh from the hardware exponential and
reciprocal (absolute error below 1e-6), where the reference sums and takes tanh in
float64.  Now and then that moves a hidden activation across a bfloat16 rounding boundary:
the activation then changes by one bfloat16 step (at most 2^-8 for |h| < 1), which
reaches the normalised output through weights of magnitude ~1/8 per layer, so about 1e-3
at most.  One step therefore agrees to 1e-4 of the sum of the pair-force magnitudes on
each capsule (float32 accumulation) plus 1e-3 of the output scale per partner in the
network's range (hidden-activation flips) plus the input-flip allowance plus one float32
rounding of each coordinate; twenty steps agree to 1e-3 of the distance travelled plus
twenty times the per-step flip allowances.
"""
import math

import numpy as np
import pytest

import synth
from oracle import cluster, mlp

pytestmark = pytest.mark.gpu

FLIP = 1e-3     # output change from a bfloat16 rounding flip of one hidden activation


def _theta(seed):
    rng = np.random.default_rng(seed)
    out = []
    for i in range(4):
        k, n = mlp.DIMS[i], mlp.DIMS[i + 1]
        out.append(rng.normal(0, 1 / math.sqrt(k), k * n))
        out.append(0.1 * rng.normal(size=n))
    return np.concatenate(out).astype(np.float32)


def _cfg(box):
    return dict(box=box, radius=10.0, features=[-1.2, 0.18, 90.0], in_mean=[4.0, -1.5, 0.2, 90.0],
                in_scale=[1.1, 0.5, 0.1, 1.0], out_mean=[0.0, 0.4], out_scale=[0.02, 0.3],
                r_contact=2.4, r_cut=6.0, k_contact=0.05, mobility=10.0)


def _kw(c):
    return {k: v for k, v in c.items()}


def _ulp(p):
    return np.spacing(np.abs(p).astype(np.float32)).astype(np.float64)


def _wrap(d, box):
    return (d + box / 2) % box - box / 2


def _one_step(n, packing, seed):
    from paper_2007_15405_amd import Surrogate
    th = _theta(seed)
    box, p = synth.cluster_film(n=n, packing=packing, min_sep=2.0, seed=seed)
    c = _cfg(box)
    s = Surrogate(th, 64)
    q = s.cluster(p, 1, **_kw(c))
    s.close()
    qo = cluster.step(th.astype(np.float64), p, c)
    d_gpu = _wrap(q.astype(np.float64) - p, box)
    d_or = _wrap(qo.astype(np.float64) - p, box)
    th64 = th.astype(np.float64)
    scale = c["mobility"] * cluster.pair_forces_abs(th64, p, c)
    flips = c["mobility"] * (FLIP * c["out_scale"][0] * cluster.network_partners(p, c) +
                             cluster.input_flip_allowance(th64, p, c))
    err = np.abs(d_gpu - d_or)
    bound = (1e-4 * scale + flips)[:, None] + 2 * _ulp(p)
    assert (scale > 0).mean() > 0.9
    assert np.abs(d_or).max() > 0.05
    assert np.all(err <= bound), (np.argmax(err / bound), (err / bound).max())


def test_one_step_small_ragged():
    _one_step(45, 0.3, 11)        # 2025 pairs: a ragged last tile


def test_one_step_full_size():
    _one_step(512, 0.25, 12)      # 512 capsules at 25 % coverage: 262144 pairs per step


def test_one_step_4096_capsules_sampled():
    """4096 capsules (16.8 M network evaluations per step, a 4096-block launch): 64
    sampled capsules against the oracle's step of those capsules."""
    from paper_2007_15405_amd import Surrogate
    th = _theta(15)
    box, p = synth.cluster_film(n=4096, packing=0.25, min_sep=2.0, seed=15)
    c = _cfg(box)
    s = Surrogate(th, 64)
    q = s.cluster(p, 1, **_kw(c))
    s.close()
    rows = np.random.default_rng(15).choice(4096, 64, replace=False)
    th64 = th.astype(np.float64)
    qo = cluster.step(th64, p, c, rows)
    d_gpu = _wrap(q[rows].astype(np.float64) - p[rows], box)
    d_or = _wrap(qo.astype(np.float64) - p[rows], box)
    scale = c["mobility"] * cluster.pair_forces_abs(th64, p, c, rows)
    flips = c["mobility"] * (FLIP * c["out_scale"][0] * cluster.network_partners(p, c, rows) +
                             cluster.input_flip_allowance(th64, p, c, rows))
    bound = (1e-4 * scale + flips)[:, None] + 2 * _ulp(p[rows])
    assert np.abs(d_or).max() > 0.05
    assert np.all(np.abs(d_gpu - d_or) <= bound)


def test_twenty_steps_follow_the_oracle():
    from paper_2007_15405_amd import Surrogate
    th = _theta(13)
    box, p = synth.cluster_film(n=96, packing=0.3, min_sep=2.0, seed=13)
    c = _cfg(box)
    s = Surrogate(th, 64)
    q = s.cluster(p, 20, **_kw(c))
    s.close()
    qo = p
    for _ in range(20):
        qo = cluster.step(th.astype(np.float64), qo, c)
    travel = np.abs(_wrap(qo.astype(np.float64) - p, box)).max()
    th64 = th.astype(np.float64)
    flips = 20 * c["mobility"] * (FLIP * c["out_scale"][0] * cluster.network_partners(p, c).max() +
                                  cluster.input_flip_allowance(th64, p, c).max())
    assert travel > 1.0
    assert np.abs(_wrap(q.astype(np.float64) - qo, box)).max() <= 1e-3 * travel + flips


def test_zero_steps_and_refusals():
    from paper_2007_15405_amd import LbmError, Surrogate
    th = _theta(14)
    box, p = synth.cluster_film(n=40, packing=0.3, seed=14)
    c = _cfg(box)
    s = Surrogate(th, 16)                          # the evolution needs no sample capacity
    with pytest.raises(LbmError):
        s.cluster(p[:1], 1, **_kw(c))              # a single capsule
    bad = _cfg(box)
    bad["r_cut"] = 2.0
    with pytest.raises(LbmError):
        s.cluster(p[:30], 1, **_kw(bad))           # cutoff inside contact
    small = _cfg(110.0)
    with pytest.raises(LbmError):
        s.cluster(p[:30] % 110.0, 1, **_kw(small))  # cutoff 60 above half the box
    assert np.array_equal(s.cluster(p[:30], 0, **_kw(c)), p[:30])
    one = s.cluster(p[:2], 1, **_kw(c))            # the smallest system: one pair
    assert np.all(np.isfinite(one))
    s.close()
