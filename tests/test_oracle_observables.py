"""Pins of the oracle's observables of the validation section (Section 4.1): the meniscus
height of every lattice column and the lateral force sampled on a fixed (anchored)
capsule.  Each is checked against something other than the oracle's own formula: the
geometry of the initial film of Section 3.2, an analytic density field, the capsule's
labels, and the momentum balance of a periodic box.

Meniscus convention: h is the height of the first upward crossing of
phi = (rho1 - rho2) / (rho1 + rho2) through 0, in lattice coordinates (sites at integer
z, the wall layer at z = 0, the half-way bounce-back plane at z = 0.5), so the film
thickness above the wall plane is h - 0.5.

Lateral force convention: f_anchor is the force of the fluid on the anchored capsule,
minus the sum of the anchor forces on its nodes.  In a periodic box with a body force g
on the fluid mass M and the anchor as the only momentum sink, the fluid momentum changes
per step by M g - f_anchor, and f_anchor reaches M g at steady state."""
import numpy as np
import pytest

import oracle
import synth


@pytest.mark.parametrize("H", [4, 7.0, 12])
def test_meniscus_of_the_initial_film_is_one_layer_above_it(H):
    """Film layers 1..H of (0.7, 0.04), one mixed layer (0.3, 0.3) at H + 1, gas above
    (Section 3.2): phi is exactly 0 at H + 1, so h = H + 1 in every column, i.e. a film
    thickness above the wall plane of H + 1/2 (the mixed layer counts half)."""
    cfg = synth.workload("pf", nx=6, ny=5, nz=24, film_height=float(H), capsules=[])
    o = oracle.Oracle(cfg)
    h = o.meniscus()
    assert h.shape == (5, 6)
    assert np.all(h == H + 1.0)
    assert np.all(h - 0.5 == H + 0.5)


def test_meniscus_of_a_tilted_linear_interface_is_exact():
    """rho1 = 1/2 - a (z - h(x, y)), rho2 = 1/2 + a (z - h(x, y)) gives phi = -2a (z - h)
    linear in z, so the interpolated crossing is h(x, y) itself (up to rounding) for a
    tilted plane h = 5.3 + 0.11 x + 0.07 y that crosses many layers."""
    nx, ny, nz, a = 12, 10, 16, 0.02
    x = np.arange(nx)[None, None, :]
    y = np.arange(ny)[None, :, None]
    z = np.arange(nz)[:, None, None]
    h = 5.3 + 0.11 * x + 0.07 * y
    rho = np.empty((2, nz, ny, nx))
    rho[0] = 0.5 - a * (z - h)
    rho[1] = 0.5 + a * (z - h)
    cfg = synth.workload("pf", nx=nx, ny=ny, nz=nz, init_mode=2, init_rho_array=rho,
                         capsules=[])
    got = oracle.Oracle(cfg).meniscus()
    want = h[0]
    assert np.abs(got - want).max() <= 1e-12
    assert np.ptp(np.floor(want)) >= 2        # the crossing sits in several layers


def test_meniscus_without_a_crossing_is_nan():
    """A column of pure gas or pure liquid has no crossing."""
    for dens in ([0.04, 0.7], [0.7, 0.04]):
        cfg = synth.workload("pf", nx=4, ny=4, nz=10, init_mode=0, init_rho=dens, capsules=[])
        assert np.all(np.isnan(oracle.Oracle(cfg).meniscus()))


def test_meniscus_is_nan_where_the_crossing_lies_inside_a_capsule():
    """The capsule of radius 6 centred at height 10 straddles the film's interface at
    height 11: the crossing of every column through it lies on labelled sites, so those
    columns give NaN; columns clear of the capsule keep the film's height.  The NaN disc
    has about the capsule's cross-section at the interface (radius sqrt(6^2 - 1^2))."""
    cfg = synth.workload("pf")
    o = oracle.Oracle(cfg)
    o.step(1)
    h = o.meniscus()
    lab = o.labels()
    assert np.isnan(h[16, 16])
    yy, xx = np.mgrid[0:32, 0:32]
    far = (xx - 16.0) ** 2 + (yy - 16.0) ** 2 > 8.0 ** 2
    assert not np.any(np.isnan(h[far]))
    assert np.abs(h[far] - 11.0).max() < 0.05
    n_nan = int(np.isnan(h).sum())
    r = np.sqrt(35.0)
    assert 0.8 * np.pi * (r - 1) ** 2 <= n_nan <= 1.2 * np.pi * (r + 1) ** 2
    # every NaN column has a labelled site at the film's interface layers
    inner = np.isnan(h)
    assert np.all((lab[10:13] != 0).any(axis=0)[inner])


@pytest.mark.parametrize("H,nz", [(7, 24), (10, 32), (14, 40)])
def test_meniscus_of_the_equilibrated_film_lies_between_its_gibbs_surfaces(H, nz):
    """After the film has equilibrated (3000 steps) the interface is diffuse.  Exchanging
    the components mirrors the profile about the phi = 0 crossing, so that crossing lies
    midway between the Gibbs dividing surfaces of the two components: z_G1 = 1/2 + the
    volume of liquid 1 per column above the lower wall plane, z_G2 = nz - 1/2 - the volume
    of liquid 2 below the upper wall plane (the wrap makes the wall layer bound the top at
    nz - 1/2).  The bulk densities of the thin film and the thicker gas differ slightly,
    which breaks the symmetry by a few hundredths of a lattice unit; a wrong wall-plane
    offset (1/2) or layer index (1) fails."""
    cfg = synth.workload("pf", nx=4, ny=4, nz=nz, film_height=float(H), capsules=[])
    o = oracle.Oracle(cfg)
    o.step(3000)
    h = o.meniscus()
    assert np.ptp(h) < 1e-9
    r = o.rho()[:, 1:, 0, 0]
    lo0, hi0 = r[0][-3:].mean(), r[0][:3].mean()
    lo1, hi1 = r[1][:3].mean(), r[1][-3:].mean()
    zg0 = 0.5 + float(np.sum((r[0] - lo0) / (hi0 - lo0)))
    zg1 = nz - 0.5 - float(np.sum((r[1] - lo1) / (hi1 - lo1)))
    assert zg0 < h[0, 0] < zg1
    assert abs(h[0, 0] - 0.5 * (zg0 + zg1)) <= 0.1


def _anchored_box(g=2e-6):
    cfg = synth.workload("pf", nx=16, ny=16, nz=16, wall_z0=0, init_mode=0,
                         init_rho=[1.0, 0.0], body_force=[g, 0.0, 0.0],
                         capsules=[synth.capsule((8.0, 8.0, 8.0), 4.0, 320, 0.02,
                                                 anchor_k=1.0)])
    return cfg, oracle.Oracle(cfg)


def test_anchor_force_balances_the_momentum_of_every_step():
    """Single fluid (no Shan-Chen forces, no reaction) in a periodic box driven by g along
    x: the collision adds the total force, streaming conserves momentum, the elastic node
    forces sum to zero and the spread forces keep their sum, so P(n+1) - P(n) = M g -
    f_anchor(n+1) exactly, in sign and magnitude."""
    g = 2e-6
    cfg, o = _anchored_box(g)
    M = o.summary()["mass"][0]
    P = o.summary()["momentum"].copy()
    for n in range(6):
        o.step(1)
        s = o.summary()
        fa = o.capsule(0)["f_anchor"]
        dP = s["momentum"] - P
        P = s["momentum"].copy()
        assert np.abs(dP - (np.array([M * g, 0, 0]) - fa)).max() <= 1e-12
        assert np.abs(s["pending"]).max() == 0.0
        if n >= 2:
            assert fa[0] > 0                 # the fluid drags the capsule along +x


def test_anchor_force_of_the_fixed_capsule_reaches_the_driving_force():
    """At steady state the anchored capsule is the only momentum sink: f_anchor = M g
    (the force the paper samples on fixed particles, Section 4.1)."""
    g = 2e-6
    cfg, o = _anchored_box(g)
    M = o.summary()["mass"][0]
    o.step(1500)
    fa = o.capsule(0)["f_anchor"]
    assert abs(fa[0] / (M * g) - 1.0) <= 1e-3
    assert np.abs(fa[1:]).max() <= 1e-6 * M * g
