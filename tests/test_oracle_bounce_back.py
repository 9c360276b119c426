"""Pins of the oracle's bounce-back coupling (Section 3.1: half-way bounce-back on the
moving membrane with Ladd's momentum exchange, homogeneous weighting of the three nodes of
the crossed element, the exchanged momentum spread over two consecutive steps, Newtonian
nodes of mass 25 rho0 from Section 3.2).  Each is checked against something other than the
oracle's own formulas: closed forms of the segment-triangle miss distance, the uniform rest
state as a fixed point, exact conservation of mass and of fluid + node momentum, the
momentum balance of a driven periodic box, the number of lattice links a closed surface
cuts, and the drag of a fixed sphere in a periodic array (Hasimoto)."""
import math

import numpy as np
import pytest

import oracle
import synth


def test_miss_distance_closed_forms():
    a, b, c = (0.0, 0.0, 0.0), (1.0, 0.0, 0.0), (0.0, 1.0, 0.0)
    md = oracle.miss_distance
    assert md((0.2, 0.2, -1.0), (0.2, 0.2, 1.0), a, b, c) == 0.0       # through the interior
    assert md((0.5, 0.0, -1.0), (0.5, 0.0, 1.0), a, b, c) == 0.0       # through an edge
    assert md((1.0, 0.0, -0.5), (1.0, 0.0, 1.5), a, b, c) == 0.0       # through a vertex
    # the line meets the plane at (2, 2, 0): barycentric (-3, 2, 2), t = 1/2
    assert md((2.0, 2.0, -1.0), (2.0, 2.0, 1.0), a, b, c) == pytest.approx(3.0, abs=1e-15)
    # the segment stops short of the plane: t = 2
    assert md((0.2, 0.2, -2.0), (0.2, 0.2, -1.0), a, b, c) == pytest.approx(1.0, abs=1e-15)
    # beyond the far end on the other side: t = -1
    assert md((0.2, 0.2, 1.0), (0.2, 0.2, 2.0), a, b, c) == pytest.approx(1.0, abs=1e-15)
    assert md((0.0, 0.0, 1.0), (1.0, 0.0, 1.0), a, b, c) == math.inf   # parallel


def _bb(**kw):
    return synth.workload("pf", coupling=1, **kw)


def test_uniform_rest_state_with_a_capsule_is_a_fixed_point():
    """Uniform densities at rest with a capsule in its reference shape: the reflected and
    the incoming populations are equal on both sides of every link, so nothing is exchanged,
    the Shan-Chen forces vanish and nothing moves."""
    cfg = _bb(nx=16, ny=16, nz=16, wall_z0=0, init_mode=0, init_rho=[0.5, 0.3],
              capsules=[synth.capsule((8.3, 7.6, 8.1), 4.0, 320, 0.1, kv=0.5)])
    o = oracle.Oracle(cfg)
    r0, x0 = o.rho(), o.nodes(0)
    o.step(30)
    assert o.summary()["links"] > 500
    assert np.abs(o.rho() - r0).max() <= 1e-14
    assert np.abs(o.nodes(0) - x0).max() <= 1e-14
    assert np.abs(o.capsule(0)["f_fluid"]).max() <= 1e-14


def test_mass_of_each_component_is_conserved():
    """The link swap moves populations between the two sides with the same moving-wall
    term on both, so each component's mass is conserved exactly (film with a wetting,
    volume-penalised capsule straddling the interface, 150 steps)."""
    cfg = _bb(capsules=[synth.capsule((16.0, 16.0, 10.0), 6.0, 1280, 0.05, kv=0.3,
                                      wet_drho=0.05)])
    o = oracle.Oracle(cfg)
    m0 = o.summary()["mass"]
    o.step(150)
    s = o.summary()
    assert s["unstable"] == 0 and s["lost_links"] == 0
    assert np.abs(s["mass"] - m0).max() <= 1e-13 * m0.max()
    assert np.abs(o.nodes(0) - synth.capsule_mesh(cfg["capsules"][0])[0]).max() > 1e-3


def test_momentum_of_fluid_and_nodes_is_conserved():
    """Periodic box without wall, anchor or body force, a noisy two-component mixture and a
    wetting capsule with a volume penalty: what the fluid loses at the links the nodes gain
    (half at once, half one step later), and the Shan-Chen reaction returns the
    cross-membrane force, so fluid momentum + node momentum + the pending half is
    constant."""
    rho = synth.noise_rho(18, 18, 18, (0.7, 0.04), 0.05, seed=5)
    cfg = _bb(nx=18, ny=18, nz=18, wall_z0=0, init_mode=2, init_rho_array=rho,
              capsules=[synth.capsule((9.2, 8.7, 9.4), 4.0, 320, 0.05, kv=0.5, wet_drho=0.05)])
    o = oracle.Oracle(cfg)

    def total(s):
        return s["momentum"] + s["node_momentum"] + s["pending"]

    s = o.summary()
    P0, M = total(s), s["mass"].sum()
    moved = 0.0
    for _ in range(4):
        o.step(25)
        s = o.summary()
        assert np.abs(total(s) - P0).max() <= 1e-12 * M
        moved = max(moved, float(np.abs(s["node_momentum"]).max()))
    assert moved > 1e-6                      # the nodes took up momentum


def test_driven_box_momentum_balance_per_step():
    """A body force g on the fluid of a periodic box with a free capsule: fluid + nodes +
    pending gain exactly M g per step."""
    g = 3e-6
    cfg = _bb(nx=16, ny=16, nz=16, wall_z0=0, init_mode=0, init_rho=[1.0, 0.0],
              body_force=[g, 0.0, 0.0],
              capsules=[synth.capsule((8.0, 8.0, 8.0), 4.0, 320, 0.1)])
    o = oracle.Oracle(cfg)
    M = o.summary()["mass"][0]

    def total(s):
        return s["momentum"] + s["node_momentum"] + s["pending"]

    P = total(o.summary())
    for _ in range(5):
        o.step(1)
        Pn = total(o.summary())
        assert np.abs(Pn - P - np.array([M * g, 0.0, 0.0])).max() <= 1e-13
        P = Pn
    o.step(200)
    assert o.summary()["node_momentum"][0] > 0


@pytest.mark.parametrize("center", [(16.0, 16.0, 16.0), (15.37, 16.81, 15.6),
                                    (16.5, 15.5, 16.25)])
def test_link_count_matches_the_surface_area(center):
    """Lattice lines of direction e pass a plane at density 1 (axis links) or sqrt(2)
    (face diagonals) per unit area, and cross a closed surface in |cos| of its normal on
    average 1/2, so a surface of area A cuts 3 A/2 + 6 sqrt(2) A/2 = 5.743 A links."""
    cap = synth.capsule(center, 6.0, 1280, 0.1)
    cfg = _bb(wall_z0=0, init_mode=0, init_rho=[0.5, 0.3], capsules=[cap])
    o = oracle.Oracle(cfg)
    o.step(1)
    x, t = synth.capsule_mesh(cap)
    area = 0.5 * np.linalg.norm(np.cross(x[t[:, 1]] - x[t[:, 0]], x[t[:, 2]] - x[t[:, 0]]),
                                axis=1).sum()
    want = (1.5 + 3.0 * math.sqrt(2.0)) * area
    n = o.summary()["links"]
    assert o.summary()["lost_links"] == 0
    assert abs(n / want - 1.0) <= 0.03, (n, want)


def test_fixed_sphere_in_a_periodic_array_has_hasimoto_drag():
    """A sphere held by a stiff centroid spring in a periodic box, the fluid driven by g: at
    steady state the spring carries the whole driving force M g (momentum balance), and the
    mean fluid velocity U gives the drag F / (6 pi mu R U) of Hasimoto's periodic array,
    1 / (1 - 1.7601 c^(1/3) + c - 1.5593 c^2) at volume fraction c, for a hydrodynamic
    radius within 15 % below the nominal one (the flat facets of the mesh and the
    half-way wall lie inside the sphere; measured 0.913)."""
    g, R, L = 2e-6, 4.0, 16
    cfg = _bb(nx=L, ny=L, nz=L, wall_z0=0, init_mode=0, init_rho=[1.0, 0.0],
              body_force=[g, 0.0, 0.0],
              capsules=[synth.capsule((L / 2, L / 2, L / 2), R, 320, 0.5, anchor_k=20.0)])
    o = oracle.Oracle(cfg)
    M = o.summary()["mass"][0]
    o.step(1500)
    F = o.capsule(0)["f_anchor"][0]
    U = o.summary()["momentum"][0] / M
    assert abs(F / (M * g) - 1.0) <= 1e-3
    c = 4.0 / 3.0 * math.pi * R ** 3 / L ** 3
    K = 1.0 / (1.0 - 1.7601 * c ** (1.0 / 3.0) + c - 1.5593 * c * c)
    mu = 1.0 / 6.0                    # rho c_s^2 (tau - 1/2) at rho = 1, tau = 1
    ratio = F / (6.0 * math.pi * mu * R * U * K)
    assert 0.85 <= ratio <= 1.0, ratio
