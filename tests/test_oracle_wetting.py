"""Pins of the oracle's wall wetting against Young's law: a cylindrical drop of component
0 resting on the substrate (quasi-two-dimensional box, periodic in x and y) takes the
contact angle of the wall, whatever its size, and that angle is 90 degrees for a neutral
wall (zero wetting offset), where exchanging the components maps the system onto itself.

The angle is measured as a plain geometric fit: the points where the two densities are
equal (linear interpolation along rows and columns, at least 3 sites above the wall) are
fitted with a circle by linear least squares, and the angle inside the drop between the
wall plane z = 1/2 (half-way bounce-back) and the circle is acos((1/2 - z_c) / R_c).
Finite drops carry a small size-dependent offset from the diffuse interface: 87.6 degrees
at R = 10 and 88.6 at R = 14 for the neutral wall."""
import math

import numpy as np
import pytest

import oracle
import synth

NX, NY, NZ, WALL = 80, 3, 40, 0.5


def _drop_density(radius):
    X, Z = np.meshgrid(np.arange(NX), np.arange(NZ))
    inside = ((X - (NX - 1) / 2) ** 2 + (Z - WALL) ** 2 < radius * radius) & (Z >= 1)
    rho = np.zeros((2, NZ, NY, NX))
    rho[0] = np.where(inside, 0.72, 0.036)[:, None, :]
    rho[1] = np.where(inside, 0.036, 0.72)[:, None, :]
    return rho


def contact_angle(r0, r1):
    """Contact angle (degrees) inside component 0 of a drop on the wall, from density
    planes [nz][nx]."""
    phi = r0 - r1
    nz, nx = phi.shape
    pts = []
    for z in range(3, nz // 2):
        for x in range(nx - 1):
            if phi[z, x] * phi[z, x + 1] < 0:
                pts.append((x + phi[z, x] / (phi[z, x] - phi[z, x + 1]), z))
    for x in range(nx):
        for z in range(3, nz // 2):
            if phi[z, x] * phi[z + 1, x] < 0:
                pts.append((x, z + phi[z, x] / (phi[z, x] - phi[z + 1, x])))
    P = np.array(pts)
    A = np.column_stack([2 * P[:, 0], 2 * P[:, 1], np.ones(len(P))])
    (xc, zc, c), *_ = np.linalg.lstsq(A, (P ** 2).sum(1), rcond=None)
    rc = math.sqrt(c + xc * xc + zc * zc)
    assert np.abs(np.hypot(P[:, 0] - xc, P[:, 1] - zc) - rc).max() < 0.1   # a circle
    return math.degrees(math.acos((WALL - zc) / rc))


def _angle(radius, drho, steps=4000):
    cfg = synth.workload("pf", capsules=[], wall_z0=1, nx=NX, ny=NY, nz=NZ, init_mode=2,
                         init_rho_array=_drop_density(radius), wall_drho=drho)
    o = oracle.Oracle(cfg)
    assert o.step(steps) == 0
    r = o.rho()[:, :, 1, :]
    o.close()
    return contact_angle(r[0], r[1])


def test_contact_angle_fit_of_exact_circles():
    # the measurement itself: density fields of circular caps with known angles
    X, Z = np.meshgrid(np.arange(NX, dtype=float), np.arange(NZ, dtype=float))
    for theta in (40.0, 90.0, 130.0):
        rc = 15.0
        zc = WALL - rc * math.cos(math.radians(theta))
        d = np.hypot(X - 40.0, Z - zc) - rc
        r0 = 0.4 - 0.35 * np.tanh(d / 2.0)
        assert contact_angle(r0, 0.8 - r0) == pytest.approx(theta, abs=0.2)


@pytest.mark.slow
def test_neutral_wall_gives_ninety_degrees():
    assert abs(_angle(14.0, 0.0) - 90.0) < 2.5


@pytest.mark.slow
@pytest.mark.parametrize("drho", [0.1, -0.1])
def test_contact_angle_is_a_property_of_the_wall(drho):
    a, b = _angle(10.0, drho), _angle(14.0, drho)
    assert abs(a - b) < 1.5
    # a positive offset makes the wall wet by component 0
    assert (a < 80.0) if drho > 0 else (a > 100.0)
