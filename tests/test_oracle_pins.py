"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks one part of the oracle against something other than itself: a
moment identity of the lattice, a closed form, a symmetry, an invariant of the
dynamics, brute force or a textbook solution.  A plausible slip (a dropped term, a
wrong sign or index, a transposed operand) in the oracle fails at least one of them.
"""
import math

import numpy as np
import pytest

import oracle
import synth

# ---------------------------------------------------------------------------------------
# Lattice and equilibrium (Section 3.1, eq. lbm:equilibrium)
# ---------------------------------------------------------------------------------------


def test_lattice_moments():
    e, w, opp = oracle.lattice()
    assert e.shape == (19, 3)
    assert w.sum() == pytest.approx(1.0, abs=1e-15)
    assert np.allclose(w @ e, 0.0, atol=1e-15)
    m2 = np.einsum("q,qa,qb->ab", w, e, e)
    assert np.allclose(m2, np.eye(3) / 3.0, atol=1e-15)          # c_s^2 = 1/3
    m4 = np.einsum("q,qa,qb,qc,qd->abcd", w, e, e, e, e)
    d = np.eye(3)
    iso = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
           + np.einsum("ad,bc->abcd", d, d)) / 9.0
    assert np.allclose(m4, iso, atol=1e-15)
    assert np.all(e[opp] == -e)
    assert sorted(set(np.round(w, 12))) == sorted({round(1 / 3, 12), round(1 / 18, 12),
                                                   round(1 / 36, 12)})


def test_feq_moments():
    e, w, _ = oracle.lattice()
    rng = np.random.default_rng(1)
    for _ in range(20):
        rho = rng.uniform(0.01, 2.0)
        u = rng.uniform(-0.1, 0.1, 3)
        f = oracle.feq(rho, u)
        assert f.sum() == pytest.approx(rho, rel=1e-14)
        assert np.allclose(f @ e, rho * u, atol=1e-14)
        pi = np.einsum("q,qa,qb->ab", f, e, e)
        assert np.allclose(pi, rho * (np.eye(3) / 3 + np.outer(u, u)), atol=1e-14)
    # rest state: f^eq = omega * rho
    assert np.allclose(oracle.feq(0.7, np.zeros(3)), 0.7 * w, atol=1e-16)


# ---------------------------------------------------------------------------------------
# Shan-Chen stencil (eq. shanchen)
# ---------------------------------------------------------------------------------------


@pytest.mark.parametrize("norm", [1.0, 3.0])
def test_sc_stencil_gradient(norm):
    """For psi = a + b.x + quadratic terms, sum_i w_i psi(x+e_i) e_i = (norm/3) b: the
    odd moments of the weights vanish and the second moment is c_s^2 = 1/3."""
    rng = np.random.default_rng(2)
    a, b = rng.normal(), rng.normal(size=3)
    Q = rng.normal(size=(3, 3)); Q = Q + Q.T
    psi = np.zeros((3, 3, 3))
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                x = np.array([dx, dy, dz], float)
                psi[dz + 1, dy + 1, dx + 1] = a + b @ x + 0.5 * x @ Q @ x
    assert np.allclose(oracle.sc_sum(psi, norm), norm / 3.0 * b, atol=1e-14)


# ---------------------------------------------------------------------------------------
# Immersed-boundary kernel
# ---------------------------------------------------------------------------------------


def test_phi4_moments():
    rng = np.random.default_rng(3)
    for r in list(rng.uniform(-3, 3, 40)) + [0.0, 0.5, 1.0, 1.5, 2.0]:
        js = np.arange(math.floor(r) - 3, math.floor(r) + 4)
        ph = np.array([oracle.phi4(r - j) for j in js])
        assert ph.sum() == pytest.approx(1.0, abs=1e-15)             # partition of unity
        assert (ph * (r - js)).sum() == pytest.approx(0.0, abs=1e-15)  # first moment
        assert (ph ** 2).sum() == pytest.approx(3.0 / 8.0, abs=1e-15)  # Peskin's sum rule
    assert oracle.phi4(2.0) == 0.0 and oracle.phi4(2.5) == 0.0
    assert oracle.phi4(1.0) == pytest.approx(0.25) and oracle.phi4(0.0) == pytest.approx(0.5)


# ---------------------------------------------------------------------------------------
# Hertz repulsion (Section 3.2)
# ---------------------------------------------------------------------------------------


def test_hertz_closed_form():
    assert oracle.hertz(0.5, 1.5, 1.5) == pytest.approx(1.5 * 1.0 ** 1.5)
    assert oracle.hertz(1.0, 2.0, 1.5) == pytest.approx(2.0 * 0.5 ** 1.5)
    assert oracle.hertz(1.5, 1.5, 1.5) == 0.0
    assert oracle.hertz(3.0, 1.5, 1.5) == 0.0
    # monotone: stronger when closer
    assert oracle.hertz(0.2, 1.5, 1.5) > oracle.hertz(0.8, 1.5, 1.5)


# ---------------------------------------------------------------------------------------
# Skalak membrane (Section 3.1, eq. strain)
# ---------------------------------------------------------------------------------------


def _sphere(level=2, R=5.0):
    return synth.icosphere(level, R, (0.0, 0.0, 0.0))


def _deformed(nodes, seed=4, amp=0.05):
    rng = np.random.default_rng(seed)
    A = np.eye(3) + 0.1 * rng.normal(size=(3, 3))
    return nodes @ A.T + amp * rng.normal(size=nodes.shape)


def test_skalak_rest_state_is_stress_free():
    x, t = _sphere()
    minv, a0 = oracle.reference_geometry(x, t)
    E, f = oracle.skalak(x, t, minv, a0, 0.01, 9.0)
    assert abs(E) < 1e-14 and np.abs(f).max() < 1e-14


def test_skalak_force_is_minus_energy_gradient():
    x0, t = _sphere(1, 3.0)
    minv, a0 = oracle.reference_geometry(x0, t)
    x = _deformed(x0)
    ks, Cs = 0.05, 9.0
    E, f = oracle.skalak(x, t, minv, a0, ks, Cs)
    h = 1e-6
    for n in range(0, len(x), 7):
        for d in range(3):
            xp = x.copy(); xp[n, d] += h
            xm = x.copy(); xm[n, d] -= h
            g = (oracle.skalak(xp, t, minv, a0, ks, Cs)[0] -
                 oracle.skalak(xm, t, minv, a0, ks, Cs)[0]) / (2 * h)
            assert f[n, d] == pytest.approx(-g, rel=1e-6, abs=1e-9)


def test_skalak_free_of_net_force_and_torque():
    x0, t = _sphere()
    minv, a0 = oracle.reference_geometry(x0, t)
    x = _deformed(x0, seed=5) + np.array([40.0, -3.0, 7.0])
    _, f = oracle.skalak(x, t, minv, a0, 0.02, 9.0)
    scale = np.abs(f).max()
    assert np.abs(f.sum(0)).max() < 1e-12 * scale * len(x)
    assert np.abs(np.cross(x, f).sum(0)).max() < 1e-11 * scale * len(x) * 40


def test_skalak_rigid_motion_invariance():
    x0, t = _sphere()
    minv, a0 = oracle.reference_geometry(x0, t)
    x = _deformed(x0, seed=6)
    E1, f1 = oracle.skalak(x, t, minv, a0, 0.02, 9.0)
    th = 0.7
    Rz = np.array([[math.cos(th), -math.sin(th), 0], [math.sin(th), math.cos(th), 0], [0, 0, 1]])
    E2, f2 = oracle.skalak(x @ Rz.T + 3.0, t, minv, a0, 0.02, 9.0)
    assert E2 == pytest.approx(E1, rel=1e-12)
    assert np.allclose(f2, f1 @ Rz.T, atol=1e-13 * np.abs(f1).max() * 10)
    # the reference frame of each triangle is arbitrary: a rotated reference mesh
    minv2, a02 = oracle.reference_geometry(x0 @ Rz.T, t)
    assert np.allclose(a02, a0, rtol=1e-13)
    E3, _ = oracle.skalak(x, t, minv2, a02, 0.02, 9.0)
    assert E3 == pytest.approx(E1, rel=1e-11)


def test_skalak_uniform_dilation_closed_form():
    """Uniform scaling by lambda: every element has B = lambda^2 I, so
    W = ks/4 (I1^2 + 2 I1 - 2 I2 + C I2^2) with I1 = 2(l^2-1), I2 = l^4-1, and by
    virtual work sum_n f_n . X_n = -lambda A0_tot W'(lambda),
    W'(lambda) = 2 ks lambda (l^2-1)(1 + C l^2 (l^2+1))."""
    x0, t = _sphere(3, 6.0)
    minv, a0 = oracle.reference_geometry(x0, t)
    ks, Cs = 0.01, 9.0
    for lam in (0.97, 1.01, 1.05):
        E, f = oracle.skalak(lam * x0, t, minv, a0, ks, Cs)
        I1, I2 = 2 * (lam ** 2 - 1), lam ** 4 - 1
        W = ks / 4 * (I1 ** 2 + 2 * I1 - 2 * I2 + Cs * I2 ** 2)
        assert E == pytest.approx(a0.sum() * W, rel=1e-11)
        Wp = 2 * ks * lam * (lam ** 2 - 1) * (1 + Cs * lam ** 2 * (lam ** 2 + 1))
        assert np.einsum("ij,ij->", f, lam * x0) == pytest.approx(-lam * a0.sum() * Wp, rel=1e-10)


def test_skalak_small_strain_moduli():
    """Small-deformation limit (Section 3.1): area modulus kappa_A = ks (1 + 2C) and
    2D Poisson ratio nu_s = C / (1 + C)."""
    tri = np.array([[0, 1, 2]], np.int32)
    ref = np.array([[0.0, 0, 0], [1.3, 0, 0], [0.4, 0.9, 0]])
    minv, a0 = oracle.reference_geometry(ref, tri)
    ks = 1.0
    for Cs in (0.5, 9.0):
        # isotropic: E / A0 = K/2 alpha^2 for area strain alpha = lambda^2 - 1
        eps = 1e-4
        lam = math.sqrt(1 + eps)
        E, _ = oracle.skalak(lam * ref, tri, minv, a0, ks, Cs)
        assert E / a0[0] / (0.5 * eps ** 2) == pytest.approx(ks * (1 + 2 * Cs), rel=1e-3)
        # uniaxial: stretch x by (1+e1); the energy-minimising y strain is -nu e1
        e1 = 1e-4
        ys = np.linspace(-2 * e1, 0.5 * e1, 2001)
        Es = [oracle.skalak(ref * np.array([1 + e1, 1 + y, 1.0]), tri, minv, a0, ks, Cs)[0]
              for y in ys]
        e2 = ys[int(np.argmin(Es))]
        assert -e2 / e1 == pytest.approx(Cs / (1 + Cs), abs=3e-3)


# ---------------------------------------------------------------------------------------
# Volume and its penalty (eq. vol_cons)
# ---------------------------------------------------------------------------------------


def test_volume_closed_forms():
    x, t = synth.icosphere(0, 1.0)
    a = np.linalg.norm(x[t[0, 0]] - x[t[0, 1]])
    assert oracle.volume(x, t) == pytest.approx(5.0 / 12.0 * (3 + math.sqrt(5)) * a ** 3, rel=1e-13)
    # translation invariance and the sphere limit
    x4, t4 = synth.icosphere(4, 10.0, (100.5, 3.2, 22.0))
    V = oracle.volume(x4, t4)
    assert V < 4 / 3 * math.pi * 1000 and V == pytest.approx(4 / 3 * math.pi * 1000, rel=5e-3)
    # reversed orientation flips the sign
    assert oracle.volume(x4, t4[:, [0, 2, 1]]) == pytest.approx(-V, rel=1e-13)


def test_volume_force_is_minus_penalty_gradient():
    x0, t = synth.icosphere(1, 3.0, (1.0, 2.0, 3.0))
    V0 = oracle.volume(x0, t)
    x = _deformed(x0, seed=8, amp=0.1)
    kv = 0.3
    f = oracle.volume_force(x, t, kv, V0)
    E = lambda y: kv * (oracle.volume(y, t) - V0) ** 2 / (2 * V0)
    h = 1e-6
    for n in range(0, len(x), 5):
        for d in range(3):
            xp = x.copy(); xp[n, d] += h
            xm = x.copy(); xm[n, d] -= h
            assert f[n, d] == pytest.approx(-(E(xp) - E(xm)) / (2 * h), rel=1e-6, abs=1e-10)
    assert np.abs(f.sum(0)).max() < 1e-12


# ---------------------------------------------------------------------------------------
# Side labels
# ---------------------------------------------------------------------------------------


def _box_mesh(lo, hi):
    """Closed, outward-oriented 12-triangle mesh of an axis-aligned box."""
    x0, y0, z0 = lo; x1, y1, z1 = hi
    v = np.array([[x0, y0, z0], [x1, y0, z0], [x1, y1, z0], [x0, y1, z0],
                  [x0, y0, z1], [x1, y0, z1], [x1, y1, z1], [x0, y1, z1]], float)
    f = [(0, 2, 1), (0, 3, 2), (4, 5, 6), (4, 6, 7), (0, 1, 5), (0, 5, 4),
         (1, 2, 6), (1, 6, 5), (2, 3, 7), (2, 7, 6), (3, 0, 4), (3, 4, 7)]
    t = np.array(f, np.int32)
    assert oracle.volume(v, t) > 0
    return v, t


@pytest.mark.parametrize("lo,hi", [((2.3, 1.7, 3.2), (7.6, 5.1, 9.9)),
                                   ((2.0, 2.0, 2.0), (5.0, 5.0, 5.0))])
def test_labels_box_exact(lo, hi):
    """A box's inside-site count equals the number of lattice points it contains; with
    vertices on lattice points the top-left rule counts each shared edge once."""
    v, t = _box_mesh(lo, hi)
    ins = oracle.column_labels(v, t, (0, 0, 0), (12, 12, 12))
    if lo[0] == 2.0:
        # columns x in {2,3,4} (left edge in), y in {3,4,5} (top edge in); 2 <= z < 5
        expect = np.zeros((12, 12, 12), np.uint8)
        expect[2:5, 3:6, 2:5] = 1
        assert np.array_equal(ins, expect)
    else:
        n = [len([k for k in range(12) if lo[d] < k < hi[d]]) for d in range(3)]
        assert ins.sum() == n[0] * n[1] * n[2]
    # triangle order does not matter
    perm = np.random.default_rng(0).permutation(len(t))
    assert np.array_equal(oracle.column_labels(v, t[perm], (0, 0, 0), (12, 12, 12)), ins)


def test_labels_sphere_count():
    R = 10.0
    x, t = synth.icosphere(4, R, (16.3, 15.8, 22.45))
    ins = oracle.column_labels(x, t, (0, 0, 0), (32, 32, 40))
    V = oracle.volume(x, t)
    assert abs(int(ins.sum()) - V) < 0.02 * V
    # every inside site is within R of the centre, every site within R-1.5 is inside
    zz, yy, xx = np.nonzero(ins)
    r = np.sqrt((xx - 16.3) ** 2 + (yy - 15.8) ** 2 + (zz - 22.45) ** 2)
    assert r.max() <= R
    Z, Y, X = np.mgrid[0:40, 0:32, 0:32]
    deep = np.sqrt((X - 16.3) ** 2 + (Y - 15.8) ** 2 + (Z - 22.45) ** 2) < R - 1.5
    assert ins[deep].all()


# ---------------------------------------------------------------------------------------
# Bending (Section 3.1, eq. method:curvature; edge form sqrt(3) kb sum (theta - theta0)^2)
# ---------------------------------------------------------------------------------------


def _hinge(theta):
    """Two unit equilateral triangles (x1, x2, x3) and (x2, x1, x4) on the edge x1-x2 along
    x, the second rotated about the edge so that the normals make the angle theta."""
    s3 = math.sqrt(3.0) / 2.0
    x1, x2 = np.array([0.0, 0.0, 0.0]), np.array([1.0, 0.0, 0.0])
    x3 = np.array([0.5, s3, 0.0])
    x4 = np.array([0.5, -s3 * math.cos(theta), -s3 * math.sin(theta)])
    return np.array([x1, x2, x3, x4]), np.array([[0, 1, 2], [1, 0, 3]], dtype=np.int32)


def test_bending_hinge_closed_form():
    """Two triangles hinged by theta about their shared edge: E = sqrt(3) kb (theta -
    theta0)^2, for either sign of the fold and any reference angle."""
    for th in (0.3, -0.3, 1.1):
        X, T = _hinge(th)
        flat, _ = _hinge(0.0)
        E, F = oracle.bending(X, T, flat, 0.7)
        assert E == pytest.approx(math.sqrt(3.0) * 0.7 * th * th, rel=1e-12)
        ref, _ = _hinge(0.5)
        E2, _ = oracle.bending(X, T, ref, 0.7)
        assert E2 == pytest.approx(math.sqrt(3.0) * 0.7 * (th - 0.5) ** 2, rel=1e-12, abs=1e-15)
        assert np.allclose(F.sum(0), 0.0, atol=1e-13)


def test_bending_reference_shape_is_stress_free():
    X, T = synth.icosphere(3, 6.0, (16.0, 16.0, 10.0))
    E, F = oracle.bending(X, T, X, 0.3)
    assert E == 0.0 and np.all(F == 0.0)


def test_bending_force_is_minus_gradient():
    X, T = synth.icosphere(2, 3.0)
    rng = np.random.default_rng(7)
    Y = X + 0.08 * rng.standard_normal(X.shape)
    E, F = oracle.bending(Y, T, X, 0.2)
    assert E > 0.1
    h = 1e-6
    for i in range(0, len(Y), 5):
        for d in range(3):
            Yp, Ym = Y.copy(), Y.copy()
            Yp[i, d] += h
            Ym[i, d] -= h
            g = (oracle.bending(Yp, T, X, 0.2)[0] - oracle.bending(Ym, T, X, 0.2)[0]) / (2 * h)
            assert F[i, d] == pytest.approx(-g, abs=1e-7 * max(1.0, np.abs(F).max()))


def test_bending_no_net_force_torque_and_rigid_invariance():
    X, T = synth.icosphere(2, 4.0, (1.0, 2.0, 3.0))
    rng = np.random.default_rng(3)
    Y = X + 0.1 * rng.standard_normal(X.shape)
    E, F = oracle.bending(Y, T, X, 0.5)
    assert np.abs(F.sum(0)).max() < 1e-12
    assert np.abs(np.cross(Y, F).sum(0)).max() < 1e-11
    a, b = 0.7, -1.3
    Rz = np.array([[math.cos(a), -math.sin(a), 0], [math.sin(a), math.cos(a), 0], [0, 0, 1]])
    Rx = np.array([[1, 0, 0], [0, math.cos(b), -math.sin(b)], [0, math.sin(b), math.cos(b)]])
    Rm, t = Rz @ Rx, np.array([5.0, -2.0, 9.0])
    E2, F2 = oracle.bending(Y @ Rm.T + t, T, X, 0.5)     # reference may stay put
    assert E2 == pytest.approx(E, rel=1e-10)
    assert np.allclose(F2, F @ Rm.T, atol=1e-10)


@pytest.mark.parametrize("level", [2, 3, 4])
def test_bending_energy_of_a_sphere_is_helfrichs(level):
    """Flat reference angles: the edge form of a triangulated sphere approaches the
    Helfrich energy (kb/2) oint (2H)^2 dA = 8 pi kb of the sphere at any radius (exactly on
    an equilateral triangulation; the icosphere's unequal triangles add 3.5 %)."""
    E1, _ = oracle.bending(*synth.icosphere(level, 1.0), None, 1.0)
    E10, _ = oracle.bending(*synth.icosphere(level, 10.0, (3.0, 4.0, 5.0)), None, 1.0)
    assert E10 == pytest.approx(E1, rel=1e-9)              # scale invariant, as Helfrich's
    assert 1.0 <= E1 / (8 * math.pi) <= 1.04


def test_bending_needs_a_manifold_mesh():
    X, T = synth.icosphere(1, 1.0)
    T2 = np.vstack([T, T[:1]])                              # a triangle used twice
    E, _ = oracle.bending(X, T2, X, 1.0)
    assert math.isnan(E)
