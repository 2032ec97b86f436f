"""Pins for the APIC transfers' oracle: the quadratic B-spline's moments,
brute-force particle-to-grid loops, mass and momentum conservation, the
exact round trip of affine velocity fields (the property the affine part
exists for), the first moments of the grid momentum, constant fields, and
the particle move."""
import numpy as np
import pytest

from oracle import apic, fluid


def _particles(n, P, rng, margin=1.0):
    h = 1.0 / n
    return h * margin + (1.0 - 2 * h * margin) * rng.random((P, 3))


@pytest.mark.parametrize("frac", [0.0, 0.13, 0.5, 0.77, 0.999])
def test_bspline_moments(frac):
    """Over the three nodes around a point: sum N = 1, sum N r = 0,
    sum N r^2 = 1/4 (the 4/dx^2 of the affine update)."""
    X = 5.0 + frac
    base = np.floor(X - 0.5)
    r = base + np.arange(3) - X
    N = apic.bspline2(r)
    assert abs(N.sum() - 1.0) < 1e-15
    assert abs((N * r).sum()) < 1e-15
    assert abs((N * r * r).sum() - 0.25) < 1e-15
    # the nodes outside the three carry no weight
    assert apic.bspline2(base - 1 - X) == 0.0 and apic.bspline2(base + 3 - X) == 0.0


def test_p2g_matches_loops():
    n, P = 5, 40
    rng = np.random.default_rng(0)
    xp = _particles(n, P, rng, margin=0.3)  # some stencils leave the lattices
    vp = rng.standard_normal((P, 3))
    Cp = rng.standard_normal((P, 3, 3))
    mp = 0.5 + rng.random(P)
    vel, mass = apic.p2g(n, xp, vp, Cp, mp)
    h = 1.0 / n
    for a in range(3):
        shp = fluid.face_shape(n, a)
        mom = np.zeros(shp)
        m = np.zeros(shp)
        off = [0.5, 0.5, 0.5]
        off[a] = 0.0
        for p in range(P):
            for k in range(shp[0]):
                for j in range(shp[1]):
                    for i in range(shp[2]):
                        xi = np.array([(i + off[0]) * h, (j + off[1]) * h, (k + off[2]) * h])
                        r = xp[p] / h - xi / h
                        w = float(np.prod([max(0.0, 0.75 - t * t) if abs(t) < 0.5
                                           else (0.5 * (1.5 - abs(t)) ** 2 if abs(t) < 1.5 else 0.0)
                                           for t in r]))
                        mom[k, j, i] += w * mp[p] * (vp[p, a] + Cp[p, a] @ (xi - xp[p]))
                        m[k, j, i] += w * mp[p]
        assert np.abs(m - mass[a]).max() < 1e-12
        ref = np.where(m > 0, mom / np.where(m > 0, m, 1.0), 0.0)
        assert np.abs(ref - vel[a]).max() < 1e-10 * max(1.0, np.abs(ref).max())


def test_mass_and_momentum_conserved():
    n, P = 8, 300
    rng = np.random.default_rng(1)
    xp = _particles(n, P, rng)
    vp = rng.standard_normal((P, 3))
    Cp = rng.standard_normal((P, 3, 3))
    mp = 0.5 + rng.random(P)
    vel, mass = apic.p2g(n, xp, vp, Cp, mp)
    for a in range(3):
        assert abs(mass[a].sum() - mp.sum()) < 1e-12 * mp.sum()
        # the affine parts carry no net momentum (first moment of the spline is 0)
        assert abs((mass[a] * vel[a]).sum() - (mp * vp[:, a]).sum()) < 1e-10


def test_affine_field_round_trip_is_exact():
    """Particles carrying v = A x + b with C = A: every node with mass gets
    A x_i + b, and grid to particles gives back v_p and C_p = A."""
    n, P = 10, 400
    rng = np.random.default_rng(2)
    A = rng.standard_normal((3, 3))
    b = rng.standard_normal(3)
    xp = _particles(n, P, rng)
    vp = xp @ A.T + b
    Cp = np.broadcast_to(A, (P, 3, 3)).copy()
    mp = 0.5 + rng.random(P)
    vel, mass = apic.p2g(n, xp, vp, Cp, mp)
    h = 1.0 / n
    for a in range(3):
        shp = fluid.face_shape(n, a)
        off = [0.5, 0.5, 0.5]
        off[a] = 0.0
        k, j, i = np.meshgrid(*[np.arange(s) for s in shp], indexing="ij")
        pos = np.stack([(i + off[0]) * h, (j + off[1]) * h, (k + off[2]) * h], -1)
        lin = pos @ A[a] + b[a]
        has = mass[a] > 0
        assert has.sum() > 100
        assert np.abs(vel[a][has] - lin[has]).max() < 1e-12
    v2, C2 = apic.g2p(n, vel, xp)
    assert np.abs(v2 - vp).max() < 1e-12
    assert np.abs(C2 - A).max() < 1e-9


def test_constant_field_and_move():
    n, P = 6, 50
    rng = np.random.default_rng(3)
    xp = _particles(n, P, rng)
    c = np.array([0.3, -1.2, 0.7])
    grid = tuple(np.full(fluid.face_shape(n, a), c[a]) for a in range(3))
    vp, Cp = apic.g2p(n, grid, xp)
    assert np.abs(vp - c).max() < 1e-13
    assert np.abs(Cp).max() < 1e-11
    x2 = apic.advect(xp, vp, 0.01)
    assert np.abs(x2 - (xp + 0.01 * c)).max() < 1e-15


def test_first_moments_of_momentum():
    """sum_i m_i v_ai x_ib = sum_p m_p (v_pa x_pb + (h^2/4) C_p[a, b]) for all
    components a and axes b (all stencils inside the lattices): the moments
    behind APIC's conservation of angular momentum."""
    n, P = 9, 250
    rng = np.random.default_rng(11)
    xp = _particles(n, P, rng)
    vp = rng.standard_normal((P, 3))
    Cp = rng.standard_normal((P, 3, 3))
    mp = 0.5 + rng.random(P)
    vel, mass = apic.p2g(n, xp, vp, Cp, mp)
    h = 1.0 / n
    for a in range(3):
        shp = fluid.face_shape(n, a)
        off = [0.5, 0.5, 0.5]
        off[a] = 0.0
        k, j, i = np.meshgrid(*[np.arange(s) for s in shp], indexing="ij")
        pos = np.stack([(i + off[0]) * h, (j + off[1]) * h, (k + off[2]) * h], -1)
        mom = mass[a] * vel[a]
        for b in range(3):
            grid = float((mom * pos[..., b]).sum())
            part = float((mp * (vp[:, a] * xp[:, b] + 0.25 * h * h * Cp[:, a, b])).sum())
            assert abs(grid - part) <= 1e-11 * max(1.0, abs(part)), (a, b, grid, part)
