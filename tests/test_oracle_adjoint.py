"""Pins for the oracle's exact discrete adjoint and rollout gradient.

The adjoint is checked against central finite differences of the oracle's
own forward map, which it does not share code with: a plausible slip in the
scatter (a wrong node, a missing position term, a sign) fails these.
"""
import numpy as np
import pytest

from paper_2503_00868_amd import inputs


def _rand_faces(orc, n, rng, scale=1.0):
    return tuple(scale * rng.standard_normal(orc.face_shape(n, c)) for c in range(3))


def _dot(a, b):
    return sum(float((x * y).sum()) for x, y in zip(a, b))


def test_advect_adjoint_dot_product(orc):
    """<(A(u + e d) - A(u - e d)) / 2e, lam> = <d, A'(u)^T lam>."""
    n = 8
    dt = 1 / 30
    cell, ug = inputs.gen_case(n, 11)
    u = orc.mask_faces(cell, ug)
    u = tuple(4.0 * f for f in u)  # back-traces reach neighbouring cells
    rng = np.random.default_rng(0)
    d = orc.mask_faces(cell, _rand_faces(orc, n, rng))
    lam = orc.mask_faces(cell, _rand_faces(orc, n, rng))
    eps = 1e-7
    up = tuple(a + eps * b for a, b in zip(u, d))
    um = tuple(a - eps * b for a, b in zip(u, d))
    fd = _dot(tuple((p - m) / (2 * eps) for p, m in zip(orc.advect(cell, up, dt),
                                                         orc.advect(cell, um, dt))), lam)
    adj = _dot(d, orc.advect_adjoint(cell, u, dt, lam))
    assert abs(fd - adj) < 1e-6 * abs(adj)


def test_advect_adjoint_field_part_is_transpose_of_sampling(orc):
    """With dt = 0 the advection is the identity on active faces, so its
    transpose is the identity on active faces too."""
    n = 6
    cell, ug = inputs.gen_case(n, 12)
    u = orc.mask_faces(cell, ug)
    rng = np.random.default_rng(1)
    lam = orc.mask_faces(cell, _rand_faces(orc, n, rng))
    g = orc.advect_adjoint(cell, u, 0.0, lam)
    for a, b in zip(g, lam):
        np.testing.assert_allclose(a, b, atol=1e-15)


@pytest.mark.parametrize("nu", [1e-3, 3e-2])
def test_diffusion_and_projection_adjoint_dot_product(orc, nu):
    n = 8
    dt = 1 / 120
    cell = inputs.gen_mask(n, 13)
    rng = np.random.default_rng(2)
    a = orc.mask_faces(cell, _rand_faces(orc, n, rng))
    b = orc.mask_faces(cell, _rand_faces(orc, n, rng))
    for mode in ("explicit", "implicit"):
        Da, _, _ = orc.diffuse(cell, a, nu, dt, mode, 1e-13)
        Db, _, _ = orc.diffuse(cell, b, nu, dt, mode, 1e-13)
        assert abs(_dot(Da, b) - _dot(a, Db)) < 1e-10 * abs(_dot(Da, b))


def _fd_theta(orc, cell, ug, nu, s, steps, dt, target, which, h=1e-3, mode="auto"):
    def J(th_nu, th_s):
        st = orc.rollout(cell, ug, np.exp(th_nu), np.exp(th_s), steps, dt, mode=mode)
        return orc.loss(cell, st[-1], target)
    t_nu, t_s = np.log(nu), np.log(s)
    if which == "nu":
        return (J(t_nu + h, t_s) - J(t_nu - h, t_s)) / (2 * h)
    return (J(t_nu, t_s + h) - J(t_nu, t_s - h)) / (2 * h)


@pytest.mark.parametrize("mode,nu_t,nu_e", [("explicit", 4e-3, 2e-3), ("implicit", 8e-2, 5e-2)])
def test_rollout_gradient_matches_fd_in_theta(orc, mode, nu_t, nu_e):
    """Exact discrete gradient of the MSE loss after a short rollout against
    central FD in theta = log(param), h = 1e-3."""
    n, steps, dt = 8, 3, 1 / 60
    cell, ug = inputs.gen_case(n, 21)
    ug = tuple(3.0 * f for f in ug)
    target = orc.rollout(cell, ug, nu_t, 1.2, steps, dt, mode=mode)[-1]
    s = 0.8
    g = orc.rollout_grad(cell, ug, nu_e, s, steps, dt, target, mode=mode)
    for which, key in (("nu", "dtheta_nu"), ("s", "dtheta_s")):
        fd = _fd_theta(orc, cell, ug, nu_e, s, steps, dt, target, which, mode=mode)
        assert abs(fd - g[key]) <= 1e-4 * abs(fd) + 1e-12, (which, fd, g[key])


def test_rollout_gradient_initial_velocity_directional(orc):
    """dJ/du_gen against a central FD along a random direction."""
    n, steps, dt = 8, 2, 1 / 60
    cell, ug = inputs.gen_case(n, 22)
    ug = tuple(3.0 * f for f in ug)
    target = orc.rollout(cell, ug, 2e-3, 1.1, steps, dt)[-1]
    rng = np.random.default_rng(5)
    d = _rand_faces(orc, n, rng)
    g = orc.rollout_grad(cell, ug, 1e-3, 1.0, steps, dt, target)
    eps = 1e-6
    Jp = orc.loss(cell, orc.rollout(cell, tuple(a + eps * b for a, b in zip(ug, d)), 1e-3, 1.0,
                                    steps, dt)[-1], target)
    Jm = orc.loss(cell, orc.rollout(cell, tuple(a - eps * b for a, b in zip(ug, d)), 1e-3, 1.0,
                                    steps, dt)[-1], target)
    fd = (Jp - Jm) / (2 * eps)
    assert abs(fd - _dot(d, g["du_gen"])) < 1e-5 * abs(fd)


def test_advect_ddt_matches_fd(orc):
    """The departure-point derivative d advect / d dt against a central
    difference of the oracle's own advection in dt, face by face."""
    n, dt, eps = 8, 1 / 30, 1e-7
    cell, ug = inputs.gen_case(n, 31)
    u = tuple(4.0 * f for f in orc.mask_faces(cell, ug))
    got = orc.advect_ddt(cell, u, dt)
    for c, (p, m) in enumerate(zip(orc.advect(cell, u, dt + eps), orc.advect(cell, u, dt - eps))):
        fd = (p - m) / (2 * eps)
        scale = np.abs(fd).max()
        assert scale > 0
        assert np.abs(fd - got[c]).max() <= 1e-6 * scale, c


@pytest.mark.parametrize("mode", ["explicit", "implicit"])
def test_rollout_gradient_dt_and_gravity_match_fd(orc, mode):
    """dJ/dtheta_dt (theta_dt = log dt) and dJ/dg against central FD of the
    oracle rollout (h = 1e-3 in theta_dt; 1e-4 m/s^2 in each g component:
    at 1e-3 a back-trace of this case crosses a lattice cell, where the
    piecewise-trilinear step has a kink), the viscosity mode held fixed."""
    n, steps, dt, s = 8, 3, 1 / 60, 0.9
    nu = 4e-3 if mode == "explicit" else 8e-2
    g0 = np.array([0.7, -9.8, -1.3])
    cell, ug = inputs.gen_case(n, 23)
    ug = tuple(3.0 * f for f in ug)
    target = orc.rollout(cell, ug, nu, 1.1, steps, dt * 1.1, g=tuple(0.9 * g0), mode=mode)[-1]
    ref = orc.rollout_grad(cell, ug, nu, s, steps, dt, target, g=tuple(g0), mode=mode)

    def J(dt_, g_):
        st = orc.rollout(cell, ug, nu, s, steps, dt_, g=tuple(g_), mode=mode)
        return orc.loss(cell, st[-1], target)

    h = 1e-3
    fd_dt = (J(dt * np.exp(h), g0) - J(dt * np.exp(-h), g0)) / (2 * h)
    assert abs(fd_dt - ref["dtheta_dt"]) <= 1e-4 * abs(fd_dt), (fd_dt, ref["dtheta_dt"])
    hg = 1e-4
    for c in range(3):
        e = np.zeros(3)
        e[c] = hg
        fd = (J(dt, g0 + e) - J(dt, g0 - e)) / (2 * hg)
        assert abs(fd - ref["dg"][c]) <= 1e-4 * abs(fd) + 1e-12, (c, fd, ref["dg"][c])


def test_upwind_convection_rollout(orc):
    """The rollout gradient with the paper's upwind convection surrogate:
    from rest (u_gen = 0) the first step's convected field is zero, where the
    surrogate and the exact transpose are both the identity on active faces,
    so a one-step gradient agrees; a moving field makes them differ, and the
    dt and g derivatives stay those of the exact mode only where the
    adjoint states agree (one step)."""
    n, dt = 8, 1 / 60
    cell, ug = inputs.gen_case(n, 24)
    zero = tuple(0.0 * f for f in ug)
    target = orc.rollout(cell, ug, 2e-3, 1.0, 1, dt)[-1]
    a = orc.rollout_grad(cell, zero, 2e-3, 1.0, 1, dt, target)
    b = orc.rollout_grad(cell, zero, 2e-3, 1.0, 1, dt, target, convection="upwind")
    for x, y in zip(a["du_gen"], b["du_gen"]):
        np.testing.assert_allclose(x, y, rtol=0, atol=1e-13)
    assert abs(a["ddt"] - b["ddt"]) <= 1e-12 * abs(a["ddt"])
    ug3 = tuple(3.0 * f for f in ug)
    a = orc.rollout_grad(cell, ug3, 2e-3, 1.0, 2, dt, target)
    b = orc.rollout_grad(cell, ug3, 2e-3, 1.0, 2, dt, target, convection="upwind")
    diff = max(float(np.abs(x - y).max()) for x, y in zip(a["du_gen"], b["du_gen"]))
    assert diff > 1e-6 * max(float(np.abs(x).max()) for x in a["du_gen"])
