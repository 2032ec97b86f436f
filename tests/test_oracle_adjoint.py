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
