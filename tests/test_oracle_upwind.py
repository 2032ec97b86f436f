"""Pins for the upwind analytic convection gradient's oracle: the
vectorised form against an explicit face-by-face evaluation of the same
definition, dt = 0, and the closed form for a field affine along the face's
axis (where first-order upwind differences are exact)."""
import numpy as np
import pytest

from oracle import fluid, upwind
from paper_2503_00868_amd import inputs


def _fields(n, rng):
    return tuple(rng.standard_normal(fluid.face_shape(n, c)) for c in range(3))


@pytest.mark.parametrize("n,seed", [(5, 0), (6, 3)])
def test_vectorised_equals_face_by_face(n, seed):
    rng = np.random.default_rng(seed)
    cell = rng.choice([fluid.AIR, fluid.LIQUID, fluid.LIQUID, fluid.SOLID], size=(n, n, n)).astype(np.uint8)
    v, lam = _fields(n, rng), _fields(n, rng)
    a = upwind.gradient(cell, v, lam, 0.01)
    b = upwind.gradient_loops(cell, v, lam, 0.01)
    for x, y in zip(a, b):
        assert np.abs(x - y).max() <= 1e-12 * max(1.0, np.abs(y).max())
    # the surrogate term is present (not just the identity)
    assert max(np.abs(x - fluid.mask_faces(cell, lam)[c]).max() for c, x in enumerate(a)) > 1e-3


def test_zero_time_step_is_the_identity_on_active_faces():
    n = 8
    cell, _ = inputs.gen_case(n, 2)
    rng = np.random.default_rng(1)
    v, lam = _fields(n, rng), _fields(n, rng)
    for x, y in zip(upwind.gradient(cell, v, lam, 0.0), fluid.mask_faces(cell, lam)):
        assert np.array_equal(x, y)


@pytest.mark.parametrize("i", [0, 1, 2])
def test_affine_field_closed_form(i):
    """v_c = a_c + b_c x_i on every face and a uniform lam: at faces two
    cells away from the box the gradient is lam (1 - dt sum_c b_c)."""
    n, dt, lam0 = 10, 0.02, 0.7
    cell = np.full((n, n, n), fluid.LIQUID, np.uint8)
    a = np.array([0.3, -0.2, 0.5])
    b = np.array([1.5, -0.75, 2.0])
    v, lam = [], []
    for c in range(3):
        shp = fluid.face_shape(n, c)
        k, j, ii = np.meshgrid(*[np.arange(s) for s in shp], indexing="ij")
        # coordinate along axis i of the c-faces (face index or cell centre)
        idx = (ii, j, k)[i]
        x = (idx + (0.0 if c == i else 0.5)) / n
        v.append(a[c] + b[c] * x)
        lam.append(np.full(shp, lam0))
    g = upwind.gradient(cell, v, lam, dt)
    ref = lam0 * (1.0 - dt * b.sum())
    gi = g[i]
    inner = gi[2:-2, 2:-2, 2:-2]
    assert np.abs(inner - ref).max() <= 1e-12, (np.abs(inner - ref).max(), ref)


@pytest.mark.parametrize("i", [0, 1, 2])
def test_quadratic_field_picks_the_upwind_side(i):
    """v_c = q_c x_i^2 + a_c along the face's axis i, with v_i changing sign
    at x_i = 1/2 and a uniform lam.  At an interior i-face at x = m h the
    backward difference of q x^2 is q (2x - h), the forward one q (2x + h),
    so the closed form lam (1 - dt sum_c q_c (2x - h)) holds where v_i > 0
    and lam (1 - dt sum_c q_c (2x + h)) where v_i < 0.  The two differ by
    2 dt lam h sum q, so taking the downwind side fails this test."""
    n, dt, lam0 = 12, 0.05, 0.7
    h = 1.0 / n
    cell = np.full((n, n, n), fluid.LIQUID, np.uint8)
    q = np.array([3.0, -1.0, 2.0])
    q[i] = 4.0
    a = np.array([0.2, 0.4, -0.3])
    a[i] = -q[i] * 0.25  # v_i = q_i (x^2 - 1/4): negative below x = 1/2, positive above
    v, lam = [], []
    for c in range(3):
        shp = fluid.face_shape(n, c)
        k, j, ii = np.meshgrid(*[np.arange(s) for s in shp], indexing="ij")
        idx = (ii, j, k)[i]
        x = (idx + (0.0 if c == i else 0.5)) * h
        v.append(a[c] + q[c] * x * x)
        lam.append(np.full(shp, lam0))
    g = upwind.gradient(cell, v, lam, dt)[i]
    shp = fluid.face_shape(n, i)
    k, j, ii = np.meshgrid(*[np.arange(s) for s in shp], indexing="ij")
    m = (ii, j, k)[i]
    x = m * h
    vi = v[i]
    side = np.where(vi > 0, -h, h)
    ref = lam0 * (1.0 - dt * q.sum() * (2 * x + side))
    inner = (slice(2, -2),) * 3
    assert np.any(vi[inner] > 0) and np.any(vi[inner] < 0)
    assert np.abs(g[inner] - ref[inner]).max() <= 1e-12
    wrong = lam0 * (1.0 - dt * q.sum() * (2 * x - side))
    assert np.abs(g[inner] - wrong[inner]).min() >= dt * lam0 * h * abs(q.sum())


@pytest.mark.parametrize("comp", [0, 1, 2])
def test_face_gradient_picks_the_upwind_side(comp):
    """The face-by-face definition (used for sampled checks of large grids)
    against the same quadratic closed form, at faces on both sides of the
    sign change."""
    n, dt, lam0 = 10, 0.05, 0.5
    h = 1.0 / n
    q = np.array([1.0, 2.0, -0.5])
    q[comp] = 3.0
    a = np.zeros(3)
    a[comp] = -q[comp] * 0.25
    v, lam = [], []
    for c in range(3):
        shp = fluid.face_shape(n, c)
        k, j, ii = np.meshgrid(*[np.arange(s) for s in shp], indexing="ij")
        idx = (ii, j, k)[comp]
        x = (idx + (0.0 if c == comp else 0.5)) * h
        v.append(a[c] + q[c] * x * x)
        lam.append(np.full(shp, lam0))
    for m in (2, 3, 7, 8):
        idx = [4, 5, 3]
        idx[2 - comp] = m
        x = m * h
        side = -h if v[comp][tuple(idx)] > 0 else h
        ref = lam0 * (1.0 - dt * q.sum() * (2 * x + side))
        got = upwind.face_gradient(n, v, lam, dt, comp, tuple(idx))
        assert abs(got - ref) <= 1e-12, (m, got, ref)
