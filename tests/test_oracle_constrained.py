"""Pins for the constrained divergence projection's oracle: one iteration
against a pressure update written from the projection's own operators, the
fixed point and the limit (the exact projection), and the relaxation
parameter's scaling."""
import numpy as np
import pytest

from oracle import constrained, fluid
from paper_2503_00868_amd import inputs


def _case(n, seed):
    cell, ug = inputs.gen_case(n, seed)
    rng = np.random.default_rng(seed)
    # a divergent field: the generator's velocity plus noise, on active faces
    f = tuple(np.asarray(g, np.float64) + 0.3 * rng.standard_normal(np.shape(g)) for g in ug)
    return cell, fluid.mask_faces(cell, f)


@pytest.mark.parametrize("n,seed", [(8, 0), (12, 2)])
def test_iteration_is_a_jacobi_pressure_step(n, seed):
    """eps = 0: lambda = b / n_c with b the projection's right-hand side, and
    the face update is the projection's pressure update with p = lambda."""
    cell, f = _case(n, seed)
    out = constrained.iterate(cell, f, 0.0)
    b = fluid.divergence_rhs(cell, f)
    D = fluid.poisson_diag(cell)
    lam = np.where(D > 0, b / np.where(D > 0, D, 1.0), 0.0)
    ref = fluid.pressure_update(cell, lam, f)
    for a, r in zip(out, ref):
        assert np.abs(a - r).max() <= 1e-12 * max(1.0, np.abs(r).max())
    # the constraint is the divergence: C = -b / h^2
    C = constrained.constraints(cell, f)
    assert np.abs(C + b * n * n).max() <= 1e-9 * np.abs(b * n * n).max()


def test_divergence_free_field_is_a_fixed_point():
    n = 10
    cell, f = _case(n, 3)
    p_fields, _, _, _ = fluid.project(cell, f, tol=1e-13)
    out = constrained.iterate(cell, p_fields, 0.0)
    for a, r in zip(out, p_fields):
        assert np.abs(a - r).max() <= 1e-10 * np.abs(r).max()


def test_iterations_converge_to_the_projection():
    n = 8
    cell, f = _case(n, 1)
    ref, _, _, _ = fluid.project(cell, f, tol=1e-13)
    out, hist = constrained.project(cell, f, 3000)
    scale = max(np.abs(r).max() for r in ref)
    assert max(np.abs(a - r).max() for a, r in zip(out, ref)) <= 1e-8 * scale
    assert hist[-1] < 1e-8 * hist[0]
    assert hist[200] < hist[20] < hist[0]


def test_relaxation_scales_the_multipliers():
    """lambda = -C / (G + eps): with eps = G_max the update is between a half
    and the full eps = 0 update, and a huge eps leaves the field (almost)
    unchanged."""
    n = 8
    cell, f = _case(n, 4)
    d0 = [a - b for a, b in zip(constrained.iterate(cell, f, 0.0), f)]
    G = constrained.gradient_norms(cell)
    eps = float(G.max())
    d1 = [a - b for a, b in zip(constrained.iterate(cell, f, eps), f)]
    n0 = np.sqrt(sum(float((x * x).sum()) for x in d0))
    n1 = np.sqrt(sum(float((x * x).sum()) for x in d1))
    assert 0.25 * n0 < n1 < n0
    d2 = [a - b for a, b in zip(constrained.iterate(cell, f, 1e8 * eps), f)]
    assert max(np.abs(x).max() for x in d2) <= 1e-7 * max(np.abs(x).max() for x in d0)
