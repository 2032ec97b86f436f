"""The parameter normalisation (host side, CPU): values, inverses, ranges
and gradients of the exponential and sigmoid maps."""
import math

import pytest
import torch

from paper_2503_00868_amd.params import PhysParam


@pytest.mark.parametrize("p,v", [(PhysParam("nu", "exp", scale=1e-3), 2.7e-4),
                                 (PhysParam("dt", "exp", scale=1 / 120), 1 / 100),
                                 (PhysParam("g", "sigmoid", lo=-20.0, hi=0.0), -9.8),
                                 (PhysParam("bounce", "sigmoid"), 0.3)])
def test_value_inverts_theta(p, v):
    th = torch.tensor(p.theta(v), dtype=torch.float64)
    assert abs(float(p.value(th)) - v) <= 1e-12 * max(1.0, abs(v))


def test_ranges_and_signs():
    g = PhysParam("g", "sigmoid", lo=-20.0, hi=5.0)
    th = torch.linspace(-40, 40, 101, dtype=torch.float64)
    vals = g.value(th)
    assert float(vals.min()) >= -20.0 and float(vals.max()) <= 5.0
    assert float(vals.min()) < 0 < float(vals.max())
    nu = PhysParam("nu", "exp", scale=1e-3)
    assert float(nu.value(th).min()) > 0


def test_gradients():
    for p in (PhysParam("nu", "exp", scale=1e-3), PhysParam("g", "sigmoid", lo=-20.0, hi=0.0)):
        th = torch.tensor(0.3, dtype=torch.float64, requires_grad=True)
        assert torch.autograd.gradcheck(p.value, (th,))
    # d value / d theta: value itself for exp, (hi - lo) s (1 - s) for the sigmoid
    th = torch.tensor(0.3, dtype=torch.float64, requires_grad=True)
    v = PhysParam("nu", "exp", scale=2.0).value(th)
    v.backward()
    assert abs(float(th.grad) - float(v.detach())) < 1e-15
    th = torch.tensor(0.3, dtype=torch.float64, requires_grad=True)
    PhysParam("g", "sigmoid", lo=-20.0, hi=0.0).value(th).backward()
    s = 1 / (1 + math.exp(-0.3))
    assert abs(float(th.grad) - 20.0 * s * (1 - s)) < 1e-13


def test_invalid_settings_and_values():
    with pytest.raises(ValueError):
        PhysParam("x", "exp", scale=0.0)
    with pytest.raises(ValueError):
        PhysParam("x", "sigmoid", lo=1.0, hi=1.0)
    with pytest.raises(ValueError):
        PhysParam("x", "tanh")
    with pytest.raises(ValueError):
        PhysParam("nu", "exp").theta(-1.0)
    with pytest.raises(ValueError):
        PhysParam("g", "sigmoid", lo=-1.0, hi=1.0).theta(1.0)
