"""The paper's parameter normalisation (Section 3.4.2): every physical
parameter is optimised as a free variable theta, passed through an activation
chosen by whether the parameter may be negative, and mapped to its physical
scale, so that one learning rate suits all of them.

  * positive-only parameters (viscosity, density, time step, velocity
    scale): value = scale * exp(theta);
  * parameters that may take either sign or live in a bounded range
    (gravity, bounce and damping coefficients, inlet velocities):
    value = lo + (hi - lo) * sigmoid(theta).

`rollout` (in `autograd.py`) takes theta_nu = log(nu) and theta_s = log(s),
the exponential map with scale 1; `PhysParam.value` gives the physical value
as a differentiable torch scalar for any other parameter of the
optimisation.
"""
from __future__ import annotations

import math
from dataclasses import dataclass


@dataclass(frozen=True)
class PhysParam:
    """One normalised parameter: kind "exp" (scale) or "sigmoid" (lo, hi)."""
    name: str
    kind: str = "exp"
    scale: float = 1.0
    lo: float = 0.0
    hi: float = 1.0

    def __post_init__(self):
        if self.kind == "exp":
            if not (self.scale > 0 and math.isfinite(self.scale)):
                raise ValueError(f"{self.name}: the exponential map needs a finite scale > 0")
        elif self.kind == "sigmoid":
            if not (math.isfinite(self.lo) and math.isfinite(self.hi) and self.hi > self.lo):
                raise ValueError(f"{self.name}: the sigmoid map needs finite lo < hi")
        else:
            raise ValueError(f"{self.name}: kind must be 'exp' or 'sigmoid'")

    def value(self, theta):
        """The physical value of theta (a torch tensor: differentiable)."""
        import torch
        if self.kind == "exp":
            return self.scale * torch.exp(theta)
        return self.lo + (self.hi - self.lo) * torch.sigmoid(theta)

    def theta(self, value: float) -> float:
        """The free variable that maps to `value` (inside the range)."""
        if self.kind == "exp":
            if not value > 0:
                raise ValueError(f"{self.name}: {value} is not positive")
            return math.log(value / self.scale)
        t = (value - self.lo) / (self.hi - self.lo)
        if not 0.0 < t < 1.0:
            raise ValueError(f"{self.name}: {value} is outside ({self.lo}, {self.hi})")
        return math.log(t / (1.0 - t))
