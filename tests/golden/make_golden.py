"""Writes the stored expected values under tests/golden/ from the FP64 oracle
only (no GPU code is imported).  Run from the repository root:

    python tests/golden/make_golden.py

Each fixture is a text file of `key value...` lines; `#` lines are comments
that name the computation and the paper passage it follows.
"""
from __future__ import annotations

import math
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import fluid as orc  # noqa: E402
from oracle import unet as orc_unet  # noqa: E402
from paper_2503_00868_amd import inputs  # noqa: E402

DT = 1.0 / 120
SAMPLES = 24


def sample_index(shape, seed):
    """Fixed pseudo-random face positions (flat indices) for spot values."""
    rng = np.random.default_rng([seed, 99])
    return np.sort(rng.choice(int(np.prod(shape)), SAMPLES, replace=False))


def field_lines(prefix, fields, seed):
    out = []
    for c, f in enumerate(fields):
        idx = sample_index(f.shape, seed + c)
        flat = f.reshape(-1)
        out.append(f"{prefix}{'uvw'[c]}_sum {flat.sum():.17e}")
        out.append(f"{prefix}{'uvw'[c]}_sumsq {(flat * flat).sum():.17e}")
        out.append(f"{prefix}{'uvw'[c]}_idx " + " ".join(str(i) for i in idx))
        out.append(f"{prefix}{'uvw'[c]}_val " + " ".join(f"{flat[i]:.17e}" for i in idx))
    return out


def write(name, header, lines):
    with open(os.path.join(HERE, name), "w") as f:
        for h in header:
            f.write(f"# {h}\n")
        for line in lines:
            f.write(line + "\n")
    print("wrote", name)


def step32():
    n, seed, nu = 32, 0, 1e-3
    cell, ug = inputs.gen_case(n, seed)
    u0 = orc.mask_faces(cell, ug)
    u1, info = orc.step(cell, u0, nu, DT, tol=1e-12)
    lines = [f"n {n}", f"seed {seed}", f"nu {nu!r}", f"dt {DT!r}",
             f"explicit {int(info.explicit)}", f"max_abs_div {orc.max_abs_divergence(cell, u1):.6e}"]
    lines += field_lines("u1_", u1, 1000)
    write("step32_seed0.txt",
          ["One step of the liquid step at 32^3 (seeded slab + ellipsoids mask, curl-of-potential",
           "velocity, nu = 1e-3, dt = 1/120, gravity (0, -9.8, 0)): advection by back-tracing",
           "(Section 3.4.1), gravity and viscosity of the momentum equation (Section 3.2.2, Eq. (v)),",
           "pressure projection solved to a 1e-12 relative residual (Section 3.2.2).",
           "FP64 oracle values; spot values at fixed flat indices of each face array."], lines)


def grad16():
    n, steps, s_t, s_e = 16, 5, 1.2, 0.8
    out = []
    for mode, nu_t, nu_e in (("explicit", 4e-3, 2e-3), ("implicit", 8e-2, 5e-2)):
        cell, ug = inputs.gen_case(n, 100)
        ug = tuple(2.0 * g for g in ug)
        target = orc.rollout(cell, ug, nu_t, s_t, steps, DT, mode=mode, tol=1e-12)[-1]
        ref = orc.rollout_grad(cell, ug, nu_e, s_e, steps, DT, target, mode=mode, tol=1e-12)
        out += [f"{mode}_J {ref['J']:.17e}", f"{mode}_dtheta_nu {ref['dtheta_nu']:.17e}",
                f"{mode}_dtheta_s {ref['dtheta_s']:.17e}"]
    write("grad16.txt",
          ["Loss J = mean over active faces of (u_T - u*_T)^2 after a 5-step rollout at 16^3",
           "(mask and velocity of seed 100, velocity doubled; target (nu*, s* = 1.2), evaluation",
           "s = 0.8), and its exact gradient in theta = (log nu, log s) (Section 3.4.2,",
           "Eq. (optLoss) L2 term with exponential parameter activations).  Solves at 1e-12."], out)


def unet8():
    n = 8
    cell = inputs.gen_mask(n, 5)
    mask = cell == 1
    rng = np.random.default_rng([5, 98])
    r = np.where(mask, rng.standard_normal((n, n, n)), 0.0)
    w = orc_unet.init_weights(3).astype(np.float64)
    z = orc_unet.forward(w, r, mask, emulate_bf16=False)
    idx = sample_index(z.shape, 77)
    flat = z.reshape(-1)
    out = [f"z_sum {flat.sum():.17e}", f"z_sumsq {(flat * flat).sum():.17e}",
           "z_idx " + " ".join(str(i) for i in idx),
           "z_val " + " ".join(f"{flat[i]:.17e}" for i in idx)]
    write("unet8.txt",
          ["U-Net preconditioner output z = mask * rms(r) * U(r / rms(r), mask) at 8^3 in FP64",
           "(no bf16 rounding), seeded residual on the seed-5 mask, weights init_weights(3)",
           "(learned pressure solver of Section 3.4.1; architecture as in oracle/unet.py)."], out)


if __name__ == "__main__":
    step32()
    grad16()
    unet8()
