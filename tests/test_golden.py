"""The oracle against its stored fixtures (tests/golden/, written by
make_golden.py from the oracle only): a regression pin for the step, the
gradient and the network."""
import os

import numpy as np
import pytest

from tests.golden import make_golden as mk

HERE = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load(name):
    out = {}
    with open(os.path.join(HERE, name)) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            key, *vals = line.split()
            out[key] = vals
    return out


def check_fields(g, prefix, fields, rtol):
    for c, f in enumerate(fields):
        k = f"{prefix}{'uvw'[c]}"
        flat = f.reshape(-1)
        scale = np.abs(flat).max()
        idx = np.array([int(v) for v in g[k + "_idx"]])
        want = np.array([float(v) for v in g[k + "_val"]])
        np.testing.assert_allclose(flat[idx], want, rtol=0, atol=rtol * scale)
        assert abs(flat.sum() - float(g[k + "_sum"][0])) <= rtol * np.abs(flat).sum()
        assert abs((flat * flat).sum() - float(g[k + "_sumsq"][0])) <= rtol * (flat * flat).sum()


def test_step32_fixture(orc):
    g = load("step32_seed0.txt")
    n, seed, nu = int(g["n"][0]), int(g["seed"][0]), float(g["nu"][0])
    cell, ug = mk.inputs.gen_case(n, seed)
    u1, info = orc.step(cell, orc.mask_faces(cell, ug), nu, mk.DT, tol=1e-12)
    assert int(info.explicit) == int(g["explicit"][0])
    assert orc.max_abs_divergence(cell, u1) < 1e-10
    check_fields(g, "u1_", u1, 1e-9)


def test_grad16_fixture(orc):
    g = load("grad16.txt")
    n, steps, s_t, s_e = 16, 5, 1.2, 0.8
    for mode, nu_t, nu_e in (("explicit", 4e-3, 2e-3), ("implicit", 8e-2, 5e-2)):
        cell, ug = mk.inputs.gen_case(n, 100)
        ug = tuple(2.0 * x for x in ug)
        target = orc.rollout(cell, ug, nu_t, s_t, steps, mk.DT, mode=mode, tol=1e-12)[-1]
        ref = orc.rollout_grad(cell, ug, nu_e, s_e, steps, mk.DT, target, mode=mode, tol=1e-12)
        for key in ("J", "dtheta_nu", "dtheta_s"):
            want = float(g[f"{mode}_{key}"][0])
            assert abs(ref[key] - want) <= 1e-8 * abs(want), (mode, key, ref[key], want)


def test_unet8_fixture():
    from oracle import unet as orc_unet
    g = load("unet8.txt")
    n = 8
    cell = mk.inputs.gen_mask(n, 5)
    mask = cell == 1
    rng = np.random.default_rng([5, 98])
    r = np.where(mask, rng.standard_normal((n, n, n)), 0.0)
    z = orc_unet.forward(orc_unet.init_weights(3).astype(np.float64), r, mask, emulate_bf16=False)
    flat = z.reshape(-1)
    idx = np.array([int(v) for v in g["z_idx"]])
    want = np.array([float(v) for v in g["z_val"]])
    np.testing.assert_allclose(flat[idx], want, rtol=0, atol=1e-10 * np.abs(flat).max())
    assert abs(flat.sum() - float(g["z_sum"][0])) <= 1e-10 * np.abs(flat).sum()
