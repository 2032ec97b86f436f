"""Pins for the network oracle: convolution against brute-force loops, the
autograd gradient against central FD, the loss against its geometric
meaning, and invariances of the architecture."""
import numpy as np
import pytest
import torch
import torch.nn.functional as F

from oracle import unet
from paper_2503_00868_amd import inputs


def test_param_count():
    assert unet.param_count() == 353808


def test_conv3d_matches_brute_force_loops():
    """The library conv used by the oracle is the cross-correlation with
    zero padding and tap (kz, ky, kx) -> offset (kz-1, ky-1, kx-1)."""
    rng = np.random.default_rng(0)
    cin, cout, n = 3, 2, 4
    x = rng.standard_normal((cin, n, n, n))
    w = rng.standard_normal((cout, cin, 3, 3, 3))
    y = F.conv3d(torch.tensor(x)[None], torch.tensor(w), padding=1)[0].numpy()
    ref = np.zeros((cout, n, n, n))
    for co in range(cout):
        for z in range(n):
            for yy in range(n):
                for xx in range(n):
                    s = 0.0
                    for ci in range(cin):
                        for kz in range(3):
                            for ky in range(3):
                                for kx in range(3):
                                    zz, y2, x2 = z + kz - 1, yy + ky - 1, xx + kx - 1
                                    if 0 <= zz < n and 0 <= y2 < n and 0 <= x2 < n:
                                        s += w[co, ci, kz, ky, kx] * x[ci, zz, y2, x2]
                    ref[co, z, yy, xx] = s
    np.testing.assert_allclose(y, ref, atol=1e-12)


def test_pool_and_upsample_semantics():
    x = torch.arange(64, dtype=torch.float64).reshape(1, 1, 4, 4, 4)
    p = F.avg_pool3d(x, 2)
    assert p[0, 0, 0, 0, 0] == np.mean([0, 1, 4, 5, 16, 17, 20, 21])
    u = F.interpolate(p, scale_factor=2, mode="nearest")
    assert u[0, 0, 1, 1, 1] == p[0, 0, 0, 0, 0] and u[0, 0, 2, 3, 2] == p[0, 0, 1, 1, 1]


def test_forward_positively_homogeneous_and_masked():
    n = 8
    cell = inputs.gen_mask(n, 1)
    mask = cell == 1
    rng = np.random.default_rng(2)
    r = np.where(mask, rng.standard_normal((n, n, n)), 0.0)
    w = unet.init_weights(3)
    z1 = unet.forward(w, r, mask, emulate_bf16=False)
    z2 = unet.forward(w, 3.7 * r, mask, emulate_bf16=False)
    np.testing.assert_allclose(z2, 3.7 * z1, rtol=1e-12, atol=1e-15)
    assert np.all(z1[~mask] == 0) and np.abs(z1).max() > 0
    assert np.all(unet.forward(w, 0 * r, mask) == 0)


def test_bf16_emulation_is_close_to_exact():
    n = 8
    cell = inputs.gen_mask(n, 1)
    mask = cell == 1
    rng = np.random.default_rng(4)
    r = np.where(mask, rng.standard_normal((n, n, n)), 0.0)
    w = unet.init_weights(5)
    za = unet.forward(w, r, mask, emulate_bf16=False)
    zb = unet.forward(w, r, mask, emulate_bf16=True)
    assert np.linalg.norm(za - zb) / np.linalg.norm(za) < 3e-2


def test_anorm_loss_geometry(orc):
    """Loss is 0 for z parallel to the true error e and 1 - cos^2 in the A
    inner product otherwise."""
    n = 8
    cell = inputs.gen_mask(n, 2)
    rng = np.random.default_rng(5)
    e = np.where(cell == 1, rng.standard_normal((n, n, n)), 0.0)
    r = orc.poisson_apply(cell, e)
    assert abs(unet.anorm_loss(2.5 * e, r, e, orc.poisson_apply(cell, 2.5 * e))) < 1e-12
    z = np.where(cell == 1, rng.standard_normal((n, n, n)), 0.0)
    Az = orc.poisson_apply(cell, z)
    cos2 = (z * r).sum() ** 2 / ((e * r).sum() * (z * Az).sum())
    assert abs(unet.anorm_loss(z, r, e, Az) - (1 - cos2)) < 1e-12
    assert 0 < unet.anorm_loss(z, r, e, Az) < 1


def test_loss_gradient_matches_fd(orc):
    """Autograd gradient of the loss (without bf16 rounding, so the map is
    piecewise smooth) against central FD on random weight directions."""
    n = 8
    cell = inputs.gen_mask(n, 3)
    mask = cell == 1
    rng = np.random.default_rng(6)
    e = np.where(mask, rng.standard_normal((n, n, n)), 0.0)
    r = orc.poisson_apply(cell, e)
    w = unet.init_weights(7).astype(np.float64)
    A = lambda x: orc.poisson_apply(cell, x)

    def loss_exact(wv):
        z = unet.forward(wv, r, mask, emulate_bf16=False)
        return unet.anorm_loss(z, r, e, A(z))

    # gradient without rounding: reuse loss_and_grad's graph with rounding off
    import oracle.unet as U
    saved = U.bf16
    U.bf16 = lambda t: t
    try:
        L, g, _ = U.loss_and_grad(w, r, e, mask, A)
    finally:
        U.bf16 = saved
    assert abs(L - loss_exact(w)) < 1e-12
    for _ in range(3):
        d = rng.standard_normal(w.size)
        h = 1e-7  # small: larger steps cross ReLU kinks of the piecewise-linear net
        fd = (loss_exact(w + h * d) - loss_exact(w - h * d)) / (2 * h)
        assert abs(fd - g @ d) < 1e-5 * max(1.0, abs(fd)), (fd, g @ d)


@pytest.mark.parametrize("p", [(32, 32, 32), (33, 34, 31)])
def test_activation_support_radius(p):
    """Support of every activation for a single liquid cell, with positive
    weights (so every voxel the receptive field reaches is strictly
    positive): the Chebyshev distance in fine cells from the liquid cell to
    the farthest fine cell under a non-zero voxel.  The library's inference
    pass relies on these reaches (its maps for the encoder layers use them
    as radii); the counts are 2^(l-1) per convolution at level l, plus the
    block alignment of each pooling."""
    n = 64
    W = unet.split_weights(np.full(unet.param_count(), 0.01, np.float32))
    r = np.zeros((n, n, n))
    r[p[2], p[1], p[0]] = 1.0
    _, acts = unet.forward(W, r, r > 0, emulate_bf16=False, return_all=True)
    zz, yy, xx = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    d = np.maximum(np.maximum(abs(xx - p[0]), abs(yy - p[1])), abs(zz - p[2]))
    reach = {}
    for k in ("a1", "e1", "p1", "a2", "e2", "p2", "a3", "e3", "b2", "d2", "b1", "d1"):
        a = acts[k][0].abs().sum(0).numpy() > 0
        f = n // a.shape[0]
        reach[k] = int(d[np.kron(a, np.ones((f, f, f), bool))].max())
    odd = p[0] % 2 == 1 or p[1] % 2 == 1 or p[2] % 2 == 1
    bound = {"a1": 1, "e1": 2, "p1": 3, "a2": 5, "e2": 7, "p2": 9, "a3": 13, "e3": 17, "b2": 19,
             "d2": 21, "b1": 22, "d1": 23}
    for k, b in bound.items():
        assert reach[k] <= b, (k, reach[k])
    if odd:  # an alignment that reaches the bound exactly
        assert reach == bound, reach
    assert max(reach.values()) < 24


def test_pruned_network_keeps_the_output():
    """The library's inference pass computes each layer only within a radius
    of liquid (the smaller of where the layer can be non-zero and where it can
    still reach the liquid-masked output): c1 1, c2 2, c3 5, c4 7, c7 5, c8 3,
    c9 2, c10 1 fine cells (a coarse voxel counts when a fine cell of its
    block does).  Zeroing every activation outside its radius, voxel by voxel,
    must leave z on the liquid cells exactly as it is, in FP64."""
    n = 48
    zz, yy, xx = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    mask = ((xx - 12) ** 2 + (yy - 14) ** 2 + (zz - 10) ** 2 <= 36) | ((xx > 36) & (yy < 4))
    rng = np.random.default_rng(5)
    r = np.where(mask, rng.standard_normal((n, n, n)), 0.0)
    W = [torch.as_tensor(w) for w in unet.split_weights(unet.init_weights(7))]
    # Chebyshev distance to liquid, in fine cells
    d = np.full((n, n, n), 10 ** 6)
    pts = np.argwhere(mask)
    for z, y, x in pts:
        np.minimum(d, np.maximum(np.maximum(abs(zz - z), abs(yy - y)), abs(xx - x)), out=d)

    def keep(t, radius):
        f = n // t.shape[-1]
        near = torch.as_tensor(d <= radius)
        near = near.reshape(n // f, f, n // f, f, n // f, f).any(dim=5).any(dim=3).any(dim=1)
        return t * near.to(t.dtype)

    rms = float(np.sqrt((r * r * mask).sum() / mask.sum()))
    x0 = torch.stack([torch.as_tensor(r / rms), torch.as_tensor(mask, dtype=torch.float64)])[None]

    def run(prune):
        k = (lambda t, rad: keep(t, rad)) if prune else (lambda t, rad: t)
        conv = lambda x, w, relu=True: F.relu(F.conv3d(x, w, padding=1)) if relu else F.conv3d(x, w, padding=1)
        a1 = k(conv(x0, W[0]), 1)
        e1 = k(conv(a1, W[1]), 2)
        a2 = k(conv(F.avg_pool3d(e1, 2), W[2]), 5)
        e2 = k(conv(a2, W[3]), 7)
        e3 = conv(conv(F.avg_pool3d(e2, 2), W[4]), W[5])
        b2 = k(conv(torch.cat([F.interpolate(e3, scale_factor=2, mode="nearest"), e2], 1), W[6]), 5)
        d2 = k(conv(b2, W[7]), 3)
        b1 = k(conv(torch.cat([F.interpolate(d2, scale_factor=2, mode="nearest"), e1], 1), W[8]), 2)
        d1 = k(conv(b1, W[9]), 1)
        return conv(d1, W[10], relu=False)[0, 0].numpy()

    dense, pruned = run(False), run(True)
    # the dense pass is the oracle's network
    np.testing.assert_allclose(mask * rms * dense, unet.forward(W, r, mask, emulate_bf16=False),
                               rtol=0, atol=1e-12 * np.abs(dense).max() * rms)
    assert np.abs(dense[mask]).max() > 0
    assert np.array_equal(dense[mask], pruned[mask])
    # the radii are tight enough to matter: pruning changes the activations
    assert not np.array_equal(dense, pruned)
