"""FP64 oracle of the recurrent convolutional pressure solver (test
infrastructure only: the tests, the smoke check and the benchmark's CPU leg
may use it; the GPU path never does).

The paper solves the pressure Poisson equation during its optimisation with
a PeRCNN-style recurrent network: a convolution over the pressure latent,
fed with the boundary-condition and velocity latents, applied recurrently
like the sweeps of an iterative solver, with the kernel fitted on pressure
pairs from an implicit solve (Section 3.4.1, Fig. "percnn_str_fit").  The
paper does not print the layer; the reading used here (R19) is

    p_{k+1}(c) = L(c) * s(c) * ( sum_t W_t p_k(c + t) + w_b * b(c) )

over the 27 offsets t of a 3x3x3 stencil (t = (dx, dy, dz) in {-1,0,1}^3,
tap index (dx+1) + 3 (dy+1) + 9 (dz+1)), with p_k = 0 outside the box.  The
boundary-condition latent is the pair (L, s): L(c) = 1 on liquid cells and 0
elsewhere (air is the p = 0 Dirichlet side, solid cells carry no pressure),
and s(c) = 6 / n_c with n_c the number of non-solid faces of c (the diagonal
of the Poisson matrix).  b is the velocity latent: the right-hand side
b = -h div u of the projection.  With the Jacobi kernel (W = 1/6 on the six
face neighbours, 0 elsewhere, w_b = 1/6) one layer is exactly one Jacobi
sweep of that Poisson system, which is the second-order discretisation the
fitted kernel is expected to reproduce.

The fit takes pairs (p_before, p_after) with their b and minimises
sum over liquid cells of (layer^K(p_before) - p_after)^2 over (W, w_b); its
gradient is the reverse pass below.

Arrays are [z][y][x] float64.
"""
from __future__ import annotations

import numpy as np

from . import fluid

NTAPS = 27


def tap_offset(t: int):
    """(dx, dy, dz) of tap t."""
    return (t % 3 - 1, (t // 3) % 3 - 1, t // 9 - 1)


def shifted(a, dx, dy, dz):
    """out(c) = a(c + (dx, dy, dz)) with zero outside the box."""
    n = a.shape[0]
    out = np.zeros_like(a)
    zs, ys, xs = [slice(max(0, -d), n - max(0, d)) for d in (dz, dy, dx)]
    zd, yd, xd = [slice(max(0, d), n - max(0, -d)) for d in (dz, dy, dx)]
    out[zs, ys, xs] = a[zd, yd, xd]
    return out


def latents(cell):
    """(L, s): liquid indicator and 6 / n_c (0 off liquid)."""
    cell = np.asarray(cell, dtype=np.uint8)
    nc = fluid.poisson_diag(cell)
    liquid = (cell == fluid.LIQUID).astype(np.float64)
    s = np.where(liquid > 0, 6.0 / np.where(nc > 0, nc, 1.0), 0.0)
    return liquid, s


def jacobi_kernel():
    """(W, w_b) of one Jacobi sweep."""
    W = np.zeros(NTAPS)
    for t in range(NTAPS):
        dx, dy, dz = tap_offset(t)
        if abs(dx) + abs(dy) + abs(dz) == 1:
            W[t] = 1.0 / 6.0
    return W, 1.0 / 6.0


def layer(cell, p, b, W, wb, lat=None):
    """One recurrent layer (the definition above)."""
    L, s = lat if lat is not None else latents(cell)
    acc = wb * np.asarray(b, dtype=np.float64)
    for t in range(NTAPS):
        if W[t] != 0.0:
            acc = acc + W[t] * shifted(np.asarray(p, dtype=np.float64), *tap_offset(t))
    return L * s * acc


def forward(cell, p0, b, W, wb, K):
    """K layers from p0; returns the list of states p_0 .. p_K."""
    lat = latents(cell)
    ps = [np.asarray(p0, dtype=np.float64)]
    for _ in range(K):
        ps.append(layer(cell, ps[-1], b, W, wb, lat))
    return ps


def backward(cell, ps, b, W, wb, g):
    """Reverse pass of forward() for a loss with dL/dp_K = g.

    Returns (dL/dp_0, dL/db, dL/dW (27), dL/dw_b).  One layer is
    p' = L s (sum_t W_t S_t p + w_b b) with S_t the shift by t, so with
    u = L s g':  dL/dp = sum_t W_t S_t^T u,  dL/db += w_b u,
    dL/dW_t += <u, S_t p>,  dL/dw_b += <u, b>;  S_t^T is the shift by -t
    (both drop what leaves the box)."""
    L, s = latents(cell)
    b = np.asarray(b, dtype=np.float64)
    gp = np.asarray(g, dtype=np.float64)
    gb = np.zeros_like(b)
    gW = np.zeros(NTAPS)
    gwb = 0.0
    for k in range(len(ps) - 1, 0, -1):
        u = L * s * gp
        p = ps[k - 1]
        gb += wb * u
        gwb += float(np.sum(u * b))
        nxt = np.zeros_like(u)
        for t in range(NTAPS):
            dx, dy, dz = tap_offset(t)
            gW[t] += float(np.sum(u * shifted(p, dx, dy, dz)))
            nxt += W[t] * shifted(u, -dx, -dy, -dz)
        gp = nxt
    return gp, gb, gW, gwb


def fit_loss(cell, pairs, W, wb, K):
    """(loss, dW, dw_b) of the fit: pairs is a list of (p_before, p_after, b);
    the loss is the mean over pairs of the sum over liquid cells of the
    squared error of layer^K(p_before) against p_after."""
    L, _ = latents(cell)
    loss, gW, gwb = 0.0, np.zeros(NTAPS), 0.0
    for p_before, p_after, b in pairs:
        ps = forward(cell, p_before, b, W, wb, K)
        err = L * (ps[-1] - p_after)
        loss += float(np.sum(err * err))
        _, _, dW, dwb = backward(cell, ps, b, W, wb, 2.0 * err)
        gW += dW
        gwb += dwb
    m = len(pairs)
    return loss / m, gW / m, gwb / m
