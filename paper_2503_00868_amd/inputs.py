"""Seeded synthetic liquid volumes: cell types and initial face velocities.

This module only builds inputs. It holds none of the fluid step's arithmetic
(no advection, diffusion, projection or face classification), so both the
GPU path and the FP64 oracle can take their inputs from it.

Stand-in for the paper's workloads (single-view videos of rivers over a fixed
bed and of viscous liquids, Section 4): the videos and their reconstructed
grids are not available, so every input here is synthetic.

Grid convention (unit box, ``n`` cells per axis, ``h = 1/n``):

* cell ``(i, j, k)`` has centre ``((i+1/2)h, (j+1/2)h, (k+1/2)h)``;
  arrays are C-ordered ``[k][j][i]`` so ``i`` is the fastest index;
* ``u`` lives on x-faces ``(i h, (j+1/2)h, (k+1/2)h)``, shape ``(n, n, n+1)``;
  ``v`` on y-faces, shape ``(n, n+1, n)``; ``w`` on z-faces, shape ``(n+1, n, n)``.

Cell types: 0 = air, 1 = liquid, 2 = solid.  Everything outside the box is
solid; the generator itself only emits air and liquid.
"""
from __future__ import annotations

import numpy as np

AIR, LIQUID, SOLID = 0, 1, 2

# Independent random streams per quantity, so changing one recipe does not
# shift the others.
_STREAM_MASK, _STREAM_VEL, _STREAM_NU, _STREAM_S = 0, 1, 2, 3


def _rng(seed: int, stream: int) -> np.random.Generator:
    return np.random.default_rng([int(seed), int(stream)])


def gen_mask(n: int, seed: int, slab_depth: float = 0.25, n_ellipsoids: int = 3,
             centre_range=(0.2, 0.8), axis_range=(0.15, 0.3)) -> np.ndarray:
    """Liquid mask: a bottom slab ``y < slab_depth`` plus ``n_ellipsoids``
    axis-aligned ellipsoids with seeded centres and semi-axes.

    Returns uint8 ``[k][j][i]`` with values AIR/LIQUID.
    """
    rng = _rng(seed, _STREAM_MASK)
    c = (np.arange(n) + 0.5) / n
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    liquid = y < slab_depth
    for _ in range(n_ellipsoids):
        ctr = rng.uniform(centre_range[0], centre_range[1], size=3)
        ax = rng.uniform(axis_range[0], axis_range[1], size=3)
        q = ((x - ctr[0]) / ax[0]) ** 2 + ((y - ctr[1]) / ax[1]) ** 2 + ((z - ctr[2]) / ax[2]) ** 2
        liquid |= q <= 1.0
    return np.where(liquid, LIQUID, AIR).astype(np.uint8)


def gen_velocity(n: int, seed: int, n_modes: int = 8, kmax: int = 4,
                 max_speed: float = 0.5):
    """Face velocities from the discrete curl of a random vector potential.

    The potential is a sum of ``n_modes`` separable Fourier modes with integer
    wave numbers in ``[1, kmax]^3`` and N(0,1) amplitudes; its tangential
    components vanish on the box walls, so the curl is exactly divergence-free
    on the MAC grid and carries no flux through the walls.  The field is then
    scaled so the largest face speed equals ``max_speed``.  No liquid masking
    is applied here.

    Returns float64 ``(u, v, w)`` with the shapes in the module docstring.
    """
    rng = _rng(seed, _STREAM_VEL)
    h = 1.0 / n
    node = np.arange(n + 1) * h          # edge/face coordinates on lattice lines
    mid = (np.arange(n) + 0.5) * h       # coordinates at cell centres
    pi = np.pi

    def sin_node(kk):
        s = np.sin(kk * pi * node)
        s[0] = s[-1] = 0.0  # exact zero on the walls, not sin(k pi) rounding
        return s
    # psi_x on x-edges ((i+1/2)h, j h, k h): shape [n+1][n+1][n]
    # psi_y on y-edges (i h, (j+1/2)h, k h): shape [n+1][n][n+1]
    # psi_z on z-edges (i h, j h, (k+1/2)h): shape [n][n+1][n+1]
    px = np.zeros((n + 1, n + 1, n))
    py = np.zeros((n + 1, n, n + 1))
    pz = np.zeros((n, n + 1, n + 1))
    for _ in range(n_modes):
        kx, ky, kz = rng.integers(1, kmax + 1, size=3)
        ax, ay, az = rng.standard_normal(3)
        px += ax * (sin_node(kz)[:, None, None] * sin_node(ky)[None, :, None]
                    * np.cos(kx * pi * mid)[None, None, :])
        py += ay * (sin_node(kz)[:, None, None] * np.cos(ky * pi * mid)[None, :, None]
                    * sin_node(kx)[None, None, :])
        pz += az * (np.cos(kz * pi * mid)[:, None, None] * sin_node(ky)[None, :, None]
                    * sin_node(kx)[None, None, :])
    # curl on the staggered grid
    u = (pz[:, 1:, :] - pz[:, :-1, :]) / h - (py[1:, :, :] - py[:-1, :, :]) / h
    v = (px[1:, :, :] - px[:-1, :, :]) / h - (pz[:, :, 1:] - pz[:, :, :-1]) / h
    w = (py[:, :, 1:] - py[:, :, :-1]) / h - (px[:, 1:, :] - px[:, :-1, :]) / h
    peak = max(np.abs(u).max(), np.abs(v).max(), np.abs(w).max())
    scale = max_speed / peak if peak > 0 else 0.0
    return u * scale, v * scale, w * scale


def gen_nu(seed: int, lo: float = 1e-4, hi: float = 1e-1) -> float:
    """Kinematic viscosity drawn log-uniformly from ``[lo, hi]``."""
    rng = _rng(seed, _STREAM_NU)
    return float(10.0 ** rng.uniform(np.log10(lo), np.log10(hi)))


def gen_scale(seed: int, lo: float = 0.5, hi: float = 1.5) -> float:
    """Initial-velocity scale ``s`` drawn uniformly from ``[lo, hi]``."""
    rng = _rng(seed, _STREAM_S)
    return float(rng.uniform(lo, hi))


def gen_case(n: int, seed: int):
    """Mask and unmasked velocities for one seed (float64)."""
    cell = gen_mask(n, seed)
    u, v, w = gen_velocity(n, seed)
    return cell, (u, v, w)


def liquid_fraction(cell: np.ndarray) -> float:
    return float(np.mean(cell == LIQUID))


_STREAM_SCREEN = 4


def gen_screen(H: int, W: int, seed: int, n_blobs: int = 6, blob_range=(0.05, 0.2)):
    """Inputs of the screen-space constrained projection (Section 3.3) for an
    H x W image, standing in for one frame of the paper's videos:

    * the interpolated screen velocity on pixel edges, a (H, W+1) and
      b (H+1, W): a few smooth modes plus small noise, as a mainstream-guided
      interpolation would leave it;
    * the out-of-plane velocity vz (H, W), smooth, and the depth z (H, W) in
      [1, 2];
    * the region where detection failed: a union of n_blobs discs (radii a
      fraction blob_range of min(H, W)) that never covers the whole image.

    Returns float32 (a, b, vz, z) and uint8 mask."""
    rng = _rng(seed, _STREAM_SCREEN)

    def smooth(shape, modes=4):
        yy, xx = np.meshgrid(np.linspace(0, 1, shape[0]), np.linspace(0, 1, shape[1]),
                             indexing="ij")
        f = np.zeros(shape)
        for _ in range(modes):
            kx, ky = rng.integers(1, 4, size=2)
            ph = rng.uniform(0, 2 * np.pi, size=2)
            f += rng.standard_normal() * np.sin(np.pi * kx * xx + ph[0]) * np.cos(np.pi * ky * yy + ph[1])
        return f

    a = smooth((H, W + 1)) + 0.05 * rng.standard_normal((H, W + 1))
    b = smooth((H + 1, W)) + 0.05 * rng.standard_normal((H + 1, W))
    vz = 0.3 * smooth((H, W))
    z = 1.0 + rng.random((H, W)) * 0.2 + 0.8 * (0.5 + 0.5 * np.tanh(smooth((H, W), 2)))
    jj, ii = np.meshgrid(np.arange(H), np.arange(W), indexing="ij")
    mask = np.zeros((H, W), dtype=bool)
    m = min(H, W)
    for _ in range(n_blobs):
        cj, ci = rng.uniform(0, H), rng.uniform(0, W)
        rad = rng.uniform(blob_range[0], blob_range[1]) * m
        mask |= (jj - cj) ** 2 + (ii - ci) ** 2 <= rad * rad
    if mask.all():
        mask[0, 0] = False
    return (a.astype(np.float32), b.astype(np.float32), vz.astype(np.float32),
            z.astype(np.float32), mask.astype(np.uint8))
