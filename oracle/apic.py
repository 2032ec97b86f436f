"""FP64 oracle of the paper's affine particle-in-cell (APIC) transfers (test
infrastructure only: the tests, the smoke check and the benchmark's CPU leg
may use it; the GPU path never does).

Section 3.2.2 (Eqs. (particle_map) and the transfer back) moves velocity
between particles and the grid around the grid step:

  * particles to grid: each grid node takes the mass-weighted sum of the
    particles' velocities extended by their affine part C_p (x_i - x_p), and
    divides by the weighted mass;
  * grid to particles: each particle takes the weighted sum of the updated
    grid velocities, and its new affine matrix is 4 / dx^2 times the weighted
    sum of v_i (x_i - x_p)^T (the factor of the quadratic kernel);
  * the particle moves by dt times its new velocity.

The weights are the quadratic B-spline, a product over the three axes.
Reading R23 on the MAC grid (the paper writes the transfer for a collocated
grid):
  * each velocity component a lives on its own lattice, the centres of the
    a-faces: node (i, j, k) of component 0 sits at h (i, j + 1/2, k + 1/2),
    and likewise for the others;
  * row a of C_p is the affine part of component a, so P2G for component a
    uses v_pa + C_p[a] . (x_i - x_p) and G2P forms C_p[a] from component a's
    nodes;
  * nodes outside a component's lattice take no part (their weight is 0 for
    particles at least one cell inside the box);
  * a node with no weighted mass keeps velocity 0.

Arrays: positions (P, 3) as (x, y, z) in the unit box; velocities (P, 3);
C (P, 3, 3); masses (P,); grid components [z][y][x] with the face axis one
longer.
"""
from __future__ import annotations

import numpy as np

from . import fluid


def bspline2(r):
    """Quadratic B-spline N(r) (support |r| < 3/2)."""
    a = np.abs(np.asarray(r, dtype=np.float64))
    return np.where(a < 0.5, 0.75 - a * a, np.where(a < 1.5, 0.5 * (1.5 - a) ** 2, 0.0))


def _offset(comp):
    """Lattice offset of component comp's nodes, in cells, per axis (x, y, z)."""
    off = np.full(3, 0.5)
    off[comp] = 0.0
    return off


def stencil(n, comp, xp):
    """For each particle the 27 nodes of component comp around it: node
    indices (P, 27, 3) as (i, j, k), their weights (P, 27) and positions
    (P, 27, 3); nodes outside the lattice get weight 0 (index clipped)."""
    xp = np.asarray(xp, dtype=np.float64)
    h = 1.0 / n
    X = xp / h - _offset(comp)                     # lattice units
    base = np.floor(X - 0.5).astype(np.int64)      # first of the three nodes
    shape = np.array(fluid.face_shape(n, comp))[::-1]   # (nx, ny, nz)
    offs = np.array([(a, b, c) for c in range(3) for b in range(3) for a in range(3)])
    idx = base[:, None, :] + offs[None, :, :]
    w = np.prod(bspline2(X[:, None, :] - idx), axis=-1)
    inside = np.all((idx >= 0) & (idx < shape), axis=-1)
    w = np.where(inside, w, 0.0)
    pos = (idx + _offset(comp)) * h
    return np.clip(idx, 0, shape - 1), w, pos


def p2g(n, xp, vp, Cp, mp):
    """Particles to grid: (grid velocity components, grid masses per component)."""
    xp = np.asarray(xp, dtype=np.float64)
    vp = np.asarray(vp, dtype=np.float64)
    Cp = np.asarray(Cp, dtype=np.float64)
    mp = np.asarray(mp, dtype=np.float64)
    vel, mass = [], []
    for a in range(3):
        idx, w, pos = stencil(n, a, xp)
        contrib = vp[:, a, None] + np.einsum("pj,pkj->pk", Cp[:, a, :], pos - xp[:, None, :])
        shp = fluid.face_shape(n, a)
        mom = np.zeros(shp)
        m = np.zeros(shp)
        flat = (idx[..., 2], idx[..., 1], idx[..., 0])
        np.add.at(mom, flat, w * mp[:, None] * contrib)
        np.add.at(m, flat, w * mp[:, None])
        with np.errstate(divide="ignore", invalid="ignore"):
            vel.append(np.where(m > 0, mom / np.where(m > 0, m, 1.0), 0.0))
        mass.append(m)
    return tuple(vel), tuple(mass)


def g2p(n, grid, xp):
    """Grid to particles: (velocities (P, 3), affine matrices (P, 3, 3))."""
    xp = np.asarray(xp, dtype=np.float64)
    h = 1.0 / n
    P = xp.shape[0]
    vp = np.zeros((P, 3))
    Cp = np.zeros((P, 3, 3))
    for a in range(3):
        idx, w, pos = stencil(n, a, xp)
        g = np.asarray(grid[a], dtype=np.float64)[idx[..., 2], idx[..., 1], idx[..., 0]]
        vp[:, a] = (w * g).sum(1)
        Cp[:, a, :] = (4.0 / (h * h)) * np.einsum("pk,pkj->pj", w * g, pos - xp[:, None, :])
    return vp, Cp


def advect(xp, vp, dt):
    """x_p + dt v_p."""
    return np.asarray(xp, dtype=np.float64) + dt * np.asarray(vp, dtype=np.float64)
