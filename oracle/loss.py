"""FP64 oracle of the paper's masked cosine + L2 velocity loss (test
infrastructure only: the tests, the smoke check and the benchmark's CPU leg
may use it; the GPU path never does).

Eq. (optLoss) (Section 3.4.2) scores a simulated velocity field against a
reference one cell by cell: alpha times one minus the cosine of the angle
between the two velocities, plus beta times their squared L2 distance, each
cell weighted by a grid mask that tells surface, occupied and empty cells
apart.  The reading used here (R22) on the MAC grid:

  * velocities are compared at cell centres: component c of a cell's
    velocity is the mean of its two c-faces;
  * classes: a liquid cell with an air cell among its six neighbours is a
    surface cell, any other liquid cell an occupied cell, an air cell an
    empty cell; solid cells take no part (outside the box counts as solid);
  * cos = a.b / sqrt((|a|^2 + eps^2)(|b|^2 + eps^2)), with a small velocity
    eps that keeps it defined at rest (eps = 0 gives the plain cosine);
  * per cell l = alpha (1 - cos) + beta |a - b|^2, and
    J = sum_cells w(class) l / sum_cells w(class), one weight per class.

The gradient with respect to the simulated face velocities is the chain
rule through the cell-centre mean: each face takes half of dJ/da of each of
the (up to two) cells it separates.

Arrays: cells [z][y][x]; face components [z][y][x] with the face axis one
longer.
"""
from __future__ import annotations

import numpy as np

from . import fluid

EMPTY, OCCUPIED, SURFACE, NONE = 0, 1, 2, 3


def classes(cell):
    """Per-cell class: EMPTY (air), OCCUPIED, SURFACE (liquid) or NONE (solid)."""
    cell = np.asarray(cell, dtype=np.uint8)
    padded = np.pad(cell, 1, constant_values=fluid.SOLID)
    air_nb = np.zeros(cell.shape, dtype=bool)
    n0, n1, n2 = cell.shape
    for axis in range(3):
        for s in (-1, 1):
            sl = [slice(1, n0 + 1), slice(1, n1 + 1), slice(1, n2 + 1)]
            sl[axis] = slice(1 + s, (n0, n1, n2)[axis] + 1 + s)
            air_nb |= padded[tuple(sl)] == fluid.AIR
    out = np.full(cell.shape, NONE, dtype=np.uint8)
    out[cell == fluid.AIR] = EMPTY
    liq = cell == fluid.LIQUID
    out[liq & air_nb] = SURFACE
    out[liq & ~air_nb] = OCCUPIED
    return out


def cell_vectors(fields):
    """Cell-centred velocity (..., 3) from the three face components."""
    u, v, w = (np.asarray(f, dtype=np.float64) for f in fields)
    return np.stack([0.5 * (u[:, :, 1:] + u[:, :, :-1]),
                     0.5 * (v[:, 1:, :] + v[:, :-1, :]),
                     0.5 * (w[1:, :, :] + w[:-1, :, :])], axis=-1)


def loss(cell, sim, ref, alpha, beta, eps, weights):
    """J and dJ/d(simulated face velocities) (three arrays).

    weights = (w_empty, w_occupied, w_surface)."""
    cls = classes(cell)
    wt = np.zeros(cls.shape)
    for k, c in enumerate((EMPTY, OCCUPIED, SURFACE)):
        wt[cls == c] = float(weights[k])
    W = float(wt.sum())
    a = cell_vectors(sim)
    b = cell_vectors(ref)
    aa = (a * a).sum(-1) + eps * eps
    bb = (b * b).sum(-1) + eps * eps
    ab = (a * b).sum(-1)
    A = np.sqrt(aa)
    B = np.sqrt(bb)
    with np.errstate(divide="ignore", invalid="ignore"):
        cos = np.where(A * B > 0, ab / (A * B), 0.0)
        dcos = np.where((A * B > 0)[..., None],
                        b / (A * B)[..., None] - (ab / (aa * A * B))[..., None] * a, 0.0)
    d = a - b
    l = alpha * (1.0 - cos) + beta * (d * d).sum(-1)
    if W <= 0:
        n = cell.shape[0]
        return 0.0, tuple(np.zeros(fluid.face_shape(n, c)) for c in range(3))
    J = float((wt * l).sum()) / W
    ga = (wt / W)[..., None] * (-alpha * dcos + 2.0 * beta * d)
    grads = []
    for c in range(3):
        g = ga[..., c]
        ax = 2 - c  # array axis of this component's face direction
        pad = [(0, 0)] * 3
        pad[ax] = (1, 1)
        gp = np.pad(g, pad)
        m = g.shape[ax]
        lo = np.take(gp, range(0, m + 1), axis=ax)   # the cell before the face
        hi = np.take(gp, range(1, m + 2), axis=ax)   # the cell after it
        grads.append(0.5 * (lo + hi))
    return J, tuple(grads)
