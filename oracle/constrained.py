"""FP64 oracle of the constrained divergence projection (test infrastructure
only: the tests, the smoke check and the benchmark's CPU leg may use it; the
GPU path never does).

The paper makes its reconstructed 3-D velocity divergence-free with a
constraint projection (Section 3.3, Eq. (divProj)): per cell i a constraint
C_i = (div v)_i = 0; each iteration sets

    lambda_i = -C_i / (sum_k |dC_i/dv_k|^2 + eps),
    v_j <- v_j + sum_i lambda_i dC_i/dv_j,

over all constraints at once, eps a relaxation parameter.  On the MAC grid
here (reading R20): the constraints are those of the liquid cells, the
variables are the active faces (non-active faces hold 0, as after a
projection), and C_i = (1/h) sum over the faces of i of the signed outflow,
so dC_i/dv_f = +1/h on the high face of i and -1/h on its low face.  The
sums below are written from that incidence, face by face, independently of
the projection's operators in ``fluid``.

Arrays: velocity components [z][y][x] with the face axis one longer.
"""
from __future__ import annotations

import numpy as np

from . import fluid


def _active(cell):
    return tuple(fluid.face_classes(cell, c) == fluid.ACTIVE for c in range(3))


def constraints(cell, fields):
    """C_i on liquid cells (0 elsewhere) from the active faces."""
    cell = np.asarray(cell, dtype=np.uint8)
    n = cell.shape[0]
    h = 1.0 / n
    act = _active(cell)
    u, v, w = (np.where(a, np.asarray(f, dtype=np.float64), 0.0) for a, f in zip(act, fields))
    C = ((u[:, :, 1:] - u[:, :, :-1]) + (v[:, 1:, :] - v[:, :-1, :]) + (w[1:, :, :] - w[:-1, :, :])) / h
    return np.where(cell == fluid.LIQUID, C, 0.0)


def gradient_norms(cell):
    """sum_k |dC_i/dv_k|^2 = (active faces of i) / h^2 on liquid cells."""
    cell = np.asarray(cell, dtype=np.uint8)
    n = cell.shape[0]
    act = [a.astype(np.float64) for a in _active(cell)]
    cnt = (act[0][:, :, 1:] + act[0][:, :, :-1] + act[1][:, 1:, :] + act[1][:, :-1, :]
           + act[2][1:, :, :] + act[2][:-1, :, :])
    return np.where(cell == fluid.LIQUID, cnt * n * n, 0.0)


def iterate(cell, fields, eps):
    """One iteration of Eq. (divProj) over every liquid-cell constraint."""
    cell = np.asarray(cell, dtype=np.uint8)
    n = cell.shape[0]
    h = 1.0 / n
    act = _active(cell)
    C = constraints(cell, fields)
    G = gradient_norms(cell)
    lam = np.where(cell == fluid.LIQUID, -C / np.where(G > 0, G + eps, 1.0), 0.0)
    # a face receives +lambda/h from the cell below it along its axis (its
    # high face) and -lambda/h from the cell above (its low face)
    out = []
    for comp, f in enumerate(fields):
        pad = [(0, 0)] * 3
        ax = 2 - comp  # array axis of this component's face direction
        pad[ax] = (1, 1)
        lp = np.pad(lam, pad)  # cells -1 .. n along the axis, zero outside
        below = np.take(lp, range(0, n + 1), axis=ax)      # cell index f - 1
        above = np.take(lp, range(1, n + 2), axis=ax)      # cell index f
        d = (below - above) / h
        g = np.where(act[comp], np.asarray(f, dtype=np.float64) + d, 0.0)
        out.append(g)
    return tuple(out)


def project(cell, fields, iters, eps=0.0):
    """`iters` iterations; returns the fields and max|C| after each."""
    out = tuple(np.asarray(f, dtype=np.float64) for f in fields)
    hist = []
    for _ in range(iters):
        out = iterate(cell, out, eps)
        hist.append(float(np.abs(constraints(cell, out)).max()))
    return out, hist
