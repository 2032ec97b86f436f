"""FP64 oracle of the upwind analytic convection gradient (test
infrastructure only: the tests, the smoke check and the benchmark's CPU leg
may use it; the GPU path never does).

The paper does not differentiate its semi-Lagrangian back-trace (grid
indexing and rounding make it a poor gradient); it uses the analytic
gradient of the split convection equation dv/dt = -(v . grad) v instead:
the derivative of the convected velocity v with respect to the component
v'_i before convection is -dt dv/dx_i, discretised by first-order upwind
differences (Section 3.4.1).  The reading used here (R21) on the MAC grid,
for a loss with gradient lam = dJ/dv (one array per face component):

    dJ/dv'_i (f) = [f active] ( lam_i(f) - dt sum_c Lam_c(f) D_i V_c(f) )

for every face f of component i, where
  * V_c and Lam_c are v_c and lam_c at the position of f: the value itself
    for c = i, else the mean of the four c-faces around that position (zero
    outside the box), as the advection interpolates velocity to faces;
  * D_i V_c(f) is the first-order upwind difference of V_c along axis i at
    f, against the sign of the advecting component v_i(f):
    (V_c(f) - V_c(f - e_i)) / h if v_i(f) > 0, else (V_c(f + e_i) - V_c(f)) / h,
    with V_c = 0 at positions outside the box;
  * the identity term lam_i is the derivative of the transported value.

This is the paper's surrogate, not the derivative of the step as computed
(R13 keeps that one); the two are compared in the design notes.

Arrays: face components [z][y][x], axis of the face direction one longer.
"""
from __future__ import annotations

import numpy as np

from . import fluid


def _at_faces(n, src, c, i):
    """Component c (array src) at the positions of the i-faces: the value for
    c == i, else the mean of the four c-faces around each i-face position."""
    if c == i:
        return np.asarray(src, dtype=np.float64).copy()
    shape = fluid.face_shape(n, i)
    out = np.zeros(shape)
    src = np.asarray(src, dtype=np.float64)
    ai, ac = 2 - i, 2 - c  # array axes of the two face directions
    # the i-face at index m along axis ai sits between cells m-1 and m of that
    # axis; the c-faces around it are at cells m-1 and m (axis ai) and at
    # face indices q and q+1 (axis ac) for its cell q along ac
    for da in (-1, 0):
        for dc in (0, 1):
            # source index along ai: m + da (cell), along ac: q + dc (face)
            sl_out = [slice(None)] * 3
            sl_src = [slice(None)] * 3
            # ai: out m in [0, n]; src cell m + da must be in [0, n)
            lo = max(0, -da)
            hi = min(n + 1, n - da)
            sl_out[ai] = slice(lo, hi)
            sl_src[ai] = slice(lo + da, hi + da)
            # ac: out cell q in [0, n); src face q + dc in [0, n]
            sl_out[ac] = slice(0, n)
            sl_src[ac] = slice(dc, n + dc)
            out[tuple(sl_out)] += 0.25 * src[tuple(sl_src)]
    return out


def _upwind_diff(V, vi, axis, h):
    """First-order upwind difference of V along `axis` against the sign of
    vi (same shape), zero outside the array."""
    pad = [(0, 0)] * 3
    pad[axis] = (1, 1)
    Vp = np.pad(V, pad)
    n1 = V.shape[axis]
    back = V - np.take(Vp, range(0, n1), axis=axis)
    fwd = np.take(Vp, range(2, n1 + 2), axis=axis) - V
    return np.where(vi > 0, back, fwd) / h


def gradient(cell, v, lam, dt):
    """dJ/dv' (three arrays) from the convected field v and lam = dJ/dv."""
    cell = np.asarray(cell, dtype=np.uint8)
    n = cell.shape[0]
    h = 1.0 / n
    out = []
    for i in range(3):
        act = fluid.face_classes(cell, i) == fluid.ACTIVE
        vi = np.asarray(v[i], dtype=np.float64)
        acc = np.asarray(lam[i], dtype=np.float64).copy()
        for c in range(3):
            Vc = _at_faces(n, v[c], c, i)
            Lc = _at_faces(n, lam[c], c, i)
            acc -= dt * Lc * _upwind_diff(Vc, vi, 2 - i, h)
        out.append(np.where(act, acc, 0.0))
    return tuple(out)


def _face_val(n, arr, c, idx):
    """Face idx = (k, j, i) of component c, zero outside its array."""
    k, j, i = idx
    shp = fluid.face_shape(n, c)
    if 0 <= k < shp[0] and 0 <= j < shp[1] and 0 <= i < shp[2]:
        return float(arr[c][k, j, i])
    return 0.0


def _at_pos(n, arr, c, comp, idx):
    """arr's component c at the position of the comp-face idx = (k, j, i)."""
    if c == comp:
        return _face_val(n, arr, c, idx)
    shp = fluid.face_shape(n, comp)
    if not all(0 <= x < s for x, s in zip(idx, shp)):
        return 0.0
    ai, ac = 2 - comp, 2 - c
    s = 0.0
    for da in (-1, 0):
        for dc in (0, 1):
            q = list(idx)
            q[ai] = idx[ai] + da
            q[ac] = idx[ac] + dc
            if not (0 <= q[ai] < n):
                continue
            s += 0.25 * _face_val(n, arr, c, tuple(q))
    return s


def face_gradient(n, v, lam, dt, comp, idx):
    """dJ/dv'_comp at the comp-face idx = (k, j, i), taken as active (the
    caller zeroes non-active faces), by the definition face by face."""
    h = 1.0 / n
    ax = 2 - comp
    lo, hi = list(idx), list(idx)
    lo[ax] -= 1
    hi[ax] += 1
    acc = float(lam[comp][tuple(idx)])
    for c in range(3):
        V0 = _at_pos(n, v, c, comp, tuple(idx))
        d = ((V0 - _at_pos(n, v, c, comp, tuple(lo))) if v[comp][tuple(idx)] > 0
             else (_at_pos(n, v, c, comp, tuple(hi)) - V0)) / h
        acc -= dt * _at_pos(n, lam, c, comp, tuple(idx)) * d
    return acc


def gradient_loops(cell, v, lam, dt):
    """The same as gradient(), face by face with explicit loops (small grids
    only)."""
    cell = np.asarray(cell, dtype=np.uint8)
    n = cell.shape[0]
    v = [np.asarray(a, dtype=np.float64) for a in v]
    lam = [np.asarray(a, dtype=np.float64) for a in lam]
    out = []
    for comp in range(3):
        act = fluid.face_classes(cell, comp) == fluid.ACTIVE
        shp = fluid.face_shape(n, comp)
        g = np.zeros(shp)
        for k in range(shp[0]):
            for j in range(shp[1]):
                for i in range(shp[2]):
                    if act[k, j, i]:
                        g[k, j, i] = face_gradient(n, v, lam, dt, comp, (k, j, i))
        out.append(g)
    return tuple(out)
