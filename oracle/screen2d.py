"""FP64 oracle of the paper's screen-space constrained projection (test
infrastructure only: the tests, the smoke check and the benchmark's CPU leg
may use it; the GPU path never does).

Section 3.3 (Eq. (div2DV)): because the 3-D surface velocity is
divergence-free, the 2-D screen velocity v2D must satisfy
div_2D v2D = -(1/z)(u d/du + v d/dv + 2) v_z, with (u, v) screen
coordinates, z the depth and v_z the out-of-plane velocity.  Where optical
flow fails the paper starts v2D from its mainstream interpolation and
projects it onto this constraint with the projection method, leaving the
rest of the image as detected.  Reading R24:

  * the image is H x W pixels, rows j (v) and columns i (u); screen
    coordinates are normalised, u_i = -1 + (2i + 1)/W and
    v_j = -1 + (2j + 1)/H, with spacings du = 2/W and dv = 2/H;
  * v2D is staggered like the 3-D solver's velocity: a (the u component) on
    the H x (W + 1) vertical edges, b (the v component) on the (H + 1) x W
    horizontal edges; div at a pixel is (a_right - a_left)/du +
    (b_up - b_down)/dv;
  * the target s = -(1/z)(u D_u v_z + v D_v v_z + 2 v_z) per pixel, with
    v_z, z per pixel and D the second-order central difference (one-sided
    at the image border);
  * the corrected region is a pixel mask; an edge is free when at least one
    of its two pixels is in the region and both lie in the image; every
    other edge keeps its value;
  * the projection subtracts the gradient of a potential p that is 0 off
    the region (as air cells in the 3-D solve): on each free edge
    (p_hi - p_lo)/spacing, with p solving div(v - grad p) = s on the region.
    The result is the orthogonal (least-change) projection onto the
    constraint among fields that differ only on free edges.

Arrays: pixel fields [j][i]; a [j][i] with i the edge index (0..W);
b [j][i] with j the edge index (0..H).
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla


def coords(H, W):
    """Pixel-centre screen coordinates (u [W], v [H]) and spacings."""
    u = -1.0 + (2.0 * np.arange(W) + 1.0) / W
    v = -1.0 + (2.0 * np.arange(H) + 1.0) / H
    return u, v, 2.0 / W, 2.0 / H


def target(vz, z):
    """Right-hand side of Eq. (div2DV) per pixel."""
    vz = np.asarray(vz, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    H, W = vz.shape
    u, v, du, dv = coords(H, W)
    dvz_dv, dvz_du = np.gradient(vz, dv, du, edge_order=2)
    return -(u[None, :] * dvz_du + v[:, None] * dvz_dv + 2.0 * vz) / z


def divergence(a, b, H, W):
    _, _, du, dv = coords(H, W)
    return (a[:, 1:] - a[:, :-1]) / du + (b[1:, :] - b[:-1, :]) / dv


def free_edges(mask):
    """Free a-edges (H x (W+1)) and b-edges ((H+1) x W) of the region."""
    m = np.asarray(mask, dtype=bool)
    H, W = m.shape
    fa = np.zeros((H, W + 1), dtype=bool)
    fb = np.zeros((H + 1, W), dtype=bool)
    fa[:, 1:W] = m[:, :-1] | m[:, 1:]
    fb[1:H, :] = m[:-1, :] | m[1:, :]
    return fa, fb


def project(a, b, vz, z, mask):
    """(a', b', p): the projected screen velocity and the potential."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    m = np.asarray(mask, dtype=bool)
    H, W = m.shape
    _, _, du, dv = coords(H, W)
    fa, fb = free_edges(m)
    ids = -np.ones((H, W), dtype=np.int64)
    ids[m] = np.arange(int(m.sum()))
    N = int(m.sum())
    if N == 0:
        return a.copy(), b.copy(), np.zeros((H, W))
    # div(v - G p) = s on the region; D G = -A with A the (positive) masked
    # Laplacian over the free edges (p = 0 off the region), so A p = s - div v
    rows, cols, vals = [], [], []
    for j, i in zip(*np.nonzero(m)):
        r = ids[j, i]
        diag = 0.0
        for (free, nb, h) in ((fa[j, i], (j, i - 1), du), (fa[j, i + 1], (j, i + 1), du),
                              (fb[j, i], (j - 1, i), dv), (fb[j + 1, i], (j + 1, i), dv)):
            if not free:
                continue
            diag += 1.0 / (h * h)
            if m[nb]:
                rows.append(r)
                cols.append(ids[nb])
                vals.append(-1.0 / (h * h))
        rows.append(r)
        cols.append(r)
        vals.append(diag)
    A = sp.csr_matrix((vals, (rows, cols)), shape=(N, N))
    rhs = (target(vz, z) - divergence(a, b, H, W))[m]
    p = np.zeros((H, W))
    p[m] = spla.spsolve(A.tocsc(), rhs)
    pa = np.pad(p, ((0, 0), (1, 1)))
    pb = np.pad(p, ((1, 1), (0, 0)))
    ga = (pa[:, 1:] - pa[:, :-1]) / du   # edge i between pixels i-1 and i
    gb = (pb[1:, :] - pb[:-1, :]) / dv
    return np.where(fa, a - ga, a), np.where(fb, b - gb, b), p


def mainstream_fill(vel, detected, normal, radius):
    """The paper's mainstream-guided interpolation (Section 3.3, the equation
    before Eq. (div2DV)): for each pixel k where detection failed,
    v_k = sum_{i in B(k)} w(i) max(0, n_k . v_i / |v_i|) v_i.

    Reading R25: B(k) holds the detected pixels within Euclidean distance
    `radius` (in pixels) of k; w(i) = 1 - d(i, k) / (radius + 1), normalised
    to sum to 1 over B(k); a zero v_i contributes nothing; v_k = 0 when B(k)
    is empty.  vel (H, W, 3) velocities in NDC space, detected (H, W) bool,
    normal (H, W, 3) unit mainstream directions.  Detected pixels keep their
    velocity."""
    vel = np.asarray(vel, dtype=np.float64)
    det = np.asarray(detected, dtype=bool)
    nrm = np.asarray(normal, dtype=np.float64)
    H, W, _ = vel.shape
    r = int(radius)
    mag = np.linalg.norm(vel, axis=-1)
    unit = np.where(mag[..., None] > 0, vel / np.where(mag > 0, mag, 1.0)[..., None], 0.0)
    num = np.zeros((H, W, 3))
    wsum = np.zeros((H, W))
    for dj in range(-r, r + 1):
        for di in range(-r, r + 1):
            d = np.hypot(dj, di)
            if (dj == 0 and di == 0) or d > r:
                continue
            w = 1.0 - d / (r + 1)
            # neighbour i = k + (dj, di), for every pixel k that has one in the image
            kj = slice(max(0, -dj), min(H, H - dj))
            ki = slice(max(0, -di), min(W, W - di))
            nj = slice(max(0, dj), min(H, H + dj))
            ni = slice(max(0, di), min(W, W + di))
            ok = det[nj, ni]
            cosv = np.maximum(0.0, (nrm[kj, ki] * unit[nj, ni]).sum(-1))
            num[kj, ki] += (w * ok * cosv)[..., None] * vel[nj, ni]
            wsum[kj, ki] += w * ok
    fill = np.where(wsum[..., None] > 0, num / np.where(wsum > 0, wsum, 1.0)[..., None], 0.0)
    return np.where(det[..., None], vel, fill)

