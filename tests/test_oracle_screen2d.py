"""Pins for the screen-space constrained projection's oracle (Eq. (div2DV)):
closed forms of the target, the constraint met on the region, edges away
from the region untouched, idempotence, orthogonality to the constraint's
null space, and a dense brute-force solve."""
import numpy as np
import pytest

from oracle import screen2d as s2


def _case(H, W, seed, frac=0.35):
    rng = np.random.default_rng(seed)
    a = rng.standard_normal((H, W + 1))
    b = rng.standard_normal((H + 1, W))
    vz = rng.standard_normal((H, W))
    z = 1.0 + rng.random((H, W))
    mask = rng.random((H, W)) < frac
    mask[0, :] = False  # the region never covers the whole image
    return a, b, vz, z, mask


def test_target_closed_forms():
    H, W = 9, 13
    u, v, _, _ = s2.coords(H, W)
    # constant v_z and depth: s = -2 v_z / z
    assert np.allclose(s2.target(np.full((H, W), 0.7), np.full((H, W), 2.0)), -0.7, atol=1e-14)
    # v_z = u (depth 1): s = -(u * 1 + 2u) = -3u, also at the border (exact for linear fields)
    vz = np.broadcast_to(u[None, :], (H, W))
    assert np.allclose(s2.target(vz, np.ones((H, W))), -3.0 * vz, atol=1e-13)
    # v_z = v^2 (depth 1): s = -(2 v^2 + 2 v^2) = -4 v^2 (second order: exact for quadratics)
    vz = np.broadcast_to((v * v)[:, None], (H, W))
    assert np.allclose(s2.target(vz, np.ones((H, W))), -4.0 * vz, atol=1e-12)


@pytest.mark.parametrize("H,W,seed", [(12, 17, 0), (20, 15, 1)])
def test_constraint_met_and_rest_untouched(H, W, seed):
    a, b, vz, z, mask = _case(H, W, seed)
    a2, b2, p = s2.project(a, b, vz, z, mask)
    div = s2.divergence(a2, b2, H, W)
    t = s2.target(vz, z)
    assert np.abs(div - t)[mask].max() <= 1e-10 * np.abs(t).max()
    fa, fb = s2.free_edges(mask)
    assert np.array_equal(a2[~fa], a[~fa]) and np.array_equal(b2[~fb], b[~fb])
    assert not np.any(p[~mask])
    # projecting again changes nothing
    a3, b3, _ = s2.project(a2, b2, vz, z, mask)
    assert np.abs(a3 - a2).max() <= 1e-10 and np.abs(b3 - b2).max() <= 1e-10


def test_orthogonal_to_divergence_free_changes():
    """The change is orthogonal (plain sum over edges) to every field that
    lives on free edges and is divergence-free: discrete curls of stream
    functions on corners surrounded by region pixels."""
    H, W = 16, 16
    a, b, vz, z, mask = _case(H, W, 2, frac=0.7)
    a2, b2, _ = s2.project(a, b, vz, z, mask)
    _, _, du, dv = s2.coords(H, W)
    rng = np.random.default_rng(9)
    inner = np.zeros((H + 1, W + 1), dtype=bool)  # corners with all four pixels in the region
    inner[1:H, 1:W] = mask[:-1, :-1] & mask[:-1, 1:] & mask[1:, :-1] & mask[1:, 1:]
    assert inner.sum() > 5
    for _ in range(3):
        psi = np.where(inner, rng.standard_normal((H + 1, W + 1)), 0.0)
        wa = (psi[1:, :] - psi[:-1, :]) / dv          # on a-edges: d psi / dv
        wb = -(psi[:, 1:] - psi[:, :-1]) / du         # on b-edges: -d psi / du
        assert np.abs(s2.divergence(wa, wb, H, W)).max() < 1e-10
        fa, fb = s2.free_edges(mask)
        assert not np.any(wa[~fa]) and not np.any(wb[~fb])
        dot = float(((a2 - a) * wa).sum() + ((b2 - b) * wb).sum())
        scale = np.sqrt(float(((a2 - a) ** 2).sum() + ((b2 - b) ** 2).sum()) * float((wa ** 2).sum() + (wb ** 2).sum()))
        assert abs(dot) <= 1e-10 * scale


def test_dense_brute_force():
    """Least change subject to the constraint, as a dense KKT system over the
    free edges: minimise |x - x0|^2 subject to D x = s on the region."""
    H, W = 6, 7
    a, b, vz, z, mask = _case(H, W, 3, frac=0.5)
    a2, b2, _ = s2.project(a, b, vz, z, mask)
    fa, fb = s2.free_edges(mask)
    _, _, du, dv = s2.coords(H, W)
    edges = [("a", j, i) for j in range(H) for i in range(W + 1) if fa[j, i]] + \
            [("b", j, i) for j in range(H + 1) for i in range(W) if fb[j, i]]
    pix = [(j, i) for j in range(H) for i in range(W) if mask[j, i]]
    D = np.zeros((len(pix), len(edges)))
    for r, (j, i) in enumerate(pix):
        for c, (kind, ej, ei) in enumerate(edges):
            if kind == "a" and ej == j and ei == i + 1:
                D[r, c] = 1 / du
            if kind == "a" and ej == j and ei == i:
                D[r, c] = -1 / du
            if kind == "b" and ej == j + 1 and ei == i:
                D[r, c] = 1 / dv
            if kind == "b" and ej == j and ei == i:
                D[r, c] = -1 / dv
    x0 = np.array([a[j, i] if k == "a" else b[j, i] for k, j, i in edges])
    # the fixed edges' part of the divergence moves to the right-hand side
    full = s2.divergence(np.where(fa, 0.0, a), np.where(fb, 0.0, b), H, W)
    rhs = np.array([s2.target(vz, z)[j, i] - full[j, i] for j, i in pix])
    n, k = len(edges), len(pix)
    K = np.block([[np.eye(n), D.T], [D, np.zeros((k, k))]])
    sol = np.linalg.solve(K, np.concatenate([x0, rhs]))
    x = sol[:n]
    got = np.array([a2[j, i] if kk == "a" else b2[j, i] for kk, j, i in edges])
    assert np.abs(got - x).max() <= 1e-9 * max(1.0, np.abs(x).max())


def _fill_loops(vel, det, nrm, r):
    H, W, _ = vel.shape
    out = vel.copy()
    for j in range(H):
        for i in range(W):
            if det[j, i]:
                continue
            num = np.zeros(3)
            den = 0.0
            for jj in range(H):
                for ii in range(W):
                    d = np.hypot(jj - j, ii - i)
                    if not det[jj, ii] or d > r or (jj == j and ii == i):
                        continue
                    w = 1.0 - d / (r + 1)
                    v = vel[jj, ii]
                    m = np.linalg.norm(v)
                    c = max(0.0, float(nrm[j, i] @ v) / m) if m > 0 else 0.0
                    num += w * c * v
                    den += w
            out[j, i] = num / den if den > 0 else 0.0
    return out


def _stream_case(H, W, seed):
    rng = np.random.default_rng(seed)
    vel = rng.standard_normal((H, W, 3))
    det = rng.random((H, W)) < 0.5
    n = rng.standard_normal((H, W, 3))
    n /= np.linalg.norm(n, axis=-1, keepdims=True)
    return vel, det, n


@pytest.mark.parametrize("r", [1, 2, 3])
def test_mainstream_fill_matches_loops(r):
    vel, det, n = _stream_case(9, 11, r)
    vel[2, 3] = 0.0  # a zero velocity contributes nothing
    det[2, 3] = True
    got = s2.mainstream_fill(vel, det, n, r)
    assert np.abs(got - _fill_loops(vel, det, n, r)).max() < 1e-13


def test_mainstream_fill_closed_forms():
    """Neighbours all moving along the mainstream with speed V give V n;
    neighbours against it or across it give 0; scaling every detected
    velocity by c > 0 scales the fill by c."""
    H, W, r = 8, 8, 2
    det = np.ones((H, W), dtype=bool)
    det[4, 4] = False
    n = np.zeros((H, W, 3))
    n[..., 0] = 1.0
    vel = np.zeros((H, W, 3))
    vel[..., 0] = 2.5
    assert np.allclose(s2.mainstream_fill(vel, det, n, r)[4, 4], [2.5, 0.0, 0.0], atol=1e-14)
    assert np.allclose(s2.mainstream_fill(-vel, det, n, r)[4, 4], 0.0)
    across = np.zeros((H, W, 3))
    across[..., 1] = 1.0
    assert np.allclose(s2.mainstream_fill(across, det, n, r)[4, 4], 0.0)
    vel2, det2, n2 = _stream_case(10, 10, 7)
    a = s2.mainstream_fill(vel2, det2, n2, 2)
    b = s2.mainstream_fill(3.0 * vel2, det2, n2, 2)
    assert np.abs(b - 3.0 * a).max() < 1e-12
