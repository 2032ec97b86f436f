"""Pins for the masked cosine + L2 loss's oracle (Eq. (optLoss)): the cell
classes against neighbour loops and a hand-built mask, closed forms of the
two terms, the cosine's scale invariance, the class weights, and the
gradient against central differences."""
import numpy as np
import pytest

from oracle import fluid
from oracle import loss as orc_loss
from paper_2503_00868_amd import inputs


def _classes_loops(cell):
    n0, n1, n2 = cell.shape
    out = np.zeros(cell.shape, np.uint8)
    for k in range(n0):
        for j in range(n1):
            for i in range(n2):
                t = cell[k, j, i]
                if t == fluid.SOLID:
                    out[k, j, i] = orc_loss.NONE
                elif t == fluid.AIR:
                    out[k, j, i] = orc_loss.EMPTY
                else:
                    air = False
                    for dk, dj, di in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
                        q = (k + dk, j + dj, i + di)
                        if all(0 <= x < s for x, s in zip(q, cell.shape)) and cell[q] == fluid.AIR:
                            air = True
                    out[k, j, i] = orc_loss.SURFACE if air else orc_loss.OCCUPIED
    return out


def _vec_loops(fields, k, j, i):
    u, v, w = fields
    return np.array([0.5 * (u[k, j, i] + u[k, j, i + 1]), 0.5 * (v[k, j, i] + v[k, j + 1, i]),
                     0.5 * (w[k, j, i] + w[k + 1, j, i])])


def _fields(n, rng, scale=1.0):
    return tuple(scale * rng.standard_normal(fluid.face_shape(n, c)) for c in range(3))


@pytest.mark.parametrize("n,seed", [(8, 0), (11, 3)])
def test_classes_match_neighbour_loops(n, seed):
    cell, _ = inputs.gen_case(n, seed)
    cell = np.asarray(cell, np.uint8)
    got = orc_loss.classes(cell)
    assert np.array_equal(got, _classes_loops(cell))
    # the generator's masks hold every class
    assert all(np.any(got == c) for c in (orc_loss.EMPTY, orc_loss.OCCUPIED, orc_loss.SURFACE))


def test_classes_hand_built():
    """A 5^3 block of liquid with one air cell at its centre: the six
    neighbours of the air cell are surface cells, the other liquid cells
    occupied; the box's outside is wall, so the outer layer is not surface."""
    cell = np.full((5, 5, 5), fluid.LIQUID, np.uint8)
    cell[2, 2, 2] = fluid.AIR
    cell[0, 0, 0] = fluid.SOLID
    cls = orc_loss.classes(cell)
    assert cls[2, 2, 2] == orc_loss.EMPTY
    assert cls[0, 0, 0] == orc_loss.NONE
    assert (cls == orc_loss.SURFACE).sum() == 6
    for q in ((1, 2, 2), (3, 2, 2), (2, 1, 2), (2, 3, 2), (2, 2, 1), (2, 2, 3)):
        assert cls[q] == orc_loss.SURFACE
    assert (cls == orc_loss.OCCUPIED).sum() == 125 - 1 - 1 - 6


def test_identical_fields_give_zero_and_opposite_ones_two_alpha():
    n = 7
    cell, _ = inputs.gen_case(n, 1)
    rng = np.random.default_rng(2)
    f = _fields(n, rng)
    J, g = orc_loss.loss(cell, f, f, 0.7, 1.3, 0.0, (1.0, 1.0, 1.0))
    assert abs(J) < 1e-13
    assert max(np.abs(x).max() for x in g) < 1e-12
    neg = tuple(-x for x in f)
    J2, _ = orc_loss.loss(cell, f, neg, 0.7, 0.0, 0.0, (1.0, 1.0, 1.0))
    assert abs(J2 - 2 * 0.7) < 1e-12


def test_l2_term_and_class_weights_by_loops():
    """alpha = 0: J is the weighted mean of |a - b|^2 over the cells, with the
    cell-centred velocities formed face by face; weights (0, 0, 1) keep only
    the surface cells."""
    n = 6
    cell, _ = inputs.gen_case(n, 4)
    cell = np.asarray(cell, np.uint8)
    rng = np.random.default_rng(4)
    s, r = _fields(n, rng), _fields(n, rng)
    cls = _classes_loops(cell)
    for weights in ((1.0, 1.0, 1.0), (0.0, 0.0, 1.0), (0.5, 2.0, 3.0)):
        num = den = 0.0
        for k in range(n):
            for j in range(n):
                for i in range(n):
                    c = cls[k, j, i]
                    if c == orc_loss.NONE:
                        continue
                    wgt = weights[c]
                    d = _vec_loops(s, k, j, i) - _vec_loops(r, k, j, i)
                    num += wgt * float(d @ d)
                    den += wgt
        J, _ = orc_loss.loss(cell, s, r, 0.0, 1.0, 0.0, weights)
        assert abs(J - num / den) <= 1e-12 * abs(num / den)


def test_cosine_term_by_loops_and_scale_invariance():
    n = 6
    cell, _ = inputs.gen_case(n, 5)
    cell = np.asarray(cell, np.uint8)
    rng = np.random.default_rng(5)
    s, r = _fields(n, rng), _fields(n, rng)
    cls = _classes_loops(cell)
    num = den = 0.0
    for k in range(n):
        for j in range(n):
            for i in range(n):
                if cls[k, j, i] == orc_loss.NONE:
                    continue
                a, b = _vec_loops(s, k, j, i), _vec_loops(r, k, j, i)
                num += 1.0 - float(a @ b) / (np.linalg.norm(a) * np.linalg.norm(b))
                den += 1.0
    J, _ = orc_loss.loss(cell, s, r, 1.0, 0.0, 0.0, (1.0, 1.0, 1.0))
    assert abs(J - num / den) <= 1e-12
    J2, _ = orc_loss.loss(cell, s, tuple(3.7 * x for x in r), 1.0, 0.0, 0.0, (1.0, 1.0, 1.0))
    assert abs(J2 - J) <= 1e-12


@pytest.mark.parametrize("eps", [0.0, 0.05])
def test_gradient_matches_central_differences(eps):
    n = 6
    cell, _ = inputs.gen_case(n, 6)
    rng = np.random.default_rng(6)
    s, r = _fields(n, rng), _fields(n, rng)
    args = (0.8, 1.7, eps, (0.5, 1.0, 2.0))
    _, g = orc_loss.loss(cell, s, r, *args)
    h = 1e-6
    for _ in range(30):
        c = int(rng.integers(0, 3))
        idx = tuple(int(rng.integers(0, m)) for m in fluid.face_shape(n, c))
        plus = [x.copy() for x in s]
        minus = [x.copy() for x in s]
        plus[c][idx] += h
        minus[c][idx] -= h
        fd = (orc_loss.loss(cell, plus, r, *args)[0] - orc_loss.loss(cell, minus, r, *args)[0]) / (2 * h)
        assert abs(fd - g[c][idx]) <= 1e-6 * max(1e-3, abs(fd)), (c, idx, fd, g[c][idx])


def test_centre_velocity_of_a_linear_field_is_exact():
    """Faces carrying a field linear in position, u_c = a_c + B[c] . x_face:
    the mean of a cell's two c-faces is exactly a_c + B[c] . x_centre (a
    linear function's value at the midpoint), so the L2 term against a zero
    reference equals the closed-form sum of |a + B x_centre|^2 over the
    weighted cells.  Averaging along the wrong axis, or a shifted index,
    gives another value (B has entries along every axis)."""
    n = 7
    h = 1.0 / n
    cell, _ = inputs.gen_case(n, 1)
    cell = np.asarray(cell, np.uint8)
    a = np.array([0.3, -0.2, 0.1])
    B = np.array([[1.0, -0.5, 0.25], [0.75, 2.0, -1.0], [-0.3, 0.6, 1.5]])  # B[c][axis x, y, z]
    sim = []
    for c in range(3):
        shp = fluid.face_shape(n, c)
        k, j, i = np.meshgrid(*[np.arange(s) for s in shp], indexing="ij")
        pos = [(i + 0.5) * h, (j + 0.5) * h, (k + 0.5) * h]
        pos[c] = (i, j, k)[c] * h  # the face sits on a cell boundary along its own axis
        sim.append(a[c] + B[c, 0] * pos[0] + B[c, 1] * pos[1] + B[c, 2] * pos[2])
    k, j, i = np.meshgrid(*[np.arange(n)] * 3, indexing="ij")
    xc = np.stack([(i + 0.5) * h, (j + 0.5) * h, (k + 0.5) * h], -1)
    vel = a + xc @ B.T  # exact centre velocity (n, n, n, 3)
    assert np.abs(orc_loss.cell_vectors(sim) - vel).max() <= 1e-14
    zero = tuple(np.zeros(fluid.face_shape(n, c)) for c in range(3))
    weights = (0.2, 1.0, 2.0)
    cls = orc_loss.classes(cell)
    wt = np.choose(np.minimum(cls, 3), list(weights) + [0.0])
    ref = float((wt * (vel * vel).sum(-1)).sum() / wt.sum())
    J, _ = orc_loss.loss(cell, sim, zero, 0.0, 1.0, 0.0, weights)
    assert abs(J - ref) <= 1e-13 * ref
