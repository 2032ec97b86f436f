"""Pins for the recurrent convolutional pressure solver's oracle: the Jacobi
kernel against a Jacobi sweep written from the Poisson operator, convergence
to the Poisson solution, the reverse pass against the transpose identity and
central differences, and the fit loss at its known minimiser."""
import numpy as np
import pytest

from oracle import fluid, percnn
from paper_2503_00868_amd import inputs


def _case(n, seed):
    cell = inputs.gen_mask(n, seed)
    liquid = cell == fluid.LIQUID
    rng = np.random.default_rng(seed)
    p = np.where(liquid, rng.standard_normal((n, n, n)), 0.0)
    b = np.where(liquid, rng.standard_normal((n, n, n)), 0.0)
    return cell, liquid, p, b


def test_tap_order_and_shift():
    assert percnn.tap_offset(0) == (-1, -1, -1)
    assert percnn.tap_offset(13) == (0, 0, 0)
    assert percnn.tap_offset(14) == (1, 0, 0)
    assert percnn.tap_offset(16) == (0, 1, 0)
    assert percnn.tap_offset(22) == (0, 0, 1)
    a = np.arange(27.0).reshape(3, 3, 3)
    s = percnn.shifted(a, 1, 0, 0)  # s(c) = a(c + x)
    assert s[0, 0, 0] == a[0, 0, 1] and s[0, 0, 2] == 0.0
    s = percnn.shifted(a, 0, 0, -1)
    assert s[1, 2, 2] == a[0, 2, 2] and s[0, 1, 1] == 0.0


@pytest.mark.parametrize("n,seed", [(10, 0), (12, 3)])
def test_jacobi_kernel_is_a_jacobi_sweep(n, seed):
    """One layer with the Jacobi kernel is p + D^-1 (b - A p) on liquid
    cells (0 elsewhere), with A and D from the projection's own operator."""
    cell, liquid, p, b = _case(n, seed)
    W, wb = percnn.jacobi_kernel()
    out = percnn.layer(cell, p, b, W, wb)
    D = fluid.poisson_diag(cell)
    ref = np.where(liquid, p + (b - fluid.poisson_apply(cell, p)) / np.where(D > 0, D, 1.0), 0.0)
    assert np.abs(out - ref).max() <= 1e-13 * np.abs(ref).max()
    # a kernel missing one face tap is not a Jacobi sweep
    W2 = W.copy()
    W2[14] = 0.0
    assert np.abs(percnn.layer(cell, p, b, W2, wb) - ref).max() > 1e-3


def test_jacobi_recurrence_converges_to_the_poisson_solution():
    n = 8
    cell, liquid, _, b = _case(n, 1)
    W, wb = percnn.jacobi_kernel()
    ps = percnn.forward(cell, np.zeros((n, n, n)), b, W, wb, 1500)
    x = fluid.pcg(cell, b, tol=1e-13)
    x = x[0] if isinstance(x, tuple) else x
    assert np.abs(ps[-1] - x).max() <= 1e-9 * np.abs(x).max()
    # the error contracts from sweep to sweep
    err = [np.abs(ps[k] - x).max() for k in (10, 50, 200)]
    assert err[0] > err[1] > err[2]


def test_reverse_pass_is_the_transpose():
    """<J (v_p, v_b), w> = <v_p, J^T_p w> + <v_b, J^T_b w> for the map
    (p0, b) -> p_K at fixed weights."""
    n, K = 9, 4
    cell, _, _, _ = _case(n, 2)
    rng = np.random.default_rng(11)
    W = rng.standard_normal(27) * 0.1
    wb = 0.3
    vp, vb, w = (rng.standard_normal((n, n, n)) for _ in range(3))
    ps = percnn.forward(cell, vp, vb, W, wb, K)
    gp, gb, _, _ = percnn.backward(cell, ps, vb, W, wb, w)
    lhs = float(np.sum(ps[-1] * w))
    rhs = float(np.sum(vp * gp) + np.sum(vb * gb))
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), 1.0)


def test_weight_gradient_matches_central_differences():
    n, K = 8, 3
    cell, _, p0, b = _case(n, 4)
    rng = np.random.default_rng(5)
    W = percnn.jacobi_kernel()[0] + 0.02 * rng.standard_normal(27)
    wb = 0.2
    g = rng.standard_normal((n, n, n))
    ps = percnn.forward(cell, p0, b, W, wb, K)
    _, _, gW, gwb = percnn.backward(cell, ps, b, W, wb, g)
    J = lambda W_, wb_: float(np.sum(g * percnn.forward(cell, p0, b, W_, wb_, K)[-1]))
    h = 1e-5
    for t in (0, 4, 13, 14, 22, 26):
        e = np.zeros(27)
        e[t] = h
        fd = (J(W + e, wb) - J(W - e, wb)) / (2 * h)
        assert abs(fd - gW[t]) <= 1e-7 * max(1.0, abs(fd)), (t, fd, gW[t])
    fd = (J(W, wb + h) - J(W, wb - h)) / (2 * h)
    assert abs(fd - gwb) <= 1e-7 * max(1.0, abs(fd))


def test_fit_loss_vanishes_at_the_generating_kernel():
    """Pairs made by K Jacobi layers: the fit loss and its gradient vanish at
    the Jacobi kernel, and a perturbed kernel has a positive loss whose
    gradient matches central differences."""
    n, K = 8, 3
    cell, liquid, _, _ = _case(n, 6)
    W, wb = percnn.jacobi_kernel()
    rng = np.random.default_rng(8)
    pairs = []
    for _ in range(3):
        p_before = np.where(liquid, rng.standard_normal((n, n, n)), 0.0)
        b = np.where(liquid, rng.standard_normal((n, n, n)), 0.0)
        p_after = percnn.forward(cell, p_before, b, W, wb, K)[-1]
        pairs.append((p_before, p_after, b))
    loss, gW, gwb = percnn.fit_loss(cell, pairs, W, wb, K)
    assert loss < 1e-25 and np.abs(gW).max() < 1e-12 and abs(gwb) < 1e-12
    W1 = W + 0.01 * rng.standard_normal(27)
    loss1, gW1, _ = percnn.fit_loss(cell, pairs, W1, wb, K)
    assert loss1 > 1e-6
    h = 1e-6
    e = np.zeros(27)
    e[14] = h
    fd = (percnn.fit_loss(cell, pairs, W1 + e, wb, K)[0] - percnn.fit_loss(cell, pairs, W1 - e, wb, K)[0]) / (2 * h)
    assert abs(fd - gW1[14]) <= 1e-6 * max(1.0, abs(fd))
