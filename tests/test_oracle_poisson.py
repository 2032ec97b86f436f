"""Pins for the oracle's pressure projection (Poisson matrix, solvers, MIC(0)).

Each test checks the oracle against something other than itself: a closed
form, a LAPACK dense solve, an identity between two independently coded
operators, or a special case with a known exact answer.
"""
import numpy as np
import pytest

from paper_2503_00868_amd import inputs

AIR, LIQ, SOL = 0, 1, 2


def _dense_poisson(orc, cell):
    """Dense matrix of the oracle's Poisson apply, restricted to liquid cells."""
    n = cell.shape[0]
    liq = np.flatnonzero(cell.ravel() == LIQ)
    A = np.zeros((liq.size, liq.size))
    for col, c in enumerate(liq):
        e = np.zeros(n ** 3)
        e[c] = 1.0
        A[:, col] = orc.poisson_apply(cell, e.reshape(n, n, n)).ravel()[liq]
    return A, liq


def _random_mask(n, seed, frac=0.5):
    rng = np.random.default_rng(seed)
    cell = np.where(rng.random((n, n, n)) < frac, LIQ, AIR).astype(np.uint8)
    return cell


def _face_basis(n):
    sizes = [int(np.prod((n + (c == 2), n + (c == 1), n + (c == 0)))) for c in range(3)]
    return sizes


def _divergence_matrix(orc, cell):
    """Columns: b-vector produced by a unit velocity on one face (all faces)."""
    n = cell.shape[0]
    sizes = _face_basis(n)
    cols = []
    for comp in range(3):
        shp = (n + (comp == 2), n + (comp == 1), n + (comp == 0))
        for q in range(sizes[comp]):
            f = [np.zeros((n + (c == 2), n + (c == 1), n + (c == 0))) for c in range(3)]
            f[comp].ravel()[q] = 1.0
            cols.append(orc.divergence_rhs(cell, f).ravel())
    return np.array(cols).T, sizes


def test_poisson_matrix_equals_divergence_gram(orc):
    """A = D_a D_a^T / h^2 where D_a is the divergence restricted to active
    faces: pins the diagonal count, the neighbour couplings and their sign
    against the independently coded divergence."""
    n = 5
    cell = _random_mask(n, 1, 0.6)
    cell[2, 2, 2] = SOL
    A, liq = _dense_poisson(orc, cell)
    B, sizes = _divergence_matrix(orc, cell)
    act = np.concatenate([(orc.face_classes(cell, c).ravel() == orc.ACTIVE) for c in range(3)])
    Bl = B[liq][:, act]
    G = Bl @ Bl.T * n * n
    np.testing.assert_allclose(A, G, atol=1e-12)


def test_poisson_matrix_spd(orc):
    cell = inputs.gen_mask(8, 3)
    A, _ = _dense_poisson(orc, cell)
    np.testing.assert_array_equal(A, A.T)
    assert np.linalg.eigvalsh(A).min() > 1e-8


def test_dense_direct_solve_8cubed(orc):
    """PCG (all three preconditioners) to 1e-12 against LAPACK on 8^3."""
    n = 8
    cell = inputs.gen_mask(n, 5)
    A, liq = _dense_poisson(orc, cell)
    rng = np.random.default_rng(0)
    b = np.zeros(n ** 3)
    b[liq] = rng.standard_normal(liq.size)
    x_ref = np.linalg.solve(A, b[liq])
    for pc in (orc.PRECOND_NONE, orc.PRECOND_JACOBI, orc.PRECOND_MIC0):
        x, it, rr = orc.pcg(cell, b.reshape(n, n, n), pc, 1e-12)
        assert rr < 1e-11
        np.testing.assert_allclose(x.ravel()[liq], x_ref, rtol=0, atol=1e-9 * np.abs(x_ref).max())
        assert np.all(x.ravel()[cell.ravel() != LIQ] == 0.0)


def _interior_box(n):
    cell = np.full((n, n, n), AIR, np.uint8)
    cell[1:-1, 1:-1, 1:-1] = LIQ
    return cell


def test_discrete_eigenvector_dirichlet(orc):
    """Liquid interior ringed by air: sin modes vanishing at the air cell
    centres are exact eigenvectors, eigenvalue sum_a (2 - 2 cos(theta_a))."""
    n = 12
    h = 1.0 / n
    cell = _interior_box(n)
    c = (np.arange(n) + 0.5) * h
    L = 1.0 - h
    kx, ky, kz = 1, 2, 3
    sx = np.sin(kx * np.pi * (c - h / 2) / L)
    sy = np.sin(ky * np.pi * (c - h / 2) / L)
    sz = np.sin(kz * np.pi * (c - h / 2) / L)
    p = sz[:, None, None] * sy[None, :, None] * sx[None, None, :]
    p[cell != LIQ] = 0.0
    lam = sum(2 - 2 * np.cos(k * np.pi * h / L) for k in (kx, ky, kz))
    Ap = orc.poisson_apply(cell, p)
    np.testing.assert_allclose(Ap, lam * p, atol=1e-12)


def test_discrete_eigenvector_walls_and_surface(orc):
    """Full-width slab under air: cosine modes are exact eigenvectors with
    Neumann walls on the sides and bottom and p = 0 at the first air row."""
    n = 10
    h = 1.0 / n
    J = 4
    cell = np.full((n, n, n), AIR, np.uint8)
    cell[:, :J, :] = LIQ
    c = (np.arange(n) + 0.5) * h
    Y = (J + 0.5) * h
    kx, kz = 2, 1
    p = (np.cos(kz * np.pi * c)[:, None, None] * np.cos(np.pi * c / (2 * Y))[None, :, None]
         * np.cos(kx * np.pi * c)[None, None, :])
    p[cell != LIQ] = 0.0
    lam = (2 - 2 * np.cos(kx * np.pi * h)) + (2 - 2 * np.cos(kz * np.pi * h)) + \
        (2 - 2 * np.cos(np.pi * h / (2 * Y)))
    np.testing.assert_allclose(orc.poisson_apply(cell, p), lam * p, atol=1e-12)


def test_manufactured_solution_second_order(orc):
    """-lap p = f with p = prod sin on the liquid box; the discrete solution
    converges to the continuous one at O(h^2)."""
    errs, hs = [], []
    for n in (8, 16, 32):
        h = 1.0 / n
        cell = _interior_box(n)
        c = (np.arange(n) + 0.5) * h
        L = 1.0 - h
        s = np.sin(np.pi * (c - h / 2) / L)
        pe = s[:, None, None] * s[None, :, None] * s[None, None, :]
        pe[cell != LIQ] = 0.0
        b = h * h * 3 * (np.pi / L) ** 2 * pe
        x, it, rr = orc.pcg(cell, b, orc.PRECOND_NONE, 1e-13)
        errs.append(np.abs(x - pe).max())
        hs.append(h / L)  # grid spacing relative to the liquid box width
    orders = [np.log(errs[q] / errs[q + 1]) / np.log(hs[q] / hs[q + 1]) for q in range(2)]
    assert all(1.85 < o < 2.15 for o in orders), (errs, orders)


def test_hydrostatic_slab_returns_to_rest(orc):
    """A resting full-width slab given the gravity kick is projected back to
    exactly zero velocity, with pressure linear in depth (rho g depth dt)."""
    n = 8
    J = 3
    dt = 1.0 / 120
    cell = np.full((n, n, n), AIR, np.uint8)
    cell[:, :J, :] = LIQ
    f = tuple(np.zeros(orc.face_shape(n, c)) for c in range(3))
    f = orc.add_force(cell, f, dt)
    out, p, it, rr = orc.project(cell, f, 1e-13)
    for a in out:
        assert np.abs(a).max() < 1e-12
    h = 1.0 / n
    expect = 9.8 * dt * h * (J - np.arange(J))
    for j in range(J):
        np.testing.assert_allclose(p[:, j, :], expect[j], rtol=1e-10)


def test_projection_symmetric_idempotent_divfree(orc):
    n = 10
    cell = inputs.gen_mask(n, 2)
    rng = np.random.default_rng(4)
    a = tuple(rng.standard_normal(orc.face_shape(n, c)) for c in range(3))
    b = tuple(rng.standard_normal(orc.face_shape(n, c)) for c in range(3))
    Pa, _, _, _ = orc.project(cell, a, 1e-13)
    Pb, _, _, _ = orc.project(cell, b, 1e-13)
    PPa, _, _, _ = orc.project(cell, Pa, 1e-13)
    dot = lambda x, y: sum(float((p * q).sum()) for p, q in zip(x, y))
    assert abs(dot(Pa, b) - dot(a, Pb)) < 1e-9 * abs(dot(Pa, b))
    for x, y in zip(Pa, PPa):
        np.testing.assert_allclose(x, y, atol=1e-9)
    assert orc.max_abs_divergence(cell, Pa) < 1e-8 * n


def test_post_projection_divergence_generated_input(orc):
    """After a 1e-12 solve the discrete divergence is below 1e-10."""
    n = 32
    cell, ug = inputs.gen_case(n, 0)
    f = orc.mask_faces(cell, ug)
    f = orc.add_force(cell, orc.advect(cell, f, 1 / 120), 1 / 120)
    out, p, it, rr = orc.project(cell, f, 1e-12)
    assert rr <= 1e-12
    assert orc.max_abs_divergence(cell, out) < 1e-10


def _mic_factor(orc, cell, precon):
    """Dense lower factor L from the MIC(0) precon vector: diagonal
    1/precon, below-diagonal A_mc * precon_m for lower neighbours m."""
    n = cell.shape[0]
    liq = np.flatnonzero(cell.ravel() == LIQ)
    pos = {c: q for q, c in enumerate(liq)}
    Lf = np.zeros((liq.size, liq.size))
    pr = precon.ravel()
    for q, c in enumerate(liq):
        Lf[q, q] = 1.0 / pr[c]
        i, j, k = c % n, (c // n) % n, c // (n * n)
        for (di, dj, dk) in ((1, 0, 0), (0, 1, 0), (0, 0, 1)):
            ii, jj, kk = i - di, j - dj, k - dk
            if min(ii, jj, kk) < 0:
                continue
            m = ii + n * (jj + n * kk)
            if m in pos:
                Lf[q, pos[m]] = -1.0 * pr[m]
    return Lf, liq


def test_mic0_is_ic0_when_tau_zero(orc):
    """tau = 0, sigma = 0: L L^T reproduces A on A's sparsity pattern."""
    n = 6
    cell = inputs.gen_mask(n, 7)
    A, liq = _dense_poisson(orc, cell)
    pc = orc.mic0_setup(cell, 0.0, 0.0)
    Lf, _ = _mic_factor(orc, cell, pc)
    M = Lf @ Lf.T
    pat = A != 0
    np.testing.assert_allclose(M[pat], A[pat], atol=1e-12)


def test_mic0_row_sums_when_tau_one(orc):
    """tau = 1 (full modification): row sums of L L^T equal those of A,
    wherever the sigma safeguard did not fire."""
    n = 6
    cell = _interior_box(n)
    A, liq = _dense_poisson(orc, cell)
    pc = orc.mic0_setup(cell, 1.0, 0.0)
    Lf, _ = _mic_factor(orc, cell, pc)
    M = Lf @ Lf.T
    np.testing.assert_allclose(M.sum(1), A.sum(1), atol=1e-12)


def test_mic0_apply_inverts_factor(orc):
    n = 6
    cell = inputs.gen_mask(n, 9)
    pc = orc.mic0_setup(cell)
    Lf, liq = _mic_factor(orc, cell, pc)
    rng = np.random.default_rng(1)
    r = np.zeros(n ** 3)
    r[liq] = rng.standard_normal(liq.size)
    z = orc.mic0_apply(cell, pc, r.reshape(n, n, n)).ravel()
    np.testing.assert_allclose(z[liq], np.linalg.solve(Lf @ Lf.T, r[liq]), atol=1e-10)


def test_mic0_exact_on_a_line(orc):
    """On a single row of liquid cells the matrix is tridiagonal, IC(0) has no
    dropped fill, so MIC(0) applies the exact inverse."""
    n = 9
    cell = np.full((n, n, n), AIR, np.uint8)
    cell[3, 4, 1:8] = LIQ
    A, liq = _dense_poisson(orc, cell)
    pc = orc.mic0_setup(cell)
    r = np.zeros(n ** 3)
    r[liq] = np.arange(1, liq.size + 1, dtype=float)
    z = orc.mic0_apply(cell, pc, r.reshape(n, n, n)).ravel()
    np.testing.assert_allclose(z[liq], np.linalg.solve(A, r[liq]), atol=1e-12)


def test_pcg_zero_rhs(orc):
    cell = inputs.gen_mask(8, 1)
    x, it, rr = orc.pcg(cell, np.zeros((8, 8, 8)), orc.PRECOND_JACOBI, 1e-6)
    assert it == 0 and np.all(x == 0)


def test_iteration_counts_ordering(orc):
    """MIC(0) needs far fewer iterations than Jacobi on the generated mask."""
    n = 24
    cell, ug = inputs.gen_case(n, 0)
    f = orc.add_force(cell, orc.mask_faces(cell, ug), 1 / 120)
    b = orc.divergence_rhs(cell, f)
    _, itj, _ = orc.pcg(cell, b, orc.PRECOND_JACOBI, 1e-6)
    _, itm, _ = orc.pcg(cell, b, orc.PRECOND_MIC0, 1e-6)
    assert itm * 2 < itj
