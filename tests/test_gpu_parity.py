"""GPU parity: every kernel of the step, called through the C ABI, against
the FP64 oracle on the same seeded inputs.

Tolerances: single operators without a solve are compared element by element
at FP32 rounding level (a few ulp of the field scale); anything with a
Poisson solve is compared to the oracle's 1e-12 solve with the 1e-5 relative
velocity bound of the target (the GPU stops at a 1e-6 FP64 true residual,
which leaves about 4e-7 of velocity error; the rest is FP32 rounding).
"""
import numpy as np
import pytest

from paper_2503_00868_amd import inputs
from tests.gpu_util import banner, case, f32, rel_err, to_np

pytestmark = pytest.mark.gpu

DT = 1.0 / 120


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _sim(cell, **kw):
    from paper_2503_00868_amd.fluidsim import Sim
    return Sim(cell, **kw)


@pytest.mark.parametrize("n,seed,scale", [(32, 0, 1.0), (20, 1, 4.0), (13, 2, 6.0)])
def test_advect_parity(torch_gpu, orc, n, seed, scale):
    banner(f"advect n={n} seed={seed}")
    cell, u = case(n, seed, scale)
    u = orc.mask_faces(cell, u)
    sim = _sim(cell)
    sim.set_params(nu=1e-3, dt=DT)
    out = to_np(sim.op_advect(sim.to_faces(u)))
    ref = orc.add_force(cell, orc.advect(cell, u, DT), DT)
    for a, b in zip(out, ref):
        np.testing.assert_allclose(a, b, rtol=0, atol=4e-6 * max(1.0, np.abs(b).max()))


@pytest.mark.parametrize("n,nu,mode", [(32, 1e-3, "explicit"), (24, 2e-2, "implicit"),
                                       (17, 5e-1, "implicit")])
def test_diffuse_parity(torch_gpu, orc, n, nu, mode):
    banner(f"diffuse n={n} nu={nu} {mode}")
    cell, u = case(n, 3)
    u = orc.mask_faces(cell, u)
    sim = _sim(cell, diffusion=mode, diff_tol=1e-7)
    sim.set_params(nu=nu, dt=DT)
    out, st = sim.op_diffuse(sim.to_faces(u))
    out = to_np(out)
    ref, explicit, _ = orc.diffuse(cell, u, nu, DT, mode, 1e-12)
    l2, mx = rel_err(out, ref)
    assert mx < 2e-6, (l2, mx, st)
    if mode == "implicit":
        assert st["diff_iters"] > 0 and st["diff_rel_residual"] <= 1e-7


def test_diffuse_early_stop_inside_a_block(torch_gpu, orc):
    """The viscosity CG checks its FP64 residual every check_every
    iterations; when the recursive residual meets the tolerance inside a
    block, the block's remaining iterations are skipped and the block-end
    check decides.  Iteration counts then need not be multiples of the check
    period, and the result still matches the oracle's 1e-12 solve."""
    counts = []
    for n, nu, seed in ((24, 2e-2, 3), (24, 6e-2, 4), (28, 1e-1, 5), (20, 3e-1, 6)):
        banner(f"diffuse early stop n={n} nu={nu}")
        cell, u = case(n, seed)
        u = orc.mask_faces(cell, u)
        sim = _sim(cell, diffusion="implicit", diff_tol=1e-7, check_every=8)
        sim.set_params(nu=nu, dt=DT)
        out, st = sim.op_diffuse(sim.to_faces(u))
        counts.append(st["diff_iters"])
        ref, _, _ = orc.diffuse(cell, u, nu, DT, "implicit", 1e-12)
        l2, mx = rel_err(to_np(out), ref)
        assert mx < 2e-6, (n, nu, l2, mx, st)
        assert st["diff_rel_residual"] <= 1e-7, st
    banner(f"  iterations: {counts}")
    assert any(k % 8 != 0 for k in counts), counts


@pytest.mark.parametrize("n", [32, 19])
def test_divergence_and_poisson_apply_parity(torch_gpu, orc, n):
    banner(f"divergence/poisson n={n}")
    cell = inputs.gen_mask(n, 4)
    rng = np.random.default_rng(n)
    # a random (divergent) field: the generator's own field is exactly
    # divergence-free, which would leave only rounding noise to compare
    u = orc.mask_faces(cell, f32(tuple(rng.standard_normal(orc.face_shape(n, c)) for c in range(3))))
    sim = _sim(cell)
    b = sim.op_divergence(sim.to_faces(u)).cpu().numpy().astype(np.float64)
    ref = orc.divergence_rhs(cell, u)
    np.testing.assert_allclose(b, ref, rtol=0, atol=1e-6 * np.abs(ref).max())
    rng = np.random.default_rng(0)
    x = np.where(cell == 1, rng.standard_normal(cell.shape), 0.0).astype(np.float32)
    y = sim.op_poisson_apply(sim.cells_tensor(x)).cpu().numpy().astype(np.float64)
    yref = orc.poisson_apply(cell, x.astype(np.float64))
    # FP32 sums of up to 7 terms: a few ulp of the largest row value
    np.testing.assert_allclose(y, yref, rtol=0, atol=1e-6 * np.abs(yref).max())


@pytest.mark.parametrize("n", [16, 27])
def test_mic0_apply_parity(torch_gpu, orc, n):
    banner(f"mic0 apply n={n}")
    cell = inputs.gen_mask(n, 5)
    sim = _sim(cell, precond="mic0")
    rng = np.random.default_rng(1)
    r = np.where(cell == 1, rng.standard_normal(cell.shape), 0.0).astype(np.float32)
    z = sim.op_precond_apply("mic0", sim.cells_tensor(r)).cpu().numpy().astype(np.float64)
    ref = orc.mic0_apply(cell, orc.mic0_setup(cell), r.astype(np.float64))
    assert np.linalg.norm(z - ref) / np.linalg.norm(ref) < 2e-5
    assert np.all(z[cell != 1] == 0)
    zj = sim.op_precond_apply("jacobi", sim.cells_tensor(r)).cpu().numpy()
    d = orc.poisson_diag(cell)
    np.testing.assert_allclose(zj, np.where(d > 0, r / np.maximum(d, 1), 0), rtol=1e-6)


@pytest.mark.parametrize("precond", ["jacobi", "mic0"])
@pytest.mark.parametrize("n,seed", [(32, 0), (23, 6)])
def test_project_parity(torch_gpu, orc, precond, n, seed):
    banner(f"project n={n} seed={seed} {precond}")
    cell, u = case(n, seed)
    u = orc.add_force(cell, orc.mask_faces(cell, u), DT)
    sim = _sim(cell, precond=precond, check_every=4)
    U = sim.to_faces(u)
    st, p = sim.project(U, want_p=True)
    out = to_np(U)
    ref, p_ref, _, _ = orc.project(cell, u, 1e-12)
    l2, mx = rel_err(out, ref)
    assert mx < 1e-5, (l2, mx)
    assert st["rel_residual"] <= 1e-6
    # the FP64 true residual, recomputed by the oracle from the GPU pressure
    b = orc.divergence_rhs(cell, u)
    assert orc.true_relres(cell, b, p.cpu().numpy()) <= 1.01e-6
    # iteration count: the oracle's PCG with the same preconditioner, plus at
    # most one check period
    pc = orc.PRECOND_JACOBI if precond == "jacobi" else orc.PRECOND_MIC0
    _, it_ref, _ = orc.pcg(cell, b, pc, 1e-6)
    assert it_ref - 2 <= st["iters"] <= it_ref + 4 + 2, (st["iters"], it_ref)


def test_step_parity_small_config(torch_gpu, orc):
    """32^3, seed 0, nu = 1e-3 (explicit), Jacobi-PCG to 1e-6, one step."""
    banner("step 32^3 jacobi explicit")
    n, seed, nu = 32, 0, 1e-3
    cell, u = case(n, seed)
    u0 = orc.mask_faces(cell, u)
    sim = _sim(cell, precond="jacobi")
    sim.set_params(nu=nu, dt=DT)
    U = sim.to_faces(u0)
    st = sim.step(U, 1)[0]
    ref, info = orc.step(cell, u0, nu, DT)
    l2, mx = rel_err(to_np(U), ref)
    assert mx <= 1e-5 and l2 <= 1e-5, (l2, mx)
    assert st["rel_residual"] <= 1e-6 and st["diff_iters"] == 0
    assert orc.max_abs_divergence(cell, ref) < 1e-10
    banner(f"  iters gpu={st['iters']} oracle(1e-12)={info.proj_iters} rel={l2:.2e}/{mx:.2e}")


def test_step32_matches_stored_fixture(torch_gpu):
    """The same step against the stored oracle values (tests/golden)."""
    from tests.test_golden import load
    g = load("step32_seed0.txt")
    n, seed, nu = int(g["n"][0]), int(g["seed"][0]), float(g["nu"][0])
    cell, u = case(n, seed)
    sim = _sim(cell, precond="jacobi")
    sim.set_params(nu=nu, dt=DT)
    from oracle import fluid as orc
    U = sim.to_faces(orc.mask_faces(cell, u))
    assert sim.step(U, 1)[0]["rel_residual"] <= 1e-6
    for c, f in enumerate(to_np(U)):
        k = f"u1_{'uvw'[c]}"
        flat = f.reshape(-1)
        idx = np.array([int(v) for v in g[k + "_idx"]])
        want = np.array([float(v) for v in g[k + "_val"]])
        assert np.abs(flat[idx] - want).max() <= 1e-5 * np.abs(flat).max(), k


@pytest.mark.parametrize("precond,nu,steps", [("mic0", 5e-2, 3), ("jacobi", 2e-3, 4)])
def test_rollout_parity(torch_gpu, orc, precond, nu, steps):
    banner(f"rollout n=24 {precond} nu={nu}")
    n = 24
    cell, u = case(n, 7, 2.0)
    u0 = orc.mask_faces(cell, u)
    sim = _sim(cell, precond=precond)
    sim.set_params(nu=nu, dt=DT)
    U = sim.to_faces(u0)
    stats = sim.step(U, steps)
    ref = u0
    for _ in range(steps):
        ref, _ = orc.step(cell, ref, nu, DT)
    l2, mx = rel_err(to_np(U), ref)
    assert mx <= 1e-5 * steps and l2 <= 1e-5 * steps, (l2, mx)
    assert all(s["rel_residual"] <= 1e-6 for s in stats)


@pytest.mark.parametrize("precond", ["jacobi", "mic0"])
def test_rollout_warm_start_parity(torch_gpu, orc, precond):
    """Each solve of a warm-started rollout begins at the previous step's
    pressure: the fields still match the oracle's cold 1e-12 solves, every
    solve meets the 1e-6 residual, and the later solves need fewer
    iterations than the cold ones."""
    banner(f"warm rollout n=24 {precond}")
    n, steps, nu = 24, 4, 2e-3
    cell, u = case(n, 7, 2.0)
    u0 = orc.mask_faces(cell, u)
    iters = {}
    for warm in (False, True):
        sim = _sim(cell, precond=precond, warm_start=warm)
        sim.set_params(nu=nu, dt=DT)
        U = sim.to_faces(u0)
        stats = sim.step(U, steps)
        iters[warm] = [s["iters"] for s in stats]
        assert all(s["rel_residual"] <= 1e-6 for s in stats)
    ref = u0
    for _ in range(steps):
        ref, _ = orc.step(cell, ref, nu, DT)
    l2, mx = rel_err(to_np(U), ref)
    assert mx <= 1e-5 * steps and l2 <= 1e-5 * steps, (l2, mx)
    assert iters[True][0] == iters[False][0]
    assert sum(iters[True][1:]) < sum(iters[False][1:]), iters


def test_solid_cells_and_ragged_size(torch_gpu, orc):
    banner("solid obstacle n=18")
    n = 18
    cell, u = case(n, 8, 2.0)
    cell = cell.copy()
    cell[2:6, 0:3, 5:9] = 2  # an obstacle in the riverbed
    u0 = orc.mask_faces(cell, u)
    sim = _sim(cell, precond="mic0")
    sim.set_params(nu=3e-3, dt=DT)
    U = sim.to_faces(u0)
    sim.step(U, 2)
    ref = u0
    for _ in range(2):
        ref, _ = orc.step(cell, ref, 3e-3, DT)
    l2, mx = rel_err(to_np(U), ref)
    assert mx <= 2e-5, (l2, mx)


def test_no_liquid_and_zero_rhs(torch_gpu, orc):
    banner("all-air and resting slab")
    n = 16
    cell = np.zeros((n, n, n), np.uint8)
    sim = _sim(cell)
    sim.set_params(nu=1e-3, dt=DT)
    U = sim.faces(1.0)
    st = sim.step(U, 1)[0]
    assert st["iters"] == 0 and all(float(t.abs().max()) == 0.0 for t in U)
    # a resting full-width slab stays at rest (gravity kick removed by the projection)
    cell = np.zeros((n, n, n), np.uint8)
    cell[:, :5, :] = 1
    sim = _sim(cell, precond="mic0")
    sim.set_params(nu=1e-3, dt=DT)
    U = sim.faces(0.0)
    st = sim.step(U, 2)
    assert max(float(t.abs().max()) for t in U) < 1e-5 * 9.8 * DT


def test_determinism(torch_gpu, orc):
    banner("determinism")
    n = 32
    cell, u = case(n, 9)
    u0 = orc.mask_faces(cell, u)
    outs = []
    for _ in range(2):
        sim = _sim(cell, precond="jacobi")
        sim.set_params(nu=1e-3, dt=DT)
        U = sim.to_faces(u0)
        sim.step(U, 2)
        outs.append(to_np(U))
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


def test_not_converged_reports_status(torch_gpu, orc):
    banner("max_iter too small")
    from paper_2503_00868_amd.fluidsim import SIM_ERR_NOT_CONVERGED
    n = 16
    cell, u = case(n, 10)
    for precond, want in (("jacobi", 4), ("mic0", 3)):  # Jacobi iterates in groups of 4
        sim = _sim(cell, precond=precond, max_iter=3, check_every=2)
        sim.set_params(nu=1e-3, dt=DT)
        U = sim.to_faces(orc.mask_faces(cell, u))
        st, _ = sim.project(U, allow=(SIM_ERR_NOT_CONVERGED,))
        assert st["status"] == SIM_ERR_NOT_CONVERGED and st["iters"] == want, st
        assert st["rel_residual"] > 1e-6


def test_loss_parity(torch_gpu, orc):
    banner("loss")
    n = 20
    cell, u = case(n, 11)
    cell2, t = case(n, 12)
    u, t = orc.mask_faces(cell, u), orc.mask_faces(cell, t)
    sim = _sim(cell)
    J, g = sim.loss_mse(sim.to_faces(u), sim.to_faces(t))
    assert abs(J - orc.loss(cell, u, t)) <= 1e-6 * orc.loss(cell, u, t)
    for a, b in zip(to_np(g), orc.loss_grad(cell, u, t)):
        np.testing.assert_allclose(a, b, rtol=1e-5, atol=1e-12)
