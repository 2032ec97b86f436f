"""GPU gradient parity: the checkpointed adjoint behind the autograd
Function against the FP64 oracle's exact discrete gradient at 16^3 (1e-4
relative), and a central FD of the GPU rollout in theta as a sanity check."""
import numpy as np
import pytest
import math

from paper_2503_00868_amd import inputs
from tests.gpu_util import banner, case, rel_err, to_np

pytestmark = pytest.mark.gpu

DT = 1.0 / 120


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    assert torch.cuda.is_available()
    return torch


@pytest.mark.parametrize("mode,nu_t,nu_e,K,warm", [("explicit", 4e-3, 2e-3, 2, False),
                                                   ("implicit", 8e-2, 5e-2, 3, False),
                                                   ("explicit", 4e-3, 2e-3, 2, True),
                                                   ("implicit", 8e-2, 5e-2, 3, True)])
def test_gradient_matches_oracle(torch_gpu, orc, mode, nu_t, nu_e, K, warm):
    """With warm starts the solves begin from the previous pressures (forward
    and adjoint) and the segment recompute from the pressures stored at the
    checkpoints; the gradient is the same to the solver tolerance."""
    torch = torch_gpu
    from paper_2503_00868_amd.fluidsim import Sim
    from paper_2503_00868_amd.autograd import mse_loss, rollout
    banner(f"gradient 16^3 {mode} K={K} warm={warm}")
    n, steps, s_t, s_e = 16, 5, 1.2, 0.8
    cell, ug = case(n, 100, 2.0)
    target = orc.rollout(cell, ug, nu_t, s_t, steps, DT, mode=mode, tol=1e-12)[-1]
    ref = orc.rollout_grad(cell, ug, nu_e, s_e, steps, DT, target, mode=mode, tol=1e-12)
    sim = Sim(cell, precond="mic0", diffusion=mode, tol=1e-9, diff_tol=1e-9, max_steps=steps,
              checkpoint_every=K, warm_start=warm)
    th_nu = torch.tensor(math.log(nu_e), dtype=torch.float64, requires_grad=True)
    th_s = torch.tensor(math.log(s_e), dtype=torch.float64, requires_grad=True)
    ugen = tuple(t.requires_grad_(True) for t in sim.to_faces(ug))
    uT = rollout(th_nu, th_s, ugen, sim, steps, DT)
    J = mse_loss(sim, uT, sim.to_faces(target))
    J.backward()
    assert abs(J.item() - ref["J"]) <= 1e-4 * ref["J"]
    for got, want, name in ((th_nu.grad.item(), ref["dtheta_nu"], "nu"),
                            (th_s.grad.item(), ref["dtheta_s"], "s")):
        assert abs(got - want) <= 1e-4 * abs(want), (name, got, want)
    l2, mx = rel_err(to_np(tuple(t.grad for t in ugen)), ref["du_gen"])
    assert l2 <= 1e-4, (l2, mx)


@pytest.mark.parametrize("mode", ["explicit", "implicit"])
def test_pressure_history_gives_the_same_gradient(torch_gpu, mode):
    """With store_pressures the backward's recompute starts each projection
    from the forward's own pressure (no iteration) and, for implicit
    viscosity, copies the forward's viscosity output.  The recomputed states
    are those of the recompute that repeats the warm-started solves, so the
    gradients agree to the run-to-run noise of the advection adjoint's FP32
    atomic scatter (1e-6 relative here; two identical runs differ likewise)."""
    from paper_2503_00868_amd.fluidsim import Sim
    banner(f"pressure history, {mode}")
    n, steps, K = 20, 5, 2
    nu = 4e-3 if mode == "explicit" else 8e-2
    cell, ug = case(n, 100, 2.0)
    out = []
    for store in (False, True, False):
        sim = Sim(cell, precond="jacobi", diffusion=mode, tol=1e-8, max_steps=steps,
                  checkpoint_every=K, warm_start=True, store_pressures=store)
        sim.set_params(nu=nu, dt=DT, s=0.9)
        ugen = sim.to_faces(ug)
        u = sim.faces()
        sim.init_state(ugen, u)
        sim.step(u, steps, record=True)
        J, gT = sim.loss_mse(u, sim.faces())
        g0, dnu, ds, _ = sim.backward(gT, ugen=ugen)
        out.append((dnu, ds, to_np(g0)))
    for other in (out[1], out[2]):
        assert abs(out[0][0] - other[0]) <= 1e-6 * abs(out[0][0])
        assert abs(out[0][1] - other[1]) <= 1e-6 * abs(out[0][1])
        l2, _ = rel_err(other[2], out[0][2])
        assert l2 <= 1e-6, l2


def test_gradient_fd_sanity_on_gpu(torch_gpu, orc):
    """Central FD (h = 1e-3 in theta) of the GPU rollout itself; FP32 rollouts
    make FD noisy, so this is a loose check (2e-2) of the analytic gradient."""
    torch = torch_gpu
    from paper_2503_00868_amd.fluidsim import Sim
    from paper_2503_00868_amd.autograd import mse_loss, rollout
    banner("gradient FD sanity 24^3")
    n, steps = 24, 4
    cell, ug = case(n, 101, 2.0)
    sim = Sim(cell, precond="mic0", tol=1e-8, diff_tol=1e-8, max_steps=steps, checkpoint_every=2)
    ugen = sim.to_faces(ug)
    target = tuple(t.clone() for t in rollout(torch.tensor(math.log(3e-3)), torch.tensor(0.1),
                                              ugen, sim, steps, DT))

    def J(tn, ts):
        u = rollout(torch.tensor(tn, dtype=torch.float64), torch.tensor(ts, dtype=torch.float64),
                    ugen, sim, steps, DT)
        return mse_loss(sim, u, target).item()

    tn0, ts0 = math.log(1.5e-3), -0.2
    th_nu = torch.tensor(tn0, dtype=torch.float64, requires_grad=True)
    th_s = torch.tensor(ts0, dtype=torch.float64, requires_grad=True)
    mse_loss(sim, rollout(th_nu, th_s, ugen, sim, steps, DT), target).backward()
    h = 1e-3
    fd_nu = (J(tn0 + h, ts0) - J(tn0 - h, ts0)) / (2 * h)
    fd_s = (J(tn0, ts0 + h) - J(tn0, ts0 - h)) / (2 * h)
    assert abs(fd_nu - th_nu.grad.item()) <= 2e-2 * abs(fd_nu), (fd_nu, th_nu.grad.item())
    assert abs(fd_s - th_s.grad.item()) <= 2e-2 * abs(fd_s), (fd_s, th_s.grad.item())


# (n, velocity scale): the benchmark's kind of flow on a small grid; a grid
# whose rows are one wave long (y and z faces), where neighbouring lanes'
# scatter targets line up and are merged; and departure points many cells
# away, clamped at the walls, where many lanes share one base node.
@pytest.mark.parametrize("n,scale", [(20, 4.0), (64, 4.0), (33, 60.0)])
def test_advect_adjoint_parity(torch_gpu, orc, n, scale):
    banner(f"advect adjoint {n}^3, velocity x{scale}")
    from paper_2503_00868_amd.fluidsim import Sim
    cell, u = case(n, 102, scale)
    u = orc.mask_faces(cell, u)
    rng = np.random.default_rng(3)
    lam = orc.mask_faces(cell, tuple(rng.standard_normal(orc.face_shape(n, c)) for c in range(3)))
    lam = tuple(np.asarray(l, np.float32).astype(np.float64) for l in lam)
    sim = Sim(cell)
    sim.set_params(nu=1e-3, dt=DT)
    g = to_np(sim.op_advect_adjoint(sim.to_faces(u), sim.to_faces(lam)))
    ref = orc.advect_adjoint(cell, u, DT, lam)
    l2, mx = rel_err(g, ref)
    assert l2 < 1e-5 and mx < 1e-4, (l2, mx)


def test_backward_requires_recording(torch_gpu, orc):
    from paper_2503_00868_amd.fluidsim import Sim, FluidSimError, SIM_ERR_STATE
    n = 8
    cell = inputs.gen_mask(n, 0)
    sim = Sim(cell, max_steps=2)
    sim.set_params(nu=1e-3, dt=DT)
    with pytest.raises(FluidSimError) as e:
        sim.backward(sim.faces())
    assert e.value.code == SIM_ERR_STATE


@pytest.mark.parametrize("n,warm", [(16, False), (16, True), (32, True)])
def test_learned_gradient_matches_oracle(torch_gpu, orc, n, warm):
    """The benchmark's preconditioner in both directions: the forward and the
    adjoint projections run flexible CG with the committed network (its
    Jacobi-PCG restart included), to 1e-9.  The gradient must still be the
    oracle's exact discrete one to 1e-4, since every solve meets the same
    residual test whatever the preconditioner."""
    torch = torch_gpu
    from paper_2503_00868_amd import unet as net_weights
    from paper_2503_00868_amd.autograd import mse_loss, rollout
    from paper_2503_00868_amd.fluidsim import Sim
    from paper_2503_00868_amd.train import DEFAULT_WEIGHTS
    banner(f"gradient {n}^3 learned preconditioner warm={warm}")
    steps, K, nu_t, nu_e, s_t, s_e = 5, 2, 4e-3, 2e-3, 1.2, 0.8
    cell, ug = case(n, 100, 2.0)
    target = orc.rollout(cell, ug, nu_t, s_t, steps, DT, mode="explicit", tol=1e-12)[-1]
    ref = orc.rollout_grad(cell, ug, nu_e, s_e, steps, DT, target, mode="explicit", tol=1e-12)
    sim = Sim(cell, precond="learned", diffusion="explicit", tol=1e-9, check_every=4,
              max_steps=steps, checkpoint_every=K, warm_start=warm)
    sim.net_set_weights(net_weights.load_weights(DEFAULT_WEIGHTS, device="cuda"))
    th_nu = torch.tensor(math.log(nu_e), dtype=torch.float64, requires_grad=True)
    th_s = torch.tensor(math.log(s_e), dtype=torch.float64, requires_grad=True)
    ugen = tuple(t.requires_grad_(True) for t in sim.to_faces(ug))
    uT = rollout(th_nu, th_s, ugen, sim, steps, DT)
    J = mse_loss(sim, uT, sim.to_faces(target))
    J.backward()
    banner(f"  J {J.item():.6e} vs {ref['J']:.6e}; dth_nu {th_nu.grad.item():.6e} vs "
           f"{ref['dtheta_nu']:.6e}; dth_s {th_s.grad.item():.6e} vs {ref['dtheta_s']:.6e}")
    assert abs(J.item() - ref["J"]) <= 1e-4 * ref["J"]
    for got, want, name in ((th_nu.grad.item(), ref["dtheta_nu"], "nu"),
                            (th_s.grad.item(), ref["dtheta_s"], "s")):
        assert abs(got - want) <= 1e-4 * abs(want), (name, got, want)
    l2, mx = rel_err(to_np(tuple(t.grad for t in ugen)), ref["du_gen"])
    assert l2 <= 1e-4, (l2, mx)
