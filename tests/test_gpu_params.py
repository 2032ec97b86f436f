"""GPU parity of the rollout's gradients in dt and gravity (Section 3.4.2:
every simulation parameter of Eq. (optLoss) is fitted), of the paper's
upwind convection surrogate as the rollout's convection gradient (Section
3.4.1), and of the parameter normalisation (exponential and sigmoid maps)
around the rollout; plus the guards against a stale recording."""
import math

import numpy as np
import pytest

from tests.gpu_util import banner, case, rel_err, to_np

pytestmark = pytest.mark.gpu

DT = 1.0 / 120
G0 = (0.6, -9.8, -1.1)


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    assert torch.cuda.is_available()
    return torch


def _run(torch, sim, ug, nu, s, dt, g, steps, target):
    from paper_2503_00868_amd.autograd import mse_loss, rollout
    th_nu = torch.tensor(math.log(nu), dtype=torch.float64, requires_grad=True)
    th_s = torch.tensor(math.log(s), dtype=torch.float64, requires_grad=True)
    dt_t = torch.tensor(dt, dtype=torch.float64, requires_grad=True)
    g_t = torch.tensor(g, dtype=torch.float64, requires_grad=True)
    ugen = tuple(t.requires_grad_(True) for t in sim.to_faces(ug))
    J = mse_loss(sim, rollout(th_nu, th_s, ugen, sim, steps, dt_t, g_t), sim.to_faces(target))
    J.backward()
    return {"J": J.item(), "dtheta_nu": th_nu.grad.item(), "dtheta_s": th_s.grad.item(),
            "ddt": dt_t.grad.item(), "dg": g_t.grad.numpy().copy(),
            "du_gen": to_np(tuple(t.grad for t in ugen))}


def _compare(got, ref, tol=1e-4):
    assert abs(got["J"] - ref["J"]) <= tol * ref["J"]
    for key in ("dtheta_nu", "dtheta_s", "ddt"):
        assert abs(got[key] - ref[key]) <= tol * abs(ref[key]), (key, got[key], ref[key])
    scale = np.abs(ref["dg"]).max()
    assert np.abs(got["dg"] - ref["dg"]).max() <= tol * scale, (got["dg"], ref["dg"])
    l2, mx = rel_err(got["du_gen"], ref["du_gen"])
    assert l2 <= tol, (l2, mx)


@pytest.mark.parametrize("mode,conv", [("explicit", "exact"), ("implicit", "exact"),
                                       ("explicit", "upwind"), ("implicit", "upwind")])
def test_parameter_gradients_match_oracle(torch_gpu, orc, mode, conv):
    """dJ/dnu, ds, ddt, dg and du_gen of a 5-step 16^3 rollout against the
    FP64 oracle (solves at 1e-12 there, 1e-9 here), for the exact transpose
    of the advection and for the paper's upwind surrogate."""
    torch = torch_gpu
    from paper_2503_00868_amd.fluidsim import Sim
    banner(f"parameter gradients 16^3 {mode} convection={conv}")
    n, steps, K = 16, 5, 2
    nu_t, nu_e = (4e-3, 2e-3) if mode == "explicit" else (8e-2, 5e-2)
    cell, ug = case(n, 100, 2.0)
    target = orc.rollout(cell, ug, nu_t, 1.2, steps, DT, g=(0.0, -9.8, 0.0), mode=mode,
                         tol=1e-12)[-1]
    ref = orc.rollout_grad(cell, ug, nu_e, 0.8, steps, DT, target, g=G0, mode=mode, tol=1e-12,
                           convection=conv)
    sim = Sim(cell, precond="mic0", diffusion=mode, tol=1e-9, diff_tol=1e-9, max_steps=steps,
              checkpoint_every=K, convection_grad=conv)
    got = _run(torch, sim, ug, nu_e, 0.8, DT, G0, steps, target)
    banner(f"  ddt {got['ddt']:.6e} vs {ref['ddt']:.6e}; dg {got['dg']} vs {ref['dg']}")
    _compare(got, ref)


def test_normalised_parameters(torch_gpu, orc):
    """The paper's normalisation around the rollout: dt = (1/120) exp(theta_dt)
    and g_y = -20 sigmoid(theta_gy) through params.PhysParam; the gradients in
    theta are the oracle's physical ones times the maps' derivatives."""
    torch = torch_gpu
    from paper_2503_00868_amd.autograd import mse_loss, rollout_params
    from paper_2503_00868_amd.fluidsim import Sim
    from paper_2503_00868_amd.params import PhysParam
    banner("normalised dt and gravity 16^3")
    n, steps = 16, 4
    cell, ug = case(n, 101, 2.0)
    maps = {"dt": PhysParam("dt", "exp", scale=1 / 120), "g_y": PhysParam("g_y", "sigmoid", lo=-20.0,
                                                                          hi=0.0)}
    dt, gy = 1 / 100, -9.0
    theta = {k: torch.tensor(maps[k].theta(v), dtype=torch.float64, requires_grad=True)
             for k, v in (("dt", dt), ("g_y", gy))}
    base = {"nu": 2e-3, "s": 0.9, "g_x": 0.0, "g_z": 0.0}
    target = orc.rollout(cell, ug, 3e-3, 1.1, steps, DT, mode="explicit", tol=1e-12)[-1]
    ref = orc.rollout_grad(cell, ug, 2e-3, 0.9, steps, dt, target, g=(0.0, gy, 0.0),
                           mode="explicit", tol=1e-12)
    sim = Sim(cell, precond="jacobi", diffusion="explicit", tol=1e-9, max_steps=steps,
              checkpoint_every=2)
    ugen = sim.to_faces(ug)
    J = mse_loss(sim, rollout_params(theta, maps, ugen, sim, steps, base), sim.to_faces(target))
    J.backward()
    want_dt = dt * ref["ddt"]
    # g_y = lo + (hi - lo) sigmoid = -20 + 20 sigmoid: d g_y / d theta = 20 s (1 - s)
    sig = 1.0 / (1.0 + math.exp(-float(theta["g_y"].detach())))
    want_gy = 20.0 * sig * (1.0 - sig) * ref["dg"][1]
    assert abs(theta["dt"].grad.item() - want_dt) <= 1e-4 * abs(want_dt)
    assert abs(theta["g_y"].grad.item() - want_gy) <= 1e-4 * abs(want_gy)


def test_stale_recording_is_refused(torch_gpu):
    """Two rollouts on one Sim before the first one's backward, or a
    set_params in between, leave the first rollout without its recording:
    the autograd Function raises, and the library reports SIM_ERR_STATE."""
    torch = torch_gpu
    from paper_2503_00868_amd.autograd import mse_loss, rollout
    from paper_2503_00868_amd.fluidsim import SIM_ERR_STATE, FluidSimError, Sim
    n, steps = 12, 2
    cell, ug = case(n, 5, 1.0)
    sim = Sim(cell, precond="jacobi", max_steps=steps, checkpoint_every=1)
    ugen = sim.to_faces(ug)
    th = [torch.tensor(v, dtype=torch.float64, requires_grad=True) for v in (-6.0, 0.0, -5.0, 0.1)]
    J1 = mse_loss(sim, rollout(th[0], th[1], ugen, sim, steps, DT), sim.faces())
    J2 = mse_loss(sim, rollout(th[2], th[3], ugen, sim, steps, DT), sim.faces())
    with pytest.raises(RuntimeError, match="recording is gone"):
        J1.backward()
    J2.backward()  # the current recording still differentiates
    assert th[2].grad is not None
    # set_params after a recorded rollout: the library forgets it
    sim.set_params(nu=1e-3, dt=DT)
    u = sim.faces()
    sim.init_state(ugen, u)
    sim.step(u, steps, record=True)
    sim.set_params(nu=2e-3, dt=DT)
    with pytest.raises(FluidSimError) as e:
        sim.backward(sim.faces())
    assert e.value.code == SIM_ERR_STATE
