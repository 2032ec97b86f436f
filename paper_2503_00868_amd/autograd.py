"""torch.autograd.Function over a recorded rollout of the HIP step.

Forward: u0 = s * mask(ugen), then `steps` steps recorded by the library.
Backward: the library's checkpointed reverse pass (the exact discrete
adjoint, or the paper's upwind convection surrogate when the context was
created with convection_grad="upwind").  The fitted parameters enter through
the normalisation of Section 3.4.2: nu = exp(theta_nu), s = exp(theta_s), so
dJ/dtheta = param * dJ/dparam; dt and gravity may be plain numbers or torch
tensors that depend on free variables through any map (for example
params.PhysParam: exponential for dt, sigmoid onto a range for gravity), and
then receive dJ/ddt and dJ/dg.
"""
from __future__ import annotations

import math

import torch


def _as_f64(x, shape):
    t = x.detach() if torch.is_tensor(x) else torch.tensor(x, dtype=torch.float64)
    t = t.to("cpu", torch.float64).reshape(shape)
    return t


class FluidRollout(torch.autograd.Function):
    @staticmethod
    def forward(ctx, theta_nu, theta_s, dt, gravity, ugen_u, ugen_v, ugen_w, sim, steps):
        nu = math.exp(float(theta_nu))
        s = math.exp(float(theta_s))
        dt_v = float(dt)
        g_v = tuple(float(x) for x in gravity.reshape(3))
        sim.set_params(nu=nu, dt=dt_v, s=s, gravity=g_v)
        ugen = tuple(t.contiguous() for t in (ugen_u, ugen_v, ugen_w))
        u = sim.faces()
        sim.init_state(ugen, u)
        ctx.stats = sim.step(u, steps, record=True)
        ctx.sim, ctx.nu, ctx.s, ctx.gen = sim, nu, s, sim.record_gen
        ctx.save_for_backward(theta_nu, theta_s, dt, gravity, *ugen)
        return u

    @staticmethod
    def backward(ctx, gu, gv, gw):
        theta_nu, theta_s, dt, gravity, ug_u, ug_v, ug_w = ctx.saved_tensors
        sim = ctx.sim
        if sim.record_gen != ctx.gen:
            raise RuntimeError(
                "FluidRollout.backward: the Sim has recorded another rollout or had its "
                "parameters set since this rollout ran; its recording is gone.  Give each "
                "rollout whose gradient is needed its own Sim, or call backward before the next "
                "rollout.")
        g = tuple(torch.zeros_like(ref) if t is None else t.contiguous()
                  for t, ref in zip((gu, gv, gw), (ug_u, ug_v, ug_w)))
        out, gr, _ = sim.backward(g, ugen=(ug_u, ug_v, ug_w), full=True)
        return (theta_nu.new_tensor(ctx.nu * gr["nu"]), theta_s.new_tensor(ctx.s * gr["s"]),
                dt.new_tensor(gr["dt"]), gravity.new_tensor(gr["gravity"]).reshape(gravity.shape),
                out[0], out[1], out[2], None, None)


def rollout(theta_nu, theta_s, ugen, sim, steps, dt, gravity=(0.0, -9.8, 0.0)):
    """u_T of a recorded rollout; differentiable in theta_nu, theta_s, ugen,
    and in dt and gravity when they are tensors that require grad."""
    dt_t = dt if torch.is_tensor(dt) else _as_f64(dt, ())
    g_t = gravity if torch.is_tensor(gravity) else _as_f64(list(gravity), (3,))
    return FluidRollout.apply(theta_nu, theta_s, dt_t, g_t, ugen[0], ugen[1], ugen[2], sim, steps)


def rollout_params(theta, maps, ugen, sim, steps, base):
    """A rollout whose parameters come from free variables through the
    paper's normalisation (Section 3.4.2).  theta: dict name -> tensor, maps:
    dict name -> params.PhysParam, for names among "nu", "s", "dt", "g_x",
    "g_y", "g_z"; base: the fixed values of the others (same names).  nu and s
    use the exponential map with scale 1 inside FluidRollout, so a scale other
    than 1 is folded into theta_nu/theta_s."""
    def val(name):
        if name in theta:
            return maps[name].value(theta[name])
        return torch.tensor(float(base[name]), dtype=torch.float64)
    tnu = torch.log(val("nu"))
    ts = torch.log(val("s"))
    dt = val("dt")
    g = torch.stack([val("g_x"), val("g_y"), val("g_z")])
    return rollout(tnu, ts, ugen, sim, steps, dt, g)


def mse_loss(sim, u, target):
    """Mean squared error over active faces (L2 term of Eq. (optLoss)),
    computed by the library; differentiable in u."""
    return _MSE.apply(sim, u[0], u[1], u[2], target[0], target[1], target[2])


class _MSE(torch.autograd.Function):
    @staticmethod
    def forward(ctx, sim, u0, u1, u2, t0, t1, t2):
        J, g = sim.loss_mse((u0, u1, u2), (t0, t1, t2), want_grad=True)
        ctx.g = g
        return u0.new_tensor(J, dtype=torch.float64)

    @staticmethod
    def backward(ctx, gJ):
        s = gJ.to(torch.float32)
        return (None, ctx.g[0] * s, ctx.g[1] * s, ctx.g[2] * s, None, None, None)


class PercnnSolve(torch.autograd.Function):
    """K layers of the recurrent convolutional pressure solver (Section
    3.4.1; sim_percnn_forward) with its reverse pass (sim_percnn_backward):
    gradients flow to the 28 weights (W_0 .. W_26, w_b; a float64 tensor on
    any device), to the starting pressure p0 and to the right-hand side b."""

    @staticmethod
    def forward(ctx, w, p0, b, sim, K):
        n = sim.n
        wn = w.detach().to("cpu", torch.float64).numpy()
        hist = torch.empty((K + 1, n, n, n), dtype=torch.float32, device=p0.device)
        p0c, bc = p0.contiguous(), b.contiguous()
        sim.percnn_forward(wn, K, p0c, bc, hist=hist)
        ctx.sim, ctx.K, ctx.wn = sim, K, wn
        ctx.save_for_backward(w, bc, hist)
        return hist[K].clone()

    @staticmethod
    def backward(ctx, g):
        w, b, hist = ctx.saved_tensors
        sim = ctx.sim
        gp0, gb = torch.empty_like(b), torch.empty_like(b)
        gw = sim.percnn_backward(ctx.wn, ctx.K, b, hist, g.contiguous(), gp0=gp0, gb=gb)
        return torch.as_tensor(gw, dtype=w.dtype, device=w.device), gp0, gb, None, None


def percnn_solve(w, p0, b, sim, K):
    """p_K of K recurrent layers, differentiable in (w, p0, b)."""
    return PercnnSolve.apply(w, p0, b, sim, K)
