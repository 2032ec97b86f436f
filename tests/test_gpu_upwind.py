"""GPU parity of the paper's upwind analytic convection gradient
(sim_op_convection_grad_upwind) against its FP64 oracle, and its comparison
with the exact advection adjoint and central differences (the surrogate is
measured, not expected to match them)."""
import numpy as np
import pytest

from oracle import fluid
from oracle import upwind as orc_up
from paper_2503_00868_amd import inputs
from tests.gpu_util import banner, f32, to_np

pytestmark = pytest.mark.gpu
DT = 1.0 / 120


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    assert torch.cuda.is_available()
    return torch


def _sim(cell):
    from paper_2503_00868_amd.fluidsim import Sim
    sim = Sim(cell, precond="jacobi")
    sim.set_params(nu=1e-3, dt=DT)
    return sim


@pytest.mark.parametrize("n,seed", [(24, 0), (33, 1)])
def test_matches_oracle(torch_gpu, n, seed):
    banner(f"upwind convection gradient n={n}")
    cell, ug = inputs.gen_case(n, seed)
    rng = np.random.default_rng(seed)
    v = f32(fluid.mask_faces(cell, tuple(np.asarray(g) + 0.2 * rng.standard_normal(np.shape(g)) for g in ug)))
    lam = f32(tuple(rng.standard_normal(fluid.face_shape(n, c)) for c in range(3)))
    sim = _sim(cell)
    g = to_np(sim.op_convection_grad_upwind(sim.to_faces(v), sim.to_faces(lam)))
    ref = orc_up.gradient(cell, v, lam, DT)
    err = max(float(np.abs(a - b).max()) for a, b in zip(g, ref)) / max(float(np.abs(b).max()) for b in ref)
    banner(f"  max rel err {err:.2e}")
    assert err < 1e-5, err


def test_against_exact_adjoint_and_central_differences(torch_gpu):
    """J(u) = <lam, advect(u)>: the exact adjoint reproduces the FP64
    oracle's central difference along a random direction; the surrogate is
    reported beside it (its cosine with the exact gradient, its directional
    derivative)."""
    n = 32
    banner(f"upwind surrogate vs exact adjoint, n={n}")
    cell, ug = inputs.gen_case(n, 4)
    u = f32(fluid.mask_faces(cell, ug))
    rng = np.random.default_rng(5)
    lam = f32(fluid.mask_faces(cell, tuple(rng.standard_normal(fluid.face_shape(n, c)) for c in range(3))))
    d = fluid.mask_faces(cell, tuple(rng.standard_normal(fluid.face_shape(n, c)) for c in range(3)))
    sim = _sim(cell)
    U = sim.to_faces(u)
    A = sim.op_advect(U)
    g_ex = to_np(sim.op_advect_adjoint(U, sim.to_faces(lam)))
    g_up = to_np(sim.op_convection_grad_upwind(A, sim.to_faces(lam)))
    J = lambda f: sum(float((l * a).sum()) for l, a in zip(lam, fluid.advect(cell, f, DT)))
    eps = 1e-6
    fd = (J(tuple(x + eps * y for x, y in zip(u, d))) - J(tuple(x - eps * y for x, y in zip(u, d)))) / (2 * eps)
    dd_ex = sum(float((a * b).sum()) for a, b in zip(g_ex, d))
    dd_up = sum(float((a * b).sum()) for a, b in zip(g_up, d))
    num = sum(float((a * b).sum()) for a, b in zip(g_ex, g_up))
    cos = num / np.sqrt(sum(float((a * a).sum()) for a in g_ex) * sum(float((b * b).sum()) for b in g_up))
    banner(f"  directional derivative: FD {fd:.6e}, exact adjoint {dd_ex:.6e}, upwind surrogate {dd_up:.6e}; "
           f"cosine(exact, surrogate) {cos:.4f}")
    assert abs(dd_ex - fd) <= 1e-4 * abs(fd)
    assert np.isfinite(dd_up) and cos > 0.5


def test_full_size_sampled(torch_gpu):
    """256^3, the benchmark's size and launch: non-active faces exactly 0;
    sampled active faces (random ones, and some on the first, second, middle
    and last planes and on a few fixed rows) against the oracle's face-by-face
    definition."""
    n = 256
    banner(f"upwind convection gradient n={n}, sampled faces")
    cell, ug = inputs.gen_case(n, 4)
    rng = np.random.default_rng(6)
    v = f32(fluid.mask_faces(cell, tuple(np.asarray(g) + 0.2 * rng.standard_normal(np.shape(g)) for g in ug)))
    lam = f32(tuple(rng.standard_normal(fluid.face_shape(n, c)) for c in range(3)))
    sim = _sim(cell)
    g = to_np(sim.op_convection_grad_upwind(sim.to_faces(v), sim.to_faces(lam)))
    v64 = [np.asarray(a, np.float64) for a in v]
    l64 = [np.asarray(a, np.float64) for a in lam]
    worst, scale = 0.0, 0.0
    for comp in range(3):
        act = fluid.face_classes(cell, comp) == fluid.ACTIVE
        assert not np.any(g[comp][~act]), comp
        shp = act.shape
        picks = [tuple(rng.integers(0, s) for s in shp) for _ in range(800)]
        for y in (7, 8, 15, 16, shp[1] - 1):
            for z in (0, 1, shp[0] // 2, shp[0] - 1):
                picks += [(z, y, int(x)) for x in rng.integers(0, shp[2], 4)]
        picks = [p for p in picks if act[p]]
        assert len(picks) > 250
        for p in picks:
            ref = orc_up.face_gradient(n, v64, l64, DT, comp, p)
            worst = max(worst, abs(float(g[comp][p]) - ref))
            scale = max(scale, abs(ref))
    banner(f"  max rel err {worst / scale:.2e}")
    assert worst <= 1e-5 * scale, (worst, scale)
