"""GPU parity of the constrained divergence projection (sim_constrained_project)
against its FP64 oracle: iterations at 32^3 and 40^3 with and without the
relaxation parameter, the relative divergence it reports, convergence to the
library's own projection, and one iteration at 256^3 over every face."""
import numpy as np
import pytest

from oracle import constrained as orc_cp
from oracle import fluid
from paper_2503_00868_amd import inputs
from tests.gpu_util import banner, f32, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    assert torch.cuda.is_available()
    return torch


def _case(n, seed):
    cell, ug = inputs.gen_case(n, seed)
    rng = np.random.default_rng(seed)
    f = f32(tuple(np.asarray(g, np.float64) + 0.3 * rng.standard_normal(np.shape(g)) for g in ug))
    return cell, f


def _sim(cell):
    from paper_2503_00868_amd.fluidsim import Sim
    return Sim(cell, precond="jacobi", tol=1e-9)


def _rel_max(a, b):
    return max(float(np.abs(x - y).max()) for x, y in zip(a, b)) / max(float(np.abs(y).max()) for y in b)


@pytest.mark.parametrize("n,seed,relax", [(32, 0, False), (32, 1, True), (40, 2, False)])
def test_iterations_match_oracle(torch_gpu, n, seed, relax):
    K = 20
    banner(f"constrained projection n={n} K={K} relax={relax}")
    cell, f = _case(n, seed)
    eps = 0.5 * float(orc_cp.gradient_norms(cell).max()) if relax else 0.0
    sim = _sim(cell)
    U = sim.to_faces(f)
    rel = sim.constrained_project(U, K, eps)
    ref, _ = orc_cp.project(cell, fluid.mask_faces(cell, f), K, eps)
    err = _rel_max(to_np(U), ref)
    b0 = fluid.divergence_rhs(cell, fluid.mask_faces(cell, f))
    bK = fluid.divergence_rhs(cell, ref)
    rel_ref = np.linalg.norm(bK) / np.linalg.norm(b0)
    banner(f"  max rel err {err:.2e}; rel divergence {rel:.4e} (oracle {rel_ref:.4e})")
    assert err < 1e-5, err
    assert abs(rel - rel_ref) <= 1e-4 * rel_ref + 1e-7


def test_converges_to_the_projection(torch_gpu):
    n = 16
    banner(f"constrained projection -> sim_project, n={n}")
    cell, f = _case(n, 3)
    sim = _sim(cell)
    U = sim.to_faces(f)
    rel = sim.constrained_project(U, 3000)
    P = sim.to_faces(f)
    sim.project(P)
    err = _rel_max(to_np(U), to_np(P))
    banner(f"  rel divergence left {rel:.2e}; max rel difference to the projection {err:.2e}")
    assert rel < 1e-5 and err < 1e-4, (rel, err)
    # iters = 0 only masks the field to the active faces
    U0 = sim.to_faces(f)
    assert sim.constrained_project(U0, 0) == 1.0
    for a, b in zip(to_np(U0), fluid.mask_faces(cell, f)):
        assert np.array_equal(a, b)


def test_full_size_iteration(torch_gpu):
    n = 256
    banner(f"constrained projection, one iteration at n={n}")
    cell, f = _case(n, 4)
    sim = _sim(cell)
    U = sim.to_faces(f)
    sim.constrained_project(U, 1)
    ref = orc_cp.iterate(cell, fluid.mask_faces(cell, f), 0.0)
    err = _rel_max(to_np(U), ref)
    banner(f"  max rel err {err:.2e}")
    assert err < 1e-5, err
