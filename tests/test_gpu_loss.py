"""GPU parity of the paper's masked cosine + L2 velocity loss
(sim_loss_cos_l2) against its FP64 oracle: J and dJ/du at small sizes with a
ragged tail, the degenerate cases, and the full 256^3 grid."""
import numpy as np
import pytest

from oracle import fluid
from oracle import loss as orc_loss
from paper_2503_00868_amd import inputs
from tests.gpu_util import banner, f32, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    assert torch.cuda.is_available()
    return torch


def _sim(cell):
    from paper_2503_00868_amd.fluidsim import Sim
    return Sim(cell, precond="jacobi")


def _fields(n, rng):
    return f32(tuple(rng.standard_normal(fluid.face_shape(n, c)) for c in range(3)))


def _check(J, g, Jr, gr, what):
    eJ = abs(J - Jr) / max(abs(Jr), 1e-30)
    scale = max(float(np.abs(b).max()) for b in gr)
    eg = max(float(np.abs(a - b).max()) for a, b in zip(g, gr)) / scale
    banner(f"  {what}: J {J:.8e} (oracle {Jr:.8e}, rel err {eJ:.1e}); grad rel err {eg:.1e}")
    assert eJ <= 1e-5, eJ
    assert eg <= 1e-5, eg


@pytest.mark.parametrize("n,seed,eps,weights", [(24, 0, 0.0, (1.0, 1.0, 1.0)),
                                                (33, 1, 0.05, (0.5, 1.0, 2.0)),
                                                (33, 2, 0.0, (0.0, 0.0, 1.0))])
def test_matches_oracle(torch_gpu, n, seed, eps, weights):
    banner(f"masked cosine + L2 loss n={n} eps={eps} weights={weights}")
    cell, _ = inputs.gen_case(n, seed)
    rng = np.random.default_rng(seed)
    s, r = _fields(n, rng), _fields(n, rng)
    sim = _sim(cell)
    J, g = sim.loss_cos_l2(sim.to_faces(s), sim.to_faces(r), 0.8, 1.3, eps, weights)
    Jr, gr = orc_loss.loss(cell, s, r, 0.8, 1.3, eps, weights)
    _check(J, to_np(g), Jr, gr, "parity")
    # the value alone (no gradient outputs) is the same
    J2, _ = sim.loss_cos_l2(sim.to_faces(s), sim.to_faces(r), 0.8, 1.3, eps, weights, want_grad=False)
    assert J2 == J


def test_degenerate_cases(torch_gpu):
    """All weights 0: J = 0 and a zero gradient; identical fields: J and the
    gradient vanish (eps = 0); opposite fields with beta = 0: J = 2 alpha."""
    n = 20
    cell, _ = inputs.gen_case(n, 3)
    rng = np.random.default_rng(3)
    s = _fields(n, rng)
    sim = _sim(cell)
    S = sim.to_faces(s)
    J, g = sim.loss_cos_l2(S, sim.to_faces(_fields(n, rng)), 1.0, 1.0, 0.0, (0.0, 0.0, 0.0))
    assert J == 0.0 and all(not np.any(x) for x in to_np(g))
    J, g = sim.loss_cos_l2(S, sim.to_faces(s), 0.7, 1.3, 0.0, (1.0, 1.0, 1.0))
    assert abs(J) <= 1e-6 and max(float(np.abs(x).max()) for x in to_np(g)) <= 1e-6
    J, _ = sim.loss_cos_l2(S, sim.to_faces(tuple(-x for x in s)), 0.7, 0.0, 0.0, (1.0, 1.0, 1.0))
    assert abs(J - 1.4) <= 1e-6


def test_full_size(torch_gpu):
    """256^3: J and the whole gradient against the oracle."""
    n = 256
    banner(f"masked cosine + L2 loss n={n}")
    cell = inputs.gen_mask(n, 4)
    rng = np.random.default_rng(7)
    shapes = [fluid.face_shape(n, c) for c in range(3)]
    r = tuple(rng.standard_normal(sh, dtype=np.float32).astype(np.float64) for sh in shapes)
    s = tuple((a + 0.3 * rng.standard_normal(a.shape, dtype=np.float32)).astype(np.float32)
              .astype(np.float64) for a in r)
    sim = _sim(cell)
    J, g = sim.loss_cos_l2(sim.to_faces(s), sim.to_faces(r), 1.0, 1.0, 1e-3, (0.2, 1.0, 2.0))
    Jr, gr = orc_loss.loss(cell, s, r, 1.0, 1.0, 1e-3, (0.2, 1.0, 2.0))
    _check(J, to_np(g), Jr, gr, "256^3")
