"""The allocation-free entry point sim_loss_mse_noalloc, called through the C
ABI, against sim_loss_mse (the context-based entry point it varies): two
calls in a row on one device, the second with a smaller grid, so the second
call reuses the library's fixed scratch array after a larger use."""
import numpy as np
import pytest

from paper_2503_00868_amd import inputs
from tests.gpu_util import banner

pytestmark = pytest.mark.gpu


def test_noalloc_loss_matches_context_loss():
    import torch
    from paper_2503_00868_amd import fluidsim as fsb
    from paper_2503_00868_amd.fluidsim import Sim
    assert torch.cuda.is_available()
    for n, seed in ((48, 3), (20, 5)):
        banner(f"allocation-free MSE loss n={n}")
        cell, ug = inputs.gen_case(n, seed)
        rng = np.random.default_rng(seed)
        sim = Sim(cell)
        u = sim.to_faces(ug)
        t = sim.to_faces(tuple(g + 0.1 * rng.standard_normal(g.shape) for g in ug))
        J_ref, g_ref = sim.loss_mse(u, t)
        d_cell = torch.as_tensor(np.ascontiguousarray(cell, np.uint8), device="cuda")
        d_loss = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
        g = sim.faces(fill=float("nan"))
        fsb.loss_mse_noalloc(n, d_cell, u, t, d_loss, g, stream=torch.cuda.current_stream())
        torch.cuda.synchronize()
        J = float(d_loss.item())
        banner(f"  J {J:.15e} vs {J_ref:.15e}")
        assert abs(J - J_ref) <= 1e-12 * abs(J_ref)
        for a, b in zip(g, g_ref):
            assert torch.equal(a, b)
        # without gradient outputs: J alone, the same value
        d_loss.fill_(float("nan"))
        fsb.loss_mse_noalloc(n, d_cell, u, t, d_loss, None, stream=torch.cuda.current_stream())
        torch.cuda.synchronize()
        assert abs(float(d_loss.item()) - J_ref) <= 1e-12 * abs(J_ref)
