"""GPU parity of the learned preconditioner: the U-Net forward pass and its
weight gradient (MFMA bf16 kernels through the C ABI) against the fp64 oracle
with bf16 emulation, the Adam step against its closed form, and flexible CG
with the network inside (including the Jacobi-PCG fallback).

Tolerances: bf16 has 8 mantissa bits (relative step 2^-8 = 3.9e-3); the
oracle rounds at the same points, so the two differ only where fp32 and fp64
accumulation round an activation to different bf16 neighbours.  The forward
output is compared at 1e-2 relative L2; gradients, whose intermediate
tensors the GPU also stores in bf16, at 3e-2 relative L2 and a cosine above
0.999.
"""
import numpy as np
import pytest

from oracle import unet as oracle_unet
from paper_2503_00868_amd import inputs
from paper_2503_00868_amd import unet as net_weights
from tests.gpu_util import banner, case, f32, rel_err, to_np

pytestmark = pytest.mark.gpu
DT = 1.0 / 120


@pytest.fixture(scope="module")
def torch_gpu():
    import torch
    assert torch.cuda.is_available()
    return torch


def _sim(cell, **kw):
    from paper_2503_00868_amd.fluidsim import Sim
    return Sim(cell, precond="learned", **kw)


def test_param_count_matches_oracle():
    assert net_weights.param_count() == oracle_unet.param_count()


@pytest.mark.parametrize("n,seed", [(16, 0), (20, 1), (32, 2), (40, 3)])
def test_net_forward_parity(torch_gpu, n, seed):
    torch = torch_gpu
    banner(f"unet forward n={n}")
    cell = inputs.gen_mask(n, seed)
    mask = cell == 1
    rng = np.random.default_rng(seed)
    r = np.where(mask, rng.standard_normal((n, n, n)), 0.0).astype(np.float32)
    w = net_weights.init_weights(seed)
    sim = _sim(cell)
    sim.net_set_weights(torch.as_tensor(w, device="cuda"))
    z = sim.net_forward(sim.cells_tensor(r)).cpu().numpy().astype(np.float64)
    zr = oracle_unet.forward(w, r.astype(np.float64), mask, emulate_bf16=True)
    err = np.linalg.norm(z - zr) / np.linalg.norm(zr)
    assert err < 1e-2, err
    assert np.all(z[~mask] == 0)
    # positive homogeneity survives the bf16 pipeline up to rounding
    z2 = sim.net_forward(sim.cells_tensor(4.0 * r)).cpu().numpy()
    assert np.linalg.norm(z2 - 4.0 * z) / np.linalg.norm(4.0 * z) < 1e-5


def _local_max(a):
    """Max of |a| over each cell's 3x3x3 neighbourhood (zero outside)."""
    from scipy import ndimage
    return ndimage.maximum_filter(np.abs(a), size=3, mode="constant")


@pytest.mark.parametrize("n,window,weights", [(40, None, "random"), (40, None, "trained"),
                                              (96, (40, 0, 80), "trained"),
                                              (96, (100, 30, 100), "random")])
def test_net_forward_elementwise(torch_gpu, n, window, weights):
    """Every element of z against the oracle's network (BF16 rounding at the
    same points), on a mask of the generator (n = 40) or on 96^3 windows cut
    from the benchmark's 256^3 mask, random and trained weights.  The two
    sides differ by accumulation order, which can move a BF16 activation by
    one step (2^-8 relative) and spreads through the later layers' 3x3x3
    neighbourhoods, and by the decoder's coarse-grid halves (their summed
    weights are rounded to BF16 once, their partial sums held in FP16).  The
    bound is therefore 2^-8 times the local magnitude: per element,
    |z - z_ref| <= 8 * 2^-8 * (max |z_ref| over its 3x3x3 neighbourhood
    + rms(z_ref))."""
    torch = torch_gpu
    from paper_2503_00868_amd.train import DEFAULT_WEIGHTS
    banner(f"unet forward element-wise n={n} window={window} weights={weights}")
    if window is None:
        cell = inputs.gen_mask(n, 3)
    else:
        z0, y0, x0 = window
        cell = np.ascontiguousarray(inputs.gen_mask(256, 4)[z0:z0 + n, y0:y0 + n, x0:x0 + n])
    mask = cell == inputs.LIQUID
    rng = np.random.default_rng(n + 11)
    r = np.where(mask, rng.standard_normal((n, n, n)), 0.0).astype(np.float32)
    w = (net_weights.init_weights(7) if weights == "random"
         else net_weights.load_weights(DEFAULT_WEIGHTS))
    sim = _sim(cell)
    sim.net_set_weights(torch.as_tensor(np.asarray(w), device="cuda"))
    z = sim.net_forward(sim.cells_tensor(r)).cpu().numpy().astype(np.float64)
    zr = oracle_unet.forward(np.asarray(w), r.astype(np.float64), mask, emulate_bf16=True)
    err = np.abs(z - zr)
    rms = float(np.sqrt((zr[mask] ** 2).mean()))
    ratio = err / (2.0 ** -8 * (_local_max(zr) + rms))
    q = np.quantile(ratio[mask], [0.5, 0.99, 0.9999])
    banner(f"  max |dz| / max |z_ref| {err.max() / np.abs(zr).max():.2e}; bound ratio median "
           f"{q[0]:.3f}, 99% {q[1]:.3f}, 99.99% {q[2]:.3f}, max {ratio.max():.3f}")
    assert np.all(z[~mask] == 0)
    assert ratio.max() <= 8.0


def test_net_zero_input(torch_gpu):
    torch = torch_gpu
    n = 16
    cell = inputs.gen_mask(n, 0)
    sim = _sim(cell)
    sim.net_set_weights(torch.as_tensor(net_weights.init_weights(1), device="cuda"))
    z = sim.net_forward(sim.cells_tensor(np.zeros((n, n, n), np.float32)))
    assert float(z.abs().max()) == 0.0


def _ball_mask(n, centre, radius):
    """Air everywhere but one liquid ball: most tiles lie far from liquid."""
    zz, yy, xx = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
    d2 = (xx - centre[0]) ** 2 + (yy - centre[1]) ** 2 + (zz - centre[2]) ** 2
    return np.where(d2 <= radius * radius, inputs.LIQUID, inputs.AIR).astype(np.uint8)


@pytest.mark.parametrize("n,which", [(128, "ball"), (128, "seed4"), (96, "ball"), (64, "seed4")])
def test_tile_skip_is_bitwise_dense(torch_gpu, n, which):
    """The inference pass skips, per layer, the tiles beyond the smaller of
    two distances to liquid: where the layer's activations must be zero, and
    where they can still reach the liquid-masked output.  Its output must be
    bitwise the dense pass's, for random and for the trained weights, and
    for an FCG projection the iteration count and the pressure must agree
    bitwise."""
    torch = torch_gpu
    from paper_2503_00868_amd.train import DEFAULT_WEIGHTS
    banner(f"tile skipping vs dense, n={n} {which}")
    cell = _ball_mask(n, (n // 5, n // 4, n // 3), n // 10) if which == "ball" else inputs.gen_mask(n, 4)
    mask = cell == inputs.LIQUID
    rng = np.random.default_rng(n)
    r = np.where(mask, rng.standard_normal((n, n, n)), 0.0).astype(np.float32)
    sim = _sim(cell)
    for w in (torch.as_tensor(net_weights.init_weights(3), device="cuda"),
              net_weights.load_weights(DEFAULT_WEIGHTS, device="cuda")):
        sim.net_set_weights(w)
        out = []
        for on in (True, False, True):
            sim.net_set_tile_skip(on)
            out.append(sim.net_forward(sim.cells_tensor(r)).cpu().numpy())
        assert np.abs(out[0]).max() > 0
        assert np.array_equal(out[0], out[1]) and np.array_equal(out[0], out[2])
    if which == "seed4" and n == 64:
        _, ug = inputs.gen_case(n, 4)
        res = []
        for on in (True, False):
            sim.net_set_tile_skip(on)
            U = sim.to_faces(ug)
            st, p = sim.project(U, want_p=True)
            res.append((st["iters"], p.cpu().numpy(), to_np(U)))
        assert res[0][0] == res[1][0]
        assert np.array_equal(res[0][1], res[1][1])
        for a, b in zip(res[0][2], res[1][2]):
            assert np.array_equal(a, b)
    sim.net_set_tile_skip(True)


@pytest.mark.parametrize("n,batch", [(16, 1), (16, 2), (24, 1), (40, 1)])
def test_net_grad_parity(torch_gpu, orc, n, batch):
    torch = torch_gpu
    banner(f"unet grad n={n} batch={batch}")
    cell = inputs.gen_mask(n, 3)
    mask = cell == 1
    rng = np.random.default_rng(7)
    es, rs = [], []
    for _ in range(batch):
        e = np.where(mask, rng.standard_normal((n, n, n)), 0.0)
        es.append(e.astype(np.float32))
        rs.append(orc.poisson_apply(cell, e).astype(np.float32))
    w = net_weights.init_weights(5)
    sim = _sim(cell)
    sim.net_set_weights(torch.as_tensor(w, device="cuda"))
    R = torch.as_tensor(np.stack(rs), device="cuda")
    E = torch.as_tensor(np.stack(es), device="cuda")
    G = torch.zeros(w.size, dtype=torch.float32, device="cuda")
    loss = sim.net_grad(R, E, batch, G)
    A = lambda x: orc.poisson_apply(cell, x)
    ref_l, ref_g = 0.0, np.zeros(w.size)
    for b in range(batch):
        l, g, _ = oracle_unet.loss_and_grad(w, rs[b].astype(np.float64), es[b].astype(np.float64),
                                            mask, A)
        ref_l += l / batch
        ref_g += g / batch
    g = G.cpu().numpy().astype(np.float64)
    assert abs(loss - ref_l) < 1e-2 * abs(ref_l), (loss, ref_l)
    err = np.linalg.norm(g - ref_g) / np.linalg.norm(ref_g)
    cos = g @ ref_g / (np.linalg.norm(g) * np.linalg.norm(ref_g))
    banner(f"  loss {loss:.6f} vs {ref_l:.6f}; grad rel err {err:.2e} cos {cos:.6f}")
    assert err < 3e-2 and cos > 0.999, (err, cos)
    # per-layer: every convolution receives a gradient of the right size
    off = 0
    for cin, cout in net_weights.CONVS:
        m = 27 * cin * cout
        gl, rl = g[off:off + m], ref_g[off:off + m]
        assert np.linalg.norm(gl - rl) <= 0.1 * np.linalg.norm(rl) + 1e-12
        off += m


def test_adam_step_closed_form(torch_gpu, orc):
    torch = torch_gpu
    n = 16
    cell = inputs.gen_mask(n, 4)
    mask = cell == 1
    rng = np.random.default_rng(9)
    e = np.where(mask, rng.standard_normal((n, n, n)), 0.0).astype(np.float32)
    r = orc.poisson_apply(cell, e.astype(np.float64)).astype(np.float32)
    w = net_weights.init_weights(6)
    sim = _sim(cell)
    R = torch.as_tensor(r[None], device="cuda")
    E = torch.as_tensor(e[None], device="cuda")
    master = torch.as_tensor(w.copy(), device="cuda")
    sim.net_set_weights(master)
    G = torch.zeros(w.size, dtype=torch.float32, device="cuda")
    sim.net_grad(R, E, 1, G)
    adam = torch.zeros(2 * w.size, dtype=torch.float32, device="cuda")
    lr = 1e-3
    sim.net_train_step(R, E, 1, master, adam, 1, lr)
    g = G.cpu().numpy().astype(np.float64)
    # first Adam step: m_hat = g, v_hat = g^2 -> w - lr g / (|g| + eps)
    expect = w - lr * g / (np.abs(g) + 1e-8)
    np.testing.assert_allclose(master.cpu().numpy(), expect, rtol=0, atol=2e-6)


def test_fcg_with_untrained_net_falls_back_and_converges(torch_gpu, orc):
    """With random weights the flexible CG may stall; the Jacobi-PCG restart
    from its iterate must still deliver the 1e-6 projection."""
    torch = torch_gpu
    from paper_2503_00868_amd.fluidsim import SIM_OK, SIM_OK_FALLBACK
    banner("fcg fallback n=24")
    n = 24
    cell, u = case(n, 8)
    u = orc.add_force(cell, orc.mask_faces(cell, u), DT)
    sim = _sim(cell, learned_max_iter=6, check_every=2)
    sim.net_set_weights(torch.as_tensor(net_weights.init_weights(2), device="cuda"))
    U = sim.to_faces(u)
    st, _ = sim.project(U)
    assert st["rel_residual"] <= 1e-6
    assert st["status"] in (SIM_OK, SIM_OK_FALLBACK)
    ref, _, _, _ = orc.project(cell, u, 1e-12)
    l2, mx = rel_err(to_np(U), ref)
    assert mx < 1e-5, (l2, mx)


def test_learned_context_without_weights_uses_jacobi(torch_gpu, orc):
    n = 16
    cell, u = case(n, 9)
    u = orc.add_force(cell, orc.mask_faces(cell, u), DT)
    sim = _sim(cell)
    U = sim.to_faces(u)
    st, _ = sim.project(U)
    assert st["rel_residual"] <= 1e-6 and st["fallback_used"] == 0


def test_harvest_pairs_consistent(torch_gpu, orc):
    """r_0 = b, A e_k = r_k, and e_0 = x* (the exact solve) for harvested pairs."""
    from paper_2503_00868_amd.fluidsim import Sim
    banner("harvest n=24")
    n = 24
    cell, u = case(n, 10)
    u = orc.add_force(cell, orc.mask_faces(cell, u), DT)
    sim = Sim(cell)
    R, E, st = sim.harvest_pairs(sim.to_faces(u), [0, 4, 10], tol=1e-10, mode=0)
    R = R.cpu().numpy().astype(np.float64)
    E = E.cpu().numpy().astype(np.float64)
    b = orc.divergence_rhs(cell, u)
    np.testing.assert_allclose(R[0], b, rtol=0, atol=1e-6 * np.abs(b).max())
    for j in range(3):
        Ae = orc.poisson_apply(cell, E[j])
        assert np.linalg.norm(Ae - R[j]) <= 1e-4 * np.linalg.norm(R[j]), j
    x_ref, _, _ = orc.pcg(cell, b, orc.PRECOND_NONE, 1e-12)
    assert np.linalg.norm(E[0] - x_ref) <= 1e-6 * np.linalg.norm(x_ref)
    assert np.linalg.norm(R[2]) < np.linalg.norm(R[0])


def test_harvest_pairs_from_flexible_cg_consistent(torch_gpu, orc):
    """Mode 1 (iterates of the flexible CG with the network): A e_k = r_k with
    e_k formed in FP64 against the reference solution."""
    from paper_2503_00868_amd.fluidsim import Sim
    banner("harvest mode 1 n=24")
    n = 24
    cell, u = case(n, 11)
    u = orc.add_force(cell, orc.mask_faces(cell, u), DT)
    sim = Sim(cell, precond="learned")
    sim.net_set_weights(torch_gpu.as_tensor(net_weights.init_weights(4), device="cuda"))
    R, E, st = sim.harvest_pairs(sim.to_faces(u), [0, 1, 2, 5], tol=1e-10, mode=1)
    R = R.cpu().numpy().astype(np.float64)
    E = E.cpu().numpy().astype(np.float64)
    last = 4 if not st["fallback_used"] else 1
    for j in range(last):
        Ae = orc.poisson_apply(cell, E[j])
        assert np.linalg.norm(Ae - R[j]) <= 1e-4 * np.linalg.norm(R[j]), j
        assert float((R[j] * E[j]).sum()) > 0


@pytest.mark.parametrize("seed", [900, 901])
def test_trained_network_gain(torch_gpu, orc, seed):
    """What the trained network gains: on held-out volumes (seeds never used
    in training) the committed weights make the flexible CG converge to the
    1e-6 residual without the Jacobi-PCG fallback, in a fraction of Jacobi-PCG's
    iterations and fewer than MIC(0)-PCG's, while an untrained network of the
    same architecture falls back or needs far more iterations.  The fields
    still match the oracle's 1e-12 projection."""
    import os
    from paper_2503_00868_amd import train
    from paper_2503_00868_amd.fluidsim import Sim
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "paper_2503_00868_amd", "weights", "unet.safetensors")
    assert os.path.exists(path), "trained weights are part of the repository"
    n = 64
    banner(f"trained network gain n={n} seed={seed}")
    cell = inputs.gen_mask(n, seed)
    iters = {}
    for name, w in (("trained", net_weights.load_weights(path)), ("untrained", net_weights.init_weights(3))):
        sim = Sim(cell, precond="learned", check_every=2, learned_max_iter=200)
        sim.net_set_weights(torch_gpu.as_tensor(w, device="cuda"))
        u = train.pre_projection_field(sim, seed)
        u_in = to_np(u)
        st, _ = sim.project(u)
        iters[name] = (st["iters"], st["fallback_used"])
        assert st["rel_residual"] <= 1e-6
        if name == "trained":
            ref, _, _, _ = orc.project(cell, tuple(x.astype(np.float64) for x in u_in), 1e-12)
            l2, mx = rel_err(to_np(u), ref)
            assert mx < 1e-5, (l2, mx)
    for pc in ("jacobi", "mic0"):
        sim = Sim(cell, precond=pc, check_every=2)
        u = train.pre_projection_field(sim, seed)
        st, _ = sim.project(u)
        iters[pc] = (st["iters"], 0)
    banner(f"  iterations: {iters}")
    t_it, t_fb = iters["trained"]
    assert t_fb == 0
    assert t_it * 5 <= iters["jacobi"][0]
    assert t_it < iters["mic0"][0]
    u_it, u_fb = iters["untrained"]
    assert u_fb == 1 or u_it >= 2 * t_it


def test_fcg_early_stop_inside_a_block(torch_gpu, orc):
    """The flexible CG runs in blocks of four iterations with the FP64 check
    at each block's end; when the recursive residual meets the tolerance
    inside a block, the block's remaining iterations (and their network
    applications) are skipped, the iterate takes only the steps that ran and
    the check decides.  Solves then end at iteration counts that are not
    multiples of four, without the fallback, and the fields still match the
    oracle's 1e-12 projection."""
    import os
    from paper_2503_00868_amd import train
    from paper_2503_00868_amd.fluidsim import SIM_OK, Sim
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "paper_2503_00868_amd", "weights", "unet.safetensors")
    w = torch_gpu.as_tensor(net_weights.load_weights(path), device="cuda")
    n = 48
    counts = []
    for seed in (902, 903, 904, 905):
        banner(f"fcg early stop n={n} seed={seed}")
        cell = inputs.gen_mask(n, seed)
        sim = Sim(cell, precond="learned", check_every=4, learned_max_iter=200)
        sim.net_set_weights(w)
        u = train.pre_projection_field(sim, seed)
        u_in = to_np(u)
        st, _ = sim.project(u)
        counts.append(st["iters"])
        assert st["status"] == SIM_OK and st["fallback_used"] == 0, st
        assert st["rel_residual"] <= 1e-6, st
        ref, _, _, _ = orc.project(cell, tuple(x.astype(np.float64) for x in u_in), 1e-12)
        l2, mx = rel_err(to_np(u), ref)
        assert mx < 1e-5, (seed, l2, mx)
    banner(f"  iterations: {counts}")
    assert any(k % 4 != 0 for k in counts), counts
