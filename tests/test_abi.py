"""Host-side checks of the C ABI: the library loads, exports every entry
point the header declares, and rejects bad arguments before touching the
device (these run without a GPU)."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2503_00868_amd import fluidsim as fsb
from paper_2503_00868_amd import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    txt = open(os.path.join(ROOT, "include", "fluidsim.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(sim_[a-z0-9_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    L = fsb.lib()
    names = _declared_symbols()
    assert len(names) >= 20
    for name in names:
        assert hasattr(L, name), name
    assert set(names) == set(fsb.SIGNATURES)


def _desc(**kw):
    d = dict(n=16, precond="jacobi", diffusion="auto", tol=1e-6, diff_tol=1e-6, max_iter=100,
             check_every=8, checkpoint_every=4, max_steps=8, learned_max_iter=50)
    d.update(kw)
    return fsb.make_desc(**d)


def _ws_size(desc):
    out = ctypes.c_size_t()
    rc = fsb.lib().sim_workspace_size(ctypes.byref(desc), ctypes.byref(out))
    return rc, out.value


@pytest.mark.parametrize("bad", [dict(n=3), dict(n=2000), dict(precond=7), dict(diffusion=5),
                                 dict(max_iter=0), dict(check_every=0), dict(checkpoint_every=0),
                                 dict(max_steps=-1), dict(tol=0.0), dict(tol=1.5),
                                 dict(diff_tol=-1.0), dict(precond="learned", n=18),
                                 dict(precond="learned", learned_max_iter=0)])
def test_workspace_size_rejects_bad_desc(bad):
    rc, _ = _ws_size(_desc(**bad))
    assert rc == fsb.SIM_ERR_INVALID_ARG


def test_workspace_size_rejects_bad_warm_start():
    d = _desc()
    d.warm_start = 2
    assert _ws_size(d)[0] == fsb.SIM_ERR_INVALID_ARG
    d = _desc()
    d.store_pressures = 2
    assert _ws_size(d)[0] == fsb.SIM_ERR_INVALID_ARG
    # the pressure history belongs to a recorded rollout
    assert _ws_size(_desc(max_steps=0, store_pressures=True))[0] == fsb.SIM_ERR_INVALID_ARG


def test_workspace_size_pressure_history():
    n = 16
    _, rec = _ws_size(_desc(max_steps=8))
    _, hist = _ws_size(_desc(max_steps=8, store_pressures=True))
    assert hist - rec >= 8 * 8 * n ** 3


def test_workspace_size_grows_with_recording_and_precond():
    _, base = _ws_size(_desc(max_steps=0))
    _, rec = _ws_size(_desc(max_steps=16))
    _, mic = _ws_size(_desc(max_steps=0, precond="mic0"))
    _, learned = _ws_size(_desc(max_steps=0, precond="learned"))
    # Jacobi keeps two extra direction buffers, MIC(0) its factor and sweep
    # temporary (the same size); the network adds its activations
    assert rec > base and mic == base and learned > mic
    # warm start: four FP64 pressures (the forward's last three, for their
    # extrapolation, and the adjoint's last), plus the forward's three per
    # checkpoint (16 / 4 = 4) when recording
    n = 16
    _, warm = _ws_size(_desc(max_steps=0, warm_start=True))
    _, warm_rec = _ws_size(_desc(max_steps=16, warm_start=True))
    assert warm - base >= 4 * 8 * n ** 3
    assert warm_rec - rec >= (4 + 3 * 4) * 8 * n ** 3
    n = 16
    assert base > (3 * (n + 1) * n * n) * 4 * 7  # at least the face-domain buffers


def _create(desc, cell, ws_ptr=256, ws_bytes=None):
    if ws_bytes is None:
        ws_bytes = _ws_size(desc)[1]
    cell = np.ascontiguousarray(cell, dtype=np.uint8)
    ctx = ctypes.c_void_p()
    rc = fsb.lib().sim_create(ctypes.byref(desc), cell.ctypes.data_as(ctypes.c_void_p),
                              ctypes.c_void_p(ws_ptr), ws_bytes, None, ctypes.byref(ctx))
    return rc, ctx


def test_create_rejects_before_device_work():
    n = 16
    cell = inputs.gen_mask(n, 0)
    d = _desc()
    assert _create(d, cell, ws_bytes=10)[0] == fsb.SIM_ERR_WORKSPACE_TOO_SMALL
    assert _create(d, cell, ws_ptr=100)[0] == fsb.SIM_ERR_INVALID_ARG  # misaligned
    bad = cell.copy()
    bad[0, 0, 0] = 7
    assert _create(d, bad)[0] == fsb.SIM_ERR_INVALID_ARG


def test_create_detects_singular_mask():
    """A liquid region enclosed by solid (no air face) has a pure-Neumann
    pressure system."""
    n = 8
    cell = np.zeros((n, n, n), np.uint8)
    cell[:, :2, :] = 1  # a slab touching air: fine...
    cell[4:7, 4:7, 4:7] = 2
    cell[5, 5, 5] = 1                # ...but this cell is boxed in by solid
    assert _create(_desc(n=n), cell)[0] == fsb.SIM_ERR_SINGULAR_MASK
    full = np.ones((n, n, n), np.uint8)  # all liquid: no air anywhere
    assert _create(_desc(n=n), full)[0] == fsb.SIM_ERR_SINGULAR_MASK


def test_null_arguments():
    L = fsb.lib()
    assert L.sim_workspace_size(None, None) == fsb.SIM_ERR_INVALID_ARG
    assert L.sim_destroy(None) == fsb.SIM_ERR_INVALID_ARG
    assert L.sim_set_params(None, None) == fsb.SIM_ERR_INVALID_ARG
    assert L.sim_step(None, None, None, None, 1, 0, None) == fsb.SIM_ERR_INVALID_ARG
    assert L.sim_backward(None, *([None] * 9), None, None) == fsb.SIM_ERR_INVALID_ARG
    assert L.sim_percnn_forward(None, None, 1, None, None, None, None) == fsb.SIM_ERR_INVALID_ARG
    assert L.sim_percnn_backward(None, None, 1, *([None] * 6)) == fsb.SIM_ERR_INVALID_ARG
    assert L.sim_constrained_project(None, None, None, None, 1, 0.0, None) == fsb.SIM_ERR_INVALID_ARG
    assert L.sim_op_convection_grad_upwind(None, *([None] * 9)) == fsb.SIM_ERR_INVALID_ARG
    assert L.sim_loss_cos_l2(None, *([None] * 6), 1.0, 1.0, 0.0, None, None, None, None,
                             None) == fsb.SIM_ERR_INVALID_ARG
    assert L.sim_apic_p2g(None, 0, *([None] * 10)) == fsb.SIM_ERR_INVALID_ARG
    assert L.sim_apic_g2p(None, 0, None, None, None, 0.0, None, None, None) == fsb.SIM_ERR_INVALID_ARG
    assert fsb.lib().sim_last_error(None) == b"NULL context"


def test_net_param_count_matches_architecture():
    # 3x3x3 bias-free convs: 2->16, 16->16, 16->32, 32->32, 32->64, 64->64,
    # (64+32)->32, 32->32, (32+16)->16, 16->16, 16->1
    chans = [(2, 16), (16, 16), (16, 32), (32, 32), (32, 64), (64, 64), (96, 32), (32, 32),
             (48, 16), (16, 16), (16, 1)]
    assert fsb.net_param_count() == sum(27 * a * b for a, b in chans)


def test_workspace_size_rejects_bad_convection_grad():
    d = _desc()
    d.convection_grad = 2
    assert _ws_size(d)[0] == fsb.SIM_ERR_INVALID_ARG
    d.convection_grad = fsb.SIM_CONVGRAD_UPWIND
    assert _ws_size(d)[0] == fsb.SIM_OK


@pytest.mark.parametrize("n", [3, 1025, -1])
def test_noalloc_loss_rejects_sizes_beyond_its_limit(n):
    """The allocation-free loss validates on the host before any device
    work (so this runs without a GPU)."""
    L = fsb.lib()
    p = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    rc = L.sim_loss_mse_noalloc(n, p, p, p, p, p, p, p, p, None, None, None, None)
    assert rc == fsb.SIM_ERR_INVALID_ARG


def test_noalloc_loss_rejects_null_and_partial_gradients():
    L = fsb.lib()
    p = [ctypes.c_void_p(0x1000 + 0x100 * q) for q in range(12)]
    assert L.sim_loss_mse_noalloc(16, None, *p[1:8], None, None, None, None) == fsb.SIM_ERR_INVALID_ARG
    assert L.sim_loss_mse_noalloc(16, *p[:8], p[8], None, None, None) == fsb.SIM_ERR_INVALID_ARG
    # a gradient output aliasing an input
    assert L.sim_loss_mse_noalloc(16, *p[:8], p[1], p[9], p[10], None) == fsb.SIM_ERR_INVALID_ARG


@pytest.mark.parametrize("H,W,tol,it", [(2, 10, 1e-8, 10), (10, 20000, 1e-8, 10), (10, 10, 0.0, 10),
                                        (10, 10, 1e-8, 0)])
def test_screen_project_rejects_bad_arguments(H, W, tol, it):
    """Host validation before any device work (runs without a GPU)."""
    L = fsb.lib()
    p = ctypes.c_void_p(0x1000)
    ws = ctypes.c_void_p(0x10000)
    rc = L.sim_screen_project(H, W, p, p, p, p, p, tol, it, ws, 1 << 30, None, None, None)
    assert rc == fsb.SIM_ERR_INVALID_ARG
    out = ctypes.c_size_t()
    assert L.sim_screen_workspace_size(10, 10, ctypes.byref(out)) == fsb.SIM_OK and out.value > 0
    assert L.sim_screen_workspace_size(2, 10, ctypes.byref(out)) == fsb.SIM_ERR_INVALID_ARG
