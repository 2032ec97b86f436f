"""ctypes binding of ``libfluidsim.so`` (the C ABI in ``include/fluidsim.h``).

Argument marshalling only: every operation runs in the library's HIP
kernels.  PyTorch provides device memory (the caller-owned workspace and
fields) and the stream.  If the library is missing this module raises; there
is no fallback implementation.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, byref, c_double, c_float, c_int32, c_int64, c_size_t, c_void_p

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfluidsim.so")

SIM_OK = 0
SIM_OK_FALLBACK = 1
SIM_ERR_INVALID_ARG = -1
SIM_ERR_WORKSPACE_TOO_SMALL = -2
SIM_ERR_HIP = -3
SIM_ERR_NOT_CONVERGED = -4
SIM_ERR_SINGULAR_MASK = -5
SIM_ERR_STATE = -6

SIM_PRECOND_JACOBI, SIM_PRECOND_MIC0, SIM_PRECOND_LEARNED = 0, 1, 2
KERNEL_KINDS = ["pcg_dir_spmv", "pcg_update", "pcg_check", "advect", "diffuse_explicit",
                "dcg_dir_spmv", "dcg_update", "mic0", "net", "advect_adjoint", "percnn",
                "percnn_adj"]
SIM_DIFFUSION_AUTO, SIM_DIFFUSION_EXPLICIT, SIM_DIFFUSION_IMPLICIT = 0, 1, 2

SIM_CONVGRAD_EXACT, SIM_CONVGRAD_UPWIND = 0, 1

PRECONDS = {"jacobi": SIM_PRECOND_JACOBI, "mic0": SIM_PRECOND_MIC0, "learned": SIM_PRECOND_LEARNED}
CONVGRADS = {"exact": SIM_CONVGRAD_EXACT, "upwind": SIM_CONVGRAD_UPWIND}
DIFFUSIONS = {"auto": SIM_DIFFUSION_AUTO, "explicit": SIM_DIFFUSION_EXPLICIT,
              "implicit": SIM_DIFFUSION_IMPLICIT}


class sim_desc(ctypes.Structure):
    _fields_ = [("n", c_int32), ("precond", c_int32), ("diffusion", c_int32),
                ("max_iter", c_int32), ("check_every", c_int32), ("checkpoint_every", c_int32),
                ("max_steps", c_int32), ("learned_max_iter", c_int32), ("tol", c_double),
                ("diff_tol", c_double), ("warm_start", c_int32), ("store_pressures", c_int32),
                ("convection_grad", c_int32)]


class sim_params(ctypes.Structure):
    _fields_ = [("nu", c_double), ("s", c_double), ("dt", c_double), ("gravity", c_double * 3)]


class sim_stats(ctypes.Structure):
    _fields_ = [("status", c_int32), ("iters", c_int32), ("diff_iters", c_int32),
                ("fallback_used", c_int32), ("rel_residual", c_double),
                ("diff_rel_residual", c_double)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class FluidSimError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"fluidsim error {code}: {msg}")
        self.code = code


# every entry point declared in include/fluidsim.h: name -> (restype, argtypes)
_P = c_void_p
SIGNATURES = {
    "sim_workspace_size": (c_int32, [POINTER(sim_desc), POINTER(c_size_t)]),
    "sim_create": (c_int32, [POINTER(sim_desc), _P, _P, c_size_t, _P, POINTER(_P)]),
    "sim_set_params": (c_int32, [_P, POINTER(sim_params)]),
    "sim_init_state": (c_int32, [_P, _P, _P, _P, _P, _P, _P]),
    "sim_step": (c_int32, [_P, _P, _P, _P, c_int32, c_int32, POINTER(sim_stats)]),
    "sim_project": (c_int32, [_P, _P, _P, _P, _P, POINTER(sim_stats)]),
    "sim_backward": (c_int32, [_P, _P, _P, _P, _P, _P, _P, _P, _P, _P, POINTER(c_double),
                               POINTER(sim_stats)]),
    "sim_loss_mse": (c_int32, [_P, _P, _P, _P, _P, _P, _P, POINTER(c_double), _P, _P, _P]),
    "sim_loss_cos_l2": (c_int32, [_P, _P, _P, _P, _P, _P, _P, c_double, c_double, c_double,
                                  POINTER(c_double), POINTER(c_double), _P, _P, _P]),
    "sim_loss_mse_noalloc": (c_int32, [c_int32, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "sim_screen_workspace_size": (c_int32, [c_int32, c_int32, POINTER(c_size_t)]),
    "sim_screen_project": (c_int32, [c_int32, c_int32, _P, _P, _P, _P, _P, c_double, c_int32, _P,
                                     c_size_t, _P, POINTER(c_int32), POINTER(c_double)]),
    "sim_apic_p2g": (c_int32, [_P, c_int64, _P, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "sim_apic_g2p": (c_int32, [_P, c_int64, _P, _P, _P, c_double, _P, _P, _P]),
    "sim_net_param_count": (c_int32, [POINTER(c_int64)]),
    "sim_net_set_weights": (c_int32, [_P, _P, c_int64]),
    "sim_net_forward": (c_int32, [_P, _P, _P]),
    "sim_net_set_tile_skip": (c_int32, [_P, c_int32]),
    "sim_harvest_pairs": (c_int32, [_P, _P, _P, _P, POINTER(c_int32), c_int32, c_int32, c_double,
                                    _P, _P, POINTER(sim_stats)]),
    "sim_net_grad": (c_int32, [_P, _P, _P, c_int32, _P, POINTER(c_double)]),
    "sim_net_train_step": (c_int32, [_P, _P, _P, c_int32, _P, _P, c_int32, c_float,
                                     POINTER(c_double)]),
    "sim_op_advect": (c_int32, [_P, _P, _P, _P, _P, _P, _P]),
    "sim_op_diffuse": (c_int32, [_P, _P, _P, _P, _P, _P, _P, POINTER(sim_stats)]),
    "sim_op_divergence": (c_int32, [_P, _P, _P, _P, _P]),
    "sim_op_poisson_apply": (c_int32, [_P, _P, _P]),
    "sim_op_precond_apply": (c_int32, [_P, c_int32, _P, _P]),
    "sim_op_advect_adjoint": (c_int32, [_P, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "sim_op_convection_grad_upwind": (c_int32, [_P, _P, _P, _P, _P, _P, _P, _P, _P, _P]),
    "sim_percnn_forward": (c_int32, [_P, POINTER(c_float), c_int32, _P, _P, _P, _P]),
    "sim_percnn_backward": (c_int32, [_P, POINTER(c_float), c_int32, _P, _P, _P, _P, _P,
                                      POINTER(c_double)]),
    "sim_percnn_fit_step": (c_int32, [_P, POINTER(c_double), POINTER(c_double), c_int32, c_double,
                                      c_int32, c_int32, _P, _P, _P, _P, POINTER(c_double)]),
    "sim_constrained_project": (c_int32, [_P, _P, _P, _P, c_int32, c_double, POINTER(c_double)]),
    "sim_profile_enable": (c_int32, [_P, c_int32]),
    "sim_profile_read": (c_int32, [_P, POINTER(c_double), POINTER(c_int64)]),
    "sim_destroy": (c_int32, [_P]),
    "sim_last_error": (ctypes.c_char_p, [_P]),
}

_lib = None


def lib():
    """Load libfluidsim.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise FluidSimError(SIM_ERR_STATE, f"{LIB_PATH} is not built; run "
                                "`python -m paper_2503_00868_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def _ptr(t):
    if t is None:
        return None
    return c_void_p(t.data_ptr())


def last_error(ctx):
    msg = lib().sim_last_error(ctx)
    return msg.decode() if msg else ""


def check(rc, ctx=None, allow=(SIM_OK, SIM_OK_FALLBACK)):
    if rc not in allow:
        raise FluidSimError(rc, last_error(ctx) if ctx else "")
    return rc


# ------------------------------------------------------------------ raw ABI

def screen_project(a, b, vz, z, mask, tol=1e-10, max_iter=20000, workspace=None, stream=None):
    """sim_screen_project in place on the float32 device tensors a (H, W+1)
    and b (H+1, W), with vz, z (H, W) float32 and mask (H, W) uint8 on the
    device.  The workspace is a torch uint8 tensor (allocated here when not
    given).  Returns (iterations, true relative residual)."""
    import torch
    H, W = int(vz.shape[0]), int(vz.shape[1])
    size = c_size_t(0)
    check(lib().sim_screen_workspace_size(H, W, byref(size)))
    if workspace is None:
        workspace = torch.empty(size.value, dtype=torch.uint8, device=vz.device)
    it, rel = c_int32(0), c_double(0.0)
    st = stream if stream is not None else torch.cuda.current_stream(vz.device)
    rc = lib().sim_screen_project(H, W, _ptr(a), _ptr(b), _ptr(vz), _ptr(z), _ptr(mask), float(tol),
                                  int(max_iter), _ptr(workspace),
                                  workspace.numel() * workspace.element_size(),
                                  c_void_p(st.cuda_stream), byref(it), byref(rel))
    if rc != SIM_OK:
        raise FluidSimError(rc, f"sim_screen_project returned {rc} (iterations {it.value}, "
                            f"relative residual {rel.value:.3e})")
    return it.value, rel.value


def loss_mse_noalloc(n, d_cell, u, target, d_loss, g=None, stream=None):
    """sim_loss_mse_noalloc: J into the device float64 tensor d_loss (one
    element), dJ/du into g (three face tensors) when given.  Enqueue only."""
    gg = g if g is not None else (None, None, None)
    rc = lib().sim_loss_mse_noalloc(int(n), _ptr(d_cell), *map(_ptr, u), *map(_ptr, target),
                                    _ptr(d_loss), *map(_ptr, gg),
                                    c_void_p(stream.cuda_stream if stream is not None else 0))
    if rc == SIM_ERR_INVALID_ARG:
        raise FluidSimError(rc, "sim_loss_mse_noalloc: n outside [4, 1024], a NULL input, a "
                            "partial gradient set or an aliased output")
    return check(rc)


def sim_workspace_size(desc: sim_desc) -> int:
    out = c_size_t(0)
    check(lib().sim_workspace_size(byref(desc), byref(out)))
    return out.value


def sim_create(desc: sim_desc, cell_host: np.ndarray, workspace, stream_handle: int):
    cell = np.ascontiguousarray(cell_host, dtype=np.uint8)
    ctx = c_void_p()
    rc = lib().sim_create(byref(desc), cell.ctypes.data_as(c_void_p), _ptr(workspace),
                          workspace.numel() * workspace.element_size(), c_void_p(stream_handle),
                          byref(ctx))
    check(rc)
    return ctx


def make_desc(n, precond="jacobi", diffusion="auto", tol=1e-6, diff_tol=1e-6, max_iter=20000,
              check_every=8, checkpoint_every=8, max_steps=0, learned_max_iter=200,
              warm_start=False, store_pressures=False, convection_grad="exact"):
    return sim_desc(n=n, precond=PRECONDS[precond] if isinstance(precond, str) else precond,
                    diffusion=DIFFUSIONS[diffusion] if isinstance(diffusion, str) else diffusion,
                    max_iter=max_iter, check_every=check_every, checkpoint_every=checkpoint_every,
                    max_steps=max_steps, learned_max_iter=learned_max_iter, tol=tol,
                    diff_tol=diff_tol, warm_start=int(bool(warm_start)),
                    store_pressures=int(bool(store_pressures)),
                    convection_grad=(CONVGRADS[convection_grad] if isinstance(convection_grad, str)
                                     else convection_grad))


def face_shapes(n):
    return [(n, n, n + 1), (n, n + 1, n), (n + 1, n, n)]


class Sim:
    """One context: owns the device workspace (a torch uint8 tensor) and
    forwards every call to the C ABI on torch's current stream."""

    def __init__(self, cell, precond="jacobi", diffusion="auto", tol=1e-6, diff_tol=1e-6,
                 max_iter=20000, check_every=8, checkpoint_every=8, max_steps=0,
                 learned_max_iter=200, warm_start=False, store_pressures=False,
                 convection_grad="exact", device="cuda"):
        import torch
        self.torch = torch
        cell = np.ascontiguousarray(cell, dtype=np.uint8)
        self.n = n = cell.shape[0]
        self.device = torch.device(device)
        self.desc = make_desc(n, precond, diffusion, tol, diff_tol, max_iter, check_every,
                              checkpoint_every, max_steps, learned_max_iter, warm_start,
                              store_pressures, convection_grad)
        size = sim_workspace_size(self.desc)
        self.ws = torch.empty(size, dtype=torch.uint8, device=self.device)
        assert self.ws.data_ptr() % 256 == 0
        self.stream = torch.cuda.current_stream(self.device)
        self.ctx = sim_create(self.desc, cell, self.ws, self.stream.cuda_stream)
        self.cell = cell
        self.params = None
        # bumped by every recorded rollout and every set_params (which makes
        # the library forget its recording): a backward can tell whether the
        # recording it needs is still the current one
        self.record_gen = 0

    def close(self):
        if getattr(self, "ctx", None):
            lib().sim_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- helpers
    def faces(self, fill=0.0):
        t = self.torch
        return tuple(t.full(s, fill, dtype=t.float32, device=self.device)
                     for s in face_shapes(self.n))

    def to_faces(self, arrays):
        t = self.torch
        return tuple(t.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device=self.device)
                     for a in arrays)

    def cells_tensor(self, arr=None, dtype=None):
        t = self.torch
        dtype = dtype or t.float32
        if arr is None:
            return t.zeros((self.n,) * 3, dtype=dtype, device=self.device)
        return t.as_tensor(np.ascontiguousarray(arr), device=self.device).to(dtype)

    def _chk(self, rc, allow=(SIM_OK, SIM_OK_FALLBACK)):
        return check(rc, self.ctx, allow)

    # -- ABI
    def set_params(self, nu, dt, s=1.0, gravity=(0.0, -9.8, 0.0)):
        p = sim_params(nu=nu, s=s, dt=dt, gravity=(c_double * 3)(*gravity))
        self._chk(lib().sim_set_params(self.ctx, byref(p)))
        self.params = dict(nu=nu, dt=dt, s=s, gravity=tuple(gravity))
        self.record_gen += 1

    def init_state(self, ugen, out):
        self._chk(lib().sim_init_state(self.ctx, *map(_ptr, ugen), *map(_ptr, out)))
        return out

    def step(self, u, nsteps=1, record=False, allow=(SIM_OK, SIM_OK_FALLBACK)):
        st = (sim_stats * max(nsteps, 1))()
        if record:
            self.record_gen += 1
        rc = lib().sim_step(self.ctx, *map(_ptr, u), nsteps, int(record), st)
        self._chk(rc, allow)
        return [st[q].as_dict() for q in range(nsteps)]

    def project(self, u, want_p=False, allow=(SIM_OK, SIM_OK_FALLBACK)):
        t = self.torch
        p = t.zeros((self.n,) * 3, dtype=t.float64, device=self.device) if want_p else None
        st = sim_stats()
        rc = lib().sim_project(self.ctx, *map(_ptr, u), _ptr(p), byref(st))
        self._chk(rc, allow)
        return st.as_dict(), p

    def backward(self, g, ugen=None, out=None, full=False):
        """Gradient of the last recorded rollout.  Returns (dJ/du0 or dJ/dugen,
        dJ/dnu, dJ/ds, stats), or with full=True (dJ/du0, grads, stats) where
        grads = {"nu", "s", "dt", "gravity" (3-tuple)}."""
        out = out if out is not None else self.faces()
        grad = (c_double * 6)()
        st = sim_stats()
        ug = ugen if ugen is not None else (None, None, None)
        rc = lib().sim_backward(self.ctx, *map(_ptr, g), *map(_ptr, ug), *map(_ptr, out), grad,
                                byref(st))
        self._chk(rc)
        if full:
            return out, {"nu": grad[0], "s": grad[1], "dt": grad[2],
                         "gravity": (grad[3], grad[4], grad[5])}, st.as_dict()
        return out, grad[0], grad[1], st.as_dict()

    def loss_mse(self, u, target, want_grad=True):
        g = self.faces() if want_grad else (None, None, None)
        J = c_double()
        self._chk(lib().sim_loss_mse(self.ctx, *map(_ptr, u), *map(_ptr, target), byref(J),
                                     *map(_ptr, g)))
        return J.value, (g if want_grad else None)

    def loss_cos_l2(self, u, ref, alpha, beta, eps, weights, want_grad=True, out=None):
        """The paper's masked cosine + L2 velocity loss of u against ref, and
        dJ/du (into `out` when given); weights = (empty, occupied, surface)."""
        g = (out if out is not None else self.faces()) if want_grad else (None, None, None)
        J = c_double()
        w = (c_double * 3)(*[float(x) for x in weights])
        self._chk(lib().sim_loss_cos_l2(self.ctx, *map(_ptr, u), *map(_ptr, ref), float(alpha),
                                        float(beta), float(eps), w, byref(J), *map(_ptr, g)))
        return J.value, (g if want_grad else None)

    def apic_p2g(self, x, vp, C, m, out=None, mass=None):
        """The paper's particle-to-grid transfer: (grid velocity, grid masses).
        x, vp: (P, 3); C: (P, 3, 3); m: (P,); float32 device tensors."""
        out = out if out is not None else self.faces()
        mass = mass if mass is not None else self.faces()
        P = int(m.shape[0])
        self._chk(lib().sim_apic_p2g(self.ctx, P, _ptr(x), _ptr(vp), _ptr(C), _ptr(m),
                                     *map(_ptr, out), *map(_ptr, mass)))
        return out, mass

    def apic_g2p(self, grid, x, dt, vp=None, C=None):
        """The paper's grid-to-particle transfer with the affine update; moves
        x (in place) by dt times the new velocity.  Returns (vp, C)."""
        t = self.torch
        P = int(x.shape[0])
        vp = vp if vp is not None else t.empty((P, 3), dtype=t.float32, device=self.device)
        C = C if C is not None else t.empty((P, 3, 3), dtype=t.float32, device=self.device)
        self._chk(lib().sim_apic_g2p(self.ctx, P, *map(_ptr, grid), float(dt), _ptr(x), _ptr(vp),
                                     _ptr(C)))
        return vp, C

    def op_advect(self, u, out=None):
        out = out if out is not None else self.faces()
        self._chk(lib().sim_op_advect(self.ctx, *map(_ptr, u), *map(_ptr, out)))
        return out

    def op_diffuse(self, u, out=None):
        out = out if out is not None else self.faces()
        st = sim_stats()
        self._chk(lib().sim_op_diffuse(self.ctx, *map(_ptr, u), *map(_ptr, out), byref(st)))
        return out, st.as_dict()

    def op_divergence(self, u, b=None):
        b = b if b is not None else self.cells_tensor()
        self._chk(lib().sim_op_divergence(self.ctx, *map(_ptr, u), _ptr(b)))
        return b

    def op_poisson_apply(self, x, y=None):
        y = y if y is not None else self.cells_tensor()
        self._chk(lib().sim_op_poisson_apply(self.ctx, _ptr(x), _ptr(y)))
        return y

    def op_precond_apply(self, precond, r, z=None):
        z = z if z is not None else self.cells_tensor()
        pc = PRECONDS[precond] if isinstance(precond, str) else precond
        self._chk(lib().sim_op_precond_apply(self.ctx, pc, _ptr(r), _ptr(z)))
        return z

    def op_advect_adjoint(self, u, lam, out=None):
        out = out if out is not None else self.faces()
        self._chk(lib().sim_op_advect_adjoint(self.ctx, *map(_ptr, u), *map(_ptr, lam),
                                              *map(_ptr, out)))
        return out

    def op_convection_grad_upwind(self, u, lam, out=None):
        """The paper's upwind convection gradient for the convected field u."""
        out = out if out is not None else self.faces()
        self._chk(lib().sim_op_convection_grad_upwind(self.ctx, *map(_ptr, u), *map(_ptr, lam),
                                                      *map(_ptr, out)))
        return out

    def harvest_pairs(self, u, iters, tol=1e-10, r_out=None, e_out=None, mode=0):
        t = self.torch
        k = len(iters)
        shape = (k,) + (self.n,) * 3
        r_out = r_out if r_out is not None else t.zeros(shape, dtype=t.float32, device=self.device)
        e_out = e_out if e_out is not None else t.zeros(shape, dtype=t.float32, device=self.device)
        arr = (c_int32 * k)(*iters)
        st = sim_stats()
        self._chk(lib().sim_harvest_pairs(self.ctx, *map(_ptr, u), arr, k, mode, tol,
                                          _ptr(r_out), _ptr(e_out), byref(st)))
        return r_out, e_out, st.as_dict()

    # -- recurrent convolutional pressure solver
    @staticmethod
    def _percnn_w(w):
        w = np.ascontiguousarray(np.asarray(w, dtype=np.float32).ravel())
        if w.size != 28:
            raise ValueError("28 weights: W_0 .. W_26, w_b")
        return w, w.ctypes.data_as(POINTER(c_float))

    def percnn_forward(self, w, K, p0, b, out=None, hist=None):
        """K recurrent layers from p0 (cell tensors); returns out (p_K) or,
        with hist ((K+1, n, n, n) float32), the recorded states."""
        wa, wp = self._percnn_w(w)
        if out is None and hist is None:
            out = self.cells_tensor()
        self._chk(lib().sim_percnn_forward(self.ctx, wp, int(K), _ptr(p0), _ptr(b),
                                           _ptr(out) if out is not None else None,
                                           _ptr(hist) if hist is not None else None))
        return out if out is not None else hist

    def percnn_fit_step(self, w, adam, step, lr, K, p0, target, b, hist):
        """sim_percnn_fit_step: w (28) and adam (56) are float64 numpy arrays
        updated in place; p0, target, b stacked (npairs, n, n, n) float32
        device tensors; hist ((K+1), n, n, n) float32.  Returns the mean loss
        before the update."""
        assert w.dtype == np.float64 and w.size == 28 and adam.dtype == np.float64 and adam.size == 56
        loss = c_double(0.0)
        self._chk(lib().sim_percnn_fit_step(
            self.ctx, w.ctypes.data_as(POINTER(c_double)), adam.ctypes.data_as(POINTER(c_double)),
            int(step), float(lr), int(K), int(p0.shape[0]), _ptr(p0), _ptr(target), _ptr(b),
            _ptr(hist), byref(loss)))
        return loss.value

    def percnn_backward(self, w, K, b, hist, g, gp0=None, gb=None):
        """Reverse pass: returns dL/d(W, w_b) (28 float64) and fills gp0, gb."""
        wa, wp = self._percnn_w(w)
        gw = (c_double * 28)()
        self._chk(lib().sim_percnn_backward(self.ctx, wp, int(K), _ptr(b), _ptr(hist), _ptr(g),
                                            _ptr(gp0) if gp0 is not None else None,
                                            _ptr(gb) if gb is not None else None, gw))
        return np.array(gw[:], dtype=np.float64)

    def constrained_project(self, u, iters, eps=0.0):
        """Constrained divergence projection in place; returns the relative
        L2 divergence left (|b(u_K)| / |b(u_0)|)."""
        rel = c_double()
        self._chk(lib().sim_constrained_project(self.ctx, *map(_ptr, u), int(iters), float(eps),
                                                byref(rel)))
        return rel.value

    # -- kernel timing
    def profile_enable(self, on=True):
        self._chk(lib().sim_profile_enable(self.ctx, int(on)))

    def profile_read(self):
        k = len(KERNEL_KINDS)
        ms = (c_double * k)()
        cnt = (c_int64 * k)()
        self._chk(lib().sim_profile_read(self.ctx, ms, cnt))
        return {name: (ms[q], cnt[q]) for q, name in enumerate(KERNEL_KINDS)}

    # -- learned preconditioner
    def net_set_weights(self, w):
        self._chk(lib().sim_net_set_weights(self.ctx, _ptr(w), w.numel()))

    def net_forward(self, r, z=None):
        z = z if z is not None else self.cells_tensor()
        self._chk(lib().sim_net_forward(self.ctx, _ptr(r), _ptr(z)))
        return z

    def net_set_tile_skip(self, on):
        self._chk(lib().sim_net_set_tile_skip(self.ctx, int(bool(on))))

    def net_grad(self, r, e, batch, grad):
        loss = c_double()
        self._chk(lib().sim_net_grad(self.ctx, _ptr(r), _ptr(e), batch, _ptr(grad), byref(loss)))
        return loss.value

    def net_train_step(self, r, e, batch, master, adam, step, lr):
        loss = c_double()
        self._chk(lib().sim_net_train_step(self.ctx, _ptr(r), _ptr(e), batch, _ptr(master),
                                           _ptr(adam), step, c_float(lr), byref(loss)))
        return loss.value


def net_param_count():
    out = c_int64()
    check(lib().sim_net_param_count(byref(out)))
    return out.value
