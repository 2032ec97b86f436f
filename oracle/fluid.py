"""FP64 oracle of the MAC-grid liquid step, its rollout, loss and gradient.

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the benchmark's
CPU-baseline leg may use it; the GPU path never does.

The grid operators are plain C loops in ``oracle.c`` (FP64); this module
marshals numpy arrays into them and composes them in the order the step
defines.  Paper passages (arXiv 2503.00868):

* momentum equation with body force, viscosity and pressure: Section 3.2.2,
  Eq. (v); operator splitting after Chorin: Section 3.2.2;
* semi-Lagrangian back-tracing of the convection term: Section 3.4.1;
* the parameters being fitted and their exp/sigmoid normalisation, the L2
  velocity loss over a grid mask: Section 3.4.2, Eq. (optLoss).

Readings where the paper is silent or differs (numbered as in the design
notes): R2 non-active faces hold zero; R3 one Euler back-trace; R5 viscosity
as a componentwise Laplacian; R6 explicit/implicit switch at nu*dt/h^2 = 1/12;
R7 p = 0 at air cell centres; R9 the step order advect -> force -> diffuse ->
project (the paper lists force -> project -> viscosity), so every step ends
divergence-free; R10 the liquid mask is fixed over a rollout; R13 the
gradient is the exact discrete adjoint, not the paper's upwind surrogate.
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass

import numpy as np

from . import build as _build

AIR, LIQUID, SOLID = 0, 1, 2
INACTIVE, ACTIVE, WALL = 0, 1, 2
PRECOND_NONE, PRECOND_JACOBI, PRECOND_MIC0 = 0, 1, 2
GRAVITY = (0.0, -9.8, 0.0)
MIC_TAU, MIC_SIGMA = 0.97, 0.25

_lib = None
_D = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_U8 = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")
_i, _d, _l = ctypes.c_int, ctypes.c_double, ctypes.c_long
_dp = ctypes.POINTER(ctypes.c_double)


def lib():
    global _lib
    if _lib is None:
        L = ctypes.CDLL(_build.ensure_built())
        sig = {
            "orc_face_count": (_l, [_i, _i]),
            "orc_face_classes": (None, [_i, _U8, _i, _U8]),
            "orc_mask_faces": (None, [_i, _U8, _i, _D]),
            "orc_sample": (_d, [_i, _i, _D, _D, ctypes.c_void_p]),
            "orc_advect": (None, [_i, _U8, _D, _D, _D, _d, _D, _D, _D]),
            "orc_add_force": (None, [_i, _U8, _D, _D, _D, _d, _D]),
            "orc_laplacian": (None, [_i, _U8, _i, _D, _D]),
            "orc_diffuse_explicit": (None, [_i, _U8, _i, _d, _D, _D]),
            "orc_diffuse_implicit": (_i, [_i, _U8, _i, _d, _D, _D, _d, _i, _dp]),
            "orc_poisson_diag": (None, [_i, _U8, _D]),
            "orc_poisson_apply": (None, [_i, _U8, _D, _D]),
            "orc_divergence_rhs": (None, [_i, _U8, _D, _D, _D, _D]),
            "orc_pressure_update": (None, [_i, _U8, _D, _D, _D, _D]),
            "orc_mic0_setup": (None, [_i, _U8, _d, _d, _D]),
            "orc_mic0_apply": (None, [_i, _U8, _D, _D, _D]),
            "orc_pcg": (_i, [_i, _U8, _D, _D, _i, _d, _i, _dp]),
            "orc_true_relres": (_d, [_i, _U8, _D, _D]),
            "orc_advect_adjoint": (None, [_i, _U8, _D, _D, _D, _d, _D, _D, _D, _D, _D, _D]),
            "orc_advect_ddt": (None, [_i, _U8, _D, _D, _D, _d, _D, _D, _D]),
        }
        for name, (res, args) in sig.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


# ------------------------------------------------------------------ shapes

def face_shape(n: int, comp: int):
    """Array shape ``[k][j][i]`` of the faces of one velocity component."""
    return (n + (comp == 2), n + (comp == 1), n + (comp == 0))


def zeros_faces(n: int):
    return tuple(np.zeros(face_shape(n, c)) for c in range(3))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _cell(cell):
    return np.ascontiguousarray(cell, dtype=np.uint8)


def _n(cell):
    n = cell.shape[0]
    assert cell.shape == (n, n, n)
    return n


# --------------------------------------------------------------- operators

def face_classes(cell, comp):
    cell = _cell(cell)
    n = _n(cell)
    out = np.zeros(face_shape(n, comp), np.uint8)
    lib().orc_face_classes(n, cell, comp, out)
    return out


def mask_faces(cell, fields):
    """Zero every non-active face (R2)."""
    cell = _cell(cell)
    n = _n(cell)
    out = []
    for c, f in enumerate(fields):
        g = _f64(f).copy()
        lib().orc_mask_faces(n, cell, c, g)
        out.append(g)
    return tuple(out)


def sample(n, comp, field, g):
    """Trilinear sample of one component at grid-unit position g, and its
    gradient with respect to g (zero along clamped axes)."""
    grad = np.zeros(3)
    val = lib().orc_sample(n, comp, _f64(field), _f64(np.asarray(g, float)),
                           grad.ctypes.data_as(ctypes.c_void_p))
    return val, grad


def advect(cell, fields, dt):
    """Semi-Lagrangian advection of the face velocities by themselves."""
    cell = _cell(cell)
    n = _n(cell)
    u, v, w = (_f64(f) for f in fields)
    out = zeros_faces(n)
    lib().orc_advect(n, cell, u, v, w, dt * n, *out)
    return out


def add_force(cell, fields, dt, g=GRAVITY):
    cell = _cell(cell)
    n = _n(cell)
    out = tuple(_f64(f).copy() for f in fields)
    lib().orc_add_force(n, cell, *out, dt, _f64(np.asarray(g, float)))
    return out


def laplacian(cell, comp, f):
    cell = _cell(cell)
    n = _n(cell)
    out = np.zeros(face_shape(n, comp))
    lib().orc_laplacian(n, cell, comp, _f64(f), out)
    return out


def diffusion_is_explicit(n, nu, dt, mode="auto"):
    """R6: the explicit step is taken iff nu*dt/h^2 <= 1/12 (half the
    stability limit of the 7-point explicit scheme) unless forced."""
    if mode == "explicit":
        return True
    if mode == "implicit":
        return False
    return nu * dt * n * n <= 1.0 / 12.0


def diffuse(cell, fields, nu, dt, mode="auto", tol=1e-12, max_iter=100000):
    """Viscosity sub-step (Section 3.2.2, Eq. (v), viscous term; R5)."""
    cell = _cell(cell)
    n = _n(cell)
    out = zeros_faces(n)
    explicit = diffusion_is_explicit(n, nu, dt, mode)
    iters = 0
    for c in range(3):
        if explicit:
            lib().orc_diffuse_explicit(n, cell, c, nu * dt, _f64(fields[c]), out[c])
        else:
            rr = ctypes.c_double()
            iters += lib().orc_diffuse_implicit(n, cell, c, nu * dt, _f64(fields[c]), out[c], tol,
                                                max_iter, ctypes.byref(rr))
    return out, explicit, iters


def poisson_diag(cell):
    cell = _cell(cell)
    n = _n(cell)
    d = np.zeros((n, n, n))
    lib().orc_poisson_diag(n, cell, d)
    return d


def poisson_apply(cell, p):
    cell = _cell(cell)
    n = _n(cell)
    out = np.zeros((n, n, n))
    lib().orc_poisson_apply(n, cell, _f64(p), out)
    return out


def divergence_rhs(cell, fields):
    cell = _cell(cell)
    n = _n(cell)
    b = np.zeros((n, n, n))
    lib().orc_divergence_rhs(n, cell, *(_f64(f) for f in fields), b)
    return b


def pressure_update(cell, p, fields):
    cell = _cell(cell)
    n = _n(cell)
    out = tuple(_f64(f).copy() for f in fields)
    lib().orc_pressure_update(n, cell, _f64(p), *out)
    return out


def mic0_setup(cell, tau=MIC_TAU, sigma=MIC_SIGMA):
    cell = _cell(cell)
    n = _n(cell)
    pc = np.zeros((n, n, n))
    lib().orc_mic0_setup(n, cell, tau, sigma, pc)
    return pc


def mic0_apply(cell, precon, r):
    cell = _cell(cell)
    n = _n(cell)
    z = np.zeros((n, n, n))
    lib().orc_mic0_apply(n, cell, _f64(precon), _f64(r), z)
    return z


def pcg(cell, b, precond=PRECOND_NONE, tol=1e-12, max_iter=100000, x0=None):
    """PCG on the Poisson matrix.  Returns (x, iterations, true relres)."""
    cell = _cell(cell)
    n = _n(cell)
    x = np.zeros((n, n, n)) if x0 is None else _f64(x0).copy()
    rr = ctypes.c_double()
    it = lib().orc_pcg(n, cell, _f64(b), x, precond, tol, max_iter, ctypes.byref(rr))
    return x, it, rr.value


def true_relres(cell, b, x):
    cell = _cell(cell)
    return lib().orc_true_relres(_n(cell), cell, _f64(b), _f64(x))


def project(cell, fields, tol=1e-12, precond=PRECOND_NONE, max_iter=100000):
    """Pressure projection: mask, solve A p = b to tol, subtract the pressure
    gradient.  Returns (fields, p, iterations, relres)."""
    fields = mask_faces(cell, fields)
    b = divergence_rhs(cell, fields)
    p, it, rr = pcg(cell, b, precond, tol, max_iter)
    return pressure_update(cell, p, fields), p, it, rr


@dataclass
class StepInfo:
    explicit: bool
    diff_iters: int
    proj_iters: int
    relres: float


def step(cell, fields, nu, dt, g=GRAVITY, mode="auto", tol=1e-12, diff_tol=None):
    """One liquid step: advect -> force -> diffuse -> project (R9)."""
    a = advect(cell, fields, dt)
    a = add_force(cell, a, dt, g)
    d, explicit, diters = diffuse(cell, a, nu, dt, mode, tol if diff_tol is None else diff_tol)
    out, _, it, rr = project(cell, d, tol)
    return out, StepInfo(explicit, diters, it, rr)


def initial_state(cell, u_gen, s):
    """u0 = s * (u_gen with non-active faces zeroed); s is the fitted
    initial-velocity scale."""
    return tuple(s * f for f in mask_faces(cell, u_gen))


def rollout(cell, u_gen, nu, s, steps, dt, g=GRAVITY, mode="auto", tol=1e-12):
    """Returns the list of states [u0, u1, ..., u_steps]."""
    states = [initial_state(cell, u_gen, s)]
    for _ in range(steps):
        nxt, _ = step(cell, states[-1], nu, dt, g, mode, tol)
        states.append(nxt)
    return states


def active_count(cell):
    return int(sum(int((face_classes(cell, c) == ACTIVE).sum()) for c in range(3)))


def loss(cell, uT, target):
    """L2 term of Eq. (optLoss): mean squared error over active faces."""
    m = active_count(cell)
    diff = mask_faces(cell, tuple(a - b for a, b in zip(uT, target)))
    return sum(float((d * d).sum()) for d in diff) / m


def loss_grad(cell, uT, target):
    m = active_count(cell)
    return mask_faces(cell, tuple(2.0 * (a - b) / m for a, b in zip(uT, target)))


def _dot(a, b):
    return sum(float((x * y).sum()) for x, y in zip(a, b))


def advect_adjoint(cell, fields, dt, lam):
    """(d advect / d fields)^T lam."""
    cell = _cell(cell)
    n = _n(cell)
    out = zeros_faces(n)
    lib().orc_advect_adjoint(n, cell, *(_f64(f) for f in fields), dt * n,
                             *(_f64(l) for l in lam), *out)
    return out


def advect_ddt(cell, fields, dt):
    """d(advect(fields))/d(dt) per face: the departure point's motion with the
    time step (active faces; zero elsewhere)."""
    cell = _cell(cell)
    n = _n(cell)
    u, v, w = (_f64(f) for f in fields)
    out = zeros_faces(n)
    lib().orc_advect_ddt(n, cell, u, v, w, dt * n, *out)
    return out


def step_adjoint(cell, u_n, lam, nu, dt, g=GRAVITY, mode="auto", tol=1e-12, convection="exact"):
    """Reverse one step.  Given lam = dJ/du_{n+1}, returns dJ/du_n and this
    step's partial derivatives {"dnu", "ddt", "dg"} of J.

    The projection is a symmetric projector on the active faces and the
    diffusion operator is symmetric, so each is its own transpose.  The
    scaled pressure does not depend on dt (R8).  dt enters the step three
    times: the back-trace distance, the body-force increment dt*g on active
    faces, and the viscous factor nu*dt (so the viscous part of dJ/ddt is
    nu/dt times that of dJ/dnu).  convection="upwind" replaces the exact
    transpose of the velocity dependence of advection by the paper's upwind
    surrogate (Section 3.4.1; upwind.py); the dt and g derivatives are the
    same in both modes."""
    from . import upwind
    n = _n(_cell(cell))
    g = tuple(float(x) for x in g)
    a = add_force(cell, advect(cell, u_n, dt), dt, g)
    explicit = diffusion_is_explicit(n, nu, dt, mode)
    lam1, _, _, _ = project(cell, lam, tol)
    if explicit:
        la = tuple(laplacian(cell, c, a[c]) for c in range(3))
        visc = _dot(lam1, la)
        lam2, _, _ = diffuse(cell, lam1, nu, dt, "explicit")
    else:
        uss, _, _ = diffuse(cell, a, nu, dt, "implicit", tol)
        mu, _, _ = diffuse(cell, lam1, nu, dt, "implicit", tol)
        lu = tuple(laplacian(cell, c, uss[c]) for c in range(3))
        visc = _dot(mu, lu)
        lam2 = mu
    lam3 = mask_faces(cell, lam2)
    lsum = [float(l.sum()) for l in lam3]  # lam3 is zero off the active faces
    parts = {
        "dnu": dt * visc,
        "dg": np.array([dt * x for x in lsum]),
        "ddt": nu * visc + sum(gc * x for gc, x in zip(g, lsum))
        + _dot(lam3, advect_ddt(cell, u_n, dt)),
    }
    if convection == "exact":
        lam_n = advect_adjoint(cell, u_n, dt, lam3)
    elif convection == "upwind":
        lam_n = upwind.gradient(cell, u_n, lam3, dt)
    else:
        raise ValueError("convection must be 'exact' or 'upwind'")
    return lam_n, parts


def rollout_grad(cell, u_gen, nu, s, steps, dt, target, g=GRAVITY, mode="auto", tol=1e-12,
                 convection="exact"):
    """Loss and its gradient (the exact discrete one, or with the paper's
    upwind convection surrogate).

    Returns a dict with J, dJ/dnu, dJ/ds, dJ/ddt, dJ/dg (3), dJ/du_gen, and
    the gradients in the normalised parameters theta_nu = log nu, theta_s =
    log s, theta_dt = log dt (exponential activation, Section 3.4.2)."""
    states = rollout(cell, u_gen, nu, s, steps, dt, g, mode, tol)
    J = loss(cell, states[-1], target)
    lam = loss_grad(cell, states[-1], target)
    dnu, ddt, dg = 0.0, 0.0, np.zeros(3)
    for t in range(steps - 1, -1, -1):
        lam, parts = step_adjoint(cell, states[t], lam, nu, dt, g, mode, tol, convection)
        dnu += parts["dnu"]
        ddt += parts["ddt"]
        dg = dg + parts["dg"]
    lam0 = mask_faces(cell, lam)
    ugm = mask_faces(cell, u_gen)
    ds = _dot(lam0, ugm)
    dug = tuple(s * l for l in lam0)
    return {"J": J, "dnu": dnu, "ds": ds, "ddt": ddt, "dg": dg, "du_gen": dug,
            "dtheta_nu": nu * dnu, "dtheta_s": s * ds, "dtheta_dt": dt * ddt,
            "uT": states[-1]}


def max_abs_divergence(cell, fields):
    """max over liquid cells of |discrete divergence| = |b|/h^2."""
    cell = _cell(cell)
    n = _n(cell)
    b = divergence_rhs(cell, fields)
    return float(np.abs(b).max()) * n * n
