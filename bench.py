"""Benchmark of the MAC-grid liquid step on one MI355X.

One bench step = one differentiable rollout of the whole hot path on the
256^3 workload (seeded slab + 3 ellipsoids liquid mask, curl-of-potential
initial velocity, nu drawn log-uniformly from [1e-4, 1e-1] for seed 4,
gravity (0,-9.8,0), dt = 1/120): u0 = s * mask(ugen), `--rollout` steps of
advection + viscosity + pressure projection to a 1e-6 FP64 relative
residual (recorded, checkpoint every 16 steps), the MSE loss against a
target rollout, and the full checkpointed reverse pass (adjoint projection
solves included).  Each solve starts from the previous step's pressure
(--cold: from zero); the stopping test is the same.  The recorded rollout
keeps every step's pressure (8.6 GB at 256^3 x 64), so the backward's segment
recompute starts each projection from the forward's solution and skips its
iterations (--no-pressure-history: repeat them).  Inputs are resident in HBM
before timing starts.

value = cell-steps/s = n^3 * rollout / (seconds per bench step).

Also reported: ms per projection and iterations for each preconditioner on
the same state (learned-FCG vs plain PCG), the roofline of the dominant
kernel from HIP-event timing inside the timed region, and the FP64 CPU
oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BF16_PEAK_TFLOPS = 2500.0

# Algorithmic bytes of each timed kernel kind: every array the operation
# must read or write once.  Cell kinds count per cell (they stream every
# cell).  Face kinds are (bytes per face over all 3F faces, bytes per active
# face): the face code and the outputs a kernel writes on every face, plus
# what it moves only on the active faces (the others it skips).
BYTES_PER_UNIT = {
    "pcg_dir_spmv": 17.0,   # r 4 + diag 1 + d 4 in; d 4 + q 4 out (Jacobi; 21 flexible CG)
    # Jacobi PCG and the flexible CG update the FP64 iterate every fourth
    # iteration: three of four iterations move r 4+4, q 4, diag 1 (13 B), the
    # fourth also x 8+8 and four directions 4x4 (45 B); the average is 21 B.
    # The flexible CG's fourth iteration ends a block, whose FP64 check
    # recomputes r, so it moves x and the directions alone (32 B): 17.75 B.
    # (MIC(0)-PCG updates x every iteration: 33 B.)
    "pcg_update": 21.0,
    "pcg_check": 17.0,      # x 8, b 4, diag 1 in; r 4 out
}
FACE_BYTES = {
    "advect": (5.0, 4.0),            # code 1 in, value 4 out everywhere; own component 4 in if active
    "diffuse_explicit": (9.0, 0.0),  # value and code in, value out, every face
    "dcg_dir_spmv": (17.0, 0.0),     # r 4, d 4, code 1 in; d 4, q 4 out, every face
    "dcg_update": (1.0, 32.0),       # code 1 everywhere; x 8 + 8, r 4 + 4, d 4, q 4 if active
    "advect_adjoint": (1.0, 20.0),   # code 1 everywhere; state 4, lambda 4 in, 3 x 4 scattered if active
}
FACE_KINDS = set(FACE_BYTES)


def active_faces(cell):
    """Faces that touch liquid and no solid cell (the box's outside is solid)."""
    import numpy as np
    c = np.pad(np.asarray(cell), 1, constant_values=2)
    total = 0
    for axis in (2, 1, 0):  # x, y, z faces
        lo = [slice(1, -1)] * 3
        hi = [slice(1, -1)] * 3
        lo[axis] = slice(0, -1)
        hi[axis] = slice(1, None)
        a, b = c[tuple(lo)], c[tuple(hi)]
        total += int(((a != 2) & (b != 2) & ((a == 1) | (b == 1))).sum())
    return total


# Recurrent convolutional pressure solver, per cell and layer: forward p 4,
# b 4, diag 1 in, p 4 out; reverse g 4, diag 1, p 4, b 4 in, g 4 out, and the
# b gradient 4 + 4 read-modify-write.
PERCNN_BYTES = {"percnn": 13.0, "percnn_adj": 25.0}
# One constrained-projection iteration, per cell, as its two kernels move it
# at most: divergence and multipliers (three face arrays 12, diagonal 1 in;
# lambda 8 out), pressure update (lambda 8, face codes 3, faces 12 in; faces
# 12 out).
CONSTRAINED_BYTES = 56.0
# The paper's upwind convection gradient, per face: own component of the
# convected field 4, lambda 4, face code 1 in; gradient 4 out (the other
# components' values around the face are re-reads of cached lines).
UPWIND_BYTES = 13.0
# The paper's masked cosine + L2 velocity loss with its gradient, per cell:
# simulated and reference faces 12 + 12, cell type 1 in; gradient 12 out.
LOSS_BYTES = 37.0

# Algorithmic FLOPs of one U-Net application per fine cell: 2 * 27 * c_in *
# c_out per voxel of each convolution (real channel counts), with the level-2
# and level-3 voxel counts 1/8 and 1/64 of the fine level.
UNET_LEVEL_CONVS = {1: [(2, 16), (16, 16), (48, 16), (16, 16), (16, 1)],
                    2: [(16, 32), (32, 32), (96, 32), (32, 32)],
                    3: [(32, 64), (64, 64)]}
NET_FLOP_PER_CELL = sum(54 * a * b / 8 ** (lvl - 1)
                        for lvl, convs in UNET_LEVEL_CONVS.items() for a, b in convs)


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=1)
    p.add_argument("--warmup", type=int, default=1)
    p.add_argument("--n", type=int, default=256)
    p.add_argument("--rollout", type=int, default=64)
    p.add_argument("--checkpoint", type=int, default=16)
    p.add_argument("--warmup-rollout", type=int, default=2,
                   help="rollout length of the untimed warmup steps")
    p.add_argument("--precond", default="auto", choices=["auto", "jacobi", "mic0", "learned"])
    p.add_argument("--weights", default=os.path.join(ROOT, "paper_2503_00868_amd", "weights",
                                                     "unet.safetensors"))
    p.add_argument("--seed", type=int, default=4)
    p.add_argument("--cold", action="store_true",
                   help="start every pressure solve of the rollout at zero (default: from the "
                        "previous step's pressure)")
    p.add_argument("--no-pressure-history", action="store_true",
                   help="recompute the backward's forward solves instead of starting them from "
                        "the stored pressures of the recorded rollout")
    p.add_argument("--check-every", type=int, default=0,
                   help="FP64 residual-check period (0: 16 for Jacobi, 4 otherwise)")
    p.add_argument("--no-plain", action="store_true",
                   help="skip the plain (Jacobi) PCG rollout timed beside a learned headline")
    p.add_argument("--no-compare", action="store_true")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-percnn", action="store_true",
                   help="skip the recurrent convolutional solver's measurement")
    p.add_argument("--percnn-layers", type=int, default=100)
    p.add_argument("--no-percnn-fit", action="store_true",
                   help="skip the recurrent solver's kernel fit and its equal-time comparison")
    p.add_argument("--no-constrained", action="store_true",
                   help="skip the constrained divergence projection's measurement")
    p.add_argument("--constrained-iters", type=int, default=100)
    p.add_argument("--no-upwind", action="store_true",
                   help="skip the upwind convection gradient's measurement")
    p.add_argument("--no-loss", action="store_true",
                   help="skip the masked cosine + L2 loss's measurement")
    p.add_argument("--no-grad-fd", action="store_true",
                   help="skip the central-FD check of the headline gradient (exact and upwind "
                        "convection adjoints)")
    p.add_argument("--no-history-leg", action="store_true",
                   help="skip the rollout timed without the pressure history")
    p.add_argument("--no-heldout", action="store_true",
                   help="skip learned vs plain on the held-out mask")
    p.add_argument("--heldout-seed", type=int, default=5)
    p.add_argument("--no-screen", action="store_true",
                   help="skip the screen-space constrained projection's measurement")
    p.add_argument("--no-apic", action="store_true",
                   help="skip the APIC transfers' measurement")
    p.add_argument("--grad-table", default="",
                   help="only measure adjoint vs central FD (exact and upwind convection "
                        "gradients) for these comma-separated rollout lengths and exit")
    p.add_argument("--cpu-n", type=int, default=128)
    p.add_argument("--workload", default="rollout",
                   choices=["rollout", "forward128", "grad128", "learned128"],
                   help="rollout: the benchmark (default).  The others measure the smaller "
                        "workloads the method is also checked on and print their own JSON line: "
                        "forward128 = 16-step MIC(0)-PCG forward rollout at 128^3; grad128 = "
                        "32-step differentiable rollout at 128^3 (checkpoint every 8), adjoint "
                        "gradient against central FD; learned128 = learned preconditioner "
                        "against MIC(0)-PCG at 128^3 (held-out masks)")
    p.add_argument("--summarize-trace", nargs=4, metavar=("TRACE_CSV", "OUT", "TITLE", "COMMAND"),
                   help="write a kernel-trace summary for profiles/ and exit (no GPU)")
    p.add_argument("--summarize-traffic", nargs=3, metavar=("RUN_CSV", "COPY_CSV", "PRECOND"),
                   help="write the per-kind traffic summaries for profiles/ and exit (no GPU)")
    p.add_argument("--summarize-counters", nargs=3, metavar=("COUNTER_CSV", "OUT", "TITLE"),
                   help="write a per-kernel MFMA / LDS counter summary for profiles/ and exit")
    p.add_argument("--commands", nargs="*", default=[],
                   help="the commands that produced the counter files (for --summarize-traffic)")
    p.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                   help="only run 20 plain device copies of MIB MiB (calibrates the HBM "
                        "byte counters) and exit")
    return p.parse_args()


def copy_probe(mib):
    """Twenty device-to-device copies of `mib` MiB with torch's copy kernel:
    the check of the HBM byte counters' readings."""
    import torch
    a = torch.ones(mib * (1 << 20) // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(20):
        b.copy_(a)
    torch.cuda.synchronize()
    log(f"copy probe: 20 copies of {mib} MiB")


def load_traffic(kind, n, precond):
    """HBM bytes per launch of `kind` at n^3 with this pressure
    preconditioner, from the committed counter summary; None when there is
    none or a kernel source changed since the counters were taken (the
    summary stores each source's SHA-256)."""
    import hashlib
    path = os.path.join(ROOT, "profiles", f"{kind}_{precond}_{n}_traffic.md")
    if not os.path.exists(path):
        return None
    rec = None
    with open(path) as f:
        for line in f:
            if line.startswith("bench-traffic:"):
                rec = json.loads(line.split(":", 1)[1])
    if not rec:
        return None
    for src, sha in rec["sources"].items():
        with open(os.path.join(ROOT, src), "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != sha:
                return None
    return rec["bytes_per_launch"]


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(n, seed):
    """The FP64 oracle on the bench step's unit of work: one forward step
    (advect, force, viscosity, projection to a 1e-6 relative residual) and
    one adjoint step of it (projection solve, viscosity adjoint, advection
    transpose, parameter terms), on one seed at n^3, timed on the host."""
    from oracle import fluid as orc
    from paper_2503_00868_amd import inputs
    cell, ug = inputs.gen_case(n, seed)
    nu = inputs.gen_nu(101)
    s = inputs.gen_scale(101)
    u0 = tuple(s * f for f in orc.mask_faces(cell, ug))
    orc.lib()
    t0 = time.perf_counter()
    u1, info = orc.step(cell, u0, nu, 1.0 / 120, tol=1e-6, diff_tol=1e-6)
    t_fwd = time.perf_counter() - t0
    lam = orc.loss_grad(cell, u1, u0)
    t0 = time.perf_counter()
    orc.step_adjoint(cell, u0, lam, nu, 1.0 / 120, tol=1e-6)
    t_adj = time.perf_counter() - t0
    dt = t_fwd + t_adj
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": n ** 3 / dt, "unit": "cell-steps/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"one forward step ({t_fwd:.1f} s: plain CG to 1e-6, {info.proj_iters} "
                      f"iterations, {'explicit' if info.explicit else 'implicit'} viscosity) and "
                      f"one adjoint step ({t_adj:.1f} s) of the FP64 oracle at {n}^3, seed {seed}; "
                      f"the headline is this unit at 256^3 (8x the cells, and about 2x the "
                      f"iterations per solve)"}


def rooflines(prof, n, precond, n_active):
    """Roofline of the kernel kind with the most time in the timed region
    (the U-Net against the BF16 MFMA peak, every other kind against HBM),
    and of the top HBM-bound kind.  n_active: active faces of the mask."""
    C, F3 = n ** 3, 3 * (n + 1) * n * n

    def hbm(kind):
        ms_tot, launches = prof[kind]
        if kind in FACE_BYTES:
            every, active = FACE_BYTES[kind]
            per_launch = every * F3 + active * n_active
        else:
            per_unit = BYTES_PER_UNIT[kind]
            if kind == "pcg_update" and precond == "mic0":
                per_unit = 33.0
            if kind == "pcg_update" and precond == "learned":
                per_unit = 17.75
            if kind == "pcg_dir_spmv" and precond == "learned":
                per_unit = 21.0  # z 4 + d 4 + r 4 (the flexible-CG dot) + diag 1 in; d 4 + q 4 out
            per_launch = per_unit * C
        avg_s = ms_tot / launches / 1e3
        achieved = per_launch / avg_s / 1e9
        return {"bound": "hbm", "kernel": kind, "achieved": round(achieved, 1),
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": load_traffic(kind, n, precond), "avg_us": round(avg_s * 1e6, 2),
                "launches": launches, "bytes_per_launch": per_launch}

    kinds = {k: v for k, v in prof.items() if (k in BYTES_PER_UNIT or k in FACE_BYTES) and v[1] > 0}
    r_hbm = hbm(max(kinds, key=lambda k: kinds[k][0]))
    net_ms, net_launches = prof.get("net", (0.0, 0))
    if net_launches and net_ms > max(v[0] for v in kinds.values()):
        avg_s = net_ms / net_launches / 1e3
        flop = NET_FLOP_PER_CELL * C
        achieved = flop / avg_s / 1e12
        return ({"bound": "mfma", "kernel": "net", "achieved": round(achieved, 1),
                 "peak": BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                 "frac": round(achieved / BF16_PEAK_TFLOPS, 4), "traffic": load_traffic("net", n, precond),
                 "avg_us": round(avg_s * 1e6, 1), "launches": net_launches,
                 "flop_per_launch": flop}, r_hbm)
    return r_hbm, None


def inputs_gen_case(n, seed):
    from paper_2503_00868_amd import inputs
    return inputs.gen_case(n, seed)


def percnn_bench(cell, ugen, nu, s, dt, g, dev, K):
    """The recurrent convolutional pressure solver on the benchmark's state:
    K layers with the Jacobi kernel from p = 0 (states recorded) and their
    reverse pass for the squared error against the projection's pressure,
    timed per layer with HIP events; plus the relative error reached."""
    import torch
    from paper_2503_00868_amd import percnn
    from paper_2503_00868_amd.fluidsim import Sim
    n = cell.shape[0]
    sim = Sim(cell, precond="jacobi", tol=1e-8, check_every=16, device=dev)
    sim.set_params(nu=nu, dt=dt, s=s, gravity=g)
    u = sim.faces()
    sim.init_state(ugen, u)
    a = sim.op_advect(u)
    b = sim.cells_tensor()
    sim.op_divergence(a, b)
    _, p_star = sim.project(tuple(x.clone() for x in a), want_p=True)
    p_star = p_star.to(torch.float32)
    L = percnn.liquid_mask(sim)
    w = percnn.jacobi_weights()
    hist = torch.empty((K + 1, n, n, n), dtype=torch.float32, device=dev)
    p0 = torch.zeros_like(b)
    sim.percnn_forward(w, 2, p0, b, hist=hist[:3])  # warm-up
    torch.cuda.synchronize()
    sim.profile_enable(True)
    t0 = time.perf_counter()
    sim.percnn_forward(w, K, p0, b, hist=hist)
    torch.cuda.synchronize()
    t_fwd = time.perf_counter() - t0
    err = L * (hist[K] - p_star)
    rel = float(torch.linalg.norm(err) / torch.linalg.norm(p_star))
    gK = (2.0 * err).contiguous()
    gp0, gb = torch.zeros_like(b), torch.zeros_like(b)
    t0 = time.perf_counter()
    sim.percnn_backward(w, K, b, hist, gK, gp0=gp0, gb=gb)
    t_bwd = time.perf_counter() - t0
    prof = sim.profile_read()
    sim.profile_enable(False)
    sim.close()
    del hist
    out = {"layers": K, "kernel": "jacobi", "rel_error_vs_projection": rel,
           "fwd_ms": round(t_fwd * 1e3, 2), "bwd_ms": round(t_bwd * 1e3, 2),
           "cell_layers_per_s": n ** 3 * K / t_fwd}
    for kind, bpc in PERCNN_BYTES.items():
        ms_tot, launches = prof[kind]
        avg_s = ms_tot / launches / 1e3
        achieved = bpc * n ** 3 / avg_s / 1e9
        out["roofline_" + kind] = {"bound": "hbm", "kernel": kind, "achieved": round(achieved, 1),
                                   "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                   "frac": round(achieved / HBM_PEAK_GBS, 4),
                                   "traffic": load_traffic(kind, n, "jacobi"),
                                   "avg_us": round(avg_s * 1e6, 2), "launches": launches,
                                   "bytes_per_launch": bpc * n ** 3}
    return out


def percnn_fitted_bench(cell, dev, weights, K=100, steps=60, layer_us=None):
    """The paper's recurrent convolutional solver with a fitted kernel (Section
    3.4.1): the kernel is fitted at the benchmark's size on (0, projection
    pressure, right-hand side) pairs of three seeded velocity fields, one
    sim_percnn_fit_step per Adam step; then, on a held-out field, the
    relative pressure error ||p - p*|| / ||p*|| against wall time for the
    fitted and the Jacobi kernels (K' layers at the measured time per layer),
    for the flexible CG with the network and for Jacobi-PCG (their iterates
    from sim_harvest_pairs, at the measured time per iteration)."""
    import torch
    from paper_2503_00868_amd import percnn
    from paper_2503_00868_amd.fluidsim import Sim
    n = cell.shape[0]
    sim = Sim(cell, precond="learned", tol=1e-8, check_every=4, device=dev)
    sim.net_set_weights(weights)
    seeds = [1000, 1001, 1002, 1003]
    pairs = percnn.make_pairs(sim, seeds)
    train, test = pairs[:3], pairs[3:]
    t0 = time.perf_counter()
    # Adam's first steps move every weight by about lr, and K layers compound
    # a change of the recurrence's spectral radius K times: the step size
    # falls as 1/K (2e-3 at K = 16, where fits at 32^3 and 64^3 converge)
    lr = 0.032 / K
    w, losses = percnn.fit(sim, train, K, steps=steps, lr=lr)
    torch.cuda.synchronize()
    t_fit = time.perf_counter() - t0
    wj = percnn.jacobi_weights()
    out = {"K_fit": K, "fit_steps": steps, "lr": lr, "fit_s": round(t_fit, 2), "loss_first": losses[0],
           "loss_last": losses[-1], "weights": [round(float(x), 5) for x in w]}
    # time per layer, per network-preconditioned CG iteration, per Jacobi-PCG iteration
    pb, pa, b = test[0]
    if layer_us is None:
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        sim.percnn_forward(w, 10, pb, b)
        ev[0].record()
        sim.percnn_forward(w, 100, pb, b)
        ev[1].record()
        torch.cuda.synchronize()
        layer_us = ev[0].elapsed_time(ev[1]) * 10.0
    # the held-out field's pre-projection velocity (as make_pairs builds it)
    _, ug = inputs_gen_case(n, seeds[-1])
    sim.set_params(nu=1e-4, dt=1.0 / 120, s=1.0)
    u = sim.faces()
    sim.init_state(sim.to_faces(ug), u)
    a = sim.op_advect(u)
    per_it = {}
    for pc in ("learned", "jacobi"):
        s2 = Sim(cell, precond=pc, tol=1e-6, check_every=4 if pc == "learned" else 16, device=dev)
        if pc == "learned":
            s2.net_set_weights(weights)
        uu = tuple(x.clone() for x in a)
        s2.project(tuple(x.clone() for x in a))  # warm-up
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        st, _ = s2.project(uu)
        torch.cuda.synchronize()
        per_it[pc] = (time.perf_counter() - t1) * 1e3 / max(st["iters"], 1)
        s2.close()
    L = percnn.liquid_mask(sim)
    norm = float(torch.linalg.norm(pa))
    curves = {"percnn_fitted": [], "percnn_jacobi": [], "fcg_learned": [], "pcg_jacobi": []}
    for Kp in (25, 50, 100, 200, 400, 800):
        for name, ww in (("percnn_fitted", w), ("percnn_jacobi", wj)):
            p = sim.percnn_forward(ww, Kp, pb, b)
            curves[name].append({"ms": round(Kp * layer_us * 1e-3, 3), "layers": Kp,
                                 "rel_error": float(torch.linalg.norm(L * (p - pa))) / norm})
    for name, mode, its in (("fcg_learned", 1, [1, 2, 4, 8, 16, 32]),
                            ("pcg_jacobi", 0, [2, 16, 64, 128, 256, 512])):
        hs = sim if mode == 1 else Sim(cell, precond="jacobi", device=dev)
        _, E, _ = hs.harvest_pairs(tuple(x.clone() for x in a), [0] + its, tol=1e-10, mode=mode)
        e0 = float(torch.linalg.norm(E[0]))
        key = "learned" if mode == 1 else "jacobi"
        for q, k in enumerate(its):
            curves[name].append({"ms": round(k * per_it[key], 3), "iters": k,
                                 "rel_error": float(torch.linalg.norm(E[q + 1])) / e0})
        del E
        if mode == 0:
            hs.close()
    out.update({"layer_us": round(layer_us, 2), "fcg_iter_ms": round(per_it["learned"], 3),
                "pcg_iter_ms": round(per_it["jacobi"], 4), "curves": curves})
    sim.close()
    return out


def constrained_bench(cell, ugen, nu, s, dt, g, dev, K):
    """The constrained divergence projection on the benchmark's advected
    state: K iterations without and with relaxation (eps = half the largest
    constraint-gradient norm), timed with HIP events on the library's
    stream, and the relative divergence left."""
    import torch
    from paper_2503_00868_amd.fluidsim import Sim
    n = cell.shape[0]
    sim = Sim(cell, precond="jacobi", device=dev)
    sim.set_params(nu=nu, dt=dt, s=s, gravity=g)
    u = sim.faces()
    sim.init_state(ugen, u)
    a = sim.op_advect(u)
    out = {"iters": K}
    for name, eps in (("eps0", 0.0), ("relaxed", 3.0 * n * n)):
        uu = tuple(x.clone() for x in a)
        sim.constrained_project(tuple(x.clone() for x in a), 2, eps)  # warm-up
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
        ev[0].record()
        rel = sim.constrained_project(uu, K, eps)
        ev[1].record()
        torch.cuda.synchronize()
        ms = ev[0].elapsed_time(ev[1])
        out[name] = {"eps": eps, "ms": round(ms, 2), "us_per_iter": round(ms / K * 1e3, 2),
                     "rel_divergence_left": rel}
    us = out["eps0"]["us_per_iter"]
    achieved = CONSTRAINED_BYTES * n ** 3 / (us * 1e-6) / 1e9
    out["roofline"] = {"bound": "hbm", "kernel": "constrained iteration (k_cp_lambda + k_pressure_update)",
                       "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": round(achieved / HBM_PEAK_GBS, 4),
                       "traffic": load_traffic("constrained", n, "jacobi"),
                       "avg_us": us, "bytes_per_iter": CONSTRAINED_BYTES * n ** 3}
    sim.close()
    return out


def upwind_bench(cell, ugen, nu, s, dt, g, dev, reps=10):
    """The paper's upwind convection gradient at the benchmark's state (the
    convected field after one advection, a seeded lambda), timed over `reps`
    calls with HIP events, with its HBM roofline."""
    import torch
    from paper_2503_00868_amd.fluidsim import Sim
    n = cell.shape[0]
    sim = Sim(cell, precond="jacobi", device=dev)
    sim.set_params(nu=nu, dt=dt, s=s, gravity=g)
    u = sim.faces()
    sim.init_state(ugen, u)
    a = sim.op_advect(u)
    gen = torch.Generator(device=dev).manual_seed(0)
    lam = tuple(torch.randn(x.shape, device=dev, generator=gen) for x in a)
    out = sim.faces()
    sim.op_convection_grad_upwind(a, lam, out)  # warm-up
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(reps):
        sim.op_convection_grad_upwind(a, lam, out)
    ev[1].record()
    torch.cuda.synchronize()
    us = ev[0].elapsed_time(ev[1]) / reps * 1e3
    faces = 3 * (n + 1) * n * n
    achieved = UPWIND_BYTES * faces / (us * 1e-6) / 1e9
    sim.close()
    return {"us_per_call": round(us, 2),
            "roofline": {"bound": "hbm", "kernel": "k_convection_grad_upwind",
                         "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(achieved / HBM_PEAK_GBS, 4),
                         "traffic": load_traffic("upwind", n, "jacobi"), "avg_us": round(us, 2),
                         "bytes_per_call": UPWIND_BYTES * faces}}


def loss_bench(cell, ugen, nu, s, dt, g, dev, reps=10):
    """The paper's masked cosine + L2 velocity loss and its gradient at the
    benchmark's state (the field after one advection against the initial
    one; weights 0.2 / 1 / 2 for empty / occupied / surface cells), timed
    over `reps` calls with HIP events (each call reads J back to the host),
    with its HBM roofline."""
    import torch
    from paper_2503_00868_amd.fluidsim import Sim
    n = cell.shape[0]
    sim = Sim(cell, precond="jacobi", device=dev)
    sim.set_params(nu=nu, dt=dt, s=s, gravity=g)
    u = sim.faces()
    sim.init_state(ugen, u)
    a = sim.op_advect(u)
    out = sim.faces()
    args = (1.0, 1.0, 1e-3, (0.2, 1.0, 2.0))
    J, _ = sim.loss_cos_l2(a, u, *args, out=out)  # warm-up
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ev[0].record()
    for _ in range(reps):
        sim.loss_cos_l2(a, u, *args, out=out)
    ev[1].record()
    torch.cuda.synchronize()
    us = ev[0].elapsed_time(ev[1]) / reps * 1e3
    cells = n ** 3
    achieved = LOSS_BYTES * cells / (us * 1e-6) / 1e9
    sim.close()
    return {"J": J, "us_per_call": round(us, 2),
            "roofline": {"bound": "hbm", "kernel": "k_loss_cells + k_loss_fold + k_loss_face_grad",
                         "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(achieved / HBM_PEAK_GBS, 4),
                         "traffic": load_traffic("loss", n, "jacobi"),
                         "avg_us": round(us, 2), "bytes_per_call": LOSS_BYTES * cells}}


# The screen-space constrained projection, per pixel and CG iteration: the
# direction + stencil kernel reads z 8, d 8, mask 1 and writes d 8, q 8; the
# update reads the mask and, on region pixels (fraction f), d 8, q 8, x 8,
# r 8 and writes x 8, r 8, z 8.
def screen_bytes_per_iter(f):
    return 33.0 + 1.0 + 56.0 * f


def screen_bench(dev, H=1080, W=1920, seed=7, reps=3, traffic_n=256):
    """The paper's screen-space constrained projection on a 1080 x 1920 frame
    of the seeded generator, to a 1e-9 relative residual: ms per call,
    iterations, and the HBM rate of its CG iterations."""
    import torch
    from paper_2503_00868_amd import inputs
    from paper_2503_00868_amd.fluidsim import screen_project
    a, b, vz, z, mask = inputs.gen_screen(H, W, seed)
    dv = lambda x: torch.as_tensor(x, device=dev)
    VZ, Z, M = dv(vz), dv(z), dv(mask)
    A0, B0 = dv(a), dv(b)
    A, B = A0.clone(), B0.clone()
    screen_project(A, B, VZ, Z, M, tol=1e-9)  # warm-up (also allocates the workspace once)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    ms = []
    for _ in range(reps):
        A.copy_(A0)
        B.copy_(B0)
        ev[0].record()
        it, rel = screen_project(A, B, VZ, Z, M, tol=1e-9)
        ev[1].record()
        torch.cuda.synchronize()
        ms.append(ev[0].elapsed_time(ev[1]))
    t = min(ms)
    f = float(mask.mean())
    per_iter_s = t * 1e-3 / max(it, 1)
    achieved = screen_bytes_per_iter(f) * H * W / per_iter_s / 1e9
    return {"H": H, "W": W, "region_fraction": round(f, 4), "iters": it, "rel_residual": rel,
            "ms_per_call": round(t, 3),
            "roofline": {"bound": "hbm", "kernel": "k_s2_dir_spmv + k_s2_update (+ 2 finalize)",
                         "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                         "frac": round(achieved / HBM_PEAK_GBS, 4),
                         "traffic": load_traffic("screen", traffic_n, "jacobi"),
                         "avg_us_per_iter": round(per_iter_s * 1e6, 2),
                         "bytes_per_iter": screen_bytes_per_iter(f) * H * W}}


def apic_bench(cell, dev, per_cell=8, reps=5):
    """The paper's APIC transfers at the benchmark's mask: `per_cell`
    particles jittered in every liquid cell (one cell from the walls), a
    smooth velocity field, C = 0; particles to grid (zero, scatter with FP32
    atomics, normalise) and grid to particles (gather, affine update, move),
    timed with HIP events, with their HBM rates: P2G moves 64 B per particle
    in and 24 B per face (mass and velocity, three components) out; G2P 12 B
    per particle in, 60 out, and 12 B per face in."""
    import torch
    from paper_2503_00868_amd.fluidsim import Sim
    n = cell.shape[0]
    sim = Sim(cell, precond="jacobi", device=dev)
    liq = torch.as_tensor(cell, device=dev)[1:-1, 1:-1, 1:-1] == 1
    k, j, i = torch.nonzero(liq, as_tuple=True)
    base = torch.stack([i + 1, j + 1, k + 1], -1).to(torch.float32)
    del liq, k, j, i
    gen = torch.Generator(device=dev).manual_seed(11)
    x = (base.repeat_interleave(per_cell, 0) +
         torch.rand((base.shape[0] * per_cell, 3), device=dev, generator=gen)) / n
    del base
    P = x.shape[0]
    v = torch.stack([torch.sin(6.0 * x[:, 1]), torch.cos(5.0 * x[:, 2]), 0.5 * torch.sin(4.0 * x[:, 0])], -1)
    C = torch.zeros((P, 3, 3), dtype=torch.float32, device=dev)
    m = torch.ones(P, dtype=torch.float32, device=dev)
    grid, mass = sim.faces(), sim.faces()
    vp, Cp = torch.empty_like(v), torch.empty_like(C)
    xm = x.clone()
    sim.apic_p2g(x, v, C, m, out=grid, mass=mass)  # warm-up
    sim.apic_g2p(grid, xm, 0.0, vp=vp, C=Cp)
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ev[0].record()
    for _ in range(reps):
        sim.apic_p2g(x, v, C, m, out=grid, mass=mass)
    ev[1].record()
    for _ in range(reps):
        sim.apic_g2p(grid, xm, 0.0, vp=vp, C=Cp)
    ev[2].record()
    torch.cuda.synchronize()
    p2g_us = ev[0].elapsed_time(ev[1]) / reps * 1e3
    g2p_us = ev[1].elapsed_time(ev[2]) / reps * 1e3
    F = (n + 1) * n * n
    p2g_bytes = 64.0 * P + 24.0 * F
    g2p_bytes = 72.0 * P + 12.0 * F
    sim.close()

    def rl(name, kind, byts, us):
        ach = byts / (us * 1e-6) / 1e9
        return {"bound": "hbm", "kernel": name, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4),
                "traffic": load_traffic(kind, n, "jacobi") if per_cell == 8 else None,
                "avg_us": round(us, 2), "bytes_per_call": byts}
    return {"particles": P, "per_liquid_cell": per_cell, "p2g_us": round(p2g_us, 1),
            "g2p_us": round(g2p_us, 1),
            "p2g_particles_per_s": P / (p2g_us * 1e-6),
            "g2p_particles_per_s": P / (g2p_us * 1e-6),
            "roofline_p2g": rl("k_apic_zero + k_apic_p2g + k_apic_normalize", "apic_p2g", p2g_bytes,
                               p2g_us),
            "roofline_g2p": rl("k_apic_g2p", "apic_g2p", g2p_bytes, g2p_us)}


def fd_gradient(sim, ugen, target, nu, s, dt, g, T, h=1e-3):
    """Central FD of J in theta_nu = log nu and theta_s = log s (h = 1e-3),
    from forward-only rollouts of `sim`."""
    def J(tn, ts):
        sim.set_params(nu=math.exp(tn), dt=dt, s=math.exp(ts), gravity=g)
        u = sim.faces()
        sim.init_state(ugen, u)
        sim.step(u, T)
        return sim.loss_mse(u, target, want_grad=False)[0]
    a, b = math.log(nu), math.log(s)
    return {"dtheta_nu": (J(a + h, b) - J(a - h, b)) / (2 * h),
            "dtheta_s": (J(a, b + h) - J(a, b - h)) / (2 * h)}


def adjoint_gradient(sim, ugen, target, nu, s, dt, g, T):
    sim.set_params(nu=nu, dt=dt, s=s, gravity=g)
    u = sim.faces()
    sim.init_state(ugen, u)
    sim.step(u, T, record=True)
    J, gT = sim.loss_mse(u, target)
    _, gr, st = sim.backward(gT, ugen=ugen, full=True)
    return {"J": J, "dtheta_nu": nu * gr["nu"], "dtheta_s": s * gr["s"], "dJ_ddt": gr["dt"],
            "dJ_dg": list(gr["gravity"]), "adjoint_iters": st["iters"]}


def _rel(a, b):
    return abs(a - b) / abs(b) if b != 0 else float("inf")


# ------------------------------------------------------------------ profiles
# Summaries of rocprofv3 output for profiles/: the per-kind kernel patterns,
# and the sources each kind's counters depend on (a summary whose sources
# changed is no longer read).

TRAFFIC_KINDS = {
    # kind: (precond the run used, kernel name patterns, sources)
    "pcg_dir_spmv": {"jacobi": ["k_dir_spmv_zm<0, false>"], "learned": ["k_dir_spmv_zm<1, true>"]},
    # (prefixes: the names carry the update's last template argument too)
    "pcg_update": {"jacobi": ["k_update4<4, true, false", "k_update4<4, false, false"],
                   "learned": ["k_update4<4, true, true", "k_update4<4, false, true"]},
    "pcg_check": {"jacobi": ["k_check_zm<0>"], "learned": ["k_check_zm<1>"]},
    "dcg_dir_spmv": {"learned": ["k_dcg_dir_spmv_zm"]},
    "dcg_update": {"learned": ["k_dcg_update"]},
    "net": {"learned": ["k_conv_in", "k_conv_zm", "k_upconv", "k_conv_out", "k_conv<",
                        "k_convILi", "k_conv_cat", "k_dot_cells"]},
    "percnn": {"jacobi": ["k_percnn_layer("]},
    "percnn_adj": {"jacobi": ["k_percnn_layer_adj"]},
    "upwind": {"jacobi": ["k_convection_grad_upwind"]},
    "advect": {"learned": ["k_advect("]},
    "advect_adjoint": {"learned": ["k_advect_adjoint"]},
    "constrained": {"jacobi": ["k_cp_lambda", "k_pressure_update"]},
    "loss": {"jacobi": ["k_loss_cells", "k_loss_fold", "k_loss_face_grad"]},
    "screen": {"jacobi": ["k_s2_dir_spmv", "k_s2_update"]},
    "apic_p2g": {"jacobi": ["k_apic_zero", "k_apic_p2g", "k_apic_normalize"]},
    "apic_g2p": {"jacobi": ["k_apic_g2p"]},
}
TRAFFIC_SOURCES = {
    "pcg_dir_spmv": ["k_pcg.hip", "common.h"], "pcg_update": ["k_pcg.hip", "common.h"],
    "pcg_check": ["k_pcg.hip", "common.h"], "dcg_dir_spmv": ["k_pcg.hip", "common.h"],
    "dcg_update": ["k_pcg.hip", "common.h"],
    "net": ["k_conv_zm.hip", "k_conv_in.hip", "k_conv_out.hip", "k_upconv.hip", "k_unet.hip",
            "net.cpp", "common.h", "block_or.h"],
    "percnn": ["k_percnn.hip"], "percnn_adj": ["k_percnn.hip"], "upwind": ["upwind.hip"],
    "advect": ["k_step.hip", "common.h"], "advect_adjoint": ["k_step.hip", "common.h"],
    "constrained": ["constrained.hip", "common.h"], "loss": ["loss.hip", "common.h"],
    "screen": ["screen2d.hip", "common.h"], "apic_p2g": ["apic.hip"], "apic_g2p": ["apic.hip"],
}
# Counter passes the summaries read: the L2's read and write requests to the
# memory side in 32-byte units (a 64-byte request counts 2, a 128-byte read 4),
# so bytes = 32 x count with no assumption about request sizes; both fit one
# pass (two TCC counters).
DRAM_READ = "TCC_EA0_RDREQ_DRAM_32B_sum"
DRAM_WRITE = "TCC_EA0_WRREQ_WRITE_DRAM_32B_sum"


def _rows(path):
    import csv
    with open(path) as f:
        return list(csv.DictReader(f))


def _demangle(name):
    """A readable kernel name: strip argument lists of plain names (keeping
    the names of kernels in anonymous namespaces)."""
    name = name.replace("(anonymous namespace)::", "")
    return name.split("(")[0] if "(" in name else name


def _matches(name, pats):
    return any(p in name for p in pats)


def summarize_trace(trace_csv, out, title, command, net_launch_ratio=None):
    """Markdown summary of a rocprofv3 --kernel-trace run (per-dispatch CSV):
    per kernel the calls, total, and the average over the dispatches that did
    work (longer than 5% of the kernel's longest; dispatches of a solve that
    had already converged return at once), and the network's time per working
    application (the sum of its kernels' working averages)."""
    import collections
    rows = _rows(trace_csv)
    dur = collections.defaultdict(list)
    for r in rows:
        dur[r["Kernel_Name"]].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3)
    total_all = sum(sum(v) for v in dur.values())
    table = []
    for k, v in dur.items():
        mx = max(v)
        work = [d for d in v if d >= 0.05 * mx]
        table.append((sum(v), k, len(v), len(work), sum(work) / len(work), min(v), mx))
    table.sort(reverse=True)
    net_pats = TRAFFIC_KINDS["net"]["learned"]
    net_us = sum(t[4] for t in table if _matches(t[1], net_pats))
    lines = [f"# Kernel trace: {title}", "",
             "Command (repository root on one MI355X; `cd /tmp && export TMPDIR=/tmp` first, "
             "R = repository path):", "", "```", command, "```", "",
             "Per kernel: calls, total time, and the average over the dispatches that did work "
             "(longer than 5% of the kernel's longest: the CG kernels and the network return at "
             "once when the solve has already converged).", "",
             "| kernel | calls | working | total ms | avg us (working) | min us | max us | % |",
             "|---|---:|---:|---:|---:|---:|---:|---:|"]
    for tot, k, calls, nw, avg, mn, mx in table[:40]:
        lines.append(f"| `{_demangle(k)}` | {calls} | {nw} | {tot / 1e3:.1f} | {avg:.2f} | "
                     f"{mn:.2f} | {mx:.2f} | {100 * tot / total_all:.2f} |")
    lines += ["", f"The network's kernels per working application add up to **{net_us:.1f} us** "
              "(one dispatch of each per application)."]
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(f"wrote {out}; network {net_us:.1f} us per application")


def _counter_by_dispatch(path, counter):
    out = {}
    for r in _rows(path):
        if r["Counter_Name"] != counter:
            continue
        d = r["Dispatch_Id"]
        out.setdefault(d, [r["Kernel_Name"], 0.0])
        out[d][1] += float(r["Counter_Value"])
    return out


def summarize_traffic(run_csv, copy_csv, precond, n, commands, out_dir, copy_mib=1024, seed=4):
    """Per-kind HBM traffic summaries from one counter pass over a bench run
    (DRAM_READ and DRAM_WRITE per dispatch, 32-byte units), averaged over the
    working dispatches (above 5% of the kernel's largest reading), with the
    same counters' reading for plain copies of copy_mib MiB as the check of
    the byte count, and the SHA-256 of the sources each kind depends on."""
    import hashlib
    rd = _counter_by_dispatch(run_csv, DRAM_READ)
    wr = _counter_by_dispatch(run_csv, DRAM_WRITE)
    crd = sorted(v for _, v in _counter_by_dispatch(copy_csv, DRAM_READ).values())[-20:]
    cwr = sorted(v for _, v in _counter_by_dispatch(copy_csv, DRAM_WRITE).values())[-20:]
    copy_bytes = copy_mib * (1 << 20)
    copy_r = 32.0 * sum(crd) / len(crd) / copy_bytes
    copy_w = 32.0 * sum(cwr) / len(cwr) / copy_bytes
    C, F3 = n ** 3, 3 * (n + 1) * n * n
    n_active = None
    written = []
    for kind, per in TRAFFIC_KINDS.items():
        pats = per.get(precond)
        if not pats:
            continue

        def per_kernel(table):
            acc = {}
            for name, v in table.values():
                if _matches(name, pats):
                    acc.setdefault(name, []).append(32.0 * v)
            res = {}
            for name, vs in acc.items():
                mx = max(vs)
                w = [x for x in vs if x >= 0.05 * mx]
                res[name] = (len(w), sum(w) / len(w))
            return res
        kr, kw = per_kernel(rd), per_kernel(wr)
        if not kr:
            continue
        rows, tot_r, tot_w = [], 0.0, 0.0
        for name in sorted(kr):
            nr, ar = kr[name]
            nw, aw = kw.get(name, (0, 0.0))
            share = 1.0
            if kind == "pcg_update":  # one dispatch in four updates the FP64 iterate
                share = 0.25 if "true" in name.split(",")[1] else 0.75
            tot_r += share * ar
            tot_w += share * aw
            rows.append(f"| `{_demangle(name)}` | {nr} | {ar / 1e6:.1f} | {aw / 1e6:.1f} | "
                        f"{(ar + aw) / 1e6:.1f} |")
        alg = None
        if kind in BYTES_PER_UNIT:
            per_unit = BYTES_PER_UNIT[kind]
            if kind == "pcg_dir_spmv" and precond == "learned":
                per_unit = 21.0
            if kind == "pcg_update" and precond == "learned":
                per_unit = 17.75
            alg = per_unit * C
        elif kind in FACE_BYTES:
            if n_active is None:
                from paper_2503_00868_amd import inputs
                n_active = active_faces(inputs.gen_mask(n, seed))
            every, active = FACE_BYTES[kind]
            alg = every * F3 + active * n_active
        else:
            alg = {"percnn": PERCNN_BYTES["percnn"] * C, "percnn_adj": PERCNN_BYTES["percnn_adj"] * C,
                   "upwind": UPWIND_BYTES * F3, "loss": LOSS_BYTES * C}.get(kind)
        srcs = {f"paper_2503_00868_amd/csrc/{f}": hashlib.sha256(
            open(os.path.join(ROOT, "paper_2503_00868_amd", "csrc", f), "rb").read()).hexdigest()
            for f in TRAFFIC_SOURCES[kind]}
        total = tot_r + tot_w
        unit = {"screen": "iteration (direction + stencil, update)", "apic_p2g": "call",
                "apic_g2p": "call", "loss": "call", "constrained": "iteration (multipliers, pressure update)"
                }.get(kind, "launch")
        lines = [f"# HBM traffic: `{kind}` at {n}^3 ({precond} run)", "",
                 "Commands (repository root on one MI355X; `cd /tmp && export TMPDIR=/tmp` first, "
                 "R = repository path):", "", "```"] + commands + [
                 "```", "",
                 f"Counters: `{DRAM_READ}` and `{DRAM_WRITE}`, the L2's read and write requests "
                 "to the memory side in 32-byte units (a 64-byte request counts 2, a 128-byte "
                 "read 4); bytes = 32 x count.  The same pass over 20 plain copies of "
                 f"{copy_mib} MiB reads {copy_r:.3f} x the bytes copied and writes {copy_w:.3f} x "
                 "(the check of the count).  Averages are over the dispatches that did work "
                 "(above 5% of the kernel's largest reading).", "",
                 "| kernel | working dispatches | read MB | written MB | MB |",
                 "|---|---:|---:|---:|---:|"] + rows + [
                 "", f"Per {unit} of the `{kind}` kind: **{total / 1e6:.1f} MB** "
                 f"(reads {tot_r / 1e6:.1f} MB, writes {tot_w / 1e6:.1f} MB)"
                 + (f" against {alg / 1e6:.1f} MB algorithmic ({total / alg:.2f}x)." if alg else "."),
                 "", "bench-traffic: " + json.dumps({"kind": kind, "precond": precond, "n": n,
                                                     "bytes_per_launch": int(total),
                                                     "read_bytes": int(tot_r),
                                                     "write_bytes": int(tot_w),
                                                     "algorithmic_bytes": int(alg) if alg else None,
                                                     "copy_check": [round(copy_r, 4), round(copy_w, 4)],
                                                     "sources": srcs})]
        path = os.path.join(out_dir, f"{kind}_{precond}_{n}_traffic.md")
        with open(path, "w") as f:
            f.write("\n".join(lines) + "\n")
        written.append(path)
        print(f"wrote {path}: {total / 1e6:.1f} MB per {unit}")
    return written


def summarize_counters(csv_path, out, title, commands, cu_num=256, simd_per_cu=4, xcc=8):
    """Per-kernel MFMA and LDS utilisation from one rocprofv3 --pmc pass with
    SQ_VALU_MFMA_BUSY_CYCLES, GRBM_GUI_ACTIVE, SQ_LDS_IDX_ACTIVE,
    SQ_LDS_BANK_CONFLICT, SQ_INSTS_MFMA, SQ_INSTS_LDS, SQ_INSTS_VALU and
    SQ_WAVE_CYCLES: MFMA busy = MFMA-busy cycles over (GPU-active cycles x
    SIMDs), LDS active = LDS-busy cycles over (GPU-active cycles x CUs), bank
    conflicts as a share of the LDS-busy cycles; averages over the working
    dispatches (GPU-active cycles above 5% of the kernel's longest).
    GRBM_GUI_ACTIVE comes summed over the xcc XCDs, each of which counts the
    dispatch's active cycles."""
    import collections
    per = collections.defaultdict(lambda: collections.defaultdict(float))
    names = {}
    for r in _rows(csv_path):
        d = r["Dispatch_Id"]
        names[d] = r["Kernel_Name"]
        per[d][r["Counter_Name"]] += float(r["Counter_Value"])
    by_kernel = collections.defaultdict(list)
    for d, cs in per.items():
        by_kernel[names[d]].append(cs)
    rows = []
    for k, lst in by_kernel.items():
        mx = max(c.get("GRBM_GUI_ACTIVE", 0.0) for c in lst)
        w = [c for c in lst if c.get("GRBM_GUI_ACTIVE", 0.0) >= 0.05 * mx]
        if not w or mx <= 0:
            continue
        avg = {key: sum(c.get(key, 0.0) for c in w) / len(w) for key in w[0]}
        gui = avg["GRBM_GUI_ACTIVE"] / xcc
        mfma = 100.0 * avg.get("SQ_VALU_MFMA_BUSY_CYCLES", 0.0) / (gui * cu_num * simd_per_cu)
        lds = 100.0 * avg.get("SQ_LDS_IDX_ACTIVE", 0.0) / (gui * cu_num)
        bc = avg.get("SQ_LDS_BANK_CONFLICT", 0.0)
        conf = 100.0 * bc / avg["SQ_LDS_IDX_ACTIVE"] if avg.get("SQ_LDS_IDX_ACTIVE") else 0.0
        valu_per_mfma = (avg.get("SQ_INSTS_VALU", 0.0) / avg["SQ_INSTS_MFMA"]
                         if avg.get("SQ_INSTS_MFMA") else float("nan"))
        lds_per_mfma = (avg.get("SQ_INSTS_LDS", 0.0) / avg["SQ_INSTS_MFMA"]
                        if avg.get("SQ_INSTS_MFMA") else float("nan"))
        rows.append((gui, _demangle(k), len(w), mfma, lds, conf, valu_per_mfma, lds_per_mfma))
    rows.sort(reverse=True)
    lines = [f"# Counters: {title}", "",
             "Commands (repository root on one MI355X; `cd /tmp && export TMPDIR=/tmp` first, "
             "R = repository path):", "", "```"] + list(commands) + ["```", "",
             "MFMA busy: `SQ_VALU_MFMA_BUSY_CYCLES` / (active cycles x 1024 SIMDs); LDS active: "
             "`SQ_LDS_IDX_ACTIVE` / (active cycles x 256 CUs), active cycles = `GRBM_GUI_ACTIVE` "
             "/ 8 (the counter comes summed over the 8 XCDs); bank conflicts: "
             "`SQ_LDS_BANK_CONFLICT` / `SQ_LDS_IDX_ACTIVE`; instruction ratios from `SQ_INSTS_*` "
             "(VALU counts the MFMAs too).  Averages over the working dispatches.", "",
             "| kernel | dispatches | GPU-active cycles | MFMA busy % | LDS active % | "
             "bank-conflict % of LDS cycles | VALU / MFMA | LDS / MFMA |",
             "|---|---:|---:|---:|---:|---:|---:|---:|"]
    for gui, k, nw, mfma, lds, conf, vpm, lpm in rows:
        lines.append(f"| `{k}` | {nw} | {gui:.0f} | {mfma:.1f} | {lds:.1f} | {conf:.1f} | "
                     f"{vpm:.2f} | {lpm:.2f} |")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")
    print(f"wrote {out}")


def workload_128(args, dev, weights):
    """The smaller workloads at 128^3 (one JSON line each; not the benchmark).

    forward128: 16 steps of the forward step with MIC(0)-PCG to 1e-6 on the
    seed's mask and velocity, nu drawn log-uniformly from [1e-4, 1e-1] for the
    seed (implicit viscosity when nu dt / h^2 > 1/12), timed after a warmup,
    with every HBM kind's roofline from the timing hooks and the FP64 oracle's
    forward step on the same state timed on the host.
    grad128: a 32-step differentiable rollout (checkpoint every 8, MSE against
    a target from (nu*, s*)), the adjoint's dJ/dtheta_nu and dJ/dtheta_s (exact
    and upwind convection gradients) against central FD with h = 1e-3 in
    theta = log(param), solves to 1e-7.
    learned128: one cold projection per held-out mask (seeds 900..903, state
    after one step) with the learned preconditioner and with MIC(0)-PCG, and
    the 16-step rollout of forward128 with each: iterations and wall time."""
    import numpy as np
    import torch

    from paper_2503_00868_amd import inputs
    from paper_2503_00868_amd.fluidsim import Sim

    n, dt, g = 128, 1.0 / 120, (0.0, -9.8, 0.0)
    seed = args.seed
    cell, ug = inputs.gen_case(n, seed)
    nu = inputs.gen_nu(seed)
    lam = nu * dt * n * n
    out = {"workload": args.workload, "n": n, "seed": seed, "nu": nu,
           "viscosity": "explicit" if lam <= 1.0 / 12 else "implicit",
           "liquid_fraction": round(inputs.liquid_fraction(cell), 4), "dtype": "f32 (FP64 iterate, dots and residual)",
           "data": "synthetic (seeded slab + ellipsoids mask, curl-of-potential velocity)"}

    def rollout_time(pc, steps, on_cell=cell, on_ug=ug, profile=False):
        s = Sim(on_cell, precond=pc, tol=1e-6, diff_tol=1e-6, max_iter=20000,
                check_every=4 if pc != "jacobi" else 16, warm_start=True, device=dev)
        if pc == "learned":
            s.net_set_weights(weights)
        s.set_params(nu=nu, dt=dt, s=1.0, gravity=g)
        ugen = s.to_faces(on_ug)
        u = s.faces()
        s.init_state(ugen, u)
        s.step(u, 2)
        s.init_state(ugen, u)
        torch.cuda.synchronize()
        if profile:
            s.profile_enable(True)
        t0 = time.perf_counter()
        st = s.step(u, steps)
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        prof = s.profile_read() if profile else None
        s.close()
        return el, st, prof

    if args.workload == "forward128":
        el, st, prof = rollout_time("mic0", 16, profile=True)
        out["precond"] = "mic0"
        out["steps"] = 16
        out["ms"] = round(el * 1e3, 1)
        out["value"] = n ** 3 * 16 / el
        out["unit"] = "cell-steps/s"
        out["pressure_iters_mean"] = float(np.mean([q["iters"] for q in st]))
        n_active = active_faces(cell)
        out["rooflines"] = {}
        for k, v in prof.items():
            if v[1] > 0 and (k in BYTES_PER_UNIT or k in FACE_BYTES):
                r1, _ = rooflines({k: v}, n, "mic0", n_active)
                out["rooflines"][k] = {q: r1[q] for q in ("achieved", "frac", "avg_us", "launches",
                                                         "bytes_per_launch")}
        out["kernel_ms"] = {k: round(v[0], 2) for k, v in prof.items() if v[1]}
        log(f"forward128: {el * 1e3:.1f} ms for 16 steps, {out['value']:.3e} cell-steps/s, "
            f"{out['pressure_iters_mean']:.1f} MIC(0) iterations per projection")
        if not args.no_cpu_baseline:
            from oracle import fluid as orc
            u0 = orc.mask_faces(cell, ug)
            orc.lib()
            t0 = time.perf_counter()
            _, info = orc.step(cell, u0, nu, dt, tol=1e-6, diff_tol=1e-6)
            t_f = time.perf_counter() - t0
            threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
            out["cpu_baseline"] = {"value": n ** 3 / t_f, "unit": "cell-steps/s", "cores": threads,
                                   "kind": "oracle", "cpu_model": cpu_model(),
                                   "sample": f"one forward step of the FP64 oracle at {n}^3 from the "
                                             f"same state ({t_f:.1f} s; plain CG to 1e-6, "
                                             f"{info.proj_iters} iterations)"}
            log(f"oracle forward step: {t_f:.1f} s")
    elif args.workload == "grad128":
        T, K = 32, 8
        nu_t, s_t = inputs.gen_nu(100), inputs.gen_scale(100)
        nu_e, s_e = inputs.gen_nu(101), inputs.gen_scale(101)
        tsim = Sim(cell, precond="jacobi", tol=1e-7, diff_tol=1e-7, max_iter=20000,
                   check_every=16, warm_start=True, device=dev)
        ugen = tsim.to_faces(ug)
        tsim.set_params(nu=nu_t, dt=dt, s=s_t, gravity=g)
        target = tsim.faces()
        tsim.init_state(ugen, target)
        tsim.step(target, T)
        torch.cuda.synchronize()
        tsim.close()
        out.update({"rollout": T, "checkpoint_every": K, "nu_eval": nu_e, "s_eval": s_e,
                    "target": {"nu": nu_t, "s": s_t}, "tol": 1e-7, "fd_h": 1e-3, "precond": "mic0"})
        for conv in ("exact", "upwind"):
            gs = Sim(cell, precond="mic0", tol=1e-7, diff_tol=1e-7, max_iter=20000, check_every=4,
                     checkpoint_every=K, max_steps=T, warm_start=True, store_pressures=False,
                     convection_grad=conv, device=dev)
            t0 = time.perf_counter()
            out[conv] = adjoint_gradient(gs, ugen, target, nu_e, s_e, dt, g, T)
            torch.cuda.synchronize()
            out[conv]["ms_forward_backward"] = round((time.perf_counter() - t0) * 1e3, 1)
            if conv == "exact":
                out["fd"] = fd_gradient(gs, ugen, target, nu_e, s_e, dt, g, T)
            gs.close()
        for conv in ("exact", "upwind"):
            for key in ("dtheta_nu", "dtheta_s"):
                out[conv]["rel_err_" + key] = _rel(out[conv][key], out["fd"][key])
        log(f"grad128: FD {out['fd']}; exact {out['exact']['dtheta_nu']:.5e} "
            f"{out['exact']['dtheta_s']:.5e}; upwind {out['upwind']['dtheta_nu']:.5e} "
            f"{out['upwind']['dtheta_s']:.5e}")
    else:
        if weights is None:
            raise SystemExit("learned128 needs the trained weights")
        proj = []
        for hs in range(900, 904):
            hcell, hug = inputs.gen_case(n, hs)
            row = {"seed": hs}
            for pc in ("learned", "mic0"):
                s = Sim(hcell, precond=pc, tol=1e-6, max_iter=20000, check_every=4, device=dev)
                if pc == "learned":
                    s.net_set_weights(weights)
                s.set_params(nu=nu, dt=dt, s=1.0, gravity=g)
                ugen = s.to_faces(hug)
                u = s.faces()
                s.init_state(ugen, u)
                s.step(u, 1)
                s.project(u)  # warm the code path; the timed solve starts cold below
                s.init_state(ugen, u)
                s.step(u, 1)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                st, _ = s.project(u)
                torch.cuda.synchronize()
                row[pc] = {"ms": round((time.perf_counter() - t0) * 1e3, 2), "iters": st["iters"],
                           "rel_residual": st["rel_residual"]}
                s.close()
            log(f"learned128 seed {hs}: learned {row['learned']}, mic0 {row['mic0']}")
            proj.append(row)
        out["projections"] = proj
        out["rollout16"] = {}
        for pc in ("learned", "mic0"):
            el, st, _ = rollout_time(pc, 16)
            out["rollout16"][pc] = {"ms": round(el * 1e3, 1),
                                    "pressure_iters_mean": float(np.mean([q["iters"] for q in st]))}
            log(f"learned128 rollout with {pc}: {el * 1e3:.1f} ms")
        out["rollout16"]["learned_over_mic0"] = (out["rollout16"]["mic0"]["ms"] /
                                                 out["rollout16"]["learned"]["ms"])
    print(json.dumps(out), flush=True)


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU "
              "decomposition is a design note, not built.", file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.summarize_trace:
        summarize_trace(*args.summarize_trace)
        return
    if args.summarize_counters:
        summarize_counters(*args.summarize_counters, args.commands)
        return
    if args.summarize_traffic:
        rc, cc, pc = args.summarize_traffic
        summarize_traffic(rc, cc, pc, args.n, args.commands, os.path.join(ROOT, "profiles"))
        return
    import numpy as np
    import torch

    from paper_2503_00868_amd import inputs
    from paper_2503_00868_amd.fluidsim import Sim

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    n, T, K = args.n, args.rollout, args.checkpoint
    dt = 1.0 / 120
    g = (0.0, -9.8, 0.0)

    precond = args.precond
    weights = None
    if precond in ("auto", "learned"):
        if os.path.exists(args.weights):
            from paper_2503_00868_amd import unet
            weights = unet.load_weights(args.weights, dev)
            precond = "learned"
        elif precond == "learned":
            raise SystemExit(f"no trained weights at {args.weights}")
        else:
            precond = "jacobi"
    if args.workload != "rollout":
        workload_128(args, dev, weights)
        return
    log(f"n={n} rollout={T} checkpoint={K} precond={precond}")

    cell, ug = inputs.gen_case(n, args.seed)
    nu_t, s_t = inputs.gen_nu(100), inputs.gen_scale(100)
    nu_e, s_e = inputs.gen_nu(101), inputs.gen_scale(101)
    log(f"liquid fraction {inputs.liquid_fraction(cell):.3f}; nu*={nu_t:.3e} s*={s_t:.3f}; "
        f"eval nu={nu_e:.3e} s={s_e:.3f}")

    def check_period(pc):
        return args.check_every or (16 if pc == "jacobi" else 4)

    def make_sim(pc, on_cell=None, history=None, conv="exact", tol=1e-6, steps=None):
        s = Sim(cell if on_cell is None else on_cell, precond=pc, tol=tol, diff_tol=tol,
                max_iter=20000, check_every=check_period(pc), checkpoint_every=K,
                max_steps=T if steps is None else steps, warm_start=not args.cold,
                store_pressures=(not args.no_pressure_history) if history is None else history,
                convection_grad=conv, device=dev)
        if pc == "learned":
            s.net_set_weights(weights)
        return s

    def make_target(on_cell, steps):
        tsim = Sim(on_cell, precond="jacobi", tol=1e-6, diff_tol=1e-6, max_iter=20000,
                   check_every=16, warm_start=True, device=dev)
        ug_dev = tsim.to_faces(inputs.gen_velocity(n, args.seed) if on_cell is cell else
                               inputs.gen_case(n, args.heldout_seed)[1])
        tsim.set_params(nu=nu_t, dt=dt, s=s_t, gravity=g)
        tgt = tsim.faces()
        tsim.init_state(ug_dev, tgt)
        tsim.step(tgt, steps)
        torch.cuda.synchronize()
        tsim.close()
        return ug_dev, tgt

    if args.grad_table:
        rows = []
        for TT in [int(x) for x in args.grad_table.split(",")]:
            ugen_t, tgt = make_target(cell, TT)
            row = {"rollout": TT}
            for conv in ("exact", "upwind"):
                gs = make_sim(precond, history=True, conv=conv, tol=1e-7, steps=TT)
                row[conv] = adjoint_gradient(gs, ugen_t, tgt, nu_e, s_e, dt, g, TT)
                if conv == "exact":
                    row["fd"] = fd_gradient(gs, ugen_t, tgt, nu_e, s_e, dt, g, TT)
                gs.close()
                del gs
            for conv in ("exact", "upwind"):
                for key in ("dtheta_nu", "dtheta_s"):
                    row[conv]["rel_err_" + key] = _rel(row[conv][key], row["fd"][key])
            log(f"grad table T={TT}: FD {row['fd']}; exact {row['exact']['dtheta_nu']:.4e} "
                f"{row['exact']['dtheta_s']:.4e}; upwind {row['upwind']['dtheta_nu']:.4e} "
                f"{row['upwind']['dtheta_s']:.4e}")
            rows.append(row)
            del tgt, ugen_t
        print(json.dumps({"grad_table": rows, "n": n, "precond": precond, "tol": 1e-7,
                          "seed": args.seed}), flush=True)
        return

    # target rollout (untimed setup; the target does not depend on the
    # preconditioner, so the fastest plain one computes it)
    tsim = Sim(cell, precond="jacobi", tol=1e-6, diff_tol=1e-6, max_iter=20000, check_every=16,
               warm_start=True, device=dev)
    ugen = tsim.to_faces(ug)
    tsim.set_params(nu=nu_t, dt=dt, s=s_t, gravity=g)
    target = tsim.faces()
    tsim.init_state(ugen, target)
    tsim.step(target, T)
    torch.cuda.synchronize()
    tsim.close()
    del tsim
    log("target rollout done")

    torch.cuda.reset_peak_memory_stats(dev)
    sim = make_sim(precond)
    u = sim.faces()

    def bench_step(rollout):
        sim.set_params(nu=nu_e, dt=dt, s=s_e, gravity=g)
        sim.init_state(ugen, u)
        st = sim.step(u, rollout, record=True)
        log(f"forward rollout of {rollout} steps done")  # progress line (host only)
        J, gT = sim.loss_mse(u, target)
        _, dnu, ds, bst = sim.backward(gT, ugen=ugen)
        return st, bst, J, dnu, ds

    for _ in range(args.warmup):
        bench_step(args.warmup_rollout)
    torch.cuda.synchronize()
    log("warmup done")

    sim.profile_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fwd_stats, bwd_stats = [], []
    for _ in range(args.steps):
        st, bst, J, dnu, ds = bench_step(T)
        fwd_stats += st
        bwd_stats.append(bst)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    prof = sim.profile_read()
    sim.profile_enable(False)
    peak_mem = torch.cuda.max_memory_allocated(dev)
    ws_bytes = sim.ws.numel()

    ms_per_step = elapsed * 1e3 / args.steps
    value = n ** 3 * T / (elapsed / args.steps)
    fwd_iters = [s["iters"] for s in fwd_stats]
    log(f"{ms_per_step:.1f} ms per bench step; {value:.3e} cell-steps/s; pressure iters "
        f"fwd mean {np.mean(fwd_iters):.1f}; adjoint iters {bwd_stats[-1]['iters']}; J={J:.4e} "
        f"dJ/dnu={dnu:.4e} dJ/ds={ds:.4e}")

    n_active = active_faces(cell)
    roofline, roofline_hbm = rooflines(prof, n, precond, n_active)
    # every HBM kind of the timed region, for the record
    roofline_all = {}
    for k, v in prof.items():
        if v[1] > 0 and (k in BYTES_PER_UNIT or k in FACE_BYTES):
            r1, _ = rooflines({k: v}, n, precond, n_active)
            roofline_all[k] = {q: r1[q] for q in ("achieved", "frac", "avg_us", "launches",
                                                   "bytes_per_launch")}
    log("kernel time in the timed region (ms, launches): " +
        ", ".join(f"{k}={v[0]:.1f}/{v[1]}" for k, v in prof.items() if v[1]))

    # the headline gradient against central FD, for the exact transpose of the
    # advection (the timed reverse pass) and for the paper's upwind surrogate
    grad_fd = None
    if not args.no_grad_fd:
        fd = fd_gradient(sim, ugen, target, nu_e, s_e, dt, g, T)
        exact = {"dtheta_nu": nu_e * dnu, "dtheta_s": s_e * ds}
        log(f"FD dJ/dtheta: nu {fd['dtheta_nu']:.4e} s {fd['dtheta_s']:.4e}; exact adjoint "
            f"nu {exact['dtheta_nu']:.4e} s {exact['dtheta_s']:.4e}")
        sim.close()
        del sim
        usim = make_sim(precond, conv="upwind")
        up = adjoint_gradient(usim, ugen, target, nu_e, s_e, dt, g, T)
        usim.close()
        del usim
        log(f"upwind-surrogate adjoint nu {up['dtheta_nu']:.4e} s {up['dtheta_s']:.4e}")
        grad_fd = {"h": 1e-3, "fd": fd, "exact": exact,
                   "upwind": {k: up[k] for k in ("dtheta_nu", "dtheta_s")}}
        for conv in ("exact", "upwind"):
            for key in ("dtheta_nu", "dtheta_s"):
                grad_fd[conv]["rel_err_" + key] = _rel(grad_fd[conv][key], fd[key])
    else:
        sim.close()
        del sim

    # the headline rollout once more without the pressure history: the
    # backward's segment recompute repeats every forward solve
    no_hist = None
    if not args.no_history_leg and not args.no_pressure_history:
        hsim = make_sim(precond, history=False)
        hu = hsim.faces()

        def hist_step(rollout):
            hsim.set_params(nu=nu_e, dt=dt, s=s_e, gravity=g)
            hsim.init_state(ugen, hu)
            hsim.step(hu, rollout, record=True)
            _, gT = hsim.loss_mse(hu, target)
            return hsim.backward(gT, ugen=ugen)[3]

        hist_step(args.warmup_rollout)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        hb = hist_step(T)
        torch.cuda.synchronize()
        hel = time.perf_counter() - t1
        no_hist = {"ms_per_step": round(hel * 1e3, 1), "value": n ** 3 * T / hel,
                   "adjoint_iters": hb["iters"], "workspace_bytes": hsim.ws.numel()}
        log(f"without the pressure history: {hel * 1e3:.1f} ms, {no_hist['value']:.3e} cell-steps/s")
        hsim.close()
        del hsim

    # learned vs plain on a mask no weight was selected on
    heldout = None
    if precond == "learned" and not args.no_heldout:
        hcell = inputs.gen_mask(n, args.heldout_seed)
        hugen, htarget = make_target(hcell, T)
        heldout = {"seed": args.heldout_seed,
                   "liquid_fraction": round(inputs.liquid_fraction(hcell), 4)}
        for pc in ("learned", "jacobi"):
            xs = make_sim(pc, on_cell=hcell)
            xu = xs.faces()

            def xstep(rollout):
                xs.set_params(nu=nu_e, dt=dt, s=s_e, gravity=g)
                xs.init_state(hugen, xu)
                st = xs.step(xu, rollout, record=True)
                _, gT = xs.loss_mse(xu, htarget)
                return st, xs.backward(gT, ugen=hugen)[3]

            xstep(args.warmup_rollout)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            xst, xb = xstep(T)
            torch.cuda.synchronize()
            xel = time.perf_counter() - t1
            heldout[pc] = {"ms_per_step": round(xel * 1e3, 1), "value": n ** 3 * T / xel,
                           "pressure_iters_mean": float(np.mean([q["iters"] for q in xst])),
                           "adjoint_iters": xb["iters"]}
            log(f"held-out mask seed {args.heldout_seed}, {pc}: {xel * 1e3:.1f} ms")
            xs.close()
            del xs
        heldout["learned_over_plain"] = heldout["jacobi"]["ms_per_step"] / heldout["learned"]["ms_per_step"]
        del htarget, hugen

    # the same workload with plain (Jacobi) PCG, beside a learned headline
    plain = None
    if precond != "jacobi" and not args.no_plain:
        psim = make_sim("jacobi")
        pu = psim.faces()

        def plain_step(rollout):
            psim.set_params(nu=nu_e, dt=dt, s=s_e, gravity=g)
            psim.init_state(ugen, pu)
            st = psim.step(pu, rollout, record=True)
            _, gT = psim.loss_mse(pu, target)
            psim.backward(gT, ugen=ugen)
            return st

        plain_step(args.warmup_rollout)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        pst = plain_step(T)
        torch.cuda.synchronize()
        pel = time.perf_counter() - t1
        plain = {"precond": "jacobi", "ms_per_step": round(pel * 1e3, 1),
                 "value": n ** 3 * T / pel,
                 "pressure_iters_mean": float(np.mean([s["iters"] for s in pst])),
                 "check_every": check_period("jacobi")}
        log(f"plain Jacobi-PCG rollout: {pel * 1e3:.1f} ms, {plain['value']:.3e} cell-steps/s")
        psim.close()
        del psim

    compare = None
    if not args.no_compare:
        compare = {}
        for pc in ("jacobi", "mic0", "learned"):
            if pc == "learned" and weights is None:
                continue
            s2 = Sim(cell, precond=pc, tol=1e-6, check_every=check_period(pc), device=dev)
            if pc == "learned":
                s2.net_set_weights(weights)
            s2.set_params(nu=nu_e, dt=dt, s=s_e, gravity=g)
            uu = s2.faces()
            s2.init_state(ugen, uu)
            s2.step(uu, 1)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            st2, _ = s2.project(uu)
            torch.cuda.synchronize()
            ms = (time.perf_counter() - t1) * 1e3
            compare[pc] = {"ms_per_projection": round(ms, 2), "iters": st2["iters"],
                           "rel_residual": st2["rel_residual"]}
            log(f"projection with {pc}: {ms:.1f} ms, {st2['iters']} iterations")
            s2.close()
            del s2

    cpu = None
    if not args.no_cpu_baseline:
        log(f"CPU oracle sample at {args.cpu_n}^3 ...")
        cpu = cpu_baseline(args.cpu_n, args.seed)
        log(f"CPU oracle: {cpu['value']:.3e} cell-steps/s ({cpu['sample']})")

    pc_out = None
    if not args.no_percnn:
        pc_out = percnn_bench(cell, ugen, nu_e, s_e, dt, g, dev,
                              args.percnn_layers)
        log(f"recurrent conv solver: {pc_out['layers']} layers {pc_out['fwd_ms']:.1f} ms forward, "
            f"{pc_out['bwd_ms']:.1f} ms reverse; rel error {pc_out['rel_error_vs_projection']:.3e}")

    if pc_out is not None and weights is not None and not args.no_percnn_fit:
        pc_out["fitted"] = percnn_fitted_bench(cell, dev, weights)
        f = pc_out["fitted"]
        log(f"recurrent conv solver fitted at {n}^3 (K={f['K_fit']}, {f['fit_steps']} steps, "
            f"{f['fit_s']:.1f} s): loss {f['loss_first']:.3e} -> {f['loss_last']:.3e}")
        for name, pts in f["curves"].items():
            log(f"  {name}: " + ", ".join(f"{q['ms']:.1f} ms {q['rel_error']:.3e}" for q in pts))

    cp_out = None
    if not args.no_constrained:
        cp_out = constrained_bench(cell, ugen, nu_e, s_e, dt, g, dev, args.constrained_iters)
        log(f"constrained projection: {cp_out['iters']} iterations {cp_out['eps0']['ms']:.1f} ms "
            f"({cp_out['eps0']['us_per_iter']:.1f} us each), divergence left "
            f"{cp_out['eps0']['rel_divergence_left']:.3e} (relaxed {cp_out['relaxed']['rel_divergence_left']:.3e})")

    up_out = None
    if not args.no_upwind:
        up_out = upwind_bench(cell, ugen, nu_e, s_e, dt, g, dev)
        log(f"upwind convection gradient: {up_out['us_per_call']:.1f} us per call")

    loss_out = None
    if not args.no_loss:
        loss_out = loss_bench(cell, ugen, nu_e, s_e, dt, g, dev)
        log(f"masked cosine + L2 loss with gradient: {loss_out['us_per_call']:.1f} us per call")

    screen_out = None
    if not args.no_screen:
        screen_out = screen_bench(dev, traffic_n=n)
        log(f"screen-space projection 1080x1920: {screen_out['ms_per_call']:.2f} ms, "
            f"{screen_out['iters']} iterations")

    apic_out = None
    if not args.no_apic:
        apic_out = apic_bench(cell, dev)
        log(f"APIC transfers, {apic_out['particles']} particles: P2G {apic_out['p2g_us']:.0f} us, "
            f"G2P {apic_out['g2p_us']:.0f} us")

    out = {
        "metric": "cell-steps/s to 1e-6 Poisson residual at 256^3; learned-PCG vs plain PCG",
        "value": value,
        "unit": "cell-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (FP64 iterate, dots and residual)",
        "data": "synthetic (seeded slab + ellipsoids mask, curl-of-potential velocity)",
        "config": {"workload": f"differentiable rollout {n}^3 x {T} steps, forward + "
                               f"checkpointed adjoint (K={K}), {precond} pressure "
                               f"preconditioner, {'cold' if args.cold else 'warm'}-started "
                               f"solves{'' if args.no_pressure_history else ', pressure history'}"
                               f", tol 1e-6",
                   "n": n, "rollout": T, "checkpoint_every": K, "precond": precond,
                   "seed": args.seed, "nu": nu_e, "s": s_e, "warm_start": not args.cold,
                   "pressure_history": not args.no_pressure_history},
        "roofline": roofline,
        "roofline_hbm": roofline_hbm,
        "roofline_all_hbm": roofline_all,
        "active_faces": n_active,
        "peak_mem_bytes": peak_mem,
        "workspace_bytes": ws_bytes,
        "grad_fd": grad_fd,
        "no_pressure_history": no_hist,
        "heldout": heldout,
        "plain_pcg": plain,
        "cpu_baseline": cpu,
        "compare": compare,
        "pressure_iters_mean": float(np.mean(fwd_iters)),
        "percnn": pc_out,
        "constrained": cp_out,
        "upwind": up_out,
        "loss": loss_out,
        "screen": screen_out,
        "apic": apic_out,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
