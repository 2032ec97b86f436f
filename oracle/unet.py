"""FP64 oracle of the learned preconditioner network (test infrastructure only).

The paper replaces the iterative pressure solve by a recurrent convolutional
network whose kernels are fitted on pressure pairs taken before and after an
implicit solve (Section 3.4.1, PeRCNN; Fig. "percnn_str_fit").  The network
built here is a 3-level 3-D U-Net used as a preconditioner inside flexible
CG; its architecture is a reading (R14), not a paper listing:

  x0 = (r / rms(r), liquid mask)                               2 channels
  e1 = relu(c2(relu(c1(x0))))                 16 ch at n^3      c1: 2->16, c2: 16->16
  e2 = relu(c4(relu(c3(pool(e1)))))           32 ch at (n/2)^3  c3: 16->32, c4: 32->32
  e3 = relu(c6(relu(c5(pool(e2)))))           64 ch at (n/4)^3  c5: 32->64, c6: 64->64
  d2 = relu(c8(relu(c7(cat(up(e3), e2)))))    32 ch at (n/2)^3  c7: 96->32, c8: 32->32
  d1 = relu(c10(relu(c9(cat(up(d2), e1)))))   16 ch at n^3      c9: 48->16, c10: 16->16
  o  = c11(d1)                                 1 ch              c11: 16->1
  z  = mask * rms(r) * o

Every convolution is 3x3x3, zero padded ("same"), bias free; pool is the 2x2x2
average, up the nearest-neighbour 2x upsampling.  rms is over liquid cells.
Bias-free ReLU layers keep z positively homogeneous in r.

Precision: the GPU stores weights, the input and every activation in bf16
and accumulates in fp32.  The oracle computes in fp64 and rounds to bf16
(round to nearest even) at the same points, so the two differ only by
accumulation order (and the rare bf16 rounding flip that causes).

Weights are one flat float32 blob: the 11 convolutions in order c1..c11, each
in PyTorch Conv3d layout [c_out][c_in][kz][ky][kx].
"""
from __future__ import annotations

import numpy as np
import torch
import torch.nn.functional as F

CONVS = [(2, 16), (16, 16), (16, 32), (32, 32), (32, 64), (64, 64), (96, 32), (32, 32),
         (48, 16), (16, 16), (16, 1)]


def param_count():
    return sum(27 * a * b for a, b in CONVS)


def split_weights(blob):
    """Flat blob (float32, or float64 for smooth FD checks) -> list of 11 fp64
    tensors [c_out, c_in, 3, 3, 3]."""
    blob = torch.as_tensor(np.asarray(blob), dtype=torch.float64)
    out, off = [], 0
    for cin, cout in CONVS:
        m = 27 * cin * cout
        out.append(blob[off:off + m].reshape(cout, cin, 3, 3, 3))
        off += m
    assert off == blob.numel()
    return out


def bf16(t):
    """Round to bfloat16 (nearest even) and back to fp64."""
    return t.to(torch.bfloat16).to(torch.float64)


def init_weights(seed=0):
    """He-normal init (fan-in 27 c_in); the output conv scaled by 0.1."""
    rng = np.random.default_rng(seed)
    parts = []
    for q, (cin, cout) in enumerate(CONVS):
        std = np.sqrt(2.0 / (27 * cin)) * (0.1 if q == len(CONVS) - 1 else 1.0)
        parts.append(rng.standard_normal(27 * cin * cout) * std)
    return np.concatenate(parts).astype(np.float32)


def forward(weights, r, mask, emulate_bf16=True, return_all=False):
    """z for one residual field r (n^3, [z][y][x]) and liquid mask (bool/0-1).

    weights: flat blob or list from split_weights."""
    W = split_weights(weights) if not isinstance(weights, list) else weights
    q = bf16 if emulate_bf16 else (lambda t: t)
    Wq = [q(w) for w in W]
    r = torch.as_tensor(np.asarray(r), dtype=torch.float64)
    m = torch.as_tensor(np.asarray(mask), dtype=torch.float64)
    nl = float(m.sum())
    rms = float(torch.sqrt((r * r * m).sum() / nl)) if nl > 0 else 0.0
    if rms == 0.0:
        return np.zeros(r.shape) if not return_all else (np.zeros(r.shape), {})
    x0 = torch.stack([q(r / rms), q(m)])[None]  # [1, 2, n, n, n]

    def conv(x, w, relu=True):
        y = F.conv3d(x, w, padding=1)
        return q(F.relu(y)) if relu else y

    a1 = conv(x0, Wq[0])
    e1 = conv(a1, Wq[1])
    p1 = q(F.avg_pool3d(e1, 2))
    a2 = conv(p1, Wq[2])
    e2 = conv(a2, Wq[3])
    p2 = q(F.avg_pool3d(e2, 2))
    a3 = conv(p2, Wq[4])
    e3 = conv(a3, Wq[5])
    c2 = torch.cat([F.interpolate(e3, scale_factor=2, mode="nearest"), e2], dim=1)
    b2 = conv(c2, Wq[6])
    d2 = conv(b2, Wq[7])
    c1 = torch.cat([F.interpolate(d2, scale_factor=2, mode="nearest"), e1], dim=1)
    b1 = conv(c1, Wq[8])
    d1 = conv(b1, Wq[9])
    o = conv(d1, Wq[10], relu=False)
    if emulate_bf16:
        o = o.to(torch.float32).to(torch.float64)
    z = (m * rms * o[0, 0]).numpy()
    if return_all:
        return z, {"x0": x0, "a1": a1, "e1": e1, "p1": p1, "a2": a2, "e2": e2, "p2": p2, "a3": a3,
                   "e3": e3, "b2": b2, "d2": d2, "b1": b1, "d1": d1, "o": o, "rms": rms}
    return z


def anorm_loss(z, r, e, Az):
    """1 - (r.z)^2 / ((r.e)(z.Az)): the squared sine of the A-norm angle
    between the correction z and the true error e (A e = r)."""
    rz = float((r * z).sum())
    re = float((r * e).sum())
    zAz = float((z * Az).sum())
    return 1.0 - rz * rz / (re * zAz)


def loss_and_grad(weights, r, e, mask, apply_A):
    """Loss of one pair and its gradient with respect to the float32 blob
    (fp64 autograd through the bf16-emulated forward: rounding is treated as
    identity in the backward pass, straight-through).

    apply_A: numpy function x -> A x (the oracle Poisson apply)."""
    W = [w.clone().requires_grad_(True) for w in split_weights(weights)]

    class RoundST(torch.autograd.Function):
        @staticmethod
        def forward(ctx, t):
            return bf16(t)

        @staticmethod
        def backward(ctx, g):
            return g

    q = RoundST.apply
    r_t = torch.as_tensor(np.asarray(r), dtype=torch.float64)
    m = torch.as_tensor(np.asarray(mask), dtype=torch.float64)
    nl = float(m.sum())
    rms = float(torch.sqrt((r_t * r_t * m).sum() / nl))
    x0 = torch.stack([bf16(r_t / rms), bf16(m)])[None]

    def conv(x, w, relu=True):
        y = F.conv3d(x, q(w), padding=1)
        return q(F.relu(y)) if relu else y

    a1 = conv(x0, W[0])
    e1 = conv(a1, W[1])
    p1 = q(F.avg_pool3d(e1, 2))
    a2 = conv(p1, W[2])
    e2 = conv(a2, W[3])
    p2 = q(F.avg_pool3d(e2, 2))
    a3 = conv(p2, W[4])
    e3 = conv(a3, W[5])
    b2 = conv(torch.cat([F.interpolate(e3, scale_factor=2, mode="nearest"), e2], dim=1), W[6])
    d2 = conv(b2, W[7])
    b1 = conv(torch.cat([F.interpolate(d2, scale_factor=2, mode="nearest"), e1], dim=1), W[8])
    d1 = conv(b1, W[9])
    o = conv(d1, W[10], relu=False)[0, 0]
    z = m * rms * o
    zn = z.detach().numpy()

    class Quad(torch.autograd.Function):
        """z.Az with A symmetric: gradient 2 Az."""

        @staticmethod
        def forward(ctx, zz):
            Az = torch.as_tensor(apply_A(zz.detach().numpy()), dtype=torch.float64)
            ctx.save_for_backward(Az)
            return (zz * Az).sum()

        @staticmethod
        def backward(ctx, g):
            (Az,) = ctx.saved_tensors
            return 2.0 * g * Az

    e_t = torch.as_tensor(np.asarray(e), dtype=torch.float64)
    rz = (r_t * z).sum()
    re = float((r_t * e_t).sum())
    zAz = Quad.apply(z)
    loss = 1.0 - rz * rz / (re * zAz)
    loss.backward()
    grad = torch.cat([w.grad.reshape(-1) for w in W]).numpy()
    return float(loss.detach()), grad, zn
