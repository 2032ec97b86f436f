"""Helpers for the GPU parity tests (the HIP path through the C ABI against
the FP64 oracle on the same seeded float32 inputs)."""
import numpy as np

from paper_2503_00868_amd import inputs


def f32(arrs):
    """Round to float32 (what the GPU receives) and back to float64 (what the
    oracle receives), so both start from identical values."""
    return tuple(np.asarray(a, np.float32).astype(np.float64) for a in arrs)


def to_np(ts):
    return tuple(t.detach().cpu().numpy().astype(np.float64) for t in ts)


def rel_err(a, b):
    """(L2 relative, max-norm relative) error of field tuple a against b."""
    num = sum(float(((x - y) ** 2).sum()) for x, y in zip(a, b))
    den = sum(float((y ** 2).sum()) for y in b)
    mx = max(float(np.abs(x - y).max()) for x, y in zip(a, b))
    my = max(float(np.abs(y).max()) for y in b)
    return (np.sqrt(num / den) if den > 0 else np.sqrt(num)), (mx / my if my > 0 else mx)


def case(n, seed, scale=1.0):
    cell, ug = inputs.gen_case(n, seed)
    return cell, f32(tuple(scale * g for g in ug))


def banner(msg):
    print(f"[gpu-test] {msg}", flush=True)
