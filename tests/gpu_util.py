"""Helpers shared by the GPU parity tests: host<->device conversion of the
seeded inputs and the normwise error metric.

Error metric: for each (b, h), ||X - X_ref||_F / ||X_ref||_F, and the test
takes the maximum over (b, h).  Elementwise relative error is not used:
outputs of attention over zero-mean values are weighted means close to
zero, so individual entries can sit arbitrarily near 0.
"""
import numpy as np
import torch

from paper_2604_16590_amd import inputs

TOL = {"bf16": 2e-2, "fp32": 1e-5}


def require_gpu():
    if not torch.cuda.is_available():
        raise RuntimeError("GPU test run without a visible GPU")
    return torch.device("cuda:0")


def to_device(a: np.ndarray, dev) -> torch.Tensor:
    if a.dtype == np.uint16:
        return torch.from_numpy(a.view(np.int16).copy()).to(dev).view(torch.bfloat16)
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def to_host(t: torch.Tensor) -> np.ndarray:
    """Stored values as numpy: bf16 as uint16 bit patterns, else float."""
    t = t.detach().cpu()
    if t.dtype == torch.bfloat16:
        return t.contiguous().view(torch.int16).numpy().view(np.uint16)
    return t.numpy()


def as64(t) -> np.ndarray:
    a = to_host(t) if isinstance(t, torch.Tensor) else t
    return inputs.as_float64(a)


def normwise(x: np.ndarray, ref: np.ndarray) -> float:
    """max over leading (b, h) of the Frobenius relative error."""
    x = np.asarray(x, np.float64)
    ref = np.asarray(ref, np.float64)
    lead = x.shape[:2]
    xe = x.reshape(lead + (-1,))
    re = ref.reshape(lead + (-1,))
    num = np.linalg.norm(xe - re, axis=-1)
    den = np.linalg.norm(re, axis=-1)
    return float((num / np.maximum(den, 1e-300)).max())


def max_rel(x, ref) -> float:
    """max |x - ref| / max |ref| (reported beside the normwise error)."""
    x = np.asarray(x, np.float64)
    ref = np.asarray(ref, np.float64)
    return float(np.abs(x - ref).max() / max(np.abs(ref).max(), 1e-300))


def make_inputs(shape, dtype, seed, streams=(0, 1, 2), std=1.0, grid=None):
    """Seeded inputs (host copies: bf16 bits or float32), one per stream id,
    made by the device generator (liblagen.so, the same definition as the
    host module paper_2604_16590_amd.inputs, which is much slower)."""
    import paper_2604_16590_amd as la
    dev = require_gpu()
    tdt = torch.bfloat16 if dtype == "bf16" else torch.float32
    out = []
    for s in streams:
        x = torch.empty(shape, dtype=tdt, device=dev)
        la.gen_fill(x, seed=seed, stream_id=s, std=std, grid=grid, tensor_id=s)
        out.append(to_host(x))
    return out
