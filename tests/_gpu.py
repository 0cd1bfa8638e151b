"""Helpers for the GPU parity tests: device transfer and storage rounding.

Inputs are drawn in float64 (paper_cs_9809105_amd.inputs), rounded once to
the storage type, and the *same* rounded values go to the GPU and, promoted
back to float64, to the oracle.
"""
import sys

import numpy as np

try:
    import torch
except ImportError:  # pragma: no cover
    torch = None

STORAGE = {"f64": "float64", "f32": "float32", "bf16": "bfloat16", "f16": "float16",
           "split3_bf16": "float32", "fp8_e4m3": "float32", "fp8_e4m3_r1": "float32"}


def gpu_available():
    return torch is not None and torch.cuda.is_available()


def note(*args):
    """Name the case before a GPU step, so a fault can be traced to it."""
    print("[gpu-case]", *args, file=sys.stderr, flush=True)


def to_dev(x64, dtype):
    """float64 numpy -> (device tensor in storage type, float64 numpy of the stored values)."""
    t = torch.from_numpy(np.ascontiguousarray(x64)).to(getattr(torch, STORAGE[dtype]))
    stored = t.to(torch.float64).numpy()
    return t.cuda(), stored


def host(t):
    return t.detach().to("cpu", torch.float64).numpy()


def poisoned(shape, dtype, device="cuda"):
    """Output buffer pre-filled with NaN to expose elements never written."""
    return torch.full(shape, float("nan"), dtype=dtype, device=device)
