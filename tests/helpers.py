"""Shared helpers for the GPU parity tests (test infrastructure)."""

import math
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def ensure_built():
    from paper_2605_18389_amd import binding
    if not os.path.exists(binding.LIB_PATH):
        from paper_2605_18389_amd.build import build
        build()


def announce(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


def to_dev(x, dtype):
    import torch
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def to_np(t):
    return t.detach().double().cpu().numpy()
