"""Helpers shared by the GPU tests: build contexts and compare against the oracle."""
import sys

import numpy as np


def say(msg):
    print(f"[gpu-test] {msg}", flush=True)
    sys.stdout.flush()


def to_complex(t):
    a = t.detach().cpu().numpy().astype(np.float64)
    return a[..., 0] + 1j * a[..., 1]


def rel_err(got, ref):
    """Per-trial relative Frobenius error ||got - ref|| / ||ref|| (max over trials)."""
    got = np.asarray(got)
    ref = np.asarray(ref)
    num = np.sqrt(np.sum(np.abs(got - ref) ** 2, axis=tuple(range(1, ref.ndim))))
    den = np.sqrt(np.sum(np.abs(ref) ** 2, axis=tuple(range(1, ref.ndim))))
    return float(np.max(num / np.maximum(den, 1e-300)))
