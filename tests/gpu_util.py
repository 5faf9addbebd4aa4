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
    """Per-trial error of got against ref, the larger of the relative Frobenius
    error ||got - ref|| / ||ref|| and the element-wise error
    max |got - ref| / max |ref|, maximised over the trials (leading axis)."""
    got = np.asarray(got)
    ref = np.asarray(ref)
    assert got.shape == ref.shape, (got.shape, ref.shape)
    ax = tuple(range(1, ref.ndim))
    d = np.abs(got - ref)
    fro = np.sqrt(np.sum(d ** 2, axis=ax)) / np.maximum(np.sqrt(np.sum(np.abs(ref) ** 2, axis=ax)),
                                                          1e-300)
    elem = np.max(d, axis=ax) / np.maximum(np.max(np.abs(ref), axis=ax), 1e-300)
    return float(max(np.max(fro), np.max(elem)))


def max_elem_err(got, ref):
    """max |got - ref| / max |ref| over the whole array."""
    got = np.asarray(got)
    ref = np.asarray(ref)
    return float(np.max(np.abs(got - ref)) / max(np.max(np.abs(ref)), 1e-300))
