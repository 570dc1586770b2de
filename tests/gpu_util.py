"""Helpers shared by the GPU tests (no arithmetic of the method)."""
import numpy as np
import pytest


def need_gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    return torch


def rel_err(a, b):
    """(max-norm, 2-norm) relative difference of a against reference b."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    d = a - b
    nb_inf = max(np.abs(b).max(), 1e-300)
    nb_2 = max(np.linalg.norm(b), 1e-300)
    return float(np.abs(d).max() / nb_inf), float(np.linalg.norm(d) / nb_2)


def banner(msg):
    print(f"\n[gpu-test] {msg}", flush=True)
