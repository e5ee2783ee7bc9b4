"""Helpers for the GPU parity tests (device placement, oracle comparisons)."""
import numpy as np
import torch

from paper_1702_02241_amd import torch_api as T


def device():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return torch.device("cuda:0")


def rel(a, b):
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    den = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (den if den > 0 else 1.0))


def upload(p):
    """(Xcm, U-shape) device copies for a synth.Problem."""
    return T.to_device_X(p.X, device())


def f32(a):
    """Round a host array to FP32 and back to FP64 (the GPU sees FP32 inputs)."""
    return np.asarray(a, np.float32).astype(np.float64)
