"""Helpers shared by the GPU tests (marshalling and error metrics only)."""
import numpy as np
import torch


def dev():
    return torch.device("cuda", 0)


def to_gpu(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device=dev())


def to_np(t):
    return t.detach().cpu().double().numpy()


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def announce(msg):
    print("[gpu-case] " + msg, flush=True)
