"""Shared helpers of the GPU tests: move oracle-side numpy arrays to the device and back."""
import numpy as np
import torch

DEV = torch.device("cuda:0")


def cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to(DEV)


def host(t):
    return t.detach().cpu().numpy()


def relmax(a, b):
    """max |a - b| / max |b|"""
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def print_case(*args):
    print("CASE", *args, flush=True)
