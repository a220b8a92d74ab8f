"""Shared helpers of the GPU tests: seeded inputs on the device and tolerance models."""
import numpy as np
import torch

from paper_2112_04556_amd import api, inputs


def dev():
    return torch.device("cuda:0")


def setup(L, kind="eps", eps=0.3, seed=1, n=1, dtype=torch.float64):
    """(U_complex numpy, P numpy, U_soa device, P device) from the seeded generators."""
    U = inputs.random_links(L, kind, eps, seed=seed)
    P = inputs.gaussian_fields(L, n, seed=seed)
    Ud = api.pack_links(L, U.to(dev()), dtype)
    Pd = P.to(dev()).to(dtype)
    return U.numpy(), P.numpy(), Ud, Pd


def rel_max(a, b):
    """max |a - b| / max |b|."""
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def announce(msg):
    print(f"[gpu-test] {msg}", flush=True)
