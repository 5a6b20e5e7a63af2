"""Helpers shared by the GPU tests: moving states between numpy and torch."""
import numpy as np

TOL = {"c128": 1e-12, "c64": 1e-5}


def torch_dtype(name):
    import torch
    return torch.complex128 if name == "c128" else torch.complex64


def to_gpu(psi, name):
    import torch
    return torch.from_numpy(np.ascontiguousarray(psi)).to(torch_dtype(name)).cuda()


def to_np(t):
    return t.detach().cpu().numpy().astype(np.complex128)


def rand_state(n, rng, name="c128"):
    v = rng.standard_normal(1 << n) + 1j * rng.standard_normal(1 << n)
    v = v / np.linalg.norm(v)
    if name == "c64":
        v = v.astype(np.complex64).astype(np.complex128)
    return v


def raw_bits(a):
    a = np.ascontiguousarray(a)
    return a.view(np.uint32 if a.dtype == np.complex64 else np.uint64)


def say(*args):
    print("[case]", *args, flush=True)
