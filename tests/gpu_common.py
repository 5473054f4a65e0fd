"""Helpers shared by the GPU tests: inputs from lattice_inputs, the oracle
on the CPU, and the library through its ctypes binding."""
import numpy as np
import torch

from lattice_inputs import gauge_links, gaussian_spinor, load_m0

DEV = "cuda:0"


def to_dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.complex128).to(DEV)


def links(dims, eps, seed):
    U = gauge_links(dims, eps, seed)
    return U, to_dev(U)


def spinors(dims, seed, n):
    s = gaussian_spinor(dims, seed, n=n)
    return s, to_dev(s)


def kappa_of(m0):
    return 1.0 / (2.0 * m0 + 8.0)


def rel(a, b):
    a = torch.as_tensor(a).to(torch.complex128).cpu()
    b = torch.as_tensor(b).to(torch.complex128).cpu()
    return float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))


def field(x):
    """canonical spinor(s) [..., 4, 3] -> oracle field [..., 12] (cpu)."""
    t = torch.as_tensor(x).cpu()
    return t.reshape(*t.shape[:-2], 12)


def maxabs_rel(a, b):
    """Largest elementwise deviation relative to the largest entry of the
    reference: catches a wrong value at a few sites that an l2 ratio over
    the whole field would average away."""
    a = torch.as_tensor(a).to(torch.complex128).cpu()
    b = torch.as_tensor(b).to(torch.complex128).cpu()
    return float((a - b).abs().max() / b.abs().max())
