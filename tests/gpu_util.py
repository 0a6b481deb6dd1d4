"""Helpers shared by the GPU tests: upload a seeded problem, build a context."""
import sys

import numpy as np

import sninputs
from sninputs import Problem


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a, dtype=None):
    import torch
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda").contiguous()


def context(p: Problem, eta=None):
    import torch
    from paper_2001_09196_amd import Context
    st = dev(p.sigma_t, torch.float64)
    ss = dev(p.sigma_s, torch.float64)
    return Context(p.dim, p.nx, p.ny, p.nz, p.h, p.omega, p.w, st, ss, eta=p.eta if eta is None else eta,
                   order=p.order)


def random_problem(dim, nx, ny, nz, order=4, seed=0, voids=True, h=(1.0, 0.8, 1.2)):
    rng = np.random.default_rng(seed)
    nc = nx * ny * nz
    om, w = sninputs.level_symmetric(order, dim)
    kind = rng.integers(0, 3, nc) if voids else rng.integers(1, 3, nc)
    st = np.where(kind == 2, rng.uniform(20, 500, nc), np.where(kind == 1, rng.uniform(0.2, 3, nc), 0.0))
    ss = np.where(kind == 2, st * rng.uniform(0.99, 0.9999, nc), np.where(kind == 1, st * rng.uniform(0, 0.9, nc), 0.0))
    q = np.where(kind == 1, rng.uniform(0, 2, nc), 0.0)
    hh = h if dim == 3 else (h[0], h[1], 1.0)
    return Problem(f"rand{dim}d_{nx}x{ny}x{nz}", dim, nx, ny, nz, hh, st, ss, q, om, w)


def rel_max(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300))


def rel_l2(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))
