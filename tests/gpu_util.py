"""Helpers shared by the GPU parity tests (no method arithmetic here)."""
import sys

import numpy as np
import torch

import oracle

DEV = torch.device("cuda:0")
EPS = {torch.float64: np.finfo(np.float64).eps, torch.float32: np.finfo(np.float32).eps}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def host(t):
    torch.cuda.synchronize()
    return t.detach().double().cpu().numpy()


def abs_scale(grid, s, u, mask, springs):
    """(|K_bc| |u|): the natural magnitude of the rounding error of K u."""
    KE = np.abs(oracle.element_stiffness())
    sp = None
    if springs:
        sp = tuple((d, abs(k)) for d, k in springs)
    return oracle.apply_K(grid, s, np.abs(u), mask, sp, KE=KE)
