"""Shared helpers of the GPU parity tests (imported only by -m gpu tests)."""
import numpy as np

import oracle


def oracle_run(D, Q, Nf, Pr, tau, dims, fields, steps, kappa=0.2):
    sim = oracle.Sim(D, Q, Nf, Pr, tau, dims, kappa=kappa)
    sim.init(*fields)
    if steps:
        sim.step(steps)
    return sim


def pop_error(w, a, b):
    """max |a - b| / w_i over all cells and directions (populations as
    (Q, ...) planes)."""
    w = np.asarray(w).reshape((-1,) + (1,) * (a.ndim - 1))
    return float(np.max(np.abs(a - b) / w))


def rel_l2(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def pert_l2(a, b, ref=1.0):
    """relative L2 of the perturbation about ref"""
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm((b - ref).ravel()))


def neighbourhood(dims, cells, c):
    """Flat indices of x - c_i for each sampled cell x and direction i:
    shape (len(cells), Q), periodic."""
    D = len(dims)
    cells = np.asarray(cells, dtype=np.int64)
    coords = []
    rem = cells.copy()
    for d in range(D):
        coords.append(rem % dims[d])
        rem //= dims[d]
    out = np.zeros((cells.size, c.shape[0]), dtype=np.int64)
    for i in range(c.shape[0]):
        idx = np.zeros(cells.size, dtype=np.int64)
        stride = 1
        for d in range(D):
            idx += ((coords[d] - c[i, d]) % dims[d]) * stride
            stride *= dims[d]
        out[:, i] = idx
    return out
