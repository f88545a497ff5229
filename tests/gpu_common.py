"""Shared helpers of the GPU parity tests (HIP path through the C ABI vs the CPU oracle)."""
import numpy as np

from oracle.lattice import Lattice, transport
from oracle.systems import Advection, Burgers, Euler, ShallowWater, equilibrium

PARITY_RTOL = 1e-12   # per conserved component: max |df_{k,m}| / max |f_{k,m}|


def oracle_system(lattice, system, param):
    lat = Lattice(lattice)
    d = lat.d
    if system == "advection":
        sys = Advection(tuple(param[:d]))
    elif system == "burgers":
        sys = Burgers(tuple(param[:d]))
    elif system == "shallow_water":
        sys = ShallowWater(param[0], d)
    elif system == "euler":
        sys = Euler(param[0], d)
    else:
        raise ValueError(system)
    return lat, sys


def componentwise_error(a, b):
    """max over (k, x) of |a - b| / max |b|, per conserved component m; arrays (q, M, ny, nx)."""
    a = np.asarray(a)
    b = np.asarray(b)
    out = []
    for m in range(b.shape[1]):
        den = np.max(np.abs(b[:, m]))
        out.append(float(np.max(np.abs(a[:, m] - b[:, m])) / (den if den > 0 else 1.0)))
    return out


def to_gpu(arr):
    import torch
    return torch.from_numpy(np.ascontiguousarray(arr)).to("cuda")


def to_host(t):
    return t.detach().cpu().numpy()


def off_equilibrium(lat, sys, V, u, shift=1):
    """f^eq(u) moved by one transport: a realistic stage input (d != 0), logical layout."""
    return transport(lat, equilibrium(lat, sys, V, u), shift)


def shifted_logical(lat, stored, offsets):
    """Logical state of a stored state with per-velocity offsets: f_k(x) = stored_k(x - o_k c_k)."""
    out = np.empty_like(stored)
    for k in range(lat.q):
        out[k] = transport(lat, stored, int(offsets[k]))[k]
    return out
