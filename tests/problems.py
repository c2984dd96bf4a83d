"""Shared problem setup for the GPU parity tests: seeded inputs from
paper_1911_03973_amd.inputs, oracle reference values, and the SoA <-> element-
major layout conversions between the GPU arrays and the oracle's arrays."""
from __future__ import annotations

import numpy as np
import torch

import oracle
from paper_1911_03973_amd import inputs


def to_soa(Ke):
    """(n_elems, nb, nb) -> (nb*nb, n_elems)."""
    ne, nb, _ = Ke.shape
    return np.ascontiguousarray(Ke.reshape(ne, nb * nb).T)


def from_soa(A, nb):
    """(nb*nb, n_elems) -> (n_elems, nb, nb)."""
    return np.ascontiguousarray(A.T.reshape(-1, nb, nb))


def pair_value(t):
    """FP64 value of an F32X2 tensor (2, nb*nb, ne)."""
    a = t.double().cpu().numpy()
    return a[0] + a[1]


class Problem:
    def __init__(self, mesh, nu=0.0, dirichlet="all", f=None, seed=0):
        self.mesh = mesh
        self.nu = float(nu)
        self.nd = inputs.boundary_nodes(mesh, dirichlet) if dirichlet else np.zeros(0, np.int32)
        self.mask = oracle.mask_from_nodes(mesh.n_nodes, self.nd)
        self.K, self.M, self.vol = oracle.local_matrices(mesh.coords, mesh.elems)
        if f is None:
            f = np.ones(mesh.n_nodes)
        elif isinstance(f, str) and f == "sine":
            f = inputs.random_sine(mesh.coords, seed)
        self.f = np.asarray(f, dtype=np.float64)
        self.b = oracle.rhs(mesh.n_nodes, mesh.elems, self.M, self.f)

    @property
    def n(self):
        return self.mesh.n_nodes


def cuda(a, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def max_rel(a, b, scale=None):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    s = np.abs(b).max() if scale is None else scale
    return float(np.abs(a - b).max() / max(s, 1e-300))


def bf16_params(net):
    """The network's parameters in the oracle's layout with the weights rounded
    to BF16 as the kernels use them (the 1x1 output layer and all biases stay
    FP32)."""
    from oracle import unet as U

    w = net.get_params()
    torch.cuda.synchronize()
    p = w.double().cpu().numpy()
    layers = U.unpack(p, net.channels)
    out = []
    for k, (W, b) in enumerate(layers):
        Wr = torch.from_numpy(W.astype(np.float32)).to(torch.bfloat16).double().numpy()
        if k == len(layers) - 1:
            Wr = W
        out.append((Wr, b))
    return U.pack(out)
