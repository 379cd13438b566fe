"""Shared helpers of the GPU parity tests: seeded inputs (from gen), oracle fields, device upload."""
from __future__ import annotations

import math

import numpy as np
import pytest
import torch

import gen
from oracle import dirac as odirac
from oracle import geometry as geo


# number of launch shapes in the hop kernel's shape table (csrc/hop_kernels.h), which DIRAC_HOP_SHAPE
# indexes; test_abi checks it against the table and bench.py's names
N_HOP_SHAPES = 48


def need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2502_02490_amd import _lib

    _lib.load()  # fails loudly when the HIP library is missing


class Case:
    """A lattice with seeded SU(3) x U(1) fields, the oracle's view of it and the GPU operator."""

    def __init__(self, dims, eps=0.5, kappa=0.1245, csw=1.6, csw_qed=1.0, qhat=-1, seed=201,
                 bc_phase=(math.pi, 0.0, 0.0, 0.0), theta_max=0.3, cstar=0):
        import paper_2502_02490_amd as P

        self.dims = tuple(dims)
        self.V = geo.volume(dims)
        self.U = gen.su3_field(dims, eps, seed)
        self.theta = gen.u1_field(dims, theta_max, seed)
        self.p = odirac.Params(self.dims, kappa, csw, csw_qed, qhat, tuple(bc_phase), cstar)
        self.f = odirac.Fields(self.U, self.theta, self.p)
        self.Ud = torch.from_numpy(self.U).cuda()
        self.thd = torch.from_numpy(self.theta).cuda()
        self.D = P.Dirac(self.Ud, self.thd, self.dims, kappa, csw, csw_qed, qhat, bc_phase, cstar=cstar)
        self.even, self.odd = odirac.even_odd(self.f)

    def spinor(self, seed, index=0):
        return gen.gaussian_spinor(self.dims, seed, index)


def to_dev(a: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def rel(a, b) -> float:
    """The larger of the norm-wise error |a - b| / |b| and the element-wise one
    max_i |a_i - b_i| / max_i |b_i|: one wrong site, which a norm dilutes by the square root of
    the number of sites, shows in full in the second."""
    a = np.asarray(a)
    b = np.asarray(b)
    return max(float(np.linalg.norm(a - b) / np.linalg.norm(b)), float(np.abs(a - b).max() / np.abs(b).max()))


def rel_norm(a, b) -> float:
    """|a - b| / |b| alone (for diagnostics where isolated entries are expected to differ)."""
    a = np.asarray(a)
    b = np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def flush(msg: str):
    print(msg, flush=True)
