"""Properties the GPU operator must have at any size, checked with the GPU alone (no oracle
values): gamma_5-hermiticity <chi, D^dag psi> = <D chi, psi> at the full 32^3 x 64 production
size in FP64 (full operator) and on the Schur complement, and covariance under a random local
SU(3) x U(1) transformation (the transformed fields go through the whole GPU set-up: link
compression, clover build, inversion).  Plus the whole-lattice parity of the Schur apply
against the oracle at 16^3 x 32."""
import math

import numpy as np
import pytest
import torch

import gen
from gpu_util import Case, flush, need_gpu, rel, to_dev
from oracle import dirac as odirac
from oracle import geometry as geo

pytestmark = pytest.mark.gpu


def _vdot(a: torch.Tensor, b: torch.Tensor) -> complex:
    return complex(torch.vdot(a.reshape(-1), b.reshape(-1)).item())


def test_gamma5_hermiticity_32c64():
    need_gpu()
    import paper_2502_02490_amd as P

    dims = (64, 32, 32, 32)
    flush(f"[gpu] gamma5 hermiticity {dims}")
    U = to_dev(gen.su3_field(dims, 0.5, 211))
    th = to_dev(gen.u1_field(dims, 0.3, 211))
    D = P.Dirac(U, th, dims, 0.1245, 1.6, 1.0, -1)
    try:
        chi = to_dev(gen.gaussian_spinor(dims, 212))
        psi = to_dev(gen.gaussian_spinor(dims, 213))
        a, b = torch.empty_like(chi), torch.empty_like(psi)
        D.apply(a, chi)                  # D chi
        D.apply(b, psi, dagger=True)     # D^dag psi
        lhs, rhs = _vdot(chi, b), _vdot(a, psi)
        assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
        # the Schur complement inherits it: <chi_e, D-hat^dag psi_e> = <D-hat chi_e, psi_e>
        vh = math.prod(dims) // 2
        ce, pe = chi[:vh].contiguous(), psi[:vh].contiguous()  # any half-lattice vectors in EO order
        a2, b2 = torch.empty_like(ce), torch.empty_like(pe)
        D.apply_eo(a2, ce)
        D.apply_eo(b2, pe, dagger=True)
        lhs, rhs = _vdot(ce, b2), _vdot(a2, pe)
        assert abs(lhs - rhs) <= 1e-12 * abs(lhs)
    finally:
        D.close()


def test_gauge_covariance_on_gpu():
    """U -> W U W(x+mu)^dag, theta -> theta + lam(x) - lam(x+mu), psi -> e^{i qhat lam} W psi:
    D'(psi') = (D psi)' with both operators built on the GPU."""
    need_gpu()
    import paper_2502_02490_amd as P

    dims = (16, 8, 8, 8)
    qhat = 2
    U = gen.su3_field(dims, 0.5, 221)
    th = gen.u1_field(dims, 0.3, 221)
    W, lam = gen.gauge_transform(dims, 222)
    V = geo.volume(dims)
    sites = np.arange(V)
    U2, th2 = np.empty_like(U), np.empty_like(th)
    for mu in range(4):
        fw = geo.shift(sites, dims, mu, 1)
        U2[:, mu] = W @ U[:, mu] @ np.conj(np.swapaxes(W[fw], 1, 2))
        th2[:, mu] = th[:, mu] + lam - lam[fw]
    tr = lambda v: np.exp(1j * qhat * lam)[:, None, None] * np.einsum("nab,nsb->nsa", W, v)  # noqa: E731
    D1 = P.Dirac(to_dev(U), to_dev(th), dims, 0.1245, 1.6, 1.0, qhat, (math.pi, 0.3, 0.0, 0.0))
    D2 = P.Dirac(to_dev(U2), to_dev(th2), dims, 0.1245, 1.6, 1.0, qhat, (math.pi, 0.3, 0.0, 0.0))
    try:
        psi = gen.gaussian_spinor(dims, 223)
        y1 = torch.empty_like(to_dev(psi))
        y2 = torch.empty_like(y1)
        D1.apply(y1, to_dev(psi))
        D2.apply(y2, to_dev(tr(psi)))
        assert rel(y2.cpu().numpy(), tr(y1.cpu().numpy())) <= 1e-13
        # and the solver: D2^-1 (b') = (D1^-1 b)'
        x1, x2 = torch.zeros_like(y1), torch.zeros_like(y1)
        D1.solve(x1, to_dev(psi), tol=1e-12)
        D2.solve(x2, to_dev(tr(psi)), tol=1e-12)
        assert rel(x2.cpu().numpy(), tr(x1.cpu().numpy())) <= 1e-9
    finally:
        D1.close()
        D2.close()


def test_schur_16c32_whole_lattice():
    """Every even site of a 16^3 x 32 lattice, FP64 and FP32, against the oracle."""
    need_gpu()
    flush("[gpu] 16^3x32 whole-lattice Schur parity")
    c = Case((32, 16, 16, 16), seed=231, qhat=-1)
    try:
        psi_e = c.spinor(232)[c.even]
        out = torch.empty_like(to_dev(psi_e))
        c.D.apply_eo(out, to_dev(psi_e), "f64", "eo")
        exp = odirac.apply_schur(c.f, psi_e)
        assert rel(out.cpu().numpy(), exp) <= 1e-13
        nat = c.D.to_native(to_dev(psi_e.astype(np.complex64)), "f32", "eo", sites=1)
        o32 = c.D.native_empty("f32", 1)
        c.D.apply_eo(o32, nat, "f32", "native")
        g32 = c.D.from_native(o32, "f32", "eo", sites=1).cpu().numpy()
        assert rel(g32, odirac.apply_schur(c.f, psi_e.astype(np.complex64).astype(np.complex128))) <= 1e-6
    finally:
        c.D.close()
