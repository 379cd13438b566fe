"""Rounding envelope of the even-odd Schur operator with 16-bit field storage.

Test infrastructure: a tolerance, derived from the storage format before any GPU result is seen,
for comparing a Schur apply whose fields are stored in FP16 or BF16 (FP32 arithmetic) with the
plain FP64 oracle.

What 16-bit storage rounds: the input spinor, the two stored rows of every SU(3) link (the third
row is rebuilt from them as the conjugate cross product, so it inherits their rounding), the
U(1) phase of the link kept as the pair (cos, sin), the packed clover blocks A_ee and the packed
inverse blocks A_oo^-1, the intermediate odd-site vector t = A_oo^-1 D_oe psi, and the output.
Rounding to a format with unit roundoff u changes a real number by at most u times its size.

The envelope applies perturbations of that largest size, u |x| with a random sign on every
real component, at each of these points and pushes them through the exact operator (the
oracle's hopping term and clover products in FP64), then takes the relative change of the
output, in norm and element-wise (largest deviation relative to the largest entry).  Real
rounding errors are spread uniformly below u |x|, so a 16-bit evaluation lands well inside; a
wrong sign, index, phase or boundary term moves the output by O(1).
"""
from __future__ import annotations

import numpy as np

from oracle import dirac as odirac

U_FP16 = 2.0 ** -11
U_BF16 = 2.0 ** -8


def _perturb(rng, x, u):
    x = np.asarray(x)
    if np.iscomplexobj(x):
        sr = rng.choice([-1.0, 1.0], x.shape)
        si = rng.choice([-1.0, 1.0], x.shape)
        return x + u * (x.real * sr + 1j * x.imag * si)
    return x + u * x * rng.choice([-1.0, 1.0], x.shape)


def perturbed_fields(f: odirac.Fields, rng, u: float) -> odirac.Fields:
    """A copy of f whose links and clover blocks carry storage-sized perturbations."""
    g = odirac.Fields(f.U, f.theta, f.p)
    r0 = _perturb(rng, f.U[..., 0, :], u)
    r1 = _perturb(rng, f.U[..., 1, :], u)
    r2 = np.conj(np.cross(r0, r1))
    Up = np.stack([r0, r1, r2], axis=-2)
    z = _perturb(rng, np.exp(1j * f.p.qhat * f.theta), u)
    g.Vlink = z[:, :, None, None] * Up
    A = odirac.pack_clover(f.clover())
    Ai = odirac.pack_clover(f.clover_inv())
    g._clover = {"A": odirac.unpack_clover(_perturb(rng, A, u)), "Ainv": odirac.unpack_clover(_perturb(rng, Ai, u))}
    return g


class Env:
    def __init__(self):
        self.norm = 0.0
        self.max = 0.0

    def add(self, a, b):
        self.norm = max(self.norm, float(np.linalg.norm(a - b) / np.linalg.norm(b)))
        self.max = max(self.max, float(np.abs(a - b).max() / np.abs(b).max()))

    def check(self, got, exact, what=""):
        n = float(np.linalg.norm(got - exact) / np.linalg.norm(exact))
        m = float(np.abs(got - exact).max() / np.abs(exact).max())
        msg = f"{what}: |d|/|y| {n:.2e} (envelope {self.norm:.2e}), max|d|/max|y| {m:.2e} (envelope {self.max:.2e})"
        assert n <= self.norm and m <= self.max, msg
        return msg


def schur_envelope(f: odirac.Fields, psi_e: np.ndarray, u: float, samples: int = 2, seed: int = 0) -> Env:
    """Envelope of D-hat psi_e with every stored operand perturbed by u (see the module text)."""
    exact = odirac.apply_schur(f, psi_e)
    rng = np.random.default_rng(seed)
    env = Env()
    for _ in range(samples):
        g = perturbed_fields(f, rng, u)
        x = _perturb(rng, psi_e, u)
        t = _perturb(rng, odirac.apply_clover(g, odirac.apply_Doe(g, x), 1, inverse=True), u)
        y = _perturb(rng, odirac.apply_clover(g, x, 0) - odirac.apply_Deo(g, t), u)
        env.add(y, exact)
    return env
