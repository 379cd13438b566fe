"""Site indexing of the oracle (paper Sec. 4.1.1, Space-time coordinates).

Coordinates x = (x0, x1, x2, x3) with x0 the time direction (txyz).
  eq. (lexi):  Lambda(x, L) = L3 L2 L1 x0 + L3 L2 x1 + L3 x2 + x3
  parity:      P(x) = (sum_mu x_mu) mod 2
  eq. (ipt):   xhat = floor((V_B Lambda(n, N_B) + Lambda(b, B)) / 2) + P(x) V / 2
               with b_mu = x_mu mod B_mu and n_mu = floor(x_mu / B_mu).
With one block (B = L) eq. (ipt) reduces to xhat = floor(Lambda(x, L) / 2) + P(x) V / 2,
the even-odd (EO) order of the library boundary.

Reading (the paper is silent): every extent L_mu is even, so that the
checkerboard is consistent across the periodic wrap and floor(Lambda/2) is
one-to-one within a parity.
"""
from __future__ import annotations

import numpy as np


def volume(L) -> int:
    return int(np.prod([int(v) for v in L]))


def lex(x, L) -> np.ndarray:
    """eq. (lexi). x: integer array [..., 4]."""
    x = np.asarray(x, dtype=np.int64)
    L = [int(v) for v in L]
    return L[3] * L[2] * L[1] * x[..., 0] + L[3] * L[2] * x[..., 1] + L[3] * x[..., 2] + x[..., 3]


def coords(lam, L) -> np.ndarray:
    """Inverse of eq. (lexi): Lambda -> x [..., 4]."""
    lam = np.asarray(lam, dtype=np.int64)
    L = [int(v) for v in L]
    x3 = lam % L[3]
    r = lam // L[3]
    x2 = r % L[2]
    r = r // L[2]
    x1 = r % L[1]
    x0 = r // L[1]
    return np.stack([x0, x1, x2, x3], axis=-1)


def parity(x) -> np.ndarray:
    """P(x) = (1 - (-1)^(sum x)) / 2."""
    return np.asarray(x, dtype=np.int64).sum(axis=-1) % 2


def ipt(x, L, B) -> np.ndarray:
    """eq. (ipt): cache-block, even-odd site index of openQxD."""
    x = np.asarray(x, dtype=np.int64)
    L = [int(v) for v in L]
    B = [int(v) for v in B]
    NB = [L[m] // B[m] for m in range(4)]
    b = np.stack([x[..., m] % B[m] for m in range(4)], axis=-1)
    n = np.stack([x[..., m] // B[m] for m in range(4)], axis=-1)
    VB = volume(B)
    return (VB * lex(n, NB) + lex(b, B)) // 2 + parity(x) * (volume(L) // 2)


def eo_index(x, L) -> np.ndarray:
    """eq. (ipt) with a single block B = L: floor(Lambda / 2) + P(x) V / 2."""
    return lex(x, L) // 2 + parity(x) * (volume(L) // 2)


def shift(lam, L, mu: int, step: int, cstar: int = 0) -> np.ndarray:
    """Lambda(x + step * mu-hat) with periodic wrap of the coordinate x_mu (step = +1 or -1).

    C* boundary conditions (Sec. 4.2: the lattice doubled in direction 1, shifted boundaries):
    cstar = number of C* directions, 1 .. cstar.  L[1] is then the doubled extent and direction 1
    is plainly periodic; crossing the boundary of a further C* direction mu (2 <= mu <= cstar)
    also moves x1 by L[1] / 2, into the mirror copy."""
    x = coords(lam, L)
    y = x[..., mu] + step
    cross = (y < 0) | (y >= int(L[mu]))
    x[..., mu] = y % int(L[mu])
    if 2 <= mu <= cstar:
        x[..., 1] = np.where(cross, (x[..., 1] + int(L[1]) // 2) % int(L[1]), x[..., 1])
    return lex(x, L)


def sites_of_parity(L, p: int) -> np.ndarray:
    """Lambda of all sites of parity p, ascending; position k in this list is the EO index k (+ p V/2)."""
    lam = np.arange(volume(L), dtype=np.int64)
    return lam[parity(coords(lam, L)) == p]


def lex_to_eo_perm(L) -> np.ndarray:
    """perm[xhat] = Lambda: an EO-ordered field is field_lex[perm]."""
    lam = np.arange(volume(L), dtype=np.int64)
    perm = np.empty_like(lam)
    perm[eo_index(coords(lam, L), L)] = lam
    return perm


def check_dims(L, cstar: int = 0) -> None:
    if len(L) != 4 or any(int(v) < 2 or int(v) % 2 for v in L):
        raise ValueError(f"lattice extents must be four even numbers >= 2, got {tuple(L)}")
    if not 0 <= cstar <= 3:
        raise ValueError("cstar must be 0 .. 3")
    if cstar >= 2 and int(L[1]) % 4:
        # the mirror shift L1 / 2 must be even, or it would join sites of equal parity
        raise ValueError("with C* boundaries in more than one direction the doubled extent L1 must be a multiple of 4")
