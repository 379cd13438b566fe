"""openQxD's storage of the fields (Sec. 4.1, Fig. gauge), FP64 reference permutations.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Site order: eq. (ipt) with cache block B (geometry.ipt).  Spinors and clover blocks are stored
per site in that order with the same per-site layout as the library's LEX boundary (12 complex
spinor components, spin-major, colour fastest; 2 x 36 clover reals).

Gauge field: openQxD keeps, for every odd point only, the 8 links attached to it -- the forward
link in each direction and the forward link of the neighbour behind it (Fig. gauge: arrows at the
odd points in every direction, none at the even points).  Every link of the lattice is one of
them exactly once, since the forward link of an even point y in direction mu ends at the odd
point y + mu.  The paper does not give the order of the 8; the reading taken is
    slot 2 mu     : U_mu(x)          (from x to x + mu)
    slot 2 mu + 1 : U_mu(x - mu)     (from x - mu to x)
for the odd point with index ipt(x) = V/2 + k, stored at position k.  The U(1) angles are stored
in the same slots.
"""
from __future__ import annotations

import numpy as np

from . import geometry as geo


def check_block(L, B) -> None:
    """Cache blocks must tile the lattice, and B3 must be even so that the two sites of every pair
    (2j, 2j + 1) of block-lexicographic order have opposite parity (floor(./2) is then one-to-one
    on each parity)."""
    for m in range(4):
        if B[m] < 1 or L[m] % B[m] != 0:
            raise ValueError("every cache-block extent must divide the lattice extent")
    if B[3] % 2 != 0:
        raise ValueError("the cache-block extent B3 must be even")


def site_order(L, B) -> np.ndarray:
    """perm[ipt] = Lambda: the LEX site stored at each position of openQxD's order."""
    check_block(L, B)
    lam = np.arange(geo.volume(L), dtype=np.int64)
    xh = geo.ipt(geo.coords(lam, L), L, B)
    perm = np.empty_like(lam)
    perm[xh] = lam
    return perm


def links_to_openqxd(U: np.ndarray, theta, L, B, cstar: int = 0):
    """LEX links U [V][4][3][3] (and angles theta [V][4] or None) -> openQxD's odd-point storage
    u [V/2][8][3][3], a [V/2][8] (None without angles)."""
    check_block(L, B)
    V = geo.volume(L)
    perm = site_order(L, B)
    odd = perm[V // 2:]                     # Lambda of the odd point at position k
    u = np.empty((V // 2, 8, 3, 3), dtype=np.complex128)
    a = None if theta is None else np.empty((V // 2, 8))
    for mu in range(4):
        back = geo.shift(odd, L, mu, -1, cstar)    # Lambda(x - mu)
        u[:, 2 * mu] = U[odd, mu]
        u[:, 2 * mu + 1] = U[back, mu]
        if a is not None:
            a[:, 2 * mu] = theta[odd, mu]
            a[:, 2 * mu + 1] = theta[back, mu]
    return u, a


def links_from_openqxd(u: np.ndarray, a, L, B, cstar: int = 0):
    """The inverse of links_to_openqxd: LEX U [V][4][3][3], theta [V][4] (None without angles)."""
    check_block(L, B)
    V = geo.volume(L)
    perm = site_order(L, B)
    odd = perm[V // 2:]
    U = np.full((V, 4, 3, 3), np.nan, dtype=np.complex128)
    th = None if a is None else np.full((V, 4), np.nan)
    for mu in range(4):
        back = geo.shift(odd, L, mu, -1, cstar)
        U[odd, mu] = u[:, 2 * mu]
        U[back, mu] = u[:, 2 * mu + 1]
        if th is not None:
            th[odd, mu] = a[:, 2 * mu]
            th[back, mu] = a[:, 2 * mu + 1]
    return U, th


def sites_to_openqxd(f: np.ndarray, L, B) -> np.ndarray:
    """Per-site data [V][...] in LEX order -> openQxD's site order."""
    return f[site_order(L, B)]
