"""Schwarz alternating procedure (SAP), the block preconditioner of openQxD's solver
(the paper's outlook names SAP-preconditioned GCR as openQxD's solver); FP64 reference.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Reading (the paper gives the name only; the method is Luscher's multiplicative Schwarz
preconditioner, restated here):
  * blocks: the lattice is tiled by blocks of extent bs (bs_mu divides L_mu, an even number of
    blocks in every direction); a block's colour is the parity of the sum of its block
    coordinates, so blocks of one colour never share a face;
  * D_blk: the operator restricted to a block, hops that leave the block dropped (Dirichlet);
  * block solver: nmr minimal-residual steps on D_blk from zero, each
        v = D_blk r,  w = <v, r> / <v, v>,  delta += w r,  r -= w v;
  * one application psi = M r: psi = 0, rho = r; ncy times, for colour 0 then colour 1: on every
    block of that colour delta = (block solver)(rho on the block); psi += delta; rho = r - D psi.
Fields are full LEX spinor fields [V, 4, 3].
"""
from __future__ import annotations

import numpy as np

from . import dirac
from . import geometry as geo


def check_blocks(L, bs, cstar: int = 0) -> None:
    for m in range(4):
        if bs[m] < 1 or L[m] % bs[m] != 0 or (L[m] // bs[m]) % 2 != 0:
            raise ValueError("block extents must divide the lattice into an even number of blocks per direction")
    if cstar >= 2 and (L[1] // 2) % (2 * bs[1]) != 0:
        # crossing a shifted boundary moves x1 by L1/2: an odd number of blocks would join two
        # blocks of one colour across that face
        raise ValueError("with C* boundaries the mirror shift L1/2 must be an even number of blocks")


def block_index(L, bs, cstar: int = 0):
    """(block id [V], colour [V]) of every LEX site; ids lexicographic in the block coordinates."""
    check_blocks(L, bs, cstar)
    x = geo.coords(np.arange(geo.volume(L)), L)
    n = x // np.asarray(bs)
    nb = [L[m] // bs[m] for m in range(4)]
    return geo.lex(n, nb), n.sum(axis=1) % 2


def restricted_apply(f: dirac.Fields, psi: np.ndarray, mask: np.ndarray) -> np.ndarray:
    """D_blk on every block selected by the boolean site mask at once.  Blocks of one colour do
    not touch, so masking the input and the output drops exactly the hops that leave a block."""
    m = mask[:, None, None]
    return m * dirac.apply_D(f, m * psi)


def mr_blocks(f: dirac.Fields, rho: np.ndarray, colour: int, bs, nmr: int, history=None) -> np.ndarray:
    """nmr minimal-residual steps on every block of the given colour (one step length per block:
    the inner products are sums over the sites of each block)."""
    ids, col = block_index(f.p.dims, bs, f.p.cstar)
    mask = col == colour
    nblk = int(ids.max()) + 1
    r = np.where(mask[:, None, None], rho, 0.0)
    delta = np.zeros_like(rho)
    for _ in range(nmr):
        v = restricted_apply(f, r, mask)
        vr = (np.conj(v) * r).sum(axis=(1, 2))                                # <v, r> per site
        vv = (np.abs(v) ** 2).sum(axis=(1, 2))
        num = np.bincount(ids, weights=vr.real, minlength=nblk) + 1j * np.bincount(ids, weights=vr.imag, minlength=nblk)
        den = np.bincount(ids, weights=vv, minlength=nblk)
        w = np.where(den > 0, num / np.where(den > 0, den, 1.0), 0.0)[ids]   # per site, its block's w
        w = np.where(mask, w, 0.0)[:, None, None]
        delta += w * r
        r = r - w * v
        if history is not None:
            rb = np.bincount(ids, weights=(np.abs(r) ** 2).sum(axis=(1, 2)), minlength=nblk)
            history.append({b: np.sqrt(rb[b]) for b in np.unique(ids[mask])})
    return delta


def sap(f: dirac.Fields, r: np.ndarray, bs=(4, 4, 4, 4), ncy: int = 4, nmr: int = 4) -> np.ndarray:
    """psi = M_SAP r."""
    psi = np.zeros_like(r)
    rho = r.copy()
    for _ in range(ncy):
        for colour in (0, 1):
            psi += mr_blocks(f, rho, colour, bs, nmr)
            rho = r - dirac.apply_D(f, psi)
    return psi
