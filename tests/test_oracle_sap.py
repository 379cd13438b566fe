"""Pins of the oracle's Schwarz (SAP) preconditioner: many minimal-residual steps reach the exact
block solve (dense block matrix from unit vectors), an exact colour step zeroes the residual on
that colour, the block residuals never grow, the colouring is a checkerboard of blocks, and SAP
preconditioning cuts the iterations of flexible GCR."""
import numpy as np
import pytest

import gen
from oracle import dirac, geometry as geo, sap, solvers


def fields(L=(4, 4, 4, 8), seed=7):
    return dirac.Fields(gen.su3_field(L, 0.5, seed), gen.u1_field(L, 0.3, seed),
                        dirac.Params(L, 0.124, 1.3, 0.9, -1, (np.pi, 0.0, 0.0, 0.0)))


BS = (2, 2, 2, 2)


@pytest.mark.parametrize("L,cs", [((4, 4, 4, 8), 0), ((4, 8, 4, 4), 3)])
def test_colouring_is_a_block_checkerboard(L, cs):
    ids, col = sap.block_index(L, BS, cs)
    assert len(np.unique(ids)) == geo.volume(L) // 16
    lam = np.arange(geo.volume(L))
    for mu in range(4):
        nb = geo.shift(lam, L, mu, 1, cs)
        cross = ids[nb] != ids
        assert np.all(col[nb][cross] != col[cross])   # a face always joins the two colours
        assert np.all(col[nb][~cross] == col[~cross])
    with pytest.raises(ValueError):
        sap.block_index((4, 4, 4, 6), (2, 2, 2, 2))   # three blocks in direction 3
    with pytest.raises(ValueError):
        sap.block_index((4, 4, 4, 4), (2, 2, 2, 2), 3)  # C* shift of one block: same colours meet


def test_many_mr_steps_reach_the_exact_block_solve():
    f = fields(L=(4, 4, 4, 4))
    ids, col = sap.block_index(f.p.dims, BS)
    rho = gen.gaussian_spinor(f.p.dims, 3)
    delta = sap.mr_blocks(f, rho, 0, BS, 150)
    b = ids[np.argmax(col == 0)]
    s = np.where(ids == b)[0]
    n = 12 * len(s)
    M = np.zeros((n, n), dtype=complex)
    mask = ids == b
    for k in range(n):
        e = np.zeros((f.V, 4, 3), dtype=complex)
        e.reshape(f.V, 12)[s[k // 12], k % 12] = 1.0
        M[:, k] = sap.restricted_apply(f, e, mask)[s].reshape(-1)
    exact = np.linalg.solve(M, rho[s].reshape(-1))
    assert np.abs(delta[s].reshape(-1) - exact).max() < 1e-10 * np.abs(exact).max()
    assert np.all(delta[col == 1] == 0)


def test_exact_colour_step_zeroes_its_residual_and_mr_is_monotone():
    f = fields(L=(4, 4, 4, 4))
    ids, col = sap.block_index(f.p.dims, BS)
    r = gen.gaussian_spinor(f.p.dims, 4)
    hist = []
    delta = sap.mr_blocks(f, r, 1, BS, 150, history=hist)
    res = r - dirac.apply_D(f, delta)
    assert np.abs(res[col == 1]).max() < 1e-9 * np.abs(r).max()
    for b in hist[0]:
        norms = [h[b] for h in hist]
        assert all(n1 <= n0 * (1 + 1e-12) for n0, n1 in zip(norms, norms[1:]))


def test_sap_preconditioned_fgcr_takes_fewer_iterations():
    f = fields(L=(4, 4, 4, 8))
    b = gen.gaussian_spinor(f.p.dims, 5)
    D = lambda v: dirac.apply_D(f, v)  # noqa: E731
    x0, i0 = solvers.gcr(D, b, tol=1e-8, restart=32, maxiter=500)
    x1, i1 = solvers.gcr(D, b, tol=1e-8, restart=32, maxiter=500, precond=lambda v: sap.sap(f, v, BS, ncy=2, nmr=4))
    assert i0.converged and i1.converged
    assert np.linalg.norm(b - D(x1)) < 1e-8 * np.linalg.norm(b)
    assert i1.iters * 3 < i0.iters
