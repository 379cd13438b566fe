"""Pins of the oracle's C* boundary conditions (Sec. 4.2: the lattice doubled in direction 1,
shifted boundaries; reading: crossing the boundary of a C* direction mu >= 2 moves x1 by half the
doubled extent).  Graph facts (bijection, inverse, parity, closed plaquettes), a free-field closed
form whose momenta carry the shift, gamma_5-hermiticity and gauge covariance."""
import numpy as np
import pytest

import gen
from oracle import dirac, geometry as geo

G5 = np.array([1, 1, -1, -1])
SHAPES = [((4, 8, 4, 6), 2), ((2, 8, 6, 4), 3), ((4, 4, 2, 2), 3)]


@pytest.mark.parametrize("L,cs", SHAPES)
def test_shift_is_a_parity_flipping_bijection_with_inverse(L, cs):
    lam = np.arange(geo.volume(L))
    par = geo.parity(geo.coords(lam, L))
    for mu in range(4):
        f = geo.shift(lam, L, mu, 1, cs)
        assert np.array_equal(np.sort(f), lam)
        assert np.array_equal(geo.shift(f, L, mu, -1, cs), lam)
        assert np.all(geo.parity(geo.coords(f, L)) != par)


@pytest.mark.parametrize("L,cs", SHAPES)
def test_shift_by_hand_and_plaquettes_close(L, cs):
    # crossing the x3 boundary forward from x = (1, 1, 0, L3 - 1) lands at (1, 1 + L1/2, 0, 0) when cs = 3
    x = np.array([1, 1, 0, L[3] - 1])
    y = geo.coords(geo.shift(geo.lex(x, L), L, 3, 1, cs), L)
    assert list(y) == [1, 1 + (L[1] // 2 if cs >= 3 else 0), 0, 0]
    # x2 boundary backward from (0, L1 - 1, 0, 1): x1 + L1/2 wraps
    x = np.array([0, L[1] - 1, 0, 1])
    y = geo.coords(geo.shift(geo.lex(x, L), L, 2, -1, cs), L)
    assert list(y) == [0, (L[1] - 1 + L[1] // 2) % L[1], L[2] - 1, 1]
    lam = np.arange(geo.volume(L))
    for mu in range(4):
        for nu in range(4):
            if mu != nu:
                s = lambda v, d, k: geo.shift(v, L, d, k, cs)  # noqa: E731
                assert np.array_equal(s(s(s(s(lam, mu, 1), nu, 1), mu, -1), nu, -1), lam)


def test_cstar_rejects_extents_that_break_the_checkerboard():
    with pytest.raises(ValueError):
        geo.check_dims((4, 6, 4, 4), 2)   # L1 / 2 = 3 is odd
    geo.check_dims((4, 6, 4, 4), 1)       # one C* direction: plain doubling, any even L1


@pytest.mark.parametrize("cs", [2, 3])
def test_free_field_with_shifted_momenta(cs):
    """Constant diagonal links: e^{ip.x} u is an eigenvector when the momenta follow the shifted
    boundaries, p_k L_k = 2 pi n_k + phi_k + p_1 L1/2 for the C* directions k >= 2, with
    D(p') = m0 + sum (1 - cos p'_mu) + i sum gamma_mu sin p'_mu per colour."""
    L = (4, 8, 4, 6)
    rng = np.random.default_rng(5)
    V = geo.volume(L)
    phi = (np.pi, 0.0, 0.3, -0.7)
    kappa, qhat = 0.127, -1
    alpha = rng.uniform(-0.5, 0.5, (4, 3))
    alpha -= alpha.mean(axis=1, keepdims=True)
    thc = rng.uniform(-0.3, 0.3, 4)
    U = np.zeros((V, 4, 3, 3), dtype=complex)
    for mu in range(4):
        U[:, mu] = np.diag(np.exp(1j * alpha[mu]))
    f = dirac.Fields(U, np.tile(thc, (V, 1)), dirac.Params(L, kappa, 1.1, 0.7, qhat, phi, cstar=cs))
    x = geo.coords(np.arange(V), L)
    m0 = 1 / (2 * kappa) - 4
    s1 = np.array([[0, 1], [1, 0]]); s2 = np.array([[0, -1j], [1j, 0]]); s3 = np.array([[1, 0], [0, -1]])
    z, e = np.zeros((2, 2)), np.eye(2)
    gam = [np.block([[z, -e], [-e, z]])] + [np.block([[z, -1j * s], [1j * s, z]]) for s in (s1, s2, s3)]
    for n in [(0, 1, 0, 0), (1, 3, 2, 1), (3, 5, 1, 4)]:
        p = np.zeros(4)
        p[0] = (2 * np.pi * n[0] + phi[0]) / L[0]
        p[1] = (2 * np.pi * n[1] + phi[1]) / L[1]
        for k in (2, 3):
            shift = p[1] * (L[1] // 2) if k <= cs else 0.0
            p[k] = (2 * np.pi * n[k] + phi[k] + shift) / L[k]
        u = rng.normal(size=(4, 3)) + 1j * rng.normal(size=(4, 3))
        psi = np.exp(1j * (x @ p))[:, None, None] * u[None]
        expect = np.zeros_like(psi)
        for a in range(3):
            pp = p + qhat * thc + alpha[:, a]
            Dp = (m0 + np.sum(1 - np.cos(pp))) * np.eye(4) + 1j * sum(gam[m] * np.sin(pp[m]) for m in range(4))
            expect[:, :, a] = np.exp(1j * (x @ p))[:, None] * (Dp @ u[:, a])[None, :]
        got = dirac.apply_D(f, psi)
        assert np.abs(got - expect).max() < 1e-12 * np.abs(expect).max()
        # the same wave on the unshifted lattice is not an eigenvector (the shift matters)
        f0 = dirac.Fields(U, np.tile(thc, (V, 1)), dirac.Params(L, kappa, 1.1, 0.7, qhat, phi, cstar=0))
        if abs(p[1] * (L[1] // 2)) % (2 * np.pi) > 1e-9:
            assert np.abs(dirac.apply_D(f0, psi) - expect).max() > 1e-3 * np.abs(expect).max()


@pytest.mark.parametrize("L,cs", SHAPES[:2])
def test_gamma5_hermiticity_and_gauge_covariance(L, cs):
    U = gen.su3_field(L, 0.5, 13)
    th = gen.u1_field(L, 0.3, 13)
    p = dirac.Params(L, 0.121, 1.4, 0.8, 2, (np.pi, 0.0, 0.5, -0.3), cstar=cs)
    f = dirac.Fields(U, th, p)
    psi, chi = gen.gaussian_spinor(L, 1), gen.gaussian_spinor(L, 2)
    g5 = lambda v: v * G5[None, :, None]  # noqa: E731
    lhs = np.vdot(chi, g5(dirac.apply_D(f, g5(psi))))
    rhs = np.vdot(dirac.apply_D(f, chi), psi)
    assert abs(lhs - rhs) < 1e-12 * abs(lhs)
    assert np.abs(dirac.apply_Ddag(f, psi) - g5(dirac.apply_D(f, g5(psi)))).max() < 1e-12
    # gauge transformation along the shifted graph: U -> W(x) U W(n(x, mu))^dag
    W, lam = gen.gauge_transform(L, 71)
    V = geo.volume(L)
    sites = np.arange(V)
    U2, th2 = np.empty_like(U), np.empty_like(th)
    for mu in range(4):
        fw = geo.shift(sites, L, mu, 1, cs)
        U2[:, mu] = W @ U[:, mu] @ np.conj(np.swapaxes(W[fw], 1, 2))
        th2[:, mu] = th[:, mu] + lam - lam[fw]
    f2 = dirac.Fields(U2, th2, p)
    tr = lambda v: np.exp(1j * p.qhat * lam)[:, None, None] * np.einsum("nab,nsb->nsa", W, v)  # noqa: E731
    a, b = dirac.apply_D(f2, tr(psi)), tr(dirac.apply_D(f, psi))
    assert np.abs(a - b).max() < 1e-12 * np.abs(b).max()
    # with the plain neighbours the transformed field is not covariant (the shift matters)
    f3 = dirac.Fields(U2, th2, dirac.Params(L, 0.121, 1.4, 0.8, 2, (np.pi, 0.0, 0.5, -0.3), cstar=0))
    assert np.abs(dirac.apply_D(f3, tr(psi)) - b).max() > 1e-3 * np.abs(b).max()
