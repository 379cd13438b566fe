"""Pins of the oracle operator: closed forms, invariants and brute force, none of which reuses
the oracle's own formula.  A dropped term, a wrong sign, a transposed link, a wrong gamma matrix
or a misplaced boundary phase each fail at least one test here."""
import functools

import numpy as np
import pytest

import gen
from oracle import dirac, geometry as geo

G5 = np.array([1, 1, -1, -1])


def g5(v):
    return v * G5[None, :, None]


def random_fields(L, eps=0.5, kappa=0.12, csw=1.3, csw_qed=0.9, qhat=-1, seed=11, phase=(np.pi, 0.4, -0.9, 1.7)):
    U = gen.su3_field(L, eps, seed)
    th = gen.u1_field(L, 0.3, seed)
    return dirac.Fields(U, th, dirac.Params(L, kappa, csw, csw_qed, qhat, phase))


# ---------------------------------------------------------------- gamma basis (reading R1)
def test_gamma_algebra():
    G = dirac.GAMMA
    for m in range(4):
        assert np.allclose(G[m], G[m].conj().T)
        for n in range(4):
            assert np.allclose(G[m] @ G[n] + G[n] @ G[m], 2 * (m == n) * np.eye(4))
    assert np.array_equal(dirac.GAMMA5, np.diag([1, 1, -1, -1]).astype(complex))
    # sigma_{mu nu} commutes with gamma_5: block-diagonal in chirality
    for m in range(4):
        for n in range(4):
            S = dirac.SIGMA[m][n]
            assert np.abs(S[:2, 2:]).max() == 0 and np.abs(S[2:, :2]).max() == 0


# ---------------------------------------------------------------- free field closed form
@pytest.mark.parametrize("L,qhat", [((4, 2, 6, 4), 2), ((2, 4, 4, 6), -1)])
def test_free_field_plane_wave(L, qhat):
    """U = diag(e^{i alpha_{mu a}}) constant, theta_mu constant: a plane wave e^{ip.x} u is an
    eigenvector with D(p') = m0 + sum_mu (1 - cos p'_mu) + i sum_mu gamma_mu sin p'_mu per colour,
    p'_{mu a} = p_mu + qhat theta_mu + alpha_{mu a}, p_mu = (2 pi n_mu + phi_mu) / L_mu."""
    rng = np.random.default_rng(3)
    V = geo.volume(L)
    phi = (np.pi, 0.37, -1.1, 2.3)
    kappa = 0.131
    alpha = rng.uniform(-0.5, 0.5, (4, 3))
    alpha -= alpha.mean(axis=1, keepdims=True)  # SU(3): phases sum to zero
    thc = rng.uniform(-0.3, 0.3, 4)
    U = np.zeros((V, 4, 3, 3), dtype=complex)
    for mu in range(4):
        U[:, mu] = np.diag(np.exp(1j * alpha[mu]))
    th = np.tile(thc, (V, 1))
    f = dirac.Fields(U, th, dirac.Params(L, kappa, 1.7, 1.3, qhat, phi))
    x = geo.coords(np.arange(V), L)
    m0 = 1 / (2 * kappa) - 4
    # gamma matrices written out independently of the oracle module
    s1 = np.array([[0, 1], [1, 0]]); s2 = np.array([[0, -1j], [1j, 0]]); s3 = np.array([[1, 0], [0, -1]])
    z, e = np.zeros((2, 2)), np.eye(2)
    gam = [np.block([[z, -e], [-e, z]])] + [np.block([[z, -1j * s], [1j * s, z]]) for s in (s1, s2, s3)]
    for n in [(0, 0, 0, 0), (1, 0, 2, 1), (L[0] - 1, 1, 1, L[3] - 1)]:
        p = np.array([(2 * np.pi * n[m] + phi[m]) / L[m] for m in range(4)])
        u = rng.normal(size=(4, 3)) + 1j * rng.normal(size=(4, 3))
        psi = np.exp(1j * (x @ p))[:, None, None] * u[None]
        expect = np.zeros_like(psi)
        for a in range(3):
            pp = p + qhat * thc + alpha[:, a]
            Dp = (m0 + np.sum(1 - np.cos(pp))) * np.eye(4) + 1j * sum(gam[m] * np.sin(pp[m]) for m in range(4))
            expect[:, :, a] = np.exp(1j * (x @ p))[:, None] * (Dp @ u[:, a])[None, :]
        got = dirac.apply_D(f, psi)
        assert np.abs(got - expect).max() < 1e-13 * np.abs(expect).max()


# ---------------------------------------------------------------- invariants
def test_gamma5_hermiticity_and_adjoint():
    f = random_fields((4, 2, 2, 4))
    psi, chi = gen.gaussian_spinor(f.p.dims, 1), gen.gaussian_spinor(f.p.dims, 2)
    lhs = np.vdot(chi, g5(dirac.apply_D(f, g5(psi))))
    rhs = np.vdot(dirac.apply_D(f, chi), psi)
    assert abs(lhs - rhs) < 1e-13 * abs(rhs)
    # D^dag written term by term agrees with the adjoint
    assert abs(np.vdot(chi, dirac.apply_Ddag(f, psi)) - rhs) < 1e-13 * abs(rhs)


def test_gauge_covariance():
    """U -> W(x) U W(x+mu)^dag, theta -> theta + lam(x) - lam(x+mu), psi -> e^{i qhat lam} W psi: D' psi' = (D psi)'."""
    L = (4, 2, 4, 2)
    f = random_fields(L, qhat=2)
    W, lam = gen.gauge_transform(L, 77)
    V = geo.volume(L)
    sites = np.arange(V)
    U2 = np.empty_like(f.U)
    th2 = np.empty_like(f.theta)
    for mu in range(4):
        fw = geo.shift(sites, L, mu, 1)
        U2[:, mu] = W @ f.U[:, mu] @ np.conj(np.swapaxes(W[fw], 1, 2))
        th2[:, mu] = f.theta[:, mu] + lam - lam[fw]
    f2 = dirac.Fields(U2, th2, f.p)
    psi = gen.gaussian_spinor(L, 5)
    tr = lambda v: np.exp(1j * f.p.qhat * lam)[:, None, None] * np.einsum("nab,nsb->nsa", W, v)  # noqa: E731
    lhs = dirac.apply_D(f2, tr(psi))
    rhs = tr(dirac.apply_D(f, psi))
    assert np.abs(lhs - rhs).max() < 1e-12 * np.abs(rhs).max()
    # the clover matrix transforms as W A W^dag (colour only)
    A, A2 = f.clover(), f2.clover()
    Wbig = np.einsum("st,nab->nsatb", np.eye(4), W).reshape(V, 12, 12)
    assert np.abs(A2 - Wbig @ A @ np.conj(np.swapaxes(Wbig, 1, 2))).max() < 1e-13


def test_clover_structure():
    f = random_fields((2, 4, 2, 4))
    A = f.clover()
    assert np.abs(A - np.conj(np.swapaxes(A, 1, 2))).max() == 0.0  # Hermitian (Sec. 2, Sec. 4.3)
    assert np.abs(A[:, :6, 6:]).max() == 0.0 and np.abs(A[:, 6:, :6]).max() == 0.0  # chirality blocks
    assert np.abs(dirac.unpack_clover(dirac.pack_clover(A)) - A).max() == 0.0


def test_unit_links_give_zero_clover():
    L = (4, 2, 2, 2)
    V = geo.volume(L)
    f = dirac.Fields(gen.unit_links(L), np.zeros((V, 4)), dirac.Params(L, 0.125, 1.9, 1.4, 2))
    assert np.abs(f.clover() - 4.0 * np.eye(12)).max() == 0.0  # 4 + m0 = 1/(2 kappa) = 4


def test_u1_only_clover_is_colour_diagonal():
    L = (4, 2, 2, 4)
    V = geo.volume(L)
    f = dirac.Fields(gen.unit_links(L), gen.u1_field(L, 0.3, 9), dirac.Params(L, 0.12, 1.6, 1.0, -1))
    A = f.clover().reshape(V, 4, 3, 4, 3)
    off = A.copy()
    for a in range(3):
        off[:, :, a, :, a] = 0
    assert np.abs(off).max() == 0.0
    assert np.abs(A[:, :, 0, :, 0] - A[:, :, 1, :, 1]).max() == 0.0
    assert np.abs(A[:, :, 0, :, 0] - np.eye(4) / 0.24).max() > 1e-3  # the U(1) term is there


def test_clover_constant_abelian_flux_closed_form():
    """Constant flux B in the (1,2) plane and B' in the (0,3) plane (quantised so the plaquette is
    e^{iB} everywhere, wrap included): the SW term reduces by hand to
      A = 1/(2 kappa) + 1/2 [ S_12 (c_sw diag sin B_a + c_qed qhat sin B) - S_03 (c_sw diag sin B'_a + c_qed qhat sin B') ]
    with S_12 = diag(1,-1,1,-1), S_03 = diag(1,-1,-1,1) in spin (sigma_12 = -S_12, sigma_03 = S_03)."""
    L = (6, 4, 2, 2)
    V = geo.volume(L)
    x = geo.coords(np.arange(V), L)
    kappa, csw, cq, qhat = 0.13, 1.7, 0.8, -2
    B = 2 * np.pi * 1 / L[1]
    Bp = 2 * np.pi * 1 / L[0]
    Ba = 2 * np.pi * np.array([1, 2, -3]) / L[1]
    Bpa = 2 * np.pi * np.array([-1, 2, -1]) / L[0]
    th = np.zeros((V, 4))
    th[:, 2] = B * x[:, 1]
    th[:, 3] = Bp * x[:, 0]
    U = gen.unit_links(L)
    U[:, 2] = np.exp(1j * np.outer(x[:, 1], Ba))[:, :, None] * np.eye(3)
    U[:, 3] = np.exp(1j * np.outer(x[:, 0], Bpa))[:, :, None] * np.eye(3)
    f = dirac.Fields(U, th, dirac.Params(L, kappa, csw, cq, qhat))
    S12 = np.diag([1, -1, 1, -1])
    S03 = np.diag([1, -1, -1, 1])
    c12 = np.diag(csw * np.sin(Ba) + cq * qhat * np.sin(B))
    c03 = np.diag(csw * np.sin(Bpa) + cq * qhat * np.sin(Bp))
    expect = np.eye(12) / (2 * kappa) + 0.5 * (np.kron(S12, c12) - np.kron(S03, c03))
    assert np.abs(f.clover() - expect[None]).max() < 1e-14


def _su2_mul(p, q):
    """(s, v) pairs for the SU(2) element s + i v.sigma: (s1 s2 - v1.v2, s1 v2 + s2 v1 - v1 x v2)."""
    return p[0] * q[0] - np.dot(p[1], q[1]), p[0] * q[1] + q[0] * p[1] - np.cross(p[1], q[1])


def _su2_dag(p):
    return p[0], -p[1]


def _su2_in_su3(p):
    """s + i v.sigma on colours 0, 1 and 1 on colour 2."""
    s, (v1, v2, v3) = p
    return np.array([[s + 1j * v3, 1j * v1 + v2, 0], [1j * v1 - v2, s - 1j * v3, 0], [0, 0, 1]], dtype=complex)


def test_clover_non_abelian_constant_links_closed_form():
    """Constant links g = exp(i a m.sigma) in direction 0 and h = exp(i b n.sigma) in direction 1 (unit
    vectors m, n in general position), in the SU(2) of colours 0 and 1, unit links elsewhere and
    theta = 0.  Every leaf of the (0, 1)
    plane is then a group commutator (g h g^-1 h^-1, h g^-1 h^-1 g, g^-1 h^-1 g h, h^-1 g h g^-1),
    computed here with the SU(2) product rule.  With s + i w.tau the sum of the four leaves
    (tau the Pauli matrices on colours 0, 1), F_01 = (Q - Q^dag)/8 = (i/4) w.tau, and the two
    terms (0, 1) and (1, 0) of the clover sum are equal, so
    A = (4 + m0) 1 + c_sw (i/2) sigma_01 (x) F_01 = 1/(2 kappa) - (c_sw / 8) diag(s1, -s1) (x) w.tau
    (sigma_01 = diag(sigma_1, -sigma_1) in the chiral basis).  The commutators point along m x n,
    which has all three components here, so the clover block mixes colours 0 and 1: the SU(3) term
    on a field whose plaquettes do not commute with the links."""
    L = (4, 4, 2, 2)
    a, b = 0.37, -0.61
    kappa, csw = 0.124, 1.7
    m = np.array([np.cos(0.8), np.sin(0.8), 0.0])
    n = np.array([0.0, np.cos(0.3), np.sin(0.3)])
    g = (np.cos(a), np.sin(a) * m)
    h = (np.cos(b), np.sin(b) * n)
    gd, hd = _su2_dag(g), _su2_dag(h)
    prod = lambda *ps: functools.reduce(_su2_mul, ps)  # noqa: E731
    leaves = [prod(g, h, gd, hd), prod(h, gd, hd, g), prod(gd, hd, g, h), prod(hd, g, h, gd)]
    w = sum(l[1] for l in leaves)
    assert np.min(np.abs(w)) > 1e-3  # genuinely non-abelian: every colour Pauli component present
    V = int(np.prod(L))
    U = gen.unit_links(L)
    U[:, 0] = _su2_in_su3(g)
    U[:, 1] = _su2_in_su3(h)
    f = dirac.Fields(U, np.zeros((V, 4)), dirac.Params(L, kappa, csw, 0.9, -1))
    pauli = [np.array([[0, 1], [1, 0]]), np.array([[0, -1j], [1j, 0]]), np.array([[1, 0], [0, -1]])]
    wt = np.zeros((3, 3), dtype=complex)
    wt[:2, :2] = sum(wk * pk for wk, pk in zip(w, pauli))
    s01 = np.zeros((4, 4), dtype=complex)
    s01[:2, :2] = pauli[0]
    s01[2:, 2:] = -pauli[0]
    expect = np.eye(12) / (2 * kappa) - (csw / 8) * np.kron(s01, wt)
    assert np.abs(f.clover() - expect[None]).max() < 1e-14


def test_clover_linear_in_coefficients():
    L = (2, 2, 4, 2)
    f0 = random_fields(L, csw=0.0, csw_qed=0.0)
    f1 = random_fields(L, csw=1.0, csw_qed=0.0)
    f2 = random_fields(L, csw=0.0, csw_qed=1.0)
    f3 = random_fields(L, csw=2.5, csw_qed=-0.7)
    A0 = f0.clover()
    assert np.abs(f3.clover() - A0 - 2.5 * (f1.clover() - A0) + 0.7 * (f2.clover() - A0)).max() < 1e-13


# ---------------------------------------------------------------- even-odd blocks against dense D
def _eo_dense(f):
    V = f.V
    perm = geo.lex_to_eo_perm(f.p.dims)  # EO position -> Lambda
    def apply_eo(v):
        full = np.zeros((V, 4, 3), dtype=complex)
        full[perm] = v.reshape(V, 4, 3)
        return dirac.apply_D(f, full)[perm].reshape(-1)
    return dirac.dense(apply_eo, 12 * V)


def test_schur_equals_dense_schur_complement():
    f = random_fields((2, 2, 2, 2))
    D = _eo_dense(f)
    n = D.shape[0] // 2
    Dee, Deo, Doe, Doo = D[:n, :n], D[:n, n:], D[n:, :n], D[n:, n:]
    S = Dee - Deo @ np.linalg.solve(Doo, Doe)
    Shat = dirac.dense(lambda v: dirac.apply_schur(f, v.reshape(-1, 4, 3)), n)
    assert np.abs(Shat - S).max() < 1e-13 * np.abs(S).max()
    # the single blocks
    assert np.abs(dirac.dense(lambda v: dirac.apply_Doe(f, v.reshape(-1, 4, 3)), n) - Doe).max() < 1e-14
    assert np.abs(dirac.dense(lambda v: dirac.apply_Deo(f, v.reshape(-1, 4, 3)), n) - Deo).max() < 1e-14
    assert np.abs(dirac.dense(lambda v: dirac.apply_clover(f, v.reshape(-1, 4, 3), 1), n) - Doo).max() < 1e-14
    # the adjoint Schur operator is the conjugate transpose, and gamma_5-hermitian
    Sd = dirac.dense(lambda v: dirac.apply_schur_dag(f, v.reshape(-1, 4, 3)), n)
    assert np.abs(Sd - S.conj().T).max() < 1e-13 * np.abs(S).max()
    g = np.tile(np.repeat(G5, 3), n // 12)
    assert np.abs(g[:, None] * S * g[None, :] - S.conj().T).max() < 1e-13 * np.abs(S).max()


def test_schur_at_sampled_sites_matches_full():
    f = random_fields((4, 4, 2, 4))
    ev, _ = dirac.even_odd(f)
    psi_e = gen.gaussian_spinor(f.p.dims, 3)[ev]
    full = dirac.apply_schur(f, psi_e)
    pick = np.array([0, 5, 17, len(ev) - 1])
    f_fresh = random_fields((4, 4, 2, 4))  # no cached clover: the per-site path
    assert np.abs(dirac.schur_at(f_fresh, psi_e, ev[pick]) - full[pick]).max() < 1e-13


def test_singular_block_rule():
    A = np.tile(np.eye(12, dtype=complex), (3, 1, 1))
    A[1, 7, 7] = 0.0  # site 1, lower block: exactly singular
    A[2, :6, :6] = np.outer(np.arange(1, 7), np.arange(1, 7))  # rank one
    bad = dirac.singular_blocks(A)
    assert bad.tolist() == [[False, False], [False, True], [True, False]]
