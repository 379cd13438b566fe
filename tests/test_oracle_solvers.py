"""Oracle solvers against LAPACK dense solves and the defining properties of each method."""
import numpy as np
import pytest

import gen
from oracle import dirac, geometry as geo, solvers


def cfg1_fields(L=(4, 4, 4, 4), seed=101):
    # the 4^4 plain-method parameters: eps 0.3, theta in (-0.3, 0.3), qhat -1, kappa 0.12, c_sw = c_sw^QED = 1
    return dirac.Fields(gen.su3_field(L, 0.3, seed), gen.u1_field(L, 0.3, seed), dirac.Params(L, 0.12, 1.0, 1.0, -1))


def dense_D(f):
    V = f.V
    return dirac.dense(lambda v: dirac.apply_D(f, v.reshape(V, 4, 3)), 12 * V)


@pytest.fixture(scope="module")
def small():
    L = (2, 2, 2, 4)
    f = dirac.Fields(gen.su3_field(L, 0.5, 3), gen.u1_field(L, 0.3, 3), dirac.Params(L, 0.1245, 1.6, 1.0, 2))
    eta = gen.gaussian_spinor(L, 4)
    exact = np.linalg.solve(dense_D(f), eta.reshape(-1)).reshape(eta.shape)
    return f, eta, exact


def test_eo_gcr_matches_lapack(small):
    f, eta, exact = small
    psi, info = solvers.solve_eo(f, eta, 1e-12)
    assert info.converged
    assert np.linalg.norm(psi - exact) < 1e-10 * np.linalg.norm(exact)
    assert solvers.rel_residual(f, psi, eta) < 1e-12


def test_cgls_matches_lapack(small):
    f, eta, exact = small
    psi, info = solvers.cgls(lambda v: dirac.apply_D(f, v), lambda v: dirac.apply_Ddag(f, v), eta, 1e-12)
    assert info.converged
    assert np.linalg.norm(psi - exact) < 1e-10 * np.linalg.norm(exact)


def test_gcr_residual_monotone_and_restarted(small):
    f, eta, exact = small
    ev, _ = dirac.even_odd(f)
    apply = lambda v: dirac.apply_schur(f, v.reshape(-1, 4, 3)).reshape(-1)  # noqa: E731
    b = eta[ev].reshape(-1)
    x, info = solvers.gcr(apply, b, 1e-12, restart=4)
    assert info.converged and info.restarts > 0
    h = np.array(info.history)
    # within a cycle GCR minimises ||r|| over a growing space: non-increasing
    assert np.all(np.diff(h[:4]) <= 1e-14 * h[0])
    assert np.linalg.norm(b - apply(x)) <= 1e-12 * np.linalg.norm(b)


def test_fgcr_with_exact_preconditioner_converges_in_one_step(small):
    f, eta, exact = small
    D = dense_D(f)
    b = eta.reshape(-1)
    x, info = solvers.gcr(lambda v: D @ v, b, 1e-12, precond=lambda r: np.linalg.solve(D, r))
    assert info.iters == 1 and np.linalg.norm(x - exact.reshape(-1)) < 1e-11 * np.linalg.norm(exact)


def test_full_residual_equals_schur_residual(small):
    """After reconstruction, eta - D psi = (r-hat_e, 0): the odd half of the residual vanishes."""
    f, eta, _ = small
    ev, od = dirac.even_odd(f)
    rng = np.random.default_rng(0)
    psi_e = rng.normal(size=(len(ev), 4, 3)) + 0j
    eta_hat = eta[ev] - dirac.apply_Deo(f, dirac.apply_clover(f, eta[od], 1, inverse=True))
    psi_o = dirac.apply_clover(f, eta[od] - dirac.apply_Doe(f, psi_e), 1, inverse=True)
    psi = np.zeros_like(eta)
    psi[ev], psi[od] = psi_e, psi_o
    r = eta - dirac.apply_D(f, psi)
    assert np.abs(r[od]).max() < 1e-13
    assert np.abs(r[ev] - (eta_hat - dirac.apply_schur(f, psi_e))).max() < 1e-13


def test_4c4_cgls_and_eo_gcr_agree():
    """4^4 at the plain-method parameters: CGLS to 1e-10 and even-odd GCR to 1e-12 agree within the
    error bound cond(D) * 1e-10 (cond(D) is about 10 here) and both pass the a-posteriori check."""
    f = cfg1_fields()
    eta = gen.gaussian_spinor(f.p.dims, 101)
    psi, info = solvers.cgls(lambda v: dirac.apply_D(f, v), lambda v: dirac.apply_Ddag(f, v), eta, 1e-10)
    assert info.converged and solvers.rel_residual(f, psi, eta) < 1e-10
    psi2, info2 = solvers.solve_eo(f, eta, 1e-12)
    assert info2.converged and solvers.rel_residual(f, psi2, eta) < 1e-12
    assert np.linalg.norm(psi - psi2) < 1e-8 * np.linalg.norm(psi2)
