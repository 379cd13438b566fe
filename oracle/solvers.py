"""Textbook Krylov solvers in FP64 for the oracle.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper names GCR as the solver family it offloads (Sec. 5.1) and fixes the
stopping rule as a relative residual (1e-12 there).  The methods are written from
their textbook definitions:
  * CGLS: conjugate gradients on the normal equations D^dag D x = D^dag b, tracking the
    residual s = b - D x of the original system (Bjorck, Numerical Methods for Least
    Squares Problems, Sec. 7.4).
  * GCR(m): generalised conjugate residuals with restart m (Eisenstat, Elman, Schultz,
    SIAM J. Numer. Anal. 20 (1983) 345); modified Gram-Schmidt on the q_k = A p_k,
    x updated at the end of each cycle by back-substitution.  With a preconditioner
    p_k = M(r_k) the same recurrence is flexible GCR (FGCR).
  * Even-odd solve (reading R5 of the dirac module): eta-hat_e = eta_e - D_eo A_oo^-1 eta_o,
    solve D-hat psi_e = eta-hat_e, psi_o = A_oo^-1 (eta_o - D_oe psi_e).  The residual of
    the Schur system is normalised by the norm of the full right-hand side: after the
    reconstruction the full residual equals (r-hat_e, 0) in exact arithmetic.
Inner product <a, b> = sum conj(a_i) b_i.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import dirac


@dataclass
class SolveInfo:
    iters: int = 0
    restarts: int = 0
    converged: bool = False
    history: list = field(default_factory=list)  # ||r|| after every iteration


def _norm(v) -> float:
    return float(np.sqrt(np.vdot(v, v).real))


def cgls(apply, apply_dag, b, tol: float, maxiter: int = 10000, x0=None):
    """CG on D^dag D; stops when ||b - D x|| / ||b|| < tol, confirmed by a recomputed residual."""
    info = SolveInfo()
    bnorm = _norm(b)
    x = np.zeros_like(b) if x0 is None else x0.copy()
    s = b - apply(x)
    while info.iters < maxiter:
        r = apply_dag(s)
        p = r.copy()
        rho = np.vdot(r, r).real
        while info.iters < maxiter and _norm(s) >= tol * bnorm:
            w = apply(p)
            alpha = rho / np.vdot(w, w).real
            x = x + alpha * p
            s = s - alpha * w
            r = apply_dag(s)
            rho_new = np.vdot(r, r).real
            p = r + (rho_new / rho) * p
            rho = rho_new
            info.iters += 1
            info.history.append(_norm(s))
        s = b - apply(x)  # a-posteriori check of the recursion
        if _norm(s) < tol * bnorm:
            info.converged = True
            break
        info.restarts += 1
    return x, info


def gcr(apply, b, tol: float, restart: int = 32, maxiter: int = 10000, x0=None, precond=None, norm_ref=None):
    """GCR(restart) (FGCR when `precond` is given); stops when ||b - A x|| <= tol * norm_ref."""
    info = SolveInfo()
    ref = _norm(b) if norm_ref is None else float(norm_ref)
    x = np.zeros_like(b) if x0 is None else x0.copy()
    r = b - apply(x)
    if _norm(r) <= tol * ref:
        info.converged = True
        return x, info
    while info.iters < maxiter:
        P, Q = [], []
        alpha = []
        beta = np.zeros((restart, restart), dtype=np.complex128)
        gamma = []
        for k in range(restart):
            p = precond(r) if precond is not None else r.copy()
            q = apply(p)
            for j in range(k):
                beta[j, k] = np.vdot(Q[j], q)
                q = q - beta[j, k] * Q[j]
            g = _norm(q)
            q = q / g
            a = np.vdot(q, r)
            r = r - a * q
            P.append(p)
            Q.append(q)
            alpha.append(a)
            gamma.append(g)
            info.iters += 1
            info.history.append(_norm(r))
            if info.history[-1] <= tol * ref or info.iters >= maxiter:
                break
        n = len(P)
        c = np.zeros(n, dtype=np.complex128)
        for j in range(n - 1, -1, -1):
            c[j] = (alpha[j] - sum(beta[j, k] * c[k] for k in range(j + 1, n))) / gamma[j]
        for k in range(n):
            x = x + c[k] * P[k]
        r = b - apply(x)
        if _norm(r) <= tol * ref:
            info.converged = True
            break
        info.restarts += 1
    return x, info


def solve_eo(f: dirac.Fields, eta: np.ndarray, tol: float, restart: int = 32, maxiter: int = 10000):
    """Even-odd preconditioned GCR solve of D psi = eta (full LEX fields [V, 4, 3])."""
    ev, od = dirac.even_odd(f)
    eta_e, eta_o = eta[ev], eta[od]
    eta_hat = eta_e - dirac.apply_Deo(f, dirac.apply_clover(f, eta_o, 1, inverse=True))
    apply = lambda v: dirac.apply_schur(f, v.reshape(-1, 4, 3)).reshape(-1)  # noqa: E731
    psi_e, info = gcr(apply, eta_hat.reshape(-1), tol, restart, maxiter, norm_ref=_norm(eta))
    psi_e = psi_e.reshape(-1, 4, 3)
    psi_o = dirac.apply_clover(f, eta_o - dirac.apply_Doe(f, psi_e), 1, inverse=True)
    psi = np.zeros_like(eta)
    psi[ev], psi[od] = psi_e, psi_o
    return psi, info


def rel_residual(f: dirac.Fields, psi: np.ndarray, eta: np.ndarray) -> float:
    """||eta - D psi|| / ||eta||, recomputed with the oracle's operator (the a-posteriori check)."""
    return _norm(eta - dirac.apply_D(f, psi)) / _norm(eta)
