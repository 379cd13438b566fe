"""GPU solvers against the FP64 oracle: the a-posteriori residual is recomputed with the oracle's
operator, and solutions are compared with the oracle's own solve.  Bar on solutions: 1e-9
relative at tolerance 1e-12 (the relative residual the paper uses, Sec. 5.1); at 1e-10 the
error bound is cond(D) * 1e-10."""
import math

import numpy as np
import pytest
import torch

import paper_2502_02490_amd as P
from gpu_util import Case, flush, need_gpu, rel, to_dev
from oracle import dirac as odirac
from oracle import solvers as osolvers

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def case4():
    """4^4, eps = 0.3, kappa = 0.12, c_sw = c_sw^QED = 1, qhat = -1 (the plain-method small case)."""
    need_gpu()
    flush("[gpu] solve case 4^4")
    c = Case((4, 4, 4, 4), eps=0.3, kappa=0.12, csw=1.0, csw_qed=1.0, qhat=-1, seed=101)
    eta = c.spinor(101)
    exact, info = osolvers.solve_eo(c.f, eta, 1e-13)
    assert info.converged
    yield c, eta, exact
    c.D.close()


def test_cgls_4c4(case4):
    c, eta, exact = case4
    x = torch.zeros_like(to_dev(eta))
    info = c.D.solve(x, to_dev(eta), method=P.CGLS, tol=1e-10, max_iter=5000)
    xs = x.cpu().numpy()
    assert info.true_rel_res < 1e-10
    assert osolvers.rel_residual(c.f, xs, eta) < 1e-10
    assert rel(xs, exact) < 20 * 1e-10  # cond(D) ~ 10 on 4^4
    flush(f"[gpu] CGLS 4^4: {info.iters} iterations, residual {info.true_rel_res:.2e}")


@pytest.mark.parametrize("layout", ["lex", "eo"])
def test_eo_gcr_f64_tight(case4, layout):
    c, eta, exact = case4
    from oracle import geometry as geo

    perm = geo.lex_to_eo_perm(c.dims) if layout == "eo" else np.arange(c.V)
    b = to_dev(eta[perm])
    x = torch.zeros_like(b)
    info = c.D.solve(x, b, method=P.GCR, tol=1e-12, restart=32, layout=layout)
    xs = np.empty_like(eta)
    xs[perm] = x.cpu().numpy()
    assert info.true_rel_res < 1e-12
    assert rel(xs, exact) < 1e-9
    assert osolvers.rel_residual(c.f, xs, eta) < 2e-12


def test_gcr_polls_convergence_every_four_iterations():
    """Plain GCR decides convergence on the device and the host reads it every 4 iterations.  A
    cycle of n iterations waits ceil(n / 4) <= (n + 3) / 4 times for the polls and 3 more (the
    back-substitution and the true-residual reads), and a solve adds at most 5 (the start of the
    first cycle and the final checks): at most iters / 4 + 3.75 cycles + 5 <= iters // 4 + 4 cycles
    + 6 waits, against iters + 3 cycles + 5 with one read per iteration.  The solution is the
    oracle's.  Restarts of 5 (not a multiple of 4) make the last poll of a cycle fall on its last
    iteration."""
    need_gpu()
    c = Case((8, 8, 8, 8), eps=0.4, kappa=0.124, seed=111)
    try:
        eta = c.spinor(111)
        for restart in (32, 5):
            x = torch.zeros_like(to_dev(eta))
            info = c.D.solve(x, to_dev(eta), method=P.GCR, tol=1e-11, restart=restart, layout="lex")
            cycles = info.restarts + 1
            flush(f"[gpu] GCR({restart}) 8^4: {info.iters} iterations, {cycles} cycles, {info.host_syncs} host waits")
            assert info.true_rel_res < 1e-11
            assert info.host_syncs <= info.iters // 4 + 4 * cycles + 6, (restart, info.iters, info.host_syncs)
            assert osolvers.rel_residual(c.f, x.cpu().numpy(), eta) < 2e-11
    finally:
        c.D.close()


@pytest.mark.parametrize("inner,itol", [("f32", None), ("f16", None), ("bf16", None)])
def test_mixed_precision_4c4(case4, inner, itol):
    c, eta, exact = case4
    x = torch.zeros_like(to_dev(eta))
    info = c.D.solve(x, to_dev(eta), method=P.MIXED_GCR, tol=1e-10, inner_prec=inner, max_iter=4000)
    xs = x.cpu().numpy()
    res = osolvers.rel_residual(c.f, xs, eta)
    err = rel(xs, exact)
    flush(f"[gpu] mixed {inner} 4^4: {info.iters} inner iterations, {info.outer} outer, residual {res:.2e}, "
          f"error vs oracle {err:.2e}, fell_back {info.fell_back}")
    assert res < 1.5e-10 and info.true_rel_res < 1e-10
    assert err < 20 * 1e-10


def test_gcr_ragged_mixed_extents():
    need_gpu()
    flush("[gpu] solve case 6x6x6x10")
    c = Case((6, 6, 6, 10), qhat=2, seed=77, bc_phase=(math.pi, 0.4, 0.0, -0.9))
    try:
        eta = c.spinor(3)
        exact, _ = osolvers.solve_eo(c.f, eta, 1e-13)
        x = torch.zeros_like(to_dev(eta))
        info = c.D.solve(x, to_dev(eta), method=P.GCR, tol=1e-12, restart=16)
        assert info.restarts >= 1
        assert rel(x.cpu().numpy(), exact) < 1e-9
        x2 = torch.zeros_like(x)
        info2 = c.D.solve(x2, to_dev(eta), method=P.MIXED_GCR, tol=1e-12, inner_prec="f32", restart=16)
        assert rel(x2.cpu().numpy(), exact) < 1e-9
        flush(f"[gpu] 6x6x6x10: GCR {info.iters} it, mixed f32 {info.iters} inner / {info2.outer} outer")
    finally:
        c.D.close()


def test_warm_start_returns_immediately(case4):
    c, eta, exact = case4
    x = to_dev(exact.copy())
    info = c.D.solve(x, to_dev(eta), method=P.GCR, tol=1e-10, x0_given=True)
    assert info.iters == 0 and info.true_rel_res < 1e-10


# ---------------------------------------------------------------- failure handling
def test_max_iter_gives_noconv(case4):
    c, eta, _ = case4
    x = torch.zeros_like(to_dev(eta))
    with pytest.raises(P.DiracError) as e:
        c.D.solve(x, to_dev(eta), method=P.GCR, tol=1e-10, max_iter=1)
    assert e.value.status == P._lib.ENOCONV
    info = c.D.solve(x, to_dev(eta), method=P.GCR, tol=1e-10, max_iter=1, raise_on_noconv=False)
    assert info.iters == 1 and info.true_rel_res < 1.0  # best iterate returned


def test_nan_rhs_is_reported(case4):
    c, eta, _ = case4
    bad = eta.copy()
    bad[7, 1, 2] = np.nan
    x = torch.zeros_like(to_dev(bad))
    for method in (P.GCR, P.CGLS, P.MIXED_GCR):
        with pytest.raises(P.DiracError) as e:
            c.D.solve(x, to_dev(bad), method=method, tol=1e-10)
        assert e.value.status == P._lib.ENONFINITE


def test_argument_errors(case4):
    c, eta, _ = case4
    b = to_dev(eta)
    with pytest.raises(P.DiracError) as e:
        c.D.apply(b, b)  # output aliases input
    assert e.value.status == P._lib.EINVAL
    with pytest.raises(P.DiracError) as e:
        c.D.apply(torch.empty_like(b), b, prec="f16", layout="lex")
    assert e.value.status == P._lib.EUNSUPPORTED
    with pytest.raises(ValueError):  # too small: refused before any device work
        c.D.apply(torch.empty(10, dtype=torch.complex128, device="cuda"), b)
    with pytest.raises(P.DiracError) as e:
        c.D.solve(torch.empty_like(b), b, tol=0.0)
    assert e.value.status == P._lib.EINVAL
    U = to_dev(c.U)
    with pytest.raises(P.DiracError) as e:
        P.Dirac(U, None, (4, 4, 4, 3), 0.12, 1.0, 1.0, -1)
    assert e.value.status == P._lib.EINVAL
    bad = c.U.copy()
    bad[3, 1] *= 1.01  # not unitary: the two-row compression would be wrong
    with pytest.raises(P.DiracError) as e:
        P.Dirac(to_dev(bad), None, c.dims, 0.12, 1.0, 1.0, -1)
    assert e.value.status == P._lib.EINVAL


def test_singular_clover_block_is_reported():
    need_gpu()
    c = Case((2, 2, 2, 4), seed=5)
    try:
        A = odirac.pack_clover(c.f.clover())
        # odd site Lambda = 1: make its upper block exactly singular (zero first row and column)
        lam = 1
        blk = odirac.unpack_clover(A[lam:lam + 1])[0]
        blk[0, :] = 0.0
        blk[:, 0] = 0.0
        A[lam] = odirac.pack_clover(blk[None])[0]
        c.D.load_clover(to_dev(A))
        with pytest.raises(P.DiracError) as e:
            c.D.clover_invert(2)
        assert e.value.status == P._lib.ESINGULAR and "Lambda = 1" in str(e.value)
        assert odirac.singular_blocks(odirac.unpack_clover(A[lam:lam + 1]))[0, 0]
        # even sites are fine
        c.D.clover_invert(1)
    finally:
        c.D.close()


def test_loaded_clover_is_used(case4):
    """Uploading the clover field the oracle computes (Sec. 4.1.3 path) gives the same operator."""
    need_gpu()
    c = Case((4, 2, 2, 4), seed=9)
    try:
        c.D.load_clover(to_dev(odirac.pack_clover(c.f.clover())))
        c.D.clover_invert(3)
        psi = c.spinor(4)
        out = torch.empty_like(to_dev(psi))
        c.D.apply(out, to_dev(psi))
        assert rel(out.cpu().numpy(), odirac.apply_D(c.f, psi)) < 1e-13
    finally:
        c.D.close()


# ---------------------------------------------------------------- production shape
def test_gcr_32c64_fp64_and_mixed():
    """32^3 x 64 plain-method solve (GCR(32), FP64, 1e-10) and its FP32-inner defect-correction
    form; the residual is checked by the oracle at 64 sampled sites."""
    need_gpu()
    flush("[gpu] 32^3x64 solve")
    c = Case((64, 32, 32, 32), seed=201)
    try:
        eta = c.spinor(201)
        b = to_dev(eta)
        rng = np.random.default_rng(1)
        pick = rng.choice(c.V, 64, replace=False)
        sols = {}
        for name, kw in (("f64", dict(method=P.GCR)), ("mixed_f32", dict(method=P.MIXED_GCR, inner_prec="f32"))):
            x = torch.zeros_like(b)
            info = c.D.solve(x, b, tol=1e-10, restart=32, max_iter=20000, **kw)
            xs = x.cpu().numpy()
            r = eta[pick] - odirac.apply_D(c.f, xs, pick)
            flush(f"[gpu] 32^3x64 {name}: {info.iters} it, {info.outer} outer, {info.seconds:.2f} s, "
                  f"residual {info.true_rel_res:.2e}, sampled {np.linalg.norm(r) / np.linalg.norm(eta[pick]):.2e}")
            assert info.true_rel_res < 1e-10
            assert np.linalg.norm(r) < 1e-8 * np.linalg.norm(eta[pick])
            sols[name] = xs
        assert rel(sols["mixed_f32"], sols["f64"]) < 1e-7
    finally:
        c.D.close()
