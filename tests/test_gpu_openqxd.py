"""openQxD field storage on the GPU (Sec. 4.1): spinors and clover blocks in eq. (ipt) order with a
cache block, and contexts created from the odd-point 8-link gauge storage, against the oracle's
permutations (oracle/openqxd.py).  Permutations are exact, so every comparison is bitwise."""
import math

import numpy as np
import pytest
import torch

import paper_2502_02490_amd as P
from gpu_util import Case, flush, need_gpu, to_dev
from oracle import openqxd as oq

pytestmark = pytest.mark.gpu

CASES = [((4, 2, 6, 8), (2, 2, 3, 4)), ((6, 4, 2, 4), (3, 2, 1, 2)), ((4, 4, 4, 4), (4, 4, 4, 4))]


@pytest.fixture(scope="module", params=CASES, ids=lambda c: "L" + "x".join(map(str, c[0])) + "_B" + "x".join(map(str, c[1])))
def case(request):
    need_gpu()
    L, B = request.param
    flush(f"[gpu] openqxd case L {L} B {B}")
    c = Case(L, seed=91, bc_phase=(math.pi, 0.3, 0.0, -0.2))
    c.D.set_cache_block(B)
    yield c, L, B
    c.D.close()


def test_spinor_order(case):
    c, L, B = case
    psi = c.spinor(3)
    nat = c.D.to_native(to_dev(psi), "f64", "lex")
    q = c.D.from_native(nat, "f64", "openqxd").cpu().numpy()
    assert np.array_equal(q, oq.sites_to_openqxd(psi, L, B))
    # back, and the two halves as half vectors (even sites first in eq. (ipt))
    nat2 = c.D.to_native(to_dev(q), "f64", "openqxd")
    assert torch.equal(c.D.from_native(nat2, "f64", "lex"), to_dev(psi))
    vh = c.V // 2
    for sites, sl in ((1, slice(0, vh)), (2, slice(vh, None))):
        h = c.D.to_native(to_dev(np.ascontiguousarray(q[sl])), "f64", "openqxd", sites=sites)
        back = c.D.from_native(h, "f64", "openqxd", sites=sites).cpu().numpy()
        assert np.array_equal(back, q[sl])
    # FP32 user buffers take the same order
    q32 = c.D.from_native(c.D.to_native(to_dev(psi.astype(np.complex64)), "f32", "lex"), "f32", "openqxd")
    assert np.array_equal(q32.cpu().numpy(), oq.sites_to_openqxd(psi.astype(np.complex64), L, B))


def test_clover_order(case):
    c, L, B = case
    lex = c.D.clover(layout="lex").cpu().numpy()
    q = c.D.clover(layout="openqxd").cpu().numpy()
    assert np.array_equal(q, oq.sites_to_openqxd(lex, L, B))
    # loading it back in that order leaves the operator unchanged
    psi = to_dev(c.spinor(4))
    y0 = torch.empty_like(psi)
    c.D.apply(y0, psi)
    c.D.load_clover(to_dev(q), layout="openqxd")
    c.D.clover_invert(3)
    y1 = torch.empty_like(psi)
    c.D.apply(y1, psi)
    assert torch.equal(y0, y1)


def test_context_from_odd_point_storage(case):
    c, L, B = case
    u, a = oq.links_to_openqxd(c.U, c.theta, L, B)
    p = c.p
    D2 = P.Dirac(to_dev(u), to_dev(a), L, p.kappa, p.csw, p.csw_qed, p.qhat, p.bc_phase, openqxd_block=B)
    try:
        psi = to_dev(c.spinor(5))
        y0, y1 = torch.empty_like(psi), torch.empty_like(psi)
        c.D.apply(y0, psi)
        D2.apply(y1, psi)
        assert torch.equal(y0, y1)
        assert torch.equal(c.D.clover(layout="lex"), D2.clover(layout="lex"))
        # the new context took B as its cache block; a solve in openQxD order is the LEX solve permuted
        b = c.spinor(6)
        x_lex = torch.zeros_like(psi)
        c.D.solve(x_lex, to_dev(b), method=P.GCR, tol=1e-12)
        bq = to_dev(oq.sites_to_openqxd(b, L, B))
        x_q = torch.zeros_like(bq)
        D2.solve(x_q, bq, method=P.GCR, tol=1e-12, layout="openqxd")
        assert np.array_equal(x_q.cpu().numpy(), oq.sites_to_openqxd(x_lex.cpu().numpy(), L, B))
    finally:
        D2.close()


def test_bad_cache_blocks_are_rejected():
    need_gpu()
    c = Case((4, 4, 4, 4), seed=3)
    try:
        for bad in ((3, 4, 4, 4), (4, 4, 4, 1), (0, 4, 4, 4)):
            with pytest.raises(P.DiracError) as e:
                c.D.set_cache_block(bad)
            assert e.value.status == P._lib.EINVAL
        u, a = oq.links_to_openqxd(c.U, c.theta, (4, 4, 4, 4), (4, 4, 4, 4))
        with pytest.raises(P.DiracError):
            P.Dirac(to_dev(u), to_dev(a), (4, 4, 4, 4), 0.12, 1.0, 1.0, -1, openqxd_block=(4, 4, 4, 3))
    finally:
        c.D.close()
