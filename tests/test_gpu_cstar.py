"""C* boundary conditions on the GPU (Sec. 4.2; the lattice doubled in direction 1, crossing the
boundary of a C* direction mu >= 2 moves x1 by half the doubled extent) against the oracle:
operator, Schur operator, clover field, every hop launch shape, solves, the network's transports
and the openQxD gauge storage."""
import math

import numpy as np
import pytest
import torch

import gen
import paper_2502_02490_amd as P
from gpu_util import N_HOP_SHAPES, Case, flush, need_gpu, rel, rel_norm, to_dev
from ptc_envelope import envelope
from oracle import dirac as odirac
from oracle import openqxd as oq
from oracle import ptc as optc

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", params=[((4, 8, 4, 6), 2), ((2, 8, 6, 4), 3), ((6, 4, 2, 2), 3)],
                ids=lambda c: "L" + "x".join(map(str, c[0])) + f"_cstar{c[1]}")
def case(request):
    need_gpu()
    L, cs = request.param
    flush(f"[gpu] cstar case {L} cstar {cs}")
    c = Case(L, seed=81, qhat=2, bc_phase=(math.pi, 0.0, 0.4, -0.2), cstar=cs)
    yield c
    c.D.close()


@pytest.mark.parametrize("dagger", [False, True])
def test_full_and_schur_apply(case, dagger):
    psi = case.spinor(1)
    out = torch.empty_like(to_dev(psi))
    case.D.apply(out, to_dev(psi), "f64", "lex", dagger=dagger)
    exp = odirac.apply_Ddag(case.f, psi) if dagger else odirac.apply_D(case.f, psi)
    assert rel(out.cpu().numpy(), exp) <= 1e-13
    psi_e = psi[case.even]
    oe = torch.empty_like(to_dev(psi_e))
    case.D.apply_eo(oe, to_dev(psi_e), "f64", "eo", dagger=dagger)
    exp = odirac.apply_schur_dag(case.f, psi_e) if dagger else odirac.apply_schur(case.f, psi_e)
    assert rel(oe.cpu().numpy(), exp) <= 1e-13


def test_clover_field(case):
    got = case.D.clover(layout="lex").cpu().numpy()
    exp = odirac.pack_clover(case.f.clover())
    assert np.abs(got - exp).max() <= 1e-13 * np.abs(exp).max()


def test_solve(case):
    b = case.spinor(2)
    x = torch.zeros_like(to_dev(b))
    info = case.D.solve(x, to_dev(b), method=P.GCR, tol=1e-12)
    r = b - odirac.apply_D(case.f, x.cpu().numpy())
    assert np.linalg.norm(r) / np.linalg.norm(b) < 2e-12, info.true_rel_res


def test_network_transports(case):
    net = P.PTC((1, 4, 1))
    try:
        ws = optc.init_weights((1, 4, 1), seed=9, scale=1.0)
        net.set_weights(ws)
        r = case.spinor(3).astype(np.complex64).astype(np.complex128)
        out = case.D.native_empty("f32")
        net.forward(case.D, out, case.D.to_native(to_dev(r.astype(np.complex64)), "f32", "lex"))
        got = case.D.from_native(out, "f32", "lex").cpu().numpy().astype(np.complex128)
        wq = [optc.round_bf16(np.asarray(w, dtype=np.complex64).astype(np.complex128)) for w in ws]
        y, _ = optc.forward(case.f, wq, r)  # the plain network with the BF16 weights
        env, _, _ = envelope(case.f, wq, r)
        env.check(got, y, "C* network forward")
        # the same network with the plain neighbours is far off (the transports take the shift)
        f0 = odirac.Fields(case.U, case.theta, odirac.Params(case.dims, case.p.kappa, case.p.csw, case.p.csw_qed,
                                                           case.p.qhat, case.p.bc_phase, 0))
        y0, _ = optc.forward(f0, ws, r)
        assert rel_norm(y0, y) > 0.05
    finally:
        net.close()


def test_openqxd_storage_with_cstar(case):
    B = case.dims
    u, a = oq.links_to_openqxd(case.U, case.theta, case.dims, B, case.p.cstar)
    p = case.p
    D2 = P.Dirac(to_dev(u), to_dev(a), case.dims, p.kappa, p.csw, p.csw_qed, p.qhat, p.bc_phase,
                 openqxd_block=B, cstar=p.cstar)
    try:
        psi = to_dev(case.spinor(4))
        y0, y1 = torch.empty_like(psi), torch.empty_like(psi)
        case.D.apply(y0, psi)
        D2.apply(y1, psi)
        assert torch.equal(y0, y1)
    finally:
        D2.close()


def test_hop_launch_shapes_with_cstar(monkeypatch):
    """Every hop launch shape applies the shifted boundaries (bitwise equal outputs)."""
    need_gpu()
    c = Case((8, 8, 16, 32), seed=57, qhat=-1, cstar=3)  # the slab and x1-split sweeps fit
    try:
        psi_e = c.spinor(3)[c.even]
        nat = c.D.to_native(to_dev(psi_e), "f64", "eo", sites=1)
        ref = None
        for shape in range(N_HOP_SHAPES):
            monkeypatch.setenv("DIRAC_HOP_SHAPE", str(shape))
            out = c.D.native_empty("f64", 1)
            c.D.apply_eo(out, nat, "f64", "native")
            if ref is None:
                ref = out.clone()
            else:
                assert torch.equal(out, ref), shape
        monkeypatch.delenv("DIRAC_HOP_SHAPE")
        o = torch.empty_like(to_dev(psi_e))
        c.D.apply_eo(o, to_dev(psi_e), "f64", "eo")
        assert rel(o.cpu().numpy(), odirac.apply_schur(c.f, psi_e)) <= 1e-13
    finally:
        c.D.close()


def test_bad_cstar_rejected():
    need_gpu()
    for dims, cs in (((4, 6, 4, 4), 2), ((4, 4, 4, 4), 4), ((4, 4, 4, 4), -1)):  # odd mirror shift, bad counts
        U, th = to_dev(gen.su3_field(dims, 0.5, 3)), to_dev(gen.u1_field(dims, 0.3, 3))
        with pytest.raises(P.DiracError) as e:
            P.Dirac(U, th, dims, 0.12, 1.0, 1.0, -1, cstar=cs)
        assert e.value.status == P._lib.EINVAL
