"""GPU parallel-transport convolution network against the FP64 oracle (forward, input and
weight gradients, Adam, one training step), and the flexible-GCR deployment with its fallback.

Parity: the library's network (BF16 weights, BF16 matrix-core operands, FP32 accumulation,
hidden activations stored in BF16) is compared with the plain FP64 oracle of the network with
the same BF16 weights (oracle/ptc.py with every rounding option off), element by element and in
norm, within the rounding envelope of tests/ptc_envelope.py: BF16 rounding (unit roundoff 2^-8)
at every point where a BF16 evaluation rounds, pushed through the exact network, so the bar
follows from the arithmetic before any GPU result is seen.  A diagnostic comparison with the
oracle's model of the kernel's own rounding points (bf16_inputs, last_contract_first,
bf16_storage) is kept beside it: it shows where the kernel rounds, not that the network is right.
"""
import math

import numpy as np
import pytest
import torch

import gen
import paper_2502_02490_amd as P
from gpu_util import Case, flush, need_gpu, rel, rel_norm, to_dev
from ptc_envelope import envelope
from oracle import dirac as odirac
from oracle import ptc as optc
from oracle import solvers as osolvers

pytestmark = pytest.mark.gpu

# the oracle's model of the library's own rounding points (diagnostics only)
MODEL = dict(bf16_inputs=True, last_contract_first=True, bf16_storage=True)


def bf16(a):
    """Round complex weights to BF16 (round to nearest even) per real component."""
    f = np.ascontiguousarray(np.asarray(a, dtype=np.complex64)).view(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = (((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16).astype(np.uint32)
    return r.view(np.float32).view(np.complex64).astype(np.complex128).reshape(np.shape(a))


def to_f32_native(D, psi):
    return D.to_native(to_dev(psi.astype(np.complex64)), "f32", "lex")


def from_f32_native(D, nat):
    return D.from_native(nat, "f32", "lex").cpu().numpy().astype(np.complex128)


@pytest.fixture(scope="module", params=[(4, 4, 4, 4), (6, 2, 6, 10)], ids=lambda d: "x".join(map(str, d)))
def case(request):
    need_gpu()
    flush(f"[gpu] ptc case {request.param}")
    c = Case(request.param, seed=41, bc_phase=(math.pi, 0.2, 0.0, -0.4))
    net = P.PTC((1, 8, 8, 1))
    yield c, net
    net.close()
    c.D.close()


def test_forward_matches_oracle(case):
    c, net = case
    ws = optc.init_weights((1, 8, 8, 1), seed=3, scale=1.0)
    net.set_weights(ws)
    wq = [bf16(w) for w in ws]
    r = c.spinor(7).astype(np.complex64).astype(np.complex128)
    y, _ = optc.forward(c.f, wq, r)
    env, _, _ = envelope(c.f, wq, r)
    out = c.D.native_empty("f32")
    net.forward(c.D, out, to_f32_native(c.D, r))
    got = from_f32_native(c.D, out)
    flush("[gpu] ptc forward vs plain oracle " + env.check(got, y, "forward"))
    # diagnostic: the oracle's model of the kernel's rounding points
    ym, _ = optc.forward(c.f, wq, r, **MODEL)
    flush(f"[gpu] ptc forward vs rounding model (diagnostic) {rel_norm(got, ym):.2e}")
    assert rel_norm(got, ym) < 3e-4


def test_backward_matches_oracle(case):
    c, net = case
    ws = optc.init_weights((1, 8, 8, 1), seed=4, scale=1.0)
    net.set_weights(ws)
    wq = [bf16(w) for w in ws]
    r = c.spinor(8).astype(np.complex64).astype(np.complex128)
    g = c.spinor(9).astype(np.complex64).astype(np.complex128)
    _, acts = optc.forward(c.f, wq, r)
    gx, gW = optc.backward(c.f, wq, acts, g)
    _, env_gin, env_gw = envelope(c.f, wq, r, g)
    net.zero_grad()
    gin = c.D.native_empty("f32")
    net.backward(c.D, gin, to_f32_native(c.D, r), to_f32_native(c.D, g))
    got_gin = from_f32_native(c.D, gin)
    flush("[gpu] ptc " + env_gin.check(got_gin, gx, "input gradient"))
    got = net.get_grad()
    for l in range(3):
        flush("[gpu] ptc " + env_gw[l].check(got[l], gW[l], f"weight gradient layer {l}"))
    # diagnostic: the rounding model
    _, am = optc.forward(c.f, wq, r, **MODEL)
    gxm, gWm = optc.backward(c.f, wq, am, g, bf16_inputs=True)
    assert rel_norm(got_gin, gxm) < 3e-4
    for l in range(3):
        assert rel_norm(got[l], gWm[l]) < 3e-4, l


@pytest.mark.parametrize("channels", [(1, 4, 1), (1, 2, 2, 1), (1, 8, 4, 8, 1)], ids=str)
def test_other_networks_forward(case, channels):
    """Other channel counts: the contract-first last layer formed after a 1 -> 4, a 2 -> 2 and a
    4 -> 8 layer (the network maps one channel to one channel, so a network of more than one
    layer always ends contract-first); forward and gradients within the rounding envelope."""
    c, _ = case
    net = P.PTC(channels)
    try:
        ws = optc.init_weights(channels, seed=12, scale=1.0)
        net.set_weights(ws)
        wq = [bf16(w) for w in ws]
        r = c.spinor(13).astype(np.complex64).astype(np.complex128)
        g = c.spinor(14).astype(np.complex64).astype(np.complex128)
        y, acts = optc.forward(c.f, wq, r)
        gx, gW = optc.backward(c.f, wq, acts, g)
        env, env_gin, env_gw = envelope(c.f, wq, r, g)
        out = c.D.native_empty("f32")
        net.forward(c.D, out, to_f32_native(c.D, r))
        got = from_f32_native(c.D, out)
        flush(f"[gpu] ptc {channels} " + env.check(got, y, "forward"))
        net.zero_grad()
        gin = c.D.native_empty("f32")
        net.backward(c.D, gin, to_f32_native(c.D, r), to_f32_native(c.D, g))
        flush(f"[gpu] ptc {channels} " + env_gin.check(from_f32_native(c.D, gin), gx, "input gradient"))
        gw_got = net.get_grad()
        for l in range(len(wq)):
            env_gw[l].check(gw_got[l], gW[l], f"weight gradient layer {l}")
        # diagnostic only: distance from the oracle's model of the kernel's rounding points
        ym, _ = optc.forward(c.f, wq, r, **MODEL)
        flush(f"[gpu] ptc {channels} forward vs rounding model (diagnostic, not asserted) {rel_norm(got, ym):.2e}")
    finally:
        net.close()


@pytest.mark.parametrize("channels", [(1, 8, 8, 1), (1, 4, 1), (1, 1)], ids=str)
def test_forward_eo_is_the_even_half(case, channels):
    """ptc_forward_eo(r_e) is bitwise the even half of ptc_forward((r_e, 0)) -- the skipped work
    only adds exact zeros or feeds the odd half -- and matches the oracle's model."""
    c, _ = case
    net = P.PTC(channels)
    try:
        ws = optc.init_weights(channels, seed=21, scale=1.0)
        net.set_weights(ws)
        wq = [bf16(w) for w in ws]
        r = c.spinor(22).astype(np.complex64).astype(np.complex128)
        r[c.odd] = 0.0
        full_in = to_f32_native(c.D, r)
        half = full_in.numel() // 2
        out_full = c.D.native_empty("f32")
        net.forward(c.D, out_full, full_in)
        in_e = full_in[:half].clone()
        out_e = torch.zeros_like(in_e)
        net.forward_eo(c.D, out_e, in_e)
        # compare at the lattice sites (the padding of the NATIVE layout is never written)
        got = from_f32_native(c.D, torch.cat([out_e, torch.zeros_like(out_e)]))[c.even]
        y_gpu = from_f32_native(c.D, out_full)
        assert np.array_equal(got, y_gpu[c.even])
        y, _ = optc.forward(c.f, wq, r)
        env, _, _ = envelope(c.f, wq, r)
        flush(f"[gpu] ptc {channels} even-odd " + env.check(y_gpu, y, "forward"))
    finally:
        net.close()


def test_gradients_over_many_tiles():
    """16^4: more 64-site tiles than weight-gradient work-groups, so each work-group sums several
    tiles into its slice; forward, input and weight gradients against the oracle."""
    need_gpu()
    flush("[gpu] ptc gradients 16^4")
    c = Case((16, 16, 16, 16), seed=71, bc_phase=(math.pi, 0.0, 0.3, 0.0))
    net = P.PTC((1, 2, 1))
    try:
        ws = optc.init_weights((1, 2, 1), seed=6, scale=1.0)
        net.set_weights(ws)
        wq = [bf16(w) for w in ws]
        r = c.spinor(8).astype(np.complex64).astype(np.complex128)
        g = c.spinor(9).astype(np.complex64).astype(np.complex128)
        y, acts = optc.forward(c.f, wq, r)
        gx, gW = optc.backward(c.f, wq, acts, g)
        env, env_gin, env_gw = envelope(c.f, wq, r, g)
        out = c.D.native_empty("f32")
        net.forward(c.D, out, to_f32_native(c.D, r))
        env.check(from_f32_native(c.D, out), y, "forward")
        net.zero_grad()
        gin = c.D.native_empty("f32")
        net.backward(c.D, gin, to_f32_native(c.D, r), to_f32_native(c.D, g))
        env_gin.check(from_f32_native(c.D, gin), gx, "input gradient")
        got = net.get_grad()
        for l in range(2):
            flush("[gpu] ptc 16^4 " + env_gw[l].check(got[l], gW[l], f"weight gradient layer {l}"))
    finally:
        net.close()
        c.D.close()


def test_dirac_as_single_layer():
    """With c_sw = c_sw^QED = 0 and 1/(2 kappa) = 4 (exact in BF16), one layer is D itself."""
    need_gpu()
    c = Case((4, 2, 4, 6), kappa=0.125, csw=0.0, csw_qed=0.0, seed=5)
    net = P.PTC((1, 1))
    try:
        net.set_weights([optc.dirac_as_layer(c.f)])
        psi = c.spinor(3).astype(np.complex64).astype(np.complex128)
        out = c.D.native_empty("f32")
        net.forward(c.D, out, to_f32_native(c.D, psi))
        got = from_f32_native(c.D, out)
        # the weights are exact in BF16; the transported inputs are rounded to BF16
        assert rel_norm(got, optc.layer(c.f, optc.dirac_as_layer(c.f), [psi], bf16_inputs=True)[0]) < 3e-4
        assert rel_norm(got, odirac.apply_D(c.f, psi)) < 2.0 ** -7
    finally:
        net.close()
        c.D.close()


def test_train_step_loss_and_update(case):
    c, net = case
    ws = optc.init_weights((1, 8, 8, 1), seed=5, scale=0.3)
    net.set_weights(ws)
    wq = [bf16(w) for w in ws]
    pairs = [(c.spinor(20 + k).astype(np.complex64).astype(np.complex128),
              c.spinor(30 + k).astype(np.complex64).astype(np.complex128)) for k in range(2)]
    L, g = optc.loss_and_grads(c.f, wq, pairs)
    rs = [to_f32_native(c.D, r) for r, _ in pairs]
    es = [to_f32_native(c.D, e) for _, e in pairs]
    lr = 1e-3
    loss = net.train_step(c.D, rs, es, lr)
    assert abs(loss - L) <= loss_bound(c, wq, pairs)
    new = net.get_weights()
    ref = optc.Adam(ws, lr=lr).step(ws, g)  # first Adam step: -lr sign(gradient) per real part
    for l in range(3):
        d_gpu, d_ref = new[l] - ws[l], ref[l] - ws[l]
        big = (np.abs(g[l].real) > 1e-3 * np.abs(g[l]).max())
        assert np.mean(np.sign(d_gpu.real[big]) == np.sign(d_ref.real[big])) > 0.99
        assert np.abs(d_gpu).max() < 1.5 * lr * math.sqrt(2)


def test_adam_five_steps_match_oracle(case):
    """Five Adam steps (moments, bias correction for t = 1..5) against the oracle's Adam on the
    same gradients, element by element: FP32 master weights and moments against FP64."""
    c, net = case
    ws = optc.init_weights((1, 8, 8, 1), seed=15, scale=0.3)
    net.set_weights(ws)
    w_ref = [np.asarray(w, dtype=np.complex64).astype(np.complex128) for w in ws]
    lr = 2e-3
    adam = optc.Adam(w_ref, lr=lr)
    for t in range(1, 6):
        r = c.spinor(40 + t).astype(np.complex64).astype(np.complex128)
        g = c.spinor(50 + t).astype(np.complex64).astype(np.complex128)
        net.zero_grad()
        net.backward(c.D, None, to_f32_native(c.D, r), to_f32_native(c.D, g))
        G = [x.astype(np.complex128) for x in net.get_grad()]
        net.adam_step(lr)
        w_ref = adam.step(w_ref, G)
        w_gpu = net.get_weights()
        m_gpu, v_gpu, step = net.get_adam_state()
        assert step == t
        m_ref = np.concatenate([m.ravel() for m in adam.m])
        v_ref = np.concatenate([v.ravel() for v in adam.v])
        # moments: a few FP32 roundings per step (relative 2^-24 each) against FP64
        assert np.abs(m_gpu - m_ref).max() <= 1e-5 * np.abs(m_ref).max(), t
        assert np.abs(v_gpu - v_ref).max() <= 1e-5 * np.abs(v_ref).max(), t
        # weights: the FP32 master weight (2^-24 relative per rounding) plus an FP32 update of at
        # most lr per step computed to a few 2^-24
        for l in range(3):
            d = np.abs(w_gpu[l] - w_ref[l])
            assert (d <= 4 * 2.0 ** -24 * np.abs(w_ref[l]) * t + 1e-5 * lr * t).all(), (t, l, d.max())
    flush("[gpu] ptc Adam: 5 steps match the oracle")


def test_nonfinite_pair_leaves_weights_unchanged(case):
    """A pair holding NaN makes ptc_train_step return DIRAC_ENONFINITE before any update: the
    weights and Adam state stay bit for bit what they were."""
    c, net = case
    ws = optc.init_weights((1, 8, 8, 1), seed=16, scale=0.3)
    net.set_weights(ws)
    r0 = to_f32_native(c.D, c.spinor(60))
    e0 = to_f32_native(c.D, c.spinor(61))
    net.train_step(c.D, [r0], [e0], 1e-3)
    w_before = net.get_weights()
    m_before, v_before, s_before = net.get_adam_state()
    bad = c.spinor(62)
    bad[3, 1, 2] = np.nan
    with pytest.raises(P.DiracError) as ei:
        net.train_step(c.D, [r0, to_f32_native(c.D, bad)], [e0, e0], 1e-3)
    assert ei.value.status == P._lib.ENONFINITE
    for a, b in zip(net.get_weights(), w_before):
        assert np.array_equal(a, b)
    m, v, s_after = net.get_adam_state()
    assert s_after == s_before and np.array_equal(m, m_before) and np.array_equal(v, v_before)


def loss_bound(c, wq, pairs):
    """Bound on |L_gpu - L| from the forward envelope: per pair, with y = N(r) and an output error
    dy, |y + dy - e|^2 - |y - e|^2 <= 2 |y - e| |dy| + |dy|^2, |dy| <= env |y|; averaged."""
    tot = 0.0
    for k, (r, e) in enumerate(pairs):
        y, _ = optc.forward(c.f, wq, r)
        env, _, _ = envelope(c.f, wq, r, seed=k)
        dy = env.norm * np.linalg.norm(y)
        tot += (2 * np.linalg.norm(y - e) * dy + dy * dy) / np.vdot(e, e).real
    return tot / len(pairs)


def test_loss_entry_point_matches_oracle(case):
    """ptc_loss (no update) equals the loss of the plain oracle within the forward envelope, and
    leaves the weights untouched."""
    c, net = case
    ws = optc.init_weights((1, 8, 8, 1), seed=17, scale=0.3)
    net.set_weights(ws)
    wq = [bf16(w) for w in ws]
    pairs = [(c.spinor(70 + k).astype(np.complex64).astype(np.complex128),
              c.spinor(80 + k).astype(np.complex64).astype(np.complex128)) for k in range(2)]
    L, _ = optc.loss_and_grads(c.f, wq, pairs)
    got = net.loss(c.D, [to_f32_native(c.D, r) for r, _ in pairs], [to_f32_native(c.D, e) for _, e in pairs])
    bound = loss_bound(c, wq, pairs)
    flush(f"[gpu] ptc_loss {got:.6f} oracle {L:.6f} (bound {bound:.2e})")
    assert abs(got - L) <= bound
    assert all(np.array_equal(a, np.asarray(b, dtype=np.complex64)) for a, b in zip(net.get_weights(), ws))


def test_training_reduces_loss():
    need_gpu()
    flush("[gpu] ptc training 4^4")
    c = Case((4, 4, 4, 4), seed=61)
    net = P.PTC((1, 8, 8, 1))
    try:
        # pairs (r, e = D^-1 r) from the GPU solver: snapshots x_k of GCR, e = x* - x_k, r = b - D x_k
        rs, es = [], []
        for k in range(4):
            b = to_dev(c.spinor(100 + k))
            xs = torch.zeros_like(b)
            c.D.solve(xs, b, method=P.GCR, tol=1e-12)
            for it in (2, 6):
                xk = torch.zeros_like(b)
                c.D.solve(xk, b, method=P.GCR, tol=1e-12, max_iter=it, raise_on_noconv=False)
                rk = torch.empty_like(b)
                c.D.apply(rk, xk)
                rk = b - rk
                rs.append(c.D.to_native(rk.to(torch.complex64), "f32", "lex"))
                es.append(c.D.to_native((xs - xk).to(torch.complex64), "f32", "lex"))
        net.set_weights(optc.init_weights((1, 8, 8, 1), seed=7, scale=0.3))
        first = net.train_step(c.D, rs, es, 1e-2)
        for _ in range(40):
            last = net.train_step(c.D, rs, es, 1e-2)
        flush(f"[gpu] ptc loss {first:.4f} -> {last:.4f}")
        assert last < 0.7 * first
    finally:
        net.close()
        c.D.close()


@pytest.mark.parametrize("method", ["full", "eo"])
def test_fgcr_ptc_solves_and_falls_back(case, method):
    c, net = case
    m = P.FGCR_PTC if method == "full" else P.FGCR_PTC_EO
    eta = c.spinor(50)
    exact, _ = osolvers.solve_eo(c.f, eta, 1e-13)
    b = to_dev(eta)
    # zero weights: N(r) = 0 gives no direction; the solver must fall back and still converge
    net.set_weights([np.zeros(s, dtype=np.complex64) for s in net.shapes()])
    x = torch.zeros_like(b)
    info = c.D.solve(x, b, method=m, ptc=net, tol=1e-12)
    assert info.fell_back == 1 and rel(x.cpu().numpy(), exact) < 1e-9
    # the identity network (W_0 = 1 on one channel) is a fine preconditioner direction
    ws = [np.zeros(s, dtype=np.complex64) for s in net.shapes()]
    for w in ws:
        w[0, 0, 0] = np.eye(4)
    net.set_weights(ws)
    x = torch.zeros_like(b)
    info = c.D.solve(x, b, method=m, ptc=net, tol=1e-12)
    assert rel(x.cpu().numpy(), exact) < 1e-9 and info.true_rel_res < 1e-12
    if method == "eo":
        # the identity network returns r rounded to BF16: flexible GCR on D-hat then needs about
        # as many iterations as plain GCR
        x2 = torch.zeros_like(b)
        info2 = c.D.solve(x2, b, method=P.GCR, tol=1e-12)
        assert abs(info.iters - info2.iters) <= max(2, info2.iters // 10) and info.fell_back == 0


def test_checkpoint_resume_is_exact(tmp_path):
    """Weights and Adam state written mid-training and read back give bitwise the same weights
    after further steps as the uninterrupted run; NaN weights make FGCR fall back."""
    need_gpu()
    from paper_2502_02490_amd import ptc_train as T

    c = Case((4, 2, 2, 4), seed=62)
    net = P.PTC((1, 4, 1))
    net2 = None
    try:
        rs, es = T.generate_pairs(c.D, 6, seed=3, snapshots=(0, 2, 4))
        ops = [(c.D, rs, es)]
        net.set_weights(T.init_weights((1, 4, 1), seed=1))
        T.train(ops, net, epochs=2, batch=3, lr=1e-2, seed=5)
        ck = str(tmp_path / "ptc.npz")
        T.save_checkpoint(ck, net, epochs_done=2, seed=5, meta={"note": "test"})
        T.train(ops, net, epochs=4, batch=3, lr=1e-2, seed=5, start_epoch=2)
        net2, head = T.load_checkpoint(ck)
        assert head["epochs_done"] == 2 and head["adam_step"] == 4 and head["meta"]["note"] == "test"
        T.train(ops, net2, epochs=4, batch=3, lr=1e-2, seed=5, start_epoch=head["epochs_done"])
        for a, b in zip(net.get_weights(), net2.get_weights()):
            assert np.array_equal(a, b)
        m1, v1, s1 = net.get_adam_state()
        m2, v2, s2 = net2.get_adam_state()
        assert s1 == s2 == 8 and np.array_equal(m1, m2) and np.array_equal(v1, v2)
        # non-finite weights: the preconditioner output is not finite, the solver falls back
        bad = net2.get_weights()
        bad[0][:] = np.nan
        net2.set_weights(bad)
        b = to_dev(c.spinor(1))
        x = torch.zeros_like(b)
        info = c.D.solve(x, b, method=P.FGCR_PTC, ptc=net2, tol=1e-12)
        assert info.fell_back == 1 and info.true_rel_res < 1e-12
        with pytest.raises(P.DiracError):
            m, v, _ = net2.get_adam_state()
            v[0] = -1.0
            net2.set_adam_state(m, v, 3)
    finally:
        net.close()
        if net2 is not None:
            net2.close()
        c.D.close()
