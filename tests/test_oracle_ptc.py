"""Pins of the oracle's parallel-transport convolution network: it reduces to D, its transports
are adjoint pairs, its gradients match central finite differences, and it is gauge equivariant."""
import numpy as np

import gen
from oracle import dirac, geometry as geo, ptc


def fields(L=(2, 2, 2, 4), csw=0.0, cq=0.0, seed=3):
    return dirac.Fields(gen.su3_field(L, 0.5, seed), gen.u1_field(L, 0.3, seed),
                        dirac.Params(L, 0.124, csw, cq, -1, (np.pi, 0.5, 0.0, -0.3)))


def test_single_layer_equals_dirac_without_clover():
    f = fields()
    psi = gen.gaussian_spinor(f.p.dims, 1)
    y = ptc.layer(f, ptc.dirac_as_layer(f), [psi])[0]
    assert np.abs(y - dirac.apply_D(f, psi)).max() < 1e-13


def test_transport_adjoint_pairs():
    f = fields()
    x, y = gen.gaussian_spinor(f.p.dims, 2), gen.gaussian_spinor(f.p.dims, 3)
    for p in range(ptc.NPATH):
        lhs = np.vdot(y, ptc.transport(f, x, p))
        rhs = np.vdot(ptc.transport(f, y, ptc.ADJ[p]), x)
        assert abs(lhs - rhs) < 1e-12 * abs(lhs)


def _loss(f, ws, r, e):
    y, _ = ptc.forward(f, ws, r)
    d = y - e
    return np.vdot(d, d).real / np.vdot(e, e).real


def test_gradients_match_finite_differences():
    f = fields()
    r, e = gen.gaussian_spinor(f.p.dims, 4), gen.gaussian_spinor(f.p.dims, 5)
    ws = ptc.init_weights((1, 2, 1), seed=1, scale=0.5)
    L, g = ptc.loss_and_grads(f, ws, [(r, e)])
    assert abs(L - _loss(f, ws, r, e)) < 1e-12
    rng = np.random.default_rng(0)
    h = 1e-6
    for l in range(len(ws)):
        for _ in range(6):
            idx = tuple(rng.integers(0, n) for n in ws[l].shape)
            for part, unit in ((0, 1.0), (1, 1j)):
                wp = [w.copy() for w in ws]
                wm = [w.copy() for w in ws]
                wp[l][idx] += h * unit
                wm[l][idx] -= h * unit
                fd = (_loss(f, wp, r, e) - _loss(f, wm, r, e)) / (2 * h)
                an = 2 * (g[l][idx].real if part == 0 else g[l][idx].imag)
                assert abs(fd - an) < 1e-7 * max(1.0, abs(an)), (l, idx, part, fd, an)
    # input gradient
    y, acts = ptc.forward(f, ws, r)
    ne2 = np.vdot(e, e).real
    gr, _ = ptc.backward(f, ws, acts, (y - e) / ne2)
    for _ in range(4):
        idx = (rng.integers(0, f.V), rng.integers(0, 4), rng.integers(0, 3))
        for unit in (1.0, 1j):
            rp, rm = r.copy(), r.copy()
            rp[idx] += h * unit
            rm[idx] -= h * unit
            fd = (_loss(f, ws, rp, e) - _loss(f, ws, rm, e)) / (2 * h)
            an = 2 * (gr[idx].real if unit == 1.0 else gr[idx].imag)
            assert abs(fd - an) < 1e-7 * max(1.0, abs(an))


def test_gauge_equivariance():
    f = fields(csw=1.0, cq=1.0)
    L = f.p.dims
    W, lam = gen.gauge_transform(L, 11)
    sites = np.arange(f.V)
    U2, th2 = np.empty_like(f.U), np.empty_like(f.theta)
    for mu in range(4):
        fw = geo.shift(sites, L, mu, 1)
        U2[:, mu] = W @ f.U[:, mu] @ np.conj(np.swapaxes(W[fw], 1, 2))
        th2[:, mu] = f.theta[:, mu] + lam - lam[fw]
    f2 = dirac.Fields(U2, th2, f.p)
    tr = lambda v: np.exp(1j * f.p.qhat * lam)[:, None, None] * np.einsum("nab,nsb->nsa", W, v)  # noqa: E731
    ws = ptc.init_weights((1, 2, 1), seed=2, scale=0.5)
    r = gen.gaussian_spinor(L, 6)
    y1, _ = ptc.forward(f2, ws, tr(r))
    y0, _ = ptc.forward(f, ws, r)
    assert np.abs(y1 - tr(y0)).max() < 1e-12 * np.abs(y0).max()


def test_adam_first_step_moves_by_lr_against_gradient_sign():
    ws = [np.array([[1.0 + 2.0j, -0.5j]])]
    g = [np.array([[0.3 - 0.1j, 2.0 + 0.0j]])]
    new = ptc.Adam(ws, lr=0.01).step(ws, g)[0]
    # first Adam step: m/sqrt(v) = sign(g) per real component (up to eps)
    expect = ws[0] - 0.01 * (np.sign(g[0].real) + 1j * np.sign(g[0].imag))
    assert np.abs(new - expect).max() < 1e-8


def test_round_bf16_known_values():
    """Round-to-nearest-even on 8 significant bits, from the FP32 value."""
    e = 2.0 ** -8
    vals = np.array([1.0, 1 + e, 1 + 1.5 * e, 1 + 0.5 * e, 1 + 2 * e + e, -1.5, 3.0, 1 + e + 2.0 ** -30,
                     2.0 ** -130, np.inf, -np.inf, 65504.0, 1 + 2 * e])
    want = np.array([1.0, 1.0, 1 + 2 * e, 1.0, 1 + 4 * e, -1.5, 3.0, 1.0, 2.0 ** -130, np.inf, -np.inf, 65536.0,
                     1 + 2 * e])
    got = ptc.round_bf16(vals)
    assert np.array_equal(got, want)
    assert np.isnan(ptc.round_bf16(np.array([np.nan]))[0])
    z = ptc.round_bf16(np.array([(1 + 1.5 * e) - 1j * (1 + 0.5 * e)]))
    assert z[0] == (1 + 2 * e) - 1j


def _exact_fields(L=(2, 2, 2, 4)):
    """Unit links, zero angles, phases 0 / pi: every transport of an integer field is a
    small-integer field (up to the 1e-16 imaginary part of exp(i pi)), so rounding to BF16
    changes nothing beyond that."""
    V = int(np.prod(L))
    U = np.broadcast_to(np.eye(3, dtype=np.complex128), (V, 4, 3, 3)).copy()
    th = np.zeros((V, 4))
    return dirac.Fields(U, th, dirac.Params(L, 0.124, 0.0, 0.0, -1, (np.pi, 0.0, np.pi, 0.0)))


def test_bf16_inputs_exact_when_transports_are_representable():
    f = _exact_fields()
    rng = np.random.default_rng(7)
    r = (rng.integers(-20, 20, size=(f.V, 4, 3)) + 1j * rng.integers(-20, 20, size=(f.V, 4, 3))).astype(np.complex128)
    g = (rng.integers(-20, 20, size=(f.V, 4, 3)) + 1j * rng.integers(-20, 20, size=(f.V, 4, 3))).astype(np.complex128)
    ws = ptc.init_weights((1, 3, 2, 1), seed=2, scale=1.0)
    y0, a0 = ptc.forward(f, ws, r)
    # the first layer sees integer transports: identical; later layers see non-integer inputs
    l1 = ptc.layer(f, ws[0], [r], bf16_inputs=True)
    assert all(np.abs(u - v).max() <= 1e-13 * np.abs(v).max() for u, v in zip(l1, a0[1]))
    # backward of a single layer with an integer gradient: the rounded form equals the exact one
    W = ws[2]  # 2 -> 1: input gradient of a 1-channel output gradient
    acts = [[r, 2 * r], ptc.layer(f, W, [r, 2 * r])]
    gx_exact, gw_exact = ptc.backward(f, [W], acts, g)
    gx_round, gw_round = ptc.backward(f, [W], acts, g, bf16_inputs=True)
    assert np.abs(gx_round - gx_exact).max() <= 1e-12 * np.abs(gx_exact).max()
    assert np.array_equal(gw_round[0], gw_exact[0])
    # a plausible slip in the rounded branch (dagger dropped) is caught
    Wbad = [np.swapaxes(W, -1, -2)]
    gx_bad, _ = ptc.backward(f, Wbad, acts, g, bf16_inputs=True)
    assert np.abs(gx_bad - gx_exact).max() > 1e-3 * np.abs(gx_exact).max()


def test_bf16_inputs_error_is_bounded_by_the_unit_roundoff():
    """On a random field the rounded network differs from the exact one by about 2^-9 per
    element of every transported input (and no more than 2^-8 relative in norm)."""
    f = fields()
    r = gen.gaussian_spinor(f.p.dims, 8)
    g = gen.gaussian_spinor(f.p.dims, 9)
    ws = ptc.init_weights((1, 2, 1), seed=3, scale=1.0)
    y, acts = ptc.forward(f, ws, r)
    yr, actsr = ptc.forward(f, ws, r, bf16_inputs=True)
    d = np.linalg.norm(yr - y) / np.linalg.norm(y)
    assert 1e-5 < d < 2.0 ** -7
    gx, _ = ptc.backward(f, ws, acts, g)
    gxr, _ = ptc.backward(f, ws, acts, g, bf16_inputs=True)
    d = np.linalg.norm(gxr - gx) / np.linalg.norm(gx)
    assert 1e-5 < d < 2.0 ** -7


def test_contract_first_equals_transport_first():
    """Spin weights commute with the transports: summing the layer as sum_p T_p (sum_c' W x_c')
    gives the transport-first layer up to FP64 rounding, for several channel counts and with the
    boundary phases and U(1) angles on."""
    f = fields(csw=1.0, cq=1.0)
    for n_in, n_out in ((8, 1), (2, 3), (1, 2)):
        W = ptc.init_weights((n_in, n_out), seed=10 + n_in, scale=1.0)[0]
        xs = [gen.gaussian_spinor(f.p.dims, 20 + k) for k in range(n_in)]
        a = ptc.layer(f, W, xs)
        b = ptc.layer_contract_first(f, W, xs)
        for u, v in zip(a, b):
            assert np.abs(u - v).max() < 1e-13 * np.abs(u).max()
        # a slip (the weights of path p applied after the transport of another path) is caught
        Wp = W[[0, 2, 1, 3, 4, 5, 6, 7, 8]]
        bad = ptc.layer_contract_first(f, Wp, xs)
        assert np.abs(bad[0] - a[0]).max() > 1e-2 * np.abs(a[0]).max()


def test_contract_first_rounds_the_untransported_inputs():
    """On fields whose transports are signed permutations (unit links, phases 0 / pi), rounding
    commutes with transport, so the contract-first layer with BF16 inputs equals the
    transport-first one with BF16 inputs; rounding z instead of x would not.  On a random field
    the rounded forms stay within the BF16 unit roundoff of the exact one."""
    f = _exact_fields()
    rng = np.random.default_rng(9)
    xs = [rng.standard_normal((f.V, 4, 3)) + 1j * rng.standard_normal((f.V, 4, 3)) for _ in range(2)]
    W = ptc.init_weights((2, 1), seed=4, scale=1.0)[0]
    a = ptc.layer(f, W, xs, bf16_inputs=True)[0]
    b = ptc.layer_contract_first(f, W, xs, bf16_inputs=True)[0]
    assert np.abs(a - b).max() < 1e-12 * np.abs(a).max()
    exact = ptc.layer(f, W, xs)[0]
    assert np.abs(b - exact).max() > 1e-4 * np.abs(exact).max()  # the rounding happened
    z_rounded = sum(ptc.transport(f, ptc.round_bf16(sum(np.einsum("st,ntc->nsc", W[p, 0, cp], xs[cp])
                                                        for cp in range(2))), p) for p in range(ptc.NPATH))
    assert np.abs(z_rounded - a).max() > 1e-4 * np.abs(a).max()
    f2 = fields()
    xs2 = [gen.gaussian_spinor(f2.p.dims, 30 + k) for k in range(2)]
    e = ptc.layer(f2, W, xs2)[0]
    r = ptc.layer_contract_first(f2, W, xs2, bf16_inputs=True)[0]
    d = np.linalg.norm(r - e) / np.linalg.norm(e)
    assert 1e-5 < d < 2.0 ** -7
    ws = ptc.init_weights((1, 2, 1), seed=3, scale=1.0)
    y, _ = ptc.forward(f2, ws, xs2[0])
    yc, _ = ptc.forward(f2, ws, xs2[0], last_contract_first=True)
    assert np.abs(y - yc).max() < 1e-13 * np.abs(y).max()


def test_bf16_storage_rounds_the_hidden_activations_only():
    """With BF16 storage every hidden activation is a BF16 value (rounding it again changes
    nothing) while input and output are untouched; on signed-permutation transports with an
    integer input, the transported values of BF16 activations are BF16 values themselves, so the
    extra input rounding changes nothing; on a random field the stored form stays within the
    BF16 unit roundoff of the exact network."""
    f = _exact_fields()
    rng = np.random.default_rng(11)
    r = (rng.integers(-8, 8, size=(f.V, 4, 3)) + 1j * rng.integers(-8, 8, size=(f.V, 4, 3))).astype(np.complex128)
    ws = ptc.init_weights((1, 3, 2, 1), seed=5, scale=1.0)
    y_s, acts = ptc.forward(f, ws, r, bf16_storage=True)
    for a in acts[1:-1]:
        for v in a:
            assert np.array_equal(ptc.round_bf16(v), v)
    assert acts[0][0] is r
    y_plain, acts_plain = ptc.forward(f, ws, r)
    assert not np.array_equal(acts_plain[1][0], acts[1][0])  # the hidden layer was rounded
    assert np.abs(y_s - y_plain).max() > 1e-4 * np.abs(y_plain).max()
    y_both, _ = ptc.forward(f, ws, r, bf16_inputs=True, last_contract_first=True, bf16_storage=True)
    y_cf, _ = ptc.forward(f, ws, r, last_contract_first=True, bf16_storage=True)
    assert np.abs(y_both - y_cf).max() < 1e-12 * np.abs(y_cf).max()
    f2 = fields()
    r2 = gen.gaussian_spinor(f2.p.dims, 12)
    ws2 = ptc.init_weights((1, 2, 2, 1), seed=6, scale=1.0)
    e, _ = ptc.forward(f2, ws2, r2)
    m, _ = ptc.forward(f2, ws2, r2, bf16_inputs=True, last_contract_first=True, bf16_storage=True)
    d = np.linalg.norm(m - e) / np.linalg.norm(e)
    assert 1e-5 < d < 2.0 ** -6


def test_adam_bias_correction_closed_forms():
    """Adam beyond its first step.  A constant gradient g keeps m_hat = g and v_hat = g^2 exactly
    (the bias corrections cancel the zero start), so every step moves each real part by
    lr g / (|g| + eps).  A single gradient g at step 1 followed by zeros gives
    m_t = (1 - b1) b1^(t-1) g, v_t = (1 - b2) b2^(t-1) g^2, hence the step at t is
    lr (1 - b1) b1^(t-1) / (1 - b1^t) g / (sqrt((1 - b2) b2^(t-1) / (1 - b2^t)) |g| + eps)."""
    lr, b1, b2, eps = 0.01, 0.9, 0.999, 1e-8
    w0 = [np.array([[1.0 + 2.0j, -0.5j, 0.25]])]
    g = [np.array([[0.3 - 0.1j, 2.0 + 0.0j, -0.7 + 0.2j]])]
    # the real gradient of (Re W, Im W) is 2 (Re, Im) of dL/dW*
    gr, gi = 2 * g[0].real, 2 * g[0].imag
    opt = ptc.Adam(w0, lr=lr)
    w = w0
    for t in range(1, 7):
        prev = w[0]
        w = opt.step(w, g)
        d = w[0] - prev
        exp = -lr * (gr / (np.abs(gr) + eps) + 1j * gi / (np.abs(gi) + eps))
        assert np.abs(d - exp).max() < 1e-12, t
    opt = ptc.Adam(w0, lr=lr)
    w = opt.step(w0, g)
    zero = [np.zeros_like(g[0])]
    for t in range(2, 8):
        prev = w[0]
        w = opt.step(w, zero)
        mh = (1 - b1) * b1 ** (t - 1) / (1 - b1 ** t)
        vh = np.sqrt((1 - b2) * b2 ** (t - 1) / (1 - b2 ** t))
        exp = -lr * mh * (gr / (vh * np.abs(gr) + eps) + 1j * gi / (vh * np.abs(gi) + eps))
        assert np.abs((w[0] - prev) - exp).max() < 1e-12, t
        assert np.abs(opt.m[0][..., 0] - (1 - b1) * b1 ** (t - 1) * gr).max() < 1e-15
        assert np.abs(opt.v[0][..., 1] - (1 - b2) * b2 ** (t - 1) * gi ** 2).max() < 1e-15


def test_rounding_envelope_separates_rounding_from_mistakes():
    """The envelope the GPU network is held to (tests/ptc_envelope.py) is neither vacuous nor too
    tight: an evaluation that rounds every layer input and hidden activation to BF16 (the
    oracle's rounding model) lies well inside it -- forward, input gradient and every weight
    gradient, element-wise and in norm -- while a network with one path's transport direction
    reversed, or one boundary phase dropped, lies far outside."""
    import math

    from ptc_envelope import envelope, max_rel

    L = (4, 4, 2, 4)
    f = dirac.Fields(gen.su3_field(L, 0.5, 41), gen.u1_field(L, 0.3, 41),
                     dirac.Params(L, 0.1245, 1.6, 1.0, -1, (math.pi, 0.2, 0.0, -0.4)))
    for chans in [(1, 4, 1), (1, 2, 4, 1)]:
        ws = [ptc.round_bf16(w) for w in ptc.init_weights(chans, seed=3, scale=1.0)]
        r = ptc.round_bf16(gen.gaussian_spinor(L, 7))
        g = ptc.round_bf16(gen.gaussian_spinor(L, 9))
        env, env_gin, env_gw = envelope(f, ws, r, g)
        y, acts = ptc.forward(f, ws, r)
        gx, gW = ptc.backward(f, ws, acts, g)
        ym, am = ptc.forward(f, ws, r, bf16_inputs=True, last_contract_first=True, bf16_storage=True)
        gxm, gWm = ptc.backward(f, ws, am, g, bf16_inputs=True)
        for e, a, b in [(env, ym, y), (env_gin, gxm, gx)] + list(zip(env_gw, gWm, gW)):
            assert np.linalg.norm(a - b) / np.linalg.norm(b) < 0.6 * e.norm
            assert max_rel(a, b) < 0.7 * e.max
        # planted mistakes: path +1 replaced by -1 in the first layer; boundary phase of mu = 1 dropped
        bad = [w.copy() for w in ws]
        bad[0][3], bad[0][4] = ws[0][4], ws[0][3]
        yb, _ = ptc.forward(f, bad, r)
        assert np.linalg.norm(yb - y) / np.linalg.norm(y) > 20 * env.norm
        f0 = dirac.Fields(f.U, f.theta, dirac.Params(L, 0.1245, 1.6, 1.0, -1, (math.pi, 0.0, 0.0, -0.4)))
        y0, _ = ptc.forward(f0, ws, r)
        assert np.linalg.norm(y0 - y) / np.linalg.norm(y) > 5 * env.norm
