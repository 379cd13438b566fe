"""Rounding envelope of a BF16 matrix-core evaluation of the parallel-transport network.

Test infrastructure: a tolerance, derived before any GPU result is seen, for comparing the
library's network with the plain FP64 oracle (oracle/ptc.py with every rounding option off).

What any BF16 matrix-core evaluation has to round: the operands of each layer's contraction (the
layer inputs, taken before or after their transport) and, when they are stored in BF16, the
hidden activations and hidden gradients.  Rounding to BF16 (8 significant bits, round to
nearest) changes a real number by a relative amount of at most u = 2^-8.  FP32 accumulation adds
a relative 2^-24 per addition, four orders of magnitude below, and the weights are BF16 in both
evaluations (the network's weights are specified in BF16).

The envelope pushes perturbations of the largest size a rounding can make, u |x| with a random
sign on every real component, through the exact (FP64) network at each of those points, and
measures the relative change of the output: the amplification of each layer's rounding by the
layers after it, measured rather than bounded by operator norms (a worst-case bound through the
layers' norms exceeds the rounding effect by about two orders of magnitude, since rounding errors
are not aligned with the network's leading singular vectors).  Both placements of the input
rounding are evaluated (before the transport: one rounding per input field; after it: one per
path) and the larger result is the envelope.  Real rounding errors are spread uniformly below
u |x| (RMS u |x| / sqrt(3)), so an evaluation that rounds at these points lands near 0.4 of the
envelope; a sign, index or transport mistake moves the output by O(1).
"""
from __future__ import annotations

import numpy as np

from oracle import ptc as optc

U_BF16 = 2.0 ** -8


def _perturb(rng, x: np.ndarray, u: float) -> np.ndarray:
    sr = rng.choice([-1.0, 1.0], x.shape)
    si = rng.choice([-1.0, 1.0], x.shape)
    return x + u * (x.real * sr + 1j * x.imag * si)


def _layer(f, W, xs, rng, u, after_transport):
    """One layer y_c = sum_{c', p} W[p, c, c'] T_p x_{c'} with its contraction operands perturbed."""
    n_out, n_in = W.shape[1], W.shape[2]
    ys = [np.zeros_like(xs[0]) for _ in range(n_out)]
    xr = xs if after_transport else [_perturb(rng, x, u) for x in xs]
    for cp in range(n_in):
        for p in range(optc.NPATH):
            t = optc.transport(f, xr[cp], p)
            if after_transport:
                t = _perturb(rng, t, u)
            for c in range(n_out):
                ys[c] += np.einsum("st,ntc->nsc", W[p, c, cp], t)
    return ys


def _adjoint_layer(f, W, gs, rng, u, after_transport):
    """dL/dx*_{c'} = sum_{p, c} T_p^dag W[p, c, c']^dag g_c with the operands g perturbed."""
    n_out, n_in = W.shape[1], W.shape[2]
    gx = [np.zeros_like(gs[0]) for _ in range(n_in)]
    gr = gs if after_transport else [_perturb(rng, g, u) for g in gs]
    for c in range(n_out):
        for p in range(optc.NPATH):
            t = optc.transport(f, gr[c], optc.ADJ[p])
            if after_transport:
                t = _perturb(rng, t, u)
            for cp in range(n_in):
                gx[cp] += np.einsum("ts,nta->nsa", np.conj(W[p, c, cp]), t)
    return gx


def _perturbed_network(f, weights, r, g, rng, u, after_transport):
    """Forward activations, input gradient and weight gradients of the network with every rounding
    point perturbed (hidden activations and hidden gradients count as stored in BF16)."""
    acts = [[r]]
    for l, W in enumerate(weights):
        y = _layer(f, W, acts[-1], rng, u, after_transport)
        if l < len(weights) - 1:
            y = [_perturb(rng, v, u) for v in y]
        acts.append(y)
    out = acts[-1][0]
    if g is None:
        return out, None, None
    grads = [None] * len(weights)
    gs = [g]
    for l in range(len(weights) - 1, -1, -1):
        W = weights[l]
        gW = np.zeros_like(W)
        for cp in range(W.shape[2]):
            for p in range(optc.NPATH):
                t = optc.transport(f, acts[l][cp], p)
                for c in range(W.shape[1]):
                    gW[p, c, cp] += np.einsum("nsa,nta->st", gs[c], np.conj(t))
        grads[l] = gW
        gx = _adjoint_layer(f, W, gs, rng, u, after_transport)
        if l > 0:
            gx = [_perturb(rng, v, u) for v in gx]
        gs = gx
    return out, gs[0], grads


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


class Env:
    """Envelope of one result: `norm` bounds |a - b| / |b| (2-norms), `max` bounds
    max_i |a_i - b_i| / max_i |b_i| (the same statistic taken on the envelope's own perturbed
    result, so the element-wise bar needs no further factor)."""

    def __init__(self):
        self.norm = 0.0
        self.max = 0.0

    def add(self, perturbed, exact):
        self.norm = max(self.norm, _rel(perturbed, exact))
        self.max = max(self.max, max_rel(perturbed, exact))

    def check(self, got, exact, what: str):
        n, m = _rel(got, exact), max_rel(got, exact)
        msg = f"{what}: |d|/|y| {n:.2e} (envelope {self.norm:.2e}), max|d|/max|y| {m:.2e} (envelope {self.max:.2e})"
        assert n <= self.norm and m <= self.max, msg
        return msg


def envelope(f, weights, r, g=None, seed: int = 0, u: float = U_BF16):
    """Envelopes (Env) of the forward output, and with g = dL/dN(r)* of the input gradient and of
    each layer's weight gradient, for a BF16 evaluation of the network with the given (BF16)
    weights on the FP32 input r: (env_out, env_gin, [env_gW per layer])."""
    y, acts = optc.forward(f, weights, r)
    gx = gW = None
    if g is not None:
        gx, gW = optc.backward(f, weights, acts, g)
    rng = np.random.default_rng(seed)
    e_out, e_gin, e_gw = Env(), Env(), [Env() for _ in weights]
    for after in (False, True):
        yp, gxp, gWp = _perturbed_network(f, weights, r, g, rng, u, after)
        e_out.add(yp, y)
        if g is not None:
            e_gin.add(gxp, gx)
            for e, a, b in zip(e_gw, gWp, gW):
                e.add(a, b)
    return e_out, (e_gin if g is not None else None), (e_gw if g is not None else None)


def max_rel(a, b) -> float:
    """max_i |a_i - b_i| / max_i |b_i| (element-wise comparison, relative to the largest entry)."""
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / np.abs(b).max())
