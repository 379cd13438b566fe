"""Gauge-covariant parallel-transport convolution (PTC) network, FP64 reference.

TEST INFRASTRUCTURE ONLY (see the package docstring).

The learned preconditioner is not in the paper; this is the reading of it that the library
builds (after Lehner and Wettig, gauge-equivariant neural networks as preconditioners, 2023):

  layer:   y_c(x) = sum_{c'} sum_{p in P} W[p, c, c'] (T_p x_{c'})(x)
  paths:   P = (0, +0, -0, +1, -1, +2, -2, +3, -3)
           T_0 = 1
           T_{+mu} psi(x) = V_mu(x) b+_mu(x) psi(x + mu)
           T_{-mu} psi(x) = V_mu(x - mu)^dag b-_mu(x) psi(x - mu)
  W[p, c, c'] is a complex 4x4 matrix acting on spin (colour untouched, hence gauge
  equivariant); channels 1 -> 8 -> 8 -> 1, no nonlinearity, no bias.
  loss:    L = mean_i |N(r_i) - e_i|^2 / |e_i|^2
  gradients (Wirtinger, L real):  with g = dL/dy*,
           dL/dx*_{c'} = sum_{p, c} T_p^dag W[p, c, c']^dag g_c
           dL/dW*[p, c, c'] = sum_{x, colour} g_c(x) (T_p x_{c'})(x)^dag
  The adjoint transport is T_{+mu}^dag = T_{-mu}.
  A real parameter w = Re W or Im W has dL/dw = 2 Re(dL/dW*) or 2 Im(dL/dW*).
  Adam (Kingma and Ba 2015) on the real and imaginary parts.
Fields are full LEX spinor fields [V, 4, 3]; weights of a layer are [9, n_out, n_in, 4, 4].
"""
from __future__ import annotations

import numpy as np

from . import dirac
from . import geometry as geo

PATHS = [(None, 0), (0, 1), (0, -1), (1, 1), (1, -1), (2, 1), (2, -1), (3, 1), (3, -1)]
NPATH = len(PATHS)
ADJ = [0, 2, 1, 4, 3, 6, 5, 8, 7]  # T_p^dag = T_{ADJ[p]}


def transport(f: dirac.Fields, psi: np.ndarray, p: int) -> np.ndarray:
    """T_p psi for a full LEX field psi [V, 4, 3]."""
    mu, d = PATHS[p]
    if mu is None:
        return psi.copy()
    L = f.p.dims
    sites = np.arange(f.V)
    x = geo.coords(sites, L)
    phi = f.p.bc_phase[mu]
    if d > 0:
        nb = geo.shift(sites, L, mu, 1, f.p.cstar)
        b = np.where(x[:, mu] == L[mu] - 1, np.exp(1j * phi), 1.0)
        return b[:, None, None] * np.einsum("nab,nsb->nsa", f.Vlink[:, mu], psi[nb])
    nb = geo.shift(sites, L, mu, -1, f.p.cstar)
    b = np.where(x[:, mu] == 0, np.exp(-1j * phi), 1.0)
    Vd = np.conj(np.swapaxes(f.Vlink[nb, mu], -1, -2))
    return b[:, None, None] * np.einsum("nab,nsb->nsa", Vd, psi[nb])


def round_bf16(a: np.ndarray) -> np.ndarray:
    """Each real component rounded to the nearest BF16 value (8 significant bits, ties to even),
    taken from its FP32 value: the precision in which the network's matrix-core inputs are formed."""
    a = np.asarray(a)
    cplx = np.iscomplexobj(a)
    f = np.ascontiguousarray(a.view(np.float64) if cplx else a.astype(np.float64)).astype(np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = (((u + 0x7FFF + ((u >> 16) & 1)) >> 16) << 16).astype(np.uint32)
    nan = np.isnan(f)
    out = r.view(np.float32).astype(np.float64)
    out[nan] = np.nan
    return out.view(np.complex128).reshape(a.shape) if cplx else out.reshape(a.shape)


def layer(f: dirac.Fields, W: np.ndarray, xs, bf16_inputs: bool = False) -> list:
    """y_c = sum_{c', p} W[p, c, c'] T_p x_{c'}; xs a list of n_in fields, W [9, n_out, n_in, 4, 4].
    With bf16_inputs each transported field T_p x_{c'} is rounded to BF16 before the spin
    contraction (the form the matrix-core kernel computes)."""
    n_out, n_in = W.shape[1], W.shape[2]
    assert len(xs) == n_in
    ys = [np.zeros_like(xs[0]) for _ in range(n_out)]
    for cp in range(n_in):
        for p in range(NPATH):
            t = transport(f, xs[cp], p)
            if bf16_inputs:
                t = round_bf16(t)
            for c in range(n_out):
                ys[c] += np.einsum("st,ntc->nsc", W[p, c, cp], t)
    return ys


def layer_contract_first(f: dirac.Fields, W: np.ndarray, xs, bf16_inputs: bool = False) -> list:
    """The same layer summed in the other order: z_{p,c} = sum_{c'} W[p, c, c'] x_{c'} at every
    site, then y_c = sum_p T_p z_{p,c}.  W acts on spin only and T_p on colour and position, so
    W[p, c, c'] T_p = T_p W[p, c, c'] and this equals layer() in exact arithmetic; it needs
    9 n_out transports instead of 9 n_in.  With bf16_inputs each input field x_{c'} is rounded to
    BF16 before the contraction (the form the library uses for a last layer with one output
    channel); z and the transports stay exact."""
    n_out, n_in = W.shape[1], W.shape[2]
    assert len(xs) == n_in
    xr = [round_bf16(x) for x in xs] if bf16_inputs else xs
    ys = [np.zeros_like(xs[0]) for _ in range(n_out)]
    for c in range(n_out):
        for p in range(NPATH):
            z = np.zeros_like(xs[0])
            for cp in range(n_in):
                z += np.einsum("st,ntc->nsc", W[p, c, cp], xr[cp])
            ys[c] += transport(f, z, p)
    return ys


def forward(f: dirac.Fields, weights, r: np.ndarray, bf16_inputs: bool = False, last_contract_first: bool = False,
            bf16_storage: bool = False):
    """N(r) and the activations of every layer (inputs of layer l are acts[l]).  With
    last_contract_first the last layer is summed as in layer_contract_first (the library does so
    when the network has more than one layer and one output channel).  With bf16_storage the
    output of every layer but the last is rounded to BF16 before the next layer reads it (the
    library stores those activations in BF16); the input and the output stay unrounded."""
    acts = [[r]]
    for l, W in enumerate(weights):
        last = l == len(weights) - 1
        if last_contract_first and last:
            y = layer_contract_first(f, W, acts[-1], bf16_inputs)
        else:
            y = layer(f, W, acts[-1], bf16_inputs)
        if bf16_storage and not last:
            y = [round_bf16(v) for v in y]
        acts.append(y)
    return acts[-1][0], acts


def backward(f: dirac.Fields, weights, acts, g_out: np.ndarray, bf16_inputs: bool = False):
    """Given g = dL/dN(r)*, return (dL/dr*, [dL/dW*] per layer).  With bf16_inputs the input
    gradient is formed as the matrix-core kernel forms it: each transported gradient
    T_{adj p} g_c is rounded to BF16, then contracted with W[p, c, c']^dag (spin matrices commute
    with the transports, so without rounding this equals T_p^dag W^dag g).  The weight gradient
    is exact in both cases."""
    grads = [None] * len(weights)
    g = [g_out]
    for l in range(len(weights) - 1, -1, -1):
        W = weights[l]
        xs = acts[l]
        n_out, n_in = W.shape[1], W.shape[2]
        gW = np.zeros_like(W)
        gx = [np.zeros_like(xs[0]) for _ in range(n_in)]
        for cp in range(n_in):
            for p in range(NPATH):
                t = transport(f, xs[cp], p)
                for c in range(n_out):
                    # dL/dW*[p, c, c'] = sum_{x, colour} g_c (T_p x_{c'})^dag
                    gW[p, c, cp] += np.einsum("nsa,nta->st", g[c], np.conj(t))
        if bf16_inputs:
            for c in range(n_out):
                for p in range(NPATH):
                    t = round_bf16(transport(f, g[c], ADJ[p]))
                    for cp in range(n_in):
                        gx[cp] += np.einsum("ts,nta->nsa", np.conj(W[p, c, cp]), t)
        else:
            for cp in range(n_in):
                for p in range(NPATH):
                    acc = np.zeros_like(xs[0])
                    for c in range(n_out):
                        acc += np.einsum("ts,nta->nsa", np.conj(W[p, c, cp]), g[c])  # W^dag g
                    gx[cp] += transport(f, acc, ADJ[p])  # T_p^dag = T_{ADJ[p]}
        grads[l] = gW
        g = gx
    return g[0], grads


def loss_and_grads(f: dirac.Fields, weights, pairs, bf16_inputs: bool = False, last_contract_first: bool = False,
                   bf16_storage: bool = False):
    """L = mean_i |N(r_i) - e_i|^2 / |e_i|^2 and dL/dW* per layer (forward as in forward(); the
    gradients treat each rounding as the identity, with the rounded activations)."""
    total = 0.0
    gsum = [np.zeros_like(W) for W in weights]
    n = len(pairs)
    for r, e in pairs:
        y, acts = forward(f, weights, r, bf16_inputs, last_contract_first, bf16_storage)
        ne2 = np.vdot(e, e).real
        d = y - e
        total += np.vdot(d, d).real / ne2 / n
        _, gw = backward(f, weights, acts, d / ne2 / n, bf16_inputs)
        for k in range(len(weights)):
            gsum[k] += gw[k]
    return total, gsum


def dirac_as_layer(f: dirac.Fields) -> np.ndarray:
    """The single 1 -> 1 layer that equals D when the clover term vanishes:
    W_0 = (4 + m0) 1, W_{+mu} = -1/2 (1 - gamma_mu), W_{-mu} = -1/2 (1 + gamma_mu)."""
    W = np.zeros((NPATH, 1, 1, 4, 4), dtype=np.complex128)
    W[0, 0, 0] = (4.0 + f.p.m0) * np.eye(4)
    for p in range(1, NPATH):
        mu, d = PATHS[p]
        W[p, 0, 0] = -0.5 * (dirac.ONE4 - d * dirac.GAMMA[mu])
    return W


def init_weights(channels, seed: int, scale: float = 0.1):
    """Random complex weights [9, c_out, c_in, 4, 4] per layer, N(0, scale^2 / fan_in) per real part."""
    rng = np.random.default_rng(seed)
    ws = []
    for cin, cout in zip(channels[:-1], channels[1:]):
        s = scale / np.sqrt(NPATH * cin)
        ws.append(s * (rng.normal(size=(NPATH, cout, cin, 4, 4)) + 1j * rng.normal(size=(NPATH, cout, cin, 4, 4))))
    return ws


class Adam:
    """Adam on the real and imaginary parts of complex weights (Kingma and Ba 2015)."""

    def __init__(self, weights, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
        self.lr, self.b1, self.b2, self.eps = lr, b1, b2, eps
        self.m = [np.zeros(W.shape + (2,)) for W in weights]
        self.v = [np.zeros(W.shape + (2,)) for W in weights]
        self.t = 0

    def step(self, weights, grads_conj):
        """grads_conj: dL/dW*; the real gradient of (Re W, Im W) is 2 (Re, Im) of it."""
        self.t += 1
        out = []
        for k, (W, G) in enumerate(zip(weights, grads_conj)):
            g = 2.0 * np.stack([G.real, G.imag], axis=-1)
            self.m[k] = self.b1 * self.m[k] + (1 - self.b1) * g
            self.v[k] = self.b2 * self.v[k] + (1 - self.b2) * g * g
            mh = self.m[k] / (1 - self.b1 ** self.t)
            vh = self.v[k] / (1 - self.b2 ** self.t)
            w = np.stack([W.real, W.imag], axis=-1) - self.lr * mh / (np.sqrt(vh) + self.eps)
            out.append(w[..., 0] + 1j * w[..., 1])
        return out
