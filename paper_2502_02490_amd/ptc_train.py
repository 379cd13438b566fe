"""Training driver of the learned preconditioner (a parallel-transport convolution network).

Training pairs (r, e) with e = D^-1 r come from the library's own FP64 solver.  For a Gaussian
right-hand side b with solution x* (FP64 even-odd GCR to 1e-12), the iterate x_k after k GCR
iterations from zero has residual r_k = b - D x_k and error e_k = x* - x_k, and D e_k = r_k.
k = 0 gives the broadband pair (b, x*); larger k give the low-mode dominated residuals a
flexible GCR hands its preconditioner late in a solve.  Each pair is scaled so that |e| = 1
(the network is linear and the loss is scale free).

The loss is mean_i |N(r_i) - e_i|^2 / |e_i|^2; ptc_train_step runs the forward pass, the
loss, the input and weight gradients and one Adam step in the library's kernels.  Minibatches
are drawn from one gauge field at a time (the network transports with that field's links).

Checkpoints are .npz files without pickled objects: a JSON header (version, channels, dtype,
Adam step, epochs done, shuffling seed, free-form metadata) and float32 arrays of weights and
Adam moments, so that a resumed run continues bit-for-bit where it stopped.
"""
from __future__ import annotations

import json
import math
import time

import numpy as np
import torch

from . import FGCR_PTC, FGCR_PTC_EO, GCR, PTC, Dirac

CHECKPOINT_VERSION = 1
DEFAULT_SNAPSHOTS = (0, 2, 4, 8, 16, 32)


def _scaled_pair_f32(D: Dirac, r64, e64):
    """(r, e) scaled so that |e| = 1 and rounded once to NATIVE F32 (library calls)."""
    ne = math.sqrt(D.dot(e64, e64, "f64").real)
    r32, e32 = D.native_empty("f32"), D.native_empty("f32")
    D.lincomb(r32, 1.0 / ne, r64, out_prec="f32", in_prec="f64")
    D.lincomb(e32, 1.0 / ne, e64, out_prec="f32", in_prec="f64")
    return r32, e32


def generate_pairs(D: Dirac, n_pairs: int, seed: int, snapshots=DEFAULT_SNAPSHOTS, restart: int = 32, log=None):
    """n_pairs (r, e) pairs on the lattice of D as NATIVE F32 full vectors (two lists).  The
    solves, residuals r_k = b - D x_k, errors e_k = x* - x_k and the scaling run in the library
    on NATIVE FP64 vectors; only the Gaussian right-hand sides are drawn here."""
    g = torch.Generator(device="cpu").manual_seed(seed)
    rs, es = [], []
    t0 = time.perf_counter()
    while len(rs) < n_pairs:
        b = D.to_native(torch.randn((D.V, 4, 3), dtype=torch.complex128, generator=g).cuda(), "f64", "lex")
        xs = D.native_empty("f64")
        D.solve(xs, b, method=GCR, tol=1e-12, restart=restart, layout="native")
        for k in snapshots:
            if len(rs) == n_pairs:
                break
            if k == 0:
                r, e = b, xs
            else:
                xk = D.native_empty("f64")
                D.solve(xk, b, method=GCR, tol=1e-12, max_iter=k, restart=restart, layout="native",
                        raise_on_noconv=False)
                r, e = D.native_empty("f64"), D.native_empty("f64")
                D.residual(r, b, xk)
                D.lincomb(e, 1.0, xs, -1.0, xk)
            r32, e32 = _scaled_pair_f32(D, r, e)
            rs.append(r32)
            es.append(e32)
        if log and len(rs) % (10 * len(snapshots)) < len(snapshots):
            log(f"pairs {len(rs)}/{n_pairs} ({time.perf_counter() - t0:.1f} s)")
    torch.cuda.synchronize()
    return rs, es


def generate_apply_pairs(D: Dirac, n_pairs: int, seed: int):
    """n_pairs (r, e) pairs with a Gaussian e and r = D e (one operator application each, no
    solve): the error distribution of a converged smoother, dominated by the high modes."""
    g = torch.Generator(device="cpu").manual_seed(seed)
    rs, es = [], []
    for _ in range(n_pairs):
        e = D.to_native(torch.randn((D.V, 4, 3), dtype=torch.complex128, generator=g).cuda(), "f64", "lex")
        r = D.native_empty("f64")
        D.apply(r, e, "f64", "native")
        r32, e32 = _scaled_pair_f32(D, r, e)
        rs.append(r32)
        es.append(e32)
    torch.cuda.synchronize()
    return rs, es


def init_weights(channels, seed: int, scale: float = 0.1):
    """Small random complex weights (N(0, scale^2 / (9 c_in)) per real part) plus, on the
    unshifted path, 1/c of the identity from channel min(c, c') to min(c, c'), so that the
    untrained network is close to a multiple of the identity map."""
    rng = np.random.default_rng(seed)
    ws = []
    for cin, cout in zip(channels[:-1], channels[1:]):
        s = scale / math.sqrt(9 * cin)
        w = s * (rng.normal(size=(9, cout, cin, 4, 4)) + 1j * rng.normal(size=(9, cout, cin, 4, 4)))
        for c in range(cout):
            w[0, c, c % cin] += np.eye(4) / (cin if cin > cout else 1)
        ws.append(w.astype(np.complex64))
    return ws


def evaluate(ops_pairs, net: PTC):
    """Mean loss |N(r) - e|^2 / |e|^2 over all pairs, without an update (held-out pairs)."""
    tot, n = 0.0, 0
    for D, rs, es in ops_pairs:
        if rs:
            tot += net.loss(D, rs, es) * len(rs)
            n += len(rs)
    return tot / max(n, 1)


def train(ops_pairs, net: PTC, epochs: int, batch: int, lr: float, seed: int = 0, start_epoch: int = 0,
          log=None, lr_decay: float = 1.0, time_budget: float | None = None):
    """ops_pairs: list of (Dirac, rs, es).  Epoch ep shuffles with a generator seeded by
    (seed, ep), so that a run resumed at start_epoch repeats the same minibatches.  The
    learning rate of epoch ep is lr * lr_decay**ep.  With time_budget (seconds) no new epoch
    starts once the budget is spent.  Returns the mean loss of every epoch run."""
    history = []
    t_start = time.perf_counter()
    for ep in range(start_epoch, epochs):
        if time_budget is not None and history and time.perf_counter() - t_start > time_budget:
            break
        rng = np.random.default_rng([seed, ep])
        batches = []
        for j, (_, rs, _) in enumerate(ops_pairs):
            idx = rng.permutation(len(rs))
            batches += [(j, idx[k:k + batch]) for k in range(0, len(idx), batch)]
        order = rng.permutation(len(batches))
        tot, n = 0.0, 0
        t0 = time.perf_counter()
        lr_ep = lr * lr_decay ** ep
        for bi in order:
            j, sel = batches[bi]
            D, rs, es = ops_pairs[j]
            loss = net.train_step(D, [rs[i] for i in sel], [es[i] for i in sel], lr_ep)
            tot += loss * len(sel)
            n += len(sel)
        history.append(tot / n)
        if log:
            log(f"epoch {ep}: loss {history[-1]:.5f} lr {lr_ep:.2e} ({time.perf_counter() - t0:.1f} s)")
    return history


def save_checkpoint(path: str, net: PTC, epochs_done: int, seed: int, meta: dict | None = None):
    ws = net.get_weights()
    m, v, step = net.get_adam_state()
    header = {"version": CHECKPOINT_VERSION, "channels": list(net.channels), "dtype": "complex64",
              "adam_step": step, "epochs_done": epochs_done, "shuffle_seed": seed, "meta": meta or {}}
    arrays = {f"layer{k}": w for k, w in enumerate(ws)}
    np.savez(path, header=np.frombuffer(json.dumps(header).encode(), dtype=np.uint8), adam_m=m, adam_v=v,
             **arrays)


def load_checkpoint(path: str):
    """Returns (PTC with the stored weights and Adam state, header dict)."""
    with np.load(path, allow_pickle=False) as z:
        header = json.loads(bytes(z["header"]).decode())
        if header.get("version") != CHECKPOINT_VERSION:
            raise ValueError(f"unsupported checkpoint version {header.get('version')}")
        net = PTC(tuple(header["channels"]))
        net.set_weights([z[f"layer{k}"] for k in range(len(header["channels"]) - 1)])
        net.set_adam_state(z["adam_m"], z["adam_v"], int(header["adam_step"]))
    return net, header


def compare_solvers(D: Dirac, net: PTC, b: torch.Tensor, tol: float = 1e-10, restart: int = 32, reps: int = 1,
                    flex_restart: int = 8):
    """Solve D x = b with plain even-odd FP64 GCR(restart), flexible GCR(flex_restart) on D with
    the network, and flexible GCR(flex_restart) on D-hat with the network's even block; returns a
    dict of iterations, restart lengths, seconds (best of reps) and residuals for each.  The
    flexible forms take the same iterations at restart 8 as at 32 on the 32^3 x 64 field of the
    measurements, for a quarter of the orthogonalisation work."""
    out = {}
    for name, kw in (("eo_gcr", dict(method=GCR, restart=restart)),
                     ("fgcr_ptc", dict(method=FGCR_PTC, ptc=net, restart=flex_restart)),
                     ("fgcr_ptc_eo", dict(method=FGCR_PTC_EO, ptc=net, restart=flex_restart))):
        best = None
        for _ in range(reps):
            x = torch.zeros_like(b)
            info = D.solve(x, b, tol=tol, max_iter=20000, **kw)
            if best is None or info.seconds < best.seconds:
                best = info
        out[name] = {"iters": best.iters, "restart": kw["restart"], "restarts": best.restarts, "seconds": best.seconds,
                     "true_rel_res": best.true_rel_res, "fell_back": bool(best.fell_back)}
    return out
