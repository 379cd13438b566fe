"""What the trained network gains: a (1, 8, 8, 1) and a (1, 4, 1) network, each trained briefly with
the library's own kernels on pairs from two 16^3 x 32 fields (eps = 0.5, kappa = 0.1245, c_sw = 1.6, c_sw^QED = 1.0,
qhat = -1), then used as the preconditioner of flexible GCR on the Schur system of a third,
held-out field, against plain even-odd GCR (the method without it) on the same field and source,
both to 1e-10; the held-out loss falls during training."""
import time

import numpy as np
import pytest
import torch

import gen
import paper_2502_02490_amd as P
from gpu_util import Case, flush, need_gpu, to_dev
from oracle import dirac as odirac
from paper_2502_02490_amd import ptc_train as T

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("channels", [(1, 8, 8, 1), (1, 4, 1)])
def test_trained_network_cuts_iterations_on_a_held_out_field(channels):
    need_gpu()
    dims = (32, 16, 16, 16)
    train = []
    try:
        t0 = time.perf_counter()
        for j, seed in enumerate((501, 502)):
            flush(f"[gpu] ptc gain: pairs on field {seed}")
            c = Case(dims, kappa=0.1245, seed=seed)
            rs, es = T.generate_pairs(c.D, 80, seed=seed)
            ra, ea = T.generate_apply_pairs(c.D, 80, seed=seed + 100)
            train.append((c, rs + ra, es + ea))
        held = Case(dims, kappa=0.1245, seed=503)
        hr, he = T.generate_pairs(held.D, 6, seed=10503)
        har, hae = T.generate_apply_pairs(held.D, 6, seed=10603)
        net = P.PTC(channels)
        try:
            net.set_weights(T.init_weights(channels, seed=7))
            loss0 = T.evaluate([(held.D, hr + har, he + hae)], net)
            T.train([(c.D, rs, es) for c, rs, es in train], net, epochs=6, batch=16, lr=2e-3, seed=11, lr_decay=0.8)
            loss1 = T.evaluate([(held.D, hr + har, he + hae)], net)
            flush(f"[gpu] ptc gain: held-out loss {loss0:.3f} -> {loss1:.3f} ({time.perf_counter() - t0:.1f} s)")
            assert loss1 < 0.5 * loss0
            eta = held.spinor(505)
            b = to_dev(eta)
            T.compare_solvers(held.D, net, b, tol=1e-10)  # warm-up: tuner, work buffers
            res = T.compare_solvers(held.D, net, b, tol=1e-10)
            flush(f"[gpu] ptc gain on the held-out field: plain even-odd GCR {res['eo_gcr']['iters']} it "
                  f"{res['eo_gcr']['seconds'] * 1e3:.1f} ms, FGCR with the network on D-hat "
                  f"{res['fgcr_ptc_eo']['iters']} it {res['fgcr_ptc_eo']['seconds'] * 1e3:.1f} ms, on D "
                  f"{res['fgcr_ptc']['iters']} it {res['fgcr_ptc']['seconds'] * 1e3:.1f} ms")
            assert not res["fgcr_ptc_eo"]["fell_back"]
            assert res["fgcr_ptc_eo"]["true_rel_res"] < 1e-10
            assert res["fgcr_ptc_eo"]["iters"] < (0.8 if len(channels) > 3 else 0.9) * res["eo_gcr"]["iters"]
            # the solution the network-preconditioned solve returns satisfies the oracle's operator
            x = torch.zeros_like(b)
            held.D.solve(x, b, method=P.FGCR_PTC_EO, ptc=net, tol=1e-10)
            r = eta - odirac.apply_D(held.f, x.cpu().numpy())
            assert np.linalg.norm(r) / np.linalg.norm(eta) < 1e-10
        finally:
            net.close()
            held.D.close()
    finally:
        for c, _, _ in train:
            c.D.close()
