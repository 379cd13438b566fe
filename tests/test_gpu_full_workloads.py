"""The solve workloads at their full sizes, checked by the FP64 oracle's own operator.

48^3 x 96 (the mixed-precision workload: kappa = 0.125, c_sw = 1.6, c_sw^QED = 1.0, qhat = +2,
eps = 0.5, seed 301) in plain FP64 GCR and in FP64 defect correction around FP32, FP16 and BF16
inner solves; the batched workload's 16^3 x 32 and 8^4 lattices with their 12 point sources; FP16
and BF16 inner solves on 16^3 x 32.

At 48^3 x 96 the oracle cannot solve, so it recomputes the true residual r = b - D x of every GPU
solution from the definition at sampled sites (several hundred random sites, plus sites on the
time boundary where the antiperiodic phase enters).  The norm of r over any subset of sites is at
most its norm over the lattice, so |r_S| <= tol |b| is a necessary condition of the solve's
stopping test that holds however the sites are picked, and an error of the operator at a
sampled site (a wrong phase, link or clover entry) leaves r_S of the size of b there."""
import math

import numpy as np
import pytest
import torch

import gen
import paper_2502_02490_amd as P
from gpu_util import Case, flush, need_gpu, rel, to_dev
from oracle import dirac as odirac
from oracle import geometry as geo

pytestmark = pytest.mark.gpu


def sampled_sites(dims, n, seed):
    """n random sites plus the sites at both ends of the time direction in the first row."""
    V = geo.volume(dims)
    rng = np.random.default_rng(seed)
    s = rng.choice(V, n, replace=False)
    L3L2L1 = dims[1] * dims[2] * dims[3]
    edge = np.concatenate([np.arange(8), (dims[0] - 1) * L3L2L1 + np.arange(8)])
    return np.unique(np.concatenate([s, edge]))


def sampled_residual(f, x, b, sites):
    """|b - D x| over `sites` (oracle, from the definition) divided by |b| over the lattice."""
    r = b[sites] - odirac.apply_D(f, x, sites)
    return float(np.linalg.norm(r) / np.linalg.norm(b))


def test_48c96_solves_sampled_residual():
    need_gpu()
    dims = (96, 48, 48, 48)
    flush("[gpu] 48^3x96: generating fields")
    U = gen.su3_field(dims, 0.5, 301)
    th = gen.u1_field(dims, 0.3, 301)
    b = gen.gaussian_spinor(dims, 301)
    p = odirac.Params(dims, 0.1250, 1.6, 1.0, 2, (math.pi, 0.0, 0.0, 0.0))
    D = P.Dirac(torch.from_numpy(U).cuda(), torch.from_numpy(th).cuda(), dims, 0.1250, 1.6, 1.0, 2)
    try:
        f = odirac.Fields(U, th, p)
        sites = sampled_sites(dims, 512, 3)
        bd = torch.from_numpy(b).cuda()
        x64 = None
        for name, kw in (("fp64", dict(method=P.GCR)),) + tuple(
                (f"mixed_{pr}", dict(method=P.MIXED_GCR, inner_prec=pr)) for pr in ("f32", "f16", "bf16")):
            flush(f"[gpu] 48^3x96 solve {name}")
            x = torch.zeros_like(bd)
            info = D.solve(x, bd, tol=1e-10, restart=32, max_iter=100000, **kw)
            xh = x.cpu().numpy()
            res = sampled_residual(f, xh, b, sites)
            msg = f"[gpu] 48^3x96 {name}: {info.iters} it, GPU true residual {info.true_rel_res:.2e}, " \
                  f"oracle residual over {len(sites)} sites / |b| {res:.2e}"
            if x64 is None:
                x64 = xh
            else:
                msg += f", max|x - x_fp64| / max|x_fp64| {np.abs(xh - x64).max() / np.abs(x64).max():.2e}"
            flush(msg)
            assert info.true_rel_res < 1e-10
            assert res <= 1e-10
            del x, xh
    finally:
        D.close()


@pytest.mark.parametrize("inner", ["f32", "bf16"])
def test_batched_point_sources_16c32_and_8c4(inner):
    """The batched workload's 16^3 x 32 lattice (kappa_2 = 0.120 + 0.005 * 2 / 7, seed 403) and 8^4
    lattice (kappa_0 = 0.120, seed 401) with 12 spin-colour point sources at the origin each,
    FP64 defect correction around batched FP32 GCR (the configuration) and around batched BF16
    GCR(16): every solution's residual recomputed by the oracle at the source's neighbourhood and
    at random sites."""
    need_gpu()
    lat = [((32, 16, 16, 16), 0.120 + 0.005 * 2 / 7, 403), ((8, 8, 8, 8), 0.120, 401)]
    cases = []
    try:
        for dims, kappa, seed in lat:
            flush(f"[gpu] batched point sources {dims}")
            cases.append(Case(dims, kappa=kappa, seed=seed))
        bs = []
        for c in cases:
            bb = np.zeros((12, c.V, 4, 3), dtype=np.complex128)
            for s_ in range(4):
                for a in range(3):
                    bb[3 * s_ + a, 0, s_, a] = 1.0
            bs.append(bb)
        xs = [torch.zeros((12, c.V, 4, 3), dtype=torch.complex128, device="cuda") for c in cases]
        infos = P.solve_batched([c.D for c in cases], xs, [to_dev(bb) for bb in bs], 12, method=P.MIXED_GCR,
                                inner_prec=inner, tol=1e-10, restart=8 if inner == "f32" else 16)
        for c, bb, x, row in zip(cases, bs, xs, infos):
            nbh = np.unique(np.concatenate([[0]] + [geo.shift(np.array([0]), c.dims, mu, s, 0)
                                                    for mu in range(4) for s in (1, -1)]))
            sites = np.unique(np.concatenate([nbh, sampled_sites(c.dims, 256, 5)]))
            xh = x.cpu().numpy()
            worst = 0.0
            for r in range(12):
                assert row[r].true_rel_res < 1e-10
                worst = max(worst, sampled_residual(c.f, xh[r], bb[r], sites))
            flush(f"[gpu] batched {inner} {c.dims}: worst oracle residual over {len(sites)} sites {worst:.2e}")
            assert worst <= 1e-10
    finally:
        for c in cases:
            c.D.close()


@pytest.mark.parametrize("inner", ["f16", "bf16"])
def test_mixed_16bit_inner_16c32(inner):
    """FP64 defect correction around FP16 / BF16 inner GCR on 16^3 x 32: the oracle recomputes
    the full residual of the solution, which also agrees with the plain FP64 solution to the
    accuracy the stopping test allows."""
    need_gpu()
    flush(f"[gpu] mixed {inner} 16^3x32")
    c = Case((32, 16, 16, 16), seed=501)
    try:
        eta = c.spinor(11)
        bd = to_dev(eta)
        x64 = torch.zeros_like(bd)
        c.D.solve(x64, bd, method=P.GCR, tol=1e-10)
        x = torch.zeros_like(bd)
        info = c.D.solve(x, bd, method=P.MIXED_GCR, inner_prec=inner, tol=1e-10, max_iter=100000)
        xh = x.cpu().numpy()
        res = float(np.linalg.norm(eta - odirac.apply_D(c.f, xh)) / np.linalg.norm(eta))
        diff = rel(xh, x64.cpu().numpy())
        flush(f"[gpu] mixed {inner} 16^3x32: {info.iters} inner it, {info.outer} outer, oracle residual "
              f"{res:.2e}, difference from the FP64 solution {diff:.2e}")
        assert res < 1e-10 and info.true_rel_res < 1e-10
        # both solutions satisfy |b - D x| < 1e-10 |b|; their difference is bounded by
        # |D^-1| 2e-10 |b| (|D^-1| |b| / |x| <= cond(D) ~ 10 at these parameters)
        assert diff < 2e-9
    finally:
        c.D.close()
