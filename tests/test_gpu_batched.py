"""Batched solves (many right-hand sides on lattices of uneven size) against single solves and
the oracle: every system's solution must match, graphs on or off must agree bitwise."""
import os

import numpy as np
import pytest
import torch

import gen
import paper_2502_02490_amd as P
from gpu_util import Case, flush, need_gpu, rel, to_dev
from oracle import geometry as geo
from oracle import solvers as osolvers

pytestmark = pytest.mark.gpu


def point_sources(dims, site=0):
    """The 12 spin-colour point sources at one site, stacked [12, V, 4, 3]."""
    V = geo.volume(dims)
    b = np.zeros((12, V, 4, 3), dtype=np.complex128)
    for s in range(4):
        for a in range(3):
            b[3 * s + a, site, s, a] = 1.0
    return b


@pytest.fixture(scope="module")
def lattices():
    need_gpu()
    flush("[gpu] batched cases")
    cs = [Case((4, 4, 4, 4), kappa=0.120, seed=401), Case((6, 2, 4, 8), kappa=0.1236, seed=402),
          Case((2, 4, 2, 4), kappa=0.125, seed=403)]
    yield cs
    for c in cs:
        c.D.close()


def test_batched_fp64_matches_oracle(lattices):
    bs = [point_sources(c.dims) for c in lattices]
    xs = [torch.zeros_like(to_dev(b)) for b in bs]
    infos = P.solve_batched([c.D for c in lattices], xs, [to_dev(b) for b in bs], 12, method=P.GCR, tol=1e-12)
    for c, b, x, inf in zip(lattices, bs, xs, infos):
        xg = x.cpu().numpy()
        for r in (0, 5, 11):
            exact, _ = osolvers.solve_eo(c.f, b[r], 1e-13)
            assert rel(xg[r], exact) < 1e-9, (c.dims, r)
        assert all(i.true_rel_res < 1e-12 for i in inf)
    # convergence is decided on the device: the host waits for a value once per 4 iterations of a
    # cycle and once per cycle end, plus a few set-up and final reads per lattice
    iters = max(i.iters for row in infos for i in row)
    cycles = max(i.restarts for row in infos for i in row) + 1
    syncs = infos[0][0].host_syncs
    flush(f"[gpu] batched FP64: {iters} iterations, {cycles} cycles, {syncs} host waits")
    assert syncs <= iters // 4 + 2 * cycles + 3 * len(lattices) + 4, (syncs, iters)


def test_batched_mixed_f32_matches_single(lattices):
    bs = [point_sources(c.dims) for c in lattices]
    xs = [torch.zeros_like(to_dev(b)) for b in bs]
    infos = P.solve_batched([c.D for c in lattices], xs, [to_dev(b) for b in bs], 12, method=P.MIXED_GCR,
                            inner_prec="f32", tol=1e-10)
    for c, b, x, inf in zip(lattices, bs, xs, infos):
        for r in (1, 7):
            single = torch.zeros_like(to_dev(b[r]))
            c.D.solve(single, to_dev(b[r]), method=P.GCR, tol=1e-12)
            assert rel(x[r].cpu().numpy(), single.cpu().numpy()) < 1e-8
        assert all(i.true_rel_res < 1e-10 for i in inf)
        flush(f"[gpu] batched mixed {c.dims}: inner iters {[i.iters for i in inf]}, outer {[i.outer for i in inf]}")


def test_graphs_replay_bitwise(lattices):
    """The hipGraph replays give exactly the eager launches' results (many replays per solve)."""
    c = lattices[0]
    b = to_dev(point_sources(c.dims))
    x1, x2 = torch.zeros_like(b), torch.zeros_like(b)
    P.solve_batched([c.D], [x1], [b], 12, method=P.MIXED_GCR, inner_prec="f32", tol=1e-10)
    os.environ["DIRAC_GRAPHS"] = "0"
    try:
        P.solve_batched([c.D], [x2], [b], 12, method=P.MIXED_GCR, inner_prec="f32", tol=1e-10)
    finally:
        del os.environ["DIRAC_GRAPHS"]
    assert torch.equal(x1, x2)


def test_batched_gaussian_rhs_and_f16(lattices):
    c = lattices[1]
    b = np.stack([gen.gaussian_spinor(c.dims, 900, k) for k in range(5)])
    x = torch.zeros_like(to_dev(b))
    infos = P.solve_batched([c.D], [x], [to_dev(b)], 5, method=P.MIXED_GCR, inner_prec="f16", tol=1e-10)
    for r in range(5):
        exact, _ = osolvers.solve_eo(c.f, b[r], 1e-13)
        assert rel(x[r].cpu().numpy(), exact) < 1e-8
    assert all(i.true_rel_res < 1e-10 for i in infos[0])


@pytest.mark.parametrize("shape", [41, 46])
def test_batched_column_walk_with_frozen_systems(monkeypatch, shape):
    """The batched mixed solve on a lattice where the column walk fits (8 x 8 x 16 x 32, 12 point
    sources at two sites, so the systems converge after different iterations and the active mask
    freezes some while the others go on), with its inner FP32 operator forced to a column-walk
    shape (single- or double-buffered), gives bitwise the solutions of the default shape, and the
    oracle's residual of one solution is below the tolerance."""
    need_gpu()
    c = Case((8, 8, 16, 32), kappa=0.124, seed=404)
    try:
        b = point_sources(c.dims)
        b[6:] = point_sources(c.dims, site=c.V // 2 + 37)[6:]
        sols = {}
        for sh in (None, shape):
            if sh is not None:
                monkeypatch.setenv("DIRAC_HOP_SHAPE", str(sh))
            x = torch.zeros_like(to_dev(b))
            infos = P.solve_batched([c.D], [x], [to_dev(b)], 12, method=P.MIXED_GCR, inner_prec="f32", tol=1e-10,
                                    restart=8)
            its = [i.iters for i in infos[0]]
            flush(f"[gpu] batched column walk shape {sh}: iterations {its}")
            sols[sh] = x.cpu().numpy()
        assert np.array_equal(sols[None], sols[shape])
        assert osolvers.rel_residual(c.f, sols[shape][9], b[9]) < 1e-10
    finally:
        c.D.close()
