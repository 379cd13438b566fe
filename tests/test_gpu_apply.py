"""GPU parity of the operator kernels against the FP64 oracle, through the C ABI.

Bars: FP64 apply relative error <= 1e-13, FP32 <= 1e-6, both in norm and element-wise (largest
deviation relative to the largest entry) on the same seeded inputs; 16-bit storage within its
rounding envelope.  Lattices span one tile (2^4), several tiles with a ragged tail (6x6x6x10:
V/2 = 1080 sites, 4 full work-groups of 256 and a partial one), mixed extents, and the
32^3 x 64 production shape on sampled output sites."""
import math

import numpy as np
import pytest
import torch

from gpu_util import N_HOP_SHAPES, Case, flush, need_gpu, rel, to_dev
from storage_envelope import U_BF16, U_FP16, schur_envelope
from oracle import dirac as odirac
from oracle import geometry as geo

pytestmark = pytest.mark.gpu

SHAPES = [(2, 2, 2, 2), (4, 4, 4, 4), (2, 4, 6, 8), (6, 6, 6, 10), (8, 4, 4, 12)]


@pytest.fixture(scope="module", params=SHAPES, ids=lambda d: "x".join(map(str, d)))
def case(request):
    need_gpu()
    flush(f"[gpu] case dims={request.param}")
    phase = (math.pi, 0.3, -0.8, 1.3) if request.param == (2, 4, 6, 8) else (math.pi, 0.0, 0.0, 0.0)
    qhat = 2 if request.param == (6, 6, 6, 10) else -1
    c = Case(request.param, qhat=qhat, bc_phase=phase, seed=301 + sum(request.param))
    yield c
    c.D.close()


def test_clover_field_matches_oracle(case):
    got = case.D.clover().cpu().numpy()
    exp = odirac.pack_clover(case.f.clover())
    assert np.abs(got - exp).max() <= 1e-13 * np.abs(exp).max()


def test_clover_inverse_matches_oracle(case):
    case.D.clover_invert(3)
    got = case.D.clover(inverse=True).cpu().numpy()
    exp = odirac.pack_clover(case.f.clover_inv())
    assert np.abs(got - exp).max() <= 1e-13 * np.abs(exp).max()


@pytest.mark.parametrize("dagger", [0, 1])
def test_full_apply_f64_lex(case, dagger):
    psi = case.spinor(11)
    out = torch.empty_like(to_dev(psi))
    case.D.apply(out, to_dev(psi), "f64", "lex", dagger=bool(dagger))
    exp = odirac.apply_Ddag(case.f, psi) if dagger else odirac.apply_D(case.f, psi)
    assert rel(out.cpu().numpy(), exp) <= 1e-13


@pytest.mark.parametrize("dagger", [0, 1])
def test_schur_apply_f64_eo(case, dagger):
    psi_e = case.spinor(12)[case.even]  # EO order = even sites by ascending Lambda
    out = torch.empty_like(to_dev(psi_e))
    case.D.apply_eo(out, to_dev(psi_e), "f64", "eo", dagger=bool(dagger))
    exp = odirac.apply_schur_dag(case.f, psi_e) if dagger else odirac.apply_schur(case.f, psi_e)
    assert rel(out.cpu().numpy(), exp) <= 1e-13


def test_hop_and_clover_native(case):
    D = case.D
    psi = case.spinor(13)
    nat = D.to_native(to_dev(psi), "f64", "lex")
    half = nat.numel() // 2
    ev, od = nat[:half], nat[half:]
    out = D.native_empty("f64", 1)
    # D_oe psi_e, exported as the odd half of an EO vector
    D.apply_hop(out, ev, 1, "f64")
    got = D.from_native(out, "f64", "eo", sites=2).cpu().numpy()
    assert rel(got, odirac.apply_Doe(case.f, psi[case.even])) <= 1e-13
    D.apply_hop(out, od, 0, "f64", dagger=True)
    got = D.from_native(out, "f64", "eo", sites=1).cpu().numpy()
    g5 = np.array([1, 1, -1, -1])[None, :, None]
    assert rel(got, g5 * odirac.apply_Deo(case.f, g5 * psi[case.odd])) <= 1e-13
    D.clover_invert(3)
    for par, sites in ((0, case.even), (1, case.odd)):
        src = ev if par == 0 else od
        for inv in (False, True):
            D.apply_clover(out, src, par, inverse=inv, prec="f64")
            got = D.from_native(out, "f64", "eo", sites=1 + par).cpu().numpy()
            assert rel(got, odirac.apply_clover(case.f, psi[sites], par, inverse=inv)) <= 1e-13


def test_layout_round_trip_is_exact(case):
    D = case.D
    psi = to_dev(case.spinor(14))
    for lay in ("lex", "eo"):
        back = D.from_native(D.to_native(psi, "f64", lay), "f64", lay)
        assert torch.equal(back, psi)
    # EO export of a LEX import reorders by eq. (ipt) with one block
    eo = D.from_native(D.to_native(psi, "f64", "lex"), "f64", "eo").cpu().numpy()
    perm = geo.lex_to_eo_perm(case.dims)
    assert np.array_equal(eo, psi.cpu().numpy()[perm])


def test_full_apply_f32(case):
    psi = case.spinor(15)
    inp = to_dev(psi.astype(np.complex64))
    out = torch.empty_like(inp)
    case.D.apply(out, inp, "f32", "lex")
    exp = odirac.apply_D(case.f, psi.astype(np.complex64).astype(np.complex128))
    assert rel(out.cpu().numpy(), exp) <= 1e-6


def test_schur_apply_f32_native(case):
    D = case.D
    psi_e = case.spinor(16)[case.even]
    nat = D.to_native(to_dev(psi_e.astype(np.complex64)), "f32", "eo", sites=1)
    out = D.native_empty("f32", 1)
    D.apply_eo(out, nat, "f32", "native")
    got = D.from_native(out, "f32", "eo", sites=1).cpu().numpy()
    exp = odirac.apply_schur(case.f, psi_e.astype(np.complex64).astype(np.complex128))
    assert rel(got, exp) <= 1e-6


@pytest.mark.parametrize("prec", ["f16", "bf16"])
def test_schur_apply_half_precision_storage(case, prec):
    """16-bit storage with FP32 arithmetic against the plain FP64 oracle, within the storage
    rounding envelope (tests/storage_envelope.py: unit roundoff 2^-11 for FP16, 2^-8 for BF16 at
    the spinor, the link rows and phase pair, both clover fields, the intermediate and the
    output), in norm and element-wise."""
    D = case.D
    psi_e = case.spinor(17)[case.even]
    nat = D.to_native(to_dev(psi_e), prec, "eo", sites=1)
    out = D.native_empty(prec, 1)
    D.apply_eo(out, nat, prec, "native")
    got = D.from_native(out, prec, "eo", sites=1).cpu().numpy()
    env = schur_envelope(case.f, psi_e, U_FP16 if prec == "f16" else U_BF16)
    flush(f"[gpu] {prec} Schur dims={case.dims} " + env.check(got, odirac.apply_schur(case.f, psi_e)))


def test_repeat_is_bitwise_identical(case):
    psi_e = to_dev(case.spinor(18)[case.even])
    a, b = torch.empty_like(psi_e), torch.empty_like(psi_e)
    case.D.apply_eo(a, psi_e)
    case.D.apply_eo(b, psi_e)
    assert torch.equal(a, b)


# ---------------------------------------------------------------- production shape, sampled
@pytest.mark.parametrize("qhat", [-1, 2])
def test_schur_32c64_sampled_sites(qhat):
    """32^3 x 64 (config shape of the plain-method solve): the whole Schur apply on the GPU,
    checked at 64 sampled even sites, each recomputed by the oracle from the definition."""
    need_gpu()
    flush(f"[gpu] 32^3x64 Schur sampled qhat={qhat}")
    c = Case((64, 32, 32, 32), qhat=qhat, seed=201)
    try:
        psi_e = c.spinor(21)[c.even]
        out = torch.empty_like(to_dev(psi_e))
        c.D.apply_eo(out, to_dev(psi_e), "f64", "eo")
        got = out.cpu().numpy()
        rng = np.random.default_rng(qhat + 5)
        pick = np.concatenate([[0, len(c.even) - 1], rng.choice(len(c.even), 62, replace=False)])
        exp = odirac.schur_at(c.f, psi_e, c.even[pick])
        assert rel(got[pick], exp) <= 1e-13
        # FP32 at the same sites
        nat = c.D.to_native(to_dev(psi_e.astype(np.complex64)), "f32", "eo", sites=1)
        o32 = c.D.native_empty("f32", 1)
        c.D.apply_eo(o32, nat, "f32", "native")
        g32 = c.D.from_native(o32, "f32", "eo", sites=1).cpu().numpy()
        exp32 = odirac.schur_at(c.f, psi_e.astype(np.complex64).astype(np.complex128), c.even[pick])
        assert rel(g32[pick], exp32) <= 1e-6
    finally:
        c.D.close()


# (8, 8, 16, 32): L0 % 8 == 0, (L1 L2 L3 / 2) % 64 == 0, (L2 L3 / 2) % 256 == 0, L1 % 8 == 0 and
# (L1 / 8) (L2 L3 / 2) % 256 == 0: the time tiles, the slab and the x1-split sweeps fit, so every
# shape runs its own kernel.  (4, 8, 12, 48): an XCD's part of a time slice is 288 sites, so the
# x1-split sweeps end each slice with a partial chunk (32 of 256 or 128 sites).
@pytest.mark.parametrize("dims", [(8, 8, 16, 32), (4, 8, 12, 48)], ids=lambda d: "x".join(map(str, d)))
def test_hop_launch_shapes_bitwise_identical(monkeypatch, dims):
    """Every launch shape the tuner may pick (work-group size, occupancy hint, work-group order,
    time-tiled LDS staging, persistent sweeps) gives bitwise the same Schur output, in every
    precision."""
    need_gpu()
    c = Case(dims, seed=55, qhat=2)
    try:
        psi_e = c.spinor(3)[c.even]
        for prec in ("f64", "f32", "f16", "bf16"):
            nat = c.D.to_native(to_dev(psi_e.astype(np.complex64) if prec == "f32" else psi_e), prec, "eo", sites=1)
            ref = None
            for shape in range(N_HOP_SHAPES):
                monkeypatch.setenv("DIRAC_HOP_SHAPE", str(shape))
                out = c.D.native_empty(prec, 1)
                c.D.apply_eo(out, nat, prec, "native")
                full = c.D.native_empty(prec, 0)
                c.D.apply(full, torch.cat([nat, nat]), prec, "native", dagger=True)
                if ref is None:
                    ref = (out.clone(), full.clone())
                else:
                    assert torch.equal(out, ref[0]) and torch.equal(full, ref[1]), (prec, shape)
        exp = odirac.apply_schur(c.f, psi_e)
        monkeypatch.setenv("DIRAC_HOP_SHAPE", "5")
        out = torch.empty_like(to_dev(psi_e))
        c.D.apply_eo(out, to_dev(psi_e), "f64", "eo")
        assert rel(out.cpu().numpy(), exp) <= 1e-13
    finally:
        c.D.close()


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16"])
def test_multi_rhs_schur_equals_single(case, prec, monkeypatch):
    """dirac_apply_eo_multi on 5 right-hand sides equals five single applies bit for bit, with
    the tuner's shape and with the shapes that take 2 or 4 right-hand sides per work-item (5 is
    a multiple of neither, so the last chunk is partial)."""
    D = case.D
    nr = 5
    vecs = [case.spinor(40 + r)[case.even] for r in range(nr)]
    nats = [D.to_native(to_dev(v.astype(np.complex64) if prec == "f32" else v), prec, "eo", sites=1) for v in vecs]
    inp = torch.cat(nats)
    n = nats[0].numel()
    singles = []
    for r in range(nr):
        one = torch.zeros_like(nats[r])  # padding sites of a NATIVE vector are never written
        D.apply_eo(one, nats[r], prec, "native")
        singles.append(one)
    one_dag = torch.zeros_like(nats[nr - 1])
    D.apply_eo(one_dag, nats[nr - 1], prec, "native", dagger=True)
    for shape in (None, 20, 21, 22, 23, 24, 25, 26, 27, 38, 39, 41, 42, 43, 44, 45, 46, 47):
        if shape is not None:
            monkeypatch.setenv("DIRAC_HOP_SHAPE", str(shape))
        out = torch.zeros_like(inp)
        D.apply_eo_multi(out, inp, nr, prec)
        for r in range(nr):
            assert torch.equal(out[r * n:(r + 1) * n], singles[r]), (shape, r)
        dag = torch.zeros_like(inp)
        D.apply_eo_multi(dag, inp, nr, prec, dagger=True)
        assert torch.equal(dag[(nr - 1) * n:], one_dag), shape


# shapes of the right-hand-side blocked column walk (k_hop_rbc in csrc/hop_kernels.h)
COLUMN_SHAPES = (41, 42, 43, 44, 45, 46, 47)


@pytest.mark.parametrize("dims", [(8, 8, 16, 32), (4, 8, 12, 48)], ids=lambda d: "x".join(map(str, d)))
def test_column_walk_equals_single_applies(monkeypatch, dims):
    """The column walk keeps each -t half-spinor in registers for two time slices instead of
    loading it again: with 12 and 7 right-hand sides (all waves busy, and some idle) its Schur
    output and that of its dagger equal single applies bit for bit in FP32, FP16 and BF16.
    (8, 8, 16, 32): 32 spatial blocks per slice (the x1-split order applies) in two chunks of four
    slices, so the kept half-spinors cross no chunk boundary; (4, 8, 12, 48): 36 blocks (plain
    order), one chunk of four slices."""
    need_gpu()
    c = Case(dims, seed=61, qhat=2)
    try:
        for prec in ("f32", "f16", "bf16"):
            for nr in (12, 7):
                flush(f"[gpu] column walk {dims} {prec} nrhs={nr}")
                vecs = [c.spinor(70 + r)[c.even] for r in range(nr)]
                nats = [c.D.to_native(to_dev(v.astype(np.complex64) if prec == "f32" else v), prec, "eo", sites=1)
                        for v in vecs]
                monkeypatch.setenv("DIRAC_HOP_SHAPE", "0")
                singles, sdag = [], []
                for r in range(nr):
                    one = torch.zeros_like(nats[r])
                    c.D.apply_eo(one, nats[r], prec, "native")
                    singles.append(one)
                    d = torch.zeros_like(nats[r])
                    c.D.apply_eo(d, nats[r], prec, "native", dagger=True)
                    sdag.append(d)
                inp = torch.cat(nats)
                n = nats[0].numel()
                for shape in COLUMN_SHAPES:
                    monkeypatch.setenv("DIRAC_HOP_SHAPE", str(shape))
                    out = torch.zeros_like(inp)
                    c.D.apply_eo_multi(out, inp, nr, prec)
                    dag = torch.zeros_like(inp)
                    c.D.apply_eo_multi(dag, inp, nr, prec, dagger=True)
                    for r in range(nr):
                        assert torch.equal(out[r * n:(r + 1) * n], singles[r]), (prec, nr, shape, r)
                        assert torch.equal(dag[r * n:(r + 1) * n], sdag[r]), (prec, nr, shape, r, "dagger")
    finally:
        c.D.close()


def test_multi_rhs_shapes_on_x1split_lattice(monkeypatch):
    """On a lattice where the x1-split block order fits (L1 % 8 == 0), every multi-right-hand-side
    shape, the x1-split ones included, equals single applies bit for bit, in FP64 and FP32."""
    need_gpu()
    c = Case((8, 8, 16, 32), seed=58, qhat=-1)
    try:
        nr = 3
        for prec in ("f64", "f32"):
            vecs = [c.spinor(60 + r)[c.even] for r in range(nr)]
            nats = [c.D.to_native(to_dev(v.astype(np.complex64) if prec == "f32" else v), prec, "eo", sites=1)
                    for v in vecs]
            singles = []
            monkeypatch.setenv("DIRAC_HOP_SHAPE", "0")
            for r in range(nr):
                one = torch.zeros_like(nats[r])
                c.D.apply_eo(one, nats[r], prec, "native")
                singles.append(one)
            inp = torch.cat(nats)
            n = nats[0].numel()
            for shape in range(N_HOP_SHAPES):
                monkeypatch.setenv("DIRAC_HOP_SHAPE", str(shape))
                out = torch.zeros_like(inp)
                c.D.apply_eo_multi(out, inp, nr, prec)
                for r in range(nr):
                    assert torch.equal(out[r * n:(r + 1) * n], singles[r]), (prec, shape, r)
    finally:
        c.D.close()
