"""dirac_apply_eo_noalloc, the even-odd Schur apply that allocates nothing (its odd-site
intermediate sits in the library's static device buffer), called through the C ABI and held to
the existing dirac_apply_eo: the two run the same kernels, so the bar is bit-for-bit equality.
Two calls in a row, the second on a smaller lattice (the buffer keeps the first call's
contents), both precisions of the solvers, the dagger, the oracle's D-hat for the first call,
and a lattice whose F64 intermediate exceeds the buffer (refused) while its F16 one fits."""
from __future__ import annotations

import ctypes
import math

import numpy as np
import pytest
import torch

from gpu_util import Case, flush, need_gpu, rel, to_dev
from oracle import dirac as odirac

pytestmark = pytest.mark.gpu

PREC = {"f64": 0, "f32": 1, "f16": 2, "bf16": 3}


def noalloc(D, out, inp, prec, dagger=0):
    """One call of the entry point through ctypes, on torch's current stream; returns the status."""
    return D.lib.dirac_apply_eo_noalloc(D._ctx, ctypes.c_void_p(out.data_ptr()), ctypes.c_void_p(inp.data_ptr()),
                                        PREC[prec], int(dagger),
                                        ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))


def native_even(case, seed, prec):
    v = case.spinor(seed)[case.even]
    if prec == "f32":
        v = v.astype(np.complex64)
    return case.D.to_native(to_dev(v), prec, "eo", sites=1)


def test_noalloc_equals_apply_eo_twice_second_smaller():
    need_gpu()
    big, small = Case((8, 8, 4, 8), seed=211), Case((4, 4, 4, 4), seed=212)
    try:
        for prec in ("f64", "f32"):
            for dagger in (0, 1):
                for case in (big, small):  # the second call runs on the smaller lattice
                    flush(f"[gpu] noalloc Schur {case.dims} {prec} dagger={dagger}")
                    x = native_even(case, 300 + dagger, prec)
                    ref = torch.zeros_like(x)
                    case.D.apply_eo(ref, x, prec, "native", dagger=bool(dagger))
                    out = torch.zeros_like(x)
                    assert noalloc(case.D, out, x, prec, dagger) == 0, case.D.lib.dirac_last_error()
                    torch.cuda.synchronize()
                    assert torch.equal(out, ref), (case.dims, prec, dagger)
        # the first lattice's result against the oracle's D-hat (FP64 parity bar)
        psi_e = big.spinor(300)[big.even]
        x = big.D.to_native(to_dev(psi_e), "f64", "eo", sites=1)
        out = torch.zeros_like(x)
        assert noalloc(big.D, out, x, "f64") == 0
        got = big.D.from_native(out, "f64", "eo", sites=1).cpu().numpy().reshape(psi_e.shape)
        assert rel(got, odirac.apply_schur(big.f, psi_e)) <= 1e-13
    finally:
        big.D.close()
        small.D.close()


def test_noalloc_rejects_sizes_beyond_the_buffer():
    """32^3x32: the F64 intermediate (524,288 odd sites x 192 B) exceeds the 64 MiB buffer and is
    refused with DIRAC_EINVAL; the F16 one (48 B per site) fits and equals dirac_apply_eo."""
    need_gpu()
    import gen
    import paper_2502_02490_amd as P

    dims = (32, 32, 32, 32)
    U = torch.from_numpy(gen.su3_field(dims, 0.5, 213)).cuda()
    th = torch.from_numpy(gen.u1_field(dims, 0.3, 213)).cuda()
    with P.Dirac(U, th, dims, 0.1245, 1.6, 1.0, -1, (math.pi, 0.0, 0.0, 0.0)) as D:
        del U, th
        x = D.native_empty("f64", 1).normal_()
        out = torch.zeros_like(x)
        assert noalloc(D, out, x, "f64") == P._lib.EINVAL
        assert b"static buffer" in D.lib.dirac_last_error()
        # F16 fields do not exist before an apply in F16 builds them: refused, not built
        h = D.native_empty("f16", 1)
        h.copy_(torch.randn(h.shape, dtype=torch.float32, device="cuda").to(torch.float16))
        hout = torch.zeros_like(h)
        assert noalloc(D, hout, h, "f16") == P._lib.EINVAL
        ref = torch.zeros_like(h)
        D.apply_eo(ref, h, "f16", "native")
        flush("[gpu] noalloc Schur 32^4 f16")
        assert noalloc(D, hout, h, "f16") == 0, D.lib.dirac_last_error()
        torch.cuda.synchronize()
        assert torch.equal(hout, ref)
