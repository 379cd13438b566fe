"""MI355X library for the QCD+QED O(a)-improved Wilson-Dirac operator (arXiv:2502.02490).

A thin binding over the C ABI of include/dirac.h: PyTorch supplies device memory and the
current stream, every step of the operator and the solvers runs in the library's HIP
kernels.  There is no CPU fallback: without libdirac.so every call raises.
"""
from __future__ import annotations

import ctypes
import math

import torch

from . import _lib
from ._lib import (BF16, CGLS, EO, F16, F32, F64, GCR, LEX, MIXED_GCR, NATIVE, DiracError,  # noqa: F401
                   SolveInfo, SolverParams)

_TORCH_REAL = {F64: torch.float64, F32: torch.float32, F16: torch.float16, BF16: torch.bfloat16}
_TORCH_USER = {F64: torch.complex128, F32: torch.complex64, F16: torch.complex128, BF16: torch.complex128}
_PREC = {"f64": F64, "f32": F32, "f16": F16, "bf16": BF16}
_LAYOUT = {"lex": LEX, "eo": EO, "native": NATIVE}


def _prec(p):
    return _PREC[p] if isinstance(p, str) else int(p)


def _layout(l):
    return _LAYOUT[l] if isinstance(l, str) else int(l)


def _ptr(t: torch.Tensor):
    if not t.is_cuda:
        raise ValueError("tensors passed to the library must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensors passed to the library must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


class Dirac:
    """One operator D (and its even-odd Schur form) on a fixed gauge background.

    U:     complex128 [V, 4, 3, 3] SU(3) links on the GPU, LEX order (x0 = time slowest).
    theta: float64 [V, 4] U(1) angles, or None.
    """

    def __init__(self, U: torch.Tensor, theta, dims, kappa: float, csw: float, csw_qed: float, qhat: int,
                 bc_phase=(math.pi, 0.0, 0.0, 0.0), stream=None, allow_singular: bool = False):
        self.lib = _lib.load()
        self.dims = tuple(int(d) for d in dims)
        self.V = int(math.prod(self.dims))
        self.vh = self.V // 2
        p = _lib.Params()
        for m in range(4):
            p.dims[m] = self.dims[m]
            p.bc_phase[m] = float(bc_phase[m])
        p.kappa, p.csw, p.csw_qed, p.qhat = float(kappa), float(csw), float(csw_qed), int(qhat)
        self.params = p
        self._ctx = ctypes.c_void_p()
        st = self.lib.dirac_create(ctypes.byref(p), _ptr(U), _ptr(theta) if theta is not None else None,
                                   _stream(stream), ctypes.byref(self._ctx))
        self.singular = st == _lib.ESINGULAR
        if st != _lib.OK and not (self.singular and allow_singular and self._ctx.value):
            if self._ctx.value:
                self.lib.dirac_destroy(self._ctx)
                self._ctx = ctypes.c_void_p()
            _lib.check(st)

    # -------------------------------------------------------------- lifetime
    def close(self):
        if getattr(self, "_ctx", None) is not None and self._ctx.value:
            torch.cuda.synchronize()
            _lib.check(self.lib.dirac_destroy(self._ctx))
            self._ctx = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -------------------------------------------------------------- buffers
    def native_empty(self, prec="f64", sites: int = 0) -> torch.Tensor:
        """A NATIVE vector: sites = 0 full lattice, 1 one parity."""
        pr = _prec(prec)
        n = self.lib.dirac_native_bytes(self._ctx, pr, sites) // torch.empty(0, dtype=_TORCH_REAL[pr]).element_size()
        return torch.empty(int(n), dtype=_TORCH_REAL[pr], device="cuda")

    def to_native(self, user: torch.Tensor, prec="f64", layout="lex", sites: int = 0, out=None, stream=None):
        pr = _prec(prec)
        out = self.native_empty(pr, 0 if sites == 0 else 1) if out is None else out
        _lib.check(self.lib.dirac_import(self._ctx, _ptr(out), _ptr(user), sites, pr, _layout(layout), _stream(stream)))
        return out

    def from_native(self, native: torch.Tensor, prec="f64", layout="lex", sites: int = 0, out=None, stream=None):
        pr = _prec(prec)
        n = self.V if sites == 0 else self.vh
        out = torch.empty((n, 4, 3), dtype=_TORCH_USER[pr] if pr == F32 else torch.complex128,
                          device="cuda") if out is None else out
        _lib.check(self.lib.dirac_export(self._ctx, _ptr(out), _ptr(native), sites, pr, _layout(layout), _stream(stream)))
        return out

    # -------------------------------------------------------------- operators
    def apply(self, out, inp, prec="f64", layout="lex", dagger=False, stream=None):
        """out = D inp (full lattice)."""
        _lib.check(self.lib.dirac_apply(self._ctx, _ptr(out), _ptr(inp), _prec(prec), _layout(layout), int(dagger),
                                        _stream(stream)))
        return out

    def apply_eo(self, out, inp, prec="f64", layout="eo", dagger=False, stream=None):
        """out_e = D-hat inp_e (even-odd Schur operator on even half-vectors)."""
        _lib.check(self.lib.dirac_apply_eo(self._ctx, _ptr(out), _ptr(inp), _prec(prec), _layout(layout), int(dagger),
                                           _stream(stream)))
        return out

    def apply_hop(self, out, inp, out_parity: int, prec="f64", dagger=False, stream=None):
        """out_p = D_{p,1-p} inp = -1/2 H inp (NATIVE half-vectors)."""
        _lib.check(self.lib.dirac_apply_hop(self._ctx, _ptr(out), _ptr(inp), int(out_parity), _prec(prec),
                                            int(dagger), _stream(stream)))
        return out

    def apply_clover(self, out, inp, parity: int, inverse=False, prec="f64", stream=None):
        """out_p = A_pp inp or A_pp^-1 inp (NATIVE half-vectors)."""
        _lib.check(self.lib.dirac_apply_clover(self._ctx, _ptr(out), _ptr(inp), int(parity), int(inverse),
                                               _prec(prec), _stream(stream)))
        return out

    # -------------------------------------------------------------- clover field
    def clover(self, inverse=False, layout="lex", stream=None) -> torch.Tensor:
        """Packed clover field (or inverse) [V, 2, 36] float64 (Sec. 4.1.3 packing)."""
        out = torch.empty((self.V, 2, 36), dtype=torch.float64, device="cuda")
        _lib.check(self.lib.dirac_get_clover(self._ctx, _ptr(out), int(inverse), _layout(layout), _stream(stream)))
        return out

    def load_clover(self, packed: torch.Tensor, layout="lex", stream=None):
        _lib.check(self.lib.dirac_load_clover(self._ctx, _ptr(packed), _layout(layout), _stream(stream)))

    def clover_invert(self, parity_mask: int = 2, stream=None):
        _lib.check(self.lib.clover_invert(self._ctx, int(parity_mask), _stream(stream)))

    # -------------------------------------------------------------- solvers
    def solve(self, x, b, method=GCR, tol=1e-10, restart=32, max_iter=10000, layout="lex", precision="f64",
              inner_prec="f32", inner_tol=None, x0_given=False, stream=None, raise_on_noconv=True):
        sp = SolverParams()
        sp.method, sp.restart, sp.max_iter, sp.tol = int(method), int(restart), int(max_iter), float(tol)
        sp.inner_prec = _prec(inner_prec)
        sp.inner_tol = float(inner_tol) if inner_tol is not None else 0.0
        sp.x0_given, sp.precision = int(x0_given), _prec(precision)
        info = SolveInfo()
        st = self.lib.dirac_solve(self._ctx, _ptr(x), _ptr(b), _layout(layout), ctypes.byref(sp), ctypes.byref(info),
                                  _stream(stream))
        if st == _lib.ENOCONV and not raise_on_noconv:
            return info
        _lib.check(st)
        return info
