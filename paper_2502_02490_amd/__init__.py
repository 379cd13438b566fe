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
from ._lib import (BF16, CGLS, EO, F16, F32, F64, FGCR_PTC, FGCR_PTC_EO, FGCR_SAP, GCR, LEX, MIXED_GCR,  # noqa: F401
                   NATIVE, OPENQXD, DiracError, SolveInfo, SolverParams)

_TORCH_REAL = {F64: torch.float64, F32: torch.float32, F16: torch.float16, BF16: torch.bfloat16}
_TORCH_USER = {F64: torch.complex128, F32: torch.complex64, F16: torch.complex128, BF16: torch.complex128}
_PREC = {"f64": F64, "f32": F32, "f16": F16, "bf16": BF16}
_LAYOUT = {"lex": LEX, "eo": EO, "native": NATIVE, "openqxd": OPENQXD}


def _prec(p):
    return _PREC[p] if isinstance(p, str) else int(p)


def _layout(l):
    return _LAYOUT[l] if isinstance(l, str) else int(l)


def _ptr(t: torch.Tensor, nbytes: int = 0):
    """Device address of a contiguous GPU tensor holding at least nbytes (the library can only
    check the size of the underlying allocation, not of a tensor carved out of it)."""
    if not t.is_cuda:
        raise ValueError("tensors passed to the library must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensors passed to the library must be contiguous")
    if t.numel() * t.element_size() < nbytes:
        raise ValueError(f"tensor of {t.numel() * t.element_size()} bytes where {nbytes} are needed")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream):
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


class Dirac:
    """One operator D (and its even-odd Schur form) on a fixed gauge background.

    U:     complex128 [V, 4, 3, 3] SU(3) links on the GPU, LEX order (x0 = time slowest).
    theta: float64 [V, 4] U(1) angles, or None.
    cstar: C* boundary conditions in directions 1 .. cstar (dims[1] the doubled extent).
    With openqxd_block = (B0, B1, B2, B3) the gauge field is given in openQxD's storage instead:
    U complex128 [V/2, 8, 3, 3] and theta float64 [V/2, 8] (or None), the 8 links attached to each
    odd point in eq. (ipt) order with that cache block (see dirac_create_openqxd).
    """

    def __init__(self, U: torch.Tensor, theta, dims, kappa: float, csw: float, csw_qed: float, qhat: int,
                 bc_phase=(math.pi, 0.0, 0.0, 0.0), stream=None, allow_singular: bool = False, openqxd_block=None,
                 cstar: int = 0):
        self.lib = _lib.load()
        self.dims = tuple(int(d) for d in dims)
        self.V = int(math.prod(self.dims))
        self.vh = self.V // 2
        p = _lib.Params()
        for m in range(4):
            p.dims[m] = self.dims[m]
            p.bc_phase[m] = float(bc_phase[m])
        p.kappa, p.csw, p.csw_qed, p.qhat = float(kappa), float(csw), float(csw_qed), int(qhat)
        p.cstar = int(cstar)
        self.params = p
        self._ctx = ctypes.c_void_p()
        if openqxd_block is None:
            st = self.lib.dirac_create(ctypes.byref(p), _ptr(U, self.V * 576),
                                       _ptr(theta, self.V * 32) if theta is not None else None,
                                       _stream(stream), ctypes.byref(self._ctx))
        else:
            blk = (ctypes.c_int * 4)(*[int(b) for b in openqxd_block])
            st = self.lib.dirac_create_openqxd(ctypes.byref(p), blk, _ptr(U, self.V * 576),
                                               _ptr(theta, self.V * 32) if theta is not None else None,
                                               _stream(stream), ctypes.byref(self._ctx))
        self.singular = st == _lib.ESINGULAR
        if st != _lib.OK and not (self.singular and allow_singular and self._ctx.value):
            if self._ctx.value:
                self.lib.dirac_destroy(self._ctx)
                self._ctx = ctypes.c_void_p()
            _lib.check(st)

    def set_cache_block(self, block):
        """Cache block B of the "openqxd" user layout (eq. (ipt)); default B = dims."""
        blk = (ctypes.c_int * 4)(*[int(b) for b in block])
        _lib.check(self.lib.dirac_set_cache_block(self._ctx, blk))

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
    def native_bytes(self, prec="f64", sites: int = 0) -> int:
        return int(self.lib.dirac_native_bytes(self._ctx, _prec(prec), sites))

    def user_bytes(self, prec="f64", sites: int = 0) -> int:
        n = self.V if sites == 0 else self.vh
        return n * 24 * (4 if _prec(prec) == F32 else 8)

    def _vec_bytes(self, prec, layout, sites):
        return self.native_bytes(prec, sites) if _layout(layout) == NATIVE else self.user_bytes(prec, sites)

    def native_empty(self, prec="f64", sites: int = 0) -> torch.Tensor:
        """A NATIVE vector: sites = 0 full lattice, 1 one parity."""
        pr = _prec(prec)
        n = self.lib.dirac_native_bytes(self._ctx, pr, sites) // torch.empty(0, dtype=_TORCH_REAL[pr]).element_size()
        return torch.empty(int(n), dtype=_TORCH_REAL[pr], device="cuda")

    def to_native(self, user: torch.Tensor, prec="f64", layout="lex", sites: int = 0, out=None, stream=None):
        pr = _prec(prec)
        out = self.native_empty(pr, 0 if sites == 0 else 1) if out is None else out
        _lib.check(self.lib.dirac_import(self._ctx, _ptr(out, self.native_bytes(pr, min(sites, 1))),
                                         _ptr(user, self.user_bytes(pr, sites)), sites, pr, _layout(layout),
                                         _stream(stream)))
        return out

    def from_native(self, native: torch.Tensor, prec="f64", layout="lex", sites: int = 0, out=None, stream=None):
        pr = _prec(prec)
        n = self.V if sites == 0 else self.vh
        out = torch.empty((n, 4, 3), dtype=_TORCH_USER[pr] if pr == F32 else torch.complex128,
                          device="cuda") if out is None else out
        _lib.check(self.lib.dirac_export(self._ctx, _ptr(out, self.user_bytes(pr, sites)),
                                         _ptr(native, self.native_bytes(pr, min(sites, 1))), sites, pr,
                                         _layout(layout), _stream(stream)))
        return out

    # -------------------------------------------------------------- operators
    def apply(self, out, inp, prec="f64", layout="lex", dagger=False, stream=None):
        """out = D inp (full lattice)."""
        nb = self._vec_bytes(prec, layout, 0)
        _lib.check(self.lib.dirac_apply(self._ctx, _ptr(out, nb), _ptr(inp, nb), _prec(prec), _layout(layout),
                                        int(dagger), _stream(stream)))
        return out

    def apply_eo(self, out, inp, prec="f64", layout="eo", dagger=False, stream=None):
        """out_e = D-hat inp_e (even-odd Schur operator on even half-vectors)."""
        nb = self._vec_bytes(prec, layout, 1)
        _lib.check(self.lib.dirac_apply_eo(self._ctx, _ptr(out, nb), _ptr(inp, nb), _prec(prec), _layout(layout),
                                           int(dagger), _stream(stream)))
        return out

    def apply_eo_multi(self, out, inp, nrhs: int, prec="f64", dagger=False, stream=None):
        """out[r] = D-hat inp[r] for nrhs NATIVE half vectors stored back to back."""
        nb = self.native_bytes(prec, 1) * int(nrhs)
        _lib.check(self.lib.dirac_apply_eo_multi(self._ctx, _ptr(out, nb), _ptr(inp, nb), int(nrhs), _prec(prec),
                                                 int(dagger), _stream(stream)))
        return out

    def apply_eo_noalloc(self, out, inp, prec="f64", dagger=False, stream=None):
        """out_e = D-hat inp_e on NATIVE half vectors without any device allocation (the odd
        intermediate sits in the library's static buffer; see dirac_apply_eo_noalloc)."""
        nb = self.native_bytes(prec, 1)
        _lib.check(self.lib.dirac_apply_eo_noalloc(self._ctx, _ptr(out, nb), _ptr(inp, nb), _prec(prec), int(dagger),
                                                   _stream(stream)))
        return out

    def apply_hop(self, out, inp, out_parity: int, prec="f64", dagger=False, stream=None):
        """out_p = D_{p,1-p} inp = -1/2 H inp (NATIVE half-vectors)."""
        nb = self.native_bytes(prec, 1)
        _lib.check(self.lib.dirac_apply_hop(self._ctx, _ptr(out, nb), _ptr(inp, nb), int(out_parity), _prec(prec),
                                            int(dagger), _stream(stream)))
        return out

    def apply_clover(self, out, inp, parity: int, inverse=False, prec="f64", stream=None):
        """out_p = A_pp inp or A_pp^-1 inp (NATIVE half-vectors)."""
        nb = self.native_bytes(prec, 1)
        _lib.check(self.lib.dirac_apply_clover(self._ctx, _ptr(out, nb), _ptr(inp, nb), int(parity), int(inverse),
                                               _prec(prec), _stream(stream)))
        return out

    # -------------------------------------------------------------- vector arithmetic (NATIVE)
    def residual(self, r, b, x, prec="f64", rel=False, stream=None):
        """r = b - D x on full NATIVE vectors; returns |r| / |b| when rel (blocking), else None."""
        pr = _prec(prec)
        nb = self.native_bytes(pr, 0)
        out = ctypes.c_double() if rel else None
        _lib.check(self.lib.dirac_residual(self._ctx, _ptr(r, nb), _ptr(b, nb), _ptr(x, nb), pr,
                                           ctypes.byref(out) if rel else None, _stream(stream)))
        return out.value if rel else None

    def lincomb(self, out, alpha, a, beta=0.0, b=None, out_prec="f64", in_prec="f64", sites=0, norm=False,
                stream=None):
        """out = alpha a + beta b on NATIVE vectors (in_prec in, out_prec out); returns |out|^2 when norm."""
        po, pi = _prec(out_prec), _prec(in_prec)
        nbo, nbi = self.native_bytes(po, sites), self.native_bytes(pi, sites)
        n2 = ctypes.c_double() if norm else None
        _lib.check(self.lib.dirac_lincomb(self._ctx, _ptr(out, nbo), po, float(alpha), _ptr(a, nbi), float(beta),
                                          _ptr(b, nbi) if b is not None else None, pi, int(sites),
                                          ctypes.byref(n2) if norm else None, _stream(stream)))
        return n2.value if norm else None

    def dot(self, a, b, prec="f64", sites=0, stream=None) -> complex:
        """<a, b> = sum conj(a) b over NATIVE vectors (FP64 sums, blocking)."""
        pr = _prec(prec)
        nb = self.native_bytes(pr, sites)
        d = (ctypes.c_double * 2)()
        _lib.check(self.lib.dirac_dot(self._ctx, _ptr(a, nb), _ptr(b, nb), pr, int(sites), d, _stream(stream)))
        return complex(d[0], d[1])

    # -------------------------------------------------------------- clover field
    def clover(self, inverse=False, layout="lex", stream=None) -> torch.Tensor:
        """Packed clover field (or inverse) [V, 2, 36] float64 (Sec. 4.1.3 packing)."""
        out = torch.empty((self.V, 2, 36), dtype=torch.float64, device="cuda")
        _lib.check(self.lib.dirac_get_clover(self._ctx, _ptr(out, self.V * 576), int(inverse), _layout(layout),
                                             _stream(stream)))
        return out

    def load_clover(self, packed: torch.Tensor, layout="lex", stream=None):
        _lib.check(self.lib.dirac_load_clover(self._ctx, _ptr(packed, self.V * 576), _layout(layout), _stream(stream)))

    def clover_invert(self, parity_mask: int = 2, stream=None):
        _lib.check(self.lib.clover_invert(self._ctx, int(parity_mask), _stream(stream)))

    def sap(self, out, inp, ncy=4, nmr=4, stream=None):
        """out = M_SAP inp (Schwarz preconditioner) on NATIVE F32 full vectors."""
        nb = self.native_bytes("f32", 0)
        _lib.check(self.lib.dirac_sap(self._ctx, _ptr(out, nb), _ptr(inp, nb), int(ncy), int(nmr), _stream(stream)))
        return out

    # -------------------------------------------------------------- solvers
    def solve(self, x, b, method=GCR, tol=1e-10, restart=32, max_iter=10000, layout="lex", precision="f64",
              inner_prec="f32", inner_tol=None, x0_given=False, ptc=None, stream=None, raise_on_noconv=True,
              sap_ncy=0, sap_nmr=0):
        """Solve D x = b (full-lattice FP64 vectors in `layout`); returns the SolveInfo."""
        sp = SolverParams()
        sp.method, sp.restart, sp.max_iter, sp.tol = int(method), int(restart), int(max_iter), float(tol)
        sp.inner_prec = _prec(inner_prec)
        sp.inner_tol = float(inner_tol) if inner_tol is not None else 0.0
        sp.x0_given, sp.precision = int(x0_given), _prec(precision)
        sp.ptc = ptc._net if ptc is not None else None
        sp.sap_ncy, sp.sap_nmr = int(sap_ncy), int(sap_nmr)
        info = SolveInfo()
        nb = self._vec_bytes("f64", layout, 0)
        st = self.lib.dirac_solve(self._ctx, _ptr(x, nb), _ptr(b, nb), _layout(layout), ctypes.byref(sp),
                                  ctypes.byref(info), _stream(stream))
        if st == _lib.ENOCONV and not raise_on_noconv:
            return info
        _lib.check(st)
        return info


def solve_batched(ops, xs, bs, nrhs, method=GCR, tol=1e-10, restart=32, max_iter=100000, layout="lex",
                  inner_prec="f32", inner_tol=None, stream=None):
    """Solve D_l x = b for nrhs right-hand sides on each lattice l (ops: Dirac objects).
    xs[l], bs[l]: tensors holding nrhs full-lattice FP64 vectors in `layout`.  Returns a list
    (per lattice) of lists (per right-hand side) of SolveInfo."""
    lib = _lib.load()
    n = len(ops)
    sp = SolverParams()
    sp.method, sp.restart, sp.max_iter, sp.tol = int(method), int(restart), int(max_iter), float(tol)
    sp.inner_prec = _prec(inner_prec)
    sp.inner_tol = float(inner_tol) if inner_tol is not None else 0.0
    sp.x0_given, sp.precision, sp.ptc = 0, F64, None
    ctx = (ctypes.c_void_p * n)(*[D._ctx.value for D in ops])
    xa = (ctypes.c_void_p * n)(*[_ptr(x, nrhs * D._vec_bytes("f64", layout, 0)).value for x, D in zip(xs, ops)])
    ba = (ctypes.c_void_p * n)(*[_ptr(b, nrhs * D._vec_bytes("f64", layout, 0)).value for b, D in zip(bs, ops)])
    infos = (SolveInfo * (n * nrhs))()
    _lib.check(lib.dirac_solve_batched(ctx, n, xa, ba, int(nrhs), _layout(layout), ctypes.byref(sp), infos,
                                       _stream(stream)))
    return [[infos[l * nrhs + r] for r in range(nrhs)] for l in range(n)]


class PTC:
    """Parallel-transport convolution network (the learned preconditioner), e.g. channels (1, 8, 8, 1).

    Weights: complex [9][c_out][c_in][4][4] per layer; get/set as numpy complex64 arrays."""

    def __init__(self, channels=(1, 8, 8, 1)):
        self.lib = _lib.load()
        self.channels = tuple(int(c) for c in channels)
        arr = (ctypes.c_int * len(self.channels))(*self.channels)
        self._net = ctypes.c_void_p()
        _lib.check(self.lib.ptc_create(arr, len(self.channels) - 1, ctypes.byref(self._net)))
        self.n = int(self.lib.ptc_num_weights(self._net))

    def shapes(self):
        return [(9, co, ci, 4, 4) for ci, co in zip(self.channels[:-1], self.channels[1:])]

    def _flat(self, layers):
        import numpy as np

        flat = np.concatenate([np.asarray(w, dtype=np.complex64).reshape(-1) for w in layers])
        if flat.size * 2 != self.n:
            raise ValueError("weight shapes do not match the network")
        return np.ascontiguousarray(flat.view(np.float32))

    def _unflat(self, flat):
        import numpy as np

        c = flat.view(np.complex64)
        out, o = [], 0
        for sh in self.shapes():
            k = int(np.prod(sh))
            out.append(c[o:o + k].reshape(sh).copy())
            o += k
        return out

    def set_weights(self, layers):
        flat = self._flat(layers)
        _lib.check(self.lib.ptc_set_weights(self._net, flat.ctypes.data_as(ctypes.c_void_p), flat.size))

    def get_weights(self):
        import numpy as np

        flat = np.empty(self.n, dtype=np.float32)
        _lib.check(self.lib.ptc_get_weights(self._net, flat.ctypes.data_as(ctypes.c_void_p), self.n))
        return self._unflat(flat)

    def get_grad(self):
        import numpy as np

        flat = np.empty(self.n, dtype=np.float32)
        _lib.check(self.lib.ptc_get_grad(self._net, flat.ctypes.data_as(ctypes.c_void_p), self.n))
        return self._unflat(flat)

    def zero_grad(self, stream=None):
        _lib.check(self.lib.ptc_zero_grad(self._net, _stream(stream)))

    def forward(self, D: Dirac, out, inp, stream=None):
        nb = D.native_bytes("f32", 0)
        _lib.check(self.lib.ptc_forward(D._ctx, self._net, _ptr(out, nb), _ptr(inp, nb), _stream(stream)))
        return out

    def forward_eo(self, D: Dirac, out_e, inp_e, stream=None):
        """out_e = [N((inp_e, 0))]_e on NATIVE F32 even halves (the Schur-system preconditioner)."""
        nb = D.native_bytes("f32", 1)
        _lib.check(self.lib.ptc_forward_eo(D._ctx, self._net, _ptr(out_e, nb), _ptr(inp_e, nb), _stream(stream)))
        return out_e

    def backward(self, D: Dirac, grad_in, inp, grad_out, stream=None):
        nb = D.native_bytes("f32", 0)
        _lib.check(self.lib.ptc_backward(D._ctx, self._net, _ptr(grad_in, nb) if grad_in is not None else None,
                                         _ptr(inp, nb), _ptr(grad_out, nb), _stream(stream)))

    def adam_step(self, lr, stream=None):
        _lib.check(self.lib.ptc_adam_step(self._net, float(lr), _stream(stream)))

    def get_adam_state(self):
        """(first moments, second moments, step): moments as float32 arrays in weight order."""
        import numpy as np

        m = np.empty(self.n, dtype=np.float32)
        v = np.empty(self.n, dtype=np.float32)
        step = ctypes.c_int()
        _lib.check(self.lib.ptc_get_adam_state(self._net, m.ctypes.data_as(ctypes.c_void_p),
                                               v.ctypes.data_as(ctypes.c_void_p), self.n, ctypes.byref(step)))
        return m, v, step.value

    def set_adam_state(self, m, v, step: int):
        import numpy as np

        m = np.ascontiguousarray(m, dtype=np.float32)
        v = np.ascontiguousarray(v, dtype=np.float32)
        if m.size != self.n or v.size != self.n:
            raise ValueError("moment sizes do not match the network")
        _lib.check(self.lib.ptc_set_adam_state(self._net, m.ctypes.data_as(ctypes.c_void_p),
                                               v.ctypes.data_as(ctypes.c_void_p), self.n, int(step)))

    def train_step(self, D: Dirac, rs, es, lr, stream=None) -> float:
        nb = D.native_bytes("f32", 0)
        n = len(rs)
        ra = (ctypes.c_void_p * n)(*[_ptr(r, nb).value for r in rs])
        ea = (ctypes.c_void_p * n)(*[_ptr(e, nb).value for e in es])
        loss = ctypes.c_double()
        _lib.check(self.lib.ptc_train_step(D._ctx, self._net, ra, ea, n, float(lr), ctypes.byref(loss),
                                           _stream(stream)))
        return loss.value

    def loss(self, D: Dirac, rs, es, stream=None) -> float:
        """Mean |N(r_i) - e_i|^2 / |e_i|^2 over the pairs, without an update (blocking)."""
        nb = D.native_bytes("f32", 0)
        n = len(rs)
        ra = (ctypes.c_void_p * n)(*[_ptr(r, nb).value for r in rs])
        ea = (ctypes.c_void_p * n)(*[_ptr(e, nb).value for e in es])
        out = ctypes.c_double()
        _lib.check(self.lib.ptc_loss(D._ctx, self._net, ra, ea, n, ctypes.byref(out), _stream(stream)))
        return out.value

    def close(self):
        if getattr(self, "_net", None) is not None and self._net.value:
            torch.cuda.synchronize()
            _lib.check(self.lib.ptc_destroy(self._net))
            self._net = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
