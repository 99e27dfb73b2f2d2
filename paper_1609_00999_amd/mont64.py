"""Python binding of the 64-bit-residue entry points (include/mont64.h).

Argument marshalling only: every operation runs in libmont's HIP kernels.
Tensors are torch ROCm tensors of dtype uint64 or int64 (bit patterns).
"""
from __future__ import annotations

import ctypes

from . import mont

c_u64 = ctypes.c_uint64
c_vp = ctypes.c_void_p
c_size = ctypes.c_size_t


class Mont64Params(ctypes.Structure):
    """Mirror of ``mont64_params``: section 3.1 constants for R = 2^64."""
    _fields_ = [("P", c_u64), ("Pprime", c_u64), ("R1", c_u64), ("R2", c_u64), ("k", ctypes.c_uint32),
                ("reserved", ctypes.c_uint32)]

    def __repr__(self):
        return "Mont64Params(P=%d, Pprime=%d, R1=%d, R2=%d, k=%d)" % (self.P, self.Pprime, self.R1, self.R2, self.k)


_registered = False


def lib():
    global _registered
    L = mont.lib()
    if not _registered:
        pp = ctypes.POINTER(Mont64Params)
        L.mont64_setup.argtypes = [c_u64, pp]
        for name in ("mont64_to", "mont64_from"):
            getattr(L, name).argtypes = [pp, c_vp, c_vp, c_size, c_vp]
        for name in ("mont64_mul", "mont64_pow"):
            getattr(L, name).argtypes = [pp, c_vp, c_vp, c_vp, c_size, c_vp]
        L.mont64_muladd.argtypes = [pp, c_vp, c_vp, c_vp, c_vp, c_size, c_vp]
        _registered = True
    return L


def setup(P: int) -> Mont64Params:
    """Precomputation for odd 3 <= P < 2^63 with R = 2^64."""
    out = Mont64Params()
    mont.check(lib().mont64_setup(P, ctypes.byref(out)), "mont64_setup(%d)" % P)
    return out


def dev_ptr(t, name: str = "tensor") -> int:
    torch = mont._torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch.Tensor" % name)
    if not t.is_cuda:
        raise ValueError("%s must be a ROCm device tensor" % name)
    if t.dtype not in (torch.uint64, torch.int64):
        raise TypeError("%s must be uint64 or int64, got %s" % (name, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return t.data_ptr()


def _out(like, out):
    torch = mont._torch()
    if out is None:
        out = torch.empty(like.shape, dtype=like.dtype, device=like.device)
    if out.numel() != like.numel():
        raise ValueError("out has %d elements, input %d" % (out.numel(), like.numel()))
    return out


def _same(*xs):
    if len({x.numel() for x in xs}) != 1:
        raise ValueError("operand sizes differ")


def to_mont(prm: Mont64Params, x, out=None):
    """Residues x*2^64 mod P (any uint64 input)."""
    out = _out(x, out)
    mont.check(lib().mont64_to(ctypes.byref(prm), dev_ptr(x, "x"), dev_ptr(out, "out"), x.numel(),
                               mont.stream_handle()), "mont64_to")
    return out


def from_mont(prm: Mont64Params, x, out=None):
    """x*2^-64 mod P (any uint64 input)."""
    out = _out(x, out)
    mont.check(lib().mont64_from(ctypes.byref(prm), dev_ptr(x, "x"), dev_ptr(out, "out"), x.numel(),
                                 mont.stream_handle()), "mont64_from")
    return out


def mul(prm: Mont64Params, a, b, out=None):
    """REDC(a*b) elementwise; operands are residues in [0, P)."""
    _same(a, b)
    out = _out(a, out)
    mont.check(lib().mont64_mul(ctypes.byref(prm), dev_ptr(a, "a"), dev_ptr(b, "b"), dev_ptr(out, "out"),
                                a.numel(), mont.stream_handle()), "mont64_mul")
    return out


def muladd(prm: Mont64Params, a, b, c, out=None):
    """(REDC(a*b) + c) mod P elementwise; out may be c."""
    _same(a, b, c)
    out = _out(a, out)
    mont.check(lib().mont64_muladd(ctypes.byref(prm), dev_ptr(a, "a"), dev_ptr(b, "b"), dev_ptr(c, "c"),
                                   dev_ptr(out, "out"), a.numel(), mont.stream_handle()), "mont64_muladd")
    return out


def pow(prm: Mont64Params, base, exp, out=None):  # noqa: A001 - mirrors mont64_pow
    """Residue of a^e for residues ``base`` and ordinary uint64 exponents."""
    _same(base, exp)
    out = _out(base, out)
    mont.check(lib().mont64_pow(ctypes.byref(prm), dev_ptr(base, "base"), dev_ptr(exp, "exp"),
                                dev_ptr(out, "out"), base.numel(), mont.stream_handle()), "mont64_pow")
    return out
