"""Python binding of libmont (argument marshalling only).

Every function takes ROCm device tensors (torch.uint32, or torch.int32 read
as uint32 bit patterns), checks shapes on the host and calls the C ABI on
torch's current HIP stream.  All arithmetic happens in libmont's HIP kernels;
there is no host fallback: if libmont.so is missing the call raises.
"""
from __future__ import annotations

import ctypes
import os

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libmont.so")

c_u32 = ctypes.c_uint32
c_size = ctypes.c_size_t
c_vp = ctypes.c_void_p


class MontParams(ctypes.Structure):
    """Mirror of ``mont_params`` (include/mont.h)."""
    _fields_ = [("P", c_u32), ("Pprime", c_u32), ("R1", c_u32), ("R2", c_u32), ("k", c_u32)]

    def __repr__(self):
        return "MontParams(P=%d, Pprime=%d, R1=%d, R2=%d, k=%d)" % (self.P, self.Pprime, self.R1, self.R2,
                                                                    self.k)


# mont_status values (include/mont.h)
OK, EINVAL, ERANGE, ENOROOT, ENOMEM, EHIP, ETIMEOUT = 0, -1, -2, -3, -4, -5, -6


class MontError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        super().__init__("%s: %s (status %d)" % (what or "libmont", strerror(status), status))


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded libmont.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libmont.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    pp = ctypes.POINTER(MontParams)
    L.mont_strerror.argtypes = [ctypes.c_int]
    L.mont_strerror.restype = ctypes.c_char_p
    L.mont_setup.argtypes = [c_u32, pp]
    for name in ("mont_to", "mont_from"):
        getattr(L, name).argtypes = [pp, c_vp, c_vp, c_size, c_vp]
    for name in ("mont_mul", "mont_pow"):
        getattr(L, name).argtypes = [pp, c_vp, c_vp, c_vp, c_size, c_vp]
    L.mont_muladd.argtypes = [pp, c_vp, c_vp, c_vp, c_vp, c_size, c_vp]
    for name in ("mont_mul_fourier", "mont_pow_fourier", "mont_modmul"):
        getattr(L, name).argtypes = [pp, c_vp, c_vp, c_vp, c_size, c_vp]
    for name in ("modmul_barrett", "modpow_barrett"):
        getattr(L, name).argtypes = [c_u32, c_vp, c_vp, c_vp, c_size, c_vp]
    L.mont_check_range.argtypes = [c_u32, c_vp, c_size, c_vp, c_vp]
    L.mont_batch_reserve.argtypes = [ctypes.c_int, ctypes.POINTER(c_vp)]
    L.mont_batch_update.argtypes = [c_vp, c_vp, ctypes.c_int, c_vp]
    L.mont_batch_mul.argtypes = [c_vp, c_vp]
    L.mont_batch_destroy.argtypes = [c_vp]
    L.mont_elem_tune_set.argtypes = [ctypes.c_int] * 4
    L.mont_elem_tune_get.argtypes = [ctypes.c_int] + [ctypes.POINTER(ctypes.c_int)] * 3
    _register_ntt(L)
    _lib = L
    _apply_tuning(L)
    return L


def _apply_tuning(L) -> None:
    """Apply the autotuner's cached launch shapes for this GPU (MONT_TUNE=0
    keeps the built-in defaults)."""
    if os.environ.get("MONT_TUNE", "1") == "0":
        return
    try:
        import torch
        if not torch.cuda.is_available():
            return
        from . import tune
        tune.applied = tune.apply(tune.load(), tune.device_arch(), L)
    except Exception as e:   # tuning is an optimisation: say so, keep the defaults
        import warnings
        warnings.warn("libmont tuning not applied (%s: %s); built-in launch shapes stay in force"
                      % (type(e).__name__, e), RuntimeWarning)


def _register_ntt(L):
    """Argument types of the transform entry points (filled in by ntt.py)."""
    from . import ntt as _ntt
    _ntt.register(L)


def strerror(status: int) -> str:
    try:
        return lib().mont_strerror(status).decode()
    except RuntimeError:
        return "status %d" % status


def check(status: int, what: str = "") -> None:
    if status != 0:
        raise MontError(status, what)


def setup(P: int) -> MontParams:
    """Section 3.1 precomputation for modulus P (R = 2^32)."""
    out = MontParams()
    check(lib().mont_setup(P, ctypes.byref(out)), "mont_setup(%d)" % P)
    return out


# --------------------------------------------------------------------------
# tensor helpers
# --------------------------------------------------------------------------

def _torch():
    import torch
    return torch


def stream_handle(stream=None) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return s.cuda_stream


def dev_ptr(t, name: str = "tensor") -> int:
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError("%s must be a torch.Tensor" % name)
    if not t.is_cuda:
        raise ValueError("%s must be a ROCm device tensor" % name)
    if t.dtype not in (torch.uint32, torch.int32):
        raise TypeError("%s must be uint32 or int32, got %s" % (name, t.dtype))
    if not t.is_contiguous():
        raise ValueError("%s must be contiguous" % name)
    return t.data_ptr()


def empty_like_u32(t):
    torch = _torch()
    return torch.empty(t.shape, dtype=t.dtype, device=t.device)


# --------------------------------------------------------------------------
# checked mode: operands must lie in [0, P) (Algorithm 2 needs a*b < R P);
# when on, every call first enqueues mont_check_range on its operands
# --------------------------------------------------------------------------

_checked_depth = 0
_status_words = {}


def _status_word(device):
    torch = _torch()
    key = device.index if device.index is not None else torch.cuda.current_device()
    w = _status_words.get(key)
    if w is None:
        w = _status_words[key] = torch.zeros(1, dtype=torch.int32, device=device)
    return w


def check_range(P: int, x, status=None):
    """Enqueue the device-side check that every element of x is below P.  An
    offending element sets the int32 device word ``status`` (default: this
    device's checked-mode word) to MONT_ERANGE; the word is never cleared here."""
    if status is None:
        status = _status_word(x.device)
    check(lib().mont_check_range(P, dev_ptr(x, "x"), x.numel(), dev_ptr(status, "status"), stream_handle()),
          "mont_check_range")
    return status


def _maybe_check(P, *xs):
    if _checked_depth:
        for x in xs:
            check_range(P, x)


def checked_status(device=None, reset: bool = True) -> int:
    """Synchronize and return the checked-mode status word of ``device``
    (0, or MONT_ERANGE if an operand was out of range since the last reset)."""
    torch = _torch()
    dev = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
    w = _status_word(dev)
    v = int(w.item())
    if reset:
        w.zero_()
    return v


class checked:
    """Checked mode for a block: ``with mont.checked(): ...``.  Every
    elementwise call inside verifies its residue operands on the device; on
    exit the block synchronizes and raises MontError(MONT_ERANGE) if any
    operand was outside [0, P).  Blocks nest."""

    def __enter__(self):
        global _checked_depth
        if _checked_depth == 0:
            for w in _status_words.values():
                w.zero_()
        _checked_depth += 1
        return self

    def __exit__(self, et, ev, tb):
        global _checked_depth
        _checked_depth -= 1
        if _checked_depth == 0 and et is None:
            for key in list(_status_words):
                st = checked_status("cuda:%d" % key)
                if st != 0:
                    raise MontError(st, "checked mode: operand outside [0, P)")
        return False


def _unary(fn, prm, x, out, name):
    if out is None:
        out = empty_like_u32(x)
    if out.numel() != x.numel():
        raise ValueError("out has %d elements, input %d" % (out.numel(), x.numel()))
    check(fn(ctypes.byref(prm), dev_ptr(x, "x"), dev_ptr(out, "out"), x.numel(), stream_handle()), name)
    return out


def to_mont(prm: MontParams, x, out=None):
    """Residues x*R mod P (any uint32 input)."""
    return _unary(lib().mont_to, prm, x, out, "mont_to")


def from_mont(prm: MontParams, x, out=None):
    """x*R^-1 mod P (any uint32 input)."""
    return _unary(lib().mont_from, prm, x, out, "mont_from")


def mul(prm: MontParams, a, b, out=None):
    """REDC(a*b) elementwise (Algorithm 2); operands are residues in [0, P)."""
    if a.numel() != b.numel():
        raise ValueError("operand sizes differ")
    if out is None:
        out = empty_like_u32(a)
    if out.numel() != a.numel():
        raise ValueError("out size differs")
    _maybe_check(prm.P, a, b)
    check(lib().mont_mul(ctypes.byref(prm), dev_ptr(a, "a"), dev_ptr(b, "b"), dev_ptr(out, "out"), a.numel(),
                         stream_handle()), "mont_mul")
    return out


def muladd(prm: MontParams, a, b, c, out=None):
    """(REDC(a*b) + c) mod P elementwise; out may be c (in place)."""
    if not (a.numel() == b.numel() == c.numel()):
        raise ValueError("operand sizes differ")
    if out is None:
        out = empty_like_u32(a)
    if out.numel() != a.numel():
        raise ValueError("out size differs")
    _maybe_check(prm.P, a, b, c)
    check(lib().mont_muladd(ctypes.byref(prm), dev_ptr(a, "a"), dev_ptr(b, "b"), dev_ptr(c, "c"),
                            dev_ptr(out, "out"), a.numel(), stream_handle()), "mont_muladd")
    return out


def pow(prm: MontParams, base, exp, out=None):  # noqa: A001 - mirrors mont_pow
    """Residue of a^e for residues ``base`` and ordinary uint32 exponents."""
    if base.numel() != exp.numel():
        raise ValueError("operand sizes differ")
    if out is None:
        out = empty_like_u32(base)
    if out.numel() != base.numel():
        raise ValueError("out size differs")
    _maybe_check(prm.P, base)
    check(lib().mont_pow(ctypes.byref(prm), dev_ptr(base, "base"), dev_ptr(exp, "exp"), dev_ptr(out, "out"),
                         base.numel(), stream_handle()), "mont_pow")
    return out


def _binary(fn, first, a, b, out, name, P, check_b):
    if a.numel() != b.numel():
        raise ValueError("operand sizes differ")
    _maybe_check(P, a, *((b,) if check_b else ()))
    if out is None:
        out = empty_like_u32(a)
    if out.numel() != a.numel():
        raise ValueError("out size differs")
    check(fn(first, dev_ptr(a, "a"), dev_ptr(b, "b"), dev_ptr(out, "out"), a.numel(), stream_handle()), name)
    return out


def modmul(prm: MontParams, a, b, out=None):
    """a*b mod P of ORDINARY uint32 values in one pass (mont_modmul); no
    conversion to residues needed, any uint32 operand accepted."""
    if a.numel() != b.numel():
        raise ValueError("operand sizes differ")
    if out is None:
        out = empty_like_u32(a)
    if out.numel() != a.numel():
        raise ValueError("out size differs")
    check(lib().mont_modmul(ctypes.byref(prm), dev_ptr(a, "a"), dev_ptr(b, "b"), dev_ptr(out, "out"), a.numel(),
                            stream_handle()), "mont_modmul")
    return out


def mul_fourier(prm: MontParams, a, b, out=None):
    """Algorithm 3 (Fourier-prime REDC) elementwise; same result as mul()."""
    return _binary(lib().mont_mul_fourier, ctypes.byref(prm), a, b, out, "mont_mul_fourier", prm.P, True)


def pow_fourier(prm: MontParams, base, exp, out=None):
    """pow() with Algorithm 3 in place of Algorithm 2; same result."""
    return _binary(lib().mont_pow_fourier, ctypes.byref(prm), base, exp, out, "mont_pow_fourier", prm.P, False)


def mul_barrett(P: int, a, b, out=None):
    """Algorithm 1 (Barrett) on ordinary residues: a*b mod P."""
    return _binary(lib().modmul_barrett, P, a, b, out, "modmul_barrett", P, True)


def pow_barrett(P: int, base, exp, out=None):
    """Ordinary a^e mod P with Algorithm 1 products."""
    return _binary(lib().modpow_barrett, P, base, exp, out, "modpow_barrett", P, False)


class VecDesc(ctypes.Structure):
    """Mirror of ``mont_vec_desc`` (include/mont.h)."""
    _fields_ = [("a", c_vp), ("b", c_vp), ("out", c_vp), ("n", ctypes.c_uint64), ("P", c_u32), ("Pprime", c_u32)]


class Batch:
    """Reusable batch of vectors, each with its own modulus (mont_batch)."""

    def __init__(self, max_vectors: int):
        h = c_vp()
        check(lib().mont_batch_reserve(max_vectors, ctypes.byref(h)), "mont_batch_reserve")
        self.handle = h
        self.cap = max_vectors
        self._keep = None

    def close(self):
        if self.handle:
            check(lib().mont_batch_destroy(self.handle), "mont_batch_destroy")
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def update(self, items):
        """items: list of (prm, a, b, out) with device tensors of equal length."""
        arr = (VecDesc * max(1, len(items)))()
        for i, (prm, a, b, out) in enumerate(items):
            if not (a.numel() == b.numel() == out.numel()):
                raise ValueError("vector %d: sizes differ" % i)
            arr[i] = VecDesc(dev_ptr(a, "a"), dev_ptr(b, "b"), dev_ptr(out, "out"), a.numel(), prm.P, prm.Pprime)
        self._keep = items
        check(lib().mont_batch_update(self.handle, arr, len(items), stream_handle()), "mont_batch_update")

    def update_raw(self, descs, stream=None):
        """descs: a ctypes array of VecDesc (pointers already resolved); uploaded
        on `stream` (the current stream if None)."""
        check(lib().mont_batch_update(self.handle, descs, len(descs), stream_handle(stream)), "mont_batch_update")

    def mul(self, stream=None):
        check(lib().mont_batch_mul(self.handle, stream_handle(stream)), "mont_batch_mul")


ELEM_OPS = {"to": 0, "from": 1, "mul": 2, "muladd": 3, "pow": 4, "modmul": 5}


def elem_tune_set(op: str, block: int, vpt: int, nontemporal: bool) -> None:
    check(lib().mont_elem_tune_set(ELEM_OPS[op], block, vpt, int(bool(nontemporal))), "mont_elem_tune_set")


def elem_tune_get(op: str):
    b, v, n = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
    check(lib().mont_elem_tune_get(ELEM_OPS[op], ctypes.byref(b), ctypes.byref(v), ctypes.byref(n)),
          "mont_elem_tune_get")
    return b.value, v.value, bool(n.value)
