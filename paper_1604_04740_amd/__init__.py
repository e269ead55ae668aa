"""Numerical entanglement on MI355X: Python binding of the C ABI (libne.so).

Argument marshalling only: every function here checks tensor placement,
dtype and shape, passes raw device pointers and the current HIP stream to
the function of the same name in include/ne.h, and raises NEError on a
non-zero return code.  All computation happens in the library's HIP
kernels; there is no other code path.  Importing works without a GPU (the
library's argument checks and parameter rules run on the host), but any call
that launches work needs a ROCm device.
"""
from __future__ import annotations

import ctypes
import math
import os

import torch

__all__ = [
    "NEError", "Params", "lib", "ne_version", "ne_strerror", "ne_params_default", "ne_range_bound",
    "ne_entangle", "ne_lsb_gemm", "ne_lsb_circconv", "ne_lsb_permute_scale",
    "ne_disentangle_check", "ne_recover", "ne_gemm_fused", "ne_plain_gemm_i8", "ne_abft_gemm_i8",
    "ne_abft_workspace", "ne_abft_rc_gemm_i8", "ne_abft_rc_check_i8", "ne_abft_rc_workspace",
    "ne_circconv_fused", "ne_circconv_workspace", "ne_linconv_workspace", "linconv_planes_default", "ne_permute_scale_fused", "ne_permute_workspace", "Inject", "Problem", "Batch", "ne_batch_plan",
    "ne_batch_run", "ne_batch_autotune", "NE_OP_GEMM", "NE_OP_CONV", "NE_OP_PERM",
]

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libne.so")

NE_I8, NE_I32, NE_I64 = 1, 4, 8
NE_OK, NE_EINVAL, NE_ERANGE, NE_EALIAS, NE_EALIGN, NE_EUNSUP, NE_ELAUNCH = 0, -1, -2, -3, -4, -5, -6
_DT = {torch.int8: NE_I8, torch.int32: NE_I32, torch.int64: NE_I64}


class NEError(RuntimeError):
    def __init__(self, code: int, where: str):
        super().__init__(f"{where}: {ne_strerror(code)} (code {code})")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [("M", ctypes.c_int32), ("w", ctypes.c_int32), ("l", ctypes.c_int32),
                ("k", ctypes.c_int32), ("r_check", ctypes.c_int32)]

    def __repr__(self):
        return f"Params(M={self.M}, w={self.w}, l={self.l}, k={self.k}, r_check={self.r_check})"


NE_OP_GEMM, NE_OP_CONV, NE_OP_PERM = 0, 1, 2


class _Problem(ctypes.Structure):
    _fields_ = [("op", ctypes.c_int32), ("M", ctypes.c_int32), ("r_check", ctypes.c_int32),
                ("out_dtype", ctypes.c_int32), ("n", ctypes.c_int64), ("K", ctypes.c_int64),
                ("N", ctypes.c_int64), ("c", ctypes.c_void_p), ("g", ctypes.c_void_p),
                ("perm", ctypes.c_void_p), ("scale", ctypes.c_void_p), ("add", ctypes.c_void_p),
                ("d_hat", ctypes.c_void_p), ("flags", ctypes.c_void_p), ("n_bad", ctypes.c_void_p)]


class _Tuning(ctypes.Structure):
    _fields_ = [("gemm_bn", (ctypes.c_int32 * 3) * 6), ("perm_chunk", (ctypes.c_int64 * 3) * 6)]


NE_SERIES_GEMM, NE_SERIES_CONV, NE_SERIES_SCALE_ADD, NE_SERIES_PERMUTE = 0, 1, 2, 3


class _SeriesOp(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("length", ctypes.c_int64), ("operand_max", ctypes.c_int64)]


class _Inject(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int64), ("position", ctypes.c_void_p),
                ("stream", ctypes.c_void_p), ("xor_mask", ctypes.c_void_p)]


_lib = None
_vp, _i32, _i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64


def lib():
    """The loaded libne.so (raises ImportError if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER(Params)
        sig = {
            "ne_strerror": ([ctypes.c_int], ctypes.c_char_p),
            "ne_version": ([], ctypes.c_int),
            "ne_params_default": ([_i32, _i32, P], ctypes.c_int),
            "ne_range_bound": ([P, ctypes.POINTER(_i64)], ctypes.c_int),
            "ne_entangle": ([_vp, _i32, _vp, _i64, P, _vp], ctypes.c_int),
            "ne_lsb_gemm": ([_vp, _i32, _vp, _vp, _i64, _i64, _i64, P, _vp], ctypes.c_int),
            "ne_lsb_circconv": ([_vp, _i32, _vp, _vp, _i64, P, _vp, _i64, _vp], ctypes.c_int),
            "ne_circconv_workspace": ([_i64, _i32, _i32], _i64),
            "ne_lsb_permute_scale": ([_vp, _vp, _vp, _vp, _vp, _i64, P, _vp], ctypes.c_int),
            "ne_disentangle_check": ([_vp, _vp, _vp, _vp, _i64, P, _vp], ctypes.c_int),
            "ne_recover": ([ctypes.POINTER(_vp), _i32, _vp, _vp, _i64, P, _vp], ctypes.c_int),
            "ne_gemm_fused": ([_vp, _vp, _vp, _i32, _vp, _vp, _i64, _i64, _i64, P,
                               ctypes.POINTER(_Inject), _vp], ctypes.c_int),
            "ne_plain_gemm_i8": ([_vp, _vp, _vp, _i64, _i64, _i64, _vp], ctypes.c_int),
            "ne_abft_workspace": ([_i64, _i64], _i64),
            "ne_abft_rc_workspace": ([_i32, _i64, _i64], _i64),
            "ne_abft_rc_gemm_i8": ([_vp, _vp, _vp, _vp, _vp, _vp, _i32, _i64, _i64, _i64, _vp, _i64,
                                    _vp], ctypes.c_int),
            "ne_abft_rc_check_i8": ([_vp, _vp, _vp, _vp, _vp, _vp, _i32, _i64, _i64, _i64, _vp, _i64,
                                     _vp], ctypes.c_int),
            "ne_abft_gemm_i8": ([_vp, _vp, _vp, _vp, _vp, _i32, _i64, _i64, _i64, _vp, _i64, _vp],
                                ctypes.c_int),
            "ne_circconv_fused": ([_vp, _i32, _i32, _vp, _vp, _i32, _vp, _vp, _i64, P, _vp,
                                   _i64, _vp], ctypes.c_int),
            "ne_permute_scale_fused": ([_vp, _i32, _vp, _vp, _vp, _vp, _i32, _vp, _vp, _i64, P,
                                        _vp, _i64, _vp], ctypes.c_int),
            "ne_permute_workspace": ([_i64, _i32, _i32], _i64),
            "ne_lsb_linconv": ([_vp, _i32, _vp, _i64, _vp, _i64, P, _vp, _i64, _vp], ctypes.c_int),
            "ne_linconv_workspace": ([_i64, _i64, _i32, _i32, _i32], _i64),
            "ne_linconv_fused": ([_vp, _i32, _i32, _vp, _i64, _vp, _i32, _vp, _vp, _i64, P, _vp,
                                  _i64, _vp],
                                 ctypes.c_int),
            "ne_series_range": ([P, _i64, _i32, ctypes.POINTER(_SeriesOp),
                                 ctypes.POINTER(_i32), ctypes.POINTER(_i64)], ctypes.c_int),
            "ne_series_gemm_scale_permute": ([_vp, _vp, _vp, _vp, _vp, _i64, _i64, _vp, _i32, _vp,
                                              _vp, _i64, _i64, _i64, P, _vp, _i64, _vp],
                                             ctypes.c_int),
            "ne_series_workspace": ([_i64, _i64, _i32], _i64),
            "ne_batch_plan": ([ctypes.POINTER(_Problem), _i32, ctypes.POINTER(_Tuning), _vp, _i64,
                               ctypes.POINTER(_i64), ctypes.POINTER(_vp)], ctypes.c_int),
            "ne_batch_run": ([_vp, _vp], ctypes.c_int),
            "ne_batch_items": ([_vp], ctypes.c_int),
            "ne_batch_free": ([_vp], None),
            "ne_batch_autotune": ([ctypes.POINTER(_Problem), _i32, _vp, _i64, _i32,
                                   ctypes.POINTER(_Tuning), _vp], ctypes.c_int),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def ne_strerror(code: int) -> str:
    return lib().ne_strerror(code).decode()


def ne_version() -> int:
    return lib().ne_version()


def _ok(code: int, where: str):
    if code != 0:
        raise NEError(code, where)


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev(t: torch.Tensor, name: str, dtype=None):
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.device.type != "cuda":
        raise ValueError(f"{name} must be on a ROCm device")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _opt(t, name, dtype):
    return _dev(t, name, dtype) if t is not None else None


def _word(p: Params):
    """torch dtype of the words (eps, delta, d_hat, scale, add) for p.w."""
    return torch.int32 if p.w == 32 else torch.int64


# --------------------------------------------------------------- parameters

def ne_params_default(M: int, w: int = 64) -> Params:
    p = Params()
    _ok(lib().ne_params_default(M, w, ctypes.byref(p)), "ne_params_default")
    return p


def ne_range_bound(p: Params) -> int:
    D = _i64()
    _ok(lib().ne_range_bound(ctypes.byref(p), ctypes.byref(D)), "ne_range_bound")
    return D.value


# --------------------------------------------------------------- staged path

def ne_entangle(c: torch.Tensor, p: Params, out: torch.Tensor | None = None) -> torch.Tensor:
    """c: [M, ...] int8/int32/int64 -> eps [M, ...] words (int64; int32 for
    p.w == 32; out may be c when c has the word type)."""
    if c.dtype not in _DT:
        raise TypeError("c must be int8, int32 or int64")
    M = c.shape[0]
    if M != p.M:
        raise ValueError("leading dimension must be M")
    if out is None:
        out = torch.empty(c.shape, dtype=_word(p), device=c.device)
    if out.shape != c.shape:
        raise ValueError("out must have the shape of c")
    N = c.numel() // M if M else 0
    _ok(lib().ne_entangle(_dev(c, "c"), _DT[c.dtype], _dev(out, "out", _word(p)), N,
                          ctypes.byref(p), _stream()), "ne_entangle")
    return out


def ne_lsb_gemm(eps: torch.Tensor, eps_bits: int, Gt: torch.Tensor, p: Params,
                out: torch.Tensor | None = None) -> torch.Tensor:
    """eps: [M, n, K] int64, Gt: [N, K] int8 -> delta [M, n, N] int64."""
    M, n, K = eps.shape
    N, K2 = Gt.shape
    if K2 != K or M != p.M:
        raise ValueError("shape mismatch")
    if out is None:
        out = torch.empty((M, n, N), dtype=torch.int64, device=eps.device)
    _ok(lib().ne_lsb_gemm(_dev(eps, "eps", torch.int64), eps_bits, _dev(Gt, "Gt", torch.int8),
                          _dev(out, "out", torch.int64), n, K, N, ctypes.byref(p), _stream()),
        "ne_lsb_gemm")
    return out


def ne_permute_workspace(N: int, M: int, c_dtype: torch.dtype) -> int:
    return int(lib().ne_permute_workspace(N, M, _DT[c_dtype]))


def ne_circconv_workspace(N: int, M: int, fused: bool) -> int:
    return int(lib().ne_circconv_workspace(N, M, 1 if fused else 0))


def _conv_ws(workspace, N, M, fused, device):
    """workspace=True: allocate what the library asks for; None/False: none."""
    if workspace is True:
        need = ne_circconv_workspace(N, M, fused)
        return torch.empty((max(need, 8) // 8,), dtype=torch.int64, device=device) if need else None
    if workspace is None or workspace is False:
        return None
    return workspace


def ne_lsb_circconv(eps: torch.Tensor, eps_bits: int, g: torch.Tensor, p: Params,
                    out: torch.Tensor | None = None, workspace=True) -> torch.Tensor:
    """eps: [M, N] int64, g: [N] int8 -> delta [M, N] int64."""
    M, N = eps.shape
    if g.shape != (N,) or M != p.M:
        raise ValueError("shape mismatch")
    if out is None:
        out = torch.empty_like(eps)
    ws = _conv_ws(workspace, N, M, False, eps.device)
    _ok(lib().ne_lsb_circconv(_dev(eps, "eps", torch.int64), eps_bits, _dev(g, "g", torch.int8),
                              _dev(out, "out", torch.int64), N, ctypes.byref(p), _opt(ws, "ws", None),
                              ws.numel() * ws.element_size() if ws is not None else 0, _stream()),
        "ne_lsb_circconv")
    return out


def ne_linconv_workspace(N: int, L: int, M: int, bits: int, fused: bool) -> int:
    return int(lib().ne_linconv_workspace(N, L, M, bits, 1 if fused else 0))


def linconv_planes_default(M: int, L: int) -> bool:
    """Whether workspace=None stages a linear convolution from digit planes:
    for kernels longer than four 256-tap steps (the blocks slide over the
    taps) and six or more streams, where the per-step staging of the direct
    path costs more than the pre-pass."""
    return M >= 6 and L + 32 > 1024


def _linconv_ws(workspace, N, L, M, bits, fused, device):
    """workspace=True: allocate the digit planes the library asks for;
    None: the same where linconv_planes_default says so; False: none."""
    if workspace is None:
        workspace = linconv_planes_default(M, L)
    if workspace is True:
        need = ne_linconv_workspace(N, L, M, bits, fused)
        if need <= 0:
            raise ValueError("invalid linear convolution sizes")
        return torch.empty(((need + 15) // 16 * 2,), dtype=torch.int64, device=device)
    if workspace is False:
        return None
    return workspace


def _ws_args(ws):
    return _opt(ws, "ws", None), ws.numel() * ws.element_size() if ws is not None else 0


def ne_lsb_linconv(eps: torch.Tensor, eps_bits: int, g: torch.Tensor, p: Params,
                   out: torch.Tensor | None = None, workspace=None) -> torch.Tensor:
    """eps: [M, N] int64, g: [L] int8 -> delta [M, N + L - 1] int64 (linear convolution).
    workspace=True stages from digit planes written by a pre-pass (a tensor:
    that buffer), False from eps directly, None as linconv_planes_default."""
    M, N = eps.shape
    (L,) = g.shape
    if M != p.M:
        raise ValueError("shape mismatch")
    if out is None:
        out = torch.empty((M, N + L - 1), dtype=torch.int64, device=eps.device)
    ws = _linconv_ws(workspace, N, L, M, eps_bits, False, eps.device)
    _ok(lib().ne_lsb_linconv(_dev(eps, "eps", torch.int64), eps_bits, _dev(g, "g", torch.int8), L,
                             _dev(out, "out", torch.int64), N, ctypes.byref(p), *_ws_args(ws),
                             _stream()), "ne_lsb_linconv")
    return out


def ne_lsb_permute_scale(eps: torch.Tensor, perm: torch.Tensor, scale: torch.Tensor | None,
                         add: torch.Tensor | None, p: Params,
                         out: torch.Tensor | None = None) -> torch.Tensor:
    """eps: [M, N] words; perm [N] int32; scale/add [N] words or None (words:
    int64, or int32 for p.w == 32)."""
    M, N = eps.shape
    if M != p.M or perm.shape != (N,):
        raise ValueError("shape mismatch")
    if out is None:
        out = torch.empty_like(eps)
    W = _word(p)
    _ok(lib().ne_lsb_permute_scale(_dev(eps, "eps", W), _dev(perm, "perm", torch.int32),
                                   _opt(scale, "scale", W), _opt(add, "add", W),
                                   _dev(out, "out", W), N, ctypes.byref(p), _stream()),
        "ne_lsb_permute_scale")
    return out


def ne_disentangle_check(delta: torch.Tensor, p: Params, out: torch.Tensor | None = None,
                         flags: bool | torch.Tensor = True, n_bad: torch.Tensor | None = None):
    """delta: [M, ...] words -> (d_hat [M, ...] words, flags uint32 words or
    None, n_bad); words are int64, or int32 for p.w == 32."""
    M = delta.shape[0]
    if M != p.M:
        raise ValueError("leading dimension must be M")
    N = delta.numel() // M
    if out is None:
        out = torch.empty_like(delta)
    if flags is True:
        flags = torch.empty(((N + 31) // 32,), dtype=torch.int32, device=delta.device)
    elif flags is False:
        flags = None
    if n_bad is None:
        n_bad = torch.zeros((1,), dtype=torch.int64, device=delta.device)
    _ok(lib().ne_disentangle_check(_dev(delta, "delta", _word(p)), _dev(out, "out", _word(p)),
                                   _opt(flags, "flags", torch.int32), _dev(n_bad, "n_bad", torch.int64),
                                   N, ctypes.byref(p), _stream()), "ne_disentangle_check")
    return out, flags, n_bad


def ne_recover(deltas, lost: int, p: Params, rebuild: bool = False, out: torch.Tensor | None = None):
    """deltas: list of M tensors [N] of words (int64; int32 for p.w == 32;
    deltas[lost] may be None).  Returns (d_hat [M, N], rebuilt [N] or None)."""
    M = p.M
    if len(deltas) != M:
        raise ValueError("need M stream pointers")
    ref = next(d for i, d in enumerate(deltas) if i != lost)
    N = ref.numel()
    ptrs = (_vp * M)()
    for i, d in enumerate(deltas):
        if i == lost:
            ptrs[i] = None
            continue
        if d.numel() != N:
            raise ValueError("every stream must have N words")
        ptrs[i] = _dev(d, f"deltas[{i}]", _word(p)).value
    if out is None:
        out = torch.empty((M,) + tuple(ref.shape), dtype=_word(p), device=ref.device)
    rb = torch.empty_like(ref) if rebuild else None
    _ok(lib().ne_recover(ptrs, lost, _dev(out, "out", _word(p)), _opt(rb, "rebuilt", _word(p)),
                         N, ctypes.byref(p), _stream()), "ne_recover")
    return out, rb


# --------------------------------------------------------------- fused path

class Inject:
    """Device-side fault list for ne_gemm_fused: XOR xor_mask into the entangled
    output word of `stream` at flat position `position` (row * N + col)."""

    def __init__(self, position: torch.Tensor, stream: torch.Tensor, xor_mask: torch.Tensor):
        order = torch.argsort(position)
        self.position = position[order].to(torch.int64).contiguous()
        self.stream = stream[order].to(torch.int32).contiguous()
        self.xor_mask = xor_mask[order].to(torch.int64).contiguous()

    def struct(self):
        s = _Inject()
        s.count = self.position.numel()
        s.position = _dev(self.position, "position", torch.int64)
        s.stream = _dev(self.stream, "stream", torch.int32)
        s.xor_mask = _dev(self.xor_mask, "xor_mask", torch.int64)
        return s


def ne_gemm_fused(c: torch.Tensor, Gt: torch.Tensor, p: Params, out_dtype=torch.int32,
                  out: torch.Tensor | None = None, flags: bool | torch.Tensor = True,
                  n_bad: torch.Tensor | None = None, inject: Inject | None = None):
    """c: [M, n, K] int8, Gt: [N, K] int8 -> (d_hat [M, n, N], flags [n, ceil(N/32)], n_bad)."""
    M, n, K = c.shape
    N, K2 = Gt.shape
    if K2 != K or M != p.M:
        raise ValueError("shape mismatch")
    if out is None:
        out = torch.empty((M, n, N), dtype=out_dtype, device=c.device)
    if flags is True:
        flags = torch.empty((n, (N + 31) // 32), dtype=torch.int32, device=c.device)
    elif flags is False:
        flags = None
    if n_bad is None:
        n_bad = torch.zeros((1,), dtype=torch.int64, device=c.device)
    inj = ctypes.byref(inject.struct()) if inject is not None else None
    _ok(lib().ne_gemm_fused(_dev(c, "c", torch.int8), _dev(Gt, "Gt", torch.int8),
                            _dev(out, "out", out_dtype), _DT[out_dtype],
                            _opt(flags, "flags", torch.int32), _dev(n_bad, "n_bad", torch.int64),
                            n, K, N, ctypes.byref(p), inj, _stream()), "ne_gemm_fused")
    return out, flags, n_bad


def ne_plain_gemm_i8(A: torch.Tensor, Bt: torch.Tensor, out: torch.Tensor | None = None):
    """A: [R, K] int8 (or [M, n, K]), Bt: [N, K] int8 -> C int32 [R, N] (or [M, n, N])."""
    K = A.shape[-1]
    R = math.prod(A.shape[:-1])
    N, K2 = Bt.shape
    if K2 != K:
        raise ValueError("shape mismatch")
    if out is None:
        out = torch.empty(tuple(A.shape[:-1]) + (N,), dtype=torch.int32, device=A.device)
    _ok(lib().ne_plain_gemm_i8(_dev(A, "A", torch.int8), _dev(Bt, "Bt", torch.int8),
                               _dev(out, "out", torch.int32), R, K, N, _stream()), "ne_plain_gemm_i8")
    return out


def ne_abft_workspace(n: int, K: int) -> int:
    return int(lib().ne_abft_workspace(n, K))


def ne_abft_rc_workspace(M: int, K: int, N: int) -> int:
    return int(lib().ne_abft_rc_workspace(M, K, N))


def _abft_rc(c, Gt, d, gemm, row_flags, col_flags, n_bad, workspace):
    M, n, K = c.shape
    N, K2 = Gt.shape
    if K2 != K:
        raise ValueError("shape mismatch")
    if d is None:
        d = torch.empty((M, n, N), dtype=torch.int32, device=c.device)
    elif tuple(d.shape) != (M, n, N):
        raise ValueError("shape mismatch")
    if row_flags is True:
        row_flags = torch.empty((M, (n + 31) // 32), dtype=torch.int32, device=c.device)
    elif row_flags is False:
        row_flags = None
    if col_flags is True:
        col_flags = torch.empty((M, (N + 31) // 32), dtype=torch.int32, device=c.device)
    elif col_flags is False:
        col_flags = None
    if n_bad is None:
        n_bad = torch.zeros((1,), dtype=torch.int64, device=c.device)
    if workspace is None:
        need = ne_abft_rc_workspace(M, K, N)
        if need <= 0:
            raise ValueError("invalid sizes")
        workspace = torch.empty((need // 8 + 2,), dtype=torch.int64, device=c.device)
    fn = lib().ne_abft_rc_gemm_i8 if gemm else lib().ne_abft_rc_check_i8
    _ok(fn(_dev(c, "c", torch.int8), _dev(Gt, "Gt", torch.int8), _dev(d, "d", torch.int32),
           _opt(row_flags, "row_flags", torch.int32), _opt(col_flags, "col_flags", torch.int32),
           _dev(n_bad, "n_bad", torch.int64), M, n, K, N, *_ws_args(workspace), _stream()),
        "ne_abft_rc_gemm_i8" if gemm else "ne_abft_rc_check_i8")
    return d, row_flags, col_flags, n_bad


def ne_abft_rc_gemm_i8(c: torch.Tensor, Gt: torch.Tensor, out: torch.Tensor | None = None,
                       row_flags: bool | torch.Tensor = True, col_flags: bool | torch.Tensor = True,
                       n_bad: torch.Tensor | None = None, workspace: torch.Tensor | None = None):
    """Row/column checksum ABFT: c [M, n, K] int8, Gt [N, K] int8 -> (d [M, n, N]
    int32, row_flags [M, ceil(n/32)], col_flags [M, ceil(N/32)], n_bad).
    workspace: a tensor of ne_abft_rc_workspace(M, K, N) bytes, or None to
    allocate one."""
    return _abft_rc(c, Gt, out, True, row_flags, col_flags, n_bad, workspace)


def ne_abft_rc_check_i8(c: torch.Tensor, Gt: torch.Tensor, d: torch.Tensor,
                        row_flags: bool | torch.Tensor = True, col_flags: bool | torch.Tensor = True,
                        n_bad: torch.Tensor | None = None, workspace: torch.Tensor | None = None):
    """The check of ne_abft_rc_gemm_i8 on a given product d [M, n, N] int32."""
    return _abft_rc(c, Gt, d, False, row_flags, col_flags, n_bad, workspace)[1:]


def ne_abft_gemm_i8(c: torch.Tensor, Gt: torch.Tensor, out: torch.Tensor | None = None,
                    flags: bool | torch.Tensor = True, n_bad: torch.Tensor | None = None,
                    workspace=True):
    """c: [M, n, K] int8, Gt: [N, K] int8 -> (d [M, n, N] int32, flags, n_bad).
    workspace=True allocates the checksum planes (DMA pipeline); None: the
    single-launch form; or a caller tensor of ne_abft_workspace(n, K) bytes."""
    M, n, K = c.shape
    N, K2 = Gt.shape
    if K2 != K:
        raise ValueError("shape mismatch")
    if out is None:
        out = torch.empty((M, n, N), dtype=torch.int32, device=c.device)
    if flags is True:
        flags = torch.empty((n, (N + 31) // 32), dtype=torch.int32, device=c.device)
    elif flags is False:
        flags = None
    if n_bad is None:
        n_bad = torch.zeros((1,), dtype=torch.int64, device=c.device)
    if workspace is True:
        need = int(lib().ne_abft_workspace(n, K))
        workspace = torch.empty((max(need, 16) // 8 + 2,), dtype=torch.int64, device=c.device)
    ws = workspace if workspace is not None and workspace is not False else None
    _ok(lib().ne_abft_gemm_i8(_dev(c, "c", torch.int8), _dev(Gt, "Gt", torch.int8),
                              _dev(out, "out", torch.int32), _opt(flags, "flags", torch.int32),
                              _dev(n_bad, "n_bad", torch.int64), M, n, K, N,
                              _opt(ws, "workspace", None),
                              ws.numel() * ws.element_size() if ws is not None else 0, _stream()),
        "ne_abft_gemm_i8")
    return out, flags, n_bad



# ----------------------------------------------------------- fused conv/perm

def ne_circconv_fused(c: torch.Tensor, g: torch.Tensor, p: Params, c_bits: int,
                      out_dtype=torch.int64, out: torch.Tensor | None = None,
                      flags: bool | torch.Tensor = True, n_bad: torch.Tensor | None = None,
                      workspace=True):
    """c: [M, N] int8/int32/int64, g: [N] int8 -> (d_hat [M, N], flags [ceil(N/32)], n_bad)."""
    M, N = c.shape
    if M != p.M or g.shape != (N,):
        raise ValueError("shape mismatch")
    if c.dtype not in _DT:
        raise TypeError("c must be int8, int32 or int64")
    if out is None:
        out = torch.empty((M, N), dtype=out_dtype, device=c.device)
    if flags is True:
        flags = torch.empty(((N + 31) // 32,), dtype=torch.int32, device=c.device)
    elif flags is False:
        flags = None
    if n_bad is None:
        n_bad = torch.zeros((1,), dtype=torch.int64, device=c.device)
    ws = _conv_ws(workspace, N, M, True, c.device)
    _ok(lib().ne_circconv_fused(_dev(c, "c"), _DT[c.dtype], c_bits, _dev(g, "g", torch.int8),
                                _dev(out, "out", out_dtype), _DT[out_dtype],
                                _opt(flags, "flags", torch.int32), _dev(n_bad, "n_bad", torch.int64),
                                N, ctypes.byref(p), _opt(ws, "ws", None),
                                ws.numel() * ws.element_size() if ws is not None else 0, _stream()),
        "ne_circconv_fused")
    return out, flags, n_bad


def ne_linconv_fused(c: torch.Tensor, g: torch.Tensor, p: Params, c_bits: int,
                     out_dtype=torch.int64, out: torch.Tensor | None = None,
                     flags: bool | torch.Tensor = True, n_bad: torch.Tensor | None = None,
                     workspace=None):
    """c: [M, N] int8/int32/int64, g: [L] int8 -> (d_hat [M, N + L - 1],
    flags [ceil((N + L - 1) / 32)], n_bad).  workspace as for ne_lsb_linconv."""
    M, N = c.shape
    (L,) = g.shape
    if M != p.M:
        raise ValueError("shape mismatch")
    if c.dtype not in _DT:
        raise TypeError("c must be int8, int32 or int64")
    No = N + L - 1
    if out is None:
        out = torch.empty((M, No), dtype=out_dtype, device=c.device)
    if flags is True:
        flags = torch.empty(((No + 31) // 32,), dtype=torch.int32, device=c.device)
    elif flags is False:
        flags = None
    if n_bad is None:
        n_bad = torch.zeros((1,), dtype=torch.int64, device=c.device)
    ws = _linconv_ws(workspace, N, L, M, c_bits, True, c.device)
    _ok(lib().ne_linconv_fused(_dev(c, "c"), _DT[c.dtype], c_bits, _dev(g, "g", torch.int8), L,
                               _dev(out, "out", out_dtype), _DT[out_dtype],
                               _opt(flags, "flags", torch.int32), _dev(n_bad, "n_bad", torch.int64),
                               N, ctypes.byref(p), *_ws_args(ws), _stream()), "ne_linconv_fused")
    return out, flags, n_bad


def ne_permute_scale_fused(c: torch.Tensor, perm: torch.Tensor, scale: torch.Tensor | None,
                           add: torch.Tensor | None, p: Params, out_dtype=torch.int64,
                           out: torch.Tensor | None = None, flags: bool | torch.Tensor = True,
                           n_bad: torch.Tensor | None = None, workspace=True):
    """c: [M, N]; perm [N] int32; scale/add [N] int64 or None -> (d_hat, flags, n_bad).
    workspace=True allocates the row copy the library gathers from; None: direct gather."""
    M, N = c.shape
    if M != p.M or perm.shape != (N,):
        raise ValueError("shape mismatch")
    if c.dtype not in _DT:
        raise TypeError("c must be int8, int32 or int64")
    if out is None:
        out = torch.empty((M, N), dtype=out_dtype, device=c.device)
    if flags is True:
        flags = torch.empty(((N + 31) // 32,), dtype=torch.int32, device=c.device)
    elif flags is False:
        flags = None
    if n_bad is None:
        n_bad = torch.zeros((1,), dtype=torch.int64, device=c.device)
    if workspace is True:
        need = int(lib().ne_permute_workspace(N, M, _DT[c.dtype]))
        workspace = torch.empty((need // 8,), dtype=torch.int64, device=c.device)
    ws = workspace if workspace is not None and workspace is not False else None
    _ok(lib().ne_permute_scale_fused(_dev(c, "c"), _DT[c.dtype], _dev(perm, "perm", torch.int32),
                                     _opt(scale, "scale", _word(p)), _opt(add, "add", _word(p)),
                                     _dev(out, "out", out_dtype), _DT[out_dtype],
                                     _opt(flags, "flags", torch.int32),
                                     _dev(n_bad, "n_bad", torch.int64), N, ctypes.byref(p),
                                     _opt(ws, "workspace", None),
                                     ws.numel() * ws.element_size() if ws is not None else 0,
                                     _stream()), "ne_permute_scale_fused")
    return out, flags, n_bad


# ------------------------------------------------------- operation series

def ne_series_range(p: Params, c_max: int, ops):
    """ops: (kind, length, operand_max) tuples (NE_SERIES_*).  Returns
    (eps_bits per operation, bound on the final output, whether it is within
    the entangled range).  Invalid arguments raise NEError."""
    n = len(ops)
    arr = (_SeriesOp * max(n, 1))()
    for i, (kind, length, omax) in enumerate(ops):
        arr[i].kind, arr[i].length, arr[i].operand_max = kind, length, omax
    bits = (ctypes.c_int32 * max(n, 1))()
    out = ctypes.c_int64()
    rc = lib().ne_series_range(ctypes.byref(p), c_max, n, arr, bits, ctypes.byref(out))
    if rc not in (0, NE_ERANGE):
        raise NEError(rc, "ne_series_range")
    return [bits[i] for i in range(n)], out.value, rc == 0


def ne_series_workspace(n: int, N: int, M: int) -> int:
    return int(lib().ne_series_workspace(n, N, M))


def ne_series_gemm_scale_permute(c: torch.Tensor, Gt: torch.Tensor, scale: torch.Tensor | None,
                                 add: torch.Tensor | None, perm: torch.Tensor, p: Params, *,
                                 scale_max: int | None = None, add_max: int | None = None,
                                 out_dtype=torch.int32, out: torch.Tensor | None = None,
                                 flags: bool | torch.Tensor = True,
                                 n_bad: torch.Tensor | None = None,
                                 workspace: torch.Tensor | None = None):
    """c: [M, n, K] int8, Gt: [N, K] int8, scale/add [n*N] int64 or None,
    perm [n*N] int32 -> (d_hat [M, n*N], flags [ceil(n*N/32)], n_bad).
    scale_max / add_max bound |scale| / |add| and are required with them."""
    M, n, K = c.shape
    N, K2 = Gt.shape
    Q = n * N
    if M != p.M or K2 != K or perm.shape != (Q,):
        raise ValueError("shape mismatch")
    if (scale is not None and scale_max is None) or (add is not None and add_max is None):
        raise ValueError("scale_max / add_max are required with scale / add")
    if out is None:
        out = torch.empty((M, Q), dtype=out_dtype, device=c.device)
    if flags is True:
        flags = torch.empty(((Q + 31) // 32,), dtype=torch.int32, device=c.device)
    elif flags is False:
        flags = None
    if n_bad is None:
        n_bad = torch.zeros((1,), dtype=torch.int64, device=c.device)
    need = ne_series_workspace(n, N, M)
    if workspace is None:
        workspace = torch.empty((max(need, 16) // 8,), dtype=torch.int64, device=c.device)
    _ok(lib().ne_series_gemm_scale_permute(
        _dev(c, "c", torch.int8), _dev(Gt, "Gt", torch.int8), _opt(scale, "scale", torch.int64),
        _opt(add, "add", torch.int64), _dev(perm, "perm", torch.int32),
        scale_max if scale is not None else 1, add_max if add is not None else 0,
        _dev(out, "out", out_dtype), _DT[out_dtype], _opt(flags, "flags", torch.int32),
        _dev(n_bad, "n_bad", torch.int64), n, K, N, ctypes.byref(p),
        _dev(workspace, "workspace"), workspace.numel() * workspace.element_size(),
        _stream()), "ne_series_gemm_scale_permute")
    return out, flags, n_bad


# -------------------------------------------------------------------- batch

class Problem:
    """One problem of a batch (see ne_problem_t in include/ne.h); keeps its
    tensors alive.  Outputs (d_hat, flags, n_bad) are allocated here."""

    def __init__(self, op: int, c: torch.Tensor, g: torch.Tensor | None = None, *,
                 perm: torch.Tensor | None = None, scale: torch.Tensor | None = None,
                 add: torch.Tensor | None = None, r_check: int = 0, out_dtype=torch.int32):
        self.op, self.c, self.g, self.perm, self.scale, self.add = op, c, g, perm, scale, add
        self.M = c.shape[0]
        dev = c.device
        if op == NE_OP_GEMM:
            self.n, self.K = c.shape[1], c.shape[2]
            self.N = g.shape[0]
            self.d_hat = torch.empty((self.M, self.n, self.N), dtype=out_dtype, device=dev)
            self.flags = torch.empty((self.n, (self.N + 31) // 32), dtype=torch.int32, device=dev)
        else:
            self.n, self.K, self.N = 1, 1, c.shape[1]
            self.d_hat = torch.empty((self.M, self.N), dtype=out_dtype, device=dev)
            self.flags = torch.empty(((self.N + 31) // 32,), dtype=torch.int32, device=dev)
        self.n_bad = torch.zeros((1,), dtype=torch.int64, device=dev)
        self.r_check, self.out_dtype = r_check, out_dtype

    def struct(self) -> _Problem:
        s = _Problem()
        s.op, s.M, s.r_check, s.out_dtype = self.op, self.M, self.r_check, _DT[self.out_dtype]
        s.n, s.K, s.N = self.n, self.K, self.N
        s.c = _dev(self.c, "c", torch.int8)
        s.g = _dev(self.g, "g", torch.int8) if self.g is not None else None
        s.perm = _opt(self.perm, "perm", torch.int32)
        s.scale = _opt(self.scale, "scale", torch.int64)
        s.add = _opt(self.add, "add", torch.int64)
        s.d_hat = _dev(self.d_hat, "d_hat", self.out_dtype)
        s.flags = _dev(self.flags, "flags", torch.int32)
        s.n_bad = _dev(self.n_bad, "n_bad", torch.int64)
        return s


def _problem_array(problems):
    arr = (_Problem * len(problems))()
    for i, q in enumerate(problems):
        arr[i] = q.struct()
    return arr


class Batch:
    """A planned batch: owns the device table and the library's host plan."""

    def __init__(self, problems, tuning=None):
        self.problems = list(problems)
        self._arr = _problem_array(self.problems)
        need = _i64()
        t = ctypes.byref(tuning) if tuning is not None else None
        _ok(lib().ne_batch_plan(self._arr, len(self.problems), t, None, 0, ctypes.byref(need),
                                None), "ne_batch_plan")
        dev = self.problems[0].c.device if self.problems else torch.device("cuda")
        self.table = torch.empty((max(need.value, 256),), dtype=torch.uint8, device=dev)
        plan = _vp()
        _ok(lib().ne_batch_plan(self._arr, len(self.problems), t, _dev(self.table, "table"),
                                self.table.numel(), ctypes.byref(need), ctypes.byref(plan)),
            "ne_batch_plan")
        self._plan = plan

    @property
    def items(self) -> int:
        return lib().ne_batch_items(self._plan)

    def run(self):
        _ok(lib().ne_batch_run(self._plan, _stream()), "ne_batch_run")

    def __del__(self):
        try:
            if getattr(self, "_plan", None):
                lib().ne_batch_free(self._plan)
                self._plan = None
        except Exception:
            pass


def ne_batch_plan(problems, tuning=None) -> Batch:
    return Batch(problems, tuning)


def ne_batch_run(batch: Batch):
    batch.run()


def ne_batch_autotune(problems, reps: int = 3) -> _Tuning:
    """Time every bucket's candidates on the device; returns the tuning struct."""
    arr = _problem_array(problems)
    need = _i64()
    _ok(lib().ne_batch_plan(arr, len(problems), None, None, 0, ctypes.byref(need), None),
        "ne_batch_plan")
    table = torch.empty((max(need.value, 256),), dtype=torch.uint8, device=problems[0].c.device)
    out = _Tuning()
    _ok(lib().ne_batch_autotune(arr, len(problems), _dev(table, "table"), table.numel(), reps,
                                ctypes.byref(out), _stream()), "ne_batch_autotune")
    return out
