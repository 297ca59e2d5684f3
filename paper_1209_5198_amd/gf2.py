"""Thin ctypes binding of libgf2 (include/gf2.h).

The functions named like the C ABI (``gf2_matmul``, ``gf2_decompose``,
``gf2_rank``, ``gf2_solve`` ...) only marshal arguments; every step of the
computation runs in the library's HIP kernels.  Device memory comes from torch
(``int64`` tensors viewed as raw 64-bit words) and the default stream is
torch's current HIP stream.  There is no CPU fallback: if ``libgf2.so`` is not
built the first call raises.

:class:`Mat` describes a device bit matrix in the ABI's column-blocked layout
(word (i, q) at ``(q // w) * ld * w + i * w + q % w``); its helpers only move
words between that layout and plain row-major numpy arrays.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgf2.so")

GF2_OK = 0
GF2_EINVAL = -1
GF2_ENOMEM = -2
GF2_EHIP = -3

EXPORTED = ("gf2_matmul", "gf2_decompose", "gf2_rank", "gf2_solve", "gf2_set_param",
            "gf2_profile", "gf2_profile_read", "gf2_release", "gf2_last_error", "gf2_version")


class Gf2Error(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libgf2 error {code}: {msg}")
        self.code = code


class _Mat(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("rows", ctypes.c_int64), ("cols", ctypes.c_int64),
                ("w", ctypes.c_int64), ("ld", ctypes.c_int64)]


_lib = None


def load():
    """Load libgf2.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_1209_5198_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER(_Mat)
        vp = ctypes.c_void_p
        i64 = ctypes.c_int64
        lib.gf2_matmul.argtypes = [P, P, P, ctypes.c_int, vp]
        lib.gf2_decompose.argtypes = [P, P, P, vp, vp, vp, vp]
        lib.gf2_rank.argtypes = [P, vp, vp]
        lib.gf2_solve.argtypes = [P, P, P, vp, vp, vp]
        lib.gf2_set_param.argtypes = [ctypes.c_char_p, i64]
        lib.gf2_profile.argtypes = [ctypes.c_int]
        lib.gf2_profile_read.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64),
                                         ctypes.POINTER(ctypes.c_double)]
        lib.gf2_release.argtypes = []
        lib.gf2_last_error.restype = ctypes.c_char_p
        lib.gf2_version.restype = ctypes.c_char_p
        for name in ("gf2_matmul", "gf2_decompose", "gf2_rank", "gf2_solve", "gf2_set_param",
                     "gf2_profile", "gf2_profile_read", "gf2_release"):
            getattr(lib, name).restype = ctypes.c_int
        _lib = lib
    return _lib


def _check(rc: int):
    if rc != GF2_OK:
        raise Gf2Error(rc, load().gf2_last_error().decode())


def _stream(stream):
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(int(stream.cuda_stream) if hasattr(stream, "cuda_stream") else int(stream))


def _ptr(t):
    return None if t is None else ctypes.c_void_p(int(t.data_ptr()))


def wpr(bits: int) -> int:
    return (int(bits) + 63) // 64


class Mat:
    """Device bit matrix: an int64 torch tensor of words plus its layout."""

    def __init__(self, tensor, rows: int, cols: int, w: int, ld: int):
        self.t = tensor
        self.rows, self.cols, self.w, self.ld = int(rows), int(cols), int(w), int(ld)
        need = self.nblocks() * self.ld * self.w
        assert tensor.numel() >= need, (tensor.numel(), need)

    def nblocks(self) -> int:
        nw = wpr(self.cols)
        return (nw + self.w - 1) // self.w if nw else 0

    def desc(self) -> _Mat:
        return _Mat(ctypes.c_void_p(int(self.t.data_ptr())), self.rows, self.cols, self.w, self.ld)

    @staticmethod
    def _shape(rows, cols, w, ld):
        nw = wpr(cols)
        w = max(1, nw) if w is None else int(w)
        ld = max(rows, 1) if ld is None else int(ld)
        return w, ld

    @classmethod
    def zeros(cls, rows: int, cols: int, w=None, ld=None, device="cuda"):
        import torch

        w, ld = cls._shape(rows, cols, w, ld)
        nb = (wpr(cols) + w - 1) // w
        t = torch.zeros(max(nb * ld * w, 1), dtype=torch.int64, device=device)
        return cls(t, rows, cols, w, ld)

    @staticmethod
    def blocked_words(words: np.ndarray, rows: int, cols: int, w: int, ld: int) -> np.ndarray:
        """Row-major words (rows x ceil(cols/64)) -> flat column-blocked array."""
        nw = wpr(cols)
        nb = (nw + w - 1) // w
        buf = np.zeros((ld, nb * w), dtype=np.uint64)
        buf[:rows, :nw] = np.asarray(words, dtype=np.uint64).reshape(rows, nw)
        return np.ascontiguousarray(buf.reshape(ld, nb, w).transpose(1, 0, 2)).reshape(-1)

    @classmethod
    def from_rowmajor(cls, words: np.ndarray, rows: int, cols: int, w=None, ld=None, device="cuda"):
        import torch

        w, ld = cls._shape(rows, cols, w, ld)
        flat = cls.blocked_words(words, rows, cols, w, ld)
        if flat.size == 0:
            flat = np.zeros(1, dtype=np.uint64)
        t = torch.from_numpy(flat.view(np.int64).copy()).to(device)
        return cls(t, rows, cols, w, ld)

    def to_rowmajor(self) -> np.ndarray:
        nw = wpr(self.cols)
        nb = self.nblocks()
        flat = self.t.detach().cpu().numpy().view(np.uint64)[: nb * self.ld * self.w]
        arr = flat.reshape(nb, self.ld, self.w).transpose(1, 0, 2).reshape(self.ld, nb * self.w)
        return np.ascontiguousarray(arr[: self.rows, :nw])


# ----------------------------------------------------------------- the ABI, one to one
def gf2_matmul(C: Mat, A: Mat, B: Mat, accumulate: bool = False, stream=None) -> None:
    _check(load().gf2_matmul(ctypes.byref(C.desc()), ctypes.byref(A.desc()), ctypes.byref(B.desc()),
                             1 if accumulate else 0, _stream(stream)))


def gf2_decompose(A: Mat, L, E, perm, pivcols, rank, stream=None) -> None:
    Ld = ctypes.byref(L.desc()) if L is not None else None
    Ed = ctypes.byref(E.desc()) if E is not None else None
    _check(load().gf2_decompose(ctypes.byref(A.desc()), Ld, Ed, _ptr(perm), _ptr(pivcols), _ptr(rank),
                                _stream(stream)))


def gf2_rank(A: Mat, rank, stream=None) -> None:
    _check(load().gf2_rank(ctypes.byref(A.desc()), _ptr(rank), _stream(stream)))


def gf2_solve(A: Mat, B: Mat, X: Mat, consistent, rank=None, stream=None) -> None:
    _check(load().gf2_solve(ctypes.byref(A.desc()), ctypes.byref(B.desc()), ctypes.byref(X.desc()),
                            _ptr(consistent), _ptr(rank), _stream(stream)))


def gf2_set_param(name: str, value: int) -> None:
    _check(load().gf2_set_param(name.encode(), int(value)))


def gf2_profile(enable: bool) -> None:
    _check(load().gf2_profile(1 if enable else 0))


def gf2_profile_read():
    ms = ctypes.c_double()
    n = ctypes.c_int64()
    work = ctypes.c_double()
    _check(load().gf2_profile_read(ctypes.byref(ms), ctypes.byref(n), ctypes.byref(work)))
    return ms.value, n.value, work.value


def gf2_release() -> None:
    _check(load().gf2_release())


def gf2_last_error() -> str:
    return load().gf2_last_error().decode()


def gf2_version() -> str:
    return load().gf2_version().decode()


# ----------------------------------------------------------------- conveniences (still ABI calls)
def decompose(A: Mat, want_le: bool = True, stream=None, L=None, E=None):
    """Allocate outputs and call gf2_decompose; returns a dict of device tensors/Mats."""
    import torch

    n, m = A.rows, A.cols
    kmin = min(n, m)
    dev = A.t.device
    if want_le:
        L = L if L is not None else Mat.zeros(n, kmin, device=dev)
        E = E if E is not None else Mat.zeros(kmin, m, device=dev)
    perm = torch.empty(max(n, 1), dtype=torch.int64, device=dev)
    piv = torch.empty(max(kmin, 1), dtype=torch.int64, device=dev)
    rank = torch.empty(1, dtype=torch.int64, device=dev)
    gf2_decompose(A, L if want_le else None, E if want_le else None, perm, piv, rank, stream)
    return dict(L=L if want_le else None, E=E if want_le else None, perm=perm[:n], pivcols=piv[:kmin], rank=rank)


def matmul(A: Mat, B: Mat, stream=None, w=None) -> Mat:
    C = Mat.zeros(A.rows, B.cols, w=w, device=A.t.device)
    gf2_matmul(C, A, B, False, stream)
    return C


def solve(A: Mat, B: Mat, stream=None):
    import torch

    X = Mat.zeros(A.cols, B.cols, device=A.t.device)
    cons = torch.zeros(wpr(B.cols), dtype=torch.int64, device=A.t.device)
    rank = torch.empty(1, dtype=torch.int64, device=A.t.device)
    gf2_solve(A, B, X, cons, rank, stream)
    return dict(X=X, consistent=cons, rank=rank)
