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

import atexit
import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgf2.so")

GF2_OK = 0
GF2_EINVAL = -1
GF2_ENOMEM = -2
GF2_EHIP = -3

EXPORTED = ("gf2_matmul", "gf2_decompose", "gf2_rank", "gf2_solve", "gf2_decompose_batched",
            "gf2_solve_batched", "gf2_rref", "gf2_nullspace", "gf2_inverse", "gf2_autotune", "gf2_autotune_table",
            "gf2_autotune_params", "gf2_set_param", "gf2_profile", "gf2_profile_read", "gf2_microbench", "gf2_workspace_bytes",
            "gf2_matmul_ws", "gf2_decompose_ws", "gf2_rank_ws", "gf2_solve_ws", "gf2_decompose_batched_ws",
            "gf2_solve_batched_ws", "gf2_decompose_noalloc", "gf2_decompose_graph", "gf2_graph_launch",
            "gf2_graph_destroy", "gf2_release", "gf2_last_error", "gf2_version")
# operation codes of gf2_workspace_bytes
OP_MATMUL, OP_DECOMPOSE, OP_RANK, OP_SOLVE, OP_DECOMPOSE_BATCHED, OP_SOLVE_BATCHED = range(6)
SIZE_MAX = 2 ** 64 - 1
BATCH_MAX_DIM = 2048


class Gf2Error(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libgf2 error {code}: {msg}")
        self.code = code


class _Mat(ctypes.Structure):
    _fields_ = [("data", ctypes.c_void_p), ("rows", ctypes.c_int64), ("cols", ctypes.c_int64),
                ("w", ctypes.c_int64), ("ld", ctypes.c_int64)]


class BatchItem(ctypes.Structure):
    """gf2_batch_item: shape of one batch matrix and the offsets of its pieces."""
    _fields_ = [(f, ctypes.c_int64) for f in ("rows", "cols", "a", "l", "e", "p", "c", "b", "x")]


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
        PB = ctypes.POINTER(BatchItem)
        lib.gf2_decompose_batched.argtypes = [PB, i64, vp, vp, vp, vp, vp, vp, vp]
        lib.gf2_solve_batched.argtypes = [PB, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp]
        lib.gf2_rref.argtypes = [P, P, vp, vp, vp]
        lib.gf2_nullspace.argtypes = [P, P, vp, vp]
        lib.gf2_inverse.argtypes = [P, P, vp, vp]
        lib.gf2_autotune.argtypes = [i64, vp]
        lib.gf2_autotune_table.argtypes = [ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(i64)]
        i32p = ctypes.POINTER(ctypes.c_int32)
        lib.gf2_autotune_params.argtypes = [i64, i64, i32p, i32p, i32p, ctypes.POINTER(i64)]
        lib.gf2_set_param.argtypes = [ctypes.c_char_p, i64]
        lib.gf2_profile.argtypes = [ctypes.c_int]
        lib.gf2_profile_read.argtypes = [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64),
                                         ctypes.POINTER(ctypes.c_double)]
        lib.gf2_microbench.argtypes = [ctypes.c_int, i64, ctypes.c_int, ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_double), vp]
        sz = ctypes.c_size_t
        lib.gf2_workspace_bytes.argtypes = [ctypes.c_int, i64, i64, i64]
        lib.gf2_workspace_bytes.restype = sz
        lib.gf2_matmul_ws.argtypes = [P, P, P, ctypes.c_int, vp, sz, vp]
        lib.gf2_decompose_ws.argtypes = [P, P, P, vp, vp, vp, vp, sz, vp]
        lib.gf2_rank_ws.argtypes = [P, vp, vp, sz, vp]
        lib.gf2_solve_ws.argtypes = [P, P, P, vp, vp, vp, sz, vp]
        lib.gf2_decompose_batched_ws.argtypes = [PB, i64, vp, vp, vp, vp, vp, vp, vp, sz, vp]
        lib.gf2_solve_batched_ws.argtypes = [PB, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, sz, vp]
        lib.gf2_decompose_noalloc.argtypes = [P, P, P, vp, vp, vp, vp]
        lib.gf2_decompose_graph.argtypes = [P, P, P, vp, vp, vp, vp, sz, vp, ctypes.POINTER(vp)]
        lib.gf2_graph_launch.argtypes = [vp, vp]
        lib.gf2_graph_destroy.argtypes = [vp]
        lib.gf2_release.argtypes = []
        lib.gf2_last_error.restype = ctypes.c_char_p
        lib.gf2_version.restype = ctypes.c_char_p
        for name in ("gf2_matmul", "gf2_decompose", "gf2_rank", "gf2_solve", "gf2_decompose_batched",
                     "gf2_solve_batched", "gf2_rref", "gf2_nullspace", "gf2_inverse", "gf2_autotune",
                     "gf2_autotune_table", "gf2_autotune_params", "gf2_set_param", "gf2_profile", "gf2_profile_read", "gf2_microbench",
                     "gf2_matmul_ws", "gf2_decompose_ws", "gf2_rank_ws", "gf2_solve_ws", "gf2_decompose_batched_ws",
                     "gf2_solve_batched_ws", "gf2_decompose_noalloc", "gf2_decompose_graph", "gf2_graph_launch",
                     "gf2_graph_destroy", "gf2_release"):
            getattr(lib, name).restype = ctypes.c_int
        _lib = lib
        atexit.register(_release_at_exit)
    return _lib


def _release_at_exit():
    """Free the library's streams, events and workspace while the HIP runtime
    is still fully alive (only if this process used a GPU)."""
    import sys

    torch = sys.modules.get("torch")
    if _lib is not None and torch is not None and torch.cuda.is_initialized():
        _lib.gf2_release()


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


def gf2_decompose_batched(items, A, L, E, perm, pivcols, rank, stream=None) -> None:
    """items: a ctypes array of BatchItem (host); the pools are device tensors (or None)."""
    _check(load().gf2_decompose_batched(items, len(items), _ptr(A), _ptr(L), _ptr(E), _ptr(perm),
                                        _ptr(pivcols), _ptr(rank), _stream(stream)))


def gf2_solve_batched(items, L, E, perm, pivcols, rank, B, X, consistent, stream=None) -> None:
    _check(load().gf2_solve_batched(items, len(items), _ptr(L), _ptr(E), _ptr(perm), _ptr(pivcols),
                                    _ptr(rank), _ptr(B), _ptr(X), _ptr(consistent), _stream(stream)))


def gf2_rref(A: Mat, R, pivcols, rank, stream=None) -> None:
    Rd = ctypes.byref(R.desc()) if R is not None else None
    _check(load().gf2_rref(ctypes.byref(A.desc()), Rd, _ptr(pivcols), _ptr(rank), _stream(stream)))


def gf2_nullspace(A: Mat, N: Mat, nullity, stream=None) -> None:
    _check(load().gf2_nullspace(ctypes.byref(A.desc()), ctypes.byref(N.desc()), _ptr(nullity), _stream(stream)))


def gf2_inverse(A: Mat, X: Mat, invertible=None, stream=None) -> None:
    _check(load().gf2_inverse(ctypes.byref(A.desc()), ctypes.byref(X.desc()), _ptr(invertible), _stream(stream)))


def gf2_autotune(max_size: int = 65536, stream=None) -> None:
    _check(load().gf2_autotune(int(max_size), _stream(stream)))


def gf2_autotune_table():
    """(variants as a 9 x 4 list (row class x block class), strassen cutoff)."""
    v = (ctypes.c_int32 * 36)()
    c = ctypes.c_int64()
    _check(load().gf2_autotune_table(v, ctypes.byref(c)))
    return [list(v[4 * r:4 * r + 4]) for r in range(9)], c.value


def gf2_autotune_params(rows: int, cols: int) -> dict:
    """The panel width and table size an n x m decomposition uses, beside the
    paper's analytic table size and Strassen point (Section 6)."""
    w, c, ca = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    st = ctypes.c_int64()
    _check(load().gf2_autotune_params(int(rows), int(cols), ctypes.byref(w), ctypes.byref(c), ctypes.byref(ca),
                                      ctypes.byref(st)))
    return {"panel_words": w.value, "table_bits": c.value, "analytic_table_bits": ca.value,
            "analytic_strassen": st.value}


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


MICROBENCH_KINDS = {"hbm_read": 0, "hbm_copy": 1, "valu_xor32": 2, "lds_read": 3, "mfma_int8": 4, "mfma_fp4": 5}


def gf2_microbench(kind, nbytes=0, iters=0, stream=None):
    """One microbenchmark (name or number, see MICROBENCH_KINDS): returns
    (rate, ms) -- bytes/s, operations/s or multiply-accumulates/s, and the mean
    launch time."""
    k = MICROBENCH_KINDS[kind] if isinstance(kind, str) else int(kind)
    rate = ctypes.c_double()
    ms = ctypes.c_double()
    _check(load().gf2_microbench(k, int(nbytes), int(iters), ctypes.byref(rate), ctypes.byref(ms), _stream(stream)))
    return rate.value, ms.value


def gf2_workspace_bytes(op: int, rows: int, cols: int, k: int = 0) -> int:
    """Device bytes a *_ws call needs (op: one of the OP_* codes)."""
    v = load().gf2_workspace_bytes(int(op), int(rows), int(cols), int(k))
    if v == SIZE_MAX:
        raise Gf2Error(GF2_EINVAL, load().gf2_last_error().decode())
    return int(v)


def _ws(workspace):
    """(pointer, bytes) of a caller workspace tensor (or (None, 0))."""
    if workspace is None:
        return None, 0
    return ctypes.c_void_p(int(workspace.data_ptr())), int(workspace.numel() * workspace.element_size())


def gf2_matmul_ws(C: Mat, A: Mat, B: Mat, accumulate: bool, workspace, stream=None) -> None:
    p, nb = _ws(workspace)
    _check(load().gf2_matmul_ws(ctypes.byref(C.desc()), ctypes.byref(A.desc()), ctypes.byref(B.desc()),
                                1 if accumulate else 0, p, nb, _stream(stream)))


def gf2_decompose_ws(A: Mat, L, E, perm, pivcols, rank, workspace, stream=None) -> None:
    Ld = ctypes.byref(L.desc()) if L is not None else None
    Ed = ctypes.byref(E.desc()) if E is not None else None
    p, nb = _ws(workspace)
    _check(load().gf2_decompose_ws(ctypes.byref(A.desc()), Ld, Ed, _ptr(perm), _ptr(pivcols), _ptr(rank), p, nb,
                                   _stream(stream)))


def gf2_decompose_noalloc(A: Mat, L, E, perm, pivcols, rank, stream=None) -> None:
    """gf2_decompose with the library's static scratch (no device allocation)."""
    Ld = ctypes.byref(L.desc()) if L is not None else None
    Ed = ctypes.byref(E.desc()) if E is not None else None
    _check(load().gf2_decompose_noalloc(ctypes.byref(A.desc()), Ld, Ed, _ptr(perm), _ptr(pivcols), _ptr(rank),
                                        _stream(stream)))


class DecomposeGraph:
    """gf2_decompose_graph: one captured decomposition, replayed by launch()."""

    def __init__(self, A: Mat, L, E, perm, pivcols, rank, workspace, stream):
        Ld = ctypes.byref(L.desc()) if L is not None else None
        Ed = ctypes.byref(E.desc()) if E is not None else None
        p, nb = _ws(workspace)
        h = ctypes.c_void_p()
        _check(load().gf2_decompose_graph(ctypes.byref(A.desc()), Ld, Ed, _ptr(perm), _ptr(pivcols), _ptr(rank), p,
                                          nb, _stream(stream), ctypes.byref(h)))
        self.h = h

    def launch(self, stream=None):
        _check(load().gf2_graph_launch(self.h, _stream(stream)))

    def close(self):
        if self.h:
            _check(load().gf2_graph_destroy(self.h))
            self.h = None


def gf2_rank_ws(A: Mat, rank, workspace, stream=None) -> None:
    p, nb = _ws(workspace)
    _check(load().gf2_rank_ws(ctypes.byref(A.desc()), _ptr(rank), p, nb, _stream(stream)))


def gf2_solve_ws(A: Mat, B: Mat, X: Mat, consistent, rank, workspace, stream=None) -> None:
    p, nb = _ws(workspace)
    _check(load().gf2_solve_ws(ctypes.byref(A.desc()), ctypes.byref(B.desc()), ctypes.byref(X.desc()),
                               _ptr(consistent), _ptr(rank), p, nb, _stream(stream)))


def gf2_decompose_batched_ws(items, A, L, E, perm, pivcols, rank, workspace, stream=None) -> None:
    p, nb = _ws(workspace)
    _check(load().gf2_decompose_batched_ws(items, len(items), _ptr(A), _ptr(L), _ptr(E), _ptr(perm),
                                           _ptr(pivcols), _ptr(rank), p, nb, _stream(stream)))


def gf2_solve_batched_ws(items, L, E, perm, pivcols, rank, B, X, consistent, workspace, stream=None) -> None:
    p, nb = _ws(workspace)
    _check(load().gf2_solve_batched_ws(items, len(items), _ptr(L), _ptr(E), _ptr(perm), _ptr(pivcols),
                                       _ptr(rank), _ptr(B), _ptr(X), _ptr(consistent), p, nb, _stream(stream)))


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


def inverse(A: Mat, stream=None):
    """A^-1 of a square A: dict(X (Mat, zero when A is singular), invertible (1-element tensor))."""
    import torch

    X = Mat.zeros(A.rows, A.cols, device=A.t.device)
    inv = torch.zeros(1, dtype=torch.int64, device=A.t.device)
    gf2_inverse(A, X, inv, stream)
    return dict(X=X, invertible=inv)


def solve(A: Mat, B: Mat, stream=None):
    import torch

    X = Mat.zeros(A.cols, B.cols, device=A.t.device)
    cons = torch.zeros(wpr(B.cols), dtype=torch.int64, device=A.t.device)
    rank = torch.empty(1, dtype=torch.int64, device=A.t.device)
    gf2_solve(A, B, X, cons, rank, stream)
    return dict(X=X, consistent=cons, rank=rank)


class Batch:
    """Device pools of a batch of row-major bit matrices (the gf2_batch_item layout).

    ``shapes`` is a list of (rows, cols).  Offsets are assigned in order; every
    pool is an int64 torch tensor of raw words.  ``set_matrices`` / ``set_rhs``
    upload numpy word arrays, ``decompose`` / ``solve`` call the ABI, and
    ``fetch`` copies every pool back once so that ``result(i)`` can slice it.
    """

    def __init__(self, shapes, device="cuda"):
        import torch

        self.shapes = [(int(n), int(m)) for n, m in shapes]
        cnt = len(self.shapes)
        self.items = (BatchItem * cnt)()
        offs = dict(a=0, l=0, e=0, p=0, c=0, b=0, x=0)
        self.off = []
        for i, (n, m) in enumerate(self.shapes):
            k = min(n, m)
            o = dict(offs)
            self.off.append(o)
            it = self.items[i]
            it.rows, it.cols = n, m
            it.a, it.l, it.e, it.p, it.c, it.b, it.x = o["a"], o["l"], o["e"], o["p"], o["c"], o["b"], o["x"]
            offs["a"] += n * wpr(m)
            offs["l"] += n * wpr(k)
            offs["e"] += k * wpr(m)
            offs["p"] += n
            offs["c"] += k
            offs["b"] += wpr(n)
            offs["x"] += wpr(m)
        self.size = offs

        def pool(words, dtype=torch.int64):
            return torch.zeros(max(words, 1), dtype=dtype, device=device)

        self.A, self.L, self.E = pool(offs["a"]), pool(offs["l"]), pool(offs["e"])
        self.perm, self.pivcols = pool(offs["p"]), pool(offs["c"])
        self.B, self.X = pool(offs["b"]), pool(offs["x"])
        self.rank = pool(cnt)
        self.consistent = pool(cnt, torch.int32)
        self.host = None

    def __len__(self):
        return len(self.shapes)

    def _upload(self, dst, arrays, key, rows_of):
        import torch

        flat = np.zeros(max(self.size[key], 1), dtype=np.uint64)
        for i, a in enumerate(arrays):
            o = self.off[i][key]
            a = np.ascontiguousarray(a, dtype=np.uint64).reshape(-1)
            assert a.size == rows_of(i), (i, a.size, rows_of(i))
            flat[o:o + a.size] = a
        dst.copy_(torch.from_numpy(flat.view(np.int64)))

    def set_matrices(self, mats):
        """mats[i]: numpy uint64 array of rows x ceil(cols/64) words."""
        self._upload(self.A, mats, "a", lambda i: self.shapes[i][0] * wpr(self.shapes[i][1]))

    def set_rhs(self, rhs):
        """rhs[i]: numpy uint64 array of ceil(rows/64) words (bit j = entry j)."""
        self._upload(self.B, rhs, "b", lambda i: wpr(self.shapes[i][0]))

    def mat_view(self, i) -> "Mat":
        """Matrix i of the A pool as a row-major Mat (a view; for gf2_matmul)."""
        n, m = self.shapes[i]
        o = self.off[i]["a"]
        return Mat(self.A[o:o + max(n * wpr(m), 1)], n, m, max(wpr(m), 1), max(n, 1))

    def decompose(self, want_le=True, stream=None):
        gf2_decompose_batched(self.items, self.A, self.L if want_le else None, self.E if want_le else None,
                              self.perm, self.pivcols, self.rank, stream)

    def solve(self, stream=None):
        gf2_solve_batched(self.items, self.L, self.E, self.perm, self.pivcols, self.rank, self.B, self.X,
                          self.consistent, stream)

    def fetch(self):
        self.host = {k: getattr(self, k).cpu().numpy() for k in
                     ("L", "E", "perm", "pivcols", "rank", "X", "consistent")}
        return self.host

    def result(self, i):
        h = self.host if self.host is not None else self.fetch()
        n, m = self.shapes[i]
        k = min(n, m)
        o = self.off[i]
        return dict(rank=int(h["rank"][i]),
                    perm=h["perm"][o["p"]:o["p"] + n],
                    pivcols=h["pivcols"][o["c"]:o["c"] + k],
                    L=h["L"][o["l"]:o["l"] + n * wpr(k)].view(np.uint64).reshape(n, wpr(k)),
                    E=h["E"][o["e"]:o["e"] + k * wpr(m)].view(np.uint64).reshape(k, wpr(m)),
                    x=h["X"][o["x"]:o["x"] + wpr(m)].view(np.uint64),
                    consistent=int(h["consistent"][i]))
