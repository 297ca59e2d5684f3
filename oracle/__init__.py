"""CPU oracle for dense GF(2) linear algebra -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The GPU library and its Python binding
never import, link or call it; it shares no code, header, table or helper with
them.

All matrices here are numpy ``uint64`` arrays of plain row-major bit rows
(``wpr = ceil(cols/64)`` words per row, column ``c`` = bit ``c % 64`` of word
``c // 64``), the bit order of Section 3 of the paper with b = 64.

Functions (each cites the passage it follows; see ``gf2_oracle.c``):

* :func:`ple`    -- P*A = L*E, Lemma 4.1 in its b = 1 (PLE) form (Remark after
  Lemma 4.1); pivot = first row in current order (row search of procedure
  buildZ, Section 4.4), transposition swaps, no column swaps.
* :func:`matmul` -- C = A*B from the definition of the product.
* :func:`solve`  -- A*x = b through the decomposition, free variables zero.
* :func:`nullspace` -- null space basis read off the reduced row echelon form
                    (back-substitution of the echelon rows), Section 1's use.
* :func:`inverse` -- the inverse of a square matrix from its definition
                    A*X = I (Gauss-Jordan elimination of [A | I]).
* :func:`pack_bits` / :func:`unpack_bits` -- the b-bit packing of Section 3
  (a_ij is bit r of word q, j = q*b + r), for any b <= 64.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gf2_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile ``gf2_oracle.c`` into ``liboracle.so`` with gcc (-fopenmp)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        lib = ctypes.CDLL(_LIB)
        p64 = ctypes.POINTER(ctypes.c_uint64)
        pi64 = ctypes.POINTER(ctypes.c_int64)
        i64 = ctypes.c_int64
        lib.or_ple.argtypes = [i64, i64, p64, p64, p64, pi64, pi64]
        lib.or_ple.restype = i64
        lib.or_matmul.argtypes = [i64, i64, i64, p64, p64, p64, ctypes.c_int]
        lib.or_matmul.restype = None
        lib.or_solve.argtypes = [i64, i64, i64, p64, p64, p64, p64]
        lib.or_solve.restype = i64
        lib.or_nullspace.argtypes = [i64, i64, p64, p64, p64]
        lib.or_nullspace.restype = i64
        lib.or_inverse.argtypes = [i64, p64, p64]
        lib.or_inverse.restype = i64
        lib.or_num_threads.argtypes = []
        lib.or_num_threads.restype = ctypes.c_int
        lib.or_set_threads.argtypes = [ctypes.c_int]
        lib.or_set_threads.restype = None
        _lib = lib
    return _lib


def wpr(bits: int) -> int:
    return (int(bits) + 63) // 64


def _u64(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64))


def _i64(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64))


def _check(A, rows, cols):
    A = np.ascontiguousarray(A, dtype=np.uint64)
    assert A.shape == (rows, wpr(cols)), (A.shape, rows, cols)
    return A


def num_threads() -> int:
    return int(_load().or_num_threads())


def set_threads(n: int) -> None:
    _load().or_set_threads(int(n))


def ple(A, n: int, m: int, want_le: bool = True):
    """Decomposition P*A = L*E (Lemma 4.1, b = 1 form).

    Returns dict(rank, perm[n], pivcols[min(n,m)], L (n x min(n,m)), E (min(n,m) x m)).
    """
    lib = _load()
    A = _check(A, n, m)
    kmin = min(n, m)
    perm = np.zeros(max(n, 1), dtype=np.int64)
    piv = np.zeros(max(kmin, 1), dtype=np.int64)
    if want_le:
        E = np.zeros((max(kmin, 1), wpr(m)), dtype=np.uint64)
        L = np.zeros((max(n, 1), wpr(max(kmin, 1))), dtype=np.uint64)
        r = lib.or_ple(n, m, _u64(A), _u64(E), _u64(L), _i64(perm), _i64(piv))
    else:
        E = L = None
        r = lib.or_ple(n, m, _u64(A), None, None, _i64(perm), _i64(piv))
    if r < 0:
        raise MemoryError("oracle ple: out of memory")
    out = dict(rank=int(r), perm=perm[:n], pivcols=piv[:kmin])
    if want_le:
        out["E"] = E[:kmin]
        out["L"] = L[:n]
    return out


def matmul(A, B, n: int, k: int, m: int, C=None):
    """C = A*B (or C ^= A*B when C is given), from the definition of the product."""
    lib = _load()
    A = _check(A, n, k)
    B = _check(B, k, m)
    acc = C is not None
    if C is None:
        C = np.zeros((n, wpr(m)), dtype=np.uint64)
    else:
        C = _check(C, n, m).copy()
    lib.or_matmul(n, k, m, _u64(A), _u64(B), _u64(C), 1 if acc else 0)
    return C


def solve(A, B, n: int, m: int, nrhs: int):
    """Solve A*X = B (nrhs systems); returns dict(X (m x nrhs), consistent (wpr(nrhs) words), rank)."""
    lib = _load()
    A = _check(A, n, m)
    B = _check(B, n, nrhs)
    X = np.zeros((max(m, 1), wpr(nrhs)), dtype=np.uint64)
    cons = np.zeros(wpr(nrhs), dtype=np.uint64)
    r = lib.or_solve(n, m, nrhs, _u64(A), _u64(B), _u64(X), _u64(cons))
    if r < 0:
        raise MemoryError("oracle solve: out of memory")
    return dict(X=X[:m], consistent=cons, rank=int(r))


def nullspace(A, n: int, m: int):
    """Null space basis (one vector per free column, free variables unit) and the RREF.

    Returns dict(N ((m - rank) x wpr(m)), R (min(n,m) x wpr(m)), nullity).
    """
    lib = _load()
    A = _check(A, n, m)
    kmin = min(n, m)
    N = np.zeros((max(m, 1), wpr(m)), dtype=np.uint64)
    R = np.zeros((max(kmin, 1), wpr(m)), dtype=np.uint64)
    k = lib.or_nullspace(n, m, _u64(A), _u64(N), _u64(R))
    if k < 0:
        raise MemoryError("oracle nullspace: out of memory")
    return dict(N=N[:k], R=R[:kmin], nullity=int(k))


def inverse(A, n: int):
    """Inverse of a square A (n x n) by Gauss-Jordan elimination of [A | I].

    Returns dict(X (n x wpr(n), zero when singular), invertible (bool)).
    """
    lib = _load()
    A = _check(A, n, n)
    X = np.zeros((max(n, 1), wpr(n)), dtype=np.uint64)
    r = lib.or_inverse(n, _u64(A), _u64(X))
    if r < 0:
        raise MemoryError("oracle inverse: out of memory")
    return dict(X=X[:n], invertible=bool(r))


def rank(A, n: int, m: int) -> int:
    return ple(A, n, m, want_le=False)["rank"]


def pack_bits(bits, b: int = 64):
    """Pack a 0/1 array (rows x cols) into b-bit words: a_ij is bit r of word q, j = q*b + r."""
    bits = np.asarray(bits, dtype=np.uint8)
    rows, cols = bits.shape
    nw = (cols + b - 1) // b
    if b == 64:
        padded = np.zeros((rows, nw * 64), dtype=np.uint8)
        padded[:, :cols] = bits
        return np.packbits(padded, axis=1, bitorder="little").view("<u8").astype(np.uint64)
    out = np.zeros((rows, nw), dtype=np.uint64)
    for j in range(cols):
        q, r = divmod(j, b)
        out[:, q] |= bits[:, j].astype(np.uint64) << np.uint64(r)
    return out


def unpack_bits(words, cols: int, b: int = 64):
    """Inverse of :func:`pack_bits`."""
    words = np.asarray(words, dtype=np.uint64)
    rows = words.shape[0]
    if b == 64:
        w8 = np.ascontiguousarray(words).astype("<u8").view(np.uint8).reshape(rows, -1)
        return np.unpackbits(w8, axis=1, bitorder="little")[:, :cols].copy()
    out = np.zeros((rows, cols), dtype=np.uint8)
    for j in range(cols):
        q, r = divmod(j, b)
        out[:, j] = ((words[:, q] >> np.uint64(r)) & np.uint64(1)).astype(np.uint8)
    return out
