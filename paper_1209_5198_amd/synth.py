"""Seeded synthetic GF(2) inputs, shared by the oracle side and the GPU side.

This module holds random bits only -- none of the method's arithmetic.  A
planted-rank matrix is returned as its two random factors; each side forms the
product with its own code.

Random source: the SplitMix64 generator of Steele, Lea and Flood ("Fast
splittable pseudorandom number generators", OOPSLA 2014), used counter-style:
the 64-bit output for (seed, stream, index) is the SplitMix64 mixing function
applied to ``key(seed, stream) + (index + 1) * GAMMA`` with
``GAMMA = 0x9E3779B97F4A7C15`` and
``key(seed, stream) = mix(seed * GAMMA + stream)``.

Layout of every matrix returned: numpy ``uint64`` array of plain row-major bit
rows, ``ceil(cols/64)`` words per row, column c = bit (c % 64) of word c // 64,
bits at or beyond ``cols`` zero (Section 3 of the paper: a_ij is bit r of word
q with j = 64q + r; the unused high bits of the last word are padding).

Workloads (shapes, value distributions and structure of the paper's tests):
  * ``dense``      iid Bernoulli(1/2) entries -- the random dense matrices of
                   the paper's timing tables (Section 7).
  * ``bernoulli``  iid Bernoulli(p) entries, one 32-bit draw per entry,
                   entry = draw < floor(p * 2^32).
  * ``sparse_rows`` exactly ``k`` ones per row at distinct uniform positions
                   (the shape of the low-rank sample S_n of Section 7).
  * ``planted``    factors X (n x r), Y (r x m) of a rank-<=r product X*Y.
  * ``batch_specs`` shapes and kinds of a batch of independent matrices (sides
                   uniform in [lo, hi], density 1/2 or 1/10, half of them with
                   a planted rank), ``batch_matrix`` / ``batch_rhs`` their
                   entries and right-hand sides.
  * ``serving_specs`` a request stream: rank / solve / decompose requests,
                   square sides log-uniform in [lo, hi] or 1:4 rectangles with
                   the long side log-uniform in [4 lo, hi], Poisson arrivals.
"""
from __future__ import annotations

import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix(z):
    """SplitMix64 output function (vectorised over uint64 arrays)."""
    with np.errstate(over="ignore"):
        z = np.asarray(z, dtype=np.uint64)
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def key(seed: int, stream: int) -> np.uint64:
    with np.errstate(over="ignore"):
        return _mix(np.uint64(seed & 0xFFFFFFFFFFFFFFFF) * GAMMA + np.uint64(stream & 0xFFFFFFFFFFFFFFFF))[()]


def words(seed: int, stream: int, start: int, count: int) -> np.ndarray:
    """``count`` consecutive 64-bit outputs starting at counter ``start``."""
    k = key(seed, stream)
    idx = np.arange(start + 1, start + 1 + count, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix(k + idx * GAMMA)


def wpr(bits: int) -> int:
    return (int(bits) + 63) // 64


def pad_mask(cols: int) -> np.uint64:
    r = cols & 63
    return np.uint64(0xFFFFFFFFFFFFFFFF) if r == 0 else np.uint64((1 << r) - 1)


def dense(seed: int, stream: int, rows: int, cols: int, row0: int = 0, nrows=None) -> np.ndarray:
    """Bernoulli(1/2) matrix rows [row0, row0+nrows) of a rows x cols matrix."""
    nw = wpr(cols)
    nrows = rows - row0 if nrows is None else nrows
    out = words(seed, stream, row0 * nw, nrows * nw).reshape(nrows, nw)
    if nw:
        out[:, -1] &= pad_mask(cols)
    return out


def bernoulli(seed: int, stream: int, rows: int, cols: int, p: float) -> np.ndarray:
    """iid Bernoulli(p) entries: entry (i, j) = draw_{i*cols+j} < floor(p * 2^32)."""
    if p == 0.5:
        return dense(seed, stream, rows, cols)
    thr = np.uint64(min(int(p * 4294967296.0), 4294967296))
    nw = wpr(cols)
    out = np.zeros((rows, nw), dtype=np.uint64)
    chunk = max(1, (1 << 22) // max(cols, 1))
    for r0 in range(0, rows, chunk):
        r1 = min(rows, r0 + chunk)
        n = (r1 - r0) * cols
        first = r0 * cols
        w = words(seed, stream, first // 2, (n + (first & 1) + 1) // 2 + 1)
        halves = np.empty(2 * w.size, dtype=np.uint64)
        halves[0::2] = w & np.uint64(0xFFFFFFFF)
        halves[1::2] = w >> np.uint64(32)
        draws = halves[(first & 1):(first & 1) + n]
        bits = (draws < thr).astype(np.uint8).reshape(r1 - r0, cols)
        padded = np.zeros((r1 - r0, nw * 64), dtype=np.uint8)
        padded[:, :cols] = bits
        out[r0:r1] = np.packbits(padded, axis=1, bitorder="little").view("<u8").astype(np.uint64)
    return out


def sparse_rows(seed: int, stream: int, rows: int, cols: int, k: int) -> np.ndarray:
    """Exactly k ones per row at distinct uniformly drawn positions."""
    k = min(k, cols)
    nw = wpr(cols)
    out = np.zeros((rows, nw), dtype=np.uint64)
    for i in range(rows):
        keys = words(seed, stream, i * cols, cols)
        pos = np.argsort(keys, kind="stable")[:k]
        for c in pos:
            out[i, c >> 6] |= np.uint64(1) << np.uint64(c & 63)
    return out


def planted(seed: int, stream: int, rows: int, cols: int, r: int, p: float = 0.5):
    """Random factors (X: rows x r, Y: r x cols) of a planted rank-<=r product."""
    X = bernoulli(seed, 2 * stream, rows, r, p)
    Y = bernoulli(seed, 2 * stream + 1, r, cols, p)
    return X, Y


# ---------------------------------------------------------------- batches
BATCH_SPEC_STREAM = 0x6261  # draws of the batch shapes
BATCH_MAT_STREAM = 1_000_000  # + i: entries of matrix i (planted: 2 * (this + i) and + 1)
BATCH_RHS_STREAM = 5_000_000  # + i: right-hand side of matrix i


def batch_specs(seed: int, count: int, lo: int = 64, hi: int = 2048, densities=(0.5, 0.1)):
    """Per-matrix workload parameters of a batch.

    Matrix i uses draws 4i..4i+3 of stream BATCH_SPEC_STREAM: n = lo + d0 mod
    (hi-lo+1), m likewise from d1 (independent sides), density densities[d2 & 1],
    planted iff bit 1 of d2 (probability 1/2), with planted rank
    r = r_lo + d3 mod (kmin - r_lo + 1), r_lo = min(ceil(m/4), kmin); r = 0 means
    an iid matrix.
    """
    d = words(seed, BATCH_SPEC_STREAM, 0, 4 * count).reshape(count, 4) if count else np.zeros((0, 4), np.uint64)
    span = hi - lo + 1
    out = []
    for i in range(count):
        n = lo + int(d[i, 0] % np.uint64(span))
        m = lo + int(d[i, 1] % np.uint64(span))
        p = densities[int(d[i, 2] & np.uint64(1))]
        r = 0
        if int(d[i, 2] >> np.uint64(1)) & 1:
            kmin = min(n, m)
            r_lo = min((m + 3) // 4, kmin)
            r = r_lo + int(d[i, 3] % np.uint64(kmin - r_lo + 1))
        out.append(dict(i=i, n=n, m=m, p=p, r=r))
    return out


def batch_matrix(seed: int, spec):
    """Entries of a batch matrix: ('iid', A) or ('planted', X, Y) with X n x r and Y r x m
    of the matrix's density (each side forms the product with its own code)."""
    i, n, m, p, r = spec["i"], spec["n"], spec["m"], spec["p"], spec["r"]
    if r:
        X, Y = planted(seed, BATCH_MAT_STREAM + i, n, m, r, p)
        return ("planted", X, Y)
    return ("iid", bernoulli(seed, BATCH_MAT_STREAM + i, n, m, p))


def batch_rhs(seed: int, spec) -> np.ndarray:
    """Right-hand side of batch matrix i: n Bernoulli(1/2) bits, bit j of the vector
    is bit j % 64 of word j // 64."""
    n = spec["n"]
    out = words(seed, BATCH_RHS_STREAM + spec["i"], 0, wpr(n))
    if out.size:
        out[-1] &= pad_mask(n)
    return out


# ---------------------------------------------------------------- request streams
SERVE_SPEC_STREAM = 0x7365  # draws of the request kinds and shapes
SERVE_ARRIVAL_STREAM = 0x7366  # draws of the inter-arrival gaps
SERVE_MAT_STREAM = 10_000_000  # + id: entries of request id
SERVE_RHS_STREAM = 20_000_000  # + id: right-hand side of request id
SERVE_KINDS = ("rank", "solve", "decompose")


def _unit(d):
    """64-bit draws -> floats in (0, 1)."""
    return (d >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0) + 0.5 / 9007199254740992.0


def serving_specs(seed: int, count: int, lo: int = 128, hi: int = 16384):
    """Request i uses draws 4i..4i+3 of stream SERVE_SPEC_STREAM: kind uniform over
    SERVE_KINDS; square (n = m = s, s log-uniform in [lo, hi]) or, with probability
    1/2, a 1:4 rectangle whose long side is log-uniform in [4 lo, hi], tall or wide
    with probability 1/2 each."""
    d = words(seed, SERVE_SPEC_STREAM, 0, 4 * count).reshape(count, 4) if count else np.zeros((0, 4), np.uint64)
    u = _unit(d[:, 1]) if count else np.zeros(0)
    out = []
    for i in range(count):
        kind = SERVE_KINDS[int(d[i, 0] % np.uint64(3))]
        if int(d[i, 2]) & 1:
            s_ = int(round(lo * (hi / lo) ** u[i]))
            n = m = s_
        else:
            long_ = int(round(4 * lo * (hi / (4 * lo)) ** u[i]))
            short = max(1, long_ // 4)
            n, m = (long_, short) if (int(d[i, 2]) >> 1) & 1 else (short, long_)
        out.append(dict(id=i, kind=kind, n=n, m=m))
    return out


def poisson_arrivals(seed: int, count: int, rate: float) -> np.ndarray:
    """Arrival times (s) of a Poisson stream of the given rate (1/s): cumulative sums
    of exponential gaps -ln(U)/rate from stream SERVE_ARRIVAL_STREAM."""
    if count == 0:
        return np.zeros(0)
    gaps = -np.log(_unit(words(seed, SERVE_ARRIVAL_STREAM, 0, count))) / float(rate)
    return np.cumsum(gaps)


def serving_matrix(seed: int, spec) -> np.ndarray:
    """Bernoulli(1/2) entries of request ``spec``."""
    return dense(seed, SERVE_MAT_STREAM + spec["id"], spec["n"], spec["m"])


def serving_rhs(seed: int, spec) -> np.ndarray:
    """Right-hand side of request ``spec`` as a bit vector (wpr(n) words)."""
    n = spec["n"]
    out = words(seed, SERVE_RHS_STREAM + spec["id"], 0, wpr(n))
    if out.size:
        out[-1] &= pad_mask(n)
    return out
