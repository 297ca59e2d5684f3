"""The paper's own block method, written out in pure Python for small inputs.

Test infrastructure: an independent route to the decomposition that the oracle
must agree with (same P, same rank, same row spaces per block), so that the
oracle's tie-break and swap rule is pinned to the paper rather than to itself.

Rows are Python ints (bit c = column c).  Word size b is arbitrary.

* :func:`build_z` -- procedure buildZ of Section 4.4: per bit k, the test
  vector c from the bookkeeping words M; the first row at or after i_b with odd
  popcount(c AND row) becomes the pivot and is exchanged with row i_b; Z and M
  are updated; finally the columns of Z that belong to bits with no pivot are
  squeezed out.
* :func:`block_decompose` -- the non-recursive block decomposition of
  Section 4: per panel of b columns, buildZ gives P^(j) and Z; Y = D*Z
  (Section 4.1, D*Z = Y) and the Schur complement E xor Y*C (eq. (Aj)) with the
  raw pivot rows [B C]; the permutation of later steps also moves the rows of
  L already written (final form of the decomposition before Lemma 4.1).
"""
from __future__ import annotations


def popcount(x: int) -> int:
    return bin(x).count("1")


def build_z(rows, start, col0, b, perm=None, lrows=None):
    """buildZ on bits [col0, col0+b) of rows[start:] (rows are swapped in place).

    Returns (P, Z, r): P[k] = panel-relative row chosen for bit k before the
    swap, or -1; Z = list of b words with r bits each.
    """
    mask = (1 << b) - 1
    ib = 0
    Z = [1 << j for j in range(b)]
    M = [1 << j for j in range(b)]
    P = [-1] * b
    nrow = len(rows) - start
    for k in range(b):
        c = 1 << k
        for i in range(k):
            if (M[i] >> k) & 1:
                c ^= 1 << i
        for i in range(ib, nrow):
            w = (rows[start + i] >> col0) & mask
            if popcount(c & w) & 1:
                P[k] = i
                a, z = start + i, start + ib
                rows[a], rows[z] = rows[z], rows[a]
                if perm is not None:
                    perm[a], perm[z] = perm[z], perm[a]
                if lrows is not None:
                    lrows[a], lrows[z] = lrows[z], lrows[a]
                M[k] = (rows[z] >> col0) & mask
                ib += 1
                break
        y = M[k]
        for j in range(k):
            if (y >> j) & 1:
                Z[k] ^= Z[j]
                M[k] ^= M[j]
        for j in range(k):
            if (c >> j) & 1:
                Z[j] ^= Z[k]
                M[j] ^= M[k]
    kept = 0
    for i in range(b):
        if P[i] == -1:
            for j in range(b):
                Z[j] = ((Z[j] >> 1) & ~kept) ^ (Z[j] & kept)
        else:
            kept = 2 * kept + 1
    return P, Z, ib


def block_decompose(rows_in, n, m, b):
    """Section 4 block decomposition with word size b.

    Returns dict(perm, rank, L (list of n ints, bit t = column t),
    U (list of rank ints: raw pivot rows, block staircase), blocks (list of
    (R_j, r_j, col0_j))).
    """
    rows = list(rows_in)
    perm = list(range(n))
    lrows = [0] * n
    U = []
    blocks = []
    R = 0
    col0 = 0
    while col0 < m and R < n:
        bw = min(b, m - col0)
        _, Z, r = build_z(rows, R, col0, bw, perm, lrows)
        for t in range(r):
            lrows[R + t] |= 1 << (R + t)
            U.append(rows[R + t])
        pmask = (1 << bw) - 1
        for i in range(R + r, n):
            d = (rows[i] >> col0) & pmask
            y = 0
            for j in range(bw):
                if (d >> j) & 1:
                    y ^= Z[j]
            for t in range(r):
                if (y >> t) & 1:
                    rows[i] ^= rows[R + t]
                    lrows[i] |= 1 << (R + t)
            assert (rows[i] >> col0) & pmask == 0, "D xor Y*B must vanish (D = Y*B)"
        blocks.append((R, r, col0))
        R += r
        col0 += bw
    return dict(perm=perm, rank=R, L=lrows, U=U, blocks=blocks)
