"""GPU parity at the full benchmark sizes, in the launch configuration bench.py times.

* 65536 x 65536 and 16384 x 16384 decompositions (Bernoulli(1/2)): SHA-256 of
  every output (perm, pivcols, L, E) equals the digest of the oracle's output
  stored in tests/golden/fullsize_hashes.json (written by
  tests/golden/make_fullsize_hashes.py, which calls only the oracle), rank equal.
* planted rank: X (32768 x 20000) and Y (20000 x 65536) from the generator; the
  GPU forms A = X*Y with gf2_matmul (its digest must equal the oracle product's)
  and decomposes it: rank 20000 and every output digest equal.
* 16384^3 product, and a 32768^3 product with one Strassen-Winograd level
  (cutoff 16384): SHA-256 of C equals the oracle product's digest.
"""
import hashlib
import json
import os
import sys

import numpy as np
import pytest

from paper_1209_5198_amd import synth

pytestmark = pytest.mark.gpu
GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "fullsize_hashes.json")


def digest(a) -> str:
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint64:
        a = a.astype("<u8", copy=False)
    elif a.dtype == np.int64:
        a = a.astype("<i8", copy=False)
    return hashlib.sha256(a.tobytes()).hexdigest()


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def g():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1209_5198_amd import gf2

    gf2.load()
    return gf2


@pytest.fixture(scope="module")
def gold():
    with open(GOLD) as f:
        return json.load(f)


def check_decomposition(g, A, n, m, ref):
    import torch

    out = g.decompose(A)
    torch.cuda.synchronize()
    rank = int(out["rank"].item())
    say("  rank", rank)
    assert rank == ref["rank"]
    assert digest(out["perm"].cpu().numpy()) == ref["perm"]
    assert digest(out["pivcols"].cpu().numpy()) == ref["pivcols"]
    E = out["E"].to_rowmajor()
    assert digest(E) == ref["E"]
    del E
    L = out["L"].to_rowmajor()
    assert digest(L) == ref["L"]


@pytest.mark.parametrize("case,sp", [("dense16384", 0), ("dense65536", 0), ("dense16384", 2), ("dense65536", 4)])
def test_fullsize_dense_decompose(g, gold, case, sp):
    """Full-size digests with the one-level schedule and with super-panels."""
    ref = gold.get(case)
    if ref is None:
        pytest.skip(f"no golden digests for {case}")
    n, m = ref["n"], ref["m"]
    say("fullsize", case, n, m, "sp_panels", sp)
    A = g.Mat.from_rowmajor(synth.dense(ref["seed"], ref["stream"], n, m), n, m)
    g.gf2_set_param("sp_panels", sp)
    try:
        check_decomposition(g, A, n, m, ref)
    finally:
        g.gf2_set_param("sp_panels", 0)


def test_fullsize_planted_rank(g, gold):
    import torch

    ref = gold.get("planted")
    if ref is None:
        pytest.skip("no golden digests for planted")
    n, m, r = ref["n"], ref["m"], ref["r_planted"]
    say("fullsize planted", n, r, m)
    X, Y = synth.planted(ref["seed"], ref["stream"], n, m, r)
    Xg = g.Mat.from_rowmajor(X, n, r)
    Yg = g.Mat.from_rowmajor(Y, r, m)
    del X, Y
    A = g.matmul(Xg, Yg)
    torch.cuda.synchronize()
    del Xg, Yg
    assert digest(A.to_rowmajor()) == ref["A"]
    check_decomposition(g, A, n, m, ref)


def fullsize_product(g, gold, name, cutoff=None):
    """C = A*B at a full size: SHA-256 of C equals the oracle product's digest."""
    import torch

    ref = gold.get(name)
    if ref is None:
        pytest.skip("no golden digest for " + name)
    n, seed = ref["n"], ref["seed"]
    say("fullsize matmul", n, "strassen_cutoff", cutoff)
    A = synth.dense(seed, ref["streams"][0], n, n)
    B = synth.dense(seed, ref["streams"][1], n, n)
    Ag, Bg = g.Mat.from_rowmajor(A, n, n), g.Mat.from_rowmajor(B, n, n)
    del A, B
    if cutoff is not None:
        g.gf2_set_param("strassen_cutoff", cutoff)
    try:
        C = g.matmul(Ag, Bg)
        torch.cuda.synchronize()
    finally:
        if cutoff is not None:
            g.gf2_set_param("strassen_cutoff", 65536)
    assert digest(C.to_rowmajor()) == ref["C"]


def test_fullsize_matmul_16384(g, gold):
    fullsize_product(g, gold, "matmul16384")


def test_fullsize_matmul_32768_strassen(g, gold):
    # one Strassen-Winograd level (32768 > 16384), leaves of 16384^3
    fullsize_product(g, gold, "matmul32768", cutoff=16384)
