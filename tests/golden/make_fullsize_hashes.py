"""Write tests/golden/fullsize_hashes.json: SHA-256 digests of the CPU oracle's
outputs at the full benchmark sizes.

Calls only the oracle package and the seeded generator.  Hashes are taken over
the oracle's own representation (row-major uint64 words, little-endian; int64
perm / pivcols), so a GPU result matches iff it is bit-identical.

Cases:
  dense65536   65536 x 65536 Bernoulli(1/2), generator seed 65536 stream 1
               (the matrix bench.py decomposes)
  dense16384   16384 x 16384 Bernoulli(1/2), seed 16384 stream 1
  planted      A = X*Y, X 32768 x 20000, Y 20000 x 65536 Bernoulli(1/2),
               seed 20000 (factors from synth.planted stream 9); the product is
               formed by the oracle's matmul
  matmul16384  C = A*B, A and B 16384 x 16384 Bernoulli(1/2), seed 16384
               streams 2 and 3
  matmul32768  C = A*B, A and B 32768 x 32768 Bernoulli(1/2), seed 32768
               streams 2 and 3 (the GPU test runs it with one Strassen level)
  planted_rref the planted matrix above: its reduced row echelon form R and
               null-space basis N (oracle Gauss-Jordan)

Usage: python tests/golden/make_fullsize_hashes.py [case ...]
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1209_5198_amd import synth  # noqa: E402

OUT = os.path.join(HERE, "fullsize_hashes.json")


def digest(a) -> str:
    a = np.ascontiguousarray(a)
    if a.dtype == np.uint64:
        a = a.astype("<u8", copy=False)
    elif a.dtype == np.int64:
        a = a.astype("<i8", copy=False)
    return hashlib.sha256(a.tobytes()).hexdigest()


def ple_hashes(A, n, m):
    t0 = time.time()
    res = oracle.ple(A, n, m)
    dt = time.time() - t0
    return {"n": n, "m": m, "rank": res["rank"], "perm": digest(res["perm"]),
            "pivcols": digest(res["pivcols"]), "L": digest(res["L"]), "E": digest(res["E"]),
            "oracle_seconds": round(dt, 1), "oracle_threads": oracle.num_threads()}


def case_dense65536():
    n = 65536
    return ple_hashes(synth.dense(65536, 1, n, n), n, n) | {"seed": 65536, "stream": 1}


def case_dense16384():
    n = 16384
    return ple_hashes(synth.dense(16384, 1, n, n), n, n) | {"seed": 16384, "stream": 1}


def case_planted():
    n, r, m = 32768, 20000, 65536
    X, Y = synth.planted(20000, 9, n, m, r)
    t0 = time.time()
    A = oracle.matmul(X, Y, n, r, m)
    dt = time.time() - t0
    out = ple_hashes(A, n, m)
    out.update({"seed": 20000, "stream": 9, "r_planted": r, "A": digest(A), "matmul_seconds": round(dt, 1)})
    return out


def product_case(seed, n):
    A = synth.dense(seed, 2, n, n)
    B = synth.dense(seed, 3, n, n)
    t0 = time.time()
    C = oracle.matmul(A, B, n, n, n)
    dt = time.time() - t0
    return {"n": n, "k": n, "m": n, "seed": seed, "streams": [2, 3], "C": digest(C),
            "oracle_seconds": round(dt, 1), "oracle_threads": oracle.num_threads()}


def case_matmul16384():
    return product_case(16384, 16384)


def case_matmul32768():
    return product_case(32768, 32768)


def case_planted_rref():
    n, r, m = 32768, 20000, 65536
    X, Y = synth.planted(20000, 9, n, m, r)
    A = oracle.matmul(X, Y, n, r, m)
    del X, Y
    t0 = time.time()
    res = oracle.nullspace(A, n, m)
    dt = time.time() - t0
    return {"n": n, "m": m, "seed": 20000, "stream": 9, "r_planted": r, "nullity": res["nullity"],
            "R": digest(res["R"]), "N": digest(res["N"]), "oracle_seconds": round(dt, 1),
            "oracle_threads": oracle.num_threads()}


CASES = {"dense16384": case_dense16384, "planted": case_planted, "dense65536": case_dense65536,
         "matmul16384": case_matmul16384, "matmul32768": case_matmul32768, "planted_rref": case_planted_rref}


def main(argv):
    oracle.build()
    want = argv or list(CASES)
    data = {}
    if os.path.exists(OUT):
        with open(OUT) as f:
            data = json.load(f)
    for name in want:
        print("computing", name, flush=True)
        data[name] = CASES[name]()
        print(name, data[name], flush=True)
        with open(OUT, "w") as f:
            json.dump(data, f, indent=1, sort_keys=True)
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
