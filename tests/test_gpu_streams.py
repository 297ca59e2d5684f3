"""Stream ordering of gf2_decompose and gf2_rank on a caller's side stream.

The input's packed words are copied to the device on the side stream (a
non-blocking copy from pinned host memory, issued right before the call), the
call is made on that stream, and the outputs are cloned on it before the host
synchronises: any launch of the library that ran outside the stream's order
would read a partial input or leave a partial output.  Factorizations of at most
two 512-column panels run on the caller's stream itself; larger ones use the
library's look-ahead streams, linked to it.  Both kinds are covered, and every
output is compared with the oracle bit for bit.
"""
import sys

import numpy as np
import pytest

from paper_1209_5198_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def g():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1209_5198_amd import gf2

    gf2.load()
    return gf2


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


# (rows, cols): one panel and two panels (one stream); three and five panels (look-ahead)
SHAPES = [(700, 450), (1024, 1024), (1500, 1100), (2600, 2300)]


def staged_input(g, A, n, m):
    """An empty device matrix of A's layout and A's packed words in pinned host memory."""
    import torch

    packed = g.Mat.from_rowmajor(A, n, m)
    host = packed.t.cpu().pin_memory()
    dev = g.Mat(torch.empty_like(packed.t), n, m, packed.w, packed.ld)
    torch.cuda.synchronize()
    return dev, host


@pytest.mark.parametrize("n,m", SHAPES)
def test_decompose_on_side_stream(g, orc, n, m):
    import torch

    say("decompose on a side stream", n, m)
    A = synth.dense(7 * n + m, 3, n, m)
    ref = orc.ple(A, n, m)
    k = min(n, m)
    Ad, host = staged_input(g, A, n, m)
    L, E = g.Mat.zeros(n, k), g.Mat.zeros(k, m)
    perm = torch.empty(n, dtype=torch.int64, device="cuda")
    piv = torch.empty(k, dtype=torch.int64, device="cuda")
    rank = torch.empty(1, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        Ad.t.copy_(host, non_blocking=True)  # the input arrives on s, right before the call
    g.gf2_decompose(Ad, L, E, perm, piv, rank, s)
    with torch.cuda.stream(s):
        outs = [t.clone() for t in (perm, piv, rank, L.t, E.t)]
    torch.cuda.synchronize()
    assert int(outs[2].item()) == ref["rank"]
    assert np.array_equal(outs[0].cpu().numpy(), ref["perm"])
    assert np.array_equal(outs[1].cpu().numpy()[:k], ref["pivcols"])
    Lc = g.Mat(outs[3], n, k, L.w, L.ld)
    Ec = g.Mat(outs[4], k, m, E.w, E.ld)
    assert np.array_equal(Lc.to_rowmajor(), ref["L"])
    assert np.array_equal(Ec.to_rowmajor(), ref["E"])


@pytest.mark.parametrize("n,m", SHAPES)
def test_rank_on_side_stream(g, orc, n, m):
    import torch

    say("rank on a side stream", n, m)
    X, Y = synth.planted(5, n + m, n, m, 97, 0.5)
    A = orc.matmul(X, Y, n, 97, m)  # rank at most 97
    ref = orc.ple(A, n, m)
    Ad, host = staged_input(g, A, n, m)
    rank = torch.full((1,), -1, dtype=torch.int64, device="cuda")
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        Ad.t.copy_(host, non_blocking=True)
    g.gf2_rank(Ad, rank, s)
    with torch.cuda.stream(s):
        r = rank.clone()
    torch.cuda.synchronize()
    assert int(r.item()) == ref["rank"] <= 97
