"""Captured decompositions (gf2_decompose_graph): a graph recorded once and
replayed on new contents of A gives, on every replay, the outputs of an eager
gf2_decompose of the same matrix, bit for bit (with eager work and
synchronisations between the replays), and the oracle's on small shapes."""
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


def outs(g, n, m):
    import torch

    k = min(n, m)
    return (g.Mat.zeros(n, k), g.Mat.zeros(k, m), torch.zeros(n, dtype=torch.int64, device="cuda"),
            torch.zeros(max(k, 1), dtype=torch.int64, device="cuda"), torch.zeros(1, dtype=torch.int64, device="cuda"))


@pytest.mark.parametrize("n,m,sp", [(1300, 1700, 0), (2300, 2900, 2), (4100, 3000, 0)])
def test_graph_replays_equal_eager(g, orc, n, m, sp):
    import torch

    say("graph", n, m, sp)
    g.gf2_set_param("sp_panels", sp)
    try:
        s = torch.cuda.Stream()
        A = g.Mat.zeros(n, m)
        L, E, perm, piv, rank = outs(g, n, m)
        ws = torch.empty((g.gf2_workspace_bytes(g.OP_DECOMPOSE, n, m) + 255) // 8, dtype=torch.int64, device="cuda")
        graph = g.DecomposeGraph(A, L, E, perm, piv, rank, ws, s)
        try:
            for rep in range(3):
                words = synth.dense(300 + rep, 1, n, m) if rep != 1 else orc.matmul(
                    *synth.planted(300 + rep, 9, n, m, 700), n, 700, m)
                A.t.copy_(g.Mat.from_rowmajor(words, n, m).t)  # refill A in place
                torch.cuda.synchronize()
                graph.launch(s)
                s.synchronize()
                ref = g.decompose(g.Mat.from_rowmajor(words, n, m))  # eager, default stream
                torch.cuda.synchronize()
                assert int(rank.item()) == int(ref["rank"].item()), rep
                assert np.array_equal(perm.cpu().numpy(), ref["perm"].cpu().numpy()), rep
                k = min(n, m)
                assert np.array_equal(piv.cpu().numpy()[:k], ref["pivcols"].cpu().numpy()[:k]), rep
                assert np.array_equal(L.to_rowmajor(), ref["L"].to_rowmajor()), rep
                assert np.array_equal(E.to_rowmajor(), ref["E"].to_rowmajor()), rep
                if rep == 0:
                    o = orc.ple(words, n, m)
                    assert int(rank.item()) == o["rank"] and np.array_equal(E.to_rowmajor(), o["E"])
        finally:
            graph.close()
    finally:
        g.gf2_set_param("sp_panels", 0)


def test_graph_rejects_null_stream(g):
    import torch

    n = m = 256
    A = g.Mat.zeros(n, m)
    L, E, perm, piv, rank = outs(g, n, m)
    ws = torch.empty((g.gf2_workspace_bytes(g.OP_DECOMPOSE, n, m) + 255) // 8, dtype=torch.int64, device="cuda")
    with pytest.raises(g.Gf2Error):
        g.DecomposeGraph(A, L, E, perm, piv, rank, ws, 0)
