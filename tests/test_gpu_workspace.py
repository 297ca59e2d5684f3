"""Caller-owned workspace (the *_ws calls): every output equals the oracle's bit
for bit, the workspace is reused across calls of different shapes without any
state carried over, and the exact size gf2_workspace_bytes reports suffices
(the workspace is a slice of a larger buffer that is pre-filled with ones)."""
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


def exact_ws(nbytes):
    """A workspace of exactly nbytes (rounded to 256) inside a larger buffer of ones."""
    import torch

    words = max((nbytes + 255) // 256 * 32, 32)
    buf = torch.full((words + 64,), -1, dtype=torch.int64, device="cuda")
    return buf[:words]


@pytest.mark.parametrize("n,m", [(1, 1), (300, 70), (1300, 1700), (2300, 2900), (3000, 1030)])
def test_decompose_ws_parity(g, orc, n, m):
    import torch

    say("decompose_ws", n, m)
    A = synth.dense(41 * n + m, 1, n, m)
    ref = orc.ple(A, n, m)
    k = min(n, m)
    L, E = g.Mat.zeros(n, k), g.Mat.zeros(k, m)
    perm = torch.empty(n, dtype=torch.int64, device="cuda")
    piv = torch.empty(max(k, 1), dtype=torch.int64, device="cuda")
    rank = torch.empty(1, dtype=torch.int64, device="cuda")
    ws = exact_ws(g.gf2_workspace_bytes(g.OP_DECOMPOSE, n, m))
    g.gf2_decompose_ws(g.Mat.from_rowmajor(A, n, m), L, E, perm, piv, rank, ws)
    torch.cuda.synchronize()
    assert int(rank.item()) == ref["rank"]
    assert np.array_equal(perm.cpu().numpy(), ref["perm"])
    assert np.array_equal(piv.cpu().numpy()[:k], ref["pivcols"])
    assert np.array_equal(L.to_rowmajor(), ref["L"])
    assert np.array_equal(E.to_rowmajor(), ref["E"])


def test_ws_reused_across_shapes_and_ops(g, orc):
    """One caller buffer serves rank, solve, decompose and product calls of
    different shapes in a row on one stream."""
    import torch

    shapes = [(2100, 2500), (700, 4000), (2600, 900)]
    need = max(max(g.gf2_workspace_bytes(g.OP_DECOMPOSE, n, m), g.gf2_workspace_bytes(g.OP_RANK, n, m),
                   g.gf2_workspace_bytes(g.OP_SOLVE, n, m, 3)) for n, m in shapes)
    need = max(need, g.gf2_workspace_bytes(g.OP_MATMUL, 1500, 1700, 1100))
    ws = exact_ws(need)
    for i, (n, m) in enumerate(shapes):
        say("ws reuse", n, m)
        A = synth.planted(60 + i, 9, n, m, min(n, m) // 2)
        Aw = orc.matmul(A[0], A[1], n, min(n, m) // 2, m)
        ref = orc.ple(Aw, n, m)
        rank = torch.empty(1, dtype=torch.int64, device="cuda")
        g.gf2_rank_ws(g.Mat.from_rowmajor(Aw, n, m), rank, ws)
        torch.cuda.synchronize()
        assert int(rank.item()) == ref["rank"]
        rhs = synth.dense(70 + i, 3, n, 3)
        X = g.Mat.zeros(m, 3)
        cons = torch.zeros(1, dtype=torch.int64, device="cuda")
        g.gf2_solve_ws(g.Mat.from_rowmajor(Aw, n, m), g.Mat.from_rowmajor(rhs, n, 3), X, cons, rank, ws)
        torch.cuda.synchronize()
        sref = orc.solve(Aw, rhs, n, m, 3)
        assert np.array_equal(X.to_rowmajor(), sref["X"])
        assert np.array_equal(cons.cpu().numpy().view(np.uint64), sref["consistent"])
    n, k, m = 1500, 1100, 1700
    Am, Bm = synth.dense(80, 1, n, k), synth.dense(80, 2, k, m)
    C = g.Mat.zeros(n, m)
    g.gf2_matmul_ws(C, g.Mat.from_rowmajor(Am, n, k), g.Mat.from_rowmajor(Bm, k, m), False, ws)
    assert np.array_equal(C.to_rowmajor(), orc.matmul(Am, Bm, n, k, m))


def test_ws_too_small_rejected(g):
    import torch

    n = m = 1000
    need = g.gf2_workspace_bytes(g.OP_DECOMPOSE, n, m)
    ws = torch.zeros((need - 256) // 8, dtype=torch.int64, device="cuda")
    rank = torch.empty(1, dtype=torch.int64, device="cuda")
    with pytest.raises(g.Gf2Error):
        g.gf2_rank_ws(g.Mat.zeros(n, m), rank, ws)


def test_batched_ws_parity(g, orc):
    import torch

    shapes = [(70, 130), (257, 64), (64, 64), (2048, 2048), (1000, 3)]
    mats = [synth.dense(90 + i, 1, n, m) for i, (n, m) in enumerate(shapes)]
    bt = g.Batch(shapes)
    bt.set_matrices(mats)
    bt.set_rhs([synth.dense(95 + i, 2, 1, n)[0] for i, (n, _) in enumerate(shapes)])
    ws = exact_ws(max(g.gf2_workspace_bytes(g.OP_DECOMPOSE_BATCHED, len(shapes), 2048, 2048),
                      g.gf2_workspace_bytes(g.OP_SOLVE_BATCHED, len(shapes), 0)))
    g.gf2_decompose_batched_ws(bt.items, bt.A, bt.L, bt.E, bt.perm, bt.pivcols, bt.rank, ws)
    g.gf2_solve_batched_ws(bt.items, bt.L, bt.E, bt.perm, bt.pivcols, bt.rank, bt.B, bt.X, bt.consistent, ws)
    torch.cuda.synchronize()
    for i, (n, m) in enumerate(shapes):
        ref = orc.ple(mats[i], n, m)
        got = bt.result(i)
        assert got["rank"] == ref["rank"] and np.array_equal(got["E"], ref["E"]), i
        assert np.array_equal(got["L"], ref["L"][:, :got["L"].shape[1]]), i
        assert np.array_equal(got["perm"], ref["perm"]) and np.array_equal(got["pivcols"], ref["pivcols"]), i
        b = synth.dense(95 + i, 2, 1, n)[0]
        col = np.zeros((n, 1), dtype=np.uint64)
        idx = np.arange(n)
        col[:, 0] = (b[idx >> 6] >> (idx & 63).astype(np.uint64)) & np.uint64(1)
        sref = orc.solve(mats[i], col, n, m, 1)
        assert got["consistent"] == int(sref["consistent"][0] & np.uint64(1)), i
        xr = sref["X"][:, 0]
        xbits = np.zeros(g.wpr(m), dtype=np.uint64)
        for j in np.nonzero(xr)[0]:
            xbits[j >> 6] |= np.uint64(1) << np.uint64(j & 63)
        assert np.array_equal(got["x"], xbits), i
