"""The autotuner: it measures a tile for every size class, a Strassen cutoff
and a panel width per decomposition size class, and no result depends on it
(decompositions in two size classes and a product stay bit-identical to the
oracle with the tuned choices in use)."""
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


def test_autotune_table_and_invariance(g, orc):
    import torch

    before, cut0 = g.gf2_autotune_table()
    try:
        g.gf2_autotune(65536)
        table, cut = g.gf2_autotune_table()
        print("tuned tiles", table, "strassen cutoff", cut, flush=True)
        assert all(v in (0, 1, 2, 3) for row in table for v in row)
        assert cut in (32768, 65536, 131072)
        # results with the tuned table equal the oracle's
        n, m = 3000, 2600
        A = synth.dense(91, 1, n, m)
        out = g.decompose(g.Mat.from_rowmajor(A, n, m))
        torch.cuda.synchronize()
        ref = orc.ple(A, n, m)
        assert int(out["rank"].item()) == ref["rank"]
        assert np.array_equal(out["perm"].cpu().numpy(), ref["perm"])
        assert np.array_equal(out["E"].to_rowmajor(), ref["E"])
        assert np.array_equal(out["L"].to_rowmajor(), ref["L"])
        # the measured panel widths, and a decomposition in the second size
        # class with its width equal to the oracle too
        for n_c in (2048, 16384, 32768):
            p = g.gf2_autotune_params(n_c, n_c)
            print("class", n_c, p, flush=True)
            assert p["panel_words"] in (2, 4, 8)
        n2, m2 = 5000, 4500
        A2 = synth.dense(91, 4, n2, m2)
        out2 = g.decompose(g.Mat.from_rowmajor(A2, n2, m2))
        torch.cuda.synchronize()
        ref2 = orc.ple(A2, n2, m2)
        assert int(out2["rank"].item()) == ref2["rank"]
        assert np.array_equal(out2["perm"].cpu().numpy(), ref2["perm"])
        assert np.array_equal(out2["E"].to_rowmajor(), ref2["E"])
        assert np.array_equal(out2["L"].to_rowmajor(), ref2["L"])
        X, Y = synth.dense(91, 2, 2100, 1500), synth.dense(91, 3, 1500, 2500)
        C = g.matmul(g.Mat.from_rowmajor(X, 2100, 1500), g.Mat.from_rowmajor(Y, 1500, 2500)).to_rowmajor()
        assert np.array_equal(C, orc.matmul(X, Y, 2100, 1500, 2500))
    finally:
        g.gf2_set_param("autotuned", 0)
        g.gf2_set_param("strassen_cutoff", cut0)
