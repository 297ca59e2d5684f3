"""GPU parity: every output of libgf2 equals the CPU oracle's, bit for bit.

Inputs come from the shared seeded generator; the oracle and the GPU each form
planted products with their own code.  Shapes span several 1024-row x
1024-column product tiles, 512-column panels and ragged tails, plus the
degenerate cases (1 x 1, one row, one column, zero, identity, all ones,
duplicate rows, widths not a multiple of 64).
"""
import sys

import numpy as np
import pytest

from paper_1209_5198_amd import synth

pytestmark = pytest.mark.gpu


def _need_gpu():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def g():
    _need_gpu()
    from paper_1209_5198_amd import gf2

    gf2.load()
    return gf2


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def gpu_decompose(g, words, n, m, w=None):
    A = g.Mat.from_rowmajor(words, n, m, w=w)
    out = g.decompose(A)
    import torch

    torch.cuda.synchronize()
    return dict(rank=int(out["rank"].item()), perm=out["perm"].cpu().numpy(),
                pivcols=out["pivcols"].cpu().numpy(), L=out["L"].to_rowmajor(), E=out["E"].to_rowmajor())


def assert_same_ple(got, ref, tag):
    assert got["rank"] == ref["rank"], (tag, got["rank"], ref["rank"])
    assert np.array_equal(got["perm"], ref["perm"]), (tag, "perm")
    assert np.array_equal(got["pivcols"], ref["pivcols"]), (tag, "pivcols")
    assert np.array_equal(got["E"], ref["E"]), (tag, "E")
    assert np.array_equal(got["L"], ref["L"]), (tag, "L")


def planted_words(orc, seed, n, m, r, p=0.5):
    X, Y = synth.planted(seed, 9, n, m, r, p)
    return orc.matmul(X, Y, n, r, m)


# ---------------------------------------------------------------- product
MATMUL_SHAPES = [(1, 1, 1), (5, 70, 3), (64, 64, 64), (100, 200, 300), (1030, 130, 1100),
                 (2100, 1500, 2500), (300, 2049, 77)]


@pytest.mark.parametrize("n,k,m", MATMUL_SHAPES)
def test_matmul_parity(g, orc, n, k, m):
    say("matmul", n, k, m)
    A = synth.dense(21, 1, n, k)
    B = synth.dense(21, 2, k, m)
    ref = orc.matmul(A, B, n, k, m)
    C = g.matmul(g.Mat.from_rowmajor(A, n, k), g.Mat.from_rowmajor(B, k, m))
    assert np.array_equal(C.to_rowmajor(), ref)


@pytest.mark.parametrize("wa,wb,wc", [(1, 1, 1), (3, 2, 5), (None, 1, None)])
def test_matmul_layouts_and_accumulate(g, orc, wa, wb, wc):
    n, k, m = 700, 650, 900
    say("matmul layouts", wa, wb, wc)
    A = synth.dense(22, 1, n, k)
    B = synth.bernoulli(22, 2, k, m, 0.2)
    C0 = synth.dense(22, 3, n, m)
    ref = orc.matmul(A, B, n, k, m, C=C0)
    Cg = g.Mat.from_rowmajor(C0, n, m, w=wc, ld=n + 5)
    g.gf2_matmul(Cg, g.Mat.from_rowmajor(A, n, k, w=wa, ld=n + 3), g.Mat.from_rowmajor(B, k, m, w=wb),
                 accumulate=True)
    assert np.array_equal(Cg.to_rowmajor(), ref)


# ---------------------------------------------------------------- decomposition
DEC_CASES = [
    ("dense", 1, 1), ("dense", 1, 200), ("dense", 200, 1), ("dense", 64, 64), ("dense", 65, 63),
    ("dense", 63, 65), ("dense", 300, 300), ("dense", 700, 520), ("dense", 520, 700),
    ("dense", 2048, 2048), ("dense", 2500, 1900), ("dense", 1900, 2500), ("dense", 1200, 4200),
    ("sparse", 1500, 1500), ("sparse", 600, 2000), ("planted", 1800, 1600), ("planted", 1000, 3000),
    ("planted", 3000, 1000),
]


@pytest.mark.parametrize("kind,n,m", DEC_CASES)
def test_decompose_parity(g, orc, kind, n, m):
    say("decompose", kind, n, m)
    seed = 31 * n + m
    if kind == "dense":
        A = synth.dense(seed, 1, n, m)
    elif kind == "sparse":
        A = synth.bernoulli(seed, 1, n, m, 0.002)
    else:
        A = planted_words(orc, seed, n, m, min(n, m) // 3)
    ref = orc.ple(A, n, m)
    got = gpu_decompose(g, A, n, m)
    assert_same_ple(got, ref, (kind, n, m))


@pytest.mark.parametrize("panel_words", [1, 2, 3, 8])
def test_decompose_panel_width_invariant(g, orc, panel_words):
    """No tuning parameter changes a result (P is independent of the panel width)."""
    n, m = 1300, 1700
    say("panel width", panel_words)
    A = planted_words(orc, 5, n, m, 900)
    ref = orc.ple(A, n, m)
    g.gf2_set_param("panel_words", panel_words)
    try:
        got = gpu_decompose(g, A, n, m)
    finally:
        g.gf2_set_param("panel_words", 0)
    assert_same_ple(got, ref, panel_words)


KNOB_DEFAULTS = {"panel_gemm_variant": -1, "overlap_lookups": 300000000, "post_follow_lookups": 1500000000,
                 "sp_panels": 0, "panel_words": 0}


@pytest.mark.parametrize("knobs", [{"panel_gemm_variant": v} for v in range(6)] + [
    # one-level schedule: the early bulk update and the post-follow schedule
    # on every panel at once, or neither
    {"overlap_lookups": 0, "post_follow_lookups": 0}, {"overlap_lookups": 10 ** 15, "post_follow_lookups": -1},
    {"overlap_lookups": 10 ** 15, "post_follow_lookups": 0},
    # super-panels of 1, 2 and 3 panels: far words (beyond this super-panel and
    # the next) exist at 2900 columns, so the deferred row exchanges, the far
    # pivot-row solve and the far products all run
    {"sp_panels": 1}, {"sp_panels": 2}, {"sp_panels": 3},
    {"sp_panels": 1, "overlap_lookups": 0}, {"sp_panels": 2, "overlap_lookups": 10 ** 15},
    # narrow panels: many super-panels, partial last ones
    {"sp_panels": 3, "panel_words": 1}, {"sp_panels": 5, "panel_words": 2}, {"sp_panels": 32, "panel_words": 3}])
def test_decompose_tuning_invariant(g, orc, knobs):
    """Look-ahead schedule, super-panel width and product-kernel variant do not change any result."""
    n, m = 2300, 2900
    say("tuning", knobs)
    A = synth.dense(17, 1, n, m)
    ref = orc.ple(A, n, m)
    for k, v in knobs.items():
        g.gf2_set_param(k, v)
    try:
        got = gpu_decompose(g, A, n, m)
    finally:
        for k in knobs:
            g.gf2_set_param(k, KNOB_DEFAULTS[k])
    assert_same_ple(got, ref, knobs)


@pytest.mark.parametrize("kind,sp", [("sparse", 1), ("planted", 1), ("planted", 2), ("dense", 2), ("sparse", 4),
                                     ("planted", 4), ("dense", 0)])
def test_decompose_super_panels(g, orc, kind, sp):
    """Far words at several super-panel widths on inputs whose pivots fall far
    from the diagonal (sparse), stop early (planted rank) or are dense, with
    more rows than columns."""
    n, m = 3100, 4700
    say("super-panels", kind, sp)
    if kind == "sparse":
        A = synth.bernoulli(91, 1, n, m, 0.002)
    elif kind == "planted":
        A = planted_words(orc, 92, n, m, 1700)
    else:
        A = synth.dense(93, 1, n, m)
    ref = orc.ple(A, n, m)
    g.gf2_set_param("sp_panels", sp)
    try:
        got = gpu_decompose(g, A, n, m)
    finally:
        g.gf2_set_param("sp_panels", 0)
    assert_same_ple(got, ref, (kind, sp))


def test_chain_cus_rejected(g):
    """CU-masked chain streams are not supported: only 0 is accepted."""
    with pytest.raises(g.Gf2Error):
        g.gf2_set_param("chain_cus", 8)
    g.gf2_set_param("chain_cus", 0)


@pytest.mark.parametrize("variant", list(range(7)))
def test_matmul_variants(g, orc, variant):
    n, k, m = 2100, 1300, 2500
    say("matmul variant", variant)
    A = synth.dense(23, 1, n, k)
    B = synth.dense(23, 2, k, m)
    ref = orc.matmul(A, B, n, k, m)
    g.gf2_set_param("gemm_variant", variant)
    try:
        C = g.matmul(g.Mat.from_rowmajor(A, n, k), g.Mat.from_rowmajor(B, k, m))
    finally:
        g.gf2_set_param("gemm_variant", -1)
    assert np.array_equal(C.to_rowmajor(), ref)


@pytest.mark.parametrize("n,k,m,acc", [(1, 1, 1, False), (1, 1, 1, True), (300, 64, 500, True), (257, 130, 1025, False),
                                        (2100, 1300, 2500, True), (64, 4100, 70, False), (1030, 2049, 1100, True),
                                        (513, 192, 4097, False), (4096, 4096, 4096, True),
                                        (512, 32768, 640, True), (700, 20000, 900, False)])
def test_matmul_mfma(g, orc, n, k, m, acc):
    """The fp4 matrix-core product (gemm_variant 6): ragged shapes, one to many
    inner words, with and without accumulation, against the oracle's product.
    Few output tiles with a long inner dimension split it across workgroups
    (64 x 4100 x 70: 3 parts, 1030 x 2049 x 1100: 2, 512 x 32768 x 640: 32,
    700 x 20000 x 900: 20), whose parity words are XORed into C."""
    say("matmul mfma", n, k, m, acc)
    A = synth.dense(25, 1, n, k)
    B = synth.dense(25, 2, k, m)
    C0 = synth.dense(25, 3, n, m) if acc else None
    ref = orc.matmul(A, B, n, k, m, C=C0) if acc else orc.matmul(A, B, n, k, m)
    g.gf2_set_param("gemm_variant", 6)
    try:
        if acc:
            Cg = g.Mat.from_rowmajor(C0, n, m)
            g.gf2_matmul(Cg, g.Mat.from_rowmajor(A, n, k), g.Mat.from_rowmajor(B, k, m), accumulate=True)
        else:
            Cg = g.matmul(g.Mat.from_rowmajor(A, n, k), g.Mat.from_rowmajor(B, k, m))
    finally:
        g.gf2_set_param("gemm_variant", -1)
    assert np.array_equal(Cg.to_rowmajor(), ref)


@pytest.mark.parametrize("n,k,m", [(2100, 1300, 2500), (5000, 1024, 3000), (300, 3000, 17000)])
def test_matmul_automatic_mfma(g, orc, n, k, m):
    """Shapes the automatic rule sends to the fp4 matrix-core product (k >= 1024,
    fewer 1024 x 1024 output tiles than CUs) against the oracle."""
    say("matmul automatic (fp4)", n, k, m)
    A = synth.dense(26, 1, n, k)
    B = synth.dense(26, 2, k, m)
    C = g.matmul(g.Mat.from_rowmajor(A, n, k), g.Mat.from_rowmajor(B, k, m))
    assert np.array_equal(C.to_rowmajor(), orc.matmul(A, B, n, k, m))


@pytest.mark.parametrize("variant", [-1, 4, 5])
@pytest.mark.parametrize("n,k,m", [(3000, 1300, 512), (2500, 700, 300), (1030, 64, 64), (700, 2049, 100)])
def test_matmul_narrow(g, orc, variant, n, k, m):
    """Products at most 8 words wide (the next-panel update shape), narrow kernels."""
    say("matmul narrow", variant, n, k, m)
    A = synth.dense(24, 1, n, k)
    B = synth.dense(24, 2, k, m)
    C0 = synth.dense(24, 3, n, m)
    ref = orc.matmul(A, B, n, k, m, C=C0)
    Cg = g.Mat.from_rowmajor(C0, n, m)
    g.gf2_set_param("gemm_variant", variant)
    try:
        g.gf2_matmul(Cg, g.Mat.from_rowmajor(A, n, k), g.Mat.from_rowmajor(B, k, m), accumulate=True)
    finally:
        g.gf2_set_param("gemm_variant", -1)
    assert np.array_equal(Cg.to_rowmajor(), ref)


@pytest.mark.parametrize("cutoff", [256, 700, 1024])
@pytest.mark.parametrize("n,k,m,acc", [(2100, 1500, 2500, False), (1030, 2049, 1100, True), (3000, 1024, 1024, True)])
def test_matmul_strassen(g, orc, cutoff, n, k, m, acc):
    """Strassen-Winograd recursion (Section 6) at 1 to 3 levels, ragged shapes, accumulate."""
    say("matmul strassen", cutoff, n, k, m, acc)
    A = synth.dense(25, 1, n, k)
    B = synth.dense(25, 2, k, m)
    C0 = synth.dense(25, 3, n, m)
    ref = orc.matmul(A, B, n, k, m, C=C0 if acc else None)
    Cg = g.Mat.from_rowmajor(C0, n, m)
    g.gf2_set_param("strassen_cutoff", cutoff)
    try:
        g.gf2_matmul(Cg, g.Mat.from_rowmajor(A, n, k), g.Mat.from_rowmajor(B, k, m), accumulate=acc)
    finally:
        g.gf2_set_param("strassen_cutoff", 65536)
    assert np.array_equal(Cg.to_rowmajor(), ref)


def test_decompose_special(g, orc):
    for n, m in [(1, 1), (5, 9), (64, 64), (130, 70), (700, 1300)]:
        say("special", n, m)
        k = min(n, m)
        cases = {
            "zero": np.zeros((n, orc.wpr(m)), np.uint64),
            "eye": orc.pack_bits(np.eye(n, m, dtype=np.uint8)),
            "ones": orc.pack_bits(np.ones((n, m), np.uint8)),
            "antieye": orc.pack_bits(np.eye(n, m, dtype=np.uint8)[::-1].copy()),
        }
        rng = np.random.default_rng(n + m)
        base = rng.integers(0, 2, size=(max(1, n // 3), m), dtype=np.uint8)
        dup = np.concatenate([base] * 3 + [base[:1]] * 3)[:n]
        cases["dup"] = orc.pack_bits(dup)
        for name, A in cases.items():
            ref = orc.ple(A, n, m)
            got = gpu_decompose(g, A, n, m)
            assert_same_ple(got, ref, (name, n, m, k))


@pytest.mark.parametrize("s", [2, 5, 21])
def test_decompose_spread_pivots(g, orc, s):
    """Only every s-th column is nonzero, so a sub-panel holds about 64 / s
    pivots and a 64-column word of L gathers its columns from about s
    sub-panels (2: the listed-segment path of the L extraction; 5 and 21: more
    segments than it lists, the per-row walk)."""
    n, m = 1500, 3000
    say("spread pivots", s)
    bits = orc.unpack_bits(synth.dense(40 + s, 1, n, m), m)
    bits[:, np.arange(m) % s != 0] = 0
    A = orc.pack_bits(bits)
    ref = orc.ple(A, n, m)
    got = gpu_decompose(g, A, n, m)
    assert_same_ple(got, ref, s)


def test_decompose_paired_columns(g, orc):
    """Columns in identical pairs: every 64-column sub-panel holds exactly 32
    pivots, so each product's inner words have rows 0..31 only and the table
    steps of rows 32..63 are skipped."""
    n, m = 3000, 5000
    say("paired columns")
    bits = orc.unpack_bits(synth.dense(61, 1, n, m), m)
    bits[:, 1::2] = bits[:, 0::2][:, :bits[:, 1::2].shape[1]]
    A = orc.pack_bits(bits)
    ref = orc.ple(A, n, m)
    assert ref["rank"] == m // 2
    got = gpu_decompose(g, A, n, m)
    assert_same_ple(got, ref, "paired")


@pytest.mark.parametrize("w", [1, 2, 5])
def test_decompose_input_layouts(g, orc, w):
    n, m = 900, 1000
    say("layout", w)
    A = synth.dense(8, 1, n, m)
    ref = orc.ple(A, n, m)
    got = gpu_decompose(g, A, n, m, w=w)
    assert_same_ple(got, ref, w)


def test_decompose_repeatable(g, orc):
    """Bit-exact repeat runs (a race in LDS or in the row lists would show here)."""
    n, m = 1500, 1500
    A = synth.dense(99, 1, n, m)
    first = gpu_decompose(g, A, n, m)
    for _ in range(3):
        again = gpu_decompose(g, A, n, m)
        assert_same_ple(again, first, "repeat")


@pytest.mark.parametrize("kind,n,m", [("dense", 2048, 2048), ("planted", 1500, 2200), ("dense", 3000, 500),
                                      ("dense", 1, 700), ("dense", 70, 5000), ("dense", 1000, 1001),
                                      ("planted", 700, 20000), ("sparse", 300, 9000), ("lead_zero", 130, 6000)])
def test_rank_parity(g, orc, kind, n, m):
    """Rank against the oracle.  Wider than tall matrices are factored as their
    transpose (rank A = rank A^T): ragged edges, planted rank, sparse, and pivots
    only in the last columns (the first 5000 columns zero)."""
    import torch

    say("rank", kind, n, m)
    if kind == "dense":
        A = synth.dense(3, 1, n, m)
    elif kind == "planted":
        A = planted_words(orc, 3, n, m, min(n, m) // 2)
    elif kind == "sparse":
        A = synth.bernoulli(3, 2, n, m, 0.001)
    else:
        bits = orc.unpack_bits(synth.dense(3, 3, n, m), m)
        bits[:, :5000] = 0
        A = orc.pack_bits(bits)
    r = torch.empty(1, dtype=torch.int64, device="cuda")
    g.gf2_rank(g.Mat.from_rowmajor(A, n, m), r)
    assert int(r.item()) == orc.rank(A, n, m)


# ---------------------------------------------------------------- solve
@pytest.mark.parametrize("kind,n,m,k", [("dense", 2048, 2048, 1), ("dense", 1000, 700, 64),
                                        ("dense", 700, 1000, 70), ("planted", 1200, 1200, 130),
                                        ("planted", 300, 900, 5)])
def test_solve_parity(g, orc, kind, n, m, k):
    say("solve", kind, n, m, k)
    A = synth.dense(4, 1, n, m) if kind == "dense" else planted_words(orc, 4, n, m, min(n, m) // 2)
    B = synth.dense(4, 2, n, k)
    # half of the systems consistent by construction: b = A x0
    x0 = synth.dense(4, 3, m, k)
    AX = orc.matmul(A, x0, n, m, k)
    bits = orc.unpack_bits(B, k)
    bits[:, ::2] = orc.unpack_bits(AX, k)[:, ::2]
    B = orc.pack_bits(bits)
    ref = orc.solve(A, B, n, m, k)
    out = g.solve(g.Mat.from_rowmajor(A, n, m), g.Mat.from_rowmajor(B, n, k))
    import torch

    torch.cuda.synchronize()
    assert int(out["rank"].item()) == ref["rank"]
    assert np.array_equal(out["consistent"].cpu().numpy().view(np.uint64), ref["consistent"])
    assert np.array_equal(out["X"].to_rowmajor(), ref["X"])


def test_errors_are_reported(g):
    import torch

    A = g.Mat.zeros(10, 20)
    B = g.Mat.zeros(30, 5)
    C = g.Mat.zeros(10, 5)
    with pytest.raises(g.Gf2Error):
        g.gf2_matmul(C, A, B)
    with pytest.raises(g.Gf2Error):
        g.gf2_set_param("panel_words", 99)
    r = torch.empty(1, dtype=torch.int64, device="cuda")
    g.gf2_rank(A, r)
    assert int(r.item()) == 0
