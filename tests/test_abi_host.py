"""CPU-side checks of the boundary: the library loads, exports every symbol the
header declares, and the binding's layout helpers place words where the
header says (pinned by the worked example of Section 3)."""
import os
import re

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_symbols():
    text = open(os.path.join(ROOT, "include", "gf2.h")).read()
    return sorted(set(re.findall(r"\b(gf2_[a-z_]+)\s*\(", text)))


def test_header_declares_the_abi():
    syms = header_symbols()
    for name in ("gf2_matmul", "gf2_decompose", "gf2_rank", "gf2_solve"):
        assert name in syms


def test_library_exports_every_declared_symbol():
    import ctypes

    from paper_1209_5198_amd import gf2

    if not os.path.exists(gf2.LIB_PATH):
        import __graft_entry__

        __graft_entry__.build()
    lib = ctypes.CDLL(gf2.LIB_PATH)
    for name in header_symbols():
        assert hasattr(lib, name), name
    assert set(gf2.EXPORTED) == set(header_symbols())
    lib.gf2_version.restype = ctypes.c_char_p
    assert lib.gf2_version().startswith(b"libgf2")


def test_set_param_validation_without_gpu():
    from paper_1209_5198_amd import gf2

    gf2.load()
    assert gf2.load().gf2_set_param(b"panel_words", -1) == gf2.GF2_EINVAL
    assert gf2.load().gf2_set_param(b"panel_words", 9) == gf2.GF2_EINVAL
    assert gf2.load().gf2_set_param(b"no_such_knob", 1) == gf2.GF2_EINVAL
    assert b"unknown" in gf2.load().gf2_last_error()
    assert gf2.load().gf2_set_param(b"panel_words", 8) == gf2.GF2_OK
    assert gf2.load().gf2_set_param(b"panel_words", 0) == gf2.GF2_OK  # automatic (the default)
    # tile rule of the trailing update: 0 plain, 1 wall-time always, 2 limited (the default)
    for v in (-1, 3):
        assert gf2.load().gf2_set_param(b"wall_tiles", v) == gf2.GF2_EINVAL
    for v in (0, 1, 2):
        assert gf2.load().gf2_set_param(b"wall_tiles", v) == gf2.GF2_OK


def test_null_descriptor_rejected_without_gpu():
    from paper_1209_5198_amd import gf2

    lib = gf2.load()
    assert lib.gf2_rank(None, None, None) == gf2.GF2_EINVAL
    assert lib.gf2_matmul(None, None, None, 0, None) == gf2.GF2_EINVAL


def test_microbench_validation_without_gpu():
    """Bad kinds, sizes and trip counts are rejected before anything touches the device."""
    import ctypes

    from paper_1209_5198_amd import gf2

    lib = gf2.load()
    rate, ms = ctypes.c_double(), ctypes.c_double()
    r, t = ctypes.byref(rate), ctypes.byref(ms)
    assert lib.gf2_microbench(-1, 0, 1, r, t, None) == gf2.GF2_EINVAL
    assert lib.gf2_microbench(6, 0, 1, r, t, None) == gf2.GF2_EINVAL
    assert lib.gf2_microbench(0, 1000, 0, r, t, None) == gf2.GF2_EINVAL    # not a multiple of 64 KiB
    assert lib.gf2_microbench(1, 0, 0, r, t, None) == gf2.GF2_EINVAL       # empty copy
    assert lib.gf2_microbench(2, 0, 0, r, t, None) == gf2.GF2_EINVAL       # no trips
    assert lib.gf2_microbench(5, 0, 1 << 25, r, t, None) == gf2.GF2_EINVAL
    assert lib.gf2_microbench(3, 0, 1, None, t, None) == gf2.GF2_EINVAL
    assert b"gf2_microbench" in lib.gf2_last_error()
    assert set(gf2.MICROBENCH_KINDS.values()) == set(range(6))


def test_blocked_layout_matches_section3_example():
    """The Section 3 example stores the 4 x 2 word matrix column-major
    (5 1 3 4 | 3 2 1 3).  With b = 64 the same rule is the layout with w = 1:
    word (i, q) at q*ld + i."""
    from paper_1209_5198_amd.gf2 import Mat

    words = np.array([[5, 3], [1, 2], [3, 1], [4, 3]], dtype=np.uint64)
    flat = Mat.blocked_words(words, 4, 128, w=1, ld=4)
    assert flat.tolist() == [5, 1, 3, 4, 3, 2, 1, 3]
    # w = 2 (both words in one block) is plain row-major
    assert Mat.blocked_words(words, 4, 128, w=2, ld=4).tolist() == words.reshape(-1).tolist()
    # ld > rows leaves padding rows inside each block
    flat = Mat.blocked_words(words, 4, 128, w=1, ld=6)
    assert flat.tolist() == [5, 1, 3, 4, 0, 0, 3, 2, 1, 3, 0, 0]


def test_blocked_layout_roundtrip():
    from paper_1209_5198_amd import synth
    from paper_1209_5198_amd.gf2 import Mat

    for rows, cols, w, ld in [(7, 200, 1, 9), (7, 200, 3, 7), (33, 1000, 4, 40), (1, 1, 1, 1)]:
        words = synth.dense(1, 1, rows, cols)
        flat = Mat.blocked_words(words, rows, cols, w, ld)
        nw = (cols + 63) // 64
        nb = (nw + w - 1) // w
        back = flat.reshape(nb, ld, w).transpose(1, 0, 2).reshape(ld, nb * w)[:rows, :nw]
        assert np.array_equal(back, words)
        # the header's formula
        for i in range(rows):
            for q in range(nw):
                assert flat[(q // w) * ld * w + i * w + q % w] == words[i, q]


def test_batched_validation_without_gpu():
    """Host-side checks of the batched entry points reject bad items before any launch."""
    import ctypes

    from paper_1209_5198_amd import gf2

    lib = gf2.load()
    items = (gf2.BatchItem * 2)()
    items[0].rows, items[0].cols = 10, 10
    items[1].rows, items[1].cols = gf2.BATCH_MAX_DIM + 1, 5
    dummy = ctypes.c_void_p(16)
    rc = lib.gf2_decompose_batched(items, 2, dummy, None, None, None, None, dummy, None)
    assert rc == gf2.GF2_EINVAL and b"rows and cols" in lib.gf2_last_error()
    items[1].rows = 5
    items[1].e = -1
    assert lib.gf2_decompose_batched(items, 2, dummy, None, None, None, None, dummy, None) == gf2.GF2_EINVAL
    assert b"negative offset" in lib.gf2_last_error()
    items[1].e = 0
    assert lib.gf2_decompose_batched(items, -1, dummy, None, None, None, None, dummy, None) == gf2.GF2_EINVAL
    assert lib.gf2_decompose_batched(None, 3, dummy, None, None, None, None, dummy, None) == gf2.GF2_EINVAL
    assert lib.gf2_decompose_batched(items, 2, dummy, None, None, None, None, None, None) == gf2.GF2_EINVAL
    assert b"null rank" in lib.gf2_last_error()
    assert lib.gf2_solve_batched(items, 2, dummy, dummy, dummy, dummy, dummy, None, dummy, dummy,
                                 None) == gf2.GF2_EINVAL
    # an empty batch is a valid no-op
    assert lib.gf2_decompose_batched(items, 0, None, None, None, None, None, None, None) == gf2.GF2_OK


def test_batch_offsets_pack_the_pools():
    """The binding's Batch offsets follow the gf2_batch_item layout (no GPU: offsets only)."""
    from paper_1209_5198_amd import gf2

    shapes = [(3, 70), (0, 5), (130, 64), (64, 1)]
    off = dict(a=0, l=0, e=0, p=0, c=0, b=0, x=0)
    want = []
    for n, m in shapes:
        k = min(n, m)
        want.append(dict(off))
        off["a"] += n * gf2.wpr(m)
        off["l"] += n * gf2.wpr(k)
        off["e"] += k * gf2.wpr(m)
        off["p"] += n
        off["c"] += k
        off["b"] += gf2.wpr(n)
        off["x"] += gf2.wpr(m)
    b = gf2.Batch(shapes, device="cpu")
    assert b.off == want and b.size == off
    assert [(it.rows, it.cols, it.a, it.l, it.e) for it in b.items] == [
        (n, m, w["a"], w["l"], w["e"]) for (n, m), w in zip(shapes, want)]


def test_autotune_entry_points_without_gpu():
    from paper_1209_5198_amd import gf2

    lib = gf2.load()
    assert lib.gf2_autotune(100, None) == gf2.GF2_EINVAL
    table, cut = gf2.gf2_autotune_table()
    assert table == [[-1] * 4 for _ in range(9)] and cut == 65536
    assert lib.gf2_set_param(b"autotuned", 2) == gf2.GF2_EINVAL
    assert lib.gf2_set_param(b"autotuned", 1) == gf2.GF2_OK  # no table yet: stays on the rule


def test_inverse_validation_without_gpu():
    """Non-square, empty and mis-shaped inverse calls are rejected before any device work."""
    import ctypes

    from paper_1209_5198_amd import gf2

    lib = gf2.load()
    def desc(rows, cols):  # the data address is never dereferenced: the shapes fail first
        return gf2._Mat(0x1000, rows, cols, 1, max(rows, 1))

    A, X = desc(5, 6), desc(5, 6)
    assert lib.gf2_inverse(ctypes.byref(A), ctypes.byref(X), None, None) == gf2.GF2_EINVAL
    assert b"square" in lib.gf2_last_error()
    A, X = desc(0, 0), desc(0, 0)
    assert lib.gf2_inverse(ctypes.byref(A), ctypes.byref(X), None, None) == gf2.GF2_EINVAL
    A, X = desc(7, 7), desc(7, 8)
    assert lib.gf2_inverse(ctypes.byref(A), ctypes.byref(X), None, None) == gf2.GF2_EINVAL
    assert b"X must be" in lib.gf2_last_error()
    assert lib.gf2_inverse(None, None, None, None) == gf2.GF2_EINVAL


def test_header_compiles_as_plain_c_and_cpp(tmp_path):
    """include/gf2.h is plain C: it compiles with gcc -std=c99 and with g++,
    neither of which sees a HIP header."""
    import shutil
    import subprocess

    src_c = tmp_path / "use.c"
    src_c.write_text('#include "gf2.h"\nint main(void) { gf2_mat m; (void)m; return (int)gf2_workspace_bytes(0, 0, 0, 0); }\n')
    inc = os.path.join(ROOT, "include")
    for cc, std, src in (("gcc", "-std=c99", src_c), ("g++", "-std=c++11", src_c)):
        exe = shutil.which(cc)
        assert exe, cc
        cmd = [exe, std, "-Wall", "-Werror", "-pedantic", "-fsyntax-only", "-I", inc]
        if cc == "g++":
            cmd += ["-x", "c++"]
        r = subprocess.run(cmd + [str(src)], capture_output=True, text=True)
        assert r.returncode == 0, (cc, r.stderr)


def test_workspace_bytes_without_gpu():
    """Sizes of the caller workspace: the working copy in 16-word column blocks
    plus the per-panel state, exact growth with the matrix, and invalid requests."""
    from paper_1209_5198_amd import gf2

    lib = gf2.load()
    d = gf2.gf2_workspace_bytes(gf2.OP_DECOMPOSE, 16384, 16384)
    assert 32 * 2 ** 20 <= d < 34 * 2 ** 20, d
    assert gf2.gf2_workspace_bytes(gf2.OP_DECOMPOSE, 0, 100) == 0
    assert gf2.gf2_workspace_bytes(gf2.OP_RANK, 0, 100) == 0
    # a wide matrix is factored as its transpose
    assert gf2.gf2_workspace_bytes(gf2.OP_RANK, 1000, 70000) == gf2.gf2_workspace_bytes(gf2.OP_DECOMPOSE, 70000, 1000)
    s1 = gf2.gf2_workspace_bytes(gf2.OP_SOLVE, 4096, 4096, 1)
    s2 = gf2.gf2_workspace_bytes(gf2.OP_SOLVE, 4096, 4096, 200)
    assert s2 - s1 == 4096 * 8 * 3  # four words of right-hand sides per row instead of one
    assert gf2.gf2_workspace_bytes(gf2.OP_SOLVE_BATCHED, 10, 0) >= 10 * 64
    assert gf2.gf2_workspace_bytes(gf2.OP_MATMUL, 300, 200, 100) > 0
    for args in ((99, 1, 1, 1), (gf2.OP_DECOMPOSE, -1, 5, 0)):
        assert lib.gf2_workspace_bytes(*args) == gf2.SIZE_MAX
    assert lib.gf2_workspace_bytes(gf2.OP_DECOMPOSE_BATCHED, 4, 4096, 64) == gf2.SIZE_MAX  # above the batch limit


def test_caller_workspace_validation_without_gpu():
    """A *_ws call rejects a null, misaligned or short workspace before any launch."""
    import ctypes

    from paper_1209_5198_amd import gf2

    lib = gf2.load()
    fake = ctypes.c_void_p(1 << 40)  # never dereferenced: the call fails on the host first
    A = gf2._Mat(fake, 64, 64, 1, 64)
    need = gf2.gf2_workspace_bytes(gf2.OP_DECOMPOSE, 64, 64)
    for ws, nb, what in ((None, need, b"null"), (ctypes.c_void_p((1 << 40) + 8), need, b"aligned"),
                         (fake, need - 256, b"needed")):
        assert lib.gf2_decompose_ws(ctypes.byref(A), None, None, None, None, fake, ws, nb, None) == gf2.GF2_EINVAL
        assert what in lib.gf2_last_error(), lib.gf2_last_error()
        assert lib.gf2_rank_ws(ctypes.byref(A), fake, ws, nb, None) == gf2.GF2_EINVAL
    assert lib.gf2_set_param(b"chain_cus", 8) == gf2.GF2_EINVAL
    assert lib.gf2_set_param(b"chain_cus", 0) == gf2.GF2_OK


def test_autotune_params_analytic_choices():
    """gf2_autotune_params reports the paper's analytic choices (Section 6): the
    table size minimising C(b, c, n) = (b/c)(2^c - 1 + n) -- the Remark there
    puts the continuous minimum of C(64, c, 64) near 4.77 and of C(128, c,
    128) near 5.5 -- and the Strassen point 44c + 6(2^c - 1) = 1882 at c = 8."""
    from paper_1209_5198_amd import gf2

    lib = gf2.load()
    try:
        assert lib.gf2_set_param(b"panel_words", 1) == gf2.GF2_OK  # b = 64
        p = gf2.gf2_autotune_params(64, 64)
        assert p["panel_words"] == 1 and p["table_bits"] == 8 and p["analytic_strassen"] == 1882
        assert p["analytic_table_bits"] == 5  # integer neighbour of 4.77
        assert lib.gf2_set_param(b"panel_words", 2) == gf2.GF2_OK  # b = 128
        assert gf2.gf2_autotune_params(128, 128)["analytic_table_bits"] in (5, 6)  # either side of 5.5
        # larger products: the minimum moves up like log2(n)
        assert gf2.gf2_autotune_params(65536, 65536)["analytic_table_bits"] > \
            gf2.gf2_autotune_params(2048, 2048)["analytic_table_bits"]
        assert lib.gf2_set_param(b"panel_words", 0) == gf2.GF2_OK
        assert gf2.gf2_autotune_params(2048, 2048)["panel_words"] == 8  # untuned default
        assert lib.gf2_autotune_params(-1, 5, None, None, None, None) == gf2.GF2_EINVAL
    finally:
        lib.gf2_set_param(b"panel_words", 0)
