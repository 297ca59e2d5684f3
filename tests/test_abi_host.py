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
    assert gf2.load().gf2_set_param(b"panel_words", 0) == gf2.GF2_EINVAL
    assert gf2.load().gf2_set_param(b"no_such_knob", 1) == gf2.GF2_EINVAL
    assert b"unknown" in gf2.load().gf2_last_error()
    assert gf2.load().gf2_set_param(b"panel_words", 8) == gf2.GF2_OK


def test_null_descriptor_rejected_without_gpu():
    from paper_1209_5198_amd import gf2

    lib = gf2.load()
    assert lib.gf2_rank(None, None, None) == gf2.GF2_EINVAL
    assert lib.gf2_matmul(None, None, None, 0, None) == gf2.GF2_EINVAL


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
