"""The unit microbenchmarks run on the device and report plausible rates:
positive and below twice the nominal ceilings the bench compares them with."""
import sys

import pytest

pytestmark = pytest.mark.gpu

NOMINAL = {  # per second: bytes, operations or multiply-accumulates
    "hbm_read": 8.0e12, "hbm_copy": 8.0e12, "valu_xor32": 78.6e12, "lds_read": 157.3e12,
    "mfma_int8": 2.5e15, "mfma_fp4": 5.05e15,
}


@pytest.fixture(scope="module")
def g():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1209_5198_amd import gf2

    gf2.load()
    return gf2


@pytest.mark.parametrize("kind,kw", [("hbm_read", dict(nbytes=256 << 20)), ("hbm_copy", dict(nbytes=256 << 20)),
                                     ("valu_xor32", dict(iters=64)), ("lds_read", dict(iters=64)),
                                     ("mfma_int8", dict(iters=256)), ("mfma_fp4", dict(iters=256))])
def test_microbench_rates(g, kind, kw):
    print("microbench", kind, kw, flush=True)
    sys.stdout.flush()
    rate, ms = g.gf2_microbench(kind, **kw)
    assert ms > 0.0
    assert 0.0 < rate < 2.0 * NOMINAL[kind], (kind, rate)
