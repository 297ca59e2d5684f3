"""GPU checks of the continuous-batching request loop.

A stream of rank / solve / decompose requests of mixed sizes (both below and
above the batched-kernel limit) arrives faster than it is served, under an
admission cap small enough that requests must wait for memory.  Every result
must equal (a) the same request computed alone through the C ABI and (b) the
CPU oracle; the run must have batched several requests into one launch and
overlapped a large request with a batched launch.
"""
import concurrent.futures
import sys

import numpy as np
import pytest

from paper_1209_5198_amd import synth

pytestmark = pytest.mark.gpu
wpr = synth.wpr


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


def bits_to_col(v, n):
    out = np.zeros((n, 1), dtype=np.uint64)
    idx = np.arange(n)
    out[:, 0] = (v[idx >> 6] >> (idx & 63).astype(np.uint64)) & np.uint64(1)
    return out


def col_to_bits(X, m):
    out = np.zeros(wpr(m), dtype=np.uint64)
    for j in np.nonzero(X[:m, 0] & np.uint64(1))[0]:
        out[j >> 6] |= np.uint64(1) << np.uint64(j & 63)
    return out


def alone(g, r, A):
    """The request computed by itself through the C ABI (batch of one or a single call)."""
    import torch

    n, m = r.n, r.m
    if r.small:
        b = g.Batch([(n, m)])
        b.set_matrices([A])
        if r.kind == "solve":
            b.set_rhs([r.b_bits])
        b.decompose(want_le=r.kind != "rank")
        if r.kind == "solve":
            b.solve()
        torch.cuda.synchronize()
        res = b.result(0)
    else:
        M = g.Mat.from_rowmajor(A, n, m)
        if r.kind == "rank":
            rank = torch.empty(1, dtype=torch.int64, device="cuda")
            g.gf2_rank(M, rank)
            res = dict(rank=int(rank.item()))
        elif r.kind == "decompose":
            out = g.decompose(M)
            res = dict(rank=int(out["rank"].item()), perm=out["perm"].cpu().numpy(),
                       pivcols=out["pivcols"].cpu().numpy(), L=out["L"].to_rowmajor(), E=out["E"].to_rowmajor())
        else:
            out = g.solve(M, g.Mat.from_rowmajor(bits_to_col(r.b_bits, n), n, 1))
            res = dict(rank=int(out["rank"].item()), x=col_to_bits(out["X"].to_rowmajor(), m),
                       consistent=int(out["consistent"][0].item()) & 1)
    return res


def oracle(orc, r, A):
    orc.set_threads(1)
    n, m = r.n, r.m
    if r.kind == "solve":
        sol = orc.solve(A, bits_to_col(r.b_bits, n), n, m, 1)
        return dict(rank=sol["rank"], x=col_to_bits(sol["X"], m), consistent=int(sol["consistent"][0]) & 1)
    res = orc.ple(A, n, m)
    if r.kind == "rank":
        return dict(rank=res["rank"])
    res["L"] = res["L"][:, :wpr(min(n, m))]
    return res


def same(a, b, kind):
    keys = {"rank": ("rank",), "solve": ("x", "consistent"), "decompose": ("rank", "perm", "pivcols", "L", "E")}[kind]
    for k in keys:
        x, y = a[k], b[k]
        if isinstance(x, np.ndarray) or isinstance(y, np.ndarray):
            if not np.array_equal(np.asarray(x), np.asarray(y)):
                return False
        elif x != y:
            return False
    return True


def test_serving_mix_equals_alone_and_oracle(g, orc):
    from paper_1209_5198_amd import serve

    seed, count = 77, 60
    specs = synth.serving_specs(seed, count, lo=64, hi=3200)
    arrivals = synth.poisson_arrivals(seed, count, 3000.0)
    data = serve.make_request_data(seed, specs)
    reqs = serve.make_requests(specs, data, arrivals)
    srv = serve.Server(cap_bytes=24 << 20, big_streams=2, verify=True)
    st = srv.run(reqs)
    say("serving stats", st)
    assert st["max_batch"] > 1, "no request joined a running stream of small work"
    assert st["small"] > 0 and st["large"] > 0
    # a large request ran while a batched launch was on the GPU
    wins = {}
    for r in reqs:
        if r.small:
            w = wins.setdefault(r.batch_id, [r.t_start, r.t_done])
            w[1] = max(w[1], r.t_done)
    big = [r for r in reqs if not r.small]
    assert any(b.t_start < w[1] and w[0] < b.t_done for b in big for w in wins.values())
    buf, offs, _ = data
    host = buf.numpy().view(np.uint64)
    mats = [host[offs[i]:offs[i + 1]].reshape(s["n"], wpr(s["m"])) for i, s in enumerate(specs)]
    with concurrent.futures.ThreadPoolExecutor(16) as ex:
        refs = list(ex.map(lambda i: oracle(orc, reqs[i], mats[i]), range(count)))
    bad = []
    for i, r in enumerate(reqs):
        a = alone(g, r, mats[i])
        if not same(r.result, a, r.kind):
            bad.append(("alone", r.id, r.kind, r.n, r.m))
        if not same(r.result, refs[i], r.kind):
            bad.append(("oracle", r.id, r.kind, r.n, r.m))
    assert not bad, bad[:10]


def test_serving_full_size_range(g, orc):
    """Requests at the serving workload's real sizes (sides 128..16384, square and
    1:4): every result equals the request alone; a sample that includes the largest
    requests equals the oracle."""
    from paper_1209_5198_amd import serve

    seed, count = 5, 64
    specs = synth.serving_specs(seed, count)
    arrivals = synth.poisson_arrivals(seed, count, 400.0)
    data = serve.make_request_data(seed, specs)
    reqs = serve.make_requests(specs, data, arrivals)
    srv = serve.Server(cap_bytes=8 << 30, big_streams=4, verify=True)
    st = srv.run(reqs)
    say("serving full-size stats", {k: st[k] for k in ("requests_per_s", "p50_ms", "p99_ms", "small", "large")})
    buf, offs, _ = data
    host = buf.numpy().view(np.uint64)
    mats = [host[offs[i]:offs[i + 1]].reshape(s["n"], wpr(s["m"])) for i, s in enumerate(specs)]
    bad = []
    for i, r in enumerate(reqs):
        if not same(r.result, alone(g, r, mats[i]), r.kind):
            bad.append(("alone", r.id, r.kind, r.n, r.m))
    order = sorted(range(count), key=lambda i: -specs[i]["n"] * specs[i]["m"])
    sample = sorted(set(order[:6]) | set(range(0, count, 6)))
    with concurrent.futures.ThreadPoolExecutor(8) as ex:
        refs = dict(zip(sample, ex.map(lambda i: oracle_mt(orc, reqs[i], mats[i]), sample)))
    for i in sample:
        if not same(reqs[i].result, refs[i], reqs[i].kind):
            bad.append(("oracle", reqs[i].id, reqs[i].kind, reqs[i].n, reqs[i].m))
    assert not bad, bad[:10]


def oracle_mt(orc, r, A):
    """The oracle with two threads per call (large requests)."""
    orc.set_threads(2)
    n, m = r.n, r.m
    if r.kind == "solve":
        sol = orc.solve(A, bits_to_col(r.b_bits, n), n, m, 1)
        return dict(rank=sol["rank"], x=col_to_bits(sol["X"], m), consistent=int(sol["consistent"][0]) & 1)
    res = orc.ple(A, n, m)
    if r.kind == "rank":
        return dict(rank=res["rank"])
    res["L"] = res["L"][:, :wpr(min(n, m))]
    return res
