"""Continuous-batching request loop for GF(2) rank / solve / decompose on one GPU.

Requests of mixed sizes arrive over time with their matrix (and right-hand
side) in host memory.  The loop:

* **admits** requests in arrival order by HBM footprint: every admitted request
  gets its input, outputs and (for a single-matrix call) the library workspace
  of that call carved from one device arena whose size is the admission cap, so
  admission is allocation and a request waits until its footprint fits; its
  data is copied to the device on a copy stream as soon as it is admitted;
* **batches continuously**: whenever the batch stream is idle, every admitted
  small request (both sides at most GF2_BATCH_MAX_DIM) whose data has arrived
  is packed into one gf2_decompose_batched launch (rank requests in a second,
  output-free one) followed by one gf2_solve_batched launch for the solve
  requests, their workspace carved from the arena for the batch's lifetime;
  requests that arrive meanwhile join the next launch;
* runs each **large** request as one call (gf2_rank_ws / gf2_decompose_ws /
  gf2_solve_ws, with the workspace from its own arena block) on one of a few
  side streams, so large and small work overlap on the device;

Every byte of device memory the library works in comes from the arena, so the
admission cap bounds the device memory of the whole loop (the library's
per-stream look-ahead streams and events hold no buffers).
* detects completion with HIP events and frees the request's memory; latency
  is completion time minus arrival time.

Concurrency of the side streams needs enough hardware queues: each large call
runs on its own pair of pipeline streams (libgf2 keys them by caller stream),
and with HIP's default of 4 queues per process, unrelated streams that share
a queue wait for each other.  Processes that serve should start the HIP
runtime with GPU_MAX_HW_QUEUES raised (16 measured best with 4 side streams).

All arithmetic runs in libgf2's kernels; this module only schedules.
"""
from __future__ import annotations

import collections
import time
from dataclasses import dataclass, field

import numpy as np

from . import gf2

wpr = gf2.wpr
GRANULE = 32  # words (256 bytes)


class Arena:
    """First-fit allocator of 64-bit words inside one device tensor."""

    def __init__(self, words: int, device="cuda"):
        self.cap = int(words) // GRANULE * GRANULE
        self.t = None  # bookkeeping only (no device memory) when device is None
        if device is not None:
            import torch

            self.t = torch.empty(max(self.cap, GRANULE), dtype=torch.int64, device=device)
        self.free = [(0, self.cap)]
        self.used = 0
        self.peak = 0

    @staticmethod
    def size(words: int) -> int:
        return max(GRANULE, (int(words) + GRANULE - 1) // GRANULE * GRANULE)

    def alloc(self, words: int):
        w = self.size(words)
        for i, (o, s) in enumerate(self.free):
            if s >= w:
                if s == w:
                    del self.free[i]
                else:
                    self.free[i] = (o + w, s - w)
                self.used += w
                self.peak = max(self.peak, self.used)
                return o
        return None

    def release(self, off: int, words: int):
        w = self.size(words)
        self.used -= w
        fl = self.free
        lo, hi = 0, len(fl)
        while lo < hi:
            mid = (lo + hi) // 2
            if fl[mid][0] < off:
                lo = mid + 1
            else:
                hi = mid
        fl.insert(lo, (off, w))
        if lo + 1 < len(fl) and fl[lo][0] + fl[lo][1] == fl[lo + 1][0]:  # merge right
            fl[lo] = (fl[lo][0], fl[lo][1] + fl[lo + 1][1])
            del fl[lo + 1]
        if lo > 0 and fl[lo - 1][0] + fl[lo - 1][1] == fl[lo][0]:  # merge left
            fl[lo - 1] = (fl[lo - 1][0], fl[lo - 1][1] + fl[lo][1])
            del fl[lo]


@dataclass
class Request:
    id: int
    kind: str            # "rank", "solve" or "decompose"
    n: int
    m: int
    arrival: float       # seconds from the start of the session
    A: object            # host words, n x wpr(m) (numpy uint64 or pinned torch int64)
    b_bits: object = None  # solve: wpr(n) words, bit i = entry i
    small: bool = False
    off: dict = field(default_factory=dict)
    span: int = 0        # arena words of this request (one block)
    base: int = 0
    ready_ev: object = None
    t_admit: float = 0.0
    t_start: float = 0.0
    t_done: float = 0.0
    batch_id: int = -1
    result: dict = None


def _layout(r: Request):
    """Word offsets (relative to the request's block) of every piece it needs."""
    n, m = r.n, r.m
    k = min(n, m)
    parts = [("A", n * wpr(m))]
    if r.kind in ("decompose", "solve") and r.small:
        parts += [("L", n * wpr(k)), ("E", k * wpr(m)), ("perm", n), ("pivcols", k)]
    if r.kind == "decompose" and not r.small:
        parts += [("L", n * wpr(k)), ("E", k * wpr(m)), ("perm", n), ("pivcols", k)]
    if r.kind == "solve":
        parts += [("b", wpr(n)), ("x", wpr(m))] if r.small else [("b", n), ("x", m)]
    parts += [("rank", 1), ("cons", 1)]
    if not r.small:  # the single-matrix call's library workspace, carved from the block
        op = {"rank": gf2.OP_RANK, "decompose": gf2.OP_DECOMPOSE, "solve": gf2.OP_SOLVE}[r.kind]
        parts += [("ws", (gf2.gf2_workspace_bytes(op, n, m, 1 if r.kind == "solve" else 0) + 7) // 8)]
    off, pos = {}, 0
    for name, w in parts:
        off[name] = pos
        pos += Arena.size(w)
    return off, pos


def _batch_ws_words(groups) -> int:
    """Arena words of the workspace the launches of one batch need (they run in
    order on one stream, so they share it): groups = lists of (rows, cols)."""
    need = 0
    for shapes, op in groups:
        if not shapes:
            continue
        cnt = len(shapes)
        if op == gf2.OP_DECOMPOSE_BATCHED:
            b = gf2.gf2_workspace_bytes(op, cnt, max(m for _, m in shapes), max(n for n, _ in shapes))
        else:
            b = gf2.gf2_workspace_bytes(op, cnt, 0, 0)
        need = max(need, b)
    return (need + 7) // 8


class Server:
    """One GPU, one arena of `cap_bytes`, one batch stream and `big_streams` side streams."""

    def __init__(self, cap_bytes: int = 64 << 30, big_streams: int = 4, verify: bool = False, device="cuda"):
        import torch

        self.torch = torch
        self.arena = Arena(cap_bytes // 8, device)
        self.copy = torch.cuda.Stream(device=device)
        self.sb = torch.cuda.Stream(device=device)
        self.sl = [torch.cuda.Stream(device=device) for _ in range(big_streams)]
        self.verify = verify
        self.batches = []  # sizes of the batched launches

    # ---------------------------------------------------------------- memory
    def _admit(self, r: Request) -> bool:
        off, span = _layout(r)
        if span > self.arena.cap:
            raise ValueError(f"request {r.id} ({r.n} x {r.m}) exceeds the admission cap")
        base = self.arena.alloc(span)
        if base is None:
            return False
        r.base, r.span, r.off = base, span, off
        t = self.arena.t
        with self.torch.cuda.stream(self.copy):
            a = r.A if hasattr(r.A, "data_ptr") else self.torch.from_numpy(np.ascontiguousarray(r.A).view(np.int64))
            nw = r.n * wpr(r.m)
            if nw:
                t[base + off["A"]:base + off["A"] + nw].copy_(a.reshape(-1)[:nw], non_blocking=True)
            if r.kind == "solve":
                bb = self._rhs_words(r)
                t[base + off["b"]:base + off["b"] + bb.numel()].copy_(bb, non_blocking=True)
            ev = self.torch.cuda.Event()
            ev.record(self.copy)
        r.ready_ev = ev
        return True

    def _rhs_words(self, r: Request):
        """Right-hand side in the layout of the path that serves r."""
        bits = np.ascontiguousarray(r.b_bits, dtype=np.uint64)
        if r.small:
            return self.torch.from_numpy(bits.view(np.int64).copy())
        col = np.zeros(max(r.n, 1), dtype=np.uint64)
        idx = np.arange(r.n)
        col[:r.n] = (bits[idx >> 6] >> (idx & 63).astype(np.uint64)) & np.uint64(1)
        return self.torch.from_numpy(col[:max(r.n, 1)].view(np.int64).copy())

    def _release(self, r: Request):
        self.arena.release(r.base, r.span)

    # ---------------------------------------------------------------- launches
    def _mat(self, r, key, rows, cols):
        o = r.base + r.off[key]
        return gf2.Mat(self.arena.t[o:o + max(rows * wpr(cols), 1)], rows, cols, max(wpr(cols), 1), max(rows, 1))

    def _launch_large(self, r: Request, s):
        t = self.arena.t
        o = r.base
        A = self._mat(r, "A", r.n, r.m)
        rank = t[o + r.off["rank"]:o + r.off["rank"] + 1]
        ws = t[o + r.off["ws"]:o + r.span]
        if r.kind == "rank":
            gf2.gf2_rank_ws(A, rank, ws, s)
        elif r.kind == "decompose":
            k = min(r.n, r.m)
            gf2.gf2_decompose_ws(A, self._mat(r, "L", r.n, k), self._mat(r, "E", k, r.m),
                                 t[o + r.off["perm"]:], t[o + r.off["pivcols"]:], rank, ws, s)
        else:
            B = gf2.Mat(t[o + r.off["b"]:o + r.off["b"] + max(r.n, 1)], r.n, 1, 1, max(r.n, 1))
            X = gf2.Mat(t[o + r.off["x"]:o + r.off["x"] + max(r.m, 1)], r.m, 1, 1, max(r.m, 1))
            cons = t[o + r.off["cons"]:o + r.off["cons"] + 1]
            gf2.gf2_solve_ws(A, B, X, cons, rank, ws, s)
        ev = self.torch.cuda.Event()
        ev.record(s)
        return ev

    def _items(self, reqs, with_out):
        items = (gf2.BatchItem * len(reqs))()
        for j, r in enumerate(reqs):
            it = items[j]
            it.rows, it.cols = r.n, r.m
            it.a = r.base + r.off["A"]
            if with_out:
                it.l, it.e = r.base + r.off["L"], r.base + r.off["E"]
                it.p, it.c = r.base + r.off["perm"], r.base + r.off["pivcols"]
            if r.kind == "solve":
                it.b, it.x = r.base + r.off["b"], r.base + r.off["x"]
        return items

    def _launch_batch(self, reqs, s):
        """Launch one batch: (event, outputs), or None while its block does not fit.
        The block holds the library workspace of its launches (they run in order
        on one stream, so they share it) and the per-item ranks and flags."""
        torch = self.torch
        t = self.arena.t
        solve = [r for r in reqs if r.kind == "solve"]
        full = solve + [r for r in reqs if r.kind == "decompose"]
        ranko = [r for r in reqs if r.kind == "rank"]
        sh = lambda rs: [(r.n, r.m) for r in rs]  # noqa: E731
        ws_words = _batch_ws_words([(sh(full), gf2.OP_DECOMPOSE_BATCHED), (sh(solve), gf2.OP_SOLVE_BATCHED),
                                    (sh(ranko), gf2.OP_DECOMPOSE_BATCHED)])
        o_rank = Arena.size(ws_words)
        o_rank2 = o_rank + Arena.size(len(full))
        o_cons = o_rank2 + Arena.size(len(ranko))
        total = o_cons + Arena.size((len(solve) + 1) // 2)
        base = self.arena.alloc(total)
        if base is None:
            return None
        ws = t[base:base + o_rank]
        out = {"block": (base, total)}
        if full:
            items = self._items(full, True)
            rank = t[base + o_rank:base + o_rank + len(full)]
            gf2.gf2_decompose_batched_ws(items, t, t, t, t, t, rank, ws, s)
            out["full"] = (full, rank)
            if solve:  # the solve requests lead `full`, so rank[j] is theirs
                cons = t[base + o_cons:base + o_cons + (len(solve) + 1) // 2].view(torch.int32)[:len(solve)]
                gf2.gf2_solve_batched_ws(self._items(solve, True), t, t, t, t, rank, t, t, cons, ws, s)
                out["cons"] = cons
        if ranko:
            rank2 = t[base + o_rank2:base + o_rank2 + len(ranko)]
            gf2.gf2_decompose_batched_ws(self._items(ranko, False), t, None, None, None, None, rank2, ws, s)
            out["rank"] = (ranko, rank2)
        ev = torch.cuda.Event()
        ev.record(s)
        self.batches.append(len(reqs))
        return ev, out

    def _launch_fitting_batch(self, ready, s):
        """The largest leading part of `ready` (halving) whose batch block fits."""
        k = len(ready)
        while k >= 1:
            launched = self._launch_batch(ready[:k], s)
            if launched is not None:
                return ready[:k], launched
            k //= 2
        return [], None

    # ---------------------------------------------------------------- results (verify mode)
    def _fetch_large(self, r):
        t = self.arena.t
        o = r.base
        res = dict(rank=int(t[o + r.off["rank"]].item()))
        if r.kind == "decompose":
            k = min(r.n, r.m)
            res["L"] = self._mat(r, "L", r.n, k).to_rowmajor()
            res["E"] = self._mat(r, "E", k, r.m).to_rowmajor()
            res["perm"] = t[o + r.off["perm"]:o + r.off["perm"] + r.n].cpu().numpy()
            res["pivcols"] = t[o + r.off["pivcols"]:o + r.off["pivcols"] + k].cpu().numpy()
        elif r.kind == "solve":
            col = t[o + r.off["x"]:o + r.off["x"] + r.m].cpu().numpy().view(np.uint64) & np.uint64(1)
            x = np.zeros(wpr(r.m), dtype=np.uint64)
            for j in np.nonzero(col)[0]:
                x[j >> 6] |= np.uint64(1) << np.uint64(j & 63)
            res["x"] = x
            res["consistent"] = int(t[o + r.off["cons"]].item()) & 1
        return res

    def _fetch_small(self, r, rank_val, cons_val):
        t = self.arena.t
        o = r.base
        res = dict(rank=int(rank_val))
        if r.kind == "decompose":
            k = min(r.n, r.m)
            res["L"] = t[o + r.off["L"]:o + r.off["L"] + r.n * wpr(k)].cpu().numpy().view(np.uint64).reshape(r.n, wpr(k))
            res["E"] = t[o + r.off["E"]:o + r.off["E"] + k * wpr(r.m)].cpu().numpy().view(np.uint64).reshape(k, wpr(r.m))
            res["perm"] = t[o + r.off["perm"]:o + r.off["perm"] + r.n].cpu().numpy()
            res["pivcols"] = t[o + r.off["pivcols"]:o + r.off["pivcols"] + k].cpu().numpy()
        elif r.kind == "solve":
            res["x"] = t[o + r.off["x"]:o + r.off["x"] + wpr(r.m)].cpu().numpy().view(np.uint64).copy()
            res["consistent"] = int(cons_val)
        return res

    # ---------------------------------------------------------------- the loop
    def run(self, requests, small_max: int = gf2.BATCH_MAX_DIM):
        """Serve `requests` (sorted by arrival); returns a statistics dict."""
        for r in requests:
            r.small = max(r.n, r.m) <= small_max
        reqs = sorted(requests, key=lambda r: r.arrival)
        N = len(reqs)
        pending = collections.deque()
        waiting_small, waiting_large = [], collections.deque()
        batch = None                       # (event, out, requests, t_start)
        large = [None] * len(self.sl)      # (event, request)
        done = 0
        nxt = 0
        self.torch.cuda.synchronize()
        t0 = time.perf_counter()
        while done < N:
            now = time.perf_counter() - t0
            while nxt < N and reqs[nxt].arrival <= now:
                pending.append(reqs[nxt])
                nxt += 1
            while pending and self._admit(pending[0]):
                r = pending.popleft()
                r.t_admit = time.perf_counter() - t0
                (waiting_small if r.small else waiting_large).append(r)
            progressed = False
            # batch stream
            if batch is not None and batch[0].query():
                tdone = time.perf_counter() - t0
                ev, out, members, _ = batch
                if self.verify:
                    self._collect_batch(out)
                self.arena.release(*out["block"])
                for r in members:
                    r.t_done = tdone
                    self._release(r)
                done += len(members)
                batch = None
                progressed = True
            if batch is None and waiting_small:
                flags = [r.ready_ev.query() for r in waiting_small]
                ready = [r for r, f in zip(waiting_small, flags) if f]
                ready, launched = self._launch_fitting_batch(ready, self.sb) if ready else ([], None)
                if launched is not None:
                    taken = set(id(r) for r in ready)
                    waiting_small = [r for r in waiting_small if id(r) not in taken]
                    ts = time.perf_counter() - t0
                    bid = len(self.batches) - 1
                    for r in ready:
                        r.t_start, r.batch_id = ts, bid
                    ev, out = launched
                    batch = (ev, out, ready, ts)
                    progressed = True
            # side streams
            for j, s in enumerate(self.sl):
                if large[j] is not None and large[j][0].query():
                    r = large[j][1]
                    r.t_done = time.perf_counter() - t0
                    if self.verify:
                        r.result = self._fetch_large(r)
                    self._release(r)
                    done += 1
                    large[j] = None
                    progressed = True
                if large[j] is None and waiting_large and waiting_large[0].ready_ev.query():
                    r = waiting_large.popleft()
                    r.t_start = time.perf_counter() - t0
                    large[j] = (self._launch_large(r, s), r)
                    progressed = True
            if not progressed:
                time.sleep(20e-6)
        return self.stats(reqs)

    def _collect_batch(self, out):
        if "full" in out:
            full, rank = out["full"]
            rv = rank.cpu().numpy()
            cons = out["cons"].cpu().numpy() if "cons" in out else None
            for j, r in enumerate(full):
                r.result = self._fetch_small(r, rv[j], cons[j] if (cons is not None and r.kind == "solve") else 0)
        if "rank" in out:
            ranko, rank2 = out["rank"]
            rv = rank2.cpu().numpy()
            for j, r in enumerate(ranko):
                r.result = dict(rank=int(rv[j]))

    def stats(self, reqs):
        lat = np.array([r.t_done - r.arrival for r in reqs]) if reqs else np.zeros(0)
        t_first = min(r.arrival for r in reqs) if reqs else 0.0
        t_last = max(r.t_done for r in reqs) if reqs else 0.0
        dur = max(t_last - t_first, 1e-9)
        out = dict(requests=len(reqs), duration_s=dur, requests_per_s=len(reqs) / dur,
                   solves_per_s=sum(1 for r in reqs if r.kind == "solve") / dur,
                   p50_ms=float(np.percentile(lat, 50) * 1e3) if len(lat) else 0.0,
                   p99_ms=float(np.percentile(lat, 99) * 1e3) if len(lat) else 0.0,
                   mean_ms=float(lat.mean() * 1e3) if len(lat) else 0.0,
                   batches=len(self.batches),
                   mean_batch=float(np.mean(self.batches)) if self.batches else 0.0,
                   max_batch=int(max(self.batches)) if self.batches else 0,
                   small=sum(1 for r in reqs if r.small), large=sum(1 for r in reqs if not r.small),
                   arena_peak_bytes=self.arena.peak * 8)
        for kind in ("rank", "solve", "decompose"):
            lk = np.array([r.t_done - r.arrival for r in reqs if r.kind == kind])
            if len(lk):
                out[f"p99_ms_{kind}"] = float(np.percentile(lk, 99) * 1e3)
        return out


def make_request_data(seed: int, specs, pin: bool = True, threads: int = 16):
    """Entries of every request (shared seeded generator) in one (pinned) host buffer."""
    import concurrent.futures

    import torch

    from . import synth

    sizes = [s["n"] * wpr(s["m"]) for s in specs]
    offs = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    buf = torch.empty(max(int(offs[-1]), 1), dtype=torch.int64, pin_memory=pin)
    view = buf.numpy().view(np.uint64)

    def fill(i):
        view[offs[i]:offs[i + 1]] = synth.serving_matrix(seed, specs[i]).reshape(-1)

    with concurrent.futures.ThreadPoolExecutor(threads) as ex:
        list(ex.map(fill, range(len(specs))))
    rhs = [synth.serving_rhs(seed, s) if s["kind"] == "solve" else None for s in specs]
    return buf, offs, rhs


def make_requests(specs, data, arrivals):
    """Fresh Request objects over prepared data (make_request_data), arriving at `arrivals` (s)."""
    buf, offs, rhs = data
    reqs = []
    for i, s in enumerate(specs):
        reqs.append(Request(id=s["id"], kind=s["kind"], n=s["n"], m=s["m"], arrival=float(arrivals[i]),
                            A=buf[offs[i]:offs[i + 1]], b_bits=rhs[i]))
    return reqs
