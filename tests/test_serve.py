"""Serving-loop scheduling without a GPU: a synchronous fake backend whose
"keys" are a deterministic function of (p, index).  Checks that every request
is served once, in key-index order per parameter set, that refills respect
the low-water mark and the HBM budget, and that the report is complete."""
import hashlib
from types import SimpleNamespace

import numpy as np
import pytest

from paper_2106_08759_amd import serve

SIZES = {761: (1237, 382), 857: (1393, 430), 1277: (2076, 640)}


def fake_key(p, i, nbytes, tag):
    h = hashlib.sha256(b"%d:%d:%s" % (p, i, tag)).digest()
    return (h * (nbytes // len(h) + 1))[:nbytes]


class FakeCtx:
    def __init__(self):
        self.ws = 0
        self.calls = 0


class FakeBackend:
    def __init__(self):
        self.keygens = []

    def params(self, p):
        return SimpleNamespace(pk_bytes=SIZES[p][0], sk_bytes=SIZES[p][1])

    def context(self):
        return FakeCtx()

    def stream(self):
        return object()

    def alloc(self, rows, cols):
        return np.zeros((rows, cols), dtype=np.uint8)

    def pinned(self, rows, cols):
        return np.zeros((rows, cols), dtype=np.uint8)

    def workspace_bytes(self, ctx, p, n):
        ctx.ws = max(ctx.ws, 3000 * n)
        return ctx.ws

    def configure(self, ctx, p, n):
        self.configured = getattr(self, "configured", []) + [(p, n)]

    def keygen(self, ctx, p, seed, first, n, pk, sk, stream):
        assert ctx.ws >= 3000 * n
        ctx.calls += 1
        self.keygens.append((p, first, n))
        for r in range(n):
            pk[r] = np.frombuffer(fake_key(p, first + r, pk.shape[1], b"pk"), dtype=np.uint8)
            sk[r] = np.frombuffer(fake_key(p, first + r, sk.shape[1], b"sk"), dtype=np.uint8)

    def event(self, stream):
        return True

    def done(self, ev):
        return True

    def wait(self, stream, ev):
        pass

    def copy_out(self, dst, src, stream):
        dst[...] = src

    def erase(self, t, stream):
        t[...] = 0

    def status(self, ctx, stream):
        return 0

    def sync(self, stream):
        pass

    def row_bytes(self, t, r):
        return bytes(t[r])


MIX = {761: 0.7, 857: 0.2, 1277: 0.1}


def test_every_request_served_in_order():
    be = FakeBackend()
    rep = serve.serve(be, rate=20000, seconds=0.2, mix=MIX, seed=bytes(32),
                      refill={761: 256, 857: 128, 1277: 64}, blocks=4, record_keys=10 ** 6)
    assert rep["served"] == rep["requests"] > 0
    for p in MIX:
        rec = rep["recorded"][p]
        assert [k for k, _, _ in rec] == list(range(len(rec)))      # indices 0, 1, 2, ...
        for k, pk, sk in rec[:50]:
            assert pk == fake_key(p, k, SIZES[p][0], b"pk") and sk == fake_key(p, k, SIZES[p][1], b"sk")
    assert rep["latency_ms"]["p50"] >= 0 and rep["latency_ms"]["p99"] >= rep["latency_ms"]["p50"]
    assert rep["occupancy"]["columns"] == ["t_s", "761", "857", "1277"]
    # refills are whole blocks with consecutive first indices
    for p in MIX:
        firsts = [f for q, f, n in be.keygens if q == p]
        assert firsts == [i * {761: 256, 857: 128, 1277: 64}[p] for i in range(len(firsts))]


def test_budget_limits_workspaces_and_defers_refills():
    be = FakeBackend()
    refill = {761: 256, 857: 128, 1277: 64}
    rings = sum(4 * refill[p] * sum(SIZES[p]) for p in MIX)
    ws = 3000 * 256
    # room for one workspace only: the three pools share it, refills defer
    rep = serve.serve(be, rate=20000, seconds=0.1, mix=MIX, seed=bytes(32), refill=refill, blocks=4,
                      budget_bytes=rings + ws, warm=False)
    assert rep["served"] == rep["requests"]
    assert rep["workspaces"] == 1 and rep["hbm_used_bytes"] <= rings + ws
    assert sum(v["deferred"] for v in rep["pools"].values()) > 0
    # a generous budget gives one workspace per pool and no deferral
    rep = serve.serve(be, rate=20000, seconds=0.1, mix=MIX, seed=bytes(32), refill=refill, blocks=4,
                      budget_bytes=1 << 30)
    assert rep["workspaces"] == 3
    with pytest.raises(MemoryError):
        serve.serve(be, rate=1000, seconds=0.01, mix=MIX, seed=bytes(32), refill=refill, blocks=4,
                    budget_bytes=rings + ws // 2)
    with pytest.raises(MemoryError):
        serve.serve(be, rate=1000, seconds=0.01, mix=MIX, seed=bytes(32), refill=refill, blocks=4,
                    budget_bytes=rings // 2)


def test_poisson_arrivals_mix_and_rate():
    t, p = serve.poisson_arrivals(1e5, 2.0, MIX, rng_seed=5)
    assert abs(len(t) - 2e5) < 5 * np.sqrt(2e5)
    assert np.all(np.diff(t) >= 0) and t[0] >= 0 and t[-1] <= 2.0
    frac = {q: np.mean(p == q) for q in MIX}
    assert abs(frac[761] - 0.7) < 0.01 and abs(frac[857] - 0.2) < 0.01 and abs(frac[1277] - 0.1) < 0.01
