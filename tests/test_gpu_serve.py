"""Serving loop on the GPU: every request of a Poisson mix is served, and each
delivered key equals the same key generated alone (batch of one) and the
oracle's key -- alone and in the mix are the same, bit for bit."""
import numpy as np
import pytest

import oracle
from paper_2106_08759_amd import workloads as wl

pytestmark = pytest.mark.gpu

MIX = {761: 0.7, 857: 0.2, 1277: 0.1}


def test_serving_mix_alone_equals_mix():
    import paper_2106_08759_amd as nk
    from paper_2106_08759_amd import serve
    be = serve.GpuBackend(0)
    rep = serve.serve(be, rate=2e5, seconds=0.5, mix=MIX, seed=wl.SEED,
                      refill={761: 4096, 857: 2048, 1277: 1024}, blocks=4, record_keys=48)
    assert rep["served"] == rep["requests"] > 50000
    assert rep["latency_ms"]["p99"] < 1000.0
    ctx = nk.Context(0)
    for p in MIX:
        rec = rep["recorded"][p]
        assert len(rec) == 48 and [k for k, _, _ in rec] == list(range(48))
        pk, sk = ctx.batch_keygen(p, wl.SEED, 0, 48)
        pk, sk = pk.cpu().numpy(), sk.cpu().numpy()
        _, q, w = wl.PQW[p]
        for k, rpk, rsk in rec:
            assert rpk == pk[k].tobytes() and rsk == sk[k].tobytes(), (p, k)
        for k in (0, 17, 47):
            o = oracle.keygen(wl.SEED, p, k)
            assert rec[k][1] == oracle.encode_pk(o["h"], p, q) and rec[k][2] == oracle.encode_sk(o["f"], o["ginv"], p)
    ctx.close()
