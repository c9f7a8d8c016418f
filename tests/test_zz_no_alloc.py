"""ntrup_batch_keygen_noalloc, the allocation-free variant of
ntrup_batch_keygen (static device scratch instead of the context workspace),
called through the C ABI: its keys equal ntrup_batch_keygen's on two calls in
a row, the second smaller, with raw outputs; the context holds no workspace
afterwards; sizes beyond the scratch are refused."""
import numpy as np
import pytest

from paper_2106_08759_amd import workloads as wl

pytestmark = pytest.mark.gpu


def test_noalloc_matches_batch_keygen():
    import torch
    import paper_2106_08759_amd as nk
    p = 761
    prm = nk.params(p)
    nmax = nk.noalloc_max_keys(p)
    assert 3000 < nmax < 6000
    ctx = nk.Context(0)          # the allocation-free calls' context: never gets a workspace
    ref = nk.Context(0)          # the workspace path, to compare against
    try:
        for first, n in ((1000, nmax), (37, 301)):
            pk = torch.full((n, prm.pk_bytes), 0xA5, dtype=torch.uint8, device="cuda")
            sk = torch.full((n, prm.sk_bytes), 0xA5, dtype=torch.uint8, device="cuda")
            raw = (torch.zeros((n, p), dtype=torch.int16, device="cuda"),
                   torch.zeros((n, p), dtype=torch.int8, device="cuda"),
                   torch.zeros((n, p), dtype=torch.int8, device="cuda"))
            torch.cuda.synchronize()
            ctx.batch_keygen_noalloc(p, wl.SEED, first, n, pk, sk, raw=raw)
            assert ctx.workspace_bytes() == 0
            rpk, rsk, rh, rf, rg = ref.batch_keygen(p, wl.SEED, first, n, raw=True)
            assert torch.equal(pk, rpk) and torch.equal(sk, rsk), (first, n)
            assert torch.equal(raw[0], rh) and torch.equal(raw[1], rf) and torch.equal(raw[2], rg), (first, n)
        big_pk = torch.empty((nmax + 1, prm.pk_bytes), dtype=torch.uint8, device="cuda")
        big_sk = torch.empty((nmax + 1, prm.sk_bytes), dtype=torch.uint8, device="cuda")
        with pytest.raises(nk.NtrupError) as e:
            ctx.batch_keygen_noalloc(p, wl.SEED, 0, nmax + 1, big_pk, big_sk, check=False)
        assert e.value.code == nk.NTRUP_ERANGE
    finally:
        ctx.close()
        ref.close()


@pytest.mark.parametrize("p", [653, 1277])
def test_noalloc_other_params_and_forms(p):
    """Resampling parameter sets, in the per-key and batched-R/3 forms."""
    import torch
    import paper_2106_08759_amd as nk
    prm = nk.params(p)
    ctx = nk.Context(0)
    ref = nk.Context(0)
    try:
        for r3b in (0, 1):
            for c in (ctx, ref):
                c.set_config(p, r3_batch=r3b, persistent=0, use_graph=0, group_size=32, inverse_share=4)
            for first, n in ((5, 700), (900, 65)):
                pk = torch.empty((n, prm.pk_bytes), dtype=torch.uint8, device="cuda")
                sk = torch.empty((n, prm.sk_bytes), dtype=torch.uint8, device="cuda")
                ctx.batch_keygen_noalloc(p, wl.SEED, first, n, pk, sk)
                rpk, rsk = ref.batch_keygen(p, wl.SEED, first, n)
                assert torch.equal(pk, rpk) and torch.equal(sk, rsk), (r3b, first, n)
        assert ctx.workspace_bytes() == 0
    finally:
        ctx.close()
        ref.close()
