"""The autotuner on the GPU: a real timed search at N = 2048 sntrup761 keys
(every phase: group knobs with the R/3 lanes per key, the R/3 knobs, the
persistent fused form, the batched-R/3 form), the choice cached and applied,
and the keys of the chosen configuration equal to the oracle's."""
import numpy as np
import pytest

from paper_2106_08759_amd import workloads as wl
import oracle_pool

pytestmark = pytest.mark.gpu


def test_tune_then_parity(tmp_path):
    import paper_2106_08759_amd as nk
    from paper_2106_08759_amd import autotune
    ctx = nk.Context(0)
    try:
        n = 2048
        path = str(tmp_path / "tune.json")
        e = autotune.tune(ctx, 761, n, reps=1, force=True, path=path, mode="eager")
        assert not e["cached"]
        rows = e["table"]
        assert any(r["persistent"] for r in rows) and any(r["r3_batch"] for r in rows)
        assert 256 in {r["group_size"] for r in rows}
        best = min(rows, key=lambda r: r["ms"])
        assert e["config"] == {k: best[k] for k in autotune.KNOBS}
        applied = ctx.get_config(761)
        assert all(applied[k] == v for k, v in e["config"].items()) and applied["use_graph"] == 0
        again = autotune.tune(ctx, 761, n, path=path, mode="eager")
        assert again["cached"] and again["config"] == e["config"]
        pk, sk, h, f, ginv = ctx.batch_keygen(761, wl.SEED, 0, n, raw=True)
        ref = oracle_pool.oracle_keys(wl.SEED, 761, range(n))
        rpk, rsk = oracle_pool.pk_sk_arrays(ref, range(n))
        assert np.array_equal(pk.cpu().numpy(), rpk) and np.array_equal(sk.cpu().numpy(), rsk), e["config"]
        hh = h.cpu().numpy()
        assert all(np.array_equal(hh[i], ref[i][2]) for i in range(n))
    finally:
        ctx.close()
