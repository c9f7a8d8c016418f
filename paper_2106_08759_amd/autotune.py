"""Autotuner for the batched KeyGen pipeline.

Knobs (see ``ntrup_config`` in include/ntrupkg.h):
  group_size     Montgomery group size G (Section 2.2's n): larger groups
                 share one R/q reciprocal among more keys but leave fewer
                 independent groups to fill the GPU;
  inverse_share  W groups (one wave each) sharing one reciprocal through a
                 second level of the same trick;
  lanes_per_key  1, 2, 4 or 8 lanes per key for the bitsliced R/3 divsteps
                 of the main pass;
  retry_lanes_per_key, retry_parallel_attempts, retry_passes
                 lanes per key, g draws tried side by side per key, and the
                 number of compacted passes for the keys whose g was not
                 invertible (matters for p = 653, 1277, where the retry
                 passes are latency-bound);
  persistent     the stage pipeline (0) or one persistent fused kernel per
                 call (1);
  r3_batch       one divstep reciprocal in R/3 per key (0) or the R/3
                 reciprocals of each Montgomery group batched as in
                 Algorithm 1 (1);
  recip_jump     the shared R/q reciprocal (bit 0) and the batched-R/3
                 group reciprocals (bit 1) by the plain divstep loop (bit
                 clear) or by jump divsteps on the matrix cores (bit set);
  group_form     the R/q batch inversion of a group as a chain (0) or as a
                 product tree over the waves of a workgroup (1).

The group knobs (G, W) and the R/3 knobs act on different kernels, but in
eager launches the prefix kernel runs beside the R/3 stage and the two compete
for the same compute units, so the first phase times (G, W) jointly with the
lanes per key of the R/3 main pass (PHASE1_LANES); the second phase then times
every R/3 setting (lanes per key, retry knobs) with the chosen (G, W), and
the persistent fused form (one kernel per call, ``persistent`` = 1) at the
settings in PERSISTENT_CANDIDATES, and the batched-R/3 form (``r3_batch`` =
1) at the (G, W) settings in R3BATCH_CANDIDATES.  Each candidate runs in the launch form of
the tuning mode (eager launches, or graph replay: one linear stream per job);
mode "auto" then compares the two forms.
The product tiles are fixed by p.
Every candidate is timed on the real pipeline with HIP events on the launch
stream; the winner per (device, p, N rounded up to a power of two) is cached
as JSON.
"""
from __future__ import annotations

import json
import os
import time

GROUP_SIZES = (8, 16, 32, 64, 128, 256)
SHARES = (1, 2, 4, 8)
PHASE1_LANES = (1, 2, 4)   # R/3 lanes per key timed jointly with (G, W)
KNOBS = ("group_size", "inverse_share", "lanes_per_key", "retry_passes", "retry_lanes_per_key",
         "retry_parallel_attempts", "persistent", "r3_batch", "recip_jump", "group_form")
# (G, W, lanes per key) settings timed for the persistent fused form
PERSISTENT_CANDIDATES = ((32, 2, 2), (32, 4, 2), (64, 2, 2), (32, 4, 4), (16, 4, 2))
# (G, W) settings timed for the batched-R/3 form (its R/3 groups are the
# Montgomery groups of the R/q stage)
R3BATCH_CANDIDATES = ((32, 8), (32, 4), (64, 4), (16, 8), (64, 2), (64, 8), (128, 2), (128, 1))
# group sizes timed for the tree form (group_form = 1) of the R/q batch inversion
TREE_SIZES = (16, 32, 64, 128)


def cache_path() -> str:
    return os.environ.get("NTRUPKG_TUNE_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "ntrupkg", "autotune.json"))


def bucket(n: int) -> int:
    b = 1
    while b < n:
        b <<= 1
    return b


def group_candidates(p: int, n: int):
    """(G, W) pairs worth timing for n keys of degree p."""
    out = []
    for g in GROUP_SIZES:
        if g > max(16, n):
            continue
        for w in SHARES:
            if p == 1277 and w > 4:   # 8 waves of p = 1277 exceed the LDS
                continue
            if g * w > max(16, 2 * n):
                continue
            out.append({"group_size": g, "inverse_share": w})
    return out


def r3_candidates(p: int):
    """R/3 knob settings worth timing for degree p."""
    lpks = (1, 2, 4, 8)
    # (retry passes, retry lanes per key, attempts side by side)
    retry = [(1, 8, 4)] if p not in (653, 1277) else [(1, 8, 2), (1, 8, 4), (1, 8, 8), (0, 8, 4), (1, 4, 4)]
    return [{"lanes_per_key": l, "retry_passes": r, "retry_lanes_per_key": rl, "retry_parallel_attempts": ra}
            for l in lpks for r, rl, ra in retry]


def candidates(p: int, n: int):
    """All configurations the two tuning phases may time (for reference)."""
    return [dict(g, **r) for g in group_candidates(p, n) for r in r3_candidates(p)]


def phase1_candidates(p: int, n: int):
    """The (G, W, lanes per key) settings of the first phase."""
    return [dict(g, lanes_per_key=l) for l in PHASE1_LANES for g in group_candidates(p, n)]


def device_id(device: int) -> str:
    """Cache key of the device: its architecture (the marketing name can read
    empty, e.g. under a profiler), else its name."""
    import torch
    props = torch.cuda.get_device_properties(device)
    return getattr(props, "gcnArchName", "") or props.name or "unknown"


MODES = ("auto", "eager", "graph")


def _key(device_name: str, p: int, n: int, mode: str = "auto") -> str:
    # v6: entries carry inverse_share, the launch form (eager / graph), the
    # kernel form (stage pipeline / persistent fused kernel) and the R/3 form
    # (per key / batched); G up to 256
    # v9: and the reciprocals' forms (plain / jump divsteps), the group form
    # (chain / tree)
    return "%s|p=%d|n<=%d|%s|v9" % (device_name, p, bucket(n), mode)


def load_cache(path: str | None = None) -> dict:
    path = path or cache_path()
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def save_cache(data: dict, path: str | None = None) -> None:
    path = path or cache_path()
    os.makedirs(os.path.dirname(path), exist_ok=True)
    tmp = path + ".tmp%d" % os.getpid()
    with open(tmp, "w") as fh:
        json.dump(data, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def lookup(device_name: str, p: int, n: int, path: str | None = None, mode: str = "auto"):
    return load_cache(path).get(_key(device_name, p, n, mode))


def time_config(ctx, p: int, n: int, cfg: dict, seed: bytes, reps: int, pk, sk, use_graph: int = 0) -> float:
    """Mean milliseconds per call of the pipeline under cfg (eager launches,
    which run the prefix kernel beside the R/3 stage, or graph replay)."""
    import torch
    ctx.set_config(p, use_graph=use_graph, **cfg)
    ctx.batch_keygen(p, seed, 0, n, pk, sk, check=True)  # warm
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        ctx.batch_keygen(p, seed, 0, n, pk, sk, check=False)
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def tune(ctx, p: int, n: int, seed: bytes | None = None, reps: int = 3, force: bool = False,
         path: str | None = None, mode: str = "auto") -> dict:
    """Pick and apply the fastest configuration for (p, n); returns the cache entry
    {"config": ..., "use_graph": 0/1, "ms": ..., "keys_per_s": ..., "table": [...],
    "cached": bool}.  mode: "eager" times and applies eager launches (the
    prefix kernel beside the R/3 stage; for calls whose arguments never repeat,
    or timed with stage events), "graph" times and applies graph replay (one
    linear stream per job, as the jobs of a mixed call run), "auto" tunes the
    knobs eagerly and then picks the faster launch form."""
    assert mode in MODES, mode
    import torch
    from . import params
    from .workloads import SEED

    seed = seed or SEED
    dev = device_id(ctx.device)
    key = _key(dev, p, n, mode)
    data = load_cache(path)
    if not force and key in data:
        entry = dict(data[key])
        ctx.set_config(p, use_graph=entry["use_graph"], **entry["config"])
        entry["cached"] = True
        return entry
    ug = 1 if mode == "graph" else 0
    prm = params(p)
    pk = torch.empty((n, prm.pk_bytes), dtype=torch.uint8, device="cuda:%d" % ctx.device)
    sk = torch.empty((n, prm.sk_bytes), dtype=torch.uint8, device="cuda:%d" % ctx.device)
    ctx.reserve(p, n)
    base = ctx.get_config(p)
    cur = {k: base[k] for k in KNOBS}
    cur["persistent"] = 0
    cur["r3_batch"] = 0
    # eager launches run the per-key R/3 stage beside the prefix kernel, and
    # the jump reciprocal's registers do not fit beside the one-lane R/3
    # waves (it then waits for them: 2.6 vs 1.8 ms at sntrup761 N = 65536):
    # the per-key phases time the plain reciprocal there, the batched-R/3
    # phase the jump form; phase 2d tries the others
    cur["recip_jump"] = 0 if ug == 0 else 1
    cur["group_form"] = 0
    ctx.set_config(p, product_engine=1)
    table = []
    # phase 1: the group stage, jointly with the R/3 main pass's lanes per key
    for lanes in PHASE1_LANES:
        for gc in group_candidates(p, n):
            cfg = dict(cur, lanes_per_key=lanes, **gc)
            table.append(dict(cfg, ms=round(time_config(ctx, p, n, cfg, seed, reps, pk, sk, ug), 4)))
    best = min(table, key=lambda r: r["ms"])
    cur.update({k: best[k] for k in ("group_size", "inverse_share")})
    # phase 2: the R/3 stage
    for rc in r3_candidates(p):
        cfg = dict(cur, **rc)
        table.append(dict(cfg, ms=round(time_config(ctx, p, n, cfg, seed, reps, pk, sk, ug), 4)))
    best = min(table, key=lambda r: r["ms"])
    # phase 2b: the persistent fused form (one kernel per call) at a few
    # (G, W, lanes per key) settings, with the chosen retry knobs
    for g_, w_, l_ in PERSISTENT_CANDIDATES:
        if (g_, w_) not in {(c["group_size"], c["inverse_share"]) for c in group_candidates(p, n)}:
            continue
        pc = dict(best, group_size=g_, inverse_share=w_, lanes_per_key=l_, persistent=1)
        pc = {k: pc[k] for k in KNOBS}
        table.append(dict(pc, ms=round(time_config(ctx, p, n, pc, seed, reps, pk, sk, ug), 4)))
    # phase 2c: batched R/3 reciprocals (Algorithm 1) at a few (G, W)
    r3b = min((r for r in table if not r["persistent"]), key=lambda r: r["ms"])
    for g_, w_ in R3BATCH_CANDIDATES:
        if (g_, w_) not in {(c["group_size"], c["inverse_share"]) for c in group_candidates(p, n)}:
            continue
        bc = dict(r3b, group_size=g_, inverse_share=w_, r3_batch=1, persistent=0, recip_jump=1)
        bc = {k: bc[k] for k in KNOBS}
        table.append(dict(bc, ms=round(time_config(ctx, p, n, bc, seed, reps, pk, sk, ug), 4)))
    best = min(table, key=lambda r: r["ms"])
    # phase 2c': the tree form of the R/q batch inversion at a few group sizes
    # (with the best R/3 form so far: its batched groups are the same size)
    tb = min((r for r in table if not r["persistent"]), key=lambda r: r["ms"])
    for g_ in TREE_SIZES:
        if g_ > max(16, n):
            continue
        tc = dict(tb, group_size=g_, inverse_share=1, group_form=1, persistent=0)
        tc = {k: tc[k] for k in KNOBS}
        table.append(dict(tc, ms=round(time_config(ctx, p, n, tc, seed, reps, pk, sk, ug), 4)))
    best = min(table, key=lambda r: r["ms"])
    # phase 2d: the other reciprocal forms at the chosen setting (plain or
    # jump R/q reciprocal; with batched R/3 also jump divsteps for its group
    # reciprocals; the persistent form always runs the plain loops)
    if not best["persistent"]:
        for rj in sorted({0, 1, 3} if best["r3_batch"] else {0, 1}):
            if rj == best["recip_jump"]:
                continue
            pc = {k: best[k] for k in KNOBS}
            pc["recip_jump"] = rj
            table.append(dict(pc, ms=round(time_config(ctx, p, n, pc, seed, reps, pk, sk, ug), 4)))
        best = min(table, key=lambda r: r["ms"])
    cfg = {k: best[k] for k in KNOBS}
    # phase 3 (auto): eager launches (stage overlap) or graph replay (one
    # linear stream, no launch overhead) for the chosen knobs
    if mode == "auto":
        eager_ms = best["ms"]
        graph_ms = round(time_config(ctx, p, n, cfg, seed, reps, pk, sk, use_graph=1), 4)
        graph = 1 if graph_ms < eager_ms else 0
        ms = min(eager_ms, graph_ms)
    else:
        graph, ms = ug, best["ms"]
        eager_ms = ms if not ug else None
        graph_ms = ms if ug else None
    entry = {"config": cfg, "use_graph": graph, "mode": mode, "ms": ms, "eager_ms": eager_ms,
             "graph_ms": graph_ms, "n": n, "table": table, "tuned_at": time.strftime("%Y-%m-%dT%H:%M:%S")}
    entry["keys_per_s"] = round(n / entry["ms"] * 1e3, 1)
    data[key] = entry
    save_cache(data, path)
    ctx.set_config(p, use_graph=graph, **cfg)
    return dict(entry, cached=False)


def main(argv=None):
    import argparse
    ap = argparse.ArgumentParser(description="tune the batched KeyGen pipeline")
    ap.add_argument("--p", type=int, nargs="+", default=[761])
    ap.add_argument("--n", type=int, default=65536)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--force", action="store_true")
    ap.add_argument("--mode", choices=MODES, default="auto")
    args = ap.parse_args(argv)
    from . import Context
    ctx = Context(0)
    for p in args.p:
        e = tune(ctx, p, args.n, reps=args.reps, force=args.force, mode=args.mode)
        print(json.dumps({"p": p, "n": args.n, "config": e["config"], "ms": e["ms"],
                          "keys_per_s": e["keys_per_s"], "cached": e["cached"]}))


if __name__ == "__main__":
    main()
