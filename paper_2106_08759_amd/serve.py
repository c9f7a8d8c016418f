"""Serving loop: device-resident key pools with continuous batched refills.

The paper's ``batch_lib`` provider (Section 4.2) keeps one pool of key pairs
per parameter set; a request pops a key (copy, then secure erase of the slot)
and an emptied pool is refilled synchronously by one batch call.  Here the
pools live in HBM, refills are asynchronous and overlap on the device:

* each pool is a ring of ``blocks`` blocks of ``refill`` slots; a block is
  FREE, PENDING (a batched KeyGen is writing it) or READY;
* the HBM budget pays for the pool rings and for K device workspaces
  (K = what fits, at most one per pool); a refill needs a free workspace:
  when READY + PENDING keys fall below ``low_water`` and a workspace is
  free, a refill of one block is enqueued on the pool's generation stream,
  otherwise it is deferred; refills of different pools overlap on the
  device, up to K at a time;
* requests queue per parameter set in arrival order and are served from
  READY blocks as soon as keys are there: one device-to-host copy per pool
  per loop turn into pinned memory, then the served slots are erased on the
  device;
* latency = time the key is in host memory minus arrival time.

Keys are a pure function of (seed, p, index); each pool hands out indices
0, 1, 2, ... in order, so any served key can be regenerated alone and must be
identical (the tests check this).

The loop talks to the device through a backend object so that the
scheduling logic can be exercised without a GPU; ``GpuBackend`` is the only
backend in this package.
"""
from __future__ import annotations

import json
import time
from dataclasses import dataclass, field

import numpy as np

FREE, PENDING, READY = 0, 1, 2


class GpuBackend:
    """Device operations of the serving loop on the HIP library."""

    def __init__(self, device: int = 0):
        import torch
        self.torch = torch
        self.device = device
        self.dev = "cuda:%d" % device

    def params(self, p):
        from . import params
        return params(p)

    def context(self):
        from . import Context
        return Context(self.device)

    def stream(self):
        return self.torch.cuda.Stream(device=self.device)

    def alloc(self, rows, cols):
        return self.torch.zeros((rows, cols), dtype=self.torch.uint8, device=self.dev)

    def pinned(self, rows, cols):
        return self.torch.empty((rows, cols), dtype=self.torch.uint8, pin_memory=True)

    def workspace_bytes(self, ctx, p, n):
        """Grow ctx's workspace to fit n keys of degree p; returns its size."""
        ctx.reserve(p, n)
        return ctx.workspace_bytes()

    def configure(self, ctx, p, n):
        """Tuned configuration of (p, n) refills for this workspace (cached).
        Refills never repeat their arguments (each starts at a new key index),
        so they launch eagerly rather than through a captured graph."""
        from . import autotune
        autotune.tune(ctx, p, n, reps=2, mode="eager")

    def keygen(self, ctx, p, seed, first_index, n, pk, sk, stream):
        ctx.batch_keygen(p, seed, first_index, n, pk, sk, stream=stream, check=False)

    def event(self, stream):
        ev = self.torch.cuda.Event()
        ev.record(stream)
        return ev

    def done(self, ev) -> bool:
        return ev.query()

    def wait(self, stream, ev):
        stream.wait_event(ev)

    def copy_out(self, dst, src, stream):
        with self.torch.cuda.stream(stream):
            dst.copy_(src, non_blocking=True)

    def erase(self, t, stream):
        with self.torch.cuda.stream(stream):
            t.zero_()

    def status(self, ctx, stream):
        return ctx.status(stream)

    def sync(self, stream):
        stream.synchronize()

    def row_bytes(self, t, r) -> bytes:
        return bytes(t[r].numpy())


@dataclass
class PoolStats:
    served: int = 0
    refills: int = 0
    deferred: int = 0
    keys_generated: int = 0


@dataclass
class Pool:
    """Ring of blocks for one parameter set."""
    p: int
    refill: int
    blocks: int
    low_water: int
    backend: object
    seed: bytes
    budget: "Budget"
    stats: PoolStats = field(default_factory=PoolStats)

    def __post_init__(self):
        b = self.backend
        prm = b.params(self.p)
        self.pkb, self.skb = prm.pk_bytes, prm.sk_bytes
        cap = self.refill * self.blocks
        self.pk = b.alloc(cap, self.pkb)
        self.sk = b.alloc(cap, self.skb)
        self.state = [FREE] * self.blocks
        self.first_key = [0] * self.blocks       # key index of slot 0 of the block
        self.taken = [0] * self.blocks           # slots of a READY block already served
        self.pending_ev = [None] * self.blocks
        self.erase_ev = [None] * self.blocks
        self.fifo = []                           # READY/PENDING blocks in key order
        self.next_key = 0
        self.gen_stream = b.stream()
        self.io_stream = b.stream()
        self.budget.reserve_static(cap * (self.pkb + self.skb))
        self.inflight = 0
        self.ctx_of = {}      # block -> workspace context of its pending refill

    # -- accounting
    def ready_keys(self) -> int:
        return sum(self.refill - self.taken[i] for i in self.fifo if self.state[i] == READY)

    def pending_keys(self) -> int:
        return sum(self.refill for i in self.fifo if self.state[i] == PENDING)

    # -- device work
    def poll(self, now: float):
        for i in self.fifo:
            if self.state[i] == PENDING and self.backend.done(self.pending_ev[i]):
                ctx = self.ctx_of.pop(i)
                rc = self.backend.status(ctx, self.gen_stream)   # the batch's key-level status
                if rc:
                    raise RuntimeError("refill of p=%d failed: status %d" % (self.p, rc))
                self.state[i] = READY
                self.pending_ev[i] = None
                self.inflight -= 1
                self.budget.release(ctx)

    def maybe_refill(self) -> bool:
        if self.ready_keys() + self.pending_keys() >= self.low_water:
            return False
        free = [i for i in range(self.blocks) if self.state[i] == FREE]
        if not free or self.inflight >= 1:   # one batch in flight per pool
            return False
        ctx = self.budget.acquire()
        if ctx is None:
            self.stats.deferred += 1
            return False
        i = free[0]
        self.ctx_of[i] = ctx
        b = self.backend
        if self.erase_ev[i] is not None:
            b.wait(self.gen_stream, self.erase_ev[i])   # the block's last erase precedes the refill
        lo = i * self.refill
        b.keygen(ctx, self.p, self.seed, self.next_key, self.refill,
                 self.pk[lo:lo + self.refill], self.sk[lo:lo + self.refill], self.gen_stream)
        self.pending_ev[i] = b.event(self.gen_stream)
        self.state[i] = PENDING
        self.first_key[i] = self.next_key
        self.taken[i] = 0
        self.next_key += self.refill
        self.fifo.append(i)
        self.inflight += 1
        self.stats.refills += 1
        self.stats.keys_generated += self.refill
        return True

    def take(self, k: int, host_pk, host_sk):
        """Copy up to k ready keys (oldest first) into host rows [0, got);
        returns (got, key indices, copy-complete event)."""
        b = self.backend
        got, idx = 0, []
        for i in list(self.fifo):
            if got == k or self.state[i] != READY:
                break
            t = min(k - got, self.refill - self.taken[i])
            lo = i * self.refill + self.taken[i]
            b.copy_out(host_pk[got:got + t], self.pk[lo:lo + t], self.io_stream)
            b.copy_out(host_sk[got:got + t], self.sk[lo:lo + t], self.io_stream)
            b.erase(self.pk[lo:lo + t], self.io_stream)
            b.erase(self.sk[lo:lo + t], self.io_stream)
            idx.extend(range(self.first_key[i] + self.taken[i], self.first_key[i] + self.taken[i] + t))
            self.taken[i] += t
            got += t
            if self.taken[i] == self.refill:
                self.erase_ev[i] = b.event(self.io_stream)
                self.state[i] = FREE
                self.fifo.remove(i)
        ev = b.event(self.io_stream) if got else None
        self.stats.served += got
        return got, idx, ev


class Budget:
    """HBM admission.  Static memory = the pool rings; the rest of the budget
    buys K device workspaces (contexts), each big enough for any pool's
    refill batch.  A refill holds one workspace until its keys are READY."""

    def __init__(self, limit_bytes: int):
        self.limit = limit_bytes
        self.static = 0
        self.ws_bytes = 0
        self.free = []
        self.contexts = []

    def reserve_static(self, n: int):
        self.static += n
        if self.static > self.limit:
            raise MemoryError("pool rings need %d bytes, budget %d" % (self.static, self.limit))

    def provision(self, backend, sizes, max_contexts: int, tune: bool = False):
        """Create as many workspaces as the budget pays for (at most
        max_contexts); sizes = [(p, n)] of the refill batches.  With tune, each
        workspace gets the autotuned configuration of every refill size."""
        probe = backend.context()
        ws = 0
        for p, n in sizes:
            ws = backend.workspace_bytes(probe, p, n)
        k = min(max_contexts, (self.limit - self.static) // max(ws, 1))
        if k < 1:
            raise MemoryError("budget %d leaves no room for a %d-byte workspace after %d bytes of pools"
                              % (self.limit, ws, self.static))
        self.ws_bytes = ws
        self.contexts = [probe]
        for _ in range(k - 1):
            c = backend.context()
            for p, n in sizes:
                backend.workspace_bytes(c, p, n)
            self.contexts.append(c)
        if tune:
            for c in self.contexts:
                for p, n in sizes:
                    backend.configure(c, p, n)
        self.free = list(self.contexts)

    def acquire(self):
        return self.free.pop() if self.free else None

    def release(self, ctx):
        self.free.append(ctx)

    @property
    def used(self) -> int:
        return self.static + self.ws_bytes * len(self.contexts)


def poisson_arrivals(rate: float, seconds: float, mix: dict, rng_seed: int = 5):
    """Arrival times (s) and parameter sets of a Poisson stream (numpy default_rng)."""
    rng = np.random.default_rng(rng_seed)
    n = rng.poisson(rate * seconds)
    t = np.sort(rng.uniform(0.0, seconds, size=n))
    ps = np.array(list(mix.keys()))
    w = np.array(list(mix.values()), dtype=float)
    which = ps[rng.choice(len(ps), size=n, p=w / w.sum())]
    return t, which


def serve(backend, rate: float, seconds: float, mix: dict, seed: bytes, refill: dict, blocks: int = 4,
          low_water: dict | None = None, budget_bytes: int = 4 << 30, warm: bool = True,
          sample_every: float = 0.01, record_keys: int = 0, rng_seed: int = 5, clock=time.perf_counter,
          tune: bool = False):
    """Run the request loop for `seconds` of Poisson arrivals.  Returns a report
    dict; with record_keys > 0 also the first record_keys delivered keys per p
    as (index, pk bytes, sk bytes)."""
    t_arr, p_arr = poisson_arrivals(rate, seconds, mix, rng_seed)
    budget = Budget(budget_bytes)
    pools = {p: Pool(p, refill[p], blocks, (low_water or {}).get(p, 2 * refill[p]), backend, seed, budget)
             for p in mix}
    budget.provision(backend, [(p, refill[p]) for p in mix], max_contexts=len(mix), tune=tune)
    maxk = max(1024, int(rate * 0.01) + 1)
    host = {p: (backend.pinned(maxk, pools[p].pkb), backend.pinned(maxk, pools[p].skb)) for p in mix}
    if warm:  # fill the pools before the clock starts
        for _ in range(blocks):
            for pool in pools.values():
                pool.maybe_refill()
            for pool in pools.values():
                while pool.inflight:
                    pool.poll(0.0)
    times = {p: t_arr[p_arr == p] for p in mix}   # arrival times per parameter set, in order
    arrived = {p: 0 for p in mix}                  # requests of p that have arrived
    taken = {p: 0 for p in mix}                    # requests of p handed a key (copy issued)
    inflight_copies = []                           # (event, p, first request, count, key idx)
    lat_chunks = []
    lat_by_p = {p: [] for p in mix}
    occupancy = []
    recorded = {p: [] for p in mix}
    t0 = clock()
    last_sample = -1.0
    while True:
        now = clock() - t0
        if now >= seconds and all(taken[p] == len(times[p]) for p in mix) and not inflight_copies:
            break
        if now > seconds * 4 + 5.0:
            break  # the device cannot keep up: stop and report what was served
        # 1. arrivals up to now
        for p in mix:
            arrived[p] = int(np.searchsorted(times[p], now, side="right"))
        # 2. finished refills and copies
        for pool in pools.values():
            pool.poll(now)
        still = []
        for ev, p, first, cnt, idx in inflight_copies:
            if backend.done(ev):
                tdone = clock() - t0
                lat_chunks.append(tdone - times[p][first:first + cnt])
                lat_by_p[p].append(lat_chunks[-1])
                if record_keys and len(recorded[p]) < record_keys:
                    hp, hs = host[p]
                    for r, key in enumerate(idx[: record_keys - len(recorded[p])]):
                        recorded[p].append((key, backend.row_bytes(hp, r), backend.row_bytes(hs, r)))
            else:
                still.append((ev, p, first, cnt, idx))
        inflight_copies = still
        # 3. serve waiting requests from ready keys (one copy batch per pool per turn;
        #    the pool's host buffer is reused only after its previous copy landed)
        busy = {c[1] for c in inflight_copies}
        for p, pool in pools.items():
            waiting = arrived[p] - taken[p]
            if waiting and p not in busy:
                hp, hs = host[p]
                got, idx, ev = pool.take(min(waiting, maxk), hp, hs)
                if got:
                    inflight_copies.append((ev, p, taken[p], got, idx))
                    taken[p] += got
        # 4. refills admitted by low water and budget
        for pool in pools.values():
            pool.maybe_refill()
        if now - last_sample >= sample_every:
            last_sample = now
            occupancy.append([round(now, 4)] + [pools[p].ready_keys() for p in mix])
    wall = clock() - t0
    for pool in pools.values():
        backend.sync(pool.gen_stream)
        backend.sync(pool.io_stream)
    lat = np.concatenate(lat_chunks) if lat_chunks else np.zeros(1)
    served = sum(pool.stats.served for pool in pools.values())
    rep = {
        "rate_req_per_s": rate, "seconds": seconds, "mix": {str(k): v for k, v in mix.items()},
        "requests": int(len(t_arr)), "served": int(served),
        "keys_per_s": round(served / max(wall, 1e-9), 1),
        "latency_ms": {"p50": round(float(np.percentile(lat, 50)) * 1e3, 4),
                       "p99": round(float(np.percentile(lat, 99)) * 1e3, 4),
                       "max": round(float(lat.max()) * 1e3, 4)},
        "latency_ms_by_p": {str(p): ({"p50": round(float(np.percentile(np.concatenate(v), 50)) * 1e3, 4),
                                      "p99": round(float(np.percentile(np.concatenate(v), 99)) * 1e3, 4)}
                                     if v else None) for p, v in lat_by_p.items()},
        "pools": {str(p): {"refill": pools[p].refill, "blocks": blocks, "low_water": pools[p].low_water,
                           "refills": pools[p].stats.refills, "deferred": pools[p].stats.deferred,
                           "generated": pools[p].stats.keys_generated} for p in mix},
        "hbm_budget_bytes": budget_bytes, "hbm_used_bytes": budget.used, "workspaces": len(budget.contexts),
        "occupancy": {"columns": ["t_s"] + [str(p) for p in mix], "samples": occupancy},
        "wall_s": round(wall, 3),
    }
    if record_keys:
        rep["recorded"] = recorded
    return rep


def main(argv=None):
    import argparse
    ap = argparse.ArgumentParser(description="key-pool serving loop under Poisson load")
    ap.add_argument("--rate", type=float, nargs="+", default=[1e5, 3e5, 1e6])
    ap.add_argument("--seconds", type=float, default=60.0)
    ap.add_argument("--budget-gib", type=float, default=4.0)
    ap.add_argument("--refill", type=int, nargs=3, default=[16384, 8192, 4096],
                    metavar=("R761", "R857", "R1277"))
    ap.add_argument("--blocks", type=int, default=4)
    ap.add_argument("--occupancy", action="store_true", help="include the occupancy time series")
    ap.add_argument("--no-tune", action="store_true", help="refill with the library defaults")
    args = ap.parse_args(argv)
    from .workloads import SEED
    mix = {761: 0.7, 857: 0.2, 1277: 0.1}
    refill = dict(zip((761, 857, 1277), args.refill))
    be = GpuBackend(0)
    for r in args.rate:
        rep = serve(be, r, args.seconds, mix, SEED, refill, blocks=args.blocks,
                    budget_bytes=int(args.budget_gib * (1 << 30)), tune=not args.no_tune)
        if not args.occupancy:
            occ = rep.pop("occupancy")
            rep["occupancy_min"] = {c: min(s[i] for s in occ["samples"]) for i, c in
                                    enumerate(occ["columns"]) if i > 0} if occ["samples"] else {}
        print(json.dumps(rep), flush=True)


if __name__ == "__main__":
    main()
