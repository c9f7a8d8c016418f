#!/usr/bin/env python3
"""Benchmark: batched sntrup761 KeyGen on one MI355X.

One step = one pass of the whole hot path over one batch: N = 65536
sntrup761 keys (Short sampling, R/3 reciprocals with resampling, Montgomery
groups in R/q, encoded pk/sk written to HBM).  Prints ONE JSON line.

value     keys/s over the timed steps (inputs: a 32-byte seed; outputs stay in
          HBM; no host copies inside the timed region)
roofline  the dominant kernel's algorithmic integer ops per launch divided by
          its average launch time, measured with HIP events recorded on the
          launch stream during the timed steps.  Peaks: 39.3 T int32
          lane-ops/s for the vector-ALU kernels (256 CU x 4 SIMD x 16 lanes x
          2.4 GHz: a wave64 int32 instruction occupies its SIMD for 4 clocks;
          R/3 divsteps, Short sampling); 5.0 P int8 ops/s for the Montgomery
          group kernels, whose R/q products run on the int8 matrix cores.
          traffic / issued: HBM bytes and VALU instructions per launch from the
          committed counter summary, null once the kernel sources differ from
          the ones they were measured on
cpu_baseline  the CPU oracle (plain C, -O2) on the host cores, bounded sample;
          its keys include 64 spread over the timed workload, against which
          the timed output is checked byte for byte (no value is printed on a
          mismatch)
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# 256 CUs x 4 SIMDs x 32 lanes per clock x 2.4 GHz = 78.6 T int32 lane-ops
# per second: the fp32 vector rate (157.3 TFLOP/s) at one operation per lane
# instead of two flops per FMA.  Simple int32 operations (add, logic,
# bitop3) measure up to 23.4 lanes per clock per SIMD by SQ_INSTS_VALU, above
# the 16 of a four-clock wave64 issue, so 16 lanes is no ceiling; funnel
# shifts and 24-bit multiply-adds run at half rate (<= 15 measured).  The
# calibration table is in profiles/valu_issue_rate.md.
VALU_PEAK = 256 * 4 * 32 * 2.4e9   # int32 lane-ops per second = 78.6 T
I8_MFMA_PEAK = 5.0e15              # dense int8 matrix-core ops per second (2 per multiply-add)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "kernel_counters.json")


def sources_digest() -> str:
    """sha256 over the HIP sources, to tell whether stored counters still apply."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2106_08759_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".h", ".hip")):
            h.update(name.encode())
            with open(os.path.join(csrc, name), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()


def stored_counter(kernel: str, field: str = "bytes_per_launch"):
    """A per-launch figure of `kernel` from the committed counter summary:
    bytes_per_launch (FETCH_SIZE and WRITE_SIZE scaled by a plain-copy
    calibration) or valu_insts (SQ_INSTS_VALU, wave instructions); None when
    there is none or the kernel sources changed since it was taken.  A stage
    of several kernels in a row ('a+b') sums theirs."""
    try:
        with open(TRAFFIC_FILE) as fh:
            data = json.load(fh)
    except (OSError, ValueError):
        return None
    if data.get("sources_sha256") != sources_digest():
        return None
    total = 0
    for part in kernel.split("+"):
        entry = data.get("kernels", {}).get(part)
        if entry is None or entry.get(field) is None:
            return None
        total += entry[field]
    return total


def stored_traffic(kernel: str):
    return stored_counter(kernel, "bytes_per_launch")


def kernel_key(name: str) -> str:
    """'void ntrup::r3_kernel<761, 4>(ntrup::R3Args)' -> 'r3_kernel<761,4>'."""
    base = name.split("(")[0].replace("void ", "").replace("ntrup::", "")
    return base.replace(" ", "")


def summarize_counters(directory: str, copy_mib: int, workload: str, steps_per_run: int = 0,
                       config: dict | None = None) -> dict:
    """profiles/kernel_counters.json from rocprofv3 --pmc runs of bench.py with
    --calib-copy-mib: <directory>/fetch and <directory>/write, each holding
    pmc_counter_collection.csv (FETCH_SIZE, WRITE_SIZE in KiB per dispatch),
    and optionally <directory>/sq (SQ_INSTS_* per dispatch).
    The plain device copy of copy_mib MiB reads and writes copy_mib MiB; the
    ratio of that to what the counters report for it scales every kernel.
    Host-only: reads CSV files, runs nothing on the GPU."""
    import csv
    per = {}
    for which, counter in (("fetch", "FETCH_SIZE"), ("write", "WRITE_SIZE")):
        path = os.path.join(directory, which, "pmc_counter_collection.csv")
        with open(path) as fh:
            for row in csv.DictReader(fh):
                if row["Counter_Name"] != counter:
                    continue
                key = kernel_key(row["Kernel_Name"])
                per.setdefault(key, {}).setdefault(which, []).append(float(row["Counter_Value"]))
    sq = os.path.join(directory, "sq", "pmc_counter_collection.csv")
    if os.path.exists(sq):
        with open(sq) as fh:
            for row in csv.DictReader(fh):
                if row["Counter_Name"] in ("SQ_INSTS_VALU", "SQ_INSTS_MFMA", "SQ_INSTS_SALU", "SQ_INSTS_LDS"):
                    key = kernel_key(row["Kernel_Name"])
                    per.setdefault(key, {}).setdefault(row["Counter_Name"], []).append(float(row["Counter_Value"]))
    copy = per.get("__amd_rocclr_copyBuffer")
    if not copy or "fetch" not in copy or "write" not in copy:
        raise SystemExit("no calibration copy in %s (run bench.py with --calib-copy-mib)" % directory)
    expected = copy_mib * 1024.0
    cal_f, cal_w = max(copy["fetch"]), max(copy["write"])
    fs, ws = expected / cal_f, expected / cal_w
    kernels = {}
    for key, d in sorted(per.items()):
        if not key.startswith(("r3_kernel", "r3b_", "r3_share", "keygen_", "sample_short", "group_", "kem_")) \
                or "fetch" not in d or "write" not in d:
            continue
        f = sum(d["fetch"]) / len(d["fetch"])
        w = sum(d["write"]) / len(d["write"])
        kernels[key] = {"fetch_kib_raw": round(f, 2), "write_kib_raw": round(w, 2),
                        "bytes_per_launch": int(round((f * fs + w * ws) * 1024)),
                        "launches_per_run": len(d["fetch"])}
        for c, field in (("SQ_INSTS_VALU", "valu_insts"), ("SQ_INSTS_MFMA", "mfma_insts"),
                         ("SQ_INSTS_SALU", "salu_insts"), ("SQ_INSTS_LDS", "lds_insts")):
            if c in d:
                kernels[key][field] = round(sum(d[c]) / len(d[c]), 1)
    return {"sources_sha256": sources_digest(),
            "calibration": {"copy_mib": copy_mib, "fetch_kib": round(cal_f, 2), "write_kib": round(cal_w, 2),
                            "fetch_scale": round(fs, 4), "write_scale": round(ws, 4)},
            "workload": workload, "config": config or {}, "steps_per_run": steps_per_run, "kernels": kernels}


def ceil_div(a, b):
    return -(-a // b)


def group_kernel_ops(p: int, n: int, G: int, W: int, split: bool = False) -> dict:
    """Algorithmic int8 matrix-core operations (2 per multiply-add) of the
    Montgomery group stages for n keys.  A ring product is p*p schoolbook
    multiply-adds per pair of int8 limbs: 2 limb pairs when one operand is
    small (3f_i, g_i), 4 when both are residues.  Prefix kernel, per group of
    g keys: g-1 prefix products (small); per W groups: 3(W-1) big products of
    the shared reciprocal (the divstep reciprocal itself runs on the vector
    ALUs and is not counted).  Back-substitution, per group: g-1 products c_i
    (big), g-1 t_i updates and g products h_i (small).  split: eager launches
    with a side stream run the c_i and t_i products there after the prefix
    kernel (group_prefix), and only the h_i products after the R/3 stage
    (group_back, keygen_h_kernel)."""
    pre = back = 0.0
    groups = 0
    for start in range(0, n, G):
        g = min(G, n - start)
        pre += (g - 1) * 2 * p * p
        if split:
            pre += ((g - 1) * 4 + (g - 1) * 2) * p * p
            back += g * 2 * p * p
        else:
            back += ((g - 1) * 4 + (g - 1) * 2 + g * 2) * p * p
        groups += 1
    for start in range(0, groups, W):
        w = min(W, groups - start)
        pre += 3 * (w - 1) * 4 * p * p
    return {"group_prefix": 2 * pre, "group_back": 2 * back}


def tree_kernel_ops(p: int, n: int, G: int) -> dict:
    """Algorithmic int8 matrix-core operations (2 per multiply-add) of the
    tree form for n keys in groups of G = 2^k: per group, G/2 leaf-pair
    products (small x small, 1 limb pair), G/2 - 1 inner up-sweep and G - 2
    inner down-sweep products (big x big, 4 limb pairs), G leaf products
    c_i = t a_sibling (small x big, 2 limb pairs) -- 3G - 3 in all -- and
    the h_i products (group_back)."""
    pre = 0.0
    for start in range(0, n, G):
        pre += (G // 2 * 1 + (G // 2 - 1 + G - 2) * 4 + G * 2) * p * p
    return {"group_prefix": 2 * pre, "group_back": 2.0 * n * 2 * p * p}


def r3_kernel_ops(p: int, keys: int) -> float:
    """Algorithmic 32-bit lane-ops of the bitsliced R/3 divsteps: per key and
    divstep j (of 2p-1), 9 ops per live word of the (f, g) pair and 9 per
    live word of the (v, r) pair (an F_3 scalar multiply-add at 5 ops, a
    2-plane select, a 2-plane shift).  Live: f and g words holding the
    min(p+1, 2p-1-j) coefficients the remaining steps read; v and r words
    holding degree <= j+1.  Layouts with several lanes per key also update
    the dead words; that work is not counted."""
    words = ceil_div(p + 1, 32)
    live = sum(ceil_div(min(p + 1, 2 * p - 1 - j), 32) + min(words, ceil_div(j + 2, 32)) for j in range(2 * p - 1))
    return float(keys) * 9 * live


def short_kernel_ops(p: int, keys: int) -> float:
    """ChaCha20 blocks the f stream needs (ceil(p/16) of 16 words; 20 rounds x
    4 quarter-rounds x 12 ops + 32 per block) plus the compare-exchanges of
    the bitonic network on the next power of two of p words (2 ops each)."""
    ns = 1 << (p - 1).bit_length()
    lg = ns.bit_length() - 1
    ce = ns // 2 * lg * (lg + 1) // 2
    blocks = ceil_div(p, 16)
    return float(keys) * (blocks * (20 * 4 * 12 + 32) + 2 * ce)


def check_indices(n: int, count: int = 64) -> list:
    """Keys of the timed workload whose bytes are checked against the oracle:
    the first, the last and evenly spread ones in between."""
    return sorted({round(i * (n - 1) / (count - 1)) for i in range(count)}) if n > 1 else [0]


def _cpu_worker(args):
    p, start, seconds, check = args
    import oracle
    _, q, _ = oracle.PARAMS[p]
    t0 = time.perf_counter()
    keys = {}
    for i in check:
        k = oracle.keygen(bytes(range(32)), p, i)
        keys[i] = (oracle.encode_pk(k["h"], p, q), oracle.encode_sk(k["f"], k["ginv"], p))
    done, idx = len(check), start
    while time.perf_counter() - t0 < seconds:
        oracle.keygen_range(bytes(range(32)), p, idx, 4)
        idx += 4
        done += 4
    return done, time.perf_counter() - t0, keys


def host_cpu() -> dict:
    """CPU model and core counts of this host."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count() or 1
    return {"model": model, "nproc": os.cpu_count() or 1, "usable": usable}


def cpu_baseline(p: int, seconds: float, check: list) -> tuple:
    """The oracle timed on this host's cores (one process per core, at most
    16: the CPU share a one-GPU job is given); the keys at `check` are part of
    the sample.  Returns (cpu_baseline entry, {index: (pk bytes, sk bytes)})."""
    import oracle
    oracle.build()
    cpu = host_cpu()
    cores = max(1, min(16, cpu["usable"]))
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        res = pool.map(_cpu_worker, [(p, 10_000_000 * (i + 1), seconds, check[i::cores]) for i in range(cores)])
    wall = time.perf_counter() - t0
    keys = sum(r[0] for r in res)
    ref = {}
    for r in res:
        ref.update(r[2])
    return ({"value": round(keys / wall, 1), "unit": "keys/s", "cores": cores, "kind": "oracle",
             "cpu_model": cpu["model"], "nproc": cpu["nproc"], "usable_cpus": cpu["usable"],
             "sample": "sntrup%d KeyGen, %d keys over %d processes (the %d checked keys of the timed workload, "
                       "then disjoint index ranges), %.1f s wall" % (p, keys, cores, len(check), wall)},
            ref)


CALIB_KINDS = {0: "arx (add, xor, rotate)", 1: "v_add_u32", 2: "v_bitop3_b32", 3: "v_alignbit_b32", 4: "v_mad_u32_u24",
               5: "v_perm_b32", 6: "v_xor_b32 + v_add_u32", 7: "v_med3_u32", 8: "v_min_u32 + v_max_u32",
               9: "v_mov_b32_dpp + v_xor_b32"}


def calib_valu(iters: int = 20000, reps: int = 5) -> dict:
    """The vector-ALU probes (csrc/calib_valu.hip): 8 independent chains per
    lane of one instruction kind (or the add-xor-rotate mix), over 1024 x k
    one-wave blocks (k waves per SIMD on 256 CUs x 4 SIMDs).  Reports, per
    kind and k, the mean launch time (HIP events) and the issue rate in lanes
    per clock per SIMD at 2.4 GHz from the instruction count; the counter run
    (SQ_INSTS_VALU) of the same command confirms the count."""
    import ctypes
    import torch
    from paper_2106_08759_amd import build
    L = ctypes.CDLL(build.CALIB_LIB)
    L.calib_valu.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_void_p, ctypes.c_void_p]
    out = {"iters": iters, "clock_ghz": 2.4, "kinds": {}}
    st = torch.cuda.current_stream()
    for kind, name in CALIB_KINDS.items():
        ops = L.calib_valu_ops_per_step(kind)
        rates = {}
        for k in (1, 2, 4, 8):
            blocks = 1024 * k
            buf = torch.empty(blocks * 64, dtype=torch.int32, device="cuda")
            assert L.calib_valu(kind, blocks, iters, buf.data_ptr(), st.cuda_stream) == 0
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(reps):
                assert L.calib_valu(kind, blocks, iters, buf.data_ptr(), st.cuda_stream) == 0
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / reps
            wave_insts = blocks * iters * ops
            rates[k] = {"ms": round(ms, 4), "wave_insts": wave_insts,
                        "lanes_per_clk_per_simd": round(wave_insts * 64 / (ms / 1e3) / 1024 / 2.4e9, 2),
                        "T_lane_ops": round(wave_insts * 64 / (ms / 1e3) / 1e12, 2)}
        out["kinds"][name] = {"ops_per_lane_step": ops, "rates": rates}
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--p", type=int, default=761)
    ap.add_argument("--n", type=int, default=65536)
    ap.add_argument("--group-size", type=int, default=0, help="0: autotuned (see --no-autotune)")
    ap.add_argument("--no-autotune", action="store_true", help="use the library defaults instead of tuning")
    ap.add_argument("--r3-batch", action="store_true",
                    help="measure the batched-R/3 form (Algorithm 1's batchInv over R/3) as the main workload")
    ap.add_argument("--persistent", action="store_true",
                    help="measure the persistent fused kernel as the main workload")
    ap.add_argument("--serve-seconds", type=float, default=3.0)
    ap.add_argument("--serve-rate", type=float, default=3e5)
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the plain-form and N=1024 side measurements")
    ap.add_argument("--summarize-counters", metavar="DIR", default=None,
                    help="host only: write profiles/kernel_counters.json from DIR/fetch, DIR/write, DIR/sq "
                         "(rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE runs of this script) and exit")
    ap.add_argument("--workload-note", default="", help="workload line stored with --summarize-counters")
    ap.add_argument("--counter-steps", type=int, default=3,
                    help="warmup + timed steps of the counter runs (--summarize-counters)")
    ap.add_argument("--counter-config", default="",
                    help="JSON of the configuration the counter runs used (stored with --summarize-counters)")
    ap.add_argument("--calib-valu", action="store_true",
                    help="time the int32 vector-ALU issue-rate probe (libcalib.so) at 1, 2, 4, 8 waves per SIMD "
                         "and exit")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one device-to-device copy of this many MiB first (HBM counter calibration)")
    args = ap.parse_args()

    if args.summarize_counters:
        data = summarize_counters(args.summarize_counters, args.calib_copy_mib or 256, args.workload_note,
                                  args.counter_steps, json.loads(args.counter_config) if args.counter_config else None)
        with open(TRAFFIC_FILE, "w") as fh:
            json.dump(data, fh, indent=1)
            fh.write("\n")
        print(json.dumps(data["kernels"], indent=1))
        return

    if args.calib_valu:
        print(json.dumps(calib_valu()), flush=True)
        return

    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(keys shard with no exchange step: each GPU would run its own key range)", file=sys.stderr)
        sys.exit(2)

    # the CPU oracle runs first, in forked workers, before this process touches
    # the GPU; its sample includes the keys the timed output is checked against
    check = check_indices(args.n)
    cb, ref_keys = (None, {}) if args.no_cpu_baseline else cpu_baseline(args.p, args.cpu_seconds, check)

    import torch
    import paper_2106_08759_amd as nk
    from paper_2106_08759_amd import workloads as wl

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    p, n, K, W = args.p, args.n, args.steps, args.warmup
    ctx = nk.Context(0)
    tuned = None
    if args.group_size:
        ctx.set_config(p, group_size=args.group_size)
    elif not args.no_autotune:
        from paper_2106_08759_amd import autotune
        # eager launches: the timed region records stage events, which
        # bypass graph replay, so the tuned launch form must be eager too
        tuned = autotune.tune(ctx, p, n, reps=2, mode="eager")
    if args.r3_batch:
        ctx.set_config(p, r3_batch=1, persistent=0, use_graph=0, group_size=32, inverse_share=8)
    elif args.persistent:
        pers = [r for r in (tuned or {}).get("table", []) if r.get("persistent")]
        pc = {k: v for k, v in min(pers, key=lambda r: r["ms"]).items() if k != "ms"} if pers else \
            {"group_size": 32, "inverse_share": 2, "lanes_per_key": 2, "persistent": 1, "r3_batch": 0}
        ctx.set_config(p, **dict(pc, use_graph=0, r3_batch=0))
    cfg = ctx.get_config(p)
    prm = nk.params(p)
    ctx.reserve(p, n)
    pk = torch.empty((n, prm.pk_bytes), dtype=torch.uint8, device="cuda")
    sk = torch.empty((n, prm.sk_bytes), dtype=torch.uint8, device="cuda")

    if args.calib_copy_mib:
        src = torch.ones(args.calib_copy_mib << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    for _ in range(W):
        ctx.batch_keygen(p, wl.SEED, 0, n, pk, sk, check=False)
    torch.cuda.synchronize()
    assert ctx.status() == 0

    # timed region: K steps, stage events recorded on the launch stream
    ctx.timing_begin(K)
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(K):
        ctx.batch_keygen(p, wl.SEED, 0, n, pk, sk, check=False)
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = ev0.elapsed_time(ev1)
    stage_ms, timed = ctx.timing_end()
    assert timed == K
    rc = ctx.status()
    assert rc == 0, "keygen status %d" % rc
    # the timed output: the checked keys byte for byte against the oracle's,
    # and every key's f of weight w (decoded from sk); no value on a mismatch
    verified = 0
    if ref_keys:
        import numpy as np
        hpk, hsk = pk[check].cpu().numpy(), sk[check].cpu().numpy()
        bad = [i for j, i in enumerate(check) if hpk[j].tobytes() != ref_keys[i][0] or hsk[j].tobytes() != ref_keys[i][1]]
        if bad:
            print("bench.py: timed output differs from the oracle at keys %s" % bad[:8], file=sys.stderr)
            sys.exit(1)
        verified = len(check)
        f, _ = nk.decode_sk(sk, p)
        if not (np.count_nonzero(f, axis=1) == prm.w).all():
            print("bench.py: some timed f is not of weight %d" % prm.w, file=sys.stderr)
            sys.exit(1)
    ms_per_step = ms / K
    keys_per_s = n * K / (ms / 1e3)

    avg = {k: v / K for k, v in stage_ms.items()}
    assert cfg["product_engine"] == 1, "the roofline below prices the matrix-core group kernel"
    # eager single-job launches use the side stream (prefix kernel and
    # back-substitution beside the R/3 stage); captured graphs run one stream
    split = not cfg["use_graph"] and not cfg.get("persistent")
    tree = cfg.get("group_form") == 1
    ops = dict(tree_kernel_ops(p, n, cfg["group_size"]) if tree else
               group_kernel_ops(p, n, cfg["group_size"], cfg["inverse_share"], split),
               r3_main=r3_kernel_ops(p, n), sample_short=short_kernel_ops(p, n))
    # the persistent fused kernel does all of it; priced on its vector-ALU work
    # (R/3 divsteps and sampling), its matrix-core work being the smaller share
    ops["fused"] = ops["r3_main"] + ops["sample_short"]
    peaks = {"group_prefix": I8_MFMA_PEAK, "group_back": I8_MFMA_PEAK, "r3_main": VALU_PEAK,
             "sample_short": VALU_PEAK, "fused": VALU_PEAK}
    units = {"group_prefix": "T int8-op/s", "group_back": "T int8-op/s", "r3_main": "T lane-op/s",
             "sample_short": "T lane-op/s", "fused": "T lane-op/s"}
    if cfg.get("r3_batch"):
        # batched R/3: per group of g keys, g-1 prefix and 2(g-1) back
        # products in R/3, one int8 limb pair each (the group divstep
        # reciprocals and the screen are not counted)
        G_ = cfg["group_size"]
        prods = sum(3 * (min(G_, n - s_) - 1) for s_ in range(0, n, G_))
        ops["r3_main"] = 2.0 * prods * p * p
        peaks["r3_main"] = I8_MFMA_PEAK
        units["r3_main"] = "T int8-op/s"
    # the dominant kernel is the longest stage on the launch stream (the
    # critical path): in eager launches one of the prefix kernel and the R/3
    # stage runs on the side stream beside the other, its wall time shared --
    # the prefix kernel with per-key R/3, the whole R/3 stage with batched R/3
    # (a chain of five kernels, not one kernel either way)
    if cfg.get("persistent"):
        dom = "fused"
    else:
        side = set() if cfg["use_graph"] else {"r3_main"} if cfg.get("r3_batch") else {"group_prefix"}
        if cfg.get("r3_batch"):
            side.add("r3_main")
        crit = [k for k in ops if k != "fused" and k not in side]
        dom = max(crit, key=lambda k: avg[k])
    achieved = ops[dom] / (avg[dom] / 1e3)
    jump = "true" if cfg["recip_jump"] & 1 else "false"
    # with the side stream, the launch stream's stage between sampling and
    # the join is the prefix kernel followed by the back-substitution kernel
    # (its time and its products are both kernels'); otherwise the prefix
    # kernel alone
    prefix_name = "keygen_prefix_kernel<%d,%d,%s>" % (p, cfg["inverse_share"], jump)
    kernel_names = {"group_prefix": ("keygen_tree_{up,root,down}_kernel<%d> (root jump %s)" % (p, jump) if tree else
                                     prefix_name + "+keygen_cinv_kernel<%d>" % p if split else prefix_name),
                    "group_back": ("keygen_h_kernel<%d>" if split or tree else "keygen_back_kernel<%d>") % p,
                    "r3_main": "r3_kernel<%d,%d>" % (p, cfg["lanes_per_key"]),
                    "sample_short": "sample_short_kernel<%d>" % p,
                    "fused": "keygen_persistent_kernel<%d,%d>" % (cfg["lanes_per_key"], p)}
    roofline = {"bound": "mfma" if peaks[dom] == I8_MFMA_PEAK else "alu", "kernel": kernel_names[dom],
                "achieved": round(achieved / 1e12, 3),
                "peak": round(peaks[dom] / 1e12, 2), "unit": units[dom], "frac": round(achieved / peaks[dom], 4),
                "traffic": stored_traffic(kernel_names[dom]),
                "ops_per_launch": ops[dom], "avg_launch_ms": round(avg[dom], 4)}
    # issued: the VALU instructions the counters saw per launch (x 64 lanes)
    # over the same launch time; the algorithmic fraction is at most this
    vi = stored_counter(kernel_names[dom], "valu_insts")
    if vi is not None and roofline["bound"] == "alu":
        roofline["issued_frac"] = round(vi * 64 / (avg[dom] / 1e3) / VALU_PEAK, 4)
    # the whole step: every kernel's VALU instructions per step over the step
    # time (how full the vector ALUs are across the pipeline)
    try:
        with open(TRAFFIC_FILE) as fh:
            tk = json.load(fh)
        if tk.get("sources_sha256") == sources_digest() and tk.get("steps_per_run"):
            per_step = sum(v.get("valu_insts", 0.0) * v.get("launches_per_run", 1)
                           for v in tk["kernels"].values()) / tk["steps_per_run"]
            roofline["step_valu_issue_frac"] = round(per_step * 64 / (ms_per_step / 1e3) / VALU_PEAK, 4)
    except (OSError, ValueError):
        pass
    stage_fracs = {k: {"ms": round(avg[k], 4),
                       "frac": (round(ops[k] / (avg[k] / 1e3) / peaks[k], 4) if k in ops and avg[k] > 0 else None)}
                   for k in avg}

    extras = {}
    if not args.no_extras:
        # the plain form (one key per launch sequence, Section 3.1) and N=1024 batches
        m = 32
        ctx.keygen_plain(p, wl.SEED, 0, m, check=True)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        ctx.keygen_plain(p, wl.SEED, 0, m, check=False)
        e1.record()
        torch.cuda.synchronize()
        plain = m / (e0.elapsed_time(e1) / 1e3)
        ctx.batch_keygen(p, wl.SEED, 0, 1024, check=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(10):
            ctx.batch_keygen(p, wl.SEED, 0, 1024, check=False)
        e1.record()
        torch.cuda.synchronize()
        b1024 = 1024 * 10 / (e0.elapsed_time(e1) / 1e3)
        extras = {"plain32_keys_per_s": round(plain, 1), "batched1024_keys_per_s": round(b1024, 1),
                  "speedup_batched65536_over_plain": round(keys_per_s / plain, 1)}
        # mixed parameter sets in one graph launch: 16384 keys each of 653/761/857/1277
        jobs = [(653, 0, 16384), (761, 0, 16384), (857, 0, 16384), (1277, 0, 16384)]
        if not args.no_autotune:
            from paper_2106_08759_amd import autotune
            # the jobs of a mixed call run as linear graph branches
            for q_ in (653, 761, 857, 1277):
                autotune.tune(ctx, q_, 16384, reps=2, mode="graph")
        ctx.batch_keygen_mixed(wl.SEED, jobs, check=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(5):
            ctx.batch_keygen_mixed(wl.SEED, jobs, check=False)
        e1.record()
        torch.cuda.synchronize()
        assert ctx.status() == 0
        mixed_ms = e0.elapsed_time(e1) / 5
        all_pers = all(ctx.get_config(q_)["persistent"] for q_ in (653, 761, 857, 1277))
        extras["mixed_4x16384"] = {"keys_per_s": round(4 * 16384 / mixed_ms * 1e3, 1), "ms": round(mixed_ms, 3),
                                   "launch": ("one persistent fused kernel (autotuned)" if all_pers else
                                              "one hipGraph, four concurrent branches (autotuned)")}
        # the same jobs as one launch of the persistent fused kernel
        saved = {q_: ctx.get_config(q_) for q_ in (653, 761, 857, 1277)}
        for q_ in saved:
            # every knob set here: the graph-mode tuning above leaves per-p
            # retry settings (up to 8 draws side by side at 8 lanes each) that
            # this form does not want
            ctx.set_config(q_, persistent=1, r3_batch=0, group_form=0, product_engine=1, lanes_per_key=2,
                           group_size=32, inverse_share=2, use_graph=1, retry_passes=1, retry_lanes_per_key=8,
                           retry_parallel_attempts=4)
        ctx.batch_keygen_mixed(wl.SEED, jobs, check=True)
        torch.cuda.synchronize()
        e0.record()
        for _ in range(5):
            ctx.batch_keygen_mixed(wl.SEED, jobs, check=False)
        e1.record()
        torch.cuda.synchronize()
        assert ctx.status() == 0
        pm_ms = e0.elapsed_time(e1) / 5
        extras["mixed_4x16384_persistent"] = {"keys_per_s": round(4 * 16384 / pm_ms * 1e3, 1), "ms": round(pm_ms, 3),
                                              "launch": "one persistent fused kernel (G=32, W=2, 2 lanes per key, "
                                                        "retries 8 lanes x 4 draws)"}
        for q_, c_ in saved.items():
            ctx.set_config(q_, **c_)
        # this workload (N keys of p) in the persistent fused form, at the
        # autotuner's best persistent setting
        pers = [r for r in (tuned or {}).get("table", []) if r.get("persistent")]
        pcfg = {k: v for k, v in min(pers, key=lambda r: r["ms"]).items() if k != "ms"} if pers else \
            {"group_size": 32, "inverse_share": 2, "lanes_per_key": 2, "persistent": 1, "r3_batch": 0}
        saved = ctx.get_config(p)
        pf = {}
        for ug in (0, 1):
            # eager launches, and the form config 3 names: the persistent
            # kernel captured in a hipGraph and replayed (outer events only)
            ctx.set_config(p, use_graph=ug, **pcfg)
            ctx.batch_keygen(p, wl.SEED, 0, n, pk, sk, check=True)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(5):
                ctx.batch_keygen(p, wl.SEED, 0, n, pk, sk, check=False)
            e1.record()
            torch.cuda.synchronize()
            assert ctx.status() == 0
            pf[ug] = e0.elapsed_time(e1) / 5
        extras["persistent_fused"] = {"keys_per_s": round(n / pf[0] * 1e3, 1), "ms": round(pf[0], 3),
                                      "graph_keys_per_s": round(n / pf[1] * 1e3, 1), "graph_ms": round(pf[1], 3),
                                      "speedup_over_plain": round(n / min(pf.values()) * 1e3 / plain, 1),
                                      "config": {k: pcfg[k] for k in ("group_size", "inverse_share", "lanes_per_key")}}
        ctx.set_config(p, **saved)
        # the paper's own form of Algorithm 1 for the R/3 side: g screened for
        # invertibility, then batchInv over R/3 (Montgomery groups on the
        # matrix cores, one divstep reciprocal per group) instead of one
        # divstep reciprocal per key; same keys
        best = None
        for G_, W_ in ((32, 8), (32, 4), (16, 8)):
            ctx.set_config(p, use_graph=0, persistent=0, r3_batch=1, group_size=G_, inverse_share=W_)
            ctx.batch_keygen(p, wl.SEED, 0, n, pk, sk, check=True)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(5):
                ctx.batch_keygen(p, wl.SEED, 0, n, pk, sk, check=False)
            e1.record()
            torch.cuda.synchronize()
            assert ctx.status() == 0
            b_ms = e0.elapsed_time(e1) / 5
            if best is None or b_ms < best[0]:
                best = (b_ms, G_, W_)
        extras["batched_r3"] = {"keys_per_s": round(n / best[0] * 1e3, 1), "ms": round(best[0], 3),
                                "config": {"group_size": best[1], "inverse_share": best[2]},
                                "method": "batchInv over R/3 after the invertibility screen (Algorithm 1)"}
        ctx.set_config(p, **saved)
        # encapsulation / decapsulation core on this batch's key pairs: r and
        # c = Round(h r); r' = decrypt(c) with the weight and re-encryption
        # checks.  Whole-call times; checked by decap(encap) = r, ok = 1 for
        # every key.
        _, _, h_raw, f_raw, gi_raw = ctx.batch_keygen(p, wl.SEED, 0, n, raw=True)
        seed_e = bytes(range(100, 132))
        c_k, r_k = ctx.batch_encap(p, seed_e, 0, h_raw)
        r_d, ok_d = ctx.batch_decap(p, c_k, f_raw, gi_raw, h_raw)
        torch.cuda.synchronize()
        if not (bool((r_d == r_k).all()) and bool((ok_d == 1).all())):
            print("bench.py: decapsulation did not return r for every key", file=sys.stderr)
            sys.exit(1)
        kem = {}
        for name, call, mfma_ops in (
                ("encap", lambda: ctx.batch_encap(p, seed_e, 0, h_raw, c_k, r_k), 4.0 * p * p),
                ("decap", lambda: ctx.batch_decap(p, c_k, f_raw, gi_raw, h_raw, r_d, ok_d), 10.0 * p * p)):
            call()
            torch.cuda.synchronize()
            e0.record()
            for _ in range(10):
                call()
            e1.record()
            torch.cuda.synchronize()
            k_ms = e0.elapsed_time(e1) / 10
            kem[name] = {"keys_per_s": round(n / k_ms * 1e3, 1), "ms": round(k_ms, 4),
                         "int8_ops_per_key": mfma_ops,
                         "frac_of_mfma_peak": round(n * mfma_ops / (k_ms / 1e3) / I8_MFMA_PEAK, 4)}
        kem["encap"]["call"] = "Short sampler (stream 0x8000) + kem_encap_kernel: one small x big product per key"
        kem["decap"]["call"] = ("kem_decap_kernel: 3f c in R/q, e (1/g) in R/3, weight check, re-encryption "
                                "Round(h r') against c")
        kem["verified"] = "decap(encap) = r with ok = 1 for all %d keys" % n
        extras["kem_core"] = kem
        del h_raw, f_raw, gi_raw, c_k, r_k, r_d, ok_d
        # serving: Poisson arrivals, 70/20/10 % sntrup761/857/1277, device pools
        if args.serve_seconds > 0:
            from paper_2106_08759_amd import serve
            rep = serve.serve(serve.GpuBackend(0), args.serve_rate, args.serve_seconds,
                              {761: 0.7, 857: 0.2, 1277: 0.1}, wl.SEED,
                              refill={761: 16384, 857: 8192, 1277: 4096}, blocks=4, tune=True)
            extras["serving"] = {k: rep[k] for k in ("rate_req_per_s", "seconds", "requests", "served",
                                                     "keys_per_s", "latency_ms", "latency_ms_by_p", "workspaces",
                                                     "hbm_used_bytes")}

    out = {
        "metric": "sntrup761 keys/sec on 1 MI355X (bit-exact)",
        "value": round(keys_per_s, 1),
        "unit": "keys/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic (seeded ChaCha20 keys; seed bytes 0x00..0x1f)",
        "config": {"workload": "sntrup%d batched KeyGen, N=%d keys, Montgomery group size %d%s" % (
                       p, n, cfg["group_size"], ", batched R/3 reciprocals" if cfg.get("r3_batch") else ""),
                   "p": p, "q": prm.q, "w": prm.w, "n_keys": n, "group_size": cfg["group_size"],
                   "inverse_share": cfg["inverse_share"], "lanes_per_key": cfg["lanes_per_key"],
                   "r3_batch": cfg["r3_batch"], "recip_jump": cfg["recip_jump"], "group_form": cfg["group_form"],
                   "product_engine": "int8 matrix cores" if cfg["product_engine"] == 1 else "v_dot2",
                   "launch": ("one persistent fused kernel per call" if cfg.get("persistent") else
                              "one captured hipGraph per call (stages on one stream)" if cfg["use_graph"] else
                              "eager launches: prefix kernel on a side stream beside the R/3 stage")},
        "roofline": roofline,
        "stages": stage_fracs,
        "output_GBps": round(n * (prm.pk_bytes + prm.sk_bytes) / (ms_per_step / 1e3) / 1e9, 2),
        "verified_keys": verified,
        "wall_s": round(wall, 3),
    }
    out.update(extras)
    if tuned is not None:
        out["autotune"] = {"config": tuned["config"], "use_graph": tuned.get("use_graph"),
                           "eager_ms": tuned.get("eager_ms"), "graph_ms": tuned.get("graph_ms"),
                           "cached": tuned["cached"],
                           "table_ms": {"%sG%d/W%d/L%d/R%dx%dx%d%s" % (
                               "P:" if r.get("persistent") else "B:" if r.get("r3_batch") else "",
                               r["group_size"], r["inverse_share"], r["lanes_per_key"], r["retry_passes"],
                               r["retry_lanes_per_key"], r["retry_parallel_attempts"],
                               {0: "/plain-recips", 1: "", 2: "/jump-r3-only", 3: "/jump-r3"}[r.get("recip_jump", 1)]
                               + ("/tree" if r.get("group_form") else "")):
                               r["ms"]
                                        for r in tuned.get("table", [])}}
    if cb is not None:
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
