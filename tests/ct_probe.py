"""Runs the secret-dependent operations of KeyGen on three different secret
inputs each (same shapes), one after the other, for a hardware-counter run
(test_gpu_constant_time.py runs it under rocprofv3 --pmc): the R/3 reciprocal
(bitsliced divsteps, 1 to 64 lanes per key), the R/q reciprocal (plain divstep
loop and jump divsteps), the R/q product with a small and with a big
operand, the Short and small samplers, and the encapsulation and
decapsulation core.  Prints one line per operation."""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)


def main():
    import torch
    import paper_2106_08759_amd as nk
    from paper_2106_08759_amd import workloads as wl

    ctx = nk.Context(0)
    p, n = 761, 256
    rng = np.random.default_rng(11)

    def dev(a):
        return torch.from_numpy(np.ascontiguousarray(a)).cuda()

    # three secret inputs per operation: random draws of the operation's domain
    smalls = [dev(rng.integers(-1, 2, size=(n, p)).astype(np.int8)) for _ in range(3)]
    bigs = [dev(wl.random_rq(p, n, tag=30 + i)) for i in range(3)]
    seeds = [bytes(rng.integers(0, 256, size=32).astype(np.uint8)) for _ in range(3)]
    torch.cuda.synchronize()
    for lpk in (1, 2, 4, 8, 16, 32, 64):
        ctx.set_config(p, lanes_per_key=lpk)
        for s in smalls:
            ctx.recip_r3(p, s)
        torch.cuda.synchronize()
        print("recip_r3 lanes_per_key=%d" % lpk, flush=True)
    for jump in (0, 1):
        ctx.set_config(p, recip_jump=jump)
        for b in bigs:
            ctx.recip_rq(p, b)
        torch.cuda.synchronize()
        print("recip_rq recip_jump=%d" % jump, flush=True)
    for b in bigs:
        ctx.mul_rq(p, bigs[0], b)
    for s in smalls:
        ctx.mul_rq(p, s.to(torch.int16), bigs[0], small_a=True)
    torch.cuda.synchronize()
    print("mul_rq big and small", flush=True)
    for sd in seeds:
        ctx.sample(p, sd, 0, n)
    torch.cuda.synchronize()
    print("samplers", flush=True)
    # encapsulation (secret: r, from the seed) and decapsulation (secret: f
    # and 1/g; the weight check and its fallback are selects)
    for sd in seeds:
        ctx.batch_encap(p, sd, 0, bigs[0])
    cts = [(3 * torch.div(b, 3, rounding_mode="trunc")).contiguous() for b in bigs]
    for i in range(3):
        ctx.batch_decap(p, cts[0], smalls[i], smalls[(i + 1) % 3], bigs[0])
    torch.cuda.synchronize()
    print("kem encap and decap", flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
