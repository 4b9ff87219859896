#!/usr/bin/env python3
"""Benchmark: CKKS key-switch rotations/s at N=2^16, L=24 on one MI355X.

A step is one batch of ROT_PER_STEP slot rotations (Galois automorphism +
hybrid key switching: ModUp -> key inner product -> ModDown) of one
ciphertext at the top level (L=24 limbs: one 60-bit + 23 50-bit primes,
K=8 60-bit special primes, dnum=3), cycling through three resident rotation
keys (3 x 96 MiB, more than the 256 MB Infinity Cache) so keys stream from
HBM.  Inputs (ciphertext and key limbs) are seeded uniform residues, which is
what RLWE ciphertexts and keys look like; they are resident in HBM before the
timed region starts.

Prints one JSON line (see the design doc for the fields).  --gpus > 1 is refused:
this build targets one GPU.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

CFG = dict(log_n=16, q_bits=[60] + [50] * 23, p_bits=[60] * 8, alpha=8, log_scale=50)
ROTATIONS = [1, -1, 32]
ROT_PER_STEP = 48
HBM_PEAK_GBS = 8000.0
# 64-bit Shoup modular product = 10 32-bit multiplies (4 for the high word,
# 3 + 3 for two low words); 32-bit multiplies issue at half the VALU rate:
# 256 CUs * 4 SIMDs * 16 lanes / 2 * 2.4 GHz = 19.66e12 mul32/s.
ALU_PEAK_GMODMUL = 256 * 4 * 16 / 2 * 2.4 / 10.0  # = 1966 Gmodmul/s


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget for the CPU baseline sample")
    return ap.parse_args()


def cpu_baseline(budget_s):
    """The oracle (test infrastructure) timed on the host on a bounded sample:
    whole single rotations at the same parameters, as many as fit the budget."""
    from oracle import ckks
    import synth

    pr = ckks.Params(**CFG)
    ctx = ckks.Context(pr)
    sk, pk = ctx.keygen(7)
    key = ctx.gen_rotation_key(sk, ROTATIONS[0], 7)
    ct = ctx.encrypt(pk, ctx.encode(synth.uniform_slots(1, pr.n // 2), pr.scale, pr.L), 7)
    done, t0 = 0, time.perf_counter()
    while True:
        ctx.rotate(ct, ROTATIONS[0], {ROTATIONS[0]: key})
        done += 1
        el = time.perf_counter() - t0
        if el > budget_s or done >= 50:
            break
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": done / el, "unit": "rotations/s", "cores": threads, "kind": "oracle",
            "sample": "%d single key-switch rotations at N=2^16 L=24 K=8 dnum=3 (%.1f s)" % (done, el)}


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: this build measures one GPU only (--gpus %d refused)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch

    import synth
    from paper_2510_03996_amd import he

    torch.cuda.init()
    dev = torch.device("cuda", 0)
    ctx = he.Context(CFG["log_n"], CFG["q_bits"], CFG["p_bits"], CFG["alpha"])
    N, L, K = ctx.n, ctx.L, ctx.K
    dnum = ctx.dnum
    # resident inputs: three rotation keys and one ciphertext (seeded residues)
    for i, r in enumerate(ROTATIONS):
        key = synth.residues(100 + i, ctx.moduli, N)  # [L+K][N] pattern, tiled to the key shape
        full = he.to_device(key).unsqueeze(0).unsqueeze(0).expand(dnum, 2, L + K, N).contiguous()
        ctx.key_upload(r, full)
    ct = ctx.ct_from_numpy(synth.residues(1, ctx.moduli[:L], N)[None].repeat(2, 0), 2.0 ** 50)
    outs = [ctx.new_ct(L), ctx.new_ct(L)]
    stream = torch.cuda.current_stream()

    def step():
        for t in range(ROT_PER_STEP):
            ctx.rotate(ct, ROTATIONS[t % len(ROTATIONS)], out=outs[t & 1], stream=stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    rot_s = args.steps * ROT_PER_STEP / el

    # live per-kernel roofline: same steps again with HIP events around each launch
    he.lib().he_profile_begin(ctx.h)
    for _ in range(args.steps):
        step()
    buf = he.ctypes.create_string_buffer(1 << 16)
    n = he.lib().he_profile_end(ctx.h, buf, len(buf))
    kern = json.loads(buf.value[:n].decode())
    dom_name = max(kern, key=lambda k: kern[k]["ms"])
    d = kern[dom_name]
    sec = d["ms"] / 1e3
    gbs = d["bytes"] / sec / 1e9
    gmm = d["modmul"] / sec / 1e9
    hbm_frac, alu_frac = gbs / HBM_PEAK_GBS, gmm / ALU_PEAK_GMODMUL
    if alu_frac >= hbm_frac:
        roof = {"bound": "alu", "achieved": round(gmm, 1), "peak": round(ALU_PEAK_GMODMUL, 1), "unit": "Gmodmul/s",
                "frac": round(alu_frac, 4)}
    else:
        roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(hbm_frac, 4)}
    roof.update({"traffic": None, "kernel": dom_name, "avg_launch_us": round(d["ms"] / d["launches"] * 1e3, 2),
                 "hbm_GBs": round(gbs, 1), "hbm_frac": round(hbm_frac, 4), "gmodmul_s": round(gmm, 1)})
    ks_bytes = 2 * L * N * 8 + 2 * dnum * (L + K) * N * 8 + 2 * L * N * 8
    result = {
        "metric": "key-switch rotations/s at N=2^16 L=24",
        "value": round(rot_s, 1),
        "unit": "rotations/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(el / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u64",
        "data": "synthetic",
        "config": {"workload": "plain he_rotate, one ciphertext at a time, N=2^16 L=24 K=8 dnum=3, "
                               "%d rotations per step cycling %d resident keys" % (ROT_PER_STEP, len(ROTATIONS)),
                   "log_n": 16, "limbs": L, "special_primes": K, "dnum": dnum},
        "keyswitch_hbm_frac": round(rot_s * ks_bytes / 1e9 / HBM_PEAK_GBS, 4),
        "roofline": roof,
        "kernels": {k: {"launches": v["launches"], "ms": round(v["ms"], 3)} for k, v in kern.items()},
    }
    if not args.no_cpu:
        result["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    ctx.close()
    print(json.dumps(result))


if __name__ == "__main__":
    main()
