#!/usr/bin/env python3
"""Benchmark of the MI355X CKKS hot path under FHEON's encrypted CNN layers.

Headline (``value``): key-switch rotations/s at N=2^16, L=24 — a step is one
batch of ROT_PER_STEP plain slot rotations (Galois automorphism + hybrid key
switching: ModUp -> key inner product -> ModDown) of one ciphertext at the
top level (one 60-bit + 23 50-bit primes, K=9 50-bit special primes,
dnum=3), cycling through three resident rotation keys (3 x 99 MiB, more than
the 256 MB Infinity Cache) so keys stream from HBM.

Measured in the same run and reported beside it:
  * roofline of the dominant kernel, from HIP events around every launch;
  * layer latencies: the tiny conv (N=2^12), the LeNet-5-shaped stack
    (N=2^14), and the ResNet-20-shaped conv A / conv B / global pooling / FC
    (N=2^16); convolutions at the library default of two layer streams, the
    ResNet-shaped ones also on one and four (`*_streams<n>_ms`);
  * batched key switching: 64 ciphertexts with seeded hoisted rotation sets
    of 9-49 indices from a 7x7-window key pool and 1-32 outputs each,
    batched + graph-captured vs the per-op path, same GPU;
  * serving: Poisson arrivals of LeNet-shaped (3/4) and ResNet-shaped (1/4)
    requests, continuous batching vs sequential FIFO on the same trace;
  * the CPU oracle on a bounded sample (a baseline, not a target).
Inputs are seeded synthetic residues (what RLWE ciphertexts, keys and
encoded plaintexts look like), resident in HBM before each timed region.

--gpus > 1 is refused: the benchmark measures one GPU.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

CFG0 = dict(log_n=12, q_bits=[54, 40, 40], p_bits=[55], alpha=1)
CFG1 = dict(log_n=14, q_bits=[60] + [45] * 7, p_bits=[60, 60], alpha=2)
CFG2 = dict(log_n=16, q_bits=[60] + [50] * 23, p_bits=[50] * 9, alpha=8)
# layer-stream counts timed besides the library default (2) for the ResNet-shaped convolutions
LAYER_STREAMS = (1, 4)
ROTATIONS = [1, -1, 32]
ROT_PER_STEP = 48
HBM_PEAK_GBS = 8000.0
# ALU peaks of one modular product from the unit counts (256 CUs * 4 SIMDs *
# 16 lanes * 2.4 GHz = 39.3e12 full-rate lane operations/s): an integer Shoup
# product (64-bit primes) is 10 32-bit multiplies at half rate; a centred FP64
# product (primes below 2^50) is 6 full-rate FP64 operations.  The library
# prices every profiled launch by the arithmetic of its limbs (`ideal_ms`);
# a kernel's peak is its products divided by that ideal time.
ALU_PEAK_GMODMUL_INT = 256 * 4 * 16 * 2.4 / 2 / 10.0  # = 1966 Gmodmul/s
ALU_PEAK_GMODMUL_F64 = 256 * 4 * 16 * 2.4 / 6.0  # = 6554 Gmodmul/s


def recorded_traffic(kernel):
    """HBM bytes per launch of `kernel` from the committed counter passes
    (profiles/traffic_*.json), or None when none were taken or the NTT sources
    changed since (the file records their sha256)."""
    import glob
    import hashlib

    src = "".join(open(os.path.join(ROOT, "paper_2510_03996_amd", "csrc", f)).read()
                  for f in ("ntt.hip", "ntt_core.h", "modarith.h"))
    h = hashlib.sha256(src.encode()).hexdigest()
    for fn in glob.glob(os.path.join(ROOT, "profiles", "traffic_*.json")):
        d = json.load(open(fn))
        if d.get("kernel") == kernel and d.get("source_sha256") == h:
            return d["traffic_bytes_per_launch"]
    return None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--no-cpu", action="store_true", help="skip the oracle CPU baseline")
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="budget for the CPU baseline sample")
    ap.add_argument("--only-headline", action="store_true", help="skip layers / batched / serving sections")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run three 256 MiB device-to-device copies (the reference kernel that scales "
                         "the FETCH_SIZE / WRITE_SIZE counters to bytes)")
    ap.add_argument("--only", choices=["hoisted", "layers", "bootstrap", "batched", "serving"], default=None,
                    help="run the headline plus one section (profiling runs)")
    ap.add_argument("--serve-requests", type=int, default=300)
    return ap.parse_args()


def log(msg):
    print("[bench] " + msg, file=sys.stderr, flush=True)


def new_ctx(cfg):
    from paper_2510_03996_amd import he

    return he.Context(cfg["log_n"], cfg["q_bits"], cfg["p_bits"], cfg["alpha"])


def upload_synthetic_keys(ctx, keys, seed, relin=False):
    import synth
    from paper_2510_03996_amd import he

    ids = list(keys) + ([he.KEY_RELIN] if relin else [])
    for t, r in enumerate(ids):
        k = synth.device_residues(seed * 7919 + t, ctx.moduli, ctx.n, lead=(ctx.dnum, 2))
        ctx.key_upload(r, k)


def register_synthetic_keys_on_host(ctx, keys, seed):
    """The keys upload_synthetic_keys(ctx, keys, seed) makes, held instead as
    host copies that the library loads on demand."""
    import synth

    for t, r in enumerate(keys):
        k = synth.device_residues(seed * 7919 + t, ctx.moduli, ctx.n, lead=(ctx.dnum, 2))
        ctx.key_host_register(r, k.cpu().numpy().view("uint64"))


def synthetic_pts(ctx, count, level, seed, scale):
    import synth
    from paper_2510_03996_amd import he

    if count == 0:
        return []
    block = synth.device_residues(seed, ctx.moduli[:level], ctx.n, lead=(count,))
    return [he.Plaintext(block[i], scale) for i in range(count)]


def synthetic_ct(ctx, level, seed, scale):
    import synth
    from paper_2510_03996_amd import he

    d = synth.device_residues(seed, ctx.moduli[:level], ctx.n, lead=(2,))
    return he.Ciphertext(d.contiguous(), level, scale)


def timed(fn, reps, stream):
    import torch

    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    stream.synchronize()
    return (time.perf_counter() - t0) / reps


# ---------------------------------------------------------------- headline
def headline(args):
    import torch

    import synth
    from paper_2510_03996_amd import he

    ctx = new_ctx(CFG2)
    N, L, K, dnum = ctx.n, ctx.L, ctx.K, ctx.dnum
    upload_synthetic_keys(ctx, ROTATIONS, 1)
    ct = synthetic_ct(ctx, L, 2, 2.0 ** 50)
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
    # live per-kernel roofline: the same steps again with HIP events around each launch
    ctx.profile_begin()
    for _ in range(args.steps):
        step()
    kern = ctx.profile_end()
    limb = N * 8
    # the algorithmic bytes of one key switch (read c0 and c1, the key, write
    # the output: 2L + 2 dnum (L+K) + 2L limbs) split over the launches that
    # move them, each counted once: c1 by its first reader (the inverse
    # pass 2), the key by the fused inner-product kernel, c0 and the output by
    # the last forward pass
    share = {"ntt_inv_pass2": L * limb, "ntt_fwd_pass2_ip": 2 * dnum * (L + K) * limb,
             "ntt_fwd_pass2_moddown": (L + 2 * L) * limb}
    ks_bytes = 2 * L * limb + 2 * dnum * (L + K) * limb + 2 * L * limb
    assert sum(share.values()) == ks_bytes
    n_ks = args.steps * ROT_PER_STEP
    table = {}
    for name, v in kern.items():
        us = v["ms"] / v["launches"] * 1e3
        table[name] = {"launches_per_keyswitch": round(v["launches"] / n_ks, 3), "avg_us": round(us, 2),
                       "io_bytes": int(v["bytes"] / v["launches"]), "io_GBs": round(v["bytes"] / v["ms"] / 1e6, 1),
                       "alg_bytes": share.get(name, 0),
                       "alg_GBs": round(share.get(name, 0) / us / 1e3, 1)}
    # the dominant kernel: the longest one that moves algorithmic bytes
    dom_name = max((k for k in kern if share.get(k)), key=lambda k: kern[k]["ms"])
    d = kern[dom_name]
    sec = d["ms"] / d["launches"] / 1e3  # per launch
    gbs = share[dom_name] / sec / 1e9
    roof = {"bound": "hbm", "achieved": round(gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(gbs / HBM_PEAK_GBS, 4), "traffic": recorded_traffic(dom_name), "kernel": dom_name,
            "avg_launch_us": round(sec * 1e6, 2), "alg_bytes_per_launch": share[dom_name],
            "io_bytes_per_launch": int(d["bytes"] / d["launches"]),
            "io_GBs": round(d["bytes"] / d["launches"] / sec / 1e9, 1),
            "keyswitch_launches": table}
    roof["ntt_autotune"] = ctx.ntt_tuning()
    roof["conv_autotune"] = ctx.conv_tuning()
    ctx.close()
    return rot_s, el, roof, kern, ks_bytes, (L, K, dnum)


def two_stream_rotations(args):
    """Reported beside the value: the headline's independent rotations issued
    alternately on two streams (each stream with its own output buffer)."""
    import torch

    ctx = new_ctx(CFG2)
    upload_synthetic_keys(ctx, ROTATIONS, 1)
    ct = synthetic_ct(ctx, ctx.L, 2, 2.0 ** 50)
    outs = [ctx.new_ct(ctx.L), ctx.new_ct(ctx.L)]
    pair = (torch.cuda.current_stream(), torch.cuda.Stream())

    def step2():
        for t in range(ROT_PER_STEP):
            ctx.rotate(ct, ROTATIONS[t % len(ROTATIONS)], out=outs[t & 1], stream=pair[t & 1])

    for _ in range(args.warmup):
        step2()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step2()
    torch.cuda.synchronize()
    out = {"rotations_per_s": round(args.steps * ROT_PER_STEP / (time.perf_counter() - t0), 1),
           "workload": "the headline's rotations, issued alternately on two streams"}
    ctx.close()
    return out


# ---------------------------------------------------------------- hoisted rotation sets
def hoisted_sets(reps=20):
    """he_rotate_hoisted at N=2^16 L=24: the 3x3 conv window (8 rotations, W=32)
    and the 7x7 window plus 1024 (49 rotations), one ModUp per set; the key
    switches of a set at the library default of two streams, and on one
    (`<set>_streams1`) and four (`<set>_streams4`)."""
    import torch

    ctx = new_ctx(CFG2)
    sets = {"set8": [dy * 32 + dx for dy in (-1, 0, 1) for dx in (-1, 0, 1) if (dy, dx) != (0, 0)],
            "set49": [dy * 32 + dx for dy in range(-3, 4) for dx in range(-3, 4) if (dy, dx) != (0, 0)] + [1024]}
    upload_synthetic_keys(ctx, sorted(set(sets["set8"]) | set(sets["set49"])), 3)
    ct = synthetic_ct(ctx, ctx.L, 4, 2.0 ** 50)
    stream = torch.cuda.current_stream()
    out = {}
    for n_streams, suffix in ((2, ""), (1, "_streams1"), (4, "_streams4")):
        ctx.layer_streams(n_streams)
        for name, rs in sets.items():
            outs = [ctx.new_ct(ctx.L) for _ in rs]
            for _ in range(2):
                ctx.rotate_hoisted(ct, rs, outs=outs, stream=stream)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                ctx.rotate_hoisted(ct, rs, outs=outs, stream=stream)
            torch.cuda.synchronize()
            el = time.perf_counter() - t0
            out[name + suffix] = {"rotations": len(rs), "ms_per_set": round(el / reps * 1e3, 3),
                                  "rotations_per_s": round(reps * len(rs) / el, 1)}
            del outs
    ctx.close()
    return out


# ---------------------------------------------------------------- layers
def layer_latencies(reps=3):
    import torch

    from paper_2510_03996_amd import he, models

    out = {}
    s = torch.cuda.current_stream()
    # tiny conv, N=2^12
    c0 = new_ctx(CFG0)
    fm = he.fmap(1, 8, 8)
    pl = c0.conv2d_plan(fm, 1, 3, 1, 1)
    upload_synthetic_keys(c0, pl.keys(), 10)
    ct = synthetic_ct(c0, 3, 11, 2.0 ** 40)
    kp = synthetic_pts(c0, pl.n_kernel_pts, 3, 12, 2.0 ** 40)
    out["conv3x3_1x8x8_n12_ms"] = round(timed(lambda: c0.conv2d(ct, fm, 1, 3, 1, 1, kp, [], stream=s), reps, s) * 1e3, 3)
    c0.close()
    # LeNet-5-shaped stack, N=2^14
    c1 = new_ctx(CFG1)
    fm0, pc, pp, keys = models.lenet_plan(c1)
    upload_synthetic_keys(c1, keys, 20, relin=True)
    chain = models.lenet_chain(c1, synthetic_pts(c1, pc.n_kernel_pts, 8, 21, 2.0 ** 45),
                               synthetic_pts(c1, pp.n_mask_pts, 8, 22, 2.0 ** 45), 2.0 ** 45)
    ct = synthetic_ct(c1, 8, 23, 2.0 ** 45)

    def run_chain(ch, x):
        for st in ch.stages:
            x = st(x, s)
        return x

    out["lenet5_stack_n14_ms"] = round(timed(lambda: run_chain(chain, ct), reps, s) * 1e3, 3)
    # the same stack with the baby-step giant-step pooling compaction
    c1.mask_chains(he.CHAIN_BSGS)
    fm0, pc_b, pp_b, keys_b = models.lenet_plan(c1)
    upload_synthetic_keys(c1, keys_b, 20, relin=True)
    chain_b = models.lenet_chain(c1, synthetic_pts(c1, pc_b.n_kernel_pts, 8, 21, 2.0 ** 45),
                                 synthetic_pts(c1, pp_b.n_mask_pts, 8, 22, 2.0 ** 45), 2.0 ** 45)
    out["lenet5_stack_n14_bsgs_ms"] = round(timed(lambda: run_chain(chain_b, ct), reps, s) * 1e3, 3)
    lenet_ks_b = pc_b.key_switches + pp_b.key_switches + 2
    c1.close()
    # ResNet-20-shaped layers, N=2^16
    c2 = new_ctx(CFG2)
    fm0, pa, pb, pg, pf, keys = models.resnet_plan(c2)
    upload_synthetic_keys(c2, keys, 30)
    sc = 2.0 ** 50
    ct = synthetic_ct(c2, 24, 31, sc)
    ak, am = synthetic_pts(c2, pa.n_kernel_pts, 24, 32, sc), synthetic_pts(c2, pa.n_mask_pts, 24, 33, sc)
    out["resnet_convA_16x32x32_n16_ms"] = round(timed(lambda: c2.conv2d(ct, fm0, 16, 3, 1, 1, ak, am, stream=s), reps, s) * 1e3, 3)
    # the library default spreads output channels over the caller's stream and
    # one helper stream; the same layer on one stream and on four (same results)
    for n in LAYER_STREAMS:
        c2.layer_streams(n)
        out["resnet_convA_16x32x32_n16_streams%d_ms" % n] = round(
            timed(lambda: c2.conv2d(ct, fm0, 16, 3, 1, 1, ak, am, stream=s), reps, s) * 1e3, 3)
    c2.layer_streams(2)
    # conv A captured once into a graph (two layer streams inside) and replayed
    gs = torch.cuda.Stream()
    gout = c2.new_ct()
    c2.conv2d(ct, fm0, 16, 3, 1, 1, ak, am, out=gout, stream=gs)
    gs.synchronize()
    c2.capture_begin(gs)
    c2.conv2d(ct, fm0, 16, 3, 1, 1, ak, am, out=gout, stream=gs)
    graph = c2.capture_end(gs)
    out["resnet_convA_16x32x32_n16_graph_ms"] = round(timed(lambda: graph.launch(gs), reps, gs) * 1e3, 3)
    graph.close()
    # the same layers with the log-step input-channel sum (keys W^2, 2 W^2, 4 W^2, 8 W^2)
    c2.conv_channel_sum(he.CHSUM_LOG)
    pal = c2.conv2d_plan(fm0, 16, 3, 1, 1)
    pbl = c2.conv2d_plan(pa.out, 32, 3, 2, 1)
    upload_synthetic_keys(c2, sorted(set(pal.keys()) | set(pbl.keys())), 30)
    out["resnet_convA_16x32x32_n16_logsum_ms"] = round(
        timed(lambda: c2.conv2d(ct, fm0, 16, 3, 1, 1, ak, am, stream=s), reps, s) * 1e3, 3)
    c2.conv_channel_sum(he.CHSUM_CHAIN)
    del ak, am
    ctb = synthetic_ct(c2, 22, 34, sc)
    bk, bm = synthetic_pts(c2, pb.n_kernel_pts, 22, 35, sc), synthetic_pts(c2, pb.n_mask_pts, 22, 36, sc)
    out["resnet_convB_s2_n16_ms"] = round(timed(lambda: c2.conv2d(ctb, pa.out, 32, 3, 2, 1, bk, bm, stream=s), reps, s) * 1e3, 3)
    for n in LAYER_STREAMS:
        c2.layer_streams(n)
        out["resnet_convB_s2_n16_streams%d_ms" % n] = round(
            timed(lambda: c2.conv2d(ctb, pa.out, 32, 3, 2, 1, bk, bm, stream=s), reps, s) * 1e3, 3)
    c2.layer_streams(2)
    c2.conv_channel_sum(he.CHSUM_LOG)
    out["resnet_convB_s2_n16_logsum_ms"] = round(
        timed(lambda: c2.conv2d(ctb, pa.out, 32, 3, 2, 1, bk, bm, stream=s), reps, s) * 1e3, 3)
    # and with the baby-step giant-step stride compaction as well
    c2.mask_chains(he.CHAIN_BSGS)
    pbb = c2.conv2d_plan(pa.out, 32, 3, 2, 1)
    upload_synthetic_keys(c2, pbb.keys(), 30)
    out["resnet_convB_s2_n16_logsum_bsgs_ms"] = round(
        timed(lambda: c2.conv2d(ctb, pa.out, 32, 3, 2, 1, bk, bm, stream=s), reps, s) * 1e3, 3)
    c2.mask_chains(he.CHAIN_HORNER)
    c2.conv_channel_sum(he.CHSUM_CHAIN)
    # the paper's other striding forms of conv B: approach 2 (log-step column
    # moves) and the multi-channel pipeline (groups of the 16 input channels)
    stride_ks = {}
    for tag, on, off in (("logstride", lambda: c2.striding(he.STRIDE_LOG), lambda: c2.striding(he.STRIDE_EXTRACT)),
                         ("groups", lambda: c2.stride_groups(he.STRIDE_GROUP_IN),
                          lambda: c2.stride_groups(he.STRIDE_JOINT))):
        on()
        pv = c2.conv2d_plan(pa.out, 32, 3, 2, 1)
        upload_synthetic_keys(c2, pv.keys(), 30)
        vm = synthetic_pts(c2, pv.n_mask_pts, 22, 36, sc)
        out["resnet_convB_s2_n16_%s_ms" % tag] = round(
            timed(lambda: c2.conv2d(ctb, pa.out, 32, 3, 2, 1, bk, vm, stream=s), reps, s) * 1e3, 3)
        stride_ks["resnet_convB_" + tag] = pv.key_switches
        off()
        del vm
    del bk, bm
    ctg = synthetic_ct(c2, 17, 37, sc)
    gm = synthetic_pts(c2, pg.n_mask_pts, 17, 38, sc)
    out["resnet_gap_32x16x16_n16_ms"] = round(timed(lambda: c2.avgpool(ctg, pb.out, 0, 1, gm, stream=s), reps, s) * 1e3, 3)
    c2.mask_chains(he.CHAIN_BSGS)
    pgb = c2.avgpool_plan(pb.out, 0, 1)
    upload_synthetic_keys(c2, pgb.keys(), 30)
    out["resnet_gap_32x16x16_n16_bsgs_ms"] = round(
        timed(lambda: c2.avgpool(ctg, pb.out, 0, 1, gm, stream=s), reps, s) * 1e3, 3)
    c2.mask_chains(he.CHAIN_HORNER)
    ctf = synthetic_ct(c2, 16, 39, sc)
    fr, fmk = synthetic_pts(c2, 10, 16, 40, sc), synthetic_pts(c2, 1, 16, 41, sc)
    out["resnet_fc_64x10_n16_ms"] = round(timed(lambda: c2.fc(ctf, 64, 10, fr, fmk, stream=s), reps, s) * 1e3, 3)
    c2.fc_form(he.FC_DIAG)
    pfd = c2.fc_plan(64, 10)
    upload_synthetic_keys(c2, pfd.keys(), 30)
    fd = synthetic_pts(c2, pfd.n_kernel_pts, 16, 40, sc)
    out["resnet_fc_64x10_n16_diag_ms"] = round(timed(lambda: c2.fc(ctf, 64, 10, fd, [], stream=s), reps, s) * 1e3, 3)
    c2.fc_form(he.FC_ROWS)
    del fd
    # zero padding by masked taps: 7x7 / stride 2 / padding 3 (the ResNet-34 stem shape), 3 x 32 x 32 -> 8
    fmp = he.fmap(3, 32, 32)
    p7 = c2.conv2d_plan(fmp, 8, 7, 2, 3)
    upload_synthetic_keys(c2, p7.keys(), 45)
    ctp = synthetic_ct(c2, 24, 46, sc)
    pk7, pm7 = synthetic_pts(c2, p7.n_kernel_pts, 24, 47, sc), synthetic_pts(c2, p7.n_mask_pts, 24, 48, sc)
    out["conv7x7_s2_p3_3x32x32_n16_ms"] = round(
        timed(lambda: c2.conv2d(ctp, fmp, 8, 7, 2, 3, pk7, pm7, stream=s), reps, s) * 1e3, 3)
    del pk7, pm7
    # the paper's secure ReLU: degree-59 Chebyshev interpolant, beta = 4 scale mask
    upload_synthetic_keys(c2, [], 42, relin=True)
    cheb = he.cheb_relu_coeffs(4.0, 59)
    ctr = synthetic_ct(c2, 24, 43, sc)
    rmask = synthetic_pts(c2, 1, 24, 44, sc)[0]
    out["relu_cheb59_n16_ms"] = round(timed(lambda: c2.cheb(ctr, cheb, sc, scale_mask=rmask, stream=s), reps, s) * 1e3, 3)
    c2.layer_streams(1)
    out["relu_cheb59_n16_streams1_ms"] = round(
        timed(lambda: c2.cheb(ctr, cheb, sc, scale_mask=rmask, stream=s), reps, s) * 1e3, 3)
    c2.layer_streams(2)
    out["key_switches"] = {"conv3x3_n12": 8, "lenet5_stack": pc.key_switches + pp.key_switches + 2,
                           "resnet_convA": pa.key_switches, "resnet_convB": pb.key_switches,
                           "resnet_gap": pg.key_switches, "resnet_fc": pf.key_switches,
                           "conv7x7_s2_p3": p7.key_switches, "relu_cheb59": he.cheb_plan(cheb, True)[1],
                           "resnet_convA_logsum": pal.key_switches, "resnet_convB_logsum": pbl.key_switches,
                           "resnet_convB_logsum_bsgs": pbb.key_switches, "resnet_gap_bsgs": pgb.key_switches,
                           **stride_ks,
                           "lenet5_stack_bsgs": lenet_ks_b, "resnet_fc_diag": pfd.key_switches}
    c2.close()
    return out


# ---------------------------------------------------------------- bootstrapping
def bootstrap_latency(reps=3):
    """Bootstrapping at N=2^16, L=24: ModRaise of a level-1 ciphertext to 24
    limbs, coefficient/slot transforms of three (or four) levels, EvalMod
    (K ~ 16) on the real and imaginary parts as the cosine of degree 39 with
    three double angles (15 levels consumed, the result at level 9; 17 and
    level 7 with four-level transforms) and as the sine of degree 159 (14
    levels, level 10).  Keys and plaintexts are synthetic residues of the
    real shapes."""
    import torch

    from paper_2510_03996_amd import he

    out = {}
    s = torch.cuda.current_stream()
    sc = 2.0 ** 50
    c2 = new_ctx(CFG2)
    plans = {lv: he.boot_plan(16, lv, key_switches=True) for lv in (3, 4)}
    keys = sorted(set(plans[3][0]) | set(plans[4][0]))
    upload_synthetic_keys(c2, keys + [he.KEY_CONJ], 60, relin=True)
    ctb1 = synthetic_ct(c2, 1, 67, sc)
    ks = {}
    for name, nl, deg, r in (("bootstrap_n16", 3, 39, 3), ("bootstrap_n16_levels4", 4, 39, 3),
                             ("bootstrap_n16_sine159", 3, 159, 0)):
        brots, bcounts, bks = plans[nl]
        bdesc = he.boot_desc(nl, deg, 12.0, sc, double_angles=r)
        bK, _, bcs, bss = c2.boot_scales(bdesc)
        bcoef = he.boot_mod_coeffs(bK, deg, r)
        blv = he.cheb_plan(bcoef, False)
        bcts = [p for g in range(nl) for p in synthetic_pts(c2, bcounts[g], 24 - g, 61 + g, bcs[g])]
        bstc = [p for g in range(nl)
                for p in synthetic_pts(c2, bcounts[nl + g], 24 - nl - blv[0] - r - g, 64 + g, bss[g])]
        out[name + "_ms"] = round(timed(lambda: c2.bootstrap(ctb1, bdesc, bcts, bstc, bcoef, stream=s), reps, s)
                                  * 1e3, 3)
        if name == "bootstrap_n16":
            # independent ciphertexts refreshed concurrently, one per stream
            # (each stream its own lane): time per ciphertext
            sts = [torch.cuda.Stream() for _ in range(4)]
            outs = [c2.new_ct() for _ in sts]

            def run_all():
                for st, o in zip(sts, outs):
                    c2.bootstrap(ctb1, bdesc, bcts, bstc, bcoef, out=o, stream=st)

            run_all()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(reps):
                run_all()
            torch.cuda.synchronize()
            out[name + "_4streams_ms_per_ct"] = round((time.perf_counter() - t0) / (reps * len(sts)) * 1e3, 3)
            del outs
        ks[name] = bks + 1 + 2 * (blv[1] + r)
        out[name + "_output_level"] = 24 - 2 * nl - blv[0] - r
        del bcts, bstc
    out["key_switches"] = ks
    out["rotation_keys"] = {"levels3": len(plans[3][0]) + 1, "levels4": len(plans[4][0]) + 1}
    c2.close()
    return out


# ---------------------------------------------------------------- batched
def batched(reps=2):
    import torch

    import synth
    from paper_2510_03996_amd import he

    ctx = new_ctx(CFG2)
    L, N = ctx.L, ctx.n
    pool_offsets = [dy * 32 + dx for dy in range(-3, 4) for dx in range(-3, 4) if (dy, dx) != (0, 0)] + [1024]
    B = 64
    sets, outs = synth.rotation_sets(7, B, pool_offsets, 9, 49, 1, 32)
    upload_synthetic_keys(ctx, pool_offsets, 50)
    inp = synth.device_residues(51, ctx.moduli[:L], N, lead=(B, 2))
    pool = synth.device_residues(52, ctx.moduli[:L], N, lead=(64,))
    pos = lambda i, t: t
    pti = [[(i + 7 * o + 13 * pos(i, t)) % 64 for o in range(outs[i]) for t in range(len(sets[i]))] for i in range(B)]
    total = sum(outs)
    out_b = torch.empty((total, 2, L - 1, N), dtype=torch.int64, device="cuda")
    out_p = torch.empty_like(out_b)
    s = torch.cuda.Stream()
    res = {}
    rot = sum(len(x) for x in sets)
    with torch.cuda.stream(s):
        bt = he.Batch(ctx, inp, L, 2.0 ** 50, sets, outs, pool, 2.0 ** 50, pti, out_b, he.BATCH_GRAPH | he.BATCH_TUNE)
        tb = timed(lambda: bt.run(s), reps, s)
        pl = he.Batch(ctx, inp, L, 2.0 ** 50, sets, outs, pool, 2.0 ** 50, pti, out_p, 0)
        tp = timed(lambda: pl.run_plain(s), 1, s)
        same = bool(torch.equal(out_b, out_p))
        ctx.profile_begin()
        bt.run(s)
        s.synchronize()
        kern = ctx.profile_end()
        info = bt.info()
        tune = bt.tuning()
        bt.close()
        pl.close()
    ctx.close()
    res = {"workload": "64 ciphertexts N=2^16 L=24, hoisted sets of 9-49 rotations from a 49-key pool, 1-32 outputs",
           "rotations": info["rotations"], "outputs": info["outputs"], "mac_terms": sum(len(a) * m for a, m in zip(sets, outs)),
           "distinct_keys": info["keys"], "batched_s": round(tb, 4), "plain_s": round(tp, 4),
           "batched_rotations_per_s": round(rot / tb, 1), "plain_rotations_per_s": round(rot / tp, 1),
           "speedup": round(tp / tb, 3), "bit_identical": same, "autotune": tune,
           "kernels_ms": {k: round(v["ms"], 2) for k, v in kern.items()}}
    return res


# ---------------------------------------------------------------- serving
def synthetic_serving_models(seed=1):
    """LeNet-shaped (N=2^14) and ResNet-shaped (N=2^16) models with synthetic
    resident keys and weight plaintexts; returns (models, make_input)."""
    from paper_2510_03996_amd import he, models, serve

    c1 = new_ctx(CFG1)
    fm0, pc, pp, k1 = models.lenet_plan(c1)
    upload_synthetic_keys(c1, k1, seed * 100 + 1, relin=True)
    lenet = models.lenet_chain(c1, synthetic_pts(c1, pc.n_kernel_pts, 8, seed * 100 + 2, 2.0 ** 45),
                               synthetic_pts(c1, pp.n_mask_pts, 8, seed * 100 + 3, 2.0 ** 45), 2.0 ** 45)
    c2 = new_ctx(CFG2)
    c2.conv_channel_sum(he.CHSUM_LOG)  # the served ResNet-shaped chain sums input channels by doubling
    c2.mask_chains(he.CHAIN_BSGS)      # and compacts / gathers with baby-step giant-step chains
    c2.fc_form(he.FC_DIAG)             # and takes the diagonal fully connected form
    fm0, pa, pb, pg, pf, k2 = models.resnet_plan(c2)
    upload_synthetic_keys(c2, k2, seed * 100 + 4)
    sc = 2.0 ** 50
    resnet = models.resnet_chain(
        c2, synthetic_pts(c2, pa.n_kernel_pts, 24, seed * 100 + 5, sc), synthetic_pts(c2, pa.n_mask_pts, 24, seed * 100 + 6, sc),
        synthetic_pts(c2, pb.n_kernel_pts, 22, seed * 100 + 7, sc), synthetic_pts(c2, pb.n_mask_pts, 22, seed * 100 + 8, sc),
        synthetic_pts(c2, pg.n_mask_pts, 17, seed * 100 + 9, sc),
        synthetic_pts(c2, pf.n_kernel_pts, 16, seed * 100 + 10, sc), synthetic_pts(c2, pf.n_mask_pts, 16, seed * 100 + 11, sc))
    nbuf = 24
    # footprint: the request's lane, its convolutions' helper lane, in/out ciphertexts
    ms = {"lenet": serve.Model("lenet", c1, lenet.stages, nbuf,
                               c1.lane_bytes(nbuf) + c1.lane_bytes(4) + 4 * 2 * 8 * c1.n * 8),
          "resnet": serve.Model("resnet", c2, resnet.stages, nbuf,
                                c2.lane_bytes(nbuf) + c2.lane_bytes(4) + 4 * 2 * 24 * c2.n * 8)}
    ms["resnet"].key_ids, ms["resnet"].key_seed = list(k2), seed * 100 + 4  # the seed regenerates them

    def make_input(kind, sd):
        if kind == "lenet":
            return synthetic_ct(c1, 8, sd, 2.0 ** 45)
        return synthetic_ct(c2, 24, sd, sc)

    return ms, make_input


def serving(n_req):
    import numpy as np

    import synth
    from paper_2510_03996_amd import serve

    ms, make_input = synthetic_serving_models(3)
    srv = serve.Server(ms, slots=4)
    # mean plain service time from requests of each kind run alone, after one
    # untimed pass (first uses create lanes and helper streams)
    def warm_set():
        return [serve.Request(i, k, 0.0, make_input(k, 900 + i)) for i, k in enumerate(["lenet", "resnet", "lenet", "resnet"])]

    srv.serve(warm_set(), "sequential")
    w = srv.serve(warm_set(), "sequential")
    t_len = np.mean([r.t_done - r.t_admit for r in w if r.kind == "lenet"])
    t_res = np.mean([r.t_done - r.t_admit for r in w if r.kind == "resnet"])
    mean_service = 0.75 * t_len + 0.25 * t_res
    warm = 20
    res = {"workload": "Poisson arrivals, LeNet-5-shaped N=2^14 (3/4) and ResNet-20-shaped N=2^16 (1/4, log-step "
                       "channel sums, baby-step giant-step mask chains, diagonal FC) requests; %d requests timed after "
                       "%d warm-up requests of the same trace" % (n_req, warm),
           "requests": n_req, "warmup_requests": warm, "slots": 4,
           "service_ms": {"lenet": round(t_len * 1e3, 2), "resnet": round(t_res * 1e3, 2)}}
    kinds = ["lenet" if k == 0 else "resnet" for k in synth.request_mix(11, warm + n_req)]
    inputs = [make_input(k, 1000 + i) for i, k in enumerate(kinds)]

    def run(srv_, load, mode):
        rate = load / mean_service
        arr = synth.poisson_arrivals(12, rate, warm + n_req)
        reqs = [serve.Request(i, k, arr[i], inputs[i]) for i, k in enumerate(kinds)]
        srv_.max_active = 0
        done = srv_.serve(reqs, mode)
        timed = [r for r in done if r.id >= warm]
        lat = [r.latency for r in timed]
        span = max(r.t_done for r in timed) - min(r.arrival for r in timed)
        return rate, {"req_per_s": round(len(timed) / span, 2), "p50_ms": round(serve.percentile(lat, 50) * 1e3, 2),
                      "p99_ms": round(serve.percentile(lat, 99) * 1e3, 2)}

    for load in (0.7, 0.9, 1.5):
        row = {}
        for mode in ("sequential", "continuous"):
            log("serving load %.1f, %s" % (load, mode))
            rate, row[mode] = run(srv, load, mode)
        row["rate_req_s"] = round(rate, 2)
        row["max_in_flight"] = srv.max_active
        res["load_%.1f" % load] = row
    # a small admission budget: one request of each kind at a time fits, so
    # requests queue for memory, not for slots
    cap = ms["lenet"].footprint + ms["resnet"].footprint
    small = serve.Server(ms, slots=4, budget_bytes=cap)
    log("serving load 0.9, continuous, small byte budget")
    rate, row = run(small, 0.9, "continuous")
    res["small_budget_load_0.9"] = {"budget_bytes": cap, "rate_req_s": round(rate, 2), "continuous": row,
                                    "max_in_flight": small.max_active, "max_bytes": small.max_bytes}
    small.close()
    # dynamic key management: the ResNet-shaped model's keys held as host copies,
    # loaded on demand into a device budget of a third of its key set (LRU)
    rm = ms["resnet"]
    register_synthetic_keys_on_host(rm.ctx, rm.key_ids, rm.key_seed)
    budget = max(1, len(rm.key_ids) // 3) * rm.ctx.key_bytes()
    rm.ctx.key_cache_limit(budget)
    log("serving load 0.7, continuous, keys on demand")
    rate, row = run(srv, 0.7, "continuous")
    st = rm.ctx.key_cache_stats()
    res["dynamic_keys_load_0.7"] = {
        "resnet_keys": len(rm.key_ids), "device_budget_keys": budget // rm.ctx.key_bytes(), "continuous": row,
        "key_loads": st["loads"], "key_evictions": st["evictions"]}
    srv.close()
    for m in ms.values():
        m.ctx.close()
    return res


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _omp_threads(n):
    """Thread count of the oracle's OpenMP loops for the calls that follow."""
    import ctypes

    ctypes.CDLL("libgomp.so.1").omp_set_num_threads(int(n))


def _timed_cpu(fn, budget_s, max_reps):
    t0 = time.perf_counter()
    n = 0
    while True:
        fn()
        n += 1
        el = time.perf_counter() - t0
        if el >= budget_s or n >= max_reps:
            return el / n, n


def _oracle_costs(cfg, levels, keysets, seed):
    """Measured oracle times (s) of the layer primitives at the given levels:
    single rotation, modup share and per-rotation share of a hoisted set,
    pt-ct product, addition, rescale, relinearised product."""
    from oracle import ckks
    import synth

    pr = ckks.Params(**cfg)
    ctx = ckks.Context(pr)
    sk, pk = ctx.keygen(seed)
    keys = {r: ctx.gen_rotation_key(sk, r, seed) for r in keysets}
    rk = ctx.gen_relin_key(sk, seed)
    out = {}
    for l in levels:
        ct = ctx.encrypt(pk, ctx.encode(synth.uniform_slots(seed, pr.n // 2), pr.scale, l), seed)
        pt = ctx.encode(synth.uniform_slots(seed + 1, pr.n // 2), pr.scale, l)
        t1, _ = _timed_cpu(lambda: ctx.rotate(ct, keysets[0], keys), 0.0, 1)
        t4, _ = _timed_cpu(lambda: ctx.rotate_hoisted(ct, keysets[:4], keys), 0.0, 1)
        modup = max(0.0, (4 * t1 - t4) / 3)
        m = ctx.mul_plain(ct, pt)
        tm, _ = _timed_cpu(lambda: ctx.mul_plain(ct, pt), 0.05, 20)
        ta, _ = _timed_cpu(lambda: ctx.add(m, m), 0.05, 20)
        tr, _ = _timed_cpu(lambda: ctx.rescale(m), 0.05, 5) if l > 1 else (0.0, 0)
        trl, _ = _timed_cpu(lambda: ctx.mul_relin(ct, ct, rk), 0.0, 1)
        out[l] = {"rot": t1, "modup": modup, "apply": max(0.0, t1 - modup), "mul": tm, "add": ta, "rescale": tr,
                  "relin": trl}
    return out


class _CostEval:
    """Runs a layer schedule on slot vectors (the oracle's float simulation)
    and adds up the measured oracle time of every operation it issues, with
    costs linear in the level between the measured levels."""

    def __init__(self, slots, costs):
        from oracle import layers as LY

        self.sim = LY.SimEval(slots)
        self.costs = costs
        self.t = 0.0

    def _c(self, op, level):
        ls = sorted(self.costs)
        if len(ls) == 1:
            return self.costs[ls[0]][op]
        lo, hi = ls[0], ls[-1]
        a, b = self.costs[lo][op], self.costs[hi][op]
        return max(0.0, a + (b - a) * (level - lo) / (hi - lo))

    def rot_hoisted(self, x, rs):
        n = sum(1 for r in rs if r % self.sim.slots)
        if n == 1:
            self.t += self._c("rot", x.level)
        elif n > 1:
            self.t += self._c("modup", x.level) + n * self._c("apply", x.level)
        return self.sim.rot_hoisted(x, rs)

    def rot(self, x, r):
        return self.rot_hoisted(x, [r])[0]

    def mul_plain(self, x, pt):
        self.t += self._c("mul", x.level)
        return self.sim.mul_plain(x, pt)

    def add(self, a, b):
        self.t += self._c("add", a.level)
        return self.sim.add(a, b)

    def rescale(self, x):
        self.t += self._c("rescale", x.level)
        return self.sim.rescale(x)

    def mul_relin(self, a, b):
        self.t += self._c("relin", a.level)
        return self.sim.mul_relin(a, b)

    def mul_const(self, x, c, scale):
        self.t += self._c("mul", x.level)
        return self.sim.mul_const(x, c, scale)

    def add_const(self, x, c):
        self.t += self._c("add", x.level)
        return self.sim.add_const(x, c)

    def drop(self, x, level):
        return self.sim.drop(x, level)

    def with_scale(self, x, sc):
        return self.sim.with_scale(x, sc)

    def modulus(self, i):
        return self.sim.modulus(i)


def _lenet_cost(costs):
    import numpy as np

    from oracle import layers as LY
    import synth

    slots = 1 << 13
    fm = LY.FMap(1, 28, 28)
    f1 = LY.conv_out_map(fm, 6, 5, 1, 0, slots)
    kern, _ = LY.conv_plaintexts(fm, synth.conv_weights(1, 6, 1, 5, 0.1), 1, 0, slots)
    ev = _CostEval(slots, costs)
    x = LY.SimCt(np.zeros(slots), 8)
    y, f1 = LY.conv2d(ev, x, fm, 6, 5, 1, 0, kern, [], slots)
    p = LY.relu_poly4(ev, y, 2.0 ** 45)
    LY.avgpool(ev, p, f1, 2, 2, LY.avgpool_plaintexts(f1, 2, 2, slots))
    return ev.t


def _resnet_costs(costs):
    """Costed times of the ResNet-shaped layers (paper's schedules, one stream)."""
    import numpy as np

    from oracle import layers as LY
    import synth

    slots = 1 << 15
    out = {}
    fm0 = LY.FMap(16, 32, 32, reps=2)
    ka, ma = LY.conv_plaintexts(fm0, synth.conv_weights(2, 16, 16, 3, 0.1), 1, 1, slots)
    ev = _CostEval(slots, costs)
    ya, fa = LY.conv2d(ev, LY.SimCt(np.zeros(slots), 24), fm0, 16, 3, 1, 1, ka, ma, slots)
    out["resnet_convA"] = ev.t
    kb, mb = LY.conv_plaintexts(fa, synth.conv_weights(3, 32, 16, 3, 0.1), 2, 1, slots)
    ev = _CostEval(slots, costs)
    yb, fb = LY.conv2d(ev, ya, fa, 32, 3, 2, 1, kb, mb, slots)
    out["resnet_convB"] = ev.t
    ev = _CostEval(slots, costs)
    yg = LY.gap(ev, yb, fb, LY.gap_plaintexts(fb, slots))
    out["resnet_gap"] = ev.t
    rows, masks = LY.fc_plaintexts(synth.fc_weights(4, 10, 64, 0.1), slots)
    ev = _CostEval(slots, costs)
    LY.fc(ev, yg if not isinstance(yg, tuple) else yg[0], 64, 10, rows, masks)
    out["resnet_fc"] = ev.t
    return out


def cpu_baseline(budget_s):
    """The oracle (test infrastructure, untuned) on the host, in this run, at
    all cores and at one thread: whole single rotations at the headline
    parameters (the value), the tiny convolution, the LeNet-shaped stack and
    (all cores only) a bootstrap at N=2^16 measured whole, and the
    ResNet-shaped layers costed from measured oracle primitives (each
    layer's schedule run on slot vectors, every operation priced by the
    oracle's measured time at its level)."""
    from oracle import ckks, layers as LY
    import numpy as np
    import synth

    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    res = {"unit": "rotations/s", "cores": cores, "kind": "oracle", "cpu_model": _cpu_model()}
    cfg2 = dict(CFG2, log_scale=50)
    pr = ckks.Params(**cfg2)
    ctx = ckks.Context(pr)
    sk, pk = ctx.keygen(7)
    key = {ROTATIONS[0]: ctx.gen_rotation_key(sk, ROTATIONS[0], 7)}
    ct = ctx.encrypt(pk, ctx.encode(synth.uniform_slots(1, pr.n // 2), pr.scale, pr.L), 7)
    layers = {}
    for threads in ((cores, 1) if cores > 1 else (1,)):
        _omp_threads(threads)
        tag = "threads_%d" % threads
        log("cpu baseline: %d thread(s)" % threads)
        t_rot, n_rot = _timed_cpu(lambda: ctx.rotate(ct, ROTATIONS[0], key), budget_s / 3 if threads > 1 else 0.0,
                                  50)
        if threads == cores:
            res["value"] = round(1.0 / t_rot, 3)
            res["sample"] = ("%d single key-switch rotations at N=2^16 L=24 K=9 dnum=3 on %d threads; "
                             "layers below per thread count" % (n_rot, cores))
        else:
            res["single_thread_rotations_per_s"] = round(1.0 / t_rot, 4)
        # tiny conv, N=2^12, measured whole
        c0 = ckks.Context(ckks.Params(**dict(CFG0, log_scale=40)))
        s0, p0 = c0.keygen(8)
        fm = LY.FMap(1, 8, 8)
        k0 = {r: c0.gen_rotation_key(s0, r, 8) for r in LY.conv_rotations(fm, 1, 3, 1, 1, c0.n // 2)}
        kern, masks = LY.conv_plaintexts(fm, synth.conv_weights(10, 1, 1, 3, 0.1), 1, 1, c0.n // 2)
        kp = [c0.encode(v, c0.pr.scale, c0.pr.L) for v in kern]
        x0 = c0.encrypt(p0, c0.encode(LY.pack(synth.image(10, 1, 8, 8), fm, c0.n // 2), c0.pr.scale, c0.pr.L), 8)
        ev0 = LY.HEEval(c0, k0)
        t_c0, _ = _timed_cpu(lambda: LY.conv2d(ev0, x0, fm, 1, 3, 1, 1, kp, masks, c0.n // 2), 0.5, 5)
        layers.setdefault("conv3x3_1x8x8_n12_ms", {})[tag] = round(t_c0 * 1e3, 2)
        # primitives for the costed layers
        c1costs = _oracle_costs(dict(CFG1, log_scale=45), [8, 2], [1, 2, 3, 4], 9)
        first = threads == cores
        c2costs = _oracle_costs(cfg2, [24, 12], [1, 2, 3, 4], 9) if first else None
        if first:
            # LeNet-shaped stack measured whole on all cores (and costed, as a check of the model)
            c1 = ckks.Context(ckks.Params(**dict(CFG1, log_scale=45)))
            s1, p1 = c1.keygen(9)
            fm1 = LY.FMap(1, 28, 28)
            slots = c1.n // 2
            f1 = LY.conv_out_map(fm1, 6, 5, 1, 0, slots)
            rots = sorted(set(LY.conv_rotations(fm1, 6, 5, 1, 0, slots)) | set(LY.avgpool_rotations(f1, 2, 2)))
            ks1 = {r: c1.gen_rotation_key(s1, r, 9) for r in rots}
            ev1 = LY.HEEval(c1, ks1, c1.gen_relin_key(s1, 9))
            kern1, _ = LY.conv_plaintexts(fm1, synth.conv_weights(11, 6, 1, 5, 0.1), 1, 0, slots)
            kp1 = [c1.encode(v, c1.pr.scale, 8) for v in kern1]
            pm1 = [c1.encode(v, c1.pr.scale, 8) for v in LY.avgpool_plaintexts(f1, 2, 2, slots)]
            x1 = c1.encrypt(p1, c1.encode(LY.pack(synth.image(11, 1, 28, 28), fm1, slots), c1.pr.scale, 8), 9)

            def lenet():
                y, f = LY.conv2d(ev1, x1, fm1, 6, 5, 1, 0, kp1, [], slots)
                p = LY.relu_poly4(ev1, y, c1.pr.scale)
                LY.avgpool(ev1, p, f, 2, 2, pm1)

            t_l, _ = _timed_cpu(lenet, 0.0, 1)
            layers.setdefault("lenet5_stack_n14_ms", {})[tag] = round(t_l * 1e3, 1)
            layers.setdefault("lenet5_stack_n14_costed_ms", {})[tag] = round(_lenet_cost(c1costs) * 1e3, 1)
            # bootstrapping at N=2^16 L=24 measured whole on all cores (the
            # cosine-with-double-angles variant of the bootstrap section; keys
            # and plaintexts made before the timing)
            log("cpu baseline: bootstrapping at N=2^16")
            from oracle import boot as BT

            sb, pb = ctx.keygen(11, hamming=32)
            bplan = BT.BootPlan(16, 3, 12.0, pr.scale, 39, 3)
            kb = {r: ctx.gen_rotation_key(sb, r, 11) for r in bplan.rotations()}
            kb[ckks.CONJ] = ctx.gen_rotation_key(sb, ckks.CONJ, 11)
            rkb = ctx.gen_relin_key(sb, 11)
            bcts, bstc = BT.boot_plaintexts(ctx, bplan, pr.L)
            xb = ctx.encrypt(pb, ctx.encode(synth.uniform_slots(2, pr.n // 2), pr.scale, 1), 11)
            t_b, _ = _timed_cpu(lambda: BT.bootstrap(ctx, xb, bplan, kb, rkb, bcts, bstc), 0.0, 1)
            layers.setdefault("bootstrap_n16_ms", {})[tag] = round(t_b * 1e3, 1)
            del kb, bcts, bstc
            for name, t in _resnet_costs(c2costs).items():
                layers.setdefault(name + "_costed_ms", {})[tag] = round(t * 1e3, 1)
            res["_c2_rot_nproc"] = c2costs[24]["rot"]
        else:
            layers.setdefault("lenet5_stack_n14_costed_ms", {})[tag] = round(_lenet_cost(c1costs) * 1e3, 1)
            # the N = 2^16 layers at one thread: the all-cores costs scaled by the
            # measured one-thread / all-cores ratio of the single rotation
            ratio = t_rot * 1.0 / res.pop("_c2_rot_nproc")
            for name in ("resnet_convA", "resnet_convB", "resnet_gap", "resnet_fc"):
                key_ = name + "_costed_ms"
                layers[key_][tag] = round(layers[key_]["threads_%d" % cores] * ratio, 1)
            res["single_thread_scale_for_n16_layers"] = round(ratio, 3)
    _omp_threads(cores)
    res["layers"] = layers
    res["method"] = ("value: rotations timed whole; *_ms measured whole; *_costed_ms: the layer's schedule "
                     "run on slot vectors with every rotation (ModUp and per-rotation share of hoisted sets), "
                     "product, addition, rescale and relinearisation priced at the oracle's measured time for "
                     "its level (linear between two measured levels); the one-thread N=2^16 layers scale the "
                     "all-core costs by the measured one-thread/all-core ratio of a single rotation")
    return res


def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py: measures one GPU only (--gpus %d refused)" % args.gpus, file=sys.stderr)
        sys.exit(2)
    import torch

    torch.cuda.init()
    if args.copy_calibration:
        src = torch.ones(1 << 25, dtype=torch.int64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes": src.numel() * 8, "copies": 3}), flush=True)
        return
    log("headline: plain key-switch rotations")
    rot_s, el, roof, kern, ks_bytes, (L, K, dnum) = headline(args)
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
        "config": {"workload": "plain he_rotate, one ciphertext at a time, N=2^16 L=24 K=9 dnum=3, "
                               "%d rotations per step cycling %d resident keys" % (ROT_PER_STEP, len(ROTATIONS)),
                   "log_n": 16, "limbs": L, "special_primes": K, "dnum": dnum},
        "keyswitch_hbm_frac": round(rot_s * ks_bytes / 1e9 / HBM_PEAK_GBS, 4),
        "roofline": roof,
        "kernels": {k: {"launches": v["launches"], "ms": round(v["ms"], 3)} for k, v in kern.items()},
    }
    sections = [] if args.only_headline else (
        [args.only] if args.only else ["hoisted", "layers", "bootstrap", "batched", "serving"])
    if not args.only_headline and not args.only:
        log("headline rotations on two streams")
        result["two_streams"] = two_stream_rotations(args)
    if "hoisted" in sections:
        log("hoisted rotation sets (8 and 49 rotations per ModUp)")
        result["hoisted"] = hoisted_sets()
    if "layers" in sections:
        log("layer latencies")
        result["layers"] = layer_latencies()
    if "bootstrap" in sections:
        log("bootstrapping at N=2^16")
        result["bootstrap"] = bootstrap_latency()
    if "batched" in sections:
        log("batched key switching (64 ciphertexts)")
        result["batched"] = batched()
    if "serving" in sections:
        log("serving")
        result["serving"] = serving(args.serve_requests)
    if not args.no_cpu:
        log("cpu baseline (oracle)")
        result["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
