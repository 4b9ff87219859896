"""GPU vs oracle parity for the layer schedules (needs MI355X).

Every layer output is compared with the oracle's ciphertext on every limb
(same keys, same encrypted input, same oracle-encoded plaintexts), and its
decryption with the paper's FP64 layer equation.
"""
import numpy as np
import pytest
import torch

import synth
from oracle import ckks
from oracle import layers as LY
from tests import helpers as H

pytestmark = pytest.mark.gpu

RELU_COEFFS = [LY.RELU4[0], LY.RELU4[1], LY.RELU4[2], 0.0, LY.RELU4[4]]


@pytest.fixture(scope="module")
def gctx():
    cache = {}

    def get(name):
        if name not in cache:
            cache[name] = H.gpu_ctx(name)
        return cache[name]

    yield get
    for c in cache.values():
        c.close()


def setup_keys(g, name, rots, relin=False):
    from paper_2510_03996_amd import he

    for r in rots:
        g.key_upload(r, H.oracle_key(name, r))
    if relin:
        g.key_upload(he.KEY_RELIN, H.oracle_key(name, "relin"))
    return LY.HEEval(H.oracle_ctx(name)[0], H.oracle_keys(name, rots),
                     H.oracle_key(name, "relin") if relin else None)


def encode(octx, vecs, level):
    return [octx.encode(v, octx.pr.scale, level) for v in vecs]


def gpts(g, pts):
    return [g.pt_from_numpy(p.data, p.scale) for p in pts]


def check_ct(got, want, what):
    H.assert_limbs_equal(got.numpy(), want.data, what)
    assert got.level == want.level and got.scale == want.scale, what


def fm_he(fm):
    from paper_2510_03996_amd import he

    return he.he_fmap(*fm.key())


def encrypt_map(name, X, fm, seed, level=None):
    octx, _, _ = H.oracle_ctx(name)
    _, ct = H.encrypt_slots(name, seed, level=level, values=LY.pack(X, fm, octx.n // 2))
    return ct


def run_conv(g, name, X, K, fm, stride, padding, seed, level=None, logstep=False, bsgs=False, streams=(2,),
             slog=False, groups=False):
    """One oracle convolution; the GPU result with each layer-stream count in
    `streams` must equal it bit for bit."""
    from paper_2510_03996_amd import he

    octx, sk, _ = H.oracle_ctx(name)
    slots = octx.n // 2
    F, _, k, _ = K.shape
    g.conv_channel_sum(he.CHSUM_LOG if logstep else he.CHSUM_CHAIN)
    g.mask_chains(he.CHAIN_BSGS if bsgs else he.CHAIN_HORNER)
    g.striding(he.STRIDE_LOG if slog else he.STRIDE_EXTRACT)
    g.stride_groups(he.STRIDE_GROUP_IN if groups else he.STRIDE_JOINT)
    sg = fm.C if groups else 0
    plan = g.conv2d_plan(fm_he(fm), F, k, stride, padding)
    assert sorted(plan.keys()) == LY.conv_rotations(fm, F, k, stride, padding, slots, logstep=logstep, bsgs=bsgs,
                                                    stride_log=slog, stride_group=sg)
    ev = setup_keys(g, name, plan.keys())
    ct = encrypt_map(name, X, fm, seed, level)
    kern, masks = LY.conv_plaintexts(fm, K, stride, padding, slots, bsgs=bsgs, stride_log=slog, stride_group=sg)
    assert (plan.n_kernel_pts, plan.n_mask_pts) == (len(kern), len(masks))
    kp, mp = encode(octx, kern, ct.level), encode(octx, masks, ct.level)
    want, fo = LY.conv2d(ev, ct, fm, F, k, stride, padding, kp, mp, slots, logstep=logstep, bsgs=bsgs,
                         stride_log=slog, stride_group=sg)
    assert ev.ks == plan.key_switches and ct.level - want.level == plan.levels
    gct, gkp, gmp = g.ct_from_numpy(ct.data, ct.scale), gpts(g, kp), gpts(g, mp)
    for n in streams:
        g.layer_streams(n)
        got, gfm = g.conv2d(gct, fm_he(fm), F, k, stride, padding, gkp, gmp)
        torch.cuda.synchronize()
        assert gfm.key() == fo.key()
        check_ct(got, want, "conv2d with %d layer stream(s)" % n)
    g.layer_streams(2)  # the library default
    dec = LY.unpack(octx.decrypt(sk, ckks.Ciphertext(got.numpy(), got.scale)), fo)
    err = np.max(np.abs(dec - LY.conv2d_ref(X, K, stride, padding)))
    assert err < 1e-3, err
    g.conv_channel_sum(he.CHSUM_CHAIN)
    g.mask_chains(he.CHAIN_HORNER)
    g.striding(he.STRIDE_EXTRACT)
    g.stride_groups(he.STRIDE_JOINT)
    return got, want, fo


def test_config0_special_conv(gctx):
    X = synth.image(20, 1, 8, 8)
    K = synth.conv_weights(20, 1, 1, 3, 0.1)
    run_conv(gctx("config0"), "config0", X, K, LY.FMap(1, 8, 8), 1, 1, 20, streams=(1, 2))


def test_config1_generic_conv_multichannel_stride(gctx):
    """C=3 -> F=4, 3x3, stride 2, pad 0 at N=2^14 (channel chain, block-0 mask, placement, compaction)."""
    X = synth.image(21, 3, 12, 12)
    K = synth.conv_weights(21, 4, 3, 3, 0.2)
    run_conv(gctx("config1"), "config1", X, K, LY.FMap(3, 12, 12), 2, 0, 21, streams=(1, 2, 3, 8))


@pytest.mark.parametrize("C,F,H,W,rs,cs,k,S,P,bsgs", [
    (2, 3, 8, 8, None, None, 3, 1, 2, False),    # 3x3 / padding 2: channels then rows, then the shift
    (3, 2, 10, 10, None, None, 1, 2, 1, True),   # 1x1 / stride 2 / padding 1, baby-step giant-step chains
    (2, 2, 6, 6, 30, 180, 3, 1, 2, False),       # wide input rows: rows first, then channels
    (1, 2, 7, 9, None, None, 5, 2, 3, False),    # one channel, rectangular, strided
])
def test_config1_relayout_padded_conv(gctx, C, F, H, W, rs, cs, k, S, P, bsgs):
    """Padding beyond (k-1)/2: the re-layout as X_p and the generic schedule
    with P = 0, bit for bit against the oracle."""
    X = synth.image(30 + k, C, H, W)
    K = synth.conv_weights(30 + k, F, C, k, 0.2)
    fm = LY.FMap(C, H, W, rs, cs)
    assert LY.conv_kind(k, P, fm, F) == "padded"
    run_conv(gctx("config1"), "config1", X, K, fm, S, P, 30 + k, bsgs=bsgs, streams=(1, 2))


@pytest.mark.parametrize("bsgs", [False, True], ids=["horner", "bsgs"])
def test_config1_log_step_striding_conv(gctx, bsgs):
    """Striding approach 2 (log-step column moves): C=3 -> F=4, 3x3, stride 2,
    pad 1 at N=2^14, bit for bit against the oracle."""
    X = synth.image(34, 3, 12, 12)
    K = synth.conv_weights(34, 4, 3, 3, 0.2)
    run_conv(gctx("config1"), "config1", X, K, LY.FMap(3, 12, 12), 2, 1, 34, bsgs=bsgs, streams=(1, 2), slog=True)


@pytest.mark.parametrize("slog,bsgs", [(False, False), (True, False), (True, True)],
                         ids=["extract", "logstride", "logstride_bsgs"])
def test_config1_grouped_striding_conv(gctx, slog, bsgs):
    """The paper's multi-channel striding pipeline (groups of the layer's 2
    input channels: 2 + 2 + 1 of the 5 outputs, merged with one more key):
    generic 3x3 / stride 2 / pad 1 at N=2^14, with both striding approaches
    and baby-step giant-step chains, bit for bit against the oracle."""
    X = synth.image(36, 2, 12, 12)
    K = synth.conv_weights(36, 5, 2, 3, 0.2)
    run_conv(gctx("config1"), "config1", X, K, LY.FMap(2, 12, 12), 2, 1, 36, streams=(1, 2), slog=slog, groups=True,
             bsgs=bsgs)


def test_config1_grouped_striding_special_conv(gctx):
    """The special schedule (replicated 4 x 32 x 32 input, 4 -> 8 channels,
    stride 2) with the multi-channel pipeline's two groups of 4 at N=2^14."""
    X = synth.image(37, 4, 32, 32)
    K = synth.conv_weights(37, 8, 4, 3, 0.1)
    run_conv(gctx("config1"), "config1", X, K, LY.FMap(4, 32, 32, reps=2), 2, 1, 37, groups=True)


def test_config1_log_step_striding_pool(gctx):
    """2x2 / stride 2 pooling of 6 x 24 x 24 (row stride 28) with approach 2."""
    from paper_2510_03996_amd import he

    name = "config1"
    g = gctx(name)
    octx, sk, _ = H.oracle_ctx(name)
    slots = octx.n // 2
    X = synth.image(35, 6, 24, 24)
    fm = LY.FMap(6, 24, 24, 28, 784)
    g.striding(he.STRIDE_LOG)
    try:
        plan = g.avgpool_plan(fm_he(fm), 2, 2)
        assert sorted(plan.keys()) == LY.avgpool_rotations(fm, 2, 2, stride_log=True)
        ev = setup_keys(g, name, plan.keys())
        ct = encrypt_map(name, X, fm, 35)
        mp = encode(octx, LY.avgpool_plaintexts(fm, 2, 2, slots, stride_log=True), ct.level)
        want, fo = LY.avgpool(ev, ct, fm, 2, 2, mp, stride_log=True)
        got, gfo = g.avgpool(g.ct_from_numpy(ct.data, ct.scale), fm_he(fm), 2, 2, gpts(g, mp))
        assert ev.ks == plan.key_switches and ct.level - want.level == plan.levels == 6
        check_ct(got, want, "log-step strided avgpool")
        dec = LY.unpack(octx.decrypt(sk, ckks.Ciphertext(got.numpy(), got.scale)), fo)
        assert np.max(np.abs(dec - LY.avgpool_ref(X, 2, 2))) < 1e-3
    finally:
        g.striding(he.STRIDE_EXTRACT)


def test_config1_lenet_stack(gctx):
    """LeNet-5-shaped stack: conv 5x5 1->6 -> degree-4 ReLU -> 2x2 avgpool (7 levels)."""
    name = "config1"
    g = gctx(name)
    octx, sk, _ = H.oracle_ctx(name)
    slots = octx.n // 2
    X = synth.image(22, 1, 28, 28)
    K = synth.conv_weights(22, 6, 1, 5, 0.1)
    fm = LY.FMap(1, 28, 28)
    got, want, f1 = run_conv(g, name, X, K, fm, 1, 0, 22)
    # polynomial ReLU
    ev = setup_keys(g, name, [], relin=True)
    pw = LY.relu_poly4(ev, want, octx.pr.scale)
    pg = g.poly4(got, RELU_COEFFS, octx.pr.scale)
    check_ct(pg, pw, "poly4")
    # pooling
    plan = g.avgpool_plan(fm_he(f1), 2, 2)
    assert sorted(plan.keys()) == LY.avgpool_rotations(f1, 2, 2)
    ev = setup_keys(g, name, plan.keys())
    mp = encode(octx, LY.avgpool_plaintexts(f1, 2, 2, slots), pw.level)
    zw, f2 = LY.avgpool(ev, pw, f1, 2, 2, mp)
    zg, gf2 = g.avgpool(pg, fm_he(f1), 2, 2, gpts(g, mp))
    assert gf2.key() == f2.key() and zw.level == 1
    check_ct(zg, zw, "avgpool")
    ref = LY.avgpool_ref(LY.relu4_ref(LY.conv2d_ref(X, K, 1, 0)), 2, 2)
    dec = LY.unpack(octx.decrypt(sk, ckks.Ciphertext(zg.numpy(), zg.scale)), f2)
    assert np.max(np.abs(dec - ref)) < 1e-2


def test_config2_small_special_conv(gctx):
    """4 replicated channels of 64x64 at N=2^16, L=24 (20 key switches)."""
    X = synth.image(23, 4, 64, 64)
    K = synth.conv_weights(23, 4, 4, 3, (2.0 / 36) ** 0.5)
    run_conv(gctx("config2"), "config2", X, K, LY.FMap(4, 64, 64, reps=2), 1, 1, 23, streams=(1, 3, 4))


def test_config2_conv_a(gctx):
    """ResNet-20-shaped conv 3x3 16->16, stride 1, pad 1 on a replicated 16x32x32 input (248 key switches)."""
    X = synth.image(24, 16, 32, 32)
    K = synth.conv_weights(24, 16, 16, 3, (2.0 / 144) ** 0.5)
    got, want, fo = run_conv(gctx("config2"), "config2", X, K, LY.FMap(16, 32, 32, reps=2), 1, 1, 24,
                             streams=(1, 4))
    assert fo.reps == 2


def test_config2_conv_b(gctx):
    """conv 3x3 16->32, stride 2, pad 1 at level 22 (549 key switches, joint stride compaction)."""
    X = synth.image(25, 16, 32, 32)
    K = synth.conv_weights(25, 32, 16, 3, (2.0 / 144) ** 0.5)
    run_conv(gctx("config2"), "config2", X, K, LY.FMap(16, 32, 32, reps=2), 2, 1, 25, level=22, streams=(1, 4))


@pytest.mark.parametrize("C,HW,level", [(32, 16, 17), (64, 8, 17)])
def test_config2_global_avgpool(gctx, C, HW, level):
    name = "config2"
    g = gctx(name)
    octx, sk, _ = H.oracle_ctx(name)
    slots = octx.n // 2
    X = synth.image(26, C, HW, HW)
    fm = LY.FMap(C, HW, HW)
    plan = g.avgpool_plan(fm_he(fm), 0, 1)
    assert sorted(plan.keys()) == LY.gap_rotations(fm)
    ev = setup_keys(g, name, plan.keys())
    ct = encrypt_map(name, X, fm, 26, level)
    mp = encode(octx, LY.gap_plaintexts(fm, slots), ct.level)
    want, fo = LY.gap(ev, ct, fm, mp)
    got, gfo = g.avgpool(g.ct_from_numpy(ct.data, ct.scale), fm_he(fm), 0, 1, gpts(g, mp))
    assert ev.ks == plan.key_switches
    check_ct(got, want, "global avgpool")
    dec = octx.decrypt(sk, ckks.Ciphertext(got.numpy(), got.scale))
    assert np.max(np.abs(dec[:C] - LY.gap_ref(X))) < 1e-3


def test_config1_pool_whole_channel(gctx):
    """A k = H = W window takes the global schedule (pooling special case)."""
    name = "config1"
    g = gctx(name)
    octx, sk, _ = H.oracle_ctx(name)
    slots = octx.n // 2
    C, HW = 16, 8
    X = synth.image(27, C, HW, HW)
    fm = LY.FMap(C, HW, HW)
    plan = g.avgpool_plan(fm_he(fm), HW, HW)
    assert sorted(plan.keys()) == LY.avgpool_rotations(fm, HW, HW) == LY.gap_rotations(fm)
    assert plan.levels == 1
    ev = setup_keys(g, name, plan.keys())
    ct = encrypt_map(name, X, fm, 27, 5)
    mp = encode(octx, LY.avgpool_plaintexts(fm, HW, HW, slots), ct.level)
    want, fo = LY.avgpool(ev, ct, fm, HW, HW, mp)
    got, gfo = g.avgpool(g.ct_from_numpy(ct.data, ct.scale), fm_he(fm), HW, HW, gpts(g, mp))
    assert ev.ks == plan.key_switches
    assert (gfo.channels, gfo.height, gfo.width) == (C, 1, 1)
    check_ct(got, want, "whole-channel avgpool")
    dec = octx.decrypt(sk, ckks.Ciphertext(got.numpy(), got.scale))
    assert np.max(np.abs(dec[:C] - LY.avgpool_ref(X, HW, HW).reshape(-1))) < 1e-3


def test_config2_fc(gctx):
    name = "config2"
    g = gctx(name)
    octx, sk, _ = H.oracle_ctx(name)
    slots = octx.n // 2
    x = np.zeros(64)
    x[:32] = synth.uniform_slots(27, 32)  # global pooling of 32 channels, zeros above (64-slot input)
    Wm = synth.fc_weights(27, 10, 64, (2.0 / 64) ** 0.5)
    plan = g.fc_plan(64, 10)
    assert sorted(plan.keys()) == LY.fc_rotations(64, 10)
    ev = setup_keys(g, name, plan.keys())
    v = np.zeros(slots)
    v[:64] = x
    _, ct = H.encrypt_slots(name, 27, level=16, values=v)
    rows, masks = LY.fc_plaintexts(Wm, slots)
    rp, mp = encode(octx, rows, ct.level), encode(octx, masks, ct.level)
    want = LY.fc(ev, ct, 64, 10, rp, mp)
    assert ev.ks == plan.key_switches == 69
    gct, grp, gmp = g.ct_from_numpy(ct.data, ct.scale), gpts(g, rp), gpts(g, mp)
    for n in (1, 2, 4):  # neurons over the caller's stream and n - 1 helpers
        g.layer_streams(n)
        got = g.fc(gct, 64, 10, grp, gmp)
        torch.cuda.synchronize()
        check_ct(got, want, "fc with %d stream(s)" % n)
    g.layer_streams(2)
    dec = octx.decrypt(sk, ckks.Ciphertext(got.numpy(), got.scale))
    assert np.max(np.abs(dec[:10] - LY.fc_ref(x, Wm))) < 1e-3


@pytest.mark.parametrize("C,F,HW,k,S,P", [(3, 2, 16, 7, 2, 3), (3, 4, 12, 3, 1, 1), (2, 3, 12, 5, 2, 2),
                                          (4, 3, 8, 1, 2, 0)])
def test_config1_padded_conv(gctx, C, F, HW, k, S, P):
    """Padding by masked taps: 7x7/s2/p3 (ResNet-34 stem shape), 3x3/p1 on a
    non-replicated multi-channel map, 5x5/s2/p2; and a 1x1 / stride 2 kernel
    (no tap rotation at all)."""
    X = synth.image(29, C, HW, HW)
    K = synth.conv_weights(29, F, C, k, 0.15)
    run_conv(gctx("config1"), "config1", X, K, LY.FMap(C, HW, HW), S, P, 29)


def test_layer_errors(gctx):
    from paper_2510_03996_amd import he

    name = "config1"
    g = gctx(name)
    fm = he.fmap(1, 28, 28)
    with pytest.raises(he.HEError) as e:
        g.conv2d_plan(fm, 6, 9, 1, 4)  # 80 tap keys: more than a plan lists
    assert e.value.name == "HE_EUNSUPPORTED"
    _, ct = H.encrypt_slots(name, 28, level=2)
    gct = g.ct_from_numpy(ct.data, ct.scale)
    plan = g.conv2d_plan(fm, 6, 5, 1, 0)
    with pytest.raises(he.HEError) as e:  # wrong plaintext count
        g.conv2d(gct, fm, 6, 5, 1, 0, [], [])
    assert e.value.name == "HE_EINVAL"
    with pytest.raises(he.HEError) as e:  # level 2 cannot afford 3-level polynomial
        g.poly4(gct, RELU_COEFFS, 2.0 ** 45)
    assert e.value.name in ("HE_ELEVEL", "HE_ENOKEY")
    assert plan.n_kernel_pts == 150


@pytest.mark.parametrize("stride", [1, 2])
def test_config2_special_conv_logstep(gctx, stride):
    """Log-step input-channel sum (he_ctx_conv_channel_sum): 4 replicated
    channels of 64x64 at N=2^16, keys W^2 and 2 W^2, stride 1 and 2."""
    X = synth.image(71, 4, 64, 64)
    K = synth.conv_weights(71, 4, 4, 3, (2.0 / 36) ** 0.5)
    run_conv(gctx("config2"), "config2", X, K, LY.FMap(4, 64, 64, reps=2), stride, 1, 71, logstep=True,
             streams=(1, 2))


def test_config1_generic_conv_logstep(gctx):
    """Log-step channel sum in the generic schedule: C=4 -> F=3, 5x5, stride 2,
    pad 2 at N=2^14 (keys cs and 2 cs)."""
    X = synth.image(72, 4, 16, 16)
    K = synth.conv_weights(72, 3, 4, 5, 0.1)
    run_conv(gctx("config1"), "config1", X, K, LY.FMap(4, 16, 16), 2, 2, 72, logstep=True, streams=(1, 4))


def test_channel_sum_mode_errors(gctx):
    from paper_2510_03996_amd import he

    g = gctx("config0")
    with pytest.raises(he.HEError) as e:
        g.conv_channel_sum(7)
    assert e.value.name == "HE_EINVAL"


def test_config2_special_conv_stride2_bsgs(gctx):
    """Baby-step giant-step stride compaction (he_ctx_mask_chains) with the
    log-step channel sum: 16 replicated channels of 32x32 -> 8, stride 2."""
    X = synth.image(73, 16, 32, 32)
    K = synth.conv_weights(73, 8, 16, 3, (2.0 / 144) ** 0.5)
    fm = LY.FMap(16, 32, 32, reps=2)
    run_conv(gctx("config2"), "config2", X, K, fm, 2, 1, 73, level=20, logstep=True, bsgs=True)


def test_config1_generic_conv_bsgs(gctx):
    """Generic schedule with both options: C=4 -> F=3, 5x5, stride 2, pad 2 (N=2^14)."""
    X = synth.image(74, 4, 16, 16)
    K = synth.conv_weights(74, 3, 4, 5, 0.1)
    run_conv(gctx("config1"), "config1", X, K, LY.FMap(4, 16, 16), 2, 2, 74, logstep=True, bsgs=True)


def test_config1_avgpool_bsgs(gctx):
    """2x2 average pooling of a 6x24x24 map with the baby-step giant-step compaction."""
    from paper_2510_03996_amd import he

    name = "config1"
    g = gctx(name)
    octx, sk, _ = H.oracle_ctx(name)
    slots = octx.n // 2
    X = synth.image(75, 6, 24, 24)
    f1 = LY.FMap(6, 24, 24, 28, 784)
    g.mask_chains(he.CHAIN_BSGS)
    try:
        plan = g.avgpool_plan(fm_he(f1), 2, 2)
        assert sorted(plan.keys()) == LY.avgpool_rotations(f1, 2, 2, bsgs=True)
        ev = setup_keys(g, name, plan.keys())
        ct = encrypt_map(name, X, f1, 75, 5)
        mp = encode(octx, LY.avgpool_plaintexts(f1, 2, 2, slots, bsgs=True), ct.level)
        zw, f2 = LY.avgpool(ev, ct, f1, 2, 2, mp, bsgs=True)
        zg, gf2 = g.avgpool(g.ct_from_numpy(ct.data, ct.scale), fm_he(f1), 2, 2, gpts(g, mp))
        assert ev.ks == plan.key_switches and gf2.key() == f2.key()
        check_ct(zg, zw, "avgpool bsgs")
        dec = LY.unpack(octx.decrypt(sk, ckks.Ciphertext(zg.numpy(), zg.scale)), f2)
        assert np.max(np.abs(dec - LY.avgpool_ref(X, 2, 2))) < 1e-3
    finally:
        g.mask_chains(he.CHAIN_HORNER)


def test_config2_global_avgpool_bsgs(gctx):
    from paper_2510_03996_amd import he

    name = "config2"
    g = gctx(name)
    octx, sk, _ = H.oracle_ctx(name)
    slots = octx.n // 2
    C, HW = 32, 16
    X = synth.image(76, C, HW, HW)
    fm = LY.FMap(C, HW, HW)
    g.mask_chains(he.CHAIN_BSGS)
    try:
        plan = g.avgpool_plan(fm_he(fm), 0, 1)
        assert sorted(plan.keys()) == LY.gap_rotations(fm, bsgs=True) and plan.key_switches == 8 + 10
        ev = setup_keys(g, name, plan.keys())
        ct = encrypt_map(name, X, fm, 76, 17)
        mp = encode(octx, LY.gap_plaintexts(fm, slots, bsgs=True), ct.level)
        want, fo = LY.gap(ev, ct, fm, mp, bsgs=True)
        got, gfo = g.avgpool(g.ct_from_numpy(ct.data, ct.scale), fm_he(fm), 0, 1, gpts(g, mp))
        assert ev.ks == plan.key_switches
        check_ct(got, want, "global avgpool bsgs")
        dec = octx.decrypt(sk, ckks.Ciphertext(got.numpy(), got.scale))
        assert np.max(np.abs(dec[:C] - LY.gap_ref(X))) < 1e-3
    finally:
        g.mask_chains(he.CHAIN_HORNER)


def test_chain_mode_errors(gctx):
    from paper_2510_03996_amd import he

    g = gctx("config0")
    with pytest.raises(he.HEError) as e:
        g.mask_chains(2)
    assert e.value.name == "HE_EINVAL"


@pytest.mark.parametrize("n_in,n_out,name", [(64, 10, "config2"), (32, 32, "config1"), (8, 3, "config0")])
def test_fc_diag(gctx, n_in, n_out, name):
    """Diagonal (baby-step giant-step) fully connected form (he_ctx_fc_form)."""
    from paper_2510_03996_amd import he

    g = gctx(name)
    octx, sk, _ = H.oracle_ctx(name)
    slots = octx.n // 2
    x = synth.uniform_slots(78 + n_in, n_in)
    Wm = synth.fc_weights(78 + n_out, n_out, n_in, (2.0 / n_in) ** 0.5)
    g.fc_form(he.FC_DIAG)
    try:
        plan = g.fc_plan(n_in, n_out)
        assert sorted(plan.keys()) == LY.fc_diag_rotations(n_in) and plan.n_mask_pts == 0
        ev = setup_keys(g, name, plan.keys())
        v = np.zeros(slots)
        v[:n_in] = x
        level = min(octx.pr.L, 16)
        _, ct = H.encrypt_slots(name, 78, level=level, values=v)
        dp = encode(octx, LY.fc_diag_plaintexts(Wm, slots), ct.level)
        want = LY.fc_diag(ev, ct, n_in, n_out, dp)
        got = g.fc(g.ct_from_numpy(ct.data, ct.scale), n_in, n_out, gpts(g, dp), [])
        assert ev.ks == plan.key_switches and got.level == ct.level - 1
        check_ct(got, want, "fc diag")
        dec = octx.decrypt(sk, ckks.Ciphertext(got.numpy(), got.scale))
        assert np.max(np.abs(dec[:n_out] - LY.fc_ref(x, Wm))) < 1e-3
    finally:
        g.fc_form(he.FC_ROWS)


def test_layer_streams_errors(gctx):
    from paper_2510_03996_amd import he

    g = gctx("config0")
    for bad in (0, 9, -1):
        with pytest.raises(he.HEError) as e:
            g.layer_streams(bad)
        assert e.value.name == "HE_EINVAL"
    g.layer_streams(2)


def test_fc_form_errors(gctx):
    from paper_2510_03996_amd import he

    g = gctx("config0")
    with pytest.raises(he.HEError) as e:
        g.fc_form(5)
    assert e.value.name == "HE_EINVAL"
    g.fc_form(he.FC_DIAG)
    try:
        with pytest.raises(he.HEError) as e:
            g.fc_plan(8, 9)  # more outputs than inputs
        assert e.value.name == "HE_EINVAL"
    finally:
        g.fc_form(he.FC_ROWS)


@pytest.mark.parametrize("name,case", [
    ("config0", (1, 8, 8, 1, 1, 3, 1, 1)),       # special, single channel
    ("config1", (3, 12, 12, 1, 4, 3, 2, 0)),     # generic, channel chain + placement + compaction
    ("config1", (2, 10, 10, 1, 2, 5, 2, 2)),     # generic 5x5 / s2 / p2
], ids=["special_n12", "generic_s2_n14", "generic_p2_n14"])
def test_conv_with_bias_from_library_recipes(gctx, name, case):
    """The library's own plaintext recipes (he_layer_plaintexts: kernel
    vectors, masks and the bias vector) drive the GPU convolution; the oracle
    runs its own recipes (conv_plaintexts, conv_bias_vector).  The vectors are
    equal, so the oracle-encoded plaintexts and the ciphertexts are too; the
    decryption matches the FP64 convolution plus bias."""
    from paper_2510_03996_amd import he

    nc, nh, nw, reps, F, k, S, P = case
    g = gctx(name)
    octx, sk, _ = H.oracle_ctx(name)
    slots = octx.n // 2
    X = synth.image(60, nc, nh, nw)
    K = synth.conv_weights(60, F, nc, k, 0.2)
    b = synth.uniform_slots(61, F, -0.5, 0.5)
    fm = LY.FMap(nc, nh, nw, reps=reps)
    plan = g.conv2d_plan(fm_he(fm), F, k, S, P)
    vecs = he.layer_plaintexts(he.LAYER_CONV, octx.pr.log_n, K, b, fm=fm_he(fm), out_ch=F, kernel=k, stride=S,
                               padding=P)
    assert vecs.shape[0] == plan.n_kernel_pts + plan.n_mask_pts + 1
    ev = setup_keys(g, name, plan.keys())
    ct = encrypt_map(name, X, fm, 62)
    L = ct.level
    kern, masks = LY.conv_plaintexts(fm, K, S, P, slots)
    fo = LY.conv_out_map(fm, F, k, S, P, slots)
    out_level = L - plan.levels
    # oracle: its own vectors; the bias at the output's scale and level
    y0, _ = LY.conv2d(ev, ct, fm, F, k, S, P, encode(octx, kern, L), encode(octx, masks, L), slots)
    bias_o = octx.encode(LY.conv_bias_vector(fo, b, slots), y0.scale, out_level)
    want = octx.add_plain(y0, bias_o)
    # GPU: the library's vectors, encoded by the same encoder
    nk = plan.n_kernel_pts
    gk = gpts(g, encode(octx, list(vecs[:nk]), L))
    gm = gpts(g, encode(octx, list(vecs[nk:nk + plan.n_mask_pts]), L))
    gb = g.pt_from_numpy(octx.encode(vecs[-1], y0.scale, out_level).data, y0.scale)
    got, gfm = g.conv2d(g.ct_from_numpy(ct.data, ct.scale), fm_he(fm), F, k, S, P, gk, gm, bias_pt=gb)
    torch.cuda.synchronize()
    assert gfm.key() == fo.key()
    check_ct(got, want, "conv2d + bias")
    dec = LY.unpack(octx.decrypt(sk, ckks.Ciphertext(got.numpy(), got.scale)), fo)
    err = np.max(np.abs(dec - LY.conv2d_ref(X, K, S, P, bias=b)))
    assert err < 1e-3, err
